/* Plain FP64 CPU oracle for the VMC energy/force estimate and the
 * covariance-preconditioned Langevin step of Sorella & Mazzola,
 * "Accelerated ab-initio Molecular Dynamics: probing the weak dispersive
 * forces in dense liquid hydrogen" (arXiv:1605.08423).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle is slow on purpose and exists to
 * check the GPU library.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the product path never links it and
 * shares no code with it.
 *
 * Parity status per function is listed in the .c file's header.
 */
#ifndef VMC_ORACLE_H
#define VMC_ORACLE_H
#include <stdint.h>

enum { OB_PERIODIC_GAUSS = 0, OB_OPEN_GAUSS = 1, OB_OPEN_STO = 2 };
enum { OP_EWALD = 0, OP_COULOMB_OPEN = 1, OP_HARMONIC = 2, OP_NONE = 3 };

typedef struct {
  int n_p;           /* protons = basis centres, charge +1 */
  int n_up, n_dn;    /* electrons per spin; electrons 0..n_up-1 are spin up */
  int n_orb;         /* columns of C (>= max(n_up, n_dn)) */
  double L;          /* cubic box side (periodic kinds) */
  int basis_kind;    /* OB_* */
  int pot_kind;      /* OP_* */
  double kappa;      /* Ewald splitting parameter */
  int nmax;          /* Ewald reciprocal cutoff: 0 < |n|^2 <= nmax^2 */
  int jastrow_on;
  double a_par, a_anti, b;   /* Pade u = a rho / (1 + b rho) */
  const double* R;     /* n_p x 3 */
  const double* zeta;  /* n_p */
  const double* C;     /* n_p x n_orb, row-major */
  double b1;           /* one-body (electron-nucleus) Jastrow U_1 of the SI, Eq. e:j1, with
                          Z_a = 1 and no orbital part: b_1 of u_1(x) = (1 - e^{-b_1 x})/(2 b_1);
                          0 = no one-body term */
  int twist;           /* twisted boundary conditions with real twists: bit m set means
                          phi(r + L e_m) = -phi(r) (twist angle pi along axis m), clear means
                          periodic (angle 0); the Jastrow stays periodic */
  int contracted;      /* 1: the SI's contracted orbital per proton, phi_1 + eta phi_2 with
                          phi_1 = e^{-Z1 r^2}, phi_2 = r^2 e^{-Z2 r^2} (O_Z1, O_Z2; zeta unused),
                          with the same image sums and twists as the single Gaussian; 0: e^{-zeta r^2} */
  double eta;          /* the contraction coefficient eta (contracted = 1) */
  double j3f[3];       /* the on-site three-body (electron-electron-nucleus) Jastrow term U_3 of the SI
                          (Eq. e:j33): f_11, f_12 = f_21, f_22 of the 2 x 2 matrix coupling the
                          orbitals chi_1 = e^{-ZJ rho^2}, chi_2 = rho^2 e^{-ZJ rho^2} (O_ZJ) of two
                          electrons on the same nucleus, the same for every nucleus; all zero = no term */
  double j1f[2];       /* the orbital part of the one-body Jastrow term U_1 of the SI (Eq. e:j1):
                          sum_a sum_i (f_1 chi_1 + f_2 chi_2)(r_i - R_a) on the three-body term's
                          orbitals, the same f for every nucleus; both zero = no such part */
} osys;

/* The exponent of the Jastrow orbitals (SI, Jastrow section). */
#define O_ZJ 0.7933844

/* The SI's exponents of the contracted minimal basis (section "Systematic setup"). */
#define O_Z1 0.6066825
#define O_Z2 0.3382168

/* The three-body term's orbitals chi_1, chi_2 of nucleus `atom` at r: out[0..13] and out[14..27]
 * are the 14 components [value, grad(3), lap, hess xx yy zz xy xz yz, grad lap(3)] of each. */
void o_j3_orbitals(const osys* s, int atom, const double r[3], double out[28]);

/* Philox4x32-10 counter-based generator (Salmon et al., SC'11). */
void o_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double o_u01(uint32_t hi, uint32_t lo);

void o_basis(const osys* s, int a, const double r[3], double out[14]);
void o_jastrow(const osys* s, const double* x, double* U, double* gradU, double* lapU);
double o_potential(const osys* s, const double* x, double* dV_dR, double* dV_dx);
/* Adds the proton derivatives of the one-body and three-body Jastrow terms to dln (d ln psi/dR)
 * and dT (dT_L/dR), given vv = grad_i U + grad_i ln|D| per electron (3 N). */
void o_jastrow_dR(const osys* s, const double* x, const double* vv, double* dln, double* dT);
int o_local(const osys* s, const double* x, double* lnpsi, double* sign, double* EL,
            double* dlnpsi_dR, double* dEL_dR);
int o_huckel(int n_p, double L, const double* R, const double* zeta, int n_orb,
             double* C, double* evals);
/* Hueckel orbitals on the contracted periodic basis (no twist): the overlaps of
 * phi_1 + eta phi_2 from one image sum of the free-space overlaps of e^{-Z r^2} and
 * r^2 e^{-Z r^2}, written out as one-dimensional Gaussian moments. */
int o_huckel_contracted(int n_p, double L, const double* R, double eta, int n_orb, double* C, double* evals);
/* The overlap matrix of the contracted periodic basis (n_p x n_p). */
void o_overlap_contracted(int n_p, double L, const double* R, double eta, double* S);
int o_huckel_twist(int n_p, double L, const double* R, const double* zeta, int n_orb, int twist,
                   double* C, double* evals);
/* d ln psi / d p for the Jastrow parameters p = (b, b_1, f_11, f_12, f_22, f_1, f_2) (O_NPAR of
 * them); the b_1 entry is 0 without the one-body cusp part, the three-body entries and those of
 * the one-body orbital part are formed for any F and f. */
#define O_NPAR 7
void o_param_derivs(const osys* s, const double* x, double O[O_NPAR]);
/* Per walker, the parameter statistics of the measured samples: [sum E_L, sum O (O_NPAR),
 * sum E_L O (O_NPAR), sum O O^T (O_NPAR x O_NPAR, row-major)]. */
#define O_NOPT (1 + 2 * O_NPAR + O_NPAR * O_NPAR)
/* o_vmc_run_from that also writes W x O_NOPT parameter sums to popt (NULL: none). */
int o_vmc_run_opt(const osys* s, int W, uint32_t w0, double* x, int n_equil, int n_meas, double delta,
                  uint32_t seed, uint32_t traj, uint32_t step, double* sums, int64_t* n_acc, double* popt,
                  int n_threads);
int o_vmc_run(const osys* s, int W, double* x, int n_equil, int n_meas, double delta,
              uint32_t seed, uint32_t traj, uint32_t step, double* sums, int64_t* n_acc,
              int n_threads);
int o_vmc_run_from(const osys* s, int W, uint32_t w0, double* x, int n_equil, int n_meas,
                   double delta, uint32_t seed, uint32_t traj, uint32_t step, double* sums,
                   int64_t* n_acc, int n_threads);
int o_reduce(int W, int n3, int M, const double* sums, double* E, double* sigma_E,
             double* f, double* f_w, double* means);
void o_build_S(int W, int n3, const double* f_w, const double* f, double* S);
int o_cholesky(int n, const double* S, double* Lc);
int o_langevin(int n3, double L, double* R, double* R_prev, double* S_prev,
               const double* f, const double* S, double T, double Delta, double alpha,
               unsigned flags, uint32_t seed, uint32_t traj, uint32_t step);
int o_langevin_harmonic_run(int n3, const double* K, const double* S, double T, double Delta,
                            double alpha, unsigned flags, uint32_t seed, int n_steps,
                            double* R, double* samples, int sample_every);
int o_toy_run(double lambda, double k, double a, double mu, int s_kind, double T, double Delta,
              double alpha, int scheme, uint32_t seed, uint32_t traj, int n_steps, double* R, double* U_mean,
              double* U_samples);
void o_normals(uint32_t seed, uint32_t traj, uint32_t step, int n, double* xi);
void o_toy_S(double lambda, double k, double a, double mu, int s_kind, const double x[2], double S[4]);

/* General (complex) twisted boundary conditions, vmc_oracle_complex.c: theta[3] the twist
 * angles, complex arrays as (real, imaginary) pairs. */
void o_cbasis(const osys* s, const double theta[3], int a, const double r[3], double out[28]);
void o_cbasis_values(const osys* s, const double theta[3], int npt, const double* pts, double* out);
void o_coverlap(int n_p, double L, const double theta[3], const double* R, const double* zeta, double* S_out);
int o_chuckel(int n_p, double L, const double theta[3], const double* R, const double* zeta, int n_orb, double* C,
              double* evals);
/* The contracted basis (phi_1 + eta phi_2) under the twist: its overlaps and Hueckel orbitals. */
void o_coverlap_contracted(int n_p, double L, const double theta[3], const double* R, double eta, double* S_out);
int o_chuckel_contracted(int n_p, double L, const double theta[3], const double* R, double eta, int n_orb, double* C,
                         double* evals);
int o_clocal(const osys* s, const double theta[3], const double* Cd, const double* x, double* lnpsi, double* phase,
             double* EL, double* dlnpsi_dR, double* dEL_dR);
int o_cvmc_run_from(const osys* s, const double theta[3], const double* Cd, int W, uint32_t w0, double* x,
                    int n_equil, int n_meas, double delta, uint32_t seed, uint32_t traj, uint32_t step, double* sums,
                    int64_t* n_acc, int n_threads);

#define O_STEP_CFOLD 1u
#define O_STEP_NOISE_CORR 2u
#define O_STEP_NO_SCORR 4u

#endif
