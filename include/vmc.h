/* vmc.h -- C ABI of the MI355X library for the variational Monte Carlo (VMC)
 * energy/force estimate and the covariance-preconditioned Langevin step of
 * Sorella & Mazzola, "Accelerated ab-initio Molecular Dynamics: probing the
 * weak dispersive forces in dense liquid hydrogen" (arXiv:1605.08423).
 *
 * Conventions (every entry point):
 *  - Arrays whose name ends in _dev are DEVICE pointers (hipMalloc'd or torch
 *    CUDA tensors) on the context's device; all others are host memory.  The
 *    caller owns every pointer it passes; the library never retains one past
 *    the call.  Arrays are dense, row-major, FP64, in atomic units (bohr,
 *    Hartree).  Vectors over ions are laid out [R_0x, R_0y, R_0z, R_1x, ...].
 *  - Work is queued on the context's stream (vmc_set_stream; default: the
 *    null stream).  Calls returning a status that depends on device results
 *    (VMC_ENOTSPD, VMC_ESINGULAR) synchronise that stream.
 *  - Every call returns VMC_OK (0) or a negative VMC_E* code; no C++ exception
 *    or abort crosses the ABI.  On failure the caller's state arrays are left
 *    unchanged unless noted.
 *  - A context is not thread-safe: one context per host thread.
 *
 * System: N protons (charge +1) and N electrons (N even; electrons 0..N/2-1
 * spin up) in a periodic cube of side L.  Wavefunction psi = D_up D_dn e^U:
 * one Slater determinant per spin, A_s[i][k] = sum_a phi_a(r_i) C[a][k], on
 * s-Gaussians phi_a made periodic by the image sum (SI, "Systematic setup"),
 * times the two-body Pade Jastrow U = sum_{i<j} a rho/(1 + b rho) on the
 * sin-periodised distance (SI, Jastrow section).  Hamiltonian: all-electron
 * Coulomb (main text, Eq. for V(R)), evaluated by Ewald summation.
 */
#ifndef VMC_H
#define VMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VMC_OK = 0,
  VMC_EINVAL = -1,     /* bad size/argument: odd N, unsupported N, W < 2, Delta <= 0, ... */
  VMC_ENOMEM = -2,     /* device allocation failed */
  VMC_ENOTSPD = -3,    /* Cholesky of S failed: S not positive definite */
  VMC_ESINGULAR = -4,  /* a Slater matrix had a zero pivot at an inverse refresh */
  VMC_EDEVICE = -5,    /* a HIP runtime error */
  VMC_ENOTBUILT = -6,  /* no device code for this GPU */
  VMC_ECANCELLED = -7, /* stopped by vmc_cancel or vmc_server_cancel; the state is as before the call */
  VMC_ENOCONV = -8     /* the host eigen-solver of the Hueckel orbitals failed (no finite eigenvector) */
};

/* `step` of vmc_energy_forces: use the trajectory's own Langevin step counter. */
#define VMC_STEP_TRAJ 0xFFFFFFFFu

enum { VMC_FP64 = 0, VMC_MIXED = 1 };

/* Flags of vmc_langevin_step. */
#define VMC_STEP_CFOLD 1u       /* S = I: conventional first-order Langevin (main text, Eq. basic with S = I) */
#define VMC_STEP_NOISE_CORR 2u  /* lower T so that 2 T Db = 2 T_target Db - Dt^2 (SI, "Noise correction") */
#define VMC_STEP_NO_SCORR 4u    /* drop the S-difference term (SI, Eq. norogna); for tests only */

typedef struct vmc_ctx vmc_ctx;
typedef struct vmc_traj vmc_traj;

typedef struct {
  int n_protons;      /* N = number of protons = number of electrons; even */
  double box_L;       /* side of the periodic cube, bohr */
  double ewald_kappa; /* Ewald splitting parameter, 1/bohr (real space uses the minimum image) */
  int ewald_nmax;     /* reciprocal vectors k = 2 pi n / L with 0 < |n|^2 <= nmax^2, half space */
  double a_par;       /* Pade cusp parameter for parallel spins (1/4) */
  double a_anti;      /* Pade cusp parameter for anti-parallel spins (1/2) */
  double b;           /* Pade b (1); finite and >= 0, else VMC_EINVAL */
  int precision;      /* VMC_FP64: all FP64; VMC_MIXED: orbital, Jastrow and Ewald real-space
                         terms in FP32, determinant ratios, inverse refresh, reductions and
                         all accumulators FP64 */
  double refine_tol;  /* inverse refresh after the first sweep: one Newton-Schulz step
                         X <- X + X (I - A X) in FP64, and Gauss-Jordan elimination for
                         every matrix with max|I - A X| > refine_tol (or not finite).
                         0 = default (1e-7); < 0 = elimination for every matrix.
                         At N = 256 the step uses the walker's measurement scratch for I - A X */
  double j1_b1;       /* one-body electron-proton Jastrow term U_1 of the SI (Eq. e:j1), its
                         homogeneous part for Z = 1 on the sin-periodised distance rho:
                         -(2Z)^{3/4} u_1((2Z)^{1/4} rho), u_1(x) = (1 - e^{-b_1 x}) / (2 b_1), summed
                         over every electron-proton pair; it gives psi the electron-nucleus cusp.
                         j1_b1 = b_1 > 0 enables it; 0 = no one-body term; < 0 or NaN: VMC_EINVAL */
  int twist;          /* twisted boundary conditions of the orbitals (SI, basis section:
                         phi(r + n L) = e^{i theta.n} phi(r)) for the real twists: bit m set means
                         theta_m = pi (the orbitals change sign across the cell along axis m),
                         clear means theta_m = 0.  0..7; the Jastrow factor stays periodic.  C must
                         be the orbitals of the same twist (vmc_huckel_params_twist) */
  int general_twist;  /* 1: twisted boundary conditions with the angles theta below (SI, basis section;
                         the paper averages over a 4 x 4 x 4 Monkhorst-Pack mesh of them): each
                         Gaussian is the Bloch sum phi_a(r) = sum_n e^{-i theta.n} g_a(r - R_a + n L),
                         so phi(r + n L) = e^{i theta.n} phi(r); orbitals, Slater matrices and
                         determinants are complex, sampling follows |psi|^2 and the estimators take
                         the real part of E_L and of its proton derivative.  The one-body and
                         three-body Jastrow terms combine with it (their proton derivatives take the
                         real part of grad ln D), and so does the contracted basis (contracted = 1:
                         its three Cartesian factors Bloch-summed alike).  Requires precision
                         VMC_FP64, twist = 0 and N_sigma <= 64 (else VMC_EINVAL).  The
                         orbital coefficients C are then complex, N x N/2 (re, im) pairs of doubles
                         (vmc_huckel_params_theta, or vmc_huckel_params_theta_contracted on the
                         contracted basis); Binv holds complex inverses (twice the bytes).
                         Both spins use the same twist.  Not for the server (VMC_EINVAL).
                         0: real orbitals, twist as above */
  double theta[3];    /* twist angles per axis, radians (general_twist = 1 only; finite) */
  int contracted;     /* 1: the SI's contracted minimal basis (section "Systematic setup"): one
                         orbital per proton, phi_1 + eta phi_2 with phi_1 = e^{-Z1 r^2},
                         phi_2 = r^2 e^{-Z2 r^2}, Z1 = 0.6066825, Z2 = 0.3382168, image-summed like the
                         single Gaussian; zeta is then not used (but must still be a valid pointer).
                         C must come from vmc_huckel_params_contracted (with a general twist: from
                         vmc_huckel_params_theta_contracted).  Requires twist = 0 (the real twists
                         through general_twist), N_sigma <= 64 and a box with Z2 (1.5 L)^2 >= 36
                         (L >= 6.88 bohr: the images |n| <= 1 of the diffuse phi_2 then reach
                         FP64 resolution); not for the server.  Else VMC_EINVAL.
                         0: one s-Gaussian e^{-zeta_a r^2} per proton */
  double eta;         /* the contraction coefficient (contracted = 1; finite) */
  double j3_f[3];     /* the on-site three-body (electron-electron-nucleus) Jastrow term U_3 of the SI
                         (Jastrow section, Eq. e:j33): U_3 = sum_a sum_{i<j} chi_a(r_i)^T F chi_a(r_j)
                         with chi_1 = e^{-ZJ rho^2}, chi_2 = rho^2 e^{-ZJ rho^2}, ZJ = 0.7933844, on
                         the sin-periodised offset rho between electron and nucleus, and
                         F = [[f11, f12], [f12, f22]] = [[j3_f[0], j3_f[1]], [j3_f[1], j3_f[2]]] the same
                         for every nucleus.  All zero: no term.  The term requires N_sigma <= 64 (it
                         combines with the real and general twists, the contracted basis and the
                         one-body term), and is not for the server (else VMC_EINVAL); its orbitals are evaluated in the precision of
                         the Jastrow terms (FP32 in VMC_MIXED), their per-nucleus sums combined and
                         accumulated in FP64 */
  double j1_f[2];     /* the orbital part of the one-body Jastrow term U_1 of the SI (Jastrow section,
                         Eq. e:j1): sum_a sum_i (f_1 chi_1 + f_2 chi_2)(r_i - R_a) on the three-body
                         term's orbitals chi_1, chi_2, with (f_1, f_2) = (j1_f[0], j1_f[1]) the same for
                         every nucleus (finite).  Both zero: no such part.  Independent of j1_b1 (the
                         cusp part) and of j3_f, with the same scope as j3_f: N_sigma <= 64, not for the
                         server (else VMC_EINVAL), evaluated and accumulated like the three-body term */
} vmc_system;

/* ---------------------------------------------------------------- context -- */
/* Creates a context on HIP device `device`.  Allocates small device scratch. */
int vmc_create(vmc_ctx** out, int device);
void vmc_destroy(vmc_ctx* ctx);
/* HBM budget of the context's trajectories (bytes; 0 = no limit, the default): vmc_traj_create
 * returns VMC_ENOMEM when the device bytes of the context's live trajectories (vmc_traj_bytes)
 * would exceed it.  vmc_hbm_in_use: the bytes they hold now. */
int vmc_set_hbm_budget(vmc_ctx* ctx, size_t bytes);
int vmc_hbm_in_use(vmc_ctx* ctx, size_t* in_use);
/* Device bytes a trajectory of this system and walker count holds (0 if invalid). */
size_t vmc_traj_bytes(const vmc_system* sys, int n_walkers);
/* Asks the vmc_energy_forces call running on this context (or, if none runs, the next one)
 * to stop: it returns VMC_ECANCELLED within a few sweeps, with the trajectory as it was
 * before the call.  The only call that may be made from another thread. */
int vmc_cancel(vmc_ctx* ctx);
/* hip_stream: a hipStream_t (NULL = null stream).  Not owned. */
int vmc_set_stream(vmc_ctx* ctx, void* hip_stream);
const char* vmc_strerror(int code);
/* Whether N is supported: N = 2 N_sigma with N_sigma in {8, 12, 16, 20, 24, 27, 32, 64, 128}
 * (N = 16, 24, 32, 40, 48, 54, 64, 128, 256; each size is a compiled kernel variant).
 * Up to N_sigma = 64 a spin's inverse is held in one wavefront's registers during a
 * sweep; at 128 it stays in device memory. */
int vmc_supported_n(int n_protons);
/* Per-kernel timing with HIP events on the context stream (0 = off). */
int vmc_set_profiling(vmc_ctx* ctx, int on);
/* Fills up to max_n entries: kernel class names (static strings), total
 * milliseconds and launch counts since the last reset; returns the count. */
int vmc_kernel_times(vmc_ctx* ctx, const char** names, double* total_ms, long long* launches, int max_n);
int vmc_reset_kernel_times(vmc_ctx* ctx);

/* ------------------------------------------------------------- trajectory -- */
/* Device-resident state of one trajectory: W walkers (electron positions,
 * cached Slater matrices and inverses, accumulators), the per-walker force
 * means of the last vmc_energy_forces call, the RNG key (seed, traj_id) and the
 * Langevin state: proton positions R, the previous step's R and S (Eq. finaldyn_new
 * needs R(t - Delta) and S(R(t - Delta))), the last S and the step counter.
 * Allocates device memory (about W * (16 N^2 + 120 N) bytes + Ewald tables; at N = 256
 * also a per-walker region for the measurement's matrix products, 323 KiB in
 * mixed precision and 645 KiB in FP64). */
int vmc_traj_create(vmc_ctx* ctx, const vmc_system* sys, int n_walkers, uint32_t seed,
                    uint32_t traj_id, vmc_traj** out);
void vmc_traj_destroy(vmc_traj* traj);
/* Copies walker positions in/out (pos_dev: W x N x 3, any values; wrapped into
 * the box on input). */
int vmc_traj_set_walkers(vmc_traj* traj, const double* pos_dev);
int vmc_traj_get_walkers(vmc_traj* traj, double* pos_dev);
/* Proton positions R (3N, device) held by the trajectory.  vmc_traj_set_R starts a new
 * Langevin history (the next vmc_traj_langevin_step is a first step: R_prev = R, S_prev = S);
 * the step counter keeps counting.  vmc_traj_get_R: VMC_EINVAL before R was set. */
int vmc_traj_set_R(vmc_traj* traj, const double* R_dev);
int vmc_traj_get_R(vmc_traj* traj, double* R_dev);
/* Completed vmc_traj_langevin_step calls (the noise counter of the next step). */
int vmc_traj_step_count(vmc_traj* traj, uint32_t* steps);

/* a1-a7 (main text, Eq. for V(R) and f = -dV/dR; SI, alpha paragraph): VMC
 * estimate of the Born-Oppenheimer energy and ionic forces at proton positions
 * R_dev (3N) with MO coefficients C_dev (N x N/2, same for both spins) and
 * Gaussian exponents zeta_dev (N).  Each walker first refreshes its Slater
 * matrices at R, runs n_equil unmeasured sweeps, then n_sweeps measured sweeps:
 * a sweep moves electrons 0..N-1 in order by r' = r + step_delta (u - 1/2),
 * accepted iff u_acc < |psi'/psi|^2; Philox4x32-10 with key (seed, traj_id) and
 * counter (step, walker, sweep*N + e, 0|1).  The inverse of a spin's Slater
 * matrix is built by FP64 Gauss-Jordan elimination with partial pivoting before
 * the first half-sweep over that spin, refreshed before every later one (see
 * refine_tol) and carried through the N/2 moves of a half-sweep by Sherman-
 * Morrison updates applied in blocks of 16 moves (delayed, same ratios).
 * After each measured sweep: E_L, dE_L/dR and dln|psi|/dR.
 * With a general twist (vmc_system.general_twist) C_dev is complex; each half-sweep forms the
 * spin's Slater matrix afresh before the first sweep and every 4th one: at the first sweep it
 * inverts it (complex Gauss-Jordan elimination with partial pivoting), at the later ones it
 * refines the carried inverse by one Newton-Schulz step (elimination where max|I - A X| >
 * refine_tol, or for every matrix when refine_tol < 0); otherwise it carries the inverse of the
 * previous half-sweep; the moves update it by Sherman-Morrison steps applied in blocks of 16
 * moves (delayed, same ratios), the acceptance is
 * u_acc < |psi'/psi|^2 with complex ratios, and E_L, dE_L/dR in the outputs are the real parts.
 * Output out_dev (3 + 3N doubles): [E, sigma_E, acceptance, f(3N)] with
 * E = mean_w e_w, sigma_E = sd_w(e_w)/sqrt(W), f = mean_w f_w,
 * f_w = -(<dE_L/dR>_w + 2(<E_L dln|psi|/dR>_w - E <dln|psi|/dR>_w)).
 * Per-walker means stay on the device for vmc_build_S / vmc_traj_walker_*.
 * R_dev == NULL uses the trajectory's R (vmc_traj_set_R); step == VMC_STEP_TRAJ uses its
 * Langevin step counter.
 * Returns VMC_ESINGULAR if an inverse refresh hit an exactly zero pivot (e.g. two same-spin
 * electrons at one point), VMC_ECANCELLED after vmc_cancel, VMC_EINVAL if no walker has finite
 * coordinates; on every failure the walkers, accepted-move counts and the last call's means
 * are left as they were before the call and out_dev is not written. */
int vmc_energy_forces(vmc_traj* traj, const double* R_dev, const double* C_dev, const double* zeta_dev,
                      int n_equil, int n_sweeps, double step_delta, uint32_t step, double* out_dev);
/* Per-walker means of the last call: means_dev W x (1 + 9N) = [e_w, d_w(3N), g_w(3N), h_w(3N)]
 * with d = dE_L/dR, g = dln|psi|/dR, h = E_L dln|psi|/dR; f_w_dev W x 3N. */
int vmc_traj_walker_means(vmc_traj* traj, double* means_dev);
int vmc_traj_walker_forces(vmc_traj* traj, double* f_w_dev);
/* Accepted moves per walker in the last call (int64, W). */
int vmc_traj_accepts(vmc_traj* traj, int64_t* n_acc_dev);
/* Walker quarantine: at the start of every vmc_energy_forces call a walker with a non-finite
 * coordinate is replaced by a copy of the next walker (cyclically) whose coordinates are all
 * finite; if no walker is finite the call returns VMC_EINVAL and changes nothing.  *n_reset:
 * the number of walkers so replaced at the start of the last call. */
int vmc_traj_walkers_reset(vmc_traj* traj, int* n_reset);

/* ------------------------------------------------ wavefunction optimisation --
 * The main text re-optimises the wavefunction before every ionic step (n_opt optimisation steps
 * per step) and cites its optimiser; these calls give stochastic reconfiguration (SR; Sorella,
 * PRB 64, 024512 (2001)) on the Jastrow parameters p = (b, b_1, f_11, f_12, f_22, f_1, f_2): the
 * Pade b of the two-body term, b_1 of the one-body term's cusp part (Eq. e:j1), the three-body
 * matrix F (Eq. e:j33) and f of the one-body term's orbital part (Eq. e:j1).
 * O_k = d ln psi / d p_k: b: sum_{i<j} -a_ij rho^2 / (1 + b rho)^2; b_1: the derivative of the
 * one-body cusp part (0 without it); f_qr: sum_a sum_{i<j} chi_q(r_ia) chi_r(r_ja) (+ the
 * transposed product for q != r), formed for any F; f_q: sum_a sum_i chi_q(r_ia), for any f.  A loop of SR steps alternates vmc_energy_forces,
 * vmc_traj_param_stats, vmc_sr_update (host) and vmc_traj_set_jastrow. */
/* on = 1: every later vmc_energy_forces call also accumulates, per walker and in FP64, the
 * samples' [E_L, O (7), E_L O (7), O O^T (49)] (one more kernel per measured sweep); 0: off
 * (the default); with real or complex orbitals. */
int vmc_traj_set_param_stats(vmc_traj* traj, int on);
/* Means over the W walkers and M measured sweeps of the last vmc_energy_forces call made with the
 * statistics on, in a fixed summation order: stats_dev (device, 64 doubles) = [E, <O> (7),
 * <E_L O> (7), <O O^T> (7 x 7 row-major)].  VMC_EINVAL if there is no such call since the
 * statistics were switched on or the parameters changed. */
int vmc_traj_param_stats(vmc_traj* traj, double* stats_dev);
/* Sets the trajectory's Jastrow parameters for later calls (host values): the Pade b (>= 0), the
 * one-body b_1 (> 0 if the trajectory was created with the one-body cusp part, 0 if not), the
 * three-body F (j3_f[3]) and the one-body orbital part's f (j1_f[2]; NULL keeps the current f),
 * finite; F and f non-zero only if the trajectory was created with a non-zero F or f, whose
 * per-walker memory they need.  The walkers are kept; VMC_EINVAL on any violation, and then
 * nothing changes. */
int vmc_traj_set_jastrow(vmc_traj* traj, double b, double j1_b1, const double* j3_f, const double* j1_f);
/* Host helper: one SR step from the 64 means of vmc_traj_param_stats (host copy).  With
 * f_k = -2 (<E_L O_k> - E <O_k>) (minus the energy gradient) and S_kl = <O_k O_l> - <O_k><O_l>
 * over the parameters whose bit k is set in `active` (bit 0: b, 1: b_1, 2..4: f_11, f_12, f_22,
 * 5..6: f_1, f_2), S_kk scaled by (1 + eps): dp = tau S^-1 f on those parameters, 0 on the others
 * (dp: host, 7 doubles).  VMC_ENOTSPD if the regularised S is not positive definite (e.g. a
 * parameter whose O is zero on every sample); VMC_EINVAL on non-finite input, eps < 0 or bits
 * above 6. */
int vmc_sr_update(const double* stats, int active, double eps, double tau, double* dp);

/* Checkpoint / resume of the state a trajectory owns between calls: its system and walker
 * count (checked on load), the RNG key (seed, traj_id), the walker positions, and the per-walker
 * means, forces and accepted-move counts of the last vmc_energy_forces call.  The Slater rows,
 * inverses and Ewald tables are rebuilt by every vmc_energy_forces call and are not saved.  The
 * trajectory's Langevin state (R, R_prev, S, S_prev, the last estimate [E, sigma_E,
 * acceptance, f] and the step counter) is saved with it.  A trajectory loaded from a checkpoint
 * continues the saved run bit for bit (vmc_energy_forces with R_dev = NULL and step =
 * VMC_STEP_TRAJ, vmc_build_S, vmc_traj_langevin_step) with no state held by the caller but C
 * and zeta.  The checkpoint carries an FNV-1a checksum of its bytes.
 * vmc_traj_save: buf == NULL sets *len to the bytes needed; otherwise writes the checkpoint to
 * host memory buf of *len bytes (VMC_EINVAL, with *len set to the need, if it is too small);
 * waits for the trajectory's work on the context stream.
 * vmc_traj_load: reads a checkpoint of len bytes from host memory into a trajectory created with
 * the same system (N, box, precision, Ewald settings, cusp parameters, twist or general twist and
 * its angles, basis and eta, the one-body and three-body terms on or off) and walker count; the
 * Jastrow parameters b, j1_b1, j3_f and j1_f are taken from the checkpoint (as vmc_traj_set_jastrow sets
 * them, so an optimised wavefunction resumes).  Anything else, or a damaged buffer (checksum,
 * size, version), returns VMC_EINVAL and leaves the trajectory unchanged. */
int vmc_traj_save(vmc_traj* traj, void* buf, size_t* len);
int vmc_traj_load(vmc_traj* traj, const void* buf, size_t len);
/* Restart at another density (SI, systematic setup: configurations made at r_s* serve at any
 * r_s after scaling by s = r_s / r_s*).  vmc_traj_load_rescaled reads a checkpoint taken in a
 * box of side L* into a trajectory whose system differs from the checkpoint's at most in box_L
 * and ewald_kappa (N, walker count, precision, n_max, Jastrow, one-body term and twist must
 * match; VMC_EINVAL otherwise, or for a damaged buffer, with the trajectory unchanged).  Every
 * walker coordinate is multiplied by s = L / L* (L = this trajectory's box_L; at fixed N,
 * L is proportional to r_s), so walkers in [0, L*) land in [0, L).  The RNG key is the
 * checkpoint's.  The means, forces and acceptance counts belong to the old density and are
 * cleared: vmc_build_S and vmc_traj_walker_* return VMC_EINVAL until the next
 * vmc_energy_forces call.  The Langevin state is cleared too: the caller sets the proton
 * positions scaled by the same s (vmc_traj_set_R), and the next step is a first step. */
int vmc_traj_load_rescaled(vmc_traj* traj, const void* buf, size_t len);

/* a8 (main text, Eq. for Cov(f); SI, alpha paragraph): the acceleration matrix
 * S = Cov of the mean force = sum_w (f_w - f)(f_w - f)^T / (W (W - 1)) from the
 * trajectory's last vmc_energy_forces call, kept by the trajectory for
 * vmc_traj_langevin_step.  S_dev: 3N x 3N, or NULL (kept on the device only). */
int vmc_build_S(vmc_traj* traj, double* S_dev);
/* The same for caller-provided per-walker forces f_w_dev (W x n3) and their mean f_dev (n3). */
int vmc_build_S_raw(vmc_ctx* ctx, int W, int n3, const double* f_w_dev, const double* f_dev, double* S_dev);

/* a9-a10 (SI, Eq. finaldyn_new): one step of the adopted scheme
 *   R' = R + Dt S^-1 [ f - (S_prev - S)(R_prev - R)/(2 Db) ] + sqrt(2 T Db) z,
 *   <z z^T> = S^-1, Dt = (1 - e^{-alpha Delta})/alpha, Db = (1 - e^{-2 alpha Delta})/(2 alpha),
 * Dt = Db = Delta at alpha = 0 (Eq. finaldyn).  S = L L^T by FP64 Cholesky,
 * z = L^-T xi with xi standard normal from Philox4x32-10 (key (seed, traj_id),
 * counter (step, 0xFFFFFFFF, j, 0), Box-Muller pairs).  box_L > 0 wraps R'
 * into [0, box_L) and takes R_prev - R by minimum image.  R_dev, R_prev_dev
 * (n3) and S_prev_dev (n3 x n3) are updated in place ((R_prev, S_prev) <- (R, S));
 * on the first step pass R_prev = R and S_prev = S.  Units: T and Delta in
 * Hartree (S in Ha^2/bohr^2 makes alpha 1/Ha).  Returns VMC_ENOTSPD (state
 * unchanged) if S is not positive definite; VMC_EINVAL (state unchanged) if Delta <= 0,
 * alpha < 0, T < 0, the noise-corrected T is negative, or a position, the force, the
 * S-difference term or the noise is not finite. */
int vmc_langevin_step(vmc_ctx* ctx, int n3, double box_L, double* R_dev, double* R_prev_dev,
                      double* S_prev_dev, const double* f_dev, const double* S_dev, double T,
                      double Delta, double alpha, unsigned flags, uint32_t seed, uint32_t traj_id,
                      uint32_t step);
/* a9-a10 on the trajectory's own state: the same step with R, R_prev, S_prev, f (the last
 * vmc_energy_forces), S (the last vmc_build_S; not needed with VMC_STEP_CFOLD), box_L, the RNG
 * key (seed, traj_id) and the step counter held by the trajectory; on its first step (after
 * vmc_traj_set_R) R_prev = R and S_prev = S.  On success R moves, (R_prev, S_prev) <- (R, S) and
 * the counter advances; on failure (VMC_ENOTSPD, VMC_EINVAL) nothing changes.  VMC_EINVAL too if
 * R, the estimate or S is missing. */
int vmc_traj_langevin_step(vmc_traj* traj, double T, double Delta, double alpha, unsigned flags);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vmc_langevin_step with the same arguments, results
 * and status codes, but no allocation of any kind.  Its Cholesky work and status word live in a
 * static device array of the library (one per device, about 4.8 MB, held until the process
 * ends; its address is taken at vmc_create), so n3 <= 768 (the 256-proton box); a larger n3
 * returns VMC_EINVAL.  Every call on a device shares that device's array: calls that overlap on
 * one device (other threads, other contexts' streams) race and must not be issued. */
int vmc_langevin_step_noalloc(vmc_ctx* ctx, int n3, double box_L, double* R_dev, double* R_prev_dev,
                              double* S_prev_dev, const double* f_dev, const double* S_dev, double T,
                              double Delta, double alpha, unsigned flags, uint32_t seed, uint32_t traj_id,
                              uint32_t step);

/* The rotating-spring toy model (SI, "A simple toy model"; main text, figure of the toy
 * model): U = k (|x| - a)^2 / 2 in the plane; S = G_lambda (radial eigenvalue 1/lambda,
 * tangential 1; s_kind 0), S = H + mu G_lambda with H the Hessian of U (s_kind 1), S = I
 * (s_kind 2) or S = H + mu I (s_kind 3; the main text's shifted Hessian).
 * scheme 0: Eq. finaldyn_new (alpha = 0 is Eq. finaldyn); 1: Eq. norogna (no S-difference
 * term); 2: Eq. standard with gamma = 0 and the drift-diffusion term of Eq. e:cumber,
 * Gamma_j = sum_i d_i (S^-1)_ji, by central differences (h = 1e-6); 3: the SI's first
 * simplified scheme (Eq. smartMarkov), a noise step to y and the drift with the half
 * S-difference between y and R, S evaluated at both. */
typedef struct {
  double lambda, k, a, mu; /* G_lambda parameter, spring constant, ring radius, regulariser of H */
  int s_kind;              /* 0 G_lambda, 1 H + mu G_lambda, 2 identity, 3 H + mu I */
  double T, Delta, alpha;  /* temperature, time step, alpha of Eq. finaldyn_new (scheme 0) */
  int scheme;              /* 0 finaldyn_new, 1 norogna, 2 explicit Gamma, 3 smartMarkov (two S) */
} vmc_toy_params;

/* n_traj independent trajectories of n_steps steps, one GPU thread each.  R0_dev (n_traj x 2,
 * device, read) are the starting points; R_dev (n_traj x 2, device, written) the end points;
 * U_mean_dev (n_traj, device, written) the mean of U over the last 90% of the steps;
 * status_dev (n_traj ints, device, written) 0, or 3 if S stopped being positive definite (the
 * trajectory then stops there).  Trajectory i draws its step-t noise from the counter-based
 * generator with key (seed, i) and counter t, like vmc_langevin_step with traj_id i.
 * Asynchronous on the context stream; VMC_EINVAL for bad sizes or parameters. */
int vmc_toy_run(vmc_ctx* ctx, const vmc_toy_params* params, int n_traj, int n_steps, uint32_t seed,
                const double* R0_dev, double* R_dev, double* U_mean_dev, int* status_dev);

/* Per-configuration quantities for K fixed electron configurations pos_dev
 * (K x N x 3): out_dev K x (2 + 6N) = [ln|psi|, E_L, dln|psi|/dR (3N), dE_L/dR (3N)]
 * at protons R_dev with C_dev, zeta_dev (main text, Eq. for V(R)). */
int vmc_eval_configs(vmc_ctx* ctx, const vmc_system* sys, const double* R_dev, const double* C_dev,
                     const double* zeta_dev, int K, const double* pos_dev, double* out_dev);

/* a1 (host helper): Hueckel MO coefficients on the periodic s-Gaussians.
 * Overlap S_ab of the periodic Gaussians, H = -S_ab / sqrt(S_aa S_bb), its N/2
 * lowest eigenvectors v (Householder reduction to tridiagonal form, the N/2 lowest eigenvalues
 * by bisection, their eigenvectors by inverse iteration), C_ak = v_ak / sqrt(S_aa).
 * R, zeta: host (3N, N); C_out: host N x N/2.  VMC_EINVAL for a non-finite R or zeta <= 0,
 * VMC_ENOCONV if an eigenvector does not come out finite. */
int vmc_huckel_params(int n_protons, double box_L, const double* R, const double* zeta, double* C_out);
/* The same for the twisted basis (twist as in vmc_system): image n of the overlap sum carries
 * prod_m (+-1)^{n_m}.  twist = 0 is vmc_huckel_params; outside 0..7: VMC_EINVAL. */
int vmc_huckel_params_twist(int n_protons, double box_L, int twist, const double* R, const double* zeta,
                            double* C_out);

/* The same for the contracted basis (vmc_system.contracted, coefficient eta): the overlaps of
 * phi_1 + eta phi_2 are one image sum of free-space Gaussian overlaps and of their derivatives
 * with respect to the exponents (r^2 e^{-Z r^2} = -d/dZ e^{-Z r^2}).  C_out: host N x N/2.
 * VMC_EINVAL for a non-finite R or eta, VMC_ENOCONV if an eigenvector does not come out finite. */
int vmc_huckel_params_contracted(int n_protons, double box_L, double eta, const double* R, double* C_out);

/* The same for a general twist (vmc_system.general_twist): image n of the overlap sum carries
 * e^{-i theta.n}, S and H are Hermitian, and C_out receives N x N/2 complex coefficients as
 * (re, im) pairs of doubles (2 N * N/2 doubles).  The lowest N/2 eigenvectors of H are those of
 * the real symmetric 2N x 2N matrix [[Re H, -Im H], [Im H, Re H]] (each eigenvalue of H appears
 * twice there); the N/2 orthonormal complex vectors are taken from the lowest N of those by
 * Gram-Schmidt with column pivoting.  Any unitary mix of the occupied orbitals gives the same
 * |psi|, so C is defined up to one.  VMC_EINVAL for a non-finite R, theta or zeta <= 0,
 * VMC_ENOCONV if an eigenvector does not come out finite. */
int vmc_huckel_params_theta(int n_protons, double box_L, const double* theta, const double* R, const double* zeta,
                            double* C_out);
/* The same on the contracted basis (phi_1 + eta phi_2 per proton, the SI's exponents Z1, Z2):
 * the overlaps of vmc_huckel_params_contracted with each axis's image k weighted e^{-i theta k};
 * C_out: N x N/2 complex (re, im) pairs.  VMC_EINVAL for odd or too small N, L <= 0, non-finite
 * theta, eta or R; VMC_ENOCONV if an eigenvector does not come out finite. */
int vmc_huckel_params_theta_contracted(int n_protons, double box_L, const double* theta, double eta, const double* R,
                                       double* C_out);

/* Twist averaging (SI: the paper averages its estimates over a mesh of twists): n_tw
 * independent runs of one box, one per twist (each its own trajectory, orbitals and
 * walkers), give the force of the average f = (1/n_tw) sum_t f_t and, since the runs share no
 * samples, the covariance of that mean S = (1/n_tw^2) sum_t S_t.  f_stack_dev n_tw x n3 and
 * S_stack_dev n_tw x n3 x n3 (row-major) hold the runs' vmc_energy_forces forces and vmc_build_S
 * matrices; writes f_dev (n3) and S_dev (n3 x n3).  All device memory; n_tw >= 1. */
int vmc_twist_average(vmc_ctx* ctx, int n_tw, int n3, const double* f_stack_dev, const double* S_stack_dev,
                      double* f_dev, double* S_dev);

/* ---------------------------------------------------------------- serving --
 * Many independent trajectories (different N, r_s, T, walker counts) on one context,
 * with continuous batching: requests are admitted as HBM budget frees up, walker and
 * S state stay resident on the device between Langevin steps, and each tick runs
 * one sweep of every resident trajectory, trajectories of equal (N, precision,
 * Gaussian images, Ewald cut-off) sharing one launch per kernel.  A trajectory's
 * step is the same sequence as vmc_energy_forces (n_equil then n_sweeps sweeps),
 * vmc_build_S and vmc_langevin_step (S_prev = S and R_prev = R at its first step),
 * with C from vmc_huckel_params_twist (its system's twist) at its current R, so its results do not depend on
 * what else is being served.  Host pointers in a request are read during
 * vmc_server_submit only.  A server drives its context's stream; do not use the
 * context for anything else between ticks. */
typedef struct vmc_server vmc_server;

typedef struct {
  vmc_system sys;
  int n_walkers;        /* W >= 2 */
  int n_equil_first;    /* sweeps before the first measured sweep of the first step */
  int n_equil;          /* re-equilibration sweeps of every later step */
  int n_sweeps;         /* measured sweeps per step (M) */
  int n_steps;          /* Langevin steps to run */
  double step_delta;    /* electron move size */
  double T, Delta, alpha;   /* Langevin temperature (Ha), time step, alpha (vmc_langevin_step) */
  unsigned flags;       /* VMC_STEP_* */
  uint32_t seed, traj_id;
  const double* R0;     /* host, 3N initial proton positions */
  const double* zeta;   /* host, N Gaussian exponents */
  const double* pos0;   /* host, W x N x 3 initial electron positions */
} vmc_request;

enum { VMC_REQ_QUEUED = 0, VMC_REQ_RUNNING = 1, VMC_REQ_DONE = 2, VMC_REQ_FAILED = 3, VMC_REQ_CANCELLED = 4 };

/* Device bytes a request holds while resident (0 if the request is invalid). */
size_t vmc_request_bytes(const vmc_request* req);
/* Admission rule (host only): how many requests at the head of a queue with these
 * byte counts are admitted, first come first served, without overtaking. */
int vmc_server_admit_count(size_t budget, size_t resident, int n_queued, const size_t* bytes);
int vmc_server_create(vmc_ctx* ctx, size_t hbm_budget_bytes, vmc_server** out);
/* Waits for the context stream, then frees every trajectory and the server. */
void vmc_server_destroy(vmc_server* srv);
/* Queues a request (inputs copied).  VMC_EINVAL if invalid (including W <= 3N
 * without VMC_STEP_CFOLD: S of W walker means would be singular), VMC_ENOMEM if it
 * can never fit the budget.  *id_out identifies it in the calls below. */
int vmc_server_submit(vmc_server* srv, const vmc_request* req, int* id_out);
/* Removes a queued request, or stops a running one and frees its memory (waits for
 * the stream); its state becomes VMC_REQ_CANCELLED with error VMC_ECANCELLED. */
int vmc_server_cancel(vmc_server* srv, int id);
/* Collects finished steps, admits, sets up the trajectories that start a step and
 * queues sweeps of every resident trajectory (returns without waiting for them):
 * one per tick for the bucket with the most work per sweep (sum of W N^2), up to 32
 * for lighter buckets, in proportion. */
int vmc_server_tick(vmc_server* srv, int* n_active, int* n_queued);
/* state: VMC_REQ_*; error: the VMC_E* code of a failed request (singular matrix,
 * S not positive definite, a non-finite R at the start of a step, the host eigen-solver, ...);
 * a failure affects that request only: vmc_server_tick returns an error only for HIP errors. */
int vmc_server_status(vmc_server* srv, int id, int* state, int* steps_done, int* error);
/* Host outputs (any may be NULL): R after the completed steps (3N), E and sigma_E
 * of every completed step, each step's latency in ms (from the step becoming
 * runnable: admission or the previous step's end, to its result being on the host),
 * and the queue wait (submit to admission, ms; -1 while queued). */
int vmc_server_result(vmc_server* srv, int id, double* R_out, double* E_out, double* sigma_out, double* latency_ms,
                      double* wait_ms);
int vmc_server_info(vmc_server* srv, size_t* resident, size_t* peak_resident, int* n_active, int* n_queued,
                    long long* ticks);

#ifdef __cplusplus
}
#endif
#endif
