// Kernel argument blocks and launchers (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmc {

struct WalkerArgs {
  int W, N, NS;
  int nimg;            // 1: images n = -1, 0, 1 of each Gaussian; 0: n = 0 only
  double L, invL;
  const double* R;     // 3N proton positions
  const double* zeta;  // N Gaussian exponents
  const double* C;     // N x NS MO coefficients
  double a_par, a_anti, b;
  double j1_beta;      // one-body Jastrow f(rho) = -(1 - e^{-beta rho}) / beta per electron-proton pair; 0 = none
  int twist;           // bit m: twist angle pi along axis m (the orbitals change sign across the cell)
  double* pos;         // W x N x 3
  double* Amat;        // W x 2 x NS x NS
  double* Binv;        // W x 2 x NS x NS
  double* ldet;        // W x 2
  double* sgn;         // W x 2
  int* status;         // set to 1 on a zero pivot
  int64_t* nacc;       // W accepted moves
  int* rflag;          // W x 2: 1 = the refinement step left a large residual, redo by elimination
  double* rscr;        // N_sigma > 64: per-walker scratch of the refinement (N_sigma^2 doubles at rscr_stride)
  size_t rscr_stride;
  int contracted;      // 1: the contracted orbital phi_1 + eta phi_2 per proton (zeta unused)
  double eta;
  int j3;              // 1: the Jastrow-orbital terms are on: the on-site three-body term with the
                       // matrix j3f = (f11, f12, f22) and/or the one-body orbital part with j1f
  double j3f[3];
  double j1f[2];       // (f_1, f_2) of the one-body term's orbital part, f^T chi_a(r_i) per pair
  double* j3G;         // W x N x 2: per walker and nucleus, G_a = sum over electrons of (chi_1, chi_2)
};

struct SweepArgs {
  int spin;        // 0 = up (electrons 0..NS-1), 1 = down
  int sweep;       // sweep index within the call (equilibration sweeps included)
  uint32_t step, seed, traj;
  double delta;    // box-move size
};

// Ewald tables of one box, built at a new R (walker independent).
struct EwaldArgs {
  int nk;              // half-space k vectors
  int nslot;           // (ny, nz) slots, k vectors grouped by slot, nx innermost
  int nmax;
  double kappa;
  const double* kvec;  // nk x 4: kx, ky, kz, W_k = (4 pi / V) e^{-k^2/(4 kappa^2)} / k^2
  const int* slot;     // nslot x 4: ny, nz, first k index, count (nx from nx0 = first nx)
  const int* slot_nx0; // nslot: first nx of the slot
  const double* rho_p; // nk x 2: proton structure factor sum_b e^{i k R_b}
  const double* Ptab;  // nk x N x 2: e^{i k R_b}
  const double* Vpp;   // device: proton-proton real-space energy (k_proton_const)
  double Vself;        // self energy of all 2N charges, -kappa/sqrt(pi) * 2N
  const double* Fconst;// 3N: walker-independent part of dV/dR (p-p real space + rho_p part of reciprocal)
};

struct MeasureArgs {
  int W, N, NS;
  int nimg;
  double L, invL;
  const double* R;
  const double* zeta;
  const double* C;
  double a_par, a_anti, b;
  double j1_beta;       // as in WalkerArgs
  int twist;            // as in WalkerArgs
  const double* pos;    // W x N x 3
  const double* Binv;   // W x 2 x NS x NS
  double* Vs;           // W  per-sample potential energy
  double* dVs;          // W x 3N per-sample real-space e-p gradient
  double* Uj;           // W  Jastrow exponent U of the sample
  double* acc;          // W x (2 + 9N): sum E_L, sum E_L^2, sum dE_L/dR, sum dlnpsi/dR, sum E_L dlnpsi/dR
  double* rho_acc;      // W x nk x 2: sum of the electron structure factor
  unsigned char* scr;   // W x slater_scratch_bytes(NS, mixed): matrix products that do not fit in LDS
  int contracted;       // as in WalkerArgs
  double eta;
  int j3;               // as in WalkerArgs
  double j3f[3];
  double j1f[2];
  double* j3scr;        // W x j3_measure_doubles(N): the term's per-electron gradient, Laplacian and U_3,
                        // then the full grad U, grad ln|D| and E_L of the sample (written by the Slater pass)
  double* ELs;          // W: E_L of the sample, written by the Slater pass when not null
  double* popt;         // W x kOptStats: the walker's parameter sums (k_opt_sample)
};

// Several trajectories of one bucket (N, precision, Gaussian images, Ewald cut-off)
// in one grid: blocks [off[j], off[j+1]) belong to jobs[j], with the kernel's usual
// block-to-walker map inside each range.  jobs == nullptr: the launch serves the
// trajectory passed by value.  Per-launch values (spin, fallback mode) stay those
// passed by value.
struct TrajJob {
  WalkerArgs a;
  SweepArgs s;
  MeasureArgs m;
  EwaldArgs e;
  double tol;
};
struct Batch {
  const TrajJob* jobs;
  const int* off;     // njobs + 1 block offsets
  int njobs;
};
__device__ __forceinline__ int batch_job(const Batch& b, int blk) {
  int lo = 0, hi = b.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.off[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

hipError_t launch_build_A(const WalkerArgs& a, int mixed, hipStream_t st);
// Walkers with non-finite coordinates take a copy of the next finite walker (flags: W ints;
// count: 2 ints, copies made and bad walkers without a source, both added to).
hipError_t launch_walker_quarantine(int W, int N, double* pos, int* flags, int* count, hipStream_t st);
hipError_t launch_invert(const WalkerArgs& a, int spin_lo, int spin_hi, int only_flagged, hipStream_t st,
                         const Batch* bt = nullptr, int nblk = 0);
hipError_t launch_refine(const WalkerArgs& a, int spin, double tol, hipStream_t st, const Batch* bt = nullptr,
                         int nblk = 0);
// Blocks of the refresh launch: two waves per matrix and two matrices per block where a matrix has
// an even number (>= 2) of 16-wide column tiles, four one-wave matrices per block otherwise, one
// block per matrix for N_sigma > 64.
constexpr bool refine_pairs(int NS) { return NS <= 64 && (NS + 15) / 16 >= 2 && ((NS + 15) / 16) % 2 == 0; }
constexpr int refine_blocks(int NS, int W) { return NS > 64 ? W : refine_pairs(NS) ? (W + 1) / 2 : (W + 3) / 4; }
hipError_t launch_sweep(const WalkerArgs& a, const SweepArgs& s, int mixed, hipStream_t st, const Batch* bt = nullptr,
                        int nblk = 0);

hipError_t launch_ewald_sample(const MeasureArgs& m, const EwaldArgs& e, int mixed, hipStream_t st,
                               const Batch* bt = nullptr, int nblk = 0);
// Per-walker device scratch of the measurement kernel (0 where everything fits in LDS).
size_t slater_scratch_bytes(int NS, int mixed);
hipError_t launch_slater_sample(const MeasureArgs& m, int mixed, hipStream_t st, const Batch* bt = nullptr,
                                int nblk = 0);
hipError_t launch_finalize(const MeasureArgs& m, const EwaldArgs& e, int M, double* means, hipStream_t st);
hipError_t launch_proton_setup(int N, double L, const double* R, EwaldArgs& e, double* rho_p, double* Ptab,
                               double* Fconst, double* Vpp, hipStream_t st);

hipError_t launch_reduce(int W, int n3, const double* means, const int64_t* nacc, double moves_per_walker,
                         double* f_w, double* partial, double* out, hipStream_t st);
hipError_t launch_syrk(int W, int n3, const double* f_w, const double* f, double* partial, double* S,
                       hipStream_t st);
hipError_t launch_langevin(int n3, double L, double* R, double* R_prev, double* S_prev, const double* f,
                           const double* S, double* Lwork, double* vwork, double T, double Delta, double alpha,
                           unsigned flags, uint32_t seed, uint32_t traj, uint32_t step, int* status,
                           hipStream_t st);
// Work of one Langevin step: Lwork needs langevin_work_doubles(n3) doubles.
size_t langevin_work_doubles(int n3);
// The per-device static scratch of the allocation-free Langevin step: largest 3N, its address on
// the current device (hipGetSymbolAddress) and the offset (doubles) of its status word.
int langevin_noalloc_max();
hipError_t langevin_scratch_address(double** ptr);
size_t langevin_scratch_status_offset();
size_t syrk_partial_doubles(int W, int n3);
size_t reduce_partial_doubles(int W, int n3);
// Independent toy-model trajectories (the rotating spring of the SI), one thread each.
hipError_t launch_toy(double lambda, double k, double a, double mu, int s_kind, double T, double Delta,
                      double alpha, int scheme, uint32_t seed, int n_traj, int n_steps, const double* R0,
                      double* Rout, double* Umean, int* status, hipStream_t st);
// f = mean of the n_tw rows of f_stack, S = sum of the n_tw matrices of S_stack / n_tw^2.
hipError_t launch_twist_average(int n_tw, int n3, const double* f_stack, const double* S_stack, double* f, double* S,
                                hipStream_t st);
// The on-site three-body Jastrow term: G_a of every walker from its positions (before the sweeps),
// and the measurement's two passes around the Slater pass (its gradient, Laplacian and U_3 before;
// its d/dR terms after, from the full grad U, grad ln|D| and E_L the Slater pass leaves).
constexpr size_t j3_measure_doubles(int N) { return (size_t)10 * N + 2; }
hipError_t launch_j3_init(const WalkerArgs& a, hipStream_t st);
// Wavefunction optimisation: per walker [sum E_L, sum O (P), sum E_L O (P), sum O O^T (P x P)] of the
// logarithmic derivatives O of the P = 7 Jastrow parameters (b, b_1, f_11, f_12, f_22, f_1, f_2),
// and their means.
constexpr int kOptPar = 7;
constexpr int kOptStats = 1 + 2 * kOptPar + kOptPar * kOptPar;
hipError_t launch_opt_sample(const MeasureArgs& m, int mixed, hipStream_t st);
hipError_t launch_opt_reduce(int W, int M, const double* popt, double* out, hipStream_t st);
hipError_t launch_j3_grad(const MeasureArgs& m, int mixed, hipStream_t st);
hipError_t launch_j3_forces(const MeasureArgs& m, int mixed, hipStream_t st);

// General twist angles (radians) per axis with their cosines and sines: the complex path.
struct TwistArgs {
  double th[3], c[3], s[3];
};
// Complex path (FP64, N_sigma <= 64): one work-group per walker for spin s.spin.  refresh 1: form the
// spin's Slater matrix at the current positions and invert it; refresh 2: form it and refine the
// inverse read from Binv by one Newton-Schulz step, inverting afresh where max |I - A X| > rtol;
// refresh 0: read the inverse from Binv.  moves: then move the spin's electrons once.  Binv holds
// complex (A^-1)[k][i], ldet ln|det A|, sgn arg det A.  A zero pivot sets *status and leaves the
// walker unchanged.
hipError_t launch_csweep(const WalkerArgs& a, const SweepArgs& s, const TwistArgs& tw, int refresh, int moves,
                         double rtol, hipStream_t st);
// The complex measurement (same accumulator layout as the real one) and its per-walker scratch.
size_t cslater_scratch_bytes(int NS);
hipError_t launch_cslater_sample(const MeasureArgs& m, const TwistArgs& tw, hipStream_t st);
hipError_t launch_pack_eval(int K, int N, const double* means, const double* ldet, const double* Uj, double* out,
                            hipStream_t st);

}  // namespace vmc
