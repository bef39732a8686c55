// Walker kernels: Slater matrices at new proton positions (a2), the FP64 inverse
// refresh (a4) and the Metropolis half-sweep with delayed Sherman-Morrison
// updates (a3).
//
// Layout in HBM (per trajectory, W walkers, N electrons, NS = N/2 per spin):
//   pos  [W][N][3]            electron positions, wrapped into [0, L)
//   Amat [W][2][NS][NS]       Slater matrix rows A[i][k] = sum_a phi_a(r_i) C[a][k]
//   Binv [W][2][NS][NS]       inverse, row-major (A^-1)[k][i]
//   ldet [W][2], sgn[W][2]    ln|det A| and sign at the last refresh
// A wavefront (64 lanes) owns one walker in the sweep: the active spin's inverse
// stays in matrix-core accumulator registers, lanes own electrons j, j+64, ...;
// the MO coefficients C are read through the caches.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "moves.hpp"

namespace vmc {

// phi_a(r); tw: bit m set = twist angle pi along axis m (real twisted boundary conditions)
template <class Real, int NIMG, bool TW>
__device__ __forceinline__ Real phi_value(double rx, double ry, double rz, const double* Ra, Real zeta,
                                          double L, double invL, int tw) {
  Real g[3][4];
  basis_axis<Real, 0, NIMG, TW>(rx - Ra[0], zeta, L, invL, tw & 1, g[0]);
  basis_axis<Real, 0, NIMG, TW>(ry - Ra[1], zeta, L, invL, (tw >> 1) & 1, g[1]);
  basis_axis<Real, 0, NIMG, TW>(rz - Ra[2], zeta, L, invL, (tw >> 2) & 1, g[2]);
  return g[0][0] * g[1][0] * g[2][0];
}

// --------------------------------------------------------------- build A ---
// One wave per walker; electrons in order, lanes over centres then orbitals.
template <int NS, class Real, int NIMG, bool TW, bool CB = false>
__global__ __launch_bounds__(256) void k_build_A(WalkerArgs a) {
  constexpr int N = 2 * NS;
  constexpr int WPB = 4;
  __shared__ Real phi_s[WPB][N];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = blockIdx.x * WPB + wv;
  if (w >= a.W) return;
  const double* p = a.pos + (size_t)w * N * 3;
  for (int e = 0; e < N; ++e) {
    double rx = p[3 * e], ry = p[3 * e + 1], rz = p[3 * e + 2];
    for (int c = lane; c < N; c += 64)
      phi_s[wv][c] = CB ? contracted_value<Real, NIMG>(rx, ry, rz, a.R + 3 * c, (Real)a.eta, a.L, a.invL)
                        : phi_value<Real, NIMG, TW>(rx, ry, rz, a.R + 3 * c, (Real)a.zeta[c], a.L, a.invL, a.twist);
    wave_lds_sync();
    for (int k = lane; k < NS; k += 64) {
      double m = 0.0;
      for (int c = 0; c < N; ++c) m += (double)phi_s[wv][c] * a.C[c * NS + k];
      int sp = e / NS, i = e % NS;
      a.Amat[(((size_t)w * 2 + sp) * NS + i) * NS + k] = m;
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------------- inverse refresh ---
// Gauss-Jordan inversion with partial pivoting, one wave per matrix, entirely
// in registers: lane i holds row i of A.  Pivoting is implicit (the pivot row
// of column p is the unused row with the largest |A[i][p]|, ties to the lowest
// row); the pivot row is broadcast by readlane and every other row is updated
// with one FMA per column.  The in-place inverse ends with rows and columns
// permuted: the row that pivoted column k holds row k of A^-1 with column c
// stored at position pi(c).  ln|det A| = sum ln|pivot|, sign from the pivots
// and the parity of pi.  A zero pivot sets *status = 1.
template <int NS, bool BATCH>
__global__ __launch_bounds__(256) void k_invert(WalkerArgs a, int spin_lo, int spin_hi, int only_flagged, Batch bt) {
  constexpr int BC = 16, NB = (NS + BC - 1) / BC;
  __shared__ double stage[4 * NS * 17];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    a = bt.jobs[j].a;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  const int blk = BATCH ? bblk : (int)blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nsp = spin_hi - spin_lo;
  const int mat = blk * 4 + wv;
  const int w = mat / nsp, sp = spin_lo + mat % nsp;
  if (w >= a.W) return;
  if (only_flagged) {
    if (a.rflag[(size_t)w * 2 + sp] == 0) return;
    if (lane == 0) a.rflag[(size_t)w * 2 + sp] = 0;
  }
  const size_t base = ((size_t)w * 2 + sp) * NS * NS;
  const bool isrow = lane < NS;
  double r[NB][BC];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int j = 0; j < BC; ++j) {
      const int c = b * BC + j;
      r[b][j] = (isrow && c < NS) ? a.Amat[base + (size_t)lane * NS + c] : 0.0;
    }
  bool used = !isrow;
  int myk = 0, mypi = 0;
  double logdet = 0.0, sgn = 1.0;
  bool singular = false;
#pragma unroll
  for (int pb = 0; pb < NB; ++pb) {
    const int qmax = (NS - pb * BC) < BC ? (NS - pb * BC) : BC;
    for (int q = 0; q < qmax; ++q) {
      const int p = pb * BC + q;
      double rp = r[pb][0];
#pragma unroll
      for (int j = 1; j < BC; ++j) rp = (j == q) ? r[pb][j] : rp;
      double bv = used ? -1.0 : fabs(rp);
      int bi = lane;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      const int piv = __builtin_amdgcn_readfirstlane(bi);
      const double pv = readlane_d(rp, piv);
      if (pv == 0.0) { singular = true; break; }
      logdet += log(fabs(pv));
      if (pv < 0.0) sgn = -sgn;
      const bool me = lane == piv;
      if (me) { used = true; myk = p; }
      if (lane == p) mypi = piv;
      // multiplier by division, not by the reciprocal: a row equal to the pivot row gets g = 1
      // exactly and becomes exactly zero, so an exactly singular matrix (two same-spin electrons
      // at one point) meets an exactly zero pivot
      const double g = (me ? (pv - 1.0) : rp) / pv;
      const double diag = (me ? 1.0 : 0.0) - g;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          if (b * BC + j >= NS) continue;
          const double pc = readlane_d(r[b][j], piv);
          const double upd = fma(-g, pc, r[b][j]);
          r[b][j] = (b == pb && j == q) ? diag : upd;
        }
    }
    if (singular) break;
  }
  if (singular) {
    if (lane == 0) {
      *a.status = 1;
      a.ldet[(size_t)w * 2 + sp] = -INFINITY;
      a.sgn[(size_t)w * 2 + sp] = 0.0;
    }
    return;
  }
  // parity of pi: lane p counts q > p with pi(q) < pi(p)
  int inv_cnt = 0;
  for (int q = 0; q < NS; ++q) {
    const int pq = __builtin_amdgcn_readlane(mypi, q);
    if (isrow && q > lane && pq < mypi) ++inv_cnt;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) inv_cnt += __shfl_xor(inv_cnt, off, 64);
  if (inv_cnt & 1) sgn = -sgn;
  // Lane myk's row of A^-1 has column pi(c) in r[c].  Stage 16 columns at a time in
  // LDS (row stride 17) and write whole row segments, so stores are coalesced.
  constexpr int CH = 16, NCH = (NS + CH - 1) / CH;
  double* st = stage + (size_t)wv * NS * (CH + 1);
  for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int j = 0; j < BC; ++j) {
        const int c = b * BC + j;
        if (c >= NS) continue;
        const int col = __builtin_amdgcn_readlane(mypi, c);
        if (col / CH == ch && isrow) st[myk * (CH + 1) + col % CH] = r[b][j];
      }
    wave_lds_sync();
    const int ncol = (NS - ch * CH) < CH ? (NS - ch * CH) : CH;
    for (int idx = lane; idx < NS * CH; idx += 64) {
      const int row = idx / CH, cc = idx % CH;
      if (cc < ncol) a.Binv[base + (size_t)row * NS + ch * CH + cc] = st[row * (CH + 1) + cc];
    }
    wave_lds_sync();
  }
  if (lane == 0) {
    a.ldet[(size_t)w * 2 + sp] = logdet;
    a.sgn[(size_t)w * 2 + sp] = sgn;
  }
}

// Gauss-Jordan for NS = 128: one 256-thread work-group per matrix, registers
// resident.  Thread (h, r) = (t / 128, t % 128) holds row r, columns 64 h .. 64 h + 63,
// in 4 blocks of 16.  The same implicit-pivot elimination as k_invert (pivot of
// column p: the unused row with the largest |A[i][p]|, ties to the lowest row) and
// the same output: row r, which pivoted column myk(r), holds row myk(r) of A^-1 with
// column c at pi(c).  Each step: the two waves that hold column p propose their best
// row; every thread takes the same pivot from LDS; the pivot row (column p set to 1)
// and the multipliers g_i go through LDS; then M[i][j] -= g_i prow[j] everywhere,
// with column p first set to e_piv so that the rank-1 step also forms the new column.
template <int NS, bool BATCH>
__global__ __launch_bounds__(256, 2) void k_invert_big(WalkerArgs a, int spin_lo, int spin_hi, int only_flagged,
                                                       Batch bt) {
  static_assert(NS == 128, "two column halves of 64 per row");
  constexpr int HALF = NS / 2, BC = 16, NBL = HALF / BC;
  __shared__ __align__(16) double prow[NS];
  __shared__ double gcol[NS];
  __shared__ double cand_v[2], cand_s[2];
  __shared__ int cand_i[2];
  __shared__ int pi_s[NS];
  __shared__ double pv_s[NS];
  __shared__ int wv_cnt[4];
  __shared__ double wv_ld[4];
  int blk = blockIdx.x;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blk);
    a = bt.jobs[j].a;
    blk -= bt.off[j];
  }
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int h = t >> 7, r = t & (NS - 1);
  const int nsp = spin_hi - spin_lo;
  const int w = blk / nsp, sp = spin_lo + blk % nsp;
  if (w >= a.W) return;
  if (only_flagged) {
    const int fl = a.rflag[(size_t)w * 2 + sp];
    __syncthreads();
    if (fl == 0) return;
    if (t == 0) a.rflag[(size_t)w * 2 + sp] = 0;
  }
  const size_t base = ((size_t)w * 2 + sp) * NS * NS;
  double x[NBL][BC];
  {
    const double* src = a.Amat + base + (size_t)r * NS + HALF * h;
#pragma unroll
    for (int b = 0; b < NBL; ++b)
#pragma unroll
      for (int j = 0; j < BC; ++j) x[b][j] = src[b * BC + j];
  }
  bool used = false;
  int myk = 0;
  bool singular = false;
#pragma unroll
  for (int pb = 0; pb < 2 * NBL; ++pb) {
    const int ph = pb / NBL, lb = pb % NBL;   // column half and block of the pivot columns
    for (int q = 0; q < BC; ++q) {
      const int p = pb * BC + q;
      // column p of this thread's row (meaningful where h == ph)
      double rp = x[lb][0];
#pragma unroll
      for (int j = 1; j < BC; ++j) rp = (j == q) ? x[lb][j] : rp;
      if (h == ph) {                                    // wave-uniform
        double bv = used ? -1.0 : fabs(rp);
        int bi = r;
        wave_argmax(bv, bi);
        const int wr = __builtin_amdgcn_readfirstlane(bi);
        const double sv = readlane_d(rp, wr & 63);
        if (lane == 0) {
          cand_v[wave & 1] = bv;
          cand_i[wave & 1] = wr;
          cand_s[wave & 1] = sv;
        }
      }
      __syncthreads();
      const int hi = cand_v[1] > cand_v[0] ? 1 : 0;   // ties to the lower rows
      const int piv = cand_i[hi];
      const double pv = cand_s[hi];
      if (pv == 0.0) { singular = true; break; }      // uniform
      const bool me = r == piv;
      if (me) { used = true; myk = p; }
      if (h == 0 && r == p) { pi_s[p] = piv; pv_s[p] = pv; }
      if (h == ph) {
        gcol[r] = (me ? (pv - 1.0) : rp) / pv;        // by division: equal rows cancel exactly
        const double dv = me ? 1.0 : 0.0;
#pragma unroll
        for (int j = 0; j < BC; ++j) x[lb][j] = (j == q) ? dv : x[lb][j];
      }
      if (me) {
        double2* pw2 = reinterpret_cast<double2*>(prow + HALF * h);
#pragma unroll
        for (int b = 0; b < NBL; ++b)
#pragma unroll
          for (int j = 0; j < BC; j += 2) pw2[(b * BC + j) / 2] = make_double2(x[b][j], x[b][j + 1]);
      }
      __syncthreads();
      const double g = gcol[r];
      const double2* pr2 = reinterpret_cast<const double2*>(prow + HALF * h);
#pragma unroll
      for (int b = 0; b < NBL; ++b)
#pragma unroll
        for (int j = 0; j < BC; j += 2) {
          const double2 pv2 = pr2[(b * BC + j) / 2];
          x[b][j] = fma(-g, pv2.x, x[b][j]);
          x[b][j + 1] = fma(-g, pv2.y, x[b][j + 1]);
        }
    }
    if (singular) break;
  }
  if (singular) {
    if (t == 0) {
      *a.status = 1;
      a.ldet[(size_t)w * 2 + sp] = -INFINITY;
      a.sgn[(size_t)w * 2 + sp] = 0.0;
    }
    return;
  }
  __syncthreads();
  // parity of pi (thread r < NS counts q > r with pi(q) < pi(r)), the signs and the
  // logarithms of the pivots, summed over the waves in a fixed order
  int inv_cnt = 0;
  double lsum = 0.0;
  if (h == 0) {
    const int mine = pi_s[r];
    for (int q = r + 1; q < NS; ++q) inv_cnt += pi_s[q] < mine ? 1 : 0;
    inv_cnt += pv_s[r] < 0.0 ? 1 : 0;
    lsum = log(fabs(pv_s[r]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    inv_cnt += __shfl_xor(inv_cnt, off, 64);
    lsum += __shfl_xor(lsum, off, 64);
  }
  if (lane == 0) { wv_cnt[wave] = inv_cnt; wv_ld[wave] = lsum; }
  // row myk of A^-1: column pi(c) from x at c (pi(c) is the same for every lane of a wave)
  double* dst = a.Binv + base + (size_t)myk * NS;
#pragma unroll
  for (int b = 0; b < NBL; ++b)
#pragma unroll
    for (int j = 0; j < BC; ++j) dst[pi_s[HALF * h + b * BC + j]] = x[b][j];
  __syncthreads();
  if (t == 0) {
    a.ldet[(size_t)w * 2 + sp] = (wv_ld[0] + wv_ld[1]) + (wv_ld[2] + wv_ld[3]);
    a.sgn[(size_t)w * 2 + sp] = ((wv_cnt[0] + wv_cnt[1] + wv_cnt[2] + wv_cnt[3]) & 1) ? -1.0 : 1.0;
  }
}

// ---------------------------------------------------------- half sweep ---
template <class T, int E>
__device__ __forceinline__ T pick(const T (&v)[E], int s) {
  T r = v[0];
#pragma unroll
  for (int t = 1; t < E; ++t) r = (s == t) ? v[t] : r;
  return r;
}

// Column c (wave-uniform) of a vector spread as element c / 64 of lane c % 64.
template <int E>
__device__ __forceinline__ double colread(const double (&v)[E], int c) {
  return readlane_d(pick(v, c >> 6), c & 63);
}

typedef double d4w_t __attribute__((ext_vector_type(4)));
// 16x16x4 FP64 matrix-core step D += A B: lane l gives A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16] in element v.
__device__ __forceinline__ d4w_t mfma_w(double av, double bv, d4w_t acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
}

// LDS per wave of the half-sweep (doubles): M' block (16 x LDM), later reused for
// the 16 inverse columns G (NSP x 17), and the P / Z block (16 x LDM).
template <int NS>
struct SweepLds {
  static constexpr int NSP = (NS + 15) / 16 * 16, LDM = NSP + 1, LDG = 17;
  static constexpr int MB = (16 * LDM > NSP * LDG) ? 16 * LDM : NSP * LDG;
  static constexpr int WAVE = MB + 16 * LDM;
  static constexpr size_t bytes(int N) { return ((size_t)4 * WAVE + 4 * (size_t)N) * sizeof(double); }
};
// With the one-body Jastrow term the sweeps keep sin and cos of pi R / L of every proton
// (6 x N values of the Jastrow precision) after the centre table, then per wave the moves'
// one-body changes in FP64 (k_sweep_half: all N_sigma of the half-sweep; k_sweep_big: the
// 16 of the current block).
template <class Real>
constexpr size_t one_body_table_bytes(int N, int per_wave) {
  return (size_t)6 * N * sizeof(Real) + (size_t)4 * per_wave * sizeof(double);
}

// Change of the one-body Jastrow term, sum over protons c of
// [-(1 - e^{-beta rho_new}) + (1 - e^{-beta rho_old})] / beta, for the proposal held by the
// lanes with this l16: quarter l4 takes the protons c = l4 mod 4 and the quarters are
// combined by lane exchanges, so the four lanes of a proposal hold the same total.
template <class Real, int N>
__device__ __forceinline__ double one_body_change(const Real* Rt, double xo, double yo, double zo, double xn,
                                                  double yn, double zn, double invL, Real LoverPi, Real beta,
                                                  int l4) {
  Real so[3], co[3], sn[3], cn[3];
  dev_sincospi<Real>((Real)(xo * invL), &so[0], &co[0]);
  dev_sincospi<Real>((Real)(yo * invL), &so[1], &co[1]);
  dev_sincospi<Real>((Real)(zo * invL), &so[2], &co[2]);
  dev_sincospi<Real>((Real)(xn * invL), &sn[0], &cn[0]);
  dev_sincospi<Real>((Real)(yn * invL), &sn[1], &cn[1]);
  dev_sincospi<Real>((Real)(zn * invL), &sn[2], &cn[2]);
  Real acc = Real(0);
#pragma unroll 2
  for (int c = l4; c < N; c += 4) {
    const Real sr[3] = {Rt[c], Rt[N + c], Rt[2 * N + c]};
    const Real cr[3] = {Rt[3 * N + c], Rt[4 * N + c], Rt[5 * N + c]};
    acc += one_body_exp<Real>(sn, cn, sr, cr, LoverPi, beta) - one_body_exp<Real>(so, co, sr, cr, LoverPi, beta);
  }
  acc += xor_lane<16>(acc);
  acc += xor_lane<32>(acc);
  return (double)(acc * dev_rcp<Real>(beta));
}

// Moves the NS electrons of spin `sp` of every walker once, in order, with
// delayed updates of the inverse in blocks of 16 moves.  A proposal depends only
// on the electron's own position, which no earlier move of the half-sweep
// changes, so the 16 proposals of a block are drawn together:
//   M' = Phi' C          MO rows of the proposals (16 x NS, FP64 matrix cores)
//   P  = M' A^-1         their products with the inverse at the block start
// Move j then needs t = m'_j (A^-1 after the accepted moves j' < j of the block),
// obtained from P_j by the left-looking recursion t -= t[i_j'] z_j' over the
// accepted j', with z_j' = (t_j' - e_i_j') / q_j' the Sherman-Morrison row of j';
// the ratio is q_j = t[i_j].  After the block the inverse takes all accepted
// updates at once: A^-1 -= A^-1[:, block] Z with Z = (I + Y)^-1 [z rows], Y the
// strictly upper coupling Y[j''][j'] = z_j''[i_j'], solved by back-substitution.
// Every LDS row access of the recursion is lane-private (lane = column).
// One wave per walker; the inverse lives in matrix-core accumulator layout
// (tile (tr, tc), element v of lane l = A^-1[16 tr + 4 v + l/16][16 tc + l%16]).
template <int NS, class Real, int NIMG, bool BATCH, bool TW, bool CB = false, bool J3 = false>
__global__ __launch_bounds__(256, 2) void k_sweep_half(WalkerArgs a, SweepArgs s, Batch bt) {
  constexpr int N = 2 * NS;
  using LY = SweepLds<NS>;
  constexpr int NSP = LY::NSP, NT = NSP / 16, NB = (NS + 15) / 16, KC = (N + 3) / 4;
  constexpr int LDM = LY::LDM, LDG = LY::LDG;
  constexpr int EPL = (N + 63) / 64;
  constexpr int CPL = (NSP + 63) / 64;   // columns of the recursion vectors per lane
  static_assert(NS <= 64 && (NS == 64 || N <= 64), "the electrons of one spin must share a slot");
  extern __shared__ __align__(16) double smem_d[];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    const int spin = s.spin;
    a = bt.jobs[j].a;
    s = bt.jobs[j].s;
    s.spin = spin;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  double* Rs = smem_d + 4 * LY::WAVE;     // centres x, y, z, zeta
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    Rs[4 * t] = a.R[3 * t]; Rs[4 * t + 1] = a.R[3 * t + 1]; Rs[4 * t + 2] = a.R[3 * t + 2];
    Rs[4 * t + 3] = a.zeta[t];
  }
  Real* Rt = reinterpret_cast<Real*>(Rs + 4 * N);   // one-body and three-body terms: sin (3 x N), then cos (3 x N)
  const bool one_body = a.j1_beta > 0.0;
  if (one_body || J3)
    for (int t = threadIdx.x; t < 3 * N; t += blockDim.x)
      dev_sincospi<Real>((Real)(a.R[3 * (t % N) + t / N] * a.invL), &Rt[t], &Rt[3 * N + t]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, l4 = lane >> 4;
  double* D1 = reinterpret_cast<double*>(Rt + 6 * N) + NSP * wv;   // one-body change of each move
  // (the block index is read at its uses: a long-lived copy costs registers here)
  const int w = (BATCH ? bblk : (int)blockIdx.x) * 4 + wv;
  if (w >= a.W) return;
  double* MB = smem_d + (size_t)wv * LY::WAVE;
  double* PB = MB + LY::MB;
  const int sp = s.spin;
  const int slot = (sp * NS) >> 6;
  const double L = a.L, invL = a.invL;
  const Real LoverPi = (Real)(L / VMC_PI);
  const size_t bbase = ((size_t)w * 2 + sp) * NS * NS;
  if (one_body) {
    // a move's one-body change depends on its electron's position at the start of the
    // half-sweep and on the protons only: all of them now, while the registers that will
    // hold the inverse are free
    const double* pw0 = a.pos + (size_t)w * N * 3;
    for (int b = 0; b < NB; ++b) {
      const int ip = 16 * b + l16;
      if (ip < NS) {
        const double* po = pw0 + 3 * (sp * NS + ip);
        double xn, yn, zn, ru;
        draw_move(s, w, N, sp * NS + ip, po, s.delta, L, invL, xn, yn, zn, ru);
        const double d1 = one_body_change<Real, N>(Rt, po[0], po[1], po[2], xn, yn, zn, invL, LoverPi,
                                                   (Real)a.j1_beta, l4);
        if (l4 == 0) D1[ip] = d1;   // read after the synchronisation that follows the first M'
      }
    }
  }

  // element (r, c) of the inverse at Bw[(16 tr + 4 v) NS] (wave-uniform) + lane offset
  double* Bw = a.Binv + bbase;
  const int loff = l4 * NS + l16;
  d4w_t binv[NT][NT];
#pragma unroll
  for (int tr = 0; tr < NT; ++tr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* rowp = Bw + (16 * tr + 4 * v) * NS;
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        const bool ok = (16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS);
        const double val = rowp[ok ? loff + 16 * tc : -(16 * tr + 4 * v) * NS];   // in range either way
        binv[tr][tc][v] = ok ? val : 0.0;
      }
    }

  // positions stay in HBM: a block reads the current positions of its 16 electrons
  // (no earlier move of the half-sweep touches them) and an accepted move writes
  // its electron's new position; lanes keep the trig caches of electrons lane, lane+64
  Real ts[EPL][3], tc_[EPL][3];
  double* pw = a.pos + (size_t)w * N * 3;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = lane + 64 * t;
    for (int m = 0; m < 3; ++m) { ts[t][m] = Real(0); tc_[t][m] = Real(1); }
    if (e < N) {
      dev_sincospi<Real>((Real)(pw[3 * e] * invL), &ts[t][0], &tc_[t][0]);
      dev_sincospi<Real>((Real)(pw[3 * e + 1] * invL), &ts[t][1], &tc_[t][1]);
      dev_sincospi<Real>((Real)(pw[3 * e + 2] * invL), &ts[t][2], &tc_[t][2]);
    }
  }
  const Real a_same = (Real)a.a_par, a_anti = (Real)a.a_anti, bj = (Real)a.b;
  const double delta = s.delta;
  int nacc = 0;
  // three-body term: lanes hold G_a = sum_i (chi_1, chi_2)(r_i - R_a) of nuclei lane, lane + 64
  double Gj[EPL][2];
  if constexpr (J3) {
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const int c = lane + 64 * t;
      Gj[t][0] = c < N ? a.j3G[((size_t)w * N + c) * 2] : 0.0;
      Gj[t][1] = c < N ? a.j3G[((size_t)w * N + c) * 2 + 1] : 0.0;
    }
  }

  for (int b = 0; b < NB; ++b) {
    const int jmax = (NS - 16 * b) < 16 ? (NS - 16 * b) : 16;
    // proposal of move 16 b + l16 (lanes with equal l16 hold the same one)
    const int ip = 16 * b + l16;
    const bool pvalid = ip < NS;
    const int ipc = pvalid ? ip : 0;
    const double* po = pw + 3 * (sp * NS + ipc);
    const double xo_p = po[0], yo_p = po[1], zo_p = po[2];
    // the move's four uniforms: displacement x, y, z and the acceptance test
    double xn, yn, zn, ru3;
    {
      const double pov[3] = {xo_p, yo_p, zo_p};
      draw_move(s, w, N, sp * NS + ipc, pov, delta, L, invL, xn, yn, zn, ru3);
    }
    // trig cache of proposal l16 along axis l4 (l4 < 3)
    Real sv = Real(0), cv = Real(1);
    {
      const double comp = (l4 == 0) ? xn : ((l4 == 1) ? yn : zn);
      dev_sincospi<Real>((Real)(comp * invL), &sv, &cv);
    }
    // M' = Phi' C on the matrix cores: lane l supplies phi of proposal l%16 at centre 4k + l/16
    d4w_t acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int k = 0; k < KC; ++k) {
      const int c = 4 * k + l4;
      const bool cv_ok = c < N;
      const int cc = cv_ok ? c : 0;
      double bvs[NT];
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        const int col = 16 * tc + l16;
        const bool ok = cv_ok && col < NS;
        const double val = a.C[ok ? cc * NS + col : 0];
        bvs[tc] = ok ? val : 0.0;
      }
      double ph = 0.0;
      if (cv_ok && pvalid) {
        const double* Rc = Rs + 4 * cc;
        if constexpr (CB)
          ph = (double)contracted_value<Real, NIMG>(xn, yn, zn, Rc, (Real)a.eta, L, invL);
        else
          ph = (double)phi_value<Real, NIMG, TW>(xn, yn, zn, Rc, (Real)Rc[3], L, invL, a.twist);
      }
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_w(ph, bvs[tc], acc[tc]);
    }
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int v = 0; v < 4; ++v) MB[(4 * v + l4) * LDM + 16 * tc + l16] = acc[tc][v];
    wave_lds_sync();
    // P = M' A^-1: the inverse registers are the B operand of k step 4 tr + v
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int tr = 0; tr < NT; ++tr) {
      double av[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) av[v] = MB[l16 * LDM + 16 * tr + 4 * v + l4];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_w(av[v], binv[tr][tc][v], acc[tc]);
      asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int v = 0; v < 4; ++v) PB[(4 * v + l4) * LDM + 16 * tc + l16] = acc[tc][v];
    wave_lds_sync();

    // the moves of the block, in order; column c of the recursion vectors is element
    // c / 64 of lane c % 64
    uint32_t amask = 0;
    for (int j = 0; j < jmax; ++j) {
      const int i = 16 * b + j, e = sp * NS + i, owner = e & 63;
      double t[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) t[u] = (lane + 64 * u < NSP) ? PB[j * LDM + lane + 64 * u] : 0.0;
      for (uint32_t mm = amask; mm; mm &= mm - 1) {
        const int jp = __builtin_ctz(mm);
        const double cf = colread(t, 16 * b + jp);
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          t[u] = fma(-cf, (lane + 64 * u < NSP) ? PB[jp * LDM + lane + 64 * u] : 0.0, t[u]);
      }
      const double q = colread(t, i);
      Real sn[3], cn[3], so[3], co[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        sn[m] = readlane<Real>(sv, j + 16 * m);
        cn[m] = readlane<Real>(cv, j + 16 * m);
        so[m] = readlane<Real>(slot == 0 ? ts[0][m] : ts[EPL - 1][m], owner);
        co[m] = readlane<Real>(slot == 0 ? tc_[0][m] : tc_[EPL - 1][m], owner);
      }
      Real du = Real(0);
#pragma unroll
      for (int tt = 0; tt < EPL; ++tt) {
        const int jj = lane + 64 * tt;
        if (jj < N && jj != e) {
          const Real aa = ((jj / NS) == sp) ? a_same : a_anti;
          du += pade_u<Real>(sn, cn, ts[tt], tc_[tt], LoverPi, aa, bj) -
                pade_u<Real>(so, co, ts[tt], tc_[tt], LoverPi, aa, bj);
        }
      }
      // three-body change over the lane's nuclei, (chi(r') - chi(r))^T F (G_a - chi(r)), and the
      // one-body orbital part's, f^T (chi(r') - chi(r))
      Real dj[EPL][2];
      if constexpr (J3) {
#pragma unroll
        for (int tt = 0; tt < EPL; ++tt) {
          const int c = lane + 64 * tt;
          dj[tt][0] = dj[tt][1] = Real(0);
          if (c < N) {
            const Real sa[3] = {Rt[c], Rt[N + c], Rt[2 * N + c]};
            const Real ca[3] = {Rt[3 * N + c], Rt[4 * N + c], Rt[5 * N + c]};
            Real n1, n2, o1, o2;
            j3_values<Real>(sn, cn, sa, ca, LoverPi, n1, n2);
            j3_values<Real>(so, co, sa, ca, LoverPi, o1, o2);
            dj[tt][0] = n1 - o1;
            dj[tt][1] = n2 - o2;
            const Real g1 = (Real)Gj[tt][0] - o1, g2 = (Real)Gj[tt][1] - o2;
            du += (Real)a.j3f[0] * dj[tt][0] * g1 + (Real)a.j3f[1] * (dj[tt][0] * g2 + dj[tt][1] * g1) +
                  (Real)a.j3f[2] * dj[tt][1] * g2;
            // the one-body term's orbital part: f^T (chi(r') - chi(r))
            du += (Real)a.j1f[0] * dj[tt][0] + (Real)a.j1f[1] * dj[tt][1];
          }
        }
      }
      // xor-butterfly sum kept in vector registers, in the precision of the pair terms: every
      // lane adds the same two partial sums at every step, so all lanes hold the identical
      // total and the acceptance test below takes the same branch in every lane
      double dU = (double)wave_allsum(du);
      if (one_body) dU += D1[i];
      // the Jastrow factor in the working precision of the Jastrow terms
      const double pacc = q * q * (double)dev_exp<Real>((Real)(2.0 * dU));
      double zrow[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) zrow[u] = 0.0;
      if (readlane_d(ru3, j) < pacc) {
        const double iq = 1.0 / q;
#pragma unroll
        for (int u = 0; u < CPL; ++u) zrow[u] = (t[u] - (lane + 64 * u == i ? 1.0 : 0.0)) * iq;
        amask |= 1u << j;
        if constexpr (J3) {
#pragma unroll
          for (int tt = 0; tt < EPL; ++tt) {
            Gj[tt][0] += (double)dj[tt][0];
            Gj[tt][1] += (double)dj[tt][1];
          }
        }
        // lanes j, j + 16, j + 32 hold move j's proposal; each writes one coordinate
        if (l16 == j && l4 < 3) pw[3 * e + l4] = (l4 == 0) ? xn : ((l4 == 1) ? yn : zn);
        if (lane == owner) {
#pragma unroll
          for (int tt = 0; tt < EPL; ++tt)
            if (tt == slot)
              for (int m = 0; m < 3; ++m) { ts[tt][m] = sn[m]; tc_[tt][m] = cn[m]; }
        }
        ++nacc;
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < NSP) PB[j * LDM + lane + 64 * u] = zrow[u];
    }
    for (int j = jmax; j < 16; ++j)
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < NSP) PB[j * LDM + lane + 64 * u] = 0.0;
    if (amask == 0) { wave_lds_sync(); continue; }
    // accepted MO rows into A
    for (uint32_t mm = amask; mm; mm &= mm - 1) {
      const int j = __builtin_ctz(mm);
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < NS) a.Amat[bbase + (size_t)(16 * b + j) * NS + lane + 64 * u] = MB[j * LDM + lane + 64 * u];
    }
    // Z = (I + Y)^-1 [z rows]: back-substitution from the last accepted move
#pragma unroll 1
    for (int j = 15; j >= 0; --j) {
      if (!((amask >> j) & 1u)) continue;
      double zo[CPL], z[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        zo[u] = (lane + 64 * u < NSP) ? PB[j * LDM + lane + 64 * u] : 0.0;
        z[u] = zo[u];
      }
      for (uint32_t mm = amask & ~((2u << j) - 1u); mm; mm &= mm - 1) {
        const int jp = __builtin_ctz(mm);
        const double cf = colread(zo, 16 * b + jp);
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          z[u] = fma(-cf, (lane + 64 * u < NSP) ? PB[jp * LDM + lane + 64 * u] : 0.0, z[u]);
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < NSP) PB[j * LDM + lane + 64 * u] = z[u];
    }
    // G = the inverse's columns of this block (column tile b) into the M' buffer
    wave_lds_sync();
    {
      auto snap = [&](auto tcc) {
        constexpr int TC = decltype(tcc)::value;
#pragma unroll
        for (int tr = 0; tr < NT; ++tr)
#pragma unroll
          for (int v = 0; v < 4; ++v) MB[(16 * tr + 4 * v + l4) * LDG + l16] = binv[tr][TC][v];
      };
      switch (b) {
        case 0: snap(std::integral_constant<int, 0>{}); break;
        case 1: if constexpr (NT > 1) snap(std::integral_constant<int, (NT > 1 ? 1 : 0)>{}); break;
        case 2: if constexpr (NT > 2) snap(std::integral_constant<int, (NT > 2 ? 2 : 0)>{}); break;
        default: if constexpr (NT > 3) snap(std::integral_constant<int, (NT > 3 ? 3 : 0)>{}); break;
      }
    }
    wave_lds_sync();
    // A^-1 -= G Z
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      double zb[NT], ga[NT];
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) zb[tc] = PB[(4 * kk + l4) * LDM + 16 * tc + l16];
#pragma unroll
      for (int tr = 0; tr < NT; ++tr) ga[tr] = -MB[(16 * tr + l16) * LDG + 4 * kk + l4];
#pragma unroll
      for (int tr = 0; tr < NT; ++tr)
#pragma unroll
        for (int tc = 0; tc < NT; ++tc) binv[tr][tc] = mfma_w(ga[tr], zb[tc], binv[tr][tc]);
      asm volatile("" ::: "memory");
    }
    wave_lds_sync();
  }
  {
    // the block's walker again from the block index (the lookup is redone rather than kept live)
    const int blk_end = BATCH ? (int)blockIdx.x - bt.off[batch_job(bt, blockIdx.x)] : (int)blockIdx.x;
    Bw = a.Binv + ((size_t)(blk_end * 4 + wv) * 2 + sp) * NS * NS;
#pragma unroll
    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double* rowp = Bw + (16 * tr + 4 * v) * NS;
#pragma unroll
        for (int tc = 0; tc < NT; ++tc)
          if ((16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS)) rowp[loff + 16 * tc] = binv[tr][tc][v];
      }
  }
  if constexpr (J3) {
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const int c = lane + 64 * t;
      if (c < N) {
        a.j3G[((size_t)w * N + c) * 2] = Gj[t][0];
        a.j3G[((size_t)w * N + c) * 2 + 1] = Gj[t][1];
      }
    }
  }
  if (lane == 0) a.nacc[w] += nacc;
}

// The half-sweep for N_sigma = 128, whose inverse (128 KB) stays in HBM: the same
// delayed-update algorithm with the inverse streamed in the register tile layout (each
// lane reads and writes only the elements it would hold as accumulators, so no other
// lane's accesses are involved), 128 recursion columns two per lane, and the electrons of
// a spin spread over two lane slots.  One LDS block of 16 rows per wave (P, then the z
// rows, then the next block's MO rows), so two work-groups share a CU:
//   * the MO rows M' of a block also go to the walker's scratch in HBM, from where the
//     accepted ones are copied to A;
//   * after the back-substitution Z moves to registers (the B operand layout of the
//     update), the next block's proposals and M' are formed, and the update
//     A^-1 -= G Z streams the inverse once, tile by tile, feeding each updated tile into
//     the next block's P = M' A^-1 (G, the inverse's columns of the block, is read from
//     HBM; row tile tr of G is read before the update writes row tile tr).
struct SweepBigLds {
  static constexpr int NS = 128, LDM = NS + 1, WAVE = 16 * LDM;
  static constexpr size_t bytes = ((size_t)4 * WAVE + 4 * 2 * NS) * sizeof(double);
};

template <class Real, int NIMG, bool BATCH, bool TW>
__global__ __launch_bounds__(256, 2) void k_sweep_big(WalkerArgs a, SweepArgs s, Batch bt) {
  constexpr int NS = 128, N = 2 * NS, NT = NS / 16, NB = NS / 16, KC = N / 4, EPL = N / 64, CPL = NS / 64;
  constexpr int LDM = SweepBigLds::LDM;
  extern __shared__ __align__(16) double smem_b[];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    const int spin = s.spin;
    a = bt.jobs[j].a;
    s = bt.jobs[j].s;
    s.spin = spin;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  double* Rs = smem_b + 4 * SweepBigLds::WAVE;     // centres x, y, z, zeta
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    Rs[4 * t] = a.R[3 * t]; Rs[4 * t + 1] = a.R[3 * t + 1]; Rs[4 * t + 2] = a.R[3 * t + 2];
    Rs[4 * t + 3] = a.zeta[t];
  }
  Real* Rt = reinterpret_cast<Real*>(Rs + 4 * N);   // one-body term: sin (3 x N), then cos (3 x N)
  const bool one_body = a.j1_beta > 0.0;
  if (one_body)
    for (int t = threadIdx.x; t < 3 * N; t += blockDim.x)
      dev_sincospi<Real>((Real)(a.R[3 * (t % N) + t / N] * a.invL), &Rt[t], &Rt[3 * N + t]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, l4 = lane >> 4;
  double* D1 = reinterpret_cast<double*>(Rt + 6 * N) + 16 * wv;   // one-body change of each proposal
  const int w = (BATCH ? bblk : (int)blockIdx.x) * 4 + wv;
  if (w >= a.W) return;
  double* PB = smem_b + (size_t)wv * SweepBigLds::WAVE;   // 16 x LDM
  const int sp = s.spin;
  const double L = a.L, invL = a.invL;
  const Real LoverPi = (Real)(L / VMC_PI);
  double* Bw = a.Binv + ((size_t)w * 2 + sp) * NS * NS;
  double* Am = a.Amat + ((size_t)w * 2 + sp) * NS * NS;
  double* Ms = a.rscr + (size_t)w * a.rscr_stride;        // MO rows of the block, 16 x NS
  Real ts[EPL][3], tc_[EPL][3];
  double* pw = a.pos + (size_t)w * N * 3;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = lane + 64 * t;
    dev_sincospi<Real>((Real)(pw[3 * e] * invL), &ts[t][0], &tc_[t][0]);
    dev_sincospi<Real>((Real)(pw[3 * e + 1] * invL), &ts[t][1], &tc_[t][1]);
    dev_sincospi<Real>((Real)(pw[3 * e + 2] * invL), &ts[t][2], &tc_[t][2]);
  }
  const Real a_same = (Real)a.a_par, a_anti = (Real)a.a_anti, bj = (Real)a.b;
  const double delta = s.delta;
  int nacc = 0;

  // proposal of move 16 b + l16 of the next block (lanes with equal l16 hold the same one)
  double xn, yn, zn, ru3;
  Real sv, cv;
  auto propose = [&](int b) {
    const int ip = 16 * b + l16;
    const double* po = pw + 3 * (sp * NS + ip);
    draw_move(s, w, N, sp * NS + ip, po, delta, L, invL, xn, yn, zn, ru3);
    sv = Real(0); cv = Real(1);
    const double comp = (l4 == 0) ? xn : ((l4 == 1) ? yn : zn);
    dev_sincospi<Real>((Real)(comp * invL), &sv, &cv);
    if (one_body) {
      const double d1 = one_body_change<Real, N>(Rt, po[0], po[1], po[2], xn, yn, zn, invL, LoverPi, (Real)a.j1_beta, l4);
      if (l4 == 0) D1[l16] = d1;   // read after the synchronisation that follows M'
    }
  };
  // M' = Phi' C on the matrix cores -> PB (left operand layout rows) and the HBM scratch
  auto mo_rows = [&]() {
    d4w_t acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int k = 0; k < KC; ++k) {
      const int c = 4 * k + l4;
      double bvs[NT];
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) bvs[tc] = a.C[c * NS + 16 * tc + l16];
      const double* Rc = Rs + 4 * c;
      const double ph = (double)phi_value<Real, NIMG, TW>(xn, yn, zn, Rc, (Real)Rc[3], L, invL, a.twist);
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_w(ph, bvs[tc], acc[tc]);
    }
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        PB[(4 * v + l4) * LDM + 16 * tc + l16] = acc[tc][v];
        Ms[(4 * v + l4) * NS + 16 * tc + l16] = acc[tc][v];
      }
    wave_lds_sync();
  };
  // P = M' A^-1 with the inverse read from HBM, M' from PB -> PB
  auto p_rows = [&]() {
    d4w_t acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tr = 0; tr < NT; ++tr) {
      double av[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) av[v] = PB[l16 * LDM + 16 * tr + 4 * v + l4];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tc = 0; tc < NT; ++tc)
          acc[tc] = mfma_w(av[v], Bw[(16 * tr + 4 * v + l4) * NS + 16 * tc + l16], acc[tc]);
    }
    wave_lds_sync();
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int v = 0; v < 4; ++v) PB[(4 * v + l4) * LDM + 16 * tc + l16] = acc[tc][v];
    wave_lds_sync();
  };

  propose(0);
  mo_rows();
  p_rows();
  for (int b = 0; b < NB; ++b) {
    const int slotb = (sp * NS + 16 * b) >> 6;   // lane slot of this block's electrons
    // the moves of the block, in order; column c of the recursion vectors is element
    // c / 64 of lane c % 64
    uint32_t amask = 0;
    for (int j = 0; j < 16; ++j) {
      const int i = 16 * b + j, e = sp * NS + i, owner = e & 63;
      double t[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) t[u] = PB[j * LDM + lane + 64 * u];
      for (uint32_t mm = amask; mm; mm &= mm - 1) {
        const int jp = __builtin_ctz(mm);
        const double cf = colread(t, 16 * b + jp);
#pragma unroll
        for (int u = 0; u < CPL; ++u) t[u] = fma(-cf, PB[jp * LDM + lane + 64 * u], t[u]);
      }
      const double q = colread(t, i);
      Real sn[3], cn[3], so[3], co[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        sn[m] = readlane<Real>(sv, j + 16 * m);
        cn[m] = readlane<Real>(cv, j + 16 * m);
        Real s0 = ts[0][m], c0 = tc_[0][m];
#pragma unroll
        for (int tt = 1; tt < EPL; ++tt) { s0 = (tt == slotb) ? ts[tt][m] : s0; c0 = (tt == slotb) ? tc_[tt][m] : c0; }
        so[m] = readlane<Real>(s0, owner);
        co[m] = readlane<Real>(c0, owner);
      }
      Real du = Real(0);
#pragma unroll
      for (int tt = 0; tt < EPL; ++tt) {
        const int jj = lane + 64 * tt;
        if (jj != e) {
          const Real aa = ((jj / NS) == sp) ? a_same : a_anti;
          du += pade_u<Real>(sn, cn, ts[tt], tc_[tt], LoverPi, aa, bj) -
                pade_u<Real>(so, co, ts[tt], tc_[tt], LoverPi, aa, bj);
        }
      }
      double dU = wave_allsum((double)du);
      if (one_body) dU += D1[j];
      const double pacc = q * q * (double)dev_exp<Real>((Real)(2.0 * dU));
      double zrow[CPL] = {0.0, 0.0};
      if (readlane_d(ru3, j) < pacc) {
        const double iq = 1.0 / q;
#pragma unroll
        for (int u = 0; u < CPL; ++u) zrow[u] = (t[u] - (lane + 64 * u == i ? 1.0 : 0.0)) * iq;
        amask |= 1u << j;
        if (l16 == j && l4 < 3) pw[3 * e + l4] = (l4 == 0) ? xn : ((l4 == 1) ? yn : zn);
        if (lane == owner) {
#pragma unroll
          for (int tt = 0; tt < EPL; ++tt)
            if (tt == slotb)
              for (int m = 0; m < 3; ++m) { ts[tt][m] = sn[m]; tc_[tt][m] = cn[m]; }
        }
        ++nacc;
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u) PB[j * LDM + lane + 64 * u] = zrow[u];
    }
    const bool more = b + 1 < NB;
    if (amask == 0) {                         // nothing to update: the next block's P from the same inverse
      wave_lds_sync();
      if (more) { propose(b + 1); mo_rows(); p_rows(); }
      continue;
    }
    // accepted MO rows into A (from the scratch copy)
    for (uint32_t mm = amask; mm; mm &= mm - 1) {
      const int j = __builtin_ctz(mm);
#pragma unroll
      for (int u = 0; u < CPL; ++u) Am[(size_t)(16 * b + j) * NS + lane + 64 * u] = Ms[j * NS + lane + 64 * u];
    }
    // Z = (I + Y)^-1 [z rows]: back-substitution from the last accepted move
#pragma unroll 1
    for (int j = 15; j >= 0; --j) {
      if (!((amask >> j) & 1u)) continue;
      double zo[CPL], z[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) { zo[u] = PB[j * LDM + lane + 64 * u]; z[u] = zo[u]; }
      for (uint32_t mm = amask & ~((2u << j) - 1u); mm; mm &= mm - 1) {
        const int jp = __builtin_ctz(mm);
        const double cf = colread(zo, 16 * b + jp);
#pragma unroll
        for (int u = 0; u < CPL; ++u) z[u] = fma(-cf, PB[jp * LDM + lane + 64 * u], z[u]);
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u) PB[j * LDM + lane + 64 * u] = z[u];
    }
    wave_lds_sync();
    // Z into registers in the update's B operand layout, which frees PB
    double zr[NT][4];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) zr[tc][kk] = PB[(4 * kk + l4) * LDM + 16 * tc + l16];
    wave_lds_sync();
    // the next block's proposals and MO rows (into PB and the scratch)
    if (more) { propose(b + 1); mo_rows(); }
    // A^-1 -= G Z tile by tile; each updated tile also feeds the next block's P = M' A^-1
    d4w_t pacc_t[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) pacc_t[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tr = 0; tr < NT; ++tr) {
      double ga[4], av[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) ga[kk] = -Bw[(16 * tr + l16) * NS + 16 * b + 4 * kk + l4];
#pragma unroll
      for (int v = 0; v < 4; ++v) av[v] = more ? PB[l16 * LDM + 16 * tr + 4 * v + l4] : 0.0;
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        double* tp = Bw + (16 * tr + l4) * NS + 16 * tc + l16;
        d4w_t tile = {tp[0], tp[4 * NS], tp[8 * NS], tp[12 * NS]};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) tile = mfma_w(ga[kk], zr[tc][kk], tile);
        tp[0] = tile[0]; tp[4 * NS] = tile[1]; tp[8 * NS] = tile[2]; tp[12 * NS] = tile[3];
#pragma unroll
        for (int v = 0; v < 4; ++v) pacc_t[tc] = mfma_w(av[v], tile[v], pacc_t[tc]);
      }
    }
    wave_lds_sync();
    if (more) {
#pragma unroll
      for (int tc = 0; tc < NT; ++tc)
#pragma unroll
        for (int v = 0; v < 4; ++v) PB[(4 * v + l4) * LDM + 16 * tc + l16] = pacc_t[tc][v];
      wave_lds_sync();
    }
  }
  if (lane == 0) a.nacc[w] += nacc;
}

// ------------------------------------------------- refinement refresh ---
// One Newton-Schulz step X <- X + X (I - A X) on the FP64 matrix cores, one
// wave per matrix.  X (the inverse carried through the previous half-sweep)
// differs from A^-1 only by accumulated rounding E, and the step leaves an error
// of order E^2, so it restores the inverse to working precision at a quarter of
// the elimination's issue cost.  If max |I - A X| over the matrix exceeds tol
// (or is not finite) the matrix is flagged for elimination instead.
// X sits in accumulator layout (tile (tr, tc), element v of lane l =
// X[16 tr + 4 v + l/16][16 tc + l%16]) and, as the left operand of X R, in LDS.
template <int NS>
struct RefineLds {
  static constexpr int NSP = (NS + 15) / 16 * 16, LDX = NSP + 1;
  static constexpr size_t bytes = (size_t)4 * NSP * LDX * sizeof(double);
};

template <int NS, bool BATCH>
__global__ __launch_bounds__(256, 1) void k_refine(WalkerArgs a, int sp, double tol, Batch bt) {
  constexpr int NSP = RefineLds<NS>::NSP, NT = NSP / 16, LDX = RefineLds<NS>::LDX;
  extern __shared__ __align__(16) double smem_r[];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    a = bt.jobs[j].a;
    tol = bt.jobs[j].tol;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  const int blk = BATCH ? bblk : (int)blockIdx.x;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, l4 = lane >> 4;
  const int w = blk * 4 + wv;
  if (w >= a.W) return;
  double* xs = smem_r + (size_t)wv * NSP * LDX;
  const size_t base = ((size_t)w * 2 + sp) * NS * NS;
  const double* Ag = a.Amat + base;
  double* Xg = a.Binv + base;
  const int loff = l4 * NS + l16;
  d4w_t xr[NT][NT];
#pragma unroll
  for (int tr = 0; tr < NT; ++tr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* rowp = Xg + (16 * tr + 4 * v) * NS;
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        const bool ok = (16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS);
        const double val = rowp[ok ? loff + 16 * tc : -(16 * tr + 4 * v) * NS];
        xr[tr][tc][v] = ok ? val : 0.0;
        xs[(16 * tr + 4 * v + l4) * LDX + 16 * tc + l16] = ok ? val : 0.0;
      }
    }
  wave_lds_sync();
  // R = I - A X (real rows and columns only)
  d4w_t rr[NT][NT];
  double rmax = 0.0;
#pragma unroll
  for (int tr = 0; tr < NT; ++tr) {
    d4w_t acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = d4w_t{0.0, 0.0, 0.0, 0.0};
    const int arow = 16 * tr + l16;
#pragma unroll
    for (int ks = 0; ks < NSP / 4; ++ks) {
      const int acol = 4 * ks + l4;
      const bool ok = arow < NS && acol < NS;
      const double val = Ag[ok ? arow * NS + acol : 0];
      const double av = ok ? val : 0.0;
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_w(av, xr[ks / 4][tc][ks % 4], acc[tc]);
    }
#pragma unroll
    for (int tc = 0; tc < NT; ++tc)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * tr + 4 * v + l4, col = 16 * tc + l16;
        const double r = (row < NS && col < NS) ? ((row == col ? 1.0 : 0.0) - acc[tc][v]) : 0.0;
        rr[tr][tc][v] = r;
        rmax = fmax(rmax, fabs(r)) + (r - r);     // NaN propagates
      }
  }
  // X + X R, written back in place
#pragma unroll
  for (int tr = 0; tr < NT; ++tr) {
    d4w_t acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = xr[tr][tc];
#pragma unroll
    for (int ks = 0; ks < NSP / 4; ++ks) {
      const double av = xs[(16 * tr + l16) * LDX + 4 * ks + l4];
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_w(av, rr[ks / 4][tc][ks % 4], acc[tc]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double* rowp = Xg + (16 * tr + 4 * v) * NS;
#pragma unroll
      for (int tc = 0; tc < NT; ++tc)
        if ((16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS)) rowp[loff + 16 * tc] = acc[tc][v];
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(rmax, off, 64);
    rmax = (o > rmax || o != o) ? o : rmax;
  }
  if (lane == 0 && !(rmax <= tol)) a.rflag[(size_t)w * 2 + sp] = 1;
}

// The same step with two waves per matrix, for matrices of an even number (>= 2) of column
// tiles: wave h of a pair owns column tiles [h NT/2, (h+1) NT/2) of R and of the new X, so it
// holds half the fragments of k_refine and two work-groups (two matrices each) fit per CU,
// letting one matrix's loads overlap another's matrix-core work.  X's LDS copy, the left
// operand of X R, is shared by the pair and taken before either wave writes X back.  Every
// output tile accumulates the same products in the same order as in k_refine, so the results
// are identical.
template <int NS>
struct RefinePairLds {
  static constexpr size_t bytes = (size_t)2 * RefineLds<NS>::NSP * RefineLds<NS>::LDX * sizeof(double);
};

template <int NS, bool BATCH>
__global__ __launch_bounds__(256, 2) void k_refine_pair(WalkerArgs a, int sp, double tol, Batch bt) {
  constexpr int NSP = RefineLds<NS>::NSP, NT = NSP / 16, LDX = RefineLds<NS>::LDX, NH = NT / 2;
  static_assert(NT >= 2 && NT % 2 == 0, "the two waves split the column tiles evenly");
  extern __shared__ __align__(16) double smem_r[];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    a = bt.jobs[j].a;
    tol = bt.jobs[j].tol;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  const int blk = BATCH ? bblk : (int)blockIdx.x;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, l4 = lane >> 4;
  const int w = blk * 2 + (wv >> 1), h = wv & 1;
  const bool active = w < a.W;
  double* xs = smem_r + (size_t)(wv >> 1) * NSP * LDX;
  const size_t base = ((size_t)(active ? w : 0) * 2 + sp) * NS * NS;
  const double* Ag = a.Amat + base;
  double* Xg = a.Binv + base;
  const int loff = l4 * NS + l16;
  d4w_t xr[NT][NH];                 // X[:, tiles h NH .. h NH + NH - 1] in accumulator layout
  if (active) {
#pragma unroll
    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double* rowp = Xg + (16 * tr + 4 * v) * NS;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const int tc = h * NH + j;
          const bool ok = (16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS);
          const double val = rowp[ok ? loff + 16 * tc : -(16 * tr + 4 * v) * NS];
          xr[tr][j][v] = ok ? val : 0.0;
          xs[(16 * tr + 4 * v + l4) * LDX + 16 * tc + l16] = ok ? val : 0.0;
        }
      }
  }
  __syncthreads();                  // the pair's halves of X are in LDS (the only barrier)
  if (!active) return;
  // R[:, own tiles] = I - A X[:, own tiles]
  d4w_t rr[NT][NH];
  double rmax = 0.0;
#pragma unroll
  for (int tr = 0; tr < NT; ++tr) {
    d4w_t acc[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) acc[j] = d4w_t{0.0, 0.0, 0.0, 0.0};
    const int arow = 16 * tr + l16;
#pragma unroll
    for (int ks = 0; ks < NSP / 4; ++ks) {
      const int acol = 4 * ks + l4;
      const bool ok = arow < NS && acol < NS;
      const double val = Ag[ok ? arow * NS + acol : 0];
      const double av = ok ? val : 0.0;
#pragma unroll
      for (int j = 0; j < NH; ++j) acc[j] = mfma_w(av, xr[ks / 4][j][ks % 4], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < NH; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * tr + 4 * v + l4, col = 16 * (h * NH + j) + l16;
        const double r = (row < NS && col < NS) ? ((row == col ? 1.0 : 0.0) - acc[j][v]) : 0.0;
        rr[tr][j][v] = r;
        rmax = fmax(rmax, fabs(r)) + (r - r);     // NaN propagates
      }
  }
  // X[:, own tiles] + X R[:, own tiles], written back in place (the other wave reads X from LDS)
#pragma unroll
  for (int tr = 0; tr < NT; ++tr) {
    d4w_t acc[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) acc[j] = xr[tr][j];
#pragma unroll
    for (int ks = 0; ks < NSP / 4; ++ks) {
      const double av = xs[(16 * tr + l16) * LDX + 4 * ks + l4];
#pragma unroll
      for (int j = 0; j < NH; ++j) acc[j] = mfma_w(av, rr[ks / 4][j][ks % 4], acc[j]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double* rowp = Xg + (16 * tr + 4 * v) * NS;
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        const int tc = h * NH + j;
        if ((16 * tr + 4 * v + l4 < NS) && (16 * tc + l16 < NS)) rowp[loff + 16 * tc] = acc[j][v];
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(rmax, off, 64);
    rmax = (o > rmax || o != o) ? o : rmax;
  }
  // either wave of the pair may flag the matrix (both store the same value)
  if (lane == 0 && !(rmax <= tol)) a.rflag[(size_t)w * 2 + sp] = 1;
}

// The refinement step for NS = 128, where X and A do not fit in registers: one 512-thread
// work-group per matrix.  Both products take the right operand's column tile w of wave w in
// registers (read once) and stage the left operand 16 rows at a time in LDS, row tiles in
// the outer loop so X can be updated in place (row tile rt of X + X R needs only row tile rt
// of X).  R = I - A X goes to the walker's scratch between the two products.  Built for four
// waves per SIMD (128 registers, a few spilled) so that two work-groups share a CU and one's
// row-tile loads and barriers overlap the other's matrix-core work.
template <int NS, bool BATCH>
__global__ __launch_bounds__(512, 4) void k_refine_big(WalkerArgs a, int sp, double tol, Batch bt) {
  static_assert(NS == 128, "eight column tiles, one per wave");
  constexpr int KK = NS / 4, NRT = NS / 16, LDS_S = NS + 1, NTH = 512;
  __shared__ double stage[16 * LDS_S];
  __shared__ double wmax[8];
  int blk = blockIdx.x;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blk);
    a = bt.jobs[j].a;
    tol = bt.jobs[j].tol;
    blk -= bt.off[j];
  }
  const int t = threadIdx.x & (NTH - 1), lane = t & 63, wave = t >> 6, l16 = lane & 15, l4 = lane >> 4;
  const int w = blk;
  if (w >= a.W) return;                      // the whole work-group
  const size_t base = ((size_t)w * 2 + sp) * NS * NS;
  double* Xg = a.Binv + base;
  const double* Ag = a.Amat + base;
  double* Rg = a.rscr + (size_t)w * a.rscr_stride;
  const int col = 16 * wave + l16;
  double breg[KK];
  auto stage_rows = [&](const double* src, int rt) {
    __syncthreads();                          // the previous tile is consumed
    for (int u = t; u < 16 * NS; u += NTH) stage[(u / NS) * LDS_S + u % NS] = src[(size_t)(16 * rt + u / NS) * NS + u % NS];
    __syncthreads();
  };
  // R = I - A X
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) breg[kk] = Xg[(4 * kk + l4) * NS + col];
  double rmax = 0.0;
  for (int rt = 0; rt < NRT; ++rt) {
    stage_rows(Ag, rt);
    d4w_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) acc = mfma_w(stage[l16 * LDS_S + 4 * kk + l4], breg[kk], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * rt + l4 + 4 * v;
      const double r = (row == col ? 1.0 : 0.0) - acc[v];
      Rg[(size_t)row * NS + col] = r;
      rmax = fmax(rmax, fabs(r)) + (r - r);     // NaN propagates
    }
  }
  // X + X R, row tile by row tile, in place (each wave reads back only its own columns of R)
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) breg[kk] = Rg[(size_t)(4 * kk + l4) * NS + col];
  for (int rt = 0; rt < NRT; ++rt) {
    stage_rows(Xg, rt);
    d4w_t acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = stage[(l4 + 4 * v) * LDS_S + col];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) acc = mfma_w(stage[l16 * LDS_S + 4 * kk + l4], breg[kk], acc);
    // row tile rt is in LDS for every wave before any wave writes it back
#pragma unroll
    for (int v = 0; v < 4; ++v) Xg[(size_t)(16 * rt + l4 + 4 * v) * NS + col] = acc[v];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(rmax, off, 64);
    rmax = (o > rmax || o != o) ? o : rmax;
  }
  if (lane == 0) wmax[wave] = rmax;
  __syncthreads();
  if (t == 0) {
    double m = wmax[0];
    for (int q = 1; q < 8; ++q) m = (wmax[q] > m || wmax[q] != wmax[q]) ? wmax[q] : m;
    if (!(m <= tol)) a.rflag[(size_t)w * 2 + sp] = 1;
  }
}

// ------------------------------------------------------ walker quarantine ---
// A walker with a non-finite coordinate (flag 1) takes a copy of the next walker, cyclically,
// whose coordinates are all finite; count[0] counts the copies, count[1] the bad walkers left
// without a source (every walker bad).  Finite walkers are not written.
__global__ __launch_bounds__(256) void k_walker_flags(int n3, const double* pos, int* flags) {
  const int w = blockIdx.x;
  int bad = 0;
  for (int u = threadIdx.x; u < n3; u += 256) bad |= !isfinite(pos[(size_t)w * n3 + u]);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flags[w] = bad;
}
__global__ __launch_bounds__(256) void k_walker_repair(int W, int n3, double* pos, const int* flags, int* count) {
  const int w = blockIdx.x;
  if (!flags[w]) return;
  int src = -1;
  for (int d = 1; d < W && src < 0; ++d) {
    const int c = (w + d) % W;
    if (!flags[c]) src = c;
  }
  if (src < 0) {
    if (threadIdx.x == 0) atomicAdd(count + 1, 1);
    return;
  }
  for (int u = threadIdx.x; u < n3; u += 256) pos[(size_t)w * n3 + u] = pos[(size_t)src * n3 + u];
  if (threadIdx.x == 0) atomicAdd(count, 1);
}
hipError_t launch_walker_quarantine(int W, int N, double* pos, int* flags, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_walker_flags, dim3(W), dim3(256), 0, st, 3 * N, pos, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_walker_repair, dim3(W), dim3(256), 0, st, W, 3 * N, pos, flags, count);
  return hipGetLastError();
}

// ----------------------------------------------------------- launchers ---
template <int NS, class Real, bool TW>
hipError_t launch_build_A_tw(const WalkerArgs& a, hipStream_t st) {
  dim3 grid((a.W + 3) / 4);
  if (a.nimg || sizeof(Real) == 8)
    hipLaunchKernelGGL((k_build_A<NS, Real, 1, TW>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_build_A<NS, Real, 0, TW>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}
template <int NS, class Real>
hipError_t launch_build_A_t(const WalkerArgs& a, hipStream_t st) {
  if (a.contracted) {
    if constexpr (NS > 64) {
      return hipErrorInvalidValue;
    } else {
      if (a.twist) return hipErrorInvalidValue;
      dim3 grid((a.W + 3) / 4);
      if (a.nimg || sizeof(Real) == 8)
        hipLaunchKernelGGL((k_build_A<NS, Real, 1, false, true>), grid, dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((k_build_A<NS, Real, 0, false, true>), grid, dim3(256), 0, st, a);
      return hipGetLastError();
    }
  }
  return a.twist ? launch_build_A_tw<NS, Real, true>(a, st) : launch_build_A_tw<NS, Real, false>(a, st);
}
inline Batch batch_or_none(const Batch* bt) { return bt ? *bt : Batch{nullptr, nullptr, 0}; }

template <int NS>
hipError_t launch_invert_t(const WalkerArgs& a, int spin_lo, int spin_hi, int only_flagged, hipStream_t st,
                           const Batch* bt, int nblk) {
  if constexpr (NS > 64) {          // one work-group per matrix
    dim3 g(bt ? nblk : a.W * (spin_hi - spin_lo));
    if (bt)
      hipLaunchKernelGGL((k_invert_big<NS, true>), g, dim3(256), 0, st, a, spin_lo, spin_hi, only_flagged, *bt);
    else
      hipLaunchKernelGGL((k_invert_big<NS, false>), g, dim3(256), 0, st, a, spin_lo, spin_hi, only_flagged,
                         batch_or_none(bt));
    return hipGetLastError();
  } else {
    dim3 grid(bt ? nblk : (a.W * (spin_hi - spin_lo) + 3) / 4);
    if (bt)
      hipLaunchKernelGGL((k_invert<NS, true>), grid, dim3(256), 0, st, a, spin_lo, spin_hi, only_flagged, *bt);
    else
      hipLaunchKernelGGL((k_invert<NS, false>), grid, dim3(256), 0, st, a, spin_lo, spin_hi, only_flagged, batch_or_none(bt));
    return hipGetLastError();
  }
}
template <int NS>
hipError_t launch_refine_t(const WalkerArgs& a, int spin, double tol, hipStream_t st, const Batch* bt, int nblk) {
  if constexpr (NS > 64) {          // one work-group per matrix, scratch for R
    if (!a.rscr) return hipErrorInvalidValue;
    dim3 g(bt ? nblk : a.W);
    if (bt)
      hipLaunchKernelGGL((k_refine_big<NS, true>), g, dim3(512), 0, st, a, spin, tol, *bt);
    else
      hipLaunchKernelGGL((k_refine_big<NS, false>), g, dim3(512), 0, st, a, spin, tol, batch_or_none(bt));
    return hipGetLastError();
  } else {
    if constexpr (refine_pairs(NS)) {             // two waves per matrix, two matrices per block
      if (bt)
        hipLaunchKernelGGL((k_refine_pair<NS, true>), dim3(nblk), dim3(256), RefinePairLds<NS>::bytes, st, a, spin,
                           tol, *bt);
      else
        hipLaunchKernelGGL((k_refine_pair<NS, false>), dim3((a.W + 1) / 2), dim3(256), RefinePairLds<NS>::bytes, st,
                           a, spin, tol, batch_or_none(bt));
      return hipGetLastError();
    }
    dim3 grid(bt ? nblk : (a.W + 3) / 4);
    if (bt)
      hipLaunchKernelGGL((k_refine<NS, true>), grid, dim3(256), RefineLds<NS>::bytes, st, a, spin, tol, *bt);
    else
      hipLaunchKernelGGL((k_refine<NS, false>), grid, dim3(256), RefineLds<NS>::bytes, st, a, spin, tol, batch_or_none(bt));
    return hipGetLastError();
  }
}
template <int NS, class Real>
size_t sweep_smem() {
  return SweepLds<NS>::bytes(2 * NS);
}
// (a batch holds only twisted or only untwisted trajectories: the request loop buckets them apart)
template <int NS, class Real, bool TW>
hipError_t launch_sweep_tw(const WalkerArgs& a, const SweepArgs& s, hipStream_t st, const Batch* bt, int nblk) {
  dim3 grid(bt ? nblk : (a.W + 3) / 4);
  const bool img = a.nimg || sizeof(Real) == 8;
  const size_t tab = a.j1_beta > 0.0 ? one_body_table_bytes<Real>(2 * NS, NS == 128 ? 16 : SweepLds<NS>::NSP) : 0;
  if constexpr (NS == 128) {
    const size_t smb = SweepBigLds::bytes + tab;
    if (bt && img)
      hipLaunchKernelGGL((k_sweep_big<Real, 1, true, TW>), grid, dim3(256), smb, st, a, s, *bt);
    else if (bt)
      hipLaunchKernelGGL((k_sweep_big<Real, 0, true, TW>), grid, dim3(256), smb, st, a, s, *bt);
    else if (img)
      hipLaunchKernelGGL((k_sweep_big<Real, 1, false, TW>), grid, dim3(256), smb, st, a, s, batch_or_none(bt));
    else
      hipLaunchKernelGGL((k_sweep_big<Real, 0, false, TW>), grid, dim3(256), smb, st, a, s, batch_or_none(bt));
    return hipGetLastError();
  } else {
    size_t sm = sweep_smem<NS, Real>() + tab;
    if (bt && img)
      hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, true, TW>), grid, dim3(256), sm, st, a, s, *bt);
    else if (bt)
      hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, true, TW>), grid, dim3(256), sm, st, a, s, *bt);
    else if (img)
      hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, false, TW>), grid, dim3(256), sm, st, a, s, batch_or_none(bt));
    else
      hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, false, TW>), grid, dim3(256), sm, st, a, s, batch_or_none(bt));
    return hipGetLastError();
  }
}

template <int NS, class Real>
hipError_t launch_sweep_t(const WalkerArgs& a, const SweepArgs& s, hipStream_t st, const Batch* bt, int nblk) {
  if (a.j3) {
    // the three-body term: single trajectories, N_sigma <= 64, with the single Gaussian (real twists
    // allowed) or the contracted orbital (no twist)
    if constexpr (NS > 64) {
      return hipErrorInvalidValue;
    } else {
      if (bt || (a.twist && a.contracted) || !a.j3G) return hipErrorInvalidValue;
      const size_t tab = one_body_table_bytes<Real>(2 * NS, SweepLds<NS>::NSP);
      const size_t sm = sweep_smem<NS, Real>() + tab;
      dim3 grid((a.W + 3) / 4);
      const bool img = a.nimg || sizeof(Real) == 8;
      if (a.contracted) {
        if (img)
          hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, false, false, true, true>), grid, dim3(256), sm, st, a, s,
                             batch_or_none(bt));
        else
          hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, false, false, true, true>), grid, dim3(256), sm, st, a, s,
                             batch_or_none(bt));
      } else if (a.twist) {
        if (img)
          hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, false, true, false, true>), grid, dim3(256), sm, st, a, s,
                             batch_or_none(bt));
        else
          hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, false, true, false, true>), grid, dim3(256), sm, st, a, s,
                             batch_or_none(bt));
      } else if (img) {
        hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, false, false, false, true>), grid, dim3(256), sm, st, a, s,
                           batch_or_none(bt));
      } else {
        hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, false, false, false, true>), grid, dim3(256), sm, st, a, s,
                           batch_or_none(bt));
      }
      return hipGetLastError();
    }
  }
  if (a.contracted) {
    // the contracted orbital: single trajectories without twist, N_sigma <= 64
    if constexpr (NS > 64) {
      return hipErrorInvalidValue;
    } else {
      if (bt || a.twist) return hipErrorInvalidValue;
      const size_t tab = a.j1_beta > 0.0 ? one_body_table_bytes<Real>(2 * NS, SweepLds<NS>::NSP) : 0;
      const size_t sm = sweep_smem<NS, Real>() + tab;
      dim3 grid((a.W + 3) / 4);
      if (a.nimg || sizeof(Real) == 8)
        hipLaunchKernelGGL((k_sweep_half<NS, Real, 1, false, false, true>), grid, dim3(256), sm, st, a, s,
                           batch_or_none(bt));
      else
        hipLaunchKernelGGL((k_sweep_half<NS, Real, 0, false, false, true>), grid, dim3(256), sm, st, a, s,
                           batch_or_none(bt));
      return hipGetLastError();
    }
  }
  return a.twist ? launch_sweep_tw<NS, Real, true>(a, s, st, bt, nblk) : launch_sweep_tw<NS, Real, false>(a, s, st, bt, nblk);
}

#define VMC_DISPATCH_NS(ns, CALL) \
  switch (ns) {                   \
    case 8: { constexpr int NSV = 8; CALL; } \
    case 12: { constexpr int NSV = 12; CALL; } \
    case 16: { constexpr int NSV = 16; CALL; } \
    case 20: { constexpr int NSV = 20; CALL; } \
    case 24: { constexpr int NSV = 24; CALL; } \
    case 27: { constexpr int NSV = 27; CALL; } \
    case 32: { constexpr int NSV = 32; CALL; } \
    case 64: { constexpr int NSV = 64; CALL; } \
    case 128: { constexpr int NSV = 128; CALL; } \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_build_A(const WalkerArgs& a, int mixed, hipStream_t st) {
  if (mixed) { VMC_DISPATCH_NS(a.NS, return (launch_build_A_t<NSV, float>(a, st))) }
  VMC_DISPATCH_NS(a.NS, return (launch_build_A_t<NSV, double>(a, st)))
}
hipError_t launch_invert(const WalkerArgs& a, int spin_lo, int spin_hi, int only_flagged, hipStream_t st,
                         const Batch* bt, int nblk) {
  VMC_DISPATCH_NS(a.NS, return (launch_invert_t<NSV>(a, spin_lo, spin_hi, only_flagged, st, bt, nblk)))
}
hipError_t launch_refine(const WalkerArgs& a, int spin, double tol, hipStream_t st, const Batch* bt, int nblk) {
  VMC_DISPATCH_NS(a.NS, return (launch_refine_t<NSV>(a, spin, tol, st, bt, nblk)))
}
hipError_t launch_sweep(const WalkerArgs& a, const SweepArgs& s, int mixed, hipStream_t st, const Batch* bt,
                        int nblk) {
  if (mixed) { VMC_DISPATCH_NS(a.NS, return (launch_sweep_t<NSV, float>(a, s, st, bt, nblk))) }
  VMC_DISPATCH_NS(a.NS, return (launch_sweep_t<NSV, double>(a, s, st, bt, nblk)))
}

}  // namespace vmc
