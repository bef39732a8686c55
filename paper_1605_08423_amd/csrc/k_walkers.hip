// Walker kernels: Slater matrices at new proton positions (a2), the FP64 inverse
// refresh (a4) and the Metropolis half-sweep with Sherman-Morrison updates (a3).
//
// Layout in HBM (per trajectory, W walkers, N electrons, NS = N/2 per spin):
//   pos  [W][N][3]            electron positions, wrapped into [0, L)
//   Amat [W][2][NS][NS]       Slater matrix rows A[i][k] = sum_a phi_a(r_i) C[a][k]
//   Binv [W][2][NS][NS]       inverse, row-major (A^-1)[k][i]
//   ldet [W][2], sgn[W][2]    ln|det A| and sign at the last refresh
// A wavefront (64 lanes) owns one walker in the sweep: lane j keeps column j of
// the active spin's inverse in registers, lanes also own electrons and basis
// centres j, j+64, ...; the MO coefficients C are shared through LDS.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

template <class Real, int NIMG>
__device__ __forceinline__ Real phi_value(double rx, double ry, double rz, const double* Ra, Real zeta,
                                          double L, double invL) {
  Real g[3][4];
  gauss1d_n<Real, 0, NIMG>((Real)min_image(rx - Ra[0], L, invL), zeta, (Real)L, g[0]);
  gauss1d_n<Real, 0, NIMG>((Real)min_image(ry - Ra[1], L, invL), zeta, (Real)L, g[1]);
  gauss1d_n<Real, 0, NIMG>((Real)min_image(rz - Ra[2], L, invL), zeta, (Real)L, g[2]);
  return g[0][0] * g[1][0] * g[2][0];
}

// --------------------------------------------------------------- build A ---
// One wave per walker; electrons in order, lanes over centres then orbitals.
template <int NS, class Real, int NIMG>
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
      phi_s[wv][c] = phi_value<Real, NIMG>(rx, ry, rz, a.R + 3 * c, (Real)a.zeta[c], a.L, a.invL);
    wave_lds_sync();
    if (lane < NS) {
      double m = 0.0;
      for (int c = 0; c < N; ++c) m += (double)phi_s[wv][c] * a.C[c * NS + lane];
      int sp = e / NS, i = e % NS;
      a.Amat[(((size_t)w * 2 + sp) * NS + i) * NS + lane] = m;
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
template <int NS>
__global__ __launch_bounds__(256) void k_invert(WalkerArgs a, int spin_lo, int spin_hi) {
  constexpr int BC = 16, NB = (NS + BC - 1) / BC;
  __shared__ double stage[4 * NS * 17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nsp = spin_hi - spin_lo;
  const int mat = blockIdx.x * 4 + wv;
  const int w = mat / nsp, sp = spin_lo + mat % nsp;
  if (w >= a.W) return;
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
      const double pinv = 1.0 / pv;
      const bool me = lane == piv;
      if (me) { used = true; myk = p; }
      if (lane == p) mypi = piv;
      const double g = (me ? (pv - 1.0) : rp) * pinv;
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

// ---------------------------------------------------------- half sweep ---
template <class T, int E>
__device__ __forceinline__ T pick(const T (&v)[E], int s) {
  T r = v[0];
#pragma unroll
  for (int t = 1; t < E; ++t) r = (s == t) ? v[t] : r;
  return r;
}

// Moves the NS electrons of spin `sp` of every walker once, in order.
template <int NS, class Real, int NIMG>
__global__ __launch_bounds__(256, ((sizeof(Real) == 8 && NS >= 27) || NS >= 64) ? 1 : 2) void k_sweep_half(WalkerArgs a, SweepArgs s) {
  constexpr int N = 2 * NS;
  constexpr int WPB = 4;
  constexpr int EPL = (N + 63) / 64;     // electrons (and centres) per lane
  extern __shared__ __align__(16) unsigned char smem[];
  double* Cs = reinterpret_cast<double*>(smem);                  // N x NS (FP64 in both modes)
  for (int t = threadIdx.x; t < N * NS; t += blockDim.x) Cs[t] = a.C[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = blockIdx.x * WPB + wv;
  if (w >= a.W) return;
  const int sp = s.spin;
  const double L = a.L, invL = a.invL;
  const Real LoverPi = (Real)(L / VMC_PI);

  double bcol[NS];
  const size_t bbase = ((size_t)w * 2 + sp) * NS * NS;
#pragma unroll
  for (int k = 0; k < NS; ++k) bcol[k] = (lane < NS) ? a.Binv[bbase + (size_t)k * NS + lane] : 0.0;

  double px[EPL], py[EPL], pz[EPL];
  Real ts[EPL][3], tc[EPL][3];
  double Rc[EPL][3];
  Real zc[EPL];
  double* pw = a.pos + (size_t)w * N * 3;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    int e = lane + 64 * t;
    px[t] = py[t] = pz[t] = 0.0;
    zc[t] = Real(1);
    Rc[t][0] = Rc[t][1] = Rc[t][2] = 0.0;
    for (int m = 0; m < 3; ++m) { ts[t][m] = Real(0); tc[t][m] = Real(1); }
    if (e < N) {
      px[t] = pw[3 * e]; py[t] = pw[3 * e + 1]; pz[t] = pw[3 * e + 2];
      dev_sincospi<Real>((Real)(px[t] * invL), &ts[t][0], &tc[t][0]);
      dev_sincospi<Real>((Real)(py[t] * invL), &ts[t][1], &tc[t][1]);
      dev_sincospi<Real>((Real)(pz[t] * invL), &ts[t][2], &tc[t][2]);
      Rc[t][0] = a.R[3 * e]; Rc[t][1] = a.R[3 * e + 1]; Rc[t][2] = a.R[3 * e + 2];
      zc[t] = (Real)a.zeta[e];
    }
  }
  // This half-sweep's random numbers: lane i holds those of move i.
  double ru0 = 0, ru1 = 0, ru2 = 0, ru3 = 0;
  if (lane < NS) {
    const uint32_t ctr2 = (uint32_t)(s.sweep * N + sp * NS + lane);
    u32x4 o0 = philox(s.step, (uint32_t)w, ctr2, 0u, s.seed, s.traj);
    u32x4 o1 = philox(s.step, (uint32_t)w, ctr2, 1u, s.seed, s.traj);
    ru0 = u01(o0.x, o0.y); ru1 = u01(o0.z, o0.w); ru2 = u01(o1.x, o1.y); ru3 = u01(o1.z, o1.w);
  }
  const Real a_same = (Real)a.a_par, a_anti = (Real)a.a_anti, bj = (Real)a.b;
  const double delta = s.delta;
  int nacc = 0;
  for (int i = 0; i < NS; ++i) {
    const int e = sp * NS + i, owner = e & 63, slot = e >> 6;
    const double ux = readlane_d(ru0, i), uy = readlane_d(ru1, i), uz = readlane_d(ru2, i);
    const double uacc = readlane_d(ru3, i);
    const double xo = readlane_d(pick(px, slot), owner);
    const double yo = readlane_d(pick(py, slot), owner);
    const double zo = readlane_d(pick(pz, slot), owner);
    const double xn = wrap_box(xo + delta * (ux - 0.5), L, invL);
    const double yn = wrap_box(yo + delta * (uy - 0.5), L, invL);
    const double zn = wrap_box(zo + delta * (uz - 0.5), L, invL);
    // basis row at the proposed position: lane keeps phi of its own centres
    Real phv[EPL];
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      int c = lane + 64 * t;
      phv[t] = Real(0);
      if (c < N) {
        Real g[3][4];
        gauss1d_n<Real, 0, NIMG>((Real)min_image(xn - Rc[t][0], L, invL), zc[t], (Real)L, g[0]);
        gauss1d_n<Real, 0, NIMG>((Real)min_image(yn - Rc[t][1], L, invL), zc[t], (Real)L, g[1]);
        gauss1d_n<Real, 0, NIMG>((Real)min_image(zn - Rc[t][2], L, invL), zc[t], (Real)L, g[2]);
        phv[t] = g[0][0] * g[1][0] * g[2][0];
      }
    }
    // trig cache of the proposed position: lanes 0..2 compute one axis each
    Real sv, cv;
    {
      const int ax = lane % 3;
      const double comp = (ax == 0) ? xn : ((ax == 1) ? yn : zn);
      dev_sincospi<Real>((Real)(comp * invL), &sv, &cv);
    }
    Real sn[3], cn[3], so[3], co[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      sn[m] = readlane<Real>(sv, m);
      cn[m] = readlane<Real>(cv, m);
      so[m] = readlane<Real>(slot == 0 ? ts[0][m] : ts[EPL - 1][m], owner);
      co[m] = readlane<Real>(slot == 0 ? tc[0][m] : tc[EPL - 1][m], owner);
    }
    // MO row m_k = sum_a phi_a C[a][k] in FP64: phi_a broadcast from its lane
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const int cmax = (N - 64 * t) < 64 ? (N - 64 * t) : 64;
#pragma unroll 8
      for (int l = 0; l < cmax; ++l)
        acc += (double)readlane<Real>(phv[t], l) * Cs[(64 * t + l) * NS + (lane < NS ? lane : 0)];
    }
    const double mk = (lane < NS) ? acc : 0.0;
    // v_j = sum_k m_k (A^-1)[k][j]; the ratio is q = v_i
    double vj = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) vj += readlane_d(mk, k) * bcol[k];
    const double q = readlane_d(vj, i);
    // Jastrow change sum_j u(r', r_j) - u(r_e, r_j)
    Real du = Real(0);
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      int j = lane + 64 * t;
      if (j < N && j != e) {
        const Real aa = ((j / NS) == sp) ? a_same : a_anti;
        du += pade_u<Real>(sn, cn, ts[t], tc[t], LoverPi, aa, bj) - pade_u<Real>(so, co, ts[t], tc[t], LoverPi, aa, bj);
      }
    }
    const double dU = wave_sum((double)du);
    const double pacc = q * q * exp(2.0 * dU);
    if (uacc < pacc) {
      const double coef = (vj - (lane == i ? 1.0 : 0.0)) / q;
#pragma unroll
      for (int k = 0; k < NS; ++k) bcol[k] -= readlane_d(bcol[k], i) * coef;
      if (lane == owner) {
#pragma unroll
        for (int t = 0; t < EPL; ++t)
          if (t == slot) {
            px[t] = xn; py[t] = yn; pz[t] = zn;
            for (int m = 0; m < 3; ++m) { ts[t][m] = sn[m]; tc[t][m] = cn[m]; }
          }
      }
      if (lane < NS) a.Amat[bbase + (size_t)i * NS + lane] = mk;
      ++nacc;
    }
  }
  if (lane < NS) {
#pragma unroll
    for (int k = 0; k < NS; ++k) a.Binv[bbase + (size_t)k * NS + lane] = bcol[k];
  }
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    int e = lane + 64 * t;
    if (e < N) { pw[3 * e] = px[t]; pw[3 * e + 1] = py[t]; pw[3 * e + 2] = pz[t]; }
  }
  if (lane == 0) a.nacc[w] += nacc;
}

// ----------------------------------------------------------- launchers ---
template <int NS, class Real>
hipError_t launch_build_A_t(const WalkerArgs& a, hipStream_t st) {
  dim3 grid((a.W + 3) / 4);
  if (a.nimg || sizeof(Real) == 8)
    hipLaunchKernelGGL((k_build_A<NS, Real, 1>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_build_A<NS, Real, 0>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}
template <int NS>
hipError_t launch_invert_t(const WalkerArgs& a, int spin_lo, int spin_hi, hipStream_t st) {
  dim3 grid((a.W * (spin_hi - spin_lo) + 3) / 4);
  hipLaunchKernelGGL((k_invert<NS>), grid, dim3(256), 0, st, a, spin_lo, spin_hi);
  return hipGetLastError();
}
template <int NS, class Real>
size_t sweep_smem() {
  constexpr int N = 2 * NS;
  return (size_t)N * NS * sizeof(double);
}
template <int NS, class Real>
hipError_t launch_sweep_t(const WalkerArgs& a, const SweepArgs& s, hipStream_t st) {
  dim3 grid((a.W + 3) / 4);
  size_t sm = sweep_smem<NS, Real>();
  if (a.nimg || sizeof(Real) == 8)
    hipLaunchKernelGGL((k_sweep_half<NS, Real, 1>), grid, dim3(256), sm, st, a, s);
  else
    hipLaunchKernelGGL((k_sweep_half<NS, Real, 0>), grid, dim3(256), sm, st, a, s);
  return hipGetLastError();
}

#define VMC_DISPATCH_NS(ns, CALL) \
  switch (ns) {                   \
    case 8: { constexpr int NSV = 8; CALL; } \
    case 16: { constexpr int NSV = 16; CALL; } \
    case 27: { constexpr int NSV = 27; CALL; } \
    case 32: { constexpr int NSV = 32; CALL; } \
    case 64: { constexpr int NSV = 64; CALL; } \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_build_A(const WalkerArgs& a, int mixed, hipStream_t st) {
  if (mixed) { VMC_DISPATCH_NS(a.NS, return (launch_build_A_t<NSV, float>(a, st))) }
  VMC_DISPATCH_NS(a.NS, return (launch_build_A_t<NSV, double>(a, st)))
}
hipError_t launch_invert(const WalkerArgs& a, int spin_lo, int spin_hi, hipStream_t st) {
  VMC_DISPATCH_NS(a.NS, return (launch_invert_t<NSV>(a, spin_lo, spin_hi, st)))
}
hipError_t launch_sweep(const WalkerArgs& a, const SweepArgs& s, int mixed, hipStream_t st) {
  if (mixed) { VMC_DISPATCH_NS(a.NS, return (launch_sweep_t<NSV, float>(a, s, st))) }
  VMC_DISPATCH_NS(a.NS, return (launch_sweep_t<NSV, double>(a, s, st)))
}

}  // namespace vmc
