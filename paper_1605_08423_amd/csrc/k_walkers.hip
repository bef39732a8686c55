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

template <class Real>
__device__ __forceinline__ Real phi_value(double rx, double ry, double rz, const double* Ra, Real zeta,
                                          double L, double invL) {
  Real g[3][4];
  gauss1d<Real, 0>((Real)min_image(rx - Ra[0], L, invL), zeta, (Real)L, g[0]);
  gauss1d<Real, 0>((Real)min_image(ry - Ra[1], L, invL), zeta, (Real)L, g[1]);
  gauss1d<Real, 0>((Real)min_image(rz - Ra[2], L, invL), zeta, (Real)L, g[2]);
  return g[0][0] * g[1][0] * g[2][0];
}

// --------------------------------------------------------------- build A ---
// One wave per walker; electrons in order, lanes over centres then orbitals.
template <int NS, class Real>
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
      phi_s[wv][c] = phi_value<Real>(rx, ry, rz, a.R + 3 * c, (Real)a.zeta[c], a.L, a.invL);
    wave_lds_sync();
    if (lane < NS) {
      Real m = Real(0);
      for (int c = 0; c < N; ++c) m += phi_s[wv][c] * (Real)a.C[c * NS + lane];
      int sp = e / NS, i = e % NS;
      a.Amat[(((size_t)w * 2 + sp) * NS + i) * NS + lane] = (double)m;
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------------- inverse refresh ---
// In-place Gauss-Jordan inversion with partial (row) pivoting, one wave per
// matrix in LDS; columns are unscrambled in reverse pivot order at the end.
// Also records ln|det| and the sign.  A zero pivot sets *status = 1.
template <int NS>
__global__ __launch_bounds__(64) void k_invert(WalkerArgs a, int spin_lo, int spin_hi) {
  constexpr int LD = NS + 1;
  __shared__ double m[NS * LD];
  __shared__ int pivots[NS];
  const int lane = threadIdx.x;
  const int nsp = spin_hi - spin_lo;
  const int w = blockIdx.x / nsp, sp = spin_lo + blockIdx.x % nsp;
  if (w >= a.W) return;
  const size_t base = ((size_t)w * 2 + sp) * NS * NS;
  for (int t = lane; t < NS * NS; t += 64) m[(t / NS) * LD + t % NS] = a.Amat[base + t];
  wave_lds_sync();
  double logdet = 0.0, sgn = 1.0;
  bool singular = false;
  for (int p = 0; p < NS; ++p) {
    double bv = -1.0;
    int bi = NS;
    for (int r = lane; r < NS; r += 64)
      if (r >= p) {
        double v = fabs(m[r * LD + p]);
        if (v > bv) { bv = v; bi = r; }
      }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      double ov = __shfl_xor(bv, off, 64);
      int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    const int piv = __builtin_amdgcn_readfirstlane(bi);
    const double pv = readlane_d(m[piv * LD + p], 0);
    if (pv == 0.0) { singular = true; break; }
    if (piv != p) {
      for (int c = lane; c < NS; c += 64) {
        double t0 = m[p * LD + c], t1 = m[piv * LD + c];
        m[p * LD + c] = t1;
        m[piv * LD + c] = t0;
      }
      sgn = -sgn;
    }
    if (lane == 0) pivots[p] = piv;
    logdet += log(fabs(pv));
    if (pv < 0.0) sgn = -sgn;
    const double pinv = 1.0 / pv;
    wave_lds_sync();
    double prow[(NS + 63) / 64];
#pragma unroll
    for (int t = 0; t < (NS + 63) / 64; ++t) {
      int c = lane + 64 * t;
      if (c < NS) {
        double v = (c == p) ? pinv : m[p * LD + c] * pinv;
        m[p * LD + c] = v;
        prow[t] = v;
      }
    }
    wave_lds_sync();
    // column p of every row (lane r holds row r's multiplier; NS <= 64)
    const double fcol = (lane < NS) ? m[lane * LD + p] : 0.0;
    wave_lds_sync();
    for (int r = 0; r < NS; ++r) {
      if (r == p) continue;
      const double f = readlane_d(fcol, r);
#pragma unroll
      for (int t = 0; t < (NS + 63) / 64; ++t) {
        int c = lane + 64 * t;
        if (c < NS) m[r * LD + c] = ((c == p) ? 0.0 : m[r * LD + c]) - f * prow[t];
      }
    }
    wave_lds_sync();
  }
  if (singular) {
    if (lane == 0) {
      *a.status = 1;
      a.ldet[(size_t)w * 2 + sp] = -INFINITY;
      a.sgn[(size_t)w * 2 + sp] = 0.0;
    }
    return;
  }
  for (int p = NS - 1; p >= 0; --p) {
    const int q = pivots[p];
    if (q != p)
      for (int r = lane; r < NS; r += 64) {
        double t0 = m[r * LD + p], t1 = m[r * LD + q];
        m[r * LD + p] = t1;
        m[r * LD + q] = t0;
      }
    wave_lds_sync();
  }
  for (int t = lane; t < NS * NS; t += 64) a.Binv[base + t] = m[(t / NS) * LD + t % NS];
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
template <int NS, class Real>
__global__ __launch_bounds__(256, (NS >= 64 ? 1 : 2)) void k_sweep_half(WalkerArgs a, SweepArgs s) {
  constexpr int N = 2 * NS;
  constexpr int WPB = 4;
  constexpr int EPL = (N + 63) / 64;     // electrons (and centres) per lane
  extern __shared__ __align__(16) unsigned char smem[];
  Real* Cs = reinterpret_cast<Real*>(smem);                      // N x NS
  Real* phi_s = Cs + N * NS;                                       // WPB x N
  double* m_s = reinterpret_cast<double*>(smem + ((N * NS + WPB * N) * sizeof(Real) + 15) / 16 * 16);  // WPB x NS
  for (int t = threadIdx.x; t < N * NS; t += blockDim.x) Cs[t] = (Real)a.C[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = blockIdx.x * WPB + wv;
  if (w >= a.W) return;
  const int sp = s.spin;
  Real* phi = phi_s + wv * N;
  double* mrow = m_s + wv * NS;
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
    // basis row at the proposed position
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      int c = lane + 64 * t;
      if (c < N) {
        Real g[3][4];
        gauss1d<Real, 0>((Real)min_image(xn - Rc[t][0], L, invL), zc[t], (Real)L, g[0]);
        gauss1d<Real, 0>((Real)min_image(yn - Rc[t][1], L, invL), zc[t], (Real)L, g[1]);
        gauss1d<Real, 0>((Real)min_image(zn - Rc[t][2], L, invL), zc[t], (Real)L, g[2]);
        phi[c] = g[0][0] * g[1][0] * g[2][0];
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
    wave_lds_sync();
    // MO row m_k = sum_a phi_a C[a][k]
    double mk = 0.0;
    if (lane < NS) {
      Real acc = Real(0);
      for (int c = 0; c < N; ++c) acc += phi[c] * Cs[c * NS + lane];
      mk = (double)acc;
      mrow[lane] = mk;
    }
    wave_lds_sync();
    // v_j = sum_k m_k (A^-1)[k][j]; the ratio is q = v_i
    double vj = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) vj += mrow[k] * bcol[k];
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
    wave_lds_sync();
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
  hipLaunchKernelGGL((k_build_A<NS, Real>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}
template <int NS>
hipError_t launch_invert_t(const WalkerArgs& a, int spin_lo, int spin_hi, hipStream_t st) {
  dim3 grid(a.W * (spin_hi - spin_lo));
  hipLaunchKernelGGL((k_invert<NS>), grid, dim3(64), 0, st, a, spin_lo, spin_hi);
  return hipGetLastError();
}
template <int NS, class Real>
size_t sweep_smem() {
  constexpr int N = 2 * NS;
  return ((N * NS + 4 * N) * sizeof(Real) + 15) / 16 * 16 + 4 * NS * sizeof(double);
}
template <int NS, class Real>
hipError_t launch_sweep_t(const WalkerArgs& a, const SweepArgs& s, hipStream_t st) {
  dim3 grid((a.W + 3) / 4);
  size_t sm = sweep_smem<NS, Real>();
  hipLaunchKernelGGL((k_sweep_half<NS, Real>), grid, dim3(256), sm, st, a, s);
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
