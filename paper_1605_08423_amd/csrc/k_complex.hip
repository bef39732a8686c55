// General twisted boundary conditions (SI, basis section): with twist angles theta the basis
// obeys phi(r + n L) = e^{i theta.n} phi(r), so orbitals, Slater matrices and determinants are
// complex, |psi|^2 = |D_up|^2 |D_dn|^2 e^{2U} and the local energy is complex; its real part is
// the estimator.  FP64 throughout.
//
//   phi_a(r) = prod_m g_m(r_m - R_am),  g_m(d) = sum_n e^{-i theta_m n} e^{-zeta_a (d + n L)^2},
// evaluated at the minimum image x = d - k L over the images n = -1, 0, 1, times e^{i theta_m k}.
//
// Layout in HBM (a complex number is a (re, im) pair of doubles):
//   C    [N][NS]           orbital coefficients
//   Binv [W][2][NS][NS]    (A^-1)[k][i] of A[i][k] = sum_a phi_a(r_i) C[a][k]
//   ldet [W][2], sgn[W][2] ln|det A| and arg det A (the moves keep them current)
// Kernels:
//   k_csweep          one work-group per walker and spin.  With `refresh` it forms A on the
//                     matrix cores and inverts it by Gauss-Jordan elimination in LDS, else it reads
//                     the inverse; then it moves the spin's electrons in order with
//                     Sherman-Morrison updates of the inverse held in LDS, delayed over blocks of
//                     16 moves.  All proposals of the spin are drawn up front and their orbital
//                     rows formed together on the matrix cores: a proposal depends only on its own
//                     electron, which no earlier move of the spin displaces.
//   k_cslater_sample  Re E_L, d ln|psi|/dR and d Re E_L/dR by the contractions of the real
//                     measurement in complex arithmetic (B = C A^-1, M = X B, W = B M).
#include "common.hpp"
#include "kernels.hpp"
#include "moves.hpp"

namespace vmc {

namespace {

struct cd {
  double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
// real part of a b
__device__ __forceinline__ double remul(cd a, cd b) { return a.r * b.r - a.i * b.i; }

typedef double v4d __attribute__((ext_vector_type(4)));
// One complex 16x16x4 step on the FP64 matrix cores, (Dr + i Di) += (A_r + i A_i)(B_r + i B_i):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element v of the result is
// D[l / 16 + 4 v][l % 16].
__device__ __forceinline__ void cmfma(cd av, cd bv, v4d& dr, v4d& di) {
  dr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.r, bv.r, dr, 0, 0, 0);
  dr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.i, bv.i, dr, 0, 0, 0);
  di = __builtin_amdgcn_mfma_f64_16x16x4f64(av.r, bv.i, di, 0, 0, 0);
  di = __builtin_amdgcn_mfma_f64_16x16x4f64(av.i, bv.r, di, 0, 0, 0);
}

// One Cartesian factor of the Bloch-summed Gaussian and its first NDER derivatives at the raw
// offset d along axis m.
template <int NDER>
__device__ __forceinline__ void cbasis_axis(double d, double zeta, double L, double invL, const TwistArgs& tw, int m,
                                            cd g[4]) {
  const double k = floor(d * invL + 0.5);
  const double x = d - L * k;
  double h[3][4];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const double t = x + (double)(n - 1) * L;
    const double e = exp(-zeta * t * t);
    h[n][0] = e;
    if (NDER >= 1) h[n][1] = -2.0 * zeta * t * e;
    if (NDER >= 2) h[n][2] = (4.0 * zeta * zeta * t * t - 2.0 * zeta) * e;
    if (NDER >= 3) h[n][3] = (-8.0 * zeta * zeta * zeta * t * t * t + 12.0 * zeta * zeta * t) * e;
  }
  // image n weighs e^{-i theta n}: n = -1 -> c + i s, n = 0 -> 1, n = 1 -> c - i s
  const double c = tw.c[m], s = tw.s[m];
#pragma unroll
  for (int q = 0; q <= NDER; ++q) g[q] = {h[1][q] + c * (h[0][q] + h[2][q]), s * (h[0][q] - h[2][q])};
  if (k != 0.0) {
    double pc, ps;
    if (k == 1.0) { pc = c; ps = s; }
    else if (k == -1.0) { pc = c; ps = -s; }
    else sincos(tw.th[m] * k, &ps, &pc);
#pragma unroll
    for (int q = 0; q <= NDER; ++q) g[q] = cmul(g[q], cd{pc, ps});
  }
}

__device__ __forceinline__ cd cphi(double rx, double ry, double rz, const double* Ra, double zeta, double L,
                                   double invL, const TwistArgs& tw) {
  cd g[3][4];
  cbasis_axis<0>(rx - Ra[0], zeta, L, invL, tw, 0, g[0]);
  cbasis_axis<0>(ry - Ra[1], zeta, L, invL, tw, 1, g[1]);
  cbasis_axis<0>(rz - Ra[2], zeta, L, invL, tw, 2, g[2]);
  return cmul(cmul(g[0][0], g[1][0]), g[2][0]);
}

// The SI's contracted orbital phi_1 + eta phi_2 under the twist: per axis the Bloch factors of
// g1 = e^{-Z1 t^2}, g2 = e^{-Z2 t^2} and h2 = t^2 e^{-Z2 t^2} with their first NDER derivatives,
// each taken like cbasis_axis (images n = -1, 0, 1 at the minimum image weighted e^{-i theta n},
// times e^{i theta k}); the orbital is g1 g1 g1 + eta (h2 g2 g2 + g2 h2 g2 + g2 g2 h2).
template <int NDER>
__device__ __forceinline__ void bloch_factor(const double h[3][4], double k, const TwistArgs& tw, int m, cd g[4]) {
  const double c = tw.c[m], s = tw.s[m];
#pragma unroll
  for (int q = 0; q <= NDER; ++q) g[q] = {h[1][q] + c * (h[0][q] + h[2][q]), s * (h[0][q] - h[2][q])};
  if (k != 0.0) {
    double pc, ps;
    if (k == 1.0) { pc = c; ps = s; }
    else if (k == -1.0) { pc = c; ps = -s; }
    else sincos(tw.th[m] * k, &ps, &pc);
#pragma unroll
    for (int q = 0; q <= NDER; ++q) g[q] = cmul(g[q], cd{pc, ps});
  }
}

template <int NDER>
__device__ __forceinline__ void ccontracted_axis(double d, double L, double invL, const TwistArgs& tw, int m, cd g1[4],
                                                 cd g2[4], cd h2[4]) {
  const double k = floor(d * invL + 0.5);
  const double x = d - L * k, z1 = kZ1, z2 = kZ2;
  double a1[3][4], a2[3][4], b2[3][4];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const double t = x + (double)(n - 1) * L, t2 = t * t;
    const double e1 = exp(-z1 * t2), e2 = exp(-z2 * t2);
    a1[n][0] = e1;
    a2[n][0] = e2;
    b2[n][0] = t2 * e2;
    if (NDER >= 1) {
      a1[n][1] = -2.0 * z1 * t * e1;
      a2[n][1] = -2.0 * z2 * t * e2;
      b2[n][1] = (2.0 * t - 2.0 * z2 * t2 * t) * e2;
    }
    if (NDER >= 2) {
      a1[n][2] = (4.0 * z1 * z1 * t2 - 2.0 * z1) * e1;
      a2[n][2] = (4.0 * z2 * z2 * t2 - 2.0 * z2) * e2;
      b2[n][2] = (2.0 - 10.0 * z2 * t2 + 4.0 * z2 * z2 * t2 * t2) * e2;
    }
    if (NDER >= 3) {
      a1[n][3] = (-8.0 * z1 * z1 * z1 * t2 * t + 12.0 * z1 * z1 * t) * e1;
      a2[n][3] = (-8.0 * z2 * z2 * z2 * t2 * t + 12.0 * z2 * z2 * t) * e2;
      b2[n][3] = (-24.0 * z2 * t + 36.0 * z2 * z2 * t2 * t - 8.0 * z2 * z2 * z2 * t2 * t2 * t) * e2;
    }
  }
  bloch_factor<NDER>(a1, k, tw, m, g1);
  bloch_factor<NDER>(a2, k, tw, m, g2);
  bloch_factor<NDER>(b2, k, tw, m, h2);
}

// Value, gradient, Hessian and gradient of the Laplacian of a complex basis function.
struct CBasisD {
  cd v, gx, gy, gz, hxx, hyy, hzz, hxy, hxz, hyz, glx, gly, glz;
};
// Adds w times the components of the product f[0](x) f[1](y) f[2](z) (FULL: all; else value
// and gradient).
template <bool FULL>
__device__ __forceinline__ void cprod_terms(const cd (&f)[3][4], double w, CBasisD& o) {
  const cd p00 = cmul(f[1][0], f[2][0]), p01 = cmul(f[0][0], f[2][0]), p02 = cmul(f[0][0], f[1][0]);
  auto add = [w](cd& acc, cd v) { acc = cadd(acc, cd{w * v.r, w * v.i}); };
  add(o.v, cmul(f[0][0], p00));
  add(o.gx, cmul(f[0][1], p00));
  add(o.gy, cmul(f[1][1], p01));
  add(o.gz, cmul(f[2][1], p02));
  if (FULL) {
    add(o.hxx, cmul(f[0][2], p00));
    add(o.hyy, cmul(f[1][2], p01));
    add(o.hzz, cmul(f[2][2], p02));
    add(o.hxy, cmul(cmul(f[0][1], f[1][1]), f[2][0]));
    add(o.hxz, cmul(cmul(f[0][1], f[1][0]), f[2][1]));
    add(o.hyz, cmul(cmul(f[0][0], f[1][1]), f[2][1]));
    add(o.glx, cadd(cmul(f[0][3], p00), cmul(f[0][1], cadd(cmul(f[1][2], f[2][0]), cmul(f[1][0], f[2][2])))));
    add(o.gly, cadd(cmul(f[1][3], p01), cmul(f[1][1], cadd(cmul(f[0][2], f[2][0]), cmul(f[0][0], f[2][2])))));
    add(o.glz, cadd(cmul(f[2][3], p02), cmul(f[2][1], cadd(cmul(f[0][2], f[1][0]), cmul(f[0][0], f[1][2])))));
  }
}

template <bool FULL>
__device__ __forceinline__ CBasisD ccontracted_derivs(double dx, double dy, double dz, double eta, double L,
                                                      double invL, const TwistArgs& tw) {
  constexpr int ND = FULL ? 3 : 1;
  cd g1[3][4], g2[3][4], h2[3][4];
  ccontracted_axis<ND>(dx, L, invL, tw, 0, g1[0], g2[0], h2[0]);
  ccontracted_axis<ND>(dy, L, invL, tw, 1, g1[1], g2[1], h2[1]);
  ccontracted_axis<ND>(dz, L, invL, tw, 2, g1[2], g2[2], h2[2]);
  const cd z = {0.0, 0.0};
  CBasisD o = {z, z, z, z, z, z, z, z, z, z, z, z, z};
  cprod_terms<FULL>(g1, 1.0, o);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    cd f[3][4];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
      for (int q = 0; q <= ND; ++q) f[mm][q] = (mm == m) ? h2[mm][q] : g2[mm][q];
    cprod_terms<FULL>(f, eta, o);
  }
  return o;
}

__device__ __forceinline__ cd ccontracted_value(double rx, double ry, double rz, const double* Ra, double eta,
                                                double L, double invL, const TwistArgs& tw) {
  cd g1[3][4], g2[3][4], h2[3][4];
  ccontracted_axis<0>(rx - Ra[0], L, invL, tw, 0, g1[0], g2[0], h2[0]);
  ccontracted_axis<0>(ry - Ra[1], L, invL, tw, 1, g1[1], g2[1], h2[1]);
  ccontracted_axis<0>(rz - Ra[2], L, invL, tw, 2, g1[2], g2[2], h2[2]);
  const cd v1 = cmul(cmul(g1[0][0], g1[1][0]), g1[2][0]);
  const cd v2 = cadd(cadd(cmul(cmul(h2[0][0], g2[1][0]), g2[2][0]), cmul(cmul(g2[0][0], h2[1][0]), g2[2][0])),
                     cmul(cmul(g2[0][0], g2[1][0]), h2[2][0]));
  return {v1.r + eta * v2.r, v1.i + eta * v2.i};
}

__device__ __forceinline__ cd ld_c(const double* p, size_t idx) {
  const double2 v = *reinterpret_cast<const double2*>(p + 2 * idx);
  return {v.x, v.y};
}
__device__ __forceinline__ void st_c(double* p, size_t idx, cd v) {
  *reinterpret_cast<double2*>(p + 2 * idx) = make_double2(v.r, v.i);
}

// Deterministic sum over a 256-thread block (waves combined in a fixed order); every thread
// gets the result.
__device__ __forceinline__ double csum256(double v, double* red4) {
  v = wave_allsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

}  // namespace

// ------------------------------------------------------------- half sweep ---
// Threads of a half-sweep work-group: eight waves, two per SIMD, so that one wave's LDS round
// trips overlap another's arithmetic (the LDS held by one walker allows one work-group per CU).
constexpr int CT = 512, CW = CT / 64;

template <int NS>
struct CSweepLds {
  static constexpr int N = 2 * NS, NSP = (NS + 15) / 16 * 16, LDA = NSP + 1;
  static constexpr int P = (CT / NS) < NS ? (CT / NS) : NS;   // partial sums of a row product
  static constexpr int CH = (NS + P - 1) / P;                    // their k range
  static constexpr int RPT = CT / NS;                           // rows per pass of an NS-wide update
  // offsets in doubles; the proposals' orbital rows come last (absent in a refresh-only launch)
  static constexpr size_t ainv = 0, pos = ainv + 2 * (size_t)NSP * LDA, trig = pos + 3 * N, prop = trig + 6 * N,
                          ptrig = prop + 4 * NSP, vpart = ptrig + 6 * NSP, colI = vpart + 2 * (size_t)P * NSP,
                          prow = colI + 2 * NSP, fcol = prow + 2 * NSP, red = fcol + 2 * NSP, misc = red + 16,
                          mp = misc + NSP + 8;
  static constexpr size_t bytes(bool moves) { return sizeof(double) * (moves ? mp + 2 * (size_t)NSP * NSP : mp); }
};

// refresh: 0 carries the previous half-sweep's inverse; 1 forms A and inverts it by elimination;
// 2 forms A and refines the carried inverse X by one Newton-Schulz step X + X (I - A X), with the
// elimination instead where max |I - A X| exceeds rtol (or is not finite).
template <int NS, bool MOVES, bool CB>
__global__ __launch_bounds__(CT, 1) void k_csweep(WalkerArgs a, SweepArgs s, TwistArgs tw, int refresh,
                                                  double rtol) {
  using LY = CSweepLds<NS>;
  constexpr int N = 2 * NS, NSP = LY::NSP, LDA = LY::LDA, P = LY::P, CH = LY::CH, RPT = LY::RPT;
  constexpr int TR = NSP / 16, TC = NSP / 16, KS = (N + 3) / 4;
  extern __shared__ __align__(16) double smem[];
  double* Ai = smem + LY::ainv;      // NSP x LDA complex: A, then A^-1
  double* pos = smem + LY::pos;      // N x 3
  double* trig = smem + LY::trig;    // N x 6: sin(pi x/L) x3, cos x3
  double* prop = smem + LY::prop;    // NSP x 4: proposal x, y, z and the acceptance uniform
  double* ptrig = smem + LY::ptrig;  // NSP x 6
  double* vpart = smem + LY::vpart;  // P x NSP complex
  double* colI = smem + LY::colI;    // NSP complex
  double* prow = smem + LY::prow;    // NSP complex
  double* fcol = smem + LY::fcol;    // NSP complex
  double* red = smem + LY::red;      // 16: per-wave partials, then the pivot
  int* perm = reinterpret_cast<int*>(smem + LY::misc);   // NSP pivot rows, then flags
  int* flag = perm + NSP;
  double* Mp = smem + LY::mp;        // NSP x NSP complex: orbital rows of the proposals
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int w = blockIdx.x, sp = s.spin;
  const double L = a.L, invL = a.invL;
  for (int u = t; u < 3 * N; u += CT) pos[u] = a.pos[(size_t)w * 3 * N + u];
  __syncthreads();
  for (int e = t; e < N; e += CT)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) sincospi(pos[3 * e + ax] * invL, &trig[6 * e + ax], &trig[6 * e + 3 + ax]);
  // the sines and cosines of pi R_c / L of every proton (one- and three-body terms), in the
  // region of the row-product partial sums, which the delayed moves do not use
  double* ptab = smem + LY::vpart;   // N x 6
  static_assert(6 * N <= 2 * P * NSP, "the proton table fits the partial-sum region");
  if (MOVES && (a.j1_beta > 0.0 || a.j3))
    for (int c = t; c < N; c += CT)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) sincospi(a.R[3 * c + ax] * invL, &ptab[6 * c + ax], &ptab[6 * c + 3 + ax]);
  if (MOVES)
    for (int i = t; i < NS; i += CT) {
      double xn, yn, zn, ru;
      draw_move(s, w, N, sp * NS + i, pos + 3 * (sp * NS + i), s.delta, L, invL, xn, yn, zn, ru);
      prop[4 * i] = xn; prop[4 * i + 1] = yn; prop[4 * i + 2] = zn; prop[4 * i + 3] = ru;
      sincospi(xn * invL, &ptrig[6 * i], &ptrig[6 * i + 3]);
      sincospi(yn * invL, &ptrig[6 * i + 1], &ptrig[6 * i + 4]);
      sincospi(zn * invL, &ptrig[6 * i + 2], &ptrig[6 * i + 5]);
    }
  if (t == 0) flag[0] = 0;
  const double* Bg = a.Binv + 2 * ((size_t)w * 2 + sp) * NS * NS;
  if (!refresh)
    for (int u = t; u < NS * NS; u += CT) st_c(Ai, (u / NS) * LDA + u % NS, ld_c(Bg, u));
  if (refresh == 2)   // X into the proposal-row region (zero outside N_sigma x N_sigma) until the rows are formed
    for (int u = t; u < NSP * NSP; u += CT) {
      const int i = u / NSP, j = u % NSP;
      st_c(Mp, u, (i < NS && j < NS) ? ld_c(Bg, (size_t)i * NS + j) : cd{0.0, 0.0});
    }
  __syncthreads();
  // row tiles [0, TR): the spin's electrons (A, refresh only); [TR, 2 TR): the proposals.  With
  // fewer tiles than waves the centres of a tile are split over CW / (tiles) waves, whose partial
  // products are added into the tile one after another in a fixed order.
  static_assert(2 * TR <= CW, "one tile per wave");
  auto form_rows = [&](const int t0, const int t1) {
    const int nt = t1 - t0;
    const int split = CW / nt, kper = (KS + split - 1) / split;
    const int part = wave / nt, tt = t0 + wave % nt;
    const bool active = part < split;
    const bool isp = tt >= TR;
    const int rt = isp ? tt - TR : tt;
    v4d dr[TC], di[TC];
#pragma unroll
    for (int tc = 0; tc < TC; ++tc) { dr[tc] = v4d{0, 0, 0, 0}; di[tc] = v4d{0, 0, 0, 0}; }
    if (active) {
      const int row = rt * 16 + (lane & 15);
      const bool rok = row < NS;
      const int rr = rok ? row : 0;
      const double* rp = isp ? prop + 4 * rr : pos + 3 * (sp * NS + rr);
      const double rx = rp[0], ry = rp[1], rz = rp[2];
      const int k1 = (part + 1) * kper < KS ? (part + 1) * kper : KS;
      for (int kk = part * kper; kk < k1; ++kk) {
        const int c = kk * 4 + (lane >> 4);
        cd ph = {0.0, 0.0};
        if (rok && c < N) {
          if constexpr (CB) ph = ccontracted_value(rx, ry, rz, a.R + 3 * c, a.eta, L, invL, tw);
          else ph = cphi(rx, ry, rz, a.R + 3 * c, a.zeta[c], L, invL, tw);
        }
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
          const int col = tc * 16 + (lane & 15);
          const cd cv = (c < N && col < NS) ? ld_c(a.C, (size_t)c * NS + col) : cd{0.0, 0.0};
          cmfma(ph, cv, dr[tc], di[tc]);
        }
      }
    }
    double* D = isp ? Mp : Ai;
    const int ldd = isp ? NSP : LDA;
    for (int q = 0; q < split; ++q) {
      if (active && part == q)
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const size_t o = (size_t)(rt * 16 + (lane >> 4) + 4 * v) * ldd + tc * 16 + (lane & 15);
            const cd x = {dr[tc][v], di[tc][v]};
            st_c(D, o, q == 0 ? x : cadd(ld_c(D, o), x));
          }
      __syncthreads();
    }
  };
  // a refinement forms A first and the proposals' rows after it, since X occupies their region
  if (refresh == 2) form_rows(0, TR);
  else if (refresh) form_rows(0, MOVES ? 2 * TR : TR);
  else if (MOVES) form_rows(TR, 2 * TR);
  bool eliminate = refresh == 1;
  if (refresh == 2) {
    // R = I - A X and X' = X + X R on the matrix cores, tile by tile (tiles w, w + CW of wave w),
    // operands read from LDS before every barrier that precedes a write
    constexpr int NT2 = TR * TR, MT = (NT2 + CW - 1) / CW;
    v4d rr[MT], ri[MT];
    double rmax = 0.0;
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const int id = wave + CW * q, tr = id / TR, tc = id % TR;
      rr[q] = v4d{0, 0, 0, 0};
      ri[q] = v4d{0, 0, 0, 0};
      if (id < NT2)
        for (int kk = 0; kk < NSP / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          cmfma(ld_c(Ai, (size_t)(16 * tr + (lane & 15)) * LDA + k), ld_c(Mp, (size_t)k * NSP + 16 * tc + (lane & 15)),
                rr[q], ri[q]);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * tr + (lane >> 4) + 4 * v, col = 16 * tc + (lane & 15);
        const bool ok = id < NT2 && row < NS && col < NS;
        rr[q][v] = ok ? (row == col ? 1.0 : 0.0) - rr[q][v] : 0.0;
        ri[q][v] = ok ? -ri[q][v] : 0.0;
        const double m2 = rr[q][v] * rr[q][v] + ri[q][v] * ri[q][v];
        rmax = (m2 > rmax || m2 != m2) ? m2 : rmax;   // a NaN is kept
      }
    }
    if (rmax != rmax) rmax = INFINITY;
    int dummy = 0;
    wave_argmax(rmax, dummy);
    if (lane == 0) red[wave] = rmax;
    __syncthreads();
    double rm = red[0];
    for (int q = 1; q < CW; ++q) rm = fmax(rm, red[q]);
    eliminate = !(rm <= rtol * rtol);
    if (!eliminate) {
      // R replaces A, then X' = X + X R replaces R
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        const int id = wave + CW * q, tr = id / TR, tc = id % TR;
        if (id < NT2)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            st_c(Ai, (size_t)(16 * tr + (lane >> 4) + 4 * v) * LDA + 16 * tc + (lane & 15), cd{rr[q][v], ri[q][v]});
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        const int id = wave + CW * q, tr = id / TR, tc = id % TR;
        if (id < NT2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const cd x = ld_c(Mp, (size_t)(16 * tr + (lane >> 4) + 4 * v) * NSP + 16 * tc + (lane & 15));
            rr[q][v] = x.r;
            ri[q][v] = x.i;
          }
          for (int kk = 0; kk < NSP / 4; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            cmfma(ld_c(Mp, (size_t)(16 * tr + (lane & 15)) * NSP + k), ld_c(Ai, (size_t)k * LDA + 16 * tc + (lane & 15)),
                  rr[q], ri[q]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        const int id = wave + CW * q, tr = id / TR, tc = id % TR;
        if (id < NT2)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            st_c(Ai, (size_t)(16 * tr + (lane >> 4) + 4 * v) * LDA + 16 * tc + (lane & 15), cd{rr[q][v], ri[q][v]});
      }
      __syncthreads();
    }
    if (MOVES) form_rows(TR, 2 * TR);
  }
  __syncthreads();
  double ldv = 0.0, phv = 0.0;   // meaningful in thread 0
  cd dprod = {1.0, 0.0};
  int dexp = 0, nswap = 0;
  if (eliminate) {
    // Gauss-Jordan elimination with partial pivoting, in place; row swaps are undone on the
    // columns at the end.  A pivot below N_sigma eps max|A_ij| counts as zero: with complex
    // multipliers even two equal rows leave a rounding-sized pivot, not an exact zero.
    {
      double am = 0.0;
      for (int u = t; u < NS * NS; u += CT) {
        const cd v = ld_c(Ai, (size_t)(u / NS) * LDA + u % NS);
        am = fmax(am, v.r * v.r + v.i * v.i);
      }
      int dummy = 0;
      wave_argmax(am, dummy);
      if (lane == 0) red[wave] = am;
      __syncthreads();
    }
    double amax = red[0];
    for (int q = 1; q < CW; ++q) amax = fmax(amax, red[q]);
    const double tol2 = amax * (NS * 2.220446049250313e-16) * (NS * 2.220446049250313e-16);
    for (int p = 0; p < NS; ++p) {
      if (wave == 0) {
        double mag = -1.0;
        int idx = lane;
        if (lane >= p && lane < NS) {
          const cd v = ld_c(Ai, (size_t)lane * LDA + p);
          mag = v.r * v.r + v.i * v.i;
        }
        wave_argmax(mag, idx);
        if (lane == 0) {
          perm[p] = idx;
          if (!(mag > tol2) || !isfinite(mag)) flag[0] = 1;
          // the pivot value, read by every thread before the row swap below moves it
          const cd v = ld_c(Ai, (size_t)idx * LDA + p);
          red[8] = v.r;
          red[9] = v.i;
        }
      }
      __syncthreads();
      if (flag[0]) break;
      const int r = perm[p];
      const cd pv = {red[8], red[9]};
      const double m2 = pv.r * pv.r + pv.i * pv.i;
      const cd ip = {pv.r / m2, -pv.i / m2};
      for (int j = t; j < NS; j += CT) {
        const cd x = ld_c(Ai, (size_t)p * LDA + j), y = ld_c(Ai, (size_t)r * LDA + j);
        st_c(Ai, (size_t)p * LDA + j, y);
        st_c(Ai, (size_t)r * LDA + j, x);
        st_c(prow, j, cmul(j == p ? cd{1.0, 0.0} : y, ip));
        if (j == p) { st_c(fcol, r, x); st_c(fcol, p, y); }
      }
      for (int i = t; i < NS; i += CT)
        if (i != p && i != r) st_c(fcol, i, ld_c(Ai, (size_t)i * LDA + p));
      __syncthreads();
      if (t < RPT * NS) {
        const int j = t % NS;
        const cd pj = ld_c(prow, j);
        for (int i = t / NS; i < NS; i += RPT) {
          cd v;
          if (i == p) {
            v = pj;
          } else {
            const cd x = (j == p) ? cd{0.0, 0.0} : ld_c(Ai, (size_t)i * LDA + j);
            v = csub(x, cmul(ld_c(fcol, i), pj));
          }
          st_c(Ai, (size_t)i * LDA + j, v);
        }
      }
      if (t == 0) {
        // the pivots' product as a mantissa and a power of two (its logarithm and angle once at
        // the end), and the row swaps, each a factor -1
        dprod = cmul(dprod, pv);
        int ex;
        (void)frexp(fmax(fabs(dprod.r), fabs(dprod.i)), &ex);
        dprod = {ldexp(dprod.r, -ex), ldexp(dprod.i, -ex)};
        dexp += ex;
        nswap += r != p ? 1 : 0;
      }
      __syncthreads();
    }
    if (t == 0) {
      ldv = 0.5 * log(dprod.r * dprod.r + dprod.i * dprod.i) + dexp * 0.69314718055994530942;
      phv = atan2(dprod.i, dprod.r) + (nswap & 1 ? VMC_PI : 0.0);
    }
    if (flag[0]) {
      if (t == 0) atomicExch(a.status, 1);
      return;
    }
    for (int i = t; i < NS; i += CT)
      for (int p = NS - 1; p >= 0; --p) {
        const int r = perm[p];
        if (r != p) {
          const cd x = ld_c(Ai, (size_t)i * LDA + p), y = ld_c(Ai, (size_t)i * LDA + r);
          st_c(Ai, (size_t)i * LDA + p, y);
          st_c(Ai, (size_t)i * LDA + r, x);
        }
      }
    __syncthreads();
  } else if (t == 0) {
    ldv = a.ldet[(size_t)w * 2 + sp];
    phv = a.sgn[(size_t)w * 2 + sp];
  }
  int64_t nadd = 0;
  // product of the accepted ratios (thread 0), kept as a complex mantissa and a power of two so
  // that the moves need no logarithm or angle; folded into ldet and the phase at the end
  cd qprod = {1.0, 0.0};
  int qexp = 0;
  if constexpr (MOVES) {
    // The moves in blocks of 16, as in the real half-sweep: the block's row products
    // P = M'[block] A^-1 on the matrix cores (waves tc < TC, column tile tc), then wave 0 alone runs
    // the 16 moves in order with no barrier: move j takes t = P_j after the accepted moves j' < j
    // of the block by the left-looking recursion t -= t[i_j'] z_j' (z_j' = (t_j' - e_i_j') / q_j'),
    // its ratio q_j = t[i_j] and its Jastrow change; after the block Z = (I + Y)^-1 [z
    // rows] by back-substitution (Y[j][j''] = z_j[i_j''], j'' > j) and every wave updates its
    // tiles of A^-1 -= A^-1[:, block] Z on the matrix cores.  P and then Z overwrite the block's
    // orbital rows, which nothing reads again.
    constexpr int EPL = (N + 63) / 64, NBK = NSP / 16, NTILE = TR * TC, MAXT = (NTILE + CW - 1) / CW;
    static_assert(NSP <= 64, "one recursion column per lane");
    const double LoP = L / VMC_PI, bj = a.b;
    const bool one_body = a.j1_beta > 0.0;
    double* D1 = fcol;   // one-body change of each move
    // A move's one-body change depends on its own electron and the protons only, so all of them
    // are formed first: move i by the eight threads 8 i .. 8 i + 7, each over the protons
    // c = t mod 8 (mod 8), combined by lane exchanges in a fixed order.
    if (one_body) {
      for (int i0 = 0; i0 < NSP; i0 += CT / 8) {
        const int i = i0 + (t >> 3);
        double acc = 0.0;
        if (i < NS) {
          const double* to = trig + 6 * (sp * NS + i);
          const double* tn = ptrig + 6 * i;
          const double so[3] = {to[0], to[1], to[2]}, co[3] = {to[3], to[4], to[5]};
          const double sn[3] = {tn[0], tn[1], tn[2]}, cn[3] = {tn[3], tn[4], tn[5]};
          for (int c = t & 7; c < N; c += 8) {
            const double* tp = ptab + 6 * c;
            const double sc[3] = {tp[0], tp[1], tp[2]}, cc[3] = {tp[3], tp[4], tp[5]};
            acc += one_body_exp<double>(sn, cn, sc, cc, LoP, a.j1_beta) -
                   one_body_exp<double>(so, co, sc, cc, LoP, a.j1_beta);
          }
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 4, 64);
        if ((t & 7) == 0 && i < NS) D1[i] = acc / a.j1_beta;
      }
    }
    // The pair terms of a move are staged per block by all threads: with the electrons where the
    // block starts, base_j = sum_{jj != e_j} u(r'_j, r_jj) - u(r_j, r_jj) (move j by the 32 threads
    // 32 j .. 32 j + 31, each over the electrons jj = t mod 32 (mod 32), combined by lane
    // exchanges in a fixed order), and for two moves j' < j of the block the correction
    // X[j][j'] = [u(r'_j, r'_j') - u(r_j, r'_j')] - [u(r'_j, r_j') - u(r_j, r_j')] that applies
    // once move j' is accepted.  The electrons' sines and cosines in LDS follow the accepted moves.
    constexpr int JB = NS < 16 ? NS : 16;
    static_assert(6 * N + JB * JB <= 2 * P * NSP, "the proton table and the pair corrections fit");
    double* Xc = ptab + 6 * N;   // JB x JB pair corrections
    double* base = colI;         // 16 staged pair changes
    // wave 0's state for the moves: lane l keeps protons l, l + 64 (their sines and cosines) and
    // the three-body sums G of nuclei l, l + 64
    double sa[EPL][3], ca[EPL][3], Gj[EPL][2];
    if (wave == 0) {
#pragma unroll
      for (int tt = 0; tt < EPL; ++tt) {
        const int c = lane + 64 * tt;
        const bool ok = c < N;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          sa[tt][m] = (ok && (one_body || a.j3)) ? ptab[6 * c + m] : 0.0;
          ca[tt][m] = (ok && (one_body || a.j3)) ? ptab[6 * c + 3 + m] : 1.0;
        }
        Gj[tt][0] = (ok && a.j3) ? a.j3G[((size_t)w * N + c) * 2] : 0.0;
        Gj[tt][1] = (ok && a.j3) ? a.j3G[((size_t)w * N + c) * 2 + 1] : 0.0;
      }
    }
    __syncthreads();
    for (int b = 0; b < NBK; ++b) {
      const int jmax = NS - 16 * b < 16 ? NS - 16 * b : 16;
      double* PB = Mp + 2 * (size_t)16 * b * NSP;   // 16 x NSP complex: M'[block], then P, then z / Z
      {
        v4d pr = {0.0, 0.0, 0.0, 0.0}, pim = {0.0, 0.0, 0.0, 0.0};
        if (wave < TC) {
          const int col = 16 * wave + (lane & 15);
          for (int kk = 0; kk < NSP / 4; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            const cd av = ld_c(PB, (size_t)(lane & 15) * NSP + k);
            const cd bv = (k < NS && col < NS) ? ld_c(Ai, (size_t)k * LDA + col) : cd{0.0, 0.0};
            cmfma(av, bv, pr, pim);
          }
        }
        {
          const int j = t >> 5;
          double acc = 0.0;
          if (j < jmax) {
            const int e = sp * NS + 16 * b + j;
            const double* to = trig + 6 * e;
            const double* tn = ptrig + 6 * (16 * b + j);
            const double so[3] = {to[0], to[1], to[2]}, co[3] = {to[3], to[4], to[5]};
            const double sn[3] = {tn[0], tn[1], tn[2]}, cn[3] = {tn[3], tn[4], tn[5]};
            for (int jj = t & 31; jj < N; jj += 32) {
              if (jj == e) continue;
              const double* tj = trig + 6 * jj;
              const double sj[3] = {tj[0], tj[1], tj[2]}, cj[3] = {tj[3], tj[4], tj[5]};
              const double aa = (jj / NS == sp) ? a.a_par : a.a_anti;
              acc += pade_u<double>(sn, cn, sj, cj, LoP, aa, bj) - pade_u<double>(so, co, sj, cj, LoP, aa, bj);
            }
          }
          acc += __shfl_xor(acc, 16, 64);
          acc += __shfl_xor(acc, 8, 64);
          acc += __shfl_xor(acc, 4, 64);
          acc += __shfl_xor(acc, 2, 64);
          acc += __shfl_xor(acc, 1, 64);
          if ((t & 31) == 0 && j < jmax) base[j] = acc;
          const int jx = t >> 4, jp = t & 15;
          if (t < 256 && jp < jx && jx < jmax) {
            const double* to = trig + 6 * (sp * NS + 16 * b + jx);
            const double* tn = ptrig + 6 * (16 * b + jx);
            const double* po = trig + 6 * (sp * NS + 16 * b + jp);
            const double* pn = ptrig + 6 * (16 * b + jp);
            const double so[3] = {to[0], to[1], to[2]}, co[3] = {to[3], to[4], to[5]};
            const double sn[3] = {tn[0], tn[1], tn[2]}, cn[3] = {tn[3], tn[4], tn[5]};
            const double qo[3] = {po[0], po[1], po[2]}, ko[3] = {po[3], po[4], po[5]};
            const double qn[3] = {pn[0], pn[1], pn[2]}, kn[3] = {pn[3], pn[4], pn[5]};
            const double ap = a.a_par;
            Xc[jx * JB + jp] = (pade_u<double>(sn, cn, qn, kn, LoP, ap, bj) - pade_u<double>(so, co, qn, kn, LoP, ap, bj)) -
                               (pade_u<double>(sn, cn, qo, ko, LoP, ap, bj) - pade_u<double>(so, co, qo, ko, LoP, ap, bj));
          }
        }
        __syncthreads();
        if (wave < TC)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            st_c(PB, (size_t)((lane >> 4) + 4 * v) * NSP + 16 * wave + (lane & 15), cd{pr[v], pim[v]});
        __syncthreads();
      }
      if (wave == 0) {
        uint32_t amask = 0;
        for (int j = 0; j < jmax; ++j) {
          const int i = 16 * b + j, e = sp * NS + i;
          cd tv = lane < NSP ? ld_c(PB, (size_t)j * NSP + lane) : cd{0.0, 0.0};
          // the Jastrow change: the staged pair change with the corrections of the block's
          // accepted moves, the three-body term on the lane's nuclei,
          // (chi(r') - chi(r))^T F (G - chi(r)), and the staged one-body change
          const double* to = trig + 6 * e;
          const double* tn = ptrig + 6 * i;
          const double so[3] = {to[0], to[1], to[2]}, co[3] = {to[3], to[4], to[5]};
          const double sn[3] = {tn[0], tn[1], tn[2]}, cn[3] = {tn[3], tn[4], tn[5]};
          double du = (lane < JB && ((amask >> lane) & 1u)) ? Xc[j * JB + lane] : 0.0, dj[EPL][2];
#pragma unroll
          for (int tt = 0; tt < EPL; ++tt) {
            const int jj = lane + 64 * tt;
            dj[tt][0] = dj[tt][1] = 0.0;
            if (a.j3 && jj < N) {
              double n1, n2, o1, o2;
              j3_values<double>(sn, cn, sa[tt], ca[tt], LoP, n1, n2);
              j3_values<double>(so, co, sa[tt], ca[tt], LoP, o1, o2);
              dj[tt][0] = n1 - o1;
              dj[tt][1] = n2 - o2;
              const double g1 = Gj[tt][0] - o1, g2 = Gj[tt][1] - o2;
              du += a.j3f[0] * dj[tt][0] * g1 + a.j3f[1] * (dj[tt][0] * g2 + dj[tt][1] * g1) +
                    a.j3f[2] * dj[tt][1] * g2;
              du += a.j1f[0] * dj[tt][0] + a.j1f[1] * dj[tt][1];   // the one-body orbital part
            }
          }
          double dU = base[j] + wave_allsum(du);
          if (one_body) dU += D1[i];
          for (uint32_t mm = amask; mm; mm &= mm - 1) {
            const int jp = __builtin_ctz(mm);
            const cd cf = {readlane_d(tv.r, 16 * b + jp), readlane_d(tv.i, 16 * b + jp)};
            const cd z = lane < NSP ? ld_c(PB, (size_t)jp * NSP + lane) : cd{0.0, 0.0};
            tv = csub(tv, cmul(cf, z));
          }
          const cd q = {readlane_d(tv.r, i), readlane_d(tv.i, i)};
          const double q2 = q.r * q.r + q.i * q.i;
          const double pacc = q2 * exp(2.0 * dU);
          cd zrow = {0.0, 0.0};
          if (prop[4 * i + 3] < pacc) {
            const double iq2 = 1.0 / q2;
            const cd iq = {q.r * iq2, -q.i * iq2};
            cd vj = tv;
            if (lane == i) vj.r -= 1.0;
            zrow = cmul(vj, iq);
            amask |= 1u << j;
#pragma unroll
            for (int tt = 0; tt < EPL; ++tt) {
              Gj[tt][0] += dj[tt][0];
              Gj[tt][1] += dj[tt][1];
            }
            if (lane < 3) pos[3 * e + lane] = prop[4 * i + lane];
            if (lane < 6) trig[6 * e + lane] = tn[lane];
            ++nadd;
            qprod = cmul(qprod, q);
            int ex;
            (void)frexp(fmax(fabs(qprod.r), fabs(qprod.i)), &ex);
            qprod = {ldexp(qprod.r, -ex), ldexp(qprod.i, -ex)};
            qexp += ex;
          }
          if (lane < NSP) st_c(PB, (size_t)j * NSP + lane, zrow);
          wave_lds_sync();
        }
        // Z = (I + Y)^-1 [z rows]: back-substitution from the last accepted move
        for (int j = 15; j >= 0; --j) {
          if (!((amask >> j) & 1u)) continue;
          const cd zo = lane < NSP ? ld_c(PB, (size_t)j * NSP + lane) : cd{0.0, 0.0};
          cd z = zo;
          for (uint32_t mm = amask & ~((2u << j) - 1u); mm; mm &= mm - 1) {
            const int jp = __builtin_ctz(mm);
            const cd cf = {readlane_d(zo.r, 16 * b + jp), readlane_d(zo.i, 16 * b + jp)};
            const cd zp = lane < NSP ? ld_c(PB, (size_t)jp * NSP + lane) : cd{0.0, 0.0};
            z = csub(z, cmul(cf, zp));
          }
          if (lane < NSP) st_c(PB, (size_t)j * NSP + lane, z);
          wave_lds_sync();
        }
        if (lane == 0) flag[1] = (int)amask;
      }
      __syncthreads();
      if (flag[1]) {
        // A^-1 -= A^-1[:, block] Z, tile by tile: every wave reads its tiles, the (negated) block
        // columns and Z first, and writes only after the barrier, since the block's column tile is
        // both read and updated
        v4d cr[MAXT], ci[MAXT];
        cd ga[MAXT][4], zb[MAXT][4];
#pragma unroll
        for (int r = 0; r < MAXT; ++r) {
          const int id = wave + CW * r;
          const int tr = id / TC, tc = id % TC;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * tr + (lane >> 4) + 4 * v, col = 16 * tc + (lane & 15);
            const cd c = (id < NTILE && row < NS && col < NS) ? ld_c(Ai, (size_t)row * LDA + col) : cd{0.0, 0.0};
            cr[r][v] = c.r;
            ci[r][v] = c.i;
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int grow = 16 * tr + (lane & 15), gcol = 16 * b + 4 * kk + (lane >> 4);
            const cd g = (id < NTILE && grow < NS && gcol < NS) ? ld_c(Ai, (size_t)grow * LDA + gcol) : cd{0.0, 0.0};
            ga[r][kk] = {-g.r, -g.i};
            zb[r][kk] = id < NTILE ? ld_c(PB, (size_t)(4 * kk + (lane >> 4)) * NSP + 16 * tc + (lane & 15))
                                   : cd{0.0, 0.0};
          }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < MAXT; ++r) {
          const int id = wave + CW * r;
          if (id >= NTILE) continue;
          const int tr = id / TC, tc = id % TC;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) cmfma(ga[r][kk], zb[r][kk], cr[r], ci[r]);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * tr + (lane >> 4) + 4 * v, col = 16 * tc + (lane & 15);
            if (row < NS && col < NS) st_c(Ai, (size_t)row * LDA + col, cd{cr[r][v], ci[r][v]});
          }
        }
      }
      __syncthreads();
    }
    if (wave == 0 && a.j3)
#pragma unroll
      for (int tt = 0; tt < EPL; ++tt) {
        const int c = lane + 64 * tt;
        if (c < N) {
          a.j3G[((size_t)w * N + c) * 2] = Gj[tt][0];
          a.j3G[((size_t)w * N + c) * 2 + 1] = Gj[tt][1];
        }
      }
  }
  double* Bo = a.Binv + 2 * ((size_t)w * 2 + sp) * NS * NS;
  for (int u = t; u < NS * NS; u += CT) st_c(Bo, u, ld_c(Ai, (size_t)(u / NS) * LDA + u % NS));
  if (MOVES)
    for (int u = t; u < 3 * NS; u += CT) a.pos[(size_t)w * 3 * N + 3 * sp * NS + u] = pos[3 * sp * NS + u];
  if (t == 0) {
    if (MOVES && nadd > 0) {
      ldv += 0.5 * log(qprod.r * qprod.r + qprod.i * qprod.i) + qexp * 0.69314718055994530942;
      phv += atan2(qprod.i, qprod.r);
    }
    a.ldet[(size_t)w * 2 + sp] = ldv;
    a.sgn[(size_t)w * 2 + sp] = remainder(phv, 2.0 * VMC_PI);
    if (MOVES) a.nacc[w] += nadd;
  }
}

// ------------------------------------------------------------ measurement ---
template <int NS>
struct CSlaterLay {
  static constexpr int N = 2 * NS, NSP = (NS + 15) / 16 * 16, NP = (N + 15) / 16 * 16;
  // per-walker scratch (complex elements): B = C A^-1 (NP x NSP), X (NSP x NP), M = X B (NSP x NSP),
  // W = B M (NP x NSP)
  static constexpr size_t b = 0, x = b + (size_t)NP * NSP, mm = x + (size_t)NSP * NP, wm = mm + (size_t)NSP * NSP,
                          scr_elems = wm + (size_t)NP * NSP;
  static constexpr int H = 256 / N;          // threads per centre in the pair passes
  static constexpr int HJ = H > 0 ? H : 1;   // threads per electron in the Jastrow pass
  // LDS (doubles)
  static constexpr size_t pos = 0, gU = pos + 3 * N, lU = gU + 3 * N, trig = lU + N, part = trig + 6 * N,
                          partn = (size_t)(HJ * N * 5 > 256 * 6 ? HJ * N * 5 : 256 * 6), red = part + partn,
                          gd = red + 8, bytes = sizeof(double) * (gd + 3 * N);
  // the partial sums of Re grad ln D (256 / NS shares x NS x 3) reuse the pair-pass region
  static_assert((256 / NS) * NS * 3 <= (int)partn, "partial sums of grad ln D exceed their region");
};

// D (TRr*16 x TCc*16) = A (x K) B (K x), complex, row-major with leading dimensions in complex
// elements; A outside rows [0, MA) or columns [0, KA), and B outside rows [0, KA) or columns
// [0, NB), read as zero.  Wave w computes the output tiles w, w + 4, ...; all 64 lanes of a
// wave run every matrix-core step.
template <int TRr, int TCc, int KA>
__device__ __forceinline__ void cgemm(const double* A, int lda, int MA, const double* B, int ldb, int NB, double* D,
                                      int ldd, int wave, int lane) {
  constexpr int K4 = (KA + 3) / 4;
  for (int tt = wave; tt < TRr * TCc; tt += 4) {
    const int tr = tt / TCc, tc = tt % TCc;
    const int arow = tr * 16 + (lane & 15), bcol = tc * 16 + (lane & 15);
    v4d dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
    for (int kk = 0; kk < K4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      const cd av = (arow < MA && k < KA) ? ld_c(A, (size_t)arow * lda + k) : cd{0.0, 0.0};
      const cd bv = (k < KA && bcol < NB) ? ld_c(B, (size_t)k * ldb + bcol) : cd{0.0, 0.0};
      cmfma(av, bv, dr, di);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) st_c(D, (size_t)(tr * 16 + (lane >> 4) + 4 * v) * ldd + bcol, cd{dr[v], di[v]});
  }
}

// Per walker (one 256-thread block): the Jastrow gradient and Laplacian per electron, then per
// spin B = C A^-1, the basis pass that forms X and the terms needing only B, M = X B, W = B M and
// the pass that adds grad phi W; the four products on the FP64 matrix cores through the
// walker's scratch.
//   Re T_L = Re sum X_ia B_ai - 1/2 sum_i (lap_i U + |grad_i U|^2),  X_ia = -1/2 [lap phi_a + 2 grad phi_a . grad_i U]
//   d ln|psi|/dR_b = -Re sum_i B_bi grad phi_b(r_i)
//   d Re T_L/dR_b = Re sum_i [1/2 (grad lap phi_b + 2 Hess phi_b . grad_i U) B_bi + grad phi_b(r_i) W_bi]
// Two work-groups per CU for the single Gaussian (a few registers spill), so that measurements of
// twists on other streams share a CU; the contracted basis needs one CU's registers per walker.
template <int NS, bool CB>
__global__ __launch_bounds__(256, CB ? 1 : 2) void k_cslater_sample(MeasureArgs m, TwistArgs tw) {
  using LY = CSlaterLay<NS>;
  constexpr int N = 2 * NS, NSP = LY::NSP, NP = LY::NP, H = LY::H, HJ = LY::HJ;
  constexpr int NT = H * N, IPT = (NS + H - 1) / H;
  extern __shared__ __align__(16) double smem[];
  double* pos = smem + LY::pos;
  double* gU = smem + LY::gU;
  double* lU = smem + LY::lU;
  double* trig = smem + LY::trig;
  double* part = smem + LY::part;
  double* red = smem + LY::red;
  double* gd = smem + LY::gd;        // N x 3: Re grad ln D per electron (one- and three-body terms)
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int w = blockIdx.x;
  const double L = m.L, invL = m.invL;
  const bool one_body = m.j1_beta > 0.0;
  double* scr = reinterpret_cast<double*>(m.scr + (size_t)w * 16 * LY::scr_elems);
  double* Bs = scr + 2 * LY::b;
  double* Xs = scr + 2 * LY::x;
  double* Ms = scr + 2 * LY::mm;
  double* Ws = scr + 2 * LY::wm;
  for (int u = t; u < 3 * N; u += 256) pos[u] = m.pos[(size_t)w * 3 * N + u];
  __syncthreads();
  for (int e = t; e < N; e += 256)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) sincospi(pos[3 * e + ax] * invL, &trig[6 * e + ax], &trig[6 * e + 3 + ax]);
  __syncthreads();
  // Jastrow: HJ threads share an electron's pairs, combined in a fixed order
  double tj = 0.0, usum = 0.0;
  {
    const double LoP = L / VMC_PI, kf = (VMC_PI * invL) * (VMC_PI * invL);
    for (int u = t; u < HJ * N; u += 256) {
      const int i = u % N, hj = u / N;
      const int j0 = hj * N / HJ, j1 = (hj + 1) * N / HJ;
      double g0 = 0, g1 = 0, g2 = 0, lp = 0, ui = 0;
      const double* ti = trig + 6 * i;
      for (int j = j0; j < j1; ++j) {
        if (j == i) continue;
        const double* tq = trig + 6 * j;
        double rt[3], cc[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          rt[ax] = LoP * (ti[ax] * tq[3 + ax] - ti[3 + ax] * tq[ax]);
          cc[ax] = ti[3 + ax] * tq[3 + ax] + ti[ax] * tq[ax];
        }
        const double r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
        const double rho = sqrt(r2), irho = 1.0 / rho;
        const double aj = ((i / NS) == (j / NS)) ? m.a_par : m.a_anti;
        const double iden = 1.0 / (1.0 + m.b * rho);
        const double up = aj * iden * iden, upp = -2.0 * aj * m.b * iden * iden * iden;
        const double gr0 = rt[0] * cc[0] * irho, gr1 = rt[1] * cc[1] * irho, gr2 = rt[2] * cc[2] * irho;
        const double gg = gr0 * gr0 + gr1 * gr1 + gr2 * gr2;
        const double lr = (cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2] - kf * r2) * irho - gg * irho;
        g0 += up * gr0; g1 += up * gr1; g2 += up * gr2;
        lp += upp * gg + up * lr;
        if (j > i) ui += aj * rho * iden;
      }
      if (one_body) {
        // the one-body term f(rho) = -(1 - e^{-beta rho}) / beta of electron i and this thread's
        // share of the protons: f' = -e^{-beta rho}, f'' = beta e^{-beta rho}; the sum of f as
        // (sum e^{-beta rho} - count) / beta
        const double beta = m.j1_beta;
        double sx = 0.0;
        for (int c = j0; c < j1; ++c) {
          double rt[3], cc[3];
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            double sc, cs;
            sincospi(min_image(pos[3 * i + ax] - m.R[3 * c + ax], L, invL) * invL, &sc, &cs);
            rt[ax] = LoP * sc;
            cc[ax] = cs;
          }
          const double r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
          const double rho = sqrt(r2), irho = 1.0 / rho;
          const double ex = exp(-beta * rho);
          const double gr0 = rt[0] * cc[0] * irho, gr1 = rt[1] * cc[1] * irho, gr2 = rt[2] * cc[2] * irho;
          const double gg = gr0 * gr0 + gr1 * gr1 + gr2 * gr2;
          const double lr = (cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2] - kf * r2) * irho - gg * irho;
          g0 -= ex * gr0; g1 -= ex * gr1; g2 -= ex * gr2;
          lp += beta * ex * gg - ex * lr;
          sx += ex;
        }
        ui += (sx - (double)(j1 - j0)) / beta;
      }
      double* q = part + ((size_t)hj * N + i) * 5;
      q[0] = g0; q[1] = g1; q[2] = g2; q[3] = lp; q[4] = ui;
    }
    __syncthreads();
    // the three-body term's gradient, Laplacian and value, from the pass before this kernel
    const double* j3in = m.j3 ? m.j3scr + (size_t)w * j3_measure_doubles(N) : nullptr;
    for (int i = t; i < N; i += 256) {
      double g0 = 0, g1 = 0, g2 = 0, lp = 0, ui = 0;
      for (int hj = 0; hj < HJ; ++hj) {
        const double* q = part + ((size_t)hj * N + i) * 5;
        g0 += q[0]; g1 += q[1]; g2 += q[2]; lp += q[3]; ui += q[4];
      }
      if (j3in) {
        g0 += j3in[3 * i]; g1 += j3in[3 * i + 1]; g2 += j3in[3 * i + 2];
        lp += j3in[3 * N + i];
        if (i == 0) ui += j3in[4 * N];
      }
      gU[3 * i] = g0; gU[3 * i + 1] = g1; gU[3 * i + 2] = g2;
      lU[i] = lp;
      tj += -0.5 * (lp + g0 * g0 + g1 * g1 + g2 * g2);
      usum += ui;
    }
  }
  __syncthreads();
  const int ca = t % N, h = t / N;
  const bool act = t < NT;
  double dln0 = 0, dln1 = 0, dln2 = 0, dT0 = 0, dT1 = 0, dT2 = 0, tsl = 0;
  const double Ra0 = m.R[3 * ca], Ra1 = m.R[3 * ca + 1], Ra2 = m.R[3 * ca + 2];
  const double za = m.zeta[ca];
  for (int sp = 0; sp < 2; ++sp) {
    const double* Bi = m.Binv + 2 * ((size_t)w * 2 + sp) * NS * NS;
    // B = C A^-1 (NP x NSP; K = orbitals)
    cgemm<NP / 16, NSP / 16, NS>(m.C, NS, N, Bi, NS, NS, Bs, NSP, wave, lane);
    // the padding of X stays zero
    for (int u = t; u < NSP * NP; u += 256) {
      const int i = u / NP, c = u % NP;
      if (i >= NS || c >= N) st_c(Xs, u, cd{0.0, 0.0});
    }
    __syncthreads();
    if (one_body || m.j3) {
      // Re grad_i ln D = Re sum_a grad phi_a(r_i) B_ai for the electrons of this spin, in HG
      // shares of the centres, combined in a fixed order
      constexpr int HG = 256 / NS;
      double* gp = part;
      for (int u = t; u < HG * NS; u += 256) {
        const int i = u % NS, hg = u / NS, e = sp * NS + i;
        const int c0 = hg * N / HG, c1 = (hg + 1) * N / HG;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int c = c0; c < c1; ++c) {
          const cd b = ld_c(Bs, (size_t)c * NSP + i);
          if constexpr (CB) {
            const CBasisD q = ccontracted_derivs<false>(pos[3 * e] - m.R[3 * c], pos[3 * e + 1] - m.R[3 * c + 1],
                                                        pos[3 * e + 2] - m.R[3 * c + 2], m.eta, L, invL, tw);
            s0 += remul(b, q.gx);
            s1 += remul(b, q.gy);
            s2 += remul(b, q.gz);
          } else {
            cd g[3][4];
            cbasis_axis<1>(pos[3 * e] - m.R[3 * c], m.zeta[c], L, invL, tw, 0, g[0]);
            cbasis_axis<1>(pos[3 * e + 1] - m.R[3 * c + 1], m.zeta[c], L, invL, tw, 1, g[1]);
            cbasis_axis<1>(pos[3 * e + 2] - m.R[3 * c + 2], m.zeta[c], L, invL, tw, 2, g[2]);
            s0 += remul(b, cmul(cmul(g[0][1], g[1][0]), g[2][0]));
            s1 += remul(b, cmul(cmul(g[0][0], g[1][1]), g[2][0]));
            s2 += remul(b, cmul(cmul(g[0][0], g[1][0]), g[2][1]));
          }
        }
        gp[3 * u] = s0; gp[3 * u + 1] = s1; gp[3 * u + 2] = s2;
      }
      __syncthreads();
      for (int u = t; u < 3 * NS; u += 256) {
        const int i = u / 3, c = u % 3;
        double sg = 0.0;
        for (int hg = 0; hg < HG; ++hg) sg += gp[3 * (hg * NS + i) + c];
        gd[3 * (sp * NS + i) + c] = sg;
      }
      __syncthreads();
    }
    // pass 1: basis derivatives -> X, and the terms that need only B
    if (act) {
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const int e = sp * NS + i;
        cd gx, gy, gz, hxx, hyy, hzz, hxy, hxz, hyz, glx, gly, glz;
        if constexpr (CB) {
          const CBasisD q = ccontracted_derivs<true>(pos[3 * e] - Ra0, pos[3 * e + 1] - Ra1, pos[3 * e + 2] - Ra2, m.eta,
                                                     L, invL, tw);
          gx = q.gx; gy = q.gy; gz = q.gz;
          hxx = q.hxx; hyy = q.hyy; hzz = q.hzz; hxy = q.hxy; hxz = q.hxz; hyz = q.hyz;
          glx = q.glx; gly = q.gly; glz = q.glz;
        } else {
          cd g[3][4];
          cbasis_axis<3>(pos[3 * e] - Ra0, za, L, invL, tw, 0, g[0]);
          cbasis_axis<3>(pos[3 * e + 1] - Ra1, za, L, invL, tw, 1, g[1]);
          cbasis_axis<3>(pos[3 * e + 2] - Ra2, za, L, invL, tw, 2, g[2]);
          const cd p00 = cmul(g[1][0], g[2][0]), p01 = cmul(g[0][0], g[2][0]), p02 = cmul(g[0][0], g[1][0]);
          gx = cmul(g[0][1], p00); gy = cmul(g[1][1], p01); gz = cmul(g[2][1], p02);
          hxx = cmul(g[0][2], p00); hyy = cmul(g[1][2], p01); hzz = cmul(g[2][2], p02);
          hxy = cmul(cmul(g[0][1], g[1][1]), g[2][0]); hxz = cmul(cmul(g[0][1], g[1][0]), g[2][1]);
          hyz = cmul(cmul(g[0][0], g[1][1]), g[2][1]);
          glx = cadd(cmul(g[0][3], p00), cmul(g[0][1], cadd(cmul(g[1][2], g[2][0]), cmul(g[1][0], g[2][2]))));
          gly = cadd(cmul(g[1][3], p01), cmul(g[1][1], cadd(cmul(g[0][2], g[2][0]), cmul(g[0][0], g[2][2]))));
          glz = cadd(cmul(g[2][3], p02), cmul(g[2][1], cadd(cmul(g[0][2], g[1][0]), cmul(g[0][0], g[1][2]))));
        }
        const cd lap = cadd(cadd(hxx, hyy), hzz);
        const double u0 = gU[3 * e], u1 = gU[3 * e + 1], u2 = gU[3 * e + 2];
        const cd X = {-0.5 * (lap.r + 2.0 * (gx.r * u0 + gy.r * u1 + gz.r * u2)),
                      -0.5 * (lap.i + 2.0 * (gx.i * u0 + gy.i * u1 + gz.i * u2))};
        st_c(Xs, (size_t)i * NP + ca, X);
        const cd b = ld_c(Bs, (size_t)ca * NSP + i);
        tsl += remul(X, b);
        dln0 -= remul(b, gx); dln1 -= remul(b, gy); dln2 -= remul(b, gz);
        const cd q0 = {0.5 * glx.r + hxx.r * u0 + hxy.r * u1 + hxz.r * u2, 0.5 * glx.i + hxx.i * u0 + hxy.i * u1 + hxz.i * u2};
        const cd q1 = {0.5 * gly.r + hxy.r * u0 + hyy.r * u1 + hyz.r * u2, 0.5 * gly.i + hxy.i * u0 + hyy.i * u1 + hyz.i * u2};
        const cd q2 = {0.5 * glz.r + hxz.r * u0 + hyz.r * u1 + hzz.r * u2, 0.5 * glz.i + hxz.i * u0 + hyz.i * u1 + hzz.i * u2};
        dT0 += remul(q0, b); dT1 += remul(q1, b); dT2 += remul(q2, b);
      }
    }
    if (one_body && act) {
      // the one-body term of proton ca at electron e moves with R_ca (d/dR = -grad_e):
      // d ln|psi|/dR -= F1 g, dT/dR += grad(lap f)/2 + hess f (grad U + Re grad ln D), with the
      // radial derivatives F1 = -x, F2 = beta x, F3 = -beta^2 x (x = e^{-beta rho}), g = grad rho,
      // p_m = c_m^2 - (pi/L)^2 rt_m^2, G = |g|^2, P = sum p_m,
      // hess f = (F2 - F1/rho) g g^T + (F1/rho) diag(p),
      // grad lap f = F3 G g + F2 (dG + (P - G) g / rho) + F1 ((dP - dG) / rho - (P - G) g / rho^2),
      // dG = 2 g (p - G) / rho, dP = -4 (pi/L)^2 rho g
      const double LoP1 = L / VMC_PI, kf1 = (VMC_PI * invL) * (VMC_PI * invL), beta1 = m.j1_beta;
      const double Ra[3] = {Ra0, Ra1, Ra2};
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const int e = sp * NS + i;
        double rt[3], cc[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          double sc, cs;
          sincospi(min_image(pos[3 * e + ax] - Ra[ax], L, invL) * invL, &sc, &cs);
          rt[ax] = LoP1 * sc;
          cc[ax] = cs;
        }
        const double r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
        const double rho = sqrt(r2), irho = 1.0 / rho;
        const double x = exp(-beta1 * rho);
        const double F1 = -x, F2 = beta1 * x, F3 = -beta1 * beta1 * x;
        double g_[3], p_[3], v_[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          g_[ax] = rt[ax] * cc[ax] * irho;
          p_[ax] = cc[ax] * cc[ax] - kf1 * rt[ax] * rt[ax];
          v_[ax] = gU[3 * e + ax] + gd[3 * e + ax];
        }
        const double G = g_[0] * g_[0] + g_[1] * g_[1] + g_[2] * g_[2];
        const double P = p_[0] + p_[1] + p_[2];
        const double gv = g_[0] * v_[0] + g_[1] * v_[1] + g_[2] * v_[2];
        const double ha = (F2 - F1 * irho) * gv, hb = F1 * irho, PG = (P - G) * irho;
        double o[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const double dG = 2.0 * g_[ax] * (p_[ax] - G) * irho, dP = -4.0 * kf1 * rho * g_[ax];
          const double glap = F3 * G * g_[ax] + F2 * (dG + PG * g_[ax]) + F1 * ((dP - dG) - PG * g_[ax]) * irho;
          o[ax] = 0.5 * glap + ha * g_[ax] + hb * p_[ax] * v_[ax];
        }
        dln0 -= F1 * g_[0]; dln1 -= F1 * g_[1]; dln2 -= F1 * g_[2];
        dT0 += o[0]; dT1 += o[1]; dT2 += o[2];
      }
    }
    __syncthreads();
    // M = X B (NSP x NSP; K = centres), then W = B M (NP x NSP; K = orbitals)
    cgemm<NSP / 16, NSP / 16, NP>(Xs, NP, NSP, Bs, NSP, NSP, Ms, NSP, wave, lane);
    __syncthreads();
    cgemm<NP / 16, NSP / 16, NSP>(Bs, NSP, NP, Ms, NSP, NSP, Ws, NSP, wave, lane);
    __syncthreads();
    // pass 2: d Re T/dR_a += Re grad phi_a(r_i) W_ai
    if (act) {
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const int e = sp * NS + i;
        const cd Wv = ld_c(Ws, (size_t)ca * NSP + i);
        if constexpr (CB) {
          const CBasisD q = ccontracted_derivs<false>(pos[3 * e] - Ra0, pos[3 * e + 1] - Ra1, pos[3 * e + 2] - Ra2,
                                                      m.eta, L, invL, tw);
          dT0 += remul(q.gx, Wv);
          dT1 += remul(q.gy, Wv);
          dT2 += remul(q.gz, Wv);
        } else {
          cd g[3][4];
          cbasis_axis<1>(pos[3 * e] - Ra0, za, L, invL, tw, 0, g[0]);
          cbasis_axis<1>(pos[3 * e + 1] - Ra1, za, L, invL, tw, 1, g[1]);
          cbasis_axis<1>(pos[3 * e + 2] - Ra2, za, L, invL, tw, 2, g[2]);
          dT0 += remul(cmul(cmul(g[0][1], g[1][0]), g[2][0]), Wv);
          dT1 += remul(cmul(cmul(g[0][0], g[1][1]), g[2][0]), Wv);
          dT2 += remul(cmul(cmul(g[0][0], g[1][0]), g[2][1]), Wv);
        }
      }
    }
    __syncthreads();
  }
  // combine the H threads of each centre in a fixed order
  double* rr = part;
  if (act) {
    double* q = rr + ((size_t)h * N + ca) * 6;
    q[0] = dln0; q[1] = dln1; q[2] = dln2; q[3] = dT0; q[4] = dT1; q[5] = dT2;
  }
  const double Tsl = csum256(tsl, red);
  const double Tj = csum256(tj, red);
  const double Us = csum256(usum, red);
  const double EL = Tsl + Tj + m.Vs[w];
  double* acc = m.acc + (size_t)w * (2 + 9 * N);
  if (t < N) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int hh = 0; hh < H; ++hh)
      for (int c = 0; c < 6; ++c) v[c] += rr[((size_t)hh * N + t) * 6 + c];
    const double* dv = m.dVs + (size_t)w * 3 * N + 3 * t;
    for (int c = 0; c < 3; ++c) {
      const double d = v[3 + c] + dv[c], gq = v[c];
      acc[2 + 3 * t + c] += d;
      acc[2 + 3 * N + 3 * t + c] += gq;
      acc[2 + 6 * N + 3 * t + c] += EL * gq;
    }
  }
  if (t == 0) {
    acc[0] += EL;
    acc[1] += EL * EL;
    m.Uj[w] = Us;
    if (m.ELs) m.ELs[w] = EL;
  }
  if (m.j3) {
    // for the three-body term's d/dR pass: grad U, Re grad ln D and Re E_L of this sample
    double* out = m.j3scr + (size_t)w * j3_measure_doubles(N) + 4 * N + 1;
    for (int u = t; u < 3 * N; u += 256) {
      out[u] = gU[u];
      out[3 * N + u] = gd[u];
    }
    if (t == 0) out[6 * N] = EL;
  }
}

// ---------------------------------------------------------------- launchers ---
size_t cslater_scratch_bytes(int NS) {
  switch (NS) {
    case 8: return 16 * CSlaterLay<8>::scr_elems;
    case 12: return 16 * CSlaterLay<12>::scr_elems;
    case 16: return 16 * CSlaterLay<16>::scr_elems;
    case 20: return 16 * CSlaterLay<20>::scr_elems;
    case 24: return 16 * CSlaterLay<24>::scr_elems;
    case 27: return 16 * CSlaterLay<27>::scr_elems;
    case 32: return 16 * CSlaterLay<32>::scr_elems;
    case 64: return 16 * CSlaterLay<64>::scr_elems;
    default: return 0;
  }
}

template <int NS>
hipError_t launch_csweep_t(const WalkerArgs& a, const SweepArgs& s, const TwistArgs& tw, int refresh, int moves,
                           double rtol, hipStream_t st) {
  static_assert(CSweepLds<NS>::bytes(true) <= 160 * 1024, "the complex half-sweep exceeds the LDS of a CU");
  if (moves && a.contracted)
    hipLaunchKernelGGL((k_csweep<NS, true, true>), dim3(a.W), dim3(CT), CSweepLds<NS>::bytes(true), st, a, s, tw,
                       refresh, rtol);
  else if (moves)
    hipLaunchKernelGGL((k_csweep<NS, true, false>), dim3(a.W), dim3(CT), CSweepLds<NS>::bytes(true), st, a, s, tw,
                       refresh, rtol);
  else if (a.contracted)
    hipLaunchKernelGGL((k_csweep<NS, false, true>), dim3(a.W), dim3(CT), CSweepLds<NS>::bytes(false), st, a, s, tw, 1, rtol);
  else
    hipLaunchKernelGGL((k_csweep<NS, false, false>), dim3(a.W), dim3(CT), CSweepLds<NS>::bytes(false), st, a, s, tw, 1, rtol);
  return hipGetLastError();
}

template <int NS>
hipError_t launch_cslater_t(const MeasureArgs& m, const TwistArgs& tw, hipStream_t st) {
  static_assert(CSlaterLay<NS>::bytes <= 160 * 1024, "the complex measurement exceeds the LDS of a CU");
  if (m.contracted)
    hipLaunchKernelGGL((k_cslater_sample<NS, true>), dim3(m.W), dim3(256), CSlaterLay<NS>::bytes, st, m, tw);
  else
    hipLaunchKernelGGL((k_cslater_sample<NS, false>), dim3(m.W), dim3(256), CSlaterLay<NS>::bytes, st, m, tw);
  return hipGetLastError();
}

#define VMC_CDISPATCH(ns, CALL)                  \
  switch (ns) {                                  \
    case 8: { constexpr int NSV = 8; CALL; }     \
    case 12: { constexpr int NSV = 12; CALL; }   \
    case 16: { constexpr int NSV = 16; CALL; }   \
    case 20: { constexpr int NSV = 20; CALL; }   \
    case 24: { constexpr int NSV = 24; CALL; }   \
    case 27: { constexpr int NSV = 27; CALL; }   \
    case 32: { constexpr int NSV = 32; CALL; }   \
    case 64: { constexpr int NSV = 64; CALL; }   \
    default: return hipErrorInvalidValue;        \
  }

hipError_t launch_csweep(const WalkerArgs& a, const SweepArgs& s, const TwistArgs& tw, int refresh, int moves,
                         double rtol, hipStream_t st) {
  if (a.W < 1 || a.N != 2 * a.NS || (s.spin != 0 && s.spin != 1) || (!moves && refresh != 1) || refresh < 0 ||
      refresh > 2)
    return hipErrorInvalidValue;
  VMC_CDISPATCH(a.NS, return (launch_csweep_t<NSV>(a, s, tw, refresh, moves, rtol, st)))
}

hipError_t launch_cslater_sample(const MeasureArgs& m, const TwistArgs& tw, hipStream_t st) {
  if (m.W < 1 || m.N != 2 * m.NS || !m.scr) return hipErrorInvalidValue;
  VMC_CDISPATCH(m.NS, return (launch_cslater_t<NSV>(m, tw, st)))
}

}  // namespace vmc
