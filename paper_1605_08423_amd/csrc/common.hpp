// Device helpers shared by the VMC kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define VMC_WAVE 64
#define VMC_PI 3.14159265358979323846

namespace vmc {

// ------------------------------------------------------------------ Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (hi*, lo*) = M * (c0, c2) mixing with the key, the key bumped by the Weyl
// constants between rounds.
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

// 53-bit uniform double in [0, 1) from two words (all 32 bits of hi, top 21 of lo).
__device__ __forceinline__ double u01(uint32_t hi, uint32_t lo) {
  uint64_t m = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
  return (double)m * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------ wave helpers --
__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, lane);
  hi = __builtin_amdgcn_readlane(hi, lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <class T> __device__ __forceinline__ T readlane(T v, int lane);
template <> __device__ __forceinline__ double readlane<double>(double v, int lane) { return readlane_d(v, lane); }
template <> __device__ __forceinline__ float readlane<float>(float v, int lane) { return readlane_f(v, lane); }

// Value held by lane (l ^ M) for M in {1, 2, 7, 15, 16, 32}: quad permutations and row
// (half-)mirrors (i -> 7 - i, 15 - i, which are xor 7, xor 15 inside a row) by DPP, and the
// gfx950 row-swap instructions across rows; all are register moves, no LDS round trip.
// The six masks span all lane bits, so a butterfly over them reaches every lane.
template <int M>
__device__ __forceinline__ int xor_lane(int v) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  } else if constexpr (M == 7) {
    return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
  } else if constexpr (M == 15) {
    return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);   // row_mirror
  } else if constexpr (M == 16) {
    // element 0: even rows keep theirs, odd rows get the even row's; element 1: the reverse
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((__lane_id() & 16) ? r[0] : r[1]);
  } else {
    static_assert(M == 32, "unsupported lane mask");
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((__lane_id() & 32) ? r[0] : r[1]);
  }
}
template <int M>
__device__ __forceinline__ double xor_lane(double v) {
  const int lo = xor_lane<M>(__double2loint(v)), hi = xor_lane<M>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int M>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane<M>(__float_as_int(v)));
}

// Sum over the 64 lanes by the xor butterfly above.  Each step adds a lane's value and its
// partner's (the same two operands in both lanes), so every lane ends with bit-identical
// totals.
template <class T>
__device__ __forceinline__ T wave_allsum(T v) {
  v += xor_lane<32>(v);
  v += xor_lane<16>(v);
  v += xor_lane<15>(v);
  v += xor_lane<7>(v);
  v += xor_lane<2>(v);
  v += xor_lane<1>(v);
  return v;
}

// Largest value over the 64 lanes and its index, ties to the lowest index (a total order,
// so every lane ends with the same pair).
template <int M>
__device__ __forceinline__ void argmax_step(double& bv, int& bi) {
  const double ov = xor_lane<M>(bv);
  const int oi = xor_lane<M>(bi);
  if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
}
__device__ __forceinline__ void wave_argmax(double& bv, int& bi) {
  argmax_step<32>(bv, bi);
  argmax_step<16>(bv, bi);
  argmax_step<15>(bv, bi);
  argmax_step<7>(bv, bi);
  argmax_step<2>(bv, bi);
  argmax_step<1>(bv, bi);
}

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane gets lane 0's result.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return readlane_d(v, 0);
}

// Orders the wave's own LDS writes before its later LDS reads (no block barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --------------------------------------------------------------- geometry --
__device__ __forceinline__ double min_image(double d, double L, double invL) {
  return d - L * floor(d * invL + 0.5);
}
__device__ __forceinline__ double wrap_box(double x, double L, double invL) {
  return x - L * floor(x * invL);
}

template <class Real> __device__ __forceinline__ Real dev_exp(Real x);
template <> __device__ __forceinline__ double dev_exp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float dev_exp<float>(float x) { return __expf(x); }

// Periodic Gaussian factor along one axis at minimum-image offset x in
// [-L/2, L/2): images n = -1, 0, +1 of e^{-zeta (x + n L)^2} (the far images are
// below e^{-zeta (1.5 L)^2}).  NDER = number of derivatives wanted (0..3).
// nimg = 0 keeps only n = 0; the caller uses it only where every dropped image is
// below e^{-zeta_min (L/2)^2} <= e^{-23}, i.e. under FP32 resolution.
template <class Real, int NDER, int NIMG>
__device__ __forceinline__ void gauss1d_n(Real x, Real zeta, Real L, Real g[4]) {
  g[0] = g[1] = g[2] = g[3] = Real(0);
#pragma unroll
  for (int n = -NIMG; n <= NIMG; ++n) {
    Real t = x + Real(n) * L;
    Real e = dev_exp<Real>(-zeta * t * t);
    g[0] += e;
    if (NDER >= 1) g[1] += Real(-2) * zeta * t * e;
    if (NDER >= 2) g[2] += (Real(4) * zeta * zeta * t * t - Real(2) * zeta) * e;
    if (NDER >= 3) g[3] += (Real(-8) * zeta * zeta * zeta * t * t * t + Real(12) * zeta * zeta * t) * e;
  }
}
// The same with image n weighted by tau^n (tau = -1: twist angle pi); the two images are
// summed apart and enter once.
template <class Real, int NDER, int NIMG>
__device__ __forceinline__ void gauss1d_n(Real x, Real zeta, Real L, Real g[4], Real tau) {
  Real h[4] = {Real(0), Real(0), Real(0), Real(0)};
  g[0] = g[1] = g[2] = g[3] = Real(0);
#pragma unroll
  for (int n = -NIMG; n <= NIMG; ++n) {
    Real t = x + Real(n) * L;
    Real e = dev_exp<Real>(-zeta * t * t);
    Real* o = (n == 0) ? g : h;
    o[0] += e;
    if (NDER >= 1) o[1] += Real(-2) * zeta * t * e;
    if (NDER >= 2) o[2] += (Real(4) * zeta * zeta * t * t - Real(2) * zeta) * e;
    if (NDER >= 3) o[3] += (Real(-8) * zeta * zeta * zeta * t * t * t + Real(12) * zeta * zeta * t) * e;
  }
  if (NIMG) {
#pragma unroll
    for (int q = 0; q <= NDER; ++q) g[q] += tau * h[q];
  }
}

// The basis factor along one axis at the offset d = r - R_a (any real value): the
// image sum at the minimum image d - k L, k = round(d / L), by gauss1d_n.  TW (a launch
// with some twist): with the twist angle pi along the axis (tw = 1: phi(r + L e) = -phi(r))
// the images carry (-1)^n and the factor at d is (-1)^k times the one at the minimum image.
// Untwisted launches use TW = false, which is the plain periodic factor.
template <class Real, int NDER, int NIMG, bool TW>
__device__ __forceinline__ void basis_axis(double d, Real zeta, double L, double invL, int tw, Real g[4]) {
  const double k = floor(d * invL + 0.5);
  if constexpr (TW) {
    gauss1d_n<Real, NDER, NIMG>((Real)(d - L * k), zeta, (Real)L, g, tw ? Real(-1) : Real(1));
    if (tw & (int)k) {
#pragma unroll
      for (int q = 0; q <= NDER; ++q) g[q] = -g[q];
    }
  } else {
    gauss1d_n<Real, NDER, NIMG>((Real)(d - L * k), zeta, (Real)L, g);
  }
}

// The SI's contracted orbital per proton, phi_1 + eta phi_2 with phi_1 = e^{-Z1 r^2} and
// phi_2 = r^2 e^{-Z2 r^2}.  Writing r^2 = x^2 + y^2 + z^2 makes it a sum of four products of
// Cartesian factors, g1 g1 g1 + eta (h2 g2 g2 + g2 h2 g2 + g2 g2 h2), with the image sums (at the
// minimum image, images n = -NIMG..NIMG) of g1 = e^{-Z1 t^2}, g2 = e^{-Z2 t^2} and
// h2 = t^2 e^{-Z2 t^2} and their first NDER derivatives.
constexpr double kZ1 = 0.6066825, kZ2 = 0.3382168;
template <class Real, int NDER, int NIMG>
__device__ __forceinline__ void contracted_axis(double d, double L, double invL, Real g1[4], Real g2[4], Real h2[4]) {
  const double k = floor(d * invL + 0.5);
  const Real x = (Real)(d - L * k), Lr = (Real)L, z1 = (Real)kZ1, z2 = (Real)kZ2;
#pragma unroll
  for (int q = 0; q < 4; ++q) g1[q] = g2[q] = h2[q] = Real(0);
#pragma unroll
  for (int n = -NIMG; n <= NIMG; ++n) {
    const Real t = x + Real(n) * Lr, t2 = t * t;
    const Real e1 = dev_exp<Real>(-z1 * t2), e2 = dev_exp<Real>(-z2 * t2);
    g1[0] += e1;
    g2[0] += e2;
    h2[0] += t2 * e2;
    if (NDER >= 1) {
      g1[1] += Real(-2) * z1 * t * e1;
      g2[1] += Real(-2) * z2 * t * e2;
      h2[1] += (Real(2) * t - Real(2) * z2 * t2 * t) * e2;
    }
    if (NDER >= 2) {
      g1[2] += (Real(4) * z1 * z1 * t2 - Real(2) * z1) * e1;
      g2[2] += (Real(4) * z2 * z2 * t2 - Real(2) * z2) * e2;
      h2[2] += (Real(2) - Real(10) * z2 * t2 + Real(4) * z2 * z2 * t2 * t2) * e2;
    }
    if (NDER >= 3) {
      g1[3] += (Real(-8) * z1 * z1 * z1 * t2 * t + Real(12) * z1 * z1 * t) * e1;
      g2[3] += (Real(-8) * z2 * z2 * z2 * t2 * t + Real(12) * z2 * z2 * t) * e2;
      h2[3] += (Real(-24) * z2 * t + Real(36) * z2 * z2 * t2 * t - Real(8) * z2 * z2 * z2 * t2 * t2 * t) * e2;
    }
  }
}

template <class Real, int NIMG>
__device__ __forceinline__ Real contracted_value(double rx, double ry, double rz, const double* Ra, Real eta,
                                                 double L, double invL) {
  Real a1[3][4], a2[3][4], b2[3][4];
  contracted_axis<Real, 0, NIMG>(rx - Ra[0], L, invL, a1[0], a2[0], b2[0]);
  contracted_axis<Real, 0, NIMG>(ry - Ra[1], L, invL, a1[1], a2[1], b2[1]);
  contracted_axis<Real, 0, NIMG>(rz - Ra[2], L, invL, a1[2], a2[2], b2[2]);
  return a1[0][0] * a1[1][0] * a1[2][0] +
         eta * (b2[0][0] * a2[1][0] * a2[2][0] + a2[0][0] * b2[1][0] * a2[2][0] + a2[0][0] * a2[1][0] * b2[2][0]);
}

// Derivative components of a basis function: gradient, Hessian and (FULL) gradient of the
// Laplacian; product_terms adds w times those of a product of Cartesian factors f[axis][order].
template <class Real>
struct BasisD {
  Real gx, gy, gz, hxx, hyy, hzz, hxy, hxz, hyz, glx, gly, glz;
};
template <class Real, bool FULL>
__device__ __forceinline__ void product_terms(const Real (&f)[3][4], Real w, BasisD<Real>& o) {
  const Real p00 = f[1][0] * f[2][0], p01 = f[0][0] * f[2][0], p02 = f[0][0] * f[1][0];
  o.gx += w * f[0][1] * p00;
  o.gy += w * f[1][1] * p01;
  o.gz += w * f[2][1] * p02;
  if (FULL) {
    o.hxx += w * f[0][2] * p00;
    o.hyy += w * f[1][2] * p01;
    o.hzz += w * f[2][2] * p02;
    o.hxy += w * f[0][1] * f[1][1] * f[2][0];
    o.hxz += w * f[0][1] * f[1][0] * f[2][1];
    o.hyz += w * f[0][0] * f[1][1] * f[2][1];
    o.glx += w * (f[0][3] * p00 + f[0][1] * (f[1][2] * f[2][0] + f[1][0] * f[2][2]));
    o.gly += w * (f[1][3] * p01 + f[1][1] * (f[0][2] * f[2][0] + f[0][0] * f[2][2]));
    o.glz += w * (f[2][3] * p02 + f[2][1] * (f[0][2] * f[1][0] + f[0][0] * f[1][2]));
  }
}
// The components of the contracted orbital at offset (dx, dy, dz) from its centre.
template <class Real, int NIMG, bool FULL>
__device__ __forceinline__ BasisD<Real> contracted_derivs(double dx, double dy, double dz, Real eta, double L,
                                                           double invL) {
  constexpr int ND = FULL ? 3 : 1;
  Real a1[3][4], a2[3][4], b2[3][4];
  contracted_axis<Real, ND, NIMG>(dx, L, invL, a1[0], a2[0], b2[0]);
  contracted_axis<Real, ND, NIMG>(dy, L, invL, a1[1], a2[1], b2[1]);
  contracted_axis<Real, ND, NIMG>(dz, L, invL, a1[2], a2[2], b2[2]);
  BasisD<Real> o = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0), Real(0), Real(0), Real(0), Real(0),
                    Real(0), Real(0)};
  product_terms<Real, FULL>(a1, Real(1), o);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Real f[3][4];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
      for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? b2[mm][q] : a2[mm][q];
    product_terms<Real, FULL>(f, eta, o);
  }
  return o;
}

// The on-site three-body Jastrow term's orbitals (SI, Jastrow section): chi_1 = e^{-ZJ rho^2} and
// chi_2 = rho^2 e^{-ZJ rho^2} of the sin-periodised offset rho_m = (L/pi) sin(pi d_m / L) between an
// electron and a nucleus; their values from the sines and cosines of pi x / L of both.
constexpr double kZJ = 0.7933844;
template <class Real>
__device__ __forceinline__ void j3_values(const Real se[3], const Real ce[3], const Real sa[3], const Real ca[3],
                                          Real LoverPi, Real& v1, Real& v2) {
  Real u = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const Real rt = LoverPi * (se[m] * ca[m] - ce[m] * sa[m]);
    u += rt * rt;
  }
  v1 = dev_exp<Real>(-(Real)kZJ * u);
  v2 = u * v1;
}

// Orders this wave's LDS writes before its later LDS reads (the wave's LDS
// operations complete in order; the clobber keeps the compiler from moving them).
__device__ __forceinline__ void lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <class Real> __device__ __forceinline__ Real dev_sqrt(Real x);
template <> __device__ __forceinline__ double dev_sqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dev_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// Reciprocal and reciprocal square root: exact in FP64, the hardware estimates
// (about 1 ulp) in FP32, where the mixed mode accepts FP32-level errors.
template <class Real> __device__ __forceinline__ Real dev_rcp(Real x);
template <> __device__ __forceinline__ double dev_rcp<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ float dev_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <class Real> __device__ __forceinline__ Real dev_rsqrt(Real x);
template <> __device__ __forceinline__ double dev_rsqrt<double>(double x) { return 1.0 / sqrt(x); }
template <> __device__ __forceinline__ float dev_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// erfc(x) for x >= 0 and e^{-x^2}.  FP64: the library functions.  FP32, without
// branches: erfc(x) = t Q(t) e^{-x^2}, t = 1 / (1 + 0.4 x), Q of degree 9 fitted to
// erfcx(x) / t on [0, 10] (relative error of the fit below 1e-8, so FP32 rounding
// dominates; csrc/fit_erfc.py makes the coefficients); e^{-x^2} takes the rounding
// error of x^2 into account to first order.
template <class Real> __device__ __forceinline__ Real dev_erfc_exp(Real x, Real* ex2);
template <> __device__ __forceinline__ double dev_erfc_exp<double>(double x, double* ex2) {
  *ex2 = exp(-x * x);
  return erfc(x);
}
template <> __device__ __forceinline__ float dev_erfc_exp<float>(float x, float* ex2) {
  constexpr float Q0 = 0.22570692f, Q1 = 0.22495188f, Q2 = 0.21491995f, Q3 = 0.12967727f, Q4 = 0.27206808f;
  constexpr float Q5 = -0.28436062f, Q6 = 0.54741645f, Q7 = -0.49878836f, Q8 = 0.19799955f, Q9 = -0.029591113f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.4f, x, 1.0f));
  float q = fmaf(Q9, t, Q8);
  q = fmaf(q, t, Q7); q = fmaf(q, t, Q6); q = fmaf(q, t, Q5); q = fmaf(q, t, Q4);
  q = fmaf(q, t, Q3); q = fmaf(q, t, Q2); q = fmaf(q, t, Q1); q = fmaf(q, t, Q0);
  const float hi = x * x, lo = fmaf(x, x, -hi);
  const float e = __expf(-hi) * (1.0f - lo);
  *ex2 = e;
  return t * q * e;
}

template <class Real> __device__ __forceinline__ void dev_sincospi(Real x, Real* s, Real* c);
template <> __device__ __forceinline__ void dev_sincospi<double>(double x, double* s, double* c) { sincospi(x, s, c); }
template <> __device__ __forceinline__ void dev_sincospi<float>(float x, float* s, float* c) { sincospif(x, s, c); }

// sin(pi x) and cos(pi x) for |x| <= 1/2 (a minimum-image offset over the box side).  FP32:
// the Taylor series of sin t and cos t, t = pi x, through t^13 and t^14 in Horner form; the
// truncation is below 1e-9 at |t| = pi/2, so FP32 rounding sets the error (about 1.6e-7
// relative for sin, small offsets included).  FP64 keeps the library's sincospi.
template <class Real> __device__ __forceinline__ void sincospi_half(Real x, Real* s, Real* c);
template <> __device__ __forceinline__ void sincospi_half<double>(double x, double* s, double* c) {
  sincospi(x, s, c);
}
template <> __device__ __forceinline__ void sincospi_half<float>(float x, float* s, float* c) {
  const float t = 3.14159265358979f * x, t2 = t * t;
  float ps = 1.0f / 6227020800.0f;
  ps = fmaf(ps, t2, -1.0f / 39916800.0f);
  ps = fmaf(ps, t2, 1.0f / 362880.0f);
  ps = fmaf(ps, t2, -1.0f / 5040.0f);
  ps = fmaf(ps, t2, 1.0f / 120.0f);
  ps = fmaf(ps, t2, -1.0f / 6.0f);
  ps = fmaf(ps, t2, 1.0f);
  float pc = -1.0f / 87178291200.0f;
  pc = fmaf(pc, t2, 1.0f / 479001600.0f);
  pc = fmaf(pc, t2, -1.0f / 3628800.0f);
  pc = fmaf(pc, t2, 1.0f / 40320.0f);
  pc = fmaf(pc, t2, -1.0f / 720.0f);
  pc = fmaf(pc, t2, 1.0f / 24.0f);
  pc = fmaf(pc, t2, -0.5f);
  *s = ps * t;
  *c = fmaf(pc, t2, 1.0f);
}

// Pade pair value u(rho) = a rho / (1 + b rho) of the Jastrow, for the
// sin-periodised offset built from the trig caches of the two electrons:
// sin(pi (x_i - x_j)/L) = s_i c_j - c_i s_j.
template <class Real>
__device__ __forceinline__ Real pade_u(const Real si[3], const Real ci[3], const Real sj[3], const Real cj[3],
                                       Real LoverPi, Real a, Real b) {
  Real r2 = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Real rt = LoverPi * (si[m] * cj[m] - ci[m] * sj[m]);
    r2 += rt * rt;
  }
  Real rho = dev_sqrt<Real>(r2);
  return a * rho * dev_rcp<Real>(Real(1) + b * rho);
}

// e^{-beta rho} on the sin-periodised distance of an electron (si, ci) and a proton
// (sj, cj).  The one-body Jastrow term of the pair is -(1 - e^{-beta rho}) / beta, so a
// move changes it by the difference of these exponentials divided by beta.
template <class Real>
__device__ __forceinline__ Real one_body_exp(const Real si[3], const Real ci[3], const Real sj[3], const Real cj[3],
                                             Real LoverPi, Real beta) {
  Real r2 = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Real rt = LoverPi * (si[m] * cj[m] - ci[m] * sj[m]);
    r2 += rt * rt;
  }
  return dev_exp<Real>(-beta * dev_sqrt<Real>(r2));
}

}  // namespace vmc
