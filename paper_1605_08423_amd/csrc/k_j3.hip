// The on-site three-body (electron-electron-nucleus) Jastrow term of the SI (Jastrow section, Eq.
// e:j33): U_3 = sum_a sum_{i<j} chi_a(r_i)^T F chi_a(r_j) with the orbitals chi_1 = e^{-ZJ rho^2},
// chi_2 = rho^2 e^{-ZJ rho^2} on the sin-periodised offsets rho_m = (L/pi) sin(pi d_m / L) and one
// symmetric 2 x 2 matrix F for every nucleus.  With G_a = sum_i chi_a(r_i):
//   U_3 = 1/2 sum_a [G_a^T F G_a - sum_i chi_ai^T F chi_ai],
//   grad_k U_3 = sum_a (grad chi_ak)^T F (G_a - chi_ak),   lap_k U_3 = sum_a (lap chi_ak)^T F (G_a - chi_ak),
// and, as chi_a moves with R_a (d/dR_a = -grad on it), with v_k = grad_k U + grad_k ln|D| and
// G_a,mu = sum_i d_mu chi_ai:
//   d ln psi/dR_a,mu = -sum_k (d_mu chi_ak)^T F (G_a - chi_ak),
//   d T_L/dR_a,mu = sum_k { 1/2 [(d_mu lap chi_ak)^T F (G_a - chi_ak) + (lap chi_ak)^T F (G_a,mu - d_mu chi_ak)]
//                 + sum_nu v_k,nu [(d_mu d_nu chi_ak)^T F (G_a - chi_ak) + (d_nu chi_ak)^T F (G_a,mu - d_mu chi_ak)] }.
// Both are bilinear in sums over k, so with X_k,mu = 1/2 d_mu lap chi_ak + sum_nu v_k,nu d_mu d_nu chi_ak,
// Y_k = 1/2 lap chi_ak + sum_nu v_k,nu d_nu chi_ak, P_mu = sum_k X_k,mu and Q = sum_k Y_k:
//   d T_L/dR_a,mu = P_mu^T F G_a + Q^T F G_a,mu - sum_k (X_k,mu^T F chi_ak + Y_k^T F d_mu chi_ak),
//   d ln psi/dR_a,mu = -G_a,mu^T F G_a + sum_k (d_mu chi_ak)^T F chi_ak,
// which one pass over the electrons forms, evaluating each pair's orbitals once.
// The orbital part of the one-body term (Eq. e:j1), U_1f = sum_a f^T G_a, is linear in the same
// orbitals: grad_k and lap_k get sum_a f^T (grad, lap) chi_ak, d ln psi/dR_a,mu gets -f^T G_a,mu and
// d T_L/dR_a,mu gets f^T P_mu; the kernels add these beside the three-body terms.
// The sweep keeps G_a of every walker current (k_sweep_half's three-body variant); k_j3_init forms
// G_a from the positions before the sweeps (FP64), and the measurement's kernels evaluate the
// orbitals and their sums in the working precision of the Jastrow terms (FP32 in mixed precision,
// with the per-nucleus and per-electron results combined and accumulated in FP64).
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

namespace {

// Orbital components [value, grad(3), lap, hess xx yy zz xy xz yz, grad lap(3)] of chi_1 and chi_2
// at the offset whose sin and cos of pi d_m / L per axis are s, c: the first NC of them (5: value,
// gradient, Laplacian; 14: all).  Per axis, with rho = (L/pi) s, u = rho^2, u1 = 2 rho c,
// u2 = 2 (c^2 - k rho^2), u3 = -8 k rho c (the first three derivatives of u; k = (pi/L)^2), the
// factors a = e^{-Z u} and b = u a have q-th derivatives A_q e^{-Z u} and B_q e^{-Z u} with
//   A = (1, -Z u1, Z^2 u1^2 - Z u2, -Z^3 u1^3 + 3 Z^2 u1 u2 - Z u3),
//   B = (u, u1 + u A_1, u2 + 2 u1 A_1 + u A_2, u3 + 3 u2 A_1 + 3 u1 A_2 + u A_3);
// chi_1 = a a a and chi_2 = b a a + a b a + a a b, so every product carries e^{-Z (u_x + u_y + u_z)}.
template <class Real, int NC>
__device__ __forceinline__ void prodc(const Real f[3][4], Real w, Real o[NC]) {
  const Real p00 = f[1][0] * f[2][0], p01 = f[0][0] * f[2][0], p02 = f[0][0] * f[1][0];
  o[0] += w * f[0][0] * p00;
  o[1] += w * f[0][1] * p00;
  o[2] += w * f[1][1] * p01;
  o[3] += w * f[2][1] * p02;
  const Real hxx = f[0][2] * p00, hyy = f[1][2] * p01, hzz = f[2][2] * p02;
  o[4] += w * (hxx + hyy + hzz);
  if constexpr (NC == 14) {
    o[5] += w * hxx;
    o[6] += w * hyy;
    o[7] += w * hzz;
    o[8] += w * f[0][1] * f[1][1] * f[2][0];
    o[9] += w * f[0][1] * f[1][0] * f[2][1];
    o[10] += w * f[0][0] * f[1][1] * f[2][1];
    o[11] += w * (f[0][3] * p00 + f[0][1] * (f[1][2] * f[2][0] + f[1][0] * f[2][2]));
    o[12] += w * (f[1][3] * p01 + f[1][1] * (f[0][2] * f[2][0] + f[0][0] * f[2][2]));
    o[13] += w * (f[2][3] * p02 + f[2][1] * (f[0][2] * f[1][0] + f[0][0] * f[1][2]));
  }
}

template <class Real, int NC>
__device__ __forceinline__ void j3_orbitals(const Real s[3], const Real c[3], Real LoP, Real kf, Real c1[NC],
                                            Real c2[NC]) {
  const Real Z = (Real)kZJ;
  Real A[3][4], B[3][4], usum = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const Real rho = LoP * s[m];
    const Real u = rho * rho, u1 = Real(2) * rho * c[m], u2 = Real(2) * (c[m] * c[m] - kf * rho * rho);
    usum += u;
    A[m][0] = Real(1);
    A[m][1] = -Z * u1;
    A[m][2] = Z * Z * u1 * u1 - Z * u2;
    B[m][0] = u;
    B[m][1] = u1 + u * A[m][1];
    B[m][2] = u2 + Real(2) * u1 * A[m][1] + u * A[m][2];
    if constexpr (NC == 14) {
      const Real u3 = Real(-8) * kf * rho * c[m];
      A[m][3] = -Z * Z * Z * u1 * u1 * u1 + Real(3) * Z * Z * u1 * u2 - Z * u3;
      B[m][3] = u3 + Real(3) * u2 * A[m][1] + Real(3) * u1 * A[m][2] + u * A[m][3];
    } else {
      A[m][3] = B[m][3] = Real(0);
    }
  }
  const Real E = dev_exp<Real>(-Z * usum);
#pragma unroll
  for (int q = 0; q < NC; ++q) c1[q] = c2[q] = Real(0);
  prodc<Real, NC>(A, E, c1);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Real f[3][4];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
      for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? B[mm][q] : A[mm][q];
    prodc<Real, NC>(f, E, c2);
  }
}

// x^T F y for 2-vectors, F = [[f0, f1], [f1, f2]]
template <class Real>
__device__ __forceinline__ Real fform(const Real f[3], Real x1, Real x2, Real y1, Real y2) {
  return f[0] * x1 * y1 + f[1] * (x1 * y2 + x2 * y1) + f[2] * x2 * y2;
}

// sin and cos of pi (x_e - R_a)_m / L from the tables of both
template <class Real>
__device__ __forceinline__ void pair_trig(const Real* te, const Real* ta, Real s[3], Real c[3]) {
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    s[m] = te[m] * ta[3 + m] - te[3 + m] * ta[m];
    c[m] = te[3 + m] * ta[3 + m] + te[m] * ta[m];
  }
}

// sin and cos of pi x / L of the walker's electrons (te, N x 6) and of the nuclei (ta, N x 6)
template <class Real>
__device__ __forceinline__ void trig_tables(const double* pos, const double* R, int N, double invL, Real* te,
                                            Real* ta) {
  for (int u = threadIdx.x; u < 3 * N; u += blockDim.x) {
    const int i = u / 3, m = u % 3;
    dev_sincospi<Real>((Real)(pos[u] * invL), &te[6 * i + m], &te[6 * i + 3 + m]);
    dev_sincospi<Real>((Real)(R[u] * invL), &ta[6 * i + m], &ta[6 * i + 3 + m]);
  }
}

// threads of a block: the particle count rounded up to whole wavefronts
inline int j3_threads(int N) { return ((N + 63) / 64) * 64; }

}  // namespace

// G_a of every walker: one block per walker, threads over nuclei.
__global__ __launch_bounds__(256) void k_j3_init(WalkerArgs a) {
  extern __shared__ __align__(16) double sm[];
  const int N = a.N, w = blockIdx.x;
  double* te = sm;            // N x 6: electrons' sin x3, cos x3
  double* ta = sm + 6 * N;    // N x 6: nuclei
  trig_tables<double>(a.pos + (size_t)w * 3 * N, a.R, N, a.invL, te, ta);
  __syncthreads();
  const double LoP = a.L / VMC_PI;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    double g1 = 0.0, g2 = 0.0;
    for (int i = 0; i < N; ++i) {
      double u = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double rt = LoP * (te[6 * i + m] * ta[6 * c + 3 + m] - te[6 * i + 3 + m] * ta[6 * c + m]);
        u += rt * rt;
      }
      const double v = exp(-kZJ * u);
      g1 += v;
      g2 += u * v;
    }
    a.j3G[((size_t)w * N + c) * 2] = g1;
    a.j3G[((size_t)w * N + c) * 2 + 1] = g2;
  }
}

// Before the Slater pass: per walker grad_k U_3 (3N), lap_k U_3 (N) and U_3 into the walker's scratch
// [gU3 (3N), lU3 (N), U3]; threads over nuclei for G_a, then over electrons for the per-electron
// sums (value, gradient and Laplacian of the orbitals only).
template <class Real>
__global__ __launch_bounds__(256) void k_j3_grad(MeasureArgs m) {
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* sm = reinterpret_cast<Real*>(smraw);
  const int N = m.N, w = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  Real* te = sm;
  Real* ta = sm + 6 * N;
  Real* G = sm + 12 * N;     // N x 2
  Real* Q = sm + 14 * N;     // N: sum_i chi_ai^T F chi_ai
  __shared__ double red[4];
  trig_tables<Real>(m.pos + (size_t)w * 3 * N, m.R, N, m.invL, te, ta);
  __syncthreads();
  const Real LoP = (Real)(m.L / VMC_PI), kf = (Real)((VMC_PI * m.invL) * (VMC_PI * m.invL)), Z = (Real)kZJ;
  const Real F[3] = {(Real)m.j3f[0], (Real)m.j3f[1], (Real)m.j3f[2]};
  const Real f1 = (Real)m.j1f[0], f2 = (Real)m.j1f[1];
  for (int c = t; c < N; c += T) {
    Real g1 = Real(0), g2 = Real(0), q = Real(0);
    for (int i = 0; i < N; ++i) {
      Real u = Real(0);
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) {
        const Real rt = LoP * (te[6 * i + mm] * ta[6 * c + 3 + mm] - te[6 * i + 3 + mm] * ta[6 * c + mm]);
        u += rt * rt;
      }
      const Real v = dev_exp<Real>(-Z * u);
      g1 += v;
      g2 += u * v;
      q += fform<Real>(F, v, u * v, v, u * v);
    }
    G[2 * c] = g1;
    G[2 * c + 1] = g2;
    Q[c] = q;
  }
  __syncthreads();
  double* out = m.j3scr + (size_t)w * j3_measure_doubles(N);
  for (int k = t; k < N; k += T) {
    Real gx = Real(0), gy = Real(0), gz = Real(0), lp = Real(0);
    for (int c = 0; c < N; ++c) {
      Real s[3], cc[3], c1[5], c2[5];
      pair_trig<Real>(te + 6 * k, ta + 6 * c, s, cc);
      j3_orbitals<Real, 5>(s, cc, LoP, kf, c1, c2);
      const Real r1 = G[2 * c] - c1[0], r2 = G[2 * c + 1] - c2[0];
      gx += fform<Real>(F, c1[1], c2[1], r1, r2) + (f1 * c1[1] + f2 * c2[1]);
      gy += fform<Real>(F, c1[2], c2[2], r1, r2) + (f1 * c1[2] + f2 * c2[2]);
      gz += fform<Real>(F, c1[3], c2[3], r1, r2) + (f1 * c1[3] + f2 * c2[3]);
      lp += fform<Real>(F, c1[4], c2[4], r1, r2) + (f1 * c1[4] + f2 * c2[4]);
    }
    out[3 * k] = (double)gx;
    out[3 * k + 1] = (double)gy;
    out[3 * k + 2] = (double)gz;
    out[3 * N + k] = (double)lp;
  }
  // U_3 = 1/2 sum_a (G^T F G - Q_a) and U_1f = sum_a f^T G_a, in a fixed order, in FP64 from the
  // per-nucleus sums
  const double Fd[3] = {m.j3f[0], m.j3f[1], m.j3f[2]};
  double part = 0.0;
  for (int c = t; c < N; c += T) {
    const double g1 = (double)G[2 * c], g2 = (double)G[2 * c + 1];
    part += 0.5 * (fform<double>(Fd, g1, g2, g1, g2) - (double)Q[c]) + (m.j1f[0] * g1 + m.j1f[1] * g2);
  }
  part = wave_allsum(part);
  if ((t & 63) == 0) red[t >> 6] = part;
  __syncthreads();
  if (t == 0) {
    double tot = red[0];
    for (int q = 1; q < T / 64; ++q) tot += red[q];
    out[4 * N] = tot;
  }
}

// After the Slater pass: the term's d/dR contributions to the accumulators, from the full grad U,
// grad ln|D| and E_L of the sample in the walker's scratch [.., gU (3N), gD (3N), E_L].  Threads over
// nuclei; each makes one pass over the electrons in order (the bilinear form above) and combines
// its sums in FP64.
template <class Real>
__global__ __launch_bounds__(256) void k_j3_forces(MeasureArgs m) {
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* sm = reinterpret_cast<Real*>(smraw);
  const int N = m.N, w = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  Real* te = sm;
  Real* ta = sm + 6 * N;
  Real* v = sm + 12 * N;     // N x 3: grad_k U + grad_k ln|D|
  const double* in = m.j3scr + (size_t)w * j3_measure_doubles(N);
  const double* gUf = in + 4 * N + 1;
  const double* gD = gUf + 3 * N;
  const double EL = gD[3 * N];
  trig_tables<Real>(m.pos + (size_t)w * 3 * N, m.R, N, m.invL, te, ta);
  for (int u = t; u < 3 * N; u += T) v[u] = (Real)(gUf[u] + gD[u]);
  __syncthreads();
  const Real LoP = (Real)(m.L / VMC_PI), kf = (Real)((VMC_PI * m.invL) * (VMC_PI * m.invL)), h = Real(0.5);
  const Real F[3] = {(Real)m.j3f[0], (Real)m.j3f[1], (Real)m.j3f[2]};
  const double Fd[3] = {m.j3f[0], m.j3f[1], m.j3f[2]};
  for (int c = t; c < N; c += T) {
    Real G1 = Real(0), G2 = Real(0), Gm1[3] = {0, 0, 0}, Gm2[3] = {0, 0, 0};
    Real P1[3] = {0, 0, 0}, P2[3] = {0, 0, 0}, Q1 = Real(0), Q2 = Real(0), sT[3] = {0, 0, 0}, sL[3] = {0, 0, 0};
    for (int k = 0; k < N; ++k) {
      Real s[3], cc[3], c1[14], c2[14];
      pair_trig<Real>(te + 6 * k, ta + 6 * c, s, cc);
      j3_orbitals<Real, 14>(s, cc, LoP, kf, c1, c2);
      const Real vx = v[3 * k], vy = v[3 * k + 1], vz = v[3 * k + 2];
      // Y_k, F chi_k and F Y_k, the pieces every axis uses
      const Real Y1 = h * c1[4] + vx * c1[1] + vy * c1[2] + vz * c1[3];
      const Real Y2 = h * c2[4] + vx * c2[1] + vy * c2[2] + vz * c2[3];
      const Real Fc1 = F[0] * c1[0] + F[1] * c2[0], Fc2 = F[1] * c1[0] + F[2] * c2[0];
      const Real FY1 = F[0] * Y1 + F[1] * Y2, FY2 = F[1] * Y1 + F[2] * Y2;
      G1 += c1[0];
      G2 += c2[0];
      Q1 += Y1;
      Q2 += Y2;
      // Hessian rows (xx xy xz), (xy yy yz), (xz yz zz) in the 14-component layout
      constexpr int hrow[3][3] = {{5, 8, 9}, {8, 6, 10}, {9, 10, 7}};
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        const Real d1 = c1[1 + mu], d2 = c2[1 + mu];
        Gm1[mu] += d1;
        Gm2[mu] += d2;
        const Real X1 = h * c1[11 + mu] + vx * c1[hrow[mu][0]] + vy * c1[hrow[mu][1]] + vz * c1[hrow[mu][2]];
        const Real X2 = h * c2[11 + mu] + vx * c2[hrow[mu][0]] + vy * c2[hrow[mu][1]] + vz * c2[hrow[mu][2]];
        P1[mu] += X1;
        P2[mu] += X2;
        sT[mu] += X1 * Fc1 + X2 * Fc2 + d1 * FY1 + d2 * FY2;
        sL[mu] += d1 * Fc1 + d2 * Fc2;
      }
    }
    double* acc = m.acc + (size_t)w * (2 + 9 * N);
    const double g1 = (double)G1, g2 = (double)G2, q1 = (double)Q1, q2 = (double)Q2;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const double gm1 = (double)Gm1[mu], gm2 = (double)Gm2[mu];
      const double dT = fform<double>(Fd, (double)P1[mu], (double)P2[mu], g1, g2) +
                        fform<double>(Fd, q1, q2, gm1, gm2) - (double)sT[mu] +
                        (m.j1f[0] * (double)P1[mu] + m.j1f[1] * (double)P2[mu]);
      const double dln = (double)sL[mu] - fform<double>(Fd, gm1, gm2, g1, g2) - (m.j1f[0] * gm1 + m.j1f[1] * gm2);
      acc[2 + 3 * c + mu] += dT;
      acc[2 + 3 * N + 3 * c + mu] += dln;
      acc[2 + 6 * N + 3 * c + mu] += EL * dln;
    }
  }
}

hipError_t launch_j3_init(const WalkerArgs& a, hipStream_t st) {
  if (a.W < 1 || a.N < 2 || a.N > 256 || !a.j3G) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_j3_init, dim3(a.W), dim3(j3_threads(a.N)), (size_t)12 * a.N * sizeof(double), st, a);
  return hipGetLastError();
}
hipError_t launch_j3_grad(const MeasureArgs& m, int mixed, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || m.N > 256 || !m.j3scr) return hipErrorInvalidValue;
  if (mixed)
    hipLaunchKernelGGL(k_j3_grad<float>, dim3(m.W), dim3(j3_threads(m.N)), (size_t)15 * m.N * sizeof(float), st, m);
  else
    hipLaunchKernelGGL(k_j3_grad<double>, dim3(m.W), dim3(j3_threads(m.N)), (size_t)15 * m.N * sizeof(double), st, m);
  return hipGetLastError();
}
hipError_t launch_j3_forces(const MeasureArgs& m, int mixed, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || m.N > 256 || !m.j3scr) return hipErrorInvalidValue;
  if (mixed)
    hipLaunchKernelGGL(k_j3_forces<float>, dim3(m.W), dim3(j3_threads(m.N)), (size_t)15 * m.N * sizeof(float), st, m);
  else
    hipLaunchKernelGGL(k_j3_forces<double>, dim3(m.W), dim3(j3_threads(m.N)), (size_t)15 * m.N * sizeof(double), st,
                       m);
  return hipGetLastError();
}

}  // namespace vmc
