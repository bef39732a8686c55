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
// The sweep keeps G_a of every walker current (k_sweep_half's three-body variant); these kernels
// form G_a from the positions before the sweeps and evaluate the measurement's terms in FP64.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

namespace {

// Orbital components [value, grad(3), lap, hess xx yy zz xy xz yz, grad lap(3)] of chi_1 and chi_2
// at the offset whose sin and cos of pi d_m / L per axis are s, c.  Per axis, with rho = (L/pi) s,
// u = rho^2, u' = 2 rho c, u'' = 2 (c^2 - k rho^2), u''' = -8 k rho c (k = (pi/L)^2), the factors
// a = e^{-Z u} and b = u a have derivatives a^(q) = A_q e^{-Z u} and b^(q) = B_q e^{-Z u} with
//   A = (1, -Z u', Z^2 u'^2 - Z u'', -Z^3 u'^3 + 3 Z^2 u' u'' - Z u'''),
//   B = (u, u' + u A_1, u'' + 2 u' A_1 + u A_2, u''' + 3 u'' A_1 + 3 u' A_2 + u A_3);
// chi_1 = a a a and chi_2 = b a a + a b a + a a b, so every product carries e^{-Z (u_x + u_y + u_z)}.
__device__ __forceinline__ void prod14(const double f[3][4], double w, double o[14]) {
  const double p00 = f[1][0] * f[2][0], p01 = f[0][0] * f[2][0], p02 = f[0][0] * f[1][0];
  o[0] += w * f[0][0] * p00;
  o[1] += w * f[0][1] * p00;
  o[2] += w * f[1][1] * p01;
  o[3] += w * f[2][1] * p02;
  const double hxx = f[0][2] * p00, hyy = f[1][2] * p01, hzz = f[2][2] * p02;
  o[4] += w * (hxx + hyy + hzz);
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

__device__ __forceinline__ void j3_orbitals(const double s[3], const double c[3], double LoP, double kf, double c1[14],
                                            double c2[14]) {
  const double Z = kZJ;
  double A[3][4], B[3][4], usum = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double rho = LoP * s[m];
    const double u = rho * rho, u1 = 2.0 * rho * c[m], u2 = 2.0 * (c[m] * c[m] - kf * rho * rho);
    const double u3 = -8.0 * kf * rho * c[m];
    usum += u;
    A[m][0] = 1.0;
    A[m][1] = -Z * u1;
    A[m][2] = Z * Z * u1 * u1 - Z * u2;
    A[m][3] = -Z * Z * Z * u1 * u1 * u1 + 3.0 * Z * Z * u1 * u2 - Z * u3;
    B[m][0] = u;
    B[m][1] = u1 + u * A[m][1];
    B[m][2] = u2 + 2.0 * u1 * A[m][1] + u * A[m][2];
    B[m][3] = u3 + 3.0 * u2 * A[m][1] + 3.0 * u1 * A[m][2] + u * A[m][3];
  }
  const double E = exp(-Z * usum);
#pragma unroll
  for (int q = 0; q < 14; ++q) c1[q] = c2[q] = 0.0;
  prod14(A, E, c1);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double f[3][4];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
      for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? B[mm][q] : A[mm][q];
    prod14(f, E, c2);
  }
}

// x^T F y for 2-vectors, F = [[f0, f1], [f1, f2]]
__device__ __forceinline__ double fform(const double f[3], double x1, double x2, double y1, double y2) {
  return f[0] * x1 * y1 + f[1] * (x1 * y2 + x2 * y1) + f[2] * x2 * y2;
}

// sin and cos of pi (x_e - R_a)_m / L from the tables of both
__device__ __forceinline__ void pair_trig(const double* te, const double* ta, double s[3], double c[3]) {
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    s[m] = te[m] * ta[3 + m] - te[3 + m] * ta[m];
    c[m] = te[3 + m] * ta[3 + m] + te[m] * ta[m];
  }
}

}  // namespace

// G_a of every walker: one 256-thread block per walker, threads over nuclei.
__global__ __launch_bounds__(256) void k_j3_init(WalkerArgs a) {
  extern __shared__ __align__(16) double sm[];
  const int N = a.N, w = blockIdx.x, t = threadIdx.x;
  double* te = sm;            // N x 6: electrons' sin x3, cos x3
  double* ta = sm + 6 * N;    // N x 6: nuclei
  for (int u = t; u < 3 * N; u += 256) {
    const int i = u / 3, m = u % 3;
    sincospi(a.pos[(size_t)w * 3 * N + u] * a.invL, &te[6 * i + m], &te[6 * i + 3 + m]);
    sincospi(a.R[u] * a.invL, &ta[6 * i + m], &ta[6 * i + 3 + m]);
  }
  __syncthreads();
  const double LoP = a.L / VMC_PI;
  for (int c = t; c < N; c += 256) {
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
// [gU3 (3N), lU3 (N), U3]; threads over electrons for the per-electron sums, nuclei for G_a.
__global__ __launch_bounds__(256) void k_j3_grad(MeasureArgs m) {
  extern __shared__ __align__(16) double sm[];
  const int N = m.N, w = blockIdx.x, t = threadIdx.x;
  double* te = sm;
  double* ta = sm + 6 * N;
  double* G = sm + 12 * N;     // N x 2
  double* Q = sm + 14 * N;     // N: sum_i chi_ai^T F chi_ai
  __shared__ double red[4];
  for (int u = t; u < 3 * N; u += 256) {
    const int i = u / 3, mm = u % 3;
    sincospi(m.pos[(size_t)w * 3 * N + u] * m.invL, &te[6 * i + mm], &te[6 * i + 3 + mm]);
    sincospi(m.R[u] * m.invL, &ta[6 * i + mm], &ta[6 * i + 3 + mm]);
  }
  __syncthreads();
  const double LoP = m.L / VMC_PI, kf = (VMC_PI * m.invL) * (VMC_PI * m.invL);
  for (int c = t; c < N; c += 256) {
    double g1 = 0.0, g2 = 0.0, q = 0.0;
    for (int i = 0; i < N; ++i) {
      double u = 0.0;
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) {
        const double rt = LoP * (te[6 * i + mm] * ta[6 * c + 3 + mm] - te[6 * i + 3 + mm] * ta[6 * c + mm]);
        u += rt * rt;
      }
      const double v = exp(-kZJ * u);
      g1 += v;
      g2 += u * v;
      q += fform(m.j3f, v, u * v, v, u * v);
    }
    G[2 * c] = g1;
    G[2 * c + 1] = g2;
    Q[c] = q;
  }
  __syncthreads();
  double* out = m.j3scr + (size_t)w * j3_measure_doubles(N);
  for (int k = t; k < N; k += 256) {
    double gx = 0.0, gy = 0.0, gz = 0.0, lp = 0.0;
    for (int c = 0; c < N; ++c) {
      double s[3], cc[3], c1[14], c2[14];
      pair_trig(te + 6 * k, ta + 6 * c, s, cc);
      j3_orbitals(s, cc, LoP, kf, c1, c2);
      const double r1 = G[2 * c] - c1[0], r2 = G[2 * c + 1] - c2[0];
      gx += fform(m.j3f, c1[1], c2[1], r1, r2);
      gy += fform(m.j3f, c1[2], c2[2], r1, r2);
      gz += fform(m.j3f, c1[3], c2[3], r1, r2);
      lp += fform(m.j3f, c1[4], c2[4], r1, r2);
    }
    out[3 * k] = gx;
    out[3 * k + 1] = gy;
    out[3 * k + 2] = gz;
    out[3 * N + k] = lp;
  }
  // U_3 = 1/2 sum_a (G^T F G - Q_a), in a fixed order
  double part = 0.0;
  for (int c = t; c < N; c += 256) part += 0.5 * (fform(m.j3f, G[2 * c], G[2 * c + 1], G[2 * c], G[2 * c + 1]) - Q[c]);
  part = wave_allsum(part);
  if ((t & 63) == 0) red[t >> 6] = part;
  __syncthreads();
  if (t == 0) out[4 * N] = ((red[0] + red[1]) + red[2]) + red[3];
}

// After the Slater pass: the term's d/dR contributions to the accumulators, from the full grad U,
// grad ln|D| and E_L of the sample in the walker's scratch [.., gU (3N), gD (3N), E_L].  Threads over
// nuclei; each sums over the electrons in order.
__global__ __launch_bounds__(256) void k_j3_forces(MeasureArgs m) {
  extern __shared__ __align__(16) double sm[];
  const int N = m.N, w = blockIdx.x, t = threadIdx.x;
  double* te = sm;
  double* ta = sm + 6 * N;
  double* v = sm + 12 * N;     // N x 3: grad_k U + grad_k ln|D|
  const double* in = m.j3scr + (size_t)w * j3_measure_doubles(N);
  const double* gUf = in + 4 * N + 1;
  const double* gD = gUf + 3 * N;
  const double EL = gD[3 * N];
  for (int u = t; u < 3 * N; u += 256) {
    const int i = u / 3, mm = u % 3;
    sincospi(m.pos[(size_t)w * 3 * N + u] * m.invL, &te[6 * i + mm], &te[6 * i + 3 + mm]);
    sincospi(m.R[u] * m.invL, &ta[6 * i + mm], &ta[6 * i + 3 + mm]);
    v[u] = gUf[u] + gD[u];
  }
  __syncthreads();
  const double LoP = m.L / VMC_PI, kf = (VMC_PI * m.invL) * (VMC_PI * m.invL);
  // hessian component index of (mu, nu) in the 14-component layout
  auto hix = [](int mu, int nu) -> int {
    if (mu == nu) return 5 + mu;
    const int lo = mu < nu ? mu : nu, hi = mu < nu ? nu : mu;
    return lo == 0 ? (hi == 1 ? 8 : 9) : 10;
  };
  for (int c = t; c < N; c += 256) {
    // G_a and G_a,mu
    double G1 = 0.0, G2 = 0.0, Gm1[3] = {0, 0, 0}, Gm2[3] = {0, 0, 0};
    for (int k = 0; k < N; ++k) {
      double s[3], cc[3], c1[14], c2[14];
      pair_trig(te + 6 * k, ta + 6 * c, s, cc);
      j3_orbitals(s, cc, LoP, kf, c1, c2);
      G1 += c1[0];
      G2 += c2[0];
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) { Gm1[mu] += c1[1 + mu]; Gm2[mu] += c2[1 + mu]; }
    }
    double dln[3] = {0, 0, 0}, dT[3] = {0, 0, 0};
    for (int k = 0; k < N; ++k) {
      double s[3], cc[3], c1[14], c2[14];
      pair_trig(te + 6 * k, ta + 6 * c, s, cc);
      j3_orbitals(s, cc, LoP, kf, c1, c2);
      const double r1 = G1 - c1[0], r2 = G2 - c2[0];
      const double* vk = v + 3 * k;
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        const double q1 = Gm1[mu] - c1[1 + mu], q2 = Gm2[mu] - c2[1 + mu];
        dln[mu] -= fform(m.j3f, c1[1 + mu], c2[1 + mu], r1, r2);
        double d = 0.5 * (fform(m.j3f, c1[11 + mu], c2[11 + mu], r1, r2) + fform(m.j3f, c1[4], c2[4], q1, q2));
#pragma unroll
        for (int nu = 0; nu < 3; ++nu) {
          const int h = hix(mu, nu);
          d += vk[nu] * (fform(m.j3f, c1[h], c2[h], r1, r2) + fform(m.j3f, c1[1 + nu], c2[1 + nu], q1, q2));
        }
        dT[mu] += d;
      }
    }
    double* acc = m.acc + (size_t)w * (2 + 9 * N);
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      acc[2 + 3 * c + mu] += dT[mu];
      acc[2 + 3 * N + 3 * c + mu] += dln[mu];
      acc[2 + 6 * N + 3 * c + mu] += EL * dln[mu];
    }
  }
}

hipError_t launch_j3_init(const WalkerArgs& a, hipStream_t st) {
  if (a.W < 1 || a.N < 2 || a.N > 256 || !a.j3G) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_j3_init, dim3(a.W), dim3(256), (size_t)12 * a.N * sizeof(double), st, a);
  return hipGetLastError();
}
hipError_t launch_j3_grad(const MeasureArgs& m, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || m.N > 256 || !m.j3scr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_j3_grad, dim3(m.W), dim3(256), (size_t)15 * m.N * sizeof(double), st, m);
  return hipGetLastError();
}
hipError_t launch_j3_forces(const MeasureArgs& m, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || m.N > 256 || !m.j3scr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_j3_forces, dim3(m.W), dim3(256), (size_t)15 * m.N * sizeof(double), st, m);
  return hipGetLastError();
}

}  // namespace vmc
