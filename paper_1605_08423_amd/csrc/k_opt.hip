// Statistics for wavefunction optimisation.  The paper re-optimises the wavefunction before every
// ionic step and cites its optimiser, stochastic reconfiguration (SR; Sorella, PRB 64, 024512
// (2001)).  SR needs, over the sampled configurations, the local energy and the logarithmic
// derivatives O_k = d ln psi / d p_k of the variational parameters; here the Jastrow parameters
// p = (b, b_1, f_11, f_12, f_22):
//   b    two-body u = a rho / (1 + b rho):  O = sum_{i<j} -a_ij rho_ij^2 / (1 + b rho_ij)^2
//   b_1  one-body f(rho) = -(1 - e^{-beta rho}) / beta, beta = b_1 2^{1/4} (Eq. e:j1 with Z = 1):
//        O = sum_{i,a} 2^{1/4} [(1 - e^{-beta rho}) / beta^2 - rho e^{-beta rho} / beta]
//   F    three-body (Eq. e:j33): with G_q = sum_i chi_q(r_ia) and T_qr = sum_i chi_q chi_r per
//        proton, O_11 = 1/2 sum_a (G_1^2 - T_11), O_12 = sum_a (G_1 G_2 - T_12),
//        O_22 = 1/2 sum_a (G_2^2 - T_22)  (the pair sums sum_{i<j}, for any F).
// k_opt_sample adds [E_L, O (5), E_L O (5), O O^T (25)] of every measured sample to its walker's
// sums; k_opt_reduce forms the means over walkers and samples in a fixed order.  FP64 throughout.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

namespace {

inline int opt_threads(int N) { return ((N + 63) / 64) * 64; }

}  // namespace

// One block per walker; thread i takes electron i (its pairs with every other electron, halved,
// and with every proton) and proton i (the three-body sums over the electrons).
__global__ __launch_bounds__(256) void k_opt_sample(MeasureArgs m) {
  extern __shared__ __align__(16) double sm[];
  const int N = m.N, NS = m.NS, w = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  double* te = sm;            // N x 6: electrons' sin x3, cos x3 of pi x / L
  double* ta = sm + 6 * N;    // N x 6: protons
  __shared__ double red[4][5];
  __shared__ double Ob[5];
  const double* pos = m.pos + (size_t)w * 3 * N;
  for (int u = t; u < 3 * N; u += T) {
    const int i = u / 3, c = u % 3;
    sincospi(pos[u] * m.invL, &te[6 * i + c], &te[6 * i + 3 + c]);
    sincospi(m.R[u] * m.invL, &ta[6 * i + c], &ta[6 * i + 3 + c]);
  }
  __syncthreads();
  const double LoP = m.L / VMC_PI;
  double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = t; i < N; i += T) {
    const double* si = te + 6 * i;
    // two-body: every other electron, half of each pair to each of its electrons
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      const double* sj = te + 6 * j;
      double r2 = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double rt = LoP * (si[c] * sj[3 + c] - si[3 + c] * sj[c]);
        r2 += rt * rt;
      }
      const double rho = sqrt(r2), a = ((i < NS) == (j < NS)) ? m.a_par : m.a_anti;
      const double den = 1.0 + m.b * rho;
      o[0] += -0.5 * a * r2 / (den * den);
    }
    // one-body
    if (m.j1_beta > 0.0) {
      const double beta = m.j1_beta, q = 1.189207115002721;   // 2^{1/4} = d beta / d b_1
      for (int c = 0; c < N; ++c) {
        const double* sa = ta + 6 * c;
        double r2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double rt = LoP * (si[d] * sa[3 + d] - si[3 + d] * sa[d]);
          r2 += rt * rt;
        }
        const double rho = sqrt(r2), e = exp(-beta * rho);
        o[1] += q * ((1.0 - e) / (beta * beta) - rho * e / beta);
      }
    }
  }
  // three-body: per proton the sums over the electrons
  for (int c = t; c < N; c += T) {
    const double* sa = ta + 6 * c;
    double g1 = 0.0, g2 = 0.0, t11 = 0.0, t12 = 0.0, t22 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double* si = te + 6 * i;
      double u = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double rt = LoP * (si[d] * sa[3 + d] - si[3 + d] * sa[d]);
        u += rt * rt;
      }
      const double v1 = exp(-kZJ * u), v2 = u * v1;
      g1 += v1;
      g2 += v2;
      t11 += v1 * v1;
      t12 += v1 * v2;
      t22 += v2 * v2;
    }
    o[2] += 0.5 * (g1 * g1 - t11);
    o[3] += g1 * g2 - t12;
    o[4] += 0.5 * (g2 * g2 - t22);
  }
  // fixed-order block sums
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double v = wave_allsum(o[k]);
    if ((t & 63) == 0) red[t >> 6][k] = v;
  }
  __syncthreads();
  if (t < 5) {
    double s = red[0][t];
    for (int q = 1; q < T / 64; ++q) s += red[q][t];
    Ob[t] = s;
  }
  __syncthreads();
  const double EL = m.ELs[w];
  double* out = m.popt + (size_t)w * kOptStats;
  if (t == 0) out[0] += EL;
  if (t < 5) {
    out[1 + t] += Ob[t];
    out[6 + t] += EL * Ob[t];
  }
  if (t < 25) out[11 + t] += Ob[t / 5] * Ob[t % 5];
}

// Means over W walkers and M samples each: column q of the per-walker sums, one block per column,
// strided partial sums then the wave and block sums in a fixed order.
__global__ __launch_bounds__(256) void k_opt_reduce(int W, double inv_samples, const double* popt, double* out) {
  __shared__ double red[4];
  const int q = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int w = t; w < W; w += 256) s += popt[(size_t)w * kOptStats + q];
  s = wave_allsum(s);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) out[q] = (((red[0] + red[1]) + red[2]) + red[3]) * inv_samples;
}

hipError_t launch_opt_sample(const MeasureArgs& m, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || m.N > 256 || !m.popt || !m.ELs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_opt_sample, dim3(m.W), dim3(opt_threads(m.N)), (size_t)12 * m.N * sizeof(double), st, m);
  return hipGetLastError();
}

hipError_t launch_opt_reduce(int W, int M, const double* popt, double* out, hipStream_t st) {
  if (W < 1 || M < 1 || !popt || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_opt_reduce, dim3(kOptStats), dim3(256), 0, st, W, 1.0 / ((double)W * (double)M), popt, out);
  return hipGetLastError();
}

}  // namespace vmc
