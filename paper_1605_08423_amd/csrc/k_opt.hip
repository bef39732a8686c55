// Statistics for wavefunction optimisation.  The paper re-optimises the wavefunction before every
// ionic step and cites its optimiser, stochastic reconfiguration (SR; Sorella, PRB 64, 024512
// (2001)).  SR needs, over the sampled configurations, the local energy and the logarithmic
// derivatives O_k = d ln psi / d p_k of the variational parameters; here the Jastrow parameters
// p = (b, b_1, f_11, f_12, f_22, f_1, f_2):
//   b    two-body u = a rho / (1 + b rho):  O = sum_{i<j} -a_ij rho_ij^2 / (1 + b rho_ij)^2
//   b_1  one-body f(rho) = -(1 - e^{-beta rho}) / beta, beta = b_1 2^{1/4} (Eq. e:j1 with Z = 1):
//        O = sum_{i,a} 2^{1/4} [(1 - e^{-beta rho}) / beta^2 - rho e^{-beta rho} / beta]
//   F    three-body (Eq. e:j33): with G_q = sum_i chi_q(r_ia) and T_qr = sum_i chi_q chi_r per
//        proton, O_11 = 1/2 sum_a (G_1^2 - T_11), O_12 = sum_a (G_1 G_2 - T_12),
//        O_22 = 1/2 sum_a (G_2^2 - T_22)  (the pair sums sum_{i<j}, for any F).
//   f    one-body orbital part (Eq. e:j1): O_1 = sum_a G_1, O_2 = sum_a G_2 (for any f).
// k_opt_sample adds [E_L, O (7), E_L O (7), O O^T (49)] of every measured sample to its walker's
// sums; k_opt_reduce forms the means over walkers and samples in a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

namespace {

inline int opt_threads(int N) { return ((N + 63) / 64) * 64; }

}  // namespace

// One block per walker.  Thread i takes electron i: its pairs with the electrons i + 1 .. i + N/2
// (cyclically; the pair at distance N/2 only from its lower electron, so every pair is taken once
// and the threads share the pairs evenly) and with every proton; and proton i: the three-body
// sums over the electrons.  The terms are evaluated in the working precision of the Jastrow terms
// (FP32 in mixed precision) and summed over the block, and accumulated, in FP64.
template <class Real>
__global__ __launch_bounds__(256) void k_opt_sample(MeasureArgs m) {
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* te = reinterpret_cast<Real*>(smraw);   // N x 6: electrons' sin x3, cos x3 of pi x / L
  Real* ta = te + 6 * m.N;                     // N x 6: protons
  const int N = m.N, NS = m.NS, w = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  constexpr int P = kOptPar;
  __shared__ double red[4][P];
  __shared__ double Ob[P];
  const double* pos = m.pos + (size_t)w * 3 * N;
  for (int u = t; u < 3 * N; u += T) {
    const int i = u / 3, c = u % 3;
    dev_sincospi<Real>((Real)(pos[u] * m.invL), &te[6 * i + c], &te[6 * i + 3 + c]);
    dev_sincospi<Real>((Real)(m.R[u] * m.invL), &ta[6 * i + c], &ta[6 * i + 3 + c]);
  }
  __syncthreads();
  const Real LoP = (Real)(m.L / VMC_PI), bb = (Real)m.b, ap = (Real)m.a_par, aa = (Real)m.a_anti;
  Real o[P] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
  const int half = N / 2;
  for (int i = t; i < N; i += T) {
    const Real* si = te + 6 * i;
    // two-body
    const int dmax = i < half ? half : half - 1;
    for (int d = 1; d <= dmax; ++d) {
      const int j = i + d < N ? i + d : i + d - N;
      const Real* sj = te + 6 * j;
      Real r2 = Real(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const Real rt = LoP * (si[c] * sj[3 + c] - si[3 + c] * sj[c]);
        r2 += rt * rt;
      }
      const Real a = ((i < NS) == (j < NS)) ? ap : aa, den = Real(1) + bb * sqrt(r2);
      o[0] -= a * r2 / (den * den);
    }
    // one-body: d/db_1 of -(1 - e^{-beta rho}) / beta with beta = 2^{1/4} b_1
    if (m.j1_beta > 0.0) {
      const Real beta = (Real)m.j1_beta, ib = (Real)(1.0 / m.j1_beta), q = (Real)1.189207115002721;
      Real s1 = Real(0);
      for (int c = 0; c < N; ++c) {
        const Real* sa = ta + 6 * c;
        Real r2 = Real(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const Real rt = LoP * (si[d] * sa[3 + d] - si[3 + d] * sa[d]);
          r2 += rt * rt;
        }
        const Real rho = sqrt(r2), e = dev_exp<Real>(-beta * rho);
        s1 += ((Real(1) - e) * ib - rho * e) * ib;
      }
      o[1] += q * s1;
    }
  }
  // three-body: per proton the sums over the electrons
  const Real Z = (Real)kZJ;
  for (int c = t; c < N; c += T) {
    const Real* sa = ta + 6 * c;
    Real g1 = Real(0), g2 = Real(0), t11 = Real(0), t12 = Real(0), t22 = Real(0);
    for (int i = 0; i < N; ++i) {
      const Real* si = te + 6 * i;
      Real u = Real(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const Real rt = LoP * (si[d] * sa[3 + d] - si[3 + d] * sa[d]);
        u += rt * rt;
      }
      const Real v1 = dev_exp<Real>(-Z * u), v2 = u * v1;
      g1 += v1;
      g2 += v2;
      t11 += v1 * v1;
      t12 += v1 * v2;
      t22 += v2 * v2;
    }
    const double G1 = (double)g1, G2 = (double)g2;
    o[2] += (Real)(0.5 * (G1 * G1 - (double)t11));
    o[3] += (Real)(G1 * G2 - (double)t12);
    o[4] += (Real)(0.5 * (G2 * G2 - (double)t22));
    o[5] += g1;
    o[6] += g2;
  }
  // fixed-order block sums in FP64
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const double v = wave_allsum((double)o[k]);
    if ((t & 63) == 0) red[t >> 6][k] = v;
  }
  __syncthreads();
  if (t < P) {
    double s = red[0][t];
    for (int q = 1; q < T / 64; ++q) s += red[q][t];
    Ob[t] = s;
  }
  __syncthreads();
  const double EL = m.ELs[w];
  double* out = m.popt + (size_t)w * kOptStats;
  if (t == 0) out[0] += EL;
  if (t < P) {
    out[1 + t] += Ob[t];
    out[1 + P + t] += EL * Ob[t];
  }
  if (t < P * P) out[1 + 2 * P + t] += Ob[t / P] * Ob[t % P];
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

hipError_t launch_opt_sample(const MeasureArgs& m, int mixed, hipStream_t st) {
  if (m.W < 1 || m.N < 2 || (m.N & 1) || m.N > 256 || !m.popt || !m.ELs) return hipErrorInvalidValue;
  if (mixed)
    hipLaunchKernelGGL(k_opt_sample<float>, dim3(m.W), dim3(opt_threads(m.N)), (size_t)12 * m.N * sizeof(float), st,
                       m);
  else
    hipLaunchKernelGGL(k_opt_sample<double>, dim3(m.W), dim3(opt_threads(m.N)), (size_t)12 * m.N * sizeof(double),
                       st, m);
  return hipGetLastError();
}

hipError_t launch_opt_reduce(int W, int M, const double* popt, double* out, hipStream_t st) {
  if (W < 1 || M < 1 || !popt || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_opt_reduce, dim3(kOptStats), dim3(256), 0, st, W, 1.0 / ((double)W * (double)M), popt, out);
  return hipGetLastError();
}

}  // namespace vmc
