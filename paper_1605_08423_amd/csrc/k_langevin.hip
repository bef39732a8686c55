// Estimators, acceleration matrix and the Langevin step (a7-a10).
//   E = mean_w e_w, sigma_E = sd_w(e_w)/sqrt(W), f_w = -(d_w + 2 (h_w - E g_w)), f = mean_w f_w
//   S = sum_w (f_w - f)(f_w - f)^T / (W (W - 1))       (covariance of the mean force)
//   R' = R + Dt S^-1 [f - (S_prev - S)(R_prev - R)/(2 Db)] + sqrt(2 T Db) z,  z = L^-T xi
// All reductions use a fixed order so results are bitwise reproducible.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

constexpr int RED_CHUNK = 256;      // walkers per partial column sum

__device__ __forceinline__ double block_sum1024(double v, double* sh) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  for (int k = 0; k < 16; ++k) r += sh[k];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void k_reduce_E(int W, int stride, const double* means, const int64_t* nacc,
                                                   double moves_per_walker, double* out) {
  __shared__ double sh[16];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int w = t; w < W; w += 1024) s += means[(size_t)w * stride];
  const double E = block_sum1024(s, sh) / (double)W;
  double v = 0.0, a = 0.0;
  for (int w = t; w < W; w += 1024) {
    const double d = means[(size_t)w * stride] - E;
    v += d * d;
    a += (double)nacc[w];
  }
  v = block_sum1024(v, sh);
  a = block_sum1024(a, sh);
  if (t == 0) {
    out[0] = E;
    out[1] = (W > 1) ? sqrt(v / (double)(W - 1)) / sqrt((double)W) : 0.0;
    out[2] = a / ((double)W * moves_per_walker);
  }
}

__global__ void k_fw(int W, int n3, const double* means, const double* out, double* f_w) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)W * n3) return;
  const int w = (int)(idx / n3), t = (int)(idx % n3);
  const double* mw = means + (size_t)w * (1 + 3 * n3);
  const double E = out[0];
  f_w[idx] = -(mw[1 + t] + 2.0 * (mw[1 + 2 * n3 + t] - E * mw[1 + n3 + t]));
}

__global__ void k_colsum_partial(int W, int n3, const double* f_w, double* partial) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x, ch = blockIdx.y;
  if (t >= n3) return;
  const int w0 = ch * RED_CHUNK, w1 = min(W, w0 + RED_CHUNK);
  double s = 0.0;
  for (int w = w0; w < w1; ++w) s += f_w[(size_t)w * n3 + t];
  partial[(size_t)ch * n3 + t] = s;
}

__global__ void k_colsum_final(int W, int n3, int nch, const double* partial, double* f) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += partial[(size_t)c * n3 + t];
  f[t] = s / (double)W;
}

size_t reduce_partial_doubles(int W, int n3) { return (size_t)((W + RED_CHUNK - 1) / RED_CHUNK) * n3; }

hipError_t launch_reduce(int W, int n3, const double* means, const int64_t* nacc, double moves_per_walker,
                         double* f_w, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_E, dim3(1), dim3(1024), 0, st, W, 1 + 3 * n3, means, nacc, moves_per_walker, out);
  size_t tot = (size_t)W * n3;
  hipLaunchKernelGGL(k_fw, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, W, n3, means, out, f_w);
  const int nch = (W + RED_CHUNK - 1) / RED_CHUNK;
  hipLaunchKernelGGL(k_colsum_partial, dim3((n3 + 255) / 256, nch), dim3(256), 0, st, W, n3, f_w, partial);
  hipLaunchKernelGGL(k_colsum_final, dim3((n3 + 255) / 256), dim3(256), 0, st, W, n3, nch, partial, out + 3);
  return hipGetLastError();
}

// ---------------------------------------------------------------- SYRK ---
// S = sum_w (f_w - f)(f_w - f)^T / (W (W - 1)) on the FP64 matrix cores.  A work-group takes
// one 64 x 64 tile (bi, bj), bi >= bj, of the lower block triangle and one chunk of walkers;
// each of its four waves owns a 32 x 32 quadrant (2 x 2 matrix-core tiles) and runs over the
// whole chunk, four walkers per step: lane l supplies a_w[i] for walker 4 s + l / 16 and
// column l % 16 of the quadrant's row and column tiles (a_w = f_w - f), so every load is a
// 128-byte row segment.  Chunks write partial sums; k_syrk_final adds them in chunk order and
// takes every element from the lower triangle, so S is exactly symmetric and the result does
// not depend on the launch.
constexpr int SYRK_T = 64;         // S tile edge
constexpr int SYRK_MAXCH = 32;     // walker chunks (partial sums)

typedef double d4s_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4s_t mfma_s(double av, double bv, d4s_t acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
}

static int syrk_chunks(int W) { return W / 512 < 1 ? 1 : (W / 512 > SYRK_MAXCH ? SYRK_MAXCH : W / 512); }

__global__ __launch_bounds__(256) void k_syrk_partial(int W, int n3, int nch, const double* f_w, const double* f,
                                                      double* partial) {
  // tile pair from the linear index over the lower block triangle: t = bi (bi + 1) / 2 + bj
  const int t = blockIdx.x, ch = blockIdx.y;
  int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, l4 = lane >> 4;
  const int r0 = bi * SYRK_T + (wv >> 1) * 32, c0 = bj * SYRK_T + (wv & 1) * 32;
  const int w0 = (int)((long long)W * ch / nch), w1 = (int)((long long)W * (ch + 1) / nch);
  int ca[2], cb[2];
  double fa[2], fb[2];
  bool oka[2], okb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    ca[q] = r0 + 16 * q + l16;
    cb[q] = c0 + 16 * q + l16;
    oka[q] = ca[q] < n3;
    okb[q] = cb[q] < n3;
    fa[q] = oka[q] ? f[ca[q]] : 0.0;
    fb[q] = okb[q] ? f[cb[q]] : 0.0;
  }
  d4s_t acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4s_t{0.0, 0.0, 0.0, 0.0};
  // 32 walkers per iteration: all 32 loads are issued before the first product, so a
  // wave keeps them in flight together
  constexpr int UN = 8;
  for (int wb = w0; wb < w1; wb += 4 * UN) {
    double av[UN][2], bv[UN][2];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int w = wb + 4 * u + l4;
      const bool okw = w < w1;
      const double* row = f_w + (size_t)(okw ? w : w0) * n3;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double x = row[oka[q] ? ca[q] : 0], y = row[okb[q] ? cb[q] : 0];
        av[u][q] = (okw && oka[q]) ? x - fa[q] : 0.0;
        bv[u][q] = (okw && okb[q]) ? y - fb[q] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = mfma_s(av[u][p], bv[u][q], acc[p][q]);
  }
  double* P = partial + (size_t)ch * n3 * n3;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + 16 * p + l4 + 4 * v, j = c0 + 16 * q + l16;
        if (i < n3 && j < n3) P[(size_t)i * n3 + j] = acc[p][q][v];
      }
}

__global__ void k_syrk_final(int W, int n3, int nch, const double* partial, double* S) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n3 * n3) return;
  const int i0 = (int)(idx / n3), j0 = (int)(idx % n3);
  const int i = i0 > j0 ? i0 : j0, j = i0 > j0 ? j0 : i0;   // the lower-triangle element
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += partial[(size_t)c * n3 * n3 + (size_t)i * n3 + j];
  S[idx] = s / ((double)W * (double)(W - 1));
}

size_t syrk_partial_doubles(int W, int n3) { return (size_t)syrk_chunks(W) * n3 * n3; }

hipError_t launch_syrk(int W, int n3, const double* f_w, const double* f, double* partial, double* S,
                       hipStream_t st) {
  const int nt = (n3 + SYRK_T - 1) / SYRK_T, nch = syrk_chunks(W);
  hipLaunchKernelGGL(k_syrk_partial, dim3(nt * (nt + 1) / 2, nch), dim3(256), 0, st, W, n3, nch, f_w, f, partial);
  const size_t tot = (size_t)n3 * n3;
  hipLaunchKernelGGL(k_syrk_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, W, n3, nch, partial, S);
  return hipGetLastError();
}

// ------------------------------------------------------------ Langevin ---
// One step of Eq. finaldyn_new as a short launch sequence on the step's work area
// (langevin_work_doubles(n3): the factor L in n3 x n3, then the vectors v, y, z and R'):
//   k_lang_prep      L <- S (or I), v = f - (S_prev - S)(R_prev - R)/(2 Db), status <- 0
//   k_chol_panel     per 64-column panel k: the diagonal block's Cholesky factor (in LDS, every
//                    work-group alike) and the panel below it, L_ik = A_ik L_kk^-T
//   k_chol_update    the trailing update A_ij -= L_ik L_jk^T on the FP64 matrix cores
//   k_lang_solve     one work-group: y = S^-1 v and z = L^-T xi by blocked triangular solves,
//                    the finite checks and R' = R + Dt y + sqrt(2 T Db) z (wrapped) into the work
//   k_lang_commit    if the step succeeded: (R_prev, R, S_prev) <- (R, R', S)
// status: 0 ok, 1 bad temperature or a non-finite position, force or noise, 3 S not positive
// definite; every kernel after the first returns at once once it is set, so a failed step
// changes nothing.  Every path writes the status word (nothing needs clearing beforehand).
constexpr int LANG_MAX = 1536;
constexpr int CHB = 64;            // panel width of the blocked Cholesky

__global__ __launch_bounds__(256) void k_lang_prep(int n3, double L, const double* R, const double* R_prev,
                                                   const double* S_prev, const double* f, const double* S,
                                                   double* Lw, double Delta, double alpha, unsigned flags,
                                                   int* status) {
  const bool cfold = flags & 1u, no_scorr = flags & 4u;
  const double Db = alpha > 0.0 ? -expm1(-2.0 * alpha * Delta) / (2.0 * alpha) : Delta;
  const int lane = threadIdx.x & 63, i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
  if (i >= n3) return;
  const double invL = L > 0.0 ? 1.0 / L : 0.0;
  double c = 0.0;
  for (int j = lane; j < n3; j += 64) {
    const double s = S[(size_t)i * n3 + j];
    Lw[(size_t)i * n3 + j] = cfold ? (i == j ? 1.0 : 0.0) : (j <= i ? s : 0.0);
    if (!no_scorr && !cfold) {
      double d = R_prev[j] - R[j];
      if (L > 0.0) d = min_image(d, L, invL);
      c = fma(S_prev[(size_t)i * n3 + j] - s, d, c);
    }
  }
  c = wave_sum(c);
  if (lane == 0) Lw[(size_t)n3 * n3 + i] = f[i] - c / (2.0 * Db);   // v
}

// Diagonal block of panel k (every work-group factors it alike, so no work-group waits for
// another), then work-group 0 writes it and work-group g >= 1 solves row block k + g of the
// panel.  A block narrower than 64 (the last one) is padded with the identity, which the
// factorisation and the solve leave as it is, so the code has no data-size branches.  The
// factorisation runs in wave 0 with lane r holding row r in registers: at column j the pivot
// comes by readlane, the column l_rj is formed in the lanes and published through LDS, and
// every lane updates its row with broadcast reads of that column.  The row-block solve
// X L_kk^T = A runs the same way, lane r holding row r of X.
__global__ __launch_bounds__(256) void k_chol_panel(int n3, int k, double* Lw, int* status) {
  __shared__ double D[CHB][CHB + 1];
  __shared__ double col[CHB];
  __shared__ int fail;
  if (*status) return;
  const int t = threadIdx.x, lane = t & 63;
  const int kb = k * CHB, nb = min(CHB, n3 - kb);
  if (t == 0) fail = 0;
  for (int u = t; u < CHB * CHB; u += 256) {
    const int r = u / CHB, c = u % CHB;
    D[r][c] = (r < nb && c < nb) ? (c <= r ? Lw[(size_t)(kb + r) * n3 + kb + c] : 0.0) : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  if (t < 64) {
    double row[CHB];
#pragma unroll
    for (int c = 0; c < CHB; ++c) row[c] = D[lane][c];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < CHB; ++j) {
      const double piv = readlane_d(row[j], j);
      bad = bad || !(piv > 0.0);
      const double ljj = sqrt(piv);
      const double lrj = lane == j ? ljj : (lane > j ? row[j] / ljj : 0.0);
      row[j] = lrj;
      col[lane] = lrj;
      wave_lds_sync();
#pragma unroll
      for (int c = j + 1; c < CHB; ++c) row[c] = fma(-lrj, col[c], row[c]);
      wave_lds_sync();
    }
    if (bad) {
      if (lane == 0) fail = 1;
    } else {
#pragma unroll
      for (int c = 0; c < CHB; ++c) D[lane][c] = row[c];
    }
  }
  __syncthreads();
  if (fail) {
    if (blockIdx.x == 0 && t == 0) *status = 3;
    return;
  }
  // every factor element is also written transposed into the unused upper triangle, where
  // the forward substitution of the solve reads it along rows
  if (blockIdx.x == 0) {
    for (int u = t; u < nb * nb; u += 256) {
      const int r = u / nb, c = u % nb;
      Lw[(size_t)(kb + r) * n3 + kb + c] = c <= r ? D[r][c] : D[c][r];
    }
    return;
  }
  // row block ib (nb = 64 here: only the last panel is narrower, and it has no blocks below)
  const int ib = kb + CHB * blockIdx.x, mb = min(CHB, n3 - ib);
  if (t < 64) {
    double row[CHB];
#pragma unroll
    for (int c = 0; c < CHB; ++c) row[c] = lane < mb ? Lw[(size_t)(ib + lane) * n3 + kb + c] : 0.0;
#pragma unroll
    for (int c = 0; c < CHB; ++c) {
      const double xc = row[c] / D[c][c];
      row[c] = xc;
#pragma unroll
      for (int c2 = c + 1; c2 < CHB; ++c2) row[c2] = fma(-xc, D[c2][c], row[c2]);
    }
    if (lane < mb) {
#pragma unroll
      for (int c = 0; c < CHB; ++c) Lw[(size_t)(ib + lane) * n3 + kb + c] = row[c];
    }
#pragma unroll
    for (int c = 0; c < CHB; ++c)
      if (lane < mb) Lw[(size_t)(kb + c) * n3 + ib + lane] = row[c];
  }
}

// Trailing update after panel k: for row and column blocks bi >= bj > k,
// A_ij -= L_ik L_jk^T; the two 64 x 64 panel blocks are staged in LDS, each wave computes a
// 32 x 32 quadrant with the FP64 matrix cores.
__global__ __launch_bounds__(256) void k_chol_update(int n3, int k, double* Lw, const int* status) {
  __shared__ double Li[CHB][CHB + 1];
  __shared__ double Lj[CHB][CHB + 1];
  if (*status) return;
  const int t = blockIdx.x;
  int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  const int bi = k + 1 + a, bj = k + 1 + (t - a * (a + 1) / 2);
  const int kb = k * CHB, ib = bi * CHB, jb = bj * CHB;
  for (int u = threadIdx.x; u < CHB * CHB; u += 256) {
    const int r = u / CHB, c = u % CHB;
    Li[r][c] = (ib + r < n3) ? Lw[(size_t)(ib + r) * n3 + kb + c] : 0.0;
    Lj[r][c] = (jb + r < n3) ? Lw[(size_t)(jb + r) * n3 + kb + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, l4 = lane >> 4;
  const int qr = (wv >> 1) * 32, qc = (wv & 1) * 32;
  d4s_t acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib + qr + 16 * p + l4 + 4 * v, j = jb + qc + 16 * q + l16;
        acc[p][q][v] = (i < n3 && j < n3) ? Lw[(size_t)i * n3 + j] : 0.0;
      }
#pragma unroll 4
  for (int s = 0; s < CHB / 4; ++s) {
    double av[2], bv[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      av[p] = -Li[qr + 16 * p + l16][4 * s + l4];
      bv[p] = Lj[qc + 16 * p + l16][4 * s + l4];
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = mfma_s(av[p], bv[q], acc[p][q]);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib + qr + 16 * p + l4 + 4 * v, j = jb + qc + 16 * q + l16;
        if (i < n3 && j < n3 && j <= i) Lw[(size_t)i * n3 + j] = acc[p][q][v];
      }
}

// One work-group of 1024 threads: Teff check, y = S^-1 v (L w = v, L^T y = w) and z = L^-T xi
// by 64-row blocks (the diagonal block's substitution by wave 0 from LDS, the off-diagonal
// products by all waves), the finite checks and R' into the work area.
__global__ __launch_bounds__(1024) void k_lang_solve(int n3, double L, const double* R, const double* R_prev,
                                                    double* Lw, double T, double Delta, double alpha,
                                                    unsigned flags, uint32_t seed, uint32_t traj, uint32_t step,
                                                    int* status) {
  __shared__ double D[CHB][CHB + 1];
  __shared__ double y[LANG_MAX];
  __shared__ double z[LANG_MAX];
  __shared__ int bad;
  if (*status) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const bool noise_corr = flags & 2u;
  double Dt = Delta, Db = Delta;
  if (alpha > 0.0) {
    Dt = -expm1(-alpha * Delta) / alpha;
    Db = -expm1(-2.0 * alpha * Delta) / (2.0 * alpha);
  }
  const double Teff = noise_corr ? T - Dt * Dt / (2.0 * Db) : T;
  if (Teff < 0.0) {
    if (t == 0) *status = 1;
    return;
  }
  const double* v = Lw + (size_t)n3 * n3;
  double* Rn = Lw + (size_t)n3 * n3 + n3;
  for (int i = t; i < n3; i += 1024) y[i] = v[i];
  // xi by Box-Muller pairs: pair j from counter (step, 0xFFFFFFFF, j, 0)
  for (int j = t; 2 * j < n3; j += 1024) {
    const u32x4 o = philox(step, 0xFFFFFFFFu, (uint32_t)j, 0u, seed, traj);
    const double u1 = u01(o.x, o.y), u2 = u01(o.z, o.w);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z[2 * j] = rad * c;
    if (2 * j + 1 < n3) z[2 * j + 1] = rad * s;
  }
  if (t == 0) bad = 0;
  const int nblk = (n3 + CHB - 1) / CHB;
  // forward: L w = v (in y)
  for (int kb = 0; kb < nblk; ++kb) {
    const int b0 = kb * CHB, nb = min(CHB, n3 - b0);
    __syncthreads();
    for (int u = t; u < CHB * CHB; u += 1024) {
      const int r = u / CHB, c = u % CHB;
      D[r][c] = (r < nb && c < nb) ? Lw[(size_t)(b0 + r) * n3 + b0 + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    if (wv == 0) {
      // lane r holds x_r; step j: x_j = x_j / L_jj goes to every lane by readlane, and the
      // lanes below subtract L_rj x_j (the division by the diagonal is a multiplication by its
      // reciprocal, formed for all j at once before the chain of steps)
      double x = lane < nb ? y[b0 + lane] : 0.0;
      const double rd = 1.0 / D[lane][lane];
#pragma unroll
      for (int j = 0; j < CHB; ++j) {
        const double wj = readlane_d(x, j) * readlane_d(rd, j);
        const double lj = D[lane][j];
        x = lane == j ? wj : (lane > j ? fma(-lj, wj, x) : x);
      }
      if (lane < nb) y[b0 + lane] = x;
    }
    __syncthreads();
    // rows below the block: y_r -= L[r][block] w_block, one thread per row, reading the
    // transposed copy of L (upper triangle) so that the threads' loads are consecutive
    for (int r = b0 + nb + t; r < n3; r += 1024) {
      double s = 0.0;
      for (int c0 = 0; c0 < nb; c0 += 16) {
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = c0 + u < nb ? Lw[(size_t)(b0 + c0 + u) * n3 + r] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < nb) s = fma(l[u], y[b0 + c0 + u], s);
      }
      y[r] -= s;
    }
  }
  // backward: L^T y = w and L^T z = xi together
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int b0 = kb * CHB, nb = min(CHB, n3 - b0);
    __syncthreads();
    for (int u = t; u < CHB * CHB; u += 1024) {
      const int r = u / CHB, c = u % CHB;
      D[r][c] = (r < nb && c < nb) ? Lw[(size_t)(b0 + r) * n3 + b0 + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    if (wv < 2) {
      double* x_v = wv == 0 ? y : z;
      double x = lane < nb ? x_v[b0 + lane] : 0.0;
      const double rd = 1.0 / D[lane][lane];
#pragma unroll
      for (int j = CHB - 1; j >= 0; --j) {
        const double xj = readlane_d(x, j) * readlane_d(rd, j);
        const double lj = D[j][lane];
        x = lane == j ? xj : (lane < j ? fma(-lj, xj, x) : x);
      }
      if (lane < nb) x_v[b0 + lane] = x;
    }
    __syncthreads();
    // rows above the block: x_r -= sum_i L[b0 + i][r] x_i, one thread per row (coalesced over r)
    for (int r = t; r < b0; r += 1024) {
      double sy = 0.0, sz = 0.0;
      for (int i0 = 0; i0 < nb; i0 += 16) {
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = i0 + u < nb ? Lw[(size_t)(b0 + i0 + u) * n3 + r] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (i0 + u < nb) {
            sy = fma(l[u], y[b0 + i0 + u], sy);
            sz = fma(l[u], z[b0 + i0 + u], sz);
          }
      }
      y[r] -= sy;
      z[r] -= sz;
    }
  }
  __syncthreads();
  // a non-finite position, force, S-difference term or noise is an argument error
  for (int i = t; i < n3; i += 1024)
    if (!isfinite(y[i]) || !isfinite(z[i]) || !isfinite(R[i]) || !isfinite(R_prev[i])) bad = 1;
  __syncthreads();
  if (bad) {
    if (t == 0) *status = 1;
    return;
  }
  const double amp = sqrt(2.0 * Teff * Db), invL = L > 0.0 ? 1.0 / L : 0.0;
  for (int i = t; i < n3; i += 1024) {
    double rn = R[i] + Dt * y[i] + amp * z[i];
    if (L > 0.0) rn = wrap_box(rn, L, invL);
    Rn[i] = rn;
  }
}

__global__ __launch_bounds__(256) void k_lang_commit(int n3, double* R, double* R_prev, double* S_prev,
                                                     const double* S, const double* Lw, const int* status) {
  if (*status) return;
  const double* Rn = Lw + (size_t)n3 * n3 + n3;
  const size_t nS = (size_t)n3 * n3;
  for (size_t u = (size_t)blockIdx.x * 256 + threadIdx.x; u < nS + n3; u += (size_t)gridDim.x * 256) {
    if (u < nS) {
      S_prev[u] = S[u];
    } else {
      const size_t i = u - nS;
      R_prev[i] = R[i];
      R[i] = Rn[i];
    }
  }
}

// Device scratch of vmc_langevin_step_noalloc: the work of one Langevin step (langevin_work_doubles)
// for 3N <= LANG_NOALLOC_MAX, then its status word.  One array per device, shared by every call on
// that device (each device holds it until the process ends).  Host code never names the array in
// a kernel argument or copy: it takes the device address from langevin_scratch_address.
constexpr int LANG_NOALLOC_MAX = 768;
static __device__ __align__(256) double scratch[(size_t)LANG_NOALLOC_MAX * LANG_NOALLOC_MAX +
                                                 16 * LANG_NOALLOC_MAX + 32];

size_t langevin_work_doubles(int n3) { return (size_t)n3 * n3 + 16 * (size_t)n3; }
int langevin_noalloc_max() { return LANG_NOALLOC_MAX; }
// With the device current: the address of that device's copy of the array.
hipError_t langevin_scratch_address(double** ptr) { return hipGetSymbolAddress((void**)ptr, HIP_SYMBOL(scratch)); }
size_t langevin_scratch_status_offset() { return langevin_work_doubles(LANG_NOALLOC_MAX); }

hipError_t launch_langevin(int n3, double L, double* R, double* R_prev, double* S_prev, const double* f,
                           const double* S, double* Lwork, double* vwork, double T, double Delta, double alpha,
                           unsigned flags, uint32_t seed, uint32_t traj, uint32_t step, int* status,
                           hipStream_t st) {
  (void)vwork;
  if (n3 < 1 || n3 > LANG_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lang_prep, dim3((n3 + 3) / 4), dim3(256), 0, st, n3, L, R, R_prev, S_prev, f, S, Lwork,
                     Delta, alpha, flags, status);
  if (!(flags & 1u)) {          // S = I needs no factorisation
    const int nblk = (n3 + CHB - 1) / CHB;
    for (int k = 0; k < nblk; ++k) {
      hipLaunchKernelGGL(k_chol_panel, dim3(nblk - k), dim3(256), 0, st, n3, k, Lwork, status);
      const int m = nblk - k - 1;
      if (m > 0) hipLaunchKernelGGL(k_chol_update, dim3(m * (m + 1) / 2), dim3(256), 0, st, n3, k, Lwork, status);
    }
  }
  hipLaunchKernelGGL(k_lang_solve, dim3(1), dim3(1024), 0, st, n3, L, R, R_prev, Lwork, T, Delta, alpha, flags,
                     seed, traj, step, status);
  const size_t tot = (size_t)n3 * n3 + n3;
  const unsigned nb = (unsigned)std::min<size_t>((tot + 255) / 256, 1024);
  hipLaunchKernelGGL(k_lang_commit, dim3(nb), dim3(256), 0, st, n3, R, R_prev, S_prev, S, Lwork, status);
  return hipGetLastError();
}

// ---------------------------------------------------------- toy model ---
// The rotating spring of the SI ("A simple toy model"): U = k (|x| - a)^2 / 2 in the plane,
// with S = G_lambda (radial eigenvalue 1/lambda, tangential 1), S = H + mu G_lambda (H the
// Hessian of U) or S = I.  One thread per independent trajectory; trajectory i draws its
// noise with key (seed, i) at counter step t, the numbers of the single-trajectory step.
// Schemes: 0 Eq. finaldyn_new (alpha = 0 gives Eq. finaldyn), 1 Eq. norogna (no
// S-difference term), 2 Eq. standard with gamma = 0 and the drift-diffusion term
// Gamma_j = sum_i d_i (S^-1)_ji by central differences.
struct ToyArgs {
  double lambda, k, a, mu, T, Delta, alpha;
  int s_kind, scheme, n_steps, n_traj;
  uint32_t seed;
};

__device__ __forceinline__ void toy_metric(const ToyArgs& p, double x, double y, double S[3]) {
  if (p.s_kind == 2) { S[0] = 1.0; S[1] = 0.0; S[2] = 1.0; return; }
  if (p.s_kind == 3) {
    // S = H + mu I
    const double r = sqrt(x * x + y * y), nx = x / r, ny = y / r, c = p.k * (r - p.a) / r;
    S[0] = p.k * nx * nx + c * (1.0 - nx * nx) + p.mu;
    S[1] = p.k * nx * ny - c * nx * ny;
    S[2] = p.k * ny * ny + c * (1.0 - ny * ny) + p.mu;
    return;
  }
  const double r = sqrt(x * x + y * y), nx = x / r, ny = y / r;
  const double il = 1.0 / p.lambda;
  // n n^T / lambda + t t^T with t = (-ny, nx)
  S[0] = nx * nx * il + ny * ny;
  S[1] = nx * ny * (il - 1.0);
  S[2] = ny * ny * il + nx * nx;
  if (p.s_kind == 1) {
    // H = k n n^T + k (r - a) / r (I - n n^T)
    const double c = p.k * (r - p.a) / r;
    S[0] = p.k * nx * nx + c * (1.0 - nx * nx) + p.mu * S[0];
    S[1] = p.k * nx * ny - c * nx * ny + p.mu * S[1];
    S[2] = p.k * ny * ny + c * (1.0 - ny * ny) + p.mu * S[2];
  }
}

// S^-1 of a symmetric 2 x 2 matrix (s00, s01, s11)
__device__ __forceinline__ void toy_inv(const double S[3], double Si[3]) {
  const double det = S[0] * S[2] - S[1] * S[1];
  Si[0] = S[2] / det; Si[1] = -S[1] / det; Si[2] = S[0] / det;
}

__global__ __launch_bounds__(256) void k_toy(ToyArgs p, const double* R0, double* Rout, double* Umean,
                                            int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n_traj) return;
  double x = R0[2 * i], y = R0[2 * i + 1], xp = x, yp = y;
  double Sp[3];
  toy_metric(p, x, y, Sp);
  double Dt = p.Delta, Db = p.Delta;
  if (p.scheme == 0 && p.alpha > 0.0) {
    Dt = -expm1(-p.alpha * p.Delta) / p.alpha;
    Db = -expm1(-2.0 * p.alpha * p.Delta) / (2.0 * p.alpha);
  }
  const int burn = p.n_steps / 10;
  double usum = 0.0;
  int st = 0;
  for (int t = 0; t < p.n_steps; ++t) {
    const double r = sqrt(x * x + y * y);
    const double fx = -p.k * (r - p.a) * x / r, fy = -p.k * (r - p.a) * y / r;
    double S[3];
    toy_metric(p, x, y, S);
    // S = L L^T and the two unit normals of step t
    const double l00 = sqrt(S[0]), l10 = S[1] / l00, d11 = S[2] - l10 * l10;
    if (!(S[0] > 0.0) || !(d11 > 0.0)) { st = 3; break; }
    const double l11 = sqrt(d11);
    const u32x4 o = philox((uint32_t)t, 0xFFFFFFFFu, 0u, 0u, p.seed, (uint32_t)i);
    const double u1 = u01(o.x, o.y), u2 = u01(o.z, o.w);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    // L^T z = xi: <z z^T> = S^-1
    const double z1 = rad * sn / l11, z0 = (rad * cs - l10 * z1) / l00;
    double dx, dy;
    if (p.scheme == 3) {
      // first simplified scheme: noise step to y, then the drift with S at R and the
      // half S-difference between y and R
      const double amp = sqrt(2.0 * p.T * p.Delta);
      const double yx = x + amp * z0, yy = y + amp * z1;
      double Sy[3], Si[3];
      toy_metric(p, yx, yy, Sy);
      toy_inv(S, Si);
      const double ex = yx - x, ey = yy - y;
      const double vx = p.Delta * fx - 0.5 * ((Sy[0] - S[0]) * ex + (Sy[1] - S[1]) * ey);
      const double vy = p.Delta * fy - 0.5 * ((Sy[1] - S[1]) * ex + (Sy[2] - S[2]) * ey);
      dx = amp * z0 + Si[0] * vx + Si[1] * vy;
      dy = amp * z1 + Si[1] * vx + Si[2] * vy;
    } else if (p.scheme == 2) {
      double Si[3];
      toy_inv(S, Si);
      // Gamma_j = sum_i d/dx_i (S^-1)_ji, central differences of step h
      const double h = 1e-6;
      double Spx[3], Smx[3], Spy[3], Smy[3], Ipx[3], Imx[3], Ipy[3], Imy[3];
      toy_metric(p, x + h, y, Spx); toy_metric(p, x - h, y, Smx);
      toy_metric(p, x, y + h, Spy); toy_metric(p, x, y - h, Smy);
      toy_inv(Spx, Ipx); toy_inv(Smx, Imx); toy_inv(Spy, Ipy); toy_inv(Smy, Imy);
      const double g0 = (Ipx[0] - Imx[0]) / (2.0 * h) + (Ipy[1] - Imy[1]) / (2.0 * h);
      const double g1 = (Ipx[1] - Imx[1]) / (2.0 * h) + (Ipy[2] - Imy[2]) / (2.0 * h);
      const double amp = sqrt(2.0 * p.T * p.Delta);
      dx = p.Delta * (Si[0] * fx + Si[1] * fy) + p.T * p.Delta * g0 + amp * z0;
      dy = p.Delta * (Si[1] * fx + Si[2] * fy) + p.T * p.Delta * g1 + amp * z1;
    } else {
      // v = f - (S_prev - S)(R_prev - R) / (2 Db), then y = S^-1 v through L
      double vx = fx, vy = fy;
      if (p.scheme == 0) {
        const double ex = xp - x, ey = yp - y;
        vx -= ((Sp[0] - S[0]) * ex + (Sp[1] - S[1]) * ey) / (2.0 * Db);
        vy -= ((Sp[1] - S[1]) * ex + (Sp[2] - S[2]) * ey) / (2.0 * Db);
      }
      const double w0 = vx / l00, w1 = (vy - l10 * w0) / l11;
      const double y1 = w1 / l11, y0 = (w0 - l10 * y1) / l00;
      const double amp = sqrt(2.0 * p.T * Db);
      dx = Dt * y0 + amp * z0;
      dy = Dt * y1 + amp * z1;
    }
    xp = x; yp = y;
    Sp[0] = S[0]; Sp[1] = S[1]; Sp[2] = S[2];
    x += dx; y += dy;
    const double rn = sqrt(x * x + y * y);
    if (t >= burn) usum += 0.5 * p.k * (rn - p.a) * (rn - p.a);
  }
  Rout[2 * i] = x;
  Rout[2 * i + 1] = y;
  const int cnt = p.n_steps - burn;
  Umean[i] = usum / (double)(cnt > 0 ? cnt : 1);
  status[i] = st;
}

hipError_t launch_toy(double lambda, double k, double a, double mu, int s_kind, double T, double Delta,
                      double alpha, int scheme, uint32_t seed, int n_traj, int n_steps, const double* R0,
                      double* Rout, double* Umean, int* status, hipStream_t st) {
  ToyArgs p{lambda, k, a, mu, T, Delta, alpha, s_kind, scheme, n_steps, n_traj, seed};
  hipLaunchKernelGGL(k_toy, dim3((n_traj + 255) / 256), dim3(256), 0, st, p, R0, Rout, Umean, status);
  return hipGetLastError();
}

// Twist averaging: element u of f (u < n3) and of S (n3 <= u < n3 + n3^2), each summed over
// the runs in run order.
__global__ __launch_bounds__(256) void k_twist_average(int n_tw, int n3, const double* f_stack,
                                                       const double* S_stack, double* f, double* S) {
  const size_t nS = (size_t)n3 * n3, total = n3 + nS;
  for (size_t u = (size_t)blockIdx.x * 256 + threadIdx.x; u < total; u += (size_t)gridDim.x * 256) {
    double s = 0.0;
    if (u < (size_t)n3) {
      for (int r = 0; r < n_tw; ++r) s += f_stack[(size_t)r * n3 + u];
      f[u] = s / n_tw;
    } else {
      const size_t v = u - n3;
      for (int r = 0; r < n_tw; ++r) s += S_stack[(size_t)r * nS + v];
      S[v] = s / ((double)n_tw * n_tw);
    }
  }
}

hipError_t launch_twist_average(int n_tw, int n3, const double* f_stack, const double* S_stack, double* f, double* S,
                                hipStream_t st) {
  const size_t total = (size_t)n3 + (size_t)n3 * n3;
  const int blocks = (int)((total + 255) / 256 < 2048 ? (total + 255) / 256 : 2048);
  hipLaunchKernelGGL(k_twist_average, dim3(blocks), dim3(256), 0, st, n_tw, n3, f_stack, S_stack, f, S);
  return hipGetLastError();
}

// Packs per-configuration results: [ln|psi|, E_L, dln|psi|/dR, dE_L/dR].
__global__ void k_pack_eval(int K, int N, const double* means, const double* ldet, const double* Uj, double* out) {
  const int k = blockIdx.x;
  const int n3 = 3 * N;
  const double* mw = means + (size_t)k * (1 + 3 * n3);
  double* o = out + (size_t)k * (2 + 2 * n3);
  for (int u = threadIdx.x; u < n3; u += blockDim.x) {
    o[2 + u] = mw[1 + n3 + u];
    o[2 + n3 + u] = mw[1 + u];
  }
  if (threadIdx.x == 0) {
    o[0] = ldet[2 * k] + ldet[2 * k + 1] + Uj[k];
    o[1] = mw[0];
  }
}

hipError_t launch_pack_eval(int K, int N, const double* means, const double* ldet, const double* Uj, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pack_eval, dim3(K), dim3(256), 0, st, K, N, means, ldet, Uj, out);
  return hipGetLastError();
}

}  // namespace vmc
