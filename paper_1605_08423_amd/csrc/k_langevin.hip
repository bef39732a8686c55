// Estimators, acceleration matrix and the Langevin step (a7-a10).
//   E = mean_w e_w, sigma_E = sd_w(e_w)/sqrt(W), f_w = -(d_w + 2 (h_w - E g_w)), f = mean_w f_w
//   S = sum_w (f_w - f)(f_w - f)^T / (W (W - 1))       (covariance of the mean force)
//   R' = R + Dt S^-1 [f - (S_prev - S)(R_prev - R)/(2 Db)] + sqrt(2 T Db) z,  z = L^-T xi
// All reductions use a fixed order so results are bitwise reproducible.
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

constexpr int RED_CHUNK = 256;      // walkers per partial column sum
constexpr int SYRK_CHUNK = 1024;    // walkers per partial S block
constexpr int SYRK_T = 64;          // S tile edge

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
// Partial sums of (f_w - f)(f_w - f)^T over walker chunks, lower block triangle.
__global__ __launch_bounds__(256) void k_syrk_partial(int W, int n3, const double* f_w, const double* f,
                                                      double* partial) {
  const int bi = blockIdx.x, bj = blockIdx.y, ch = blockIdx.z;
  if (bj > bi) return;
  __shared__ double Ai[32][SYRK_T], Aj[32][SYRK_T];
  const int t = threadIdx.x, tx = t % 16, ty = t / 16;
  const int i0 = bi * SYRK_T, j0 = bj * SYRK_T;
  const int w0 = ch * SYRK_CHUNK, w1 = min(W, w0 + SYRK_CHUNK);
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int wb = w0; wb < w1; wb += 32) {
    for (int u = t; u < 32 * SYRK_T; u += 256) {
      const int ww = u / SYRK_T, c = u % SYRK_T, w = wb + ww;
      const int ci = i0 + c, cj = j0 + c;
      Ai[ww][c] = (w < w1 && ci < n3) ? f_w[(size_t)w * n3 + ci] - f[ci] : 0.0;
      Aj[ww][c] = (w < w1 && cj < n3) ? f_w[(size_t)w * n3 + cj] - f[cj] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ww = 0; ww < 32; ++ww) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) { a[r] = Ai[ww][ty * 4 + r]; b[r] = Aj[ww][tx * 4 + r]; }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
    __syncthreads();
  }
  double* P = partial + (size_t)ch * n3 * n3;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
      if (i < n3 && j < n3) P[(size_t)i * n3 + j] = acc[r][c];
    }
}

__global__ void k_syrk_final(int W, int n3, int nch, const double* partial, double* S) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n3 * n3) return;
  int i = (int)(idx / n3), j = (int)(idx % n3);
  if (i / SYRK_T < j / SYRK_T) { int tmp = i; i = j; j = tmp; }
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += partial[(size_t)c * n3 * n3 + (size_t)i * n3 + j];
  S[idx] = s / ((double)W * (double)(W - 1));
}

size_t syrk_partial_doubles(int W, int n3) {
  return (size_t)((W + SYRK_CHUNK - 1) / SYRK_CHUNK) * n3 * n3;
}

hipError_t launch_syrk(int W, int n3, const double* f_w, const double* f, double* partial, double* S,
                       hipStream_t st) {
  const int nt = (n3 + SYRK_T - 1) / SYRK_T, nch = (W + SYRK_CHUNK - 1) / SYRK_CHUNK;
  hipLaunchKernelGGL(k_syrk_partial, dim3(nt, nt, nch), dim3(256), 0, st, W, n3, f_w, f, partial);
  size_t tot = (size_t)n3 * n3;
  hipLaunchKernelGGL(k_syrk_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, W, n3, nch, partial, S);
  return hipGetLastError();
}

// ------------------------------------------------------------ Langevin ---
// One work-group: v, Cholesky S = L L^T (right-looking, column j cached in LDS),
// y = S^-1 v, z = L^-T xi, update and state shift.  status: 0 ok, 1 bad T, 3 not SPD.
constexpr int LANG_MAX = 1536;

__global__ __launch_bounds__(1024) void k_langevin(int n3, double L, double* R, double* R_prev, double* S_prev,
                                                  const double* f, const double* S, double* Lw, double T,
                                                  double Delta, double alpha, unsigned flags, uint32_t seed,
                                                  uint32_t traj, uint32_t step, int* status) {
  __shared__ double col[LANG_MAX];
  __shared__ double dR[LANG_MAX];
  __shared__ double y[LANG_MAX];
  __shared__ double z[LANG_MAX];
  __shared__ int fail;
  const int t = threadIdx.x, nt = blockDim.x;
  const bool cfold = flags & 1u, noise_corr = flags & 2u, no_scorr = flags & 4u;
  double Dt = Delta, Db = Delta;
  if (alpha > 0.0) {
    Dt = -expm1(-alpha * Delta) / alpha;
    Db = -expm1(-2.0 * alpha * Delta) / (2.0 * alpha);
  }
  const double invL = L > 0.0 ? 1.0 / L : 0.0;
  if (t == 0) fail = 0;
  for (int i = t; i < n3; i += nt) {
    double d = R_prev[i] - R[i];
    if (L > 0.0) d = min_image(d, L, invL);
    dR[i] = d;
  }
  __syncthreads();
  for (int i = t; i < n3; i += nt) {
    double c = 0.0;
    if (!no_scorr && !cfold)
      for (int j = 0; j < n3; ++j) c += (S_prev[(size_t)i * n3 + j] - S[(size_t)i * n3 + j]) * dR[j];
    y[i] = f[i] - c / (2.0 * Db);
  }
  // Cholesky of S (or I) into the lower triangle of Lw
  for (size_t u = t; u < (size_t)n3 * n3; u += nt) {
    const int i = (int)(u / n3), j = (int)(u % n3);
    Lw[u] = cfold ? (i == j ? 1.0 : 0.0) : S[u];
  }
  __syncthreads();
  for (int j = 0; j < n3; ++j) {
    if (t == 0) {
      const double d = Lw[(size_t)j * n3 + j];
      if (!(d > 0.0)) fail = 1;
      else Lw[(size_t)j * n3 + j] = sqrt(d);
    }
    __syncthreads();
    if (fail) break;
    const double djj = Lw[(size_t)j * n3 + j];
    for (int i = j + 1 + t; i < n3; i += nt) {
      const double v = Lw[(size_t)i * n3 + j] / djj;
      Lw[(size_t)i * n3 + j] = v;
      col[i] = v;
    }
    __syncthreads();
    const int m = n3 - j - 1;
    for (int u = t; u < m * m; u += nt) {
      const int ii = u / m, kk = u % m;
      if (kk <= ii) {
        const int i = j + 1 + ii, k = j + 1 + kk;
        Lw[(size_t)i * n3 + k] -= col[i] * col[k];
      }
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) *status = 3;
    return;
  }
  const double Teff = noise_corr ? T - Dt * Dt / (2.0 * Db) : T;
  if (Teff < 0.0) {
    if (t == 0) *status = 1;
    return;
  }
  // forward: L w = v (in y)
  for (int k = 0; k < n3; ++k) {
    if (t == 0) y[k] /= Lw[(size_t)k * n3 + k];
    __syncthreads();
    const double yk = y[k];
    for (int i = k + 1 + t; i < n3; i += nt) y[i] -= Lw[(size_t)i * n3 + k] * yk;
    __syncthreads();
  }
  // backward: L^T y = w
  for (int k = n3 - 1; k >= 0; --k) {
    if (t == 0) y[k] /= Lw[(size_t)k * n3 + k];
    __syncthreads();
    const double yk = y[k];
    for (int i = t; i < k; i += nt) y[i] -= Lw[(size_t)k * n3 + i] * yk;
    __syncthreads();
  }
  // xi by Box-Muller pairs, then L^T z = xi
  for (int j = t; 2 * j < n3; j += nt) {
    const u32x4 o = philox(step, 0xFFFFFFFFu, (uint32_t)j, 0u, seed, traj);
    const double u1 = u01(o.x, o.y), u2 = u01(o.z, o.w);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z[2 * j] = rad * c;
    if (2 * j + 1 < n3) z[2 * j + 1] = rad * s;
  }
  __syncthreads();
  for (int k = n3 - 1; k >= 0; --k) {
    if (t == 0) z[k] /= Lw[(size_t)k * n3 + k];
    __syncthreads();
    const double zk = z[k];
    for (int i = t; i < k; i += nt) z[i] -= Lw[(size_t)k * n3 + i] * zk;
    __syncthreads();
  }
  // a non-finite position, force, S-difference term or noise is an argument error: the state stays
  for (int i = t; i < n3; i += nt)
    if (!isfinite(y[i]) || !isfinite(z[i]) || !isfinite(R[i]) || !isfinite(R_prev[i])) fail = 1;
  __syncthreads();
  if (fail) {
    if (t == 0) *status = 1;
    return;
  }
  const double amp = sqrt(2.0 * Teff * Db);
  for (int i = t; i < n3; i += nt) {
    double rn = R[i] + Dt * y[i] + amp * z[i];
    if (L > 0.0) rn = wrap_box(rn, L, invL);
    R_prev[i] = R[i];
    R[i] = rn;
  }
  for (size_t u = t; u < (size_t)n3 * n3; u += nt) S_prev[u] = S[u];
  if (t == 0) *status = 0;
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
  if (n3 > LANG_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_langevin, dim3(1), dim3(1024), 0, st, n3, L, R, R_prev, S_prev, f, S, Lwork, T, Delta,
                     alpha, flags, seed, traj, step, status);
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
