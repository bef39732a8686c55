/* Plain FP64 CPU oracle -- see vmc_oracle.h.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.
 *
 * What the paper fixes and what is a recorded reading:
 *  - Langevin update: Eq. finaldyn_new of the SI ("Better integration scheme,
 *    the adopted one") with the exactly integrated steps Dt = (1-e^{-aD})/a and
 *    Db = (1-e^{-2aD})/(2a); a = 0 gives Eq. finaldyn.  Noise <z z^T> = S^{-1}.
 *  - S = Cov(f): the covariance of the sampled force (main text, Eq. for Cov(f)),
 *    read as the covariance of the mean force, which scales as 1/N_c (SI, the
 *    paragraph that sets alpha = 0.122 N_c).
 *  - V(R) = <psi|H_R|psi>/<psi|psi> for a Jastrow-Slater psi and the all-electron
 *    Coulomb Hamiltonian (main text, Eq. for V(R)); the force is f = -dV/dR at
 *    frozen wavefunction parameters.  The paper defers the estimator to its
 *    references, so the textbook variational derivative with the Pulay term is used.
 *  - Basis: s-Gaussians made periodic by the image sum (SI, "Systematic setup");
 *    Jastrow: two-body Pade term on the sin-periodised distance (SI, Jastrow
 *    section, periodisation substitution and the U_2 paragraph).  The e-e cusp
 *    sign is taken as u = +a rho/(1+b rho) with J = e^{+U}, a = 1/2 (anti-parallel)
 *    and 1/4 (parallel), b = 1.  Optionally the one-body term U_1 of the same
 *    section (Eq. e:j1) for protons (Z = 1), its homogeneous part only (the f
 *    coefficients are optimised parameters), on the same periodised distance.
 *  - Ewald parameters, Metropolis details and the Hueckel orbitals are not in
 *    the paper; they are recorded readings shared with the GPU library only
 *    through their definitions.
 *  - Wavefunction optimisation (main text: the wavefunction is re-optimised before
 *    every ionic step; the optimiser is only cited): the logarithmic derivatives of
 *    the Jastrow parameters (o_param_derivs) and their per-walker sums along the
 *    chain (o_vmc_run_opt) feed stochastic reconfiguration, whose step is written
 *    from its published definition in oracle.py (sr_step).
 * Every function below is pinned by a test in tests/test_oracle_*.py; the
 * end-to-end Monte Carlo averages themselves are "parity unpinned" beyond the
 * pins of their parts (no values exist in the paper for this wavefunction).
 */
#include "vmc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O_EINVAL (-1)
#define O_ENOTSPD (-3)
#define O_ESINGULAR (-4)

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ RNG -- */
/* Philox4x32-10: ten rounds of the Philox S-box on a 4x32-bit counter with a
 * 2x32-bit key that is bumped by the Weyl constants between rounds. */
void o_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53 random bits (32 from hi, the top 21 of lo) scaled into [0, 1). */
double o_u01(uint32_t hi, uint32_t lo) {
  uint64_t m = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
  return (double)m * (1.0 / 9007199254740992.0);
}

/* Gaussian normals for the Langevin noise by the Box-Muller transform; pair j
 * uses counter (step, 0xFFFFFFFF, j, 0). */
void o_normals(uint32_t seed, uint32_t traj, uint32_t step, int n, double* xi) {
  uint32_t key[2] = {seed, traj};
  for (int j = 0; 2 * j < n; ++j) {
    uint32_t ctr[4] = {step, 0xFFFFFFFFu, (uint32_t)j, 0u}, o[4];
    o_philox(ctr, key, o);
    double u1 = o_u01(o[0], o[1]), u2 = o_u01(o[2], o[3]);
    double rad = sqrt(-2.0 * log(1.0 - u1));
    xi[2 * j] = rad * cos(2.0 * PI * u2);
    if (2 * j + 1 < n) xi[2 * j + 1] = rad * sin(2.0 * PI * u2);
  }
}

/* ------------------------------------------------------- linear algebra -- */
/* LU with partial pivoting of a copy of the n x n matrix M.  Returns 0, or
 * O_ESINGULAR if a pivot is exactly zero.  logdet = ln|det M|, sgn = sign. */
static int lu_logdet(int n, const double* M, double* logdet, double* sgn, double* inv) {
  double* a = (double*)malloc(sizeof(double) * n * n);
  int* piv = (int*)malloc(sizeof(int) * n);
  memcpy(a, M, sizeof(double) * n * n);
  double ld = 0.0, sg = 1.0;
  int rc = 0;
  for (int p = 0; p < n; ++p) {
    int best = p;
    for (int r = p + 1; r < n; ++r)
      if (fabs(a[r * n + p]) > fabs(a[best * n + p])) best = r;
    piv[p] = best;
    if (a[best * n + p] == 0.0) { rc = O_ESINGULAR; break; }
    if (best != p) {
      for (int c = 0; c < n; ++c) { double t = a[p * n + c]; a[p * n + c] = a[best * n + c]; a[best * n + c] = t; }
      sg = -sg;
    }
    double d = a[p * n + p];
    if (d < 0) sg = -sg;
    ld += log(fabs(d));
    for (int r = p + 1; r < n; ++r) {
      double l = a[r * n + p] / d;
      a[r * n + p] = l;
      for (int c = p + 1; c < n; ++c) a[r * n + c] -= l * a[p * n + c];
    }
  }
  if (rc == 0 && inv) {
    /* Solve A X = I column by column with the factors. */
    for (int j = 0; j < n; ++j) {
      double* col = (double*)calloc(n, sizeof(double));
      col[j] = 1.0;
      for (int p = 0; p < n; ++p) { double t = col[p]; col[p] = col[piv[p]]; col[piv[p]] = t; }
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < r; ++c) col[r] -= a[r * n + c] * col[c];
      for (int r = n - 1; r >= 0; --r) {
        for (int c = r + 1; c < n; ++c) col[r] -= a[r * n + c] * col[c];
        col[r] /= a[r * n + r];
      }
      for (int r = 0; r < n; ++r) inv[r * n + j] = col[r];
      free(col);
    }
  }
  *logdet = rc ? -INFINITY : ld;
  *sgn = rc ? 0.0 : sg;
  free(a);
  free(piv);
  return rc;
}

/* C = A B for n x n row-major matrices. */
static void matmul(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}

/* ------------------------------------------------------------------ basis -- */
static double min_image(double d, double L) { return d - L * floor(d / L + 0.5); }

/* One Cartesian factor of a Gaussian and its first three derivatives.  In the
 * periodic case x is the minimum-image offset and the n = -1, 0, +1 images are
 * summed (the neglected images are below e^{-zeta (1.5 L)^2}), image n weighted by
 * tau^n: tau = 1 periodic, tau = -1 for the twist angle pi (SI, twisted boundary
 * conditions, phi(r + n L) = e^{i theta n} phi(r)).  With tau = -1 the truncated sum
 * jumps by 2 e^{-zeta (1.5 L)^2} where the minimum image changes (below 1e-26 for
 * every box of the workloads). */
static void gauss_1d(double x, double zeta, double L, int periodic, double tau, double g[4]) {
  g[0] = g[1] = g[2] = g[3] = 0.0;
  int nlo = periodic ? -1 : 0, nhi = periodic ? 1 : 0;
  for (int n = nlo; n <= nhi; ++n) {
    double t = x + n * L;
    double e = (n == 0 ? 1.0 : tau) * exp(-zeta * t * t);
    g[0] += e;
    g[1] += -2.0 * zeta * t * e;
    g[2] += (4.0 * zeta * zeta * t * t - 2.0 * zeta) * e;
    g[3] += (-8.0 * zeta * zeta * zeta * t * t * t + 12.0 * zeta * zeta * t) * e;
  }
}

/* One Cartesian factor of the image sum of t^2 e^{-zeta t^2} (the r^2 part of the contracted
 * orbital's second Gaussian) and its first three derivatives, images and weights as in gauss_1d;
 * with e = e^{-zeta t^2}: first derivative (2t - 2 zeta t^3) e, second (2 - 10 zeta t^2 +
 * 4 zeta^2 t^4) e, third (-24 zeta t + 36 zeta^2 t^3 - 8 zeta^3 t^5) e. */
static void gauss2_1d(double x, double zeta, double L, int periodic, double tau, double g[4]) {
  g[0] = g[1] = g[2] = g[3] = 0.0;
  int nlo = periodic ? -1 : 0, nhi = periodic ? 1 : 0;
  for (int n = nlo; n <= nhi; ++n) {
    double t = x + n * L, t2 = t * t;
    double e = (n == 0 ? 1.0 : tau) * exp(-zeta * t2);
    g[0] += t2 * e;
    g[1] += (2.0 * t - 2.0 * zeta * t2 * t) * e;
    g[2] += (2.0 - 10.0 * zeta * t2 + 4.0 * zeta * zeta * t2 * t2) * e;
    g[3] += (-24.0 * zeta * t + 36.0 * zeta * zeta * t2 * t - 8.0 * zeta * zeta * zeta * t2 * t2 * t) * e;
  }
}

/* w times the 14 components of the product f_x(x) f_y(y) f_z(z), added to out. */
static void add_product(const double g[3][4], double w, double out[14]) {
  out[0] += w * g[0][0] * g[1][0] * g[2][0];
  out[1] += w * g[0][1] * g[1][0] * g[2][0];
  out[2] += w * g[0][0] * g[1][1] * g[2][0];
  out[3] += w * g[0][0] * g[1][0] * g[2][1];
  out[4] += w * (g[0][2] * g[1][0] * g[2][0] + g[0][0] * g[1][2] * g[2][0] + g[0][0] * g[1][0] * g[2][2]);
  out[5] += w * g[0][2] * g[1][0] * g[2][0];
  out[6] += w * g[0][0] * g[1][2] * g[2][0];
  out[7] += w * g[0][0] * g[1][0] * g[2][2];
  out[8] += w * g[0][1] * g[1][1] * g[2][0];
  out[9] += w * g[0][1] * g[1][0] * g[2][1];
  out[10] += w * g[0][0] * g[1][1] * g[2][1];
  out[11] += w * (g[0][3] * g[1][0] * g[2][0] + g[0][1] * g[1][2] * g[2][0] + g[0][1] * g[1][0] * g[2][2]);
  out[12] += w * (g[0][2] * g[1][1] * g[2][0] + g[0][0] * g[1][3] * g[2][0] + g[0][0] * g[1][1] * g[2][2]);
  out[13] += w * (g[0][2] * g[1][0] * g[2][1] + g[0][0] * g[1][2] * g[2][1] + g[0][0] * g[1][0] * g[2][3]);
}

/* Basis function a at point r: out = [phi, grad(3), lap, hess xx yy zz xy xz yz,
 * grad lap (3)]. */
void o_basis(const osys* s, int a, const double r[3], double out[14]) {
  const double* Ra = s->R + 3 * a;
  double z = s->zeta[a];
  if (s->basis_kind == OB_OPEN_STO) {
    double d[3] = {r[0] - Ra[0], r[1] - Ra[1], r[2] - Ra[2]};
    double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double f = exp(-z * rr);
    out[0] = f;
    for (int m = 0; m < 3; ++m) out[1 + m] = -z * d[m] / rr * f;
    out[4] = f * (z * z - 2.0 * z / rr);
    int hp[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int h = 0; h < 6; ++h) {
      int m = hp[h][0], n = hp[h][1];
      double dd = (m == n) ? 1.0 : 0.0;
      out[5 + h] = f * (z * z * d[m] * d[n] / (rr * rr) - z * (dd / rr - d[m] * d[n] / (rr * rr * rr)));
    }
    for (int m = 0; m < 3; ++m)
      out[11 + m] = out[1 + m] * (z * z - 2.0 * z / rr) + f * 2.0 * z * d[m] / (rr * rr * rr);
    return;
  }
  int periodic = (s->basis_kind == OB_PERIODIC_GAUSS);
  if (s->contracted) {
    /* phi_1 + eta phi_2 with r^2 = x^2 + y^2 + z^2: four separable products,
     * g1 g1 g1 + eta (h2 g2 g2 + g2 h2 g2 + g2 g2 h2) */
    double g1[3][4], g2[3][4], h2[3][4];
    for (int m = 0; m < 3; ++m) {
      double d = r[m] - Ra[m], tau = ((s->twist >> m) & 1) ? -1.0 : 1.0, sg = 1.0;
      if (periodic) {
        double k = floor(d / s->L + 0.5);
        d -= s->L * k;
        if (fmod(fabs(k), 2.0) == 1.0) sg = tau;
      }
      gauss_1d(d, O_Z1, s->L, periodic, tau, g1[m]);
      gauss_1d(d, O_Z2, s->L, periodic, tau, g2[m]);
      gauss2_1d(d, O_Z2, s->L, periodic, tau, h2[m]);
      for (int q = 0; q < 4; ++q) { g1[m][q] *= sg; g2[m][q] *= sg; h2[m][q] *= sg; }
    }
    for (int q = 0; q < 14; ++q) out[q] = 0.0;
    add_product(g1, 1.0, out);
    for (int m = 0; m < 3; ++m) {
      double f[3][4];
      for (int mm = 0; mm < 3; ++mm)
        for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? h2[mm][q] : g2[mm][q];
      add_product(f, s->eta, out);
    }
    return;
  }
  double g[3][4];
  for (int m = 0; m < 3; ++m) {
    double d = r[m] - Ra[m], tau = ((s->twist >> m) & 1) ? -1.0 : 1.0, sg = 1.0;
    if (periodic) {
      /* d = d_min + k L: the image sum at d is tau^k times the one at d_min */
      double k = floor(d / s->L + 0.5);
      d -= s->L * k;
      if (fmod(fabs(k), 2.0) == 1.0) sg = tau;
    }
    gauss_1d(d, z, s->L, periodic, tau, g[m]);
    for (int q = 0; q < 4; ++q) g[m][q] *= sg;
  }
  out[0] = g[0][0] * g[1][0] * g[2][0];
  out[1] = g[0][1] * g[1][0] * g[2][0];
  out[2] = g[0][0] * g[1][1] * g[2][0];
  out[3] = g[0][0] * g[1][0] * g[2][1];
  out[4] = g[0][2] * g[1][0] * g[2][0] + g[0][0] * g[1][2] * g[2][0] + g[0][0] * g[1][0] * g[2][2];
  out[5] = g[0][2] * g[1][0] * g[2][0];
  out[6] = g[0][0] * g[1][2] * g[2][0];
  out[7] = g[0][0] * g[1][0] * g[2][2];
  out[8] = g[0][1] * g[1][1] * g[2][0];
  out[9] = g[0][1] * g[1][0] * g[2][1];
  out[10] = g[0][0] * g[1][1] * g[2][1];
  out[11] = g[0][3] * g[1][0] * g[2][0] + g[0][1] * g[1][2] * g[2][0] + g[0][1] * g[1][0] * g[2][2];
  out[12] = g[0][2] * g[1][1] * g[2][0] + g[0][0] * g[1][3] * g[2][0] + g[0][0] * g[1][1] * g[2][2];
  out[13] = g[0][2] * g[1][0] * g[2][1] + g[0][0] * g[1][2] * g[2][1] + g[0][0] * g[1][0] * g[2][3];
}

static int hidx(int m, int n) {
  if (m == n) return 5 + m;
  if (m > n) { int t = m; m = n; n = t; }
  return (m == 0) ? (n == 1 ? 8 : 9) : 10;
}

/* ---------------------------------------------------------------- Jastrow -- */
static int spin_of(const osys* s, int e) { return e < s->n_up ? 0 : 1; }

/* Pade pair term for the offset d = r_i - r_j: u(rho), grad_i rho, and
 * u', u'', lap rho.  Periodic systems use rt_m = (L/pi) sin(pi d_m / L). */
static void jas_pair(const osys* s, const double d[3], int same, double* u, double* up, double* upp,
                     double grho[3], double* laprho) {
  double rt[3], c[3], kf;
  if (s->basis_kind == OB_PERIODIC_GAUSS) {
    for (int m = 0; m < 3; ++m) {
      rt[m] = s->L / PI * sin(PI * d[m] / s->L);
      c[m] = cos(PI * d[m] / s->L);
    }
    kf = (PI / s->L) * (PI / s->L);
  } else {
    for (int m = 0; m < 3; ++m) { rt[m] = d[m]; c[m] = 1.0; }
    kf = 0.0;
  }
  double rho = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
  double a = same ? s->a_par : s->a_anti, b = s->b;
  double den = 1.0 + b * rho;
  *u = a * rho / den;
  *up = a / (den * den);
  *upp = -2.0 * a * b / (den * den * den);
  double g2 = 0.0, c2 = 0.0;
  for (int m = 0; m < 3; ++m) {
    grho[m] = rt[m] * c[m] / rho;
    g2 += grho[m] * grho[m];
    c2 += c[m] * c[m];
  }
  *laprho = (c2 - kf * rho * rho) / rho - g2 / rho;
}

/* One-body term of the SI (Eq. e:j1), homogeneous part, for a nucleus of charge
 * Z = 1: f(rho) = -(2Z)^{3/4} u_1((2Z)^{1/4} rho), u_1(x) = (1 - e^{-b_1 x})/(2 b_1),
 * on the distance rho between electron and nucleus.  Its slope at rho = 0 is -Z,
 * the electron-nucleus cusp.  F[k] = d^k f / d rho^k, k = 0..3. */
static void j1_radial(double b1, double rho, double F[4]) {
  const double Z = 1.0, c = pow(2.0 * Z, 0.75), sc = pow(2.0 * Z, 0.25);
  double e = exp(-b1 * sc * rho);
  double u0 = (1.0 - e) / (2.0 * b1), u1 = e / 2.0, u2 = -b1 * e / 2.0, u3 = b1 * b1 * e / 2.0;
  F[0] = -c * u0;
  F[1] = -c * sc * u1;
  F[2] = -c * sc * sc * u2;
  F[3] = -c * sc * sc * sc * u3;
}

/* rho = |rt|, rt_m = (L/pi) sin(pi d_m / L) in the periodic kind, |d| otherwise. */
static double periodised_rho(const osys* s, const double d[3]) {
  double r2 = 0.0;
  for (int m = 0; m < 3; ++m) {
    double r = (s->basis_kind == OB_PERIODIC_GAUSS) ? s->L / PI * sin(PI * d[m] / s->L) : d[m];
    r2 += r * r;
  }
  return sqrt(r2);
}

/* A radial function f(rho(d)) of the offset d, with rho = |rt| on the periodised
 * components rt_m = (L/pi) sin(pi d_m / L) (d itself in the open kinds), given
 * F[k] = d^k f/d rho^k.  Chain rule with c_m = d rt_m / d d_m = cos(pi d_m / L),
 * d c_m / d d_m = -(pi/L)^2 rt_m, g_m = d rho / d d_m = rt_m c_m / rho and
 * p_m = c_m^2 - (pi/L)^2 rt_m^2:
 *   d g_m / d d_n = (delta_mn p_m - g_m g_n) / rho,
 *   grad f = F' g,  hess f = F'' g g^T + F' (diag(p) - g g^T) / rho,
 *   lap f = F'' G + F' (P - G) / rho  with G = |g|^2, P = sum_m p_m,
 * and the gradient of the Laplacian with d G / d d_n = 2 g_n (p_n - G) / rho and
 * d P / d d_n = -4 (pi/L)^2 rho g_n.  hess: xx yy zz xy xz yz. */
static void radial_field(const osys* s, const double d[3], const double F[4], double grad[3], double hess[6],
                         double* lap, double glap[3]) {
  double rt[3], c[3], kf;
  if (s->basis_kind == OB_PERIODIC_GAUSS) {
    for (int m = 0; m < 3; ++m) {
      rt[m] = s->L / PI * sin(PI * d[m] / s->L);
      c[m] = cos(PI * d[m] / s->L);
    }
    kf = (PI / s->L) * (PI / s->L);
  } else {
    for (int m = 0; m < 3; ++m) { rt[m] = d[m]; c[m] = 1.0; }
    kf = 0.0;
  }
  double rho = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
  double g[3], p[3], G = 0.0, P = 0.0;
  for (int m = 0; m < 3; ++m) {
    g[m] = rt[m] * c[m] / rho;
    p[m] = c[m] * c[m] - kf * rt[m] * rt[m];
    G += g[m] * g[m];
    P += p[m];
  }
  for (int m = 0; m < 3; ++m) grad[m] = F[1] * g[m];
  int hp[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int h = 0; h < 6; ++h) {
    int m = hp[h][0], n = hp[h][1];
    hess[h] = F[2] * g[m] * g[n] + F[1] * ((m == n ? p[m] : 0.0) - g[m] * g[n]) / rho;
  }
  *lap = F[2] * G + F[1] * (P - G) / rho;
  for (int n = 0; n < 3; ++n) {
    double dG = 2.0 * g[n] * (p[n] - G) / rho, dP = -4.0 * kf * rho * g[n];
    glap[n] = F[3] * g[n] * G + F[2] * dG + F[2] * g[n] * (P - G) / rho +
              F[1] * ((dP - dG) / rho - (P - G) * g[n] / (rho * rho));
  }
}

/* ------------------------------------------------------ three-body term -- */
static int j3_on(const osys* s) { return s->j3f[0] != 0.0 || s->j3f[1] != 0.0 || s->j3f[2] != 0.0; }
static int j1f_on(const osys* s) { return s->j1f[0] != 0.0 || s->j1f[1] != 0.0; }

/* One Cartesian factor of the Jastrow orbitals at the offset d along an axis: with the periodised
 * component rho = (L/pi) sin(pi d / L) (rho = d in the open kinds), u = rho^2 and
 * a = e^{-ZJ u}, b = u a, the derivatives in d to third order by the chain rule:
 *   u' = 2 rho c, u'' = 2 (c^2 - k rho^2), u''' = -8 k rho c   (c = cos(pi d / L), k = (pi/L)^2),
 *   a' = -Z u' a, a'' = (Z^2 u'^2 - Z u'') a, a''' = (-Z^3 u'^3 + 3 Z^2 u' u'' - Z u''') a,
 *   b' = u' a + u a', b'' = u'' a + 2 u' a' + u a'', b''' = u''' a + 3 u'' a' + 3 u' a'' + u a'''. */
static void j3_axis(const osys* s, double d, double a[4], double b[4]) {
  double rho, c, k;
  if (s->basis_kind == OB_PERIODIC_GAUSS) {
    rho = s->L / PI * sin(PI * d / s->L);
    c = cos(PI * d / s->L);
    k = (PI / s->L) * (PI / s->L);
  } else {
    rho = d; c = 1.0; k = 0.0;
  }
  const double Z = O_ZJ;
  const double u = rho * rho, u1 = 2.0 * rho * c, u2 = 2.0 * (c * c - k * rho * rho), u3 = -8.0 * k * rho * c;
  const double e = exp(-Z * u);
  a[0] = e;
  a[1] = -Z * u1 * e;
  a[2] = (Z * Z * u1 * u1 - Z * u2) * e;
  a[3] = (-Z * Z * Z * u1 * u1 * u1 + 3.0 * Z * Z * u1 * u2 - Z * u3) * e;
  b[0] = u * a[0];
  b[1] = u1 * a[0] + u * a[1];
  b[2] = u2 * a[0] + 2.0 * u1 * a[1] + u * a[2];
  b[3] = u3 * a[0] + 3.0 * u2 * a[1] + 3.0 * u1 * a[2] + u * a[3];
}

/* chi_1 = a a a and chi_2 = rho^2 e^{-Z rho^2} = b a a + a b a + a a b, each as 14 components. */
void o_j3_orbitals(const osys* s, int atom, const double r[3], double out[28]) {
  double A[3][4], B[3][4];
  for (int m = 0; m < 3; ++m) j3_axis(s, r[m] - s->R[3 * atom + m], A[m], B[m]);
  for (int q = 0; q < 28; ++q) out[q] = 0.0;
  add_product(A, 1.0, out);
  for (int m = 0; m < 3; ++m) {
    double f[3][4];
    for (int mm = 0; mm < 3; ++mm)
      for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? B[mm][q] : A[mm][q];
    add_product(f, 1.0, out + 14);
  }
}

/* chi_a(r)^T F chi'  for 14-component orbital blocks: component q of the first pair with the
 * value of the second (F symmetric: f11, f12, f22). */
static double j3_form(const osys* s, const double* ci, int q, const double* cj, int qj) {
  const double* f = s->j3f;
  return f[0] * ci[q] * cj[qj] + f[1] * (ci[q] * cj[14 + qj] + ci[14 + q] * cj[qj]) + f[2] * ci[14 + q] * cj[14 + qj];
}

/* U = sum_{i<j} u(rho_ij) + U_1 + U_3; gradU (Ne x 3) and lapU (Ne) are w.r.t. each electron.
 * U_3 = sum_a sum_{i<j} chi_a(r_i)^T F chi_a(r_j) (SI, Eq. e:j33, on-site), summed pair by pair. */
void o_jastrow(const osys* s, const double* x, double* U, double* gradU, double* lapU) {
  int ne = s->n_up + s->n_dn;
  double Ut = 0.0;
  if (gradU) memset(gradU, 0, sizeof(double) * 3 * ne);
  if (lapU) memset(lapU, 0, sizeof(double) * ne);
  if (s->b1 > 0.0)
    for (int i = 0; i < ne; ++i)
      for (int a = 0; a < s->n_p; ++a) {
        double d[3] = {x[3 * i] - s->R[3 * a], x[3 * i + 1] - s->R[3 * a + 1], x[3 * i + 2] - s->R[3 * a + 2]};
        double F[4], g[3], h[6], lp, gl[3];
        j1_radial(s->b1, periodised_rho(s, d), F);
        radial_field(s, d, F, g, h, &lp, gl);
        Ut += F[0];
        if (gradU)
          for (int m = 0; m < 3; ++m) gradU[3 * i + m] += g[m];
        if (lapU) lapU[i] += lp;
      }
  /* the orbital part of U_1 (Eq. e:j1): f^T chi_a(r_i) over every electron and nucleus */
  if (j1f_on(s))
    for (int i = 0; i < ne; ++i)
      for (int a = 0; a < s->n_p; ++a) {
        double c[28];
        o_j3_orbitals(s, a, x + 3 * i, c);
        Ut += s->j1f[0] * c[0] + s->j1f[1] * c[14];
        if (gradU)
          for (int m = 0; m < 3; ++m) gradU[3 * i + m] += s->j1f[0] * c[1 + m] + s->j1f[1] * c[15 + m];
        if (lapU) lapU[i] += s->j1f[0] * c[4] + s->j1f[1] * c[18];
      }
  if (j3_on(s)) {
    const int np = s->n_p;
    double* ch = malloc(sizeof(double) * 28 * (size_t)ne * np);
    for (int i = 0; i < ne; ++i)
      for (int a = 0; a < np; ++a) o_j3_orbitals(s, a, x + 3 * i, ch + 28 * ((size_t)i * np + a));
    for (int a = 0; a < np; ++a)
      for (int i = 0; i < ne; ++i) {
        const double* ci = ch + 28 * ((size_t)i * np + a);
        for (int j = 0; j < ne; ++j) {
          if (j == i) continue;
          const double* cj = ch + 28 * ((size_t)j * np + a);
          if (j > i) Ut += j3_form(s, ci, 0, cj, 0);
          if (gradU)
            for (int m = 0; m < 3; ++m) gradU[3 * i + m] += j3_form(s, ci, 1 + m, cj, 0);
          if (lapU) lapU[i] += j3_form(s, ci, 4, cj, 0);
        }
      }
    free(ch);
  }
  if (!s->jastrow_on) { *U = Ut; return; }
  for (int i = 0; i < ne; ++i)
    for (int j = i + 1; j < ne; ++j) {
      double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
      double u, up, upp, g[3], lr;
      jas_pair(s, d, spin_of(s, i) == spin_of(s, j), &u, &up, &upp, g, &lr);
      Ut += u;
      double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      if (gradU)
        for (int m = 0; m < 3; ++m) { gradU[3 * i + m] += up * g[m]; gradU[3 * j + m] -= up * g[m]; }
      if (lapU) { lapU[i] += upp * g2 + up * lr; lapU[j] += upp * g2 + up * lr; }
    }
  *U = Ut;
}

/* ------------------------------------------------- variational parameters -- */
/* O_k = d ln psi / d p_k for the Jastrow parameters p = (b, b_1, f_11, f_12, f_22, f_1, f_2): the
 * logarithmic derivatives that stochastic reconfiguration (Sorella, PRB 64, 024512 (2001); the
 * paper re-optimises the wavefunction before each ionic step) uses.  Each is the derivative of
 * the term's own definition, summed pair by pair:
 *   b    two-body u = a rho / (1 + b rho):        sum_{i<j} -a_ij rho_ij^2 / (1 + b rho_ij)^2
 *   b_1  one-body -(2Z)^{3/4} u_1((2Z)^{1/4} rho), u_1(y) = (1 - e^{-b_1 y}) / (2 b_1), Z = 1:
 *        d u_1 / d b_1 = [b_1 y e^{-b_1 y} - (1 - e^{-b_1 y})] / (2 b_1^2), summed over (i, a)
 *   f_qr three-body (Eq. e:j33) with f_12 = f_21:  sum_a sum_{i<j} chi_q(r_ia) chi_r(r_ja)
 *        (+ chi_r(r_ia) chi_q(r_ja) for q != r).
 *   f_q  one-body orbital part (Eq. e:j1):  sum_a sum_i chi_q(r_ia).
 * O_b1 is 0 without the one-body term (b_1 = 0 means no term); the three-body derivatives do not
 * depend on F and are formed for any F, zero included. */
void o_param_derivs(const osys* s, const double* x, double O[O_NPAR]) {
  const int ne = s->n_up + s->n_dn;
  for (int k = 0; k < O_NPAR; ++k) O[k] = 0.0;
  if (s->jastrow_on)
    for (int i = 0; i < ne; ++i)
      for (int j = i + 1; j < ne; ++j) {
        double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
        const double rho = periodised_rho(s, d), a = spin_of(s, i) == spin_of(s, j) ? s->a_par : s->a_anti;
        const double den = 1.0 + s->b * rho;
        O[0] += -a * rho * rho / (den * den);
      }
  if (s->b1 > 0.0) {
    const double Z = 1.0, c = pow(2.0 * Z, 0.75), sc = pow(2.0 * Z, 0.25), b1 = s->b1;
    for (int i = 0; i < ne; ++i)
      for (int a = 0; a < s->n_p; ++a) {
        double d[3] = {x[3 * i] - s->R[3 * a], x[3 * i + 1] - s->R[3 * a + 1], x[3 * i + 2] - s->R[3 * a + 2]};
        const double y = sc * periodised_rho(s, d), e = exp(-b1 * y);
        O[1] += -c * (b1 * y * e - (1.0 - e)) / (2.0 * b1 * b1);
      }
  }
  double* v1 = malloc(sizeof(double) * ne);
  double* v2 = malloc(sizeof(double) * ne);
  for (int a = 0; a < s->n_p; ++a) {
    for (int i = 0; i < ne; ++i) {
      double ci[28];
      o_j3_orbitals(s, a, x + 3 * i, ci);
      v1[i] = ci[0];
      v2[i] = ci[14];
      O[5] += ci[0];
      O[6] += ci[14];
    }
    for (int i = 0; i < ne; ++i)
      for (int j = i + 1; j < ne; ++j) {
        O[2] += v1[i] * v1[j];
        O[3] += v1[i] * v2[j] + v2[i] * v1[j];
        O[4] += v2[i] * v2[j];
      }
  }
  free(v1);
  free(v2);
}

/* -------------------------------------------------------------- potential -- */
/* Coulomb energy of the protons (+1 at R) and electrons (-1 at x).
 * OP_EWALD: real-space erfc sum over minimum-image pairs, reciprocal sum over
 * half-space vectors k = 2 pi n / L with 0 < |n|^2 <= nmax^2, self term; the
 * cell is neutral so there is no background term.
 * Returns V; dV_dR (n_p x 3) and dV_dx (Ne x 3) are gradients (may be NULL). */
double o_potential(const osys* s, const double* x, double* dV_dR, double* dV_dx) {
  int np = s->n_p, ne = s->n_up + s->n_dn, nq = np + ne;
  double* pos = (double*)malloc(sizeof(double) * 3 * nq);
  double* q = (double*)malloc(sizeof(double) * nq);
  double* grad = (double*)calloc(3 * nq, sizeof(double));
  for (int i = 0; i < np; ++i) { memcpy(pos + 3 * i, s->R + 3 * i, 3 * sizeof(double)); q[i] = 1.0; }
  for (int i = 0; i < ne; ++i) { memcpy(pos + 3 * (np + i), x + 3 * i, 3 * sizeof(double)); q[np + i] = -1.0; }
  double V = 0.0;
  if (s->pot_kind == OP_EWALD || s->pot_kind == OP_COULOMB_OPEN) {
    int ew = (s->pot_kind == OP_EWALD);
    double kap = s->kappa, L = s->L;
    for (int i = 0; i < nq; ++i)
      for (int j = i + 1; j < nq; ++j) {
        double d[3];
        for (int m = 0; m < 3; ++m) {
          d[m] = pos[3 * i + m] - pos[3 * j + m];
          if (ew) d[m] = min_image(d[m], L);
        }
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double qq = q[i] * q[j];
        double e, dedr;
        if (ew) {
          e = erfc(kap * r) / r;
          dedr = -erfc(kap * r) / (r * r) - 2.0 * kap / sqrt(PI) * exp(-kap * kap * r * r) / r;
        } else {
          e = 1.0 / r;
          dedr = -1.0 / (r * r);
        }
        V += qq * e;
        for (int m = 0; m < 3; ++m) {
          grad[3 * i + m] += qq * dedr * d[m] / r;
          grad[3 * j + m] -= qq * dedr * d[m] / r;
        }
      }
    if (ew) {
      double vol = L * L * L;
      int nm = s->nmax;
      for (int nx = 0; nx <= nm; ++nx)
        for (int ny = -nm; ny <= nm; ++ny)
          for (int nz = -nm; nz <= nm; ++nz) {
            int n2 = nx * nx + ny * ny + nz * nz;
            if (n2 == 0 || n2 > nm * nm) continue;
            if (!(nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0))))) continue;
            double k[3] = {2 * PI * nx / L, 2 * PI * ny / L, 2 * PI * nz / L};
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double w = exp(-k2 / (4 * kap * kap)) / k2;
            double rr = 0.0, ri = 0.0;
            for (int i = 0; i < nq; ++i) {
              double th = k[0] * pos[3 * i] + k[1] * pos[3 * i + 1] + k[2] * pos[3 * i + 2];
              rr += q[i] * cos(th);
              ri += q[i] * sin(th);
            }
            V += 4 * PI / vol * w * (rr * rr + ri * ri);
            for (int i = 0; i < nq; ++i) {
              double th = k[0] * pos[3 * i] + k[1] * pos[3 * i + 1] + k[2] * pos[3 * i + 2];
              double im = rr * sin(th) - ri * cos(th);   /* Im(conj(rho) e^{i th}) */
              for (int m = 0; m < 3; ++m) grad[3 * i + m] += -8 * PI / vol * w * k[m] * q[i] * im;
            }
          }
      V += -kap / sqrt(PI) * (double)nq;   /* every charge is +-1 */
    }
  } else if (s->pot_kind == OP_HARMONIC) {
    double z = s->zeta[0];
    for (int e = 0; e < ne; ++e)
      for (int m = 0; m < 3; ++m) {
        double d = x[3 * e + m] - s->R[m];
        V += 2.0 * z * z * d * d;
        grad[3 * (np + e) + m] += 4.0 * z * z * d;
        grad[m] -= 4.0 * z * z * d;
      }
  }
  if (dV_dR) memcpy(dV_dR, grad, sizeof(double) * 3 * np);
  if (dV_dx) memcpy(dV_dx, grad + 3 * np, sizeof(double) * 3 * ne);
  free(pos); free(q); free(grad);
  return V;
}

/* ------------------------------------------------------------ local energy -- */
/* The proton derivatives of the one-body and three-body Jastrow terms (each moves with its
 * nucleus): adds their part of d ln psi / dR to dln and of dT_L / dR to dT, given per electron
 * vv = grad_i U + grad_i ln|D| (the real part of grad_i ln D for complex orbitals). */
void o_jastrow_dR(const osys* s, const double* x, const double* vv, double* dln, double* dT) {
  const int ne = s->n_up + s->n_dn, np = s->n_p;
  /* The one-body term depends on R_a through r_i - R_a, so d/dR_a = -grad_i on it:
   * d ln psi / dR_a gets -grad_i f_ia, and the kinetic part
   * -1/2 sum_i (lap_i U + |grad_i U|^2 + 2 grad_i ln|D| . grad_i U) + (the determinant
   * terms, already differentiated above with the full grad U) gets
   * sum_i [ 1/2 grad_i lap_i f_ia + hess_i f_ia (grad_i U + grad_i ln|D|) ]. */
  if (s->b1 > 0.0)
    for (int a = 0; a < np; ++a)
      for (int i = 0; i < ne; ++i) {
        double d[3] = {x[3 * i] - s->R[3 * a], x[3 * i + 1] - s->R[3 * a + 1], x[3 * i + 2] - s->R[3 * a + 2]};
        double F[4], g[3], h[6], lp, gl[3];
        j1_radial(s->b1, periodised_rho(s, d), F);
        radial_field(s, d, F, g, h, &lp, gl);
        double v[3];
        for (int m = 0; m < 3; ++m) v[m] = vv[3 * i + m];
        for (int mu = 0; mu < 3; ++mu) {
          dln[3 * a + mu] -= g[mu];
          double hv = 0.0;
          for (int nu = 0; nu < 3; ++nu) hv += h[hidx(mu, nu) - 5] * v[nu];
          dT[3 * a + mu] += 0.5 * gl[mu] + hv;
        }
      }
  /* The orbital part of U_1, f^T chi_a(r_i - R_a), the same way: d ln psi/dR_a,mu gets
   * -f^T d_mu chi_ai and the kinetic part 1/2 f^T d_mu lap chi_ai + sum_nu v_i,nu f^T d_mu d_nu chi_ai. */
  if (j1f_on(s))
    for (int a = 0; a < np; ++a)
      for (int i = 0; i < ne; ++i) {
        double c[28];
        o_j3_orbitals(s, a, x + 3 * i, c);
        for (int mu = 0; mu < 3; ++mu) {
          dln[3 * a + mu] -= s->j1f[0] * c[1 + mu] + s->j1f[1] * c[15 + mu];
          double t = 0.5 * (s->j1f[0] * c[11 + mu] + s->j1f[1] * c[25 + mu]);
          for (int nu = 0; nu < 3; ++nu) {
            const int q = hidx(mu, nu);
            t += vv[3 * i + nu] * (s->j1f[0] * c[q] + s->j1f[1] * c[14 + q]);
          }
          dT[3 * a + mu] += t;
        }
      }
  /* The three-body term depends on R_a through chi_a(r_i - R_a), d/dR_a = -grad_i on it: with
   * v_k = grad_k U + grad_k ln|D| and the sums over the other electrons j != k,
   *   d ln psi/dR_a,mu = -sum_k sum_j (d_mu chi_ak)^T F chi_aj,
   *   d(grad_k U)_nu/dR_a,mu = -sum_j [(d_mu d_nu chi_ak)^T F chi_aj + (d_nu chi_ak)^T F d_mu chi_aj],
   *   d(lap_k U)/dR_a,mu = -sum_j [(d_mu lap chi_ak)^T F chi_aj + (lap chi_ak)^T F d_mu chi_aj],
   * and the kinetic part changes by -1/2 sum_k d(lap_k U) - sum_k v_k . d(grad_k U). */
  if (j3_on(s)) {
    double* ch = malloc(sizeof(double) * 28 * (size_t)ne * np);
    for (int i = 0; i < ne; ++i)
      for (int a = 0; a < np; ++a) o_j3_orbitals(s, a, x + 3 * i, ch + 28 * ((size_t)i * np + a));
    for (int a = 0; a < np; ++a)
      for (int mu = 0; mu < 3; ++mu) {
        double dl = 0.0, dt = 0.0;
        for (int k = 0; k < ne; ++k) {
          const double* ck = ch + 28 * ((size_t)k * np + a);
          double v[3];
          for (int m = 0; m < 3; ++m) v[m] = vv[3 * k + m];
          for (int j = 0; j < ne; ++j) {
            if (j == k) continue;
            const double* cj = ch + 28 * ((size_t)j * np + a);
            dl -= j3_form(s, ck, 1 + mu, cj, 0);
            const double dlap = -(j3_form(s, ck, 11 + mu, cj, 0) + j3_form(s, ck, 4, cj, 1 + mu));
            dt += -0.5 * dlap;
            for (int nu = 0; nu < 3; ++nu) {
              const double dg = -(j3_form(s, ck, hidx(mu, nu), cj, 0) + j3_form(s, ck, 1 + nu, cj, 1 + mu));
              dt -= v[nu] * dg;
            }
          }
        }
        dln[3 * a + mu] += dl;
        dT[3 * a + mu] += dt;
      }
    free(ch);
  }
}

/* For one electron configuration x (Ne x 3): ln|psi|, sign(psi), the local
 * energy E_L = -1/2 sum_i lap_i psi / psi + V, and the derivatives of ln|psi|
 * and E_L with respect to the proton positions at fixed C, zeta and Jastrow.
 * psi = D_up D_dn e^U, D_s = det A_s, A_s[i][k] = sum_a phi_a(r_i) C[a][k].
 * Determinant derivatives use Jacobi's formula d ln det A = tr(A^-1 dA) and
 * d A^-1 = -A^-1 dA A^-1, each written out as plain matrix products. */
int o_local(const osys* s, const double* x, double* lnpsi, double* sign, double* EL,
            double* dlnpsi_dR, double* dEL_dR) {
  int np = s->n_p, ne = s->n_up + s->n_dn, no = s->n_orb, n3 = 3 * np;
  double U;
  double* gU = (double*)malloc(sizeof(double) * 3 * ne);
  double* lU = (double*)malloc(sizeof(double) * ne);
  o_jastrow(s, x, &U, gU, lU);
  double* dVdR = (double*)malloc(sizeof(double) * n3);
  double V = o_potential(s, x, dVdR, NULL);
  double T = 0.0, lnp = U, sg = 1.0;
  for (int e = 0; e < ne; ++e)
    T += -0.5 * (lU[e] + gU[3 * e] * gU[3 * e] + gU[3 * e + 1] * gU[3 * e + 1] + gU[3 * e + 2] * gU[3 * e + 2]);
  int want = (dlnpsi_dR != NULL) || (dEL_dR != NULL);
  double* dln = (double*)calloc(n3, sizeof(double));
  double* dT = (double*)calloc(n3, sizeof(double));
  double* gDe = (double*)calloc(3 * ne, sizeof(double));   /* grad_i ln|D| per electron */
  int rc = 0;
  for (int sp = 0; sp < 2 && rc == 0; ++sp) {
    int n = sp ? s->n_dn : s->n_up, e0 = sp ? s->n_up : 0;
    if (n == 0) continue;
    double* bf = (double*)malloc(sizeof(double) * 14 * n * np);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < np; ++a) o_basis(s, a, x + 3 * (e0 + i), bf + 14 * (i * np + a));
    double *A = calloc(n * n, 8), *G = calloc(3 * n * n, 8), *Lp = calloc(n * n, 8), *Ai = malloc(8 * n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k)
        for (int a = 0; a < np; ++a) {
          const double* f = bf + 14 * (i * np + a);
          double c = s->C[a * no + k];
          A[i * n + k] += f[0] * c;
          for (int m = 0; m < 3; ++m) G[(m * n + i) * n + k] += f[1 + m] * c;
          Lp[i * n + k] += f[4] * c;
        }
    double ld, sgn;
    rc = lu_logdet(n, A, &ld, &sgn, Ai);
    if (rc) { free(bf); free(A); free(G); free(Lp); free(Ai); break; }
    lnp += ld;
    sg *= sgn;
    for (int i = 0; i < n; ++i) {
      double lapD = 0.0, gD[3] = {0, 0, 0};
      for (int k = 0; k < n; ++k) {
        lapD += Lp[i * n + k] * Ai[k * n + i];
        for (int m = 0; m < 3; ++m) gD[m] += G[(m * n + i) * n + k] * Ai[k * n + i];
      }
      const double* gu = gU + 3 * (e0 + i);
      T += -0.5 * (lapD + 2.0 * (gD[0] * gu[0] + gD[1] * gu[1] + gD[2] * gu[2]));
      for (int m = 0; m < 3; ++m) gDe[3 * (e0 + i) + m] = gD[m];
    }
    if (want) {
      double *dA = malloc(8 * n * n), *dG = malloc(8 * 3 * n * n), *dL = malloc(8 * n * n);
      double *tmp = malloc(8 * n * n), *dAi = malloc(8 * n * n);
      for (int b = 0; b < np; ++b)
        for (int mu = 0; mu < 3; ++mu) {
          /* d/dR_b acts only on phi_b(r - R_b): d phi_b/dR_b,mu = -d_mu phi_b. */
          for (int i = 0; i < n; ++i) {
            const double* f = bf + 14 * (i * np + b);
            for (int k = 0; k < n; ++k) {
              double c = s->C[b * no + k];
              dA[i * n + k] = -f[1 + mu] * c;
              for (int nu = 0; nu < 3; ++nu) dG[(nu * n + i) * n + k] = -f[hidx(mu, nu)] * c;
              dL[i * n + k] = -f[11 + mu] * c;
            }
          }
          matmul(n, Ai, dA, tmp);
          matmul(n, tmp, Ai, dAi);
          for (int t = 0; t < n * n; ++t) dAi[t] = -dAi[t];
          double tr = 0.0;
          for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) tr += Ai[k * n + i] * dA[i * n + k];
          dln[3 * b + mu] += tr;
          double dt = 0.0;
          for (int i = 0; i < n; ++i) {
            double dlap = 0.0, dgD[3] = {0, 0, 0};
            for (int k = 0; k < n; ++k) {
              dlap += dL[i * n + k] * Ai[k * n + i] + Lp[i * n + k] * dAi[k * n + i];
              for (int nu = 0; nu < 3; ++nu)
                dgD[nu] += dG[(nu * n + i) * n + k] * Ai[k * n + i] + G[(nu * n + i) * n + k] * dAi[k * n + i];
            }
            const double* gu = gU + 3 * (e0 + i);
            dt += -0.5 * (dlap + 2.0 * (dgD[0] * gu[0] + dgD[1] * gu[1] + dgD[2] * gu[2]));
          }
          dT[3 * b + mu] += dt;
        }
      free(dA); free(dG); free(dL); free(tmp); free(dAi);
    }
    free(bf); free(A); free(G); free(Lp); free(Ai);
  }
  if (rc == 0 && want && (s->b1 > 0.0 || j3_on(s) || j1f_on(s))) {
    double* vv = malloc(sizeof(double) * 3 * ne);
    for (int t = 0; t < 3 * ne; ++t) vv[t] = gU[t] + gDe[t];
    o_jastrow_dR(s, x, vv, dln, dT);
    free(vv);
  }
  if (rc == 0) {
    if (lnpsi) *lnpsi = lnp;
    if (sign) *sign = sg;
    if (EL) *EL = T + V;
    if (dlnpsi_dR) memcpy(dlnpsi_dR, dln, sizeof(double) * n3);
    if (dEL_dR)
      for (int t = 0; t < n3; ++t) dEL_dR[t] = dT[t] + dVdR[t];
  }
  free(gU); free(lU); free(dVdR); free(dln); free(dT); free(gDe);
  return rc;
}

/* ---------------------------------------------------------------- Hueckel -- */
/* Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (in place);
 * eigenvectors are the columns of V. */
static void jacobi_eigen(int n, double* A, double* V) {
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * akq;
          A[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * aqk;
          A[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
}

/* Hueckel orbitals on the periodic s-Gaussians: overlap
 * S_ab = (pi/(za+zb))^{3/2} prod_m sum_n exp(-za zb/(za+zb) (d_m + n L)^2),
 * normalised S~_ab = S_ab / sqrt(S_aa S_bb), H = -S~, the n_orb lowest
 * eigenvectors v, and C_ak = v_ak / sqrt(S_aa). */
int o_huckel(int n_p, double L, const double* R, const double* zeta, int n_orb, double* C, double* evals) {
  return o_huckel_twist(n_p, L, R, zeta, n_orb, 0, C, evals);
}

static int huckel_from_overlap(int n_p, const double* S, int n_orb, double* C, double* evals);

/* Hueckel orbitals of the twisted basis (real twists, bit m of twist = angle pi along m).
 * The cell overlap of two image sums is one image sum of the plane-space overlaps,
 * S_ab = sum_n tau^n (pi/(za+zb))^{3/2} e^{-mu |R_a - R_b + n L|^2}, tau^n = prod_m tau_m^{n_m}. */
int o_huckel_twist(int n_p, double L, const double* R, const double* zeta, int n_orb, int twist, double* C,
                   double* evals) {
  if (n_orb > n_p || n_orb < 0) return O_EINVAL;
  double* S = malloc(8 * n_p * n_p);
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) {
      double za = zeta[a], zb = zeta[b], mu = za * zb / (za + zb);
      double v = pow(PI / (za + zb), 1.5);
      for (int m = 0; m < 3; ++m) {
        double tau = ((twist >> m) & 1) ? -1.0 : 1.0;
        double d = R[3 * a + m] - R[3 * b + m], acc = 0.0;
        for (int n = -4; n <= 4; ++n) acc += ((n & 1) ? tau : 1.0) * exp(-mu * (d + n * L) * (d + n * L));
        v *= acc;
      }
      S[a * n_p + b] = v;
    }
  int rc = huckel_from_overlap(n_p, S, n_orb, C, evals);
  free(S);
  return rc;
}

/* The Hueckel step shared by the bases: H = -S_ab / sqrt(S_aa S_bb), its eigenvectors by
 * Jacobi rotations, the n_orb lowest v, C_ak = v_ak / sqrt(S_aa); evals ascending. */
static int huckel_from_overlap(int n_p, const double* S, int n_orb, double* C, double* evals) {
  double* H = malloc(8 * n_p * n_p);
  double* Vv = malloc(8 * n_p * n_p);
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) H[a * n_p + b] = -S[a * n_p + b] / sqrt(S[a * n_p + a] * S[b * n_p + b]);
  jacobi_eigen(n_p, H, Vv);
  int* order = malloc(sizeof(int) * n_p);
  for (int i = 0; i < n_p; ++i) order[i] = i;
  for (int i = 1; i < n_p; ++i) {   /* insertion sort by eigenvalue */
    int t = order[i], j = i - 1;
    while (j >= 0 && H[order[j] * n_p + order[j]] > H[t * n_p + t]) { order[j + 1] = order[j]; --j; }
    order[j + 1] = t;
  }
  for (int k = 0; k < n_orb; ++k)
    for (int a = 0; a < n_p; ++a) C[a * n_orb + k] = Vv[a * n_p + order[k]] / sqrt(S[a * n_p + a]);
  if (evals)
    for (int k = 0; k < n_p; ++k) evals[k] = H[order[k] * n_p + order[k]];
  free(H); free(Vv); free(order);
  return 0;
}

/* One-dimensional Gaussian moments of e^{-al x^2} e^{-be (x - d)^2} = e^{-p (x - P)^2} e^{-mu d^2}
 * (p = al + be, P = be d / p, mu = al be / p): with x = y + P, x - d = y - Q (Q = al d / p)
 * and the moments m0 = sqrt(pi/p), m2 = m0/(2p), m4 = 3 m0/(4 p^2) of e^{-p y^2},
 *   out[0] = int 1             = m0
 *   out[1] = int x^2           = m2 + P^2 m0
 *   out[2] = int (x-d)^2       = m2 + Q^2 m0
 *   out[3] = int x^2 (x-d)^2   = m4 + ((P - Q)^2 - 2 P Q) m2 + P^2 Q^2 m0,
 * each times e^{-mu d^2} and summed over the images d + n L, |n| <= 4. */
static void moments_1d(double al, double be, double d, double L, double out[4]) {
  const double p = al + be, mu = al * be / p;
  const double m0 = sqrt(PI / p), m2 = m0 / (2.0 * p), m4 = 3.0 * m0 / (4.0 * p * p);
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int n = -4; n <= 4; ++n) {
    const double dd = d + n * L, e = exp(-mu * dd * dd);
    const double P = be * dd / p, Q = al * dd / p;
    out[0] += e * m0;
    out[1] += e * (m2 + P * P * m0);
    out[2] += e * (m2 + Q * Q * m0);
    out[3] += e * (m4 + ((P - Q) * (P - Q) - 2.0 * P * Q) * m2 + P * P * Q * Q * m0);
  }
}

/* S_ab = <phi_a | phi_b> over the cell for phi = g1 + eta h2 (g1 = e^{-Z1 r^2},
 * h2 = r^2 e^{-Z2 r^2}): one image sum of free-space overlaps, every term separable, with x the
 * coordinate relative to R_a, d = R_b - R_a and [.]_m the moments of axis m:
 *   <g1|g1> = prod_m [1]_m                                          (Z1, Z1)
 *   <g1|h2> = sum_m [(x-d)^2]_m prod_{m' != m} [1]_m'                  (Z1, Z2)
 *   <h2|g1> = sum_m [x^2]_m prod_{m' != m} [1]_m'                      (Z2, Z1)
 *   <h2|h2> = sum_m [x^2 (x-d)^2]_m prod_{m' != m} [1]_m'
 *           + sum_{m != m'} [x^2]_m [(x-d)^2]_m' [1]_m''               (Z2, Z2) */
void o_overlap_contracted(int n_p, double L, const double* R, double eta, double* S) {
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) {
      double m11[3][4], m12[3][4], m21[3][4], m22[3][4];
      for (int m = 0; m < 3; ++m) {
        const double d = R[3 * b + m] - R[3 * a + m];
        moments_1d(O_Z1, O_Z1, d, L, m11[m]);
        moments_1d(O_Z1, O_Z2, d, L, m12[m]);
        moments_1d(O_Z2, O_Z1, d, L, m21[m]);
        moments_1d(O_Z2, O_Z2, d, L, m22[m]);
      }
      const double s11 = m11[0][0] * m11[1][0] * m11[2][0];
      double s12 = 0.0, s21 = 0.0, s22 = 0.0;
      for (int m = 0; m < 3; ++m) {
        double p12 = m12[m][2], p21 = m21[m][1], p22 = m22[m][3];
        for (int q = 0; q < 3; ++q)
          if (q != m) { p12 *= m12[q][0]; p21 *= m21[q][0]; p22 *= m22[q][0]; }
        s12 += p12;
        s21 += p21;
        s22 += p22;
        for (int m2 = 0; m2 < 3; ++m2) {
          if (m2 == m) continue;
          double pc = m22[m][1] * m22[m2][2];
          for (int q = 0; q < 3; ++q)
            if (q != m && q != m2) pc *= m22[q][0];
          s22 += pc;
        }
      }
      S[a * n_p + b] = s11 + eta * (s12 + s21) + eta * eta * s22;
    }
}

int o_huckel_contracted(int n_p, double L, const double* R, double eta, int n_orb, double* C, double* evals) {
  if (n_orb > n_p || n_orb < 0) return O_EINVAL;
  double* S = malloc(8 * n_p * n_p);
  o_overlap_contracted(n_p, L, R, eta, S);
  int rc = huckel_from_overlap(n_p, S, n_orb, C, evals);
  free(S);
  return rc;
}

/* ------------------------------------------------------------ Metropolis -- */
static void mo_row(const osys* s, const double r[3], double* m) {
  double f[14];
  for (int k = 0; k < s->n_orb; ++k) m[k] = 0.0;
  for (int a = 0; a < s->n_p; ++a) {
    o_basis(s, a, r, f);
    for (int k = 0; k < s->n_orb; ++k) m[k] += f[0] * s->C[a * s->n_orb + k];
  }
}

/* Runs n_equil unmeasured and then n_meas measured sweeps on each of W walkers.
 * Sweep: electrons e = 0..Ne-1 in order; move r' = r_e + delta (u - 1/2) (wrapped
 * into the box); accept iff u_acc < |psi'/psi|^2, strictly.  The determinant
 * ratio is det A'/det A from two fresh LU factorisations; the Jastrow change is
 * the sum of the pair changes (and of the moved electron's one-body terms).  Random numbers: Philox key (seed, traj),
 * counter (step, walker, sweep*Ne + e, 0|1).  After each measured sweep the
 * local quantities of o_local are added to sums[w] = [sum E_L, sum E_L^2,
 * sum dE_L/dR (3N), sum dln|psi|/dR (3N), sum E_L dln|psi|/dR (3N)].
 * o_vmc_run_from runs walkers w0 .. w0+W-1 of a larger set: x, sums and n_acc hold
 * only those W walkers, and walker w draws from the counter of walker w0 + w. */
int o_vmc_run(const osys* s, int W, double* x, int n_equil, int n_meas, double delta,
              uint32_t seed, uint32_t traj, uint32_t step, double* sums, int64_t* n_acc, int n_threads) {
  return o_vmc_run_opt(s, W, 0u, x, n_equil, n_meas, delta, seed, traj, step, sums, n_acc, NULL, n_threads);
}

int o_vmc_run_from(const osys* s, int W, uint32_t w0, double* x, int n_equil, int n_meas, double delta,
                   uint32_t seed, uint32_t traj, uint32_t step, double* sums, int64_t* n_acc, int n_threads) {
  return o_vmc_run_opt(s, W, w0, x, n_equil, n_meas, delta, seed, traj, step, sums, n_acc, NULL, n_threads);
}

int o_vmc_run_opt(const osys* s, int W, uint32_t w0, double* x, int n_equil, int n_meas, double delta,
                  uint32_t seed, uint32_t traj, uint32_t step, double* sums, int64_t* n_acc, double* popt,
                  int n_threads) {
  int ne = s->n_up + s->n_dn, n3 = 3 * s->n_p, nsum = 2 + 3 * n3;
  int periodic = (s->basis_kind == OB_PERIODIC_GAUSS);
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int w = 0; w < W; ++w) {
    double* xw = x + (size_t)w * 3 * ne;
    double* sw = sums + (size_t)w * nsum;
    memset(sw, 0, sizeof(double) * nsum);
    double* pw = popt ? popt + (size_t)w * O_NOPT : NULL;
    if (pw) memset(pw, 0, sizeof(double) * O_NOPT);
    int64_t acc = 0;
    double *Asp[2], ld[2] = {0, 0}, sgs[2] = {1, 1};
    int nsp[2] = {s->n_up, s->n_dn};
    for (int sp = 0; sp < 2; ++sp) {
      int n = nsp[sp], e0 = sp ? s->n_up : 0;
      Asp[sp] = malloc(8 * (n > 0 ? n * n : 1));
      for (int i = 0; i < n; ++i) {
        double* m = malloc(8 * s->n_orb);
        mo_row(s, xw + 3 * (e0 + i), m);
        memcpy(Asp[sp] + i * n, m, 8 * n);
        free(m);
      }
      if (n > 0 && lu_logdet(n, Asp[sp], &ld[sp], &sgs[sp], NULL)) err = O_ESINGULAR;
    }
    double* Anew = malloc(8 * (ne * ne + 1));
    double* m = malloc(8 * (s->n_orb + 1));
    double* dE = malloc(8 * n3);
    double* dg = malloc(8 * n3);
    uint32_t key[2] = {seed, traj};
    for (int sw_i = 0; sw_i < n_equil + n_meas; ++sw_i) {
      for (int e = 0; e < ne; ++e) {
        uint32_t c0[4] = {step, w0 + (uint32_t)w, (uint32_t)(sw_i * ne + e), 0u}, o0[4], o1[4];
        uint32_t c1[4] = {step, w0 + (uint32_t)w, (uint32_t)(sw_i * ne + e), 1u};
        o_philox(c0, key, o0);
        o_philox(c1, key, o1);
        double u[3] = {o_u01(o0[0], o0[1]), o_u01(o0[2], o0[3]), o_u01(o1[0], o1[1])};
        double uacc = o_u01(o1[2], o1[3]);
        double rn[3];
        for (int mm = 0; mm < 3; ++mm) {
          rn[mm] = xw[3 * e + mm] + delta * (u[mm] - 0.5);
          if (periodic) rn[mm] -= s->L * floor(rn[mm] / s->L);
        }
        int sp = spin_of(s, e), n = nsp[sp], i = e - (sp ? s->n_up : 0);
        mo_row(s, rn, m);
        memcpy(Anew, Asp[sp], 8 * n * n);
        memcpy(Anew + i * n, m, 8 * n);
        double ldn, sgn;
        double q = 0.0;
        if (lu_logdet(n, Anew, &ldn, &sgn, NULL) == 0) q = sgn * sgs[sp] * exp(ldn - ld[sp]);
        double dU = 0.0;
        if (s->jastrow_on)
          for (int j = 0; j < ne; ++j) {
            if (j == e) continue;
            double dn[3], dold[3], u1, u0, t1, t2, g[3], lr;
            for (int mm = 0; mm < 3; ++mm) { dn[mm] = rn[mm] - xw[3 * j + mm]; dold[mm] = xw[3 * e + mm] - xw[3 * j + mm]; }
            int same = (spin_of(s, j) == sp);
            jas_pair(s, dn, same, &u1, &t1, &t2, g, &lr);
            jas_pair(s, dold, same, &u0, &t1, &t2, g, &lr);
            dU += u1 - u0;
          }
        if (s->b1 > 0.0)
          for (int a = 0; a < s->n_p; ++a) {
            double dn[3], dold[3], F1[4], F0[4];
            for (int mm = 0; mm < 3; ++mm) { dn[mm] = rn[mm] - s->R[3 * a + mm]; dold[mm] = xw[3 * e + mm] - s->R[3 * a + mm]; }
            j1_radial(s->b1, periodised_rho(s, dn), F1);
            j1_radial(s->b1, periodised_rho(s, dold), F0);
            dU += F1[0] - F0[0];
          }
        if (j1f_on(s))
          /* the orbital part of U_1: f^T (chi(r' - R_a) - chi(r_e - R_a)) over the nuclei */
          for (int a = 0; a < s->n_p; ++a) {
            double cn[28], co[28];
            o_j3_orbitals(s, a, rn, cn);
            o_j3_orbitals(s, a, xw + 3 * e, co);
            dU += s->j1f[0] * (cn[0] - co[0]) + s->j1f[1] * (cn[14] - co[14]);
          }
        if (j3_on(s))
          /* the three-body change: sum over nuclei and the other electrons of
           * (chi(r' - R_a) - chi(r_e - R_a))^T F chi(r_j - R_a) */
          for (int a = 0; a < s->n_p; ++a) {
            double cn[28], co[28], cj[28];
            o_j3_orbitals(s, a, rn, cn);
            o_j3_orbitals(s, a, xw + 3 * e, co);
            for (int j = 0; j < ne; ++j) {
              if (j == e) continue;
              o_j3_orbitals(s, a, xw + 3 * j, cj);
              dU += j3_form(s, cn, 0, cj, 0) - j3_form(s, co, 0, cj, 0);
            }
          }
        double p = q * q * exp(2.0 * dU);
        if (uacc < p) {
          memcpy(xw + 3 * e, rn, 3 * sizeof(double));
          memcpy(Asp[sp], Anew, 8 * n * n);
          ld[sp] = ldn;
          sgs[sp] = sgn;
          ++acc;
        }
      }
      if (sw_i >= n_equil) {
        double el;
        if (o_local(s, xw, NULL, NULL, &el, dg, dE)) { err = O_ESINGULAR; continue; }
        sw[0] += el;
        sw[1] += el * el;
        for (int t = 0; t < n3; ++t) {
          sw[2 + t] += dE[t];
          sw[2 + n3 + t] += dg[t];
          sw[2 + 2 * n3 + t] += el * dg[t];
        }
        if (pw) {
          double O[O_NPAR];
          o_param_derivs(s, xw, O);
          pw[0] += el;
          for (int k = 0; k < O_NPAR; ++k) {
            pw[1 + k] += O[k];
            pw[1 + O_NPAR + k] += el * O[k];
            for (int l = 0; l < O_NPAR; ++l) pw[1 + 2 * O_NPAR + O_NPAR * k + l] += O[k] * O[l];
          }
        }
      }
    }
    if (n_acc) n_acc[w] = acc;
    free(Asp[0]); free(Asp[1]); free(Anew); free(m); free(dE); free(dg);
  }
  return err;
}

/* ------------------------------------------------------------- estimators -- */
/* Per-walker means over M samples: e_w, d_w = <dE_L/dR>, g_w = <dln|psi|/dR>,
 * h_w = <E_L dln|psi|/dR>.  E = mean_w e_w, sigma_E = sd_w(e_w)/sqrt(W),
 * f_w = -(d_w + 2 (h_w - E g_w)), f = mean_w f_w.  means (optional) receives
 * [e_w, d_w, g_w, h_w] per walker. */
int o_reduce(int W, int n3, int M, const double* sums, double* E, double* sigma_E,
             double* f, double* f_w, double* means) {
  if (W < 1 || M < 1) return O_EINVAL;
  int nsum = 2 + 3 * n3;
  double Es = 0.0;
  for (int w = 0; w < W; ++w) Es += sums[(size_t)w * nsum] / M;
  double Em = Es / W, var = 0.0;
  for (int w = 0; w < W; ++w) {
    double d = sums[(size_t)w * nsum] / M - Em;
    var += d * d;
  }
  *E = Em;
  *sigma_E = (W > 1) ? sqrt(var / (W - 1)) / sqrt((double)W) : 0.0;
  for (int t = 0; t < n3; ++t) f[t] = 0.0;
  for (int w = 0; w < W; ++w) {
    const double* sw = sums + (size_t)w * nsum;
    for (int t = 0; t < n3; ++t) {
      double d = sw[2 + t] / M, g = sw[2 + n3 + t] / M, h = sw[2 + 2 * n3 + t] / M;
      double fw = -(d + 2.0 * (h - Em * g));
      if (f_w) f_w[(size_t)w * n3 + t] = fw;
      f[t] += fw;
      if (means) {
        double* mw = means + (size_t)w * (1 + 3 * n3);
        mw[0] = sw[0] / M;
        mw[1 + t] = d;
        mw[1 + n3 + t] = g;
        mw[1 + 2 * n3 + t] = h;
      }
    }
  }
  for (int t = 0; t < n3; ++t) f[t] /= W;
  return 0;
}

/* S = Cov of the mean force: sum_w (f_w - f)(f_w - f)^T / (W (W - 1)). */
void o_build_S(int W, int n3, const double* f_w, const double* f, double* S) {
  for (int i = 0; i < n3; ++i)
    for (int j = 0; j < n3; ++j) {
      double acc = 0.0;
      for (int w = 0; w < W; ++w) acc += (f_w[(size_t)w * n3 + i] - f[i]) * (f_w[(size_t)w * n3 + j] - f[j]);
      S[i * n3 + j] = acc / ((double)W * (double)(W - 1));
    }
}

/* Cholesky S = L L^T (lower, row-major).  O_ENOTSPD if S is not positive definite. */
int o_cholesky(int n, const double* S, double* Lc) {
  memset(Lc, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double d = S[j * n + j];
    for (int k = 0; k < j; ++k) d -= Lc[j * n + k] * Lc[j * n + k];
    if (!(d > 0.0)) return O_ENOTSPD;
    Lc[j * n + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = S[i * n + j];
      for (int k = 0; k < j; ++k) v -= Lc[i * n + k] * Lc[j * n + k];
      Lc[i * n + j] = v / Lc[j * n + j];
    }
  }
  return 0;
}

/* One step of the adopted Langevin scheme (SI, Eq. finaldyn_new):
 *   R' = R + Dt S^-1 [ f - (S_prev - S)(R_prev - R) / (2 Db) ] + sqrt(2 T Db) z,
 *   <z z^T> = S^-1,  Dt = (1 - e^{-alpha D})/alpha,  Db = (1 - e^{-2 alpha D})/(2 alpha),
 * with Dt = Db = D at alpha = 0 (Eq. finaldyn).  z = L^-T xi for S = L L^T and
 * xi standard normal.  L_box > 0 wraps R' into [0, L_box) and takes R_prev - R
 * by minimum image.  Flags: CFOLD uses S = I; NO_SCORR drops the S-difference
 * term (Eq. norogna); NOISE_CORR lowers T so that 2 T Db = 2 T_target Db - Dt^2
 * (SI "Noise correction", restated for the Dt/Db form).  On success the state
 * shifts (R_prev, S_prev) <- (R, S); on failure nothing changes. */
int o_langevin(int n3, double L, double* R, double* R_prev, double* S_prev,
               const double* f, const double* S, double T, double Delta, double alpha,
               unsigned flags, uint32_t seed, uint32_t traj, uint32_t step) {
  if (n3 < 1 || !(Delta > 0.0) || alpha < 0.0 || T < 0.0) return O_EINVAL;
  double Dt = Delta, Db = Delta;
  if (alpha > 0.0) {
    Dt = (1.0 - exp(-alpha * Delta)) / alpha;
    Db = (1.0 - exp(-2.0 * alpha * Delta)) / (2.0 * alpha);
  }
  double* Se = malloc(8 * n3 * n3);
  double* Sp = malloc(8 * n3 * n3);
  if (flags & O_STEP_CFOLD) {
    for (int i = 0; i < n3 * n3; ++i) Se[i] = 0.0;
    for (int i = 0; i < n3; ++i) Se[i * n3 + i] = 1.0;
    memcpy(Sp, Se, 8 * n3 * n3);
  } else {
    memcpy(Se, S, 8 * n3 * n3);
    memcpy(Sp, S_prev, 8 * n3 * n3);
  }
  double* v = malloc(8 * n3);
  double* dR = malloc(8 * n3);
  for (int i = 0; i < n3; ++i) {
    dR[i] = R_prev[i] - R[i];
    if (L > 0.0) dR[i] = min_image(dR[i], L);
  }
  for (int i = 0; i < n3; ++i) {
    double c = 0.0;
    if (!(flags & O_STEP_NO_SCORR))
      for (int j = 0; j < n3; ++j) c += (Sp[i * n3 + j] - Se[i * n3 + j]) * dR[j];
    v[i] = f[i] - c / (2.0 * Db);
  }
  double* Lc = malloc(8 * n3 * n3);
  double* y = malloc(8 * n3);
  double* xi = malloc(8 * (n3 + 1));
  double* z = malloc(8 * n3);
  int rc = o_cholesky(n3, Se, Lc);
  double Teff = T;
  if (rc == 0) {
    if (flags & O_STEP_NOISE_CORR) Teff = T - Dt * Dt / (2.0 * Db);
    if (Teff < 0.0) rc = O_EINVAL;
  }
  if (rc == 0) {
    /* y = S^-1 v: L w = v, then L^T y = w. */
    for (int i = 0; i < n3; ++i) {
      double t = v[i];
      for (int k = 0; k < i; ++k) t -= Lc[i * n3 + k] * y[k];
      y[i] = t / Lc[i * n3 + i];
    }
    for (int i = n3 - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n3; ++k) t -= Lc[k * n3 + i] * y[k];
      y[i] = t / Lc[i * n3 + i];
    }
    o_normals(seed, traj, step, n3, xi);
    for (int i = n3 - 1; i >= 0; --i) {   /* L^T z = xi */
      double t = xi[i];
      for (int k = i + 1; k < n3; ++k) t -= Lc[k * n3 + i] * z[k];
      z[i] = t / Lc[i * n3 + i];
    }
    /* a non-finite position, force or noise (NaN input) is an argument error: no change */
    for (int i = 0; i < n3; ++i)
      if (!isfinite(y[i]) || !isfinite(z[i]) || !isfinite(R[i]) || !isfinite(R_prev[i])) rc = O_EINVAL;
  }
  if (rc == 0) {
    double amp = sqrt(2.0 * Teff * Db);
    for (int i = 0; i < n3; ++i) {
      double rn = R[i] + Dt * y[i] + amp * z[i];
      if (L > 0.0) rn -= L * floor(rn / L);
      R_prev[i] = R[i];
      R[i] = rn;
    }
    memcpy(S_prev, S, 8 * n3 * n3);
  }
  free(y); free(xi); free(z);
  free(Se); free(Sp); free(v); free(dR); free(Lc);
  return rc;
}

/* Harmonic test potential V = 1/2 R^T K R (f = -K R) with constant S.
 * Records R every sample_every steps into samples. */
int o_langevin_harmonic_run(int n3, const double* K, const double* S, double T, double Delta,
                            double alpha, unsigned flags, uint32_t seed, int n_steps,
                            double* R, double* samples, int sample_every) {
  double* Rp = malloc(8 * n3);
  double* Sp = malloc(8 * n3 * n3);
  double* f = malloc(8 * n3);
  memcpy(Rp, R, 8 * n3);
  memcpy(Sp, S, 8 * n3 * n3);
  int rc = 0, ns = 0;
  for (int t = 0; t < n_steps && rc == 0; ++t) {
    for (int i = 0; i < n3; ++i) {
      double a = 0.0;
      for (int j = 0; j < n3; ++j) a += K[i * n3 + j] * R[j];
      f[i] = -a;
    }
    rc = o_langevin(n3, 0.0, R, Rp, Sp, f, S, T, Delta, alpha, flags, seed, 0u, (uint32_t)t);
    if (samples && sample_every > 0 && (t + 1) % sample_every == 0) memcpy(samples + (size_t)(ns++) * n3, R, 8 * n3);
  }
  free(Rp); free(Sp); free(f);
  return rc;
}

/* ------------------------------------------------------- rotating spring -- */
/* SI "A simple toy model": U = k (|x| - a)^2 / 2 in the plane and the metric
 * G_lambda = n n^T / lambda + t t^T (radial eigenvalue 1/lambda, tangential 1).
 * s_kind 0: S = G_lambda; s_kind 1: S = H + mu G_lambda, H the Hessian of U; s_kind 2: S = I;
 * s_kind 3: S = H + mu I (the main text's proposal of an empirical Hessian shifted by mu > 0). */
void o_toy_S(double lambda, double k, double a, double mu, int s_kind, const double x[2], double S[4]) {
  if (s_kind == 2) {   /* S = I: the conventional first-order dynamics (black points of Fig. toy) */
    S[0] = S[3] = 1.0;
    S[1] = S[2] = 0.0;
    return;
  }
  double r = sqrt(x[0] * x[0] + x[1] * x[1]);
  double n[2] = {x[0] / r, x[1] / r}, t[2] = {-n[1], n[0]};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) S[2 * i + j] = n[i] * n[j] / lambda + t[i] * t[j];
  if (s_kind == 1 || s_kind == 3) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        double H = k * n[i] * n[j] + k * (r - a) / r * ((i == j) - n[i] * n[j]);
        S[2 * i + j] = H + mu * (s_kind == 1 ? S[2 * i + j] : (double)(i == j));
      }
  }
}

static void inv2(const double S[4], double Si[4]) {
  double det = S[0] * S[3] - S[1] * S[2];
  Si[0] = S[3] / det; Si[1] = -S[1] / det; Si[2] = -S[2] / det; Si[3] = S[0] / det;
}

/* scheme 0: Eq. finaldyn_new (alpha; alpha = 0 is Eq. finaldyn); scheme 1: Eq.
 * norogna (no S-difference term); scheme 2: Eq. standard with gamma = 0 and the
 * term Gamma_j = sum_i d_i S^-1_ji by central differences; scheme 3: the first
 * simplified scheme of the SI (Eq. smartMarkov), y = R + sqrt(2 T D) z and
 * R' = y + D S^-1(R) f(R) - 1/2 S^-1(R) [S(y) - S(R)] (y - R), S taken at R and y.
 * Returns the mean of U over the last 90% of n_steps; U_samples (optional) gets U
 * after every step. */
int o_toy_run(double lambda, double k, double a, double mu, int s_kind, double T, double Delta,
              double alpha, int scheme, uint32_t seed, uint32_t traj, int n_steps, double* R, double* U_mean,
              double* U_samples) {
  double Rp[2] = {R[0], R[1]}, S[4], Sp[4];
  o_toy_S(lambda, k, a, mu, s_kind, R, Sp);
  double acc = 0.0;
  int cnt = 0, burn = n_steps / 10;
  for (int t = 0; t < n_steps; ++t) {
    double r = sqrt(R[0] * R[0] + R[1] * R[1]);
    double f[2] = {-k * (r - a) * R[0] / r, -k * (r - a) * R[1] / r};
    o_toy_S(lambda, k, a, mu, s_kind, R, S);
    int rc;
    if (scheme == 0 || scheme == 1) {
      rc = o_langevin(2, 0.0, R, Rp, Sp, f, S, T, Delta, scheme == 0 ? alpha : 0.0,
                      scheme == 1 ? O_STEP_NO_SCORR : 0u, seed, traj, (uint32_t)t);
      if (rc) return rc;
    } else if (scheme == 3) {
      double Lc[4], xi[2], z[2], Si[4], Sy[4], y[2], amp = sqrt(2.0 * T * Delta);
      if (o_cholesky(2, S, Lc)) return O_ENOTSPD;
      o_normals(seed, traj, (uint32_t)t, 2, xi);
      z[1] = xi[1] / Lc[3];
      z[0] = (xi[0] - Lc[2] * z[1]) / Lc[0];
      for (int j = 0; j < 2; ++j) y[j] = R[j] + amp * z[j];
      o_toy_S(lambda, k, a, mu, s_kind, y, Sy);
      inv2(S, Si);
      double dS[4], v[2];
      for (int q = 0; q < 4; ++q) dS[q] = Sy[q] - S[q];
      for (int j = 0; j < 2; ++j) v[j] = Delta * f[j] - 0.5 * (dS[2 * j] * (y[0] - R[0]) + dS[2 * j + 1] * (y[1] - R[1]));
      for (int j = 0; j < 2; ++j) {
        Rp[j] = R[j];
        R[j] = y[j] + Si[2 * j] * v[0] + Si[2 * j + 1] * v[1];
      }
      memcpy(Sp, S, sizeof(S));
    } else {
      double Si[4], Gam[2] = {0, 0}, h = 1e-6;
      inv2(S, Si);
      for (int i = 0; i < 2; ++i) {
        double xp[2] = {R[0], R[1]}, xm[2] = {R[0], R[1]}, Spp[4], Smm[4], Sip[4], Sim[4];
        xp[i] += h; xm[i] -= h;
        o_toy_S(lambda, k, a, mu, s_kind, xp, Spp);
        o_toy_S(lambda, k, a, mu, s_kind, xm, Smm);
        inv2(Spp, Sip); inv2(Smm, Sim);
        for (int j = 0; j < 2; ++j) Gam[j] += (Sip[2 * j + i] - Sim[2 * j + i]) / (2 * h);
      }
      double Lc[4], xi[2], z[2];
      if (o_cholesky(2, S, Lc)) return O_ENOTSPD;
      o_normals(seed, traj, (uint32_t)t, 2, xi);
      z[1] = xi[1] / Lc[3];
      z[0] = (xi[0] - Lc[2] * z[1]) / Lc[0];
      double amp = sqrt(2.0 * T * Delta);
      for (int j = 0; j < 2; ++j) {
        double dr = Delta * (Si[2 * j] * f[0] + Si[2 * j + 1] * f[1]) + T * Delta * Gam[j] + amp * z[j];
        Rp[j] = R[j];
        R[j] += dr;
      }
      memcpy(Sp, S, sizeof(S));
    }
    double rn = sqrt(R[0] * R[0] + R[1] * R[1]);
    double U = 0.5 * k * (rn - a) * (rn - a);
    if (U_samples) U_samples[t] = U;
    if (t >= burn) { acc += U; ++cnt; }
  }
  *U_mean = acc / (cnt > 0 ? cnt : 1);
  return 0;
}
