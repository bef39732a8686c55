/* Plain FP64 CPU oracle for general (complex) twisted boundary conditions -- see
 * vmc_oracle.h.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU baseline leg of
 * the benchmark; never by the product path.
 *
 * The SI's basis obeys phi(r + n L) = e^{i theta.n} phi(r) for a twist vector theta, and its
 * estimates are averaged over a 4 x 4 x 4 Monkhorst-Pack mesh of twists.  With a twist the
 * periodic Gaussian is the Bloch sum
 *     phi_a(r) = sum_n e^{-i theta.n} exp(-zeta_a |r - R_a + n L|^2),
 * which factorises over the axes; the orbitals, Slater matrices and determinants are complex
 * and |psi|^2 = |D_up|^2 |D_dn|^2 e^{2U}.  The local energy is complex; its real part is the
 * estimator (the imaginary part integrates to zero against |psi|^2), so
 *     E = <Re E_L>,  f = -<d Re E_L / dR> - 2 <(Re E_L - E) d ln|psi| / dR>.
 * Readings: the Jastrow factor (two-body, and optionally the one-body and on-site three-body
 * terms) and the Coulomb part are the untwisted ones (they depend on distances only; the proton
 * derivatives of the one- and three-body terms couple to the real part of grad ln D); both spins
 * use the same twist and orbitals (the SI's opposite twists for
 * opposite spins would conjugate D_dn, which leaves |psi|^2, Re E_L and both force terms
 * unchanged).  Images |n| <= 1 per axis, as in the real oracle.  The SI's contracted orbital
 * phi_1 + eta phi_2 is Bloch-summed factor by factor like the single Gaussian (o_cbasis), its
 * overlaps are the real contracted overlaps' axis moments with Bloch weights.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "vmc_oracle.h"

#define O_EINVAL (-1)
#define O_ESINGULAR (-4)

typedef double complex cplx;
static const double CPI = 3.14159265358979323846;

/* One Cartesian factor of the Bloch-summed Gaussian and its first three derivatives at the
 * raw offset d (any real value): with d = x + k L, x the minimum image, the sum at d is
 * e^{i theta k} times the sum at x over the images n = -1, 0, 1. */
static void cgauss_1d(double d, double zeta, double L, double theta, cplx g[4]) {
  const double k = floor(d / L + 0.5);
  const double x = d - k * L;
  g[0] = g[1] = g[2] = g[3] = 0.0;
  for (int n = -1; n <= 1; ++n) {
    const double t = x + n * L;
    const cplx e = cexp(-I * theta * n) * exp(-zeta * t * t);
    g[0] += e;
    g[1] += -2.0 * zeta * t * e;
    g[2] += (4.0 * zeta * zeta * t * t - 2.0 * zeta) * e;
    g[3] += (-8.0 * zeta * zeta * zeta * t * t * t + 12.0 * zeta * zeta * t) * e;
  }
  const cplx ph = cexp(I * theta * k);
  for (int q = 0; q < 4; ++q) g[q] *= ph;
}

/* The contracted orbital's factors on one axis (SI, basis section): the Bloch sums of
 * e^{-z t^2} (g) and of t^2 e^{-z t^2} (h) with their first three derivatives at the raw offset
 * d, images n = -1, 0, 1 at the minimum image x weighted e^{-i theta n}, times e^{i theta k}.
 * With e = e^{-z t^2}: h' = (2 t - 2 z t^3) e, h'' = (2 - 10 z t^2 + 4 z^2 t^4) e,
 * h''' = (-24 z t + 36 z^2 t^3 - 8 z^3 t^5) e. */
static void cgauss2_1d(double d, double z, double L, double theta, cplx g[4], cplx h[4]) {
  const double k = floor(d / L + 0.5);
  const double x = d - k * L;
  for (int q = 0; q < 4; ++q) g[q] = h[q] = 0.0;
  for (int n = -1; n <= 1; ++n) {
    const double t = x + n * L, t2 = t * t;
    const cplx e = cexp(-I * theta * n) * exp(-z * t2);
    g[0] += e;
    g[1] += -2.0 * z * t * e;
    g[2] += (4.0 * z * z * t2 - 2.0 * z) * e;
    g[3] += (-8.0 * z * z * z * t2 * t + 12.0 * z * z * t) * e;
    h[0] += t2 * e;
    h[1] += (2.0 * t - 2.0 * z * t2 * t) * e;
    h[2] += (2.0 - 10.0 * z * t2 + 4.0 * z * z * t2 * t2) * e;
    h[3] += (-24.0 * z * t + 36.0 * z * z * t2 * t - 8.0 * z * z * z * t2 * t2 * t) * e;
  }
  const cplx ph = cexp(I * theta * k);
  for (int q = 0; q < 4; ++q) { g[q] *= ph; h[q] *= ph; }
}

/* Adds w times the 14 components [value, grad(3), lap, hess xx yy zz xy xz yz, grad lap(3)] of
 * the product f[0](x) f[1](y) f[2](z) of Cartesian factors (f[m][q]: q-th derivative). */
static void cprod14(const cplx f[3][4], cplx w, cplx v[14]) {
  v[0] += w * f[0][0] * f[1][0] * f[2][0];
  v[1] += w * f[0][1] * f[1][0] * f[2][0];
  v[2] += w * f[0][0] * f[1][1] * f[2][0];
  v[3] += w * f[0][0] * f[1][0] * f[2][1];
  v[4] += w * (f[0][2] * f[1][0] * f[2][0] + f[0][0] * f[1][2] * f[2][0] + f[0][0] * f[1][0] * f[2][2]);
  v[5] += w * f[0][2] * f[1][0] * f[2][0];
  v[6] += w * f[0][0] * f[1][2] * f[2][0];
  v[7] += w * f[0][0] * f[1][0] * f[2][2];
  v[8] += w * f[0][1] * f[1][1] * f[2][0];
  v[9] += w * f[0][1] * f[1][0] * f[2][1];
  v[10] += w * f[0][0] * f[1][1] * f[2][1];
  v[11] += w * (f[0][3] * f[1][0] * f[2][0] + f[0][1] * f[1][2] * f[2][0] + f[0][1] * f[1][0] * f[2][2]);
  v[12] += w * (f[0][2] * f[1][1] * f[2][0] + f[0][0] * f[1][3] * f[2][0] + f[0][0] * f[1][1] * f[2][2]);
  v[13] += w * (f[0][2] * f[1][0] * f[2][1] + f[0][0] * f[1][2] * f[2][1] + f[0][0] * f[1][0] * f[2][3]);
}

/* Basis function a at r: out = [phi, grad(3), lap, hess xx yy zz xy xz yz, grad lap (3)],
 * complex, as 28 doubles (real, imaginary) in that order. */
void o_cbasis(const osys* s, const double theta[3], int a, const double r[3], double out[28]) {
  const double* Ra = s->R + 3 * a;
  cplx v[14];
  if (s->contracted) {
    /* phi_1 + eta phi_2 = g1 g1 g1 + eta (h2 g2 g2 + g2 h2 g2 + g2 g2 h2), exponents Z1 and Z2 */
    cplx g1[3][4], g2[3][4], h2[3][4];
    for (int m = 0; m < 3; ++m) {
      cplx hd[4];
      cgauss2_1d(r[m] - Ra[m], O_Z1, s->L, theta[m], g1[m], hd);
      cgauss2_1d(r[m] - Ra[m], O_Z2, s->L, theta[m], g2[m], h2[m]);
    }
    for (int q = 0; q < 14; ++q) v[q] = 0.0;
    cprod14(g1, 1.0, v);
    for (int m = 0; m < 3; ++m) {
      cplx f[3][4];
      for (int mm = 0; mm < 3; ++mm)
        for (int q = 0; q < 4; ++q) f[mm][q] = (mm == m) ? h2[mm][q] : g2[mm][q];
      cprod14(f, s->eta, v);
    }
    for (int q = 0; q < 14; ++q) { out[2 * q] = creal(v[q]); out[2 * q + 1] = cimag(v[q]); }
    return;
  }
  cplx g[3][4];
  for (int m = 0; m < 3; ++m) cgauss_1d(r[m] - Ra[m], s->zeta[a], s->L, theta[m], g[m]);
  v[0] = g[0][0] * g[1][0] * g[2][0];
  v[1] = g[0][1] * g[1][0] * g[2][0];
  v[2] = g[0][0] * g[1][1] * g[2][0];
  v[3] = g[0][0] * g[1][0] * g[2][1];
  v[4] = g[0][2] * g[1][0] * g[2][0] + g[0][0] * g[1][2] * g[2][0] + g[0][0] * g[1][0] * g[2][2];
  v[5] = g[0][2] * g[1][0] * g[2][0];
  v[6] = g[0][0] * g[1][2] * g[2][0];
  v[7] = g[0][0] * g[1][0] * g[2][2];
  v[8] = g[0][1] * g[1][1] * g[2][0];
  v[9] = g[0][1] * g[1][0] * g[2][1];
  v[10] = g[0][0] * g[1][1] * g[2][1];
  v[11] = g[0][3] * g[1][0] * g[2][0] + g[0][1] * g[1][2] * g[2][0] + g[0][1] * g[1][0] * g[2][2];
  v[12] = g[0][2] * g[1][1] * g[2][0] + g[0][0] * g[1][3] * g[2][0] + g[0][0] * g[1][1] * g[2][2];
  v[13] = g[0][2] * g[1][0] * g[2][1] + g[0][0] * g[1][2] * g[2][1] + g[0][0] * g[1][0] * g[2][3];
  for (int q = 0; q < 14; ++q) { out[2 * q] = creal(v[q]); out[2 * q + 1] = cimag(v[q]); }
}

/* Values of every basis function at npt points (out: npt x n_p complex as pairs). */
void o_cbasis_values(const osys* s, const double theta[3], int npt, const double* pts, double* out) {
  for (int p = 0; p < npt; ++p)
    for (int a = 0; a < s->n_p; ++a) {
      double f[28];
      o_cbasis(s, theta, a, pts + 3 * p, f);
      out[2 * ((size_t)p * s->n_p + a)] = f[0];
      out[2 * ((size_t)p * s->n_p + a) + 1] = f[1];
    }
}

/* Overlap of two Bloch sums over the cell: one image sum of the free-space overlaps,
 * S_ab = (pi/(za+zb))^{3/2} sum_p e^{-i theta.p} e^{-mu |R_a - R_b + p L|^2},
 * mu = za zb/(za+zb), per axis p = -4..4.  Hermitian. */
void o_coverlap(int n_p, double L, const double theta[3], const double* R, const double* zeta, double* S_out) {
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) {
      const double za = zeta[a], zb = zeta[b], mu = za * zb / (za + zb);
      cplx v = pow(CPI / (za + zb), 1.5);
      for (int m = 0; m < 3; ++m) {
        const double d = R[3 * a + m] - R[3 * b + m];
        cplx acc = 0.0;
        for (int p = -4; p <= 4; ++p) acc += cexp(-I * theta[m] * p) * exp(-mu * (d + p * L) * (d + p * L));
        v *= acc;
      }
      S_out[2 * (a * n_p + b)] = creal(v);
      S_out[2 * (a * n_p + b) + 1] = cimag(v);
    }
}

/* One axis of the contracted overlap: moments of the free-space product of e^{-al (x - A)^2} and
 * e^{-be (x - B)^2} over the images of the second centre at d + n L (d = B - A), n = -4..4, each
 * weighted e^{i theta n} (the Bloch sum of the second factor): out = [<1>, <(x-A)^2>, <(x-B)^2>,
 * <(x-A)^2 (x-B)^2>] with the product centred at (al A + be B)/p, P = be dn/p, Q = al dn/p. */
static void cmoments_1d(double al, double be, double d, double L, double theta, cplx out[4]) {
  const double p = al + be, mu = al * be / p;
  const double m0 = sqrt(CPI / p), m2 = m0 / (2.0 * p), m4 = 3.0 * m0 / (4.0 * p * p);
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int n = -4; n <= 4; ++n) {
    const double dd = d + n * L;
    const cplx e = cexp(I * theta * n) * exp(-mu * dd * dd);
    const double P = be * dd / p, Q = al * dd / p;
    out[0] += e * m0;
    out[1] += e * (m2 + P * P * m0);
    out[2] += e * (m2 + Q * Q * m0);
    out[3] += e * (m4 + ((P - Q) * (P - Q) - 2.0 * P * Q) * m2 + P * P * Q * Q * m0);
  }
}

/* Overlaps of the contracted Bloch orbitals over the cell (Hermitian): the same term-by-term
 * product of axis moments as the real contracted basis, each axis an image sum with Bloch
 * weights (S_out: n_p x n_p complex as pairs). */
void o_coverlap_contracted(int n_p, double L, const double theta[3], const double* R, double eta, double* S_out) {
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) {
      cplx m11[3][4], m12[3][4], m21[3][4], m22[3][4];
      for (int m = 0; m < 3; ++m) {
        const double d = R[3 * b + m] - R[3 * a + m];
        cmoments_1d(O_Z1, O_Z1, d, L, theta[m], m11[m]);
        cmoments_1d(O_Z1, O_Z2, d, L, theta[m], m12[m]);
        cmoments_1d(O_Z2, O_Z1, d, L, theta[m], m21[m]);
        cmoments_1d(O_Z2, O_Z2, d, L, theta[m], m22[m]);
      }
      const cplx s11 = m11[0][0] * m11[1][0] * m11[2][0];
      cplx s12 = 0.0, s21 = 0.0, s22 = 0.0;
      for (int m = 0; m < 3; ++m) {
        cplx p12 = m12[m][2], p21 = m21[m][1], p22 = m22[m][3];
        for (int q = 0; q < 3; ++q)
          if (q != m) { p12 *= m12[q][0]; p21 *= m21[q][0]; p22 *= m22[q][0]; }
        s12 += p12;
        s21 += p21;
        s22 += p22;
        for (int m2 = 0; m2 < 3; ++m2) {
          if (m2 == m) continue;
          cplx pc = m22[m][1] * m22[m2][2];
          for (int q = 0; q < 3; ++q)
            if (q != m && q != m2) pc *= m22[q][0];
          s22 += pc;
        }
      }
      const cplx v = s11 + eta * (s12 + s21) + eta * eta * s22;
      S_out[2 * (a * n_p + b)] = creal(v);
      S_out[2 * (a * n_p + b) + 1] = cimag(v);
    }
}

/* Cyclic Jacobi for a Hermitian matrix (in place): each step zeroes A[p][q] by the unitary
 * rotation that first takes the phase of A[p][q] out and then a real Jacobi rotation;
 * eigenvectors are the columns of V. */
static void cjacobi_eigen(int n, cplx* A, cplx* V) {
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double m2 = creal(A[i * n + j] * conj(A[i * n + j]));
        tot += m2;
        if (i != j) off += m2;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cplx apq = A[p * n + q];
        const double r = cabs(apq);
        if (r == 0.0) continue;
        const cplx ph = apq / r;                       /* A[p][q] = r e^{i phi} */
        const double app = creal(A[p * n + p]), aqq = creal(A[q * n + q]);
        const double th = (aqq - app) / (2.0 * r);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        /* columns: a_p' = c a_p - s conj(ph) a_q ... with the unitary J = [[c, s ph], [-s conj(ph), c]] */
        for (int k = 0; k < n; ++k) {
          const cplx akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * conj(ph) * akq;
          A[k * n + q] = sn * ph * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const cplx apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * ph * aqk;
          A[q * n + k] = sn * conj(ph) * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const cplx vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * conj(ph) * vkq;
          V[k * n + q] = sn * ph * vkp + c * vkq;
        }
      }
  }
}

/* Hueckel orbitals of the twisted basis: H = -S~ with S~_ab = S_ab / sqrt(S_aa S_bb), the n_orb
 * lowest eigenvectors v of the Hermitian H, C_ak = v_ak / sqrt(S_aa) (complex, as pairs). */
static int chuckel_from_overlap(int n_p, double* Sd, int n_orb, double* C, double* evals);
int o_chuckel(int n_p, double L, const double theta[3], const double* R, const double* zeta, int n_orb, double* C,
              double* evals) {
  if (n_orb > n_p || n_orb < 0) return O_EINVAL;
  double* Sd = malloc(sizeof(double) * 2 * n_p * n_p);
  o_coverlap(n_p, L, theta, R, zeta, Sd);
  return chuckel_from_overlap(n_p, Sd, n_orb, C, evals);
}

/* The same on the contracted basis. */
int o_chuckel_contracted(int n_p, double L, const double theta[3], const double* R, double eta, int n_orb, double* C,
                         double* evals) {
  if (n_orb > n_p || n_orb < 0) return O_EINVAL;
  double* Sd = malloc(sizeof(double) * 2 * n_p * n_p);
  o_coverlap_contracted(n_p, L, theta, R, eta, Sd);
  return chuckel_from_overlap(n_p, Sd, n_orb, C, evals);
}

/* Hueckel orbitals from the overlap Sd (complex pairs; freed here). */
static int chuckel_from_overlap(int n_p, double* Sd, int n_orb, double* C, double* evals) {
  cplx* H = malloc(sizeof(cplx) * n_p * n_p);
  cplx* V = malloc(sizeof(cplx) * n_p * n_p);
  for (int a = 0; a < n_p; ++a)
    for (int b = 0; b < n_p; ++b) {
      const cplx sab = Sd[2 * (a * n_p + b)] + I * Sd[2 * (a * n_p + b) + 1];
      H[a * n_p + b] = -sab / sqrt(Sd[2 * (a * n_p + a)] * Sd[2 * (b * n_p + b)]);
    }
  cjacobi_eigen(n_p, H, V);
  int* order = malloc(sizeof(int) * n_p);
  for (int i = 0; i < n_p; ++i) order[i] = i;
  for (int i = 1; i < n_p; ++i) {
    int t = order[i], j = i - 1;
    while (j >= 0 && creal(H[order[j] * n_p + order[j]]) > creal(H[t * n_p + t])) { order[j + 1] = order[j]; --j; }
    order[j + 1] = t;
  }
  for (int k = 0; k < n_orb; ++k)
    for (int a = 0; a < n_p; ++a) {
      const cplx c = V[a * n_p + order[k]] / sqrt(Sd[2 * (a * n_p + a)]);
      C[2 * (a * n_orb + k)] = creal(c);
      C[2 * (a * n_orb + k) + 1] = cimag(c);
    }
  if (evals)
    for (int k = 0; k < n_p; ++k) evals[k] = creal(H[order[k] * n_p + order[k]]);
  free(Sd); free(H); free(V); free(order);
  return 0;
}

/* LU with partial pivoting (by modulus) of a copy of the complex n x n matrix M: ln|det|,
 * the phase of det, and optionally the inverse.  O_ESINGULAR on an exactly zero pivot. */
static int clu(int n, const cplx* M, double* logdet, double* phase, cplx* inv) {
  cplx* a = malloc(sizeof(cplx) * n * n);
  int* piv = malloc(sizeof(int) * n);
  memcpy(a, M, sizeof(cplx) * n * n);
  double ld = 0.0, ph = 0.0;
  int rc = 0;
  for (int p = 0; p < n; ++p) {
    int best = p;
    for (int r = p + 1; r < n; ++r)
      if (cabs(a[r * n + p]) > cabs(a[best * n + p])) best = r;
    piv[p] = best;
    if (a[best * n + p] == 0.0) { rc = O_ESINGULAR; break; }
    if (best != p) {
      for (int c = 0; c < n; ++c) { cplx t = a[p * n + c]; a[p * n + c] = a[best * n + c]; a[best * n + c] = t; }
      ph += CPI;
    }
    const cplx d = a[p * n + p];
    ld += log(cabs(d));
    ph += carg(d);
    for (int r = p + 1; r < n; ++r) {
      const cplx l = a[r * n + p] / d;
      a[r * n + p] = l;
      for (int c = p + 1; c < n; ++c) a[r * n + c] -= l * a[p * n + c];
    }
  }
  if (rc == 0 && inv) {
    cplx* col = malloc(sizeof(cplx) * n);
    for (int j = 0; j < n; ++j) {
      for (int r = 0; r < n; ++r) col[r] = (r == j) ? 1.0 : 0.0;
      for (int p = 0; p < n; ++p) { cplx t = col[p]; col[p] = col[piv[p]]; col[piv[p]] = t; }
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < r; ++c) col[r] -= a[r * n + c] * col[c];
      for (int r = n - 1; r >= 0; --r) {
        for (int c = r + 1; c < n; ++c) col[r] -= a[r * n + c] * col[c];
        col[r] /= a[r * n + r];
      }
      for (int r = 0; r < n; ++r) inv[r * n + j] = col[r];
    }
    free(col);
  }
  *logdet = rc ? -INFINITY : ld;
  *phase = rc ? 0.0 : remainder(ph, 2.0 * CPI);
  free(a);
  free(piv);
  return rc;
}

static int chidx(int m, int n) {
  if (m == n) return 5 + m;
  if (m > n) { int t = m; m = n; n = t; }
  return (m == 0) ? (n == 1 ? 8 : 9) : 10;
}

static void cmatmul(int n, const cplx* A, const cplx* B, cplx* C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cplx s = 0.0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}

/* Local quantities of the complex-twisted wavefunction at electron configuration x:
 * ln|psi|, arg psi, Re E_L and the proton derivatives of ln|psi| and of Re E_L (by Jacobi's
 * formula, d A^-1 = -A^-1 dA A^-1, as in the real oracle).  C: n_p x n_orb complex pairs.
 * The one-body and three-body Jastrow terms are real and enter as in the real oracle, their proton
 * derivatives coupling to the real part of grad ln D (o_jastrow_dR).  Single Gaussians only. */
int o_clocal(const osys* s, const double theta[3], const double* Cd, const double* x, double* lnpsi, double* phase,
             double* EL, double* dlnpsi_dR, double* dEL_dR) {
  if (s->basis_kind != OB_PERIODIC_GAUSS) return O_EINVAL;
  const int np = s->n_p, ne = s->n_up + s->n_dn, no = s->n_orb, n3 = 3 * np;
  double U;
  double* gU = malloc(sizeof(double) * 3 * ne);
  double* lU = malloc(sizeof(double) * ne);
  o_jastrow(s, x, &U, gU, lU);
  double* dVdR = malloc(sizeof(double) * n3);
  const double V = o_potential(s, x, dVdR, NULL);
  double T = 0.0, lnp = U, ph = 0.0;
  for (int e = 0; e < ne; ++e)
    T += -0.5 * (lU[e] + gU[3 * e] * gU[3 * e] + gU[3 * e + 1] * gU[3 * e + 1] + gU[3 * e + 2] * gU[3 * e + 2]);
  const int want = (dlnpsi_dR != NULL) || (dEL_dR != NULL);
  double* dln = calloc(n3, sizeof(double));
  double* dT = calloc(n3, sizeof(double));
  double* vv = malloc(sizeof(double) * 3 * ne);   /* grad_i U + Re grad_i ln D */
  memcpy(vv, gU, sizeof(double) * 3 * ne);
  int rc = 0;
  for (int sp = 0; sp < 2 && rc == 0; ++sp) {
    const int n = sp ? s->n_dn : s->n_up, e0 = sp ? s->n_up : 0;
    if (n == 0) continue;
    double* bf = malloc(sizeof(double) * 28 * n * np);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < np; ++a) o_cbasis(s, theta, a, x + 3 * (e0 + i), bf + 28 * (i * np + a));
#define BF(i, a, q) (bf[28 * ((i) * np + (a)) + 2 * (q)] + I * bf[28 * ((i) * np + (a)) + 2 * (q) + 1])
#define CC(a, k) (Cd[2 * ((a) * no + (k))] + I * Cd[2 * ((a) * no + (k)) + 1])
    cplx *A = calloc(n * n, sizeof(cplx)), *G = calloc(3 * n * n, sizeof(cplx)), *Lp = calloc(n * n, sizeof(cplx));
    cplx* Ai = malloc(sizeof(cplx) * n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k)
        for (int a = 0; a < np; ++a) {
          const cplx c = CC(a, k);
          A[i * n + k] += BF(i, a, 0) * c;
          for (int m = 0; m < 3; ++m) G[(m * n + i) * n + k] += BF(i, a, 1 + m) * c;
          Lp[i * n + k] += BF(i, a, 4) * c;
        }
    double ld, dph;
    rc = clu(n, A, &ld, &dph, Ai);
    if (rc) { free(bf); free(A); free(G); free(Lp); free(Ai); break; }
    lnp += ld;
    ph += dph;
    for (int i = 0; i < n; ++i) {
      cplx lapD = 0.0, gD[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < n; ++k) {
        lapD += Lp[i * n + k] * Ai[k * n + i];
        for (int m = 0; m < 3; ++m) gD[m] += G[(m * n + i) * n + k] * Ai[k * n + i];
      }
      const double* gu = gU + 3 * (e0 + i);
      T += -0.5 * creal(lapD + 2.0 * (gD[0] * gu[0] + gD[1] * gu[1] + gD[2] * gu[2]));
      for (int m = 0; m < 3; ++m) vv[3 * (e0 + i) + m] += creal(gD[m]);
    }
    if (want) {
      cplx *dA = malloc(sizeof(cplx) * n * n), *dG = malloc(sizeof(cplx) * 3 * n * n), *dL = malloc(sizeof(cplx) * n * n);
      cplx *tmp = malloc(sizeof(cplx) * n * n), *dAi = malloc(sizeof(cplx) * n * n);
      for (int b = 0; b < np; ++b)
        for (int mu = 0; mu < 3; ++mu) {
          /* d/dR_b acts only on phi_b(r - R_b): d phi_b / dR_b,mu = -d_mu phi_b */
          for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
              const cplx c = CC(b, k);
              dA[i * n + k] = -BF(i, b, 1 + mu) * c;
              for (int nu = 0; nu < 3; ++nu) dG[(nu * n + i) * n + k] = -BF(i, b, chidx(mu, nu)) * c;
              dL[i * n + k] = -BF(i, b, 11 + mu) * c;
            }
          cmatmul(n, Ai, dA, tmp);
          cmatmul(n, tmp, Ai, dAi);
          for (int t = 0; t < n * n; ++t) dAi[t] = -dAi[t];
          cplx tr = 0.0;
          for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) tr += Ai[k * n + i] * dA[i * n + k];
          dln[3 * b + mu] += creal(tr);
          cplx dt = 0.0;
          for (int i = 0; i < n; ++i) {
            cplx dlap = 0.0, dgD[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < n; ++k) {
              dlap += dL[i * n + k] * Ai[k * n + i] + Lp[i * n + k] * dAi[k * n + i];
              for (int nu = 0; nu < 3; ++nu)
                dgD[nu] += dG[(nu * n + i) * n + k] * Ai[k * n + i] + G[(nu * n + i) * n + k] * dAi[k * n + i];
            }
            const double* gu = gU + 3 * (e0 + i);
            dt += -0.5 * (dlap + 2.0 * (dgD[0] * gu[0] + dgD[1] * gu[1] + dgD[2] * gu[2]));
          }
          dT[3 * b + mu] += creal(dt);
        }
      free(dA); free(dG); free(dL); free(tmp); free(dAi);
    }
#undef BF
#undef CC
    free(bf); free(A); free(G); free(Lp); free(Ai);
  }
  if (rc == 0 && want) o_jastrow_dR(s, x, vv, dln, dT);
  if (rc == 0) {
    if (lnpsi) *lnpsi = lnp;
    if (phase) *phase = remainder(ph, 2.0 * CPI);
    if (EL) *EL = T + V;
    if (dlnpsi_dR) memcpy(dlnpsi_dR, dln, sizeof(double) * n3);
    if (dEL_dR)
      for (int t = 0; t < n3; ++t) dEL_dR[t] = dT[t] + dVdR[t];
  }
  free(gU); free(lU); free(dVdR); free(dln); free(dT); free(vv);
  return rc;
}

/* Complex MO row m_k = sum_a phi_a(r) C_ak. */
static void cmo_row(const osys* s, const double theta[3], const double* Cd, const double r[3], cplx* m) {
  const int no = s->n_orb;
  for (int k = 0; k < no; ++k) m[k] = 0.0;
  for (int a = 0; a < s->n_p; ++a) {
    double f[28];
    o_cbasis(s, theta, a, r, f);
    const cplx p = f[0] + I * f[1];
    for (int k = 0; k < no; ++k) m[k] += p * (Cd[2 * (a * no + k)] + I * Cd[2 * (a * no + k) + 1]);
  }
}

/* The Metropolis chains of o_vmc_run_from with the complex-twisted wavefunction: the same
 * moves, random numbers and acceptance rule u < |psi'/psi|^2, the determinant ratio from two
 * fresh complex LU factorisations, the measurement by o_clocal. */
int o_cvmc_run_from(const osys* s, const double theta[3], const double* Cd, int W, uint32_t w0, double* x,
                    int n_equil, int n_meas, double delta, uint32_t seed, uint32_t traj, uint32_t step, double* sums,
                    int64_t* n_acc, int n_threads) {

  const int ne = s->n_up + s->n_dn, n3 = 3 * s->n_p, nsum = 2 + 3 * n3;
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int w = 0; w < W; ++w) {
    double* xw = x + (size_t)w * 3 * ne;
    double* sw = sums + (size_t)w * nsum;
    memset(sw, 0, sizeof(double) * nsum);
    int64_t acc = 0;
    cplx* Asp[2];
    double ld[2] = {0, 0}, phs[2] = {0, 0};
    const int nsp[2] = {s->n_up, s->n_dn};
    cplx* m = malloc(sizeof(cplx) * (s->n_orb + 1));
    for (int sp = 0; sp < 2; ++sp) {
      const int n = nsp[sp], e0 = sp ? s->n_up : 0;
      Asp[sp] = malloc(sizeof(cplx) * (n > 0 ? n * n : 1));
      for (int i = 0; i < n; ++i) {
        cmo_row(s, theta, Cd, xw + 3 * (e0 + i), m);
        memcpy(Asp[sp] + i * n, m, sizeof(cplx) * n);
      }
      if (n > 0 && clu(n, Asp[sp], &ld[sp], &phs[sp], NULL)) err = O_ESINGULAR;
    }
    cplx* Anew = malloc(sizeof(cplx) * (ne * ne + 1));
    double* dE = malloc(sizeof(double) * n3);
    double* dg = malloc(sizeof(double) * n3);
    const uint32_t key[2] = {seed, traj};
    for (int sw_i = 0; sw_i < n_equil + n_meas; ++sw_i) {
      for (int e = 0; e < ne; ++e) {
        uint32_t c0[4] = {step, w0 + (uint32_t)w, (uint32_t)(sw_i * ne + e), 0u}, o0[4], o1[4];
        uint32_t c1[4] = {step, w0 + (uint32_t)w, (uint32_t)(sw_i * ne + e), 1u};
        o_philox(c0, key, o0);
        o_philox(c1, key, o1);
        const double u[3] = {o_u01(o0[0], o0[1]), o_u01(o0[2], o0[3]), o_u01(o1[0], o1[1])};
        const double uacc = o_u01(o1[2], o1[3]);
        double rn[3];
        for (int mm = 0; mm < 3; ++mm) {
          rn[mm] = xw[3 * e + mm] + delta * (u[mm] - 0.5);
          rn[mm] -= s->L * floor(rn[mm] / s->L);
        }
        const int sp = e < s->n_up ? 0 : 1, n = nsp[sp], i = e - (sp ? s->n_up : 0);
        cmo_row(s, theta, Cd, rn, m);
        memcpy(Anew, Asp[sp], sizeof(cplx) * n * n);
        memcpy(Anew + i * n, m, sizeof(cplx) * n);
        double ldn, phn;
        double q2 = 0.0;
        if (clu(n, Anew, &ldn, &phn, NULL) == 0) q2 = exp(2.0 * (ldn - ld[sp]));
        double dU = 0.0;
        if (s->jastrow_on) {
          /* the Jastrow change of the move, from the whole-configuration Jastrow before and after */
          double U0, U1;
          double* gtmp = malloc(sizeof(double) * 3 * ne);
          double* ltmp = malloc(sizeof(double) * ne);
          o_jastrow(s, xw, &U0, gtmp, ltmp);
          double keep[3] = {xw[3 * e], xw[3 * e + 1], xw[3 * e + 2]};
          memcpy(xw + 3 * e, rn, sizeof keep);
          o_jastrow(s, xw, &U1, gtmp, ltmp);
          memcpy(xw + 3 * e, keep, sizeof keep);
          dU = U1 - U0;
          free(gtmp);
          free(ltmp);
        }
        const double p = q2 * exp(2.0 * dU);
        if (uacc < p) {
          memcpy(xw + 3 * e, rn, 3 * sizeof(double));
          memcpy(Asp[sp], Anew, sizeof(cplx) * n * n);
          ld[sp] = ldn;
          phs[sp] = phn;
          ++acc;
        }
      }
      if (sw_i >= n_equil) {
        double el;
        if (o_clocal(s, theta, Cd, xw, NULL, NULL, &el, dg, dE)) { err = O_ESINGULAR; continue; }
        sw[0] += el;
        sw[1] += el * el;
        for (int t = 0; t < n3; ++t) {
          sw[2 + t] += dE[t];
          sw[2 + n3 + t] += dg[t];
          sw[2 + 2 * n3 + t] += el * dg[t];
        }
      }
    }
    if (n_acc) n_acc[w] = acc;
    free(Asp[0]); free(Asp[1]); free(Anew); free(m); free(dE); free(dg);
  }
  return err;
}
