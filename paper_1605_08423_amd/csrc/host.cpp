// Host-only parts of the library (see host.hpp): reciprocal vectors, the admission rule,
// the Hueckel eigen-solver and the checkpoint format.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

namespace vmc_host {

// Half-space reciprocal vectors grouped by (ny, nz), nx innermost.
// Half-space k = 2 pi n / L, 0 < |n|^2 <= nmax^2, grouped in (ny, nz) slots with nx
// innermost; the slot list is sorted by nx range (longest first, stable) so that
// the reciprocal-space lanes of a wave get slots of about equal length.
void build_kvectors(const vmc_system& s, std::vector<double>& kv, std::vector<int>& slots_out,
                    std::vector<int>& nx0_out) {
  const int nm = s.ewald_nmax;
  const double L = s.box_L, V = L * L * L, kap = s.ewald_kappa, tp = 2.0 * M_PI / L;
  std::vector<int> slots, nx0;
  int k = 0;
  for (int ny = -nm; ny <= nm; ++ny)
    for (int nz = -nm; nz <= nm; ++nz) {
      const int r2 = ny * ny + nz * nz;
      if (r2 > nm * nm) continue;
      int nxmax = 0;
      while ((nxmax + 1) * (nxmax + 1) + r2 <= nm * nm) ++nxmax;
      const bool pos_half = (ny > 0) || (ny == 0 && nz > 0);
      const int nxmin = pos_half ? 0 : 1;
      if (nxmin > nxmax) continue;
      slots.push_back(ny);
      slots.push_back(nz);
      slots.push_back(k);
      slots.push_back(nxmax - nxmin + 1);
      nx0.push_back(nxmin);
      for (int nx = nxmin; nx <= nxmax; ++nx, ++k) {
        const double kx = tp * nx, ky = tp * ny, kz = tp * nz, k2 = kx * kx + ky * ky + kz * kz;
        kv.push_back(kx);
        kv.push_back(ky);
        kv.push_back(kz);
        kv.push_back(4.0 * M_PI / V * std::exp(-k2 / (4.0 * kap * kap)) / k2);
      }
    }
  std::vector<int> order(nx0.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return nx0[x] + slots[4 * x + 3] > nx0[y] + slots[4 * y + 3];
  });
  slots_out.clear();
  nx0_out.clear();
  for (int q : order) {
    for (int c = 0; c < 4; ++c) slots_out.push_back(slots[4 * q + c]);
    nx0_out.push_back(nx0[q]);
  }
}

int admit_count(size_t budget, size_t resident, int n, const size_t* bytes) {
  int k = 0;
  for (; k < n; ++k) {
    if (bytes[k] > budget || resident > budget - bytes[k]) break;
    resident += bytes[k];
  }
  return k;
}

// ------------------------------------------------------------ checkpoint --
static constexpr char kCkptMagic[8] = {'V', 'M', 'C', 'T', 'R', 'A', 'J', '2'};

size_t ckpt_payload_bytes(int n, int w) {
  const size_t W = (size_t)w, N = (size_t)n, n3 = 3 * N;
  return sizeof(double) * (W * N * 3 + W * (1 + 9 * N) + W * n3 + (3 + n3) + 2 * n3 + 2 * n3 * n3) +
         sizeof(int64_t) * W;
}

void ckpt_init_header(CkptHeader* h, int n, int w) {
  std::memset(h, 0, sizeof *h);
  std::memcpy(h->magic, kCkptMagic, 8);
  h->version = kCkptVersion;
  h->n = n;
  h->w = w;
  h->payload_bytes = ckpt_payload_bytes(n, w);
}

// FNV-1a, 64 bit (Fowler, Noll, Vo): h = (h xor byte) * 1099511628211 from the offset basis.
static uint64_t fnv1a(uint64_t h, const unsigned char* p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

static uint64_t ckpt_checksum(const unsigned char* buf, size_t payload) {
  CkptHeader h;
  std::memcpy(&h, buf, sizeof h);
  h.checksum = 0;
  uint64_t c = fnv1a(14695981039346656037ull, reinterpret_cast<const unsigned char*>(&h), sizeof h);
  return fnv1a(c, buf + sizeof h, payload);
}

void ckpt_seal(void* buf) {
  unsigned char* p = static_cast<unsigned char*>(buf);
  CkptHeader h;
  std::memcpy(&h, p, sizeof h);
  h.checksum = ckpt_checksum(p, h.payload_bytes);
  std::memcpy(p, &h, sizeof h);
}

int ckpt_validate(const void* buf, size_t len, CkptHeader* out) {
  if (!buf || len < sizeof(CkptHeader)) return VMC_EINVAL;
  const unsigned char* p = static_cast<const unsigned char*>(buf);
  CkptHeader h;
  std::memcpy(&h, p, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion) return VMC_EINVAL;
  if (h.n < 2 || h.n > 4096 || h.w < 1) return VMC_EINVAL;
  if (h.payload_bytes != ckpt_payload_bytes(h.n, h.w) || len - sizeof h < h.payload_bytes) return VMC_EINVAL;
  if (ckpt_checksum(p, h.payload_bytes) != h.checksum) return VMC_EINVAL;
  if (out) *out = h;
  return VMC_OK;
}

}  // namespace vmc_host

using namespace vmc_host;

// ---------------------------------------------------------------- Hueckel --
// The m lowest eigenpairs of the symmetric A (n x n, overwritten): Householder reduction to the
// tridiagonal T (the reflections kept, not accumulated), the m lowest eigenvalues of T by
// bisection on Sturm counts, each eigenvector of T by inverse iteration (T - sigma I solved by
// Gaussian elimination with partial pivoting, three iterations from a fixed start; the vectors of
// eigenvalues closer than 1e-3 |T| orthogonalised by modified Gram-Schmidt, and a shift equal to
// the previous eigenvalue moved up by 10 eps |T|), carried back through the reflections.  Only the
// occupied half of the spectrum is needed, which the full QR iteration with accumulated rotations
// paid n^3 for.  evals: m ascending values; vecs: n x m, column k belonging to evals[k].
static int lowest_eigenpairs(int n, int m, std::vector<double>& A, std::vector<double>& evals,
                             std::vector<double>& vecs) {
  std::vector<double> V((size_t)n * n, 0.0), betas(n, 0.0), v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int mm = n - k - 1, o = k + 1;
    const double x0 = A[(size_t)o * n + k];
    double sigma = 0.0;
    for (int i = 1; i < mm; ++i) sigma += A[(size_t)(o + i) * n + k] * A[(size_t)(o + i) * n + k];
    if (sigma == 0.0) continue;
    const double mu = std::sqrt(x0 * x0 + sigma);
    const double v0 = (x0 <= 0.0) ? x0 - mu : -sigma / (x0 + mu);
    const double beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    v[0] = 1.0;
    for (int i = 1; i < mm; ++i) v[i] = A[(size_t)(o + i) * n + k] / v0;
    double pv = 0.0;
    for (int i = 0; i < mm; ++i) {
      double acc = 0.0;
      for (int j = 0; j < mm; ++j) acc += A[(size_t)(o + i) * n + o + j] * v[j];
      p[i] = beta * acc;
      pv += p[i] * v[i];
    }
    for (int i = 0; i < mm; ++i) w[i] = p[i] - 0.5 * beta * pv * v[i];
    for (int i = 0; i < mm; ++i)
      for (int j = 0; j < mm; ++j) A[(size_t)(o + i) * n + o + j] -= v[i] * w[j] + w[i] * v[j];
    A[(size_t)o * n + k] = A[(size_t)k * n + o] = mu;
    for (int i = 1; i < mm; ++i) A[(size_t)(o + i) * n + k] = A[(size_t)k * n + o + i] = 0.0;
    betas[k] = beta;
    for (int i = 0; i < mm; ++i) V[(size_t)k * n + o + i] = v[i];
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
  double tn = 0.0, lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
    tn = std::max(tn, std::fabs(d[i]) + r);
  }
  const double eps = 2.220446049250313e-16, tiny = eps * (tn > 0.0 ? tn : 1.0);
  // number of eigenvalues of T below x (signs of the pivots of T - x I)
  auto below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++c;
    for (int i = 1; i < n; ++i) {
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q == 0.0) q = -tiny;
      if (q < 0.0) ++c;
    }
    return c;
  };
  evals.assign(m, 0.0);
  for (int k = 0; k < m; ++k) {
    double a = (k > 0 ? evals[k - 1] : lo) - tiny, b = hi + tiny;
    for (int it = 0; it < 200 && b - a > 2.0 * eps * std::max(std::fabs(a), std::fabs(b)) + tiny * 1e-3; ++it) {
      const double c = 0.5 * (a + b);
      if (c <= a || c >= b) break;
      if (below(c) > k) b = c; else a = c;
    }
    evals[k] = 0.5 * (a + b);
  }
  vecs.assign((size_t)n * m, 0.0);
  std::vector<double> u0(n), u1(n), u2(n), ml(n), x(n), ev((size_t)m * n);
  std::vector<char> sw(n);
  const double ortol = 1e-3 * tn;
  for (int k = 0; k < m; ++k) {
    double sig = evals[k];
    if (k > 0 && sig - evals[k - 1] < 10.0 * eps * tn) sig = evals[k - 1] + 10.0 * eps * tn;
    // T - sig I = P L U, U with two super-diagonals
    double dd = d[0] - sig, s1 = n > 1 ? e[0] : 0.0, s2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = e[i], nd = d[i + 1] - sig, ns = i + 2 < n ? e[i + 1] : 0.0;
      if (std::fabs(sub) > std::fabs(dd)) {
        sw[i] = 1;
        u0[i] = sub; u1[i] = nd; u2[i] = ns;
        const double f = dd / sub;
        ml[i] = f;
        dd = s1 - f * nd;
        s1 = s2 - f * ns;
      } else {
        sw[i] = 0;
        if (dd == 0.0) dd = tiny;
        u0[i] = dd; u1[i] = s1; u2[i] = s2;
        const double f = sub / dd;
        ml[i] = f;
        dd = nd - f * s1;
        s1 = ns - f * s2;
      }
      s2 = 0.0;
    }
    if (dd == 0.0) dd = tiny;
    u0[n - 1] = dd; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    // a fixed start with every component present
    uint64_t st = 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1);
    for (int i = 0; i < n; ++i) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      x[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i + 1 < n; ++i) {
        if (sw[i]) std::swap(x[i], x[i + 1]);
        x[i + 1] -= ml[i] * x[i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        if (i + 1 < n) s -= u1[i] * x[i + 1];
        if (i + 2 < n) s -= u2[i] * x[i + 2];
        x[i] = s / u0[i];
      }
      for (int j = k - 1; j >= 0 && evals[k] - evals[j] < ortol; --j) {
        double dp = 0.0;
        for (int i = 0; i < n; ++i) dp += ev[(size_t)j * n + i] * x[i];
        for (int i = 0; i < n; ++i) x[i] -= dp * ev[(size_t)j * n + i];
      }
      double nn = 0.0;
      for (int i = 0; i < n; ++i) nn += x[i] * x[i];
      if (!(nn > 0.0) || !std::isfinite(nn)) return VMC_ENOCONV;
      const double inv = 1.0 / std::sqrt(nn);
      for (int i = 0; i < n; ++i) x[i] *= inv;
    }
    for (int i = 0; i < n; ++i) ev[(size_t)k * n + i] = x[i];
    // back through the reflections, the last one first
    for (int r = n - 3; r >= 0; --r) {
      if (betas[r] == 0.0) continue;
      const double* vr = &V[(size_t)r * n];
      double dp = 0.0;
      for (int i = r + 1; i < n; ++i) dp += vr[i] * x[i];
      dp *= betas[r];
      for (int i = r + 1; i < n; ++i) x[i] -= dp * vr[i];
    }
    for (int i = 0; i < n; ++i) vecs[(size_t)i * m + k] = x[i];
  }
  return VMC_OK;
}

extern "C" int vmc_huckel_params(int n, double L, const double* R, const double* zeta, double* C_out) {
  return vmc_huckel_params_twist(n, L, 0, R, zeta, C_out);
}

extern "C" int vmc_huckel_params_twist(int n, double L, int twist, const double* R, const double* zeta, double* C_out) {
  if (n < 2 || (n & 1) || !(L > 0.0) || !R || !zeta || !C_out || twist < 0 || twist > 7) return VMC_EINVAL;
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(R[i])) return VMC_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(zeta[i] > 0.0) || !std::isfinite(zeta[i])) return VMC_EINVAL;
  std::vector<double> S((size_t)n * n), H((size_t)n * n), Q;
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {   // the lower triangle by symmetry
      const double za = zeta[a], zb = zeta[b], mu = za * zb / (za + zb);
      double v = std::pow(M_PI / (za + zb), 1.5);
      for (int ax = 0; ax < 3; ++ax) {
        // minimum image dd - m L; with the twist angle pi image k weighs (-1)^k and the
        // sum at the raw offset is (-1)^m times the one at the minimum image
        const double tau = ((twist >> ax) & 1) ? -1.0 : 1.0;
        double dd = R[3 * a + ax] - R[3 * b + ax];
        const double m = std::floor(dd / L + 0.5);
        dd -= L * m;
        double s = 0.0;
        for (int k = -3; k <= 3; ++k) s += ((k & 1) ? tau : 1.0) * std::exp(-mu * (dd + k * L) * (dd + k * L));
        if (((long long)m) & 1) s *= tau;
        v *= s;
      }
      S[(size_t)a * n + b] = v;
      S[(size_t)b * n + a] = S[(size_t)a * n + b];
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      H[(size_t)a * n + b] = -S[(size_t)a * n + b] / std::sqrt(S[(size_t)a * n + a] * S[(size_t)b * n + b]);
  const int no = n / 2;
  std::vector<double> ev;
  const int rc = lowest_eigenpairs(n, no, H, ev, Q);
  if (rc) return rc;
  for (int k = 0; k < no; ++k)
    for (int a = 0; a < n; ++a) C_out[(size_t)a * no + k] = Q[(size_t)a * no + k] / std::sqrt(S[(size_t)a * n + a]);
  return VMC_OK;
}


// Per axis of the contracted overlap: s(al, be) = sqrt(pi/p) sum_n e^{-mu dn^2} (p = al + be,
// mu = al be / p, dn = d + n L) and its exponent derivatives; with r^2 e^{-Z r^2} = -d/dZ e^{-Z r^2}
// the overlaps <h2|g> = -ds/dal, <g|h2> = -ds/dbe, <h2|h2> = d2s/(dal dbe) on each axis, using
// dp/dal = 1, dmu/dal = be^2/p^2, dmu/dbe = al^2/p^2.
static void axis_exponent_derivs(double al, double be, double d, double L, double out[4]) {
  const double p = al + be, mu = al * be / p, c = std::sqrt(M_PI / p);
  const double ka = be * be / (p * p), kb = al * al / (p * p);
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int n = -4; n <= 4; ++n) {
    const double dn = d + n * L, d2 = dn * dn, e = c * std::exp(-mu * d2);
    const double fa = -0.5 / p - ka * d2, fb = -0.5 / p - kb * d2;
    // d/dbe of (fa) = 1/(2 p^2) - 2 be d2 / p^2 + 2 be^2 d2 / p^3
    const double fab = 0.5 / (p * p) - 2.0 * be * d2 / (p * p) + 2.0 * be * be * d2 / (p * p * p);
    out[0] += e;
    out[1] += e * fa;
    out[2] += e * fb;
    out[3] += e * (fa * fb + fab);
  }
}

extern "C" int vmc_huckel_params_contracted(int n, double L, double eta, const double* R, double* C_out) {
  if (n < 2 || (n & 1) || !(L > 0.0) || !R || !C_out || !std::isfinite(eta)) return VMC_EINVAL;
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(R[i])) return VMC_EINVAL;
  const double z1 = 0.6066825, z2 = 0.3382168;
  std::vector<double> S((size_t)n * n), H((size_t)n * n), Q;
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {   // the lower triangle by symmetry
      double s11[3][4], s12[3][4], s21[3][4], s22[3][4];
      for (int m = 0; m < 3; ++m) {
        const double d = R[3 * a + m] - R[3 * b + m];
        axis_exponent_derivs(z1, z1, d, L, s11[m]);
        axis_exponent_derivs(z1, z2, d, L, s12[m]);
        axis_exponent_derivs(z2, z1, d, L, s21[m]);
        axis_exponent_derivs(z2, z2, d, L, s22[m]);
      }
      // g1 g1; g1 h2 = -d/dbe; h2 g1 = -d/dal; h2 h2 = d2/(dal dbe), by the product rule over the axes
      double v = s11[0][0] * s11[1][0] * s11[2][0];
      double gh = 0.0, hg = 0.0, hh = 0.0;
      for (int m = 0; m < 3; ++m) {
        const int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
        gh -= s12[m][2] * s12[m1][0] * s12[m2][0];
        hg -= s21[m][1] * s21[m1][0] * s21[m2][0];
        hh += s22[m][3] * s22[m1][0] * s22[m2][0];
        for (int q = 0; q < 3; ++q)
          if (q != m) {
            const int r = 3 - m - q;
            hh += s22[m][1] * s22[q][2] * s22[r][0];
          }
      }
      S[(size_t)a * n + b] = v + eta * (gh + hg) + eta * eta * hh;
      S[(size_t)b * n + a] = S[(size_t)a * n + b];
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      H[(size_t)a * n + b] = -S[(size_t)a * n + b] / std::sqrt(S[(size_t)a * n + a] * S[(size_t)b * n + b]);
  const int no = n / 2;
  std::vector<double> ev;
  const int rc = lowest_eigenpairs(n, no, H, ev, Q);
  if (rc) return rc;
  for (int k = 0; k < no; ++k)
    for (int a = 0; a < n; ++a) C_out[(size_t)a * no + k] = Q[(size_t)a * no + k] / std::sqrt(S[(size_t)a * n + a]);
  return VMC_OK;
}

// Hueckel orbitals from the Hermitian overlap S (n x n): H = -S_ab / sqrt(S_aa S_bb) through its real
// symmetric embedding of order 2n, the n/2 lowest eigenvectors as complex (re, im) pairs in C_out.
static int hermitian_huckel(int n, const std::vector<std::complex<double>>& S, double* C_out) {
  using cplx = std::complex<double>;
  // H = -S_ab / sqrt(S_aa S_bb) (Hermitian) through its real symmetric embedding of order 2n
  const int n2 = 2 * n;
  std::vector<double> M((size_t)n2 * n2), Q;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const cplx h = -S[(size_t)a * n + b] / std::sqrt(S[(size_t)a * n + a].real() * S[(size_t)b * n + b].real());
      M[(size_t)a * n2 + b] = h.real();
      M[(size_t)(a + n) * n2 + b + n] = h.real();
      M[(size_t)a * n2 + b + n] = -h.imag();
      M[(size_t)(a + n) * n2 + b] = h.imag();
    }
  std::vector<double> ev;
  const int rc = lowest_eigenpairs(n2, n, M, ev, Q);
  if (rc) return rc;
  // the lowest n embedded eigenvectors (x, y) give n complex vectors x + i y spanning the n/2
  // lowest eigenvectors of H; Gram-Schmidt, each time on the candidate of largest residual
  const int no = n / 2;
  std::vector<std::vector<cplx>> z(n, std::vector<cplx>(n));
  for (int c = 0; c < n; ++c)
    for (int a = 0; a < n; ++a) z[c][a] = cplx(Q[(size_t)a * n + c], Q[(size_t)(a + n) * n + c]);
  std::vector<bool> used(n, false);
  for (int k = 0; k < no; ++k) {
    int best = -1;
    double bn = -1.0;
    for (int c = 0; c < n; ++c) {
      if (used[c]) continue;
      double nn = 0.0;
      for (int a = 0; a < n; ++a) nn += std::norm(z[c][a]);
      if (nn > bn) { bn = nn; best = c; }
    }
    if (best < 0 || !(bn > 0.0)) return VMC_ENOCONV;
    used[best] = true;
    const double inv = 1.0 / std::sqrt(bn);
    for (int a = 0; a < n; ++a) z[best][a] *= inv;
    for (int c = 0; c < n; ++c) {
      if (used[c]) continue;
      cplx p = 0.0;
      for (int a = 0; a < n; ++a) p += std::conj(z[best][a]) * z[c][a];
      for (int a = 0; a < n; ++a) z[c][a] -= p * z[best][a];
    }
    for (int a = 0; a < n; ++a) {
      const cplx ca = z[best][a] / std::sqrt(S[(size_t)a * n + a].real());
      C_out[2 * ((size_t)a * no + k)] = ca.real();
      C_out[2 * ((size_t)a * no + k) + 1] = ca.imag();
    }
  }
  return VMC_OK;
}


extern "C" int vmc_huckel_params_theta(int n, double L, const double* theta, const double* R, const double* zeta,
                                       double* C_out) {
  if (n < 2 || (n & 1) || !(L > 0.0) || !theta || !R || !zeta || !C_out) return VMC_EINVAL;
  for (int m = 0; m < 3; ++m)
    if (!std::isfinite(theta[m])) return VMC_EINVAL;
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(R[i])) return VMC_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(zeta[i] > 0.0) || !std::isfinite(zeta[i])) return VMC_EINVAL;
  using cplx = std::complex<double>;
  // S_ab = (pi/(za+zb))^{3/2} prod_m sum_k e^{-i theta_m k} e^{-mu (d_m + k L)^2}, d = R_a - R_b taken at
  // its minimum image d - j L, which multiplies the sum by e^{i theta_m j}
  std::vector<cplx> S((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {   // the lower triangle by symmetry
      const double za = zeta[a], zb = zeta[b], mu = za * zb / (za + zb);
      cplx v = std::pow(M_PI / (za + zb), 1.5);
      for (int ax = 0; ax < 3; ++ax) {
        double dd = R[3 * a + ax] - R[3 * b + ax];
        const double j = std::floor(dd / L + 0.5);
        dd -= L * j;
        cplx sum = 0.0;
        for (int k = -3; k <= 3; ++k) sum += std::polar(std::exp(-mu * (dd + k * L) * (dd + k * L)), -theta[ax] * k);
        v *= sum * std::polar(1.0, theta[ax] * j);
      }
      S[(size_t)a * n + b] = v;
      S[(size_t)b * n + a] = std::conj(S[(size_t)a * n + b]);
    }
  return hermitian_huckel(n, S, C_out);
}

// Per axis of the contracted overlap under a twist: the terms of axis_exponent_derivs with image k of
// d = R_a - R_b (taken at its minimum image d - j L) weighted e^{-i theta k}, times e^{i theta j}.
static void axis_exponent_derivs_theta(double al, double be, double d, double L, double theta,
                                       std::complex<double> out[4]) {
  const double p = al + be, mu = al * be / p, c = std::sqrt(M_PI / p);
  const double ka = be * be / (p * p), kb = al * al / (p * p);
  const double j = std::floor(d / L + 0.5);
  const double dd = d - L * j;
  for (int q = 0; q < 4; ++q) out[q] = 0.0;
  for (int k = -4; k <= 4; ++k) {
    const double dn = dd + k * L, d2 = dn * dn, e = c * std::exp(-mu * d2);
    const double fa = -0.5 / p - ka * d2, fb = -0.5 / p - kb * d2;
    const double fab = 0.5 / (p * p) - 2.0 * be * d2 / (p * p) + 2.0 * be * be * d2 / (p * p * p);
    const std::complex<double> w = std::polar(1.0, -theta * k);
    out[0] += w * e;
    out[1] += w * (e * fa);
    out[2] += w * (e * fb);
    out[3] += w * (e * (fa * fb + fab));
  }
  const std::complex<double> ph = std::polar(1.0, theta * j);
  for (int q = 0; q < 4; ++q) out[q] *= ph;
}

extern "C" int vmc_huckel_params_theta_contracted(int n, double L, const double* theta, double eta, const double* R,
                                                  double* C_out) {
  if (n < 2 || (n & 1) || !(L > 0.0) || !theta || !R || !C_out || !std::isfinite(eta)) return VMC_EINVAL;
  for (int m = 0; m < 3; ++m)
    if (!std::isfinite(theta[m])) return VMC_EINVAL;
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(R[i])) return VMC_EINVAL;
  using cplx = std::complex<double>;
  const double z1 = 0.6066825, z2 = 0.3382168;
  std::vector<cplx> S((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {   // the lower triangle by symmetry
      cplx s11[3][4], s12[3][4], s21[3][4], s22[3][4];
      for (int m = 0; m < 3; ++m) {
        const double d = R[3 * a + m] - R[3 * b + m];
        axis_exponent_derivs_theta(z1, z1, d, L, theta[m], s11[m]);
        axis_exponent_derivs_theta(z1, z2, d, L, theta[m], s12[m]);
        axis_exponent_derivs_theta(z2, z1, d, L, theta[m], s21[m]);
        axis_exponent_derivs_theta(z2, z2, d, L, theta[m], s22[m]);
      }
      // as vmc_huckel_params_contracted, with complex axis factors
      cplx v = s11[0][0] * s11[1][0] * s11[2][0];
      cplx gh = 0.0, hg = 0.0, hh = 0.0;
      for (int m = 0; m < 3; ++m) {
        const int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
        gh -= s12[m][2] * s12[m1][0] * s12[m2][0];
        hg -= s21[m][1] * s21[m1][0] * s21[m2][0];
        hh += s22[m][3] * s22[m1][0] * s22[m2][0];
        for (int q = 0; q < 3; ++q)
          if (q != m) {
            const int r = 3 - m - q;
            hh += s22[m][1] * s22[q][2] * s22[r][0];
          }
      }
      S[(size_t)a * n + b] = v + eta * (gh + hg) + eta * eta * hh;
      S[(size_t)b * n + a] = std::conj(S[(size_t)a * n + b]);
    }
  return hermitian_huckel(n, S, C_out);
}

extern "C" int vmc_server_admit_count(size_t budget, size_t resident, int n_queued, const size_t* bytes) {
  if (n_queued < 0 || (n_queued > 0 && !bytes)) return -1;
  return admit_count(budget, resident, n_queued, bytes);
}

// One step of stochastic reconfiguration (Sorella, PRB 64, 024512 (2001)) from the sample means
// [E, <O> (5), <E_L O> (5), <O O^T> (25)]: f_k = -2 (<E_L O_k> - E <O_k>), S_kl = <O_k O_l> -
// <O_k><O_l> over the active parameters, S_kk scaled by (1 + eps), dp = tau S^-1 f by Cholesky.
extern "C" int vmc_sr_update(const double* stats, int active, double eps, double tau, double* dp) {
  constexpr int P = 7;   // (b, b_1, f_11, f_12, f_22, f_1, f_2)
  if (!stats || !dp || (active & ~((1 << P) - 1)) || !(eps >= 0.0) || !std::isfinite(eps) || !std::isfinite(tau))
    return VMC_EINVAL;
  for (int q = 0; q < 1 + 2 * P + P * P; ++q)
    if (!std::isfinite(stats[q])) return VMC_EINVAL;
  const double E = stats[0];
  const double* O = stats + 1;
  const double* EO = stats + 1 + P;
  const double* OO = stats + 1 + 2 * P;
  int idx[P], n = 0;
  for (int k = 0; k < P; ++k)
    if ((active >> k) & 1) idx[n++] = k;
  double L[P][P] = {}, f[P], y[P];
  for (int a = 0; a < n; ++a) {
    const int k = idx[a];
    f[a] = -2.0 * (EO[k] - E * O[k]);
    for (int b = 0; b <= a; ++b) {
      const int l = idx[b];
      double s = OO[P * k + l] - O[k] * O[l];
      if (a == b) s *= 1.0 + eps;
      for (int c = 0; c < b; ++c) s -= L[a][c] * L[b][c];
      if (a == b) {
        if (!(s > 0.0)) return VMC_ENOTSPD;
        L[a][a] = std::sqrt(s);
      } else {
        L[a][b] = s / L[b][b];
      }
    }
  }
  for (int a = 0; a < n; ++a) {
    double s = tau * f[a];
    for (int c = 0; c < a; ++c) s -= L[a][c] * y[c];
    y[a] = s / L[a][a];
  }
  for (int k = 0; k < P; ++k) dp[k] = 0.0;
  for (int a = n - 1; a >= 0; --a) {
    double s = y[a];
    for (int c = a + 1; c < n; ++c) s -= L[c][a] * dp[idx[c]];
    dp[idx[a]] = s / L[a][a];
  }
  return VMC_OK;
}
