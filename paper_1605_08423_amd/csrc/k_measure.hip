// Measurement kernels (a5, a6): per sample and walker, the Ewald potential
// energy and its real-space gradient on the protons, the local kinetic energy,
// d ln|psi|/dR and dE_L/dR by the determinant adjoint, accumulated in FP64.
//
// Ewald (all 2N charges, protons +1, electrons -1, cubic box of side L):
//   V = sum_{i<j} q_i q_j erfc(kappa r_ij)/r_ij  (minimum image)
//     + sum_{k in half space, 0<|n|^2<=nmax^2} W_k |rho(k)|^2,  W_k = (4 pi/V) e^{-k^2/(4 kappa^2)}/k^2
//     - (kappa/sqrt(pi)) sum_i q_i^2.
// The reciprocal gradient on proton b, -2 sum_k W_k k Im(conj(rho(k)) e^{i k R_b}),
// is linear in rho, so its electron part is formed once per walker from the mean
// electron structure factor (k_finalize) instead of per sample.
//
// Local energy with psi = D_up D_dn e^U, B_s = C A_s^-1 (N x NS):
//   T_L = sum_s sum_{i in s, a} X_ia B_ai - 1/2 sum_i (lap_i U + |grad_i U|^2),
//   X_ia = -1/2 [lap phi_a(r_i) + 2 grad phi_a(r_i) . grad_i U].
// With C, zeta and U held fixed, d/dR_b acts on phi_b(r - R_b) only:
//   d ln|psi|/dR_b = -sum_i B_bi grad phi_b(r_i),
//   dT_L/dR_b = sum_i [1/2 (grad lap phi_b + 2 Hess phi_b . grad_i U) B_bi + grad phi_b(r_i) W_bi],
//   M = X B (NS x NS), W = B M, from d A^-1 = -A^-1 dA A^-1 with dA/dR_b = -grad phi_b c_b^T.
// With the one-body Jastrow term U also holds sum_{i,b} f(rho_ib), which moves with R_b:
//   d ln|psi|/dR_b gets -sum_i grad f_ib, and dT_L/dR_b gets
//   sum_i [1/2 grad lap f_ib + hess f_ib (grad_i U + grad_i ln|D|)].
// Twisted boundary conditions change only the basis (its image signs).
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {


// Deterministic block sum (blockDim = 256); every thread gets the result.
__device__ __forceinline__ double block_sum256(double v, double* scratch4) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) scratch4[wv] = v;
  __syncthreads();
  double r = (scratch4[0] + scratch4[1]) + (scratch4[2] + scratch4[3]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------- Ewald ---
constexpr int NMAXC = 12;   // largest supported ewald_nmax

template <int N, class Real, int NMX, bool BATCH>
__global__ __launch_bounds__(256) void k_ewald_sample(MeasureArgs m, EwaldArgs e, Batch bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  int bblk = 0;
  if constexpr (BATCH) {
    const int j = batch_job(bt, blockIdx.x);
    m = bt.jobs[j].m;
    e = bt.jobs[j].e;
    bblk = (int)blockIdx.x - bt.off[j];
  }
  const int blk = BATCH ? bblk : (int)blockIdx.x;
  double* pe = reinterpret_cast<double*>(smem);   // N x 3 electrons
  double* pp = pe + 3 * N;                         // N x 3 protons
  double* part = pp + 3 * N;                       // 4 x N x 3 partial e-p gradients
  double2* ph = reinterpret_cast<double2*>(part + 12 * N);   // 3 x N x (nmax+1) phase powers
  __shared__ double red[4];
  const int t = threadIdx.x & 255, w = blk;   // 256-thread launch
  const int NP1 = e.nmax + 1;
  const double L = m.L, invL = m.invL;
  for (int u = t; u < 3 * N; u += 256) {
    pe[u] = m.pos[(size_t)w * 3 * N + u];
    pp[u] = m.R[u];
  }
  __syncthreads();
  // e^{i 2 pi n x / L} for n = 0..nmax, per electron and axis
  for (int u = t; u < 3 * N; u += 256) {
    const int i = u / 3, ax = u % 3;
    double s, c;
    sincospi(2.0 * pe[3 * i + ax] * invL, &s, &c);
    double2* row = ph + ((size_t)ax * N + i) * NP1;
    double2 v = make_double2(1.0, 0.0);
    row[0] = v;
    for (int n = 1; n < NP1; ++n) {
      v = make_double2(v.x * c - v.y * s, v.x * s + v.y * c);
      row[n] = v;
    }
  }
  __syncthreads();
  // Reciprocal space.  The (ny, nz) slots come sorted longest first; thread u of
  // an electron half (u = t mod 128) accumulates the slots of rank base + u and
  // base + 255 - u (a long and a short one, so the two waves of a half get about the
  // same work), nx counted from 0 (the k of (slot, nx) is k0 + nx - nx0), so one load
  // of an electron's x phases serves both slots.  Every lane of a wave runs the wave's
  // longest length of each slot, taken from a few compiled trip counts so the loop has
  // no branches and its phase loads are issued together.  When all slots fit one
  // pass, waves 2 and 3 take electrons N/2..N-1 and hand their partial sums to waves
  // 0 and 1 through LDS (over the phase table, no longer needed); otherwise waves 0
  // and 1 take every electron in passes of 256 slots.
  double vrec = 0.0, vreal = 0.0;
  double* racc = m.rho_acc + (size_t)w * e.nk * 2;
  const bool split = e.nslot <= 256;
  const int u = t & 127, hf = t >> 7;
  if (split || hf == 0) {
    for (int base = 0; base < e.nslot; base += 256) {
      int ay[2], az[2], k0[2], nx0[2], nb[2];
      double sy[2], sz[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int sl = q == 0 ? base + u : base + 255 - u;
        ay[q] = az[q] = k0[q] = nx0[q] = nb[q] = 0;
        sy[q] = sz[q] = 1.0;
        if (sl < e.nslot) {
          const int ny = e.slot[4 * sl], nz = e.slot[4 * sl + 1];
          ay[q] = ny < 0 ? -ny : ny; az[q] = nz < 0 ? -nz : nz;
          sy[q] = ny < 0 ? -1.0 : 1.0; sz[q] = nz < 0 ? -1.0 : 1.0;
          k0[q] = e.slot[4 * sl + 2];
          nx0[q] = e.slot_nx0[sl];
          nb[q] = nx0[q] + e.slot[4 * sl + 3];
        }
      }
      int ma = nb[0], mb = nb[1];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        ma = max(ma, __shfl_xor(ma, off, 64));
        mb = max(mb, __shfl_xor(mb, off, 64));
      }
      const int ba = __builtin_amdgcn_readfirstlane(ma), bb = __builtin_amdgcn_readfirstlane(mb);
      double ar[NMX + 1], ai[NMX + 1], br[NMX + 1], bi[NMX + 1];
#pragma unroll
      for (int j = 0; j <= NMX; ++j) { ar[j] = ai[j] = br[j] = bi[j] = 0.0; }
      const int i_lo = split ? hf * (N / 2) : 0, i_hi = split ? (hf + 1) * (N / 2) : N;
      // NA, NBB: compiled trip counts of the two slots (>= the wave's ba, bb).  Phases
      // past a row's end fall in the next row of the table (still inside it) and feed
      // only accumulators that are never read.
      auto electrons = [&](auto na_c, auto nb_c) {
        constexpr int NA = decltype(na_c)::value, NBB = decltype(nb_c)::value;
        constexpr int NX = NA > NBB ? NA : NBB;
        for (int i = i_lo; i < i_hi; ++i) {
          const double2* ex = ph + (size_t)i * NP1;
          double2 xv[NX];
#pragma unroll
          for (int j = 0; j < NX; ++j) xv[j] = ex[j];
          const double2 eya = ph[((size_t)1 * N + i) * NP1 + ay[0]], eza = ph[((size_t)2 * N + i) * NP1 + az[0]];
          const double2 eyb = ph[((size_t)1 * N + i) * NP1 + ay[1]], ezb = ph[((size_t)2 * N + i) * NP1 + az[1]];
          const double ya_r = eya.x, ya_i = sy[0] * eya.y, za_r = eza.x, za_i = sz[0] * eza.y;
          const double yb_r = eyb.x, yb_i = sy[1] * eyb.y, zb_r = ezb.x, zb_i = sz[1] * ezb.y;
          const double tar = ya_r * za_r - ya_i * za_i, tai = ya_r * za_i + ya_i * za_r;
          const double tbr = yb_r * zb_r - yb_i * zb_i, tbi = yb_r * zb_i + yb_i * zb_r;
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            ar[j] += xv[j].x * tar - xv[j].y * tai;
            ai[j] += xv[j].x * tai + xv[j].y * tar;
          }
#pragma unroll
          for (int j = 0; j < NBB; ++j) {
            br[j] += xv[j].x * tbr - xv[j].y * tbi;
            bi[j] += xv[j].x * tbi + xv[j].y * tbr;
          }
        }
      };
      if (ba <= 8 && bb <= 7)
        electrons(std::integral_constant<int, 8>{}, std::integral_constant<int, 7>{});
      else if (ba <= 10 && bb <= 5)
        electrons(std::integral_constant<int, 10>{}, std::integral_constant<int, 5>{});
      else
        electrons(std::integral_constant<int, NMX + 1>{}, std::integral_constant<int, NMX + 1>{});
      if (split) {
        // the second half's sums go to comb[k] (over the phase table), the first half adds them
        double2* comb = ph;
        __syncthreads();
        if (hf == 1) {
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int j = 0; j <= NMX; ++j)
              if (j >= nx0[q] && j < nb[q])
                comb[k0[q] + j - nx0[q]] = q == 0 ? make_double2(ar[j], ai[j]) : make_double2(br[j], bi[j]);
        }
        __syncthreads();
        if (hf == 1) break;
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int j = 0; j <= NMX; ++j)
            if (j >= nx0[q] && j < nb[q]) {
              const double2 c = comb[k0[q] + j - nx0[q]];
              if (q == 0) { ar[j] += c.x; ai[j] += c.y; } else { br[j] += c.x; bi[j] += c.y; }
            }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j <= NMX; ++j) {
          if (j >= nx0[q] && j < nb[q]) {
            const int k = k0[q] + j - nx0[q];
            const double rer = -(q == 0 ? ar[j] : br[j]), rei = -(q == 0 ? ai[j] : bi[j]);   // electron charge -1
            const double tr = e.rho_p[2 * k] + rer, ti = e.rho_p[2 * k + 1] + rei;
            vrec += e.kvec[4 * k + 3] * (tr * tr + ti * ti);
            racc[2 * k] += rer;
            racc[2 * k + 1] += rei;
          }
        }
    }
  }
  {
  // real space in 6N tasks of about N/4 pairs: u < 2N electron-electron (half
  // circulant offsets split in two), 2N <= u < 6N electron-proton (electrons split in four)
  const Real kap = (Real)e.kappa;
  const Real tkp = (Real)(2.0 * e.kappa / 1.7724538509055160273);
  for (int u = t; u < 6 * N; u += 256) {
    if (u < 2 * N) {
      const int i = u % N, hh = u / N;
      const int d0 = hh == 0 ? 1 : N / 4 + 1, d1 = hh == 0 ? N / 4 : N / 2;
      Real vs = Real(0);
      for (int dd = d0; dd <= d1; ++dd) {
        if (dd == N / 2 && i >= N / 2) break;
        const int j = (i + dd) % N;
        Real r2 = Real(0);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const Real d = (Real)min_image(pe[3 * i + ax] - pe[3 * j + ax], L, invL);
          r2 += d * d;
        }
        const Real ir = dev_rsqrt<Real>(r2);
        Real e2;
        vs += dev_erfc_exp<Real>(kap * (r2 * ir), &e2) * ir;
      }
      vreal += (double)vs;
    } else {
      const int b = (u - 2 * N) % N, qd = (u - 2 * N) / N;
      const int i0 = qd * N / 4, i1 = (qd + 1) * N / 4;
      Real vs = Real(0), gx = Real(0), gy = Real(0), gz = Real(0);
      for (int i = i0; i < i1; ++i) {
        const Real dx = (Real)min_image(pp[3 * b] - pe[3 * i], L, invL);
        const Real dy = (Real)min_image(pp[3 * b + 1] - pe[3 * i + 1], L, invL);
        const Real dz = (Real)min_image(pp[3 * b + 2] - pe[3 * i + 2], L, invL);
        const Real r2 = dx * dx + dy * dy + dz * dz;
        const Real ir = dev_rsqrt<Real>(r2);
        Real e2;
        const Real ec = dev_erfc_exp<Real>(kap * (r2 * ir), &e2);
        vs -= ec * ir;
        // d/dR_b of -erfc(kappa r)/r with r = |R_b - r_i|
        const Real dedr = -ec * ir * ir - tkp * e2 * ir;
        const Real gsc = -dedr * ir;
        gx += gsc * dx; gy += gsc * dy; gz += gsc * dz;
      }
      vreal += (double)vs;
      double* pq = part + ((size_t)qd * N + b) * 3;
      pq[0] = (double)gx; pq[1] = (double)gy; pq[2] = (double)gz;
    }
  }
  }
  __syncthreads();
  for (int b = t; b < N; b += 256) {
    double* dv = m.dVs + (size_t)w * 3 * N + 3 * b;
    for (int c = 0; c < 3; ++c)
      dv[c] = (part[(0 * N + b) * 3 + c] + part[(1 * N + b) * 3 + c]) +
              (part[(2 * N + b) * 3 + c] + part[(3 * N + b) * 3 + c]);
  }
  const double vtot = block_sum256(vrec + vreal, red);
  if (t == 0) m.Vs[w] = vtot + (*e.Vpp + e.Vself);
}

// ------------------------------------------------- Slater and Jastrow ---
typedef double d4_t __attribute__((ext_vector_type(4)));

// One 16x16x4 FP64 matrix-core step: D += A(16x4) B(4x16).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; element v of its result is
// D[l / 16 + 4 v][l % 16] (the row interleave was read off the hardware).
__device__ __forceinline__ d4_t mfma16(double av, double bv, d4_t acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
}

// 16x16x4 step of the products whose operands are stored as Real: FP64 matrix
// cores for Real = double, FP32 ones (twice the rate) in mixed mode.  Element v of
// lane l's result is row l/16 + 4 v (FP64) or 4 (l/16) + v (FP32) of D, column l % 16
// (both read off the hardware); the operands follow the same layout in both.
typedef float f4_t __attribute__((ext_vector_type(4)));
template <class Real> struct MM16;
template <> struct MM16<double> {
  typedef d4_t acc_t;
  static __device__ __forceinline__ acc_t zero() { return d4_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) { return mfma16(a, b, c); }
  static __device__ __forceinline__ int row(int l4, int v) { return l4 + 4 * v; }
};
template <> struct MM16<float> {
  typedef f4_t acc_t;
  static __device__ __forceinline__ acc_t zero() { return f4_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l4, int v) { return 4 * l4 + v; }
};

// Per walker (one 256-thread block): Jastrow gradient/Laplacian per electron
// (one-body terms included); per spin the three contractions B = C A^-1 (FP64 matrix cores), M = X B and
// W = B M (matrix cores in Real: their operands are stored as Real), dimensions
// padded to multiples of 16 with zeros, and the elementwise basis passes that
// build X and the d/dR terms.
// LDS layout of k_slater_sample (bytes), shared with the launcher.  B/W, X and M
// are stored as Real (FP32 in mixed mode: they carry FP32-level errors already);
// the inverse staging and the partial sums are FP64.
template <int NS, class Real>
struct SlaterLds {
  static constexpr int N = 2 * NS;
  static constexpr int NSP = (NS + 15) / 16 * 16, NP = (N + 15) / 16 * 16;
  static constexpr int NT = (256 / N) * N;
  // X rows are read four consecutive k at a time; a stride of 4 mod 32 words keeps the
  // 16 rows of such a read on disjoint LDS banks
  static constexpr int LDB = NSP + 1, LDX = NP + 4, LDI = NSP + 1;
  static constexpr size_t head = (size_t)(3 * N + 3 * N + N) * sizeof(double) + (size_t)6 * N * sizeof(Real);
  static constexpr size_t bs = (size_t)NP * LDB * sizeof(Real);
  static constexpr size_t xm0 = (size_t)NSP * LDX * sizeof(Real);
  static constexpr size_t xm1 = (size_t)NSP * LDI * sizeof(double);
  static constexpr size_t xm2 = (size_t)6 * NT * sizeof(double);
  static constexpr size_t xm3 = (size_t)5 * 256 * sizeof(double);
  static constexpr size_t xm01 = xm0 > xm1 ? xm0 : xm1, xm23 = xm2 > xm3 ? xm2 : xm3;
  static constexpr size_t xm = xm01 > xm23 ? xm01 : xm23;
  static constexpr size_t pad(size_t v) { return (v + 15) / 16 * 16; }
  // NS > 64: B, X (later W) and M do not fit in LDS beside each other; they live in a
  // per-walker region of device memory and LDS keeps the per-electron data and the
  // partial sums only
  static constexpr bool GSCR = NS > 64;
  static constexpr size_t jpart = (size_t)((256 / N) > 0 ? (256 / N) : 1) * N * 5 * sizeof(double);
  static constexpr size_t small = xm23 > jpart ? xm23 : jpart;
  static constexpr size_t mreg = (size_t)NSP * LDI * sizeof(Real);
  // staging of one 16-row tile of a left operand: 16 x (K + pad) elements, K <= 2 NSP
  static constexpr size_t stage = (size_t)16 * (2 * NSP + 2) * sizeof(double);
  // grad ln|D| per electron (3 x N, Real) for the one-body Jastrow term's d/dR, after the rest
  static constexpr size_t gdoff = GSCR ? pad(head) + pad(small) + pad(stage) : pad(head) + pad(bs) + pad(xm);
  static constexpr size_t bytes = gdoff + pad((size_t)3 * N * sizeof(Real));
  static constexpr size_t scr_bytes = GSCR ? pad(bs) + pad(bs > xm0 ? bs : xm0) + pad(mreg) : 0;
};

// Four consecutive values from a 16-byte aligned LDS address.
__device__ __forceinline__ void load4(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double (&o)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// D = A B for TC = 8 column tiles: wave w computes tiles 2w and 2w + 1, one at a time, keeping
// that tile's B columns for the whole K in registers (B operand layout, read once per pass),
// while the work-group stages A one 16-row tile at a time in LDS (coalesced reads; rows padded
// to K + 1 doubles or K + 2 floats so the 16 rows of an A-operand read fall on distinct banks).
// All threads of the work-group call it.
template <class Op, class Out, int TR, int K>
__device__ __forceinline__ void gemm_stage_a(const Op* A, int lda, const Op* B, int ldb, Out* D, int ldd, Op* stage,
                                             int t, int wave, int l16, int l4) {
  constexpr int KK = K / 4, LDA_S = K + (sizeof(Op) == 8 ? 1 : 2);
  for (int c = 0; c < 2; ++c) {
    const int col = 16 * (2 * wave + c) + l16;
    Op breg[KK];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) breg[kk] = B[(4 * kk + l4) * ldb + col];
    for (int rt = 0; rt < TR; ++rt) {
      __syncthreads();                       // the previous tile is consumed
      for (int u = t; u < 16 * K; u += 256)
        stage[(u / K) * LDA_S + u % K] = A[(size_t)(16 * rt + u / K) * lda + u % K];
      __syncthreads();
      typename MM16<Op>::acc_t acc = MM16<Op>::zero();
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) acc = MM16<Op>::step(stage[l16 * LDA_S + 4 * kk + l4], breg[kk], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) D[(size_t)(16 * rt + MM16<Op>::row(l4, v)) * ldd + col] = (Out)acc[v];
    }
  }
  __syncthreads();
}

template <int NS, class Real, int NIMG, bool BATCH, bool TW, bool CB = false>
__global__ __launch_bounds__(256, sizeof(Real) == 4 ? 2 : 1) void k_slater_sample(MeasureArgs m, Batch bt) {
  using Lay = SlaterLds<NS, Real>;
  constexpr int N = 2 * NS;
  constexpr int NSP = Lay::NSP, NP = Lay::NP;
  constexpr int H = 256 / N;            // threads per basis centre in the pair passes
  constexpr int NT = H * N;
  constexpr int IPT = (NS + H - 1) / H; // electrons per thread per spin
  constexpr int LDB = Lay::LDB, LDX = Lay::LDX, LDI = Lay::LDI;
  constexpr int TI = NSP / 16, TA = NP / 16;      // tile counts along electrons / centres
  constexpr int TPW_B = (TA * TI + 3) / 4;        // N x NS outputs per wave
  constexpr int TPW_M = (TI * TI + 3) / 4;        // NS x NS outputs per wave
  extern __shared__ __align__(16) unsigned char smem[];
  if constexpr (BATCH) m = bt.jobs[batch_job(bt, blockIdx.x)].m;
  double* pos = reinterpret_cast<double*>(smem);     // N x 3
  double* gU = pos + 3 * N;                            // N x 3
  double* lU = gU + 3 * N;                             // N
  Real* trig = reinterpret_cast<Real*>(lU + N);        // N x 6 (sin x3, cos x3)
  constexpr bool GSCR = Lay::GSCR;
  __shared__ double red[4];
  const int t = threadIdx.x & 255;   // (the launch has 256 threads; the mask lets the compiler bound t)
  // the walker index is re-derived from the block index at its uses (a long-lived copy costs registers)
  auto walker = [&]() -> int {
    return BATCH ? (int)blockIdx.x - bt.off[batch_job(bt, blockIdx.x)] : (int)blockIdx.x;
  };
  unsigned char* gsc = GSCR ? m.scr + (size_t)walker() * Lay::scr_bytes : nullptr;
  unsigned char* lds2 = smem + Lay::pad(Lay::head);
  Real* Bs = reinterpret_cast<Real*>(GSCR ? gsc : lds2);                          // NP x LDB : B (later W)
  unsigned char* xmb = GSCR ? gsc + Lay::pad(Lay::bs) : lds2 + Lay::pad(Lay::bs);
  Real* Xr = reinterpret_cast<Real*>(xmb);             // NSP x LDX : X (GSCR: later W)
  double* XM = reinterpret_cast<double*>(xmb);         // NSP x LDI : A^-1, then M
  double* SM = GSCR ? reinterpret_cast<double*>(lds2) : XM;   // partial sums
  double* stg_d = reinterpret_cast<double*>(lds2 + Lay::pad(Lay::small));   // GSCR operand staging
  Real* stg_r = reinterpret_cast<Real*>(stg_d);
  Real* Ws = GSCR ? Xr : Bs;
  Real* gD = reinterpret_cast<Real*>(smem + Lay::gdoff);   // N x 3: grad ln|D| (one-body term only)
  // one-body term: proton positions (3 x N), needed by the Jastrow pass only, in LDS that B
  // (or the GEMM staging) takes later
  double* Rp = GSCR ? stg_d : reinterpret_cast<double*>(lds2);
  const bool one_body = m.j1_beta > 0.0;
  const int lane = t & 63, wave = t >> 6, l16 = lane & 15, l4 = lane >> 4;
  const double L = m.L, invL = m.invL;
  for (int u = t; u < 3 * N; u += 256) pos[u] = m.pos[(size_t)walker() * 3 * N + u];
  __syncthreads();
  for (int i = t; i < N; i += 256)
    for (int ax = 0; ax < 3; ++ax) {
      Real s, c;
      dev_sincospi<Real>((Real)(pos[3 * i + ax] * invL), &s, &c);
      trig[6 * i + ax] = s;
      trig[6 * i + 3 + ax] = c;
    }
  if (one_body)
    for (int u = t; u < 3 * N; u += 256) Rp[u] = m.R[u];
  __syncthreads();
  // Jastrow gradient and Laplacian per electron; HJ threads share an electron's pairs
  constexpr int HJ = (256 / N) > 0 ? (256 / N) : 1;
  double tj = 0.0, usum = 0.0;
  {
    const Real LoP = (Real)(L / VMC_PI), kf = (Real)((VMC_PI * invL) * (VMC_PI * invL));
    const Real ap = (Real)m.a_par, aa = (Real)m.a_anti, bb = (Real)m.b;
    double* jp = SM;                                   // HJ x N x 5 partial sums
    for (int u = t; u < HJ * N; u += 256) {
      const int i = u % N, hj = u / N;
      const int j0 = hj * N / HJ, j1 = (hj + 1) * N / HJ;
      Real g0 = 0, g1 = 0, g2 = 0, lp = 0, ui = 0;
      const Real* ti = trig + 6 * i;
      for (int j = j0; j < j1; ++j) {
        if (j == i) continue;
        const Real* tj_ = trig + 6 * j;
        Real rt[3], cc[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          rt[ax] = LoP * (ti[ax] * tj_[3 + ax] - ti[3 + ax] * tj_[ax]);
          cc[ax] = ti[3 + ax] * tj_[3 + ax] + ti[ax] * tj_[ax];
        }
        const Real r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
        const Real irho = dev_rsqrt<Real>(r2);
        const Real rho = r2 * irho;
        const Real a = ((i / NS) == (j / NS)) ? ap : aa;
        const Real den = Real(1) + bb * rho, iden = dev_rcp<Real>(den);
        const Real up = a * iden * iden, upp = Real(-2) * a * bb * iden * iden * iden;
        const Real gr0 = rt[0] * cc[0] * irho, gr1 = rt[1] * cc[1] * irho, gr2 = rt[2] * cc[2] * irho;
        const Real gg = gr0 * gr0 + gr1 * gr1 + gr2 * gr2;
        const Real lr = (cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2] - kf * r2) * irho - gg * irho;
        g0 += up * gr0; g1 += up * gr1; g2 += up * gr2;
        lp += upp * gg + up * lr;
        if (j > i) ui += a * rho * iden;
      }
      double f1sum = 0.0;
      if (one_body) {
        // one-body term f(rho) = -(1 - e^{-beta rho}) / beta of electron i and the protons of
        // this thread's share: f' = -e^{-beta rho}, f'' = beta e^{-beta rho}.  The sum of f is
        // taken as (sum e^{-beta rho} - count) / beta: the exponentials are small and varied,
        // while summing the near-constant -1/beta of the distant protons in the Jastrow
        // precision would drift by a rounding error per term
        const Real beta = (Real)m.j1_beta;
        Real sx = Real(0);
#pragma unroll 1
        for (int c = j0; c < j1; ++c) {
          // sin and cos of pi d / L from the minimum-image offset itself, so that rho keeps its
          // relative accuracy for close pairs (the cusp terms go as 1 / rho)
          Real rt[3], cc[3];
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            Real sc, cs;
            sincospi_half<Real>((Real)(min_image(pos[3 * i + ax] - Rp[3 * c + ax], L, invL) * invL), &sc, &cs);
            rt[ax] = LoP * sc;
            cc[ax] = cs;
          }
          const Real r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
          const Real irho = dev_rsqrt<Real>(r2);
          const Real rho = r2 * irho;
          const Real ex = dev_exp<Real>(-beta * rho);
          const Real gr0 = rt[0] * cc[0] * irho, gr1 = rt[1] * cc[1] * irho, gr2 = rt[2] * cc[2] * irho;
          const Real gg = gr0 * gr0 + gr1 * gr1 + gr2 * gr2;
          const Real lr = (cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2] - kf * r2) * irho - gg * irho;
          g0 -= ex * gr0; g1 -= ex * gr1; g2 -= ex * gr2;
          lp += beta * ex * gg - ex * lr;
          sx += ex;
        }
        f1sum = ((double)sx - (double)(j1 - j0)) / m.j1_beta;
      }
      double* q = jp + ((size_t)hj * N + i) * 5;
      q[0] = (double)g0; q[1] = (double)g1; q[2] = (double)g2; q[3] = (double)lp; q[4] = (double)ui + f1sum;
    }
    __syncthreads();
    // the three-body term's gradient, Laplacian and value, from the pass before this kernel
    const double* j3in = m.j3 ? m.j3scr + (size_t)walker() * j3_measure_doubles(N) : nullptr;
    for (int i = t; i < N; i += 256) {
      double g0 = 0, g1 = 0, g2 = 0, lp = 0, ui = 0;
      for (int hj = 0; hj < HJ; ++hj) {
        const double* q = jp + ((size_t)hj * N + i) * 5;
        g0 += q[0]; g1 += q[1]; g2 += q[2]; lp += q[3]; ui += q[4];
      }
      if (j3in) {
        g0 += j3in[3 * i]; g1 += j3in[3 * i + 1]; g2 += j3in[3 * i + 2];
        lp += j3in[3 * N + i];
        if (i == 0) ui += j3in[4 * N];
      }
      gU[3 * i] = g0; gU[3 * i + 1] = g1; gU[3 * i + 2] = g2;
      lU[i] = lp;
      tj += -0.5 * (lp + g0 * g0 + g1 * g1 + g2 * g2);
      usum += ui;
    }
  }
  __syncthreads();
  const int a = t % N, h = t / N;
  const bool act = t < NT;
  double dln0 = 0, dln1 = 0, dln2 = 0, dT0 = 0, dT1 = 0, dT2 = 0, tsl = 0;
  const double Ra0 = m.R[3 * a], Ra1 = m.R[3 * a + 1], Ra2 = m.R[3 * a + 2];
  const Real za = (Real)m.zeta[a];
  const Real LoP1 = (Real)(L / VMC_PI), kf1 = (Real)((VMC_PI * invL) * (VMC_PI * invL)), beta1 = (Real)m.j1_beta;
  for (int sp = 0; sp < 2; ++sp) {
    // A^-1 of this spin into XM (NSP x LDI, zero padded)
    const double* Bi = m.Binv + ((size_t)walker() * 2 + sp) * NS * NS;
    if constexpr (GSCR) {
      // B = C A^-1 with both operands read from device memory
      gemm_stage_a<double, Real, TA, NS>(m.C, NS, Bi, NS, Bs, LDB, stg_d, t, wave, l16, l4);
    } else {
      constexpr int PER = (NSP * NSP + 255) / 256;   // all loads issued before the stores
      double v[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int u = t + 256 * q, k = u / NSP, j = u % NSP;
        const bool ok = u < NSP * NSP && k < NS && j < NS;
        const double x = Bi[ok ? k * NS + j : 0];
        v[q] = ok ? x : 0.0;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int u = t + 256 * q, k = u / NSP, j = u % NSP;
        if (u < NSP * NSP) XM[k * LDI + j] = v[q];
      }
    __syncthreads();
    // B = C A^-1 (NP x NSP) on the FP64 matrix cores -> Bs.  Wave w takes the row
    // tiles w, w + 4, ... against every column tile, so each element of C is loaded
    // by one wave; the next k step's C values are loaded ahead of this step's products.
    {
      constexpr int RT = (TA + 3) / 4;
      d4_t acc[RT][TI];
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int tc = 0; tc < TI; ++tc) acc[r][tc] = d4_t{0.0, 0.0, 0.0, 0.0};
      auto cload = [&](int kk, int r) -> double {
        const int arow = (wave + 4 * r) * 16 + l16, k = kk * 4 + l4;
        const bool ok = (wave + 4 * r) < TA && arow < N && k < NS;
        const double v = m.C[ok ? arow * NS + k : 0];
        return ok ? v : 0.0;
      };
      double avn[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) avn[r] = cload(0, r);
      for (int kk = 0; kk < NSP / 4; ++kk) {
        double av[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) av[r] = avn[r];
        if (kk + 1 < NSP / 4) {
#pragma unroll
          for (int r = 0; r < RT; ++r) avn[r] = cload(kk + 1, r);
        }
        const int k = kk * 4 + l4;
        double bv[TI];
#pragma unroll
        for (int tc = 0; tc < TI; ++tc) bv[tc] = XM[k * LDI + tc * 16 + l16];
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (wave + 4 * r < TA) {
#pragma unroll
            for (int tc = 0; tc < TI; ++tc) acc[r][tc] = mfma16(av[r], bv[tc], acc[r][tc]);
          }
      }
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (wave + 4 * r < TA) {
          const int ta = wave + 4 * r;
#pragma unroll
          for (int tc = 0; tc < TI; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v) Bs[(ta * 16 + l4 + 4 * v) * LDB + tc * 16 + l16] = (Real)acc[r][tc][v];
        }
    }
    }
    __syncthreads();
    if (one_body || m.j3) {
      // grad_i ln|D| = sum_a grad phi_a(r_i) B_ai for the electrons of this spin, in HG
      // shares of the centres, combined in a fixed order
      constexpr int HG = 256 / NS;
      double* gp = SM;                                  // HG x NS x 3 partial sums
      for (int u = t; u < HG * NS; u += 256) {
        const int i = u % NS, hg = u / NS, e = sp * NS + i;
        const int c0 = hg * N / HG, c1 = (hg + 1) * N / HG;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 1
        for (int c = c0; c < c1; ++c) {
          const double b = (double)Bs[c * LDB + i];
          if constexpr (CB) {
            const BasisD<Real> q = contracted_derivs<Real, NIMG, false>(
                pos[3 * e] - m.R[3 * c], pos[3 * e + 1] - m.R[3 * c + 1], pos[3 * e + 2] - m.R[3 * c + 2],
                (Real)m.eta, L, invL);
            s0 += b * (double)q.gx;
            s1 += b * (double)q.gy;
            s2 += b * (double)q.gz;
          } else {
            const Real zc = (Real)m.zeta[c];
            Real g[3][4];
            basis_axis<Real, 1, NIMG, TW>(pos[3 * e] - m.R[3 * c], zc, L, invL, m.twist & 1, g[0]);
            basis_axis<Real, 1, NIMG, TW>(pos[3 * e + 1] - m.R[3 * c + 1], zc, L, invL, (m.twist >> 1) & 1, g[1]);
            basis_axis<Real, 1, NIMG, TW>(pos[3 * e + 2] - m.R[3 * c + 2], zc, L, invL, (m.twist >> 2) & 1, g[2]);
            s0 += b * (double)(g[0][1] * g[1][0] * g[2][0]);
            s1 += b * (double)(g[0][0] * g[1][1] * g[2][0]);
            s2 += b * (double)(g[0][0] * g[1][0] * g[2][1]);
          }
        }
        gp[3 * u] = s0; gp[3 * u + 1] = s1; gp[3 * u + 2] = s2;
      }
      __syncthreads();
      for (int u = t; u < 3 * NS; u += 256) {
        const int i = u / 3, c = u % 3;
        double s = 0.0;
        for (int hg = 0; hg < HG; ++hg) s += gp[3 * (hg * NS + i) + c];
        gD[3 * (sp * NS + i) + c] = (Real)s;
      }
      __syncthreads();
    }
    // pass 1: basis derivatives -> X, and the terms that need only B
    if (act) {
#pragma unroll 2
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const int e = sp * NS + i;
        // per-pair brackets in Real (FP32 in mixed mode, from FP32 basis values), sums in FP64
        Real gx, gy, gz, hxx, hyy, hzz, hxy, hxz, hyz, glx, gly, glz;
        if constexpr (CB) {
          const BasisD<Real> q = contracted_derivs<Real, NIMG, true>(pos[3 * e] - Ra0, pos[3 * e + 1] - Ra1,
                                                                     pos[3 * e + 2] - Ra2, (Real)m.eta, L, invL);
          gx = q.gx; gy = q.gy; gz = q.gz;
          hxx = q.hxx; hyy = q.hyy; hzz = q.hzz; hxy = q.hxy; hxz = q.hxz; hyz = q.hyz;
          glx = q.glx; gly = q.gly; glz = q.glz;
        } else {
          Real g[3][4];
          basis_axis<Real, 3, NIMG, TW>(pos[3 * e] - Ra0, za, L, invL, m.twist & 1, g[0]);
          basis_axis<Real, 3, NIMG, TW>(pos[3 * e + 1] - Ra1, za, L, invL, (m.twist >> 1) & 1, g[1]);
          basis_axis<Real, 3, NIMG, TW>(pos[3 * e + 2] - Ra2, za, L, invL, (m.twist >> 2) & 1, g[2]);
          const Real p00 = g[1][0] * g[2][0], p01 = g[0][0] * g[2][0], p02 = g[0][0] * g[1][0];
          gx = g[0][1] * p00; gy = g[1][1] * p01; gz = g[2][1] * p02;
          hxx = g[0][2] * p00; hyy = g[1][2] * p01; hzz = g[2][2] * p02;
          hxy = g[0][1] * g[1][1] * g[2][0]; hxz = g[0][1] * g[1][0] * g[2][1];
          hyz = g[0][0] * g[1][1] * g[2][1];
          glx = g[0][3] * p00 + g[0][1] * (g[1][2] * g[2][0] + g[1][0] * g[2][2]);
          gly = g[1][3] * p01 + g[1][1] * (g[0][2] * g[2][0] + g[0][0] * g[2][2]);
          glz = g[2][3] * p02 + g[2][1] * (g[0][2] * g[1][0] + g[0][0] * g[1][2]);
        }
        const Real lap = hxx + hyy + hzz;
        const Real u0 = (Real)gU[3 * e], u1 = (Real)gU[3 * e + 1], u2 = (Real)gU[3 * e + 2];
        const Real X = Real(-0.5) * (lap + Real(2) * (gx * u0 + gy * u1 + gz * u2));
        Xr[i * LDX + a] = X;
        const double b = (double)Bs[a * LDB + i];
        tsl += (double)X * b;
        dln0 -= b * (double)gx; dln1 -= b * (double)gy; dln2 -= b * (double)gz;
        dT0 += (double)(Real(0.5) * (glx + Real(2) * (hxx * u0 + hxy * u1 + hxz * u2))) * b;
        dT1 += (double)(Real(0.5) * (gly + Real(2) * (hxy * u0 + hyy * u1 + hyz * u2))) * b;
        dT2 += (double)(Real(0.5) * (glz + Real(2) * (hxz * u0 + hyz * u1 + hzz * u2))) * b;
      }
    }
    if (one_body && act) {
#pragma unroll 1
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const int e = sp * NS + i;
        // the one-body term of centre a at electron e moves with R_a (d/dR_a = -grad_e):
        // d ln psi/dR_a -= f' g and dT/dR_a += grad(lap f)/2 + hess f (grad U + grad ln|D|),
        // with g = grad rho, p_m = c_m^2 - (pi/L)^2 rt_m^2, G = |g|^2, P = sum p_m,
        // hess f = (f'' - f'/rho) g g^T + (f'/rho) diag(p),
        // grad lap f = f''' G g + f'' (dG + (P - G) g / rho) + f' ((dP - dG) / rho - (P - G) g / rho^2),
        // dG = 2 g (p - G) / rho, dP = -4 (pi/L)^2 rho g, f' = -x, f'' = beta x, f''' = -beta^2 x,
        // x = e^{-beta rho}
        // (sin and cos of pi d / L from the minimum-image offset, as in the Jastrow pass)
        const double Ra[3] = {Ra0, Ra1, Ra2};
        Real rt[3], cc[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          Real sc, cs;
          sincospi_half<Real>((Real)(min_image(pos[3 * e + ax] - Ra[ax], L, invL) * invL), &sc, &cs);
          rt[ax] = LoP1 * sc;
          cc[ax] = cs;
        }
        const Real r2 = rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2];
        const Real irho = dev_rsqrt<Real>(r2);
        const Real rho = r2 * irho;
        const Real x = dev_exp<Real>(-beta1 * rho);
        const Real F1 = -x, F2 = beta1 * x, F3 = -beta1 * beta1 * x;
        Real g_[3], p_[3], v_[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          g_[ax] = rt[ax] * cc[ax] * irho;
          p_[ax] = cc[ax] * cc[ax] - kf1 * rt[ax] * rt[ax];
          v_[ax] = (Real)gU[3 * e + ax] + gD[3 * e + ax];
        }
        const Real G = g_[0] * g_[0] + g_[1] * g_[1] + g_[2] * g_[2];
        const Real P = p_[0] + p_[1] + p_[2];
        const Real gv = g_[0] * v_[0] + g_[1] * v_[1] + g_[2] * v_[2];
        const Real ha = (F2 - F1 * irho) * gv, hb = F1 * irho, PG = (P - G) * irho;
        Real o[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const Real dG = Real(2) * g_[ax] * (p_[ax] - G) * irho, dP = Real(-4) * kf1 * rho * g_[ax];
          const Real glap = F3 * G * g_[ax] + F2 * (dG + PG * g_[ax]) + F1 * ((dP - dG) - PG * g_[ax]) * irho;
          o[ax] = Real(0.5) * glap + ha * g_[ax] + hb * p_[ax] * v_[ax];
        }
        dln0 -= (double)(F1 * g_[0]); dln1 -= (double)(F1 * g_[1]); dln2 -= (double)(F1 * g_[2]);
        dT0 += (double)o[0]; dT1 += (double)o[1]; dT2 += (double)o[2];
      }
    }
    __syncthreads();
    // M = X B (NSP x NSP), K = centres; stored as Real over the inverse staging
    Real* Mr = GSCR ? reinterpret_cast<Real*>(gsc + Lay::pad(Lay::bs) + Lay::pad(Lay::bs > Lay::xm0 ? Lay::bs : Lay::xm0))
                    : reinterpret_cast<Real*>(XM);
    if constexpr (GSCR) {
      gemm_stage_a<Real, Real, TI, N>(Xr, LDX, Bs, LDB, Mr, LDI, stg_r, t, wave, l16, l4);
      __syncthreads();
      gemm_stage_a<Real, Real, TA, NS>(Bs, LDB, Mr, LDI, Ws, LDB, stg_r, t, wave, l16, l4);
    } else {
    {
      typename MM16<Real>::acc_t acc[TPW_M];
#pragma unroll
      for (int q = 0; q < TPW_M; ++q) acc[q] = MM16<Real>::zero();
      // K in blocks of 16: step s of a block takes k = 16 kb + 4 (l / 16) + s in lane l, so
      // each lane reads its four X values of the block at once.  Every tile of a wave has
      // the same column tile (wave mod TI), so the B values are shared by the wave's tiles.
      const int tcw = wave % TI;
#pragma unroll 2
      for (int kb = 0; kb < NP / 16; ++kb) {
        const int k0 = 16 * kb + 4 * l4;
        Real bq[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) bq[s] = (k0 + s < N) ? Bs[(k0 + s) * LDB + tcw * 16 + l16] : Real(0);
#pragma unroll
        for (int q = 0; q < TPW_M; ++q) {
          const int tt = wave + 4 * q;
          if (tt < TI * TI) {
            const int irow = (tt / TI) * 16 + l16;
            Real xa[4];
            load4(Xr + irow * LDX + k0, xa);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const Real av = (irow < NS && k0 + s < N) ? xa[s] : Real(0);
              acc[q] = MM16<Real>::step(av, bq[s], acc[q]);
            }
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < TPW_M; ++q) {
        const int tt = wave + 4 * q;
        if (tt < TI * TI) {
          const int tr = tt / TI, tc = tt % TI;
#pragma unroll
          for (int v = 0; v < 4; ++v) Mr[(tr * 16 + MM16<Real>::row(l4, v)) * LDI + tc * 16 + l16] = (Real)acc[q][v];
        }
      }
    }
    __syncthreads();
    // W = B M (NP x NSP), K = orbitals; B is the A operand, W replaces it in Bs
    {
      typename MM16<Real>::acc_t acc[TPW_B];
#pragma unroll
      for (int q = 0; q < TPW_B; ++q) acc[q] = MM16<Real>::zero();
      for (int kk = 0; kk < NSP / 4; ++kk) {
        const int k = kk * 4 + l4;
#pragma unroll
        for (int q = 0; q < TPW_B; ++q) {
          const int tt = wave + 4 * q;
          if (tt < TA * TI) {
            const int ta = tt / TI, tc = tt % TI;
            const int arow = ta * 16 + l16;
            const Real av = (arow < N) ? Bs[arow * LDB + k] : Real(0);
            const Real bv = Mr[k * LDI + tc * 16 + l16];
            acc[q] = MM16<Real>::step(av, bv, acc[q]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < TPW_B; ++q) {
        const int tt = wave + 4 * q;
        if (tt < TA * TI) {
          const int ta = tt / TI, tc = tt % TI;
#pragma unroll
          for (int v = 0; v < 4; ++v) Bs[(ta * 16 + MM16<Real>::row(l4, v)) * LDB + tc * 16 + l16] = (Real)acc[q][v];
        }
      }
    }
    }
    __syncthreads();
    // pass 2: dT/dR_a += grad phi_a(r_i) W_ai
    if (act) {
#pragma unroll 2
      for (int s = 0; s < IPT; ++s) {
        const int i = h + H * s;
        if (i >= NS) continue;
        const double Wv = (double)Ws[a * LDB + i];
        const int e = sp * NS + i;
        if constexpr (CB) {
          const BasisD<Real> q = contracted_derivs<Real, NIMG, false>(pos[3 * e] - Ra0, pos[3 * e + 1] - Ra1,
                                                                      pos[3 * e + 2] - Ra2, (Real)m.eta, L, invL);
          dT0 += (double)q.gx * Wv;
          dT1 += (double)q.gy * Wv;
          dT2 += (double)q.gz * Wv;
        } else {
          Real g[3][4];
          basis_axis<Real, 1, NIMG, TW>(pos[3 * e] - Ra0, za, L, invL, m.twist & 1, g[0]);
          basis_axis<Real, 1, NIMG, TW>(pos[3 * e + 1] - Ra1, za, L, invL, (m.twist >> 1) & 1, g[1]);
          basis_axis<Real, 1, NIMG, TW>(pos[3 * e + 2] - Ra2, za, L, invL, (m.twist >> 2) & 1, g[2]);
          dT0 += (double)(g[0][1] * g[1][0] * g[2][0]) * Wv;
          dT1 += (double)(g[0][0] * g[1][1] * g[2][0]) * Wv;
          dT2 += (double)(g[0][0] * g[1][0] * g[2][1]) * Wv;
        }
      }
    }
    __syncthreads();
  }
  // combine the H threads of each centre in a fixed order
  double* rr = SM;
  if (act) {
    double* q = rr + ((size_t)h * N + a) * 6;
    q[0] = dln0; q[1] = dln1; q[2] = dln2; q[3] = dT0; q[4] = dT1; q[5] = dT2;
  }
  const double Tsl = block_sum256(tsl, red);
  const double Tj = block_sum256(tj, red);
  const double Us = block_sum256(usum, red);
  const int w = walker();
  const double EL = Tsl + Tj + m.Vs[w];
  double* acc = m.acc + (size_t)w * (2 + 9 * N);
  if (t < N) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int hh = 0; hh < H; ++hh)
      for (int c = 0; c < 6; ++c) v[c] += rr[((size_t)hh * N + t) * 6 + c];
    const double* dv = m.dVs + (size_t)w * 3 * N + 3 * t;
    for (int c = 0; c < 3; ++c) {
      const double d = v[3 + c] + dv[c], g = v[c];
      acc[2 + 3 * t + c] += d;
      acc[2 + 3 * N + 3 * t + c] += g;
      acc[2 + 6 * N + 3 * t + c] += EL * g;
    }
  }
  if (t == 0) {
    acc[0] += EL;
    acc[1] += EL * EL;
    m.Uj[w] = Us;
    if (m.ELs) m.ELs[w] = EL;
  }
  if (m.j3) {
    // for the three-body term's d/dR pass: grad U, grad ln|D| and E_L of this sample
    double* out = m.j3scr + (size_t)w * j3_measure_doubles(N) + 4 * N + 1;
    for (int u = t; u < 3 * N; u += 256) {
      out[u] = gU[u];
      out[3 * N + u] = (double)gD[u];
    }
    if (t == 0) out[6 * N] = EL;
  }
}

// --------------------------------------------------------- finalize ---
// Per-walker means [e_w, d_w(3N), g_w(3N), h_w(3N)]; d_w gets the constant
// proton gradient and the reciprocal gradient of the mean electron structure factor.
__global__ __launch_bounds__(256) void k_finalize(MeasureArgs m, EwaldArgs e, int M, double* means) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* rho = reinterpret_cast<double*>(smem);   // nk x 2
  const int t = threadIdx.x, w = blockIdx.x, N = m.N;
  const double invM = 1.0 / (double)M;
  const double* ra = m.rho_acc + (size_t)w * e.nk * 2;
  for (int u = t; u < 2 * e.nk; u += 256) rho[u] = ra[u] * invM;
  __syncthreads();
  const double* acc = m.acc + (size_t)w * (2 + 9 * N);
  double* mw = means + (size_t)w * (1 + 9 * N);
  if (t == 0) mw[0] = acc[0] * invM;
  for (int b = t; b < N; b += 256) {
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int k = 0; k < e.nk; ++k) {
      const double pr = e.Ptab[((size_t)k * N + b) * 2], pi = e.Ptab[((size_t)k * N + b) * 2 + 1];
      const double im = rho[2 * k] * pi - rho[2 * k + 1] * pr;   // Im(conj(rho) e^{i k R_b})
      const double s = e.kvec[4 * k + 3] * im;
      fx += e.kvec[4 * k] * s; fy += e.kvec[4 * k + 1] * s; fz += e.kvec[4 * k + 2] * s;
    }
    const double fr[3] = {-2.0 * fx, -2.0 * fy, -2.0 * fz};
    for (int c = 0; c < 3; ++c) {
      const int u = 3 * b + c;
      mw[1 + u] = acc[2 + u] * invM + e.Fconst[u] + fr[c];
      mw[1 + 3 * N + u] = acc[2 + 3 * N + u] * invM;
      mw[1 + 6 * N + u] = acc[2 + 6 * N + u] * invM;
    }
  }
}

// ------------------------------------------------------- proton setup ---
// e^{i k R_b} for every (k, b) and rho_p(k) = sum_b e^{i k R_b}.
__global__ __launch_bounds__(256) void k_proton_phases(int N, EwaldArgs e, const double* R, double* Ptab,
                                                      double* rho_p) {
  __shared__ double red[4];
  const int k = blockIdx.x, t = threadIdx.x;
  const double kx = e.kvec[4 * k], ky = e.kvec[4 * k + 1], kz = e.kvec[4 * k + 2];
  double sr = 0.0, si = 0.0;
  for (int b = t; b < N; b += 256) {
    const double th = kx * R[3 * b] + ky * R[3 * b + 1] + kz * R[3 * b + 2];
    double s, c;
    sincos(th, &s, &c);
    Ptab[((size_t)k * N + b) * 2] = c;
    Ptab[((size_t)k * N + b) * 2 + 1] = s;
    sr += c;
    si += s;
  }
  sr = block_sum256(sr, red);
  si = block_sum256(si, red);
  if (t == 0) { rho_p[2 * k] = sr; rho_p[2 * k + 1] = si; }
}

// Proton-proton real-space energy and the walker-independent gradient on
// each proton (p-p real space + the rho_p part of the reciprocal gradient).
__global__ __launch_bounds__(256) void k_proton_const(int N, double L, EwaldArgs e, const double* R,
                                                     const double* Ptab, const double* rho_p, double* Fconst,
                                                     double* Vpp) {
  __shared__ double red[4];
  const int t = threadIdx.x;
  const double invL = 1.0 / L, kap = e.kappa, tkp = 2.0 * kap / 1.7724538509055160273;
  double vs = 0.0;
  for (int b = t; b < N; b += 256) {
    double gx = 0, gy = 0, gz = 0;
    for (int c = 0; c < N; ++c) {
      if (c == b) continue;
      const double dx = min_image(R[3 * b] - R[3 * c], L, invL);
      const double dy = min_image(R[3 * b + 1] - R[3 * c + 1], L, invL);
      const double dz = min_image(R[3 * b + 2] - R[3 * c + 2], L, invL);
      const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2), ir = 1.0 / r;
      const double ec = erfc(kap * r);
      if (c > b) vs += ec * ir;
      const double dedr = -ec * ir * ir - tkp * exp(-kap * kap * r2) * ir;
      gx += dedr * dx * ir; gy += dedr * dy * ir; gz += dedr * dz * ir;
    }
    double fx = 0, fy = 0, fz = 0;
    for (int k = 0; k < e.nk; ++k) {
      const double pr = Ptab[((size_t)k * N + b) * 2], pi = Ptab[((size_t)k * N + b) * 2 + 1];
      const double s = e.kvec[4 * k + 3] * (rho_p[2 * k] * pi - rho_p[2 * k + 1] * pr);
      fx += e.kvec[4 * k] * s; fy += e.kvec[4 * k + 1] * s; fz += e.kvec[4 * k + 2] * s;
    }
    Fconst[3 * b] = gx - 2.0 * fx;
    Fconst[3 * b + 1] = gy - 2.0 * fy;
    Fconst[3 * b + 2] = gz - 2.0 * fz;
  }
  vs = block_sum256(vs, red);
  if (t == 0) *Vpp = vs;
}

// ----------------------------------------------------------- launchers ---
template <int N, class Real>
hipError_t launch_ewald_t(const MeasureArgs& m, const EwaldArgs& e, hipStream_t st, const Batch* bt, int nblk) {
  // the phase table region also holds the nk partial sums of the reciprocal combine
  const size_t tab = (size_t)3 * N * (e.nmax + 1), cmb = (size_t)e.nk;
  size_t sm = (size_t)18 * N * sizeof(double) + (tab > cmb ? tab : cmb) * sizeof(double2);
  const Batch b = bt ? *bt : Batch{nullptr, nullptr, 0};
  dim3 grid(bt ? nblk : m.W);
  if (e.nmax <= 9 && bt)
    hipLaunchKernelGGL((k_ewald_sample<N, Real, 9, true>), grid, dim3(256), sm, st, m, e, b);
  else if (e.nmax <= 9)
    hipLaunchKernelGGL((k_ewald_sample<N, Real, 9, false>), grid, dim3(256), sm, st, m, e, b);
  else if (bt)
    hipLaunchKernelGGL((k_ewald_sample<N, Real, NMAXC, true>), grid, dim3(256), sm, st, m, e, b);
  else
    hipLaunchKernelGGL((k_ewald_sample<N, Real, NMAXC, false>), grid, dim3(256), sm, st, m, e, b);
  return hipGetLastError();
}
template <int NS, class Real, bool TW>
hipError_t launch_slater_tw(const MeasureArgs& m, hipStream_t st, const Batch* bt, int nblk) {
  size_t sm = SlaterLds<NS, Real>::bytes;
  const Batch b = bt ? *bt : Batch{nullptr, nullptr, 0};
  dim3 grid(bt ? nblk : m.W);
  if (m.nimg && bt)
    hipLaunchKernelGGL((k_slater_sample<NS, Real, 1, true, TW>), grid, dim3(256), sm, st, m, b);
  else if (m.nimg)
    hipLaunchKernelGGL((k_slater_sample<NS, Real, 1, false, TW>), grid, dim3(256), sm, st, m, b);
  else if (bt)
    hipLaunchKernelGGL((k_slater_sample<NS, Real, 0, true, TW>), grid, dim3(256), sm, st, m, b);
  else
    hipLaunchKernelGGL((k_slater_sample<NS, Real, 0, false, TW>), grid, dim3(256), sm, st, m, b);
  return hipGetLastError();
}
// The contracted orbital: single trajectories without twist, N_sigma <= 64.
template <int NS, class Real>
hipError_t launch_slater_cb(const MeasureArgs& m, hipStream_t st, const Batch* bt) {
  if constexpr (NS > 64) {
    return hipErrorInvalidValue;
  } else {
    if (bt || m.twist) return hipErrorInvalidValue;
    const Batch b{nullptr, nullptr, 0};
    const size_t sm = SlaterLds<NS, Real>::bytes;
    if (m.nimg || sizeof(Real) == 8)
      hipLaunchKernelGGL((k_slater_sample<NS, Real, 1, false, false, true>), dim3(m.W), dim3(256), sm, st, m, b);
    else
      hipLaunchKernelGGL((k_slater_sample<NS, Real, 0, false, false, true>), dim3(m.W), dim3(256), sm, st, m, b);
    return hipGetLastError();
  }
}
// (a batch holds only twisted or only untwisted trajectories: the request loop buckets them apart)
template <int NS, class Real>
hipError_t launch_slater_t(const MeasureArgs& m, hipStream_t st, const Batch* bt, int nblk) {
  if (m.contracted) return launch_slater_cb<NS, Real>(m, st, bt);
  return m.twist ? launch_slater_tw<NS, Real, true>(m, st, bt, nblk) : launch_slater_tw<NS, Real, false>(m, st, bt, nblk);
}

#define VMC_DISPATCH_NS2(ns, CALL) \
  switch (ns) {                   \
    case 8: { constexpr int NSV = 8; CALL; } \
    case 12: { constexpr int NSV = 12; CALL; } \
    case 16: { constexpr int NSV = 16; CALL; } \
    case 20: { constexpr int NSV = 20; CALL; } \
    case 24: { constexpr int NSV = 24; CALL; } \
    case 27: { constexpr int NSV = 27; CALL; } \
    case 32: { constexpr int NSV = 32; CALL; } \
    case 64: { constexpr int NSV = 64; CALL; } \
    case 128: { constexpr int NSV = 128; CALL; } \
    default: return hipErrorInvalidValue; \
  }

size_t slater_scratch_bytes(int NS, int mixed) {
  if (NS == 128) return mixed ? SlaterLds<128, float>::scr_bytes : SlaterLds<128, double>::scr_bytes;
  return 0;
}

hipError_t launch_ewald_sample(const MeasureArgs& m, const EwaldArgs& e, int mixed, hipStream_t st, const Batch* bt,
                               int nblk) {
  if (e.nmax > NMAXC) return hipErrorInvalidValue;
  if (mixed) { VMC_DISPATCH_NS2(m.NS, return (launch_ewald_t<2 * NSV, float>(m, e, st, bt, nblk))) }
  VMC_DISPATCH_NS2(m.NS, return (launch_ewald_t<2 * NSV, double>(m, e, st, bt, nblk)))
}
template <int NS, bool TW>
hipError_t launch_slater_fp64_tw(const MeasureArgs& m, hipStream_t st, const Batch* bt, int nblk) {
  const Batch b = bt ? *bt : Batch{nullptr, nullptr, 0};
  dim3 grid(bt ? nblk : m.W);
  if (bt)
    hipLaunchKernelGGL((k_slater_sample<NS, double, 1, true, TW>), grid, dim3(256), (SlaterLds<NS, double>::bytes), st, m, b);
  else
    hipLaunchKernelGGL((k_slater_sample<NS, double, 1, false, TW>), grid, dim3(256), (SlaterLds<NS, double>::bytes), st, m, b);
  return hipGetLastError();
}
template <int NS>
hipError_t launch_slater_fp64(const MeasureArgs& m, hipStream_t st, const Batch* bt, int nblk) {
  if (m.contracted) return launch_slater_cb<NS, double>(m, st, bt);
  return m.twist ? launch_slater_fp64_tw<NS, true>(m, st, bt, nblk) : launch_slater_fp64_tw<NS, false>(m, st, bt, nblk);
}
hipError_t launch_slater_sample(const MeasureArgs& m, int mixed, hipStream_t st, const Batch* bt, int nblk) {
  if (mixed) { VMC_DISPATCH_NS2(m.NS, return (launch_slater_t<NSV, float>(m, st, bt, nblk))) }
  if (!m.nimg) return hipErrorInvalidValue;   // FP64 keeps every Gaussian image
  VMC_DISPATCH_NS2(m.NS, return (launch_slater_fp64<NSV>(m, st, bt, nblk)))
}
hipError_t launch_finalize(const MeasureArgs& m, const EwaldArgs& e, int M, double* means, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(m.W), dim3(256), (size_t)e.nk * 2 * sizeof(double), st, m, e, M, means);
  return hipGetLastError();
}
hipError_t launch_proton_setup(int N, double L, const double* R, EwaldArgs& e, double* rho_p, double* Ptab,
                               double* Fconst, double* Vpp, hipStream_t st) {
  hipLaunchKernelGGL(k_proton_phases, dim3(e.nk), dim3(256), 0, st, N, e, R, Ptab, rho_p);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_proton_const, dim3(1), dim3(256), 0, st, N, L, e, R, Ptab, rho_p, Fconst, Vpp);
  return hipGetLastError();
}

}  // namespace vmc
