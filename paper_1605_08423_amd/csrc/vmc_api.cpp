// C ABI of the VMC / Langevin library: contexts, trajectories and the launch
// sequence of one force evaluation.  See include/vmc.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/vmc.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace vmc;
using vmc_host::admit_count;
using vmc_host::build_kvectors;

namespace {

enum KClass { K_SETUP, K_BUILD_A, K_INVERT, K_REFINE, K_SWEEP, K_EWALD, K_SLATER, K_FINALIZE, K_REDUCE, K_SYRK,
              K_LANGEVIN, K_TOY, K_CSWEEP, K_CSLATER, K_J3_INIT, K_J3_GRAD, K_J3_FORCES, K_OPT, K_NCLASS };
const char* kClassName[K_NCLASS] = {"proton_setup", "build_A", "invert", "refine", "sweep_half", "ewald_sample",
                                    "slater_sample", "finalize", "reduce", "syrk", "langevin", "toy",
                                    "csweep", "cslater_sample", "j3_init", "j3_grad", "j3_forces", "opt_sample"};

struct Pending { int cls; hipEvent_t a, b; };
// vmc_energy_forces keeps at most this many sweeps queued ahead of the device, so that
// a cancellation takes effect within that many sweeps.
constexpr int kWindow = 8;
// With a general twist a half-sweep forms its Slater matrix at sweeps 0, kCRefresh,
// 2 kCRefresh, ... (inverting it at sweep 0, refining the carried inverse by a Newton-Schulz
// step at the others) and carries the previous half-sweep's inverse otherwise.
constexpr int kCRefresh = 4;

}  // namespace

struct vmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool profiling = false;
  double ms[K_NCLASS] = {0};
  long long launches[K_NCLASS] = {0};
  std::vector<hipEvent_t> free_events;
  std::vector<Pending> pending;
  int* d_status = nullptr;
  double* lang_work = nullptr;
  size_t lang_work_n = 0;
  double* syrk_work = nullptr;
  size_t syrk_work_n = 0;
  size_t budget = 0, in_use = 0;   // HBM budget of the trajectories (0 = none), bytes they hold
  std::atomic<int> cancel{0};     // set by vmc_cancel (any thread), consumed by vmc_energy_forces
  hipEvent_t window[kWindow] = {nullptr};   // sweeps in flight, see vmc_energy_forces
  double* noalloc_scratch = nullptr;         // the device's static scratch of vmc_langevin_step_noalloc
};

struct vmc_traj {
  vmc_ctx* ctx = nullptr;
  vmc_system sys{};
  int W = 0, N = 0, NS = 0;
  uint32_t seed = 0, traj_id = 0;
  double *pos = nullptr, *Amat = nullptr, *Binv = nullptr, *ldet = nullptr, *sgn = nullptr;
  double *acc = nullptr, *rho_acc = nullptr, *Vs = nullptr, *dVs = nullptr, *Uj = nullptr;
  double *means = nullptr, *f_w = nullptr, *partial = nullptr, *outv = nullptr;
  int64_t* nacc = nullptr;
  int* rflag = nullptr;
  int* qflag = nullptr;           // W + 2: per-walker non-finite flags, then the quarantine counts
  int n_reset = 0;                // walkers re-initialised at the start of the last vmc_energy_forces
  unsigned char* scr = nullptr;   // per-walker scratch of the measurement kernel (N_sigma > 64)
  double* pos_bak = nullptr;      // walker positions at the start of the running call (restored on failure)
  int64_t* nacc_bak = nullptr;    // accepted-move counts of the previous call (restored on failure)
  // Langevin state owned by the trajectory (vmc_traj_set_R, vmc_traj_langevin_step)
  double *Rd = nullptr, *Rprev = nullptr, *Sd = nullptr, *Sprev = nullptr;
  double *j3G = nullptr, *j3scr = nullptr;   // the three-body term: G_a per walker, measurement scratch
  // wavefunction-optimisation statistics (vmc_traj_set_param_stats): E_L per sample, per-walker sums
  double *ELs = nullptr, *popt = nullptr;
  bool param_stats = false, have_popt = false;
  int popt_M = 0;
  size_t bytes = 0;               // device bytes (traj_bytes), counted against the context's budget
  uint32_t lang_step = 0;         // completed vmc_traj_langevin_step calls (the noise counter)
  bool have_R = false, have_prev = false, have_S = false;
  // Ewald tables
  int nk = 0, nslot = 0;
  double *kvec = nullptr, *rho_p = nullptr, *Ptab = nullptr, *Fconst = nullptr, *Vpp = nullptr;
  int *slot = nullptr, *slot_nx0 = nullptr;
  double Vself = 0.0;
  bool have_means = false;
};

namespace {

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return map_err(e_);       \
  } while (0)

int map_err(hipError_t e) {
  if (e == hipErrorOutOfMemory) return VMC_ENOMEM;
  if (e == hipErrorInvalidValue) return VMC_EINVAL;
  if (e == hipErrorNoBinaryForGpu || e == hipErrorInvalidDeviceFunction) return VMC_ENOTBUILT;
  return VMC_EDEVICE;
}

hipEvent_t get_event(vmc_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void flush_timers(vmc_ctx* c) {
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->ms[p.cls] += ms;
      c->launches[p.cls] += 1;
    }
    c->free_events.push_back(p.a);
    c->free_events.push_back(p.b);
  }
  c->pending.clear();
}

// Runs one kernel launch, bracketed by events when profiling.
template <class F>
int timed(vmc_ctx* c, int cls, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->profiling) {
    if (c->pending.size() > 8192) flush_timers(c);
    a = get_event(c);
    b = get_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  hipError_t e = launch();
  if (c->profiling && a && b) {
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({cls, a, b});
  }
  if (e != hipSuccess) return map_err(e);
  return VMC_OK;
}

#define RUN(cls, expr)                                  \
  do {                                                  \
    int rc_ = timed(ctx, cls, [&]() { return (expr); }); \
    if (rc_) return rc_;                                \
  } while (0)

template <class T>
int dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  return e == hipSuccess ? VMC_OK : map_err(e);
}

bool supported_ns(int ns) {
  return ns == 8 || ns == 12 || ns == 16 || ns == 20 || ns == 24 || ns == 27 || ns == 32 || ns == 64 || ns == 128;
}

constexpr double kContractedZ2 = 0.3382168;   // the smaller exponent of the contracted orbital

bool has_j3(const vmc_system& s) { return s.j3_f[0] != 0.0 || s.j3_f[1] != 0.0 || s.j3_f[2] != 0.0; }
// the Jastrow-orbital terms (three-body F, one-body orbital part f) share the orbitals, the per-walker
// nucleus sums G_a and the measurement kernels
bool has_jorb(const vmc_system& s) { return has_j3(s) || s.j1_f[0] != 0.0 || s.j1_f[1] != 0.0; }

int check_sys(const vmc_system* s) {
  if (!s) return VMC_EINVAL;
  if (s->n_protons < 2 || (s->n_protons & 1) || !supported_ns(s->n_protons / 2)) return VMC_EINVAL;
  if (!(s->box_L > 0.0) || !(s->ewald_kappa > 0.0) || s->ewald_nmax < 1 || s->ewald_nmax > 12) return VMC_EINVAL;
  if (s->precision != VMC_FP64 && s->precision != VMC_MIXED) return VMC_EINVAL;
  if (s->refine_tol != s->refine_tol) return VMC_EINVAL;
  if (!(s->b >= 0.0) || !std::isfinite(s->b)) return VMC_EINVAL;
  if (!(s->j1_b1 >= 0.0) || !std::isfinite(s->j1_b1)) return VMC_EINVAL;
  if (s->twist < 0 || s->twist > 7) return VMC_EINVAL;
  if (s->general_twist != 0 && s->general_twist != 1) return VMC_EINVAL;
  if (s->general_twist) {
    if (s->precision != VMC_FP64 || s->twist != 0 || s->n_protons / 2 > 64) return VMC_EINVAL;
    for (int m = 0; m < 3; ++m)
      if (!std::isfinite(s->theta[m])) return VMC_EINVAL;
  }
  if (s->contracted != 0 && s->contracted != 1) return VMC_EINVAL;
  for (int m = 0; m < 3; ++m)
    if (!std::isfinite(s->j3_f[m])) return VMC_EINVAL;
  for (int m = 0; m < 2; ++m)
    if (!std::isfinite(s->j1_f[m])) return VMC_EINVAL;
  if (has_jorb(*s) && s->n_protons / 2 > 64) return VMC_EINVAL;
  if (s->contracted) {
    // the images |n| <= 1 of the diffuse r^2 e^{-Z2 r^2} reach FP64 resolution only if Z2 (1.5 L)^2 >= 36
    const double h = 1.5 * s->box_L;
    if (s->twist != 0 || s->n_protons / 2 > 64 || !std::isfinite(s->eta) ||
        kContractedZ2 * h * h < 36.0)
      return VMC_EINVAL;
  }
  return VMC_OK;
}

bool is_complex(const vmc_system& s) { return s.general_twist == 1; }

TwistArgs twist_args(const vmc_system& s) {
  TwistArgs tw{};
  for (int m = 0; m < 3; ++m) {
    tw.th[m] = s.theta[m];
    tw.c[m] = std::cos(s.theta[m]);
    tw.s[m] = std::sin(s.theta[m]);
  }
  return tw;
}

// Per-walker measurement scratch and the doubles of the inverse per walker and spin.
size_t meas_scratch_bytes(const vmc_system& s) {
  const int NS = s.n_protons / 2;
  return is_complex(s) ? cslater_scratch_bytes(NS) : slater_scratch_bytes(NS, s.precision == VMC_MIXED);
}
size_t inv_doubles(const vmc_system& s) {
  const size_t NS = s.n_protons / 2;
  return (is_complex(s) ? 2 : 1) * NS * NS;
}

// Gaussian images kept per axis: all three (n = -1, 0, 1) unless the mode is mixed and
// every dropped image is below e^{-zeta_min (L/2)^2} <= e^{-23} (under FP32 resolution).
int image_rule(const vmc_system& s, const double* zeta_host) {
  if (s.precision != VMC_MIXED) return 1;
  double zmin = zeta_host[0];
  for (int i = 0; i < s.n_protons; ++i) zmin = std::min(zmin, zeta_host[i]);
  const double h = 0.5 * s.box_L;
  return (zmin * h * h >= 23.0) ? 0 : 1;
}
int image_count(vmc_traj* t, const double* zeta_dev, int* nimg) {
  *nimg = 1;
  // the contracted orbital keeps all three images (its r^2 e^{-Z2 r^2} part is diffuse)
  if (t->sys.precision != VMC_MIXED || t->sys.contracted) return VMC_OK;
  std::vector<double> z(t->N);
  HIPCHK(hipMemcpyAsync(z.data(), zeta_dev, t->N * sizeof(double), hipMemcpyDeviceToHost, t->ctx->stream));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  *nimg = image_rule(t->sys, z.data());
  return VMC_OK;
}

// The one-body term -(2Z)^{3/4} u_1((2Z)^{1/4} rho) with Z = 1 equals
// -(1 - e^{-beta rho}) / beta for beta = b_1 (2Z)^{1/4}; the kernels take beta.
double j1_beta(const vmc_system& s) { return s.j1_b1 > 0.0 ? s.j1_b1 * std::pow(2.0, 0.25) : 0.0; }

WalkerArgs walker_args(vmc_traj* t, const double* R, const double* C, const double* zeta, int nimg) {
  WalkerArgs a{};
  a.W = t->W; a.N = t->N; a.NS = t->NS; a.nimg = nimg;
  a.L = t->sys.box_L; a.invL = 1.0 / t->sys.box_L;
  a.R = R; a.zeta = zeta; a.C = C;
  a.a_par = t->sys.a_par; a.a_anti = t->sys.a_anti; a.b = t->sys.b;
  a.j1_beta = j1_beta(t->sys);
  a.twist = t->sys.twist;
  a.pos = t->pos; a.Amat = t->Amat; a.Binv = t->Binv; a.ldet = t->ldet; a.sgn = t->sgn;
  a.status = t->ctx->d_status; a.nacc = t->nacc; a.rflag = t->rflag;
  // N_sigma > 64: the refinement's R uses the first N_sigma^2 doubles of the walker's
  // measurement scratch (the measurement never runs during a refresh)
  a.rscr = reinterpret_cast<double*>(t->scr);
  a.rscr_stride = slater_scratch_bytes(t->NS, t->sys.precision == VMC_MIXED) / sizeof(double);
  a.contracted = t->sys.contracted;
  a.eta = t->sys.eta;
  a.j3 = has_jorb(t->sys);
  for (int q = 0; q < 3; ++q) a.j3f[q] = t->sys.j3_f[q];
  for (int q = 0; q < 2; ++q) a.j1f[q] = t->sys.j1_f[q];
  a.j3G = t->j3G;
  return a;
}

MeasureArgs measure_args(vmc_traj* t, const double* R, const double* C, const double* zeta, int nimg) {
  MeasureArgs m{};
  m.W = t->W; m.N = t->N; m.NS = t->NS; m.nimg = nimg;
  m.L = t->sys.box_L; m.invL = 1.0 / t->sys.box_L;
  m.R = R; m.zeta = zeta; m.C = C;
  m.a_par = t->sys.a_par; m.a_anti = t->sys.a_anti; m.b = t->sys.b;
  m.j1_beta = j1_beta(t->sys);
  m.twist = t->sys.twist;
  m.pos = t->pos; m.Binv = t->Binv; m.Vs = t->Vs; m.dVs = t->dVs; m.Uj = t->Uj;
  m.acc = t->acc; m.rho_acc = t->rho_acc; m.scr = t->scr;
  m.contracted = t->sys.contracted;
  m.eta = t->sys.eta;
  m.j3 = has_jorb(t->sys);
  for (int q = 0; q < 3; ++q) m.j3f[q] = t->sys.j3_f[q];
  for (int q = 0; q < 2; ++q) m.j1f[q] = t->sys.j1_f[q];
  m.j3scr = t->j3scr;
  m.ELs = t->param_stats ? t->ELs : nullptr;
  m.popt = t->popt;
  return m;
}

EwaldArgs ewald_args(vmc_traj* t) {
  EwaldArgs e{};
  e.nk = t->nk; e.nslot = t->nslot; e.nmax = t->sys.ewald_nmax; e.kappa = t->sys.ewald_kappa;
  e.kvec = t->kvec; e.slot = t->slot; e.slot_nx0 = t->slot_nx0;
  e.rho_p = t->rho_p; e.Ptab = t->Ptab; e.Vpp = t->Vpp; e.Vself = t->Vself; e.Fconst = t->Fconst;
  return e;
}

// Proton-only Ewald quantities at R: rho_p, e^{ikR}, constant gradient, V_pp (all on the device).
int proton_setup(vmc_traj* t, const double* R) {
  vmc_ctx* ctx = t->ctx;
  EwaldArgs e = ewald_args(t);
  RUN(K_SETUP, launch_proton_setup(t->N, t->sys.box_L, R, e, t->rho_p, t->Ptab, t->Fconst, t->Vpp, ctx->stream));
  return VMC_OK;
}

int check_singular(vmc_ctx* ctx) {
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return st ? VMC_ESINGULAR : VMC_OK;
}

// One measured sample for every walker.
int measure(vmc_traj* t, const MeasureArgs& m, const EwaldArgs& e) {
  vmc_ctx* ctx = t->ctx;
  const int mixed = t->sys.precision == VMC_MIXED;
  if (m.j3) RUN(K_J3_GRAD, launch_j3_grad(m, mixed, ctx->stream));
  RUN(K_EWALD, launch_ewald_sample(m, e, mixed, ctx->stream));
  RUN(K_SLATER, launch_slater_sample(m, mixed, ctx->stream));
  if (m.j3) RUN(K_J3_FORCES, launch_j3_forces(m, mixed, ctx->stream));
  if (m.ELs) RUN(K_OPT, launch_opt_sample(m, mixed, ctx->stream));
  return VMC_OK;
}
int measure_c(vmc_traj* t, const MeasureArgs& m, const EwaldArgs& e, const TwistArgs& tw) {
  vmc_ctx* ctx = t->ctx;
  if (m.j3) RUN(K_J3_GRAD, launch_j3_grad(m, 0, ctx->stream));
  RUN(K_EWALD, launch_ewald_sample(m, e, 0, ctx->stream));
  RUN(K_CSLATER, launch_cslater_sample(m, tw, ctx->stream));
  if (m.j3) RUN(K_J3_FORCES, launch_j3_forces(m, 0, ctx->stream));
  if (m.ELs) RUN(K_OPT, launch_opt_sample(m, 0, ctx->stream));
  return VMC_OK;
}

// Device bytes vmc_traj_create allocates for this system and walker count.
size_t traj_bytes(const vmc_system& s, int W) {
  std::vector<double> kv;
  std::vector<int> slots, nx0;
  build_kvectors(s, kv, slots, nx0);
  const size_t N = s.n_protons, n3 = 3 * N, nk = kv.size() / 4, Wz = W;
  const size_t amat = is_complex(s) ? 1 : Wz * 2 * inv_doubles(s);
  const size_t d = 2 * Wz * N * 3 + amat + Wz * 2 * inv_doubles(s) + 2 * Wz * 2 + Wz * (2 + 9 * N) + Wz * nk * 2 + Wz +
                   Wz * n3 + Wz + Wz * (1 + 3 * n3) + Wz * n3 + reduce_partial_doubles(W, (int)n3) + 3 + n3 +
                   kv.size() + 2 * nk + nk * N * 2 + n3 + 1 + 2 * n3 + 2 * n3 * n3;
  const size_t j3 = has_jorb(s) ? Wz * (2 * N + j3_measure_doubles((int)N)) : 0;
  const size_t opt = Wz * (1 + kOptStats);
  return (d + j3 + opt) * sizeof(double) + 2 * Wz * sizeof(int64_t) +
         (3 * Wz + 2 + slots.size() + nx0.size()) * sizeof(int) + Wz * meas_scratch_bytes(s);
}

void free_traj(vmc_traj* t) {
  if (!t) return;
  if (t->ctx) t->ctx->in_use -= t->bytes;
  void* ptrs[] = {t->pos, t->Amat, t->Binv, t->ldet, t->sgn, t->acc, t->rho_acc, t->Vs, t->dVs, t->Uj,
                  t->means, t->f_w, t->partial, t->outv, t->nacc, t->kvec, t->rho_p, t->Ptab, t->Fconst,
                  t->Vpp, t->slot, t->slot_nx0, t->rflag, t->qflag, t->scr, t->pos_bak, t->nacc_bak,
                  t->Rd, t->Rprev, t->Sd, t->Sprev, t->j3G, t->j3scr, t->ELs, t->popt};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete t;
}

}  // namespace

extern "C" {

const char* vmc_strerror(int code) {
  switch (code) {
    case VMC_OK: return "ok";
    case VMC_EINVAL: return "invalid argument";
    case VMC_ENOMEM: return "device out of memory";
    case VMC_ENOTSPD: return "S is not positive definite";
    case VMC_ESINGULAR: return "singular Slater matrix at an inverse refresh";
    case VMC_EDEVICE: return "HIP runtime error";
    case VMC_ENOTBUILT: return "no device code for this GPU";
    case VMC_ECANCELLED: return "cancelled";
    case VMC_ENOCONV: return "host eigen-solver failed";
    default: return "unknown error";
  }
}

int vmc_supported_n(int n) { return (n > 0 && !(n & 1) && supported_ns(n / 2)) ? 1 : 0; }

// Device address of each device's copy of the allocation-free step's static scratch, taken once
// per device (with that device current) by the first vmc_create on it.
static std::mutex g_scratch_mu;
static double* g_scratch[256] = {nullptr};

int vmc_create(vmc_ctx** out, int device) {
  if (!out) return VMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev || device >= 256) return VMC_EINVAL;
  HIPCHK(hipSetDevice(device));
  double* scratch_dev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) HIPCHK(langevin_scratch_address(&g_scratch[device]));
    scratch_dev = g_scratch[device];
  }
  vmc_ctx* c = new (std::nothrow) vmc_ctx();
  if (!c) return VMC_ENOMEM;
  c->device = device;
  c->noalloc_scratch = scratch_dev;
  if (dalloc(&c->d_status, 1)) { delete c; return VMC_ENOMEM; }
  *out = c;
  return VMC_OK;
}

void vmc_destroy(vmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  flush_timers(c);
  for (hipEvent_t e : c->free_events) (void)hipEventDestroy(e);
  if (c->d_status) (void)hipFree(c->d_status);
  if (c->lang_work) (void)hipFree(c->lang_work);
  if (c->syrk_work) (void)hipFree(c->syrk_work);
  for (hipEvent_t e : c->window)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int vmc_cancel(vmc_ctx* c) {
  if (!c) return VMC_EINVAL;
  c->cancel.store(1);
  return VMC_OK;
}

int vmc_set_hbm_budget(vmc_ctx* c, size_t bytes) {
  if (!c) return VMC_EINVAL;
  c->budget = bytes;
  return VMC_OK;
}

int vmc_hbm_in_use(vmc_ctx* c, size_t* in_use) {
  if (!c || !in_use) return VMC_EINVAL;
  *in_use = c->in_use;
  return VMC_OK;
}

size_t vmc_traj_bytes(const vmc_system* sys, int W) {
  if (check_sys(sys) || W < 1) return 0;
  return traj_bytes(*sys, W);
}

int vmc_set_stream(vmc_ctx* c, void* s) {
  if (!c) return VMC_EINVAL;
  c->stream = (hipStream_t)s;
  return VMC_OK;
}

int vmc_set_profiling(vmc_ctx* c, int on) {
  if (!c) return VMC_EINVAL;
  if (!on) flush_timers(c);
  c->profiling = on != 0;
  return VMC_OK;
}

int vmc_kernel_times(vmc_ctx* c, const char** names, double* total_ms, long long* launches, int max_n) {
  if (!c) return VMC_EINVAL;
  flush_timers(c);
  int n = std::min(max_n, (int)K_NCLASS);
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = kClassName[i];
    if (total_ms) total_ms[i] = c->ms[i];
    if (launches) launches[i] = c->launches[i];
  }
  return n;
}

int vmc_reset_kernel_times(vmc_ctx* c) {
  if (!c) return VMC_EINVAL;
  flush_timers(c);
  for (int i = 0; i < K_NCLASS; ++i) { c->ms[i] = 0; c->launches[i] = 0; }
  return VMC_OK;
}

int vmc_traj_create(vmc_ctx* ctx, const vmc_system* sys, int W, uint32_t seed, uint32_t traj_id, vmc_traj** out) {
  if (!ctx || !out || W < 1) return VMC_EINVAL;
  *out = nullptr;
  int rc = check_sys(sys);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  const size_t bytes = traj_bytes(*sys, W);
  if (ctx->budget && ctx->in_use + bytes > ctx->budget) return VMC_ENOMEM;
  vmc_traj* t = new (std::nothrow) vmc_traj();
  if (!t) return VMC_ENOMEM;
  t->ctx = ctx; t->sys = *sys; t->W = W; t->N = sys->n_protons; t->NS = t->N / 2;
  t->bytes = bytes;
  ctx->in_use += bytes;
  t->seed = seed; t->traj_id = traj_id;
  std::vector<double> kv;
  std::vector<int> slots, nx0;
  build_kvectors(*sys, kv, slots, nx0);
  t->nk = (int)(kv.size() / 4);
  t->nslot = (int)nx0.size();
  t->Vself = -sys->ewald_kappa / std::sqrt(M_PI) * (2.0 * t->N);
  const size_t N = t->N, NS = t->NS, n3 = 3 * N;
  // the complex path keeps no Slater matrices between launches (one placeholder double)
  bool ok = !dalloc(&t->pos, W * N * 3) && !dalloc(&t->Amat, is_complex(*sys) ? 1 : (size_t)W * 2 * NS * NS) &&
            !dalloc(&t->Binv, (size_t)W * 2 * inv_doubles(*sys)) && !dalloc(&t->ldet, (size_t)W * 2) &&
            !dalloc(&t->sgn, (size_t)W * 2) && !dalloc(&t->acc, (size_t)W * (2 + 9 * N)) &&
            !dalloc(&t->rho_acc, (size_t)W * t->nk * 2) && !dalloc(&t->Vs, (size_t)W) &&
            !dalloc(&t->dVs, (size_t)W * n3) && !dalloc(&t->Uj, (size_t)W) &&
            !dalloc(&t->means, (size_t)W * (1 + 3 * n3)) && !dalloc(&t->f_w, (size_t)W * n3) &&
            !dalloc(&t->partial, reduce_partial_doubles(W, (int)n3)) && !dalloc(&t->outv, 3 + n3) &&
            !dalloc(&t->nacc, (size_t)W) && !dalloc(&t->rflag, (size_t)W * 2) && !dalloc(&t->qflag, (size_t)W + 2) &&
            !dalloc(&t->kvec, kv.size()) && !dalloc(&t->rho_p, 2 * t->nk) &&
            !dalloc(&t->Ptab, (size_t)t->nk * N * 2) && !dalloc(&t->Fconst, n3) && !dalloc(&t->Vpp, 1) &&
            !dalloc(&t->slot, slots.size()) && !dalloc(&t->slot_nx0, nx0.size()) &&
            !dalloc(&t->pos_bak, W * N * 3) && !dalloc(&t->nacc_bak, (size_t)W) && !dalloc(&t->Rd, n3) &&
            !dalloc(&t->Rprev, n3) && !dalloc(&t->Sd, n3 * n3) && !dalloc(&t->Sprev, n3 * n3) &&
            !dalloc(&t->ELs, (size_t)W) && !dalloc(&t->popt, (size_t)W * kOptStats);
  const size_t scr = meas_scratch_bytes(*sys);
  if (ok && scr) ok = !dalloc(&t->scr, (size_t)W * scr);
  if (ok && has_jorb(*sys))
    ok = !dalloc(&t->j3G, (size_t)W * N * 2) && !dalloc(&t->j3scr, (size_t)W * j3_measure_doubles((int)N));
  if (!ok) { free_traj(t); return VMC_ENOMEM; }
  if (hipMemcpy(t->kvec, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->slot, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->slot_nx0, nx0.data(), nx0.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(t->nacc, 0, W * sizeof(int64_t)) != hipSuccess ||
      hipMemset(t->Rd, 0, n3 * sizeof(double)) != hipSuccess ||
      hipMemset(t->Rprev, 0, n3 * sizeof(double)) != hipSuccess ||
      hipMemset(t->Sd, 0, n3 * n3 * sizeof(double)) != hipSuccess ||
      hipMemset(t->Sprev, 0, n3 * n3 * sizeof(double)) != hipSuccess ||
      hipMemset(t->outv, 0, (3 + n3) * sizeof(double)) != hipSuccess) {
    free_traj(t);
    return VMC_EDEVICE;
  }
  *out = t;
  return VMC_OK;
}

void vmc_traj_destroy(vmc_traj* t) { free_traj(t); }

int vmc_traj_set_walkers(vmc_traj* t, const double* pos_dev) {
  if (!t || !pos_dev) return VMC_EINVAL;
  HIPCHK(hipMemcpyAsync(t->pos, pos_dev, (size_t)t->W * t->N * 3 * sizeof(double), hipMemcpyDeviceToDevice,
                        t->ctx->stream));
  return VMC_OK;
}

// Checkpoint format: vmc_host::CkptHeader and its payload (host.hpp), sealed by a checksum.
static size_t ckpt_bytes(const vmc_traj* t) {
  return sizeof(vmc_host::CkptHeader) + vmc_host::ckpt_payload_bytes(t->N, t->W);
}

// The device arrays of the payload in their order, with their sizes in bytes (the
// accepted-move counts come last).
static int ckpt_parts(vmc_traj* t, double* ptr[7], size_t nb[7]) {
  const size_t W = t->W, N = t->N, n3 = 3 * N;
  double* p[7] = {t->pos, t->means, t->f_w, t->outv, t->Rd, t->Rprev, t->Sd};
  const size_t b[7] = {W * N * 3, W * (1 + 9 * N), W * n3, 3 + n3, n3, n3, n3 * n3};
  for (int k = 0; k < 7; ++k) {
    ptr[k] = p[k];
    nb[k] = b[k] * sizeof(double);
  }
  return 7;
}

int vmc_traj_save(vmc_traj* t, void* buf, size_t* len) {
  if (!t || !len) return VMC_EINVAL;
  const size_t need = ckpt_bytes(t);
  if (!buf) { *len = need; return VMC_OK; }
  if (*len < need) { *len = need; return VMC_EINVAL; }
  HIPCHK(hipSetDevice(t->ctx->device));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  vmc_host::CkptHeader h;
  vmc_host::ckpt_init_header(&h, t->N, t->W);
  h.seed = t->seed; h.traj_id = t->traj_id; h.lang_step = t->lang_step;
  h.precision = t->sys.precision; h.nmax = t->sys.ewald_nmax; h.twist = t->sys.twist;
  h.have_means = t->have_means; h.have_R = t->have_R; h.have_prev = t->have_prev; h.have_S = t->have_S;
  h.box_L = t->sys.box_L; h.kappa = t->sys.ewald_kappa; h.a_par = t->sys.a_par; h.a_anti = t->sys.a_anti;
  h.b = t->sys.b; h.j1_b1 = t->sys.j1_b1;
  h.general_twist = t->sys.general_twist; h.contracted = t->sys.contracted; h.eta = t->sys.eta;
  for (int q = 0; q < 3; ++q) { h.theta[q] = t->sys.theta[q]; h.j3_f[q] = t->sys.j3_f[q]; }
  for (int q = 0; q < 2; ++q) h.j1_f[q] = t->sys.j1_f[q];
  unsigned char* p = static_cast<unsigned char*>(buf);
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  double* src[7];
  size_t nb[7];
  const int np = ckpt_parts(t, src, nb);
  for (int k = 0; k < np; ++k) {
    HIPCHK(hipMemcpy(p, src[k], nb[k], hipMemcpyDeviceToHost));
    p += nb[k];
  }
  // S_prev sits between S and the counts in the payload
  const size_t n3 = 3 * (size_t)t->N;
  HIPCHK(hipMemcpy(p, t->Sprev, n3 * n3 * sizeof(double), hipMemcpyDeviceToHost));
  p += n3 * n3 * sizeof(double);
  HIPCHK(hipMemcpy(p, t->nacc, (size_t)t->W * sizeof(int64_t), hipMemcpyDeviceToHost));
  vmc_host::ckpt_seal(buf);
  *len = need;
  return VMC_OK;
}

// Shared by vmc_traj_load and vmc_traj_load_rescaled.  rescale: the checkpoint's box side may
// differ from the trajectory's (its Ewald kappa then follows the box); walker coordinates are
// multiplied by L / L*, the accumulators of the old density are cleared and so is the
// Langevin state (the caller sets the scaled R).
static int traj_load(vmc_traj* t, const void* buf, size_t len, bool rescale) {
  if (!t || !buf) return VMC_EINVAL;
  vmc_host::CkptHeader h;
  if (vmc_host::ckpt_validate(buf, len, &h) != VMC_OK) return VMC_EINVAL;
  const vmc_system& s = t->sys;
  // the system must match; the variational Jastrow parameters (b, b_1, F, f) come from the
  // checkpoint, as vmc_traj_set_jastrow would set them (an optimised wavefunction resumes)
  if (h.n != t->N || h.w != t->W || h.precision != s.precision || h.nmax != s.ewald_nmax || h.twist != s.twist ||
      h.general_twist != s.general_twist || h.contracted != s.contracted || h.a_par != s.a_par ||
      h.a_anti != s.a_anti)
    return VMC_EINVAL;
  if (s.contracted && h.eta != s.eta) return VMC_EINVAL;
  for (int q = 0; q < 3; ++q)
    if (s.general_twist && h.theta[q] != s.theta[q]) return VMC_EINVAL;
  vmc_system js = s;
  js.b = h.b;
  js.j1_b1 = h.j1_b1;
  for (int q = 0; q < 3; ++q) js.j3_f[q] = h.j3_f[q];
  for (int q = 0; q < 2; ++q) js.j1_f[q] = h.j1_f[q];
  if (check_sys(&js) || (js.j1_b1 > 0.0) != (s.j1_b1 > 0.0) || (has_jorb(js) && !t->j3G)) return VMC_EINVAL;
  if (!rescale && (h.box_L != s.box_L || h.kappa != s.ewald_kappa)) return VMC_EINVAL;
  if (rescale && !(h.box_L > 0.0 && std::isfinite(h.box_L))) return VMC_EINVAL;
  HIPCHK(hipSetDevice(t->ctx->device));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  const unsigned char* p = static_cast<const unsigned char*>(buf) + sizeof h;
  double* dst[7];
  size_t nb[7];
  const int np = ckpt_parts(t, dst, nb);
  const size_t W = t->W, n3 = 3 * (size_t)t->N;
  if (rescale) {
    // x -> (L / L*) x keeps every coordinate in [0, L) and every walker's shape
    const double sc = s.box_L / h.box_L;
    std::vector<double> x(nb[0] / sizeof(double));
    std::memcpy(x.data(), p, nb[0]);
    for (double& v : x) v *= sc;
    HIPCHK(hipMemcpy(t->pos, x.data(), nb[0], hipMemcpyHostToDevice));
    HIPCHK(hipMemset(t->nacc, 0, W * sizeof(int64_t)));
    t->have_means = t->have_R = t->have_prev = t->have_S = false;
  } else {
    for (int k = 0; k < np; ++k) {
      HIPCHK(hipMemcpy(dst[k], p, nb[k], hipMemcpyHostToDevice));
      p += nb[k];
    }
    HIPCHK(hipMemcpy(t->Sprev, p, n3 * n3 * sizeof(double), hipMemcpyHostToDevice));
    p += n3 * n3 * sizeof(double);
    HIPCHK(hipMemcpy(t->nacc, p, W * sizeof(int64_t), hipMemcpyHostToDevice));
    t->have_means = h.have_means != 0;
    t->have_R = h.have_R != 0;
    t->have_prev = h.have_prev != 0;
    t->have_S = h.have_S != 0;
  }
  t->seed = h.seed;
  t->traj_id = h.traj_id;
  t->lang_step = h.lang_step;
  t->sys = js;
  t->have_popt = false;
  return VMC_OK;
}

int vmc_traj_load(vmc_traj* t, const void* buf, size_t len) { return traj_load(t, buf, len, false); }

int vmc_traj_load_rescaled(vmc_traj* t, const void* buf, size_t len) { return traj_load(t, buf, len, true); }

int vmc_traj_walkers_reset(vmc_traj* t, int* n_reset) {
  if (!t || !n_reset) return VMC_EINVAL;
  *n_reset = t->n_reset;
  return VMC_OK;
}

int vmc_traj_get_walkers(vmc_traj* t, double* pos_dev) {
  if (!t || !pos_dev) return VMC_EINVAL;
  HIPCHK(hipMemcpyAsync(pos_dev, t->pos, (size_t)t->W * t->N * 3 * sizeof(double), hipMemcpyDeviceToDevice,
                        t->ctx->stream));
  return VMC_OK;
}

// Puts the walkers and accepted-move counts back to what they were when the call started
// (the call's failure leaves the trajectory as it found it).
static int restore_walkers(vmc_traj* t) {
  hipStream_t st = t->ctx->stream;
  HIPCHK(hipMemcpyAsync(t->pos, t->pos_bak, (size_t)t->W * t->N * 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(t->nacc, t->nacc_bak, (size_t)t->W * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return VMC_OK;
}

static int fail_restore(vmc_traj* t, int code) {
  const int rc = restore_walkers(t);
  return rc ? rc : code;
}

int vmc_energy_forces(vmc_traj* t, const double* R_in, const double* C, const double* zeta, int n_equil,
                      int n_sweeps, double step_delta, uint32_t step, double* out_dev) {
  if (!t || !C || !zeta || !out_dev || n_equil < 0 || n_sweeps < 1 || !(step_delta > 0.0)) return VMC_EINVAL;
  if (!R_in && !t->have_R) return VMC_EINVAL;
  const double* R = R_in ? R_in : t->Rd;
  if (step == VMC_STEP_TRAJ) step = t->lang_step;
  vmc_ctx* ctx = t->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int mixed = t->sys.precision == VMC_MIXED;
  const size_t N = t->N, n3 = 3 * N, W = t->W;
  for (hipEvent_t& e : ctx->window)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // the state a failure restores
  HIPCHK(hipMemcpyAsync(t->pos_bak, t->pos, W * N * 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(t->nacc_bak, t->nacc, W * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  // quarantine: a walker whose coordinates are not all finite restarts from a copy of the
  // next finite walker; every walker bad is an argument error (nothing is changed)
  HIPCHK(hipMemsetAsync(t->qflag + W, 0, 2 * sizeof(int), st));
  RUN(K_SETUP, launch_walker_quarantine((int)W, (int)N, t->pos, t->qflag, t->qflag + W, st));
  int qc[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(qc, t->qflag + W, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (qc[1] > 0) return VMC_EINVAL;     // no walker was touched: the quarantine had no source
  t->n_reset = qc[0];
  int rc = proton_setup(t, R);
  if (rc) return fail_restore(t, rc);
  int nimg = 1;
  rc = image_count(t, zeta, &nimg);
  if (rc) return fail_restore(t, rc);
  HIPCHK(hipMemsetAsync(t->acc, 0, W * (2 + 9 * N) * sizeof(double), st));
  HIPCHK(hipMemsetAsync(t->rho_acc, 0, W * t->nk * 2 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(t->nacc, 0, W * sizeof(int64_t), st));
  HIPCHK(hipMemsetAsync(t->rflag, 0, W * 2 * sizeof(int), st));
  HIPCHK(hipMemsetAsync(ctx->d_status, 0, sizeof(int), st));
  t->have_popt = false;
  if (t->param_stats) HIPCHK(hipMemsetAsync(t->popt, 0, W * kOptStats * sizeof(double), st));
  WalkerArgs a = walker_args(t, R, C, zeta, nimg);
  MeasureArgs m = measure_args(t, R, C, zeta, nimg);
  EwaldArgs e = ewald_args(t);
  const bool cplx = is_complex(t->sys);
  const TwistArgs tw = twist_args(t->sys);
  if (!cplx) RUN(K_BUILD_A, launch_build_A(a, mixed, st));
  if (a.j3) RUN(K_J3_INIT, launch_j3_init(a, st));
  const double rtol = t->sys.refine_tol == 0.0 ? 1e-7 : t->sys.refine_tol;
  const int total = n_equil + n_sweeps;
  for (int s = 0; s < total; ++s) {
    // keep at most kWindow sweeps queued; a pending cancellation stops the call here
    if (s >= kWindow) HIPCHK(hipEventSynchronize(ctx->window[s % kWindow]));
    if (ctx->cancel.exchange(0)) {
      HIPCHK(hipStreamSynchronize(st));
      return fail_restore(t, VMC_ECANCELLED);
    }
    if (cplx) {
      // each half-sweep refreshes its own spin's inverse where due; a singular start fails after
      // the first sweep and the walkers are restored
      for (int sp = 0; sp < 2; ++sp) {
        SweepArgs sa{sp, s, step, t->seed, t->traj_id, step_delta};
        // the first sweep inverts afresh (new R and orbitals), later refreshes refine the carried
        // inverse unless refinement is switched off
        const int mode = s % kCRefresh != 0 ? 0 : (s == 0 || rtol < 0.0) ? 1 : 2;
        RUN(K_CSWEEP, launch_csweep(a, sa, tw, mode, 1, rtol, st));
      }
      if (s == 0) {
        rc = check_singular(ctx);
        if (rc) return fail_restore(t, rc);
      }
      if (s >= n_equil) {
        rc = measure_c(t, m, e, tw);
        if (rc) return rc;
      }
      HIPCHK(hipEventRecord(ctx->window[s % kWindow], st));
      continue;
    }
    if (s == 0) {
      // elimination for both spins (a half-sweep over one spin leaves the other spin's matrix
      // as it is); a singular start, e.g. two same-spin electrons at one point, fails here,
      // before any move
      RUN(K_INVERT, launch_invert(a, 0, 2, 0, st));
      rc = check_singular(ctx);
      if (rc) return fail_restore(t, rc);
    }
    for (int sp = 0; sp < 2; ++sp) {
      if (s > 0 && rtol < 0.0) {
        RUN(K_INVERT, launch_invert(a, sp, sp + 1, 0, st));
      } else if (s > 0) {
        RUN(K_REFINE, launch_refine(a, sp, rtol, st));
        RUN(K_INVERT, launch_invert(a, sp, sp + 1, 1, st));
      }
      SweepArgs sa{sp, s, step, t->seed, t->traj_id, step_delta};
      RUN(K_SWEEP, launch_sweep(a, sa, mixed, st));
    }
    if (s >= n_equil) {
      rc = measure(t, m, e);
      if (rc) return rc;
    }
    HIPCHK(hipEventRecord(ctx->window[s % kWindow], st));
  }
  // a zero pivot at a later refresh: nothing of this call is kept
  rc = check_singular(ctx);
  if (rc) return fail_restore(t, rc);
  RUN(K_FINALIZE, launch_finalize(m, e, n_sweeps, t->means, st));
  RUN(K_REDUCE, launch_reduce((int)W, (int)n3, t->means, t->nacc, (double)N * total, t->f_w, t->partial, t->outv, st));
  HIPCHK(hipMemcpyAsync(out_dev, t->outv, (3 + n3) * sizeof(double), hipMemcpyDeviceToDevice, st));
  t->have_means = true;
  t->have_S = false;
  t->have_popt = t->param_stats;
  t->popt_M = n_sweeps;
  return VMC_OK;
}

int vmc_traj_set_param_stats(vmc_traj* t, int on) {
  if (!t || (on != 0 && on != 1)) return VMC_EINVAL;
  t->param_stats = on == 1;
  t->have_popt = false;
  return VMC_OK;
}

int vmc_traj_param_stats(vmc_traj* t, double* stats_dev) {
  if (!t || !stats_dev || !t->have_popt) return VMC_EINVAL;
  HIPCHK(hipSetDevice(t->ctx->device));
  vmc_ctx* ctx = t->ctx;
  RUN(K_REDUCE, launch_opt_reduce(t->W, t->popt_M, t->popt, stats_dev, ctx->stream));
  return VMC_OK;
}

int vmc_traj_set_jastrow(vmc_traj* t, double b, double j1_b1, const double* j3_f, const double* j1_f) {
  if (!t || !j3_f) return VMC_EINVAL;
  vmc_system s = t->sys;
  s.b = b;
  s.j1_b1 = j1_b1;
  for (int q = 0; q < 3; ++q) s.j3_f[q] = j3_f[q];
  if (j1_f)
    for (int q = 0; q < 2; ++q) s.j1_f[q] = j1_f[q];
  if (check_sys(&s)) return VMC_EINVAL;
  // the one-body term stays on or off; the three-body term may change freely only where its
  // per-walker memory exists (it was on at creation)
  if ((j1_b1 > 0.0) != (t->sys.j1_b1 > 0.0)) return VMC_EINVAL;
  if (has_jorb(s) && !t->j3G) return VMC_EINVAL;
  t->sys = s;
  t->have_means = false;
  t->have_popt = false;
  return VMC_OK;
}

int vmc_traj_walker_means(vmc_traj* t, double* means_dev) {
  if (!t || !means_dev || !t->have_means) return VMC_EINVAL;
  HIPCHK(hipMemcpyAsync(means_dev, t->means, (size_t)t->W * (1 + 9 * t->N) * sizeof(double),
                        hipMemcpyDeviceToDevice, t->ctx->stream));
  return VMC_OK;
}

int vmc_traj_walker_forces(vmc_traj* t, double* f_w_dev) {
  if (!t || !f_w_dev || !t->have_means) return VMC_EINVAL;
  HIPCHK(hipMemcpyAsync(f_w_dev, t->f_w, (size_t)t->W * 3 * t->N * sizeof(double), hipMemcpyDeviceToDevice,
                        t->ctx->stream));
  return VMC_OK;
}

int vmc_traj_accepts(vmc_traj* t, int64_t* n_acc_dev) {
  if (!t || !n_acc_dev) return VMC_EINVAL;
  HIPCHK(hipMemcpyAsync(n_acc_dev, t->nacc, (size_t)t->W * sizeof(int64_t), hipMemcpyDeviceToDevice,
                        t->ctx->stream));
  return VMC_OK;
}

int vmc_twist_average(vmc_ctx* ctx, int n_tw, int n3, const double* f_stack, const double* S_stack, double* f,
                      double* S) {
  if (!ctx || n_tw < 1 || n3 < 1 || !f_stack || !S_stack || !f || !S) return VMC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  RUN(K_REDUCE, launch_twist_average(n_tw, n3, f_stack, S_stack, f, S, ctx->stream));
  return VMC_OK;
}

int vmc_build_S_raw(vmc_ctx* ctx, int W, int n3, const double* f_w, const double* f, double* S) {
  if (!ctx || W < 2 || n3 < 1 || !f_w || !f || !S) return VMC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  const size_t need = syrk_partial_doubles(W, n3);
  if (ctx->syrk_work_n < need) {
    if (ctx->syrk_work) (void)hipFree(ctx->syrk_work);
    ctx->syrk_work = nullptr;
    ctx->syrk_work_n = 0;
    if (dalloc(&ctx->syrk_work, need)) return VMC_ENOMEM;
    ctx->syrk_work_n = need;
  }
  RUN(K_SYRK, launch_syrk(W, n3, f_w, f, ctx->syrk_work, S, ctx->stream));
  return VMC_OK;
}

int vmc_build_S(vmc_traj* t, double* S) {
  if (!t || !t->have_means) return VMC_EINVAL;
  const int n3 = 3 * t->N;
  int rc = vmc_build_S_raw(t->ctx, t->W, n3, t->f_w, t->outv + 3, t->Sd);
  if (rc) return rc;
  t->have_S = true;
  if (S)
    HIPCHK(hipMemcpyAsync(S, t->Sd, (size_t)n3 * n3 * sizeof(double), hipMemcpyDeviceToDevice, t->ctx->stream));
  return VMC_OK;
}

int vmc_traj_set_R(vmc_traj* t, const double* R_dev) {
  if (!t || !R_dev) return VMC_EINVAL;
  HIPCHK(hipSetDevice(t->ctx->device));
  HIPCHK(hipMemcpyAsync(t->Rd, R_dev, 3 * (size_t)t->N * sizeof(double), hipMemcpyDeviceToDevice, t->ctx->stream));
  t->have_R = true;
  t->have_prev = false;
  return VMC_OK;
}

int vmc_traj_get_R(vmc_traj* t, double* R_dev) {
  if (!t || !R_dev || !t->have_R) return VMC_EINVAL;
  HIPCHK(hipSetDevice(t->ctx->device));
  HIPCHK(hipMemcpyAsync(R_dev, t->Rd, 3 * (size_t)t->N * sizeof(double), hipMemcpyDeviceToDevice, t->ctx->stream));
  return VMC_OK;
}

int vmc_traj_step_count(vmc_traj* t, uint32_t* steps) {
  if (!t || !steps) return VMC_EINVAL;
  *steps = t->lang_step;
  return VMC_OK;
}

int vmc_langevin_step(vmc_ctx* ctx, int n3, double L, double* R, double* R_prev, double* S_prev, const double* f,
                      const double* S, double T, double Delta, double alpha, unsigned flags, uint32_t seed,
                      uint32_t traj_id, uint32_t step) {
  if (!ctx || n3 < 1 || n3 > 1536 || !R || !R_prev || !S_prev || !f || !S) return VMC_EINVAL;
  if (!(Delta > 0.0) || alpha < 0.0 || T < 0.0 || !(L >= 0.0) || (flags & ~7u)) return VMC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  const size_t need = langevin_work_doubles(n3);
  if (ctx->lang_work_n < need) {
    if (ctx->lang_work) (void)hipFree(ctx->lang_work);
    ctx->lang_work = nullptr;
    ctx->lang_work_n = 0;
    if (dalloc(&ctx->lang_work, need)) return VMC_ENOMEM;
    ctx->lang_work_n = need;
  }
  HIPCHK(hipMemsetAsync(ctx->d_status, 0, sizeof(int), ctx->stream));
  RUN(K_LANGEVIN, launch_langevin(n3, L, R, R_prev, S_prev, f, S, ctx->lang_work, nullptr, T, Delta, alpha, flags,
                                  seed, traj_id, step, ctx->d_status, ctx->stream));
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (st == 3) return VMC_ENOTSPD;
  if (st == 1) return VMC_EINVAL;
  return VMC_OK;
}

int vmc_langevin_step_noalloc(vmc_ctx* ctx, int n3, double L, double* R, double* R_prev, double* S_prev,
                              const double* f, const double* S, double T, double Delta, double alpha,
                              unsigned flags, uint32_t seed, uint32_t traj_id, uint32_t step) {
  if (!ctx || n3 < 1 || n3 > langevin_noalloc_max() || !R || !R_prev || !S_prev || !f || !S) return VMC_EINVAL;
  if (!(Delta > 0.0) || alpha < 0.0 || T < 0.0 || !(L >= 0.0) || (flags & ~7u)) return VMC_EINVAL;
  if (!ctx->noalloc_scratch) return VMC_EDEVICE;
  HIPCHK(hipSetDevice(ctx->device));
  // the device's static scratch (its address from hipGetSymbolAddress at vmc_create): the step's
  // work, then the status word, which the kernel writes on every path (nothing to clear)
  double* work = ctx->noalloc_scratch;
  int* status = reinterpret_cast<int*>(work + langevin_scratch_status_offset());
  RUN(K_LANGEVIN, launch_langevin(n3, L, R, R_prev, S_prev, f, S, work, nullptr, T, Delta, alpha, flags, seed,
                                  traj_id, step, status, ctx->stream));
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (st == 3) return VMC_ENOTSPD;
  if (st == 1) return VMC_EINVAL;
  return VMC_OK;
}

int vmc_traj_langevin_step(vmc_traj* t, double T, double Delta, double alpha, unsigned flags) {
  if (!t || !t->have_R || !t->have_means || (!t->have_S && !(flags & VMC_STEP_CFOLD))) return VMC_EINVAL;
  vmc_ctx* ctx = t->ctx;
  const int n3 = 3 * t->N;
  HIPCHK(hipSetDevice(ctx->device));
  if (!t->have_S) {
    // S = I replaces S (VMC_STEP_CFOLD); keep the stored matrix finite for S_prev
    HIPCHK(hipMemsetAsync(t->Sd, 0, (size_t)n3 * n3 * sizeof(double), ctx->stream));
  }
  if (!t->have_prev) {
    // first step of the trajectory: R_prev = R, S_prev = S
    HIPCHK(hipMemcpyAsync(t->Rprev, t->Rd, n3 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(t->Sprev, t->Sd, (size_t)n3 * n3 * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  const int rc = vmc_langevin_step(ctx, n3, t->sys.box_L, t->Rd, t->Rprev, t->Sprev, t->outv + 3, t->Sd, T, Delta,
                                   alpha, flags, t->seed, t->traj_id, t->lang_step);
  if (rc) return rc;
  t->have_prev = true;
  t->lang_step += 1;
  return VMC_OK;
}

int vmc_toy_run(vmc_ctx* ctx, const vmc_toy_params* p, int n_traj, int n_steps, uint32_t seed, const double* R0,
                double* R, double* U_mean, int* status) {
  if (!ctx || !p || n_traj < 1 || n_steps < 1 || !R0 || !R || !U_mean || !status) return VMC_EINVAL;
  if (!(p->lambda > 0.0) || !(p->k >= 0.0) || !(p->mu >= 0.0) || !(p->T >= 0.0) || !(p->Delta > 0.0) ||
      !(p->alpha >= 0.0) || p->s_kind < 0 || p->s_kind > 3 || p->scheme < 0 || p->scheme > 3)
    return VMC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  RUN(K_TOY, launch_toy(p->lambda, p->k, p->a, p->mu, p->s_kind, p->T, p->Delta, p->alpha, p->scheme, seed, n_traj,
                        n_steps, R0, R, U_mean, status, ctx->stream));
  return VMC_OK;
}

int vmc_eval_configs(vmc_ctx* ctx, const vmc_system* sys, const double* R, const double* C, const double* zeta,
                     int K, const double* pos, double* out) {
  if (!ctx || K < 1 || !R || !C || !zeta || !pos || !out) return VMC_EINVAL;
  vmc_traj* t = nullptr;
  int rc = vmc_traj_create(ctx, sys, K, 0, 0, &t);
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  const int mixed = t->sys.precision == VMC_MIXED;
  const size_t N = t->N;
  int nimg = 1;
  rc = vmc_traj_set_walkers(t, pos);
  if (!rc) rc = proton_setup(t, R);
  if (!rc) rc = image_count(t, zeta, &nimg);
  if (!rc) {
    auto body = [&]() -> int {
      HIPCHK(hipMemsetAsync(t->acc, 0, (size_t)K * (2 + 9 * N) * sizeof(double), st));
      HIPCHK(hipMemsetAsync(t->rho_acc, 0, (size_t)K * t->nk * 2 * sizeof(double), st));
      HIPCHK(hipMemsetAsync(ctx->d_status, 0, sizeof(int), st));
      WalkerArgs a = walker_args(t, R, C, zeta, nimg);
      MeasureArgs m = measure_args(t, R, C, zeta, nimg);
      EwaldArgs e = ewald_args(t);
      int r2 = 0;
      if (is_complex(t->sys)) {
        const TwistArgs tw = twist_args(t->sys);
        for (int sp = 0; sp < 2; ++sp) {
          SweepArgs sa{sp, 0, 0, 0, 0, 0.0};
          RUN(K_CSWEEP, launch_csweep(a, sa, tw, 1, 0, 0.0, st));
        }
        r2 = measure_c(t, m, e, tw);
      } else {
        RUN(K_BUILD_A, launch_build_A(a, mixed, st));
        RUN(K_INVERT, launch_invert(a, 0, 2, 0, st));
        r2 = measure(t, m, e);
      }
      if (r2) return r2;
      RUN(K_FINALIZE, launch_finalize(m, e, 1, t->means, st));
      HIPCHK(launch_pack_eval(K, (int)N, t->means, t->ldet, t->Uj, out, st));
      return check_singular(ctx);
    };
    rc = body();
  }
  (void)hipStreamSynchronize(st);
  vmc_traj_destroy(t);
  return rc;
}

}  // extern "C"

// ==================================================================== serving ==
// Continuous batching of independent trajectories on one context stream.  A tick
// admits queued requests while the HBM budget allows (FIFO, no overtaking), runs
// the set-up of every trajectory that starts a Langevin step (host Hueckel at its
// current R, proton tables, Slater rows, elimination), then one sweep for every
// sweeping trajectory: per bucket of equal (N, precision, Gaussian images, Ewald
// cut-off) one launch per kernel serves all of them (job tables, see Batch), and a
// trajectory whose last sweep this was gets its reduction, S, Langevin update and
// an asynchronous copy of the new R and E to pinned host memory.  The host polls
// that copy's event at later ticks, so no trajectory waits on another.  Every
// walker computes in a batched launch exactly what it computes alone.

namespace {

enum { SV_QUEUED = 0, SV_RUNNING = 1, SV_DONE = 2, SV_FAILED = 3, SV_CANCELLED = 4 };
enum { PH_SETUP = 0, PH_SWEEP = 1, PH_WAIT = 2 };

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Served {
  int id = 0;
  vmc_request req{};
  std::vector<double> R0, zeta, Rh;
  double* stage = nullptr;     // pinned: pos0 (W x N x 3), copied to the device at admission
  size_t bytes = 0;
  int state = SV_QUEUED, phase = PH_SETUP, err = VMC_OK;
  vmc_traj* t = nullptr;
  double *R = nullptr, *R_prev = nullptr, *S = nullptr, *S_prev = nullptr, *C = nullptr, *zeta_d = nullptr;
  int* status = nullptr;       // [0]: a refresh hit a zero pivot, [1]: the Langevin update failed (3 = S not SPD)
  double* hbuf = nullptr;      // pinned: R (3N), E, sigma_E, the two status words
  double* hC = nullptr;        // pinned: C staging (N x N/2)
  hipEvent_t done = nullptr;
  int nimg = 1, steps_done = 0, sweep = 0, n_equil_cur = 0;
  double t_submit = 0, t_admit = 0, t_step = 0;
  std::vector<double> E, sigE, lat;
};

struct BucketKey {
  int n, prec, nimg, nmax, j1;   // j1: the one-body term is on (the sweep's LDS holds a proton table)
  int tw;                        // some twist: the kernels' twisted instantiation
  bool operator<(const BucketKey& o) const {
    return std::tie(n, prec, nimg, nmax, j1, tw) < std::tie(o.n, o.prec, o.nimg, o.nmax, o.j1, o.tw);
  }
};

// Device bytes a request holds while resident: its trajectory (vmc_traj_bytes) plus the
// server's C, zeta and status.
size_t request_bytes(const vmc_system& s, int W) {
  const size_t N = s.n_protons;
  return traj_bytes(s, W) + (N * (N / 2) + N) * sizeof(double) + 2 * sizeof(int);
}

}  // namespace

struct vmc_server {
  vmc_ctx* ctx = nullptr;
  size_t budget = 0, resident = 0, peak = 0;
  int next_id = 1;
  std::deque<Served*> queue;
  std::vector<Served*> active;
  std::map<int, Served*> all;
  // job tables: ring of pinned host buffers and device buffers, one per tick in flight
  static constexpr int RING = 4;
  unsigned char* htab[RING] = {nullptr};
  unsigned char* dtab[RING] = {nullptr};
  size_t tab_cap = 0;
  hipEvent_t tab_ev[RING] = {nullptr};
  bool tab_used[RING] = {false};
  int ring = 0;
  long long ticks = 0;
};

namespace {

void release(vmc_server* s, Served* q) {
  if (q->t) {
    vmc_traj_destroy(q->t);
    q->t = nullptr;
    s->resident -= q->bytes;
  }
  q->R = q->R_prev = q->S = q->S_prev = nullptr;     // the trajectory's own arrays
  double** ds[] = {&q->C, &q->zeta_d};
  for (double** p : ds)
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  if (q->status) { (void)hipFree(q->status); q->status = nullptr; }
  if (q->hbuf) { (void)hipHostFree(q->hbuf); q->hbuf = nullptr; }
  if (q->hC) { (void)hipHostFree(q->hC); q->hC = nullptr; }
  if (q->stage) { (void)hipHostFree(q->stage); q->stage = nullptr; }
  if (q->done) { (void)hipEventDestroy(q->done); q->done = nullptr; }
}

int ensure_workspaces(vmc_ctx* ctx, int W, int n3) {
  const size_t need_s = syrk_partial_doubles(W, n3);
  if (ctx->syrk_work_n < need_s || ctx->lang_work_n < langevin_work_doubles(n3))
    HIPCHK(hipStreamSynchronize(ctx->stream));       // queued kernels may still use the old buffers
  if (ctx->syrk_work_n < need_s) {
    if (ctx->syrk_work) (void)hipFree(ctx->syrk_work);
    ctx->syrk_work = nullptr;
    ctx->syrk_work_n = 0;
    if (dalloc(&ctx->syrk_work, need_s)) return VMC_ENOMEM;
    ctx->syrk_work_n = need_s;
  }
  const size_t need_l = langevin_work_doubles(n3);
  if (ctx->lang_work_n < need_l) {
    if (ctx->lang_work) (void)hipFree(ctx->lang_work);
    ctx->lang_work = nullptr;
    ctx->lang_work_n = 0;
    if (dalloc(&ctx->lang_work, need_l)) return VMC_ENOMEM;
    ctx->lang_work_n = need_l;
  }
  return VMC_OK;
}

// Allocates and fills a trajectory's device state (admission).
int admit(vmc_server* s, Served* q) {
  vmc_ctx* ctx = s->ctx;
  const vmc_request& r = q->req;
  const int N = r.sys.n_protons, NS = N / 2, n3 = 3 * N;
  int rc = vmc_traj_create(ctx, &r.sys, r.n_walkers, r.seed, r.traj_id, &q->t);
  if (rc) return rc;
  s->resident += q->bytes;
  s->peak = std::max(s->peak, s->resident);
  // R, R_prev, S and S_prev are the trajectory's Langevin state
  q->R = q->t->Rd;
  q->R_prev = q->t->Rprev;
  q->S = q->t->Sd;
  q->S_prev = q->t->Sprev;
  if (dalloc(&q->C, (size_t)N * NS) || dalloc(&q->zeta_d, N) || dalloc(&q->status, 2)) return VMC_ENOMEM;
  if (hipHostMalloc((void**)&q->hbuf, (n3 + 3) * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&q->hC, (size_t)N * NS * sizeof(double)) != hipSuccess)
    return VMC_ENOMEM;
  if (hipEventCreateWithFlags(&q->done, hipEventDisableTiming) != hipSuccess) return VMC_EDEVICE;
  rc = ensure_workspaces(ctx, r.n_walkers, n3);
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  // zeta and R0 follow the electrons in the pinned staging buffer, so the copies need no wait
  double* zs = q->stage + (size_t)r.n_walkers * N * 3;
  HIPCHK(hipMemcpyAsync(q->t->pos, q->stage, (size_t)r.n_walkers * N * 3 * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(q->zeta_d, zs, N * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(q->R, zs + N, n3 * sizeof(double), hipMemcpyHostToDevice, st));
  q->nimg = image_rule(r.sys, q->zeta.data());
  q->Rh = q->R0;
  q->state = SV_RUNNING;
  q->phase = PH_SETUP;
  q->t_admit = now_ms();
  q->t_step = q->t_admit;
  return VMC_OK;
}

// Start of a Langevin step: C at the current R, proton tables, Slater rows, elimination.
int setup_step(vmc_server* s, Served* q) {
  vmc_ctx* ctx = s->ctx;
  vmc_traj* t = q->t;
  const vmc_request& r = q->req;
  const int N = r.sys.n_protons, NS = N / 2;
  hipStream_t st = ctx->stream;
  for (double x : q->Rh)
    if (!std::isfinite(x)) return VMC_EINVAL;
  std::vector<double> Cv((size_t)N * NS);
  int rc = vmc_huckel_params_twist(N, r.sys.box_L, r.sys.twist, q->Rh.data(), q->zeta.data(), Cv.data());
  if (rc) return rc;
  std::memcpy(q->hC, Cv.data(), Cv.size() * sizeof(double));   // the previous copy from hC has completed
  HIPCHK(hipMemcpyAsync(q->C, q->hC, Cv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  rc = proton_setup(t, q->R);
  if (rc) return rc;
  const size_t W = t->W, Nz = N;
  HIPCHK(hipMemsetAsync(t->acc, 0, W * (2 + 9 * Nz) * sizeof(double), st));
  HIPCHK(hipMemsetAsync(t->rho_acc, 0, W * t->nk * 2 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(t->nacc, 0, W * sizeof(int64_t), st));
  HIPCHK(hipMemsetAsync(t->rflag, 0, W * 2 * sizeof(int), st));
  HIPCHK(hipMemsetAsync(q->status, 0, 2 * sizeof(int), st));
  // walker quarantine as in vmc_energy_forces (asynchronous here: with no finite walker left
  // the trajectory's S is not finite and the step fails, for this request only)
  HIPCHK(hipMemsetAsync(t->qflag + W, 0, 2 * sizeof(int), st));
  RUN(K_SETUP, launch_walker_quarantine((int)W, N, t->pos, t->qflag, t->qflag + W, st));
  WalkerArgs a = walker_args(t, q->R, q->C, q->zeta_d, q->nimg);
  a.status = q->status;
  RUN(K_BUILD_A, launch_build_A(a, r.sys.precision == VMC_MIXED, st));
  RUN(K_INVERT, launch_invert(a, 0, 2, 0, st));
  q->sweep = 0;
  q->n_equil_cur = q->steps_done == 0 ? r.n_equil_first : r.n_equil;
  q->phase = PH_SWEEP;
  return VMC_OK;
}

TrajJob make_job(Served* q, int sweep) {
  vmc_traj* t = q->t;
  TrajJob j{};
  j.a = walker_args(t, q->R, q->C, q->zeta_d, q->nimg);
  j.a.status = q->status;
  j.m = measure_args(t, q->R, q->C, q->zeta_d, q->nimg);
  j.e = ewald_args(t);
  j.s = SweepArgs{0, sweep, (uint32_t)q->steps_done, t->seed, t->traj_id, q->req.step_delta};
  j.tol = q->req.sys.refine_tol == 0.0 ? 1e-7 : q->req.sys.refine_tol;
  return j;
}

// End of a Langevin step: reduction, S, update, result copy to the host.
int finish_step(vmc_server* s, Served* q) {
  vmc_ctx* ctx = s->ctx;
  vmc_traj* t = q->t;
  const vmc_request& r = q->req;
  const int N = r.sys.n_protons, n3 = 3 * N, W = t->W;
  hipStream_t st = ctx->stream;
  MeasureArgs m = measure_args(t, q->R, q->C, q->zeta_d, q->nimg);
  EwaldArgs e = ewald_args(t);
  const int total = q->n_equil_cur + r.n_sweeps;
  RUN(K_FINALIZE, launch_finalize(m, e, r.n_sweeps, t->means, st));
  RUN(K_REDUCE, launch_reduce(W, n3, t->means, t->nacc, (double)N * total, t->f_w, t->partial, t->outv, st));
  RUN(K_SYRK, launch_syrk(W, n3, t->f_w, t->outv + 3, ctx->syrk_work, q->S, st));
  if (q->steps_done == 0) {
    HIPCHK(hipMemcpyAsync(q->S_prev, q->S, (size_t)n3 * n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(q->R_prev, q->R, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  RUN(K_LANGEVIN, launch_langevin(n3, r.sys.box_L, q->R, q->R_prev, q->S_prev, t->outv + 3, q->S, ctx->lang_work,
                                  nullptr, r.T, r.Delta, r.alpha, r.flags, t->seed, t->traj_id,
                                  (uint32_t)q->steps_done, q->status + 1, st));
  HIPCHK(hipMemcpyAsync(q->hbuf, q->R, n3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(q->hbuf + n3, t->outv, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(q->hbuf + n3 + 2, q->status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(q->done, st));
  q->phase = PH_WAIT;
  return VMC_OK;
}

// One batched sweep of the sweeping trajectories of one bucket.
int bucket_sweep(vmc_server* s, const std::vector<Served*>& qs) {
  vmc_ctx* ctx = s->ctx;
  hipStream_t st = ctx->stream;
  const int nq = (int)qs.size();
  // host tables: [jobs sweep | jobs refresh | jobs measure] then offsets
  std::vector<TrajJob> js, jr, jm;
  std::vector<int> os{0}, orf{0}, orp{0}, om{0};
  for (Served* q : qs) {
    const TrajJob j = make_job(q, q->sweep);
    js.push_back(j);
    os.push_back(os.back() + (q->t->W + 3) / 4);
    // fallback elimination blocks: four walkers each, or one matrix each for N_sigma > 64; the
    // refresh's own blocks (refine_blocks) may pack matrices differently
    if (q->sweep >= 1) {
      jr.push_back(j);
      orf.push_back(orf.back() + (q->t->NS > 64 ? q->t->W : (q->t->W + 3) / 4));
      orp.push_back(orp.back() + refine_blocks(q->t->NS, q->t->W));
    }
    if (q->sweep >= q->n_equil_cur) { jm.push_back(j); om.push_back(om.back() + q->t->W); }
  }
  const size_t nj = js.size() + jr.size() + jm.size();
  const size_t bytes_jobs = nj * sizeof(TrajJob);
  // every piece is padded to 16 bytes: at most 15 more bytes for each of the seven
  const size_t bytes = bytes_jobs + (os.size() + orf.size() + orp.size() + om.size()) * sizeof(int) + 7 * 16;
  const int k = s->ring;
  s->ring = (s->ring + 1) % vmc_server::RING;
  if (s->tab_used[k]) HIPCHK(hipEventSynchronize(s->tab_ev[k]));      // its previous upload has been consumed
  if (s->tab_cap < bytes) {
    HIPCHK(hipStreamSynchronize(st));                 // queued kernels may still read the old tables
    for (int i = 0; i < vmc_server::RING; ++i) {
      if (s->tab_used[i]) HIPCHK(hipEventSynchronize(s->tab_ev[i]));
      if (s->htab[i]) (void)hipHostFree(s->htab[i]);
      if (s->dtab[i]) (void)hipFree(s->dtab[i]);
      s->htab[i] = s->dtab[i] = nullptr;
      s->tab_used[i] = false;
    }
    const size_t cap = bytes * 2;
    for (int i = 0; i < vmc_server::RING; ++i) {
      if (hipHostMalloc((void**)&s->htab[i], cap) != hipSuccess) return VMC_ENOMEM;
      if (hipMalloc((void**)&s->dtab[i], cap) != hipSuccess) return VMC_ENOMEM;
    }
    s->tab_cap = cap;
  }
  unsigned char* h = s->htab[k];
  unsigned char* d = s->dtab[k];
  size_t off = 0;
  auto put = [&](const void* src, size_t n) -> size_t {
    const size_t o = off;
    if (n) std::memcpy(h + o, src, n);
    off += (n + 15) / 16 * 16;
    return o;
  };
  const size_t o_js = put(js.data(), js.size() * sizeof(TrajJob));
  const size_t o_jr = put(jr.data(), jr.size() * sizeof(TrajJob));
  const size_t o_jm = put(jm.data(), jm.size() * sizeof(TrajJob));
  const size_t o_os = put(os.data(), os.size() * sizeof(int));
  const size_t o_or = put(orf.data(), orf.size() * sizeof(int));
  const size_t o_op = put(orp.data(), orp.size() * sizeof(int));
  const size_t o_om = put(om.data(), om.size() * sizeof(int));
  HIPCHK(hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(s->tab_ev[k], st));
  s->tab_used[k] = true;
  const Batch bsw{(const TrajJob*)(d + o_js), (const int*)(d + o_os), (int)js.size()};
  const Batch brf{(const TrajJob*)(d + o_jr), (const int*)(d + o_or), (int)jr.size()};
  const Batch brp{(const TrajJob*)(d + o_jr), (const int*)(d + o_op), (int)jr.size()};
  const Batch bms{(const TrajJob*)(d + o_jm), (const int*)(d + o_om), (int)jm.size()};
  const int mixed = qs[0]->req.sys.precision == VMC_MIXED;
  const TrajJob& j0 = js[0];
  for (int sp = 0; sp < 2; ++sp) {
    if (!jr.empty()) {
      RUN(K_REFINE, launch_refine(j0.a, sp, j0.tol, st, &brp, orp.back()));
      RUN(K_INVERT, launch_invert(j0.a, sp, sp + 1, 1, st, &brf, orf.back()));
    }
    SweepArgs sa = j0.s;
    sa.spin = sp;
    RUN(K_SWEEP, launch_sweep(j0.a, sa, mixed, st, &bsw, os.back()));
  }
  if (!jm.empty()) {
    RUN(K_EWALD, launch_ewald_sample(jm[0].m, jm[0].e, mixed, st, &bms, om.back()));
    RUN(K_SLATER, launch_slater_sample(jm[0].m, mixed, st, &bms, om.back()));
  }
  (void)nq;
  return VMC_OK;
}

int check_request(const vmc_request* r) {
  if (!r || check_sys(&r->sys) || r->sys.general_twist || r->sys.contracted || has_jorb(r->sys)) return VMC_EINVAL;
  if (r->n_walkers < 2 || r->n_sweeps < 1 || r->n_equil < 0 || r->n_equil_first < 0 || r->n_steps < 1)
    return VMC_EINVAL;
  if (!(r->step_delta > 0.0) || !(r->Delta > 0.0) || r->alpha < 0.0 || r->T < 0.0 || (r->flags & ~7u))
    return VMC_EINVAL;
  if (!r->R0 || !r->zeta || !r->pos0 || 3 * r->sys.n_protons > 1536) return VMC_EINVAL;
  // S from W walker means has rank <= W - 1: it can be positive definite only if W > 3N
  if (!(r->flags & VMC_STEP_CFOLD) && r->n_walkers <= 3 * r->sys.n_protons) return VMC_EINVAL;
  return VMC_OK;
}

}  // namespace

extern "C" {

size_t vmc_request_bytes(const vmc_request* r) {
  if (check_request(r)) return 0;
  return request_bytes(r->sys, r->n_walkers);
}

int vmc_server_create(vmc_ctx* ctx, size_t hbm_budget_bytes, vmc_server** out) {
  if (!ctx || !out || hbm_budget_bytes == 0) return VMC_EINVAL;
  vmc_server* s = new (std::nothrow) vmc_server();
  if (!s) return VMC_ENOMEM;
  s->ctx = ctx;
  s->budget = hbm_budget_bytes;
  for (int i = 0; i < vmc_server::RING; ++i)
    if (hipEventCreateWithFlags(&s->tab_ev[i], hipEventDisableTiming) != hipSuccess) {
      vmc_server_destroy(s);
      return VMC_EDEVICE;
    }
  *out = s;
  return VMC_OK;
}

void vmc_server_destroy(vmc_server* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->ctx->stream);
  for (auto& kv : s->all) {
    release(s, kv.second);
    delete kv.second;
  }
  for (int i = 0; i < vmc_server::RING; ++i) {
    if (s->htab[i]) (void)hipHostFree(s->htab[i]);
    if (s->dtab[i]) (void)hipFree(s->dtab[i]);
    if (s->tab_ev[i]) (void)hipEventDestroy(s->tab_ev[i]);
  }
  delete s;
}

int vmc_server_submit(vmc_server* s, const vmc_request* r, int* id_out) {
  if (!s || !id_out) return VMC_EINVAL;
  int rc = check_request(r);
  if (rc) return rc;
  const size_t b = request_bytes(r->sys, r->n_walkers);
  if (b > s->budget) return VMC_ENOMEM;
  Served* q = new (std::nothrow) Served();
  if (!q) return VMC_ENOMEM;
  const int N = r->sys.n_protons;
  q->id = s->next_id++;
  q->req = *r;
  q->R0.assign(r->R0, r->R0 + 3 * N);
  q->zeta.assign(r->zeta, r->zeta + N);
  const size_t npos = (size_t)r->n_walkers * N * 3;
  if (hipHostMalloc((void**)&q->stage, (npos + 4 * N) * sizeof(double)) != hipSuccess) {
    delete q;
    return VMC_ENOMEM;
  }
  std::memcpy(q->stage, r->pos0, npos * sizeof(double));
  std::memcpy(q->stage + npos, r->zeta, N * sizeof(double));
  std::memcpy(q->stage + npos + N, r->R0, 3 * N * sizeof(double));
  q->req.R0 = q->req.zeta = q->req.pos0 = nullptr;
  q->req.sys.refine_tol = r->sys.refine_tol;
  q->bytes = b;
  q->t_submit = now_ms();
  s->queue.push_back(q);
  s->all[q->id] = q;
  *id_out = q->id;
  return VMC_OK;
}

int vmc_server_cancel(vmc_server* s, int id) {
  if (!s) return VMC_EINVAL;
  auto it = s->all.find(id);
  if (it == s->all.end()) return VMC_EINVAL;
  Served* q = it->second;
  if (q->state == SV_QUEUED) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), q), s->queue.end());
    q->state = SV_CANCELLED;
    q->err = VMC_ECANCELLED;
  } else if (q->state == SV_RUNNING) {
    HIPCHK(hipStreamSynchronize(s->ctx->stream));   // its queued work finishes before its memory goes
    s->active.erase(std::remove(s->active.begin(), s->active.end(), q), s->active.end());
    release(s, q);
    q->state = SV_CANCELLED;
    q->err = VMC_ECANCELLED;
  }
  return VMC_OK;
}

int vmc_server_tick(vmc_server* s, int* n_active, int* n_queued) {
  if (!s) return VMC_EINVAL;
  vmc_ctx* ctx = s->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  ++s->ticks;
  // 1. finished steps
  for (size_t i = 0; i < s->active.size();) {
    Served* q = s->active[i];
    bool drop = false;
    if (q->phase == PH_WAIT) {
      const hipError_t e = hipEventQuery(q->done);
      if (e == hipSuccess) {
        const int n3 = 3 * q->req.sys.n_protons;
        int stv[2] = {0, 0};
        std::memcpy(stv, q->hbuf + n3 + 2, 2 * sizeof(int));
        if (stv[0] != 0 || stv[1] != 0) {
          q->state = SV_FAILED;
          q->err = stv[0] ? VMC_ESINGULAR : (stv[1] == 3 ? VMC_ENOTSPD : VMC_EINVAL);
          drop = true;
        } else {
          q->Rh.assign(q->hbuf, q->hbuf + n3);
          q->E.push_back(q->hbuf[n3]);
          q->sigE.push_back(q->hbuf[n3 + 1]);
          q->lat.push_back(now_ms() - q->t_step);
          q->steps_done += 1;
          if (q->steps_done == q->req.n_steps) {
            q->state = SV_DONE;
            drop = true;
          } else {
            q->phase = PH_SETUP;
            q->t_step = now_ms();
          }
        }
      } else if (e != hipErrorNotReady) {
        return map_err(e);
      }
    }
    if (drop) {
      release(s, q);
      s->active.erase(s->active.begin() + i);
    } else {
      ++i;
    }
  }
  // 2. admission, FIFO within the budget
  {
    std::vector<size_t> b;
    for (Served* q : s->queue) b.push_back(q->bytes);
    const int k = admit_count(s->budget, s->resident, (int)b.size(), b.data());
    for (int i = 0; i < k; ++i) {
      Served* q = s->queue.front();
      s->queue.pop_front();
      const int rc = admit(s, q);
      if (rc) {
        q->state = SV_FAILED;
        q->err = rc;
        release(s, q);
        continue;
      }
      s->active.push_back(q);
    }
  }
  // 3. set-up of trajectories starting a step.  A host-side or argument failure of one
  // request (a non-finite R, the eigen-solver) fails that request only; HIP errors end the tick.
  for (size_t i = 0; i < s->active.size();) {
    Served* q = s->active[i];
    if (q->phase == PH_SETUP) {
      const int rc = setup_step(s, q);
      if (rc == VMC_EDEVICE || rc == VMC_ENOTBUILT) return rc;
      if (rc) {
        HIPCHK(hipStreamSynchronize(ctx->stream));   // none of its work may still be queued
        q->state = SV_FAILED;
        q->err = rc;
        release(s, q);
        s->active.erase(s->active.begin() + i);
        continue;
      }
    }
    ++i;
  }
  // 4. batched sweeps per bucket, then the steps that end here.  A bucket runs
  // k = clamp(c_max / c, 1, 32) sweeps per tick, c = sum of W N^2 over its
  // trajectories (their work per sweep), so a tick advances every bucket by about
  // the same device time and small systems are not held to the pace of large ones.
  std::map<BucketKey, std::vector<Served*>> buckets;
  for (Served* q : s->active)
    if (q->phase == PH_SWEEP)
      buckets[BucketKey{q->req.sys.n_protons, q->req.sys.precision, q->nimg, q->req.sys.ewald_nmax,
                         q->req.sys.j1_b1 > 0.0 ? 1 : 0, q->req.sys.twist != 0 ? 1 : 0}].push_back(q);
  double cmax = 0.0;
  std::map<BucketKey, double> cost;
  for (auto& kv : buckets) {
    double c = 0.0;
    for (Served* q : kv.second) c += (double)q->req.n_walkers * q->req.sys.n_protons * q->req.sys.n_protons;
    cost[kv.first] = c;
    cmax = std::max(cmax, c);
  }
  for (auto& kv : buckets) {
    const int reps = (int)std::min(32.0, std::max(1.0, std::floor(cmax / cost[kv.first])));
    std::vector<Served*> live = kv.second;
    for (int rep = 0; rep < reps && !live.empty(); ++rep) {
      const int rc = bucket_sweep(s, live);
      if (rc) return rc;
      std::vector<Served*> still;
      for (Served* q : live) {
        q->sweep += 1;
        if (q->sweep == q->n_equil_cur + q->req.n_sweeps) {
          const int r2 = finish_step(s, q);
          if (r2) return r2;
        } else {
          still.push_back(q);
        }
      }
      live.swap(still);
    }
  }
  if (n_active) *n_active = (int)s->active.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  return VMC_OK;
}

int vmc_server_status(vmc_server* s, int id, int* state, int* steps_done, int* error) {
  if (!s) return VMC_EINVAL;
  auto it = s->all.find(id);
  if (it == s->all.end()) return VMC_EINVAL;
  if (state) *state = it->second->state;
  if (steps_done) *steps_done = it->second->steps_done;
  if (error) *error = it->second->err;
  return VMC_OK;
}

int vmc_server_result(vmc_server* s, int id, double* R_out, double* E_out, double* sigma_out, double* latency_ms,
                      double* wait_ms) {
  if (!s) return VMC_EINVAL;
  auto it = s->all.find(id);
  if (it == s->all.end()) return VMC_EINVAL;
  Served* q = it->second;
  const int n3 = 3 * q->req.sys.n_protons, k = q->steps_done;
  if (R_out) std::memcpy(R_out, (k ? q->Rh : q->R0).data(), n3 * sizeof(double));
  for (int i = 0; i < k; ++i) {
    if (E_out) E_out[i] = q->E[i];
    if (sigma_out) sigma_out[i] = q->sigE[i];
    if (latency_ms) latency_ms[i] = q->lat[i];
  }
  if (wait_ms) *wait_ms = q->t_admit > 0 ? q->t_admit - q->t_submit : -1.0;
  return VMC_OK;
}

int vmc_server_info(vmc_server* s, size_t* resident, size_t* peak_resident, int* n_active, int* n_queued,
                    long long* ticks) {
  if (!s) return VMC_EINVAL;
  if (resident) *resident = s->resident;
  if (peak_resident) *peak_resident = s->peak;
  if (n_active) *n_active = (int)s->active.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  if (ticks) *ticks = s->ticks;
  return VMC_OK;
}

}  // extern "C"
