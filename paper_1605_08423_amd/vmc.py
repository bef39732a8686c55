"""Thin ctypes binding of libvmc.so (include/vmc.h).  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.  Device arrays
are torch CUDA float64 tensors; the library runs on torch's current stream.

Raises RuntimeError if the HIP library has not been built -- there is no
fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmc.so")

VMC_OK, VMC_EINVAL, VMC_ENOMEM, VMC_ENOTSPD, VMC_ESINGULAR, VMC_EDEVICE, VMC_ENOTBUILT = 0, -1, -2, -3, -4, -5, -6
VMC_ECANCELLED, VMC_ENOCONV = -7, -8
VMC_STEP_TRAJ = 0xFFFFFFFF
VMC_FP64, VMC_MIXED = 0, 1
VMC_STEP_CFOLD, VMC_STEP_NOISE_CORR, VMC_STEP_NO_SCORR = 1, 2, 4
# the Jastrow parameters that stochastic reconfiguration covers, (b, b_1, f_11, f_12, f_22, f_1, f_2),
# and the length of the statistics vector [E, <O>, <E_L O>, <O O^T>]
OPT_PAR = 7
OPT_STATS = 1 + 2 * OPT_PAR + OPT_PAR * OPT_PAR

EXPORTED = ["vmc_create", "vmc_destroy", "vmc_set_stream", "vmc_strerror", "vmc_supported_n",
            "vmc_set_profiling", "vmc_kernel_times", "vmc_reset_kernel_times", "vmc_traj_create",
            "vmc_traj_destroy", "vmc_traj_set_walkers", "vmc_traj_get_walkers", "vmc_energy_forces",
            "vmc_traj_walker_means", "vmc_traj_walker_forces", "vmc_traj_accepts", "vmc_build_S",
            "vmc_build_S_raw", "vmc_langevin_step", "vmc_eval_configs", "vmc_huckel_params",
            "vmc_request_bytes", "vmc_server_admit_count", "vmc_server_create", "vmc_server_destroy",
            "vmc_server_submit", "vmc_server_cancel", "vmc_server_tick", "vmc_server_status",
            "vmc_server_result", "vmc_server_info", "vmc_toy_run", "vmc_huckel_params_twist",
            "vmc_twist_average", "vmc_traj_save", "vmc_traj_load", "vmc_traj_load_rescaled", "vmc_traj_walkers_reset",
            "vmc_set_hbm_budget", "vmc_hbm_in_use", "vmc_traj_bytes", "vmc_cancel", "vmc_traj_set_R", "vmc_traj_get_R",
            "vmc_traj_step_count", "vmc_traj_langevin_step", "vmc_langevin_step_noalloc", "vmc_huckel_params_theta",
            "vmc_huckel_params_contracted", "vmc_traj_set_param_stats", "vmc_traj_param_stats",
            "vmc_traj_set_jastrow", "vmc_sr_update", "vmc_huckel_params_theta_contracted"]
VMC_REQ_QUEUED, VMC_REQ_RUNNING, VMC_REQ_DONE, VMC_REQ_FAILED, VMC_REQ_CANCELLED = 0, 1, 2, 3, 4


class VMCError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {_lib().vmc_strerror(code).decode()} ({code})")


class vmc_system(C.Structure):
    _fields_ = [("n_protons", C.c_int), ("box_L", C.c_double), ("ewald_kappa", C.c_double),
                ("ewald_nmax", C.c_int), ("a_par", C.c_double), ("a_anti", C.c_double), ("b", C.c_double),
                ("precision", C.c_int), ("refine_tol", C.c_double), ("j1_b1", C.c_double), ("twist", C.c_int),
                ("general_twist", C.c_int), ("theta", C.c_double * 3), ("contracted", C.c_int),
                ("eta", C.c_double), ("j3_f", C.c_double * 3), ("j1_f", C.c_double * 2)]


class vmc_request(C.Structure):
    _fields_ = [("sys", vmc_system), ("n_walkers", C.c_int), ("n_equil_first", C.c_int), ("n_equil", C.c_int),
                ("n_sweeps", C.c_int), ("n_steps", C.c_int), ("step_delta", C.c_double), ("T", C.c_double),
                ("Delta", C.c_double), ("alpha", C.c_double), ("flags", C.c_uint), ("seed", C.c_uint32),
                ("traj_id", C.c_uint32), ("R0", C.POINTER(C.c_double)), ("zeta", C.POINTER(C.c_double)),
                ("pos0", C.POINTER(C.c_double))]


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built (run __graft_entry__.build())")
        _L = C.CDLL(LIB_PATH)
        _declare(_L)
    return _L


def _declare(l):
    P, vp, d, i, u32 = C.POINTER, C.c_void_p, C.c_double, C.c_int, C.c_uint32
    l.vmc_strerror.restype = C.c_char_p
    l.vmc_strerror.argtypes = [i]
    l.vmc_create.argtypes = [P(vp), i]
    l.vmc_destroy.argtypes = [vp]
    l.vmc_destroy.restype = None
    l.vmc_set_stream.argtypes = [vp, vp]
    l.vmc_supported_n.argtypes = [i]
    l.vmc_set_profiling.argtypes = [vp, i]
    l.vmc_kernel_times.argtypes = [vp, P(C.c_char_p), P(d), P(C.c_longlong), i]
    l.vmc_reset_kernel_times.argtypes = [vp]
    l.vmc_traj_create.argtypes = [vp, P(vmc_system), i, u32, u32, P(vp)]
    l.vmc_traj_destroy.argtypes = [vp]
    l.vmc_traj_destroy.restype = None
    l.vmc_traj_set_walkers.argtypes = [vp, vp]
    l.vmc_traj_get_walkers.argtypes = [vp, vp]
    l.vmc_energy_forces.argtypes = [vp, vp, vp, vp, i, i, d, u32, vp]
    l.vmc_traj_walker_means.argtypes = [vp, vp]
    l.vmc_traj_walker_forces.argtypes = [vp, vp]
    l.vmc_traj_accepts.argtypes = [vp, vp]
    l.vmc_build_S.argtypes = [vp, vp]
    l.vmc_build_S_raw.argtypes = [vp, i, i, vp, vp, vp]
    l.vmc_langevin_step.argtypes = [vp, i, d, vp, vp, vp, vp, vp, d, d, d, C.c_uint, u32, u32, u32]
    l.vmc_langevin_step_noalloc.argtypes = [vp, i, d, vp, vp, vp, vp, vp, d, d, d, C.c_uint, u32, u32, u32]
    l.vmc_eval_configs.argtypes = [vp, P(vmc_system), vp, vp, vp, i, vp, vp]
    l.vmc_toy_run.argtypes = [vp, P(vmc_toy_params), i, i, u32, vp, vp, vp, vp]
    l.vmc_huckel_params.argtypes = [i, d, P(d), P(d), P(d)]
    l.vmc_huckel_params_twist.argtypes = [i, d, i, P(d), P(d), P(d)]
    l.vmc_huckel_params_theta.argtypes = [i, d, P(d), P(d), P(d), P(d)]
    l.vmc_huckel_params_contracted.argtypes = [i, d, d, P(d), P(d)]
    l.vmc_traj_set_param_stats.argtypes = [vp, i]
    l.vmc_traj_param_stats.argtypes = [vp, vp]
    l.vmc_traj_set_jastrow.argtypes = [vp, d, d, P(d), P(d)]
    l.vmc_sr_update.argtypes = [P(d), i, d, d, P(d)]
    l.vmc_huckel_params_theta_contracted.argtypes = [i, d, P(d), d, P(d), P(d)]
    l.vmc_twist_average.argtypes = [vp, i, i, vp, vp, vp, vp]
    l.vmc_traj_save.argtypes = [vp, vp, P(C.c_size_t)]
    l.vmc_traj_walkers_reset.argtypes = [vp, P(i)]
    l.vmc_traj_load.argtypes = [vp, vp, C.c_size_t]
    l.vmc_traj_load_rescaled.argtypes = [vp, vp, C.c_size_t]
    sz = C.c_size_t
    l.vmc_request_bytes.restype = sz
    l.vmc_request_bytes.argtypes = [P(vmc_request)]
    l.vmc_server_admit_count.argtypes = [sz, sz, i, P(sz)]
    l.vmc_server_create.argtypes = [vp, sz, P(vp)]
    l.vmc_server_destroy.argtypes = [vp]
    l.vmc_server_destroy.restype = None
    l.vmc_server_submit.argtypes = [vp, P(vmc_request), P(i)]
    l.vmc_server_cancel.argtypes = [vp, i]
    l.vmc_server_tick.argtypes = [vp, P(i), P(i)]
    l.vmc_server_status.argtypes = [vp, i, P(i), P(i), P(i)]
    l.vmc_server_result.argtypes = [vp, i, P(d), P(d), P(d), P(d), P(d)]
    l.vmc_server_info.argtypes = [vp, P(sz), P(sz), P(i), P(i), P(C.c_longlong)]
    l.vmc_set_hbm_budget.argtypes = [vp, sz]
    l.vmc_hbm_in_use.argtypes = [vp, P(sz)]
    l.vmc_traj_bytes.restype = sz
    l.vmc_traj_bytes.argtypes = [P(vmc_system), i]
    l.vmc_cancel.argtypes = [vp]
    l.vmc_traj_set_R.argtypes = [vp, vp]
    l.vmc_traj_get_R.argtypes = [vp, vp]
    l.vmc_traj_step_count.argtypes = [vp, P(u32)]
    l.vmc_traj_langevin_step.argtypes = [vp, d, d, d, C.c_uint]


def _check(rc, where):
    if rc != VMC_OK:
        raise VMCError(rc, where)


def _dev(t, n=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous CUDA float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def make_system(n, L, kappa=None, nmax=9, a_par=0.25, a_anti=0.5, b=1.0, precision=VMC_FP64, refine_tol=0.0,
                b1=0.0, twist=0, theta=None, eta=None, j3=None, j1f=None):
    """b1 > 0 adds the one-body electron-proton Jastrow term with that b_1 (0: none); twist:
    bit m = twist angle pi along axis m; theta (3 angles, radians): a general twist with complex
    orbitals (FP64 only); eta: the contracted orbital phi_1 + eta phi_2 per proton; j3: (f11, f12, f22) of
    the on-site three-body Jastrow term; j1f: (f_1, f_2) of the one-body term's orbital part."""
    th = (C.c_double * 3)(*([0.0] * 3 if theta is None else [float(v) for v in theta]))
    return vmc_system(int(n), float(L), float(8.0 / L if kappa is None else kappa), int(nmax), a_par, a_anti, b,
                      int(precision), float(refine_tol), float(b1), int(twist), int(theta is not None), th,
                      int(eta is not None), float(eta or 0.0),
                      (C.c_double * 3)(*(j3 if j3 is not None else (0.0, 0.0, 0.0))),
                      (C.c_double * 2)(*(j1f if j1f is not None else (0.0, 0.0))))


def _c_doubles(system):
    """Doubles of the orbital coefficients C for this system (complex pairs with a general twist)."""
    n = system.n_protons
    return n * (n // 2) * (2 if system.general_twist else 1)


class Context:
    def __init__(self, device=0):
        import torch
        self.h = C.c_void_p()
        _check(_lib().vmc_create(C.byref(self.h), device), "vmc_create")
        self.sync_stream()

    def sync_stream(self):
        import torch
        _check(_lib().vmc_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream)), "vmc_set_stream")

    def set_profiling(self, on=True):
        _check(_lib().vmc_set_profiling(self.h, int(on)), "vmc_set_profiling")

    def kernel_times(self):
        n = 32
        names = (C.c_char_p * n)()
        ms = (C.c_double * n)()
        cnt = (C.c_longlong * n)()
        k = _lib().vmc_kernel_times(self.h, names, ms, cnt, n)
        return {names[j].decode(): (ms[j], cnt[j]) for j in range(k)}

    def reset_kernel_times(self):
        _check(_lib().vmc_reset_kernel_times(self.h), "vmc_reset_kernel_times")

    def set_hbm_budget(self, nbytes):
        _check(_lib().vmc_set_hbm_budget(self.h, int(nbytes)), "vmc_set_hbm_budget")

    def hbm_in_use(self):
        n = C.c_size_t(0)
        _check(_lib().vmc_hbm_in_use(self.h, C.byref(n)), "vmc_hbm_in_use")
        return n.value

    def cancel(self):
        """Asks the running (or the next) vmc_energy_forces call to stop (any thread)."""
        _check(_lib().vmc_cancel(self.h), "vmc_cancel")

    def close(self):
        if self.h:
            _lib().vmc_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trajectory:
    def __init__(self, ctx: Context, system: vmc_system, n_walkers: int, seed: int = 0, traj_id: int = 0):
        self.ctx, self.sys, self.W, self.N = ctx, system, n_walkers, system.n_protons
        self.h = C.c_void_p()
        _check(_lib().vmc_traj_create(ctx.h, C.byref(system), n_walkers, seed, traj_id, C.byref(self.h)),
               "vmc_traj_create")

    def set_walkers(self, pos):
        _check(_lib().vmc_traj_set_walkers(self.h, _dev(pos, self.W * self.N * 3)), "vmc_traj_set_walkers")

    def get_walkers(self):
        import torch
        out = torch.empty((self.W, self.N, 3), dtype=torch.float64, device="cuda")
        _check(_lib().vmc_traj_get_walkers(self.h, _dev(out)), "vmc_traj_get_walkers")
        return out

    def energy_forces(self, R, Cmo, zeta, n_equil, n_sweeps, delta, step=0, out=None):
        return vmc_energy_forces(self, R, Cmo, zeta, n_equil, n_sweeps, delta, step, out)

    def walker_means(self):
        import torch
        out = torch.empty((self.W, 1 + 9 * self.N), dtype=torch.float64, device="cuda")
        _check(_lib().vmc_traj_walker_means(self.h, _dev(out)), "vmc_traj_walker_means")
        return out

    def walker_forces(self):
        import torch
        out = torch.empty((self.W, 3 * self.N), dtype=torch.float64, device="cuda")
        _check(_lib().vmc_traj_walker_forces(self.h, _dev(out)), "vmc_traj_walker_forces")
        return out

    def accepts(self):
        import torch
        out = torch.empty(self.W, dtype=torch.int64, device="cuda")
        _check(_lib().vmc_traj_accepts(self.h, C.c_void_p(out.data_ptr())), "vmc_traj_accepts")
        return out

    def set_param_stats(self, on=True):
        """Accumulate the Jastrow parameters' logarithmic derivatives in later energy_forces calls."""
        _check(_lib().vmc_traj_set_param_stats(self.h, int(bool(on))), "vmc_traj_set_param_stats")

    def param_stats(self):
        """[E, <O> (7), <E_L O> (7), <O O^T> (49)] of the last energy_forces call (device tensor);
        the parameters are (b, b_1, f_11, f_12, f_22, f_1, f_2)."""
        import torch
        out = torch.empty(OPT_STATS, dtype=torch.float64, device="cuda")
        _check(_lib().vmc_traj_param_stats(self.h, C.c_void_p(out.data_ptr())), "vmc_traj_param_stats")
        return out

    def set_jastrow(self, b, b1, j3, j1f=None):
        """New Jastrow parameters (Pade b, one-body b_1, three-body (f11, f12, f22), one-body orbital
        part (f1, f2); None keeps the current f) for later calls."""
        _check(_lib().vmc_traj_set_jastrow(self.h, float(b), float(b1), (C.c_double * 3)(*j3),
                                           None if j1f is None else (C.c_double * 2)(*j1f)),
               "vmc_traj_set_jastrow")

    def build_S(self, S=None, keep_only=False):
        """S of the last estimate; keep_only: leave it on the device in the trajectory only."""
        if keep_only:
            _check(_lib().vmc_build_S(self.h, None), "vmc_build_S")
            return None
        return vmc_build_S(self, S)

    def set_R(self, R):
        _check(_lib().vmc_traj_set_R(self.h, _dev(R, 3 * self.N)), "vmc_traj_set_R")

    def get_R(self):
        import torch
        out = torch.empty(3 * self.N, dtype=torch.float64, device="cuda")
        _check(_lib().vmc_traj_get_R(self.h, _dev(out)), "vmc_traj_get_R")
        return out

    def step_count(self):
        n = C.c_uint32(0)
        _check(_lib().vmc_traj_step_count(self.h, C.byref(n)), "vmc_traj_step_count")
        return n.value

    def langevin_step(self, T, Delta, alpha, flags=0):
        """vmc_traj_langevin_step on the trajectory's own state; returns the status code."""
        return _lib().vmc_traj_langevin_step(self.h, float(T), float(Delta), float(alpha), int(flags))

    def walkers_reset(self) -> int:
        """Walkers re-initialised (non-finite coordinates) at the start of the last call."""
        n = C.c_int(0)
        _check(_lib().vmc_traj_walkers_reset(self.h, C.byref(n)), "vmc_traj_walkers_reset")
        return n.value

    def save(self) -> bytes:
        """Checkpoint of the trajectory's own state (see vmc_traj_save)."""
        n = C.c_size_t(0)
        _check(_lib().vmc_traj_save(self.h, None, C.byref(n)), "vmc_traj_save")
        buf = C.create_string_buffer(n.value)
        _check(_lib().vmc_traj_save(self.h, buf, C.byref(n)), "vmc_traj_save")
        return buf.raw[:n.value]

    def load(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(_lib().vmc_traj_load(self.h, buf, len(data)), "vmc_traj_load")

    def load_rescaled(self, data: bytes):
        """Restart from a checkpoint taken in another box: walkers scaled by L / L*
        (see vmc_traj_load_rescaled); the caller scales R by the same factor."""
        buf = C.create_string_buffer(data, len(data))
        _check(_lib().vmc_traj_load_rescaled(self.h, buf, len(data)), "vmc_traj_load_rescaled")

    def close(self):
        if self.h:
            _lib().vmc_traj_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vmc_energy_forces(traj: Trajectory, R, Cmo, zeta, n_equil, n_sweeps, delta, step=0, out=None):
    """R None: the trajectory's R; step None: its Langevin step counter (VMC_STEP_TRAJ)."""
    import torch
    N = traj.N
    if out is None:
        out = torch.empty(3 + 3 * N, dtype=torch.float64, device="cuda")
    _check(_lib().vmc_energy_forces(traj.h, None if R is None else _dev(R, 3 * N), _dev(Cmo, _c_doubles(traj.sys)),
                                    _dev(zeta, N), int(n_equil), int(n_sweeps), float(delta),
                                    VMC_STEP_TRAJ if step is None else int(step), _dev(out, 3 + 3 * N)),
           "vmc_energy_forces")
    return out


def vmc_build_S(traj: Trajectory, S=None):
    import torch
    n3 = 3 * traj.N
    if S is None:
        S = torch.empty((n3, n3), dtype=torch.float64, device="cuda")
    _check(_lib().vmc_build_S(traj.h, _dev(S, n3 * n3)), "vmc_build_S")
    return S


def vmc_build_S_raw(ctx: Context, f_w, f, S=None):
    import torch
    W, n3 = f_w.shape
    if S is None:
        S = torch.empty((n3, n3), dtype=torch.float64, device="cuda")
    _check(_lib().vmc_build_S_raw(ctx.h, W, n3, _dev(f_w), _dev(f, n3), _dev(S, n3 * n3)), "vmc_build_S_raw")
    return S


def vmc_langevin_step(ctx: Context, R, R_prev, S_prev, f, S, T, Delta, alpha, flags=0, seed=0, traj_id=0, step=0,
                      box_L=0.0):
    """One adopted-scheme step; R, R_prev, S_prev are updated in place.  Returns the status code
    (VMC_OK or VMC_ENOTSPD/VMC_EINVAL) instead of raising, so callers can test failure handling."""
    n3 = R.numel()
    return _lib().vmc_langevin_step(ctx.h, n3, float(box_L), _dev(R), _dev(R_prev, n3), _dev(S_prev, n3 * n3),
                                    _dev(f, n3), _dev(S, n3 * n3), float(T), float(Delta), float(alpha), int(flags),
                                    int(seed), int(traj_id), int(step))


def vmc_langevin_step_noalloc(ctx: Context, R, R_prev, S_prev, f, S, T, Delta, alpha, flags=0, seed=0, traj_id=0,
                              step=0, box_L=0.0):
    """vmc_langevin_step without any allocation (the library's static device scratch, 3N <= 768);
    returns the status code."""
    n3 = R.numel()
    return _lib().vmc_langevin_step_noalloc(ctx.h, n3, float(box_L), _dev(R), _dev(R_prev, n3),
                                            _dev(S_prev, n3 * n3), _dev(f, n3), _dev(S, n3 * n3), float(T),
                                            float(Delta), float(alpha), int(flags), int(seed), int(traj_id),
                                            int(step))


class vmc_toy_params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("k", C.c_double), ("a", C.c_double), ("mu", C.c_double),
                ("s_kind", C.c_int), ("T", C.c_double), ("Delta", C.c_double), ("alpha", C.c_double),
                ("scheme", C.c_int)]


TOY_S_G, TOY_S_HESSIAN, TOY_S_IDENTITY, TOY_S_HESSIAN_SHIFT = 0, 1, 2, 3
TOY_FINALDYN_NEW, TOY_NOROGNA, TOY_EXPLICIT_GAMMA, TOY_TWO_S = 0, 1, 2, 3


def vmc_toy_run(ctx: Context, R0, n_steps, lam, k, a, mu, s_kind, T, Delta, alpha, scheme, seed=0):
    """Independent toy-model trajectories (one GPU thread each) from R0 (n x 2 CUDA float64).
    Returns (R, U_mean, status) tensors on the device."""
    import torch
    n = R0.shape[0]
    R = torch.empty_like(R0)
    U = torch.empty(n, dtype=torch.float64, device=R0.device)
    st = torch.empty(n, dtype=torch.int32, device=R0.device)
    p = vmc_toy_params(float(lam), float(k), float(a), float(mu), int(s_kind), float(T), float(Delta),
                       float(alpha), int(scheme))
    _check(_lib().vmc_toy_run(ctx.h, C.byref(p), n, int(n_steps), int(seed), _dev(R0, 2 * n), _dev(R, 2 * n),
                              _dev(U, n), C.c_void_p(st.data_ptr())), "vmc_toy_run")
    return R, U, st


def vmc_eval_configs(ctx: Context, system: vmc_system, R, Cmo, zeta, pos, out=None):
    import torch
    N = system.n_protons
    K = pos.shape[0]
    if out is None:
        out = torch.empty((K, 2 + 6 * N), dtype=torch.float64, device="cuda")
    _check(_lib().vmc_eval_configs(ctx.h, C.byref(system), _dev(R, 3 * N), _dev(Cmo, _c_doubles(system)), _dev(zeta, N),
                                   K, _dev(pos, K * N * 3), _dev(out, K * (2 + 6 * N))), "vmc_eval_configs")
    return out


def vmc_huckel_params(R, zeta, L, twist=0):
    """Host helper (numpy in, numpy out); twist: bit m = twist angle pi along axis m."""
    import numpy as np
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    n = zeta.size
    Cm = np.zeros((n, n // 2))
    P = C.POINTER(C.c_double)
    if twist == 0:
        _check(_lib().vmc_huckel_params(n, float(L), R.ctypes.data_as(P), zeta.ctypes.data_as(P),
                                        Cm.ctypes.data_as(P)), "vmc_huckel_params")
    else:
        _check(_lib().vmc_huckel_params_twist(n, float(L), int(twist), R.ctypes.data_as(P), zeta.ctypes.data_as(P),
                                              Cm.ctypes.data_as(P)), "vmc_huckel_params_twist")
    return Cm


def vmc_sr_update(stats, active, eps, tau):
    """Host helper: one stochastic-reconfiguration step dp (numpy, 7) from the 64 means of
    Trajectory.param_stats (a tensor or an array)."""
    import numpy as np
    st = np.ascontiguousarray(stats.cpu().numpy() if hasattr(stats, "cpu") else stats, dtype=np.float64)
    assert st.shape == (OPT_STATS,)
    dp = np.zeros(OPT_PAR)
    P = C.POINTER(C.c_double)
    _check(_lib().vmc_sr_update(st.ctypes.data_as(P), int(active), float(eps), float(tau), dp.ctypes.data_as(P)),
           "vmc_sr_update")
    return dp


def vmc_huckel_params_contracted(R, L, eta):
    """Host helper: real N x N/2 orbital coefficients on the contracted basis (numpy)."""
    import numpy as np
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    n = R.size // 3
    Cm = np.zeros((n, n // 2))
    P = C.POINTER(C.c_double)
    _check(_lib().vmc_huckel_params_contracted(n, float(L), float(eta), R.ctypes.data_as(P), Cm.ctypes.data_as(P)),
           "vmc_huckel_params_contracted")
    return Cm


def vmc_huckel_params_theta(R, zeta, L, theta):
    """Host helper for a general twist: complex N x N/2 orbital coefficients (numpy complex128)."""
    import numpy as np
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    n = zeta.size
    Cm = np.zeros((n, n // 2, 2))
    P = C.POINTER(C.c_double)
    _check(_lib().vmc_huckel_params_theta(n, float(L), th.ctypes.data_as(P), R.ctypes.data_as(P),
                                          zeta.ctypes.data_as(P), Cm.ctypes.data_as(P)), "vmc_huckel_params_theta")
    return Cm.view(np.complex128)[..., 0]


def vmc_huckel_params_theta_contracted(R, L, theta, eta):
    """Host helper for a general twist on the contracted basis: complex N x N/2 coefficients."""
    import numpy as np
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    n = R.size // 3
    Cm = np.zeros((n, n // 2, 2))
    P = C.POINTER(C.c_double)
    _check(_lib().vmc_huckel_params_theta_contracted(n, float(L), th.ctypes.data_as(P), float(eta), R.ctypes.data_as(P),
                                                     Cm.ctypes.data_as(P)), "vmc_huckel_params_theta_contracted")
    return Cm.view(np.complex128)[..., 0]


def vmc_twist_average(ctx: Context, f_stack, S_stack, f=None, S=None):
    """Force and covariance of the twist average: f_stack (n_tw x n3), S_stack (n_tw x n3 x n3)."""
    import torch
    n_tw, n3 = f_stack.shape
    if f is None:
        f = torch.empty(n3, dtype=torch.float64, device="cuda")
    if S is None:
        S = torch.empty((n3, n3), dtype=torch.float64, device="cuda")
    _check(_lib().vmc_twist_average(ctx.h, n_tw, n3, _dev(f_stack, n_tw * n3), _dev(S_stack, n_tw * n3 * n3),
                                    _dev(f, n3), _dev(S, n3 * n3)), "vmc_twist_average")
    return f, S


def traj_bytes(system: vmc_system, n_walkers: int) -> int:
    return int(_lib().vmc_traj_bytes(C.byref(system), int(n_walkers)))


def supported_n(n):
    return bool(_lib().vmc_supported_n(int(n)))


def library_path():
    return LIB_PATH


def _host(a, n):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} elements, got {a.size}")
    return a


def make_request(sysd, W, R0, zeta, pos0, n_steps, n_sweeps, T, Delta, alpha, n_equil_first=20, n_equil=5,
                 step_delta=1.0, flags=0, seed=1, traj_id=0):
    """A vmc_request (the arrays are kept alive on the returned object until submit)."""
    n = sysd.n_protons
    R0, zeta, pos0 = _host(R0, 3 * n), _host(zeta, n), _host(pos0, W * n * 3)
    P = C.POINTER(C.c_double)
    r = vmc_request(sysd, int(W), int(n_equil_first), int(n_equil), int(n_sweeps), int(n_steps), float(step_delta),
                    float(T), float(Delta), float(alpha), int(flags), int(seed), int(traj_id),
                    R0.ctypes.data_as(P), zeta.ctypes.data_as(P), pos0.ctypes.data_as(P))
    r._keep = (R0, zeta, pos0)
    return r


def request_bytes(req):
    return int(_lib().vmc_request_bytes(C.byref(req)))


def admit_count(budget, resident, queued_bytes):
    arr = (C.c_size_t * max(len(queued_bytes), 1))(*[int(b) for b in queued_bytes])
    return int(_lib().vmc_server_admit_count(int(budget), int(resident), len(queued_bytes), arr))


class Server:
    """Continuous-batching request loop over one context (vmc_server_*)."""

    def __init__(self, ctx, hbm_budget_bytes):
        self.ctx = ctx
        self.h = C.c_void_p()
        _check(_lib().vmc_server_create(ctx.h, int(hbm_budget_bytes), C.byref(self.h)), "vmc_server_create")
        self._n = {}

    def submit(self, req):
        i = C.c_int()
        _check(_lib().vmc_server_submit(self.h, C.byref(req), C.byref(i)), "vmc_server_submit")
        self._n[i.value] = (req.sys.n_protons, req.n_steps)
        return i.value

    def cancel(self, rid):
        _check(_lib().vmc_server_cancel(self.h, int(rid)), "vmc_server_cancel")

    def tick(self):
        a, q = C.c_int(), C.c_int()
        _check(_lib().vmc_server_tick(self.h, C.byref(a), C.byref(q)), "vmc_server_tick")
        return a.value, q.value

    def status(self, rid):
        s, k, e = C.c_int(), C.c_int(), C.c_int()
        _check(_lib().vmc_server_status(self.h, int(rid), C.byref(s), C.byref(k), C.byref(e)), "vmc_server_status")
        return s.value, k.value, e.value

    def result(self, rid):
        import numpy as np
        n, steps = self._n[rid]
        R = np.zeros(3 * n)
        E, sg, lat = np.zeros(steps), np.zeros(steps), np.zeros(steps)
        w = C.c_double()
        P = C.POINTER(C.c_double)
        _check(_lib().vmc_server_result(self.h, int(rid), R.ctypes.data_as(P), E.ctypes.data_as(P),
                                        sg.ctypes.data_as(P), lat.ctypes.data_as(P), C.byref(w)),
               "vmc_server_result")
        k = self.status(rid)[1]
        return dict(R=R, E=E[:k], sigma_E=sg[:k], latency_ms=lat[:k], wait_ms=w.value)

    def info(self):
        r, p, a, q, t = C.c_size_t(), C.c_size_t(), C.c_int(), C.c_int(), C.c_longlong()
        _check(_lib().vmc_server_info(self.h, C.byref(r), C.byref(p), C.byref(a), C.byref(q), C.byref(t)),
               "vmc_server_info")
        return dict(resident=r.value, peak_resident=p.value, active=a.value, queued=q.value, ticks=t.value)

    def run_until_idle(self, max_ticks=10 ** 7):
        for _ in range(max_ticks):
            a, q = self.tick()
            if a == 0 and q == 0:
                return
        raise RuntimeError("server did not drain")

    def close(self):
        if self.h:
            _lib().vmc_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
