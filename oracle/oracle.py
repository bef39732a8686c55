"""ctypes wrapper of the plain FP64 CPU oracle (oracle/vmc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py; never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OB_PERIODIC_GAUSS, OB_OPEN_GAUSS, OB_OPEN_STO = 0, 1, 2
OP_EWALD, OP_COULOMB_OPEN, OP_HARMONIC, OP_NONE = 0, 1, 2, 3
STEP_CFOLD, STEP_NOISE_CORR, STEP_NO_SCORR = 1, 2, 4


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) and OpenMP over walkers."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", LIB_PATH,
           os.path.join(HERE, "vmc_oracle.c"), os.path.join(HERE, "vmc_oracle_complex.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return LIB_PATH


class OSys(C.Structure):
    _fields_ = [("n_p", C.c_int), ("n_up", C.c_int), ("n_dn", C.c_int), ("n_orb", C.c_int),
                ("L", C.c_double), ("basis_kind", C.c_int), ("pot_kind", C.c_int),
                ("kappa", C.c_double), ("nmax", C.c_int), ("jastrow_on", C.c_int),
                ("a_par", C.c_double), ("a_anti", C.c_double), ("b", C.c_double),
                ("R", C.POINTER(C.c_double)), ("zeta", C.POINTER(C.c_double)),
                ("C", C.POINTER(C.c_double)), ("b1", C.c_double), ("twist", C.c_int),
                ("contracted", C.c_int), ("eta", C.c_double), ("j3f", C.c_double * 3),
                ("j1f", C.c_double * 2)]


Z1, Z2 = 0.6066825, 0.3382168   # the SI's exponents of the contracted minimal basis
ZJ = 0.7933844                  # the exponent of the Jastrow orbitals


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _setup(_lib)
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _setup(l):
    P = C.POINTER
    d, i, u32 = C.c_double, C.c_int, C.c_uint32
    l.o_philox.argtypes = [P(u32), P(u32), P(u32)]
    l.o_u01.argtypes = [u32, u32]
    l.o_u01.restype = d
    l.o_normals.argtypes = [u32, u32, u32, i, P(d)]
    l.o_basis.argtypes = [P(OSys), i, P(d), P(d)]
    l.o_jastrow.argtypes = [P(OSys), P(d), P(d), P(d), P(d)]
    l.o_potential.argtypes = [P(OSys), P(d), P(d), P(d)]
    l.o_potential.restype = d
    l.o_local.argtypes = [P(OSys), P(d), P(d), P(d), P(d), P(d), P(d)]
    l.o_huckel.argtypes = [i, d, P(d), P(d), i, P(d), P(d)]
    l.o_huckel_twist.argtypes = [i, d, P(d), P(d), i, i, P(d), P(d)]
    l.o_vmc_run.argtypes = [P(OSys), i, P(d), i, i, d, u32, u32, u32, P(d), P(C.c_int64), i]
    l.o_vmc_run_from.argtypes = [P(OSys), i, u32, P(d), i, i, d, u32, u32, u32, P(d), P(C.c_int64), i]
    l.o_vmc_run_opt.argtypes = [P(OSys), i, u32, P(d), i, i, d, u32, u32, u32, P(d), P(C.c_int64), P(d), i]
    l.o_param_derivs.argtypes = [P(OSys), P(d), P(d)]
    l.o_reduce.argtypes = [i, i, i, P(d), P(d), P(d), P(d), P(d), P(d)]
    l.o_build_S.argtypes = [i, i, P(d), P(d), P(d)]
    l.o_build_S.restype = None
    l.o_cholesky.argtypes = [i, P(d), P(d)]
    l.o_langevin.argtypes = [i, d, P(d), P(d), P(d), P(d), P(d), d, d, d, C.c_uint, u32, u32, u32]
    l.o_langevin_harmonic_run.argtypes = [i, P(d), P(d), d, d, d, C.c_uint, u32, i, P(d), P(d), i]
    l.o_toy_run.argtypes = [d, d, d, d, i, d, d, d, i, u32, u32, i, P(d), P(d), P(d)]
    l.o_toy_S.argtypes = [d, d, d, d, i, P(d), P(d)]
    l.o_toy_S.restype = None
    l.o_cbasis.argtypes = [P(OSys), P(d), i, P(d), P(d)]
    l.o_cbasis.restype = None
    l.o_cbasis_values.argtypes = [P(OSys), P(d), i, P(d), P(d)]
    l.o_cbasis_values.restype = None
    l.o_coverlap.argtypes = [i, d, P(d), P(d), P(d), P(d)]
    l.o_coverlap.restype = None
    l.o_chuckel.argtypes = [i, d, P(d), P(d), P(d), i, P(d), P(d)]
    l.o_coverlap_contracted.argtypes = [i, d, P(d), P(d), d, P(d)]
    l.o_coverlap_contracted.restype = None
    l.o_chuckel_contracted.argtypes = [i, d, P(d), P(d), d, i, P(d), P(d)]
    l.o_clocal.argtypes = [P(OSys), P(d), P(d), P(d), P(d), P(d), P(d), P(d), P(d)]
    l.o_j3_orbitals.argtypes = [P(OSys), i, P(d), P(d)]
    l.o_j3_orbitals.restype = None
    l.o_huckel_contracted.argtypes = [i, d, P(d), d, i, P(d), P(d)]
    l.o_overlap_contracted.argtypes = [i, d, P(d), d, P(d)]
    l.o_overlap_contracted.restype = None
    l.o_cvmc_run_from.argtypes = [P(OSys), P(d), P(d), i, u32, P(d), i, i, d, u32, u32, u32, P(d), P(C.c_int64), i]


class System:
    """Holds the arrays an OSys points to (keeps them alive)."""

    def __init__(self, R, zeta, C_mo, L=0.0, n_up=None, n_dn=None, basis=OB_PERIODIC_GAUSS,
                 pot=OP_EWALD, kappa=None, nmax=9, jastrow=True, a_par=0.25, a_anti=0.5, b=1.0,
                 b1=0.0, twist=0, eta=None, j3=None, j1f=None):
        self.R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, 3)
        n_p = self.R.shape[0]
        self.zeta = np.ascontiguousarray(zeta, dtype=np.float64).reshape(n_p)
        self.C = np.ascontiguousarray(C_mo, dtype=np.float64).reshape(n_p, -1)
        if n_up is None:
            n_up = n_p // 2
        if n_dn is None:
            n_dn = n_p - n_up
        self.n_up, self.n_dn, self.L = n_up, n_dn, float(L)
        if kappa is None:
            kappa = 8.0 / L if L > 0 else 0.0
        # eta given: the contracted orbital phi_1 + eta phi_2 (zeta unused)
        self.s = OSys(n_p, n_up, n_dn, self.C.shape[1], float(L), basis, pot, float(kappa), int(nmax),
                      int(bool(jastrow)), a_par, a_anti, b, _dp(self.R), _dp(self.zeta), _dp(self.C),
                      float(b1), int(twist), int(eta is not None), float(eta or 0.0),
                      (C.c_double * 3)(*(j3 if j3 is not None else (0.0, 0.0, 0.0))),
                      (C.c_double * 2)(*(j1f if j1f is not None else (0.0, 0.0))))

    @property
    def n_p(self):
        return self.R.shape[0]

    @property
    def ne(self):
        return self.n_up + self.n_dn

    def basis(self, a, r):
        out = np.zeros(14)
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().o_basis(C.byref(self.s), a, _dp(r), _dp(out))
        return out

    def j3_orbitals(self, a, r):
        out = np.zeros(28)
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().o_j3_orbitals(C.byref(self.s), a, _dp(r), _dp(out))
        return out[:14], out[14:]

    def jastrow(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        U = np.zeros(1)
        g = np.zeros((self.ne, 3))
        lp = np.zeros(self.ne)
        lib().o_jastrow(C.byref(self.s), _dp(x), _dp(U), _dp(g), _dp(lp))
        return U[0], g, lp

    def potential(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        dR = np.zeros((self.n_p, 3))
        dx = np.zeros((self.ne, 3))
        V = lib().o_potential(C.byref(self.s), _dp(x), _dp(dR), _dp(dx))
        return V, dR, dx

    def local(self, x, derivs=True):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lnpsi, sign, EL = np.zeros(1), np.zeros(1), np.zeros(1)
        dl = np.zeros(3 * self.n_p)
        de = np.zeros(3 * self.n_p)
        rc = lib().o_local(C.byref(self.s), _dp(x), _dp(lnpsi), _dp(sign), _dp(EL),
                           _dp(dl) if derivs else None, _dp(de) if derivs else None)
        if rc:
            raise RuntimeError(f"o_local failed rc={rc}")
        return dict(lnpsi=lnpsi[0], sign=sign[0], EL=EL[0], dlnpsi=dl, dEL=de)

    def vmc_run(self, x, n_equil, n_meas, delta, seed, traj=0, step=0, threads=0, walker0=0, params=False):
        """Runs the Metropolis chains in place on x (W, Ne, 3); returns (sums, n_acc), and with
        params=True also the per-walker parameter sums (W, NOPT): [sum E_L, sum O (NPAR),
        sum E_L O (NPAR), sum O O^T (NPAR^2)] over the measured samples.  x holds walkers walker0 .. walker0+W-1 of a
        larger set (their random streams)."""
        assert x.dtype == np.float64 and x.flags.c_contiguous
        W = x.shape[0]
        n3 = 3 * self.n_p
        sums = np.zeros((W, 2 + 3 * n3))
        nacc = np.zeros(W, dtype=np.int64)
        popt = np.zeros((W, NOPT)) if params else None
        rc = lib().o_vmc_run_opt(C.byref(self.s), W, walker0, _dp(x), n_equil, n_meas, delta, seed, traj, step,
                                 _dp(sums), nacc.ctypes.data_as(C.POINTER(C.c_int64)),
                                 _dp(popt) if params else None, threads)
        if rc:
            raise RuntimeError(f"o_vmc_run failed rc={rc}")
        return (sums, nacc, popt) if params else (sums, nacc)

    def param_derivs(self, x):
        """O_k = d ln psi / d p_k for p = (b, b_1, f_11, f_12, f_22, f_1, f_2) at the configuration x."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        O = np.zeros(NPAR)
        lib().o_param_derivs(C.byref(self.s), _dp(x), _dp(O))
        return O


class CSystem(System):
    """A System with a general twist theta (radians, per axis) and complex orbitals Cc
    (n_p x n_orb complex): the Bloch-summed Gaussian basis of vmc_oracle_complex.c."""

    def __init__(self, R, zeta, Cc, theta, L, **kw):
        Cc = np.ascontiguousarray(Cc, dtype=np.complex128).reshape(len(zeta), -1)
        super().__init__(R, zeta, np.zeros(Cc.shape), L=L, **kw)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
        self.Cc = Cc
        self.Cpairs = np.ascontiguousarray(Cc.view(np.float64))

    def cbasis(self, a, r):
        out = np.zeros(28)
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().o_cbasis(C.byref(self.s), _dp(self.theta), a, _dp(r), _dp(out))
        return out.view(np.complex128)

    def cbasis_values(self, pts):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        out = np.zeros((pts.shape[0], self.n_p, 2))
        lib().o_cbasis_values(C.byref(self.s), _dp(self.theta), pts.shape[0], _dp(pts), _dp(out))
        return out.view(np.complex128)[..., 0]

    def local(self, x, derivs=True):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lnpsi, phase, EL = np.zeros(1), np.zeros(1), np.zeros(1)
        dl = np.zeros(3 * self.n_p)
        de = np.zeros(3 * self.n_p)
        rc = lib().o_clocal(C.byref(self.s), _dp(self.theta), _dp(self.Cpairs), _dp(x), _dp(lnpsi), _dp(phase),
                            _dp(EL), _dp(dl) if derivs else None, _dp(de) if derivs else None)
        if rc:
            raise RuntimeError(f"o_clocal failed rc={rc}")
        return dict(lnpsi=lnpsi[0], phase=phase[0], EL=EL[0], dlnpsi=dl, dEL=de)

    def vmc_run(self, x, n_equil, n_meas, delta, seed, traj=0, step=0, threads=0, walker0=0):
        assert x.dtype == np.float64 and x.flags.c_contiguous
        W = x.shape[0]
        n3 = 3 * self.n_p
        sums = np.zeros((W, 2 + 3 * n3))
        nacc = np.zeros(W, dtype=np.int64)
        rc = lib().o_cvmc_run_from(C.byref(self.s), _dp(self.theta), _dp(self.Cpairs), W, walker0, _dp(x), n_equil,
                                   n_meas, delta, seed, traj, step, _dp(sums),
                                   nacc.ctypes.data_as(C.POINTER(C.c_int64)), threads)
        if rc:
            raise RuntimeError(f"o_cvmc_run failed rc={rc}")
        return sums, nacc


def coverlap(R, zeta, L, theta):
    R = np.ascontiguousarray(R, dtype=np.float64)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = zeta.size
    S = np.zeros((n, n, 2))
    lib().o_coverlap(n, L, _dp(theta), _dp(R), _dp(zeta), _dp(S))
    return S.view(np.complex128)[..., 0]


def chuckel(R, zeta, L, n_orb, theta):
    R = np.ascontiguousarray(R, dtype=np.float64)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = zeta.size
    Cm = np.zeros((n, n_orb, 2))
    ev = np.zeros(n)
    rc = lib().o_chuckel(n, L, _dp(theta), _dp(R), _dp(zeta), n_orb, _dp(Cm), _dp(ev))
    if rc:
        raise RuntimeError("o_chuckel failed")
    return Cm.view(np.complex128)[..., 0], ev


def coverlap_contracted(R, L, eta, theta):
    R = np.ascontiguousarray(R, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = R.size // 3
    S = np.zeros((n, n, 2))
    lib().o_coverlap_contracted(n, L, _dp(theta), _dp(R), float(eta), _dp(S))
    return S.view(np.complex128)[..., 0]


def chuckel_contracted(R, L, n_orb, eta, theta):
    R = np.ascontiguousarray(R, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = R.size // 3
    Cm = np.zeros((n, n_orb, 2))
    ev = np.zeros(n)
    rc = lib().o_chuckel_contracted(n, L, _dp(theta), _dp(R), float(eta), n_orb, _dp(Cm), _dp(ev))
    if rc:
        raise RuntimeError("o_chuckel_contracted failed")
    return Cm.view(np.complex128)[..., 0], ev


def monkhorst_pack(q=4):
    """Twists of the q x q x q Monkhorst-Pack mesh: theta_m = 2 pi (2 n - q - 1) / (2 q), n = 1..q."""
    t = [2.0 * np.pi * (2 * n - q - 1) / (2 * q) for n in range(1, q + 1)]
    return np.array([(a, b, c) for a in t for b in t for c in t])


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().o_philox(c, k, o)
    return list(o)


def u01(hi, lo):
    return lib().o_u01(hi, lo)


def normals(seed, traj, step, n):
    xi = np.zeros(n)
    lib().o_normals(seed, traj, step, n, _dp(xi))
    return xi


def huckel(R, zeta, L, n_orb, twist=0):
    R = np.ascontiguousarray(R, dtype=np.float64)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    n_p = R.shape[0]
    Cm = np.zeros((n_p, n_orb))
    ev = np.zeros(n_p)
    rc = lib().o_huckel_twist(n_p, L, _dp(R), _dp(zeta), n_orb, int(twist), _dp(Cm), _dp(ev))
    if rc:
        raise RuntimeError("o_huckel failed")
    return Cm, ev


def huckel_contracted(R, L, n_orb, eta):
    """Hueckel orbitals on the contracted basis phi_1 + eta phi_2 and all eigenvalues."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    n_p = R.shape[0]
    Cm = np.zeros((n_p, n_orb))
    ev = np.zeros(n_p)
    rc = lib().o_huckel_contracted(n_p, float(L), _dp(R), float(eta), n_orb, _dp(Cm), _dp(ev))
    if rc:
        raise RuntimeError("o_huckel_contracted failed")
    return Cm, ev


def overlap_contracted(R, L, eta):
    R = np.ascontiguousarray(R, dtype=np.float64)
    n_p = R.shape[0]
    S = np.zeros((n_p, n_p))
    lib().o_overlap_contracted(n_p, float(L), _dp(R), float(eta), _dp(S))
    return S


def reduce(sums, M):
    W, nsum = sums.shape
    n3 = (nsum - 2) // 3
    E, sig = np.zeros(1), np.zeros(1)
    f = np.zeros(n3)
    fw = np.zeros((W, n3))
    means = np.zeros((W, 1 + 3 * n3))
    rc = lib().o_reduce(W, n3, M, _dp(np.ascontiguousarray(sums)), _dp(E), _dp(sig), _dp(f), _dp(fw), _dp(means))
    if rc:
        raise RuntimeError("o_reduce failed")
    return dict(E=E[0], sigma_E=sig[0], f=f, f_w=fw, means=means)


# the Jastrow parameters (two-body b, one-body cusp b_1, three-body F, one-body orbital part f) and
# the per-walker parameter sums of o_vmc_run_opt: [sum E_L, sum O (7), sum E_L O (7), sum O O^T (49)]
PARAM_NAMES = ("b", "b1", "f11", "f12", "f22", "f1", "f2")
NPAR = len(PARAM_NAMES)
NOPT = 1 + 2 * NPAR + NPAR * NPAR


def param_stats(popt, M):
    """Means over the W M samples of a run: [E, <O> (NPAR), <E_L O> (NPAR), <O O^T> (NPAR^2)]."""
    popt = np.asarray(popt, dtype=np.float64)
    return popt.sum(axis=0) / (popt.shape[0] * M)


def sr_step(stats, active, eps, tau):
    """One step of stochastic reconfiguration (Sorella, PRB 64, 024512 (2001)) from the sample
    means of param_stats: the generalised forces f_k = -dE/dp_k = -2 (<E_L O_k> - E <O_k>), the
    covariance S_kl = <O_k O_l> - <O_k><O_l> of the logarithmic derivatives, its diagonal scaled
    by (1 + eps), and the change dp = tau S^-1 f over the parameters whose bit is set in active
    (the others stay).  Returns (dp, f, S)."""
    stats = np.asarray(stats, dtype=np.float64)
    n = NPAR
    E, O, EO, OO = stats[0], stats[1:1 + n], stats[1 + n:1 + 2 * n], stats[1 + 2 * n:NOPT].reshape(n, n)
    f = -2.0 * (EO - E * O)
    S = OO - np.outer(O, O)
    idx = [k for k in range(n) if (active >> k) & 1]
    dp = np.zeros(n)
    if idx:
        Sa = S[np.ix_(idx, idx)].copy()
        Sa[np.diag_indices_from(Sa)] *= 1.0 + eps
        dp[idx] = tau * np.linalg.solve(Sa, f[idx])
    return dp, f, S


def build_S(f_w, f):
    f_w = np.ascontiguousarray(f_w, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    W, n3 = f_w.shape
    S = np.zeros((n3, n3))
    lib().o_build_S(W, n3, _dp(f_w), _dp(f), _dp(S))
    return S


def cholesky(S):
    S = np.ascontiguousarray(S, dtype=np.float64)
    Lc = np.zeros_like(S)
    rc = lib().o_cholesky(S.shape[0], _dp(S), _dp(Lc))
    return rc, Lc


def langevin(R, R_prev, S_prev, f, S, T, Delta, alpha, flags=0, seed=0, traj=0, step=0, L=0.0):
    """One step; R, R_prev, S_prev are updated in place (float64 contiguous arrays)."""
    for a in (R, R_prev, S_prev):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    f = np.ascontiguousarray(f, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    return lib().o_langevin(R.size, L, _dp(R), _dp(R_prev), _dp(S_prev), _dp(f), _dp(S), T, Delta,
                            alpha, flags, seed, traj, step)


def langevin_harmonic_run(K, S, T, Delta, alpha, n_steps, R0, flags=0, seed=0, sample_every=1):
    K = np.ascontiguousarray(K, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    n3 = K.shape[0]
    R = np.ascontiguousarray(R0, dtype=np.float64).copy()
    ns = n_steps // sample_every
    samples = np.zeros((ns, n3))
    rc = lib().o_langevin_harmonic_run(n3, _dp(K), _dp(S), T, Delta, alpha, flags, seed, n_steps,
                                       _dp(R), _dp(samples), sample_every)
    if rc:
        raise RuntimeError(f"harmonic run failed rc={rc}")
    return samples


def toy_run(lam, k, a, mu, s_kind, T, Delta, alpha, scheme, seed, n_steps, R0=(1.4, 0.0), keep=False, traj=0,
            final=False):
    """The rotating spring of the SI: s_kind 0 S = G_lambda, 1 S = H + mu G_lambda, 2 S = I;
    scheme 0 Eq. finaldyn_new (alpha = 0: Eq. finaldyn), 1 Eq. norogna, 2 Eq. standard with the
    Gamma term by central differences.  Noise key (seed, traj), counter = step.  Returns the
    mean U over the last 90% of the steps (and the U samples with keep, the final R with final)."""
    R = np.array(R0, dtype=np.float64)
    Um = np.zeros(1)
    Us = np.zeros(n_steps) if keep else None
    rc = lib().o_toy_run(lam, k, a, mu, s_kind, T, Delta, alpha, scheme, seed, traj, n_steps, _dp(R), _dp(Um),
                         _dp(Us) if keep else None)
    if rc:
        raise RuntimeError(f"toy run failed rc={rc}")
    out = (Um[0], Us) if keep else Um[0]
    return (out, R) if final else out


def toy_S(lam, k, a, mu, s_kind, x):
    """The toy model's acceleration matrix at the point x (2 x 2)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    S = np.zeros(4)
    lib().o_toy_S(lam, k, a, mu, int(s_kind), _dp(x), _dp(S))
    return S.reshape(2, 2)
