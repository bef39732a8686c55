"""Pins of the oracle's contracted minimal basis (SI, "Systematic setup": one orbital per proton,
phi_1 + eta phi_2 with phi_1 = e^{-Z1 r^2}, phi_2 = r^2 e^{-Z2 r^2}, Z1 = 0.6066825,
Z2 = 0.3382168), made periodic by the same image sum as the single Gaussian: the image sum of
r^2 e^{-Z r^2} is minus the Z-derivative of the Gaussian's, every derivative component by finite
differences, the closed-form cell overlaps against quadrature and against the single-Gaussian
formula at eta = 0, the Hueckel orbitals against numpy's eigen-solver, and the local energy,
proton derivatives, decisions and force estimator with the contracted basis."""
import ctypes
import itertools
import math

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system

ETAS = [0.3, -0.15]
# The image sums keep the images n = -1, 0, 1 per axis; the diffuse second Gaussian needs a box
# with Z2 (1.5 L)^2 >= 36 for the dropped images to stay below FP64 resolution: L >= 6.9 bohr.
LB = 7.5


def _box(n):
    """Synthetic boxes large enough for the contracted basis (r_s chosen so that L >= 7.3)."""
    return small_system(n, {6: 2.5, 16: 1.9}[n], seed=4)


def _one(oracle, L, eta, twist=0, zeta=1.0):
    return oracle.System(R=[[0.3, -0.2, 0.1]], zeta=[zeta], C_mo=[[1.0]], L=L, n_up=1, n_dn=0,
                         pot=oracle.OP_NONE, jastrow=False, twist=twist, eta=eta)


@pytest.mark.parametrize("eta,twist", [(0.3, 0), (-0.15, 0), (0.3, 5)])
def test_contracted_basis_is_gaussian_plus_minus_dZ(oracle, eta, twist):
    """The image sum of r^2 e^{-Z r^2} is -d/dZ of the image sum of e^{-Z r^2}: every component
    of the contracted orbital equals the single Gaussian at Z1 plus eta times the central
    difference in the exponent of the single Gaussian at Z2 (the single-Gaussian code path)."""
    L = LB
    c = _one(oracle, L, eta, twist)
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(6):
        r = c.R[0] + rng.uniform(-L, L, 3)
        g1 = _one(oracle, L, None, twist, zeta=oracle.Z1).basis(0, r)
        gp = _one(oracle, L, None, twist, zeta=oracle.Z2 + h).basis(0, r)
        gm = _one(oracle, L, None, twist, zeta=oracle.Z2 - h).basis(0, r)
        ref = g1 + eta * (gm - gp) / (2 * h)
        got = c.basis(0, r)
        assert np.allclose(got, ref, rtol=1e-7, atol=1e-8 * np.max(np.abs(ref)))


@pytest.mark.parametrize("eta,twist", [(0.3, 0), (-0.15, 3)])
def test_contracted_basis_derivatives_by_finite_differences(oracle, eta, twist):
    s = _one(oracle, LB, eta, twist)
    rng = np.random.default_rng(3)
    H = {(0, 0): 5, (1, 1): 6, (2, 2): 7, (0, 1): 8, (0, 2): 9, (1, 2): 10}
    for _ in range(5):
        r = s.R[0] + rng.uniform(-2.0, 2.0, 3)
        b = s.basis(0, r)
        h = 2e-5
        for m in range(3):
            e = np.zeros(3)
            e[m] = h
            bp, bm = s.basis(0, r + e), s.basis(0, r - e)
            assert b[1 + m] == pytest.approx((bp[0] - bm[0]) / (2 * h), rel=1e-7, abs=1e-10)
            assert b[11 + m] == pytest.approx((bp[4] - bm[4]) / (2 * h), rel=1e-7, abs=1e-9)
            for n in range(3):
                key = (min(m, n), max(m, n))
                assert b[H[key]] == pytest.approx((bp[1 + n] - bm[1 + n]) / (2 * h), rel=1e-7, abs=1e-9)
        assert b[4] == pytest.approx(b[5] + b[6] + b[7], rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("eta", ETAS)
def test_contracted_overlap_equals_cell_quadrature(oracle, eta):
    """The closed-form moments give S_ab = int_cell phi_a phi_b: against a 40^3 trapezoid rule
    of the periodic basis values (spectrally accurate for a smooth periodic integrand)."""
    wl = _box(6)
    S = oracle.overlap_contracted(wl.R, wl.L, eta)
    s = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, eta=eta)
    ng = 40
    g = (np.arange(ng) + 0.5) * wl.L / ng
    pts = np.array(list(itertools.product(g, g, g)))
    phi = np.array([[s.basis(a, p)[0] for a in range(6)] for p in pts])
    Sq = (phi.T @ phi) * (wl.L / ng) ** 3
    assert np.max(np.abs(S - Sq)) < 1e-10 * np.max(np.abs(S))
    assert np.max(np.abs(S - S.T)) < 1e-15 * np.max(np.abs(S))


def test_contracted_overlap_at_eta_zero_is_the_gaussian_formula(oracle):
    """eta = 0 leaves e^{-Z1 r^2}: the moment formula equals the single-Gaussian overlap (the
    Hueckel orbitals on zeta = Z1 span the same space with the same eigenvalues)."""
    wl = _box(16)
    C0, ev0 = oracle.huckel_contracted(wl.R, wl.L, 8, 0.0)
    Cg, evg = oracle.huckel(wl.R, np.full(wl.n, oracle.Z1), wl.L, 8)
    assert np.allclose(ev0, evg, atol=1e-13)
    assert np.allclose(C0 @ C0.T, Cg @ Cg.T, atol=1e-12)


@pytest.mark.parametrize("eta", ETAS)
def test_contracted_huckel_against_eigh(oracle, eta):
    wl = _box(16)
    Cm, ev = oracle.huckel_contracted(wl.R, wl.L, 8, eta)
    S = oracle.overlap_contracted(wl.R, wl.L, eta)
    d = np.sqrt(np.diag(S))
    w, v = np.linalg.eigh(-S / np.outer(d, d))
    assert np.allclose(ev, w, atol=1e-12)
    Cn = v[:, :8] / d[:, None]
    assert np.allclose(Cm @ Cm.T, Cn @ Cn.T, atol=1e-12)
    assert np.allclose(Cm.T @ S @ Cm, np.diag(-w[:8]), atol=1e-12)


def _csys(oracle, wl, eta, b1=0.0):
    Cm, _ = oracle.huckel_contracted(wl.R, wl.L, wl.n // 2, eta)
    return Cm, oracle.System(wl.R, wl.zeta, Cm, L=wl.L, b1=b1, eta=eta)


@pytest.mark.parametrize("name,eta,b1", [("h6", 0.3, 0.0), ("h16", -0.15, 0.0), ("h6", 0.3, 1.7)])
def test_contracted_kinetic_energy_against_fd_laplacian(oracle, name, eta, b1):
    wl = _box(16 if name == "h16" else 6)
    _, s = _csys(oracle, wl, eta, b1)
    x = wl.electrons(W=1)[0]
    res = s.local(x, derivs=False)
    V, _, _ = s.potential(x)
    lp0 = res["lnpsi"]

    def T_fd(h):
        T = 0.0
        for i in range(x.shape[0]):
            for m in range(3):
                xp, xm = x.copy(), x.copy()
                xp[i, m] += h
                xm[i, m] -= h
                lpp, lpm = s.local(xp, False)["lnpsi"], s.local(xm, False)["lnpsi"]
                T += -0.5 * ((lpp - 2 * lp0 + lpm) / h ** 2 + ((lpp - lpm) / (2 * h)) ** 2)
        return T

    # the r^2 term makes psi vary faster than a single Gaussian: Richardson's combination of the
    # steps h and h/2 removes the O(h^2) error of the second differences
    T = (4 * T_fd(1e-4) - T_fd(2e-4)) / 3
    assert res["EL"] - V == pytest.approx(T, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("name,eta,b1", [("h6", 0.3, 0.0), ("h16", -0.15, 0.0), ("h6", -0.15, 1.7)])
def test_contracted_proton_derivatives_by_finite_differences(oracle, name, eta, b1):
    wl = _box(16 if name == "h16" else 6)
    Cm, s = _csys(oracle, wl, eta, b1)
    x = wl.electrons(W=1)[0]
    res = s.local(x)
    h = 1e-5
    for t in range(0, 3 * wl.n, 1 if wl.n <= 6 else 5):
        Rp = wl.R.reshape(-1).copy()
        Rm = Rp.copy()
        Rp[t] += h
        Rm[t] -= h
        a = oracle.System(Rp.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, eta=eta).local(x, False)
        b = oracle.System(Rm.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, eta=eta).local(x, False)
        assert res["dlnpsi"][t] == pytest.approx((a["lnpsi"] - b["lnpsi"]) / (2 * h), rel=1e-7, abs=1e-8)
        assert res["dEL"][t] == pytest.approx((a["EL"] - b["EL"]) / (2 * h), rel=1e-6, abs=1e-7)


def test_contracted_sweep_decisions_follow_psi_ratios(oracle):
    wl = _box(6)
    _, s = _csys(oracle, wl, 0.3)
    W, seed, traj, step = 4, 21, 2, 3
    x0 = wl.electrons(W=W)
    xs = x0.copy()
    _, nacc = s.vmc_run(xs, 1, 0, wl.delta, seed, traj=traj, step=step)
    lib = oracle.lib()
    for w in range(W):
        x = x0[w].copy()
        n = 0
        for e in range(wl.n):
            u = []
            for half in (0, 1):
                out = (ctypes.c_uint32 * 4)()
                lib.o_philox((ctypes.c_uint32 * 4)(step, w, e, half), (ctypes.c_uint32 * 2)(seed, traj), out)
                u += [lib.o_u01(out[0], out[1]), lib.o_u01(out[2], out[3])]
            xn = x.copy()
            xn[e] = np.mod(x[e] + wl.delta * (np.array(u[:3]) - 0.5), wl.L)
            p = math.exp(2 * (s.local(xn, False)["lnpsi"] - s.local(x, False)["lnpsi"]))
            if u[3] < p:
                x, n = xn, n + 1
        assert n == nacc[w]
        assert np.allclose(x, xs[w], rtol=0, atol=1e-12)


def test_contracted_force_estimator_equals_correlated_sampling_derivative(oracle):
    wl = _box(6)
    eta = -0.15
    Cm, s = _csys(oracle, wl, eta)
    x = wl.electrons(W=4)
    xs = []
    for k in range(6):
        s.vmc_run(x, 1, 0, wl.delta, 5, traj=0, step=k)
        xs.append(x.copy())
    xs = np.array(xs).reshape(-1, wl.n, 3)
    n3 = 3 * wl.n
    sums = np.zeros((1, 2 + 3 * n3))
    base = []
    for y in xs:
        r = s.local(y)
        base.append(r["lnpsi"])
        sums[0, 0] += r["EL"]
        sums[0, 1] += r["EL"] ** 2
        sums[0, 2:2 + n3] += r["dEL"]
        sums[0, 2 + n3:2 + 2 * n3] += r["dlnpsi"]
        sums[0, 2 + 2 * n3:] += r["EL"] * r["dlnpsi"]
    f = oracle.reduce(sums, len(xs))["f"]
    base = np.array(base)

    def E_of(Rflat):
        sp = oracle.System(Rflat.reshape(-1, 3), wl.zeta, Cm, L=wl.L, eta=eta)
        res = [sp.local(y, False) for y in xs]
        lw = 2 * (np.array([q["lnpsi"] for q in res]) - base)
        w = np.exp(lw - lw.max())
        return float((w * np.array([q["EL"] for q in res])).sum() / w.sum())

    h = 1e-5
    for t in range(n3):
        Rp, Rm = wl.R.reshape(-1).copy(), wl.R.reshape(-1).copy()
        Rp[t] += h
        Rm[t] -= h
        assert -f[t] == pytest.approx((E_of(Rp) - E_of(Rm)) / (2 * h), rel=1e-6, abs=1e-7)
