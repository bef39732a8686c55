"""Pins of the oracle's on-site three-body (electron-electron-nucleus) Jastrow term U_3 (SI, Jastrow
section, Eq. e:j33): U_3 = sum_a sum_{i<j} chi_a(r_i)^T F chi_a(r_j) with the orbitals
chi_1 = e^{-ZJ rho^2}, chi_2 = rho^2 e^{-ZJ rho^2} (ZJ = 0.7933844) on the sin-periodised offsets
rho_m = (L/pi) sin(pi d_m / L), F a symmetric 2 x 2 matrix.  The orbitals against their closed form
and finite differences, U_3 against the pair sum written out here, the gradient and Laplacian of U,
the kinetic energy, the proton derivatives, the decisions and the force estimator with the term."""
import ctypes
import math

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload

F3 = (-0.3, 0.1, 0.05)


def _chi_closed(L, d):
    rho = L / np.pi * np.sin(np.pi * np.asarray(d) / L)
    r2 = float(np.sum(rho * rho))
    e = math.exp(-0.7933844 * r2)
    return e, r2 * e


@pytest.mark.parametrize("periodic", [True, False])
def test_j3_orbitals_closed_form_and_fd(oracle, periodic):
    wl = workload("h16")
    basis = oracle.OB_PERIODIC_GAUSS if periodic else oracle.OB_OPEN_GAUSS
    s = oracle.System(wl.R, wl.zeta, np.eye(wl.n)[:, :8], L=wl.L, basis=basis, j3=F3)
    rng = np.random.default_rng(5)
    H = {(0, 0): 5, (1, 1): 6, (2, 2): 7, (0, 1): 8, (0, 2): 9, (1, 2): 10}
    for _ in range(5):
        a = int(rng.integers(wl.n))
        r = wl.R[a] + rng.uniform(-2.0, 2.0, 3)
        c1, c2 = s.j3_orbitals(a, r)
        d = r - wl.R[a]
        if periodic:
            e1, e2 = _chi_closed(wl.L, d)
        else:
            rr = float(d @ d)
            e1, e2 = math.exp(-0.7933844 * rr), rr * math.exp(-0.7933844 * rr)
        assert c1[0] == pytest.approx(e1, rel=1e-13)
        assert c2[0] == pytest.approx(e2, rel=1e-13, abs=1e-300)
        h = 2e-5
        for c, k in ((c1, 0), (c2, 1)):
            for m in range(3):
                e = np.zeros(3)
                e[m] = h
                p, q = s.j3_orbitals(a, r + e)[k], s.j3_orbitals(a, r - e)[k]
                assert c[1 + m] == pytest.approx((p[0] - q[0]) / (2 * h), rel=1e-7, abs=1e-10)
                assert c[11 + m] == pytest.approx((p[4] - q[4]) / (2 * h), rel=1e-7, abs=1e-9)
                for n in range(3):
                    assert c[H[(min(m, n), max(m, n))]] == pytest.approx((p[1 + n] - q[1 + n]) / (2 * h),
                                                                         rel=1e-7, abs=1e-9)
            assert c[4] == pytest.approx(c[5] + c[6] + c[7], rel=1e-13, abs=1e-15)


def test_j3_value_is_the_pair_sum(oracle):
    """U with the term minus U without it equals sum_a sum_{i<j} chi_ai^T F chi_aj, written out here
    from the closed-form orbitals."""
    wl = small_system(6, 1.3, seed=4)
    x = wl.electrons(W=1)[0]
    s0 = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L)
    s3 = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=F3)
    F = np.array([[F3[0], F3[1]], [F3[1], F3[2]]])
    ref = 0.0
    for a in range(wl.n):
        chi = [np.array(_chi_closed(wl.L, x[i] - wl.R[a])) for i in range(wl.n)]
        for i in range(wl.n):
            for j in range(i + 1, wl.n):
                ref += chi[i] @ F @ chi[j]
    assert s3.jastrow(x)[0] - s0.jastrow(x)[0] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_j3_gradient_laplacian_and_periodicity(oracle):
    wl = small_system(6, 1.3, seed=4)
    s = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=F3)
    x = wl.electrons(W=1)[0]
    U, g, lp = s.jastrow(x)
    h = 1e-4
    for i in range(wl.n):
        lap = 0.0
        for m in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, m] += h
            xm[i, m] -= h
            Up, Um = s.jastrow(xp)[0], s.jastrow(xm)[0]
            assert g[i, m] == pytest.approx((Up - Um) / (2 * h), rel=1e-7, abs=1e-9)
            lap += (Up - 2 * U + Um) / h ** 2
        assert lp[i] == pytest.approx(lap, rel=1e-5, abs=1e-6)
        xs = x.copy()
        xs[i] += wl.L * np.array([1.0, -1.0, 2.0])
        assert s.jastrow(xs)[0] == pytest.approx(U, rel=1e-12, abs=1e-12)


def _sys(oracle, wl, b1=0.0):
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    return Cm, oracle.System(wl.R, wl.zeta, Cm, L=wl.L, b1=b1, j3=F3)


@pytest.mark.parametrize("name,b1", [("h6", 0.0), ("h16", 0.0), ("h6", 1.7)])
def test_j3_kinetic_energy_against_fd_laplacian(oracle, name, b1):
    wl = workload("h16") if name == "h16" else small_system(6, 1.3, seed=4)
    _, s = _sys(oracle, wl, b1)
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

    # a step where the O(h^2) error and the rounding of the second differences are both small
    T = T_fd(3e-4)
    assert res["EL"] - V == pytest.approx(T, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("name,b1", [("h6", 0.0), ("h16", 0.0), ("h6", 1.7)])
def test_j3_proton_derivatives_by_finite_differences(oracle, name, b1):
    wl = workload("h16") if name == "h16" else small_system(6, 1.3, seed=4)
    Cm, s = _sys(oracle, wl, b1)
    x = wl.electrons(W=1)[0]
    res = s.local(x)
    h = 1e-5
    for t in range(0, 3 * wl.n, 1 if wl.n <= 6 else 5):
        Rp = wl.R.reshape(-1).copy()
        Rm = Rp.copy()
        Rp[t] += h
        Rm[t] -= h
        a = oracle.System(Rp.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, j3=F3).local(x, False)
        b = oracle.System(Rm.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, j3=F3).local(x, False)
        assert res["dlnpsi"][t] == pytest.approx((a["lnpsi"] - b["lnpsi"]) / (2 * h), rel=1e-7, abs=1e-8)
        assert res["dEL"][t] == pytest.approx((a["EL"] - b["EL"]) / (2 * h), rel=1e-6, abs=1e-7)


def test_j3_sweep_decisions_follow_psi_ratios(oracle):
    wl = small_system(6, 1.3, seed=4)
    _, s = _sys(oracle, wl)
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


def test_j3_force_estimator_equals_correlated_sampling_derivative(oracle):
    wl = small_system(6, 1.3, seed=4)
    Cm, s = _sys(oracle, wl)
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
        sp = oracle.System(Rflat.reshape(-1, 3), wl.zeta, Cm, L=wl.L, j3=F3)
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
