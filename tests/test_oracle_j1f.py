"""Pins of the oracle's orbital part of the one-body Jastrow term U_1 (SI, Jastrow section, Eq. e:j1):
sum_a sum_i (f_1 chi_1 + f_2 chi_2)(r_i - R_a) with the Jastrow orbitals chi_1 = e^{-ZJ rho^2},
chi_2 = rho^2 e^{-ZJ rho^2} (ZJ = 0.7933844) on the sin-periodised offsets, the same f for every
nucleus.  The value against the one-body sum written out here from the closed-form orbitals, the
electron gradient and Laplacian by finite differences, the kinetic energy against a finite-difference
Laplacian of ln psi, the proton derivatives of ln psi and E_L by finite differences, the sweep's
decisions against |psi'/psi|^2 and the force estimator against the correlated-sampling derivative,
each with the cusp b_1 and the three-body matrix F on as well as off."""
import ctypes
import math

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload

F1 = (0.35, -0.6)
F3 = (-0.3, 0.1, 0.05)


def _chi_closed(L, d):
    rho = L / np.pi * np.sin(np.pi * np.asarray(d) / L)
    r2 = float(np.sum(rho * rho))
    e = math.exp(-0.7933844 * r2)
    return e, r2 * e


def _sys(oracle, wl, b1=0.0, j3=None, R=None, j1f=F1):
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    R = wl.R if R is None else R
    return Cm, oracle.System(R, wl.zeta, Cm, L=wl.L, b1=b1, j3=j3, j1f=j1f)


def test_j1f_value_is_the_one_body_sum(oracle):
    wl = small_system(6, 1.3, seed=4)
    x = wl.electrons(W=1)[0]
    s0 = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=F3)
    s1 = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=F3, j1f=F1)
    ref = 0.0
    for a in range(wl.n):
        for i in range(wl.n):
            c1, c2 = _chi_closed(wl.L, x[i] - wl.R[a])
            ref += F1[0] * c1 + F1[1] * c2
    assert s1.jastrow(x)[0] - s0.jastrow(x)[0] == pytest.approx(ref, rel=1e-12, abs=1e-14)
    # linear in f: doubling f doubles the change
    s2 = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=F3, j1f=(2 * F1[0], 2 * F1[1]))
    assert s2.jastrow(x)[0] - s0.jastrow(x)[0] == pytest.approx(2 * ref, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("j3", [None, F3])
def test_j1f_gradient_laplacian_and_periodicity(oracle, j3):
    wl = small_system(6, 1.3, seed=4)
    s = oracle.System(wl.R, wl.zeta, np.eye(6)[:, :3], L=wl.L, j3=j3, j1f=F1)
    x = wl.electrons(W=1)[0]
    U, g, lp = s.jastrow(x)
    h, hg = 1e-4, 1e-5   # second differences at h, the gradient's central differences at hg
    for i in range(wl.n):
        lap = 0.0
        for m in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, m] += hg
            xm[i, m] -= hg
            assert g[i, m] == pytest.approx((s.jastrow(xp)[0] - s.jastrow(xm)[0]) / (2 * hg), rel=1e-7, abs=1e-9)
            xp, xm = x.copy(), x.copy()
            xp[i, m] += h
            xm[i, m] -= h
            Up, Um = s.jastrow(xp)[0], s.jastrow(xm)[0]
            lap += (Up - 2 * U + Um) / h ** 2
        assert lp[i] == pytest.approx(lap, rel=1e-5, abs=1e-6)
        xs = x.copy()
        xs[i] += wl.L * np.array([1.0, -1.0, 2.0])
        assert s.jastrow(xs)[0] == pytest.approx(U, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("name,b1,j3", [("h6", 0.0, None), ("h16", 0.0, F3), ("h6", 1.7, F3)])
def test_j1f_kinetic_energy_against_fd_laplacian(oracle, name, b1, j3):
    wl = workload("h16") if name == "h16" else small_system(6, 1.3, seed=4)
    _, s = _sys(oracle, wl, b1, j3)
    x = wl.electrons(W=1)[0]
    res = s.local(x, derivs=False)
    V, _, _ = s.potential(x)
    lp0 = res["lnpsi"]
    h = 3e-4
    T = 0.0
    for i in range(x.shape[0]):
        for m in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, m] += h
            xm[i, m] -= h
            lpp, lpm = s.local(xp, False)["lnpsi"], s.local(xm, False)["lnpsi"]
            T += -0.5 * ((lpp - 2 * lp0 + lpm) / h ** 2 + ((lpp - lpm) / (2 * h)) ** 2)
    assert res["EL"] - V == pytest.approx(T, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("name,b1,j3", [("h6", 0.0, None), ("h16", 0.0, F3), ("h6", 1.7, F3)])
def test_j1f_proton_derivatives_by_finite_differences(oracle, name, b1, j3):
    wl = workload("h16") if name == "h16" else small_system(6, 1.3, seed=4)
    Cm, s = _sys(oracle, wl, b1, j3)
    x = wl.electrons(W=1)[0]
    res = s.local(x)
    h = 1e-5
    for t in range(0, 3 * wl.n, 1 if wl.n <= 6 else 5):
        Rp = wl.R.reshape(-1).copy()
        Rm = Rp.copy()
        Rp[t] += h
        Rm[t] -= h
        a = oracle.System(Rp.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, j3=j3, j1f=F1).local(x, False)
        b = oracle.System(Rm.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, j3=j3, j1f=F1).local(x, False)
        assert res["dlnpsi"][t] == pytest.approx((a["lnpsi"] - b["lnpsi"]) / (2 * h), rel=1e-7, abs=1e-8)
        assert res["dEL"][t] == pytest.approx((a["EL"] - b["EL"]) / (2 * h), rel=1e-6, abs=1e-7)


def test_j1f_sweep_decisions_follow_psi_ratios(oracle):
    wl = small_system(6, 1.3, seed=4)
    _, s = _sys(oracle, wl, 1.7, F3)
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


def test_j1f_force_estimator_equals_correlated_sampling_derivative(oracle):
    wl = small_system(6, 1.3, seed=4)
    Cm, s = _sys(oracle, wl, 1.7, F3)
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
        sp = oracle.System(Rflat.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=1.7, j3=F3, j1f=F1)
        res = [sp.local(y, False) for y in xs]
        lw = 2 * (np.array([q["lnpsi"] for q in res]) - base)
        w = np.exp(lw - lw.max())
        return float((w * np.array([q["EL"] for q in res])).sum() / w.sum())

    h = 1e-5
    for t in range(n3):
        Rp = wl.R.reshape(-1).copy()
        Rm = Rp.copy()
        Rp[t] += h
        Rm[t] -= h
        assert f[t] == pytest.approx(-(E_of(Rp) - E_of(Rm)) / (2 * h), rel=1e-6, abs=1e-7)
