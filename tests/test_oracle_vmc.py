"""Pins of the oracle's Metropolis sampler and VMC force estimator.

* Sampling: a single electron in a periodic box with one Gaussian must be
  distributed as |psi|^2 (its x-marginal is g(x)^2, known in closed form).
* Zero variance: a hydrogenic orbital in an open box gives E = -1/2, sigma_E = 0.
* Force estimator: on a FIXED sample set drawn at R, the correlated-sampling
  energy E(R') = sum_s w_s E_L(s; R') / sum_s w_s with w_s = |psi_R'(s)/psi_R(s)|^2
  has the exact derivative <dE_L/dR> + 2 (<E_L dln|psi|/dR> - E <dln|psi|/dR>)
  at R' = R; central differences of E(R +- h) must give -f to O(h^2).
"""
import ctypes
import math

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload


def _samples(sys_, x0, n_sweeps, delta, seed):
    """Positions after each of n_sweeps sweeps (one oracle call per sweep)."""
    x = x0.copy()
    out = []
    for s in range(n_sweeps):
        sys_.vmc_run(x, 1, 0, delta, seed, traj=0, step=s)
        out.append(x.copy())
    return np.array(out)   # (n_sweeps, W, Ne, 3)


def test_single_electron_samples_psi_squared(oracle):
    L, z = 4.0, 0.6
    s = oracle.System(R=[[1.0, 1.5, 2.0]], zeta=[z], C_mo=[[1.0]], L=L, n_up=1, n_dn=0,
                      pot=oracle.OP_NONE, jastrow=False)
    W = 64
    x0 = np.mod(np.random.default_rng(0).uniform(0, L, size=(W, 1, 3)), L)
    xs = _samples(s, x0, 300, 1.5, seed=3)[20:, :, 0, 0].ravel()
    edges = np.linspace(0, L, 21)
    hist, _ = np.histogram(xs, bins=edges)
    # closed-form marginal g(x - X)^2 with the image sum, integrated per bin
    fine = np.linspace(0, L, 200001)
    d = fine - 1.0
    d = d - L * np.floor(d / L + 0.5)
    g = sum(np.exp(-z * (d + n * L) ** 2) for n in (-1, 0, 1)) ** 2
    p = np.array([g[(fine >= a) & (fine < b)].sum() for a, b in zip(edges[:-1], edges[1:])])
    p /= p.sum()
    expect = p * xs.size
    # chains are correlated: inflate the variance by an integrated autocorrelation bound of 6
    chi2 = ((hist - expect) ** 2 / (6 * expect)).sum()
    assert chi2 < 40.0


def test_hydrogen_atom_zero_variance_chain(oracle):
    s = oracle.System(R=[[0.0, 0.0, 0.0]], zeta=[1.0], C_mo=[[1.0]], n_up=1, n_dn=0,
                      basis=oracle.OB_OPEN_STO, pot=oracle.OP_COULOMB_OPEN, jastrow=False)
    x = np.random.default_rng(1).normal(size=(8, 1, 3))
    sums, nacc = s.vmc_run(x, 5, 20, 1.0, seed=9)
    r = oracle.reduce(sums, 20)
    assert r["E"] == pytest.approx(-0.5, abs=1e-13)
    assert r["sigma_E"] < 1e-13
    assert np.all(nacc > 0) and np.all(nacc < 8 * 25)


def test_chain_is_deterministic(oracle):
    wl = workload("h16")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    x1 = wl.electrons(W=4)
    x2 = x1.copy()
    a, na = s.vmc_run(x1, 2, 3, wl.delta, seed=1, step=4)
    b, nb = s.vmc_run(x2, 2, 3, wl.delta, seed=1, step=4)
    assert np.array_equal(a, b) and np.array_equal(na, nb) and np.array_equal(x1, x2)
    acc = na.sum() / (4 * 5 * 16)
    assert 0.2 < acc < 0.9


def test_walker_slice_runs_the_walkers_own_streams(oracle):
    """Walkers w0 .. w0+k-1 run alone with walker0 = w0 give exactly rows w0 .. w0+k-1 of the run
    over the whole set (each walker's chain depends only on its own start and counter), and a
    slice run at the wrong offset gives other chains."""
    wl = workload("h16")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    x = wl.electrons(W=7)
    full = x.copy()
    a, na = s.vmc_run(full, 1, 2, wl.delta, seed=5, traj=2, step=3)
    part = np.ascontiguousarray(x[4:7])
    b, nb = s.vmc_run(part, 1, 2, wl.delta, seed=5, traj=2, step=3, walker0=4)
    assert np.array_equal(b, a[4:7]) and np.array_equal(nb, na[4:7]) and np.array_equal(part, full[4:7])
    wrong = np.ascontiguousarray(x[4:7])
    c, _ = s.vmc_run(wrong, 1, 2, wl.delta, seed=5, traj=2, step=3, walker0=3)
    assert not np.array_equal(c, a[4:7])


def test_sweep_decisions_follow_psi_ratios_with_one_body_term(oracle):
    """Each Metropolis decision of a sweep equals u < |psi(x')/psi(x)|^2 with ln|psi| taken
    from the local-energy routine (one-body term included) on the move drawn from the same
    Philox counters: the sweep's own Jastrow differences agree with ln|psi|."""
    wl = small_system(6, 1.3, seed=4)
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 3)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, b1=1.2)
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
                ctr = (ctypes.c_uint32 * 4)(step, w, e, half)
                key = (ctypes.c_uint32 * 2)(seed, traj)
                lib.o_philox(ctr, key, out)
                u += [lib.o_u01(out[0], out[1]), lib.o_u01(out[2], out[3])]
            xn = x.copy()
            xn[e] = np.mod(x[e] + wl.delta * (np.array(u[:3]) - 0.5), wl.L)
            p = math.exp(2 * (s.local(xn, False)["lnpsi"] - s.local(x, False)["lnpsi"]))
            if u[3] < p:
                x, n = xn, n + 1
        assert n == nacc[w]
        assert np.allclose(x, xs[w], rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,b1,twist", [("h6", 0.0, 0), ("h16", 0.0, 0), ("h6", 1.0, 0), ("h16", 0.0, 5)])
def test_force_estimator_equals_correlated_sampling_derivative(oracle, name, b1, twist):
    wl = small_system(6, 1.3, seed=4) if name == "h6" else workload("h16")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2, twist=twist)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, b1=b1, twist=twist)
    xs = _samples(s, wl.electrons(W=4), 6, wl.delta, seed=5).reshape(-1, wl.n, 3)
    n3 = 3 * wl.n
    sums = np.zeros((1, 2 + 3 * n3))
    base = []
    for x in xs:
        r = s.local(x)
        base.append(r["lnpsi"])
        sums[0, 0] += r["EL"]; sums[0, 1] += r["EL"] ** 2
        sums[0, 2:2 + n3] += r["dEL"]
        sums[0, 2 + n3:2 + 2 * n3] += r["dlnpsi"]
        sums[0, 2 + 2 * n3:] += r["EL"] * r["dlnpsi"]
    f = oracle.reduce(sums, len(xs))["f"]
    base = np.array(base)

    def E_of(Rflat):
        sp = oracle.System(Rflat.reshape(-1, 3), wl.zeta, Cm, L=wl.L, b1=b1, twist=twist)
        res = [sp.local(x, False) for x in xs]
        lw = 2 * (np.array([q["lnpsi"] for q in res]) - base)
        w = np.exp(lw - lw.max())
        return float((w * np.array([q["EL"] for q in res])).sum() / w.sum())

    h = 1e-5
    for t in range(0, n3, 1 if wl.n <= 6 else 7):
        Rp = wl.R.reshape(-1).copy(); Rm = Rp.copy()
        Rp[t] += h; Rm[t] -= h
        fd = (E_of(Rp) - E_of(Rm)) / (2 * h)
        assert -f[t] == pytest.approx(fd, rel=1e-6, abs=1e-7)
