"""Pins of the oracle's wavefunction-optimisation pieces: the logarithmic derivatives
O_k = d ln psi / d p_k of the Jastrow parameters p = (b, b_1, f_11, f_12, f_22, f_1, f_2) against finite
differences of ln psi, the generalised forces of stochastic reconfiguration (SR; Sorella,
PRB 64, 024512 (2001)) against the correlated-sampling derivative of the energy, the SR step's
invariances and closed form, the chain's parameter sums against the per-sample definitions, and
an SR run that lowers the energy."""
import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload

F3 = (-0.3, 0.1, 0.05)
F1 = (0.35, -0.6)
NP = 7


def _sys(oracle, wl, p):
    """The oracle system at parameters p = (b, b1, f11, f12, f22, f1, f2)."""
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    b, b1, f11, f12, f22, f1, f2 = p
    j3 = (f11, f12, f22) if (f11, f12, f22) != (0.0, 0.0, 0.0) else None
    return oracle.System(wl.R, wl.zeta, Cm, L=wl.L, b=b, b1=b1, j3=j3, j1f=(f1, f2))


@pytest.mark.parametrize("name,p", [("h6", (1.0, 1.7, *F3, *F1)), ("h6", (0.7, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)),
                                    ("h16", (1.0, 2.5, *F3, 0.0, 0.0))])
def test_log_derivatives_are_finite_differences_of_ln_psi(oracle, name, p):
    """Each O_k against (ln psi(p_k + h) - ln psi(p_k - h)) / 2h at fixed electrons; the three-body
    and orbital-part entries also at F = 0 and f = 0, where the terms are off but their derivatives
    are not zero."""
    wl = workload("h16") if name == "h16" else small_system(6, 1.3, seed=4)
    x = wl.electrons(W=2, seed_offset=1)
    s = _sys(oracle, wl, p)
    h = 1e-5
    for xk in x:
        O = s.param_derivs(xk)
        for k in range(NP):
            if k == 1 and p[1] == 0.0:
                assert O[1] == 0.0          # no one-body term: b_1 is not a parameter
                continue
            pp, pm = list(p), list(p)
            pp[k] += h
            pm[k] -= h
            lp = _sys(oracle, wl, pp).local(xk, derivs=False)["lnpsi"]
            lm = _sys(oracle, wl, pm).local(xk, derivs=False)["lnpsi"]
            assert O[k] == pytest.approx((lp - lm) / (2 * h), rel=1e-7, abs=1e-8), (k, O[k])


def _samples(oracle, s, wl, W=4, n=6, seed=5):
    x = wl.electrons(W=W)
    xs = []
    for k in range(n):
        s.vmc_run(x, 1, 0, wl.delta, seed, traj=0, step=k)
        xs.append(x.copy())
    return np.array(xs).reshape(-1, wl.n, 3)


def _stats_from_samples(s, xs):
    """[E, <O>, <E_L O>, <O O^T>] over the samples, from local() and param_derivs()."""
    E = np.array([s.local(y, derivs=False)["EL"] for y in xs])
    O = np.array([s.param_derivs(y) for y in xs])
    return np.concatenate([[E.mean()], O.mean(0), (E[:, None] * O).mean(0),
                           (O[:, :, None] * O[:, None, :]).mean(0).ravel()])


def test_generalised_force_is_the_correlated_sampling_derivative(oracle):
    """On fixed samples the reweighted energy E(p) = sum w E_L(p) / sum w, w = |psi_p / psi_p0|^2,
    has dE/dp_k = 2 <(E_L - E)(O_k - <O_k>)> + <dE_L/dp_k>; the SR force is minus the first part,
    so -f_k + <dE_L/dp_k> (the latter by finite differences of E_L) must equal the central
    difference of E(p)."""
    wl = small_system(6, 1.3, seed=4)
    p0 = (1.0, 1.7, *F3, *F1)
    s0 = _sys(oracle, wl, p0)
    xs = _samples(oracle, s0, wl)
    st = _stats_from_samples(s0, xs)
    _, f, _ = oracle.sr_step(st, 0b1111111, 0.0, 1.0)
    base = np.array([s0.local(y, derivs=False)["lnpsi"] for y in xs])
    h = 1e-5

    def at(p):
        sp = _sys(oracle, wl, p)
        res = [sp.local(y, derivs=False) for y in xs]
        return np.array([r["lnpsi"] for r in res]), np.array([r["EL"] for r in res])

    for k in range(NP):
        pp, pm = list(p0), list(p0)
        pp[k] += h
        pm[k] -= h
        lpp, epp = at(pp)
        lpm, epm = at(pm)
        wp, wm = np.exp(2 * (lpp - base)), np.exp(2 * (lpm - base))
        dE = ((wp * epp).sum() / wp.sum() - (wm * epm).sum() / wm.sum()) / (2 * h)
        dEL = ((epp - epm) / (2 * h)).mean()
        assert -f[k] + dEL == pytest.approx(dE, rel=1e-6, abs=1e-7), k


def _random_stats(rng, n=400):
    O = rng.normal(size=(n, NP)) @ rng.normal(size=(NP, NP)) + rng.normal(size=NP)
    E = -3.0 + O @ rng.normal(size=NP) + 0.3 * rng.normal(size=n)
    st = np.concatenate([[E.mean()], O.mean(0), (E[:, None] * O).mean(0),
                         (O[:, :, None] * O[:, None, :]).mean(0).ravel()])
    return st, O, E


def _stats(O, E):
    return np.concatenate([[E.mean()], O.mean(0), (E[:, None] * O).mean(0),
                           (O[:, :, None] * O[:, None, :]).mean(0).ravel()])


def test_sr_step_invariances_and_closed_form(oracle):
    """SR depends on the O_k only through their fluctuations and is covariant under a rescaling
    of the parameters: a constant shift of O leaves dp unchanged, O_k -> c_k O_k gives
    dp_k -> dp_k / c_k (the diagonal shift scales with S_kk); with one active parameter
    dp = tau f / ((1 + eps) S); inactive parameters do not move."""
    rng = np.random.default_rng(3)
    st, O, E = _random_stats(rng)
    eps, tau = 1e-3, 0.3
    dp, f, S = oracle.sr_step(st, 0b1111111, eps, tau)
    np.testing.assert_allclose(S, np.cov(O.T, bias=True), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(f, -2 * ((E - E.mean())[:, None] * (O - O.mean(0))).mean(0), rtol=1e-10)
    shift = np.array([5.0, -2.0, 0.5, 30.0, -7.0, 1.5, -0.25])
    dp_shift, _, _ = oracle.sr_step(_stats(O + shift, E), 0b1111111, eps, tau)
    np.testing.assert_allclose(dp_shift, dp, rtol=1e-8, atol=1e-12)
    c = np.array([2.0, 0.5, -3.0, 10.0, 0.1, 4.0, -0.7])
    dp_scaled, _, _ = oracle.sr_step(_stats(O * c, E), 0b1111111, eps, tau)
    np.testing.assert_allclose(dp_scaled * c, dp, rtol=1e-8, atol=1e-12)
    for k in range(NP):
        d1, f1, S1 = oracle.sr_step(st, 1 << k, eps, tau)
        assert d1[k] == pytest.approx(tau * f1[k] / ((1 + eps) * S1[k, k]), rel=1e-12)
        assert np.all(np.delete(d1, k) == 0.0)
    # the step solves the regularised system over the active block
    act = [0, 2, 4]
    d2, f2, S2 = oracle.sr_step(st, 0b10101, eps, tau)
    Sa = S2[np.ix_(act, act)] + eps * np.diag(np.diag(S2)[act])
    np.testing.assert_allclose(Sa @ d2[act], tau * f2[act], rtol=1e-10, atol=1e-13)
    assert d2[1] == 0.0 and d2[3] == 0.0


def test_chain_parameter_sums_match_the_samples(oracle):
    """The per-walker sums of o_vmc_run_opt equal the definitions evaluated on the chain's own
    measured configurations (replayed sweep by sweep from the same counters)."""
    wl = small_system(6, 1.3, seed=4)
    s = _sys(oracle, wl, (1.0, 1.7, *F3, *F1))
    x0 = wl.electrons(W=3)
    xa = x0.copy()
    sums, _, popt = s.vmc_run(xa, 1, 3, wl.delta, 9, traj=2, step=4, params=True)
    # replay: the same sweeps one call at a time keep the counters only when the call covers all
    # of them, so reconstruct the measured positions from calls with growing sweep counts
    for w in range(3):
        ref = np.zeros(oracle.NOPT)
        for m in range(3):
            xb = x0[w:w + 1].copy()
            s.vmc_run(xb, 1 + m + 1, 0, wl.delta, 9, traj=2, step=4, walker0=w)
            el = s.local(xb[0], derivs=False)["EL"]
            O = s.param_derivs(xb[0])
            ref += np.concatenate([[el], O, el * O, np.outer(O, O).ravel()])
        np.testing.assert_allclose(popt[w], ref, rtol=1e-12, atol=1e-14)
        assert popt[w, 0] == pytest.approx(sums[w, 0], rel=1e-14)


def test_sr_lowers_the_energy(oracle):
    """From a poor three-body matrix (f_11 = +0.5 pushes two electrons onto one proton) a few SR
    steps on F with the same chains lower the energy by many standard errors."""
    wl = small_system(6, 1.3, seed=4)
    p = [1.0, 1.7, 0.5, 0.0, 0.0, 0.0, 0.0]

    def run(p, step, W, M):
        s = _sys(oracle, wl, p)
        x = wl.electrons(W=W, seed_offset=2)
        sums, _, popt = s.vmc_run(x, 4, M, wl.delta, 13, traj=0, step=step, params=True)
        return oracle.reduce(sums, M), oracle.param_stats(popt, M)

    r0, _ = run(p, 0, 96, 10)
    for it in range(6):
        _, st = run(p, 1 + it, 32, 8)
        dp, _, _ = oracle.sr_step(st, 0b11100, 0.1, 0.2)
        p = list(np.array(p) + dp)
    r1, _ = run(p, 0, 96, 10)
    assert p[2] < 0.0
    assert r1["E"] < r0["E"] - 3 * np.hypot(r0["sigma_E"], r1["sigma_E"]), (r0["E"], r1["E"], p)


def test_sr_on_the_orbital_part_lowers_the_energy(oracle):
    """From a poor orbital part of the one-body term (f_1 = +0.6 piles electrons onto the protons)
    a few SR steps on (f_1, f_2) alone lower the energy by many standard errors."""
    wl = small_system(6, 1.3, seed=4)
    p = [1.0, 1.7, 0.0, 0.0, 0.0, 0.6, 0.0]

    def run(p, step, W, M):
        s = _sys(oracle, wl, p)
        x = wl.electrons(W=W, seed_offset=2)
        sums, _, popt = s.vmc_run(x, 4, M, wl.delta, 13, traj=0, step=step, params=True)
        return oracle.reduce(sums, M), oracle.param_stats(popt, M)

    r0, _ = run(p, 0, 384, 10)
    for it in range(6):
        _, st = run(p, 1 + it, 32, 8)
        dp, _, _ = oracle.sr_step(st, 0b1100000, 0.1, 0.2)
        assert np.all(dp[:5] == 0.0)
        p = list(np.array(p) + dp)
    r1, _ = run(p, 0, 384, 10)
    assert p[5] < 0.6
    assert r1["E"] < r0["E"] - 3 * np.hypot(r0["sigma_E"], r1["sigma_E"]), (r0["E"], r1["E"], p)
