"""Pins of the oracle's Langevin step, S assembly and Cholesky against closed
forms of the harmonic problem (main text, harmonic solution and Newton step;
SI, exact integration that defines Dt and Db) and the rotating-spring toy model
(SI, "A simple toy model")."""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLD, "paper_constants.json")))


def _rot(n, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(n, n)))
    return q


def test_newton_step_reaches_minimum(oracle):
    """T = 0, alpha = 0, S = K, Delta = 1: R' = R + K^-1 f = 0 in one step for any K_cond."""
    n = 12
    Q = _rot(n, 1)
    K = Q @ np.diag(np.geomspace(1.0, 200.0, n)) @ Q.T
    R = np.random.default_rng(2).normal(size=n)
    Rp, Sp = R.copy(), K.copy()
    rc = oracle.langevin(R, Rp, Sp, -K @ R, K, T=0.0, Delta=1.0, alpha=0.0)
    assert rc == 0
    assert np.abs(R).max() < 1e-11


def test_zero_temperature_cfold_is_steepest_descent(oracle):
    n = 6
    K = np.diag(np.arange(1.0, n + 1))
    R = np.linspace(-1, 1, n)
    R0 = R.copy()
    oracle.langevin(R, R.copy(), np.eye(n), -K @ R0, np.eye(n), T=0.0, Delta=0.1, alpha=0.0,
                    flags=oracle.STEP_CFOLD)
    np.testing.assert_allclose(R, R0 - 0.1 * K @ R0, rtol=1e-15, atol=1e-16)


def test_cfold_harmonic_variance_and_autocorrelation(oracle):
    """S = I Euler steps: stationary var = T / (K (1 - K D / 2)), lag-1 correlation 1 - K D."""
    k = np.linspace(1.0, 4.0, 16)
    T, D = 0.3, 0.2
    x = oracle.langevin_harmonic_run(np.diag(k), np.eye(16), T, D, 0.0, 60000, np.zeros(16),
                                     flags=oracle.STEP_CFOLD, seed=3)[2000:]
    var = x.var(0)
    ratio = var * k * (1 - k * D / 2) / T
    assert abs(ratio.mean() - 1.0) < 0.02
    ac = np.array([np.corrcoef(x[:-1, i], x[1:, i])[0, 1] for i in range(16)])
    np.testing.assert_allclose(ac, 1 - k * D, atol=0.03)


@pytest.mark.parametrize("aD", [0.5, 1.0, 3.0])
def test_adopted_scheme_exact_for_harmonic_S_proportional_to_K(oracle, aD):
    """S = K/alpha: R' = e^{-alpha D} R + sqrt(2 T Db) z, so <R R^T> = T K^-1 for every D
    and every mode decorrelates by e^{-alpha D} per step, whatever K_cond (= 200 here)."""
    n = 10
    Q = _rot(n, 4)
    kv = np.geomspace(1.0, 200.0, n)
    K = Q @ np.diag(kv) @ Q.T
    alpha, T = 2.0, 0.05
    D = aD / alpha
    x = oracle.langevin_harmonic_run(K, K / alpha, T, D, alpha, 40000, np.zeros(n), seed=5)[200:]
    cov = np.cov(x.T)
    target = T * np.linalg.inv(K)
    # compare in the eigenbasis of K: each mode's variance times k / T must be 1
    m = Q.T @ cov @ Q
    np.testing.assert_allclose(np.diag(m) * kv / T, np.ones(n), atol=0.06)
    assert np.linalg.norm(cov - target) / np.linalg.norm(target) < 0.05
    y = x @ Q
    ac = np.array([np.corrcoef(y[:-1, i], y[1:, i])[0, 1] for i in range(n)])
    np.testing.assert_allclose(ac, np.full(n, math.exp(-aD)), atol=0.03)


def test_adopted_scheme_identity_S(oracle):
    """S = I, general alpha: var = 2 T Db / (1 - (1 - Dt K)^2)."""
    k = np.linspace(0.5, 2.0, 12)
    alpha, D, T = 0.7, 0.6, 0.2
    Dt = (1 - math.exp(-alpha * D)) / alpha
    Db = (1 - math.exp(-2 * alpha * D)) / (2 * alpha)
    x = oracle.langevin_harmonic_run(np.diag(k), np.eye(12), T, D, alpha, 50000, np.zeros(12), seed=6)[1000:]
    pred = 2 * T * Db / (1 - (1 - Dt * k) ** 2)
    np.testing.assert_allclose(x.var(0) / pred, np.ones(12), atol=0.05)


def test_noise_correction_temperature(oracle):
    """NOISE_CORR lowers T so that 2 T Db = 2 T_target Db - Dt^2; with S = K/alpha the
    variance is then T_eff K^-1 exactly."""
    kv = np.array([1.0, 3.0, 9.0])
    K = np.diag(kv)
    alpha, D, T = 1.0, 0.5, 0.4
    Dt = (1 - math.exp(-alpha * D)) / alpha
    Db = (1 - math.exp(-2 * alpha * D)) / (2 * alpha)
    Teff = T - Dt ** 2 / (2 * Db)
    x = oracle.langevin_harmonic_run(K, K / alpha, T, D, alpha, 80000, np.zeros(3),
                                     flags=oracle.STEP_NOISE_CORR, seed=7)[100:]
    np.testing.assert_allclose(x.var(0) * kv / Teff, np.ones(3), atol=0.03)


def test_noise_covariance_is_S_inverse(oracle):
    """With f = 0 and alpha = 0, R' - R = sqrt(2 T D) z, <z z^T> = S^-1."""
    n = 5
    Q = _rot(n, 8)
    S = Q @ np.diag([0.5, 1.0, 2.0, 4.0, 8.0]) @ Q.T
    x = oracle.langevin_harmonic_run(np.zeros((n, n)), S, 0.5, 1.0, 0.0, 60000, np.zeros(n), seed=9)
    inc = np.diff(np.vstack([np.zeros(n), x]), axis=0)
    cov = inc.T @ inc / len(inc)
    target = np.linalg.inv(S)
    assert np.linalg.norm(cov - target) / np.linalg.norm(target) < 0.03


def test_S_difference_term_and_first_step(oracle):
    """First step (R_prev = R, S_prev = S): no correction.  Otherwise the drift gets
    -Dt S^-1 (S_prev - S)(R_prev - R)/(2 Db); checked at T = 0 against the formula."""
    n = 4
    rng = np.random.default_rng(10)
    A = rng.normal(size=(n, n)); S = A @ A.T + n * np.eye(n)
    B = rng.normal(size=(n, n)); Sp = B @ B.T + n * np.eye(n)
    R = rng.normal(size=n); Rp = rng.normal(size=n); f = rng.normal(size=n)
    alpha, D = 0.3, 0.8
    Dt = (1 - math.exp(-alpha * D)) / alpha
    Db = (1 - math.exp(-2 * alpha * D)) / (2 * alpha)
    expect = R + Dt * np.linalg.solve(S, f - (Sp - S) @ (Rp - R) / (2 * Db))
    R1, Rp1, Sp1 = R.copy(), Rp.copy(), Sp.copy()
    assert oracle.langevin(R1, Rp1, Sp1, f, S, T=0.0, Delta=D, alpha=alpha) == 0
    np.testing.assert_allclose(R1, expect, rtol=1e-13)
    np.testing.assert_allclose(Rp1, R, rtol=0, atol=0)
    np.testing.assert_allclose(Sp1, S, rtol=0, atol=0)
    R2, Rp2, Sp2 = R.copy(), R.copy(), S.copy()
    oracle.langevin(R2, Rp2, Sp2, f, S, T=0.0, Delta=D, alpha=alpha)
    np.testing.assert_allclose(R2, R + Dt * np.linalg.solve(S, f), rtol=1e-13)


def test_periodic_wrap_and_minimum_image(oracle):
    L = 5.0
    R = np.array([4.9, 0.05, 2.5]); Rp = np.array([0.1, 4.95, 2.5])   # R_prev - R is small by min image
    S = np.eye(3); f = np.zeros(3)
    R1 = R.copy()
    oracle.langevin(R1, Rp.copy(), 2.0 * S, f, S, T=0.0, Delta=1.0, alpha=0.0, L=L)
    dR = np.array([0.2, -0.1, 0.0])
    expect = np.mod(R - 0.5 * (2.0 - 1.0) * dR, L)
    np.testing.assert_allclose(R1, expect, rtol=1e-14)
    assert np.all((R1 >= 0) & (R1 < L))


def test_cholesky_and_failure_leaves_state(oracle):
    rng = np.random.default_rng(11)
    A = rng.normal(size=(30, 30)); S = A @ A.T + 0.1 * np.eye(30)
    rc, Lc = oracle.cholesky(S)
    assert rc == 0
    np.testing.assert_allclose(Lc @ Lc.T, S, rtol=1e-13, atol=1e-12)
    assert np.allclose(Lc, np.tril(Lc))
    bad = S.copy(); bad[3, 3] = -1.0
    R = rng.normal(size=30); Rp = R.copy() + 0.1; Sp = S.copy()
    R0, Rp0, Sp0 = R.copy(), Rp.copy(), Sp.copy()
    assert oracle.langevin(R, Rp, Sp, np.zeros(30), bad, T=0.1, Delta=0.1, alpha=0.0) == -3
    assert np.array_equal(R, R0) and np.array_equal(Rp, Rp0) and np.array_equal(Sp, Sp0)
    assert oracle.langevin(R, Rp, Sp, np.zeros(30), S, T=0.1, Delta=0.0, alpha=0.0) == -1


def test_build_S_covariance_of_the_mean(oracle):
    """S = Cov(f_w) / W: equals numpy's unbiased covariance over W, and for Gaussian
    f_w with covariance Sigma, W S -> Sigma."""
    rng = np.random.default_rng(12)
    n3, W = 6, 40000
    A = rng.normal(size=(n3, n3)); Sig = A @ A.T / n3 + 0.2 * np.eye(n3)
    fw = rng.multivariate_normal(np.arange(n3, dtype=float), Sig, size=W)
    f = fw.mean(0)
    S = oracle.build_S(fw, f)
    np.testing.assert_allclose(S, np.cov(fw.T) / W, rtol=1e-10)
    assert np.linalg.norm(W * S - Sig) / np.linalg.norm(Sig) < 0.03


def test_reduce_two_walkers_closed_form(oracle):
    n3 = 3
    sums = np.zeros((2, 2 + 3 * n3))
    sums[0, 0], sums[1, 0] = 2.0 * 4, 3.0 * 4          # M = 4 samples: e_w = 2, 3
    sums[0, 2:5] = [4, 8, 12]; sums[1, 2:5] = [0, 4, 0]  # d_w
    sums[0, 5:8] = [1, 0, 0]; sums[1, 5:8] = [0, 1, 0]   # g_w * 4
    sums[0, 8:11] = [4, 0, 0]; sums[1, 8:11] = [0, 4, 0]
    r = oracle.reduce(sums, 4)
    assert r["E"] == 2.5 and r["sigma_E"] == pytest.approx(0.5)
    g = np.array([[0.25, 0, 0], [0, 0.25, 0]]); h = np.array([[1, 0, 0], [0, 1, 0]]); d = np.array([[1, 2, 3], [0, 1, 0]])
    fw = -(d + 2 * (h - 2.5 * g))
    np.testing.assert_allclose(r["f_w"], fw)
    np.testing.assert_allclose(r["f"], fw.mean(0))


# ----------------------------------------------------------- toy model ------
def _toy(oracle, scheme, D, alpha=0.0, n=60000, seed=1, s_kind=0):
    tm = PAPER["toy_model"]
    return oracle.toy_run(tm["lambda_used"], tm["k"], tm["a"], tm["mu"], s_kind, tm["T"], D, alpha,
                          scheme, seed, n)


def _radial_mean_U(power):
    """<U> for the radial density r^power e^{-k (r-a)^2 / (2T)} by quadrature."""
    tm = PAPER["toy_model"]
    r = np.linspace(0.5, 2.5, 400001)
    w = r ** power * np.exp(-tm["k"] * (r - tm["a"]) ** 2 / (2 * tm["T"]))
    return float((w * 0.5 * tm["k"] * (r - tm["a"]) ** 2).sum() / w.sum())


def test_toy_model_equilibrium_and_time_step_error(oracle):
    """Canonical <U> = T/2 (planar measure r dr; exact up to e^{-196}).  Eq. finaldyn,
    Eq. finaldyn_new and the explicit-Gamma Ito step reach it as D -> 0."""
    T = PAPER["toy_model"]["T"]
    assert _radial_mean_U(1) == pytest.approx(T / 2, rel=1e-5)
    for scheme, alpha in [(0, 0.0), (0, PAPER["toy_model"]["alpha"]), (2, 0.0)]:
        u = np.mean([_toy(oracle, scheme, 0.05, alpha, seed=s) for s in range(4)])
        assert abs(u / (T / 2) - 1.0) < 0.04, (scheme, alpha, u)


def test_toy_model_adopted_scheme_removes_time_step_error(oracle):
    """At D = 1 the adopted scheme (alpha = 0.2) stays at T/2 while Eq. finaldyn drifts
    (SI, caption of Fig. toy: the alpha scheme 'basically gets rid of the time step error')."""
    T = PAPER["toy_model"]["T"]
    u_new = np.mean([_toy(oracle, 0, 1.0, PAPER["toy_model"]["alpha"], seed=s) for s in range(4)])
    u_old = np.mean([_toy(oracle, 0, 1.0, 0.0, seed=s) for s in range(4)])
    assert abs(u_new / (T / 2) - 1.0) < 0.03
    assert u_old / (T / 2) - 1.0 > 0.08


def test_toy_model_without_S_term_samples_wrong_distribution(oracle):
    """Eq. norogna drops the S-difference (Gamma) term: its Fokker-Planck equation is
    stationary for P ~ r^{(1-lambda)/lambda} e^{-U/T} (radial mobility lambda), not the
    canonical one -- the SI's 'the sampled distribution is simply wrong', made quantitative."""
    tm = PAPER["toy_model"]
    lam = tm["lambda_used"]
    wrong = _radial_mean_U(1 + (1 - lam) / lam)
    assert wrong / (tm["T"] / 2) - 1.0 > 0.15
    un = np.mean([_toy(oracle, 1, 0.02, seed=s) for s in range(4)])
    assert un == pytest.approx(wrong, rel=0.04)


def test_toy_model_conventional_dynamics_time_step_error(oracle):
    """S = I (the conventional dynamics, black points of Fig. toy): the radial Euler step of an
    Ornstein-Uhlenbeck mode of stiffness k has stationary variance T / (k (1 - k D / 2)), so <U>
    exceeds T/2 by the factor 1 / (1 - k D / 2), up to corrections of order T / (k a^2) from the
    planar geometry."""
    tm = PAPER["toy_model"]
    T, k = tm["T"], tm["k"]
    for D in (0.01, 0.05, 0.2):
        u = np.mean([_toy(oracle, 0, D, 0.0, seed=10 + s, s_kind=2) for s in range(4)])
        assert u / (T / 2) == pytest.approx(1.0 / (1.0 - k * D / 2), rel=0.03), (D, u)


def test_toy_noise_stream_follows_the_trajectory_id(oracle):
    """Trajectory ids key the noise: equal ids give equal paths, different ids different ones."""
    tm = PAPER["toy_model"]
    args = (tm["lambda_used"], tm["k"], tm["a"], tm["mu"], 0, tm["T"], 0.3, 0.2, 0, 5, 50)
    (_, r0) = oracle.toy_run(*args, traj=0, final=True)
    (_, r0b) = oracle.toy_run(*args, traj=0, final=True)
    (_, r1) = oracle.toy_run(*args, traj=1, final=True)
    assert np.array_equal(r0, r0b) and not np.allclose(r0, r1)


@pytest.mark.parametrize("s_kind", [0, 1, 2, 3])
def test_toy_acceleration_matrices(oracle, s_kind):
    """The toy model's S at points of the plane against its definitions: G_lambda has radial
    eigenvalue 1/lambda and tangential eigenvalue 1; H is the Hessian of U = k (|x| - a)^2 / 2,
    taken here by central differences of U; S = H + mu G_lambda, I, or H + mu I (the main
    text's shifted Hessian)."""
    tm = PAPER["toy_model"]
    lam, k, a, mu = tm["lambda_used"], tm["k"], tm["a"], tm["mu"]
    U = lambda x: 0.5 * k * (np.hypot(x[0], x[1]) - a) ** 2
    rng = np.random.default_rng(s_kind)
    for _ in range(6):
        x = rng.uniform(-2.0, 2.0, 2)
        if np.hypot(*x) < 0.3:
            continue
        n = x / np.hypot(*x)
        tv = np.array([-n[1], n[0]])
        G = np.outer(n, n) / lam + np.outer(tv, tv)
        h = 1e-4
        H = np.zeros((2, 2))
        for i in range(2):
            for j in range(2):
                ei, ej = np.eye(2)[i] * h, np.eye(2)[j] * h
                H[i, j] = (U(x + ei + ej) - U(x + ei - ej) - U(x - ei + ej) + U(x - ei - ej)) / (4 * h * h)
        want = {0: G, 1: H + mu * G, 2: np.eye(2), 3: H + mu * np.eye(2)}[s_kind]
        np.testing.assert_allclose(oracle.toy_S(lam, k, a, mu, s_kind, x), want, rtol=1e-6, atol=1e-6)
    if s_kind == 0:
        w = np.linalg.eigvalsh(oracle.toy_S(lam, k, a, mu, 0, np.array([0.3, 1.1])))
        np.testing.assert_allclose(sorted(w), sorted([1.0 / lam, 1.0]), rtol=1e-12)


def test_toy_model_shifted_hessian_equilibrium(oracle):
    """S = H + mu I is positive definite only where r > a k / (k + mu); with mu = 1 (the main
    text leaves mu to be chosen; the figure's 1/2 belongs to H + mu G_lambda) that region is seven
    thermal widths inside the ring, and the adopted scheme samples the canonical <U> = T/2 at a
    small step."""
    tm = PAPER["toy_model"]
    T = tm["T"]
    u = np.mean([oracle.toy_run(tm["lambda_used"], tm["k"], tm["a"], 1.0, 3, T, 0.05, tm["alpha"], 0, 20 + s, 60000)
                 for s in range(4)])
    assert abs(u / (T / 2) - 1.0) < 0.04, u


def test_toy_model_two_S_scheme_samples_canonical(oracle):
    """The SI's first simplified scheme (Eq. smartMarkov: a noise step to y, then the drift with
    the half S-difference between y and R) implies the right Fokker-Planck equation without the
    Gamma term: with S = G_lambda it samples <U> = T/2 at D = 0.2, where Eq. norogna (no
    S-difference at all) is 20-40% off."""
    tm = PAPER["toy_model"]
    T = tm["T"]
    u = np.mean([_toy(oracle, 3, 0.2, seed=40 + s) for s in range(6)])
    assert abs(u / (T / 2) - 1.0) < 0.04, u
    un = np.mean([_toy(oracle, 1, 0.2, seed=40 + s) for s in range(2)])
    assert un / (T / 2) - 1.0 > 0.15
