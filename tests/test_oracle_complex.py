"""Pins of the oracle's general-twist (complex) wavefunction, vmc_oracle_complex.c, against what
mathematics fixes: the Poisson sum of the Bloch-summed Gaussian (reciprocal frequencies
shifted by theta / L), the Bloch condition phi(r + L e_m) = e^{i theta_m} phi(r) of the SI's
twisted boundary conditions, reduction to the real oracle at the real twists, quadrature of
the overlaps, Leibniz determinants, finite differences of the local energy and of the proton
derivatives, the Metropolis decisions against |psi'/psi|^2, and the force estimator against the
derivative of the correlated-sampling energy.  None of these tests touch the GPU library."""
import ctypes
import itertools
import math

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload

THETAS = [(0.3, -1.1, 2.0), (np.pi / 4, 3 * np.pi / 4, -np.pi / 4)]
# the Jastrow factor: the two-body term alone, with the one-body and three-body terms, and with
# the orbital part of the one-body term as well
JAS = [dict(), dict(b1=1.7, j3=(-0.3, 0.1, 0.05)), dict(b1=1.7, j3=(-0.3, 0.1, 0.05), j1f=(0.35, -0.6))]


def _sys(oracle, wl, theta, **kw):
    Cc, _ = oracle.chuckel(wl.R, wl.zeta, wl.L, wl.n // 2, theta)
    return oracle.CSystem(wl.R, wl.zeta, Cc, theta, wl.L, **kw)


@pytest.mark.parametrize("theta", THETAS)
def test_bloch_sum_equals_shifted_poisson_sum(oracle, theta):
    """sum_n e^{-i theta n} e^{-zeta (d + n L)^2} = (sqrt(pi/zeta)/L) sum_m e^{i k_m d - k_m^2/(4 zeta)},
    k_m = (theta + 2 pi m)/L, for every axis; its d-derivatives bring (i k_m)^q.  All 14 basis
    components (value, gradient, Laplacian, Hessian, gradient of the Laplacian) agree."""
    wl = workload("h16")
    s = _sys(oracle, wl, theta)
    rng = np.random.default_rng(3)
    L, m = wl.L, np.arange(-30, 31)
    for _ in range(6):
        a = int(rng.integers(wl.n))
        r = rng.uniform(-L, 2 * L, size=3)                 # raw offsets beyond the cell too
        z = wl.zeta[a]
        G = []
        for ax in range(3):
            k = (theta[ax] + 2 * np.pi * m) / L
            d = r[ax] - wl.R[a, ax]
            base = math.sqrt(math.pi / z) / L * np.exp(1j * k * d - k * k / (4 * z))
            G.append([np.sum(base * (1j * k) ** q) for q in range(4)])
        gx, gy, gz = G
        ref = np.array([
            gx[0] * gy[0] * gz[0], gx[1] * gy[0] * gz[0], gx[0] * gy[1] * gz[0], gx[0] * gy[0] * gz[1],
            gx[2] * gy[0] * gz[0] + gx[0] * gy[2] * gz[0] + gx[0] * gy[0] * gz[2],
            gx[2] * gy[0] * gz[0], gx[0] * gy[2] * gz[0], gx[0] * gy[0] * gz[2],
            gx[1] * gy[1] * gz[0], gx[1] * gy[0] * gz[1], gx[0] * gy[1] * gz[1],
            gx[3] * gy[0] * gz[0] + gx[1] * gy[2] * gz[0] + gx[1] * gy[0] * gz[2],
            gx[2] * gy[1] * gz[0] + gx[0] * gy[3] * gz[0] + gx[0] * gy[1] * gz[2],
            gx[2] * gy[0] * gz[1] + gx[0] * gy[2] * gz[1] + gx[0] * gy[0] * gz[3]])
        got = s.cbasis(a, r)
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("theta", THETAS)
def test_bloch_condition(oracle, theta):
    wl = workload("h16")
    s = _sys(oracle, wl, theta)
    rng = np.random.default_rng(4)
    for _ in range(8):
        a = int(rng.integers(wl.n))
        r = rng.uniform(0, wl.L, size=3)
        for ax in range(3):
            for n in (1, -1, 2):
                r2 = r.copy()
                r2[ax] += n * wl.L
                assert np.allclose(s.cbasis(a, r2), np.exp(1j * theta[ax] * n) * s.cbasis(a, r), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("jas", JAS)
def test_real_twists_reduce_to_the_real_oracle(oracle, jas):
    """At the eight real twists (theta_m in {0, pi}) the complex wavefunction is the real one:
    the same occupied space, ln|psi|, E_L and proton derivatives (the sign of psi is its phase),
    also with the one-body and three-body Jastrow terms."""
    wl = workload("h16")
    x = wl.electrons(W=2, seed_offset=9)
    for tw in range(8):
        theta = np.array([np.pi * ((tw >> m) & 1) for m in range(3)])
        s = _sys(oracle, wl, theta, **jas)
        Cr, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8, twist=tw)
        sr = oracle.System(wl.R, wl.zeta, Cr, L=wl.L, twist=tw, **jas)
        assert np.allclose(s.Cc @ s.Cc.conj().T, Cr @ Cr.T, atol=1e-12)
        for k in range(2):
            a, b = s.local(x[k]), sr.local(x[k])
            assert a["lnpsi"] == pytest.approx(b["lnpsi"], rel=1e-12, abs=1e-12)
            assert a["EL"] == pytest.approx(b["EL"], rel=1e-12)
            assert np.allclose(a["dlnpsi"], b["dlnpsi"], rtol=1e-10, atol=1e-11)
            assert np.allclose(a["dEL"], b["dEL"], rtol=1e-10, atol=1e-10)
            assert math.cos(a["phase"]) == pytest.approx(b["sign"], abs=1e-10)


@pytest.mark.parametrize("theta", THETAS)
def test_overlap_equals_cell_quadrature(oracle, theta):
    """S_ab (one image sum of free-space overlaps) against the trapezoid rule over the cell of
    conj(phi_a) phi_b from the Bloch-summed basis values (spectrally accurate for a smooth
    periodic integrand); the Hueckel orbitals then satisfy C^H S C = diag(-eigenvalues)."""
    wl = small_system(6, 1.3, seed=4, zeta_lo=0.9, zeta_hi=1.1)
    s = _sys(oracle, wl, theta)
    ng = 40
    g = (np.arange(ng) + 0.5) * wl.L / ng
    pts = np.array(list(itertools.product(g, g, g)))
    phi = s.cbasis_values(pts)                         # (npts, n)
    Sq = (phi.conj().T @ phi) * (wl.L / ng) ** 3
    S = oracle.coverlap(wl.R, wl.zeta, wl.L, theta)
    assert np.max(np.abs(S - Sq)) < 1e-10 * np.max(np.abs(S))
    assert np.max(np.abs(S - S.conj().T)) < 1e-15 * np.max(np.abs(S))
    Cc, ev = oracle.chuckel(wl.R, wl.zeta, wl.L, 3, theta)
    assert np.allclose(Cc.conj().T @ S @ Cc, np.diag(-ev[:3]), atol=1e-12)
    # the occupied space is that of numpy's Hermitian eigen-solver
    d = np.sqrt(np.real(np.diag(S)))
    w, v = np.linalg.eigh(-S / np.outer(d, d))
    Cn = v[:, :3] / d[:, None]
    assert np.allclose(Cc @ Cc.conj().T, Cn @ Cn.conj().T, atol=1e-12)


def _leibniz(A):
    n = A.shape[0]
    tot = 0j
    for p in itertools.permutations(range(n)):
        sg = 1
        for i in range(n):
            for j in range(i + 1, n):
                if p[i] > p[j]:
                    sg = -sg
        tot += sg * np.prod([A[i, p[i]] for i in range(n)])
    return tot


@pytest.mark.parametrize("n", [2, 4])
def test_determinants_equal_leibniz(oracle, n):
    """psi without the Jastrow factor is the product of the two spins' Slater determinants of
    MO values; the oracle's complex LU gives the Leibniz sum of each (modulus and phase)."""
    wl = small_system(n, 1.3, seed=8)
    theta = np.array(THETAS[0])
    s = _sys(oracle, wl, theta, jastrow=False)
    x = wl.electrons(W=3, seed_offset=2)
    ns = n // 2
    for k in range(3):
        phi = s.cbasis_values(x[k])                     # electrons x centres
        M = phi @ s.Cc                                  # MO values
        D = _leibniz(M[:ns, :ns]) * _leibniz(M[ns:, :ns])
        r = s.local(x[k], False)
        assert r["lnpsi"] == pytest.approx(math.log(abs(D)), rel=1e-12, abs=1e-12)
        assert np.exp(1j * r["phase"]) == pytest.approx(D / abs(D), abs=1e-10)


@pytest.mark.parametrize("jas", JAS)
@pytest.mark.parametrize("theta", THETAS)
def test_kinetic_energy_equals_fd_laplacian(oracle, theta, jas):
    """Re E_L - V = Re(-1/2 sum_i lap_i psi / psi), the Laplacian of psi = e^{ln|psi| + i arg psi}
    by central differences in every electron coordinate."""
    wl = small_system(6, 1.3, seed=4)
    s = _sys(oracle, wl, theta, **jas)
    x = wl.electrons(W=1, seed_offset=5)[0]
    r = s.local(x, False)
    V, _, _ = s.potential(x)
    psi = lambda y: np.exp(s.local(y, False)["lnpsi"] + 1j * s.local(y, False)["phase"])
    p0 = psi(x)
    h = 1e-4
    lap = 0j
    for e in range(wl.n):
        for m in range(3):
            xp, xm = x.copy(), x.copy()
            xp[e, m] += h
            xm[e, m] -= h
            lap += (psi(xp) - 2 * p0 + psi(xm)) / (h * h)
    T_fd = float(np.real(-0.5 * lap / p0))
    assert r["EL"] - V == pytest.approx(T_fd, rel=2e-6, abs=2e-6)


@pytest.mark.parametrize("theta", THETAS)
def test_many_body_bloch_condition_and_exchange(oracle, theta):
    """Moving one electron by L e_m multiplies psi by e^{i theta_m} (ln|psi|, E_L and the
    derivatives unchanged); exchanging two same-spin electrons adds pi to the phase."""
    wl = workload("h16")
    s = _sys(oracle, wl, theta)
    x = wl.electrons(W=1, seed_offset=6)[0]
    r0 = s.local(x)
    for e, m in [(0, 0), (5, 1), (12, 2)]:
        x2 = x.copy()
        x2[e, m] += wl.L
        r = s.local(x2)
        assert r["lnpsi"] == pytest.approx(r0["lnpsi"], abs=1e-11)
        assert np.exp(1j * r["phase"]) == pytest.approx(np.exp(1j * (r0["phase"] + theta[m])), abs=1e-10)
        assert r["EL"] == pytest.approx(r0["EL"], rel=1e-11)
        assert np.allclose(r["dEL"], r0["dEL"], rtol=1e-9, atol=1e-10)
    x3 = x.copy()
    x3[[1, 4]] = x3[[4, 1]]
    r = s.local(x3)
    assert np.exp(1j * r["phase"]) == pytest.approx(-np.exp(1j * r0["phase"]), abs=1e-10)
    assert r["EL"] == pytest.approx(r0["EL"], rel=1e-11)


@pytest.mark.parametrize("jas", JAS)
@pytest.mark.parametrize("theta", THETAS)
def test_proton_derivatives_equal_fd(oracle, theta, jas):
    """d ln|psi| / dR and d Re E_L / dR against central differences in the proton positions
    (orbital coefficients held fixed)."""
    wl = small_system(6, 1.3, seed=4)
    s = _sys(oracle, wl, theta, **jas)
    x = wl.electrons(W=1, seed_offset=7)[0]
    r = s.local(x)
    h = 1e-5
    for t in range(3 * wl.n):
        Rp, Rm = wl.R.reshape(-1).copy(), wl.R.reshape(-1).copy()
        Rp[t] += h
        Rm[t] -= h
        sp = oracle.CSystem(Rp.reshape(-1, 3), wl.zeta, s.Cc, theta, wl.L, **jas)
        sm = oracle.CSystem(Rm.reshape(-1, 3), wl.zeta, s.Cc, theta, wl.L, **jas)
        a, b = sp.local(x, False), sm.local(x, False)
        assert r["dlnpsi"][t] == pytest.approx((a["lnpsi"] - b["lnpsi"]) / (2 * h), rel=1e-6, abs=1e-7)
        assert r["dEL"][t] == pytest.approx((a["EL"] - b["EL"]) / (2 * h), rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("jas", JAS)
def test_sweep_decisions_follow_psi_ratios(oracle, jas):
    """Each Metropolis decision of a sweep equals u < |psi(x')/psi(x)|^2 with ln|psi| from the
    local-energy routine, on the move drawn from the same Philox counters."""
    wl = small_system(6, 1.3, seed=4)
    s = _sys(oracle, wl, np.array(THETAS[0]), **jas)
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


@pytest.mark.parametrize("jas", JAS)
def test_force_estimator_equals_correlated_sampling_derivative(oracle, jas):
    wl = small_system(6, 1.3, seed=4)
    theta = np.array(THETAS[1])
    s = _sys(oracle, wl, theta, **jas)
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
        sp = oracle.CSystem(Rflat.reshape(-1, 3), wl.zeta, s.Cc, theta, wl.L, **jas)
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


def test_monkhorst_pack_mesh():
    from oracle import oracle as O
    th = O.monkhorst_pack(4)
    assert th.shape == (64, 3)
    assert np.allclose(np.sort(np.unique(np.round(th[:, 0], 12))), [-3 * np.pi / 4, -np.pi / 4, np.pi / 4, 3 * np.pi / 4])
    assert np.allclose(th.sum(0), 0.0)                  # symmetric about the origin


# ---- the contracted basis (phi_1 + eta phi_2) under general twists, in a box with Z2 (1.5 L)^2 >= 36
ETA = 0.1


def _cbox():
    return small_system(6, 2.5, seed=4)


def _csys(oracle, wl, theta, **kw):
    Cc, _ = oracle.chuckel_contracted(wl.R, wl.L, wl.n // 2, ETA, theta)
    return oracle.CSystem(wl.R, wl.zeta, Cc, theta, wl.L, eta=ETA, **kw)


def test_contracted_bloch_basis_reduces_to_the_real_one_at_real_twists(oracle):
    wl = _cbox()
    assert oracle.Z2 * (1.5 * wl.L) ** 2 >= 36.0
    rng = np.random.default_rng(2)
    for tw in range(8):
        theta = np.array([np.pi * ((tw >> m) & 1) for m in range(3)])
        sc = oracle.CSystem(wl.R, wl.zeta, np.eye(wl.n, 3, dtype=complex), theta, wl.L, eta=ETA)
        sr = oracle.System(wl.R, wl.zeta, np.eye(wl.n, 3), L=wl.L, twist=tw, eta=ETA)
        for _ in range(4):
            a = int(rng.integers(wl.n))
            r = wl.R[a] + rng.uniform(-1.5 * wl.L, 1.5 * wl.L, 3)
            c, v = sc.cbasis(a, r), sr.basis(a, r)
            assert np.allclose(c.real, v, rtol=1e-12, atol=1e-14 * np.max(np.abs(v)))
            assert np.max(np.abs(c.imag)) < 1e-13 * np.max(np.abs(v))


@pytest.mark.parametrize("theta", THETAS)
def test_contracted_bloch_condition(oracle, theta):
    wl = _cbox()
    s = oracle.CSystem(wl.R, wl.zeta, np.eye(wl.n, 3, dtype=complex), np.array(theta), wl.L, eta=ETA)
    rng = np.random.default_rng(3)
    for _ in range(4):
        a = int(rng.integers(wl.n))
        r = rng.uniform(0.0, wl.L, 3)
        f0 = s.cbasis(a, r)
        for m in range(3):
            r2 = r.copy()
            r2[m] += wl.L
            assert np.allclose(s.cbasis(a, r2), np.exp(1j * theta[m]) * f0, rtol=1e-12,
                               atol=1e-13 * np.max(np.abs(f0)))


@pytest.mark.parametrize("theta", THETAS)
def test_contracted_overlap_equals_cell_quadrature(oracle, theta):
    """The contracted overlaps (axis moments with Bloch weights) against the trapezoid rule over
    the cell of conj(phi_a) phi_b; Hermitian; the Hueckel orbitals against numpy's eigh."""
    wl = _cbox()
    th = np.array(theta)
    s = oracle.CSystem(wl.R, wl.zeta, np.eye(wl.n, 3, dtype=complex), th, wl.L, eta=ETA)
    ng = 40
    g = (np.arange(ng) + 0.5) * wl.L / ng
    pts = np.array(list(itertools.product(g, g, g)))
    phi = s.cbasis_values(pts)
    Sq = (phi.conj().T @ phi) * (wl.L / ng) ** 3
    S = oracle.coverlap_contracted(wl.R, wl.L, ETA, th)
    assert np.max(np.abs(S - Sq)) < 1e-9 * np.max(np.abs(S))
    assert np.max(np.abs(S - S.conj().T)) < 1e-15 * np.max(np.abs(S))
    Cc, ev = oracle.chuckel_contracted(wl.R, wl.L, 3, ETA, th)
    assert np.allclose(Cc.conj().T @ S @ Cc, np.diag(-ev[:3]), atol=1e-12)
    d = np.sqrt(np.real(np.diag(S)))
    w, v = np.linalg.eigh(-S / np.outer(d, d))
    Cn = v[:, :3] / d[:, None]
    assert np.allclose(Cc @ Cc.conj().T, Cn @ Cn.conj().T, atol=1e-12)


@pytest.mark.parametrize("jas", JAS)
def test_contracted_complex_wavefunction_at_zero_twist_is_the_real_one(oracle, jas):
    wl = _cbox()
    s = _csys(oracle, wl, np.zeros(3), **jas)
    Cr, _ = oracle.huckel_contracted(wl.R, wl.L, 3, ETA)
    sr = oracle.System(wl.R, wl.zeta, Cr, L=wl.L, eta=ETA, **jas)
    assert np.allclose(s.Cc @ s.Cc.conj().T, Cr @ Cr.T, atol=1e-12)
    for x in wl.electrons(W=2, seed_offset=9):
        a, b = s.local(x), sr.local(x)
        assert a["lnpsi"] == pytest.approx(b["lnpsi"], rel=1e-12, abs=1e-12)
        assert a["EL"] == pytest.approx(b["EL"], rel=1e-12)
        assert np.allclose(a["dlnpsi"], b["dlnpsi"], rtol=1e-10, atol=1e-11)
        assert np.allclose(a["dEL"], b["dEL"], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("jas", JAS)
def test_contracted_complex_kinetic_energy_and_proton_derivatives_by_fd(oracle, jas):
    wl = _cbox()
    th = np.array(THETAS[1])
    s = _csys(oracle, wl, th, **jas)
    x = wl.electrons(W=1, seed_offset=5)[0]
    r = s.local(x)
    V, _, _ = s.potential(x)
    psi = lambda y: np.exp(s.local(y, False)["lnpsi"] + 1j * s.local(y, False)["phase"])
    p0 = psi(x)
    h = 1e-4
    lap = 0j
    for e in range(wl.n):
        for m in range(3):
            xp, xm = x.copy(), x.copy()
            xp[e, m] += h
            xm[e, m] -= h
            lap += (psi(xp) - 2 * p0 + psi(xm)) / (h * h)
    assert r["EL"] - V == pytest.approx(float(np.real(-0.5 * lap / p0)), rel=2e-6, abs=2e-6)
    hr = 1e-5
    for t in range(0, 3 * wl.n, 2):
        Rp, Rm = wl.R.reshape(-1).copy(), wl.R.reshape(-1).copy()
        Rp[t] += hr
        Rm[t] -= hr
        a = oracle.CSystem(Rp.reshape(-1, 3), wl.zeta, s.Cc, th, wl.L, eta=ETA, **jas).local(x, False)
        b = oracle.CSystem(Rm.reshape(-1, 3), wl.zeta, s.Cc, th, wl.L, eta=ETA, **jas).local(x, False)
        assert r["dlnpsi"][t] == pytest.approx((a["lnpsi"] - b["lnpsi"]) / (2 * hr), rel=1e-6, abs=1e-7)
        assert r["dEL"][t] == pytest.approx((a["EL"] - b["EL"]) / (2 * hr), rel=1e-6, abs=1e-6)
