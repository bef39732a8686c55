"""Edge cases of the HIP path through the C ABI: ragged walker counts (the sweep
kernels pack four walkers per work-group), a single walker/configuration, the
smallest covariance (W = 2), a one-coordinate Langevin step and argument errors."""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_1605_08423_amd import vmc
    return torch, vmc, vmc.Context(0)


def T(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("W", [1, 5, 7, 13])
def test_ragged_walker_counts_fp64_chain(oracle, dev, W):
    torch, vmc, ctx = dev
    wl = workload("h16")
    say(f"[ragged chain] W={W}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8)
    x0 = wl.electrons(W=W, seed_offset=40 + W)
    tr = vmc.Trajectory(ctx, vmc.make_system(16, wl.L), W, seed=9, traj_id=2)
    tr.set_walkers(T(torch, x0))
    out = tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), 1, 3, wl.delta, 5).cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    means = tr.walker_means().cpu().numpy()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    sums, nacc = s.vmc_run(x0.copy(), 1, 3, wl.delta, seed=9, traj=2, step=5)
    red = oracle.reduce(sums, 3)
    assert np.array_equal(acc, nacc)
    assert rel(means, red["means"]) < 1e-10
    assert rel(out[0], red["E"]) < 1e-10
    if W > 1:
        assert rel(out[3:], red["f"]) < 1e-10


def test_single_configuration(oracle, dev):
    torch, vmc, ctx = dev
    wl = workload("h54")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 27)
    pos = wl.electrons(W=1, seed_offset=3)
    g = vmc.vmc_eval_configs(ctx, vmc.make_system(54, wl.L), T(torch, wl.R.reshape(-1)), T(torch, Cm),
                             T(torch, wl.zeta), T(torch, pos)).cpu().numpy()
    r = oracle.System(wl.R, wl.zeta, Cm, L=wl.L).local(pos[0])
    assert rel(g[0, 1], r["EL"]) < 1e-10 and rel(g[0, 2 + 162:], r["dEL"]) < 1e-10


def test_build_S_two_walkers_and_1d_langevin(oracle, dev):
    torch, vmc, ctx = dev
    fw = np.array([[1.0, 2.0, -1.0], [0.5, -1.0, 3.0]])
    f = fw.mean(0)
    S = vmc.vmc_build_S_raw(ctx, T(torch, fw), T(torch, f)).cpu().numpy()
    np.testing.assert_allclose(S, oracle.build_S(fw, f), rtol=1e-14)
    R, Rp, Sp = T(torch, [0.3]), T(torch, [0.3]), T(torch, [[2.0]])
    assert vmc.vmc_langevin_step(ctx, R, Rp, Sp, T(torch, [0.5]), T(torch, [[2.0]]), 0.1, 0.2, 0.0, 0, 1, 0, 3) == 0
    Ro, Rpo, Spo = np.array([0.3]), np.array([0.3]), np.array([[2.0]])
    oracle.langevin(Ro, Rpo, Spo, np.array([0.5]), np.array([[2.0]]), 0.1, 0.2, 0.0, seed=1, traj=0, step=3)
    assert rel(R.cpu().numpy(), Ro) < 1e-14


def test_argument_errors(dev):
    torch, vmc, ctx = dev
    with pytest.raises(vmc.VMCError) as e:
        vmc.Trajectory(ctx, vmc.make_system(17, 6.0), 4)
    assert e.value.code == vmc.VMC_EINVAL
    with pytest.raises(vmc.VMCError):
        vmc.Trajectory(ctx, vmc.make_system(100, 10.0), 4)         # unsupported size
    with pytest.raises(vmc.VMCError):
        vmc.vmc_build_S_raw(ctx, T(torch, np.ones((1, 3))), T(torch, np.ones(3)))   # W < 2


def _chain(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, refine_tol, precision=None):
    prec = vmc.VMC_FP64 if precision is None else precision
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, precision=prec, refine_tol=refine_tol), W, seed=4,
                        traj_id=3)
    tr.set_walkers(T(torch, x0))
    out = tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), ne, ns, wl.delta, 2)
    res = out.cpu().numpy(), tr.accepts().cpu().numpy(), tr.walker_means().cpu().numpy()
    tr.close()
    return res


@pytest.mark.parametrize("name,W,ne,ns", [("h54", 8, 1, 4), ("h128", 4, 1, 3), ("h256", 3, 1, 1)])
def test_refinement_refresh_matches_elimination_and_oracle(oracle, dev, name, W, ne, ns):
    """The Newton-Schulz refresh (default), elimination for every matrix (refine_tol < 0)
    and the oracle's fresh determinants give the same chain: identical acceptances and
    FP64-level agreement of the estimates.  A tolerance no residual can meet sends every
    matrix through the refinement's elimination fallback, which must reproduce the
    elimination path bit for bit."""
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[refresh paths] {name} W={W} sweeps={ne}+{ns}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    x0 = wl.electrons(W=W, seed_offset=61)
    o_ref, a_ref, m_ref = _chain(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, 0.0)
    o_gj, a_gj, m_gj = _chain(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, -1.0)
    o_fb, a_fb, m_fb = _chain(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, 1e-300)
    assert np.array_equal(a_ref, a_gj) and np.array_equal(a_fb, a_gj)
    assert np.array_equal(m_fb, m_gj) and np.array_equal(o_fb, o_gj)
    assert rel(m_ref, m_gj) < 1e-11
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    sums, nacc = s.vmc_run(x0.copy(), ne, ns, wl.delta, seed=4, traj=3, step=2)
    red = oracle.reduce(sums, ns)
    assert np.array_equal(a_ref, nacc)
    assert rel(m_ref, red["means"]) < 1e-10
    say(f"  refine vs elimination {rel(m_ref, m_gj):.2e}  refine vs oracle {rel(m_ref, red['means']):.2e}")


def test_refine_tol_nan_rejected(dev):
    torch, vmc, ctx = dev
    with pytest.raises(vmc.VMCError):
        vmc.Trajectory(ctx, vmc.make_system(16, 6.0, refine_tol=float("nan")), 4)


@pytest.mark.parametrize("precision", [0, 1])
def test_runs_are_deterministic(dev, precision):
    """Two trajectories with the same seed, walkers and inputs give bitwise-equal results: every
    reduction runs in a fixed order (no floating-point atomics), so a run is reproducible."""
    import torch
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload
    _, _, ctx = dev
    wl = workload("h54")
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L)
    T_ = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    res = []
    for _ in range(2):
        tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, precision=precision, b1=2.5), 200, seed=6, traj_id=1)
        tr.set_walkers(T_(wl.electrons(W=200, seed_offset=4)))
        out = tr.energy_forces(T_(wl.R.reshape(-1)), T_(Cm), T_(wl.zeta), 2, 3, wl.delta, 0)
        S = tr.build_S()
        res.append((out.cpu().numpy(), S.cpu().numpy(), tr.walker_means().cpu().numpy(), tr.get_walkers().cpu().numpy()))
        tr.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_walker_quarantine(dev):
    """A walker with a non-finite coordinate restarts from a copy of the next finite walker at
    the start of vmc_energy_forces and is counted; the call then equals one started from those
    copies.  With every walker non-finite the call is refused and changes nothing."""
    import torch
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload
    _, _, ctx = dev
    wl = workload("h16")
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L)
    T_ = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    x = wl.electrons(W=16, seed_offset=2)
    bad = x.copy()
    bad[5, 3, 1] = np.nan
    bad[9, 0, 2] = np.inf
    fixed = x.copy()
    fixed[5], fixed[9] = x[6], x[10]
    outs = []
    for start, expect in ((bad, 2), (fixed, 0)):
        tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L), 16, seed=3, traj_id=0)
        tr.set_walkers(T_(start))
        out = tr.energy_forces(T_(wl.R.reshape(-1)), T_(Cm), T_(wl.zeta), 1, 2, wl.delta, 0).cpu().numpy()
        assert tr.walkers_reset() == expect
        assert np.all(np.isfinite(out))
        outs.append(out)
        tr.close()
    assert np.array_equal(outs[0], outs[1])
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L), 4, seed=3, traj_id=0)
    allbad = np.full((4, wl.n, 3), np.nan)
    tr.set_walkers(T_(allbad))
    with pytest.raises(vmc.VMCError):
        tr.energy_forces(T_(wl.R.reshape(-1)), T_(Cm), T_(wl.zeta), 1, 1, wl.delta, 0)
    assert np.all(np.isnan(tr.get_walkers().cpu().numpy()))
    tr.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_singular_slater_matrix_changes_nothing(oracle, dev, precision):
    """Two same-spin electrons at one point make that spin's Slater matrix exactly singular: the
    oracle's LU and the GPU's elimination both meet an exactly zero pivot (VMC_ESINGULAR), and
    the failing call leaves the walkers, the accepted-move counts, the last call's means and the
    output as they were."""
    torch, vmc, ctx = dev
    wl = workload("h16")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8)
    W = 4
    x = wl.electrons(W=W, seed_offset=44)
    x[2, 1] = x[2, 0]                         # electrons 0 and 1 are both spin up
    say(f"[singular] h16 precision={precision}")
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    with pytest.raises(RuntimeError, match="rc=-4"):
        s.local(x[2])
    with pytest.raises(RuntimeError, match="rc=-4"):
        s.vmc_run(x.copy(), 1, 1, wl.delta, seed=3)
    R, C, z = T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta)
    sysd = vmc.make_system(wl.n, wl.L, precision=precision)
    with pytest.raises(vmc.VMCError) as e:
        vmc.vmc_eval_configs(ctx, sysd, R, C, z, T(torch, x))
    assert e.value.code == vmc.VMC_ESINGULAR
    tr = vmc.Trajectory(ctx, sysd, W, seed=3, traj_id=0)
    tr.set_walkers(T(torch, wl.electrons(W=W, seed_offset=45)))
    tr.energy_forces(R, C, z, 1, 2, wl.delta, 0)
    means0, acc0, S0 = tr.walker_means().cpu().numpy(), tr.accepts().cpu().numpy(), tr.build_S().cpu().numpy()
    tr.set_walkers(T(torch, x))
    out = torch.full((3 + 3 * wl.n,), 123.0, dtype=torch.float64, device="cuda")
    with pytest.raises(vmc.VMCError) as e:
        tr.energy_forces(R, C, z, 1, 2, wl.delta, 1, out=out)
    assert e.value.code == vmc.VMC_ESINGULAR
    assert np.array_equal(tr.get_walkers().cpu().numpy(), x)
    assert np.array_equal(tr.walker_means().cpu().numpy(), means0)
    assert np.array_equal(tr.accepts().cpu().numpy(), acc0)
    assert np.array_equal(tr.build_S().cpu().numpy(), S0)
    assert bool((out == 123.0).all())
    tr.close()


def test_cancel_leaves_trajectory_unchanged(dev):
    """vmc_cancel: the call returns VMC_ECANCELLED with the walkers, counts and means of the
    previous call; the cancellation is consumed, so the next call runs and equals the same call
    on a trajectory that was never cancelled."""
    torch, vmc, ctx = dev
    wl = workload("h16")
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L)
    R, C, z = T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta)
    sysd = vmc.make_system(wl.n, wl.L)
    say("[cancel]")
    runs = []
    for cancel in (True, False):
        tr = vmc.Trajectory(ctx, sysd, 32, seed=8, traj_id=2)
        tr.set_walkers(T(torch, wl.electrons(W=32, seed_offset=2)))
        tr.energy_forces(R, C, z, 1, 2, wl.delta, 0)
        x1, m1 = tr.get_walkers().cpu().numpy(), tr.walker_means().cpu().numpy()
        if cancel:
            ctx.cancel()
            with pytest.raises(vmc.VMCError) as e:
                tr.energy_forces(R, C, z, 1, 20, wl.delta, 1)
            assert e.value.code == vmc.VMC_ECANCELLED
            assert np.array_equal(tr.get_walkers().cpu().numpy(), x1)
            assert np.array_equal(tr.walker_means().cpu().numpy(), m1)
        out = tr.energy_forces(R, C, z, 1, 2, wl.delta, 1).cpu().numpy()
        runs.append((out, tr.get_walkers().cpu().numpy()))
        tr.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("what", ["f", "R"])
def test_langevin_nonfinite_input_refused(oracle, dev, what):
    """A NaN force or position is an argument error on both sides; the state is unchanged."""
    torch, vmc, ctx = dev
    rng = np.random.default_rng(3)
    n3 = 12
    A = rng.standard_normal((n3, n3))
    S = A @ A.T + n3 * np.eye(n3)
    f = rng.standard_normal(n3)
    R = rng.uniform(0, 5.0, n3)
    if what == "f":
        f[4] = np.nan
    else:
        R[7] = np.nan
    Ro, Rpo, Spo = R.copy(), R.copy(), S.copy()
    assert oracle.langevin(Ro, Rpo, Spo, f, S, 0.01, 0.5, 0.0, L=6.0) == -1
    assert np.array_equal(Ro, R, equal_nan=True) and np.array_equal(Spo, S)
    Rg, Rpg, Spg = T(torch, R), T(torch, R), T(torch, S)
    rc = vmc.vmc_langevin_step(ctx, Rg, Rpg, Spg, T(torch, f), T(torch, S), 0.01, 0.5, 0.0, 0, 1, 0, 0, 6.0)
    assert rc == vmc.VMC_EINVAL
    assert np.array_equal(Rg.cpu().numpy(), R, equal_nan=True) and np.array_equal(Spg.cpu().numpy(), S)


def test_hbm_budget_of_context(dev):
    """vmc_set_hbm_budget: trajectories beyond the budget are refused with VMC_ENOMEM; the bytes
    in use follow creation and destruction."""
    torch, vmc, _ = dev
    ctx = vmc.Context(0)
    wl = workload("h16")
    sysd = vmc.make_system(wl.n, wl.L)
    b = vmc.traj_bytes(sysd, 64)
    assert b > 64 * wl.n * 3 * 8
    ctx.set_hbm_budget(2 * b + b // 2)
    t1 = vmc.Trajectory(ctx, sysd, 64)
    t2 = vmc.Trajectory(ctx, sysd, 64)
    assert ctx.hbm_in_use() == 2 * b
    with pytest.raises(vmc.VMCError) as e:
        vmc.Trajectory(ctx, sysd, 64)
    assert e.value.code == vmc.VMC_ENOMEM
    t1.close()
    assert ctx.hbm_in_use() == b
    t3 = vmc.Trajectory(ctx, sysd, 64)
    t2.close()
    t3.close()
    assert ctx.hbm_in_use() == 0
    ctx.close()
