"""Real twisted boundary conditions (twist angle 0 or pi per axis; SI, basis section) on the
GPU against the CPU oracle, through the C ABI: per-configuration quantities with the orbitals
of each twist (FP64 1e-10, mixed per-quantity bars), Metropolis chains on the oracle's Philox
stream, the request loop, and the twist average of forces and their covariance."""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
TOLMIX = {"lnpsi": 1e-6, "EL": 5e-5, "dlnpsi": 2e-5, "dEL": 2e-5}


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


@pytest.mark.parametrize("name,K,precision,twist", [("h16", 8, 0, 1), ("h16", 8, 0, 7), ("h54", 4, 0, 5),
                                                    ("h128", 2, 0, 6), ("h256", 1, 0, 3), ("h16", 8, 1, 2),
                                                    ("h54", 4, 1, 7), ("h128", 2, 1, 5), ("h256", 1, 1, 6)])
def test_eval_configs_twisted(oracle, dev, name, K, precision, twist):
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[twisted eval_configs] {name} K={K} precision={precision} twist={twist}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2, twist=twist)
    pos = wl.electrons(W=K, seed_offset=6)
    g = vmc.vmc_eval_configs(ctx, vmc.make_system(wl.n, wl.L, precision=precision, twist=twist),
                             T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), T(torch, pos)).cpu().numpy()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, twist=twist)
    s0 = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    n3 = 3 * wl.n
    worst = dict.fromkeys(TOLMIX, 0.0)
    differs = False
    for k in range(K):
        r = s.local(pos[k])
        worst["lnpsi"] = max(worst["lnpsi"], rel(g[k, 0], r["lnpsi"]))
        worst["EL"] = max(worst["EL"], rel(g[k, 1], r["EL"]))
        worst["dlnpsi"] = max(worst["dlnpsi"], rel(g[k, 2:2 + n3], r["dlnpsi"]))
        worst["dEL"] = max(worst["dEL"], rel(g[k, 2 + n3:], r["dEL"]))
        differs |= abs(s0.local(pos[k], False)["EL"] - r["EL"]) > 1e-6 * abs(r["EL"])
    say("  worst relative errors", {k: f"{v:.2e}" for k, v in worst.items()})
    for q, v in worst.items():
        assert v < (TOL64 if precision == 0 else TOLMIX[q]), (q, v)
    assert differs     # the twist changes the local energy (the test is not the periodic case)


@pytest.mark.parametrize("name,W,ne,ns,twist", [("h16", 24, 2, 3, 7), ("h54", 6, 1, 2, 3), ("h128", 2, 1, 1, 5),
                                                ("h256", 2, 1, 1, 6)])
def test_chain_twisted_fp64(oracle, dev, name, W, ne, ns, twist):
    """Sweeps and measurements on the oracle's Philox stream: identical acceptances and
    per-walker means at 1e-10.  Moves that cross the cell boundary flip the sign of the moved
    orbital row; the ratio's square, and so the chain, does not change."""
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[twisted chain] {name} W={W} sweeps={ne}+{ns} twist={twist}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2, twist=twist)
    x0 = wl.electrons(W=W, seed_offset=10)
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, twist=twist), W, seed=13, traj_id=6)
    tr.set_walkers(T(torch, x0))
    out = tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), ne, ns, wl.delta, 1)
    out = out.cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    means = tr.walker_means().cpu().numpy()
    posg = tr.get_walkers().cpu().numpy()
    tr.close()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, twist=twist)
    xo = x0.copy()
    sums, nacc = s.vmc_run(xo, ne, ns, wl.delta, seed=13, traj=6, step=1)
    red = oracle.reduce(sums, ns)
    flips = int(np.sum(acc != nacc))
    say(f"  accepted gpu/oracle {acc.sum()}/{nacc.sum()}  walkers with a flipped decision: {flips}")
    assert flips == 0
    assert rel(posg, xo) < 1e-12
    n3 = 3 * wl.n
    mo = red["means"]
    for q, sl in [("e_w", slice(0, 1)), ("d_w", slice(1, 1 + n3)), ("g_w", slice(1 + n3, 1 + 2 * n3)),
                  ("h_w", slice(1 + 2 * n3, 1 + 3 * n3))]:
        e = max(rel(means[w, sl], mo[w, sl]) for w in range(W))
        say(f"  {q} worst walker rel err {e:.3e}")
        assert e < TOL64, q
    assert rel(out[0], red["E"]) < TOL64 and rel(out[3:], red["f"]) < TOL64


@pytest.mark.parametrize("name,precision,twist", [("h54", 0, 6), ("h128", 1, 3)])
def test_twist_with_one_body_term(oracle, dev, name, precision, twist):
    """A twist and the one-body Jastrow term together (the term stays periodic): per-configuration
    quantities and, in FP64, a two-sweep chain against the oracle.  The mixed-precision bars hold
    for Slater matrices of ordinary condition (these configurations: below 2e4); near a node
    (condition number kappa) the FP32 products lose about kappa * 6e-8 relative accuracy, so the
    configurations are fixed by seed."""
    torch, vmc, ctx = dev
    wl = workload(name)
    b1 = 2.5
    say(f"[twist + one-body] {name} precision={precision} twist={twist}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2, twist=twist)
    sysd = vmc.make_system(wl.n, wl.L, precision=precision, twist=twist, b1=b1)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, twist=twist, b1=b1)
    pos = wl.electrons(W=2, seed_offset=6)
    g = vmc.vmc_eval_configs(ctx, sysd, T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta),
                             T(torch, pos)).cpu().numpy()
    n3 = 3 * wl.n
    tol = TOL64 if precision == 0 else None
    for k in range(2):
        r = s.local(pos[k])
        errs = {"lnpsi": rel(g[k, 0], r["lnpsi"]), "EL": rel(g[k, 1], r["EL"]),
                "dlnpsi": rel(g[k, 2:2 + n3], r["dlnpsi"]), "dEL": rel(g[k, 2 + n3:], r["dEL"])}
        say("  config", k, {q: f"{v:.2e}" for q, v in errs.items()})
        for q, v in errs.items():
            assert v < (tol if tol else TOLMIX[q]), (q, v)
    if precision == 0:
        W = 4
        x0 = wl.electrons(W=W, seed_offset=14)
        tr = vmc.Trajectory(ctx, sysd, W, seed=15, traj_id=2)
        tr.set_walkers(T(torch, x0))
        out = tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), 1, 1, wl.delta, 0)
        out = out.cpu().numpy()
        acc = tr.accepts().cpu().numpy()
        tr.close()
        xo = x0.copy()
        sums, nacc = s.vmc_run(xo, 1, 1, wl.delta, seed=15, traj=2, step=0)
        red = oracle.reduce(sums, 1)
        assert np.array_equal(acc, nacc)
        assert rel(out[0], red["E"]) < TOL64 and rel(out[3:], red["f"]) < TOL64


def test_twist_average(dev):
    torch, vmc, ctx = dev
    rng = np.random.default_rng(4)
    for n_tw, n3 in [(1, 5), (8, 48), (3, 384)]:
        fs = rng.normal(size=(n_tw, n3))
        Ss = rng.normal(size=(n_tw, n3, n3))
        f, S = vmc.vmc_twist_average(ctx, T(torch, fs), T(torch, Ss))
        np.testing.assert_allclose(f.cpu().numpy(), fs.mean(axis=0), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(S.cpu().numpy(), Ss.sum(axis=0) / n_tw ** 2, rtol=1e-14, atol=1e-15)


def test_served_twisted_equals_single_trajectory_calls(dev):
    """A served trajectory with a twist (the request loop takes the Hueckel orbitals of its
    twist) equals the same trajectory through the single-trajectory calls, bit for bit."""
    torch, vmc, ctx = dev
    wl = workload("h16")
    W, M, steps, twist, seed, traj = 64, 4, 2, 5, 5, 7
    alpha = 0.122 * W * M
    sysd = vmc.make_system(wl.n, wl.L, twist=twist)
    req = vmc.make_request(sysd, W, wl.R, wl.zeta, wl.electrons(W=W, seed_offset=traj), n_steps=steps, n_sweeps=M,
                           T=wl.T_hartree, Delta=1.0 / alpha, alpha=alpha, n_equil_first=2, n_equil=1,
                           step_delta=wl.delta, seed=seed, traj_id=traj)
    srv = vmc.Server(ctx, 8 << 30)
    rid = srv.submit(req)
    srv.run_until_idle()
    st, res = srv.status(rid), srv.result(rid)
    srv.close()
    assert st[0] == vmc.VMC_REQ_DONE
    tr = vmc.Trajectory(ctx, sysd, W, seed=seed, traj_id=traj)
    tr.set_walkers(T(torch, wl.electrons(W=W, seed_offset=traj)))
    R = T(torch, wl.R.reshape(-1))
    zeta = T(torch, wl.zeta)
    Rp, Sp = R.clone(), None
    Es = []
    for k in range(steps):
        Cm = vmc.vmc_huckel_params(R.cpu().numpy(), wl.zeta, wl.L, twist=twist)
        out = tr.energy_forces(R, T(torch, Cm), zeta, 2 if k == 0 else 1, M, wl.delta, k)
        S = tr.build_S()
        if k == 0:
            Sp = S.clone()
            Rp.copy_(R)
        assert vmc.vmc_langevin_step(ctx, R, Rp, Sp, out[3:], S, wl.T_hartree, 1.0 / alpha, alpha, 0, seed, traj, k,
                                     wl.L) == 0
        Es.append(float(out[0]))
    tr.close()
    assert np.array_equal(res["R"], R.cpu().numpy())
    assert np.array_equal(res["E"], np.array(Es))


def test_served_twists_alone_equal_mixed_batch(dev):
    """Mixed precision, N = 54: trajectories with different twists and one untwisted one in one
    request loop (the twisted ones share launches) equal each served alone, bit for bit."""
    torch, vmc, ctx = dev
    wl = workload("h54")
    W, M = 176, 3
    alpha = 0.122 * W * M
    reqs = []
    for traj, tw in [(60, 3), (61, 0), (62, 5)]:
        sysd = vmc.make_system(wl.n, wl.L, precision=1, twist=tw)
        reqs.append(vmc.make_request(sysd, W, wl.R, wl.zeta, wl.electrons(W=W, seed_offset=traj), n_steps=2,
                                     n_sweeps=M, T=wl.T_hartree, Delta=1.0 / alpha, alpha=alpha, n_equil_first=2,
                                     n_equil=1, step_delta=wl.delta, seed=3, traj_id=traj))

    def serve(rs):
        srv = vmc.Server(ctx, 16 << 30)
        ids = [srv.submit(r) for r in rs]
        srv.run_until_idle()
        out = [(srv.status(i), srv.result(i)) for i in ids]
        srv.close()
        return out

    say("[twists served] h54 mixed, twists 3, 0, 5")
    alone = [serve([r])[0] for r in reqs]
    together = serve(reqs)
    for (sa, ra), (sm, rm) in zip(alone, together):
        assert sa[0] == sm[0] == vmc.VMC_REQ_DONE
        assert np.array_equal(ra["R"], rm["R"]) and np.array_equal(ra["E"], rm["E"])


def test_twist_parameter_checked(dev):
    torch, vmc, ctx = dev
    wl = workload("h16")
    for bad in (-1, 8):
        with pytest.raises(vmc.VMCError):
            vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, twist=bad), 8, seed=1, traj_id=0)
