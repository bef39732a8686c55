"""The contracted minimal basis (phi_1 + eta phi_2 per proton, the SI's Z1 and Z2) on the GPU
against the oracle's contracted basis on the same seeded inputs, through the C ABI: fixed
configurations and same-seed chains in FP64 (bar 1e-10, as for the single Gaussian) and in mixed
precision (the bars of the mixed single-Gaussian path), plus the argument checks."""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import small_system, workload

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
TOLM = {"lnpsi": 1e-6, "EL": 5e-5, "dlnpsi": 2e-5, "dEL": 2e-5}
ETA = 0.1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem(a, b):
    a, b = np.atleast_1d(np.asarray(a, dtype=np.float64)), np.atleast_1d(np.asarray(b, dtype=np.float64))
    return float(np.max(np.abs(a - b) / (np.abs(b) + np.max(np.abs(b)) + 1e-300)))


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_1605_08423_amd import vmc
    return torch, vmc, vmc.Context(0)


def _T(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _box(name):
    """Boxes with L >= 6.9 bohr (the contracted basis needs Z2 (1.5 L)^2 >= 36)."""
    if name in ("h54", "h128"):
        return workload(name)
    n = int(name[1:])
    return small_system(n, {16: 1.9, 32: 1.45}[n], seed=21)


@pytest.mark.parametrize("name,K,prec", [("h16", 16, 0), ("h32", 6, 0), ("h54", 6, 0), ("h128", 3, 0),
                                         ("h16", 16, 1), ("h54", 6, 1), ("h128", 3, 1)])
def test_contracted_eval_configs(oracle, dev, name, K, prec):
    torch, vmc, ctx = dev
    wl = _box(name)
    say(f"[contracted eval_configs] {name} K={K} {'mixed' if prec else 'fp64'}")
    Cm, _ = oracle.huckel_contracted(wl.R, wl.L, wl.n // 2, ETA)
    pos = wl.electrons(W=K, seed_offset=3)
    sysd = vmc.make_system(wl.n, wl.L, precision=prec, eta=ETA)
    g = vmc.vmc_eval_configs(ctx, sysd, _T(torch, wl.R.reshape(-1)), _T(torch, Cm), _T(torch, wl.zeta),
                             _T(torch, pos)).cpu().numpy()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, eta=ETA)
    n3 = 3 * wl.n
    worst = {}
    for k in range(K):
        r = s.local(pos[k])
        for q, a, b in [("lnpsi", g[k, 0], r["lnpsi"]), ("EL", g[k, 1], r["EL"]),
                        ("dlnpsi", g[k, 2:2 + n3], r["dlnpsi"]), ("dEL", g[k, 2 + n3:], r["dEL"])]:
            worst[q] = max(worst.get(q, 0.0), rel(a, b) if q in ("lnpsi", "EL") else elem(a, b))
    say("  worst errors", worst)
    for q, v in worst.items():
        assert v < (TOL64 if prec == 0 else TOLM[q]), (q, v)


@pytest.mark.parametrize("name,W,ne,ns", [("h16", 32, 2, 4), ("h54", 8, 1, 3), ("h128", 2, 1, 2)])
def test_contracted_chain_fp64(oracle, dev, name, W, ne, ns):
    torch, vmc, ctx = dev
    wl = _box(name)
    say(f"[contracted chain fp64] {name} W={W} equil={ne} sweeps={ns}")
    Cm, _ = oracle.huckel_contracted(wl.R, wl.L, wl.n // 2, ETA)
    pos = wl.electrons(W=W, seed_offset=7)
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, eta=ETA), W, seed=11, traj_id=3)
    tr.set_walkers(_T(torch, pos))
    out = tr.energy_forces(_T(torch, wl.R.reshape(-1)), _T(torch, Cm), _T(torch, wl.zeta), ne, ns, wl.delta,
                           2).cpu().numpy()
    means, acc, posg = tr.walker_means().cpu().numpy(), tr.accepts().cpu().numpy(), tr.get_walkers().cpu().numpy()
    tr.close()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, eta=ETA)
    xo = pos.copy()
    sums, nacc = s.vmc_run(xo, ne, ns, wl.delta, seed=11, traj=3, step=2)
    red = oracle.reduce(sums, ns)
    flips = int(np.sum(acc != nacc))
    say("  accepted moves gpu/oracle", acc.sum(), nacc.sum(), "walkers with a flipped decision:", flips)
    assert flips == 0
    assert rel(posg, xo) < 1e-12
    worst = max(elem(means[w], red["means"][w]) for w in range(W))
    say(f"  worst walker element-wise error of the means {worst:.3e}")
    assert worst < TOL64
    assert rel(out[0], red["E"]) < TOL64 and elem(out[3:], red["f"]) < TOL64


@pytest.mark.parametrize("name,W,ne,ns", [("h16", 64, 4, 8), ("h54", 128, 2, 3)])
def test_contracted_chain_mixed_same_seed(oracle, dev, name, W, ne, ns):
    """Mixed precision against the FP64 oracle on the same Philox stream: E and f within the
    mixed bars when no decision flipped, else within 2 sigma of the oracle's estimate."""
    torch, vmc, ctx = dev
    wl = _box(name)
    say(f"[contracted chain mixed] {name} W={W}")
    Cm, _ = oracle.huckel_contracted(wl.R, wl.L, wl.n // 2, ETA)
    pos = wl.electrons(W=W, seed_offset=9)
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, precision=vmc.VMC_MIXED, eta=ETA), W, seed=5, traj_id=1)
    tr.set_walkers(_T(torch, pos))
    out = tr.energy_forces(_T(torch, wl.R.reshape(-1)), _T(torch, Cm), _T(torch, wl.zeta), ne, ns, wl.delta,
                           0).cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    tr.close()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L, eta=ETA)
    xo = pos.copy()
    sums, nacc = s.vmc_run(xo, ne, ns, wl.delta, seed=5, traj=1, step=0)
    red = oracle.reduce(sums, ns)
    flips = int(np.sum(acc != nacc))
    say("  E gpu/oracle", out[0], red["E"], "flipped walkers", flips)
    if flips == 0:
        assert rel(out[0], red["E"]) < 1e-6
        assert rel(out[3:], red["f"]) < 1e-5
    else:
        assert abs(out[0] - red["E"]) < 2 * red["sigma_E"]


def test_contracted_system_validation(dev):
    torch, vmc, ctx = dev
    small = small_system(16, 1.3, seed=2)     # L = 5.3: Z2 (1.5 L)^2 < 36
    wl = _box("h16")
    bad = [vmc.make_system(small.n, small.L, eta=ETA),
           vmc.make_system(wl.n, wl.L, eta=ETA, twist=1),
           vmc.make_system(256, 14.0, eta=ETA),
           vmc.make_system(wl.n, wl.L, eta=float("nan"))]
    for sysd in bad:
        with pytest.raises(vmc.VMCError) as ei:
            vmc.Trajectory(ctx, sysd, 4)
        assert ei.value.code == vmc.VMC_EINVAL
