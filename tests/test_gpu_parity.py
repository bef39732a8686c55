"""GPU (HIP) path against the CPU oracle on the same seeded inputs, through the C ABI.

FP64 bar: 1e-10 relative (norm-wise per quantity) on fixed configurations and on
per-walker chain averages (the chains share the Philox stream, so FP64 chains
coincide unless an acceptance decision flips, which is reported)."""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload, small_system

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem(a, b):
    """Largest element-wise error relative to the element plus an absolute floor of the largest
    element, max_i |a_i - b_i| / (|b_i| + max_j |b_j|): bounds every component, small ones too."""
    a, b = np.atleast_1d(np.asarray(a, dtype=np.float64)), np.atleast_1d(np.asarray(b, dtype=np.float64))
    return float(np.max(np.abs(a - b) / (np.abs(b) + np.max(np.abs(b)) + 1e-300)))


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_1605_08423_amd import vmc
    ctx = vmc.Context(0)
    return torch, vmc, ctx


def _setup(oracle, wl, n_conf, seed_offset=0):
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    pos = wl.electrons(W=n_conf, seed_offset=seed_offset)
    return Cm, pos


def _eval_gpu(torch, vmc, ctx, wl, Cm, pos, precision):
    sysd = vmc.make_system(wl.n, wl.L, precision=precision)
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = vmc.vmc_eval_configs(ctx, sysd, T(wl.R.reshape(-1)), T(Cm), T(wl.zeta), T(pos))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name,K", [("h16", 24), ("h54", 8), ("h32", 8), ("h64", 4), ("h128", 3)])
def test_eval_configs_fp64(oracle, dev, name, K):
    torch, vmc, ctx = dev
    wl = workload(name) if name in ("h16", "h54", "h128") else small_system(int(name[1:]), 1.35, seed=21)
    say(f"[eval_configs fp64] {name} K={K}")
    Cm, pos = _setup(oracle, wl, K)
    g = _eval_gpu(torch, vmc, ctx, wl, Cm, pos, vmc.VMC_FP64)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    n3 = 3 * wl.n
    worst = {"lnpsi": 0.0, "EL": 0.0, "dlnpsi": 0.0, "dEL": 0.0, "dlnpsi_elem": 0.0, "dEL_elem": 0.0}
    for k in range(K):
        r = s.local(pos[k])
        worst["lnpsi"] = max(worst["lnpsi"], rel(g[k, 0], r["lnpsi"]))
        worst["EL"] = max(worst["EL"], rel(g[k, 1], r["EL"]))
        worst["dlnpsi"] = max(worst["dlnpsi"], rel(g[k, 2:2 + n3], r["dlnpsi"]))
        worst["dEL"] = max(worst["dEL"], rel(g[k, 2 + n3:], r["dEL"]))
        worst["dlnpsi_elem"] = max(worst["dlnpsi_elem"], elem(g[k, 2:2 + n3], r["dlnpsi"]))
        worst["dEL_elem"] = max(worst["dEL_elem"], elem(g[k, 2 + n3:], r["dEL"]))
    say("  worst relative errors", worst)
    for q, v in worst.items():
        assert v < TOL64, (q, v)


def _chain(oracle, dev, wl, W, n_equil, n_sweeps, seed, step, precision):
    torch, vmc, ctx = dev
    Cm, pos = _setup(oracle, wl, W, seed_offset=7)
    sysd = vmc.make_system(wl.n, wl.L, precision=precision)
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    tr = vmc.Trajectory(ctx, sysd, W, seed=seed, traj_id=3)
    tr.set_walkers(T(pos))
    out = tr.energy_forces(T(wl.R.reshape(-1)), T(Cm), T(wl.zeta), n_equil, n_sweeps, wl.delta, step)
    means = tr.walker_means().cpu().numpy()
    fw = tr.walker_forces().cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    posg = tr.get_walkers().cpu().numpy()
    S = tr.build_S().cpu().numpy()
    out = out.cpu().numpy()
    tr.close()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    xo = pos.copy()
    sums, nacc = s.vmc_run(xo, n_equil, n_sweeps, wl.delta, seed=seed, traj=3, step=step)
    red = oracle.reduce(sums, n_sweeps)
    So = oracle.build_S(red["f_w"], red["f"])
    return dict(out=out, means=means, fw=fw, acc=acc, pos=posg, S=S), dict(red=red, nacc=nacc, pos=xo, S=So)


@pytest.mark.parametrize("name,W,ne,ns", [("h16", 32, 3, 6), ("h54", 8, 2, 3), ("h128", 2, 1, 2)])
def test_chain_fp64(oracle, dev, name, W, ne, ns):
    wl = workload(name)
    say(f"[chain fp64] {name} W={W} equil={ne} sweeps={ns}")
    g, o = _chain(oracle, dev, wl, W, ne, ns, seed=11, step=2, precision=0)
    flips = int(np.sum(g["acc"] != o["nacc"]))
    say("  accepted moves gpu/oracle", g["acc"].sum(), o["nacc"].sum(), "walkers with a flipped decision:", flips)
    assert flips == 0
    assert rel(g["pos"], o["pos"]) < 1e-12
    n3 = 3 * wl.n
    mo = o["red"]["means"]
    for q, sl in [("e_w", slice(0, 1)), ("d_w", slice(1, 1 + n3)), ("g_w", slice(1 + n3, 1 + 2 * n3)),
                  ("h_w", slice(1 + 2 * n3, 1 + 3 * n3))]:
        e = max(rel(g["means"][w, sl], mo[w, sl]) for w in range(W))
        ee = max(elem(g["means"][w, sl], mo[w, sl]) for w in range(W))
        say(f"  {q} worst walker rel err {e:.3e} (element-wise {ee:.3e})")
        assert e < TOL64 and ee < TOL64, q
    assert rel(g["out"][0], o["red"]["E"]) < TOL64
    assert rel(g["out"][1], o["red"]["sigma_E"]) < 1e-8
    assert rel(g["out"][3:], o["red"]["f"]) < TOL64 and elem(g["out"][3:], o["red"]["f"]) < TOL64
    assert rel(g["fw"], o["red"]["f_w"]) < TOL64
    assert rel(g["S"], o["S"]) < 1e-9
    acc_rate = o["nacc"].sum() / (W * wl.n * (ne + ns))
    assert g["out"][2] == pytest.approx(acc_rate, rel=1e-14)


def test_build_S_raw(oracle, dev):
    torch, vmc, ctx = dev
    say("[build_S_raw] W=3000 n3=162 and W=2500 n3=384")
    for W, n3 in [(3000, 162), (2500, 384), (7, 48)]:
        rng = np.random.default_rng(W)
        fw = rng.normal(size=(W, n3)) * rng.uniform(0.1, 3.0, size=n3)
        f = fw.mean(0)
        S = vmc.vmc_build_S_raw(ctx, torch.tensor(fw, device="cuda"), torch.tensor(f, device="cuda"))
        So = oracle.build_S(fw, f)
        assert rel(S.cpu().numpy(), So) < 1e-12
        assert np.array_equal(S.cpu().numpy(), S.cpu().numpy().T)


@pytest.mark.parametrize("n3,L,alpha,flags", [(48, 5.85, 0.0, 0), (162, 8.04, 1561.6, 0), (384, 10.9, 3.0, 2),
                                              (30, 0.0, 0.5, 1), (9, 0.0, 0.0, 4), (770, 13.9, 2.0, 0)])
def test_langevin_step(oracle, dev, n3, L, alpha, flags):
    torch, vmc, ctx = dev
    say(f"[langevin] n3={n3} L={L} alpha={alpha} flags={flags}")
    rng = np.random.default_rng(n3)
    A = rng.normal(size=(n3, n3)); S = A @ A.T / n3 + 0.5 * np.eye(n3)
    B = rng.normal(size=(n3, n3)); Sp = B @ B.T / n3 + 0.5 * np.eye(n3)
    R = rng.uniform(0, L if L > 0 else 3.0, n3); Rp = R + rng.normal(scale=0.05, size=n3)
    if L > 0:
        Rp = np.mod(Rp, L)
    f = rng.normal(size=n3)
    D = 1.0 / max(alpha, 1.0)
    T = 0.5 if flags & 2 else 3e-3          # the noise correction needs T > Dt^2 / (2 Db)
    Ro, Rpo, Spo = R.copy(), Rp.copy(), Sp.copy()
    rco = oracle.langevin(Ro, Rpo, Spo, f, S, T, D, alpha, flags=flags, seed=5, traj=2, step=9, L=L)
    td = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    Rg, Rpg, Spg = td(R), td(Rp), td(Sp)
    rcg = vmc.vmc_langevin_step(ctx, Rg, Rpg, Spg, td(f), td(S), T, D, alpha, flags, 5, 2, 9, L)
    assert rco == 0 and rcg == 0
    assert rel(Rg.cpu().numpy(), Ro) < 1e-12
    dg, do = Rg.cpu().numpy() - R, Ro - R           # the step itself, element by element
    if L > 0:
        dg, do = dg - L * np.round(dg / L), do - L * np.round(do / L)
    assert elem(dg, do) < 1e-11
    assert np.array_equal(Rpg.cpu().numpy(), Rpo) and np.array_equal(Spg.cpu().numpy(), Spo)


def test_langevin_negative_corrected_temperature(oracle, dev):
    """Both sides reject NOISE_CORR when T < Dt^2/(2 Db) and leave the state alone."""
    torch, vmc, ctx = dev
    n3 = 6
    td = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    R = np.linspace(0, 1, n3); Rp = R.copy(); S = np.eye(n3); f = np.ones(n3)
    rco = oracle.langevin(R.copy(), Rp.copy(), S.copy(), f, S, 1e-3, 1.0 / 3, 3.0, flags=2)
    Rg = td(R)
    rcg = vmc.vmc_langevin_step(ctx, Rg, td(Rp), td(S), td(f), td(S), 1e-3, 1.0 / 3, 3.0, 2)
    assert rco == -1 and rcg == vmc.VMC_EINVAL
    assert np.array_equal(Rg.cpu().numpy(), R)


def test_langevin_not_spd_leaves_state(dev):
    torch, vmc, ctx = dev
    say("[langevin] non-SPD S")
    n3 = 12
    S = np.eye(n3); S[4, 4] = -1.0
    td = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    R = td(np.arange(n3, dtype=float)); Rp = td(np.arange(n3, dtype=float) + 0.5); Sp = td(np.eye(n3))
    R0, Rp0, Sp0 = R.clone(), Rp.clone(), Sp.clone()
    rc = vmc.vmc_langevin_step(ctx, R, Rp, Sp, td(np.zeros(n3)), td(S), 0.1, 0.1, 0.0)
    assert rc == vmc.VMC_ENOTSPD
    assert torch.equal(R, R0) and torch.equal(Rp, Rp0) and torch.equal(Sp, Sp0)
    assert vmc.vmc_langevin_step(ctx, R, Rp, Sp, td(np.zeros(n3)), td(np.eye(n3)), 0.1, -1.0, 0.0) == vmc.VMC_EINVAL
