"""Mixed precision (orbitals, Jastrow and Ewald real-space terms in FP32; ratios,
inverse refresh, contractions, reductions and accumulators in FP64) against the
FP64 oracle, through the C ABI.

Stated tolerances (relative, norm-wise).  FP32 rounding (2^-24 ~ 6e-8) of the
Gaussian, Jastrow and erfc values is amplified by sums over N centres / pairs and,
for E_L, by the cancellation of kinetic against potential energy (|T| ~ |V| ~ 3-4 |E_L|);
the MO rows are accumulated in FP64 so the Slater inverse does not amplify FP32 sums.
Measured worst cases over h16/h54/h128 configurations: ln|psi| 1.6e-7, E_L 1.5e-5,
dln|psi|/dR 2.0e-6, dE_L/dR 3.7e-6; same-seed chains: E 5e-8, f 1.4e-6, Langevin
displacement 1.1e-6.  Tolerances (about 3-5x above the measured values):
  per configuration: ln|psi| 1e-6, E_L 5e-5, dln|psi|/dR 2e-5, dE_L/dR 2e-5
  same-seed chain:   E 1e-6, f 1e-5, Langevin displacement 1e-5 (when no acceptance
                     decision flipped); independent seeds: E within 2 sigma.
"""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload

pytestmark = pytest.mark.gpu

TOL = {"lnpsi": 1e-6, "EL": 5e-5, "dlnpsi": 2e-5, "dEL": 2e-5}


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


@pytest.mark.parametrize("name,K", [("h16", 16), ("h54", 6), ("h128", 3)])
def test_eval_configs_mixed(oracle, dev, name, K):
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[eval_configs mixed] {name} K={K}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    pos = wl.electrons(W=K, seed_offset=5)
    sysd = vmc.make_system(wl.n, wl.L, precision=vmc.VMC_MIXED)
    g = vmc.vmc_eval_configs(ctx, sysd, T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta),
                             T(torch, pos)).cpu().numpy()
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    n3 = 3 * wl.n
    worst = dict.fromkeys(TOL, 0.0)
    for k in range(K):
        r = s.local(pos[k])
        worst["lnpsi"] = max(worst["lnpsi"], rel(g[k, 0], r["lnpsi"]))
        worst["EL"] = max(worst["EL"], rel(g[k, 1], r["EL"]))
        worst["dlnpsi"] = max(worst["dlnpsi"], rel(g[k, 2:2 + n3], r["dlnpsi"]))
        worst["dEL"] = max(worst["dEL"], rel(g[k, 2 + n3:], r["dEL"]))
    say("  worst relative errors (mixed vs FP64 oracle)", {k: f"{v:.2e}" for k, v in worst.items()})
    for q, v in worst.items():
        assert v < TOL[q], (q, v, TOL[q])


def _gpu_step(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, seed, precision):
    sysd = vmc.make_system(wl.n, wl.L, precision=precision)
    tr = vmc.Trajectory(ctx, sysd, W, seed=seed, traj_id=1)
    tr.set_walkers(T(torch, x0))
    R = T(torch, wl.R.reshape(-1))
    out = tr.energy_forces(R, T(torch, Cm), T(torch, wl.zeta), ne, ns, wl.delta, 0)
    S = tr.build_S()
    alpha = 0.122 * W * ns
    D = 1.0 / alpha
    Rn, Rp, Sp = R.clone(), R.clone(), S.clone()
    rc = vmc.vmc_langevin_step(ctx, Rn, Rp, Sp, out[3:], S, wl.T_hartree, D, alpha, 0, seed, 1, 0, wl.L)
    assert rc == 0
    res = dict(out=out.cpu().numpy(), acc=tr.accepts().cpu().numpy(), fw=tr.walker_forces().cpu().numpy(),
               dR=(Rn - R).cpu().numpy(), S=S.cpu().numpy())
    tr.close()
    return res


@pytest.mark.parametrize("name,W,ne,ns", [("h16", 64, 4, 8), ("h54", 256, 2, 3)])   # W > 3N: S full rank
def test_chain_mixed_same_seed(oracle, dev, name, W, ne, ns):
    """Mixed GPU chain vs FP64 oracle chain on the same Philox stream: report the error of
    E, f and the Langevin displacement of one step."""
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[chain mixed same seed] {name} W={W}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    x0 = wl.electrons(W=W, seed_offset=11)
    g = _gpu_step(torch, vmc, ctx, wl, Cm, x0, W, ne, ns, 21, vmc.VMC_MIXED)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    sums, nacc = s.vmc_run(x0.copy(), ne, ns, wl.delta, seed=21, traj=1, step=0)
    red = oracle.reduce(sums, ns)
    S = oracle.build_S(red["f_w"], red["f"])
    alpha = 0.122 * W * ns
    R = wl.R.reshape(-1).copy()
    Rn, Rp, Sp = R.copy(), R.copy(), S.copy()
    assert oracle.langevin(Rn, Rp, Sp, red["f"], S, wl.T_hartree, 1.0 / alpha, alpha, seed=21, traj=1, step=0,
                           L=wl.L) == 0
    dRo = Rn - R
    dRo -= wl.L * np.round(dRo / wl.L)
    dRg = g["dR"] - wl.L * np.round(g["dR"] / wl.L)
    flips = int(np.sum(g["acc"] != nacc))
    eE, ef, edR = rel(g["out"][0], red["E"]), rel(g["out"][3:], red["f"]), rel(dRg, dRo)
    say(f"  flipped-walkers={flips}  rel err: E {eE:.2e}  f {ef:.2e}  Langevin displacement {edR:.2e}")
    if flips == 0:
        assert eE < 1e-6 and ef < 1e-5 and edR < 1e-5
    else:
        sig = red["sigma_E"]
        assert abs(g["out"][0] - red["E"]) < 4 * sig


def test_energy_independent_seeds_within_2sigma(oracle, dev):
    """Different seeds: the mixed GPU estimate and the FP64 oracle estimate of E agree
    within 2 combined standard errors (walker means as independent bins)."""
    torch, vmc, ctx = dev
    wl = workload("h16")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, 8)
    W, ne, ns = 256, 20, 20
    g = _gpu_step(torch, vmc, ctx, wl, Cm, wl.electrons(W=W, seed_offset=31), W, ne, ns, 77, vmc.VMC_MIXED)
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    sums, _ = s.vmc_run(wl.electrons(W=W, seed_offset=32), ne, ns, wl.delta, seed=78, traj=0, step=0)
    red = oracle.reduce(sums, ns)
    comb = np.hypot(g["out"][1], red["sigma_E"])
    say(f"[independent seeds] E_gpu={g['out'][0]:.6f}+-{g['out'][1]:.6f}  E_oracle={red['E']:.6f}+-{red['sigma_E']:.6f}")
    assert abs(g["out"][0] - red["E"]) < 2 * comb
