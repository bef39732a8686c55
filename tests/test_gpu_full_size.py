"""The HIP path at the full sizes of the hydrogen workloads, in the launch configuration the
benchmark times (one trajectory of W walkers, every walker in one launch per sweep), through the
C ABI.  The oracle cannot run thousands of N = 128 walkers, so:

* sampled walkers (the first, one in the middle, the last) are run by the oracle one by one on
  their own Philox streams (walker index = the walker's place in the full set): identical
  acceptance counts, per-walker means e_w, d_w, g_w, h_w at 1e-10 in FP64 and within the
  mixed-precision bars (ln|psi| 1e-6, E_L 5e-5, dln|psi|/dR 2e-5, dE_L/dR 2e-5) in mixed precision;
* the reductions over all W walkers are recomputed from the GPU's own per-walker means (E,
  sigma_E, f_w, f by the oracle's estimator; S as (F - f)^T (F - f) / (W (W - 1)) by a numpy
  product; the acceptance from the counts), at 1e-10 whatever the precision, since every
  reduction is FP64;
* the Langevin step on the GPU's f and S (3N = 384 and 768) against the oracle's at 1e-12."""
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
TOLMIX = {"e_w": 5e-5, "d_w": 2e-5, "g_w": 2e-5, "h_w": 5e-5}


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


# (workload, walkers, precision (0 FP64, 1 mixed), unmeasured sweeps, measured sweeps, sampled walkers)
CASES = [("h16", 128, 0, 2, 3, (0, 63, 127)),
         ("h54", 4096, 0, 1, 2, (0, 2049, 4095)),
         ("h128", 16384, 1, 1, 2, (0, 8191, 16383)),
         ("h128", 16384, 0, 1, 1, (5, 16382)),
         ("h256", 32768, 1, 1, 1, (0, 32767))]


@pytest.mark.parametrize("name,W,precision,ne,ns,sampled", CASES)
def test_full_size_step(oracle, dev, name, W, precision, ne, ns, sampled):
    torch, vmc, ctx = dev
    wl = workload(name)
    N, n3 = wl.n, 3 * wl.n
    say(f"[full size] {name} W={W} precision={precision} sweeps={ne}+{ns} sampled={sampled}")
    Cm, _ = oracle.huckel(wl.R, wl.zeta, wl.L, N // 2)
    x0 = wl.electrons(W=W, seed_offset=17)
    tr = vmc.Trajectory(ctx, vmc.make_system(N, wl.L, precision=precision), W, seed=wl.seed, traj_id=4)
    tr.set_walkers(T(torch, x0))
    out = tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), ne, ns, wl.delta, 6)
    S = tr.build_S()
    out_h, S_h = out.cpu().numpy(), S.cpu().numpy()
    means = tr.walker_means().cpu().numpy()
    fw = tr.walker_forces().cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    pos = tr.get_walkers().cpu().numpy()
    tr.close()
    assert np.all(np.isfinite(out_h)) and np.all(np.isfinite(S_h))

    # sampled walkers, each on its own stream
    s = oracle.System(wl.R, wl.zeta, Cm, L=wl.L)
    parts = {"e_w": slice(0, 1), "d_w": slice(1, 1 + n3), "g_w": slice(1 + n3, 1 + 2 * n3),
             "h_w": slice(1 + 2 * n3, 1 + 3 * n3)}
    for w in sampled:
        xo = np.ascontiguousarray(x0[w:w + 1])
        sums, nacc = s.vmc_run(xo, ne, ns, wl.delta, seed=wl.seed, traj=4, step=6, walker0=w)
        mo = oracle.reduce(sums, ns)["means"][0]
        errs = {q: rel(means[w, sl], mo[sl]) for q, sl in parts.items()}
        say(f"  walker {w}: accepted gpu/oracle {acc[w]}/{nacc[0]}  ",
            {q: f"{v:.2e}" for q, v in errs.items()})
        assert acc[w] == nacc[0]
        if precision == 0:
            assert rel(pos[w], xo[0]) < 1e-12
            for q, v in errs.items():
                assert v < TOL64, (w, q, v)
        else:
            for q, v in errs.items():
                assert v < TOLMIX[q], (w, q, v)

    # every reduction over the W walkers, from the GPU's per-walker means
    M = ns
    sums_all = np.zeros((W, 2 + 3 * n3))
    sums_all[:, 0] = means[:, 0] * M
    sums_all[:, 2:] = means[:, 1:] * M
    red = oracle.reduce(sums_all, M)
    F = fw - red["f"]
    S_ref = F.T @ F / (W * (W - 1.0))
    acc_rate = acc.sum() / (W * (ne + ns) * N)
    errs = {"E": rel(out_h[0], red["E"]), "sigma_E": rel(out_h[1], red["sigma_E"]),
            "acceptance": rel(out_h[2], acc_rate), "f_w": rel(fw, red["f_w"]), "f": rel(out_h[3:], red["f"]),
            "S": rel(S_h, S_ref)}
    say("  reductions over all walkers", {q: f"{v:.2e}" for q, v in errs.items()})
    for q, v in errs.items():
        assert v < TOL64, (q, v)
    assert np.array_equal(S_h, S_h.T)
    assert 0.2 < acc_rate < 0.95

    # the Langevin step on this f and S (alpha Delta = 1, N_c = W M samples)
    if W > n3:
        alpha = 0.122 * W * M
        D = 1.0 / alpha
        R = wl.R.reshape(-1).copy()
        Ro, Rpo, Spo = R.copy(), R.copy(), S_h.copy()
        rco = oracle.langevin(Ro, Rpo, Spo, out_h[3:].copy(), S_h, wl.T_hartree, D, alpha, flags=0, seed=wl.seed,
                              traj=4, step=6, L=wl.L)
        Rg, Rpg, Spg = T(torch, R), T(torch, R), T(torch, S_h)
        rcg = vmc.vmc_langevin_step(ctx, Rg, Rpg, Spg, T(torch, out_h[3:]), T(torch, S_h), wl.T_hartree, D, alpha, 0,
                                    wl.seed, 4, 6, wl.L)
        assert rco == 0 and rcg == 0
        dR = rel(Rg.cpu().numpy(), Ro)
        say(f"  Langevin step 3N={n3}: R against the oracle {dR:.2e}")
        assert dR < 1e-12
        assert np.array_equal(Rpg.cpu().numpy(), Rpo) and np.array_equal(Spg.cpu().numpy(), Spo)


@pytest.mark.parametrize("name,K,precision,twist", [("h128", 16384, 0, 0), ("h128", 16384, 1, 0), ("h128", 16384, 0, 5),
                                                     ("h256", 32768, 1, 0), ("h256", 32768, 0, 3)])
def test_full_size_symmetries(oracle, dev, name, K, precision, twist):
    """Symmetries of psi on the GPU over all configurations of a full-size batch (16,384 at N = 128,
    32,768 at N = 256) in one launch: a
    translation of every particle with re-wrapping into the box (orbital rows carried along), an exchange
    of two same-spin electrons in every configuration, and a relabelling of the protons (with their
    exponents and orbital rows) leave ln|psi| and E_L unchanged and permute the proton derivatives.
    Per configuration: the 99th percentile within 1e-10 in FP64 (median below 1e-12) and within the
    mixed-precision bars in mixed.  The maximum is held to 1e-7 (FP64) and 5e-2 (mixed).  The tail
    comes from a few unequilibrated configurations.  Some have ill-conditioned Slater matrices, where
    FP64 rounding fixes E_L only to about 1e-9 (the oracle's own translation discrepancy there is the
    same size) and the proton derivatives to about 1e-8.  Others have E_L near zero against
    |V| ~ 400 Ha, where FP32 rounding of V is a large relative error in E_L."""
    torch, vmc, ctx = dev
    wl = workload(name)
    N = wl.n
    say(f"[full size symmetries] {name} K={K} precision={precision} twist={twist}")
    sysd = vmc.make_system(N, wl.L, precision=precision, twist=twist)
    pos = wl.electrons(W=K, seed_offset=23)

    def run(R, zeta, p, C=None):
        if C is None:
            C, _ = oracle.huckel(R, zeta, wl.L, N // 2, twist=twist)
        g = vmc.vmc_eval_configs(ctx, sysd, T(torch, R.reshape(-1)), T(torch, C), T(torch, zeta), T(torch, p))
        return g.cpu().numpy(), C

    g0, C0 = run(wl.R, wl.zeta, pos)
    tol = ({"lnpsi": 1e-10, "EL": 1e-10, "dlnpsi": 1e-10, "dEL": 1e-10} if precision == 0 else
           {"lnpsi": 1e-6, "EL": 5e-5, "dlnpsi": 2e-5, "dEL": 2e-5})
    tail = 1e-7 if precision == 0 else 5e-2      # worst measured: 1.2e-8 (FP64), 1.1e-2 (mixed, N = 256)

    def per_config(a, b):
        a, b = a.reshape(K, -1), b.reshape(K, -1)
        return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)

    def check(g, label, perm=None):
        d0 = g0[:, 2:].reshape(K, 2, N, 3)
        if perm is not None:
            d0 = d0[:, :, perm, :]
        d = g[:, 2:].reshape(K, 2, N, 3)
        errs = {"lnpsi": per_config(g[:, 0], g0[:, 0]), "EL": per_config(g[:, 1], g0[:, 1]),
                "dlnpsi": per_config(d[:, 0], d0[:, 0]), "dEL": per_config(d[:, 1], d0[:, 1])}
        say(f"  {label}: per-configuration relative error median / 99th percentile / max",
            {q: f"{np.median(v):.1e} / {np.quantile(v, 0.99):.1e} / {v.max():.1e}" for q, v in errs.items()})
        for q, v in errs.items():
            assert np.quantile(v, 0.99) < tol[q], (label, q)
            assert v.max() < tail, (label, q)
            if precision == 0:
                assert np.median(v) < 1e-12, (label, q)

    # the moved protons' orbitals exactly: wrapping proton a by k_am box lengths along axis m
    # multiplies its basis function by prod_m tau_m^k_am (tau_m = -1 on a twisted axis), which its
    # row of C takes over (a fresh Hueckel solve would add the eigensolver's rounding)
    c = np.array([0.37, -0.81, 0.55]) * wl.L
    k = np.floor((wl.R + c) / wl.L).astype(np.int64)
    R2, pos2 = wl.R + c - wl.L * k, np.mod(pos + c, wl.L)
    tw_bits = np.array([(twist >> m) & 1 for m in range(3)])
    D = (-1.0) ** ((k * tw_bits).sum(axis=1) % 2)
    check(run(R2, wl.zeta, pos2, np.ascontiguousarray(D[:, None] * C0))[0], "translation")
    px = pos.copy()
    for i, j in ((3, N // 2 - 24), (N // 2 + 6, N - 1)):      # one pair of each spin
        px[:, [i, j]] = px[:, [j, i]]
    check(run(wl.R, wl.zeta, px, C0)[0], "same-spin exchanges")
    perm = np.random.default_rng(8).permutation(N)
    check(run(np.ascontiguousarray(wl.R[perm]), np.ascontiguousarray(wl.zeta[perm]), pos,
              np.ascontiguousarray(C0[perm]))[0], "proton relabelling", perm)
