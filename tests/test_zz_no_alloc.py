"""The allocation-free Langevin step (vmc_langevin_step_noalloc, the library's static device
scratch) against vmc_langevin_step through the C ABI: bit-identical state on two calls in a row,
the second with a smaller system (the shared scratch keeps the first call's contents), the
error paths, and the size limit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n3, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n3, n3))
    S = A @ A.T / n3 + 0.5 * np.eye(n3)
    B = rng.normal(size=(n3, n3))
    Sp = B @ B.T / n3 + 0.5 * np.eye(n3)
    L = 10.9
    R = rng.uniform(0, L, n3)
    Rp = np.mod(R + rng.normal(scale=0.05, size=n3), L)
    f = rng.normal(size=n3)
    return S, Sp, R, Rp, f, L


def test_noalloc_equals_langevin_step():
    import torch
    from paper_1605_08423_amd import vmc
    ctx = vmc.Context(0)
    td = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    # two calls in a row, the second smaller: 3N = 768 (256 protons), then 3N = 162 (54 protons)
    for n3, alpha, flags in [(768, 2.0, 0), (162, 1561.6, 0), (384, 3.0, vmc.VMC_STEP_NOISE_CORR)]:
        say(f"[noalloc] n3={n3} alpha={alpha} flags={flags}")
        S, Sp, R, Rp, f, L = _case(n3, n3)
        T = 0.5 if flags else 3e-3
        D = 1.0 / alpha
        outs = []
        for fn in (vmc.vmc_langevin_step, vmc.vmc_langevin_step_noalloc):
            Rg, Rpg, Spg = td(R), td(Rp), td(Sp)
            rc = fn(ctx, Rg, Rpg, Spg, td(f), td(S), T, D, alpha, flags, 5, 2, 9, L)
            assert rc == vmc.VMC_OK
            outs.append((Rg.cpu().numpy(), Rpg.cpu().numpy(), Spg.cpu().numpy()))
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        assert not np.array_equal(outs[0][0], R)
    # error paths leave the state unchanged, as in vmc_langevin_step
    n3 = 12
    bad = np.eye(n3)
    bad[4, 4] = -1.0
    R0 = np.arange(n3, dtype=float)
    Rg, Rpg, Spg = td(R0), td(R0 + 0.5), td(np.eye(n3))
    assert vmc.vmc_langevin_step_noalloc(ctx, Rg, Rpg, Spg, td(np.zeros(n3)), td(bad), 0.1, 0.1, 0.0) == \
        vmc.VMC_ENOTSPD
    f_nan = np.zeros(n3)
    f_nan[3] = np.nan
    assert vmc.vmc_langevin_step_noalloc(ctx, Rg, Rpg, Spg, td(f_nan), td(np.eye(n3)), 0.1, 0.1, 0.0) == \
        vmc.VMC_EINVAL
    assert np.array_equal(Rg.cpu().numpy(), R0) and np.array_equal(Spg.cpu().numpy(), np.eye(n3))
    # beyond the static scratch: refused
    big = 769
    z = torch.zeros(big, dtype=torch.float64, device="cuda")
    I = torch.eye(big, dtype=torch.float64, device="cuda")
    assert vmc.vmc_langevin_step_noalloc(ctx, z, z.clone(), I.clone(), z.clone(), I, 0.1, 0.1, 0.0) == \
        vmc.VMC_EINVAL
    ctx.close()
