"""The device's Philox4x32-10 words against the oracle's generator, which the published
known-answer vectors pin (tests/test_oracle_parts.py): the Langevin noise of a step with
S = I, f = 0 and 2 T Delta = 1 is the standard normal vector itself, and the proposals of a
sweep with a tiny move size are accepted and expose their uniforms."""
import math
import sys

import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_1605_08423_amd import vmc
    return torch, vmc, vmc.Context(0)


def T(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_langevin_noise_words(oracle, dev):
    torch, vmc, ctx = dev
    n3, seed, traj, step = 96, 0x243F6A88, 0x85A308D3, 7
    say("[rng] Langevin noise words")
    R = torch.zeros(n3, dtype=torch.float64, device="cuda")
    Rp, Sp = R.clone(), torch.eye(n3, dtype=torch.float64, device="cuda")
    f = torch.zeros(n3, dtype=torch.float64, device="cuda")
    # S = I, alpha = 0, Delta = 1, T = 1/2: R' = xi
    assert vmc.vmc_langevin_step(ctx, R, Rp, Sp, f, Sp.clone(), 0.5, 1.0, 0.0, vmc.VMC_STEP_CFOLD, seed, traj,
                                 step, 0.0) == 0
    xi = R.cpu().numpy()
    worst = 0.0
    for j in range(n3 // 2):
        a, b = xi[2 * j], xi[2 * j + 1]
        u1 = -math.expm1(-(a * a + b * b) / 2.0)
        u2 = (math.atan2(b, a) / (2.0 * math.pi)) % 1.0
        w = oracle.philox([step, 0xFFFFFFFF, j, 0], [seed, traj])
        r1, r2 = oracle.u01(w[0], w[1]), oracle.u01(w[2], w[3])
        d2 = min(abs(u2 - r2), 1.0 - abs(u2 - r2))
        worst = max(worst, abs(u1 - r1), d2)
    say(f"  worst |u - u_ref| = {worst:.2e}")
    assert worst < 1e-12


def test_move_proposal_words(oracle, dev):
    torch, vmc, ctx = dev
    wl = workload("h16")
    W, delta, seed, traj, step = 8, 1e-6, 0xA4093822, 3, 5
    say("[rng] move proposal words")
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L)
    x0 = wl.electrons(W=W, seed_offset=6)
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L), W, seed=seed, traj_id=traj)
    tr.set_walkers(T(torch, x0))
    tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), 0, 1, delta, step)
    x1 = tr.get_walkers().cpu().numpy()
    acc = tr.accepts().cpu().numpy()
    tr.close()
    d = x1 - x0
    d -= wl.L * np.round(d / wl.L)
    worst, moved = 0.0, 0
    for w in range(W):
        for e in range(wl.n):
            if not np.any(d[w, e]):
                continue                    # rejected (probability about delta)
            moved += 1
            o0 = oracle.philox([step, w, e, 0], [seed, traj])
            o1 = oracle.philox([step, w, e, 1], [seed, traj])
            u = np.array([oracle.u01(o0[0], o0[1]), oracle.u01(o0[2], o0[3]), oracle.u01(o1[0], o1[1])])
            worst = max(worst, float(np.max(np.abs(d[w, e] / delta + 0.5 - u))))
    say(f"  {moved} of {W * wl.n} moves accepted (counted {int(acc.sum())}); worst |u - u_ref| = {worst:.2e}")
    assert moved == int(acc.sum()) and moved >= W * wl.n - 2
    assert worst < 1e-7
