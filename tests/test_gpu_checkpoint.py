"""Checkpoint / resume of a trajectory through the C ABI: a trajectory saved after one Langevin
step and loaded into a fresh trajectory continues the run bit for bit; mismatched or damaged
checkpoints are refused and leave the target unchanged; a checkpoint restarts a trajectory at
another density with its walkers scaled by the ratio of the box sides."""
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


def _steps(torch, vmc, ctx, tr, wl, R, Rp, Sp, k0, k1, first, twist=0):
    """Langevin steps k0..k1-1 of trajectory tr (R, R_prev, S_prev updated in place)."""
    zeta = T(torch, wl.zeta)
    alpha = 0.122 * tr.W * 3
    outs = []
    for k in range(k0, k1):
        Cm = vmc.vmc_huckel_params(R.cpu().numpy(), wl.zeta, wl.L, twist=twist)
        out = tr.energy_forces(R, T(torch, Cm), zeta, 2 if k == 0 else 1, 3, wl.delta, k)
        S = tr.build_S()
        if first and k == k0:
            Sp.copy_(S)
            Rp.copy_(R)
        assert vmc.vmc_langevin_step(ctx, R, Rp, Sp, out[3:], S, wl.T_hartree, 1.0 / alpha, alpha, 0, 4, 9, k,
                                     wl.L) == 0
        outs.append(out.cpu().numpy())
    return outs


@pytest.mark.parametrize("name,W,precision,b1,twist", [("h16", 64, 0, 0.0, 0), ("h54", 176, 1, 2.5, 3)])
def test_resume_continues_bit_for_bit(dev, name, W, precision, b1, twist):
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[checkpoint] {name} W={W} precision={precision} b1={b1} twist={twist}")
    sysd = vmc.make_system(wl.n, wl.L, precision=precision, b1=b1, twist=twist)
    n3 = 3 * wl.n

    def fresh(seed):
        tr = vmc.Trajectory(ctx, sysd, W, seed=seed, traj_id=9)
        tr.set_walkers(T(torch, wl.electrons(W=W, seed_offset=3)))
        R = T(torch, wl.R.reshape(-1))
        return tr, R, R.clone(), torch.empty((n3, n3), dtype=torch.float64, device="cuda")

    # uninterrupted: three steps
    tr, R, Rp, Sp = fresh(21)
    ref = _steps(torch, vmc, ctx, tr, wl, R, Rp, Sp, 0, 3, True, twist)
    ref_pos = tr.get_walkers().cpu().numpy()
    ref_R = R.cpu().numpy()
    tr.close()
    # one step, checkpoint (with the caller's R, R_prev, S_prev), then resume in a new trajectory
    tr, R, Rp, Sp = fresh(21)
    first = _steps(torch, vmc, ctx, tr, wl, R, Rp, Sp, 0, 1, True, twist)
    blob = tr.save()
    saved = (R.cpu().numpy(), Rp.cpu().numpy(), Sp.cpu().numpy())
    tr.close()
    tr2, R2, Rp2, Sp2 = fresh(777)            # a different seed: the checkpoint's key replaces it
    tr2.set_walkers(T(torch, wl.electrons(W=W, seed_offset=8)))
    tr2.load(blob)
    R2.copy_(T(torch, saved[0])); Rp2.copy_(T(torch, saved[1])); Sp2.copy_(T(torch, saved[2]))
    rest = _steps(torch, vmc, ctx, tr2, wl, R2, Rp2, Sp2, 1, 3, False, twist)
    pos2 = tr2.get_walkers().cpu().numpy()
    tr2.close()
    for a, b in zip(ref, first + rest):
        assert np.array_equal(a, b)
    assert np.array_equal(ref_pos, pos2)
    assert np.array_equal(ref_R, R2.cpu().numpy())


def test_mismatched_or_damaged_checkpoint_refused(dev):
    torch, vmc, ctx = dev
    wl = workload("h16")
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L), 32, seed=1, traj_id=0)
    tr.set_walkers(T(torch, wl.electrons(W=32)))
    blob = tr.save()
    x_before = tr.get_walkers().cpu().numpy()
    for bad in (vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L), 40, seed=1, traj_id=0),
                vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, precision=1), 32, seed=1, traj_id=0),
                vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, twist=1), 32, seed=1, traj_id=0)):
        with pytest.raises(vmc.VMCError):
            bad.load(blob)
        bad.close()
    with pytest.raises(vmc.VMCError):
        tr.load(blob[:-8])
    damaged = bytearray(blob)
    damaged[0] ^= 0xFF
    with pytest.raises(vmc.VMCError):
        tr.load(bytes(damaged))
    assert np.array_equal(tr.get_walkers().cpu().numpy(), x_before)
    tr.close()


@pytest.mark.parametrize("precision,twist", [(0, 0), (1, 5)])
def test_restart_at_another_density(dev, precision, twist):
    """A checkpoint taken at r_s* = 1.32 restarts a trajectory at r_s = 1.40 (SI, systematic setup:
    configurations scaled by s = r_s / r_s*): the walkers arrive multiplied by s = L / L*, bit for
    bit; the old density's means are gone until the next call; the next step equals that of a
    fresh trajectory at the new density started from the scaled walkers with the checkpoint's key.
    A plain load into the new box and a rescaled load of another size are refused."""
    torch, vmc, ctx = dev
    wl = workload("h54")
    W = 64
    L1 = wl.L * (1.40 / 1.32)
    say(f"[rescaled restart] h54 W={W} precision={precision} twist={twist} L {wl.L:.4f} -> {L1:.4f}")
    tr = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, precision=precision, twist=twist), W, seed=31, traj_id=6)
    tr.set_walkers(T(torch, wl.electrons(W=W, seed_offset=12)))
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L, twist=twist)
    tr.energy_forces(T(torch, wl.R.reshape(-1)), T(torch, Cm), T(torch, wl.zeta), 2, 2, wl.delta, 0)
    blob = tr.save()
    x_saved = tr.get_walkers().cpu().numpy()
    tr.close()

    sys1 = vmc.make_system(wl.n, L1, precision=precision, twist=twist)
    s = L1 / wl.L
    R1 = wl.R * s
    C1 = vmc.vmc_huckel_params(R1, wl.zeta, L1, twist=twist)
    a = vmc.Trajectory(ctx, sys1, W, seed=5, traj_id=0)
    with pytest.raises(vmc.VMCError):
        a.load(blob)                                  # the box differs: only the rescaled load takes it
    a.load_rescaled(blob)
    assert np.array_equal(a.get_walkers().cpu().numpy(), x_saved * s)
    assert x_saved.max() * s < L1
    with pytest.raises(vmc.VMCError):
        a.walker_means()
    with pytest.raises(vmc.VMCError):
        a.build_S()
    out_a = a.energy_forces(T(torch, R1.reshape(-1)), T(torch, C1), T(torch, wl.zeta), 1, 2, wl.delta, 1).cpu().numpy()
    m_a = a.walker_means().cpu().numpy()
    a.close()
    b = vmc.Trajectory(ctx, sys1, W, seed=31, traj_id=6)
    b.set_walkers(T(torch, x_saved * s))
    out_b = b.energy_forces(T(torch, R1.reshape(-1)), T(torch, C1), T(torch, wl.zeta), 1, 2, wl.delta, 1).cpu().numpy()
    m_b = b.walker_means().cpu().numpy()
    b.close()
    assert np.array_equal(out_a, out_b) and np.array_equal(m_a, m_b)
    for bad in (vmc.Trajectory(ctx, sys1, W + 4, seed=5, traj_id=0),
                vmc.Trajectory(ctx, vmc.make_system(wl.n, L1, precision=1 - precision, twist=twist), W, seed=5, traj_id=0)):
        with pytest.raises(vmc.VMCError):
            bad.load_rescaled(blob)
        bad.close()


def _owned_steps(torch, vmc, tr, wl, n, twist=0, save_before_last_update=False):
    """n Langevin steps on the trajectory's own state (R, R_prev, S, S_prev and the step
    counter held by the trajectory; the caller computes only C at the trajectory's R).  With
    save_before_last_update the last step stops after vmc_build_S and returns a checkpoint."""
    zeta = T(torch, wl.zeta)
    alpha = 0.122 * tr.W * 3
    outs = []
    for j in range(n):
        Cm = vmc.vmc_huckel_params(tr.get_R().cpu().numpy(), wl.zeta, wl.L, twist=twist)
        out = tr.energy_forces(None, T(torch, Cm), zeta, 2 if tr.step_count() == 0 else 1, 3, wl.delta, step=None)
        tr.build_S(keep_only=True)
        outs.append(out.cpu().numpy())
        if save_before_last_update and j == n - 1:
            return outs, tr.save()
        assert tr.langevin_step(wl.T_hartree, 1.0 / alpha, alpha) == 0
    return outs, None


@pytest.mark.parametrize("name,W,precision,twist,mid", [("h16", 64, 0, 0, False), ("h54", 176, 1, 3, False),
                                                         ("h16", 64, 1, 0, True)])
def test_resume_with_trajectory_owned_langevin_state(dev, name, W, precision, twist, mid):
    """The trajectory owns R, R_prev, S, S_prev and the step counter (Eq. finaldyn_new needs
    R(t - Delta) and S(R(t - Delta))): a checkpoint taken after the first step (or, with mid,
    between vmc_build_S and the update of the second step) and loaded into a fresh trajectory
    with another seed, other walkers and another R continues R, E and the walkers bit for bit
    with no state held by the caller."""
    torch, vmc, ctx = dev
    wl = workload(name)
    say(f"[owned Langevin state] {name} W={W} precision={precision} twist={twist} mid={mid}")
    sysd = vmc.make_system(wl.n, wl.L, precision=precision, twist=twist)

    def fresh(seed, off):
        tr = vmc.Trajectory(ctx, sysd, W, seed=seed, traj_id=9)
        tr.set_walkers(T(torch, wl.electrons(W=W, seed_offset=off)))
        tr.set_R(T(torch, (wl.R if off == 3 else wl.R[::-1]).reshape(-1)))
        return tr

    tr = fresh(21, 3)
    ref, _ = _owned_steps(torch, vmc, tr, wl, 3, twist)
    ref_R, ref_pos, ref_k = tr.get_R().cpu().numpy(), tr.get_walkers().cpu().numpy(), tr.step_count()
    tr.close()
    assert ref_k == 3
    tr = fresh(21, 3)
    if mid:
        first, blob = _owned_steps(torch, vmc, tr, wl, 2, twist, save_before_last_update=True)
    else:
        first, _ = _owned_steps(torch, vmc, tr, wl, 1, twist)
        blob = tr.save()
    tr.close()
    tr2 = fresh(777, 8)
    tr2.load(blob)
    alpha = 0.122 * W * 3
    if mid:
        assert tr2.langevin_step(wl.T_hartree, 1.0 / alpha, alpha) == 0
    rest, _ = _owned_steps(torch, vmc, tr2, wl, 1 if mid else 2, twist)
    assert tr2.step_count() == 3
    assert all(np.array_equal(a, b) for a, b in zip(ref, first + rest))
    assert np.array_equal(tr2.get_R().cpu().numpy(), ref_R)
    assert np.array_equal(tr2.get_walkers().cpu().numpy(), ref_pos)
    tr2.close()


def test_damaged_payload_refused(dev):
    """A checkpoint with one flipped bit inside the walker block, the means block or the
    Langevin state is refused (checksum) and leaves the target as it was."""
    torch, vmc, ctx = dev
    wl = workload("h16")
    W = 32
    sysd = vmc.make_system(wl.n, wl.L)
    tr = vmc.Trajectory(ctx, sysd, W, seed=1, traj_id=0)
    tr.set_walkers(T(torch, wl.electrons(W=W)))
    tr.set_R(T(torch, wl.R.reshape(-1)))
    Cm = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L)
    tr.energy_forces(None, T(torch, Cm), T(torch, wl.zeta), 1, 2, wl.delta, step=None)
    blob = tr.save()
    tgt = vmc.Trajectory(ctx, sysd, W, seed=2, traj_id=0)
    tgt.set_walkers(T(torch, wl.electrons(W=W, seed_offset=5)))
    x_before = tgt.get_walkers().cpu().numpy()
    n3 = 3 * wl.n
    payload = 8 * (W * wl.n * 3 + W * (1 + 9 * wl.n) + W * n3 + 3 + n3 + 2 * n3 + 2 * n3 * n3) + 8 * W
    hdr = len(blob) - payload
    for off in (hdr + 100, hdr + 8 * W * wl.n * 3 + 100, len(blob) - 8 * W - 1000):
        damaged = bytearray(blob)
        damaged[off] ^= 0x10
        with pytest.raises(vmc.VMCError) as e:
            tgt.load(bytes(damaged))
        assert e.value.code == vmc.VMC_EINVAL
    assert np.array_equal(tgt.get_walkers().cpu().numpy(), x_before)
    with pytest.raises(vmc.VMCError):
        tgt.get_R()                       # never set: the refused loads left no R behind
    tgt.load(blob)
    assert np.array_equal(tgt.get_R().cpu().numpy(), wl.R.reshape(-1))
    tgt.close()
    tr.close()


def test_optimised_jastrow_resumes_from_a_checkpoint(dev):
    """A trajectory whose Jastrow parameters were changed (as an SR loop does) is saved; a fresh
    trajectory created with the original parameters takes b, b_1 and F from the checkpoint and
    continues the run bit for bit.  A checkpoint of another basis, eta, twist angle or without
    the three-body memory is refused."""
    torch, vmc, ctx = dev
    from oracle import oracle as O
    wl = workload("h16")
    F3 = (-0.3, 0.1, 0.05)
    Cm = T(torch, O.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)[0])
    R, z = T(torch, wl.R.reshape(-1)), T(torch, wl.zeta)
    sysd = vmc.make_system(wl.n, wl.L, b1=2.5, j3=F3)
    new = (0.8, 2.2, (-0.2, 0.02, 0.06))

    def run(tr, k):
        return tr.energy_forces(R, Cm, z, 1, 2, wl.delta, k).cpu().numpy()

    tr = vmc.Trajectory(ctx, sysd, 32, seed=5, traj_id=2)
    tr.set_walkers(T(torch, wl.electrons(W=32)))
    tr.set_jastrow(*new)
    run(tr, 0)
    blob = tr.save()
    ref = run(tr, 1)
    tr.close()
    tr2 = vmc.Trajectory(ctx, sysd, 32, seed=99, traj_id=0)
    tr2.load(blob)
    assert np.array_equal(run(tr2, 1), ref)
    tr2.close()
    bad = [vmc.make_system(wl.n, wl.L, b1=2.5),                                    # no three-body memory
           vmc.make_system(wl.n, wl.L, j3=F3),                                     # no one-body term
           vmc.make_system(wl.n, wl.L, b1=2.5, j3=F3, theta=None, twist=2)]
    for sd in bad:
        t = vmc.Trajectory(ctx, sd, 32)
        with pytest.raises(vmc.VMCError):
            t.load(blob)
        t.close()
    wc = workload("h54")
    eta_blob = None
    for eta in (0.1, 0.2):
        t = vmc.Trajectory(ctx, vmc.make_system(wc.n, wc.L, eta=eta), 8, seed=1)
        if eta_blob is None:
            eta_blob = t.save()
        else:
            with pytest.raises(vmc.VMCError):
                t.load(eta_blob)
        t.close()
    th_blob = None
    for th in ((0.1, 0.2, 0.3), (0.1, 0.2, 0.4)):
        t = vmc.Trajectory(ctx, vmc.make_system(wl.n, wl.L, theta=th), 8, seed=1)
        if th_blob is None:
            th_blob = t.save()
        else:
            with pytest.raises(vmc.VMCError):
                t.load(th_blob)
        t.close()
