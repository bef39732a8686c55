"""Benchmark: VMC walker-sweeps/s with forces at N = 128 H (mixed precision), one
MI355X.  A step is one full pass of the hot path: Hueckel orbitals and proton
Ewald tables at R, the VMC energy/force estimate (5 re-equilibration + M measured
sweeps on every walker), S = Cov of the mean force, and the Langevin update.

Prints ONE JSON line (see the keys below).  Inputs are synthetic and seeded and
already resident on the device when the timed region starts."""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VMC walker-sweeps/s with forces at N=128 H; Langevin steps/s, p99 latency"
# MI355X published peaks per execution unit, TFLOP/s: FP64 (vector and matrix cores alike), FP32
# matrix cores, FP32 vector.  The kernels issue FP32 vector arithmetic unpacked (one FMA per lane
# per cycle, 78.6 TFLOP/s), so FP32 vector work can reach at most half of its published peak.
PEAK = {"f64": 78.6, "f32_mfma": 157.3, "f32": 157.3}


def _add(d: dict, unit: str, flops: float) -> dict:
    d[unit] = d.get(unit, 0.0) + flops
    return d


def work_model(cls: str, N: int, nk: int, nslot: int, nimg: int, mixed: bool, one_body: bool = False,
               acc: float = 0.57, contracted: bool = False, three_body: bool = False) -> dict:
    """Algorithmic work of the method in one walker's share of a launch, by the unit it runs on:
    {unit: flops} (FMA = 2 flops; exp, erfc, sqrt, rcp, sincos count 1).  img: Gaussian images
    evaluated per axis (3, or 1 when the dropped ones are below FP32 resolution); acc: the
    acceptance rate (a rejected move costs no inverse update); one_body: the electron-proton
    Jastrow term; contracted: the orbital phi_1 + eta phi_2 (two exps per image and axis and four
    products of Cartesian factors instead of one); three_body: the on-site electron-electron-nucleus
    Jastrow term.  In mixed precision the basis, Jastrow and Ewald real-space terms are FP32."""
    NS = N // 2
    img = 3 if nimg else 1
    lo = "f32" if mixed else "f64"
    if cls == "slater_sample":
        gemm = 2 * N * NS * NS                                   # one of B = C A^-1, M = X B, W = B M, one spin
        pair1 = 3 * (3 + 9 * img) + 29 + 8 + 32                  # Gaussian with 3 derivatives, products, X, sums
        pair2 = 3 * (3 + 5 * img) + 12                           # Gaussian gradient, W term
        if contracted:
            pair1 = 3 * (3 + 27 * img) + 4 * 45 + 8 + 32         # g1, g2, h2 with 3 derivatives; four products
            pair2 = 3 * (3 + 13 * img) + 4 * 6 + 6
        valu = N * N * (pair1 + pair2) + N * (N - 1) * 45        # both spins' (electron, centre) pairs; Jastrow
        if one_body:
            # per (electron, proton) pair: its Jastrow gradient and Laplacian (30), grad ln|D| from
            # the Gaussian gradient (3 (3 + 5 img) + 8) and the d/dR terms (80)
            valu += N * N * (30 + 3 * (3 + 5 * img) + 8 + 80)
        w = {"f64": 2 * gemm}                                    # B = C A^-1 for both spins
        _add(w, "f32_mfma" if mixed else "f64", 4 * gemm)        # M = X B, W = B M
        return _add(w, lo, valu)
    if cls == "sweep_half":
        # one move: the proposal's basis values (per centre and axis an offset, its square and an
        # exp per image; the product), its Jastrow change (old and new pair terms, 15 flops each),
        # the MO row m = phi C (2 N NS), the ratio q = m . (A^-1 column) (2 NS) and, if accepted,
        # the Sherman-Morrison update (m^T A^-1 and the rank-1 update, 4 NS^2)
        basis = N * (3 * (3 + 2 * img) + 2) if not contracted else N * (3 * (3 + 8 * img) + 14)
        jas = 30 * (N - 1) + (30 * N if one_body else 0) + (J3_MOVE * N if three_body else 0)
        w = {"f64": NS * (2 * N * NS + 2 * NS + acc * 4 * NS * NS)}
        return _add(w, lo, NS * (basis + jas))
    if cls == "ewald_sample":
        recip = nk * N * 8 + nslot * N * 6
        real = (N * (N - 1) // 2) * 30 + N * N * 40
        return _add({"f64": recip}, lo, real)
    if cls == "refine":
        return {"f64": 4 * NS ** 3}
    if cls == "csweep":
        # general twist, complex FP64 (a complex multiply-add is 8 flops).  One move: the proposal's
        # Bloch-summed basis values (per centre 3 axes x 3 images of an exp and its twist phase, and
        # the complex product, 93), the orbital row (8 N NS), the ratio (8 NS), the Jastrow change and,
        # if accepted, the Sherman-Morrison row product and update (16 NS^2).  Every CREFRESH-th
        # half-sweep also forms its Slater matrix (NS N 93 + 8 NS N NS) and inverts it (8 NS^3).
        move = N * 93 + 8 * N * NS + 8 * NS + 30 * (N - 1) + acc * 16 * NS * NS
        refresh = NS * N * 93 + 8 * NS * N * NS + 8 * NS ** 3
        return {"f64": NS * move + refresh / CREFRESH}
    if cls == "opt_sample":
        # per sample: the two-body derivative over the N(N-1)/2 electron pairs (periodised
        # distance 18, sqrt, the Pade derivative 6), the one-body derivative over the N^2
        # electron-proton pairs (distance 18, exp, 6), the three-body sums per proton (distance 15,
        # exp, 8) in the working precision of the Jastrow terms, and the 64 moments of the seven
        # parameters in FP64
        return _add({"f64": 128}, lo, N * (N - 1) // 2 * 25 + (N * N * 25 if one_body else 0) + N * N * 24)
    if cls == "j3_init":
        # G_a = sum_i chi_a(r_i) of every nucleus: per (electron, nucleus) pair the squared
        # periodised distance (15), an exp and two sums
        return {"f64": N * N * 19}
    if cls == "j3_grad":
        # G_a and sum_i chi_ai^T F chi_ai (N^2 x 26); per (electron, nucleus) pair the orbitals'
        # value, gradient and Laplacian (J3_VGL) and four F-forms with G_a - chi (28); in the working
        # precision of the Jastrow terms
        return {lo: N * N * (26 + J3_VGL + 28)}
    if cls == "j3_forces":
        # per (electron, nucleus) pair the orbitals with their Hessian and gradient of the Laplacian
        # (J3_FULL), then G_a, G_a,mu, the two velocity contractions per axis and the self terms (150)
        return {lo: N * N * (J3_FULL + 150)}
    if cls == "cslater_sample":
        # B = C A^-1, M = X B, W = B M per spin (complex, 8 N NS^2 each); the (electron, centre) passes
        # with the complex basis and its derivatives (295 + 110 flops); the Jastrow pass
        return {"f64": 2 * 3 * 8 * N * NS * NS + N * N * (295 + 110) + N * (N - 1) * 45}
    return {}


# the complex half-sweep forms and inverts its Slater matrix afresh every CREFRESH-th sweep
CREFRESH = 4
# F of the three-body leg: the lowest VMC energy of a scan at 54 protons with b_1 = 2.5
J3_LEG_F = (-0.2, 0.0, 0.05)
# f of the one-body term's orbital part in the paper-wavefunction leg: ten SR iterations on f at 54
# protons with b_1 = 2.5 and the F above (the energy is flat within 0.03 Ha between f = 0 and here)
J1F_LEG = (0.011, 0.053)


def _f3(text: str):
    """'f11,f12,f22' -> a 3-tuple of floats; 'none' -> None."""
    if text.strip().lower() == "none":
        return None
    v = tuple(float(x) for x in text.split(","))
    if len(v) != 3:
        raise argparse.ArgumentTypeError("three numbers f11,f12,f22")
    return v
# Three-body flops per (electron, nucleus) pair: a move's change (chi at the new and the old
# position, 2 x 20, and the F-form with G_a - chi, 10); the orbitals chi_1, chi_2 with value,
# gradient and Laplacian (per axis the sin-periodised offset and its polynomial factors, 3 x 30,
# the exp and the products, 60) and with every component up to the gradient of the Laplacian
# (3 x 42 and 4 products of 14 components, 250)
J3_MOVE, J3_VGL, J3_FULL = 50, 150, 376


def executed_model(cls: str, N: int, nk: int, nslot: int, nimg: int, mixed: bool, one_body: bool = False,
                   acc: float = 0.57, contracted: bool = False, three_body: bool = False) -> dict:
    """The arithmetic a launch executes, where it differs from the method's count: the sweep applies
    its Sherman-Morrison updates in blocks of 16 moves on the matrix cores, forming the full rows
    P = M' A^-1 of every proposal and a rank-16 update whatever the acceptance (2 NS N NS + 4 NS^3
    on the FP64 matrix cores per half-sweep; the SQ_INSTS_VALU_MFMA_MOPS_F64 counter gives it)."""
    if cls == "csweep":
        # the row product m A^-1 is formed for every proposal, accepted or not
        NS = N // 2
        w = work_model(cls, N, nk, nslot, nimg, mixed, one_body, acc)
        return {"f64": w["f64"] + NS * (1 - acc) * 8 * NS * NS}
    if cls != "sweep_half":
        return work_model(cls, N, nk, nslot, nimg, mixed, one_body, acc, contracted, three_body)
    NS = N // 2
    img = 3 if nimg else 1
    lo = "f32" if mixed else "f64"
    basis = N * (3 * (3 + 2 * img) + 2) if not contracted else N * (3 * (3 + 8 * img) + 14)
    per_move = basis + 30 * (N - 1) + (30 * N if one_body else 0) + (J3_MOVE * N if three_body else 0)
    w = {"f64": 2 * NS * N * NS + 4 * NS ** 3 + NS * 16 * NS}    # matrix cores; the recursion t -= t[i] z
    return _add(w, lo, NS * per_move)


def roofline_numbers(parts: dict, walkers: int, avg_s: float):
    """Achieved TFLOP/s of a launch and the peak it is measured against: the time-weighted
    combination of the unit peaks, sum(f) / sum(f_u / peak_u)."""
    total = sum(parts.values()) * walkers
    t_peak = sum(f * walkers / (PEAK[u] * 1e12) for u, f in parts.items())
    achieved = total / avg_s / 1e12 if avg_s > 0 else 0.0
    peak = total / t_peak / 1e12 if t_peak > 0 else PEAK["f64"]
    return total, achieved, peak


# the sources the real-orbital kernels of the measured workloads are built from (the complex,
# three-body and optimisation kernels live in files of their own)
REAL_PATH_SOURCES = ("k_walkers.hip", "k_measure.hip", "k_langevin.hip", "common.hpp", "kernels.hpp", "moves.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources of the real-orbital kernels, their launchers and headers; a committed
    traffic measurement applies only to this hash."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1605_08423_amd", "csrc")
    for f in REAL_PATH_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_workload_key(workload: str, precision: str, walkers: int, j1: float = 0.0, rs=None, j3=None) -> str:
    """Names the run a traffic measurement belongs to, as profiles/traffic.json records it."""
    key = f"{workload} {precision}, W={walkers}"
    if j1 > 0:
        key += f", b1={j1}"
    if j3 is not None:
        key += f", F3={','.join(f'{x:g}' for x in j3)}"
    if rs is not None:
        key += f", r_s={rs}"
    return key


def measured_traffic(kernel: str, workload_key: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy), if taken on these sources and on
    this workload (size, precision and wavefunction change every kernel's traffic)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("source_hash") != kernel_source_hash() or d.get("workload") != workload_key:
        return None
    return k["bytes_per_launch"]


def run_cpu_baseline(wl, Cm, walkers: int, sweeps: int, threads: int, b1: float = 0.0):
    from oracle import oracle as O
    s = O.System(wl.R, wl.zeta, Cm, L=wl.L, b1=b1)
    x = wl.electrons(W=walkers, seed_offset=99)
    t0 = time.perf_counter()
    s.vmc_run(x, 1, sweeps, wl.delta, seed=3, traj=0, step=0, threads=threads)
    dt = time.perf_counter() - t0
    return walkers * sweeps / dt, dt


# FP64 operations of one toy-model trajectory step (FMA = 2; sqrt, division, log and sincos
# count 1): metric and force 30, 2 x 2 Cholesky and solves 20, Box-Muller 8, S-difference
# term and update 22, U 6; Philox's integer rounds are not counted.
TOY_FLOP_PER_STEP = 86
# the series of the toy figure, and the main text's shifted Hessian: (label, s_kind, scheme, alpha, mu)
# (mu = None: the figure's mu; H + mu I takes mu = 1, which keeps it positive definite where
# the trajectories go)
TOY_SERIES = [("S=I, Eq. finaldyn", 2, 0, 0.0, None), ("S=G, Eq. finaldyn", 0, 0, 0.0, None),
              ("S=G, explicit Gamma", 0, 2, 0.0, None), ("S=G, Eq. finaldyn_new a=0.2", 0, 0, 0.2, None),
              ("S=H+mu G, Eq. finaldyn_new a=0.2", 1, 0, 0.2, None), ("S=G, Eq. norogna", 0, 1, 0.0, None),
              ("S=H+I, Eq. finaldyn_new a=0.2", 3, 0, 0.2, 1.0), ("S=G, two-S (Eq. smartMarkov)", 0, 3, 0.0, None)]
TOY_DELTAS = [0.05, 0.1, 0.2, 0.4, 0.7, 1.0]


def run_toy(args):
    """The toy figure as a GPU workload: every (series, Delta) point is an ensemble of
    independent trajectories; prints one JSON line with the trajectory-step rate and the
    figure's data (<U>/(T/2) - 1 with its standard error)."""
    import torch
    from paper_1605_08423_amd import vmc
    tm = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))["toy_model"]
    ctx = vmc.Context(0)
    n, steps = args.toy_traj, args.toy_steps
    rng = np.random.default_rng(7)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    R0 = torch.tensor(np.stack([tm["a"] * np.cos(th), tm["a"] * np.sin(th)], axis=1), dtype=torch.float64,
                      device="cuda")
    half_T = tm["T"] / 2
    run = lambda sk, sc, D, al, seed, mu=None: vmc.vmc_toy_run(ctx, R0, steps, tm["lambda_used"], tm["k"], tm["a"],
                                                                tm["mu"] if mu is None else mu, sk, tm["T"], D, al, sc,
                                                                seed)
    run(0, 0, 0.1, 0.2, 1)                     # warm-up
    torch.cuda.synchronize()
    ctx.reset_kernel_times()
    ctx.set_profiling(True)
    figure, unstable = {}, {}
    t0 = time.perf_counter()
    outs = []
    for label, sk, sc, al, mu in TOY_SERIES:
        for D in TOY_DELTAS:
            outs.append((label, D, run(sk, sc, D, al, 1000 + len(outs), mu)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = ctx.kernel_times()
    ctx.set_profiling(False)
    for label, D, (_, U, st) in outs:
        Uh, sth = U.cpu().numpy(), st.cpu().numpy()
        ok = (sth == 0) & np.isfinite(Uh) & (Uh < 1e3 * half_T)
        key = f"{D:g}"
        figure.setdefault(label, {})[key] = (
            [round(float(Uh[ok].mean() / half_T - 1.0), 5), round(float(Uh[ok].std() / np.sqrt(ok.sum()) / half_T), 5)]
            if ok.sum() > 1 else None)
        if (~ok).sum():
            unstable.setdefault(label, {})[key] = int((~ok).sum())
    n_points = len(outs)
    total_steps = n_points * n * steps
    ms, nl = times["toy"]
    avg_s = ms / max(nl, 1) / 1e3
    achieved = TOY_FLOP_PER_STEP * n * steps / avg_s / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        ncpu, t1 = 40000, time.perf_counter()       # about 10 s of one CPU thread
        for i in range(ncpu):
            O.toy_run(tm["lambda_used"], tm["k"], tm["a"], tm["mu"], 0, tm["T"], 0.2, 0.2, 0, 3, steps, traj=i)
        dt = time.perf_counter() - t1
        cpu = {"value": round(ncpu * steps / dt, 1), "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{ncpu} trajectories x {steps} steps (S=G, Eq. finaldyn_new), one thread, {dt:.1f} s"}
    line = {
        "metric": "toy-model Langevin trajectory-steps/s (rotating spring, SI)", "value": round(total_steps / wall, 1),
        "unit": "trajectory-steps/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"toy figure: {len(TOY_SERIES)} series x {len(TOY_DELTAS)} time steps, {n} independent "
                               f"trajectories x {steps} steps per point, T={tm['T']}, k={tm['k']}, a={tm['a']}, "
                               f"lambda={tm['lambda_used']}, mu={tm['mu']}"},
        "wall_s": round(wall, 3),
        "roofline": {"bound": "alu", "kernel": "toy", "achieved": round(achieved, 3), "peak": PEAK["f64"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64"], 4), "traffic": None,
                     "avg_launch_ms": round(avg_s * 1e3, 3), "flop_per_trajectory_step": TOY_FLOP_PER_STEP},
        "cpu_baseline": cpu,
        "figure_U_over_half_T_minus_1": figure, "unstable_trajectories": unstable,
    }
    print(json.dumps(line))


SERVE_WALKERS = {16: 1024, 32: 2048, 54: 4096, 128: 16384}


def serve_stream(n_req: int, steps: int, sweeps: int, rate: float, budget_gb: float, large: bool = False) -> dict:
    """Served stream: independent trajectories with N in {16, 32, 54, 128}, r_s ~ U[1.25, 1.50],
    T ~ U[600, 3000] K and walker counts scaling with N, all in mixed precision, arriving as a
    Poisson stream; continuous batching on one GPU (vmc_server_*).  large: one N = 256 box
    (r_s 1.36, 900 K, 32768 walkers) with eight N = 54 boxes instead."""
    import torch
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import KB_HA_PER_K, small_system, workload
    rng = np.random.default_rng(20240605)
    if large:
        n_req = 9
    ctx = vmc.Context(0)
    reqs, meta = [], []
    for i in range(n_req):
        if large:
            n = 256 if i == 0 else 54
            rs = 1.36 if i == 0 else float(rng.uniform(1.25, 1.50))
            T_k = 900.0 if i == 0 else float(rng.uniform(600.0, 3000.0))
            W = 32768 if i == 0 else SERVE_WALKERS[54]
        else:
            n = int(rng.choice([16, 32, 54, 128]))
            rs = float(rng.uniform(1.25, 1.50))
            T_k = float(rng.uniform(600.0, 3000.0))
            W = SERVE_WALKERS[n]
        wl = workload("h256") if (large and i == 0) else small_system(n, rs, seed=1000 + i)
        sysd = vmc.make_system(n, wl.L, precision=vmc.VMC_MIXED)
        alpha = 0.122 * W * sweeps
        reqs.append(vmc.make_request(sysd, W, wl.R, wl.zeta, wl.electrons(W=W, seed_offset=i), n_steps=steps,
                                     n_sweeps=sweeps, T=T_k * KB_HA_PER_K, Delta=1.0 / alpha, alpha=alpha,
                                     n_equil_first=5, n_equil=5, step_delta=rs, seed=77, traj_id=i))
        meta.append((n, W))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    srv = vmc.Server(ctx, int(budget_gb * 1e9))
    ids = [None] * n_req
    nxt = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while nxt < n_req and arrivals[nxt] <= now:
            ids[nxt] = srv.submit(reqs[nxt])
            nxt += 1
        a, q = srv.tick()
        if a == 0 and q == 0:
            if nxt == n_req:
                break
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat, waits, nsteps, wsweeps, failed = [], [], 0, 0, 0
    by_n = {}
    for i, rid in enumerate(ids):
        st, k, err = srv.status(rid)
        r = srv.result(rid)
        if st != vmc.VMC_REQ_DONE:
            failed += 1
        lat.extend(r["latency_ms"].tolist())
        waits.append(r["wait_ms"])
        nsteps += k
        n, W = meta[i]
        wsweeps += k * W * (sweeps + 5)
        by_n.setdefault(n, []).extend(r["latency_ms"].tolist())
    info = srv.info()
    srv.close()
    ctx.close()
    pct = lambda v, q: round(float(np.percentile(np.asarray(v), q)), 1) if len(v) else None
    return {
        "workload": (f"one N=256 box (r_s 1.36, 900 K, 32768 walkers) with eight N=54 boxes (r_s~U[1.25,1.50], "
                     f"T~U[600,3000] K, 4096 walkers), " if large else
                     f"{n_req} trajectories, N in {{16,32,54,128}}, r_s~U[1.25,1.50], T~U[600,3000] K, "
                     f"W = 1024/2048/4096/16384 by N, ") +
                    f"all mixed precision, {steps} Langevin steps x (5 + {sweeps}) sweeps each, Poisson arrivals at "
                    f"{rate}/s, HBM budget {budget_gb} GB",
        "langevin_steps_per_s": round(nsteps / wall, 3), "wall_s": round(wall, 3), "steps": nsteps, "failed": failed,
        "walker_sweeps_per_s": round(wsweeps / wall, 1),
        "step_latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "step_latency_ms_by_N": {str(n): {"p50": pct(v, 50), "p99": pct(v, 99), "steps": len(v)}
                                 for n, v in sorted(by_n.items())},
        "queue_wait_ms": {"p50": pct(waits, 50), "p99": pct(waits, 99)},
        "peak_resident_GB": round(info["peak_resident"] / 1e9, 2), "ticks": info["ticks"],
    }


def run_serve(args):
    """The served stream as its own benchmark line."""
    r = serve_stream(args.serve, args.serve_steps, args.serve_sweeps, args.serve_rate, args.serve_budget_gb,
                     large=args.serve_mix == "large")
    line = {"metric": "served stream: Langevin steps/s and step latency p50/p99", "value": r["langevin_steps_per_s"],
            "unit": "Langevin steps/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": "f32/f64", "config": {"workload": r["workload"]}}
    line.update({k: v for k, v in r.items() if k not in ("workload", "langevin_steps_per_s")})
    print(json.dumps(line))


def run_twists(args):
    """Twist-averaged Langevin steps: one trajectory per real twist (twist angle 0 or pi per
    axis, bitmasks 0..n-1), the walkers split evenly, each with the Hueckel orbitals of its
    twist; the step takes the twist average of the forces and of their covariance."""
    import torch
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload
    wl = workload(args.workload, rs=args.rs)
    N, M, n_tw = wl.n, args.sweeps, args.twists
    Wtot = args.walkers or wl.walkers
    W = Wtot // n_tw
    prec = vmc.VMC_MIXED if args.precision == "mixed" else vmc.VMC_FP64
    ctx = vmc.Context(0)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    trajs = []
    for tw in range(n_tw):
        tr = vmc.Trajectory(ctx, vmc.make_system(N, wl.L, precision=prec, b1=args.j1, twist=tw), W, seed=wl.seed,
                            traj_id=tw)
        tr.set_walkers(dev(wl.electrons(W=W, seed_offset=tw)))
        trajs.append(tr)
    R = dev(wl.R.reshape(-1))
    R_prev = R.clone()
    zeta = dev(wl.zeta)
    n3 = 3 * N
    S_prev = torch.empty((n3, n3), dtype=torch.float64, device="cuda")
    f_stack = torch.empty((n_tw, n3), dtype=torch.float64, device="cuda")
    S_stack = torch.empty((n_tw, n3, n3), dtype=torch.float64, device="cuda")
    alpha = 0.122 * W * n_tw * M
    Delta = 1.0 / alpha
    state = {"first": True}
    Es = []

    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=n_tw)   # the host Hueckel solves of the twists run side by side

    def one_step(k, n_equil):
        Rh = R.cpu().numpy()
        Cs = list(pool.map(lambda tw: vmc.vmc_huckel_params(Rh, wl.zeta, wl.L, twist=tw), range(n_tw)))
        E = 0.0
        for tw, tr in enumerate(trajs):
            out = tr.energy_forces(R, dev(Cs[tw]), zeta, n_equil, M, wl.delta, step=k)
            f_stack[tw].copy_(out[3:])
            tr.build_S(S_stack[tw])
            E += float(out[0]) / n_tw
        f, S = vmc.vmc_twist_average(ctx, f_stack, S_stack)
        if state["first"]:
            S_prev.copy_(S)
            R_prev.copy_(R)
            state["first"] = False
        rc = vmc.vmc_langevin_step(ctx, R, R_prev, S_prev, f, S, wl.T_hartree, Delta, alpha, 0, wl.seed, 0, k, wl.L)
        if rc != 0:
            raise RuntimeError(f"langevin step failed: {vmc._lib().vmc_strerror(rc).decode()}")
        Es.append(E)

    for k in range(args.warmup):
        one_step(k, 20 if k == 0 else 5)
    torch.cuda.synchronize()
    ctx.reset_kernel_times()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        one_step(k, 20 if k == 0 else 5)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = ctx.kernel_times()
    ctx.set_profiling(False)
    value = W * n_tw * M * args.steps / elapsed
    nm = 9
    kset = [(nx, ny, nz) for nx in range(0, nm + 1) for ny in range(-nm, nm + 1) for nz in range(-nm, nm + 1)
            if 0 < nx * nx + ny * ny + nz * nz <= nm * nm and (nx > 0 or (nx == 0 and (ny > 0 or (ny == 0 and nz > 0))))]
    nk, nslot = len(kset), len({(ny, nz) for _, ny, nz in kset})
    nimg = int(not (prec == vmc.VMC_MIXED and float(np.min(wl.zeta)) * (wl.L / 2) ** 2 >= 23.0))
    dom_name, (dom_ms, dom_n) = max(times.items(), key=lambda kv: kv[1][0])
    avg_s = dom_ms / max(dom_n, 1) / 1e3
    flops, achieved, peak = roofline_numbers(work_model(dom_name, N, nk, nslot, nimg, prec == vmc.VMC_MIXED,
                                                        args.j1 > 0), W, avg_s)
    for tr in trajs:
        tr.close()
    print(json.dumps({
        "metric": "twist-averaged VMC walker-sweeps/s with forces", "value": round(value, 1),
        "unit": "walker-sweeps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64" if prec == vmc.VMC_MIXED else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N} H, r_s={wl.rs}, {n_tw} real twists x {W} walkers x {M} "
                               f"measured sweeps per Langevin step, {args.precision} precision",
                   "N": N, "twists": n_tw, "walkers_per_twist": W, "sweeps": M, "precision": args.precision},
        "langevin_steps_per_s": round(args.steps / elapsed, 4), "E_Ha_twist_average": Es[-1],
        "roofline": {"bound": "alu", "kernel": dom_name, "achieved": round(achieved, 3), "peak": round(peak, 2),
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if peak else None, "traffic": None,
                     "avg_launch_ms": round(avg_s * 1e3, 4)},
        "kernel_ms": {k: round(v[0], 2) for k, v in times.items()},
    }))


def monkhorst_pack(q: int) -> np.ndarray:
    """Twist angles of the q x q x q Monkhorst-Pack mesh: theta_m = 2 pi (2 n - q - 1) / (2 q), n = 1..q."""
    t = [2.0 * math.pi * (2 * n - q - 1) / (2 * q) for n in range(1, q + 1)]
    return np.array([(a, b, c) for a in t for b in t for c in t])


def twist_mesh_leg(name: str, q: int, W: int, M: int, steps: int, warmup: int, wavefunction: str = "gaussian",
                   streams: int = 4) -> dict:
    """Twist-averaged Langevin steps over the q x q x q Monkhorst-Pack mesh of general twists (the
    paper's production setup is q = 4): one trajectory per twist with W walkers and the complex
    orbitals of its twist (FP64); a step solves the q^3 Hueckel problems on the host, runs every
    twist's estimate (5 re-equilibration + M measured sweeps; 20 at the first step), forms the
    twist averages of the forces and of their covariance and takes the Langevin step.
    wavefunction "gaussian": one s-Gaussian per proton and the two-body Jastrow; "paper": the
    contracted orbital phi_1 + eta phi_2 (eta = 0.1), the one-body term (b_1 = 2.5) and the
    three-body term (F of the three-body leg).
    The host solves the twists' Hueckel problems on a pool of threads while the GPU runs the
    twists whose orbitals are ready.  The twists are independent: with streams > 1 they run on
    that many HIP streams (one library context and one host thread each, twists dealt
    round-robin), so that the launches of different twists overlap on the GPU (a launch of one
    twist fills each CU with one work-group of 256 walkers); the averages are taken in twist
    order after all streams finish.  Kernel times are then summed over the streams, and a
    launch's duration includes the time it shares the GPU with other streams' launches."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload
    wl = workload(name)
    N, n3 = wl.n, 3 * wl.n
    mesh = monkhorst_pack(q)
    n_tw = len(mesh)
    ctx = vmc.Context(0)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    paper = wavefunction == "paper"
    wkw = dict(eta=0.1, b1=2.5, j3=J3_LEG_F, j1f=J1F_LEG) if paper else {}
    ns = max(1, min(streams, n_tw))
    strs = [torch.cuda.Stream() for _ in range(ns)] if ns > 1 else [torch.cuda.current_stream()]
    ctxs = []
    for st in strs:
        with torch.cuda.stream(st):
            ctxs.append(vmc.Context(0) if ns > 1 else ctx)
    trajs = []
    for k, th in enumerate(mesh):
        with torch.cuda.stream(strs[k % ns]):
            tr = vmc.Trajectory(ctxs[k % ns], vmc.make_system(N, wl.L, theta=th, **wkw), W, seed=wl.seed, traj_id=k)
            tr.set_walkers(dev(wl.electrons(W=W, seed_offset=k)))
        trajs.append(tr)
    torch.cuda.synchronize()
    R = dev(wl.R.reshape(-1))
    R_prev = R.clone()
    zeta = dev(wl.zeta)
    S_prev = torch.empty((n3, n3), dtype=torch.float64, device="cuda")
    f_stack = torch.empty((n_tw, n3), dtype=torch.float64, device="cuda")
    S_stack = torch.empty((n_tw, n3, n3), dtype=torch.float64, device="cuda")
    alpha = 0.122 * W * n_tw * M
    Delta = 1.0 / alpha
    pool = ThreadPoolExecutor(max_workers=16)
    sgroups = ThreadPoolExecutor(max_workers=ns)
    state = {"first": True, "E": None, "acc": 0.0}

    def one_step(k):
        Rh = R.cpu().numpy()
        # the host Hueckel solves, in twist order on the pool; a twist's estimate starts as soon as
        # its orbitals are ready, so the GPU works while the later twists are solved
        if paper:
            Cs = [pool.submit(vmc.vmc_huckel_params_theta_contracted, Rh, wl.L, th, 0.1) for th in mesh]
        else:
            Cs = [pool.submit(vmc.vmc_huckel_params_theta, Rh, wl.zeta, wl.L, th) for th in mesh]
        Ej, accj = [0.0] * n_tw, [0.0] * n_tw

        def group(c):
            with torch.cuda.stream(strs[c]):
                for j in range(c, n_tw, ns):
                    Cj = np.ascontiguousarray(Cs[j].result()).view(np.float64)
                    out = trajs[j].energy_forces(R, dev(Cj), zeta, 20 if k == 0 else 5, M, wl.delta, step=k)
                    f_stack[j].copy_(out[3:])
                    trajs[j].build_S(S_stack[j])
                    Ej[j], accj[j] = float(out[0]), float(out[2])

        list(sgroups.map(group, range(ns)))
        torch.cuda.synchronize()
        E = sum(e / n_tw for e in Ej)
        acc = sum(x / n_tw for x in accj)
        f, S = vmc.vmc_twist_average(ctx, f_stack, S_stack)
        if state["first"]:
            S_prev.copy_(S)
            R_prev.copy_(R)
            state["first"] = False
        rc = vmc.vmc_langevin_step(ctx, R, R_prev, S_prev, f, S, wl.T_hartree, Delta, alpha, 0, wl.seed, 0, k, wl.L)
        if rc != 0:
            raise RuntimeError(f"langevin step failed: {vmc._lib().vmc_strerror(rc).decode()}")
        state["E"], state["acc"] = E, acc

    for k in range(warmup):
        one_step(k)
    torch.cuda.synchronize()
    for c in set(ctxs) | {ctx}:
        c.reset_kernel_times()
        c.set_profiling(True)
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        one_step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = {}
    for c in set(ctxs) | {ctx}:
        for kname, (ms, n) in c.kernel_times().items():
            t_ms, t_n = times.get(kname, (0.0, 0))
            times[kname] = (t_ms + ms, t_n + n)
        c.set_profiling(False)
    for tr in trajs:
        tr.close()
    for c in ctxs:
        if c is not ctx:
            c.close()
    pool.shutdown()
    sgroups.shutdown()
    ranked = sorted(times.items(), key=lambda kv: -kv[1][0])
    rl = {}
    # the work model counts the single-Gaussian, two-body wavefunction
    for kname, (ms, n) in (ranked[:2] if not paper else []):
        avg_s = ms / max(n, 1) / 1e3
        parts = work_model(kname, N, 0, 0, 1, False, False, state["acc"])
        flops, achieved, peak = roofline_numbers(parts, W, avg_s)
        ex = executed_model(kname, N, 0, 0, 1, False, False, state["acc"])
        rl[kname] = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4) if peak else None, "avg_launch_ms": round(avg_s * 1e3, 4),
                     "algorithmic_flop_per_launch": round(flops),
                     "executed_tflops": round(sum(ex.values()) * W / avg_s / 1e12, 3)}
        if ns > 1:
            # launches of different streams share the GPU, so these rates are lower bounds
            rl[kname]["overlapped_streams"] = ns
    return {"value": round(W * n_tw * M * steps / elapsed, 1), "unit": "walker-sweeps/s",
            "workload": f"{name}: {N} H, r_s={wl.rs}, {q}x{q}x{q} Monkhorst-Pack twists x {W} walkers x {M} measured "
                        f"(+5 re-equilibration) sweeps per Langevin step, complex orbitals, FP64"
                        + (", contracted basis eta=0.1, one-body b_1=2.5 and f="
                           + ",".join(f"{x:g}" for x in J1F_LEG) + ", three-body F="
                           + ",".join(f"{x:g}" for x in J3_LEG_F) if paper else ""),
            "twists": n_tw, "walkers_per_twist": W, "sweeps": M, "steps": steps, "warmup": warmup,
            "ms_per_step": round(1e3 * elapsed / steps, 1), "langevin_steps_per_s": round(steps / elapsed, 4),
            "E_Ha_twist_average": state["E"], "acceptance": round(state["acc"], 4),
            "dominant_kernel": ranked[0][0], "roofline": rl or None, "wavefunction": wavefunction, "streams": ns,
            "kernel_ms": {k: round(v[0], 2) for k, v in ranked if v[0] > 0}}


def run_mesh(args):
    r = twist_mesh_leg(args.workload if args.workload != "h256" else "h128", args.mesh, args.mesh_walkers,
                       args.sweeps, args.steps, args.warmup, args.mesh_wavefunction, args.mesh_streams)
    dom = (r["roofline"] or {}).get(r["dominant_kernel"], {"bound": "alu", "achieved": None, "peak": PEAK["f64"],
                                                           "unit": "TFLOP/s", "frac": None})
    line = {"metric": "twist-averaged VMC walker-sweeps/s with forces (general twists)", "value": r["value"],
            "unit": r["unit"], "n_gpus": 1, "steps": r["steps"], "warmup": r["warmup"],
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic", "config": {"workload": r["workload"]},
            "roofline": dict(dom, kernel=r["dominant_kernel"], traffic=None)}
    line.update({k: v for k, v in r.items() if k not in ("value", "unit", "workload", "steps", "warmup", "ms_per_step")})
    print(json.dumps(line))


def cpu_host_info() -> dict:
    """The host the CPU baseline runs on: logical CPUs, those this process may use, the model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable": usable, "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def kernel_space(sysd, wl, prec_mixed: bool):
    """Reciprocal vectors, their (ny, nz) slots and the Gaussian image rule of a workload."""
    nm = sysd.ewald_nmax
    kset = [(nx, ny, nz) for nx in range(0, nm + 1) for ny in range(-nm, nm + 1) for nz in range(-nm, nm + 1)
            if 0 < nx * nx + ny * ny + nz * nz <= nm * nm and (nx > 0 or (nx == 0 and (ny > 0 or (ny == 0 and nz > 0))))]
    nk, nslot = len(kset), len({(ny, nz) for _, ny, nz in kset})
    nimg = int(not (prec_mixed and float(np.min(wl.zeta)) * (wl.L / 2) ** 2 >= 23.0))
    return nk, nslot, nimg


def run_opt_leg(wl, W: int, M: int, prec: int, b1: float, F, n_opt: int, m_opt: int, steps: int, mask: int = 0b11101,
                eps: float = 0.1, tau: float = 0.1) -> dict:
    """Langevin steps with the wavefunction re-optimised before each (the paper's n_opt steps of
    optimisation per ionic step): n_opt stochastic-reconfiguration iterations, each m_opt measured
    sweeps (+5 re-equilibration) with the parameter statistics, the SR step on the parameters in
    `mask` (bits: b, b_1, f11, f12, f22, f1, f2) and the new parameters, then the energy/force estimate, S
    and the update as in run_leg.  The first step is the warm-up; `steps` are timed."""
    import torch
    from paper_1605_08423_amd import vmc
    ctx = vmc.Context(0)
    p = np.array([1.0, b1, *F, 0.0, 0.0], dtype=np.float64)   # the leg's wavefunction has no orbital part f
    sysd = vmc.make_system(wl.n, wl.L, precision=prec, b=p[0], b1=p[1], j3=tuple(p[2:5]))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    traj = vmc.Trajectory(ctx, sysd, W, seed=wl.seed, traj_id=0)
    traj.set_walkers(dev(wl.electrons(W=W)))
    traj.set_R(dev(wl.R.reshape(-1)))
    zeta = dev(wl.zeta)
    alpha = 0.122 * W * M
    Delta = 1.0 / alpha
    path, energies, sr_s = [p.copy()], [], []

    def one_step(k):
        nonlocal p
        Cm = dev(vmc.vmc_huckel_params(traj.get_R().cpu().numpy(), wl.zeta, wl.L))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        traj.set_param_stats(True)
        for i in range(n_opt):
            # optimisation sweeps draw from counters of their own, apart from the trajectory's
            traj.energy_forces(None, Cm, zeta, 20 if k == 0 and i == 0 else 5, m_opt, wl.delta,
                               step=0x80000000 | (k << 8) | i)
            st = traj.param_stats()
            energies.append(float(st[0].item()))
            dp = vmc.vmc_sr_update(st, mask, eps, tau)
            p = p + dp
            traj.set_jastrow(p[0], p[1], tuple(p[2:5]), tuple(p[5:7]))
            path.append(p.copy())
        traj.set_param_stats(False)
        sr_s.append(time.perf_counter() - ts)
        out = traj.energy_forces(None, Cm, zeta, 5, M, wl.delta, step=None)
        traj.build_S(keep_only=True)
        rc = traj.langevin_step(wl.T_hartree, Delta, alpha)
        if rc != 0:
            raise RuntimeError(f"langevin step failed: {vmc._lib().vmc_strerror(rc).decode()}")
        return out

    one_step(0)
    torch.cuda.synchronize()
    ctx.reset_kernel_times()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for k in range(1, 1 + steps):
        out = one_step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = ctx.kernel_times()
    ctx.set_profiling(False)
    out_h = out.cpu().numpy()
    traj.close()
    ctx.close()
    return {"elapsed": elapsed, "steps": steps, "times": times, "out": out_h, "path": path, "sr_E": energies,
            "sweeps_per_step": n_opt * (m_opt + 5) + M + 5, "sr_s": sum(sr_s[1:]) / max(steps * n_opt, 1)}


def run_leg(wl, W: int, M: int, prec: int, b1: float, steps: int, warmup: int, log=None, eta=None, j3=None) -> dict:
    """Langevin steps of one trajectory, each one full pass of the hot path: Hueckel orbitals and
    proton tables at R, the energy/force estimate (20 equilibration sweeps at the first step, 5
    after), S and the update on the trajectory's own state.  Times `steps` steps after `warmup`."""
    import torch
    from paper_1605_08423_amd import vmc
    ctx = vmc.Context(0)
    sysd = vmc.make_system(wl.n, wl.L, precision=prec, b1=b1, eta=eta, j3=j3)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    traj = vmc.Trajectory(ctx, sysd, W, seed=wl.seed, traj_id=0)
    traj.set_walkers(dev(wl.electrons(W=W)))
    traj.set_R(dev(wl.R.reshape(-1)))
    zeta = dev(wl.zeta)
    alpha = 0.122 * W * M             # N_c = W M samples per step
    Delta = 1.0 / alpha               # alpha Delta = 1

    def one_step(k):
        Rh = traj.get_R().cpu().numpy()
        Cm = (vmc.vmc_huckel_params(Rh, wl.zeta, wl.L) if eta is None
              else vmc.vmc_huckel_params_contracted(Rh, wl.L, eta))
        out = traj.energy_forces(None, dev(Cm), zeta, 20 if k == 0 else 5, M, wl.delta, step=None)
        S = traj.build_S() if log is not None else traj.build_S(keep_only=True)
        rc = traj.langevin_step(wl.T_hartree, Delta, alpha)
        if rc != 0:
            raise RuntimeError(f"langevin step failed: {vmc._lib().vmc_strerror(rc).decode()}")
        return out, S

    for k in range(warmup):
        one_step(k)
    torch.cuda.synchronize()
    ctx.reset_kernel_times()
    ctx.set_profiling(True)
    lat = []
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        ts = time.perf_counter()
        out, S = one_step(k)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        if log is not None:
            oh = out.cpu().numpy()
            log.write(json.dumps({"step": k, "E_Ha": float(oh[0]), "sigma_E_Ha": float(oh[1]), "acceptance": float(oh[2]),
                                  "force_norm": float(np.linalg.norm(oh[3:])),
                                  "cond_S": float(np.linalg.cond(S.cpu().numpy())), "ms": round(1e3 * lat[-1], 2)}) + "\n")
            log.flush()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = ctx.kernel_times()
    ctx.set_profiling(False)
    out_h = out.cpu().numpy()
    traj.close()
    ctx.close()
    lat_ms = sorted(1e3 * x for x in lat)
    p = lambda q: lat_ms[min(len(lat_ms) - 1, int(math.ceil(q * len(lat_ms))) - 1)]
    return {"value": W * M * steps / elapsed, "elapsed": elapsed, "steps": steps, "times": times, "out": out_h,
            "p50": p(0.5), "p99": p(0.99), "sysd": sysd}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["h128", "h256"], default="h128",
                    help="h128: 128 H, r_s 1.34, T 1000 K, 16384 walkers (the headline); "
                         "h256: 256 H, r_s 1.36, T 900 K, 32768 walkers")
    ap.add_argument("--walkers", type=int, default=None, help="default: the workload's walker count")
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--rs", type=float, default=None, help="default: the workload's r_s")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--log", default=None, metavar="PATH",
                    help="write one JSON line per timed Langevin step: E, sigma_E, |f|, acceptance, cond(S), time")
    ap.add_argument("--j1", type=float, default=0.0, metavar="B1",
                    help="add the one-body electron-proton Jastrow term with this b_1 (0: none)")
    ap.add_argument("--eta", type=float, default=None,
                    help="the contracted orbital phi_1 + eta phi_2 per proton (the SI's Z1, Z2) instead of one "
                         "s-Gaussian")
    ap.add_argument("--contracted-leg", type=float, default=0.1, metavar="ETA",
                    help="eta of the short contracted-basis leg of the default line (nan: skip)")
    ap.add_argument("--j3", type=_f3, default=None, metavar="F11,F12,F22",
                    help="add the on-site three-body Jastrow term with this symmetric F")
    ap.add_argument("--opt-leg", type=int, default=4, metavar="N_OPT",
                    help="SR iterations per ionic step of the short wavefunction-optimisation leg of the default "
                         "line (10 sweeps each; b_1 = 2.5 and the three-body leg's F to start; 0: skip)")
    ap.add_argument("--three-body-leg", type=_f3, default=J3_LEG_F, metavar="F11,F12,F22",
                    help="F of the short three-body leg of the default line (run with b_1 = 2.5; 'none': skip)")
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed steps of the plain FP64 leg beside a mixed-precision headline (0: skip)")
    ap.add_argument("--serve-leg", type=int, default=12, metavar="K",
                    help="trajectories of the short served-stream leg of the default line (0: skip)")
    ap.add_argument("--cpu-walkers", type=int, default=None, help="default: 192 (h128), 16 (h256)")
    ap.add_argument("--cpu-sweeps", type=int, default=None, help="default: 6 (h128), 2 (h256)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads: the CPU share of one GPU on the GPU host (capped at the usable CPUs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="print per-kernel times to stderr")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration) and exit")
    ap.add_argument("--serve", type=int, default=0, metavar="K",
                    help="served-stream benchmark of K trajectories instead of the single-trajectory step")
    ap.add_argument("--serve-mix", choices=["stream", "large"], default="stream",
                    help="stream: K trajectories with N in {16,32,54,128}; large: one N=256 box and eight N=54 boxes")
    ap.add_argument("--serve-rate", type=float, default=16.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-steps", type=int, default=3)
    ap.add_argument("--serve-sweeps", type=int, default=20)
    ap.add_argument("--serve-budget-gb", type=float, default=160.0)
    ap.add_argument("--twists", type=int, default=1, metavar="N",
                    help="twist-averaged steps over the first N of the 8 real twists (2..8), walkers split evenly")
    ap.add_argument("--mesh", type=int, default=0, metavar="Q",
                    help="twist-averaged steps over the Q x Q x Q Monkhorst-Pack mesh of general twists (complex "
                         "orbitals, FP64) instead")
    ap.add_argument("--mesh-walkers", type=int, default=256, help="walkers per twist of --mesh and the mesh leg")
    ap.add_argument("--paper-mesh-leg", type=int, default=4, metavar="Q",
                    help="Q of the short twist-mesh leg with the paper's wavefunction terms (0: skip)")
    ap.add_argument("--mesh-streams", type=int, default=4,
                    help="HIP streams the twists of --mesh and of the mesh legs run on (one library context each)")
    ap.add_argument("--mesh-wavefunction", choices=["gaussian", "paper"], default="gaussian",
                    help="the wavefunction of --mesh: one s-Gaussian and the two-body Jastrow, or the paper's terms "
                         "(contracted basis, one- and three-body Jastrow)")
    ap.add_argument("--mesh-leg", type=int, default=4, metavar="Q",
                    help="Q of the short twist-mesh leg of the default line (0: skip)")
    ap.add_argument("--toy", action="store_true", help="the toy-model figure as a GPU workload instead")
    ap.add_argument("--toy-traj", type=int, default=65536)
    ap.add_argument("--toy-steps", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the walker-sharded multi-GPU path is a design "
              f"that is not built, so --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)
    if args.toy:
        run_toy(args)
        return
    if args.mesh:
        run_mesh(args)
        return
    if args.twists > 1:
        if args.twists > 8:
            print("bench.py takes at most the 8 real twists.", file=sys.stderr)
            sys.exit(2)
        run_twists(args)
        return
    if args.serve or args.serve_mix == "large":
        run_serve(args)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}))
        return

    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload

    wl = workload(args.workload, rs=args.rs)
    N, W, M = wl.n, args.walkers or wl.walkers, args.sweeps
    mixed = args.precision == "mixed"
    prec = vmc.VMC_MIXED if mixed else vmc.VMC_FP64
    log = open(args.log, "w") if args.log else None
    lead = run_leg(wl, W, M, prec, args.j1, args.steps, args.warmup, log, args.eta, args.j3)
    times, out_h, sysd = lead["times"], lead["out"], lead["sysd"]
    nk, nslot, nimg = kernel_space(sysd, wl, mixed)
    acc = float(out_h[2])
    tkey = traffic_workload_key(args.workload, args.precision, W, args.j1, args.rs, args.j3)
    j3on = args.j3 is not None

    def kernel_roofline(name):
        ms, n = times[name]
        parts = work_model(name, N, nk, nslot, nimg, mixed, args.j1 > 0, acc, args.eta is not None, j3on)
        executed = executed_model(name, N, nk, nslot, nimg, mixed, args.j1 > 0, acc, args.eta is not None, j3on)
        avg_s = ms / max(n, 1) / 1e3
        flops, achieved, peak = roofline_numbers(parts, W, avg_s)
        return {"bound": "alu", "kernel": name, "achieved": round(achieved, 3), "peak": round(peak, 2),
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if peak else None,
                "traffic": measured_traffic(name, tkey), "avg_launch_ms": round(avg_s * 1e3, 4),
                "algorithmic_flop_per_launch": round(flops), "algorithmic_flop_per_walker_by_unit":
                    {u: round(f) for u, f in parts.items()},
                "executed_flop_per_launch": round(sum(executed.values()) * W),
                "executed_tflops": round(sum(executed.values()) * W / avg_s / 1e12, 3), "acceptance": round(acc, 4)}

    # the dominant kernel by total time in the timed region; the sweep and the measurement take
    # nearly the same total time at 128 protons, so the runner-up is reported beside it
    ranked = sorted(times.items(), key=lambda kv: -kv[1][0])
    roofline = kernel_roofline(ranked[0][0])
    if len(ranked) > 1 and ranked[1][1][0] > 0:
        second = kernel_roofline(ranked[1][0])
        roofline["runner_up"] = {k: second[k] for k in ("kernel", "achieved", "peak", "frac", "traffic",
                                                        "avg_launch_ms")}
        roofline["runner_up"]["time_vs_dominant"] = round(ranked[1][1][0] / ranked[0][1][0], 4)
    if args.profile:
        for kname, (ms, n) in sorted(times.items(), key=lambda kv: -kv[1][0]):
            print(f"{kname:16s} {ms:10.2f} ms  {n:6d} launches  {ms / max(n, 1):9.4f} ms/launch", file=sys.stderr)

    fp64 = None
    if mixed and args.fp64_steps > 0:
        # the plain FP64 GPU path on the same workload, a few steps
        r = run_leg(wl, W, M, vmc.VMC_FP64, args.j1, args.fp64_steps, 1)
        fp64 = {"value": round(r["value"], 1), "unit": "walker-sweeps/s", "steps": r["steps"], "warmup": 1,
                "ms_per_step": round(1e3 * r["elapsed"] / r["steps"], 2),
                "langevin_steps_per_s": round(r["steps"] / r["elapsed"], 4),
                "mixed_over_fp64": round(lead["value"] / r["value"], 3), "E_Ha": float(r["out"][0])}

    served = None
    if args.serve_leg > 0 and args.workload == "h128":
        served = serve_stream(args.serve_leg, 2, 10, args.serve_rate, args.serve_budget_gb)

    contracted = None
    if args.eta is None and args.contracted_leg == args.contracted_leg and args.workload == "h128":
        # the same workload on the contracted basis, a few steps
        r = run_leg(wl, W, M, prec, args.j1, 2, 1, None, args.contracted_leg)
        kms = {k: v for k, v in r["times"].items() if v[1]}
        dom = max(kms.items(), key=lambda kv: kv[1][0])
        avg_s = dom[1][0] / dom[1][1] / 1e3
        nk_c, nslot_c, _ = kernel_space(r["sysd"], wl, mixed)
        parts = work_model(dom[0], N, nk_c, nslot_c, 1, mixed, args.j1 > 0, float(r["out"][2]), True)
        flops, achieved, peak = roofline_numbers(parts, W, avg_s)
        contracted = {"eta": args.contracted_leg, "value": round(r["value"], 1), "unit": "walker-sweeps/s",
                      "steps": r["steps"], "warmup": 1, "ms_per_step": round(1e3 * r["elapsed"] / r["steps"], 2),
                      "over_single_gaussian": round(r["value"] / lead["value"], 3), "E_Ha": float(r["out"][0]),
                      "acceptance": round(float(r["out"][2]), 4), "dominant_kernel": dom[0],
                      "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
                                   "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if peak else None,
                                   "avg_launch_ms": round(avg_s * 1e3, 4)},
                      "kernel_ms": {k: round(v[0], 2) for k, v in kms.items()}}

    three_body = None
    if args.j3 is None and args.three_body_leg is not None and args.eta is None and args.workload == "h128":
        # the same workload with the one-body cusp (b_1 = 2.5) and the three-body term, a few steps
        b1 = args.j1 if args.j1 > 0 else 2.5
        r = run_leg(wl, W, M, prec, b1, 2, 1, None, None, args.three_body_leg)
        acc3 = float(r["out"][2])
        kms = {k: v for k, v in r["times"].items() if v[1]}
        per = {}
        for k in ("sweep_half", "slater_sample", "j3_grad", "j3_forces"):
            if k not in kms:
                continue
            avg_s = kms[k][0] / kms[k][1] / 1e3
            parts = work_model(k, N, nk, nslot, nimg, mixed, True, acc3, False, True)
            _, achieved, peak = roofline_numbers(parts, W, avg_s)
            per[k] = {"avg_launch_ms": round(avg_s * 1e3, 4), "achieved": round(achieved, 3), "peak": round(peak, 2),
                      "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if peak else None}
        three_body = {"F": list(args.three_body_leg), "b1": b1, "value": round(r["value"], 1),
                      "unit": "walker-sweeps/s", "steps": r["steps"], "warmup": 1,
                      "ms_per_step": round(1e3 * r["elapsed"] / r["steps"], 2),
                      "over_headline": round(r["value"] / lead["value"], 3), "E_Ha": float(r["out"][0]),
                      "sigma_E_Ha": float(r["out"][1]), "acceptance": round(acc3, 4), "kernels": per,
                      "kernel_ms": {k: round(v[0], 2) for k, v in kms.items()}}

    optimisation = None
    if args.opt_leg > 0 and args.j3 is None and args.eta is None and args.workload == "h128":
        F0 = args.three_body_leg or J3_LEG_F
        b1 = args.j1 if args.j1 > 0 else 2.5
        r = run_opt_leg(wl, W, M, prec, b1, F0, args.opt_leg, 10, 2)
        kms = {k: v for k, v in r["times"].items() if v[1]}
        per = {}
        if "opt_sample" in kms:
            avg_s = kms["opt_sample"][0] / kms["opt_sample"][1] / 1e3
            _, achieved, peak = roofline_numbers(work_model("opt_sample", N, nk, nslot, nimg, mixed, True), W, avg_s)
            per = {"avg_launch_ms": round(avg_s * 1e3, 4), "achieved": round(achieved, 3), "peak": round(peak, 2),
                   "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if peak else None}
        ms_step = 1e3 * r["elapsed"] / r["steps"]
        optimisation = {"n_opt": args.opt_leg, "sweeps_per_sr_step": 10, "b1": b1, "F0": list(F0),
                        "active": "b, f11, f12, f22", "eps": 0.1, "tau": 0.1, "steps": r["steps"], "warmup": 1,
                        "ms_per_ionic_step": round(ms_step, 2),
                        "ms_per_sr_iteration": round(1e3 * r["sr_s"], 2),
                        "walker_sweeps_per_s": round(W * r["sweeps_per_step"] * r["steps"] / r["elapsed"], 1),
                        "E_Ha": float(r["out"][0]), "sr_E_Ha": [round(e, 4) for e in r["sr_E"]],
                        "params_b_b1_F_f": [round(float(v), 4) for v in r["path"][-1]], "opt_sample": per,
                        "kernel_ms": {k: round(v[0], 2) for k, v in kms.items()}}

    mesh = None
    if args.mesh_leg > 0 and args.workload == "h128":
        mesh = twist_mesh_leg("h128", args.mesh_leg, args.mesh_walkers, 10, 1, 1, streams=args.mesh_streams)
    paper_mesh = None
    if args.paper_mesh_leg > 0 and args.workload == "h128":
        paper_mesh = twist_mesh_leg("h128", args.paper_mesh_leg, args.mesh_walkers, 10, 1, 1, "paper",
                                    streams=args.mesh_streams)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        host = cpu_host_info()
        Cm0, _ = O.huckel(wl.R, wl.zeta, wl.L, N // 2)
        threads = max(1, min(args.cpu_threads, host["usable"] or 1))
        cw = args.cpu_walkers or (192 if N <= 128 else 16)
        cs = args.cpu_sweeps or (6 if N <= 128 else 2)
        v, dt = run_cpu_baseline(wl, Cm0, cw, cs, threads, args.j1)
        # one thread on a smaller sample, for the per-core rate
        w1 = 8 if N <= 128 else 2
        v1, dt1 = run_cpu_baseline(wl, Cm0, w1, 2 if N <= 128 else 1, 1, args.j1)
        cpu = {"value": round(v, 3), "unit": "walker-sweeps/s", "cores": threads, "kind": "oracle",
               "value_one_core": round(v1, 3), "host": host,
               "sample": f"{cw} walkers x (1 unmeasured + {cs} measured) sweeps of the "
                         f"same N={N} box in FP64 on {threads} threads ({dt:.1f} s; the CPU share of one GPU on "
                         f"this host is 16 threads); one core: {w1} walkers x (1 + {2 if N <= 128 else 1}) "
                         f"sweeps, {dt1:.1f} s"}
    line = {
        "metric": METRIC, "value": round(lead["value"], 1), "unit": "walker-sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * lead["elapsed"] / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N} H + {N} e-, r_s={wl.rs}, T={wl.T_kelvin:g} K, {W} walkers x {M} "
                               f"measured (+5 re-equilibration) sweeps per Langevin step, {args.precision} precision"
                               + (f", one-body Jastrow b_1={args.j1:g}" if args.j1 > 0 else "")
                               + (f", contracted basis eta={args.eta:g}" if args.eta is not None else "")
                               + (f", three-body F={','.join(f'{x:g}' for x in args.j3)}" if j3on else ""),
                   "N": N, "walkers": W, "sweeps": M, "precision": args.precision, "one_body_b1": args.j1},
        "langevin_steps_per_s": round(args.steps / lead["elapsed"], 4),
        "step_latency_ms": {"p50": round(lead["p50"], 1), "p99": round(lead["p99"], 1)},
        "E_Ha": float(out_h[0]), "sigma_E_Ha": float(out_h[1]), "acceptance": acc,
        "roofline": roofline, "fp64_gpu": fp64, "served": served, "twist_mesh": mesh,
        "twist_mesh_paper_wavefunction": paper_mesh,
        "contracted_basis": contracted, "three_body": three_body, "optimisation": optimisation,
        "cpu_baseline": cpu,
        "kernel_ms": {k: round(v[0], 2) for k, v in times.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
