"""Writes tests/golden/h128_oracle_512.json: a 512-walker FP64 run of the CPU oracle on the
128-proton box (r_s = 1.34, seed 3 of the seeded inputs), the statistical reference for the
mixed-precision GPU estimate (walker averages within 2 sigma).

Calls only the oracle and the seeded input generators.  The run: Hueckel orbitals of the
box, 512 walkers started next to their protons (seed offset 512), 20 unmeasured and 20
measured sweeps, Philox key (seed 9001, trajectory 0), step 0.  Both the expectation of
the estimate and its spread depend only on the start distribution and the sweep counts,
not on the walker count or the seed, so a GPU run from the same start distribution with
the same sweep counts estimates the same quantity whether or not the chains are
equilibrated.

Usage: python tests/golden/make_h128_oracle_512.py [threads]   (about 8 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1605_08423_amd.inputs import workload  # noqa: E402

W, N_EQUIL, M, SEED, OFFSET = 512, 20, 20, 9001, 512


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    wl = workload("h128")
    Cm, _ = O.huckel(wl.R, wl.zeta, wl.L, wl.n // 2)
    s = O.System(wl.R, wl.zeta, Cm, L=wl.L)
    x = wl.electrons(W=W, seed_offset=OFFSET)
    t0 = time.time()
    sums, nacc = s.vmc_run(x, N_EQUIL, M, wl.delta, seed=SEED, traj=0, step=0, threads=threads)
    dt = time.time() - t0
    red = O.reduce(sums, M)
    S = O.build_S(red["f_w"], red["f"])
    out = {
        "_cite": "statistical reference for the walker averages of the VMC estimate (main text, Eq. for V(R) "
                 "and f = -dV/dR; SI, the alpha paragraph: S = Cov of the mean force)",
        "_made_by": "tests/golden/make_h128_oracle_512.py (oracle only)",
        "workload": "h128", "r_s": wl.rs, "n_walkers": W, "n_equil": N_EQUIL, "n_sweeps": M,
        "electron_seed_offset": OFFSET, "philox_seed": SEED, "step_delta": wl.delta,
        "E": red["E"], "sigma_E": red["sigma_E"],
        "acceptance": float(nacc.sum()) / (W * wl.n * (N_EQUIL + M)),
        "f": red["f"].tolist(), "sigma_f": np.sqrt(np.diag(S)).tolist(),
        "cpu_seconds": round(dt, 1),
    }
    with open(os.path.join(HERE, "h128_oracle_512.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"E = {red['E']:.6f} +- {red['sigma_E']:.6f} Ha, {dt:.0f} s")


if __name__ == "__main__":
    main()
