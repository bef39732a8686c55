"""Seeded synthetic inputs for the hydrogen VMC / Langevin workloads.

This module is shared by the CPU oracle's tests and by the HIP path's tests and
benchmark. It only draws inputs (proton positions, Gaussian exponents, electron
start configurations) and holds none of the method's arithmetic.

The paper simulates 64 and 128 protons in a cubic box at r_s = 1.22-1.40 bohr and
T = 900-1800 K (main text, liquid-liquid transition paragraph; SI "Systematic
setup").  Its SI proton files are not available, so every workload here is a
synthetic hydrogen box drawn from a seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Boltzmann constant in Hartree per kelvin (CODATA 2018).
KB_HA_PER_K = 3.1668115634556e-6


def box_side(n: int, rs: float) -> float:
    """Cubic box side L with N electrons at Wigner-Seitz radius r_s: (4 pi N / 3) r_s^3 = L^3."""
    return (4.0 * math.pi * n / 3.0) ** (1.0 / 3.0) * rs


def jittered_simple_cubic(n: int, L: float, rng: np.random.Generator, jitter: float = 0.1) -> np.ndarray:
    """N sites of an m^3 simple-cubic grid (m = ceil(N^(1/3)), spacing L/m) picked by a
    seeded permutation, each coordinate jittered by U(-jitter, +jitter) bohr."""
    m = int(math.ceil(round(n ** (1.0 / 3.0), 12)))
    grid = np.array([(i, j, k) for i in range(m) for j in range(m) for k in range(m)], dtype=np.float64)
    pick = rng.permutation(len(grid))[:n]
    R = (grid[pick] + 0.5) * (L / m)
    R += rng.uniform(-jitter, jitter, size=R.shape)
    return np.mod(R, L)


def random_packing(n: int, L: float, rng: np.random.Generator, dmin: float = 1.0,
                   max_tries: int = 200000) -> np.ndarray:
    """Random sequential packing: uniform trial points accepted if their minimum-image
    distance to every accepted point is at least dmin bohr."""
    R = np.zeros((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_packing: density too high for dmin")
        p = rng.uniform(0.0, L, size=3)
        if k:
            d = R[:k] - p
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                continue
        R[k] = p
        k += 1
    return R


def initial_electrons(R: np.ndarray, W: int, L: float, rng: np.random.Generator,
                      sigma: float = 0.5) -> np.ndarray:
    """Walker start configurations: electron i sits near proton i, displaced by
    sigma * N(0,1)^3, wrapped into [0, L)^3.  Shape (W, N, 3)."""
    n = R.shape[0]
    x = R[None, :, :] + sigma * rng.standard_normal((W, n, 3))
    return np.mod(x, L)


@dataclass
class Workload:
    name: str
    n: int
    rs: float
    T_kelvin: float
    walkers: int
    sweeps: int
    steps: int
    seed: int
    zeta_lo: float
    zeta_hi: float
    lattice: str            # "sc" (jittered simple cubic) or "packing"
    mixed: bool             # FP32 orbitals/Jastrow/Ewald-real when True
    n_equil: int = 20
    n_requil: int = 5
    L: float = field(init=False)
    R: np.ndarray = field(init=False, repr=False)
    zeta: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.L = box_side(self.n, self.rs)
        rng = np.random.default_rng(self.seed)
        if self.lattice == "sc":
            self.R = jittered_simple_cubic(self.n, self.L, rng)
        else:
            self.R = random_packing(self.n, self.L, rng)
        if self.zeta_lo == self.zeta_hi:
            self.zeta = np.full(self.n, self.zeta_lo)
        else:
            self.zeta = rng.uniform(self.zeta_lo, self.zeta_hi, size=self.n)

    @property
    def T_hartree(self) -> float:
        return self.T_kelvin * KB_HA_PER_K

    @property
    def delta(self) -> float:
        """Metropolis box-move size: r_s."""
        return self.rs

    @property
    def kappa(self) -> float:
        """Ewald splitting parameter kappa = 8/L."""
        return 8.0 / self.L

    nmax: int = 9

    def electrons(self, W: int | None = None, seed_offset: int = 0) -> np.ndarray:
        rng = np.random.default_rng(1000003 * (self.seed + 1) + seed_offset)
        return initial_electrons(self.R, self.walkers if W is None else W, self.L, rng)


def workload(name: str, rs: float | None = None) -> Workload:
    """The named synthetic workloads (sizes follow the hydrogen runs of the paper)."""
    if name == "h16":       # 16 H, FP64, small: the oracle runs it in seconds
        return Workload("h16", 16, 1.44, 1500.0, 128, 100, 10, 1, 1.0, 1.0, "sc", False)
    if name == "h54":       # 54 H, FP64
        return Workload("h54", 54, 1.32, 1200.0, 4096, 400, 200, 2, 0.8, 1.2, "packing", False)
    if name == "h128":      # 128 H, mixed precision
        return Workload("h128", 128, 1.34 if rs is None else rs, 1000.0, 16384, 100, 1, 3,
                        0.8, 1.2, "packing", True)
    if name == "h256":      # 256 H, mixed precision
        return Workload("h256", 256, 1.36, 900.0, 32768, 100, 1, 5, 0.8, 1.2, "packing", True)
    raise KeyError(name)


def small_system(n: int, rs: float, seed: int, zeta_lo=0.8, zeta_hi=1.2, lattice="packing") -> Workload:
    """An ad-hoc synthetic box of n protons, for tests at sizes between the named ones."""
    return Workload(f"h{n}", n, rs, 1200.0, 8, 4, 1, seed, zeta_lo, zeta_hi, lattice, False)
