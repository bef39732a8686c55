"""Serving logic that needs no GPU: the admission rule and the device-byte model of
a request (the library loads without a device; these calls touch none)."""
import numpy as np
import pytest

from paper_1605_08423_amd.inputs import workload


@pytest.fixture(scope="module")
def vmc():
    from paper_1605_08423_amd import vmc
    return vmc


def test_admission_is_fifo_without_overtaking(vmc):
    assert vmc.admit_count(100, 0, [30, 30, 30, 30]) == 3
    assert vmc.admit_count(100, 50, [30, 30]) == 1
    # a large request at the head blocks smaller ones behind it (no starvation of large requests)
    assert vmc.admit_count(100, 50, [60, 10, 10]) == 0
    assert vmc.admit_count(100, 0, []) == 0
    assert vmc.admit_count(100, 0, [100]) == 1 and vmc.admit_count(100, 1, [100]) == 0


def _req(vmc, name, W, precision=0):
    wl = workload(name)
    sysd = vmc.make_system(wl.n, wl.L, precision=precision)
    return vmc.make_request(sysd, W, wl.R, wl.zeta, wl.electrons(W=W, seed_offset=1), n_steps=2, n_sweeps=4,
                            T=wl.T_hartree, Delta=1.0, alpha=1.0)


def test_request_bytes_model(vmc):
    b1, b2, b4 = (vmc.request_bytes(_req(vmc, "h16", W)) for W in (64, 128, 256))
    assert 0 < b1 < b2 < b4
    assert b4 - b2 == 2 * (b2 - b1)                      # linear in W beyond the per-trajectory tables
    N, NS = 16, 8
    per_walker = b2 - b1
    # at least the two Slater matrices and inverses per walker (4 N_s^2 doubles) and the positions
    assert per_walker >= 64 * 8 * (4 * NS * NS + 3 * N)
    # invalid request -> 0
    bad = _req(vmc, "h16", 64)
    bad.n_walkers = 1
    assert vmc.request_bytes(bad) == 0
    big = vmc.request_bytes(_req(vmc, "h128", 16384, precision=1))
    assert 1.5e9 < big < 4e9                            # ~3 GB of walker state and tables at N = 128, W = 16384
