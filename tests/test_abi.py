"""The C-ABI library loads and exports every symbol include/vmc.h declares (no GPU
needed), and its host-side Hueckel helper spans the oracle's occupied space."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vmc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t|const char\*)\s+(vmc_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1605_08423_amd import vmc
    lib = ctypes.CDLL(vmc.library_path())
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(vmc.EXPORTED) == names


def test_error_strings_and_supported_sizes():
    from paper_1605_08423_amd import vmc
    lib = vmc._lib()
    assert lib.vmc_strerror(vmc.VMC_ENOTSPD).decode() == "S is not positive definite"
    assert vmc.supported_n(16) and vmc.supported_n(54) and vmc.supported_n(128) and vmc.supported_n(256)
    assert not vmc.supported_n(17) and not vmc.supported_n(100)


@pytest.mark.parametrize("name,twist", [("h16", 0), ("h54", 0), ("h128", 0), ("h16", 5), ("h54", 3), ("h128", 7)])
def test_host_huckel_spans_oracle_occupied_space(oracle, name, twist):
    """The library's host Hueckel helper (also with real twists) spans the oracle's occupied space."""
    from paper_1605_08423_amd import vmc
    from paper_1605_08423_amd.inputs import workload
    wl = workload(name)
    Cg = vmc.vmc_huckel_params(wl.R, wl.zeta, wl.L, twist=twist)
    Co, ev = oracle.huckel(wl.R, wl.zeta, wl.L, wl.n // 2, twist=twist)
    assert ev[wl.n // 2] - ev[wl.n // 2 - 1] > 1e-3      # non-degenerate HOMO-LUMO gap
    np.testing.assert_allclose(Cg @ Cg.T, Co @ Co.T, atol=1e-12)
