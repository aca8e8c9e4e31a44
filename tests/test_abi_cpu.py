"""CPU-side checks of the library boundary: the built HIP library loads and exports
every function declared in include/snapmd.h; the binding refuses host tensors."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "snapmd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("snap_forces", "eam_forces", "langevin_steps", "parareal_iterate", "snap_beta_grad",
              "snapmd_create", "snapmd_destroy", "snapmd_last_error", "snapmd_sync", "snapmd_bispectrum"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2212_10508_amd import snapmd
    L = snapmd.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_2212_10508_amd import snapmd
    with pytest.raises(TypeError):
        snapmd._dev(torch.zeros(3, 4, dtype=torch.float64), "x")


def test_workload_sizes():
    from paper_2212_10508_amd import workloads as W
    for n, N in ((4, 129), (6, 433), (8, 1025), (20, 16001)):
        x, box = W.bcc_sia(n)
        assert x.shape == (3, N) and np.all(x >= 0) and np.all(x < box[:, None])
    assert [W.snap_ncoeff(J) for J in (2, 4, 6, 8)] == [5, 14, 30, 55]
