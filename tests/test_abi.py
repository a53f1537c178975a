"""The C-ABI library loads without a GPU and exports every function that
include/mgmlmc.h declares; the Python binding covers all of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgmlmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(mgm_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mgm_context_create", "mgm_operator_apply", "mgm_hierarchy_create", "mgm_draw_z4",
                 "mgm_solve", "mgm_estimate", "mgm_mlmc_allocate", "mgm_net_train", "mgm_net_apply"):
        assert must in names


def test_library_exports_every_declared_function():
    from paper_2509_11424_amd.api import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2509_11424_amd.api import EXPORTED
    assert sorted(set(EXPORTED)) == declared_functions()


def test_status_strings_without_gpu():
    from paper_2509_11424_amd.api import LIB_PATH, lib
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    assert lib().mgm_status_string(0).decode() != ""
    assert lib().mgm_status_string(-4).decode() != ""


def test_mlmc_allocation_closed_form_on_host():
    # N_l = eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k): total cost and variance
    import numpy as np
    from paper_2509_11424_amd.api import LIB_PATH, mlmc_allocate
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    V = np.array([4.0, 1.0, 0.25])
    Cst = np.array([1.0, 0.1, 0.01])
    eps2 = 1e-3
    N = mlmc_allocate(V, Cst, eps2)
    assert np.all(N >= 2)
    ideal = np.sqrt(V / Cst) * np.sum(np.sqrt(V * Cst)) / eps2
    assert np.all(N >= np.floor(ideal)) and np.all(N <= np.ceil(ideal) + 1)
    assert np.sum(V / N) <= eps2 * (1 + 1e-9)
