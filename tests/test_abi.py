"""The C-ABI library loads and exports every entry point its header declares;
argument checks that need no device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "l0l2.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(l0l2_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["l0l2_create", "l0l2_set_data", "l0l2_solve_node_batch", "l0l2_refine_incumbent",
              "l0l2_bnb_solve", "l0l2_round_branch", "l0l2_dual_bound", "l0l2_admm_sweeps"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2602_04551_amd import binding
    lib = C.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.SIGNATURES) == set(declared_functions())


def test_null_arguments_are_rejected_without_a_device():
    from paper_2602_04551_amd import binding as b
    lib = b.lib
    assert lib.l0l2_create(0, None, None) == b.L0L2_E_INVALID
    assert isinstance(lib.l0l2_last_error(None), bytes)
    assert lib.l0l2_set_data(None, None, None, 1, 1, 0.0, 1.0, 1.0, 1.0, 0, 0) == b.L0L2_E_INVALID
    assert lib.l0l2_bnb_solve(None, None, None) == b.L0L2_E_INVALID
    assert lib.l0l2_solve_node_batch(None, 0, None, None, None, None, None, None, None, None) == b.L0L2_E_INVALID
    assert lib.l0l2_state_bytes(None) == b.L0L2_E_INVALID
    lib.l0l2_destroy(None)
    lib.l0l2_result_free(None)


def test_binding_names_match_the_abi():
    from paper_2602_04551_amd import binding
    for name in declared_functions():
        assert hasattr(binding.lib, name)


def test_footprint_estimate_grows_with_size_and_batch():
    from paper_2602_04551_amd.binding import lib
    f = lib.l0l2_footprint_bytes
    assert f(1000, 1000, 1, 256) > f(1000, 1000, 1, 32) > 0
    assert f(2000, 1000, 1, 256) > f(1000, 1000, 1, 256)
    assert f(1000, 2000, 1, 256) > f(1000, 1000, 1, 256)
    assert f(1000, 2100, 0, 256) > f(1000, 2100, 1, 256)  # FP64 state is twice as wide (no Gram form at p > 2 n)
    # the Gram form's p x p buffers count where that form is a candidate (padded
    # p <= 2 padded n): just inside the limit the estimate exceeds that of a
    # wider design just outside
    for prec in (1, 2):
        assert f(1000, 2000, prec, 256) > f(1000, 2100, prec, 256)
        assert f(1000, 1500, prec, 256) - f(1000, 1400, prec, 256) > 12 * 1536 ** 2 - 12 * 1408 ** 2
    assert f(1000, 1500, 2, 256) - f(1000, 1500, 1, 256) >= 4 * 1536 ** 2   # BF16 also keeps G as a BF16 pair
    assert f(1000, 2000, 3, 256) < f(1000, 2100, 3, 256)       # no Gram form in FP8 mode
    # dominated by the instance copies for a wide design
    assert f(1000, 50000, 2, 256) > 8 * 1000 * 50000
