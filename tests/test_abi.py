"""The C-ABI library loads and exports every entry point the header declares
(no GPU work: loading the shared object needs the HIP runtime only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pcsqrt.h")).read()
    return sorted(set(re.findall(r"^(?:pc_status|const char \*|int32_t)\s*(pc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_three_hot_path_calls():
    names = _declared()
    for n in ("pc_sqrt_build", "pc_gram_factor", "pc_left_inverse_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2609_13327_amd as pc
    if not os.path.exists(pc.LIB_PATH):
        pytest.fail("libpcsqrt.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(pc.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(pc.EXPORTED) == _declared()


def test_status_strings():
    import paper_2609_13327_amd as pc
    assert pc.status_string(pc.PC_OK) == "ok"
    assert "rank deficient" in pc.status_string(pc.PC_ERR_NOT_SPD)
    assert pc.status_string(12345) == "unknown status"


def test_cholesky_task_order_is_topological():
    """The persistent Cholesky kernel takes tasks in a fixed order; the host
    replay checks every task appears once and after everything it waits for."""
    import paper_2609_13327_amd as pc
    for T in (1, 2, 3, 5, 7, 8, 13, 33, 64, 97, 256, 512):
        assert pc.pc_selftest_task_order(T) == 0, T
        for G in (1, 2, 3, 4, 5, 6, 7, 8):
            if G <= T:
                assert pc.pc_selftest_task_order(T, G) == 0, (T, G)
    assert pc.pc_selftest_task_order(0) == -1
    assert pc.pc_selftest_task_order(4, 5) == -1
