"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtproj.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtproj_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for need in ["rtproj_plan_create", "rtproj_precondition", "rtproj_project_null", "rtproj_project_row",
                 "rtproj_lstsq", "rtproj_project_all", "rtproj_plan_destroy", "rtproj_batch_create",
                 "rtproj_batch_precondition", "rtproj_batch_project_all", "rtproj_batch_status"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_0912_1135_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(rt.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_without_device():
    import paper_0912_1135_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("library not built")
    L = rt.lib()
    for s in range(8):
        assert L.rtproj_status_string(s).decode()
    assert L.rtproj_status_string(99).decode() == "unknown status"


def test_binding_rejects_bad_arguments_before_device_work():
    import paper_0912_1135_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("library not built")
    h = ctypes.c_void_p()
    # sizes are validated on the host before any HIP call
    assert rt.lib().rtproj_plan_create(10, 5, 6, 0, ctypes.byref(h)) == 1
    assert rt.lib().rtproj_plan_create(0, 5, 1, 0, ctypes.byref(h)) == 1
    assert rt.lib().rtproj_plan_create(4, 10, 11, 0, ctypes.byref(h)) == 1
    assert rt.lib().rtproj_plan_create(4, 10, 3, 0, ctypes.byref(h)) == 1
    assert not h.value
    assert rt.lib().rtproj_project_null(None, None, 0, 1, None, 0) == 1


def test_batch_rejects_bad_sizes_before_device_work():
    import paper_0912_1135_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("library not built")
    L = rt.lib()
    h = ctypes.c_void_p()
    i64 = lambda v: (ctypes.c_int64 * len(v))(*v)
    assert L.rtproj_batch_create(0, i64([1]), i64([4]), i64([2]), 1, ctypes.byref(h)) == 1
    assert L.rtproj_batch_create(2, i64([4, 5]), i64([8, 8]), i64([2, 5]), 1, ctypes.byref(h)) == 1   # l < m
    assert L.rtproj_batch_create(1, i64([4]), i64([3]), i64([4]), 1, ctypes.byref(h)) == 1            # n < m
    assert L.rtproj_batch_create(1, i64([4096]), i64([9000]), i64([8192]), 1, ctypes.byref(h)) == 7  # m too large
    assert not h.value


def test_binding_checks_tensors_before_any_library_call():
    """Host tensors (or wrong dtypes) are rejected by the binding itself."""
    import paper_0912_1135_amd as rt
    torch = pytest.importorskip("torch")
    plan = object.__new__(rt.Plan)
    plan.handle, plan.m, plan.n, plan.l = None, 4, 10, 8
    B = torch.zeros((2, 10), dtype=torch.float64)
    for call in (plan.project_null, plan.project_row, plan.lstsq, plan.project_all):
        with pytest.raises(TypeError):
            call(B)
    with pytest.raises(TypeError):
        plan.precondition(torch.zeros((4, 10), dtype=torch.float32))
