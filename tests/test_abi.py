"""The C-ABI library loads and exports every entry point of include/femhip.h.

Host-only calls (size queries, argument checks that fail before any HIP call)
run here without a GPU; nothing in this file launches a kernel.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "femhip.h")
LIB = os.path.join(ROOT, "paper_1804_05156_amd", "libfemhip.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(fe_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def femhip():
    if not os.path.exists(LIB):
        from paper_1804_05156_amd import build
        build.build()
    from paper_1804_05156_amd import femhip as fh
    return fh


def test_header_lists_entry_points(femhip):
    assert _declared() == sorted(femhip.ENTRY_POINTS)


def test_library_exports_every_declared_symbol(femhip):
    lib = C.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_status_strings(femhip):
    assert "gfx950" in femhip.version()
    assert femhip.status_string(femhip.FE_OK) == "ok"
    assert "workspace" in femhip.status_string(femhip.FE_ESIZE)


def _mesh(femhip, dim=2, n=10, nt=12):
    m = femhip.fe_mesh()
    m.dim, m.n_node, m.n_elem = dim, n, nt
    m.node = C.c_void_p(0x1000)
    m.elem = C.c_void_p(0x2000)
    m.bdflag = None
    return m


def test_workspace_size_is_host_arithmetic(femhip):
    a = femhip.fe_plan_workspace_bytes(_mesh(femhip, 2, 100, 150))
    b = femhip.fe_plan_workspace_bytes(_mesh(femhip, 2, 200, 300))
    c = femhip.fe_plan_workspace_bytes(_mesh(femhip, 3, 100, 150))
    assert 0 < a < b and c > a and a % 256 == 0
    assert femhip.fe_solve_workspace_bytes(1000) >= 6 * 8 * 1000


def test_argument_errors_before_any_device_call(femhip):
    lib = femhip._lib
    n = C.c_size_t()
    assert lib.fe_plan_workspace_bytes(None, C.byref(n)) == femhip.FE_EINVAL
    assert lib.fe_plan_workspace_bytes(C.byref(_mesh(femhip, 4)), C.byref(n)) == femhip.FE_EUNSUPPORTED
    assert lib.fe_plan_workspace_bytes(C.byref(_mesh(femhip, 2, 0, 5)), C.byref(n)) == femhip.FE_EINVAL
    big = _mesh(femhip, 3, 10, 2 ** 30)
    assert lib.fe_plan_workspace_bytes(C.byref(big), C.byref(n)) == femhip.FE_EOVERFLOW
    plan, nnz = C.c_void_p(), C.c_int64()
    m = _mesh(femhip)
    # workspace too small, misaligned workspace, missing outputs
    assert lib.fe_plan_create(C.byref(m), C.c_void_p(0x10000), 16, C.byref(plan), C.byref(nnz), None) == femhip.FE_ESIZE
    assert lib.fe_plan_create(C.byref(m), C.c_void_p(0x10010), 1 << 20, C.byref(plan), C.byref(nnz), None) == femhip.FE_EINVAL
    assert lib.fe_plan_create(C.byref(m), C.c_void_p(0x10000), 1 << 20, None, C.byref(nnz), None) == femhip.FE_EINVAL
    assert lib.fe_assemble(None, None, None, None, None, None, None, None, None, None, None, None) == femhip.FE_EINVAL
    assert lib.fe_grad(None, None, None, None, None, None) == femhip.FE_EINVAL
    assert lib.fe_spmv(-1, None, None, None, None, None, None) == femhip.FE_EINVAL
    it, rel = C.c_int32(), C.c_double()
    assert lib.fe_solve(0, None, None, None, None, None, 1e-8, 10, None, 0, C.byref(it), C.byref(rel), None) == femhip.FE_EINVAL
    # the allocation-free solve: missing arguments, and more rows than its fixed array
    assert lib.fe_solve_noalloc(10, None, None, None, None, None, 1e-8, 10, C.byref(it), C.byref(rel), None) == femhip.FE_EINVAL
    fake = [C.c_void_p(0x1000 * (k + 1)) for k in range(5)]
    assert lib.fe_solve_noalloc(femhip.FE_SOLVE_NOALLOC_MAX_N + 1, *fake, 1e-8, 10, C.byref(it), C.byref(rel),
                                None) == femhip.FE_ELIMIT
    assert lib.fe_plan_status(None, None) == femhip.FE_EINVAL
    assert lib.fe_plan_destroy(None) == femhip.FE_OK
