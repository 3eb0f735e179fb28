"""ctypes binding of the HIP library ``libfemhip.so`` (C interface in include/femhip.h).

The functions named ``fe_*`` mirror the C entry points one to one (argument
marshalling only: torch tensors supply device pointers, the current torch stream
supplies the HIP stream).  :class:`Plan`, :func:`solve` and :class:`PoissonSolve`
are conveniences built only from those calls.  Every step of the computation runs
in the library's kernels; if the library is missing this module fails on import.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfemhip.so")

FE_OK, FE_EINVAL, FE_EMESH, FE_EUNSUPPORTED, FE_EOVERFLOW = 0, -1, -2, -3, -4
FE_ESIZE, FE_EHIP, FE_ENOCONV, FE_ELIMIT = -5, -6, -7, -8
FE_FN_ZERO, FE_FN_CONST, FE_FN_LINEAR, FE_FN_SINPROD, FE_FN_DUDN_SINPROD, FE_FN_NODAL = range(6)
FE_LOAD_DEFAULT, FE_LOAD_CENTROID, FE_LOAD_TRAPEZOID = range(3)

# Entry points declared in include/femhip.h.
ENTRY_POINTS = (
    "fe_version", "fe_status_string", "fe_plan_workspace_bytes", "fe_plan_create", "fe_plan_pattern",
    "fe_plan_set_launch", "fe_plan_get_info", "fe_plan_status", "fe_plan_destroy", "fe_assemble", "fe_assemble_robin",
    "fe_assemble_quad", "fe_plan_upper", "fe_assemble_upper", "fe_spmv_sym", "fe_solve_sym", "fe_spmv",
    "fe_select", "fe_solve_workspace_bytes", "fe_solve", "fe_solve_noalloc", "fe_neumann_workspace_bytes", "fe_neumann_solve",
    "fe_grad", "fe_batch_solve_workspace_bytes",
    "fe_batch_solve", "fe_batch_create", "fe_batch_set_grid", "fe_batch_get_info", "fe_batch_assemble_solve",
    "fe_batch_destroy", "fe_prof_enable", "fe_prof_read",
)


class fe_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_node", C.c_int64), ("n_elem", C.c_int64),
                ("node", C.c_void_p), ("elem", C.c_void_p), ("bdflag", C.c_void_p)]


class fe_fn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c", C.c_double * 4), ("nodal", C.c_void_p)]


class fe_plan_info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_node", C.c_int64), ("n_elem", C.c_int64), ("nnz", C.c_int64),
                ("n_inc", C.c_int64), ("max_row", C.c_int32), ("max_deg", C.c_int32),
                ("n_dirichlet", C.c_int64), ("sort_runs", C.c_int32), ("n_long", C.c_int32)]


class fe_batch_info(C.Structure):
    _fields_ = [("n_inst", C.c_int32), ("n_units", C.c_int32), ("n_rows", C.c_int64), ("grid", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("max_blocks_per_cu", C.c_int32), ("units_per_step", C.c_int32),
                ("cooperative", C.c_int32),
                ("captures", C.c_int32)]


class fe_prof_entry(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double), ("min_ms", C.c_double),
                ("max_ms", C.c_double)]


class FemhipError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1804_05156_amd.build.build() "
                          "(there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "fe_version": ([], C.c_char_p),
        "fe_status_string": ([C.c_int], C.c_char_p),
        "fe_plan_workspace_bytes": ([C.POINTER(fe_mesh), C.POINTER(SZ)], C.c_int),
        "fe_plan_create": ([C.POINTER(fe_mesh), P, SZ, C.POINTER(P), C.POINTER(I64), P], C.c_int),
        "fe_plan_pattern": ([P, P, P, P], C.c_int),
        "fe_plan_set_launch": ([P, I32], C.c_int),
        "fe_plan_get_info": ([P, C.POINTER(fe_plan_info)], C.c_int),
        "fe_plan_status": ([P, P], C.c_int),
        "fe_plan_destroy": ([P], C.c_int),
        "fe_assemble": ([P, P, P, C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), P, P, P, P, P, P],
                        C.c_int),
        "fe_assemble_robin": ([P, P, P, C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), D,
                               P, P, P, P, P, P], C.c_int),
        "fe_assemble_quad": ([P, P, P, C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), D,
                              I32, P, P, P, P, P, P], C.c_int),
        "fe_spmv": ([I64, P, P, P, P, P, P], C.c_int),
        "fe_plan_upper": ([P, P, P, P, P, P, C.POINTER(I64), P], C.c_int),
        "fe_assemble_upper": ([P, P, P, P, C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), D,
                               I32, P, P, P, P, P, P], C.c_int),
        "fe_spmv_sym": ([I64, P, P, P, P, P, P, P], C.c_int),
        "fe_solve_sym": ([I64, P, P, P, P, P, P, D, I32, P, SZ, C.POINTER(I32), C.POINTER(D), P], C.c_int),
        "fe_solve_workspace_bytes": ([I64, C.POINTER(SZ)], C.c_int),
        "fe_solve": ([I64, P, P, P, P, P, D, I32, P, SZ, C.POINTER(I32), C.POINTER(D), P], C.c_int),
        "fe_solve_noalloc": ([I64, P, P, P, P, P, D, I32, C.POINTER(I32), C.POINTER(D), P], C.c_int),
        "fe_grad": ([P, P, P, P, P, P], C.c_int),
        "fe_neumann_workspace_bytes": ([P, I64, C.POINTER(SZ)], C.c_int),
        "fe_neumann_solve": ([P, P, P, P, P, P, P, D, I32, P, SZ, C.POINTER(I32), C.POINTER(D), C.POINTER(D), P],
                             C.c_int),
        "fe_select": ([I64, P, P, P, P, P], C.c_int),
        "fe_batch_solve_workspace_bytes": ([I64, I32, C.POINTER(SZ)], C.c_int),
        "fe_batch_solve": ([I32, P, P, P, P, P, P, D, I32, I32, I32, P, SZ, P, P, P], C.c_int),
        "fe_batch_create": ([P, I32, P, I32, I32, P, SZ, C.POINTER(P), P], C.c_int),
        "fe_batch_set_grid": ([P, I32, I32], C.c_int),
        "fe_batch_get_info": ([P, C.POINTER(fe_batch_info)], C.c_int),
        "fe_batch_assemble_solve": ([P, P, P, C.POINTER(fe_fn), C.POINTER(fe_fn), C.POINTER(fe_fn), P, P, P, P, P,
                                     P, D, I32, P, P, P], C.c_int),
        "fe_batch_destroy": ([P], C.c_int),
        "fe_prof_enable": ([C.c_int], C.c_int),
        "fe_prof_read": ([C.POINTER(fe_prof_entry), I32, C.POINTER(I32)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def status_string(code: int) -> str:
    return _lib.fe_status_string(code).decode()


def version() -> str:
    return _lib.fe_version().decode()


def _check(rc: int, what: str):
    if rc != FE_OK:
        raise FemhipError(rc, what)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Fn:
    """Data function: kind FE_FN_* with coefficients c; ``nodal`` a CUDA float64 tensor."""

    kind: int = FE_FN_ZERO
    c: tuple = (0.0, 0.0, 0.0, 0.0)
    nodal: torch.Tensor | None = None

    def struct(self) -> fe_fn:
        s = fe_fn()
        s.kind = self.kind
        cc = list(self.c)[:4] + [0.0] * (4 - len(list(self.c)[:4]))
        for k in range(4):
            s.c[k] = float(cc[k])
        s.nodal = _ptr(self.nodal, torch.float64, "nodal") if self.nodal is not None else None
        return s


def _fnref(f: Fn | None):
    return None if f is None else C.byref(f.struct())


def make_mesh(node: torch.Tensor, elem: torch.Tensor, bdflag: torch.Tensor | None = None) -> fe_mesh:
    m = fe_mesh()
    m.dim = int(node.shape[0])
    m.n_node = int(node.shape[1])
    m.n_elem = int(elem.shape[1])
    m.node = _ptr(node, torch.float64, "node")
    m.elem = _ptr(elem, torch.int32, "elem")
    m.bdflag = _ptr(bdflag, torch.int8, "bdflag") if bdflag is not None else None
    return m


# ----------------------------------------------------------------------------- C entry points
def fe_plan_workspace_bytes(mesh: fe_mesh) -> int:
    n = C.c_size_t()
    _check(_lib.fe_plan_workspace_bytes(C.byref(mesh), C.byref(n)), "fe_plan_workspace_bytes")
    return int(n.value)


def fe_plan_create(mesh: fe_mesh, ws: torch.Tensor, stream=None):
    plan = C.c_void_p()
    nnz = C.c_int64()
    _check(_lib.fe_plan_create(C.byref(mesh), _ptr(ws, torch.uint8, "ws"), ws.numel(), C.byref(plan),
                               C.byref(nnz), _stream(stream)), "fe_plan_create")
    return plan, int(nnz.value)


def fe_plan_pattern(plan, rowptr: torch.Tensor, colind: torch.Tensor, stream=None):
    _check(_lib.fe_plan_pattern(plan, _ptr(rowptr, torch.int32, "rowptr"), _ptr(colind, torch.int32, "colind"),
                                _stream(stream)), "fe_plan_pattern")


def fe_plan_set_launch(plan, rows_per_block: int):
    _check(_lib.fe_plan_set_launch(plan, int(rows_per_block)), "fe_plan_set_launch")


def fe_plan_get_info(plan) -> dict:
    info = fe_plan_info()
    _check(_lib.fe_plan_get_info(plan, C.byref(info)), "fe_plan_get_info")
    return {k: getattr(info, k) for k, _ in fe_plan_info._fields_}


def fe_plan_status(plan, stream=None) -> int:
    return int(_lib.fe_plan_status(plan, _stream(stream)))


def fe_plan_destroy(plan):
    _check(_lib.fe_plan_destroy(plan), "fe_plan_destroy")


def fe_assemble(plan, node, kappa, f: Fn | None, gD: Fn | None, gN: Fn | None, val, val_bc, b, b_load, is_d,
                stream=None):
    _check(_lib.fe_assemble(plan, _ptr(node, torch.float64, "node"), _ptr(kappa, torch.float64, "kappa"),
                            _fnref(f), _fnref(gD), _fnref(gN), _ptr(val, torch.float64, "val"),
                            _ptr(val_bc, torch.float64, "val_bc"), _ptr(b, torch.float64, "b"),
                            _ptr(b_load, torch.float64, "b_load"), _ptr(is_d, torch.uint8, "is_dirichlet"),
                            _stream(stream)), "fe_assemble")


def fe_assemble_robin(plan, node, kappa, f: Fn | None, gD: Fn | None, gN: Fn | None, gR: Fn | None,
                      robin_alpha: float, val, val_bc, b, b_load, is_d, stream=None):
    _check(_lib.fe_assemble_robin(plan, _ptr(node, torch.float64, "node"), _ptr(kappa, torch.float64, "kappa"),
                                  _fnref(f), _fnref(gD), _fnref(gN), _fnref(gR), float(robin_alpha),
                                  _ptr(val, torch.float64, "val"), _ptr(val_bc, torch.float64, "val_bc"),
                                  _ptr(b, torch.float64, "b"), _ptr(b_load, torch.float64, "b_load"),
                                  _ptr(is_d, torch.uint8, "is_dirichlet"), _stream(stream)), "fe_assemble_robin")


def fe_assemble_quad(plan, node, kappa, f: Fn | None, gD: Fn | None, gN: Fn | None, gR: Fn | None,
                     robin_alpha: float, load_rule: int, val, val_bc, b, b_load, is_d, stream=None):
    _check(_lib.fe_assemble_quad(plan, _ptr(node, torch.float64, "node"), _ptr(kappa, torch.float64, "kappa"),
                                 _fnref(f), _fnref(gD), _fnref(gN), _fnref(gR), float(robin_alpha), int(load_rule),
                                 _ptr(val, torch.float64, "val"), _ptr(val_bc, torch.float64, "val_bc"),
                                 _ptr(b, torch.float64, "b"), _ptr(b_load, torch.float64, "b_load"),
                                 _ptr(is_d, torch.uint8, "is_dirichlet"), _stream(stream)), "fe_assemble_quad")


def fe_spmv(rowptr, colind, val, x, y, stream=None):
    _check(_lib.fe_spmv(rowptr.numel() - 1, _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                        _ptr(val, torch.float64), _ptr(x, torch.float64), _ptr(y, torch.float64), _stream(stream)),
           "fe_spmv")


def fe_plan_upper(plan, rowptr, colind, rowptr_u, colind_u=None, vidx=None, stream=None) -> int:
    """Pattern of triu(A) and the value index of A's entries into it; returns nnz_u.
    With colind_u = vidx = None only rowptr_u is written (to size the others)."""
    n = C.c_int64()
    _check(_lib.fe_plan_upper(plan, _ptr(rowptr, torch.int32, "rowptr"), _ptr(colind, torch.int32, "colind"),
                              _ptr(rowptr_u, torch.int32, "rowptr_u"), _ptr(colind_u, torch.int32, "colind_u"),
                              _ptr(vidx, torch.int32, "vidx"), C.byref(n), _stream(stream)), "fe_plan_upper")
    return int(n.value)


def fe_assemble_upper(plan, rowptr_u, node, kappa, f: Fn | None, gD: Fn | None, gN: Fn | None, gR: Fn | None,
                      robin_alpha: float, load_rule: int, val_u, val_bc_u, b, b_load, is_d, stream=None):
    _check(_lib.fe_assemble_upper(plan, _ptr(rowptr_u, torch.int32, "rowptr_u"), _ptr(node, torch.float64, "node"),
                                  _ptr(kappa, torch.float64, "kappa"), _fnref(f), _fnref(gD), _fnref(gN), _fnref(gR),
                                  float(robin_alpha), int(load_rule), _ptr(val_u, torch.float64, "val_u"),
                                  _ptr(val_bc_u, torch.float64, "val_bc_u"), _ptr(b, torch.float64, "b"),
                                  _ptr(b_load, torch.float64, "b_load"), _ptr(is_d, torch.uint8, "is_dirichlet"),
                                  _stream(stream)), "fe_assemble_upper")


def fe_spmv_sym(rowptr, colind, vidx, val_u, x, y, stream=None):
    _check(_lib.fe_spmv_sym(rowptr.numel() - 1, _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                            _ptr(vidx, torch.int32), _ptr(val_u, torch.float64), _ptr(x, torch.float64),
                            _ptr(y, torch.float64), _stream(stream)), "fe_spmv_sym")


def fe_solve_sym(rowptr, colind, vidx, val_u, b, u, rtol: float, maxit: int, ws, stream=None):
    it = C.c_int32()
    rel = C.c_double()
    rc = _lib.fe_solve_sym(rowptr.numel() - 1, _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                           _ptr(vidx, torch.int32), _ptr(val_u, torch.float64), _ptr(b, torch.float64),
                           _ptr(u, torch.float64), float(rtol), int(maxit), _ptr(ws, torch.uint8, "ws"), ws.numel(),
                           C.byref(it), C.byref(rel), _stream(stream))
    _check(rc, "fe_solve_sym")
    return int(it.value), float(rel.value), rc


def fe_select(mask, a, b, out, stream=None):
    _check(_lib.fe_select(out.numel(), _ptr(mask, torch.uint8, "mask"), _ptr(a, torch.float64, "a"),
                          _ptr(b, torch.float64, "b"), _ptr(out, torch.float64, "out"), _stream(stream)), "fe_select")


def fe_solve_workspace_bytes(n: int) -> int:
    s = C.c_size_t()
    _check(_lib.fe_solve_workspace_bytes(n, C.byref(s)), "fe_solve_workspace_bytes")
    return int(s.value)


def fe_solve(rowptr, colind, val, b, u, rtol: float, maxit: int, ws, stream=None, allow_noconv=False):
    it = C.c_int32()
    rel = C.c_double()
    rc = _lib.fe_solve(rowptr.numel() - 1, _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                       _ptr(val, torch.float64), _ptr(b, torch.float64), _ptr(u, torch.float64), float(rtol),
                       int(maxit), _ptr(ws, torch.uint8, "ws"), ws.numel(), C.byref(it), C.byref(rel),
                       _stream(stream))
    if rc == FE_ENOCONV and allow_noconv:
        return int(it.value), float(rel.value), rc
    _check(rc, "fe_solve")
    return int(it.value), float(rel.value), rc


FE_SOLVE_NOALLOC_MAX_N = 1310720


def fe_solve_noalloc(rowptr, colind, val, b, u, rtol: float, maxit: int, stream=None, allow_noconv=False):
    it = C.c_int32()
    rel = C.c_double()
    rc = _lib.fe_solve_noalloc(rowptr.numel() - 1, _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                               _ptr(val, torch.float64), _ptr(b, torch.float64), _ptr(u, torch.float64),
                               float(rtol), int(maxit), C.byref(it), C.byref(rel), _stream(stream))
    if rc == FE_ENOCONV and allow_noconv:
        return int(it.value), float(rel.value), rc
    _check(rc, "fe_solve_noalloc")
    return int(it.value), float(rel.value), rc


def fe_neumann_workspace_bytes(plan, nnz: int) -> int:
    s = C.c_size_t()
    _check(_lib.fe_neumann_workspace_bytes(plan, int(nnz), C.byref(s)), "fe_neumann_workspace_bytes")
    return int(s.value)


def fe_neumann_solve(plan, node, rowptr, colind, val, b, u, rtol: float, maxit: int, ws, stream=None,
                     allow_noconv=False):
    """Returns (iters, relres, mean_b, status)."""
    it = C.c_int32()
    rel = C.c_double()
    mb = C.c_double()
    rc = _lib.fe_neumann_solve(plan, _ptr(node, torch.float64, "node"), _ptr(rowptr, torch.int32),
                               _ptr(colind, torch.int32), _ptr(val, torch.float64, "val"), _ptr(b, torch.float64, "b"),
                               _ptr(u, torch.float64, "u"), float(rtol), int(maxit), _ptr(ws, torch.uint8, "ws"),
                               ws.numel(), C.byref(it), C.byref(rel), C.byref(mb), _stream(stream))
    if not (rc == FE_ENOCONV and allow_noconv):
        _check(rc, "fe_neumann_solve")
    return int(it.value), float(rel.value), float(mb.value), rc


def fe_grad(plan, node, u, lam, g, stream=None):
    _check(_lib.fe_grad(plan, _ptr(node, torch.float64, "node"), _ptr(u, torch.float64, "u"),
                        _ptr(lam, torch.float64, "lam"), _ptr(g, torch.float64, "g"), _stream(stream)), "fe_grad")


def fe_batch_solve_workspace_bytes(n: int, n_inst: int) -> int:
    s = C.c_size_t()
    _check(_lib.fe_batch_solve_workspace_bytes(n, n_inst, C.byref(s)), "fe_batch_solve_workspace_bytes")
    return int(s.value)


def _i64_array(off):
    off = [int(v) for v in off]
    return (C.c_int64 * len(off))(*off)


def fe_batch_solve(inst_row_off, rowptr, colind, val, b, u, rtol: float, maxit: int, ws, blocks_per_cu: int = 0,
                   units_per_step: int = 0, stream=None, allow_noconv=False):
    """Returns (iters list, relres list, status)."""
    n_inst = len(inst_row_off) - 1
    it = (C.c_int32 * n_inst)()
    rel = (C.c_double * n_inst)()
    rc = _lib.fe_batch_solve(n_inst, _i64_array(inst_row_off), _ptr(rowptr, torch.int32), _ptr(colind, torch.int32),
                             _ptr(val, torch.float64), _ptr(b, torch.float64), _ptr(u, torch.float64), float(rtol),
                             int(maxit), int(blocks_per_cu), int(units_per_step), _ptr(ws, torch.uint8, "ws"),
                             ws.numel(), it, rel, _stream(stream))
    if not (rc == FE_ENOCONV and allow_noconv):
        _check(rc, "fe_batch_solve")
    return list(it), list(rel), rc


def fe_batch_create(plan, inst_node_off, ws, blocks_per_cu: int = 0, units_per_step: int = 0, stream=None):
    h = C.c_void_p()
    _check(_lib.fe_batch_create(plan, len(inst_node_off) - 1, _i64_array(inst_node_off), int(blocks_per_cu),
                                int(units_per_step), _ptr(ws, torch.uint8, "ws"), ws.numel(), C.byref(h),
                                _stream(stream)),
           "fe_batch_create")
    return h


def fe_batch_set_grid(batch, blocks_per_cu: int, units_per_step: int = 0):
    _check(_lib.fe_batch_set_grid(batch, int(blocks_per_cu), int(units_per_step)), "fe_batch_set_grid")


def fe_batch_get_info(batch) -> dict:
    info = fe_batch_info()
    _check(_lib.fe_batch_get_info(batch, C.byref(info)), "fe_batch_get_info")
    return {k: getattr(info, k) for k, _ in fe_batch_info._fields_}


def fe_batch_assemble_solve(batch, node, kappa, f, gD, gN, rowptr, colind, val, val_bc, b, u, rtol: float,
                            maxit: int, n_inst: int, stream=None, allow_noconv=False):
    it = (C.c_int32 * n_inst)()
    rel = (C.c_double * n_inst)()
    rc = _lib.fe_batch_assemble_solve(batch, _ptr(node, torch.float64, "node"), _ptr(kappa, torch.float64, "kappa"),
                                      _fnref(f), _fnref(gD), _fnref(gN), _ptr(rowptr, torch.int32),
                                      _ptr(colind, torch.int32), _ptr(val, torch.float64, "val"),
                                      _ptr(val_bc, torch.float64, "val_bc"), _ptr(b, torch.float64, "b"),
                                      _ptr(u, torch.float64, "u"), float(rtol), int(maxit), it, rel, _stream(stream))
    if not (rc == FE_ENOCONV and allow_noconv):
        _check(rc, "fe_batch_assemble_solve")
    return list(it), list(rel), rc


def fe_batch_destroy(batch):
    _check(_lib.fe_batch_destroy(batch), "fe_batch_destroy")


def fe_prof_enable(on: bool):
    _check(_lib.fe_prof_enable(1 if on else 0), "fe_prof_enable")


def fe_prof_read() -> dict:
    """{kernel name: {"launches", "total_ms", "min_ms", "max_ms", "avg_ms"}} since the last read."""
    cap = 64
    buf = (fe_prof_entry * cap)()
    n = C.c_int32()
    _check(_lib.fe_prof_read(buf, cap, C.byref(n)), "fe_prof_read")
    out = {}
    for e in buf[:min(n.value, cap)]:
        out[e.name.decode()] = {"launches": int(e.launches), "total_ms": e.total_ms, "min_ms": e.min_ms,
                                "max_ms": e.max_ms, "avg_ms": e.total_ms / max(e.launches, 1)}
    return out


# ----------------------------------------------------------------------------- conveniences
@dataclass
class Assembly:
    val: torch.Tensor
    val_bc: torch.Tensor | None
    b: torch.Tensor
    b_load: torch.Tensor | None
    is_dirichlet: torch.Tensor | None


class Plan:
    """Symbolic phase of one mesh topology plus the CSR pattern of its matrix.

    node (dim, N) float64, elem (dim+1, NT) int32 and bdflag (dim+1, NT) int8 are
    CUDA tensors; elem and bdflag are kept alive by the plan.
    """

    def __init__(self, node: torch.Tensor, elem: torch.Tensor, bdflag: torch.Tensor | None = None, stream=None):
        self.node = node
        self.elem = elem
        self.bdflag = bdflag
        self.dim = int(node.shape[0])
        self.N = int(node.shape[1])
        self.NT = int(elem.shape[1])
        self.mesh = make_mesh(node, elem, bdflag)
        self.ws = torch.empty(fe_plan_workspace_bytes(self.mesh), dtype=torch.uint8, device=node.device)
        self.handle = None
        self.handle, self.nnz = fe_plan_create(self.mesh, self.ws, stream)
        self.rowptr = torch.empty(self.N + 1, dtype=torch.int32, device=node.device)
        self.colind = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=node.device)
        fe_plan_pattern(self.handle, self.rowptr, self.colind, stream)
        self.info = fe_plan_get_info(self.handle)
        self._solve_ws = None

    def assemble(self, kappa=None, f: Fn | None = None, gD: Fn | None = None, gN: Fn | None = None, node=None,
                 outputs: str = "all", stream=None, out: Assembly | None = None, gR: Fn | None = None,
                 robin_alpha: float = 0.0, load_rule: int = FE_LOAD_DEFAULT) -> Assembly:
        """outputs: "all" (val, val_bc, b, b_load, is_dirichlet) or "min" (val, b).  gR and
        robin_alpha are the Robin data (kappa grad(u).n + robin_alpha u = gR on bdflag-3 sides);
        load_rule is the quadrature of the load integrals (FE_LOAD_*)."""
        node = self.node if node is None else node
        dev = node.device
        if out is None:
            full = outputs == "all"
            out = Assembly(
                torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev),
                torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev) if full else None,
                torch.empty(self.N, dtype=torch.float64, device=dev),
                torch.empty(self.N, dtype=torch.float64, device=dev) if full else None,
                torch.empty(self.N, dtype=torch.uint8, device=dev) if full else None)
        if load_rule != FE_LOAD_DEFAULT:
            fe_assemble_quad(self.handle, node, kappa, f, gD, gN, gR, robin_alpha, load_rule, out.val, out.val_bc,
                             out.b, out.b_load, out.is_dirichlet, stream)
        elif gR is None and robin_alpha == 0.0:
            fe_assemble(self.handle, node, kappa, f, gD, gN, out.val, out.val_bc, out.b, out.b_load,
                        out.is_dirichlet, stream)
        else:
            fe_assemble_robin(self.handle, node, kappa, f, gD, gN, gR, robin_alpha, out.val, out.val_bc, out.b,
                              out.b_load, out.is_dirichlet, stream)
        return out

    def check(self, stream=None):
        _check(fe_plan_status(self.handle, stream), "kernel status")

    def set_launch(self, rows_per_block: int):
        """Rows per workgroup of the numeric row kernels (64, 128, 256; 0 = default)."""
        fe_plan_set_launch(self.handle, rows_per_block)

    def solve_workspace(self):
        if self._solve_ws is None:
            self._solve_ws = torch.empty(fe_solve_workspace_bytes(self.N), dtype=torch.uint8, device=self.node.device)
        return self._solve_ws

    def solve(self, asm: Assembly, u0=None, rtol=1e-10, maxit=100000, rhs=None, stream=None):
        """Solve val_bc u = rhs (default asm.b); u0 defaults to b at Dirichlet rows, 0 elsewhere."""
        b = asm.b if rhs is None else rhs
        if u0 is None:
            u = torch.empty_like(b)
            fe_select(asm.is_dirichlet, b, None, u, stream)
        else:
            u = u0.clone()
        it, rel, _ = fe_solve(self.rowptr, self.colind, asm.val_bc, b, u, rtol, maxit, self.solve_workspace(),
                              stream)
        return u, it, rel

    def neumann_solve(self, asm: Assembly, rtol=1e-10, maxit=100000, node=None, stream=None):
        """Pure Neumann problem: zero-mean u with A u = b - mean(b); returns (u, iters, relres, mean_b)."""
        ws = torch.empty(fe_neumann_workspace_bytes(self.handle, self.nnz), dtype=torch.uint8, device=asm.b.device)
        u = torch.empty_like(asm.b)
        it, rel, mb, _ = fe_neumann_solve(self.handle, self.node if node is None else node, self.rowptr,
                                          self.colind, asm.val, asm.b, u, rtol, maxit, ws, stream)
        return u, it, rel, mb

    def grad(self, u, lam, node=None, stream=None):
        g = torch.empty(self.NT, dtype=torch.float64, device=u.device)
        fe_grad(self.handle, self.node if node is None else node, u, lam, g, stream)
        return g

    def close(self):
        """Release the host-side plan object now (the workspace is a tensor of this object)."""
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.fe_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def solve(rowptr, colind, val, b, u0, rtol=1e-10, maxit=100000, stream=None):
    """Jacobi-PCG on a CSR matrix; returns (u, iterations, final residual ratio)."""
    n = rowptr.numel() - 1
    ws = torch.empty(fe_solve_workspace_bytes(n), dtype=torch.uint8, device=b.device)
    u = u0.clone()
    it, rel, _ = fe_solve(rowptr, colind, val, b, u, rtol, maxit, ws, stream)
    return u, it, rel


class PoissonSolve(torch.autograd.Function):
    """u = solution of the P1 problem for coefficient kappa; backward gives dJ/dkappa.

    forward(kappa, plan, f, gD, gN, rtol): assemble with kappa, solve A_bc u = b.
    backward(dJ/du): solve A_bc lam = dJ/du (zero at Dirichlet rows), then
    dJ/dkappa_t = -|t| grad(lam_h) . grad(u_h) from the adjoint kernel.
    """

    @staticmethod
    def forward(ctx, kappa, plan: Plan, f=None, gD=None, gN=None, rtol=1e-12):
        asm = plan.assemble(kappa.detach().contiguous(), f, gD, gN)
        # a kappa that is not positive and finite, or a degenerate element, is found by
        # the numeric kernel; report it here rather than solve a meaningless system
        plan.check()
        u, it, rel = plan.solve(asm, rtol=rtol)
        ctx.plan = plan
        ctx.asm = asm
        ctx.rtol = rtol
        ctx.save_for_backward(u)
        ctx.iters = it
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        plan, asm = ctx.plan, ctx.asm
        rhs = torch.empty_like(u)
        fe_select(asm.is_dirichlet, None, grad_u.contiguous(), rhs)
        lam, _, _ = plan.solve(asm, u0=torch.zeros_like(rhs), rtol=ctx.rtol, rhs=rhs)
        g = plan.grad(u, lam)
        return g, None, None, None, None, None
