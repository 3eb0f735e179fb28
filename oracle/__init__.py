"""CPU oracle for P1 Poisson assembly, solve and adjoint gradient (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``fe_oracle.c`` (plain C, double precision, single
thread) through ctypes; the GPU library shares no code with it.

Conventions follow the mesh arrays of the paper's Section 1 in structure-of-arrays
form: ``node`` (dim, N) float64, ``elem`` (dim+1, NT) int32 0-based, ``bdflag``
(dim+1, NT) int8 with face a opposite local vertex a.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FN_ZERO, FN_CONST, FN_LINEAR, FN_SINPROD, FN_DUDN_SINPROD, FN_NODAL = range(6)
OK, EINVAL, EMESH, EUNSUPPORTED, ENOCONV = 0, -1, -2, -3, -7


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Fn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c", C.c_double * 4), ("nodal", C.c_void_p)]


@dataclass
class Fn:
    """A data function: kind FN_* with coefficients c (and nodal values for FN_NODAL).

    FN_CONST c0; FN_LINEAR c0 + c1 x + c2 y (+ c3 z); FN_SINPROD c0 prod sin(pi x_i);
    FN_DUDN_SINPROD c0 grad(prod sin(pi x_i)) . n_outward; FN_NODAL piecewise-linear
    interpolant of ``nodal``.
    """

    kind: int = FN_ZERO
    c: tuple = (0.0, 0.0, 0.0, 0.0)
    nodal: np.ndarray | None = None

    def _c(self):
        s = _Fn()
        s.kind = self.kind
        for i, v in enumerate(list(self.c)[:4] + [0.0] * (4 - len(self.c))):
            s.c[i] = float(v)
        if self.nodal is not None:
            self._keep = np.ascontiguousarray(self.nodal, dtype=np.float64)
            s.nodal = self._keep.ctypes.data
        else:
            s.nodal = None
        return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        I64 = C.c_int64
        _lib.oracle_coo_to_csr.argtypes = [I64, I64, I64, P, P, P, P, P, P, P]
        _lib.oracle_local_stiffness.argtypes = [C.c_int, P, P, P, P, P]
        _lib.oracle_assemble.argtypes = [C.c_int, I64, I64, P, P, P, P, P, P, P, I64,
                                         P, P, P, P, P, P, P, P, P]
        _lib.oracle_assemble_robin.argtypes = [C.c_int, I64, I64, P, P, P, P, P, P, P, P, C.c_double, I64,
                                               P, P, P, P, P, P, P, P, P]
        _lib.oracle_assemble_rule.argtypes = [C.c_int, I64, I64, P, P, P, P, P, P, P, P, C.c_double, C.c_int,
                                              I64, P, P, P, P, P, P, P, P, P]
        _lib.oracle_solve.argtypes = [I64, P, P, P, P, P, P, C.c_double, I64, C.c_int, P, P]
        _lib.oracle_grad.argtypes = [C.c_int, I64, I64, P, P, P, P, P]
        _lib.oracle_spmv.argtypes = [I64, P, P, P, P, P]
        for name in ("oracle_coo_to_csr", "oracle_local_stiffness", "oracle_assemble",
                     "oracle_assemble_robin", "oracle_assemble_rule", "oracle_solve", "oracle_grad", "oracle_spmv"):
            getattr(_lib, name).restype = C.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def coo_to_csr(m, n, i, j, s):
    """MATLAB-style sparse(i, j, s, m, n) with 0-based indices -> (rowptr, colind, val)."""
    i = np.ascontiguousarray(i, np.int64)
    j = np.ascontiguousarray(j, np.int64)
    s = np.ascontiguousarray(s, np.float64)
    nz = i.size
    rowptr = np.zeros(m + 1, np.int64)
    colind = np.zeros(max(nz, 1), np.int64)
    val = np.zeros(max(nz, 1), np.float64)
    nnz = np.zeros(1, np.int64)
    st = lib().oracle_coo_to_csr(m, n, nz, _p(i), _p(j), _p(s), _p(rowptr), _p(colind), _p(val), _p(nnz))
    if st:
        raise OracleError(st, "coo_to_csr")
    k = int(nnz[0])
    return rowptr, colind[:k].copy(), val[:k].copy()


def local_stiffness(p):
    """Local stiffness of one simplex with vertex coordinates p[(d+1), d]."""
    p = np.ascontiguousarray(p, np.float64)
    dim = p.shape[1]
    K = np.zeros((dim + 1, dim + 1))
    G = np.zeros((dim + 1, dim))
    meas = np.zeros(1)
    sgn = np.zeros(1)
    st = lib().oracle_local_stiffness(dim, _p(p), _p(K), _p(G), _p(meas), _p(sgn))
    if st:
        raise OracleError(st, "local_stiffness")
    return K, G, float(meas[0])


@dataclass
class Assembled:
    rowptr: np.ndarray
    colind: np.ndarray
    val: np.ndarray
    val_bc: np.ndarray
    b: np.ndarray
    b_load: np.ndarray
    is_d: np.ndarray
    b_scale: np.ndarray

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def dense(self, bc: bool = False):
        n = self.rowptr.size - 1
        A = np.zeros((n, n))
        v = self.val_bc if bc else self.val
        for i in range(n):
            for q in range(self.rowptr[i], self.rowptr[i + 1]):
                A[i, self.colind[q]] += v[q]
        return A

    def diag(self):
        n = self.rowptr.size - 1
        d = np.zeros(n)
        for i in range(n):
            for q in range(self.rowptr[i], self.rowptr[i + 1]):
                if self.colind[q] == i:
                    d[i] = self.val[q]
        return d


# quadrature of the load integrals int_t f phi_a (Section 4)
LOAD_DEFAULT = 0     # three edge midpoints (2-D), symmetric four-point rule (3-D)
LOAD_CENTROID = 1    # one-point rule at the barycentre
LOAD_TRAPEZOID = 2   # vertex (trapezoidal) rule


def assemble(node, elem, bdflag=None, kappa=None, f: Fn | None = None, gD: Fn | None = None,
             gN: Fn | None = None, gR: Fn | None = None, alpha: float = 0.0,
             rule: int = LOAD_DEFAULT) -> Assembled:
    """Assemble A (CSR), the lifted right-hand side b and the boundary data.  Robin
    sides (bdflag 3) use kappa grad(u).n + alpha u = g_R; ``rule`` picks the load
    quadrature (LOAD_*)."""
    node = np.ascontiguousarray(node, np.float64)
    elem = np.ascontiguousarray(elem, np.int32)
    dim = node.shape[0]
    N = node.shape[1]
    NT = elem.shape[1]
    bd = None if bdflag is None else np.ascontiguousarray(bdflag, np.int8)
    kp = None if kappa is None else np.ascontiguousarray(kappa, np.float64)
    cap = max((dim + 1) ** 2 * NT, 1)
    rowptr = np.zeros(N + 1, np.int64)
    colind = np.zeros(cap, np.int64)
    val = np.zeros(cap)
    val_bc = np.zeros(cap)
    b = np.zeros(N)
    b_load = np.zeros(N)
    is_d = np.zeros(N, np.uint8)
    b_scale = np.zeros(N)
    nnz = np.zeros(1, np.int64)
    fs = [x._c() if x is not None else None for x in (f, gD, gN, gR)]
    refs = [C.byref(x) if x is not None else None for x in fs]
    st = lib().oracle_assemble_rule(dim, N, NT, _p(node), _p(elem), _p(bd), _p(kp), refs[0], refs[1],
                                    refs[2], refs[3], C.c_double(alpha), int(rule), cap, _p(rowptr), _p(colind),
                                    _p(val), _p(val_bc), _p(b), _p(b_load), _p(is_d), _p(b_scale), _p(nnz))
    if st:
        raise OracleError(st, "assemble")
    k = int(nnz[0])
    return Assembled(rowptr, colind[:k].copy(), val[:k].copy(), val_bc[:k].copy(), b, b_load,
                     is_d, b_scale)


def solve(asm: Assembled, u0=None, rtol: float = 1e-12, maxit: int = 100000, method: str = "auto"):
    """Solve A_bc u = b; returns (u, iters, relres). ``u0`` supplies Dirichlet values."""
    N = asm.b.size
    u = np.zeros(N) if u0 is None else np.array(u0, np.float64, copy=True)
    d = asm.is_d.astype(bool)
    u[d] = asm.b[d]
    if method == "auto":
        method = "direct" if int((~d).sum()) <= 6000 else "cg"
    m = 0 if method == "direct" else 1
    iters = np.zeros(1, np.int64)
    rel = np.zeros(1)
    st = lib().oracle_solve(N, _p(asm.rowptr), _p(asm.colind), _p(asm.val_bc), _p(asm.b), _p(asm.is_d),
                            _p(u), rtol, maxit, m, _p(iters), _p(rel))
    if st:
        raise OracleError(st, "solve")
    return u, int(iters[0]), float(rel[0])


def solve_rhs(asm: Assembled, rhs, rtol: float = 1e-12, method: str = "auto"):
    """Solve A_bc x = rhs with rhs already zero at Dirichlet rows (adjoint systems)."""
    tmp = Assembled(asm.rowptr, asm.colind, asm.val, asm.val_bc, np.ascontiguousarray(rhs, np.float64),
                    asm.b_load, asm.is_d, asm.b_scale)
    return solve(tmp, np.zeros_like(tmp.b), rtol=rtol, method=method)


def grad(node, elem, u, lam):
    """g_t = -|t| grad(lam_h) . grad(u_h) on each element."""
    node = np.ascontiguousarray(node, np.float64)
    elem = np.ascontiguousarray(elem, np.int32)
    u = np.ascontiguousarray(u, np.float64)
    lam = np.ascontiguousarray(lam, np.float64)
    g = np.zeros(elem.shape[1])
    st = lib().oracle_grad(node.shape[0], node.shape[1], elem.shape[1], _p(node), _p(elem), _p(u),
                           _p(lam), _p(g))
    if st:
        raise OracleError(st, "grad")
    return g


def spmv(rowptr, colind, val, x):
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colind = np.ascontiguousarray(colind, np.int64)
    val = np.ascontiguousarray(val, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(rowptr.size - 1)
    lib().oracle_spmv(rowptr.size - 1, _p(rowptr), _p(colind), _p(val), _p(x), _p(y))
    return y


def objective_and_grad(node, elem, bdflag, kappa, u_obs, f=None, gD=None, gN=None, rtol=1e-14):
    """J = 1/2 ||u - u_obs||^2 and dJ/dkappa by the adjoint method."""
    asm = assemble(node, elem, bdflag, kappa, f, gD, gN)
    u, _, _ = solve(asm, rtol=rtol)
    r = u - u_obs
    J = 0.5 * float(r @ r)
    rhs = np.where(asm.is_d.astype(bool), 0.0, r)
    lam, _, _ = solve_rhs(asm, rhs, rtol=rtol)
    return J, grad(node, elem, u, lam), u, lam


def measures(node, elem):
    """|t| of every simplex: |det(x_1 - x_0, ..., x_d - x_0)| / d!."""
    node = np.asarray(node, np.float64)
    elem = np.asarray(elem)
    dim = node.shape[0]
    out = np.zeros(elem.shape[1])
    for t in range(elem.shape[1]):
        x0 = node[:, elem[0, t]]
        M = np.array([node[:, elem[a, t]] - x0 for a in range(1, dim + 1)])
        out[t] = abs(np.linalg.det(M)) / (2.0 if dim == 2 else 6.0)
    return out


def neumann_solve(asm: Assembled, node, elem, rtol: float = 1e-13, method: str = "auto"):
    """Pure Neumann problem (Section 3.3, equations (compatible) and (meanb)).

    1. b <- b - mean(b), the discrete compatibility condition;
    2. fix u = 0 at the first vertex and solve A(free, free) u(free) = b(free) with
       free = all other vertices (equation (directsolve) with freeNode = 2:N);
    3. shift u by c = sum_t |t| mean(u(elem_t)) / sum_t |t|, so that u has zero mean.
    Returns (u, iters, relres, mean_b)."""
    if asm.is_d.any():
        raise ValueError("a pure Neumann problem has no Dirichlet vertex")
    N = asm.b.size
    mean_b = float(asm.b.sum()) / N
    b = asm.b - mean_b
    b[0] = 0.0
    pin = np.zeros(N, np.uint8)
    pin[0] = 1
    val_pin = asm.val.copy()
    for i in range(N):
        for q in range(asm.rowptr[i], asm.rowptr[i + 1]):
            if i == 0:
                val_pin[q] = 1.0 if asm.colind[q] == 0 else 0.0
            elif asm.colind[q] == 0:
                val_pin[q] = 0.0
    tmp = Assembled(asm.rowptr, asm.colind, asm.val, val_pin, b, asm.b_load, pin, asm.b_scale)
    u, it, rel = solve(tmp, np.zeros(N), rtol=rtol, method=method)
    area = measures(node, elem)
    elem = np.asarray(elem)
    c = float(np.sum(area * u[elem].mean(axis=0))) / float(np.sum(area))
    return u - c, it, rel, mean_b
