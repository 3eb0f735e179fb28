"""Helpers for the GPU parity tests: move meshes to the device, run the library
through its C interface, and compare with the CPU oracle.

Tolerances (FP64): the stored pattern must match bit for bit; a value a_ij must
satisfy |a_gpu - a_oracle| <= tol * sqrt(a_ii a_jj) (oracle diagonals).  Each
element contribution obeys |K_t[i][j]| <= sqrt(K_t[i][i] K_t[j][j]) (K_t is
positive semidefinite), and by Cauchy-Schwarz the sum over t of those bounds is at
most sqrt(a_ii a_jj), so this scale bounds the forward rounding error of any
summation route.  For b the scale is the oracle's sum of |load and Neumann terms|
plus sum_{Dirichlet j} sqrt(a_ii a_jj) |g_D(x_j)| (the lifting may be summed
element by element), and |g_D(x_i)| at Dirichlet rows.  The two sides evaluate the
data functions by different routes (sinpi on the GPU, sin(pi*x) in the oracle), so
near a zero of f their values differ by ~1e-16 |f|max, not relative to f(x); the b
scale therefore also holds the load of the bound |f|max (and |g_N|max on Neumann
sides), computed by the oracle with constant data, and |g_D|max enters the lifting
and Dirichlet-row scales.  tol = 1e-12.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

TOL = 1e-12


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(m, dev="cuda"):
    return (torch.from_numpy(np.ascontiguousarray(m.node)).to(dev),
            torch.from_numpy(np.ascontiguousarray(m.elem)).to(dev),
            torch.from_numpy(np.ascontiguousarray(m.bdflag)).to(dev),
            None if m.kappa is None else torch.from_numpy(np.ascontiguousarray(m.kappa)).to(dev))


def fns(kind_f=None, kind_gd=None, kind_gn=None):
    """Build matching (femhip.Fn, oracle.Fn) pairs from (kind, coeffs, nodal-numpy) tuples."""
    from paper_1804_05156_amd import femhip
    out = []
    for spec in (kind_f, kind_gd, kind_gn):
        if spec is None:
            out.append((None, None))
            continue
        kind, c, nodal = (spec + (None,))[:3]
        gf = femhip.Fn(kind, c, None if nodal is None else torch.from_numpy(nodal).cuda())
        of = oracle.Fn(kind, c, nodal)
        out.append((gf, of))
    return out


def run_gpu(m, kappa_dev=None, f=None, gd=None, gn=None, dev_arrays=None):
    from paper_1804_05156_amd import femhip
    node, elem, bd, kap = dev_arrays if dev_arrays is not None else to_dev(m)
    kappa = kap if kappa_dev is None else kappa_dev
    plan = femhip.Plan(node, elem, bd)
    asm = plan.assemble(kappa, f, gd, gn)
    plan.check()
    torch.cuda.synchronize()
    return plan, asm


def host(plan, asm):
    nnz = plan.nnz
    return dict(rowptr=plan.rowptr.cpu().numpy(), colind=plan.colind[:nnz].cpu().numpy(),
                val=asm.val[:nnz].cpu().numpy(), val_bc=asm.val_bc[:nnz].cpu().numpy(),
                b=asm.b.cpu().numpy(), b_load=asm.b_load.cpu().numpy(), is_d=asm.is_dirichlet.cpu().numpy())


def fn_bound(spec, dim, xmax=1.5):
    """Upper bound of |value| of a data function spec (kind, coeffs[, nodal]) on the domain."""
    if spec is None:
        return 0.0
    kind, c = spec[0], spec[1]
    c = list(c) + [0.0] * 4
    if kind == 1:
        return abs(c[0])
    if kind == 2:
        return abs(c[0]) + xmax * sum(abs(x) for x in c[1:1 + dim])
    if kind == 3:
        return abs(c[0])
    if kind == 4:
        return abs(c[0]) * np.pi * np.sqrt(dim)
    if kind == 5:
        return float(np.abs(spec[2]).max())
    return 0.0


def data_scale(m, specs, gr=None):
    """Per-row size of the data: load of |f|max plus Neumann (and Robin) side terms of
    |g_N|max (|g_R|max) (oracle, constant data), and |g_D|max."""
    f, gd, gn = (list(specs) + [None] * 3)[:3]
    fb, gb, rb = fn_bound(f, m.dim), fn_bound(gn, m.dim), fn_bound(gr, m.dim)
    a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=oracle.Fn(1, (fb,)), gN=oracle.Fn(1, (gb,)),
                        gR=oracle.Fn(1, (rb,)))
    return np.abs(a.b_load), fn_bound(gd, m.dim)


def scales(ora, fscale=None, dbound=0.0):
    n = ora.rowptr.size - 1
    d = np.zeros(n)
    rows = np.repeat(np.arange(n), np.diff(ora.rowptr))
    on = ora.colind == rows
    d[rows[on]] = ora.val[on]
    vscale = np.sqrt(np.abs(d[rows] * d[ora.colind]))
    isd = ora.is_d.astype(bool)
    lift = np.zeros(n)
    dc = isd[ora.colind]
    np.add.at(lift, rows[dc], vscale[dc] * (np.abs(ora.b[ora.colind[dc]]) + dbound))
    fs = np.zeros(n) if fscale is None else fscale
    lscale = ora.b_scale + fs
    bscale = np.where(isd, np.abs(ora.b) + dbound, lscale + lift)
    return rows, vscale, bscale, lscale


def compare(g, ora, tol=TOL, rows_subset=None, data=None):
    """Element-by-element comparison of GPU outputs `g` (dict from host()) with the oracle.
    `data` = data_scale(...) of the same mesh and data functions."""
    fscale, dbound = (None, 0.0) if data is None else data
    rows, vscale, bscale, lscale = scales(ora, fscale, dbound)
    if rows_subset is None:
        assert np.array_equal(g["rowptr"], ora.rowptr), "rowptr differs"
        assert np.array_equal(g["colind"], ora.colind), "colind differs"
        ev = np.abs(g["val"] - ora.val)
        assert np.all(ev <= tol * vscale), f"val: max scaled err {np.max(ev / np.maximum(vscale, 1e-300)):.3e}"
        ebc = np.abs(g["val_bc"] - ora.val_bc)
        assert np.all(ebc <= tol * vscale), "val_bc differs"
        assert np.array_equal(g["is_d"], ora.is_d), "Dirichlet set differs"
        eb = np.abs(g["b"] - ora.b)
        assert np.all(eb <= tol * bscale), f"b: max scaled err {np.max(eb / np.maximum(bscale, 1e-300)):.3e}"
        el = np.abs(g["b_load"] - ora.b_load)
        assert np.all(el <= tol * lscale), f"b_load: max scaled err {np.max(el / np.maximum(lscale, 1e-300)):.3e}"
        return float(np.max(ev / np.maximum(vscale, 1e-300)))
    worst = 0.0
    for i in rows_subset:
        gs, ge = g["rowptr"][i], g["rowptr"][i + 1]
        os_, oe = ora.rowptr[i], ora.rowptr[i + 1]
        assert np.array_equal(g["colind"][gs:ge], ora.colind[os_:oe]), f"row {i} pattern differs"
        ev = np.abs(g["val"][gs:ge] - ora.val[os_:oe])
        assert np.all(ev <= tol * vscale[os_:oe]), f"row {i} values differ"
        ebc = np.abs(g["val_bc"][gs:ge] - ora.val_bc[os_:oe])
        assert np.all(ebc <= tol * vscale[os_:oe]), f"row {i} val_bc differs"
        assert g["is_d"][i] == ora.is_d[i]
        assert abs(g["b"][i] - ora.b[i]) <= tol * bscale[i], f"row {i} b differs"
        assert abs(g["b_load"][i] - ora.b_load[i]) <= tol * lscale[i], f"row {i} b_load differs"
        worst = max(worst, float(np.max(ev / np.maximum(vscale[os_:oe], 1e-300))))
    return worst


def two_ring_submesh(m, rows):
    """Elements around `rows` and around their neighbours: the sampled rows of the
    oracle on this submesh are complete, Dirichlet flags of their columns included."""
    e1 = np.nonzero(np.isin(m.elem, rows).any(axis=0))[0]
    nb = np.unique(m.elem[:, e1])
    e2 = np.nonzero(np.isin(m.elem, nb).any(axis=0))[0]
    return e2
