"""Seeded synthetic mesh generators (inputs only).

This module builds the mesh arrays of Section 1 of L. Chen, "Programming of Finite
Element Methods in MATLAB": vertex coordinates ``node``, element-to-vertex map
``elem`` (each simplex positively oriented, Section 1.1) and boundary-side types
``bdFlag`` (Section 1.2: face ``a`` of an element lies opposite its local vertex
``a``; 0 interior, 1 Dirichlet, 2 Neumann, 3 Robin).  It holds none of the finite
element arithmetic: every quantity here is a coordinate, an index or a random draw.
Both the GPU library's tests and the CPU oracle's tests take their inputs from here.

Layout (structure of arrays, 0-based, matching the library's C interface):
  node   float64 (dim, N)      node[c, k] = coordinate c of vertex k
  elem   int32   (dim+1, NT)   elem[a, t] = global vertex of local vertex a of t
  bdflag int8    (dim+1, NT)   bdflag[a, t] = type of the face opposite local vertex a
  kappa  float64 (NT,)         per-element coefficient

Random draws use ``numpy.random.default_rng(seed)`` in this fixed order:
(1) jitter of interior nodes, 2 (or 3) uniform draws per interior node in node order;
(2) a node relabelling ``permutation(N)``; (3) ``kappa = exp(standard_normal(NT))``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

INTERIOR, DIRICHLET, NEUMANN, ROBIN = 0, 1, 2, 3


@dataclass
class Mesh:
    """Mesh arrays in the library's structure-of-arrays layout."""

    node: np.ndarray          # (dim, N) float64
    elem: np.ndarray          # (dim+1, NT) int32
    bdflag: np.ndarray        # (dim+1, NT) int8
    kappa: np.ndarray | None = None   # (NT,) float64
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.node.shape[0])

    @property
    def n_node(self) -> int:
        return int(self.node.shape[1])

    @property
    def n_elem(self) -> int:
        return int(self.elem.shape[1])


def _relabel(node, elem, perm):
    """New label of old vertex k is perm[k]; element order is unchanged."""
    new_node = np.empty_like(node)
    new_node[:, perm] = node
    new_elem = perm[elem].astype(np.int32)
    return new_node, new_elem


def square_mesh(n: int, *, jitter: float = 0.0, permute: bool = False, seed: int | None = None,
                kappa: str = "one", sides=(DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET),
                lo=(0.0, 0.0), hi=(1.0, 1.0)) -> Mesh:
    """Uniform n x n grid of the unit square, each cell cut along its "/" diagonal.

    Cell (i, j) has corners p1=(i,j), p2=(i+1,j), p3=(i+1,j+1), p4=(i,j+1); its
    triangles are [p2,p3,p1] and [p4,p1,p3] (both counter-clockwise).  Vertex (i, j)
    has label j*n + i before any relabelling.  ``sides`` gives the boundary type of
    the bottom (y=lo), right (x=hi), top (y=hi) and left (x=lo) sides.
    ``jitter`` moves each interior node by U(-jitter*h, jitter*h) per coordinate.
    ``kappa`` is "one" or "lognormal".
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    rng = np.random.default_rng(seed)
    hx = (hi[0] - lo[0]) / (n - 1)
    hy = (hi[1] - lo[1]) / (n - 1)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")   # jj rows, ii cols
    ii = ii.ravel()
    jj = jj.ravel()
    x = lo[0] + ii * hx
    y = lo[1] + jj * hy
    if jitter:
        interior = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)
        d = rng.uniform(-jitter, jitter, size=(int(interior.sum()), 2))
        x = x.copy()
        y = y.copy()
        x[interior] += d[:, 0] * hx
        y[interior] += d[:, 1] * hy
    node = np.stack([x, y]).astype(np.float64)

    ci, cj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    p1 = cj * n + ci
    p2 = p1 + 1
    p3 = p1 + n + 1
    p4 = p1 + n
    nc = ci.size
    elem = np.empty((3, 2 * nc), dtype=np.int32)
    elem[:, 0::2] = np.stack([p2, p3, p1])
    elem[:, 1::2] = np.stack([p4, p1, p3])
    bottom, right, top, left = sides
    bd = np.zeros((3, 2 * nc), dtype=np.int8)
    # triangle [p2,p3,p1]: face opp p2 = diagonal, opp p3 = (p1,p2) bottom, opp p1 = (p2,p3) right
    bd[1, 0::2] = np.where(cj == 0, bottom, 0)
    bd[2, 0::2] = np.where(ci == n - 2, right, 0)
    # triangle [p4,p1,p3]: face opp p4 = diagonal, opp p1 = (p3,p4) top, opp p3 = (p4,p1) left
    bd[1, 1::2] = np.where(cj == n - 2, top, 0)
    bd[2, 1::2] = np.where(ci == 0, left, 0)

    if permute:
        perm = rng.permutation(n * n)
        node, elem = _relabel(node, elem, perm)
    k = _kappa(kappa, elem.shape[1], rng)
    return Mesh(node, elem, bd, k, {"kind": "square", "n": n, "jitter": jitter,
                                     "permute": permute, "seed": seed})


def _kappa(kind: str, nt: int, rng) -> np.ndarray:
    if kind == "one":
        return np.ones(nt, dtype=np.float64)
    if kind == "lognormal":
        return np.exp(rng.standard_normal(nt)).astype(np.float64)
    raise ValueError(f"unknown kappa kind {kind!r}")


def _perm_sign(p) -> int:
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def kuhn_cube(n: int, *, jitter: float = 0.0, permute: bool = False, seed: int | None = None,
              kappa: str = "one", faces=(DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN)) -> Mesh:
    """Uniform n^3 grid of the unit cube, each cell split into 6 Kuhn tetrahedra.

    Cell corner v0 = (i, j, l); for each axis permutation s (itertools order) the
    tetrahedron is [v0, v0+e_s0, v0+e_s0+e_s1, v0+(1,1,1)].  Its edge vectors from
    the first vertex are e_s0, e_s0+e_s1, e_s0+e_s1+e_s2, so its signed volume has
    the sign of s; for odd s local vertices 1 and 2 are swapped to make it positive.
    Vertex (i, j, l) has label i + n*(j + n*l).  ``faces`` gives the boundary type of
    the planes x=0, x=1, y=0, y=1, z=0, z=1.
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    ll, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    ll = ll.ravel()
    coords = np.stack([ii * h, jj * h, ll * h]).astype(np.float64)
    if jitter:
        interior = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1) & (ll > 0) & (ll < n - 1)
        d = rng.uniform(-jitter, jitter, size=(int(interior.sum()), 3)) * h
        coords[:, interior] += d.T
    cl, cj, ci = np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(n - 1), indexing="ij")
    base = [ci.ravel(), cj.ravel(), cl.ravel()]                    # cell corner per axis
    ncell = base[0].size
    eye = np.eye(3, dtype=np.int64)
    tets = []
    for s in itertools.permutations(range(3)):
        corners = [np.zeros(3, np.int64), eye[s[0]], eye[s[0]] + eye[s[1]], np.ones(3, np.int64)]
        if _perm_sign(s) < 0:
            corners[1], corners[2] = corners[2], corners[1]
        tets.append(corners)
    # element order: cell-major, then the 6 permutations (element cell * 6 + k)
    off = np.array(tets, dtype=np.int64)                          # (tet k, local vertex a, axis)

    def coord(a, axis):
        """Grid coordinate along `axis` of local vertex a of every element."""
        return (base[axis][:, None] + off[None, :, a, axis]).ravel()

    elem = np.empty((4, ncell * 6), dtype=np.int32)
    for a in range(4):
        elem[a] = coord(a, 0) + n * (coord(a, 1) + n * coord(a, 2))
    bd = np.zeros((4, ncell * 6), dtype=np.int8)
    for axis in range(3):
        for side, val in ((0, 0), (1, n - 1)):
            onv = [coord(b, axis) == val for b in range(4)]
            code = faces[2 * axis + side]
            for a in range(4):
                others = [b for b in range(4) if b != a]
                on = onv[others[0]] & onv[others[1]] & onv[others[2]]
                bd[a, on] = code
    node = coords
    if permute:
        perm = rng.permutation(n ** 3)
        node, elem = _relabel(node, elem, perm)
    k = _kappa(kappa, elem.shape[1], rng)
    return Mesh(node, elem, bd, k, {"kind": "kuhn", "n": n, "jitter": jitter,
                                     "permute": permute, "seed": seed})


def lshape_mesh(n: int, *, seed: int | None = None, kappa: str = "one") -> Mesh:
    """L-shaped domain (-1,1)^2 minus [0,1]x[-1,0] (the example domain of Section 1.1).

    Built from a (2n-1) x (2n-1) "/"-diagonal grid of (-1,1)^2 by dropping the
    cells of the removed quadrant and the vertices no element uses; every boundary
    side is Dirichlet.  ``n`` counts vertices along each half side.
    """
    m = 2 * n - 1
    full = square_mesh(m, lo=(-1.0, -1.0), hi=(1.0, 1.0), seed=seed, kappa="one")
    x, y = full.node
    cx = x[full.elem].mean(axis=0)
    cy = y[full.elem].mean(axis=0)
    keep = ~((cx > 0) & (cy < 0))
    elem = full.elem[:, keep]
    used = np.zeros(full.n_node, bool)
    used[elem.ravel()] = True
    newid = -np.ones(full.n_node, np.int64)
    newid[used] = np.arange(int(used.sum()))
    node = np.ascontiguousarray(full.node[:, used])
    elem = np.ascontiguousarray(newid[elem].astype(np.int32))
    # boundary faces: faces that belong to exactly one element
    nt = elem.shape[1]
    bd = np.zeros((3, nt), np.int8)
    keys = {}
    for a in range(3):
        u = elem[(a + 1) % 3]
        v = elem[(a + 2) % 3]
        lo_ = np.minimum(u, v).astype(np.int64)
        hi_ = np.maximum(u, v).astype(np.int64)
        keys[a] = lo_ * node.shape[1] + hi_
    allk = np.concatenate([keys[0], keys[1], keys[2]])
    uniq, cnt = np.unique(allk, return_counts=True)
    single = set(uniq[cnt == 1].tolist())
    for a in range(3):
        bd[a] = np.array([DIRICHLET if k in single else 0 for k in keys[a].tolist()], np.int8)
    rng = np.random.default_rng(seed)
    return Mesh(node, elem, bd, _kappa(kappa, nt, rng), {"kind": "lshape", "n": n})


def batch_sizes(n_inst: int = 256, lo: int = 17, hi: int = 513, seed: int = 4) -> np.ndarray:
    """Grid sides of a batch of square meshes, uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, n_inst)


def batch_meshes(sizes, *, seed_base: int = 4000, jitter: float = 0.2, permute: bool = False,
                 kappa: str = "lognormal"):
    """Instance i is ``square_mesh(sizes[i], seed=seed_base+i, ...)``."""
    return [square_mesh(int(n), jitter=jitter, permute=permute, seed=seed_base + i, kappa=kappa)
            for i, n in enumerate(sizes)]


# Named workloads: sizes and recipes of the benchmark configurations.
def workload(name: str) -> Mesh:
    """Return the mesh of a named workload.

    "square33"        33x33 uniform grid, kappa = 1, Dirichlet everywhere.
    "jitter2049"      2049x2049 grid, interior jitter +-0.2h, permuted labels,
                      lognormal kappa, Dirichlet everywhere (seed 2).
    "kuhn129"         129^3 Kuhn cube, lognormal kappa, Dirichlet on x=0,1 and
                      Neumann on the other faces (seed 3).
    "jitter1025"      1025x1025 grid, jitter +-0.2h, lognormal kappa (seed 5).
    """
    if name == "square33":
        return square_mesh(33)
    if name == "jitter2049":
        return square_mesh(2049, jitter=0.2, permute=True, seed=2, kappa="lognormal")
    if name == "kuhn129":
        return kuhn_cube(129, seed=3, kappa="lognormal")
    if name == "jitter1025":
        return square_mesh(1025, jitter=0.2, permute=False, seed=5, kappa="lognormal")
    raise KeyError(name)
