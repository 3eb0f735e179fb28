"""GPU parity of assembly (A, A_bc, b, Dirichlet set) against the CPU oracle.

Every test runs the HIP library through its C interface (ctypes binding) on the
same seeded inputs as the oracle and compares element by element: pattern bit
for bit, values within the scaled tolerance of gpu_helpers.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1804_05156_amd import meshgen
from gpu_helpers import TOL, compare, data_scale, fns, host, log, run_gpu, to_dev, two_ring_submesh

pytestmark = pytest.mark.gpu

FE_FN_CONST, FE_FN_LINEAR, FE_FN_SINPROD, FE_FN_DUDN_SINPROD, FE_FN_NODAL = 1, 2, 3, 4, 5
TWO_PI2 = 2 * math.pi ** 2


def test_uniform_square_bitwise():
    """33x33 uniform grid, kappa = 1, f = 2 pi^2 sin sin, g_D = 0 (dyadic geometry:
    every stiffness value is exact, so A matches the oracle bit for bit)."""
    log("case: uniform 33x33")
    m = meshgen.workload("square33")
    spec = [(FE_FN_SINPROD, (TWO_PI2,))]
    (f, fo), _, _ = fns(*spec)
    plan, asm = run_gpu(m, None, f)
    g = host(plan, asm)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fo)
    compare(g, ora, data=data_scale(m, spec))
    assert np.array_equal(g["val"], ora.val)
    assert np.array_equal(g["val_bc"], ora.val_bc)
    n = 33
    for j in (1, 16, 31):
        for i in (1, 7, 31):
            r = j * n + i
            c = g["colind"][g["rowptr"][r]:g["rowptr"][r + 1]]
            v = g["val"][g["rowptr"][r]:g["rowptr"][r + 1]]
            want = {r - n - 1: 0.0, r - n: -1.0, r - 1: -1.0, r: 4.0, r + 1: -1.0, r + n: -1.0, r + n + 1: 0.0}
            assert c.tolist() == sorted(want) and v.tolist() == [want[k] for k in c]


def _random_sides(rng, count):
    return tuple(int(x) for x in rng.choice([1, 2], size=count))


@pytest.mark.parametrize("seed,n", [(1, 5), (2, 9), (3, 17), (4, 33), (5, 40)])
def test_parity_2d_jittered_permuted(seed, n):
    log(f"case: 2d jitter permute seed={seed} n={n}")
    rng = np.random.default_rng(100 + seed)
    sides = _random_sides(rng, 4)
    if 1 not in sides:
        sides = (1,) + sides[1:]
    m = meshgen.square_mesh(n, jitter=0.2, permute=True, seed=seed, kappa="lognormal", sides=sides)
    specs = [(FE_FN_SINPROD, (TWO_PI2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7)),
             (FE_FN_DUDN_SINPROD, (1.3,)) if seed % 2 else (FE_FN_CONST, (0.9,))]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd, gn)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs))
    log(f"  worst scaled value error {worst:.2e}")


@pytest.mark.parametrize("dim,n", [(2, 1025), (3, 65)])
def test_both_sort_paths(dim, n):
    """The incidence sort aggregates its LDS counter updates per wavefront when labels
    follow the element order (runs of equal buckets in neighbouring lanes) and
    updates per lane when they are scattered over many buckets; the plan reports
    which it took.  The same mesh with coherent labels and with a random relabelling
    takes one path each, and the two matrices and right-hand sides are the same bits
    up to the relabelling (rows sum in ascending element order either way).  Oracle
    parity of each path is covered at full size (2049^2 permuted: per lane; 129^3:
    aggregated)."""
    from paper_1804_05156_amd import femhip
    log(f"case: both sort paths, dim {dim}, n {n}")
    if dim == 2:
        m = meshgen.square_mesh(n, jitter=0.2, seed=61, kappa="lognormal", sides=(1, 2, 1, 2))
        specs = [(FE_FN_SINPROD, (TWO_PI2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7)), (FE_FN_CONST, (0.9,))]
    else:
        m = meshgen.kuhn_cube(n, jitter=0.15, seed=62, kappa="lognormal")
        specs = [(FE_FN_SINPROD, (3 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4)),
                 (FE_FN_DUDN_SINPROD, (1.0,))]
    perm = np.random.default_rng(63).permutation(m.n_node)          # old label -> new label
    node_p = np.empty_like(m.node)
    node_p[:, perm] = m.node
    elem_p = np.ascontiguousarray(perm[m.elem].astype(np.int32))
    (f, _), (gd, _), (gn, _) = fns(*specs)
    outs = []
    for node, elem in ((m.node, m.elem), (node_p, elem_p)):
        nd = torch.from_numpy(np.ascontiguousarray(node)).cuda()
        plan = femhip.Plan(nd, torch.from_numpy(elem).cuda(), torch.from_numpy(m.bdflag).cuda())
        asm = plan.assemble(torch.from_numpy(m.kappa).cuda(), f, gd, gn)
        plan.check()
        outs.append((plan.info["sort_runs"], host(plan, asm)))
    assert [o[0] for o in outs] == [1, 0]
    g, gp = outs[0][1], outs[1][1]
    rows = np.repeat(np.arange(m.n_node), np.diff(g["rowptr"]))
    rows_p = np.repeat(np.arange(m.n_node), np.diff(gp["rowptr"]))
    key = perm[rows].astype(np.int64) * m.n_node + perm[g["colind"]]
    key_p = rows_p.astype(np.int64) * m.n_node + gp["colind"]
    o, op = np.argsort(key), np.argsort(key_p)
    assert np.array_equal(key[o], key_p[op])
    for name in ("val", "val_bc"):
        assert np.array_equal(g[name][o], gp[name][op]), name
    for name in ("b", "b_load", "is_d"):
        assert np.array_equal(g[name], gp[name][perm]), name
    log(f"  nnz {key.size}: paths {[o[0] for o in outs]}, identical up to relabelling")


@pytest.mark.parametrize("seed,n", [(1, 3), (2, 4), (3, 6), (4, 9)])
def test_parity_3d_jittered_permuted(seed, n):
    log(f"case: 3d kuhn jitter permute seed={seed} n={n}")
    rng = np.random.default_rng(200 + seed)
    faces = tuple(int(x) for x in rng.choice([0, 1, 2], size=6))
    if 1 not in faces:
        faces = (1,) + faces[1:]
    m = meshgen.kuhn_cube(n, jitter=0.15, permute=True, seed=seed, kappa="lognormal", faces=faces)
    specs = [(FE_FN_SINPROD, (3 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4)),
             (FE_FN_DUDN_SINPROD, (1.0,)) if seed % 2 else (FE_FN_LINEAR, (0.5, 0.2, 0.1, -0.3))]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd, gn)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs))
    log(f"  worst scaled value error {worst:.2e}")


@pytest.mark.parametrize("dim", [2, 3])
def test_parity_nodal_data(dim):
    log(f"case: nodal data dim={dim}")
    if dim == 2:
        m = meshgen.square_mesh(12, jitter=0.2, permute=True, seed=9, kappa="lognormal", sides=(1, 2, 2, 1))
    else:
        m = meshgen.kuhn_cube(5, jitter=0.2, permute=True, seed=9, kappa="lognormal")
    rng = np.random.default_rng(5)
    fv, gv, nv = (rng.standard_normal(m.n_node) for _ in range(3))
    specs = [(FE_FN_NODAL, (0,), fv), (FE_FN_NODAL, (0,), gv), (FE_FN_NODAL, (0,), nv)]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd, gn)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno)
    compare(host(plan, asm), ora, data=data_scale(m, specs))


def test_unused_vertex_single_elements():
    log("case: unused vertex / single elements")
    # one triangle plus an unused vertex: its row is empty, as sparse() gives
    node = np.array([[0.0, 1.0, 0.0, 5.0], [0.0, 0.0, 1.0, 5.0]])
    elem = np.array([[0], [1], [2]], np.int32)
    bd = np.array([[1], [2], [0]], np.int8)
    m = meshgen.Mesh(node, elem, bd, np.array([2.0]))
    specs = [(FE_FN_CONST, (1.0,)), (FE_FN_LINEAR, (1.0, 2.0, 3.0)), (FE_FN_CONST, (0.5,))]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd, gn)
    ora = oracle.assemble(node, elem, bd, m.kappa, f=fo, gD=gdo, gN=gno)
    g = host(plan, asm)
    assert g["rowptr"].tolist() == [0, 3, 6, 9, 9]
    compare(g, ora, data=data_scale(m, specs))
    # one tetrahedron
    node = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    elem = np.array([[0], [1], [2], [3]], np.int32)
    bd = np.array([[2], [0], [1], [2]], np.int8)
    m = meshgen.Mesh(node, elem, bd, np.array([0.7]))
    plan, asm = run_gpu(m, None, f, gd, gn)
    compare(host(plan, asm), oracle.assemble(node, elem, bd, m.kappa, f=fo, gD=gdo, gN=gno),
            data=data_scale(m, specs))


SCAN_TILE_EDGE = 4096 * 4096   # prefix sums: up to 4096 tiles of 4096 entries in two launches


@pytest.mark.parametrize("extra,labels", [(0, "leading"), (1, "scattered")])
def test_prefix_sum_tile_limit(extra, labels):
    """A 129x129 jittered mesh whose vertices sit among N = 4096^2 (+1) labels, the
    rest unused (empty rows): the per-vertex prefix sums run at the largest size of
    the two-launch form and one past it (a one-block scan of the tile sums in
    between).  Labels either lead (0.., element order: label-order processing) or
    are scattered over the whole range (the general path, which scans three
    per-vertex arrays).  With leading labels the used vertices fill a few buckets
    sized for the (tiny) average degree, far beyond their LDS capacity, so those
    buckets take the level-2 kernel's global-memory path.  f = 1, so the oracle's
    own term sums set the b scale."""
    N = SCAN_TILE_EDGE + extra
    log(f"case: prefix-sum tile limit, N = {N}, labels {labels}")
    small = meshgen.square_mesh(129, jitter=0.2, permute=False, seed=91, kappa="lognormal")
    rng = np.random.default_rng(92)
    emb = np.arange(small.n_node) if labels == "leading" else rng.choice(N, small.n_node, replace=False)
    node = np.zeros((2, N))
    node[:, emb] = small.node
    m = meshgen.Mesh(node, emb[small.elem].astype(np.int32), small.bdflag, small.kappa)
    (f, fo), _, _ = fns((FE_FN_CONST, (1.0,)))
    plan, asm = run_gpu(m, None, f)
    assert plan.info["sort_runs"] == (labels == "leading")
    g = host(plan, asm)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo)
    compare(g, ora)
    assert g["rowptr"][-1] == ora.rowptr[-1] == plan.nnz


def _fan(k):
    """k triangles around the origin (a vertex with k neighbours), outer ring Dirichlet."""
    ang = 2 * math.pi * np.arange(k) / k
    node = np.vstack([np.r_[0.0, np.cos(ang)], np.r_[0.0, np.sin(ang)]])
    elem = np.array([[0] * k, list(range(1, k + 1)), [1 + (j + 1) % k for j in range(k)]], np.int32)
    bd = np.zeros((3, k), np.int8)
    bd[0] = 1
    return meshgen.Mesh(node, elem, bd, np.exp(np.sin(np.arange(k))))


@pytest.mark.parametrize("k", [3, 15, 20, 31])
def test_high_degree_vertex(k):
    """Rows longer than 16 entries take the wider accumulator kernels."""
    log(f"case: fan k={k}")
    m = _fan(k)
    specs = [(FE_FN_SINPROD, (1.0,)), (FE_FN_LINEAR, (1.0, 0.5, 0.25))]
    (f, fo), (gd, gdo), _ = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd)
    assert plan.info["max_row"] == k + 1
    compare(host(plan, asm), oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo),
            data=data_scale(m, specs))


def _edge_fan(k):
    """k tetrahedra around the axis edge (0, 1) (its two vertices have k + 1
    neighbours); faces opposite vertex 0 Dirichlet, faces opposite vertex 1 Neumann."""
    ang = 2 * math.pi * np.arange(k) / k
    node = np.vstack([np.r_[0.0, 0.0, np.cos(ang)], np.r_[0.0, 0.0, np.sin(ang)], np.r_[0.0, 1.0, np.full(k, 0.5)]])
    ring = np.arange(k)
    elem = np.array([[0] * k, [1] * k, list(2 + ring), list(2 + (ring + 1) % k)], np.int32)
    bd = np.zeros((4, k), np.int8)
    bd[0] = 1
    bd[1] = 2
    return meshgen.Mesh(node, elem, bd, np.exp(np.cos(np.arange(k))))


@pytest.mark.parametrize("k", [20, 40])
def test_high_degree_vertex_3d(k):
    """3-D rows longer than 16 entries: the row passes take the LDS column set
    (no stored register sets) and the numeric kernel the wider accumulator."""
    log(f"case: edge fan k={k}")
    m = _edge_fan(k)
    specs = [(FE_FN_SINPROD, (1.0,)), (FE_FN_LINEAR, (1.0, 0.5, 0.25, 0.125)), (FE_FN_CONST, (0.5,))]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd, gn)
    assert plan.info["max_row"] == k + 2
    compare(host(plan, asm), oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno),
            data=data_scale(m, specs))


def _open_fan(k):
    """k triangles over a half disk around vertex 0, which sits on the straight side:
    the end spokes and the arc are boundary sides (codes set by the caller)."""
    ang = math.pi * np.arange(k + 1) / k
    node = np.vstack([np.r_[0.5, 0.5 + 0.4 * np.cos(ang)], np.r_[0.1, 0.1 + 0.4 * np.sin(ang)]])
    elem = np.array([[0] * k, list(range(1, k + 1)), list(range(2, k + 2))], np.int32)
    bd = np.zeros((3, k), np.int8)
    return meshgen.Mesh(node, elem, bd, np.exp(np.sin(np.arange(k))))


def _check_long(m, specs, gr=None, alpha=0.0, rule=0, n_long=None):
    from paper_1804_05156_amd import femhip
    (f, fo), (gd, gdo), (gn, gno) = fns(*(list(specs) + [None] * 3)[:3])
    (grf, gro), _, _ = fns(gr)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    asm = plan.assemble(kap, f, gd, gn, gR=grf, robin_alpha=alpha, load_rule=rule)
    plan.check()
    torch.cuda.synchronize()
    if n_long is not None:
        assert plan.info["n_long"] == n_long
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno, gR=gro, alpha=alpha, rule=rule)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs, gr))
    log(f"  max_row {plan.info['max_row']} n_long {plan.info['n_long']} sort_runs {plan.info['sort_runs']}, "
        f"worst scaled error {worst:.2e}")
    return plan


@pytest.mark.parametrize("k", [32, 40, 100, 1000])
def test_long_row_fan(k):
    """A vertex with more neighbours than the row kernels hold (31 in 2-D) takes the
    long-row kernels of the plan and of the numeric phase; the row is checked
    against the oracle like any other."""
    log(f"case: long row, fan k={k}")
    m = _fan(k)
    specs = [(FE_FN_SINPROD, (1.0,)), (FE_FN_LINEAR, (1.0, 0.5, 0.25))]
    plan = _check_long(m, specs, n_long=1 if k + 1 > 32 else 0)
    assert plan.info["max_row"] == k + 1


@pytest.mark.parametrize("code", [1, 2, 3])
@pytest.mark.parametrize("rule", [0, 1, 2])
def test_long_row_on_the_boundary(code, rule):
    """The long row of a boundary vertex: its two end spokes are Dirichlet (lifting),
    Neumann or Robin sides (side terms and side mass in the long-row kernel), with
    nodal data and each load rule of Section 4."""
    log(f"case: long boundary row, side code {code}, load rule {rule}")
    k = 60
    m = _open_fan(k)
    m.bdflag[2, 0] = code            # spoke (0, 1)
    m.bdflag[1, k - 1] = code        # spoke (k + 1, 0)
    m.bdflag[0, :] = 1 if code != 1 else 2
    rng = np.random.default_rng(30 + code)
    nod = [rng.standard_normal(m.n_node) for _ in range(4)]
    specs = [(FE_FN_NODAL, (0.0,), nod[0]), (FE_FN_NODAL, (0.0,), nod[1]), (FE_FN_NODAL, (0.0,), nod[2])]
    gr, alpha = ((FE_FN_NODAL, (0.0,), nod[3]), 0.8) if code == 3 else (None, 0.0)
    if rule == 0 and code != 1:
        specs = [(FE_FN_SINPROD, (2.0,)), (FE_FN_LINEAR, (0.3, 1.0, -0.5)), (FE_FN_DUDN_SINPROD, (1.0,))]
        gr = (FE_FN_DUDN_SINPROD, (0.5,)) if code == 3 else None
    _check_long(m, specs, gr, alpha, rule, n_long=1)


@pytest.mark.parametrize("k", [64, 80, 200])
def test_long_row_edge_fan(k):
    """3-D: the two vertices of an edge shared by k tetrahedra have k + 2 columns
    (more than 64 for k >= 63): Dirichlet faces on one side, Neumann faces through
    the other vertex's long row."""
    log(f"case: long rows, edge fan k={k}")
    m = _edge_fan(k)
    specs = [(FE_FN_SINPROD, (1.0,)), (FE_FN_LINEAR, (1.0, 0.5, 0.25, 0.125)), (FE_FN_CONST, (0.5,))]
    plan = _check_long(m, specs, n_long=2 if k + 2 > 64 else 0)
    assert plan.info["max_row"] == k + 2


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_long_row_edge_fan_robin(rule):
    """3-D long rows with Robin faces through them and nodal data."""
    log(f"case: long rows, edge fan with Robin faces, load rule {rule}")
    m = _edge_fan(70)
    m.bdflag[1] = 3
    rng = np.random.default_rng(40 + rule)
    nod = [rng.standard_normal(m.n_node) for _ in range(4)]
    specs = [(FE_FN_NODAL, (0.0,), nod[0]), (FE_FN_NODAL, (0.0,), nod[1]), (FE_FN_NODAL, (0.0,), nod[2])]
    _check_long(m, specs, (FE_FN_NODAL, (0.0,), nod[3]), 0.6, rule, n_long=2)


def _union(a, b):
    """Disjoint union of two meshes: b's labels follow a's."""
    node = np.hstack([a.node, b.node])
    elem = np.hstack([a.elem, b.elem + a.n_node]).astype(np.int32)
    return meshgen.Mesh(node, elem, np.hstack([a.bdflag, b.bdflag]), np.r_[a.kappa, b.kappa])


@pytest.mark.parametrize("permute", [False, True])
def test_long_rows_in_a_large_mesh(permute):
    """A 129^2 jittered mesh with a fan of 100 beside it, labels in element order or
    randomly permuted: the long row goes through both processing orders (the label-
    order copies skip it; it writes its own label-order outputs)."""
    log(f"case: long row in a large mesh, permute {permute}")
    sq = meshgen.square_mesh(129, jitter=0.2, permute=permute, seed=88, kappa="lognormal")
    fan = _fan(100)
    fan.node[0] += 2.0
    m = _union(sq, fan)
    specs = [(FE_FN_SINPROD, (2 * math.pi ** 2,)), (FE_FN_LINEAR, (0.2, 0.1, -0.3))]
    plan = _check_long(m, specs, n_long=1)
    assert plan.info["sort_runs"] == (0 if permute else 1)


@pytest.mark.parametrize("permute", [False, True])
def test_mid_degree_vertex_in_a_large_mesh(permute):
    """A 129^2 jittered mesh with a fan of 12 beside it: one row of 13 columns among
    rows of at most 7.  The register column set works at full width in the wavefronts
    around that row and at half width elsewhere, and the numeric kernel takes the
    16-column accumulators, which evaluate the source at every incidence instead of
    once per edge midpoint.  Against the oracle, and bit for bit against the square
    mesh alone (same incidences per row, so the same sums) for the square's rows."""
    log(f"case: mid-degree vertex in a large mesh, permute {permute}")
    sq = meshgen.square_mesh(129, jitter=0.2, permute=permute, seed=89, kappa="lognormal")
    fan = _fan(12)
    fan.node[0] += 2.0
    m = _union(sq, fan)
    specs = [(FE_FN_SINPROD, (2 * math.pi ** 2,)), (FE_FN_LINEAR, (0.2, 0.1, -0.3))]
    (f, fo), (gd, gdo), _ = fns(*specs)
    plan, asm = run_gpu(m, None, f, gd)
    assert plan.info["max_row"] == 13 and plan.info["n_long"] == 0
    g = host(plan, asm)
    compare(g, oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo), data=data_scale(m, specs))
    plan_sq, asm_sq = run_gpu(sq, None, f, gd)
    assert plan_sq.info["max_row"] <= 8
    h = host(plan_sq, asm_sq)
    n = sq.n_node
    nz = h["rowptr"][-1]
    assert np.array_equal(g["rowptr"][:n + 1], h["rowptr"])
    assert np.array_equal(g["colind"][:nz], h["colind"])
    for key in ("val", "val_bc"):
        assert np.array_equal(g[key][:nz], h[key]), key
    for key in ("b", "b_load", "is_d"):
        assert np.array_equal(g[key][:n], h[key]), key


def test_vertex_degree_limit_is_reported():
    """A vertex in 4096 triangles has 8193 candidate columns, one more than the long-
    row kernels hold: the plan refuses it with FE_ELIMIT.  4095 still fits."""
    from paper_1804_05156_amd import femhip
    log("case: vertex degree limit")
    node, elem, bd, _ = to_dev(_fan(4096))
    with pytest.raises(femhip.FemhipError) as e:
        femhip.Plan(node, elem, bd)
    assert e.value.code == femhip.FE_ELIMIT
    _check_long(_fan(4095), [(FE_FN_CONST, (1.0,))], n_long=1)


@pytest.mark.parametrize("labels", ["leading", "scattered", "trailing"])
def test_more_than_2_26_labels(labels):
    """A 129^2 jittered mesh whose vertices sit among N = 2^26 + 1 labels (the rest
    unused): more buckets than 2^26 labels fill at 4096 per bucket, and, with
    trailing labels in element order, element records holding labels above 2^26."""
    N = 2 ** 26 + 1
    log(f"case: N = {N}, labels {labels}")
    small = meshgen.square_mesh(129, jitter=0.2, permute=False, seed=93, kappa="lognormal")
    rng = np.random.default_rng(94)
    if labels == "leading":
        emb = np.arange(small.n_node)
    elif labels == "trailing":
        emb = N - small.n_node + np.arange(small.n_node)
    else:
        emb = rng.choice(N, small.n_node, replace=False)
        emb[-1] = N - 1
    node = np.zeros((2, N))
    node[:, emb] = small.node
    m = meshgen.Mesh(node, emb[small.elem].astype(np.int32), small.bdflag, small.kappa)
    (f, fo), _, _ = fns((FE_FN_CONST, (1.0,)))
    plan, asm = run_gpu(m, None, f)
    assert plan.info["sort_runs"] == (labels != "scattered")
    g = host(plan, asm)
    del asm
    torch.cuda.empty_cache()
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo)
    compare(g, ora)
    assert g["rowptr"][-1] == ora.rowptr[-1] == plan.nnz


@pytest.mark.parametrize("dim", [2, 3])
def test_launch_setting_bitwise(dim):
    """Rows per workgroup of the numeric row kernels (fe_plan_set_launch) change no
    result bit; other values are refused."""
    from paper_1804_05156_amd import femhip
    log(f"case: launch setting, dim {dim}")
    if dim == 2:
        m = meshgen.square_mesh(65, jitter=0.2, permute=True, seed=71, kappa="lognormal", sides=(1, 2, 1, 2))
        specs = [(FE_FN_SINPROD, (TWO_PI2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7)), (FE_FN_CONST, (0.9,))]
    else:
        m = meshgen.kuhn_cube(13, jitter=0.15, permute=False, seed=72, kappa="lognormal")
        specs = [(FE_FN_SINPROD, (3 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4)),
                 (FE_FN_DUDN_SINPROD, (1.0,))]
    (f, _), (gd, _), (gn, _) = fns(*specs)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    ref = host(plan, plan.assemble(kap, f, gd, gn))
    for rpb in (64, 128, 256, 0):
        plan.set_launch(rpb)
        g = host(plan, plan.assemble(kap, f, gd, gn))
        for name in ("val", "val_bc", "b", "b_load", "is_d"):
            assert np.array_equal(g[name], ref[name]), (rpb, name)
    for bad in (32, 100, 512, -1):
        with pytest.raises(femhip.FemhipError) as e:
            plan.set_launch(bad)
        assert e.value.code == femhip.FE_EINVAL


def test_error_paths():
    from paper_1804_05156_amd import femhip
    log("case: error paths")
    m = meshgen.square_mesh(6, jitter=0.1, seed=3)
    node, elem, bd, kap = to_dev(m)
    bad = elem.clone()
    bad[1, 3] = m.n_node                      # index out of range
    with pytest.raises(femhip.FemhipError) as e:
        femhip.Plan(node, bad, bd)
    assert e.value.code == femhip.FE_EINVAL
    bad = elem.clone()
    bad[2, 5] = bad[0, 5]                     # repeated vertex
    with pytest.raises(femhip.FemhipError) as e:
        femhip.Plan(node, bad, bd)
    assert e.value.code == femhip.FE_EMESH
    b4 = bd.clone()
    b4[1, 0] = 4                              # no such boundary type
    with pytest.raises(femhip.FemhipError) as e:
        femhip.Plan(node, elem, b4)
    assert e.value.code == femhip.FE_EINVAL
    b3 = bd.clone()
    b3[1, 0] = 3                              # Robin side: a negative coefficient is rejected
    with pytest.raises(femhip.FemhipError) as e:
        femhip.Plan(node, elem, b3).assemble(kap, robin_alpha=-1.0)
    assert e.value.code == femhip.FE_EINVAL
    cw = elem.clone()
    cw[[0, 1], 4] = cw[[1, 0], 4]             # clockwise element: found by the numeric kernel
    plan = femhip.Plan(node, cw, bd)
    plan.assemble(kap)
    with pytest.raises(femhip.FemhipError) as e:
        plan.check()
    assert e.value.code == femhip.FE_EMESH
    plan = femhip.Plan(node, elem, bd)
    k2 = kap.clone()
    k2[7] = -1.0
    plan.assemble(k2)
    with pytest.raises(femhip.FemhipError) as e:
        plan.check()
    assert e.value.code == femhip.FE_EINVAL
    plan.assemble(kap)
    plan.check()                              # status was cleared by the previous check


def test_bitwise_repeatable():
    log("case: determinism")
    m = meshgen.square_mesh(65, jitter=0.2, permute=True, seed=21, kappa="lognormal")
    (f, _), (gd, _), _ = fns((FE_FN_SINPROD, (TWO_PI2,)), (FE_FN_LINEAR, (1.0, 1.0, 1.0)))
    dev = to_dev(m)
    p1, a1 = run_gpu(m, None, f, gd, dev_arrays=dev)
    p2, a2 = run_gpu(m, None, f, gd, dev_arrays=dev)
    a3 = p1.assemble(dev[3], f, gd)
    torch.cuda.synchronize()
    for x, y in ((a1.val, a2.val), (a1.val, a3.val), (a1.b, a2.b), (a1.b, a3.b), (a1.val_bc, a2.val_bc)):
        assert torch.equal(x, y)
    assert torch.equal(p1.colind, p2.colind) and torch.equal(p1.rowptr, p2.rowptr)


def _sampled_full_size(m, specs, nsample=64, seed=0):
    (f, fo), (gd, gdo), (gn, gno) = fns(*(list(specs) + [None] * 3)[:3])
    plan, asm = run_gpu(m, None, f, gd, gn)
    log(f"  nnz={plan.nnz} max_row={plan.info['max_row']} max_deg={plan.info['max_deg']}")
    g = host(plan, asm)
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.integers(0, m.n_node, nsample), [0, m.n_node - 1]]))
    # boundary rows too: vertices of Dirichlet and Neumann sides
    bdv = np.unique(m.elem[:, np.nonzero((m.bdflag > 0).any(axis=0))[0][:8]])
    rows = np.unique(np.concatenate([rows, bdv]))
    sub = two_ring_submesh(m, rows)
    sm = meshgen.Mesh(m.node, m.elem[:, sub], m.bdflag[:, sub], m.kappa[sub])
    ora = oracle.assemble(sm.node, sm.elem, sm.bdflag, sm.kappa, f=fo, gD=gdo, gN=gno)
    worst = compare(g, ora, rows_subset=rows, data=data_scale(sm, specs))
    log(f"  sampled {rows.size} rows, worst scaled error {worst:.2e}")
    return plan, asm, g


def test_element_prefix_sum_beyond_tile_limit_sampled():
    """A 2898^2 grid with scattered labels has 16,785,218 > 4096^2 triangles, so the
    prefix sum of first incidences per element (general path) takes its three-launch
    form.  Built directly (plain grid, two triangles a cell, random labels, no
    boundary sides); sampled rows against the oracle, and the pattern size."""
    n = 2898
    log(f"case: {n}^2 grid, scattered labels, elements beyond the two-launch scan")
    N = n * n
    rng = np.random.default_rng(29)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    node = np.vstack([i.ravel() / (n - 1), j.ravel() / (n - 1)])
    c = np.arange((n - 1) * (n - 1))
    p1 = (c // (n - 1)) * n + c % (n - 1)
    elem = np.hstack([np.vstack([p1, p1 + 1, p1 + n + 1]), np.vstack([p1, p1 + n + 1, p1 + n])]).astype(np.int32)
    perm = rng.permutation(N).astype(np.int32)
    nodep = np.empty_like(node)
    nodep[:, perm] = node
    m = meshgen.Mesh(nodep, perm[elem], np.zeros(elem.shape, np.int8), np.exp(rng.standard_normal(elem.shape[1])))
    assert m.n_elem > SCAN_TILE_EDGE
    plan, asm, g = _sampled_full_size(m, [(FE_FN_CONST, (1.0,))], nsample=32)
    assert not plan.info["sort_runs"]
    assert plan.nnz == 3 * N + 2 * m.n_elem - 2


@pytest.mark.parametrize("dim,permute", [(2, False), (2, True), (3, False), (3, True)])
def test_every_element_listed_twice(dim, permute):
    """Each element listed twice (the copy with its own kappa): sparse() adds the
    duplicate contributions like any others (Section 2.2).  Every vertex then has twice
    its incidences, 12 in 2-D and 48 in the 3-D Kuhn mesh, which takes the row passes
    and numeric kernels past their per-wavefront buffers (64 rows of 8 keys in 2-D, of
    24 in the 3-D key lists, of 32 in the 3-D key copy) and the 2-D one-walk final pass
    (8 incidences), onto their direct paths."""
    log(f"case: every element twice, dim={dim} permute={permute}")
    if dim == 2:
        m = meshgen.square_mesh(65, jitter=0.2, permute=permute, seed=31, kappa="lognormal", sides=(1, 2, 1, 2))
    else:
        m = meshgen.kuhn_cube(12, jitter=0.15, permute=permute, seed=32, kappa="lognormal")
    rng = np.random.default_rng(33)
    elem = np.ascontiguousarray(np.concatenate([m.elem, m.elem], axis=1))
    bd = np.ascontiguousarray(np.concatenate([m.bdflag, m.bdflag], axis=1))
    kappa = np.concatenate([m.kappa, np.exp(rng.normal(size=m.kappa.shape))])
    m2 = meshgen.Mesh(m.node, elem, bd, kappa)
    specs = [(FE_FN_SINPROD, (TWO_PI2 if dim == 2 else 3 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.2)[:dim + 1]),
             (FE_FN_DUDN_SINPROD, (1.3,))]
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    plan, asm = run_gpu(m2, None, f, gd, gn)
    g = host(plan, asm)
    ora = oracle.assemble(m2.node, m2.elem, m2.bdflag, m2.kappa, f=fo, gD=gdo, gN=gno)
    compare(g, ora, data=data_scale(m2, specs))
    # the pattern is the single mesh's
    plan1, _ = run_gpu(m, None, f, gd, gn)
    assert np.array_equal(plan1.rowptr.cpu().numpy(), g["rowptr"])
    assert np.array_equal(plan1.colind[:plan1.nnz].cpu().numpy(), g["colind"])
