"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage (section / equation) it follows.  None of these checks
re-runs the oracle's own formula: they use worked examples printed in the paper,
closed-form stencils, invariants, exactness of quadrature, textbook special cases
and brute force on tiny inputs with a different local formula.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Fn, FN_CONST, FN_LINEAR, FN_SINPROD, FN_DUDN_SINPROD, FN_NODAL
from paper_1804_05156_amd import meshgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# --------------------------------------------------------------------------- sparse()
def test_sparse_worked_example():
    """Section 2.1, eq. (sparseA): the printed triplets give the printed 4x3 matrix,
    and the compressed-column pointer is [1 2 4 5] (1-based)."""
    g = _gold("sparse_example.json")
    i = np.array(g["i_one_based"]) - 1
    j = np.array(g["j_one_based"]) - 1
    s = np.array(g["s"], float)
    rowptr, colind, val = oracle.coo_to_csr(g["m"], g["n"], i, j, s)
    A = np.zeros((g["m"], g["n"]))
    for r in range(g["m"]):
        for q in range(rowptr[r], rowptr[r + 1]):
            A[r, colind[q]] = val[q]
    assert np.array_equal(A, np.array(g["dense"], float))
    assert rowptr.tolist() == [0, 1, 3, 3, 4]
    assert colind.tolist() == [0, 1, 2, 1]
    # compressed columns = compressed rows of the transpose
    cptr, rind, cval = oracle.coo_to_csr(g["n"], g["m"], j, i, s)
    assert (cptr + 1).tolist() == g["csc_colptr_one_based"]
    # find(A) lists entries column by column: that is the printed (i, j) order (Section 2.2)
    listed = [(int(rind[q]) + 1, c + 1) for c in range(g["n"]) for q in range(cptr[c], cptr[c + 1])]
    assert listed == list(zip(g["i_one_based"], g["j_one_based"]))


def test_spmv_worked_example_and_row_sums():
    """Section 2.1: the printed 4x3 matrix applied to unit vectors gives its printed
    columns; an assembled stiffness matrix maps constants to zero (the gradients
    of the barycentric coordinates sum to zero, Section 3.1.1)."""
    g = _gold("sparse_example.json")
    i = np.array(g["i_one_based"]) - 1
    j = np.array(g["j_one_based"]) - 1
    rowptr, colind, val = oracle.coo_to_csr(g["m"], g["n"], i, j, np.array(g["s"], float))
    dense = np.array(g["dense"], float)
    for c in range(g["n"]):
        e = np.zeros(g["n"])
        e[c] = 1.0
        assert np.array_equal(oracle.spmv(rowptr, colind, val, e), dense[:, c])
    x = np.array([0.5, -2.0, 3.0])
    expect = [sum(dense[r, c] * x[c] for c in range(g["n"])) for r in range(g["m"])]
    assert np.array_equal(oracle.spmv(rowptr, colind, val, x), np.array(expect))
    m = meshgen.square_mesh(9, jitter=0.2, permute=True, seed=61, kappa="lognormal")
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa)
    y = oracle.spmv(a.rowptr, a.colind, a.val, np.ones(m.n_node))
    assert np.abs(y).max() <= 1e-13 * np.abs(a.val).max()


def test_sparse_adds_duplicates_in_order():
    """Section 2.2: a repeated (i, j) pair is added; entries summing to zero stay stored."""
    i = np.array([1, 0, 1, 1, 0])
    j = np.array([1, 0, 1, 0, 0])
    s = np.array([2.0, 1.0, 5.0, 3.0, -1.0])
    rowptr, colind, val = oracle.coo_to_csr(2, 2, i, j, s)
    assert rowptr.tolist() == [0, 1, 3]
    assert colind.tolist() == [0, 0, 1]
    assert val.tolist() == [0.0, 3.0, 7.0]   # (0,0): 1 + (-1) = 0 kept explicitly


def test_sparse_rejects_out_of_range():
    with pytest.raises(oracle.OracleError):
        oracle.coo_to_csr(2, 2, np.array([2]), np.array([0]), np.array([1.0]))


# --------------------------------------------------------------------------- local stiffness
def test_reference_triangle():
    """Section 3.1.1: gradients of the reference barycentrics and the local matrix."""
    g = _gold("reference_simplex.json")
    K, G, area = oracle.local_stiffness(np.array(g["vertices"]))
    assert area == g["area"]
    assert np.array_equal(G, np.array(g["grad"]))
    assert np.array_equal(K, np.array(g["stiffness"]))


def test_reference_tetrahedron():
    """Unit tetrahedron 0, e1, e2, e3: lambda_2..4 = x, y, z, lambda_1 = 1-x-y-z,
    volume 1/6 (textbook closed form)."""
    p = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    K, G, vol = oracle.local_stiffness(p)
    assert vol == pytest.approx(1 / 6, rel=1e-15)
    assert np.allclose(G, [[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], atol=1e-15)
    Kx = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6
    assert np.allclose(K, Kx, atol=1e-15)


def _random_simplex(rng, dim):
    while True:
        p = rng.standard_normal((dim + 1, dim))
        E = (p[1:] - p[0]).T
        if np.linalg.det(E) > 0.05:
            return p


@pytest.mark.parametrize("dim", [2, 3])
def test_gradients_are_barycentric(dim):
    """lambda_a(x_b) = delta_ab fixes every gradient: grad lambda_a . (x_b - x_c) =
    delta_ab - delta_ac, and the gradients sum to zero (Section 3.1.3)."""
    rng = np.random.default_rng(10 + dim)
    for _ in range(20):
        p = _random_simplex(rng, dim)
        K, G, meas = oracle.local_stiffness(p)
        for a in range(dim + 1):
            for b in range(dim + 1):
                for c in range(dim + 1):
                    want = float(a == b) - float(a == c)
                    assert G[a] @ (p[b] - p[c]) == pytest.approx(want, abs=1e-12)
        assert np.allclose(G.sum(axis=0), 0, atol=1e-12)
        vol = abs(np.linalg.det((p[1:] - p[0]).T)) / math.factorial(dim)
        assert meas == pytest.approx(vol, rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_local_matrix_against_scaled_normals(dim):
    """Eq. (dlambda): a_ij = n_i . n_j / (d!^2 |t|) with n_i the scaled inward normal
    of the face opposite vertex i (edge rotation in 2-D, cross product in 3-D)."""
    rng = np.random.default_rng(20 + dim)
    for _ in range(20):
        p = _random_simplex(rng, dim)
        K, G, meas = oracle.local_stiffness(p)
        n = np.zeros((dim + 1, dim))
        if dim == 2:
            for i in range(3):
                e = p[(i + 2) % 3] - p[(i + 1) % 3]       # rotate CCW to point at vertex i
                n[i] = [-e[1], e[0]]
        else:
            for i in range(4):
                f = [k for k in range(4) if k != i]
                v = np.cross(p[f[1]] - p[f[0]], p[f[2]] - p[f[0]])
                if v @ (p[i] - p[f[0]]) < 0:
                    v = -v
                n[i] = v
        Kn = (n @ n.T) / (math.factorial(dim) ** 2 * meas)
        assert np.allclose(K, Kn, rtol=1e-12, atol=1e-12 * np.abs(Kn).max())


def test_inverted_or_flat_element_is_rejected():
    """Section 1.1 requires positive orientation."""
    with pytest.raises(oracle.OracleError) as e:
        oracle.local_stiffness(np.array([[0, 1.0], [1, 0], [0, 0]]))   # clockwise
    assert e.value.code == oracle.EMESH
    with pytest.raises(oracle.OracleError):
        oracle.local_stiffness(np.array([[0, 0.0], [1, 0], [2, 0]]))   # flat


# --------------------------------------------------------------------------- stiffness matrix
def _dense(asm):
    return asm.dense()


def test_five_point_stencil_uniform_square():
    """Uniform 33x33 grid with "/" diagonals: interior rows are 4 at the centre, -1 at
    the four axis neighbours and exactly 0 at the two diagonal neighbours; every
    intermediate is a dyadic rational, so these are exact."""
    n = 33
    m = meshgen.square_mesh(n)
    a = oracle.assemble(m.node, m.elem, m.bdflag)
    N = n * n
    assert a.nnz == 3 * N + 2 * m.n_elem - 2
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            r = j * n + i
            cols = a.colind[a.rowptr[r]:a.rowptr[r + 1]].tolist()
            vals = a.val[a.rowptr[r]:a.rowptr[r + 1]].tolist()
            want = {r - n - 1: 0.0, r - n: -1.0, r - 1: -1.0, r: 4.0, r + 1: -1.0, r + n: -1.0,
                    r + n + 1: 0.0}
            assert cols == sorted(want)
            assert vals == [want[c] for c in cols]
    # exact symmetry and zero row sums
    A = _dense(a)
    assert np.array_equal(A, A.T)
    assert np.array_equal(A.sum(axis=1), np.zeros(N))


def test_seven_point_stencil_kuhn_cube():
    """Kuhn tetrahedra of a uniform cube grid with spacing h: interior rows are 6h at
    the centre, -h at the six axis neighbours, 0 at the eight face/body-diagonal
    neighbours joined by an edge (15 stored entries)."""
    n = 5
    h = 1.0 / (n - 1)
    m = meshgen.kuhn_cube(n)
    a = oracle.assemble(m.node, m.elem, m.bdflag)
    for l in range(1, n - 1):
        for j in range(1, n - 1):
            for i in range(1, n - 1):
                r = i + n * (j + n * l)
                cols = a.colind[a.rowptr[r]:a.rowptr[r + 1]]
                vals = a.val[a.rowptr[r]:a.rowptr[r + 1]]
                assert cols.size == 15
                axis = {r + 1, r - 1, r + n, r - n, r + n * n, r - n * n}
                for c, v in zip(cols, vals):
                    if c == r:
                        assert v == pytest.approx(6 * h, rel=1e-14)
                    elif c in axis:
                        assert v == pytest.approx(-h, rel=1e-14)
                    else:
                        assert abs(v) < 1e-15
    # edge count of the Kuhn grid: axis + face-diagonal + body-diagonal edges
    E = 3 * n * n * (n - 1) + 3 * n * (n - 1) ** 2 + (n - 1) ** 3
    assert a.nnz == n ** 3 + 2 * E


@pytest.mark.parametrize("dim", [2, 3])
def test_invariants_on_jittered_mesh(dim):
    """Symmetric, A.1 = 0 (the gradients sum to zero), positive semidefinite, and the
    patch test: A x = 0 at interior rows for any linear x when kappa is constant."""
    if dim == 2:
        m = meshgen.square_mesh(9, jitter=0.2, permute=True, seed=7, kappa="lognormal")
    else:
        m = meshgen.kuhn_cube(4, jitter=0.15, permute=True, seed=7, kappa="lognormal")
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa)
    A = _dense(a)
    scale = np.sqrt(np.outer(np.diag(A), np.diag(A)))
    assert np.all(np.abs(A - A.T) <= 1e-14 * scale + 0)
    assert np.all(np.abs(A.sum(axis=1)) <= 1e-13 * np.diag(A))
    assert np.linalg.eigvalsh(A).min() > -1e-12 * np.diag(A).max()
    a1 = oracle.assemble(m.node, m.elem, m.bdflag, None)
    A1 = _dense(a1)
    onbd = np.zeros(m.n_node, bool)
    for f in range(dim + 1):
        sel = m.bdflag[f] > 0
        for e in range(dim + 1):
            if e != f:
                onbd[m.elem[e, sel]] = True
    interior = ~onbd
    for c in range(dim):
        y = A1 @ m.node[c]
        assert np.all(np.abs(y[interior]) <= 1e-13 * np.diag(A1)[interior])


@pytest.mark.parametrize("dim", [2, 3])
def test_brute_force_dense_assembly(dim):
    """Brute force on tiny meshes: a dense element loop (the straightforward assembly
    of Section 3.1.1) with the scaled-normal local matrix of eq. (dlambda)."""
    if dim == 2:
        m = meshgen.square_mesh(5, jitter=0.2, permute=True, seed=3, kappa="lognormal")
    else:
        m = meshgen.kuhn_cube(3, jitter=0.2, permute=True, seed=3, kappa="lognormal")
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa)
    N = m.n_node
    D = np.zeros((N, N))
    for t in range(m.n_elem):
        v = m.elem[:, t]
        p = m.node[:, v].T
        vol = np.linalg.det((p[1:] - p[0]).T) / math.factorial(dim)
        n = np.zeros((dim + 1, dim))
        for i in range(dim + 1):
            f = [k for k in range(dim + 1) if k != i]
            if dim == 2:
                e = p[f[1]] - p[f[0]]
                w = np.array([-e[1], e[0]])
            else:
                w = np.cross(p[f[1]] - p[f[0]], p[f[2]] - p[f[0]])
            if w @ (p[i] - p[f[0]]) < 0:
                w = -w
            n[i] = w
        Kt = m.kappa[t] * (n @ n.T) / (math.factorial(dim) ** 2 * vol)
        for i in range(dim + 1):
            for j in range(dim + 1):
                D[v[i], v[j]] += Kt[i, j]
    A = _dense(a)
    scale = np.sqrt(np.outer(np.abs(np.diag(D)), np.abs(np.diag(D))))
    assert np.all(np.abs(A - D) <= 1e-13 * scale)
    # pattern: every vertex pair sharing an element, and nothing else
    P = np.zeros((N, N), bool)
    for t in range(m.n_elem):
        v = m.elem[:, t]
        P[np.ix_(v, v)] = True
    assert a.nnz == int(P.sum())
    for r in range(N):
        assert a.colind[a.rowptr[r]:a.rowptr[r + 1]].tolist() == np.nonzero(P[r])[0].tolist()


def test_permutation_invariance():
    """Remark of Section 1.1: relabelling vertices or reordering elements describes the
    same mesh, so A changes only by the relabelling (values up to rounding)."""
    m = meshgen.square_mesh(7, jitter=0.2, seed=4, kappa="lognormal")
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa)
    rng = np.random.default_rng(99)
    perm = rng.permutation(m.n_node)
    order = rng.permutation(m.n_elem)
    node2 = np.empty_like(m.node)
    node2[:, perm] = m.node
    elem2 = perm[m.elem][:, order].astype(np.int32)
    a2 = oracle.assemble(node2, elem2, m.bdflag[:, order], m.kappa[order])
    A = _dense(a)
    A2 = _dense(a2)
    P = np.zeros_like(A, dtype=bool)
    for r in range(m.n_node):
        P[r, a.colind[a.rowptr[r]:a.rowptr[r + 1]]] = True
    P2 = np.zeros_like(A, dtype=bool)
    for r in range(m.n_node):
        P2[r, a2.colind[a2.rowptr[r]:a2.rowptr[r + 1]]] = True
    assert np.array_equal(P2[np.ix_(perm, perm)], P)
    assert np.allclose(A2[np.ix_(perm, perm)], A, rtol=0, atol=1e-13 * np.abs(A).max())
    assert a2.nnz == a.nnz
    assert np.allclose(a2.b[perm], a.b, atol=1e-15)


# --------------------------------------------------------------------------- load vector
@pytest.mark.parametrize("dim", [2, 3])
def test_load_constant_f(dim):
    """f = 1: b_i = sum over elements containing i of |t|/(d+1)."""
    m = meshgen.square_mesh(6, jitter=0.2, seed=1) if dim == 2 else meshgen.kuhn_cube(4, jitter=0.2, seed=1)
    a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_CONST, (1.0,)))
    want = np.zeros(m.n_node)
    for t in range(m.n_elem):
        p = m.node[:, m.elem[:, t]].T
        vol = np.linalg.det((p[1:] - p[0]).T) / math.factorial(dim)
        want[m.elem[:, t]] += vol / (dim + 1)
    assert np.allclose(a.b_load, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_load_exact_for_linear_f(dim):
    """The 2-D three-midpoint rule and the 3-D degree-2 rule are exact for quadratics
    (Section 4), so for linear f: b_a = sum_j f(x_j) |t| (1 + delta_aj) / ((d+1)(d+2))."""
    m = meshgen.square_mesh(6, jitter=0.2, seed=2) if dim == 2 else meshgen.kuhn_cube(4, jitter=0.2, seed=2)
    c = (0.3, -1.2, 0.7, 2.1)
    fn = Fn(FN_LINEAR, c)
    a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn)
    fv = c[0] + sum(c[1 + k] * m.node[k] for k in range(dim))
    want = np.zeros(m.n_node)
    den = (dim + 1) * (dim + 2)
    for t in range(m.n_elem):
        v = m.elem[:, t]
        p = m.node[:, v].T
        vol = np.linalg.det((p[1:] - p[0]).T) / math.factorial(dim)
        for i in range(dim + 1):
            want[v[i]] += vol * (fv[v].sum() + fv[v[i]]) / den
    assert np.allclose(a.b_load, want, rtol=1e-12, atol=1e-15)
    # nodal f interpolating the same linear function gives the same vector
    a2 = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_NODAL, nodal=fv))
    assert np.allclose(a2.b_load, want, rtol=1e-12, atol=1e-15)


def test_quadratic_exactness_of_sin_rule_limit():
    """Three-midpoint rule on the unit square: for f = sin(pi x) sin(pi y) the load
    total converges to 4/pi^2 at least at second order (rule of order 2, Section 4)."""
    errs = []
    for n in (9, 17, 33):
        m = meshgen.square_mesh(n)
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_SINPROD, (1.0,)))
        errs.append(abs(a.b_load.sum() - 4 / math.pi ** 2))
    r1 = math.log2(errs[0] / errs[1])
    r2 = math.log2(errs[1] / errs[2])
    assert r1 > 1.9 and r2 > 1.9          # at least second order (fourth on uniform grids)


# --------------------------------------------------------------------------- load rules of Section 4
def _rule_mesh(dim, seed):
    return meshgen.square_mesh(7, jitter=0.2, seed=seed) if dim == 2 else meshgen.kuhn_cube(4, jitter=0.2, seed=seed)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("rule", [oracle.LOAD_CENTROID, oracle.LOAD_TRAPEZOID])
def test_first_order_rules_exact_for_constant_f(dim, rule):
    """Section 4: the one-point and the trapezoidal rules are exact for linear
    integrands, so for constant f (integrand f phi_i, linear) they give the exact
    load, which the default rule (exact for quadratics) also gives."""
    m = _rule_mesh(dim, 11)
    fn = Fn(FN_CONST, (1.7,))
    ref = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn).b_load
    got = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn, rule=rule).b_load
    assert np.allclose(got, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_first_order_rules_error_identity_for_linear_f(dim):
    """For linear f on a simplex, int_t f phi_a = |t| (sum_e f_e + f_a) / ((d+1)(d+2))
    while the one-point rule gives |t| sum_e f_e / (d+1)^2 and the trapezoidal rule
    |t| f_a / (d+1).  Their errors satisfy trap - exact = (d+1) (exact - centroid)
    element by element, hence b_trap + (d+1) b_centroid = (d+2) b_exact for the
    assembled vectors (the default rule is exact here, test above).  A wrong point,
    weight or vertex in either first-order rule breaks the identity."""
    m = _rule_mesh(dim, 12)
    fn = Fn(FN_LINEAR, (0.4, -1.3, 0.9, 1.6))
    ex = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn).b_load
    ce = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn, rule=oracle.LOAD_CENTROID).b_load
    tr = oracle.assemble(m.node, m.elem, m.bdflag, None, f=fn, rule=oracle.LOAD_TRAPEZOID).b_load
    scale = np.abs(ex).max()
    assert np.allclose(tr + (dim + 1) * ce, (dim + 2) * ex, rtol=0, atol=1e-13 * scale)
    # the three vectors differ (the identity is not trivially met)
    assert np.abs(ce - ex).max() > 1e-6 * scale and np.abs(tr - ex).max() > 1e-6 * scale


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("rule", [oracle.LOAD_CENTROID, oracle.LOAD_TRAPEZOID])
def test_first_order_rules_integrate_linear_f(dim, rule):
    """The hat functions sum to one, so sum_i b_i is the rule applied to f itself,
    exact for linear f: on the unit square / cube, int (c0 + c . x) = c0 + sum(c)/2."""
    m = _rule_mesh(dim, 13)
    c = (0.4, -1.3, 0.9, 1.6)
    b = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_LINEAR, c), rule=rule).b_load
    assert abs(b.sum() - (c[0] + sum(c[1:1 + dim]) / 2)) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_trapezoidal_rule_is_nodal_scaling(dim):
    """The trapezoidal rule samples f at the vertices only, where phi_i is 1 at x_i and
    0 at the others: b_i = f(x_i) sum_{t containing i} |t|/(d+1), i.e. f(x_i) times
    the load of f = 1 (the lumped mass)."""
    m = _rule_mesh(dim, 14)
    one = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_CONST, (1.0,)),
                          rule=oracle.LOAD_TRAPEZOID).b_load
    b = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_SINPROD, (2.5,)),
                        rule=oracle.LOAD_TRAPEZOID).b_load
    fx = 2.5 * np.prod(np.sin(math.pi * m.node), axis=0)
    assert np.allclose(b, fx * one, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("rule", [oracle.LOAD_CENTROID, oracle.LOAD_TRAPEZOID])
def test_first_order_rules_keep_second_order_convergence(rule):
    """Section 3.2: a one-point rule is adequate for the linear element on
    quasi-uniform meshes; the L2 error of u = sin(pi x) sin(pi y) still decays like
    h^2 with either first-order rule."""
    errs = []
    for n in (9, 17, 33):
        m = meshgen.square_mesh(n)
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_SINPROD, (2 * math.pi ** 2,)), rule=rule)
        u, _, _ = oracle.solve(a, rtol=1e-13, method="direct")
        errs.append(_l2_error_2d(m, u))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(1.85 < r < 2.15 for r in rates), rates


def test_unknown_load_rule_rejected():
    m = _rule_mesh(2, 15)
    with pytest.raises(oracle.OracleError):
        oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_CONST, (1.0,)), rule=3)


# --------------------------------------------------------------------------- boundary conditions
def test_boundary_flag_example():
    """Section 1.2 example bdFlag = [1 0 2]: the side opposite vertex 1 is Dirichlet,
    the side opposite vertex 3 is Neumann (midpoint rule: |e| g / 2 to each end)."""
    g = _gold("boundary_example.json")
    node = np.array([[0.0, 2.0, 0.0], [0.0, 0.0, 1.0]])           # vertices (0,0), (2,0), (0,1)
    elem = (np.array(g["elem_one_based"], np.int32) - 1).reshape(3, 1)
    bd = np.array(g["bdflag"], np.int8).reshape(3, 1)
    a = oracle.assemble(node, elem, bd, None, gN=Fn(FN_CONST, (3.0,)))
    dset = sorted(np.nonzero(a.is_d)[0] + 1)
    assert dset == sorted(g["dirichlet_side_one_based"])
    nside = np.array(g["neumann_side_one_based"]) - 1
    L = np.linalg.norm(node[:, nside[0]] - node[:, nside[1]])
    want = np.zeros(3)
    want[nside] = L * 3.0 / 2
    assert np.allclose(a.b_load, want, rtol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_neumann_constant_total(dim):
    """Constant g_N: the Neumann part of b sums to g_N times the Neumann measure."""
    if dim == 2:
        m = meshgen.square_mesh(7, jitter=0.2, seed=5, sides=(2, 2, 2, 1))
        meas = 3.0
    else:
        m = meshgen.kuhn_cube(4, jitter=0.2, seed=5)        # x-planes Dirichlet, four Neumann faces
        meas = 4.0
    a = oracle.assemble(m.node, m.elem, m.bdflag, None, gN=Fn(FN_CONST, (1.7,)))
    assert a.b_load.sum() == pytest.approx(1.7 * meas, rel=1e-13)


def test_unsupported_and_invalid_inputs():
    m = meshgen.square_mesh(3)
    bd = m.bdflag.copy()
    bd[1, 0] = 4                                          # no such boundary type
    with pytest.raises(oracle.OracleError) as e:
        oracle.assemble(m.node, m.elem, bd)
    assert e.value.code == oracle.EINVAL
    bd[1, 0] = 3
    with pytest.raises(oracle.OracleError) as e:          # Robin coefficient must be >= 0
        oracle.assemble(m.node, m.elem, bd, alpha=-1.0)
    assert e.value.code == oracle.EINVAL
    el = m.elem.copy()
    el[0, 0] = m.n_node
    with pytest.raises(oracle.OracleError) as e:
        oracle.assemble(m.node, el, m.bdflag)
    assert e.value.code == oracle.EINVAL
    el = m.elem.copy()
    el[[0, 1], 0] = el[[1, 0], 0]                         # clockwise element
    with pytest.raises(oracle.OracleError) as e:
        oracle.assemble(m.node, el, m.bdflag)
    assert e.value.code == oracle.EMESH


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_solution_reproduced(dim):
    """Section 3.3: with f = 0, constant kappa and linear g_D the discrete solution is
    the linear function itself (it lies in the finite element space)."""
    if dim == 2:
        m = meshgen.square_mesh(17, jitter=0.2, permute=True, seed=8)
    else:
        m = meshgen.kuhn_cube(5, jitter=0.2, permute=True, seed=8,
                              faces=(1, 1, 1, 1, 1, 1))
    c = (0.5, 1.25, -2.0, 0.75)
    a = oracle.assemble(m.node, m.elem, m.bdflag, np.full(m.n_elem, 2.5), gD=Fn(FN_LINEAR, c))
    u, _, rel = oracle.solve(a)
    exact = c[0] + sum(c[1 + k] * m.node[k] for k in range(dim))
    assert np.abs(u - exact).max() < 1e-12
    assert rel < 1e-13
    ucg, it, relcg = oracle.solve(a, rtol=1e-13, method="cg")
    assert it > 0 and relcg < 1e-12
    assert np.abs(ucg - exact).max() < 1e-11


def _l2_error_2d(m, u_h):
    """sqrt(sum_t |t|/3 sum_edges (u - u_h)^2 at edge midpoints), u = sin(pi x) sin(pi y)."""
    s = 0.0
    x, y = m.node
    for t in range(m.n_elem):
        v = m.elem[:, t]
        area = 0.5 * abs((x[v[1]] - x[v[0]]) * (y[v[2]] - y[v[0]]) - (x[v[2]] - x[v[0]]) * (y[v[1]] - y[v[0]]))
        for k in range(3):
            i, j = v[(k + 1) % 3], v[(k + 2) % 3]
            mx, my = (x[i] + x[j]) / 2, (y[i] + y[j]) / 2
            e = math.sin(math.pi * mx) * math.sin(math.pi * my) - (u_h[i] + u_h[j]) / 2
            s += area / 3 * e * e
    return math.sqrt(s)


def test_second_order_convergence_2d():
    """u = sin(pi x) sin(pi y), f = 2 pi^2 u, g_D = 0: the L2 error decays like h^2."""
    errs = []
    for n in (9, 17, 33, 65):
        m = meshgen.square_mesh(n)
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_SINPROD, (2 * math.pi ** 2,)))
        u, _, _ = oracle.solve(a, rtol=1e-13, method="direct" if n <= 33 else "cg")
        errs.append(_l2_error_2d(m, u))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(1.9 < r < 2.1 for r in rates), rates
    assert errs[2] < 2e-3                                   # the 33x33 grid


@pytest.mark.slow
def test_second_order_convergence_3d_mixed():
    """u = sin sin sin on the unit cube, f = 3 pi^2 u, Dirichlet on x = 0, 1 (u = 0),
    Neumann g_N = du/dn elsewhere: the root-mean-square nodal error decays like h^2."""
    errs = []
    for n in (9, 17, 33):
        m = meshgen.kuhn_cube(n)
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_SINPROD, (3 * math.pi ** 2,)),
                            gN=Fn(FN_DUDN_SINPROD, (1.0,)))
        u, _, _ = oracle.solve(a, rtol=1e-12, method="cg")
        exact = np.prod(np.sin(math.pi * m.node), axis=0)
        errs.append(math.sqrt(np.mean((u - exact) ** 2)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(1.9 < r < 2.3 for r in rates), rates


# --------------------------------------------------------------------------- Robin sides
def test_robin_single_element_closed_form():
    """Section 1.2, type 3: on the reference triangle with the side opposite vertex 0
    (length sqrt 2) of Robin type, A = K + alpha sqrt(2)/6 [[2, 1], [1, 2]] on vertices
    1, 2 and constant g_R puts |F| g_R / 2 on each side vertex; on the reference
    tetrahedron with the face opposite vertex 0 (area sqrt(3)/2) the mass term is
    alpha |F| (1 + delta_ij) / 12."""
    alpha, g = 3.0, 2.0
    for dim in (2, 3):
        if dim == 2:
            node = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
            K = np.array([[1.0, -0.5, -0.5], [-0.5, 0.5, 0.0], [-0.5, 0.0, 0.5]])
            fm, den = math.sqrt(2.0), 6.0
        else:
            node = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
            K = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]], float) / 6.0
            fm, den = math.sqrt(3.0) / 2.0, 12.0
        nv = dim + 1
        elem = np.arange(nv, dtype=np.int32).reshape(nv, 1)
        bd = np.zeros((nv, 1), np.int8)
        bd[0, 0] = 3
        a = oracle.assemble(node, elem, bd, gR=Fn(FN_CONST, (g,)), alpha=alpha)
        M = np.zeros((nv, nv))
        for i in range(1, nv):
            for j in range(1, nv):
                M[i, j] = alpha * fm * (2.0 if i == j else 1.0) / den
        assert np.allclose(a.dense(), K + M, rtol=0, atol=1e-15)
        expect_b = np.array([0.0] + [fm * g / dim] * dim)
        assert np.allclose(a.b, expect_b, rtol=0, atol=1e-15)


def test_robin_totals_on_jittered_square():
    """All four sides Robin: the rows of K sum to zero, so 1^T A 1 = alpha |boundary| = 4
    alpha, and constant g_R loads g_R |boundary| in total."""
    m = meshgen.square_mesh(11, jitter=0.2, permute=True, seed=91, kappa="lognormal", sides=(3, 3, 3, 3))
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, gR=Fn(FN_CONST, (0.7,)), alpha=2.5)
    assert abs(float(a.val.sum()) - 4 * 2.5) <= 1e-12
    assert abs(float(a.b.sum()) - 4 * 0.7) <= 1e-12


def test_robin_second_order_convergence():
    """u = cos(pi x) cos(pi y): du/dn = 0 on the sides, so g_R = alpha u there; with
    f = 2 pi^2 u the L2 error decays like h^2 (data as nodal interpolants)."""
    errs = []
    alpha = 1.5
    for n in (9, 17, 33):
        m = meshgen.square_mesh(n, sides=(3, 3, 3, 3))
        exact = np.cos(math.pi * m.node[0]) * np.cos(math.pi * m.node[1])
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=Fn(FN_NODAL, (0.0,), 2 * math.pi ** 2 * exact),
                            gR=Fn(FN_NODAL, (0.0,), alpha * exact), alpha=alpha)
        u, _, _ = oracle.solve(a, method="direct")
        errs.append(_l2_error_cos(m, u))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(1.8 < r < 2.2 for r in rates), rates


# --------------------------------------------------------------------------- pure Neumann problem
def _cos_problem(n, seed=None, jitter=0.0):
    """u = cos(pi x) cos(pi y) on the unit square: f = 2 pi^2 u, du/dn = 0 on every side,
    zero mean.  f enters as nodal values (its P1 interpolant)."""
    m = meshgen.square_mesh(n, jitter=jitter, permute=seed is not None, seed=seed, sides=(2, 2, 2, 2))
    exact = np.cos(math.pi * m.node[0]) * np.cos(math.pi * m.node[1])
    f = Fn(FN_NODAL, (0.0,), 2 * math.pi ** 2 * exact)
    return m, f, exact


def test_pure_neumann_second_order_convergence():
    """Section 3.3: with b shifted to mean zero, one vertex fixed and the zero-mean
    shift applied, the discrete solution converges like h^2 to the zero-mean exact
    solution u = cos(pi x) cos(pi y)."""
    errs = []
    for n in (9, 17, 33):
        m, f, exact = _cos_problem(n)
        a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=f)
        u, _, _, _ = oracle.neumann_solve(a, m.node, m.elem, method="direct")
        errs.append(_l2_error_cos(m, u))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(1.8 < r < 2.2 for r in rates), rates


def _l2_error_cos(m, u_h):
    s = 0.0
    x, y = m.node
    for t in range(m.n_elem):
        v = m.elem[:, t]
        area = 0.5 * abs((x[v[1]] - x[v[0]]) * (y[v[2]] - y[v[0]]) - (x[v[2]] - x[v[0]]) * (y[v[1]] - y[v[0]]))
        for k in range(3):
            i, j = v[(k + 1) % 3], v[(k + 2) % 3]
            mx, my = (x[i] + x[j]) / 2, (y[i] + y[j]) / 2
            e = math.cos(math.pi * mx) * math.cos(math.pi * my) - (u_h[i] + u_h[j]) / 2
            s += area / 3 * e * e
    return math.sqrt(s)


def test_pure_neumann_properties():
    """Equation (meanb): after the shift b sums to zero, so A u = b - mean(b) holds at
    every row, the fixed one included (the rows of A sum to zero); the result has
    zero area-weighted mean; constant kappa scaling divides u by the constant."""
    m, f, _ = _cos_problem(13, seed=5, jitter=0.2)
    a = oracle.assemble(m.node, m.elem, m.bdflag, None, f=f)
    u, _, _, mean_b = oracle.neumann_solve(a, m.node, m.elem, method="direct")
    r = oracle.spmv(a.rowptr, a.colind, a.val, u) - (a.b - mean_b)
    assert np.abs(r).max() <= 1e-12 * np.abs(a.b).max()
    area = oracle.measures(m.node, m.elem)
    assert abs(float(np.sum(area * u[m.elem].mean(axis=0)))) <= 1e-14 * np.abs(u).max()
    a3 = oracle.assemble(m.node, m.elem, m.bdflag, np.full(m.n_elem, 3.0), f=f)
    u3, _, _, _ = oracle.neumann_solve(a3, m.node, m.elem, method="direct")
    assert np.abs(3.0 * u3 - u).max() <= 1e-12 * np.abs(u).max()
    with pytest.raises(ValueError):
        md = meshgen.square_mesh(5)
        oracle.neumann_solve(oracle.assemble(md.node, md.elem, md.bdflag), md.node, md.elem)


# --------------------------------------------------------------------------- adjoint gradient
def _fd_setup():
    m = meshgen.square_mesh(17, jitter=0.2, seed=517, kappa="lognormal")
    f = Fn(FN_SINPROD, (2 * math.pi ** 2,))
    rng = np.random.default_rng(518)
    kobs = np.exp(rng.standard_normal(m.n_elem))
    aobs = oracle.assemble(m.node, m.elem, m.bdflag, kobs, f=f)
    u_obs, _, _ = oracle.solve(aobs)
    return m, f, u_obs


def _J(m, f, kappa, u_obs):
    a = oracle.assemble(m.node, m.elem, m.bdflag, kappa, f=f)
    u, _, _ = oracle.solve(a)
    return 0.5 * float((u - u_obs) @ (u - u_obs))


@pytest.mark.slow
def test_adjoint_matches_central_differences():
    """dJ/dkappa from the adjoint equals central finite differences of J with step
    1e-4 kappa_t (direct solves), componentwise to 1e-6 where |g| >= 1e-3 max|g|."""
    m, f, u_obs = _fd_setup()
    J, g, u, lam = oracle.objective_and_grad(m.node, m.elem, m.bdflag, m.kappa, u_obs, f=f)
    gfd = np.zeros(m.n_elem)
    for t in range(m.n_elem):
        d = 1e-4 * m.kappa[t]
        kp = m.kappa.copy(); kp[t] += d
        km = m.kappa.copy(); km[t] -= d
        gfd[t] = (_J(m, f, kp, u_obs) - _J(m, f, km, u_obs)) / (2 * d)
    big = np.abs(gfd) >= 1e-3 * np.abs(gfd).max()
    rel = np.abs(g[big] - gfd[big]) / np.abs(gfd[big])
    assert rel.max() < 1e-6
    assert np.abs(g - gfd).max() < 1e-7 * np.abs(gfd).max()


def test_adjoint_homogeneity_identity():
    """With g_D = 0 and g_N = 0, u(c kappa) = u / c, so sum_t kappa_t dJ/dkappa_t =
    -(u - u_obs) . u exactly."""
    m, f, u_obs = _fd_setup()
    J, g, u, lam = oracle.objective_and_grad(m.node, m.elem, m.bdflag, m.kappa, u_obs, f=f)
    lhs = float(m.kappa @ g)
    rhs = -float((u - u_obs) @ u)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # elements whose vertices are all Dirichlet nodes see lambda = 0 there
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=f)
    alld = np.all(a.is_d[m.elem].astype(bool), axis=0)
    assert alld.sum() == 2 and np.all(g[alld] == 0.0)
