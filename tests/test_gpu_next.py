"""Rows next to the core path: the pure Neumann problem (Section 3.3, equations
(compatible) and (meanb)), Robin sides (boundary type 3 of Section 1.2) and the
L-shaped domain of Section 1.1, on the GPU against the oracle.

Pure Neumann: the oracle fixes vertex 0, solves directly and shifts u to zero
mean; the GPU runs the same steps with PCG.  Both results are the unique zero-mean
solution of A u = b - mean(b), so they agree to the solver tolerance:
||u - u*|| <= cond rtol ||u*||, checked with the generous cond <= 1e4 N used by the
other solve tests.  L-shape: assembly parity (pattern bit-exact, values in the
1e-12 scale of the other parity tests) and the solve against the direct solve.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1804_05156_amd import meshgen
from gpu_helpers import compare, data_scale, fns, host, log, run_gpu, to_dev

pytestmark = pytest.mark.gpu

FE_FN_CONST, FE_FN_LINEAR, FE_FN_SINPROD, FE_FN_DUDN_SINPROD, FE_FN_NODAL = 1, 2, 3, 4, 5


def _cos_nodal(m):
    exact = np.prod(np.cos(math.pi * m.node), axis=0)
    return exact, m.dim * math.pi ** 2 * exact


def _area_mean(m, u):
    area = oracle.measures(m.node, m.elem)
    return float(np.sum(area * u[m.elem].mean(axis=0))) / float(np.sum(area))


@pytest.mark.parametrize("dim", [2, 3])
def test_pure_neumann_matches_oracle(dim):
    log(f"case: pure Neumann vs oracle dim={dim}")
    if dim == 2:
        m = meshgen.square_mesh(25, jitter=0.2, permute=True, seed=71, kappa="lognormal", sides=(2, 2, 2, 2))
    else:
        m = meshgen.kuhn_cube(7, jitter=0.15, permute=True, seed=71, kappa="lognormal", faces=(2,) * 6)
    _, fv = _cos_nodal(m)
    specs = [(FE_FN_NODAL, (0.0,), fv)]
    (f, fo), _, _ = fns(*specs)
    plan, asm = run_gpu(m, None, f)
    u, it, rel, mb = plan.neumann_solve(asm, rtol=1e-13)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo)
    compare(host(plan, asm), ora, data=data_scale(m, specs))
    uo, _, _, mbo = oracle.neumann_solve(ora, m.node, m.elem, method="direct")
    log(f"  iterations {it}, relres {rel:.2e}, mean(b) {mb:.3e} vs {mbo:.3e}")
    assert rel <= 1e-13 and it > 0
    assert abs(mb - mbo) <= 1e-12 * np.abs(ora.b).max()
    assert np.abs(u - uo).max() <= 1e-13 * 1e4 * m.n_node * np.abs(uo).max()
    assert abs(_area_mean(m, u)) <= 1e-12 * np.abs(u).max()
    # A u = b - mean(b) at every row, the fixed one included
    r = oracle.spmv(ora.rowptr, ora.colind, ora.val, u) - (ora.b - mbo)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(ora.b - mbo)


def test_pure_neumann_second_order_convergence_gpu():
    """u = cos(pi x) cos(pi y) (zero mean, du/dn = 0): L2 error decays like h^2."""
    log("case: pure Neumann convergence")
    errs = []
    for n in (17, 33, 65, 129):
        m = meshgen.square_mesh(n, sides=(2, 2, 2, 2))
        exact, fv = _cos_nodal(m)
        (f, _), _, _ = fns((FE_FN_NODAL, (0.0,), fv))
        plan, asm = run_gpu(m, None, f)
        u, _, _, _ = plan.neumann_solve(asm, rtol=1e-12)
        u = u.cpu().numpy()
        x, y = m.node
        X, Y = x[m.elem], y[m.elem]
        area = 0.5 * np.abs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]))
        U = u[m.elem]
        s = 0.0
        for k in range(3):
            i, j = (k + 1) % 3, (k + 2) % 3
            e = np.cos(math.pi * (X[i] + X[j]) / 2) * np.cos(math.pi * (Y[i] + Y[j]) / 2) - (U[i] + U[j]) / 2
            s += float(np.sum(area / 3 * e * e))
        errs.append(math.sqrt(s))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    log(f"  L2 errors {errs} rates {rates}")
    assert all(1.9 < r < 2.1 for r in rates)


def test_pure_neumann_rejects_dirichlet_and_repeats_bitwise():
    from paper_1804_05156_amd import femhip
    log("case: pure Neumann argument checks, determinism")
    m = meshgen.square_mesh(9)
    plan, asm = run_gpu(m)
    with pytest.raises(femhip.FemhipError) as e:
        plan.neumann_solve(asm)
    assert e.value.code == femhip.FE_EINVAL
    m = meshgen.square_mesh(65, jitter=0.2, permute=True, seed=72, kappa="lognormal", sides=(2, 2, 2, 2))
    _, fv = _cos_nodal(m)
    (f, _), _, _ = fns((FE_FN_NODAL, (0.0,), fv))
    plan, asm = run_gpu(m, None, f)
    u1, i1, r1, m1 = plan.neumann_solve(asm, rtol=1e-10)
    u2, i2, r2, m2 = plan.neumann_solve(asm, rtol=1e-10)
    torch.cuda.synchronize()
    assert (i1, r1, m1) == (i2, r2, m2) and torch.equal(u1, u2)


@pytest.mark.parametrize("n", [9, 17])
def test_lshape_assembly_and_solve(n):
    """The L-shaped domain (-1,1)^2 minus the lower right quadrant, lognormal kappa,
    f = 1, g_D = 0: assembly parity and the solve against the direct solve."""
    log(f"case: L-shape n={n}")
    m = meshgen.lshape_mesh(n, seed=80 + n, kappa="lognormal")
    specs = [(FE_FN_CONST, (1.0,))]
    (f, fo), _, _ = fns(*specs)
    plan, asm = run_gpu(m, None, f)
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs))
    u, it, rel = plan.solve(asm, rtol=1e-13)
    u = u.cpu().numpy()
    uo, _, _ = oracle.solve(ora, method="direct")
    log(f"  worst scaled value error {worst:.2e}, iterations {it}")
    assert np.abs(u - uo).max() <= 1e-13 * 1e4 * m.n_node * np.abs(uo).max()


def test_lshape_linear_solution_reproduced():
    """f = 0, constant kappa, linear g_D on the L-shape: u_h is the linear function
    (the re-entrant corner does not matter for a function in the finite element space)."""
    log("case: L-shape linear reproduction")
    m = meshgen.lshape_mesh(21)
    c = (0.25, -1.5, 0.75)
    (f, _), (gd, _), _ = fns(None, (FE_FN_LINEAR, c))
    plan, asm = run_gpu(m, None, None, gd)
    u, _, _ = plan.solve(asm, rtol=1e-14)
    exact = c[0] + c[1] * m.node[0] + c[2] * m.node[1]
    assert np.abs(u.cpu().numpy() - exact).max() < 1e-10


def _robin_case(m, specs, gr_spec, alpha):
    from paper_1804_05156_amd import femhip
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    (gr, gro), _, _ = fns(gr_spec)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    asm = plan.assemble(kap, f, gd, gn, gR=gr, robin_alpha=alpha)
    plan.check()
    torch.cuda.synchronize()
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno, gR=gro, alpha=alpha)
    return plan, asm, ora


@pytest.mark.parametrize("seed,n", [(1, 6), (2, 17), (3, 33)])
def test_robin_parity_2d(seed, n):
    log(f"case: Robin 2d seed={seed} n={n}")
    rng = np.random.default_rng(300 + seed)
    sides = tuple(int(x) for x in rng.choice([1, 2, 3], size=4))
    sides = (3,) + sides[1:] if 3 not in sides else sides
    m = meshgen.square_mesh(n, jitter=0.2, permute=True, seed=seed, kappa="lognormal", sides=sides)
    specs = [(FE_FN_SINPROD, (2 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7)), (FE_FN_CONST, (0.9,))]
    gr_spec = (FE_FN_DUDN_SINPROD, (1.3,)) if seed % 2 else (FE_FN_LINEAR, (0.2, -0.5, 0.4))
    plan, asm, ora = _robin_case(m, specs, gr_spec, 1.7)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs, gr_spec))
    log(f"  sides {sides}, worst scaled value error {worst:.2e}")


@pytest.mark.parametrize("seed,n", [(1, 4), (2, 7)])
def test_robin_parity_3d(seed, n):
    log(f"case: Robin 3d seed={seed} n={n}")
    rng = np.random.default_rng(400 + seed)
    faces = tuple(int(x) for x in rng.choice([1, 2, 3], size=6))
    faces = (3,) + faces[1:] if 3 not in faces else faces
    m = meshgen.kuhn_cube(n, jitter=0.15, permute=True, seed=seed, kappa="lognormal", faces=faces)
    specs = [(FE_FN_SINPROD, (3 * math.pi ** 2,)), (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4)), (FE_FN_CONST, (0.6,))]
    gr_spec = (FE_FN_DUDN_SINPROD, (1.0,)) if seed % 2 else (FE_FN_LINEAR, (0.5, 0.2, 0.1, -0.3))
    plan, asm, ora = _robin_case(m, specs, gr_spec, 0.8)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs, gr_spec))
    log(f"  faces {faces}, worst scaled value error {worst:.2e}")


@pytest.mark.parametrize("rule", [1, 2])
@pytest.mark.parametrize("dim,n", [(2, 17), (3, 6)])
def test_load_rules_parity(rule, dim, n):
    """Section 4's one-point (centroid) and trapezoidal (vertex) load rules on the GPU
    against the oracle's, with analytic and nodal f, Neumann, Robin and Dirichlet
    sides: pattern bit-exact, values and right-hand sides to the parity tolerance."""
    from paper_1804_05156_amd import femhip
    log(f"case: load rule {rule}, dim {dim}, n {n}")
    if dim == 2:
        m = meshgen.square_mesh(n, jitter=0.2, permute=True, seed=40 + rule, kappa="lognormal", sides=(1, 2, 3, 2))
        fa = (FE_FN_SINPROD, (2 * math.pi ** 2,))
        gd, gn, gr = (FE_FN_LINEAR, (0.3, 1.1, -0.7)), (FE_FN_DUDN_SINPROD, (1.0,)), (FE_FN_LINEAR, (0.2, -0.5, 0.4))
    else:
        m = meshgen.kuhn_cube(n, jitter=0.15, permute=True, seed=50 + rule, kappa="lognormal", faces=(1, 1, 2, 3, 2, 2))
        fa = (FE_FN_SINPROD, (3 * math.pi ** 2,))
        gd, gn, gr = ((FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4)), (FE_FN_DUDN_SINPROD, (1.0,)),
                      (FE_FN_LINEAR, (0.5, 0.2, 0.1, -0.3)))
    fnod = (FE_FN_NODAL, (0.0,), np.cos(math.pi * m.node).prod(axis=0) + 0.5)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    for fspec in (fa, fnod):
        specs = [fspec, gd, gn]
        (f, fo), (gdf, gdo), (gnf, gno) = fns(*specs)
        (grf, gro), _, _ = fns(gr)
        asm = plan.assemble(kap, f, gdf, gnf, gR=grf, robin_alpha=1.2, load_rule=rule)
        plan.check()
        torch.cuda.synchronize()
        ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno, gR=gro, alpha=1.2, rule=rule)
        worst = compare(host(plan, asm), ora, data=data_scale(m, specs, gr))
        log(f"  f kind {fspec[0]}: worst scaled value error {worst:.2e}")


def test_load_rule_rejected():
    from paper_1804_05156_amd import femhip
    log("case: unknown load rule")
    m = meshgen.square_mesh(5)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    with pytest.raises(femhip.FemhipError):
        plan.assemble(kap, None, load_rule=3)


def test_robin_second_order_convergence_gpu():
    """All sides Robin, u = cos(pi x) cos(pi y) (du/dn = 0, so g_R = alpha u), f = 2 pi^2 u
    as nodal data: the GPU solution's L2 error decays like h^2."""
    log("case: Robin convergence")
    alpha = 1.5
    errs = []
    for n in (17, 33, 65, 129):
        m = meshgen.square_mesh(n, sides=(3, 3, 3, 3))
        exact, fv = _cos_nodal(m)
        plan, asm, _ = _robin_case(m, [(FE_FN_NODAL, (0.0,), fv)], (FE_FN_NODAL, (0.0,), alpha * exact), alpha)
        u, _, _ = plan.solve(asm, rtol=1e-12)
        u = u.cpu().numpy()
        x, y = m.node
        X, Y = x[m.elem], y[m.elem]
        area = 0.5 * np.abs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]))
        U = u[m.elem]
        s = 0.0
        for k in range(3):
            i, j = (k + 1) % 3, (k + 2) % 3
            e = np.cos(math.pi * (X[i] + X[j]) / 2) * np.cos(math.pi * (Y[i] + Y[j]) / 2) - (U[i] + U[j]) / 2
            s += float(np.sum(area / 3 * e * e))
        errs.append(math.sqrt(s))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    log(f"  L2 errors {errs} rates {rates}")
    assert all(1.9 < r < 2.1 for r in rates)


def test_kernel_timing_api():
    """fe_prof_enable / fe_prof_read: every kernel of one assembly is timed once, by
    name, with positive durations; disabled timing records nothing."""
    from paper_1804_05156_amd import femhip
    log("case: kernel timing")
    m = meshgen.square_mesh(65, jitter=0.2, permute=True, seed=77, kappa="lognormal")
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    asm = plan.assemble(kap)
    torch.cuda.synchronize()
    femhip.fe_prof_enable(True)
    plan.assemble(kap, out=asm)
    rec = femhip.fe_prof_read()
    femhip.fe_prof_enable(False)
    # rows processed in label order (sort_runs) need no label-order copy
    want = {"k_scatter_coords", "k_assemble_2d"} | (set() if plan.info["sort_runs"] else {"k_values_to_label"})
    assert set(rec) == want
    assert all(r["launches"] == 1 and r["total_ms"] > 0 for r in rec.values())
    plan.assemble(kap, out=asm)
    assert femhip.fe_prof_read() == {}


@pytest.mark.parametrize("permute", [False, True])
@pytest.mark.parametrize("case", ["robin", "nodal", "centroid", "trapezoid"])
@pytest.mark.parametrize("dim", [2, 3])
def test_both_processing_orders_parity(dim, case, permute):
    """Robin sides, nodal data and the load rules of Section 4 through both processing
    orders, against the oracle.  Labels that follow the element order (permute False)
    take label-order processing: rows written in place and, in 3-D, the stored
    column sets in the numeric kernel; a random relabelling takes the processing-
    order rows and the label-order copies.  The plan reports which (sort_runs 1 / 0);
    the sizes make the choice certain (at least 9 buckets, so random labels rarely
    repeat a neighbour's bucket)."""
    from paper_1804_05156_amd import femhip
    log(f"case: both orders, dim {dim}, {case}, permute {permute}")
    if dim == 2:
        m = meshgen.square_mesh(65, jitter=0.2, permute=permute, seed=500 + len(case), kappa="lognormal",
                                sides=(1, 3, 2, 3))
        lin = (FE_FN_LINEAR, (0.3, 1.1, -0.7))
        lin2 = (FE_FN_LINEAR, (0.2, -0.5, 0.4))
        fa = (FE_FN_SINPROD, (2 * math.pi ** 2,))
    else:
        m = meshgen.kuhn_cube(17, jitter=0.15, permute=permute, seed=600 + len(case), kappa="lognormal",
                              faces=(1, 3, 2, 3, 2, 1))
        lin = (FE_FN_LINEAR, (0.3, 1.1, -0.7, 0.4))
        lin2 = (FE_FN_LINEAR, (0.5, 0.2, 0.1, -0.3))
        fa = (FE_FN_SINPROD, (3 * math.pi ** 2,))
    rng = np.random.default_rng(700 + dim)
    rule, alpha = 0, 1.3
    if case == "robin":
        specs, gr = [fa, lin, (FE_FN_DUDN_SINPROD, (1.0,))], (FE_FN_DUDN_SINPROD, (0.7,))
    elif case == "nodal":
        nodal = [rng.standard_normal(m.n_node) for _ in range(4)]
        specs = [(FE_FN_NODAL, (0.0,), nodal[k]) for k in range(3)]
        gr, alpha = (FE_FN_NODAL, (0.0,), nodal[3]), 0.7
    elif case == "centroid":
        specs, gr, rule = [fa, lin, (FE_FN_CONST, (0.9,))], lin2, 1
    else:
        fnod = (FE_FN_NODAL, (0.0,), np.cos(math.pi * m.node).prod(axis=0) + 0.5)
        specs, gr, rule = [fnod, lin, (FE_FN_DUDN_SINPROD, (1.0,))], lin2, 2
    (f, fo), (gd, gdo), (gn, gno) = fns(*specs)
    (grf, gro), _, _ = fns(gr)
    node, elem, bd, kap = to_dev(m)
    plan = femhip.Plan(node, elem, bd)
    assert plan.info["sort_runs"] == (0 if permute else 1)
    asm = plan.assemble(kap, f, gd, gn, gR=grf, robin_alpha=alpha, load_rule=rule)
    plan.check()
    torch.cuda.synchronize()
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo, gN=gno, gR=gro, alpha=alpha, rule=rule)
    worst = compare(host(plan, asm), ora, data=data_scale(m, specs, gr))
    log(f"  sort_runs {plan.info['sort_runs']}, worst scaled value error {worst:.2e}")
