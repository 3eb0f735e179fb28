"""Batched assemble + solve (many meshes, one graph launch) against the plain
single-mesh path and the oracle.

The batch is the disjoint union of its meshes, so each instance's rows of the
union matrix and load vector must equal, bit for bit, what the plain path
assembles for that mesh alone, and the batched PCG, which keeps the plain solve's
units and reduction order per instance, must reproduce the plain solve's iterates:
same iteration count, same residual ratio, same solution bits, for any grid size.
The solutions are also checked against the oracle's direct solve through the true
residual ||b - A_bc u|| <= 10 rtol ||b|| (oracle matrix and vector).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1804_05156_amd import meshgen
from gpu_helpers import fns, log, run_gpu, to_dev

pytestmark = pytest.mark.gpu

FE_FN_LINEAR, FE_FN_SINPROD = 2, 3
SPECS = [(FE_FN_SINPROD, (2 * math.pi ** 2,)), (FE_FN_LINEAR, (0.5, 1.0, -1.0))]


def _batch(ms, **kw):
    from paper_1804_05156_amd import batch
    devs = [to_dev(m) for m in ms]
    B = batch.Batch([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], **kw)
    kap = torch.cat([d[3] for d in devs]).contiguous()
    return B, kap


def _check_instance(B, k, m, u, it, rel, f, gd, rtol, fo=None, gdo=None, oracle_check=True):
    """Instance k of the batch against the plain path (bitwise) and the oracle (residual)."""
    plan, asm = run_gpu(m, None, f, gd, None)
    uk, ik, rk = plan.solve(asm, rtol=rtol)
    torch.cuda.synchronize()
    r0, r1 = B.node_off[k], B.node_off[k + 1]
    p0, p1 = int(B.plan.rowptr[r0]), int(B.plan.rowptr[r1])
    assert p1 - p0 == plan.nnz
    assert torch.equal(B.plan.rowptr[r0:r1 + 1] - p0, plan.rowptr)
    assert torch.equal(B.plan.colind[p0:p1] - r0, plan.colind[:plan.nnz])
    assert torch.equal(B.val[p0:p1], asm.val[:plan.nnz])
    assert torch.equal(B.val_bc[p0:p1], asm.val_bc[:plan.nnz])
    assert torch.equal(B.b[r0:r1], asm.b)
    assert it[k] == ik and rel[k] == rk, (k, it[k], ik, rel[k], rk)
    assert torch.equal(u[r0:r1], uk)
    if oracle_check:
        ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo, gD=gdo)
        res = ora.b - oracle.spmv(ora.rowptr, ora.colind, ora.val_bc, u[r0:r1].cpu().numpy())
        assert np.linalg.norm(res) <= 10 * rtol * np.linalg.norm(ora.b)


def test_batch_matches_plain_bitwise_and_oracle():
    log("case: batch of 6 meshes vs plain path and oracle")
    ms = meshgen.batch_meshes([17, 9, 33, 12, 25, 40], seed_base=7000, permute=True)
    (f, fo), (gd, gdo), _ = fns(*SPECS)
    B, kap = _batch(ms)
    u, it, rel = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    u = u.clone()
    log(f"  iterations {it}  info {B.info()}")
    for k, m in enumerate(ms):
        _check_instance(B, k, m, u, it, rel, f, gd, 1e-10, fo, gdo)


def test_batch_solve_grid_independent():
    """fe_batch_solve (no graph) gives the same bits for every persistent grid size."""
    from paper_1804_05156_amd import femhip
    log("case: fe_batch_solve over grid sizes")
    ms = meshgen.batch_meshes([30, 7, 52, 19], seed_base=7100, permute=True)
    (f, _), (gd, _), _ = fns(*SPECS)
    B, kap = _batch(ms)
    u_ref, it_ref, rel_ref = B.assemble_solve(kap, f, gd, None, rtol=1e-11)
    u_ref = u_ref.clone()
    ws = torch.empty(femhip.fe_batch_solve_workspace_bytes(B.N, B.n_inst), dtype=torch.uint8, device="cuda")
    ran = 0
    for bpc, ups in ((1, 1), (1, 4), (2, 2), (4, 1), (2, 4), (4, 4)):
        asm = B.plan.assemble(kap, f, gd, None)
        u = torch.empty(B.N, dtype=torch.float64, device="cuda")
        femhip.fe_select(asm.is_dirichlet, asm.b, None, u)
        try:
            it, rel, rc = femhip.fe_batch_solve(B.node_off, B.plan.rowptr, B.plan.colind, asm.val_bc, asm.b, u,
                                                1e-11, 100000, ws, blocks_per_cu=bpc, units_per_step=ups)
        except femhip.FemhipError as e:
            assert e.code == femhip.FE_EINVAL   # a grid that does not fit this kernel's occupancy
            log(f"  blocks/CU {bpc}, units/step {ups}: does not fit")
            continue
        torch.cuda.synchronize()
        ran += 1
        log(f"  blocks/CU {bpc}, units/step {ups}: iterations {it}")
        assert rc == femhip.FE_OK and it == it_ref and rel == rel_ref
        assert torch.equal(u, u_ref)
    assert ran >= 4


def test_grid_bound_and_cooperative_node():
    """Grids above the verified co-resident bound (4 workgroups per compute unit) are
    refused before any launch; the captured solve node reports whether it is a
    cooperative launch (read back from the graph, not from the library's request)."""
    from paper_1804_05156_amd import femhip
    log("case: grid bound, cooperative node")
    ms = meshgen.batch_meshes([25, 18], seed_base=7300)
    (f, _), (gd, _), _ = fns(*SPECS)
    B, kap = _batch(ms)
    for bpc in (5, 7, 12):
        with pytest.raises(femhip.FemhipError) as e:
            B.set_grid(bpc, 1)
        assert e.value.code == femhip.FE_EINVAL
    B.set_grid(4, 1)
    B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    info = B.info()
    log(f"  info {info}")
    assert info["blocks_per_cu"] == 4 and info["max_blocks_per_cu"] <= 4
    assert info["cooperative"] in (0, 1)
    # a new launch setting of the assembly recaptures the graph; the bits stay
    u1, it1, _ = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    u1 = u1.clone()
    caps = B.info()["captures"]
    B.plan.set_launch(64)
    u2, it2, _ = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    assert B.info()["captures"] == caps + 1
    assert it2 == it1 and torch.equal(u2, u1)


def test_graph_replay_and_recapture():
    log("case: graph replay, in-place kappa update, recapture")
    ms = meshgen.batch_meshes([21, 14, 35], seed_base=7200)
    (f, fo), (gd, gdo), _ = fns(*SPECS)
    B, kap = _batch(ms)
    u1, it1, rel1 = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    u1 = u1.clone()
    u2, it2, rel2 = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    assert B.info()["captures"] == 1
    assert it1 == it2 and rel1 == rel2 and torch.equal(u1, u2)
    # new coefficient values behind the same pointer: the graph is replayed, the result follows kappa
    rng = np.random.default_rng(7201)
    newk = [np.exp(rng.standard_normal(m.n_elem)) for m in ms]
    kap.copy_(torch.from_numpy(np.concatenate(newk)).cuda())
    for m, kk in zip(ms, newk):
        m.kappa = kk
    u3, it3, rel3 = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    u3 = u3.clone()
    assert B.info()["captures"] == 1
    for k, m in enumerate(ms):
        _check_instance(B, k, m, u3, it3, rel3, f, gd, 1e-10, fo, gdo)
    # a different tolerance is a different graph
    u4, it4, rel4 = B.assemble_solve(kap, f, gd, None, rtol=1e-6)
    assert B.info()["captures"] == 2
    assert all(a <= b for a, b in zip(it4, it3)) and max(rel4) <= 1e-6


def test_batch_edge_cases():
    """One instance; an instance whose data vanish (converged before the first
    iteration); an iteration limit; an empty instance in fe_batch_solve."""
    from paper_1804_05156_amd import femhip
    log("case: batch edge cases")
    (f, fo), (gd, gdo), _ = fns(*SPECS)
    ms = meshgen.batch_meshes([23], seed_base=7300)
    B, kap = _batch(ms)
    u, it, rel = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    _check_instance(B, 0, ms[0], u.clone(), it, rel, f, gd, 1e-10, fo, gdo)
    # zero data: b = 0, the start vector is the solution, zero iterations
    ms = meshgen.batch_meshes([11, 16], seed_base=7310)
    B, kap = _batch(ms)
    u, it, rel = B.assemble_solve(kap, None, None, None, rtol=1e-10)
    assert it == [0, 0] and rel == [0.0, 0.0] and float(u.abs().max()) == 0.0
    # iteration limit: FE_ENOCONV, every unconverged instance stops at maxit
    u, it, rel = B.assemble_solve(kap, f, gd, None, rtol=1e-14, maxit=3, allow_noconv=True)
    assert it == [3, 3] and min(rel) > 1e-14
    # an empty instance (no rows) between two real ones
    asm = B.plan.assemble(kap, f, gd, None)
    off = [0, B.node_off[1], B.node_off[1], B.node_off[2]]
    ws = torch.empty(femhip.fe_batch_solve_workspace_bytes(B.N, 3), dtype=torch.uint8, device="cuda")
    x = torch.empty(B.N, dtype=torch.float64, device="cuda")
    femhip.fe_select(asm.is_dirichlet, asm.b, None, x)
    it3, rel3, rc = femhip.fe_batch_solve(off, B.plan.rowptr, B.plan.colind, asm.val_bc, asm.b, x, 1e-10, 100000, ws)
    u_ref, it_ref, rel_ref = B.assemble_solve(kap, f, gd, None, rtol=1e-10)
    assert rc == femhip.FE_OK and it3 == [it_ref[0], 0, it_ref[1]] and rel3[1] == 0.0
    assert torch.equal(x, u_ref)
    # argument errors (host side): bad offsets, too many instances
    with pytest.raises(femhip.FemhipError):
        femhip.fe_batch_solve([0, 5, 3], B.plan.rowptr, B.plan.colind, asm.val_bc, asm.b, x, 1e-10, 10, ws)
    with pytest.raises(femhip.FemhipError):
        femhip.fe_batch_solve_workspace_bytes(B.N, 5000)


def test_full_size_batch_sampled():
    """The 256-instance batch (grid sides uniform in [17, 513], jittered,
    lognormal kappa, rtol 1e-10) in the launch configuration of the benchmark: every
    instance converges; sampled instances (the two smallest, the median and the
    largest) equal the plain path bit for bit and satisfy the oracle residual bound."""
    log("case: 256-instance batch (full size), sampled instances")
    sizes = meshgen.batch_sizes()
    ms = meshgen.batch_meshes(sizes)
    (f, fo), _, _ = fns(SPECS[0])
    B, kap = _batch(ms)
    u, it, rel = B.assemble_solve(kap, f, None, None, rtol=1e-10)
    u = u.clone()
    log(f"  rows {B.N}, iterations min {min(it)} max {max(it)}, info {B.info()}")
    assert max(rel) <= 1e-10
    order = np.argsort(sizes)
    sample = [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]
    for k in sample:
        log(f"  instance {k}: side {sizes[k]}, iterations {it[k]}")
        _check_instance(B, k, ms[k], u, it, rel, f, None, 1e-10, fo, None)


def test_both_plain_solve_forms_match_batched():
    """The plain solve fuses its reductions into the row kernels up to 1024 workgroups
    (262144 rows) and runs separate summing kernels above; both give the bits of the
    batched solve (a 513^2 instance: 263169 rows, separate form; a 300^2 instance:
    fused form)."""
    log("case: fused and separate plain solve forms vs batched")
    ms = meshgen.batch_meshes([513, 300], seed_base=7400)
    (f, fo), _, _ = fns(SPECS[0])
    B, kap = _batch(ms)
    u, it, rel = B.assemble_solve(kap, f, None, None, rtol=1e-10)
    u = u.clone()
    for k, m in enumerate(ms):
        log(f"  instance {k}: {m.n_node} rows, iterations {it[k]}")
        _check_instance(B, k, m, u, it, rel, f, None, 1e-10, fo, None, oracle_check=False)
