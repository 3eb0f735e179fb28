"""The allocation-free solve entry point (fe_solve_noalloc) against fe_solve.

fe_solve_noalloc runs the same kernels as fe_solve on a fixed device array of the
library instead of a caller workspace, so on the same system its solution, its
iteration count and its residual ratio must equal fe_solve's bit for bit.  Two
calls in a row share that array; the second is smaller than the first, so what
the first left behind (flags, partial sums, longer vectors) must not reach it.
The first system (a 1025^2 jittered mesh, 1,050,625 rows) runs the separate
summing kernels of the large form, the second (129^2) the fused form.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1804_05156_amd import meshgen
from gpu_helpers import fns, log, run_gpu

pytestmark = pytest.mark.gpu

FE_FN_SINPROD = 3


def _system(n, seed):
    m = meshgen.square_mesh(n, jitter=0.2, permute=True, seed=seed, kappa="lognormal")
    (f, _), _, _ = fns((FE_FN_SINPROD, (2 * math.pi ** 2,)))
    plan, asm = run_gpu(m, None, f)
    return m, plan, asm


def _both(plan, asm, rtol):
    from paper_1804_05156_amd import femhip
    rp, ci = plan.rowptr, plan.colind[:plan.nnz]
    u0 = torch.empty_like(asm.b)
    femhip.fe_select(asm.is_dirichlet, asm.b, None, u0)
    u_ref = u0.clone()
    ws = torch.empty(femhip.fe_solve_workspace_bytes(plan.N), dtype=torch.uint8, device=u0.device)
    it_ref, rel_ref, _ = femhip.fe_solve(rp, ci, asm.val_bc, asm.b, u_ref, rtol, 100000, ws)
    u_na = u0.clone()
    it_na, rel_na, _ = femhip.fe_solve_noalloc(rp, ci, asm.val_bc, asm.b, u_na, rtol, 100000)
    torch.cuda.synchronize()
    return (u_ref.cpu().numpy(), it_ref, rel_ref), (u_na.cpu().numpy(), it_na, rel_na)


def test_noalloc_solve_equals_workspace_solve_twice():
    from paper_1804_05156_amd import femhip
    results = []
    for n, seed in ((1025, 71), (129, 72)):
        log(f"case: fe_solve_noalloc vs fe_solve, {n}^2 jittered mesh, seed {seed}")
        m, plan, asm = _system(n, seed)
        assert m.n_node <= femhip.FE_SOLVE_NOALLOC_MAX_N
        (u_ref, it_ref, rel_ref), (u_na, it_na, rel_na) = _both(plan, asm, 1e-10)
        log(f"  iterations {it_ref} / {it_na}, relres {rel_ref:.3e} / {rel_na:.3e}")
        assert it_na == it_ref and rel_na == rel_ref
        assert np.array_equal(u_na, u_ref)
        assert rel_na <= 1e-10
        results.append((m, u_na))
    # the smaller system's solution is also the oracle's (its own PCG at 1e-13), to
    # the solver tolerance
    m, u = results[1]
    (_, fo), _, _ = fns((FE_FN_SINPROD, (2 * math.pi ** 2,)))
    ora = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=fo)
    uo, _, _ = oracle.solve(ora, rtol=1e-13, method="cg")
    assert np.abs(u - uo).max() <= 1e-10 * 1e4 * m.n_node * np.abs(uo).max()


def test_noalloc_rejects_more_rows_than_its_array():
    from paper_1804_05156_amd import femhip
    log("case: fe_solve_noalloc above its row limit")
    n = femhip.FE_SOLVE_NOALLOC_MAX_N + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(femhip.FemhipError) as e:
        femhip.fe_solve_noalloc(rp, ci, v, b, u, 1e-10, 10)
    assert e.value.code == femhip.FE_ELIMIT
