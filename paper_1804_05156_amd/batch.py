"""Batches of independent meshes: their union, one graph launch that assembles and
solves every instance, and the autotuner of the persistent solve grid.

Only argument marshalling happens here (concatenating arrays and offsetting labels
to form the union, allocating outputs); assembly and the solves run in the
library's kernels through ``fe_batch_*``.
"""
from __future__ import annotations

import json
import os

import torch

from . import femhip


class Batch:
    """Union of ``n_inst`` meshes.  nodes[k]: (dim, N_k) float64, elems[k]: (dim+1,
    NT_k) int32 with labels local to instance k, bdflags[k]: (dim+1, NT_k) int8 (or
    all None); all CUDA tensors.  Vertex labels of instance k are offset by
    ``node_off[k]`` in the union, element labels by ``elem_off[k]``."""

    def __init__(self, nodes, elems, bdflags=None, blocks_per_cu: int = 0, units_per_step: int = 0, stream=None):
        if not nodes or len(nodes) != len(elems):
            raise ValueError("need one elem array per node array")
        self.n_inst = len(nodes)
        self.node_off = [0]
        self.elem_off = [0]
        for nd, el in zip(nodes, elems):
            self.node_off.append(self.node_off[-1] + int(nd.shape[1]))
            self.elem_off.append(self.elem_off[-1] + int(el.shape[1]))
        self.node = torch.cat(list(nodes), 1).contiguous()
        self.elem = torch.cat([el + off for el, off in zip(elems, self.node_off[:-1])], 1).to(torch.int32).contiguous()
        self.bdflag = None if bdflags is None else torch.cat(list(bdflags), 1).contiguous()
        self.handle = None
        self.plan = femhip.Plan(self.node, self.elem, self.bdflag, stream)
        self.N = self.plan.N
        self.ws = torch.empty(femhip.fe_batch_solve_workspace_bytes(self.N, self.n_inst), dtype=torch.uint8,
                              device=self.node.device)
        self.handle = femhip.fe_batch_create(self.plan.handle, self.node_off, self.ws, blocks_per_cu, units_per_step,
                                             stream)
        dev = self.node.device
        nnz = max(self.plan.nnz, 1)
        # outputs live as long as the batch, so that repeated calls replay one graph
        self.val = torch.empty(nnz, dtype=torch.float64, device=dev)
        self.val_bc = torch.empty(nnz, dtype=torch.float64, device=dev)
        self.b = torch.empty(self.N, dtype=torch.float64, device=dev)
        self.u = torch.empty(self.N, dtype=torch.float64, device=dev)

    def assemble_solve(self, kappa, f=None, gD=None, gN=None, rtol=1e-10, maxit=100000, stream=None,
                       allow_noconv=False):
        """Assemble and solve every instance; returns (u, iters, relres) with u the
        union's solution vector (``split`` cuts it per instance)."""
        it, rel, _ = femhip.fe_batch_assemble_solve(self.handle, self.node, kappa, f, gD, gN, self.plan.rowptr,
                                                    self.plan.colind, self.val, self.val_bc, self.b, self.u, rtol,
                                                    maxit, self.n_inst, stream, allow_noconv)
        return self.u, it, rel

    def split(self, x):
        return [x[self.node_off[k]:self.node_off[k + 1]] for k in range(self.n_inst)]

    def set_grid(self, blocks_per_cu: int, units_per_step: int = 0):
        femhip.fe_batch_set_grid(self.handle, blocks_per_cu, units_per_step)

    def info(self) -> dict:
        return femhip.fe_batch_get_info(self.handle)

    def close(self):
        """Release the batch (its captured graph) and the union plan now, rather than
        when the interpreter collects them."""
        if getattr(self, "handle", None) is not None and femhip is not None and femhip._lib is not None:
            femhip._lib.fe_batch_destroy(self.handle)
            self.handle = None
        plan = getattr(self, "plan", None)
        if plan is not None:
            plan.close()

    def __del__(self):
        self.close()


def _time_call(fn, reps: int) -> float:
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


# rows per workgroup of the assembly's numeric row kernels tried by autotune
ASM_ROWS_PER_BLOCK = (64, 128, 256)

# (workgroups per compute unit, 256-row units per workgroup step) tried by autotune;
# the library refuses more than 4 workgroups per compute unit (the largest grid
# verified co-resident)
CANDIDATES = ((4, 1), (2, 1), (2, 2), (4, 2), (2, 4))


def autotune(batch: Batch, kappa, f=None, gD=None, gN=None, rtol=1e-10, maxit=100000, candidates=None,
             reps: int = 1, cache_path: str | None = None, log=None) -> dict:
    """Pick the launch shapes of the batch: rows per workgroup of the assembly's row
    kernels (timing the union's assembly), then the persistent solve grid (workgroups
    per compute unit and units processed together per workgroup) by timing whole
    graph launches of this batch (results are bitwise independent of every choice).  A candidate the device
    rejects is skipped.  With ``cache_path`` the choice is stored in a JSON file
    keyed by device and batch shape and reused later.  Returns the choice and the
    measured times (ms per launch)."""
    info = batch.info()
    key = f"{torch.cuda.get_device_name()}|{info['n_inst']}|{info['n_rows']}|{batch.plan.nnz}|{rtol}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            batch.set_grid(*cache[key]["grid"])
            batch.plan.set_launch(cache[key].get("asm_rows_per_block", 0))
            return dict(cache[key], cached=True)
    # the assembly's launch setting first: rows per workgroup of the numeric row
    # kernels, by timing the union's assembly alone (results do not depend on it)
    asm_ms = {}
    for rpb in ASM_ROWS_PER_BLOCK:
        batch.plan.set_launch(rpb)
        out = batch.plan.assemble(kappa, f, gD, gN)
        asm_ms[rpb] = _time_call(lambda: batch.plan.assemble(kappa, f, gD, gN, out=out), max(reps, 3))
        if log:
            log(f"autotune: assembly, {rpb} rows per workgroup: {asm_ms[rpb]:.3f} ms")
    asm_best = min(asm_ms, key=asm_ms.get)
    batch.plan.set_launch(asm_best)
    times = {}
    for c in (candidates or CANDIDATES):
        try:
            batch.set_grid(*c)
            batch.assemble_solve(kappa, f, gD, gN, rtol, maxit)          # capture + warm
            times[c] = _time_call(lambda: batch.assemble_solve(kappa, f, gD, gN, rtol, maxit), reps)
        except femhip.FemhipError as e:
            if log:
                log(f"autotune: {c} rejected ({e})")
            continue
        if log:
            log(f"autotune: blocks/CU {c[0]}, units/step {c[1]}: {times[c]:.2f} ms")
    if not times:
        raise RuntimeError("autotune: no candidate grid ran")
    best = min(times, key=times.get)
    batch.set_grid(*best)
    out = {"grid": list(best), "ms": {f"{k[0]}x{k[1]}": v for k, v in times.items()},
           "asm_rows_per_block": asm_best, "asm_ms": {str(k): v for k, v in asm_ms.items()}}
    if cache_path:
        cache[key] = out
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dict(out, cached=False)
