"""Benchmark: P1 stiffness/load assembly of the 2049^2 jittered, permuted mesh on one GPU.

One step = the whole assembly path from the mesh arrays already in HBM to the CSR
matrix and the right-hand side with boundary conditions, nothing cached between
steps: fe_plan_create (symbolic phase: incidence lists, row pattern, Dirichlet set),
fe_plan_pattern (rowptr/colind), fe_assemble (A, A_bc, b, b_load, Dirichlet flags).
`value` = elements assembled per second over the timed steps.

Also reported (extra keys): the warm numeric phase alone (plan reused, new kappa),
the roofline of the dominant kernel measured with HIP events on its stream, the
phase split, and the CPU oracle timed on a bounded sample of the same recipe.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="jitter2049")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (for counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1804_05156_amd import femhip, meshgen

    dev = torch.device("cuda:0")
    log(f"[bench] building workload {args.workload}")
    m = meshgen.workload(args.workload)
    N, NT, dim = m.n_node, m.n_elem, m.dim
    node = torch.from_numpy(m.node).to(dev)
    elem = torch.from_numpy(m.elem).to(dev)
    bd = torch.from_numpy(m.bdflag).to(dev)
    kappa = torch.from_numpy(m.kappa).to(dev)
    kappa2 = torch.exp(torch.randn(NT, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(7)))
    if dim == 2:
        f = femhip.Fn(femhip.FE_FN_SINPROD, (2 * math.pi ** 2,))
        gn = None
    else:
        u = torch.prod(torch.sin(math.pi * node), dim=0)
        f = femhip.Fn(femhip.FE_FN_NODAL, (0,), (3 * math.pi ** 2 * u).contiguous())
        gn = femhip.Fn(femhip.FE_FN_DUDN_SINPROD, (1.0,))

    # buffers allocated once (the library allocates nothing)
    mesh = femhip.make_mesh(node, elem, bd)
    ws = torch.empty(femhip.fe_plan_workspace_bytes(mesh), dtype=torch.uint8, device=dev)
    plan, nnz = femhip.fe_plan_create(mesh, ws)
    femhip.fe_plan_destroy(plan)
    rowptr = torch.empty(N + 1, dtype=torch.int32, device=dev)
    colind = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float64, device=dev)
    val_bc = torch.empty_like(val)
    b = torch.empty(N, dtype=torch.float64, device=dev)
    b_load = torch.empty_like(b)
    isd = torch.empty(N, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    ev = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731  (events on the launch stream)

    def cold_step(times=None):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record(stream)
        p, _ = femhip.fe_plan_create(mesh, ws)
        e1.record(stream)
        femhip.fe_plan_pattern(p, rowptr, colind)
        e2.record(stream)
        femhip.fe_assemble(p, node, kappa, f, None, gn, val, val_bc, b, b_load, isd)
        e3.record(stream)
        if times is not None:
            times.append((e0, e1, e2, e3))
        return p

    log(f"[bench] N={N} NT={NT} nnz={nnz}; warmup {args.warmup}")
    for _ in range(args.warmup):
        femhip.fe_plan_destroy(cold_step())
    torch.cuda.synchronize()
    plans, times = [], []
    log(f"[bench] timing {args.steps} cold steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plans.append(cold_step(times))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc = femhip.fe_plan_status(plans[-1])
    if rc != 0:
        raise RuntimeError(f"kernel status {rc}")
    for p in plans[:-1]:
        femhip.fe_plan_destroy(p)
    plan = plans[-1]
    ms_step = wall / args.steps * 1e3
    sym_ms = np.median([a.elapsed_time(b_) for a, b_, _, _ in times])
    pat_ms = np.median([b_.elapsed_time(c) for _, b_, c, _ in times])
    num_ms = np.median([c.elapsed_time(d) for _, _, c, d in times])

    # warm numeric phase: plan reused, a different kappa each call
    log("[bench] timing warm numeric phase")
    for _ in range(3):
        femhip.fe_assemble(plan, node, kappa2, f, None, gn, val, val_bc, b, b_load, isd)
    torch.cuda.synchronize()
    wev = []
    for k in range(args.steps):
        e0, e1 = ev(), ev()
        e0.record(stream)
        femhip.fe_assemble(plan, node, kappa if k % 2 else kappa2, f, None, gn, val, val_bc, b, b_load, isd)
        e1.record(stream)
        wev.append((e0, e1))
    torch.cuda.synchronize()
    warm_ms = float(np.mean([a.elapsed_time(b_) for a, b_ in wev]))
    femhip.fe_plan_destroy(plan)

    # algorithmic bytes of fe_assemble: inputs read once, outputs written once
    in_bytes = dim * N * 8 + (dim + 1) * NT * 4 + NT * 8
    out_bytes = 2 * nnz * 8 + 2 * N * 8 + N
    if f.kind == femhip.FE_FN_NODAL:
        in_bytes += N * 8
    asm_bytes = in_bytes + out_bytes
    achieved = asm_bytes / (warm_ms * 1e-3) / 1e9
    cold_bytes = dim * N * 8 + (dim + 1) * NT * 5 + NT * 8 + (N + 1) * 4 + nnz * 4 + out_bytes

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.workload)

    out = {
        "metric": "assembled elements/s + HBM GB/s; batched & adjoint vs plain on 1 GPU",
        "value": NT / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_node": N, "n_elem": NT, "nnz": nnz, "dim": dim,
                   "step": "cold: plan + pattern + numeric assembly with boundary conditions"},
        "phases_ms": {"plan_create": sym_ms, "pattern": pat_ms, "assemble": num_ms},
        "warm": {"ms": warm_ms, "elements_per_s": NT / (warm_ms * 1e-3)},
        "effective_GBps_cold": cold_bytes / (ms_step * 1e-3) / 1e9,
        "roofline": {"kernel": "k_assemble (fe_assemble)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "bytes_per_launch": asm_bytes, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def copy_calibration(mb):
    """A plain copy of known size: reads and writes mb*2^20 bytes per launch, 5 launches."""
    import torch
    n = mb * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 8, "launches": 5}), flush=True)


def cpu_baseline(workload):
    """The oracle, single-threaded, on a bounded sample of the same recipe."""
    import numpy as np
    import oracle
    from paper_1804_05156_amd import meshgen
    if workload == "jitter2049":
        m = meshgen.square_mesh(1025, jitter=0.2, permute=True, seed=2, kappa="lognormal")
        f = oracle.Fn(oracle.FN_SINPROD, (2 * math.pi ** 2,))
        gn = None
        sample = "1025^2 jittered permuted mesh, same recipe (2,097,152 triangles), one oracle assembly"
    else:
        m = meshgen.kuhn_cube(49, seed=3, kappa="lognormal")
        u = np.prod(np.sin(math.pi * m.node), axis=0)
        f = oracle.Fn(oracle.FN_NODAL, (0,), 3 * math.pi ** 2 * u)
        gn = oracle.Fn(oracle.FN_DUDN_SINPROD, (1.0,))
        sample = "49^3 Kuhn cube, same recipe, one oracle assembly"
    log(f"[bench] cpu baseline: {sample}")
    t = time.perf_counter()
    oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=f, gN=gn)
    dt = time.perf_counter() - t
    return {"value": m.n_elem / dt, "unit": "elements/s", "cores": 1, "kind": "oracle", "sample": sample,
            "seconds": dt, "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" (nproc {os.cpu_count()})"
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
