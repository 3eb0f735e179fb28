"""Benchmark of the P1 assembly path on one GPU, with the batched and adjoint
extensions reported against the plain path.

Headline step (``value``): the whole assembly of the 2049^2 jittered, permuted
mesh from the mesh arrays already in HBM to the CSR matrix and the right-hand side
with boundary conditions, nothing cached between steps: fe_plan_create (incidence
lists, row pattern, Dirichlet set), fe_plan_pattern (rowptr/colind) and fe_assemble
(A, A_bc, b, b_load, Dirichlet flags).  value = elements assembled per second.

Also reported on the same JSON line:
  warm         fe_assemble alone (plan reused, new kappa each call)
  kernels      every kernel of the step timed with HIP events on its launch stream
  roofline     the kernel with the largest time per step (the dominant kernel): the
               compulsory bytes of the assembly per element (inputs read once,
               outputs written once: 79 B per triangle for the cold step of the
               2049^2 mesh) times the elements one launch processes, over its mean
               launch duration, against the 8 TB/s HBM peak; traffic (FETCH_SIZE +
               WRITE_SIZE per launch, copy-calibrated) and its ratio to those bytes
               when the committed counter summary matches the current sources; the
               kernel's own implementation byte model under a separate key; and the
               whole cold and warm steps' compulsory bytes over their wall time
  batched      256 uneven jittered meshes assembled + Jacobi-PCG solved (1e-10) by
               one graph launch, against a loop of the plain path over the same
               instances (plans built beforehand in both)
  adjoint      1025^2 mesh: forward solve + adjoint solve + gradient kernel against
               the forward solve alone
  next         assembly on the L-shaped domain, and the pure Neumann solve
  cpu_baseline the CPU oracle as it stands, timed before any GPU call: single thread
               pinned to one core, median of 3, on bounded samples of the 2-D and
               3-D recipes, and a process pool (one oracle assemble + solve per
               instance) over a sample of the batched workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload jitter2049|kuhn129]
                       [--no-cpu] [--no-batch] [--no-adjoint] [--no-next]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
COUNTERS = os.path.join(ROOT, "profiles", "counters_{workload}.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the library sources; counter data is valid only for the sources it was taken on."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1804_05156_amd", "csrc", "*")) +
                   [os.path.join(ROOT, "include", "femhip.h")])
    for p in files:
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bytes(name, N, NT, nnz, dim, nodal):
    """Algorithmic bytes of one launch of a kernel of the assembly step: every array
    the kernel must read or write, each element counted once."""
    nv = dim + 1
    ninc = nv * NT
    model = {
        "k_l1_hist": 5 * ninc + N,
        "k_l1_scatter": 4 * ninc + 8 * ninc,
        "k_l1_fine": 8 * ninc + 8 * ninc,
        "k_l2_bucket": 8 * ninc + N + 4 * ninc + 8 * N + N,
        "k_pi": ninc + 4 * NT + 4 * N + 8 * N + 17 * N,
        "k_unused": 8 * N,
        "k_rows_count": 12 * N + 4 * ninc + 4 * ninc + 4 * ninc + ninc + 16 * NT + 4 * N,
        "k_stats_partial": 9 * N,
        "k_rows_final": 12 * N + 4 * ninc + 16 * NT + 4 * ninc + N + 4 * nnz + 8 * ninc + 20 * N,
        "k_label_rows": 40 * N,
        "k_pattern_to_label": 20 * N + 8 * nnz,
        "k_scatter_coords": 8 * dim * N + 4 * N + 32 * N + (16 * N if nodal else 0),
        "k_assemble_2d": 8 * ninc + 8 * N + 32 * N + 8 * NT + 8 * (nnz + 2 * N) + (8 * N if nodal else 0),
        "k_assemble_3d": 8 * ninc + 8 * N + 32 * N + 8 * NT + 8 * (nnz + 2 * N) + (8 * N if nodal else 0),
        "k_values_to_label": 16 * N + 4 * N + 4 * N + 8 * (nnz + 2 * N) + 16 * nnz + 16 * N + N,
    }
    return model.get(name)


def read_counters(workload):
    """Per-dispatch FETCH/WRITE bytes from the committed counter summary, scaled by
    its copy-kernel calibration; None if absent or taken on other sources."""
    path = COUNTERS.format(workload=workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sources_sha256:\s*(\w+)", text)
    if not m or m.group(1) != source_hash():
        return None
    fcal = float(re.search(r"fetch_scale:\s*([\d.eE+-]+)", text).group(1))
    wcal = float(re.search(r"write_scale:\s*([\d.eE+-]+)", text).group(1))
    out = {}
    for line in text.splitlines():
        mm = re.match(r"\s*(k_\w+)\s+([\d.]+)\s+([\d.]+)\s*$", line)
        if mm:
            out[mm.group(1)] = (float(mm.group(2)) * 1024 * fcal, float(mm.group(3)) * 1024 * wcal)
    return out


def step_bytes(N, NT, nnz, dim, nodal):
    """Compulsory bytes of one assembly: the inputs read once (node, elem, bdflag,
    kappa, nodal f when used) and the outputs written once (rowptr, colind, val, b).
    Cold step: all of them (79 B per triangle on the 2049^2 mesh, 65.8 B per
    tetrahedron on the 129^3 cube with nodal f).  Warm step (pattern cached): without
    rowptr and colind (63 B per triangle, 55 B per tetrahedron)."""
    nv = dim + 1
    inputs = 8 * dim * N + 4 * nv * NT + nv * NT + 8 * NT + (8 * N if nodal else 0)
    cold = inputs + 4 * (N + 1) + 4 * nnz + 8 * nnz + 8 * N
    warm = inputs + 8 * nnz + 8 * N
    return cold, warm


NUMERIC = ("k_scatter_coords", "k_assemble_2d", "k_assemble_3d", "k_values_to_label")


def kernel_table(kern, steps, N, NT, nnz, dim, nodal):
    out = {}
    for name, k in kern.items():
        nb = kernel_bytes(name, N, NT, nnz, dim, nodal)
        out[name] = {"launches_per_step": k["launches"] / steps, "avg_us": k["avg_ms"] * 1e3,
                     "us_per_step": k["total_ms"] * 1e3 / steps,
                     "impl_GBps": (nb / (k["avg_ms"] * 1e-3) / 1e9) if nb else None}
    return out


def roofline(kernels, counters, N, NT, nnz, dim, nodal, cold_ms, warm_ms):
    """Roofline of the dominant kernel (largest time per step) on the compulsory bytes
    of the cold step, plus the traffic the counters measured and the whole steps'
    effective fractions."""
    cold_b, warm_b = step_bytes(N, NT, nnz, dim, nodal)
    dom = max(kernels, key=lambda n: kernels[n]["us_per_step"])
    us = kernels[dom]["avg_us"]
    achieved = cold_b / (us * 1e-6) / 1e9
    traffic = None
    if counters and dom in counters:
        traffic = counters[dom][0] + counters[dom][1]
    impl = kernel_bytes(dom, N, NT, nnz, dim, nodal)
    out = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "bytes_per_element": cold_b / NT, "elements_per_launch": NT, "algorithmic_bytes": cold_b,
           "avg_us": us,
           "traffic_ratio": (traffic / cold_b) if traffic else None,
           "impl_model": None if impl is None else {
               "bytes_per_launch": impl, "GBps": impl / (us * 1e-6) / 1e9,
               "frac": impl / (us * 1e-6) / 1e9 / HBM_PEAK_GBS},
           "cold_step": {"bytes": cold_b, "bytes_per_element": cold_b / NT, "ms": cold_ms,
                         "effective_GBps": cold_b / (cold_ms * 1e-3) / 1e9,
                         "frac": cold_b / (cold_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "warm_step": {"bytes": warm_b, "bytes_per_element": warm_b / NT, "ms": warm_ms,
                         "effective_GBps": warm_b / (warm_ms * 1e-3) / 1e9,
                         "frac": warm_b / (warm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    if counters and all(n in counters for n in kernels):
        def moved(names):
            return sum((counters[n][0] + counters[n][1]) * kernels[n]["launches_per_step"] for n in names)
        num = [n for n in kernels if n in NUMERIC]
        out["cold_step"]["counter_bytes"] = moved(list(kernels))
        out["cold_step"]["traffic_ratio"] = moved(list(kernels)) / cold_b
        out["warm_step"]["counter_bytes"] = moved(num)
        out["warm_step"]["traffic_ratio"] = moved(num) / warm_b
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="jitter2049", choices=["jitter2049", "kuhn129"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-next", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3-D (129^3 Kuhn cube) assembly section")
    ap.add_argument("--no-sym", action="store_true", help="skip the symmetric-storage (upper triangle) timings")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (for counter calibration)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only time the CPU oracle (no GPU use) and print its JSON object")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): every figure here is a single-GPU "
              "figure, and the multi-GPU sharding is a design note, not built", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, in a child process started before anything touches
    # the GPU (its pinning and its process pool stay out of this process)
    cpu = None if args.no_cpu else cpu_baseline_child()

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
    nodal = f.kind == femhip.FE_FN_NODAL

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

    ev = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731  (recorded on the launch stream)

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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plans.append(cold_step(times))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc = femhip.fe_plan_status(plans[-1])
    if rc != 0:
        raise RuntimeError(f"kernel status {rc}")
    for p in plans:
        femhip.fe_plan_destroy(p)
    ms_step = wall / args.steps * 1e3
    sym_ms = float(np.median([a.elapsed_time(b_) for a, b_, _, _ in times]))
    pat_ms = float(np.median([b_.elapsed_time(c) for _, b_, c, _ in times]))
    num_ms = float(np.median([c.elapsed_time(d) for _, _, c, d in times]))

    # the same steps with every kernel bracketed by events on its stream
    log(f"[bench] timing {args.steps} cold steps kernel by kernel")
    femhip.fe_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        femhip.fe_plan_destroy(cold_step())
    torch.cuda.synchronize()
    ms_step_prof = (time.perf_counter() - t0) / args.steps * 1e3
    kern = femhip.fe_prof_read()
    femhip.fe_prof_enable(False)
    kernels = kernel_table(kern, args.steps, N, NT, nnz, dim, nodal)
    counters = read_counters(args.workload)

    # what a plain device copy reaches on this GPU (read + write bytes over its time)
    log("[bench] timing a plain device copy")
    copy = copy_rate(torch, dev, 512)

    # warm numeric phase: plan reused, a different kappa each call
    log("[bench] timing warm numeric phase")
    plan, _ = femhip.fe_plan_create(mesh, ws)
    femhip.fe_plan_pattern(plan, rowptr, colind)
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
    sym = None
    if not args.no_sym:
        log("[bench] symmetric storage (upper triangle)")
        sym = symmetric_storage(femhip, torch, plan, node, kappa2, f, gn, rowptr, colind, val, N, args.steps)
    femhip.fe_plan_destroy(plan)
    roof = roofline(kernels, counters, N, NT, nnz, dim, nodal, ms_step, warm_ms)
    roof["copy_kernel_GBps"] = copy["GBps"]
    del node, elem, bd, kappa, kappa2, val, val_bc, b, b_load, isd, rowptr, colind, ws, mesh
    torch.cuda.empty_cache()

    c3 = None if (args.no_c3 or args.workload == "kuhn129") else bench_c3(args)
    nxt = None if args.no_next else bench_next(args)
    batched = None if args.no_batch else bench_batched(args)
    adjoint = None if args.no_adjoint else bench_adjoint(args)
    torch.cuda.synchronize()

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
        "symmetric_storage": sym,
        "kernels": {"ms_per_step_with_events": ms_step_prof, "by_kernel": kernels},
        "roofline": roof,
        "copy_kernel": copy,
        "c3": c3,
        "batched": batched,
        "next": nxt,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def symmetric_storage(femhip, torch, plan, node, kappa, f, gn, rowptr, colind, val, N, reps):
    """Upper-triangle storage on a plan whose pattern is written: warm fe_assemble_upper
    against warm fe_assemble (the same kernels, fewer entries written), and one SpMV
    in symmetric storage (A read as val_u[vidx[q]]) against one in full storage."""
    dev = node.device
    stream = torch.cuda.current_stream()
    rp_u = torch.empty(N + 1, dtype=torch.int32, device=dev)
    nnz_u = femhip.fe_plan_upper(plan, rowptr, colind, rp_u)
    ci_u = torch.empty(nnz_u, dtype=torch.int32, device=dev)
    vidx = torch.empty(colind.numel(), dtype=torch.int32, device=dev)
    femhip.fe_plan_upper(plan, rowptr, colind, rp_u, ci_u, vidx)
    val_u = torch.empty(nnz_u, dtype=torch.float64, device=dev)
    vbc_u = torch.empty_like(val_u)
    b = torch.empty(N, dtype=torch.float64, device=dev)
    bl = torch.empty_like(b)
    isd = torch.empty(N, dtype=torch.uint8, device=dev)
    full_bc = torch.empty_like(val)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    up_ms = timed(lambda: femhip.fe_assemble_upper(plan, rp_u, node, kappa, f, None, gn, None, 0.0, 0, val_u, vbc_u,
                                                   b, bl, isd))
    full_ms = timed(lambda: femhip.fe_assemble(plan, node, kappa, f, None, gn, val, full_bc, b, bl, isd))
    x = torch.randn(N, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(3))
    y = torch.empty_like(x)
    spmv_ms = timed(lambda: femhip.fe_spmv(rowptr, colind, val, x, y))
    spmv_sym_ms = timed(lambda: femhip.fe_spmv_sym(rowptr, colind, vidx, val_u, x, y))
    return {"nnz_upper": nnz_u, "warm_upper_ms": up_ms, "warm_full_ms": full_ms,
            "spmv_full_us": spmv_ms * 1e3, "spmv_symmetric_us": spmv_sym_ms * 1e3,
            "matrix_bytes_full": 12 * colind.numel(), "matrix_bytes_symmetric": 8 * nnz_u + 8 * colind.numel()}


def bench_batched(args):
    """256 jittered meshes, sides uniform in [17, 513]: one graph launch (assembly of
    the union + batched PCG) against the plain path looped over the instances."""
    import numpy as np
    import torch
    from paper_1804_05156_amd import batch, femhip, meshgen
    log("[bench] batched: generating 256 meshes")
    sizes = meshgen.batch_sizes()
    ms = meshgen.batch_meshes(sizes)
    dev = torch.device("cuda:0")
    nodes = [torch.from_numpy(m.node).to(dev) for m in ms]
    elems = [torch.from_numpy(m.elem).to(dev) for m in ms]
    bds = [torch.from_numpy(m.bdflag).to(dev) for m in ms]
    kaps = [torch.from_numpy(m.kappa).to(dev) for m in ms]
    kap = torch.cat(kaps).contiguous()
    f = femhip.Fn(femhip.FE_FN_SINPROD, (2 * math.pi ** 2,))
    rtol = 1e-10
    NT = int(sum(m.n_elem for m in ms))
    log("[bench] batched: building the union plan, autotuning the solve grid")
    B = batch.Batch(nodes, elems, bds)
    tune = batch.autotune(B, kap, f, None, None, rtol, log=lambda msg: log(f"[bench] batched: {msg}"))
    log(f"[bench] batched: autotune {tune}")
    B.assemble_solve(kap, f, None, None, rtol)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(reps):
        u, it, rel = B.assemble_solve(kap, f, None, None, rtol)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    # the plain path: one plan per instance (built beforehand), then assemble + solve each
    log("[bench] batched: plain path over the instances")
    plans = [femhip.Plan(n_, e_, b_) for n_, e_, b_ in zip(nodes, elems, bds)]
    asms = [p.assemble(k_, f) for p, k_ in zip(plans, kaps)]
    plans[0].solve(asms[0], rtol=rtol)   # first call of every kernel of the plain path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for k, (p, k_, a) in enumerate(zip(plans, kaps, asms)):
        p.assemble(k_, f, out=a)
        _, itk, _ = p.solve(a, rtol=rtol)
        its.append(itk)
        if k % 64 == 63:
            log(f"[bench] batched: plain path, {k + 1} instances done")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = its == list(it)
    info = B.info()
    # release the captured graph and every plan now, not at interpreter exit
    for p in plans:
        p.close()
    B.close()
    torch.cuda.synchronize()
    return {"workload": "256 jittered meshes, sides U{17..513}, lognormal kappa, rtol 1e-10",
            "n_inst": len(ms), "n_node": int(B.N), "n_elem": NT, "nnz": int(B.plan.nnz),
            "ms_batched": t_batch * 1e3, "ms_plain_loop": t_plain * 1e3, "speedup": t_plain / t_batch,
            "elements_per_s_batched": NT / t_batch, "iterations_max": int(max(it)),
            "iterations_sum": int(sum(it)), "iterations_equal_plain": same, "grid": info["grid"],
            "blocks_per_cu": info["blocks_per_cu"], "units_per_step": info["units_per_step"],
            "cooperative_in_graph": bool(info["cooperative"]),
            "autotune_ms": tune.get("ms")}


def bench_c3(args):
    """The 3-D configuration: 129^3 Kuhn cube (12.6M tetrahedra), lognormal kappa, nodal
    f, Dirichlet on x = 0, 1 and Neumann g_N = du/dn elsewhere.  Cold step (plan +
    pattern + numeric assembly) and warm numeric assembly, event-timed, every kernel
    of the cold step timed on its stream, and the roofline of its dominant kernel on
    the compulsory bytes of the step."""
    import numpy as np
    import torch
    from paper_1804_05156_amd import femhip, meshgen
    dev = torch.device("cuda:0")
    log("[bench] c3: 129^3 Kuhn cube")
    m = meshgen.workload("kuhn129")
    N, NT = m.n_node, m.n_elem
    node = torch.from_numpy(m.node).to(dev)
    elem = torch.from_numpy(m.elem).to(dev)
    bd = torch.from_numpy(m.bdflag).to(dev)
    kappa = torch.from_numpy(m.kappa).to(dev)
    u = torch.prod(torch.sin(math.pi * node), dim=0)
    f = femhip.Fn(femhip.FE_FN_NODAL, (0,), (3 * math.pi ** 2 * u).contiguous())
    gn = femhip.Fn(femhip.FE_FN_DUDN_SINPROD, (1.0,))
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
    reps = max(1, min(args.steps, 10))

    def cold():
        p, _ = femhip.fe_plan_create(mesh, ws)
        femhip.fe_plan_pattern(p, rowptr, colind)
        femhip.fe_assemble(p, node, kappa, f, None, gn, val, val_bc, b, b_load, isd)
        return p

    femhip.fe_plan_destroy(cold())
    torch.cuda.synchronize()
    plans = []
    t0 = time.perf_counter()
    for _ in range(reps):
        plans.append(cold())
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) / reps * 1e3
    rc = femhip.fe_plan_status(plans[-1])
    if rc != 0:
        raise RuntimeError(f"kernel status {rc}")
    for p in plans:
        femhip.fe_plan_destroy(p)
    # every kernel of the cold step on its stream
    femhip.fe_prof_enable(True)
    for _ in range(reps):
        femhip.fe_plan_destroy(cold())
    torch.cuda.synchronize()
    kern = femhip.fe_prof_read()
    femhip.fe_prof_enable(False)
    kernels = kernel_table(kern, reps, N, NT, nnz, 3, True)
    # warm numeric assembly
    plan = cold()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        femhip.fe_assemble(plan, node, kappa, f, None, gn, val, val_bc, b, b_load, isd)
    e1.record(stream)
    e1.synchronize()
    sym = None if args.no_sym else symmetric_storage(femhip, torch, plan, node, kappa, f, gn, rowptr, colind, val,
                                                     N, reps)
    femhip.fe_plan_destroy(plan)
    warm_ms = e0.elapsed_time(e1) / reps
    roof = roofline(kernels, read_counters("kuhn129"), N, NT, nnz, 3, True, cold_ms, warm_ms)
    k3 = kernels.get("k_assemble_3d")
    return {"workload": "kuhn129: 129^3 Kuhn cube, lognormal kappa, nodal f, Dirichlet x = 0, 1, Neumann elsewhere",
            "n_node": N, "n_elem": NT, "nnz": nnz, "cold_ms": cold_ms, "cold_elements_per_s": NT / (cold_ms * 1e-3),
            "warm_ms": warm_ms, "warm_elements_per_s": NT / (warm_ms * 1e-3),
            "k_assemble_3d_us": k3["avg_us"] if k3 else None, "symmetric_storage": sym,
            "kernels": kernels, "roofline": roof}


def bench_next(args):
    """The rows next to the core path: assembly on the L-shaped domain (cold and warm)
    and the pure Neumann solve (mean shift, pinned PCG, zero-mean shift)."""
    import numpy as np
    import torch
    from paper_1804_05156_amd import femhip, meshgen
    dev = torch.device("cuda:0")
    log("[bench] next: L-shape 1025 x 1025 bounding grid")
    m = meshgen.lshape_mesh(513, seed=9, kappa="lognormal")
    node = torch.from_numpy(m.node).to(dev)
    elem = torch.from_numpy(m.elem).to(dev)
    bd = torch.from_numpy(m.bdflag).to(dev)
    kap = torch.from_numpy(m.kappa).to(dev)
    f = femhip.Fn(femhip.FE_FN_CONST, (1.0,))
    reps = max(1, min(args.steps, 10))
    femhip.Plan(node, elem, bd).assemble(kap, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        p = femhip.Plan(node, elem, bd)
        a = p.assemble(kap, f)
    torch.cuda.synchronize()
    cold = (time.perf_counter() - t0) / reps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        p.assemble(kap, f, out=a)
    ev1.record()
    ev1.synchronize()
    warm = ev0.elapsed_time(ev1) / reps * 1e-3
    lshape = {"workload": "L-shape, 1025^2 bounding grid, lognormal kappa, f = 1, Dirichlet",
              "n_elem": m.n_elem, "cold_ms": cold * 1e3, "cold_elements_per_s": m.n_elem / cold,
              "warm_ms": warm * 1e3, "warm_elements_per_s": m.n_elem / warm}
    log("[bench] next: pure Neumann 1025^2")
    m = meshgen.square_mesh(1025, jitter=0.2, seed=5, kappa="lognormal", sides=(2, 2, 2, 2))
    fv = 2 * math.pi ** 2 * np.cos(math.pi * m.node[0]) * np.cos(math.pi * m.node[1])
    node = torch.from_numpy(m.node).to(dev)
    p = femhip.Plan(node, torch.from_numpy(m.elem).to(dev), torch.from_numpy(m.bdflag).to(dev))
    a = p.assemble(torch.from_numpy(m.kappa).to(dev), femhip.Fn(femhip.FE_FN_NODAL, (0.0,), torch.from_numpy(fv).to(dev)))
    p.neumann_solve(a, rtol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, it, rel, mb = p.neumann_solve(a, rtol=1e-10)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    neumann = {"workload": "1025^2 jittered, lognormal kappa, all sides Neumann, f = 2 pi^2 cos cos (nodal), rtol 1e-10",
               "ms": t * 1e3, "iterations": it, "relres": rel, "mean_b": mb, "us_per_iteration": t / max(it, 1) * 1e6}
    return {"lshape": lshape, "pure_neumann": neumann}


def bench_adjoint(args):
    """1025^2 mesh: forward solve vs forward + adjoint solve + gradient kernel."""
    import numpy as np
    import torch
    from paper_1804_05156_amd import femhip, meshgen
    log("[bench] adjoint: 1025^2 mesh")
    m = meshgen.workload("jitter1025")
    dev = torch.device("cuda:0")
    node = torch.from_numpy(m.node).to(dev)
    elem = torch.from_numpy(m.elem).to(dev)
    bd = torch.from_numpy(m.bdflag).to(dev)
    kap = torch.from_numpy(m.kappa).to(dev)
    plan = femhip.Plan(node, elem, bd)
    f = femhip.Fn(femhip.FE_FN_SINPROD, (2 * math.pi ** 2,))
    rtol = 1e-10
    kobs = torch.exp(torch.from_numpy(np.random.default_rng(55).standard_normal(m.n_elem)).to(dev))
    u_obs = femhip.PoissonSolve.apply(kobs, plan, f, None, None, rtol).detach()
    reps = max(1, min(args.steps, 3))

    def forward():
        return femhip.PoissonSolve.apply(kap, plan, f, None, None, rtol)

    def forward_backward():
        k = kap.clone().requires_grad_(True)
        u = femhip.PoissonSolve.apply(k, plan, f, None, None, rtol)
        J = 0.5 * torch.sum((u - u_obs) ** 2)
        J.backward()
        return k.grad

    for fn in (forward, forward_backward):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        forward()
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        forward_backward()
    torch.cuda.synchronize()
    t_fb = (time.perf_counter() - t0) / reps
    # the gradient kernel alone
    lam = torch.randn(m.n_node, dtype=torch.float64, device=dev)
    u = forward().detach()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        plan.grad(u, lam)
    e1.record()
    e1.synchronize()
    g_ms = e0.elapsed_time(e1) / 10
    NT = m.n_elem
    # PCG iterations of the forward solve and its time per iteration
    asm = plan.assemble(kap, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters, _ = plan.solve(asm, rtol=rtol)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    # the same solve with A_bc in symmetric (upper-triangle) storage
    N = m.n_node
    rp_u = torch.empty(N + 1, dtype=torch.int32, device=dev)
    ci = plan.colind[:plan.nnz]
    nnz_u = femhip.fe_plan_upper(plan.handle, plan.rowptr, ci, rp_u)
    ci_u = torch.empty(nnz_u, dtype=torch.int32, device=dev)
    vidx = torch.empty(plan.nnz, dtype=torch.int32, device=dev)
    femhip.fe_plan_upper(plan.handle, plan.rowptr, ci, rp_u, ci_u, vidx)
    val_u = torch.empty(nnz_u, dtype=torch.float64, device=dev)
    vbc_u = torch.empty_like(val_u)
    bu = torch.empty(N, dtype=torch.float64, device=dev)
    isd = torch.empty(N, dtype=torch.uint8, device=dev)
    femhip.fe_assemble_upper(plan.handle, rp_u, node, kap, f, None, None, None, 0.0, 0, val_u, vbc_u, bu, None, isd)
    u_sym = torch.empty_like(bu)
    femhip.fe_select(isd, bu, None, u_sym)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_sym, _, _ = femhip.fe_solve_sym(plan.rowptr, ci, vidx, vbc_u, bu, u_sym, rtol, 100000, plan.solve_workspace())
    torch.cuda.synchronize()
    t_sym = time.perf_counter() - t0
    plan.close()
    return {"workload": "1025^2 jittered mesh, lognormal kappa, u_obs from a second kappa, rtol 1e-10",
            "forward_pcg_iterations": int(iters), "us_per_pcg_iteration": t_s / max(int(iters), 1) * 1e6,
            "symmetric_storage_pcg": {"iterations": it_sym, "ms": t_sym * 1e3,
                                      "us_per_iteration": t_sym / max(it_sym, 1) * 1e6},
            "ms_forward": t_f * 1e3, "ms_forward_adjoint_grad": t_fb * 1e3, "ratio": t_fb / t_f,
            "ms_grad_kernel": g_ms, "grad_elements_per_s": NT / (g_ms * 1e-3),
            "fd_equivalent_ms": 2 * NT * t_f * 1e3}


def copy_rate(torch, dev, mb, launches=10):
    """A plain device copy of mb MiB: read + write bytes per launch over its mean time."""
    n = mb * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(launches):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / launches
    del src, dst
    return {"bytes_per_launch": 2 * n * 8, "avg_us": us, "GBps": 2 * n * 8 / (us * 1e-6) / 1e9,
            "kind": f"torch copy_ of a {mb} MiB float64 tensor"}


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


def _median_time(fn, reps=3):
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return sorted(ts)[len(ts) // 2], ts


def _pool_instance(args):
    """One instance of the batched workload on the CPU: oracle assembly and solve."""
    import oracle
    from paper_1804_05156_amd import meshgen
    k, side = args
    m = meshgen.square_mesh(int(side), jitter=0.2, seed=4000 + k, kappa="lognormal")
    t = time.perf_counter()
    a = oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=oracle.Fn(oracle.FN_SINPROD, (2 * math.pi ** 2,)))
    _, it, _ = oracle.solve(a, rtol=1e-10)
    return m.n_elem, it, time.perf_counter() - t


def cpu_baseline_child():
    """cpu_baseline() in a child interpreter (this process has not used the GPU yet)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only"], capture_output=True,
                       text=True)
    sys.stderr.write(r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline failed with status {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline():
    """The oracle as it stands (plain single-threaded C), on the host, before any GPU
    call.  Single-thread legs are pinned to one core and take the median of 3 runs:
    the 2-D recipe (jittered, permuted, lognormal kappa, analytic f) at 1025^2 and the
    3-D recipe (Kuhn cube, lognormal kappa, nodal f, Dirichlet/Neumann) at 65^3.  The
    batched leg runs one process per instance on a 16-instance sample of the batch
    (every 16th instance of the 256), oracle assembly + solve to 1e-10 each."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    import oracle
    from paper_1804_05156_amd import meshgen
    oracle.lib()
    allowed = sorted(os.sched_getaffinity(0))
    out = {"kind": "oracle", "unit": "elements/s", "cores": 1, "cpu": _cpu_model(), "host_threads": len(allowed)}
    log(f"[bench] cpu baseline: pinned to core {allowed[0]} of {len(allowed)}")
    os.sched_setaffinity(0, {allowed[0]})
    try:
        m = meshgen.square_mesh(1025, jitter=0.2, permute=True, seed=2, kappa="lognormal")
        f = oracle.Fn(oracle.FN_SINPROD, (2 * math.pi ** 2,))
        med, ts = _median_time(lambda: oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=f))
        out.update({"value": m.n_elem / med, "seconds_median": med, "seconds": ts,
                    "sample": "2-D recipe of the 2049^2 workload at 1025^2 (jittered, permuted, lognormal kappa, "
                              "analytic f, Dirichlet): 2,097,152 triangles, one oracle assembly, median of 3"})
        m = meshgen.kuhn_cube(65, seed=3, kappa="lognormal")
        u = np.prod(np.sin(math.pi * m.node), axis=0)
        f = oracle.Fn(oracle.FN_NODAL, (0,), 3 * math.pi ** 2 * u)
        gn = oracle.Fn(oracle.FN_DUDN_SINPROD, (1.0,))
        med, ts = _median_time(lambda: oracle.assemble(m.node, m.elem, m.bdflag, m.kappa, f=f, gN=gn))
        out["c3"] = {"value": m.n_elem / med, "unit": "elements/s", "cores": 1, "seconds_median": med,
                     "seconds": ts, "sample": f"3-D recipe of the 129^3 workload at 65^3: {m.n_elem} tetrahedra, "
                                               "one oracle assembly, median of 3"}
    finally:
        os.sched_setaffinity(0, set(allowed))
    sizes = meshgen.batch_sizes()
    sample = [(k, int(sizes[k])) for k in range(0, len(sizes), 16)]
    workers = min(16, len(allowed), len(sample))
    log(f"[bench] cpu baseline: batched sample of {len(sample)} instances on {workers} processes")
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_pool_instance, sample))
    wall = time.perf_counter() - t
    nel = sum(r[0] for r in res)
    out["c4_pool"] = {"value": nel / wall, "unit": "elements/s (assembly + solve)", "cores": workers,
                      "instances_per_s": len(sample) / wall, "seconds": wall,
                      "iterations_max": max(r[1] for r in res),
                      "sample": f"{len(sample)} instances of the 256-mesh batch (every 16th; sides "
                                f"{min(s for _, s in sample)}..{max(s for _, s in sample)}), one process per "
                                "instance, oracle assembly + solve to rtol 1e-10"}
    return out


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
