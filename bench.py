"""Benchmark of the space-time Biot slab solver on one MI355X.

One step = one time slab of the heterogeneous 2D workload (128 x 128 cells,
dG(1) on Gauss-Radau points, Q2/RT1/DG-Q1, log-normal K with sigma 1 and
correlation length 0.1, ramp load): slab right-hand side, preconditioned GMRES
solve to relative residual 1e-12 in FP64, state update.  The timed region
holds exactly --steps slabs of the march with all inputs resident on the GPU.

Printed JSON (one line): value = space-time DoFs advanced per second
(slab DoFs x slabs / wall time).  Extra objects: the operator-apply
throughput (space-time DoF-applies/s, FP64 and FP32), the same march in mixed
precision, the roofline of the operator-apply kernel measured with HIP events
on the stream it runs on, and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "space-time DoF-applies/s and slab solve time at 1e-10 rel. err, FP64 vs mixed"


def _apply_bytes(h, wbytes):
    # algorithmic bytes of one apply: read X, write Y (every slab DoF once), read K per cell
    ncells = sum(int(np.prod(w.n)) for w in h.wls)
    return 2 * h.slab_len * wbytes + ncells * wbytes


def time_apply(torch, h, dtype, launches=200, pool_bytes=1 << 30):
    """Average duration of one apply_operator launch (HIP events on its stream).

    X/Y rotate over a pool larger than the 256 MB last-level cache so the
    kernel streams from HBM."""
    wb = 8 if dtype == torch.float64 else 4
    per = h.slab_len * wb * 2
    npool = max(2, min(64, pool_bytes // max(per, 1)))
    xs = [torch.randn(h.slab_len, dtype=dtype, device="cuda") for _ in range(npool)]
    ys = [torch.empty_like(xs[0]) for _ in range(npool)]
    for i in range(5):
        h.apply(xs[i % npool], ys[i % npool])
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(launches):
        h.apply(xs[i % npool], ys[i % npool])
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / launches
    return ms, _apply_bytes(h, wb)


def cpu_baseline(n=32, nslabs=10):
    """FP64 oracle (assembly + sparse LU + slab solves), single thread."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import slab
    wl = W.c2_hetero2d().scaled((n, n), nslabs=nslabs)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob = slab.problem_from_workload(wl)
        prob.march(nslabs)
        dt = time.perf_counter() - t0
    dofs = prob.L * prob.N
    return {"value": nslabs * dofs / dt, "unit": "space-time DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"2D {n}x{n} cells, same physics and dG(1), {nslabs} slabs: assembly, one SuperLU "
                      f"factorisation, {nslabs} slab solves ({nslabs * dofs} space-time DoFs, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--apply-only", action="store_true", help="only launch the operator apply (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is described in "
                                   "DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1801_04984_amd import BiotSlab

    assert torch.cuda.is_available(), "bench needs a GPU"
    wl = W.ALL[args.workload]()
    theta = wl.log_k()
    h = BiotSlab([wl], [theta])
    slab_dofs = h.slab_len

    if args.apply_only:
        ms64, b64 = time_apply(torch, h, torch.float64, launches=50)
        x = torch.randn(1 << 26, device="cuda")       # 256 MiB copy for counter calibration
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"apply_ms": ms64, "apply_bytes": b64, "copy_bytes": 2 * x.numel() * 4}))
        return

    def march(nsteps, t0, state, precision):
        infos_all = []
        for k in range(nsteps):
            infos, st = h.step(1, t0 + k * wl.tau, state, precision=precision)
            if st != 0:
                raise RuntimeError(f"slab solve failed: {infos}")
            infos_all.append(infos[0])
        return infos_all

    state = h.zeros_state()
    march(args.warmup, 0.0, state, 0)
    torch.cuda.synchronize()
    t_start = args.warmup * wl.tau
    t0 = time.perf_counter()
    infos = march(args.steps, t_start, state, 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * slab_dofs / dt
    its = [i["iterations"] for i in infos]

    out = {
        "metric": METRIC, "value": value, "unit": "space-time DoF/s (slab solved to rel. residual 1e-12, FP64)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded log-normal permeability)",
        "config": {"workload": f"{wl.name}: 2D {wl.n[0]}x{wl.n[1]} cells, Q2/RT1/DG-Q1, dG({wl.r}), tau={wl.tau}, "
                               f"log-normal K sigma={wl.k_sigma} ell={wl.k_ell} seed={wl.k_seed}",
                   "slab_dofs": slab_dofs, "parallelism": "single GPU"},
        "gmres_iterations_per_slab": {"mean": float(np.mean(its)), "min": int(min(its)), "max": int(max(its))},
    }

    if not args.no_mixed:
        st2 = h.zeros_state()
        march(args.warmup, 0.0, st2, 1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        inf2 = march(args.steps, t_start, st2, 1)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t1
        diff = (torch.linalg.norm(st2 - state) / torch.linalg.norm(state)).item()
        out["mixed"] = {"value": args.steps * slab_dofs / dt2, "ms_per_step": 1e3 * dt2 / args.steps,
                        "speedup_vs_fp64": dt / dt2,
                        "end_state_rel_diff_vs_fp64": diff,
                        "inner_iterations_per_slab": float(np.mean([i["iterations"] for i in inf2])),
                        "refinement_sweeps_per_slab": float(np.mean([i["ir_sweeps"] for i in inf2]))}

    ms64, by64 = time_apply(torch, h, torch.float64)
    ms32, by32 = time_apply(torch, h, torch.float32)
    out["apply"] = {"fp64": {"dof_applies_per_s": slab_dofs / (ms64 * 1e-3), "us": ms64 * 1e3},
                    "fp32": {"dof_applies_per_s": slab_dofs / (ms32 * 1e-3), "us": ms32 * 1e3}}
    ach = by64 / (ms64 * 1e-3) / 1e9
    out["roofline"] = {"kernel": "apply2d_kernel<double, 2, false> (space-time operator apply)",
                       "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": None,
                       "algorithmic_bytes_per_launch": by64}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
