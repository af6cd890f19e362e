"""Benchmark of the space-time Biot slab solver on one MI355X.

One step = one time slab of the heterogeneous 2D workload (128 x 128 cells,
dG(1) on Gauss-Radau points, Q2/RT1/DG-Q1, log-normal K with sigma 1 and
correlation length 0.1, ramp load): slab right-hand side, preconditioned GMRES
solve to relative residual 1e-12 in FP64, state update.  The timed region
holds exactly --steps slabs of the march with all inputs resident on the GPU.

Printed JSON (one line): value = space-time DoFs advanced per second
(slab DoFs x slabs / wall time).  Extra objects:
  mixed         the same march with FP32 inner solves in FP64 refinement;
  fp32_preconditioned  the same march by FP64 flexible GMRES with the
                preconditioner in FP32;
  apply         operator-apply throughput (space-time DoF-applies/s), FP64/FP32;
  roofline      HBM roofline of the operator apply on this workload, timed with
                HIP events on the stream it runs on;
  apply_large   the same for the 3D 48^3 dG(2) workload and the 64-instance
                batch, whose vectors exceed the 256 MB last-level cache;
  batched       64 uneven 2D instances solved together (FP64 and both mixed modes) against
                the same instances solved one handle at a time (sampled);
  cpu_baseline  the FP64 oracle on a bounded sample, one host core.
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
    # algorithmic bytes of one apply: read X, write Y (every slab DoF once), read eta/K per cell
    ncells = sum(int(np.prod(w.n)) for w in h.wls)
    return 2 * h.slab_len * wbytes + ncells * wbytes


def time_apply(torch, h, dtype, launches=200, pool_bytes=1 << 30):
    """Average duration of one apply_operator launch, from HIP events recorded
    on the stream the apply is launched on.

    X/Y rotate over a pool larger than the 256 MB last-level cache so the
    kernel streams from HBM."""
    wb = 8 if dtype == torch.float64 else 4
    per = h.slab_len * wb * 2
    npool = int(max(2, min(64, pool_bytes // max(per, 1))))
    xs = [torch.randn(h.slab_len, dtype=dtype, device=h.device) for _ in range(npool)]
    ys = [torch.empty_like(xs[0]) for _ in range(npool)]
    s = torch.cuda.current_stream(h.device)   # the stream BiotSlab passes to every call
    for i in range(5):
        h.apply(xs[i % npool], ys[i % npool])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(launches):
        h.apply(xs[i % npool], ys[i % npool])
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / launches
    del xs, ys
    return ms, _apply_bytes(h, wb)


def roofline_of(ms, nbytes):
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": nbytes, "launch_us": ms * 1e3}


def measured_traffic(kernel_key):
    """HBM bytes per launch of `kernel_key` from the committed FETCH_SIZE/WRITE_SIZE
    record (copy-calibrated), or None when the record is missing or the kernel
    source changed after the counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "apply2d_2d_128_dg1_pmc.json")
    src = os.path.join(ROOT, "paper_1801_04984_amd", "csrc", "apply2d.hip")
    try:
        rec = json.load(open(rec_path))
        if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return rec["kernels"][kernel_key]["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def march(h, nsteps, t0, state, precision):
    infos_all = []
    for k in range(nsteps):
        infos, st = h.step(1, t0 + k * h.wls[0].tau, state, precision=precision)
        if st != 0:
            raise RuntimeError(f"slab solve failed: {infos}")
        infos_all.append(infos)
    return infos_all


def cpu_baseline(n=32, nslabs=30):
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


def apply_large(torch, W, BiotSlab, tuning):
    """Apply rooflines on workloads whose vectors exceed the last-level cache."""
    out = {}
    for key, wls in (("3d_48_dg2", [W.c4_adjoint3d()]), ("batch64_2d_dg1", W.c5_batch())):
        h = BiotSlab(wls, [w.log_k() for w in wls])
        tuning.tune(h, path=None)
        rec = {"slab_dofs": h.slab_len}
        for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
            ms, nb = time_apply(torch, h, dt, launches=50)
            rec[name] = dict(roofline_of(ms, nb), dof_applies_per_s=h.slab_len / (ms * 1e-3))
        rec["tile_variant"] = h.get_tuning()["apply_variant"]
        out[key] = rec
        h.close()
        del h
        torch.cuda.empty_cache()
    return out


def batched(torch, W, BiotSlab, tuning, nsteps=2, sample_every=8):
    """64 uneven instances in one handle vs the same instances one at a time."""
    wls = W.c5_batch()
    h = BiotSlab(wls, [w.log_k() for w in wls])
    tuning.tune(h, path=None)
    res = {"instances": len(wls), "slab_dofs_total": h.slab_len}
    for name, prec in (("fp64", 0), ("mixed", 1), ("fp32_preconditioned", 2)):
        st = h.zeros_state()
        march(h, 1, 0.0, st, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = march(h, nsteps, wls[0].tau, st, prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"dofs_per_s": nsteps * h.slab_len / dt, "ms_per_slab": 1e3 * dt / nsteps,
                     "max_iterations": int(max(i["iterations"] for inf in infos for i in inf))}
    h.close()
    del h
    torch.cuda.empty_cache()
    # sequential reference: every sample_every-th instance in a handle of its own
    tot_dofs, tot_t = 0, 0.0
    for w in wls[::sample_every]:
        g = BiotSlab([w], [w.log_k()])
        tuning.tune(g, path=None)
        st = g.zeros_state()
        march(g, 1, 0.0, st, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        march(g, nsteps, w.tau, st, 0)
        torch.cuda.synchronize()
        tot_t += time.perf_counter() - t0
        tot_dofs += nsteps * g.slab_len
        g.close()
    seq = tot_dofs / tot_t
    res["sequential_fp64"] = {"dofs_per_s": seq, "sample": f"instances 0,{sample_every},...: "
                              f"{len(wls[::sample_every])} of {len(wls)}, {nsteps} slabs each"}
    res["speedup_fp64_vs_sequential"] = res["fp64"]["dofs_per_s"] / seq
    res["speedup_mixed_vs_sequential"] = res["mixed"]["dofs_per_s"] / seq
    res["speedup_fp32_preconditioned_vs_sequential"] = res["fp32_preconditioned"]["dofs_per_s"] / seq
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2",
                    help="c1 2D Terzaghi 8x8 dG(0); c2 2D 128x128 dG(1) heterogeneous; c3 3D 32^3 dG(1); "
                         "c4 3D 48^3 dG(2); with --apply-only also c5 (64 uneven 2D instances)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the large-workload apply and batched objects")
    ap.add_argument("--apply-only", action="store_true", help="only time the operator apply (profiling target)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "biotst runs on one GPU only: sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1801_04984_amd import BiotSlab, tuning

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.apply_only:
        # profiling target: autotune, 50 FP64 and 50 FP32 applies, one 256 MiB copy
        # (counter calibration); --workload c5 selects the 64-instance batch
        wls = W.c5_batch() if args.workload == "c5" else [W.ALL[args.workload]()]
        h = BiotSlab(wls, [w.log_k() for w in wls])
        tuning.tune(h, path=None)
        ms64, b64 = time_apply(torch, h, torch.float64, launches=50)
        ms32, b32 = time_apply(torch, h, torch.float32, launches=50)
        x = torch.randn(1 << 26, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"workload": args.workload, "apply_ms": [ms64, ms32], "apply_bytes": [b64, b32],
                          "tile_variant": h.get_tuning()["apply_variant"], "copy_bytes": 2 * x.numel() * 4}))
        return
    wl = W.ALL[args.workload]()
    theta = wl.log_k()
    h = BiotSlab([wl], [theta])
    tune = tuning.tune(h, path=None)
    slab_dofs = h.slab_len

    state = h.zeros_state()
    march(h, args.warmup, 0.0, state, 0)
    torch.cuda.synchronize()
    t_start = args.warmup * wl.tau
    t0 = time.perf_counter()
    infos = march(h, args.steps, t_start, state, 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * slab_dofs / dt
    its = [i[0]["iterations"] for i in infos]

    out = {
        "metric": METRIC, "value": value, "unit": "space-time DoF/s (slab solved to rel. residual 1e-12, FP64)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded log-normal permeability)",
        "config": {"workload": f"{wl.name}: 2D {wl.n[0]}x{wl.n[1]} cells, Q2/RT1/DG-Q1, dG({wl.r}), tau={wl.tau}, "
                               f"log-normal K sigma={wl.k_sigma} ell={wl.k_ell} seed={wl.k_seed}",
                   "slab_dofs": slab_dofs, "parallelism": "single GPU"},
        "gmres_iterations_per_slab": {"mean": float(np.mean(its)), "min": int(min(its)), "max": int(max(its))},
        "apply_tile_variant": tune["apply_variant"],
    }

    if not args.no_mixed:
        for key, prec in (("mixed", 1), ("fp32_preconditioned", 2)):
            st2 = h.zeros_state()
            march(h, args.warmup, 0.0, st2, prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            inf2 = march(h, args.steps, t_start, st2, prec)
            torch.cuda.synchronize()
            dt2 = time.perf_counter() - t1
            diff = (torch.linalg.norm(st2 - state) / torch.linalg.norm(state)).item()
            out[key] = {"value": args.steps * slab_dofs / dt2, "ms_per_step": 1e3 * dt2 / args.steps,
                        "speedup_vs_fp64": dt / dt2,
                        "end_state_rel_diff_vs_fp64": diff,
                        "iterations_per_slab": float(np.mean([i[0]["iterations"] for i in inf2])),
                        "refinement_sweeps_per_slab": float(np.mean([i[0]["ir_sweeps"] for i in inf2]))}

    ms64, by64 = time_apply(torch, h, torch.float64)
    ms32, by32 = time_apply(torch, h, torch.float32)
    out["apply"] = {"fp64": {"dof_applies_per_s": slab_dofs / (ms64 * 1e-3), "us": ms64 * 1e3},
                    "fp32": {"dof_applies_per_s": slab_dofs / (ms32 * 1e-3), "us": ms32 * 1e3}}
    # tile variants: 0 = 16x16 tiles, 1 = 8x8 tiles, 2 = 8x8 tiles with the time levels in parallel
    ts, lp = {0: (16, "false"), 1: (8, "false"), 2: (8, "true")}[tune["apply_variant"][0]]
    kkey = f"bt::apply2d_kernel<double, 2, false, {ts}, {lp}>"
    out["roofline"] = dict(roofline_of(ms64, by64), kernel=kkey + " (space-time operator apply, FP64)",
                           traffic=measured_traffic(kkey))
    h.close()
    del h
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["apply_large"] = apply_large(torch, W, BiotSlab, tuning)
        out["batched"] = batched(torch, W, BiotSlab, tuning)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
