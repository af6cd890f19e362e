"""Benchmark of the space-time Biot slab solver on one MI355X.

Default workload: 3D 48^3 hexahedra, dG(2) on right Gauss-Radau points,
Q2/RT1/DG-Q1 (18,913,833 slab unknowns), log-normal K (sigma 1.5, correlation
length 0.15), ramp load, tau = 0.1.  One step = one time slab: slab right-hand
side, preconditioned GMRES solve to relative residual 1e-13 in FP64, state
update.  The timed region holds exactly --steps slabs of the march (after
--warmup untimed slabs) with all inputs resident on the GPU.

Printed JSON (one line): value = space-time DoFs advanced per second
(slab DoFs x slabs / wall time) of the plain FP64 path.  Extra objects:
  mixed, fp32_preconditioned  the same march with FP32 inner solves in FP64
                refinement / FP64 flexible GMRES with the preconditioner in
                FP32; per-field relative l2 difference from the FP64 march
                (last slab, all levels; and the end state);
  apply         operator-apply throughput (space-time DoF-applies/s) and its
                HBM fraction, FP64/FP32, over a buffer pool larger than the
                last-level cache;
  roofline      the dominant kernel of the step (the elasticity operator of the
                preconditioner's multigrid on the fine level in 3D, the slab
                operator in 2D), timed with HIP events on the stream it runs on;
  adjoint       (3D) forward march with checkpoints and the adjoint sweep for
                the pressure-misfit gradient at 64 sensors, FP64 and mixed;
  batched       64 uneven 2D instances (dG(1)) solved and differentiated
                together against the same instances one handle at a time;
  cpu_baseline  the FP64 oracle (sparse LU) on a bounded sample of the same
                physics, one host core; plus the oracle's CSR SpMV rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MATRIX_PEAK_TFS = 78.6
METRIC = "space-time DoF-applies/s and slab solve time at 1e-10 rel. err, FP64 vs mixed"
# Relative residual tolerance of every timed slab solve.  On the 48^3 march the
# late slabs' flux and pressure are a few hundred times smaller than at their
# peak, and 1e-12 leaves them at ~3e-9 relative error (measured against a refined
# reference); 1e-13 brings every path to ~1e-10 (the FP64 residual floor is
# ~1.5e-13).  The per-field errors are measured and reported with every run.
RTOL = 1e-13
PMC_RECORD = os.path.join(ROOT, "profiles", "counters_pmc.json")


def _apply_bytes(h, wbytes):
    # algorithmic bytes of one apply: read X, write Y (every slab DoF once), read eta/K per cell
    ncells = sum(int(np.prod(w.n)) for w in h.wls)
    return 2 * h.slab_len * wbytes + ncells * wbytes


def _pool(torch, h, dtype, pool_bytes=1 << 30):
    wb = 8 if dtype == torch.float64 else 4
    per = h.slab_len * wb * 2
    npool = int(max(2, min(64, pool_bytes // max(per, 1))))
    xs = [torch.randn(h.slab_len, dtype=dtype, device=h.device) for _ in range(npool)]
    ys = [torch.zeros_like(xs[0]) for _ in range(npool)]
    return xs, ys


def time_launches(torch, h, fn, dtype, launches):
    """Average duration of one launch of fn(x, y), from HIP events recorded on
    the stream the library is handed (torch's current stream); X/Y rotate over
    a pool larger than the 256 MB last-level cache so the kernel streams from HBM."""
    xs, ys = _pool(torch, h, dtype)
    s = torch.cuda.current_stream(h.device)
    for i in range(3):
        fn(xs[i % len(xs)], ys[i % len(ys)])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(launches):
        fn(xs[i % len(xs)], ys[i % len(ys)])
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / launches
    del xs, ys
    return ms


def hbm_roofline(ms, nbytes):
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": nbytes, "launch_us": ms * 1e3}


def measured_traffic(kernel_key):
    """HBM bytes per launch of `kernel_key` from the committed FETCH_SIZE/WRITE_SIZE
    record (copy-calibrated), or None when the record is missing or any source
    it was taken from has changed since."""
    try:
        rec = json.load(open(PMC_RECORD))
        k = rec["kernels"][kernel_key]
        for path, sha in k["sources_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, path), "rb").read()).hexdigest() != sha:
                return None
        return k["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def march(h, nsteps, t0, state, precision, slabs_last=None, state_before_last=None):
    infos_all = []
    for k in range(nsteps):
        out = slabs_last if (slabs_last is not None and k == nsteps - 1) else None
        if state_before_last is not None and k == nsteps - 1:
            state_before_last.copy_(state)
        infos, st = h.step(1, t0 + k * h.wls[0].tau, state, slabs_out=out, precision=precision, rtol=RTOL)
        if st != 0:
            raise RuntimeError(f"slab solve failed: {infos}")
        infos_all.append(infos)
    return infos_all


def field_rel(h, a, b):
    """Per-field relative l2 difference of two slab (or state) vectors of a
    single-instance handle; levels = number of levels the vectors hold."""
    N = h.level_dofs[0]
    levels = a.numel() // N
    d = h.wls[0].dim
    n = h.wls[0].n
    nu = d * int(np.prod([2 * m + 1 for m in n]))
    nq = sum((2 * n[c] + 1) * int(np.prod([2 * n[e] for e in range(d) if e != c])) for c in range(d))
    out = {}
    for name, lo, hi in (("u", 0, nu), ("q", nu, nu + nq), ("p", nu + nq, N)):
        aa = a.view(levels, N)[:, lo:hi]
        bb = b.view(levels, N)[:, lo:hi]
        nb = float(bb.norm())
        out[name] = float((aa - bb).norm()) / (nb if nb > 0 else 1.0)
    return out


def slab_error(h, state_in, t, slab, sweeps=3):
    """Per-field relative l2 error of a solved slab against a reference for the
    same slab (same entering state): FP64 GMRES to its rounding floor, then FP64
    iterative refinement (residual b - A x by the operator apply, correction by
    GMRES to 1e-6 of it), which takes the residual below the GMRES floor.
    Returns (errors, relative residual of the reference)."""
    torch = h.torch
    rhs = h.rhs(state_in, t)
    ref, info, st = h.solve(rhs, rtol=1e-14, maxit=4000)
    for _ in range(sweeps):
        r = rhs - h.apply(ref)
        d, _, _ = h.solve(r, rtol=1e-6, maxit=2000)
        ref += d
    res = float(torch.linalg.norm(rhs - h.apply(ref)) / torch.linalg.norm(rhs))
    return field_rel(h, slab, ref), res


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"host_cpu": model, "host_nproc": os.cpu_count()}


def cpu_baseline(wl_full, n, nslabs):
    """The FP64 oracle (assembly + one sparse LU + slab solves), one thread, on a
    bounded sample: the same physics, dG order and slab length on n^d cells."""
    from threadpoolctl import threadpool_limits
    from oracle import slab
    wl = wl_full.scaled((n,) * wl_full.dim)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob = slab.problem_from_workload(wl)
        prob.march(nslabs)
        dt = time.perf_counter() - t0
        A = prob.slab_matrix()
        x = np.random.default_rng(0).standard_normal(A.shape[0])
        k, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < 1.0:
            A @ x
            k += 1
        spmv_s = (time.perf_counter() - t1) / k
    dofs = prob.L * prob.N
    shape = "x".join([str(n)] * wl.dim)
    rec = {"value": nslabs * dofs / dt, "unit": "space-time DoF/s", "cores": 1, "kind": "oracle",
           "sample": f"{wl.dim}D {shape} cells, same physics, dG({wl.r}), tau {wl.tau}, {nslabs} slabs: assembly, "
                     f"one SuperLU factorisation (nested dissection), {nslabs} slab solves "
                     f"({nslabs * dofs} space-time DoFs, {dt:.1f} s)",
           "spmv": {"value": dofs / spmv_s, "unit": "space-time DoF-applies/s",
                    "sample": f"CSR product with the assembled slab matrix ({A.shape[0]} unknowns, {A.nnz} nonzeros)"}}
    rec.update(host_info())
    return rec


def adjoint_timing(torch, W, h, nslabs, precision):
    """Forward march with checkpoints, then the adjoint sweep (recompute + transposed solve per slab)."""
    wl = h.wls[0]
    sens = W.sensors(W.C4_NSENS, wl.dim, W.C4_SENSOR_SEED)
    p_obs = torch.tensor(0.05 * np.random.default_rng(W.C4_OBS_K_SEED).standard_normal(nslabs * len(sens)),
                         device=h.device)
    state = h.zeros_state()
    chk = torch.zeros(nslabs * h.state_len, dtype=torch.float64, device=h.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, st = h.step(nslabs, 0.0, state, checkpoints=chk, precision=precision, rtol=RTOL)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J, g, st2 = h.adjoint(nslabs, 0.0, chk, sens, p_obs, precision=precision, rtol=RTOL)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if st != 0 or st2 != 0:
        raise RuntimeError(f"adjoint run failed: {st}, {st2}")
    return {"slabs": nslabs, "sensors": len(sens), "params": int(g.numel()),
            "forward_ms_per_slab": 1e3 * (t1 - t0) / nslabs, "adjoint_ms_per_slab": 1e3 * (t2 - t1) / nslabs,
            "J": J[0], "grad_norm": float(g.norm())}


def batched(torch, W, BiotSlab, tuning, nsteps=4, sample_every=8):
    """64 uneven 2D instances in one handle vs the same instances one at a time."""
    wls = W.c5_batch()
    h = BiotSlab(wls, [w.log_k() for w in wls])
    tuning.tune(h, path=None)
    res = {"instances": len(wls), "slab_dofs_total": h.slab_len, "slabs_timed": nsteps}
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
        if prec == 0:
            ref_state = st.clone()
        else:
            res[name]["end_state_rel_diff_vs_fp64"] = float((st - ref_state).norm() / ref_state.norm())
    # batched forward (with checkpoints) + adjoint gradients of all 64 instances
    sens = W.sensors(16, 2, 77)
    p_obs = torch.tensor(0.05 * np.random.default_rng(78).standard_normal(len(wls) * nsteps * len(sens)),
                         device=h.device)
    state = h.zeros_state()
    chk = torch.zeros(nsteps * h.state_len, dtype=torch.float64, device=h.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, st1 = h.step(nsteps, 0.0, state, checkpoints=chk, rtol=RTOL)
    J, g, st2 = h.adjoint(nsteps, 0.0, chk, sens, p_obs, rtol=RTOL)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if st1 != 0 or st2 != 0:
        raise RuntimeError(f"batched adjoint failed: {st1}, {st2}")
    res["forward_adjoint_fp64"] = {"ms_per_slab": 1e3 * dt / nsteps, "params": int(g.numel()),
                                   "sensors_per_instance": len(sens)}
    h.close()
    del h
    torch.cuda.empty_cache()
    # sequential reference: every sample_every-th instance in a handle of its own
    tot_dofs, tot_t = 0, 0.0
    for w in wls[::sample_every]:
        g1 = BiotSlab([w], [w.log_k()])
        tuning.tune(g1, path=None)
        st = g1.zeros_state()
        march(g1, 1, 0.0, st, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        march(g1, nsteps, w.tau, st, 0)
        torch.cuda.synchronize()
        tot_t += time.perf_counter() - t0
        tot_dofs += nsteps * g1.slab_len
        g1.close()
    seq = tot_dofs / tot_t
    res["sequential_fp64"] = {"dofs_per_s": seq, "sample": f"instances 0,{sample_every},...: "
                              f"{len(wls[::sample_every])} of {len(wls)}, {nsteps} slabs each"}
    for name in ("fp64", "mixed", "fp32_preconditioned"):
        res[f"speedup_{name}_vs_sequential"] = res[name]["dofs_per_s"] / seq
    return res


def dominant_roofline(torch, h):
    """Roofline of the dominant kernel of the step.  3D: the elasticity operator
    y_u = tau A x_u on the fine level (every time level in one launch), bound by
    the FP64 matrix cores: 2 * 81^2 flops per cell and time level (dense element
    matrix-vector products).  2D: the slab operator apply, HBM-bound."""
    wl = h.wls[0]
    if wl.dim == 3:
        ms = time_launches(torch, h, lambda x, y: h.elasticity_apply(x, y), torch.float64, 50)
        flops = 2.0 * 81 * 81 * int(np.prod(wl.n)) * (wl.r + 1)
        ach = flops / (ms * 1e-3) / 1e12
        key = "bt::uapply3d_kernel<double>"
        return {"bound": "mfma", "achieved": ach, "peak": FP64_MATRIX_PEAK_TFS, "unit": "TFLOP/s",
                "frac": ach / FP64_MATRIX_PEAK_TFS, "traffic": measured_traffic(key), "kernel": key,
                "algorithmic_flops_per_launch": flops, "launch_us": ms * 1e3,
                # read x_u, write y_u: 3 (2n+1)^3 displacement DoFs per time level
                "hbm_algorithmic_bytes_per_launch": 2 * 8 * 3 * int(np.prod([2 * m + 1 for m in wl.n])) * (wl.r + 1)}
    ms = time_launches(torch, h, lambda x, y: h.apply(x, y), torch.float64, 200)
    ts, lp = {0: (16, "false"), 1: (8, "false"), 2: (8, "true")}[h.get_tuning()["apply_variant"][0]]
    key = f"bt::apply2d_kernel<double, 2, false, {ts}, {lp}>"
    return dict(hbm_roofline(ms, _apply_bytes(h, 8)), kernel=key, traffic=measured_traffic(key))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4",
                    help="c4 3D 48^3 dG(2) (default); c3 3D 32^3 dG(1); c2 2D 128x128 dG(1); c1 2D Terzaghi 8x8 "
                         "dG(0); with --kernel-only also c5 (64 uneven 2D instances)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the adjoint and batched objects")
    ap.add_argument("--kernel-only", choices=["apply", "elasticity"],
                    help="profiling target: autotune, then 50 FP64 and 50 FP32 launches of one operator "
                         "(apply: slab operator; elasticity: fine-level elasticity operator) and one 256 MiB copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "biotst runs on one GPU only: sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1801_04984_amd import BiotSlab, tuning

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.kernel_only:
        wls = W.c5_batch() if args.workload == "c5" else [W.ALL[args.workload]()]
        h = BiotSlab(wls, [w.log_k() for w in wls])
        tuning.tune(h, path=None)
        fn = (lambda x, y: h.apply(x, y)) if args.kernel_only == "apply" else (lambda x, y: h.elasticity_apply(x, y))
        ms64 = time_launches(torch, h, fn, torch.float64, 50)
        ms32 = time_launches(torch, h, fn, torch.float32, 50)
        x = torch.randn(1 << 26, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"workload": args.workload, "kernel": args.kernel_only, "launch_ms": [ms64, ms32],
                          "apply_bytes": [_apply_bytes(h, 8), _apply_bytes(h, 4)],
                          "tile_variant": h.get_tuning()["apply_variant"], "copy_bytes": 2 * x.numel() * 4}))
        return

    wl = W.ALL[args.workload]()
    theta = wl.log_k()
    # set-up cost, outside the timed region: the problem's creation (workspace carving,
    # element matrices, coarse inverses, power iterations) and the tile autotuner
    from paper_1801_04984_amd import native
    native.load_library()
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    h = BiotSlab([wl], [theta])
    torch.cuda.synchronize()
    ts1 = time.perf_counter()
    tune = tuning.tune(h, path=None)
    torch.cuda.synchronize()
    ts2 = time.perf_counter()
    slab_dofs = h.slab_len

    state = h.zeros_state()
    last64 = h.zeros_slab()
    before64 = h.zeros_state()
    march(h, args.warmup, 0.0, state, 0)
    torch.cuda.synchronize()
    t_start = args.warmup * wl.tau
    t_last = t_start + (args.steps - 1) * wl.tau
    t0 = time.perf_counter()
    infos = march(h, args.steps, t_start, state, 0, slabs_last=last64, state_before_last=before64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * slab_dofs / dt
    its = [i[0]["iterations"] for i in infos]
    err64, ref_res = slab_error(h, before64, t_last, last64)
    shape = "x".join(str(m) for m in wl.n)

    out = {
        "metric": METRIC, "value": value, "unit": "space-time DoF/s (slab solved to rel. residual 1e-13, FP64)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded log-normal permeability)",
        "config": {"workload": f"{wl.name}: {wl.dim}D {shape} cells, Q2/RT1/DG-Q1, dG({wl.r}), tau={wl.tau}, "
                               f"log-normal K sigma={wl.k_sigma} ell={wl.k_ell} seed={wl.k_seed}, ramp load",
                   "slab_dofs": slab_dofs, "parallelism": "single GPU"},
        "gmres_iterations_per_slab": {"mean": float(np.mean(its)), "min": int(min(its)), "max": int(max(its))},
        "last_slab_rel_l2_error": err64,
        "error_reference": f"the same slab solved in FP64 to the GMRES floor, then FP64 iterative refinement "
                           f"(reference relative residual {ref_res:.1e})",
        "apply_tile_variant": tune["apply_variant"],
        "setup_s": {"create": ts1 - ts0, "autotune": ts2 - ts1},
    }

    if not args.no_mixed:
        for key, prec in (("mixed", 1), ("fp32_preconditioned", 2)):
            st2 = h.zeros_state()
            last = h.zeros_slab()
            before = h.zeros_state()
            march(h, args.warmup, 0.0, st2, prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            inf2 = march(h, args.steps, t_start, st2, prec, slabs_last=last, state_before_last=before)
            torch.cuda.synchronize()
            dt2 = time.perf_counter() - t1
            out[key] = {"value": args.steps * slab_dofs / dt2, "ms_per_step": 1e3 * dt2 / args.steps,
                        "speedup_vs_fp64": dt / dt2,
                        "last_slab_rel_l2_error": slab_error(h, before, t_last, last)[0],
                        "last_slab_rel_l2_vs_fp64": field_rel(h, last, last64),
                        "end_state_rel_l2_vs_fp64": field_rel(h, st2, state),
                        "iterations_per_slab": float(np.mean([i[0]["iterations"] for i in inf2])),
                        "refinement_sweeps_per_slab": float(np.mean([i[0]["ir_sweeps"] for i in inf2]))}
            del last

    ms64 = time_launches(torch, h, lambda x, y: h.apply(x, y), torch.float64, 50)
    ms32 = time_launches(torch, h, lambda x, y: h.apply(x, y), torch.float32, 50)
    out["apply"] = {"fp64": dict(hbm_roofline(ms64, _apply_bytes(h, 8)), dof_applies_per_s=slab_dofs / (ms64 * 1e-3)),
                    "fp32": dict(hbm_roofline(ms32, _apply_bytes(h, 4)), dof_applies_per_s=slab_dofs / (ms32 * 1e-3))}
    out["roofline"] = dominant_roofline(torch, h)
    if not args.no_extra and wl.dim == 3:
        n_adj = min(args.steps, wl.nslabs)
        out["adjoint"] = {"fp64": adjoint_timing(torch, W, h, n_adj, 0),
                          "mixed": adjoint_timing(torch, W, h, n_adj, 1)}
    h.close()
    del h
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["batched"] = batched(torch, W, BiotSlab, tuning)
    if not args.no_cpu:
        n_cpu = {2: 32, 3: 5}[wl.dim]
        out["cpu_baseline"] = cpu_baseline(wl, n_cpu, 10)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
