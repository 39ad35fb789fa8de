"""Benchmark: solves/s of the background-field LS solver on one MI355X.

A step is one full solve of the hot path (layered-stack tables, background
source, outer reflection loop, GMRES on eq. (18) with the operator apply,
readouts) of the 128 x 128 x 64 contact-hole clip (256 nm, 8 holes, 20-40 nm,
60 nm absorber n = 0.95 + 0.031i on 40 Mo/Si pairs, TE, 6 deg) to a relative
residual of 1e-6, mixed precision (FP32 Arnoldi cycles, FP64 residual,
solution and reflection). Inputs are resident in HBM before timing starts.

Printed JSON line: the driver's contract plus operator applies/s, the FP64
solve rate, the TM solve, the field error of the mixed result against the
FP64 GPU solve, the roofline of the dominant apply kernel (live HIP-event
timing) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="skip the FP64 / TM / apply extras")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import ctypes as C
    import numpy as np
    import torch
    from paper_2606_25541_amd import api, clips, _lib

    dev = torch.device("cuda:0")
    prob = clips.config_problem("G3", pol=clips.TE)
    deps_np = clips.contact_holes(128, 128, 64, 256.0, 256.0, 8, seed=2001)
    deps = torch.from_numpy(deps_np).to(dev)
    N = prob.nx * prob.ny * prob.nz
    rtol = 1e-6
    plan = api.Plan(prob, rtol=rtol, precision="mixed", restart=args.restart, max_iters=20000, max_outer=200)
    em = torch.empty((3, prob.nz, prob.ny, prob.nx), dtype=torch.complex128, device=dev)
    orders = torch.empty((prob.ny, prob.nx, 3), dtype=torch.complex128, device=dev)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    log("bench: warmup", args.warmup)
    info = None
    for _ in range(args.warmup):
        _, _, info = plan.psfd_solve(deps, em, orders)
    torch.cuda.synchronize()
    log("bench: timed", args.steps, "steps")
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, _, info = plan.psfd_solve(deps, em, orders)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves_s = args.steps / dt
    log("bench: mixed", info)
    out = {
        "metric": "solves/s at 1e-6 rel. residual (mixed vs FP64) + operator applies/s + p99",
        "value": solves_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64+c128 (mixed)", "data": "synthetic",
        "config": {"workload": "contact-hole clip 128x128x64, 256 nm, 8 holes 20-40 nm, 60 nm absorber, "
                               "40 Mo/Si pairs, TE 6 deg, rtol 1e-6, mixed FP32/FP64",
                   "grid": [prob.nx, prob.ny, prob.nz], "restart": args.restart, "rtol": rtol,
                   "parallelism": "single GPU"},
        "mixed": {"iters": info["iters"], "outer_iters": info["outer_iters"], "cycles": info["cycles"],
                  "rel_residual": info["rel_residual"], "mono_residual": info["mono_residual"]},
    }
    em_mixed = em.clone()

    if not args.quick:
        # FP64 solve of the same clip
        plan64 = api.Plan(prob, rtol=rtol, precision="fp64", restart=args.restart, max_iters=20000, max_outer=200)
        em64 = torch.empty_like(em)
        plan64.psfd_solve(deps, em64, orders)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n64 = max(1, args.steps // 2)
        for _ in range(n64):
            _, _, i64 = plan64.psfd_solve(deps, em64, orders)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / n64
        log("bench: fp64", i64)
        # tight FP64 reference for the field error of both results
        planref = api.Plan(prob, rtol=1e-10, precision="fp64", restart=args.restart, max_iters=40000,
                           max_outer=400)
        emr = torch.empty_like(em)
        _, _, iref = planref.psfd_solve(deps, emr, orders)
        torch.cuda.synchronize()
        nr = torch.linalg.vector_norm(emr).item()
        out["fp64"] = {"solves_per_s": 1.0 / t64, "ms_per_solve": 1e3 * t64, "iters": i64["iters"],
                       "outer_iters": i64["outer_iters"], "mono_residual": i64["mono_residual"],
                       "field_err_vs_fp64_1e-10": torch.linalg.vector_norm(em64 - emr).item() / nr}
        out["mixed"]["field_err_vs_fp64_1e-10"] = torch.linalg.vector_norm(em_mixed - emr).item() / nr
        out["mixed_over_fp64"] = solves_s * t64
        # TM
        prob_tm = clips.config_problem("G3", pol=clips.TM)
        plantm = api.Plan(prob_tm, rtol=rtol, precision="mixed", restart=args.restart, max_iters=20000,
                          max_outer=200)
        plantm.psfd_solve(deps, em, orders)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, itm = plantm.psfd_solve(deps, em, orders)
        torch.cuda.synchronize()
        out["tm_mixed"] = {"ms_per_solve": 1e3 * (time.perf_counter() - t0), "iters": itm["iters"],
                           "outer_iters": itm["outer_iters"], "mono_residual": itm["mono_residual"]}

        # operator applies/s and per-stage roofline (live HIP events on the library's stream)
        L = _lib.lib()
        stream = torch.cuda.current_stream()
        x = torch.from_numpy(clips.random_complex((3, prob.nz, prob.ny, prob.nx), 7)).to(dev)
        res = {}
        for name, dt_, code, esz in (("fp32", torch.complex64, _lib.PSFD_C64, 8),
                                     ("fp64", torch.complex128, _lib.PSFD_C128, 16)):
            xx = x.to(dt_)
            dd = deps.to(dt_)
            y = torch.empty_like(xx)
            for _ in range(3):
                plan.psfd_apply(dd, xx, y)
            reps = 200
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                plan.psfd_apply(dd, xx, y)
            e1.record(stream)
            e1.synchronize()
            t_apply = e0.elapsed_time(e1) / reps * 1e-3
            # bytes per unit (voxel): stage 0 reads x, delta_eps, writes w; stage 1 reads and writes w;
            # stage 2 reads w, x, writes y
            per_vox = {0: 6 * esz + esz, 1: 6 * esz, 2: 9 * esz}
            stages = {}
            for st in (0, 1, 2):
                ms = C.c_float()
                _lib.check(L.psfd_bench_stage(plan._h, st, C.c_void_p(dd.data_ptr()), C.c_void_p(xx.data_ptr()),
                                              C.c_void_p(y.data_ptr()), code, 100, C.byref(ms),
                                              C.c_void_p(stream.cuda_stream)), "psfd_bench_stage")
                t = ms.value * 1e-3
                stages[st] = {"ms": ms.value, "bytes": per_vox[st] * N, "gbs": per_vox[st] * N / t / 1e9}
            b_apply = 22 * esz * N
            res[name] = {"applies_per_s": 1.0 / t_apply, "us_per_apply": 1e6 * t_apply,
                         "apply_bytes": b_apply, "apply_gbs": b_apply / t_apply / 1e9,
                         "apply_frac_hbm": b_apply / t_apply / 1e9 / HBM_PEAK_GBS, "stages": stages}
        out["apply"] = res
        st32 = res["fp32"]["stages"]
        dom = max(st32, key=lambda k: st32[k]["ms"])
        names = {0: "k_tile<float2,fwd,V*x> (transverse FFT forward)", 1: "k_pencil<float2> (z FFT, dyadic kernel)",
                 2: "k_tile<float2,inv,axpby> (transverse FFT inverse)"}
        out["roofline"] = {"bound": "hbm", "kernel": names[dom], "achieved": st32[dom]["gbs"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": st32[dom]["gbs"] / HBM_PEAK_GBS,
                           "traffic": None, "bytes_per_launch": st32[dom]["bytes"],
                           "us_per_launch": 1e3 * st32[dom]["ms"]}

    if not args.no_cpu:
        import oracle as O
        ncores = os.cpu_count() or 1
        O.set_workers(ncores)
        t0 = time.perf_counter()
        S = O.Setup(prob)
        _ = S.G
        t_setup = time.perf_counter() - t0
        xs = clips.random_complex((3, prob.nz, prob.ny, prob.nx), 3)
        V = O.potential(S, deps_np)
        e = O.background_field(S)
        rhs = O.conv_K(S, V[None] * e)
        k = 8
        t0 = time.perf_counter()
        O.gmres(lambda v: O.apply_A(S, deps_np, v), rhs, None, 1e-30, args.restart, k)
        t_it = (time.perf_counter() - t0) / k
        its = out["mixed"]["iters"]
        t_solve = t_setup + its * t_it
        out["cpu_baseline"] = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": ncores, "kind": "oracle",
                               "sample": f"{k} FP64 GMRES({args.restart}) iterations of the same solve "
                                         f"(scipy.fft workers={ncores}) plus table set-up, extrapolated to the "
                                         f"{its} iterations the GPU solve takes; {t_it:.2f} s/iteration",
                               "s_per_iteration": t_it}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
