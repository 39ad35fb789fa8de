"""Benchmark: solves/s of the background-field LS solver on one MI355X.

A step is one full solve of the hot path (layered-stack tables, background
source, monolithic coupling of the multilayer response, GMRES on eq. (18) with
the operator apply, readouts) of the 128 x 128 x 64 contact-hole clip (256 nm,
8 holes, 20-40 nm, 60 nm absorber n = 0.95 + 0.031i on 40 Mo/Si pairs, TE,
6 deg) to a relative residual of 1e-6, mixed precision (FP32 Arnoldi cycles,
FP64 residual, solution and reflection). Inputs are resident in HBM before
timing starts.

Printed JSON line: the solve rate, plus
  fp64 / tm_mixed   the plain FP64 solve and the TM solve of the same clip,
                    field errors against a tight FP64 solve;
  apply             operator applies/s and per-stage bandwidth (HIP events on
                    the library's stream), with the roofline of the dominant
                    kernel and its measured HBM traffic where the stored
                    counter summary matches the current kernel sources;
  batched           64 instances (pupil angles x {64x64x32, 128x128x64}
                    Manhattan clips) in lock-step batched solves, against the
                    same instances solved one by one;
  serving           Poisson arrivals over {64x64x32, 128x128x64, 256x256x64}
                    at 0.7 of the saturated rate (--serve-qps: several
                    rates): p50 / p99 latency, solves/s;
  isolated          the isolated-domain operator (spherical window, padding by
                    2 on all axes) on the same 128x128x64 contact holes taken
                    as a free-standing 256x256x60 nm scatterer in vacuum:
                    table precompute time, applies/s FP32 / FP64, per-pass
                    bandwidth and the roofline of its dominant kernel;
  adjoint           forward + adjoint gradient on a 256x256x64 smooth clip;
  cpu_baseline      the CPU oracle on a bounded sample of the headline solve.

--only SECTION runs one section (profiling); --quick runs the headline only;
--oracle-study times the CPU oracle on every workload (host only, no GPU) and
prints its own JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SECTIONS = ("solve", "fp64", "apply", "isolated", "batched", "serving", "adjoint", "precond", "layers", "cpu")
# sources that decide the code of the measured kernels (hashed into the counter summary)
KERNEL_SOURCES = ("common.hpp", "layout.hpp", "kernels.hpp", "fft_lds.hpp", "k_apply.hip", "krylov.hpp",
                  "givens.hpp", "k_krylov.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "apply_G3_fp32_hbm_traffic.md")
ISO_SOURCES = ("common.hpp", "fft_lds.hpp", "k_iso.hip")
ISO_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "isolated_apply_G3_hbm_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2606_25541_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(key: str, summary: str = TRAFFIC_SUMMARY, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel (key: "stage 0|1|2", "projections", "update") from the
    committed counter summary.

    None when the summary is missing or was taken on other kernel sources.
    """
    try:
        txt = open(summary).read()
    except OSError:
        return None
    m = re.search(r"kernel source hash: `([0-9a-f]+)`", txt)
    if not m or m.group(1) != kernel_source_hash(sources):
        return None
    m = re.search(r"traffic %s: (\d+) bytes" % re.escape(key), txt)
    return int(m.group(1)) if m else None


def timed(fn, n):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = None
    for _ in range(n):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n, r


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden_error(torch, case, em, od, p):
    """Field error (relative L2 over the stored lattice of E_mask samples) and largest order
    error (relative to the largest stored order) against the stored FP64 oracle solution of
    `case` (written by tests/golden/make_golden.py); None when the file is absent."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, case + ".npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    zi, yi, xi = (torch.from_numpy(z[k]).to(em.device) for k in ("zi", "yi", "xi"))
    smp = em.index_select(1, zi).index_select(2, yi).index_select(3, xi).cpu().numpy()
    ref = z["emask_sample"]
    mi = torch.from_numpy(np.arange(-8, 9)).to(em.device)
    osel = od.index_select(0, mi % p.ny).index_select(1, mi % p.nx).cpu().numpy()
    return {"field_err_vs_oracle": float(np.linalg.norm(smp - ref) / np.linalg.norm(ref)),
            "order_err_vs_oracle": float(np.abs(osel - z["orders"]).max() / np.abs(z["orders"]).max())}


def sec_solve(ctx, args, out):
    api, torch = ctx["api"], ctx["torch"]
    prob, deps = ctx["prob"], ctx["deps"]
    plan = api.Plan(prob, rtol=args.rtol, precision="mixed", restart=args.restart, max_iters=20000, max_outer=200)
    em = torch.empty((3, prob.nz, prob.ny, prob.nx), dtype=torch.complex128, device=ctx["dev"])
    orders = torch.empty((prob.ny, prob.nx, 3), dtype=torch.complex128, device=ctx["dev"])
    log("bench: warmup", args.warmup)
    for _ in range(args.warmup):
        plan.psfd_solve(deps, em, orders)
    log("bench: timed", args.steps, "steps")
    dt, (_, _, info) = timed(lambda: plan.psfd_solve(deps, em, orders), args.steps)
    log("bench: mixed", info)
    out.update({
        "value": 1.0 / dt, "ms_per_step": 1e3 * dt,
        "mixed": {"rtol": args.rtol, "iters": info["iters"], "outer_iters": info["outer_iters"],
                  "cycles": info["cycles"], "rel_residual": info["rel_residual"],
                  "mono_residual": info["mono_residual"],
                  **(golden_error(torch, "contact_holes_128x128x64_te", em, orders, prob) or {})},
    })
    ctx["plan"], ctx["em_mixed"], ctx["t_mixed"] = plan, em, dt


def sec_fp64(ctx, args, out):
    api, torch = ctx["api"], ctx["torch"]
    prob, deps = ctx["prob"], ctx["deps"]
    em = torch.empty((3, prob.nz, prob.ny, prob.nx), dtype=torch.complex128, device=ctx["dev"])
    orders = torch.empty((prob.ny, prob.nx, 3), dtype=torch.complex128, device=ctx["dev"])
    n = max(1, args.steps // 2)

    def run(prec, rtol, p=prob, case="contact_holes_128x128x64_te"):
        pl = api.Plan(p, rtol=rtol, precision=prec, restart=args.restart, max_iters=20000, max_outer=200)
        pl.psfd_solve(deps, em, orders)
        t, (_, _, inf) = timed(lambda: pl.psfd_solve(deps, em, orders), n)
        r = {"rtol": rtol, "solves_per_s": 1.0 / t, "ms_per_solve": 1e3 * t, "iters": inf["iters"],
             "rel_residual": inf["rel_residual"], **(golden_error(torch, case, em, orders, p) or {})}
        log("bench:", prec, rtol, r)
        return r

    # the plain FP64 solve at the headline tolerance and at 1e-6; the mixed solve at 1e-6
    out["fp64"] = run("fp64", args.rtol)
    out["fp64_rtol_1e-6"] = run("fp64", 1e-6)
    out["mixed_rtol_1e-6"] = run("mixed", 1e-6)
    if "t_mixed" in ctx:
        out["mixed_over_fp64"] = out["fp64"]["ms_per_solve"] * 1e-3 / ctx["t_mixed"]
    # TM, mixed at the headline tolerance
    prob_tm = ctx["clips"].config_problem("G3", pol=ctx["clips"].TM)
    out["tm_mixed"] = run("mixed", args.rtol, prob_tm, "contact_holes_128x128x64_tm")
    # workload 1: 64 nm line/space, 32x32x32, FP64 GMRES(30) to 1e-8
    clips = ctx["clips"]
    p1 = clips.config_problem("G1")
    d1 = torch.from_numpy(clips.line_space(p1.nx, p1.ny, p1.nz, p1.lx_nm, p1.ly_nm, 16.0, 48.0)).to(ctx["dev"])
    em1 = torch.empty((3, p1.nz, p1.ny, p1.nx), dtype=torch.complex128, device=ctx["dev"])
    or1 = torch.empty((p1.ny, p1.nx, 3), dtype=torch.complex128, device=ctx["dev"])
    plan1 = api.Plan(p1, rtol=1e-8, outer_rtol=1e-8, precision="fp64", restart=30, max_iters=20000)
    plan1.psfd_solve(d1, em1, or1)
    t1, (_, _, i1) = timed(lambda: plan1.psfd_solve(d1, em1, or1), 5)
    x1 = torch.from_numpy(clips.random_complex((3, p1.nz, p1.ny, p1.nx), 1)).to(ctx["dev"])
    y1 = torch.empty_like(x1)
    plan1.psfd_apply(d1, x1, y1)
    ta1, _ = timed(lambda: plan1.psfd_apply(d1, x1, y1), 200)
    out["line_space_G1_fp64"] = {"ms_per_solve": 1e3 * t1, "iters": i1["iters"], "us_per_apply": 1e6 * ta1}
    log("bench: line/space 32x32x32", out["line_space_G1_fp64"])


def sec_apply(ctx, args, out):
    """Operator applies/s and per-stage bandwidth, timed with HIP events on the launch stream."""
    import ctypes as C
    api, torch, clips, _lib = ctx["api"], ctx["torch"], ctx["clips"], ctx["_lib"]
    prob, deps, dev = ctx["prob"], ctx["deps"], ctx["dev"]
    N = prob.nx * prob.ny * prob.nz
    plan = ctx.get("plan") or api.Plan(prob, rtol=1e-6, precision="mixed", restart=args.restart)
    L = _lib.lib()
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(clips.random_complex((3, prob.nz, prob.ny, prob.nx), 7)).to(dev)
    reps = 20 if args.only == "apply" else 200
    res = {}
    for name, dt_, code, esz in (("fp32", torch.complex64, _lib.PSFD_C64, 8),
                                 ("fp64", torch.complex128, _lib.PSFD_C128, 16)):
        xx, dd = x.to(dt_), deps.to(dt_)
        y = torch.empty_like(xx)
        for _ in range(3):
            plan.psfd_apply(dd, xx, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.psfd_apply(dd, xx, y)
        e1.record(stream)
        e1.synchronize()
        t_apply = e0.elapsed_time(e1) / reps * 1e-3
        # algorithmic bytes per voxel (esz = bytes per complex value): stage 0 reads x (3 esz) and
        # delta_eps (esz), writes w (3 esz); stage 1 reads and writes w; stage 2 reads w and x, writes y
        per_vox = {0: 7 * esz, 1: 6 * esz, 2: 9 * esz}

        def time_stages():
            st_ = {}
            for st in (0, 1, 2):
                ms = C.c_float()
                _lib.check(L.psfd_bench_stage(plan._h, st, C.c_void_p(dd.data_ptr()), C.c_void_p(xx.data_ptr()),
                                              C.c_void_p(y.data_ptr()), code, reps, C.byref(ms),
                                              C.c_void_p(stream.cuda_stream)), "psfd_bench_stage")
                t = ms.value * 1e-3
                st_[st] = {"us": 1e3 * ms.value, "bytes": per_vox[st] * N, "gbs": per_vox[st] * N / t / 1e9}
            return st_
        stages = time_stages()
        b_apply = 22 * esz * N
        res[name] = {"applies_per_s": 1.0 / t_apply, "us_per_apply": 1e6 * t_apply, "apply_bytes": b_apply,
                     "apply_gbs": b_apply / t_apply / 1e9, "apply_frac_hbm": b_apply / t_apply / 1e9 / HBM_PEAK_GBS,
                     "stages": stages}
        if name == "fp32" and prob.nx == prob.ny == 128:
            # the operator apply runs the quarter-plane kernels (four blocks per 128 x 128 plane, the
            # pencil on the quarter layout); the Arnoldi steps of a solve run the one-block-per-plane
            # kernels with their fused Gram-Schmidt work, whose plain forms are timed here
            os.environ["PSFD_QUARTER_PLANES"] = "0"
            try:
                res[name]["stages_full_planes"] = time_stages()
            finally:
                os.environ.pop("PSFD_QUARTER_PLANES", None)
    out["apply"] = res
    # kernels of the Arnoldi steps of one restart cycle (columns j = 0 .. m-1) on FP32 basis vectors,
    # through psfd_bench_gram_schmidt: the projections read v_0..v_j and w, (j + 2) 3N complex64; the
    # update also writes w, (j + 3) 3N; the step's inverse transverse kernel reads the workspace and
    # writes w, 2 3N, and where it also forms the projections (FP32 128 x 128 planes) reads v_0..v_j
    # as well, (j + 3) 3N, and no separate projection pass runs
    # The forward stage of step j + 1 (pass 3) reads the slot, the contrast and writes the workspace,
    # 7N; where it also does the update of column j (FP32 128 x 128 planes, lock-step solves) it reads
    # v_0..v_j too and writes the slot back, (j + 3) 3N + 7N
    m = args.restart
    sq128 = prob.nx == prob.ny == 128
    fused = sq128 and 3 * prob.nz <= 256 and os.environ.get("PSFD_FUSE_DOTS", "1") != "0"
    fused_upd = sq128 and os.environ.get("PSFD_FUSE_UPDATE", "1") != "0"
    x32 = x.to(torch.complex64)
    gs = {}
    for pname, pas, nvec in (("projections", 0, lambda j: j + 2), ("update", 1, lambda j: j + 3),
                             ("stage 2 step", 2, lambda j: j + 3 if fused else 2),
                             ("stage 0 step", 3, lambda j: (j + 3 if fused_upd else 0) + 7 / 3)):
        us, byt = [], []
        for j in range(m):
            ms = C.c_float()
            _lib.check(L.psfd_bench_gram_schmidt(plan._h, pas, j, C.c_void_p(x32.data_ptr()), _lib.PSFD_C64,
                                                 max(5, reps // 4), C.byref(ms), C.c_void_p(stream.cuda_stream)),
                       "psfd_bench_gram_schmidt")
            us.append(1e3 * ms.value)
            byt.append(nvec(j) * 3 * N * 8)
        gs[pname] = {"us_per_column": us, "us_mean": sum(us) / m, "bytes_mean": sum(byt) / m,
                     "gbs": sum(byt) / (sum(us) * 1e-6) / 1e9}
    gs["projections_in_stage_2"] = fused
    gs["update_in_stage_0"] = fused_upd
    out["gram_schmidt_fp32"] = gs
    # the dominant kernel of an Arnoldi step (largest mean time per step over a cycle): the forward
    # stage (plain at step 0; with the previous column's update at steps 1..m-1 where fused), the
    # pencil, the inverse stage (with the projections where fused) and the separate passes
    st32 = res["fp32"].get("stages_full_planes", res["fp32"]["stages"])
    cand = {"stage 1": ("k_pencil<float2,7,16> (z FFT, dyadic kernel, stack response)", st32[1]["us"],
                        st32[1]["bytes"])}
    if fused_upd:
        g0 = gs["stage 0 step"]
        us0 = [st32[0]["us"]] + g0["us_per_column"][:m - 1]
        by0 = [st32[0]["bytes"]] + [(j + 3) * 3 * N * 8 + 7 * N * 8 for j in range(m - 1)]
        cand["stage 0 + update"] = (
            "k_plane<float2,fwd,update+V*x> (Gram-Schmidt update of the previous column + transverse FFT "
            "forward; plain at step 0; mean over the steps of a cycle)", sum(us0) / m, sum(by0) / m)
        # the last column takes no update pass: its Givens step works from the projections
    else:
        cand["stage 0"] = ("k_plane<float2,fwd,V*x> (transverse FFT forward, 128x128 planes)", st32[0]["us"],
                           st32[0]["bytes"])
        cand["update"] = ("k_update<float2> (Gram-Schmidt update, mean over j = 0..m-1)", gs["update"]["us_mean"],
                          gs["update"]["bytes_mean"])
    if fused:
        cand["stage 2 + projections"] = (
            "k_plane<float2,inv,dots> (transverse FFT inverse + Gram-Schmidt projections, mean over j = 0..m-1)",
            gs["stage 2 step"]["us_mean"], gs["stage 2 step"]["bytes_mean"])
    else:
        cand["stage 2"] = ("k_plane<float2,inv> (transverse FFT inverse)", gs["stage 2 step"]["us_mean"],
                           gs["stage 2 step"]["bytes_mean"])
        cand["projections"] = ("k_dots<float2> (Gram-Schmidt projections, mean over j = 0..m-1)",
                               gs["projections"]["us_mean"], gs["projections"]["bytes_mean"])
    dom = max(cand, key=lambda k: cand[k][1])
    name, us_d, bytes_d = cand[dom]
    gbs = bytes_d / (us_d * 1e-6) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": stored_traffic(dom),
                       "bytes_per_launch": bytes_d, "us_per_launch": us_d,
                       "kernel_source_hash": kernel_source_hash(),
                       "per_step_us": {k: round(v[1], 2) for k, v in cand.items()}}
    # the device's own copy of 256 MiB (read + write, best of five): the practical streaming
    # ceiling, against which the fraction is also given
    ca = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(5):
        e0.record()
        cb.copy_(ca)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    copy_gbs = 2 * ca.numel() * 4 / (best * 1e-3) / 1e9
    out["roofline"]["copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = gbs / copy_gbs
    del ca, cb
    if args.only == "apply":
        # plain copy of known size: the scale of the FETCH_SIZE / WRITE_SIZE counters
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_bytes"] = a.numel() * 4


def sec_isolated(ctx, args, out):
    """Isolated-domain apply: the headline contact holes as a free-standing absorber block
    (256 x 256 x 60 nm, vacuum, R = box diagonal); passes timed with HIP events on the launch stream."""
    api, torch, clips = ctx["api"], ctx["torch"], ctx["clips"]
    prob, dev = ctx["prob"], ctx["dev"]
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    spacing = (prob.t_nm / nz, prob.ly_nm / ny, prob.lx_nm / nx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = api.IsoPlan(nx, ny, nz, spacing, prob.wavelength_nm, 1.0)
    t_pre = time.perf_counter() - t0
    _, over, R = plan.table()
    N = nx * ny * nz
    x = torch.from_numpy(clips.random_complex((3, nz, ny, nx), 7)).to(dev)
    reps = 20 if args.only == "isolated" else 100
    # algorithmic bytes per voxel in complex values (esz bytes each): x rows read x (3) and
    # delta_eps (1), write half the padded rows (6); y columns read 6, write 12; the z pencils read
    # and write 12 and read the 6-entry table of the padded grid for kz = 0 .. nz (the table is even
    # or odd in kz: 24 (nz + 1) / nz); inverse y columns read 12, write 6; inverse x rows read 6 and
    # x (3), write y (3)
    per_vox = {0: 10, 1: 18, 2: 24 + 24 * (nz + 1) / nz, 3: 18, 4: 12}
    names = {0: "k_iso_lines<fwd, x rows * V>", 1: "k_iso_lines<fwd, y columns>",
             2: "k_iso_zmul (z FFT, 3x3 table product, inverse z FFT)", 3: "k_iso_lines<inv, y columns>",
             4: "k_iso_lines<inv, x rows, y = x - w>"}
    res = {"grid": [nx, ny, nz], "spacing_nm": list(spacing), "radius_nm": R, "oversampling_zyx": list(over),
           "precompute_ms": 1e3 * t_pre}
    for name, dt_, esz in (("fp32", torch.complex64, 8), ("fp64", torch.complex128, 16)):
        xx, dd = x.to(dt_), ctx["deps"].to(dt_)
        y = torch.empty_like(xx)
        ms = plan.bench_stage(-1, dd, xx, y, reps)
        stages = {}
        for st in range(5):
            t = plan.bench_stage(st, dd, xx, y, reps) * 1e-3
            stages[st] = {"kernel": names[st], "us": 1e6 * t, "bytes": int(per_vox[st] * esz * N),
                          "gbs": per_vox[st] * esz * N / t / 1e9}
        b = int(sum(per_vox.values()) * esz * N)
        res[name] = {"applies_per_s": 1e3 / ms, "us_per_apply": 1e3 * ms, "apply_bytes": b,
                     "apply_gbs": b / (ms * 1e-3) / 1e9, "stages": stages}
    st32 = res["fp32"]["stages"]
    dom = max(st32, key=lambda k: st32[k]["us"])
    gbs = st32[dom]["gbs"]
    res["roofline"] = {"bound": "hbm", "kernel": names[dom] + " FP32", "achieved": gbs, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                       "traffic": stored_traffic("z pencil fp32", ISO_TRAFFIC_SUMMARY, ISO_SOURCES) if dom == 2 else None,
                       "bytes_per_launch": st32[dom]["bytes"], "us_per_launch": st32[dom]["us"],
                       "kernel_source_hash": kernel_source_hash(ISO_SOURCES)}
    res["vs_periodic_apply_fp32"] = (res["fp32"]["us_per_apply"] / out["apply"]["fp32"]["us_per_apply"]
                                     if "apply" in out else None)
    # GMRES(20) to 1e-6 (FP64, and mixed: FP32 cycles with FP64 restarts) with b the normally
    # incident plane wave polarised along y
    k0 = 2 * math.pi / prob.wavelength_nm
    zz = torch.arange(nz, dtype=torch.float64, device=dev) * spacing[0]
    b = torch.zeros((3, nz, ny, nx), dtype=torch.complex128, device=dev)
    b[1] = torch.exp(1j * k0 * zz)[:, None, None].expand(nz, ny, nx)
    u = torch.empty_like(b)
    for prec in ("fp64", "mixed"):
        plan.solve(ctx["deps"], b, rtol=1e-6, restart=20, out=u, precision=prec)
        ts, (_, inf) = timed(lambda: plan.solve(ctx["deps"], b, rtol=1e-6, restart=20, out=u, precision=prec), 2)
        res["solve_" + prec] = {"ms_per_solve": 1e3 * ts, "iters": inf["iters"], "cycles": inf["cycles"],
                                "rel_residual": inf["rel_residual"], "rhs": "plane wave along z, E along y",
                                "restart": 20, "rtol": 1e-6}
    out["isolated"] = res
    log("bench: isolated", res)
    if args.only == "isolated":
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b2 = torch.empty_like(a)
        for _ in range(5):
            b2.copy_(a)
        torch.cuda.synchronize()
        out["copy_bytes"] = a.numel() * 4


def sec_batched(ctx, args, out):
    """64 instances over pupil angles and two grids: batched lock-step solves vs one by one."""
    import numpy as np
    api, torch, clips, dev = ctx["api"], ctx["torch"], ctx["clips"], ctx["dev"]
    items = clips.batched_set()
    opts = dict(rtol=args.rtol, precision="mixed", restart=args.restart, max_iters=20000)
    groups = {}
    for g, p, d in items:
        groups.setdefault(g, []).append((p, torch.from_numpy(d).to(dev)))
    # warm-up of both shapes
    for g, lst in groups.items():
        api.psfd_solve_batch([lst[0][0]], [lst[0][1]], **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = {}
    for g, lst in groups.items():
        _, _, infos = api.psfd_solve_batch([p for p, _ in lst], [d for _, d in lst], **opts)
        iters[g] = [i["iters"] for i in infos]
        assert all(i["status"] == 0 for i in infos), infos
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    # the same batches again: the workspaces kept from the first calls are reused
    t0 = time.perf_counter()
    res = {}
    for g, lst in groups.items():
        res[g] = api.psfd_solve_batch([p for p, _ in lst], [d for _, d in lst], **opts)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    # field error of the first instance of each grid (batched instances 0 and 1) against the oracle
    gerr = {}
    for i in range(2):
        g, p, _ = items[i]
        e = golden_error(torch, "batched_%d_%dx%dx%d" % (i, p.nx, p.ny, p.nz), res[g][0][0], res[g][1][0], p)
        if e:
            gerr["instance_%d_%s" % (i, g)] = e
    api.psfd_release_cached_workspaces()
    # the same instances one by one (plans built and their workspaces allocated before timing)
    plans = [(api.Plan(p, **opts), d) for lst in groups.values() for p, d in lst]
    for pl, d in plans:
        pl.psfd_solve(d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, d in plans:
        pl.psfd_solve(d)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del plans
    # the first four instances alone (the sample the CPU oracle is timed on)
    sample_ms = []
    for g, p, d in items[:4]:
        pl = api.Plan(p, **opts)
        dd = torch.from_numpy(d).to(dev)
        pl.psfd_solve(dd)
        t, r = timed(lambda: pl.psfd_solve(dd), 1)
        sample_ms.append({"grid": g, "ms": 1e3 * t, "iters": r[2]["iters"]})
        del pl
    out["batched"] = {"instances": len(items), "per_grid": {g: len(v) for g, v in groups.items()},
                      "rtol": args.rtol, "vs_oracle": gerr,
                      "solves_per_s": len(items) / t_batch, "sequential_solves_per_s": len(items) / t_seq,
                      "first_call_solves_per_s": len(items) / t_first,
                      "speedup_vs_sequential": t_seq / t_batch,
                      "iters_mean": {g: float(np.mean(v)) for g, v in iters.items()},
                      "iters_max": {g: int(np.max(v)) for g, v in iters.items()},
                      "first4_alone_ms": sample_ms}
    log("bench: batched", out["batched"])


def sec_serving(ctx, args, out):
    """Poisson arrivals over three grids at fractions of the saturated rate; p50/p99 latency."""
    import numpy as np
    api, torch, clips, dev = ctx["api"], ctx["torch"], ctx["clips"], ctx["dev"]
    grids = ("G2", "G3", "G4")
    opts = dict(rtol=args.rtol, precision="mixed", restart=args.restart, max_iters=20000)
    rng = np.random.default_rng(4000)
    pool = clips.serving_pool()
    pool = [(g, p, torch.from_numpy(d).to(dev)) for g, p, d in pool]

    def outputs(p):
        return (torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev),
                torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev))

    budget = int(args.serve_budget_gib * (1 << 30))
    unbounded = sum(8 * api.Plan(p, **opts).footprint() for _, p, _ in pool[:3])
    srv = api.Server(hbm_budget=budget, max_slots=8, **opts)

    def drain(tickets, deadline):
        lat = {}
        while len(lat) < len(tickets) and time.perf_counter() < deadline:
            for t in tickets:
                if t not in lat:
                    done, info, l = srv.poll(t)
                    if done:
                        assert info["status"] == 0, info
                        lat[t] = (l, time.perf_counter())
            time.sleep(0.0005)
        return lat

    # warm-up: one request per grid allocates the slot groups
    warm = [srv.submit(p, d, *outputs(p)) for g, p, d in pool[:3]]
    drain(warm, time.perf_counter() + 120)
    # saturated rate: a burst of requests all at once
    burst = [pool[int(rng.integers(len(pool)))] for _ in range(args.serve_burst)]
    bufs = [outputs(p) for _, p, _ in burst]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts = [srv.submit(p, d, *b) for (_, p, d), b in zip(burst, bufs)]
    lat = drain(ts, t0 + 300)
    t_sat = max(v[1] for v in lat.values()) - t0
    sat = len(ts) / t_sat
    log("bench: serving saturated %.2f solves/s" % sat)
    def stream(frac, nreq, seed):
        """Poisson arrivals at frac * S: latency percentiles and the completed rate.

        Output buffers are recycled once their request has completed, so a
        long stream holds only the outputs of the requests in flight.
        """
        r = np.random.default_rng(seed)
        qps = frac * sat
        reqs = [pool[int(r.integers(len(pool)))] for _ in range(nreq)]
        gaps = r.exponential(1.0 / qps, size=len(reqs))
        free = {g: [] for g in grids}
        for g, p, _ in pool[:3]:
            free[g] = [outputs(p) for _ in range(8)]
        flight, lat = {}, {}

        def collect():
            for t in list(flight):
                done, info, l = srv.poll(t)
                if done:
                    assert info["status"] == 0, info
                    g, b = flight.pop(t)
                    free[g].append(b)
                    lat[t] = (l, time.perf_counter())

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_next = t0
        tickets, kinds = [], []
        for i, ((g, p, d), gap) in enumerate(zip(reqs, gaps)):
            t_next += gap
            while time.perf_counter() < t_next:
                collect()
                time.sleep(0.0002)
            b = free[g].pop() if free[g] else outputs(p)
            t = srv.submit(p, d, *b)
            flight[t] = (g, b)
            tickets.append(t)
            kinds.append(g)
            if (i + 1) % 200 == 0:
                log("bench: serving %.1f S, %d submitted, %d in flight" % (frac, i + 1, len(flight)))
        deadline = time.perf_counter() + 600
        while flight and time.perf_counter() < deadline:
            collect()
            time.sleep(0.0005)
        assert not flight, "requests still running after the drain limit"
        t_end = max(v[1] for v in lat.values())
        ls = np.array([lat[t][0] for t in tickets])
        per = {g: np.array([lat[t][0] for t, k in zip(tickets, kinds) if k == g]) for g in grids}
        res = {"qps_frac": frac, "qps": qps, "requests": len(tickets),
               "solves_per_s": len(tickets) / (t_end - t0),
               "p50_ms": 1e3 * float(np.percentile(ls, 50)), "p99_ms": 1e3 * float(np.percentile(ls, 99)),
               "per_grid_p50_ms": {g: 1e3 * float(np.percentile(v, 50)) for g, v in per.items() if len(v)},
               "per_grid_p99_ms": {g: 1e3 * float(np.percentile(v, 99)) for g, v in per.items() if len(v)}}
        log("bench: serving stream", res)
        return res

    fracs = [float(f) for f in args.serve_qps.split(",")]
    runs = [stream(f, args.serve_requests, 4100 + i) for i, f in enumerate(fracs)]
    # served results in the mix against the oracle: the first three pool requests (one per grid)
    # submitted together with a burst of others
    mix = [pool[int(rng.integers(len(pool)))] for _ in range(12)]
    chk = [(g, p, d, outputs(p)) for g, p, d in pool[:3]]
    tk = [srv.submit(p, d, *b) for g, p, d, b in chk] + [srv.submit(p, d, *outputs(p)) for _, p, d in mix]
    drain(tk, time.perf_counter() + 300)
    verr = {}
    for i, (g, p, d, (e, o)) in enumerate(chk):
        r = golden_error(torch, "serving_pool_%d_%dx%dx%d" % (i, p.nx, p.ny, p.nz), e, o, p)
        if r:
            verr["request_%d_%s" % (i, g)] = r
    srv.close()
    main = min(runs, key=lambda x: abs(x["qps_frac"] - 0.7))
    out["serving"] = {"saturated_solves_per_s": sat, "hbm_budget_bytes": budget,
                      "groups_at_max_slots_bytes": unbounded, "rtol": args.rtol, "vs_oracle": verr, **main}
    if len(runs) > 1:
        out["serving"]["sweep"] = runs
    # the plain FP64 GPU solve of one request per grid, for comparison
    fp64 = {}
    for g, p, d in pool[:3]:
        pl = api.Plan(p, rtol=args.rtol, precision="fp64", restart=args.restart, max_iters=20000)
        pl.psfd_solve(d)
        t, _ = timed(lambda: pl.psfd_solve(d), 1)
        fp64[g] = 1e3 * t
        del pl
    out["serving"]["fp64_single_solve_ms"] = fp64
    # the first four requests of the pool alone, mixed (the sample the CPU oracle is timed on)
    alone = []
    for g, p, d in pool[:4]:
        pl = api.Plan(p, **opts)
        pl.psfd_solve(d)
        t, r = timed(lambda: pl.psfd_solve(d), 1)
        alone.append({"grid": g, "ms": 1e3 * t, "iters": r[2]["iters"]})
        del pl
    out["serving"]["first4_alone_ms"] = alone
    log("bench: serving", out["serving"])


def sec_adjoint(ctx, args, out):
    """Forward + adjoint gradient of the 0 and +-1 order intensities on a 256x256x64 smooth clip.

    The mixed-precision forward solve keeps the total field; the adjoint solve takes the
    cotangent 2 a of the selected orders (the gradient of sum ||a_q||^2). The gradient is
    checked by central differences of FP64 solves (rtol 1e-12, step 1e-2 in delta_eps) on
    16 seeded voxels, real and imaginary parts."""
    import numpy as np
    api, torch, clips, dev = ctx["api"], ctx["torch"], ctx["clips"], ctx["dev"]
    p = clips.config_problem("G4")
    de, _ = clips.smooth_density_eps(p.nx, p.ny, p.nz, p.lx_nm, p.ly_nm, p.t_nm, seed=5001)
    d = torch.from_numpy(de).to(dev)
    sel = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    idx = torch.tensor([(n % p.ny) * p.nx + (m % p.nx) for (m, n) in sel], device=dev)
    plan = api.Plan(p, rtol=1e-6, precision="mixed", restart=args.restart, max_iters=20000)
    u = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)

    def fwd_adj():
        _, od, fi = plan.psfd_solve(d, u=u)
        G = torch.zeros_like(od)
        G.view(-1, 3)[idx] = 2.0 * od.view(-1, 3)[idx]
        g, ai = plan.psfd_solve_adjoint(d, u, G)
        J = float((od.view(-1, 3)[idx].abs() ** 2).sum().item())
        return g, J, fi, ai

    fwd_adj()
    t, (g, J, fi, ai) = timed(fwd_adj, 1)
    res = {"grid": [p.nx, p.ny, p.nz], "ms_forward_plus_adjoint": 1e3 * t, "J": J,
           "forward_iters": fi["iters"], "adjoint_iters": ai["iters"],
           "grad_finite": bool(torch.isfinite(torch.view_as_real(g)).all().item())}
    if args.adjoint_fd > 0:
        g = g.cpu().numpy()
        plan64 = api.Plan(p, rtol=1e-12, precision="fp64", restart=30, max_iters=40000)
        em = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        od = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)

        def Jof(x):
            plan64.psfd_solve(x, em, od)
            return float((od.view(-1, 3)[idx].abs() ** 2).sum().item())

        rng = np.random.default_rng(5002)
        h = 1e-2
        errs, t0 = [], time.perf_counter()
        for v in range(args.adjoint_fd):
            k, j, i = int(rng.integers(0, p.nz)), int(rng.integers(0, p.ny)), int(rng.integers(0, p.nx))
            for part in (1.0, 1j):
                x = d.clone()
                x[k, j, i] += h * part
                jp = Jof(x)
                x[k, j, i] -= 2 * h * part
                jm = Jof(x)
                fd = (jp - jm) / (2 * h)
                an = g[k, j, i].real if part == 1.0 else g[k, j, i].imag
                errs.append(abs(fd - an) / max(abs(fd), 1e-300))
            log("bench: adjoint fd voxel", v, "max rel err so far %.2e" % max(errs))
        res["fd_check"] = {"voxels": args.adjoint_fd, "parts": "re and im", "step": h,
                           "fd_solver": "FP64 GMRES(30), rtol 1e-12", "max_rel_err": max(errs),
                           "median_rel_err": float(np.median(errs)), "seconds": time.perf_counter() - t0}
    out["adjoint"] = res
    log("bench: adjoint", out["adjoint"])


def _diff_layout(nz, pe, npml):
    """zc0 of an absorber of nz planes centred in an extended grid of pe planes."""
    return (pe - nz) // 2


def sec_precond(ctx, args, out):
    """The preconditioner study (the Table of Sec. 3) on synthetic clips: GMRES steps and
    wall time of the differential PSFD solve with no preconditioner and with spectral
    damping D(k) = min(1, k_bg^2 / |k|^2), against the Green's-function (Lippmann-Schwinger)
    solve of the same background-field problem (outer coupling, as in the paper, and
    monolithic), all to rtol 1e-4, GMRES(30), mixed precision. Clips: 32x32x16 Manhattan
    (64 nm, 30 nm absorber, 40 Mo/Si pairs, TE 6 deg), extended z grid of 64 planes with
    a 30 nm PML (16 planes) at each end; differential solves capped at
    --precond-max-iters steps (a capped solve counts as not converged)."""
    import numpy as np
    api, torch, clips, dev = ctx["api"], ctx["torch"], ctx["clips"], ctx["dev"]
    nclips = args.precond_clips
    rows = {"none": [], "damping": [], "ls_outer": [], "ls_mono": []}
    times = {k: [] for k in rows}
    layers, es = clips.mo_si_stack(40)
    rtol = 1e-4
    for i in range(nclips):
        p = clips.Problem(nx=32, ny=32, nz=16, lx_nm=64.0, ly_nm=64.0, t_nm=30.0, theta_deg=6.0, phi_deg=0.0,
                          pol=clips.TE, layers=layers, eps_sub=es)
        d = torch.from_numpy(clips.manhattan(p.nx, p.ny, p.nz, p.lx_nm, p.ly_nm, seed=6000 + i)).to(dev)
        pe, npml = 64, 16
        plan = api.DiffPlan(p, pe, _diff_layout(p.nz, pe, npml), p.nz, npml)
        for pc in ("none", "damping"):
            t0 = time.perf_counter()
            _, _, info = plan.solve(d, pc, rtol=rtol, restart=30, max_iters=args.precond_max_iters, max_outer=200,
                                    precision="mixed")
            torch.cuda.synchronize()
            times[pc].append(time.perf_counter() - t0)
            rows[pc].append(info["iters"] if info["status"] == 0 else None)
            log("bench: precond clip %d %s: %d steps, %d outer, status %d, %.1f s" % (
                i, pc, info["iters"], info["outer_iters"], info["status"], times[pc][-1]))
        for cp, key in (("outer", "ls_outer"), ("mono", "ls_mono")):
            ls = api.Plan(p, rtol=rtol, precision="mixed", restart=30, coupling=cp, max_outer=200, max_iters=20000)
            ls.solve(d)
            t, (_, _, li) = timed(lambda: ls.solve(d), 1)
            times[key].append(t)
            rows[key].append(li["iters"])
        log("bench: precond clip %d LS: outer %d steps, mono %d steps" % (i, rows["ls_outer"][-1], rows["ls_mono"][-1]))
        del plan
    res = {"clips": nclips, "grid": [32, 32, 16], "extended_z": 64, "rtol": rtol, "restart": 30,
           "precision": "mixed", "max_iters": args.precond_max_iters}
    for k in rows:
        its = [v for v in rows[k] if v is not None]
        res[k] = {"iters_avg_min_max": [float(np.mean(its)), int(min(its)), int(max(its))] if its else None,
                  "not_converged": sum(v is None for v in rows[k]),
                  "seconds_avg": float(np.mean(times[k])),
                  "rel_time_vs_none": float(np.mean(np.array(times[k]) / np.array(times["none"])))}
    res["paper_table_context"] = {"none": [2166, 2012, 2374], "damping": [876, 811, 930], "green": [38, 32, 46],
                                  "rel_time": {"none": 1.0, "damping": 0.43, "green": 0.11}}
    out["precond_study"] = res
    log("bench: precond", res)


def sec_layers(ctx, args, out):
    """Cost against the number of multilayer pairs (Figs. 7-8): a 30 x 30 nm absorber
    block, 44.8 nm thick (64 planes of 0.7 nm), on a 64 nm clip (32 x 32) over Mo/Si
    pairs of 7 nm (Si 4.2 nm, Mo 2.8 nm: 6 and 4 planes), the substrate being the
    background medium, TE 6 deg, rtol 1e-4, mixed precision, spectral damping (the faster
    of the two differential solves in the preconditioner study).
    Full-domain PSFD (pairs on the grid, the extended z grid grown to hold them)
    against the background-field method with the same differential operator (absorber
    only, the pairs in T_R) and the Lippmann-Schwinger solve (monolithic coupling)."""
    import numpy as np
    api, torch, clips, dev = ctx["api"], ctx["torch"], ctx["clips"], ctx["dev"]
    dz, nz, n, L, npml, gap = 0.7, 64, 32, 64.0, 43, 8
    dabs = clips.cuboid(n, n, nz, L, L, 30.0, 30.0)
    d_abs = torch.from_numpy(dabs).to(dev)
    rows = []
    for pairs in [int(v) for v in args.layer_pairs.split(",")]:
        layers, _ = clips.mo_si_stack(pairs, period_nm=7.0)
        p = clips.Problem(nx=n, ny=n, nz=nz, lx_nm=L, ly_nm=L, t_nm=nz * dz, theta_deg=6.0, phi_deg=0.0,
                          pol=clips.TE, layers=layers, eps_sub=1.0)
        row = {"pairs": pairs}
        # full domain: the pairs below the absorber on the grid
        nl = 10 * pairs
        need = 2 * npml + 2 * gap + nl + nz
        pe = 1 << (need - 1).bit_length()
        zc0 = npml + gap + (pe - need) // 2
        pf = clips.Problem(**{**p.__dict__, "layers": []})
        dc = torch.from_numpy(clips.layered_contrast(nz + nl, nz, dz, layers, dabs)).to(dev)
        plan = api.DiffPlan(pf, pe, zc0, nz + nl, npml, form="full")
        t0 = time.perf_counter()
        _, of, fi = plan.solve(dc, "damping", rtol=1e-4, restart=30, max_iters=args.layer_max_iters,
                               precision="mixed")
        torch.cuda.synchronize()
        row["full_domain"] = {"z_planes": pe, "iters": fi["iters"], "status": fi["status"],
                              "seconds": time.perf_counter() - t0}
        del plan
        # background field, differential operator: absorber only
        peb = 1 << (2 * npml + 2 * gap + nz - 1).bit_length()
        plan = api.DiffPlan(p, peb, (peb - nz) // 2, nz, npml)
        t0 = time.perf_counter()
        log("bench: layers %d pairs full domain: %d steps, status %d, %.1f s" % (
            pairs, fi["iters"], fi["status"], row["full_domain"]["seconds"]))
        _, ob, bi = plan.solve(d_abs, "damping", rtol=1e-4, restart=30, max_iters=args.layer_max_iters,
                               max_outer=200, precision="mixed")
        log("bench: layers %d pairs background (differential): %d steps, %d outer, status %d" % (
            pairs, bi["iters"], bi["outer_iters"], bi["status"]))
        torch.cuda.synchronize()
        row["background_diff"] = {"z_planes": peb, "iters": bi["iters"], "outer_iters": bi["outer_iters"],
                                  "status": bi["status"], "seconds": time.perf_counter() - t0}
        del plan
        # Lippmann-Schwinger (Green's function), monolithic coupling
        ls = api.Plan(p, rtol=1e-4, precision="mixed", restart=8, max_iters=20000)
        ls.solve(d_abs)
        t, (_, ol, li) = timed(lambda: ls.solve(d_abs), 1)
        row["ls_mono"] = {"iters": li["iters"], "seconds": t}
        a = [o.cpu().numpy()[0, 0] for o in (of, ob, ol)]
        row["specular_order"] = {"full_domain": [complex(v).__repr__() for v in a[0]],
                                 "diff_vs_full": float(np.abs(a[1] - a[0]).max() / np.abs(a[0]).max()),
                                 "ls_vs_full": float(np.abs(a[2] - a[0]).max() / np.abs(a[0]).max())}
        rows.append(row)
        log("bench: layers", row)
    out["layer_study"] = {"rows": rows, "grid": [n, n, nz], "dz_nm": dz, "pml_planes": npml,
                          "precond": "damping", "rtol": 1e-4, "max_iters_per_linear_solve": args.layer_max_iters}


def sec_cpu(ctx, args, out):
    """The CPU oracle on a bounded sample of the headline solve: table set-up plus k GMRES(30)
    iterations of the oracle's monolithic operator (I - M V), the system the GPU solves, on
    all host threads; scaled to a full solve by the oracle's own iteration count to the
    headline tolerance, recorded by tests/golden/make_golden.py --iterations (the GPU's
    count when that record is absent)."""
    import oracle as O
    prob, deps_np = ctx["prob"], ctx["deps_np"]
    ncores = os.cpu_count() or 1
    O.set_workers(ncores)
    t0 = time.perf_counter()
    S = O.Setup(prob)
    _ = S.G
    ebg = O.background_field(S)
    t_setup = time.perf_counter() - t0
    k = args.cpu_iters
    t0 = time.perf_counter()
    O.gmres(lambda v: O.apply_monolithic(S, deps_np, v), ebg, None, 1e-30, 30, k)
    t_it = (time.perf_counter() - t0) / k
    its, src = out.get("mixed", {}).get("iters", 337), "the GPU solve's count"
    try:
        with open(os.path.join(GOLDEN_DIR, "oracle_headline_iterations.json")) as f:
            rec = json.load(f)
        run = min(rec["runs"], key=lambda r: abs(math.log(r["rtol"] / args.rtol)))
        its, src = run["iters"], "the oracle's own count to rtol %g (recorded)" % run["rtol"]
    except (OSError, KeyError, ValueError):
        pass
    t_solve = t_setup + its * t_it
    out["cpu_baseline"] = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": ncores, "kind": "oracle",
                           "sample": f"table set-up plus {k} FP64 GMRES(30) iterations of the oracle's monolithic "
                                     f"operator on the same clip (scipy.fft workers={ncores}), {t_it:.2f} s per "
                                     f"iteration, scaled to {its} iterations ({src})",
                           "s_per_iteration": t_it, "s_setup": t_setup, "iterations_scaled_to": its,
                           "cpu_model": cpu_model()}


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_study(args):
    """The CPU oracle timed on the workloads' own inputs (host only; no GPU is touched).

    Per item: the oracle's table set-up, one apply of its monolithic operator
    (I - M V) (the system the GPU solves; (I - M^T V) for the adjoint), and the time per
    FP64 GMRES(m) iteration over a bounded sample of iterations (--oracle-iters),
    with scipy.fft on all host threads and, for the first two workloads, on
    one. A solve's time is then set-up + iterations x time per iteration, at
    the iteration count of the GPU solve of the same instance (the oracle's own
    outer reflection loop needs more; the 64 nm line/space clip is also solved
    in full, which takes seconds). Items: 64 nm line/space 32x32x32; the
    128x128x64 contact-hole clip; the first four instances of the batched set
    and of the serving pool; the 256x256x64 smooth clip, forward and transposed
    (adjoint) iterations. The oracle is the plain FP64 one, untuned.
    """
    import numpy as np
    import oracle as O
    from paper_2606_25541_amd import clips
    ncores = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res = {"kind": "oracle", "host_threads": ncores, "cpu_model": model, "gmres_restart": args.restart,
           "items": []}
    k = args.oracle_iters

    def sample(name, p, d, workers, transpose=False, full_rtol=None):
        O.set_workers(workers)
        t0 = time.perf_counter()
        S = O.Setup(p)
        _ = S.G
        t_setup = time.perf_counter() - t0
        x = clips.random_complex((3, p.nz, p.ny, p.nx), 1)
        V = O.potential(S, d)
        # the coupled system the GPU solves: (I - M V) u = e_bg, or its transpose
        if transpose:
            op = lambda v: v - O.apply_M_T(S, V[None] * v)
        else:
            op = lambda v: O.apply_monolithic(S, d, v)
        op(x)
        t0 = time.perf_counter()
        op(x)
        t_apply = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.gmres(op, O.background_field(S), None, 1e-30, args.restart, k)
        t_it = (time.perf_counter() - t0) / k
        it = {"item": name, "workers": workers, "transpose": transpose, "s_setup": t_setup, "s_apply": t_apply,
              "s_per_iteration": t_it, "sample_iterations": k}
        if full_rtol is not None:
            t0 = time.perf_counter()
            r = O.solve(p, d, rtol=full_rtol, restart=30, max_iters=20000)
            it.update({"s_full_solve": time.perf_counter() - t0, "full_iters": r["iters"],
                       "full_outer_iters": r["outer_iters"], "full_mono_residual": float(r["mono_residual"])})
        res["items"].append(it)
        log("oracle study:", it)

    p1 = clips.config_problem("G1")
    d1 = clips.line_space(p1.nx, p1.ny, p1.nz, p1.lx_nm, p1.ly_nm, 16.0, 48.0)
    p2 = clips.config_problem("G3", pol=clips.TE)
    d2 = clips.contact_holes(128, 128, 64, 256.0, 256.0, 8, seed=2001)
    for w in (ncores, 1):
        sample("line/space 32x32x32", p1, d1, w, full_rtol=1e-8)
        sample("contact holes 128x128x64", p2, d2, w)
    batched = clips.batched_set()
    for i, (g, p, d) in enumerate(batched[:4]):
        sample("batched instance %d (%s)" % (i, g), p, d, ncores)
    pool = clips.serving_pool()
    for i, (g, p, d) in enumerate(pool[:4]):
        sample("serving request %d (%s)" % (i, g), p, d, ncores)
    p5 = clips.config_problem("G4")
    d5, _ = clips.smooth_density_eps(p5.nx, p5.ny, p5.nz, p5.lx_nm, p5.ly_nm, p5.t_nm, seed=5001)
    sample("smooth clip 256x256x64", p5, d5, ncores)
    sample("smooth clip 256x256x64", p5, d5, ncores, transpose=True)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--rtol", type=float, default=3e-7,
                    help="headline tolerance (3e-7 brings the field error against the FP64 oracle below 1e-6)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="headline solve only")
    ap.add_argument("--only", choices=SECTIONS, default=None, help="run one section")
    ap.add_argument("--adjoint-fd", type=int, default=16, help="voxels of the adjoint's finite-difference check")
    ap.add_argument("--precond-clips", type=int, default=4, help="clips of the preconditioner study")
    ap.add_argument("--precond-max-iters", type=int, default=20000,
                    help="GMRES step limit of the differential solves")
    ap.add_argument("--layer-pairs", default="5,10,20,40", help="multilayer pairs of the layer-count study")
    ap.add_argument("--layer-max-iters", type=int, default=40000,
                    help="GMRES step limit per linear solve of the layer-count study")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-budget-gib", type=float, default=12.0,
                    help="device-memory budget of the server (binding: the three grids at 8 slots need ~24 GiB)")
    ap.add_argument("--serve-burst", type=int, default=24)
    ap.add_argument("--serve-qps", default="0.7",
                    help="comma-separated arrival rates as fractions of the saturated rate")
    ap.add_argument("--oracle-study", action="store_true",
                    help="time the CPU oracle on the workloads (host only) and exit")
    ap.add_argument("--oracle-iters", type=int, default=20, help="GMRES iterations per oracle timing sample")
    ap.add_argument("--cpu-iters", type=int, default=20, help="oracle GMRES iterations of the cpu_baseline sample")
    args = ap.parse_args()
    if args.oracle_study:
        oracle_study(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1 (there is no multi-GPU path)"}))
        sys.exit(2)

    import torch
    from paper_2606_25541_amd import api, clips, _lib

    dev = torch.device("cuda:0")
    prob = clips.config_problem("G3", pol=clips.TE)
    deps_np = clips.contact_holes(128, 128, 64, 256.0, 256.0, 8, seed=2001)
    ctx = {"api": api, "torch": torch, "clips": clips, "_lib": _lib, "dev": dev, "prob": prob,
           "deps_np": deps_np, "deps": torch.from_numpy(deps_np).to(dev)}
    out = {
        "metric": "solves/s at 1e-6 rel. residual (mixed vs FP64) + operator applies/s + p99",
        "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64+c128 (mixed)", "data": "synthetic",
        "config": {"workload": "contact-hole clip 128x128x64, 256 nm, 8 holes 20-40 nm, 60 nm absorber, "
                               "40 Mo/Si pairs, TE 6 deg, mixed FP32/FP64, rtol %g (field error <= 1e-6 "
                               "against the FP64 oracle; rtol 1e-6 reported beside it)" % args.rtol,
                   "grid": [prob.nx, prob.ny, prob.nz], "restart": args.restart, "rtol": args.rtol,
                   "parallelism": "single GPU"},
    }
    if args.only:
        todo = [args.only]
    elif args.quick:
        todo = ["solve"]
    else:
        todo = [s for s in SECTIONS if s != "cpu" or not args.no_cpu]
    fns = {"solve": sec_solve, "fp64": sec_fp64, "apply": sec_apply, "isolated": sec_isolated, "batched": sec_batched,
           "serving": sec_serving, "adjoint": sec_adjoint, "precond": sec_precond, "layers": sec_layers,
           "cpu": sec_cpu}
    for s in todo:
        log("bench: section", s)
        fns[s](ctx, args, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
