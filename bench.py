"""Benchmark: cutting voxel projector A x + A^T b on one MI355X.

Workload: 512^3 voxels of 0.25 mm, 616x480 detector of 0.616 mm, SID 749 /
SDD 1198 mm, 248 views over 200 degrees (C-arm short scan); relaxed CVP with
elevation correction; phantom of 80 seeded ellipsoids plus 1% uniform noise;
projection data U[0,1).  One step = one projection A x and one
backprojection A^T b, inputs resident in HBM.

value = 2 * n_voxels * n_views / (t_A + t_AT)   [voxel-view updates/s]

Before the timed region the geometry's cut-piece records are computed once
and cached on the device (cvp_geometry_cache_records, part of the geometry
set-up like the pixel factor tables; its size and build time are reported,
and one A / A^T pair without the cache is timed after the timed region for
comparison), and the autotuner picks the launch plan (projection band width,
backprojection stack width) on random data of the same shape.  After
it, CGLS from zero on consistent data b = A x_true is run to
|A^T (b - A x)| <= 1e-3 |A^T b| and its wall time reported ("cgls").

Prints one JSON line.  The CPU baseline times the FP64 oracle on a bounded
sample of the same workload (A x and A^T b over three views, extrapolated),
plus a one-thread run of the 64^3 workload; --cpu-baseline-full runs the
whole CPU-baseline plan instead (minutes, no GPU) and prints its record.

The roofline counts FP32 VALU lane-operations of the method per voxel-view
(costmodel.py, fixed constants per step); the instruction overhead beside it
is the kernel's measured VALU lane-instructions per voxel-view (rocprofv3
SQ_INSTS_VALU of the committed counter summary, while the kernel source
matches it) over that count.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="relaxed", choices=["relaxed", "exact"])
    ap.add_argument("--no-ec", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cgls", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the planner's default launch plan")
    ap.add_argument("--no-record-cache", action="store_true",
                    help="let every launch compute its own cut-piece records (no cached record table)")
    ap.add_argument("--launch", default=None, metavar="U,GW,KP[,WPC[,SHARED]]",
                    help="fixed launch plan (projection band columns, backprojection stack columns and passes, "
                         "backprojection workgroups per CU and one window per workgroup); no autotuning")
    ap.add_argument("--cgls-max-iter", type=int, default=200)
    ap.add_argument("--no-network", action="store_true", help="skip the warm-start network timing")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-problem batched timing")
    ap.add_argument("--no-cone", action="store_true", help="skip the 256^3 cone-beam timing")
    ap.add_argument("--no-paper-benchmarks", action="store_true",
                    help="skip the paper's two speed benchmarks (CVP and TT, one application each)")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="run only the full CPU-baseline plan of the oracle (minutes, no GPU)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def calib_copy():
    import torch
    n = 1 << 28    # 2^28 floats = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": 4 * n}))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def cpu_baseline(g, x, b, n_views=3):
    """The FP64 oracle (C, OpenMP over every host thread) on a bounded sample
    of the benchmark workload: A x and A^T b for the first n_views views of
    the whole volume, the rate extrapolated to all views (about 20 s on 16
    threads); beside it a one-thread run of the 64^3 / 32-view workload in
    full (A x and A^T b)."""
    import numpy as np
    import oracle
    from paper_2110_09841_amd import synth
    o = oracle.Options(exact=False, ec=True)
    n1, n2, n3 = g["vol_dims"]
    V = len(g["angles_rad"])
    threads = oracle.num_threads()
    tA = _time(lambda: oracle.project(g, o, x, views=(0, n_views)))
    tB = _time(lambda: oracle.backproject(g, o, b[:n_views], views=(0, n_views)))
    vv = n1 * n2 * n3 * n_views
    gs = synth.config_small()
    xs = synth.ellipsoid_phantom(64, 1.0, 10, seed=11)
    bs = synth.uniform_projections((32, 96, 96), seed=12)
    oracle.set_num_threads(1)
    try:
        t1A = _time(lambda: oracle.project(gs, o, xs))
        t1B = _time(lambda: oracle.backproject(gs, o, bs))
    finally:
        oracle.set_num_threads(threads)
    vv1 = 64 ** 3 * 32
    return {"value": 2 * vv / (tA + tB), "unit": "voxel-view updates/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": "FP64 C/OpenMP oracle, relaxed CVP with EC: A x (%.1f s) and A^T b (%.1f s) for %d of %d "
                      "views of the 512^3 volume; extrapolated to all views: A %.0f s, A^T %.0f s per application"
                      % (tA, tB, n_views, V, tA * V / n_views, tB * V / n_views),
            "project_voxel_views_per_s": vv / tA, "backproject_voxel_views_per_s": vv / tB,
            "one_thread": {"workload": "small_64c_32v (full)", "project_s": t1A, "backproject_s": t1B,
                           "voxel_views_per_s": 2 * vv1 / (t1A + t1B)}}


def cpu_baseline_full():
    """The CPU-baseline plan in full (a long run, minutes): the oracle on every
    host thread and on one thread for the 64^3 / 32-view workload (A, A^T and
    CGLS to rho <= 1e-3), every thread for the 256^3 / 360-view cone workload
    in full (exact and relaxed, EC on), and the 512^3 / 248-view workload on
    8 views, extrapolated."""
    import numpy as np
    import oracle
    from oracle.cgls import cgls
    from paper_2110_09841_amd import synth
    threads = oracle.num_threads()
    out = {"cpu": cpu_model(), "threads": threads, "kind": "oracle (FP64 C/OpenMP)"}

    def log(*a):
        print("[cpu-baseline]", *a, file=sys.stderr, flush=True)

    gs = synth.config_small()
    xs = synth.ellipsoid_phantom(64, 1.0, 10, seed=11)
    bs = synth.uniform_projections((32, 96, 96), seed=12)
    vv = 64 ** 3 * 32
    rec = {"voxel_views": vv}
    orl = oracle.Options(exact=False, ec=True)
    bcl = oracle.project(gs, orl, xs)                  # consistent data b = A x_true

    def run_cgls(n):
        return cgls(lambda v: oracle.project(gs, orl, v), lambda r: oracle.backproject(gs, orl, r), bcl, n,
                    np.zeros(xs.shape))[1]
    gam = run_cgls(100)
    rho = np.sqrt(gam / gam[0])
    it = int(np.argmax(rho <= 1e-3)) if (rho <= 1e-3).any() else len(gam) - 1
    rec["cgls_relaxed_iterations_to_1e-3"] = it
    for nthr in (threads, 1):
        oracle.set_num_threads(nthr)
        o = oracle.Options(exact=True, ec=True)
        tA = _time(lambda: oracle.project(gs, o, xs))
        tB = _time(lambda: oracle.backproject(gs, o, bs))
        tc = _time(lambda: run_cgls(it))
        rec["threads_%d" % nthr] = {"exact_project_s": tA, "exact_backproject_s": tB,
                                    "voxel_views_per_s": 2 * vv / (tA + tB), "cgls_relaxed_to_1e-3_s": tc}
        log("small", nthr, rec["threads_%d" % nthr])
    oracle.set_num_threads(threads)
    out["small_64c_32v"] = rec

    gc = synth.config_cone()
    xc = synth.ellipsoid_phantom(256, 0.5, 40, seed=21)
    bc = synth.uniform_projections((360, 384, 512), seed=22)
    vv = 256 ** 3 * 360
    rec = {"voxel_views": vv}
    for variant in ("exact", "relaxed"):
        o = oracle.Options(exact=variant == "exact", ec=True)
        tA = _time(lambda: oracle.project(gc, o, xc))
        tB = _time(lambda: oracle.backproject(gc, o, bc))
        rec[variant] = {"project_s": tA, "backproject_s": tB, "voxel_views_per_s": 2 * vv / (tA + tB)}
        log("cone", variant, rec[variant])
    out["cone_256c_360v"] = rec

    g = synth.config_carm()
    x = synth.ellipsoid_phantom(512, 0.25, 80, seed=31, noise_frac=0.01)
    b = synth.uniform_projections((248, 480, 616), seed=32)
    o = oracle.Options(exact=False, ec=True)
    nv = 8
    tA = _time(lambda: oracle.project(g, o, x, views=(0, nv)))
    tB = _time(lambda: oracle.backproject(g, o, b[:nv], views=(0, nv)))
    vv = 512 ** 3 * nv
    out["carm_512c_248v"] = {"extrapolated": True, "views_timed": nv, "project_s_8_views": tA,
                             "backproject_s_8_views": tB, "project_s_extrapolated": tA * 248 / nv,
                             "backproject_s_extrapolated": tB * 248 / nv, "voxel_views_per_s": 2 * vv / (tA + tB)}
    log("carm", out["carm_512c_248v"])
    return out


def measured_counters(kernel):
    """Counters per launch of `kernel` from the committed rocprofv3 summary
    of this workload: HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated against
    a 1 GiB copy) and VALU instructions, or None when the kernel source
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters_carm_512c_248v.json")
    src = os.path.join(ROOT, "paper_2110_09841_amd", "csrc", "cvp_kernels.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha1(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel_source_sha1") != sha or kernel not in rec:
        return None
    k = rec[kernel]
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "fetch_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "sq_insts_valu": k.get("sq_insts_valu"),
            "algorithmic_bytes": rec["algorithmic_bytes_per_launch"], "plan": rec.get("plan")}


def paper_benchmarks(reps=2):
    """The paper's two speed benchmarks (Sec. IV-A, Tables I and II) rerun on
    synthetic data: "Long" (512 x 512 x 128 voxels of 0.5 mm, 720 views, 512 x
    512 pixels of 1 mm, SID 541 / SDD 949) and "Pfeiffer" (256^3 voxels of
    0.5 mm, 100 views over 198 degrees, 1280 x 960 pixels of 0.25 mm, SID 750 /
    SDD 1000): one application of A and of A^T per projector (CVP exact and
    relaxed with EC, and TT), timed with HIP events on uniform random data,
    with the default plan; then CVP again with the cut-piece records cached
    and the plan autotuned.  The paper's times on its GPUs (context, not
    targets) go beside them."""
    import torch
    from paper_2110_09841_amd import cvp, synth
    setups = {
        "long": (dict(dims=(512, 512, 128), vox=0.5, det=(512, 512), pitch=1.0, sid=541.0, sdd=949.0, views=720,
                      arc=360.0),
                 {"cvp": [39.3, 19.7], "cvp_relaxed": [12.3, 5.2], "tt": [101.1, 18.8]}),
        "pfeiffer": (dict(dims=(256, 256, 256), vox=0.5, det=(1280, 960), pitch=0.25, sid=750.0, sdd=1000.0,
                          views=100, arc=198.0),
                     {"cvp": [22.5, 14.1], "cvp_relaxed": [7.5, 4.1], "tt": [27.6, 11.5]}),
    }
    out = {}
    gen = torch.Generator(device="cuda").manual_seed(8)
    for name, (c, paper) in setups.items():
        G = cvp.Geometry(synth.geometry(c["dims"], c["vox"], c["det"][0], c["det"][1], c["pitch"], c["sid"], c["sdd"],
                                        c["views"], c["arc"]))
        x = torch.rand(G.vol_shape, generator=gen, device="cuda")
        b = torch.rand(G.proj_shape, generator=gen, device="cuda")
        po, vo = torch.empty_like(b), torch.empty_like(x)
        res = {"voxel_views": G.n_voxels * G.n_views,
               "paper_radeon_vii_s": paper}
        for key, opts in (("cvp", cvp.Options(variant="exact", ec=True)),
                          ("cvp_relaxed", cvp.Options(variant="relaxed", ec=True)), ("tt", cvp.TT)):
            cvp.project(x, G, opts, out=po)
            cvp.backproject(b, G, opts, out=vo)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                cvp.project(x, G, opts, out=po)
            ev[1].record()
            for _ in range(reps):
                cvp.backproject(b, G, opts, out=vo)
            ev[2].record()
            torch.cuda.synchronize()
            res[key + "_ms"] = [ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps]
        # the CVP forms again with the geometry's cut-piece records cached and
        # the plan autotuned per form (as for the other workloads)
        from paper_2110_09841_amd.autotune import autotune
        res["record_cache_bytes"] = G.cache_records()
        for key, opts in (("cvp", cvp.Options(variant="exact", ec=True)),
                          ("cvp_relaxed", cvp.Options(variant="relaxed", ec=True))):
            autotune(G, opts, bands=(4, 6, 8, 12), reps=1)
            cvp.project(x, G, opts, out=po)
            cvp.backproject(b, G, opts, out=vo)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                cvp.project(x, G, opts, out=po)
            ev[1].record()
            for _ in range(reps):
                cvp.backproject(b, G, opts, out=vo)
            ev[2].record()
            torch.cuda.synchronize()
            res[key + "_cached_records_ms"] = [ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps]
            res[key + "_cached_records_launch"] = list(G.launch) + [G.bp_workgroups_per_cu, int(G.bp_shared_window)]
        out[name] = res
        del G, x, b, po, vo
        torch.cuda.empty_cache()
    return out


def cone_timing(reps=2):
    """The 12-degree cone workload (256^3 voxels of 0.5 mm, 512x384 pixels
    of 0.388 mm, SID 600 / SDD 900, 360 views): A and A^T timed separately
    for the exact and the relaxed form, EC on, autotuned plan per form."""
    import torch
    from paper_2110_09841_amd import cvp, synth
    from paper_2110_09841_amd.autotune import autotune
    G = cvp.Geometry(synth.config_cone())
    G.cache_records()
    vv = G.n_voxels * G.n_views
    gen = torch.Generator(device="cuda").manual_seed(6)
    x = torch.rand(G.vol_shape, generator=gen, device="cuda")
    b = torch.rand(G.proj_shape, generator=gen, device="cuda")
    po, vo = torch.empty_like(b), torch.empty_like(x)
    res = {"workload": "cone_256c_360v", "voxel_views": vv}
    for variant in ("exact", "relaxed"):
        opts = cvp.Options(variant=variant, ec=True)
        autotune(G, opts, bands=(6, 8, 9, 12), reps=1)
        ms = {}
        for name, fn in (("project", lambda: cvp.project(x, G, opts, out=po)),
                         ("backproject", lambda: cvp.backproject(b, G, opts, out=vo))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms[name] = e0.elapsed_time(e1) / reps
        res[variant] = {"launch": list(G.launch) + [G.bp_workgroups_per_cu, int(G.bp_shared_window)],
                        "project_ms": ms["project"],
                        "backproject_ms": ms["backproject"],
                        "voxel_views_per_s": 2 * vv / ((ms["project"] + ms["backproject"]) * 1e-3)}
    del x, b, po, vo
    torch.cuda.empty_cache()
    return res


def batched_timing(reps=2):
    """The 16-problem batch (volumes 96^3..320^3, 60..400 views): one
    persistent launch per direction against 16 single-problem launches, both
    with every member's cut-piece records cached (and, for comparison, both
    without)."""
    import torch
    from paper_2110_09841_amd import cvp, synth
    params = synth.config_batch()
    geoms = [cvp.Geometry(p) for p in params]
    opts = cvp.Options(variant="relaxed", ec=True)
    gen = torch.Generator(device="cuda").manual_seed(5)
    xs = [torch.rand(g.vol_shape, generator=gen, device="cuda") for g in geoms]
    bs = [torch.rand(g.proj_shape, generator=gen, device="cuda") for g in geoms]
    po = [torch.empty(g.proj_shape, device="cuda") for g in geoms]
    vo = [torch.empty(g.vol_shape, device="cuda") for g in geoms]

    def batched_p():
        cvp.project_batched(xs, batch, opts, outs=po)

    def batched_b():
        cvp.backproject_batched(bs, batch, opts, outs=vo)

    def single_p():
        for q, g in enumerate(geoms):
            cvp.project(xs[q], g, opts, out=po[q])

    def single_b():
        for q, g in enumerate(geoms):
            cvp.backproject(bs[q], g, opts, out=vo[q])

    def timed():
        times = {}
        for name, fn in (("batched_project", batched_p), ("batched_backproject", batched_b),
                         ("single_project", single_p), ("single_backproject", single_b)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / reps
        times["batched"] = times["batched_project"] + times["batched_backproject"]
        times["single"] = times["single_project"] + times["single_backproject"]
        return times

    batch = cvp.Batch(geoms)
    plain = timed()
    del batch
    table_bytes = sum(g.cache_records() for g in geoms)
    batch = cvp.Batch(geoms)
    times = timed()
    vv = 2 * sum(g.n_voxels * g.n_views for g in geoms)
    res = {"workload": "batch16_96c_320c", "problems": len(geoms), "voxel_views": vv,
           "record_cache_bytes": table_bytes,
           "batched_ms": times["batched"], "single_launches_ms": times["single"],
           "batched_over_single": times["batched"] / times["single"],
           "per_direction_ms": {k: times[k] for k in ("batched_project", "batched_backproject", "single_project",
                                                      "single_backproject")},
           "batched_voxel_views_per_s": vv / (times["batched"] * 1e-3),
           "without_record_cache": {"batched_ms": plain["batched"], "single_launches_ms": plain["single"],
                                    "batched_over_single": plain["batched"] / plain["single"]}}
    # CGLS on all 16 problems at once (b = the batched projections above):
    # one replay of a graph of 5 batched iterations
    cvp.project_batched(xs, batch, opts, outs=po)
    solver = cvp.BatchedCGLS(batch, opts, po)
    solver.start()
    solver.capture(5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    solver.replay()
    e1.record()
    torch.cuda.synchronize()
    res["cgls_graph5_ms"] = e0.elapsed_time(e1)
    res["cgls_ms_per_iteration"] = res["cgls_graph5_ms"] / 5
    del solver, xs, bs, po, vo, batch, geoms
    torch.cuda.empty_cache()
    return res


def network_timing(reps=5):
    """Warm-start U-Net at 128^3 (the warm-start workload's volume): forward
    pass and full training step (forward, backward, Adam), HIP events."""
    import torch
    from paper_2110_09841_amd.unet import UNet, forward_bound_seconds, forward_flops
    shape = (128, 128, 128)
    net = UNet(shape, seed=1)
    g = torch.Generator(device="cuda").manual_seed(0)
    x1, x2, t = (0.01 * torch.rand(shape, generator=g, device="cuda") for _ in range(3))
    for _ in range(2):
        net.train_step(x1, x2, t)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        net.forward(x1, x2)
    ev[1].record()
    for _ in range(reps):
        net.train_step(x1, x2, t)
    ev[2].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    step = ev[1].elapsed_time(ev[2]) / reps
    fl = forward_flops(shape)
    fla = forward_flops(shape, algorithmic=True)
    bound = forward_bound_seconds(shape)
    res = {"shape": list(shape), "forward_ms": fwd, "train_step_ms": step, "forward_gflop_executed": fl / 1e9,
           "forward_gflop_algorithmic": fla / 1e9, "forward_tflops_algorithmic": fla / (fwd * 1e-3) / 1e12,
           "peak_bf16_tflops": 2500.0, "forward_bound_ms": bound * 1e3,
           "forward_over_bound": fwd / (bound * 1e3),
           "train_step_tflops_executed": 3 * fl / (step * 1e-3) / 1e12}
    del net
    torch.cuda.empty_cache()
    return res


def cgls_to_tolerance(G, opts, x_true, max_iter):
    """CGLS from zero on b = A x_true until rho = |A^T(b - A x)| / |A^T b|
    <= 1e-3, stopped on the device: the iteration that meets the tolerance
    raises a flag and the rest of the captured 5-iteration graph (captured
    before the timed region) does nothing, so the time counts the iterations
    needed plus at most 4 empty ones.  Time runs from the start call (r = b,
    s = A^T b) to the replay boundary at which the host sees the flag."""
    import torch
    from paper_2110_09841_amd import cvp
    from paper_2110_09841_amd.cgls import CGLS
    b = cvp.project(x_true, G, opts)
    solver = CGLS(G, opts, b)
    solver.capture(5)
    it, sec, rho = solver.run(tol=1e-3, max_iter=max_iter, per_graph=5)
    res = {"tol": 1e-3, "iterations": it, "seconds": sec, "reached": bool(rho[it] <= 1e-3),
           "rho_final": float(rho[-1]), "iterations_run": len(rho) - 1, "per_graph": 5,
           "stop": "device flag (1-iteration granularity)",
           "data": "b = A x_true (consistent), x0 = 0"}
    # one replay of a graph of 20 iterations, from a fresh start
    solver.reset(b)
    solver.set_tolerance(0.0)
    solver.start()
    solver.capture(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.replay()
    torch.cuda.synchronize()
    res["graph20_replay_s"] = time.perf_counter() - t0
    res["graph20_rho"] = float(solver.rho()[-1])
    del solver, b
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); got --gpus %d" % args.gpus)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2110_09841_amd import costmodel, cvp, synth
    from paper_2110_09841_amd.autotune import autotune
    if args.calib_copy:
        calib_copy()
        return
    if args.cpu_baseline_full:
        print(json.dumps({"cpu_baseline_full": cpu_baseline_full()}), flush=True)
        return
    torch.cuda.set_device(0)
    g = synth.config_carm()
    n1, n2, n3 = g["vol_dims"]
    V = len(g["angles_rad"])
    x_h = synth.ellipsoid_phantom(512, 0.25, 80, seed=31, noise_frac=0.01)
    b_h = synth.uniform_projections((V, g["det_rows"], g["det_cols"]), seed=32)
    G = cvp.Geometry(g)
    ec = not args.no_ec
    opts = cvp.Options(variant=args.variant, ec=ec)
    record_cache = None
    if not args.no_record_cache:
        # the geometry's cut-piece records, computed once (geometry set-up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nb = G.cache_records()
        torch.cuda.synchronize()
        record_cache = {"bytes": nb, "build_ms": 1e3 * (time.perf_counter() - t0)}
    plan = {"default": list(G.launch) + [G.bp_workgroups_per_cu, int(G.bp_shared_window)]}
    if args.launch:
        G.set_launch(*(int(t) for t in args.launch.split(",")))
        plan["fixed"] = list(G.launch) + [G.bp_workgroups_per_cu, int(G.bp_shared_window)]
    elif not args.no_autotune:
        rec = autotune(G, opts, reps=2)
        plan.update(tuned=list(G.launch) + [G.bp_workgroups_per_cu, int(G.bp_shared_window)],
                    project_ms=rec["project_ms"],
                    backproject_ms=rec["backproject_ms"])
    x = torch.from_numpy(x_h).cuda()
    b = torch.from_numpy(b_h).cuda()
    p_out = torch.empty(G.proj_shape, dtype=torch.float32, device="cuda")
    v_out = torch.empty(G.vol_shape, dtype=torch.float32, device="cuda")

    for _ in range(args.warmup):
        cvp.project(x, G, opts, out=p_out)
        cvp.backproject(b, G, opts, out=v_out)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record()
        cvp.project(x, G, opts, out=p_out)
        ev[s][1].record()
        cvp.backproject(b, G, opts, out=v_out)
        ev[s][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tA = np.array([ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]) * 1e-3
    tB = np.array([ev[s][1].elapsed_time(ev[s][2]) for s in range(args.steps)]) * 1e-3
    vv = n1 * n2 * n3 * V
    value = 2 * vv / (tA.mean() + tB.mean())
    if record_cache is not None:
        # the same plan with every launch computing its own records, for comparison
        G.cache_records(False)
        e4 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        cvp.project(x, G, opts, out=p_out)
        cvp.backproject(b, G, opts, out=v_out)
        e4[0].record()
        cvp.project(x, G, opts, out=p_out)
        e4[1].record()
        cvp.backproject(b, G, opts, out=v_out)
        e4[2].record()
        torch.cuda.synchronize()
        record_cache["without_cache"] = {"project_ms": e4[0].elapsed_time(e4[1]),
                                         "backproject_ms": e4[1].elapsed_time(e4[2])}
        G.cache_records()
        torch.cuda.synchronize()

    exact = args.variant == "exact"
    counts = costmodel.estimate_counts(g)
    rA = costmodel.roofline(g, exact, ec, tA.mean(), counts)
    rB = costmodel.roofline(g, exact, ec, tB.mean(), counts)
    dom, rdom, name = (tA, rA, "cvp_project") if tA.mean() >= tB.mean() else (tB, rB, "cvp_backproject")
    traffic = measured_counters(name)

    def overhead(kernel, r):
        c = measured_counters(kernel)
        if not c or not c.get("sq_insts_valu"):
            return None
        return c["sq_insts_valu"] * 64 / vv / r["ops_per_vv"]
    out = {
        "metric": "voxel-view updates/s (CVP Ax+A^T b, 512^3, 248 views); CGLS time to 1e-3 residual",
        "value": float(value),
        "unit": "voxel-view updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ellipsoid phantom + 1% noise; U[0,1) projections)",
        "config": {"workload": "carm_512c_248v", "volume": [n1, n2, n3], "voxel_mm": 0.25,
                   "detector": [g["det_cols"], g["det_rows"]], "pitch_mm": 0.616, "views": V,
                   "arc_deg": 200, "sid_mm": 749, "sdd_mm": 1198, "variant": args.variant,
                   "elevation_correction": ec, "scaling": "solid_angle",
                   "launch": dict(zip(("proj_band_cols", "bp_stack_cols", "bp_passes", "bp_workgroups_per_cu",
                                       "bp_shared_window"),
                                      G.launch + (G.bp_workgroups_per_cu, G.bp_shared_window)))},
        "autotune": plan,
        "record_cache": record_cache,
        "project": {"ms": 1e3 * tA.mean(), "voxel_views_per_s": vv / tA.mean()},
        "backproject": {"ms": 1e3 * tB.mean(), "voxel_views_per_s": vv / tB.mean()},
        "roofline": {"bound": "alu", "kernel": name, "achieved": rdom["achieved"] / 1e12,
                     "peak": rdom["peak"] / 1e12, "unit": "TOP/s (FP32 VALU lane-ops)",
                     "frac": rdom["frac"], "ops_per_voxel_view": rdom["ops_per_vv"],
                     "counts_per_voxel_view": {"column_pieces": rdom["n_c"], "pixels": rdom["n_p"],
                                               "ec_edge_pixels": rdom["n_e"]},
                     "instruction_overhead": overhead(name, rdom),
                     "other_kernel": {"kernel": "cvp_project" if name == "cvp_backproject" else "cvp_backproject",
                                      "frac": (rA if name == "cvp_backproject" else rB)["frac"],
                                      "instruction_overhead": overhead(
                                          "cvp_project" if name == "cvp_backproject" else "cvp_backproject",
                                          rA if name == "cvp_backproject" else rB)},
                     "traffic": traffic["bytes"] if traffic else None, "traffic_unit": "bytes per launch",
                     "traffic_detail": traffic},
    }
    if not args.no_cgls:
        out["cgls"] = cgls_to_tolerance(G, opts, x, args.cgls_max_iter)
    if not args.no_network:
        out["warm_start_network"] = network_timing()
    if not args.no_batched:
        out["batched"] = batched_timing()
    if not args.no_cone:
        out["cone"] = cone_timing()
    if not args.no_paper_benchmarks:
        out["paper_benchmarks"] = paper_benchmarks()
    del x, b, p_out, v_out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, x_h, b_h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
