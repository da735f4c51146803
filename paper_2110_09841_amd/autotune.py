"""Launch-plan autotuner.

Times the projection for a set of band widths (detector columns per work
item, which also sets how many workgroups share a compute unit through their
LDS footprint) and the backprojection for each stack width and number of
64-voxel passes per stack, on seeded random
data of the geometry's own shape, with HIP events on the current stream, and
keeps the fastest of each.  Results can be cached in a JSON file keyed by the
geometry and the options, so a later process reuses them without timing.
"""
import hashlib
import json
import os

import numpy as np
import torch

from . import _lib
from .cvp import Geometry, Options, backproject, project

DEFAULT_BANDS = (4, 6, 8, 9, 10, 12, 16, 19, 24, 32)
DEFAULT_STACKS = (16, 8, 4)
DEFAULT_PASSES = (2, 1)


def _key(geom: Geometry, opts: Options):
    p = geom.params
    blob = json.dumps({
        "vol_dims": list(p["vol_dims"]), "voxel_mm": list(p["voxel_mm"]),
        "vol_offset_mm": list(p.get("vol_offset_mm", (0.0, 0.0, 0.0))),
        "det": [p["det_cols"], p["det_rows"]], "pitch_mm": list(p["pitch_mm"]),
        "principal_px": None if p.get("principal_px") is None else list(p["principal_px"]),
        "sid": p["sid_mm"], "sdd": p["sdd_mm"],
        "angles": hashlib.sha1(np.asarray(p["angles_rad"], dtype=np.float64).tobytes()).hexdigest(),
        "variant": opts.variant, "ec": bool(opts.ec), "scaling": opts.scaling,
        "device": torch.cuda.get_device_name(geom.device),
    }, sort_keys=True)
    return hashlib.sha1(blob.encode()).hexdigest()


def _time(fn, reps):
    fn()                                        # warm-up (and first-touch)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(geom: Geometry, opts: Options, bands=DEFAULT_BANDS, stacks=DEFAULT_STACKS, passes=DEFAULT_PASSES,
             reps=2, cache=None, seed=0, log=None):
    """Pick and set the fastest launch plan for (geom, opts).  Returns a dict
    with the chosen plan and the measured milliseconds per candidate.  With
    cache = path of a JSON file, a stored plan for the same key is applied
    without timing, and a newly timed plan is stored."""
    key = _key(geom, opts)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            rec = table[key]
            geom.set_launch(rec["proj_band_cols"], rec["bp_stack_cols"], rec["bp_passes"],
                            rec.get("bp_workgroups_per_cu", 0), rec.get("bp_shared_window", False))
            return dict(rec, cached=True)
    g = torch.Generator(device=geom.device).manual_seed(seed)
    x = torch.rand(geom.vol_shape, generator=g, device=geom.device)
    b = torch.rand(geom.proj_shape, generator=g, device=geom.device)
    p_out = torch.empty_like(b)
    v_out = torch.empty_like(x)
    default = geom.launch
    p_ms, b_ms = {}, {}
    for u in bands:
        try:
            geom.set_launch(u, default[1], default[2])
        except _lib.CVPError:
            continue                            # band image too large for LDS
        p_ms[u] = _time(lambda: project(x, geom, opts, out=p_out), reps)
        if log:
            log("projection band %d: %.2f ms" % (u, p_ms[u]))
    # with cached records the LDS budget (workgroups per CU) and, for stacks of
    # 8 or 16 columns, one window per workgroup are choices too
    wpcs = (4, 3) if geom.records_cached else (0,)
    for gw in stacks:
        for kp in passes:
            for wpc in wpcs:
                for shw in ((False, True) if geom.records_cached and gw >= 8 else (False,)):
                    try:
                        geom.set_launch(default[0], gw, kp, wpc, shw)
                    except _lib.CVPError:
                        continue
                    b_ms[(gw, kp, wpc, shw)] = _time(lambda: backproject(b, geom, opts, out=v_out), reps)
                    if log:
                        log("backprojection stack %d, %d passes, %d per CU%s: %.2f ms"
                            % (gw, kp, wpc, ", one window" if shw else "", b_ms[(gw, kp, wpc, shw)]))
    best_u = min(p_ms, key=p_ms.get) if p_ms else default[0]
    best_gw, best_kp, best_wpc, best_shw = min(b_ms, key=b_ms.get) if b_ms else (default[1], default[2], 0, False)
    geom.set_launch(best_u, best_gw, best_kp, best_wpc, best_shw)

    def name(k):
        s = "%d/%d/%d" % k[:3] if k[2] else "%d/%d" % k[:2]
        return s + "/s" if k[3] else s
    rec = {"proj_band_cols": best_u, "bp_stack_cols": best_gw, "bp_passes": best_kp, "bp_workgroups_per_cu": best_wpc,
           "bp_shared_window": bool(best_shw), "default": list(default),
           "project_ms": {str(k): v for k, v in p_ms.items()},
           "backproject_ms": {name(k): v for k, v in b_ms.items()}}
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = rec
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(rec, cached=False)
