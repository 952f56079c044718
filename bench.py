#!/usr/bin/env python3
"""Benchmark of the speculative progressive raycasting hot path on one MI355X.

Default workload: the RM-like mixing-layer volume, 2048x2048x1920 samples
(0..255 levels as float32, seed 3), compressed at 2 bits/value
(2,013,265,920 bytes), rendered at 1280x720 with speculation cap 64 and the
decoded-block cache capped at 2*10^9 bytes.  The timed requests visit
isovalues 64, 128 and 192 in turn, each over a 10-position seeded orbit
(the paper's protocol of isovalue changes followed by camera moves), so the
first view of each isovalue finds the cache without its blocks.

One step = one render request from start to finish: the initial rays
(set-up of the request, isovalue masks included), then passes (speculative
traversal, mark, cache update and decode, pair build, block raytrace,
composite, compaction) until every ray has terminated.  The compressed stream
and its macrocell grids are resident in HBM before the timed region starts;
the grid build (load path) is timed on its own (load_ms).

Beside the plain per-request rate (value) the line carries: the same
requests as one batch (render set-up inside both clocks), the 64-request mixed
workload batched against plain, the cold first view, per-kernel times and the
roofline of the dominant kernel, peak memory split by kind, the oracle on the
host cores on a bounded pixel subset, and the paper's figures as context.

Prints one JSON line.  --gpus N with N > 1 is refused: libspr runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s & ms/pass at 1280x720, batched vs plain, same accuracy; blocks decoded/s"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2309_10212_amd/csrc/spr_kernels.hip", "paper_2309_10212_amd/csrc/spr_internal.h",
                  "paper_2309_10212_amd/csrc/spr_launch.h", "paper_2309_10212_amd/csrc/spr_codec.h")
RM_DIMS, RM_RATE, RM_SEED = (2048, 2048, 1920), 2, 3
RM_ISOS = (64.0, 128.0, 192.0)
RM_WARM_ISOS = (96.0, 160.0)      # warm-up requests use other isovalues, so the timed ones start cold
RM_NAME = "rm2048x2048x1920_rate2_1280x720"
TRAFFIC_FILES = {"rm": os.path.join(ROOT, "profiles", f"hbm_traffic_{RM_NAME}.txt"),
                 "fourier": os.path.join(ROOT, "profiles", "hbm_traffic_fourier512_rate4_1280x720.txt")}
PASS_KERNELS = ("k_pass_begin", "k_traverse", "k_dedupe", "k_mark", "k_evict_hist",
                "k_evict", "k_assign_scatter", "k_decode", "k_raytrace", "k_finish", "k_pass_end", "k_compact")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes per kernel, in this library's data layout: every input
# and output byte the kernel must move once (cached re-reads not counted).
# Counts are summed over the timed region:
#   A rays, S pair slots (N_act*N_spec), P pairs, Ps served pairs, V visible
#   blocks, K active blocks, M decoded blocks, R bits/value; per step (load
#   path and request set-up): NB blocks, NC coarse cells, NP pixels.
def kernel_bytes(name, c, rate):
    A, S, P, Ps = c["rays"], c["pair_slots"], c["pairs"], c["served_pairs"]
    V, K, M = c["visible_blocks"], c["active_blocks"], c["blocks_decoded"]
    NB, NC, NP = c["load_blocks"], c["load_coarse"], c["setup_pixels"]
    model = {
        "k_block_ranges": (8 * rate + 8) * NB,     # record in, own range out
        "k_fine_grid": 48 * NB,                    # three in-place axis passes: range in and out each
        "k_coarse_grid": 8 * NB + 8 * NC,          # fine ranges in, coarse range out
        # coarse range in, mask word and distance seed out, the three distance passes (1 B in, 1 B out each);
        # the fine ranges of the coarse cells whose range contains the isovalue (64 blocks each)
        "k_iso_masks": 23 * c.get("mask_coarse", NC) + 8 * c.get("mask_blocks", NB),
        "k_init_rays": 40 * NP,                    # ray state, image, hit record, active entry, pass state
        # active entry + state in; candidate count, slot base and count out; slots written; per coarse cell
        # visited its isovalue-mask word and empty-space distance
        "k_traverse": 20 * A + 4 * S + c.get("coarse_steps", 0) + 8 * c.get("coarse_masks", 0),
        "k_dedupe": 4 * S + 12 * P + 12 * V,
        "k_mark": 52 * V + 12 * K + 8 * M,      # + the 8 neighbour stamps each visible block tests
        "k_assign_scatter": 32 * M + 4 * S + 28 * Ps,
        "k_decode": (8 * rate + 268) * M + 64 * V,   # + each visible block's 8 neighbour slots, read and listed
        # per served pair: sorted entry (12 B), hit t and key (16 B, hits only: an upper bound); per visible
        # block: its 5^3 dual grid once, its 8 slot ids and its list entry
        "k_raytrace": 28 * Ps + 540 * V,
        # per active ray: list entry, candidate count, best key, deferral, slot base and count, and for a hit
        # its t, block, image and hit record, ray state (an upper bound)
        "k_finish": 64 * A,
        "k_compact": 12 * A,
    }
    return model.get(name)


def hbm_fractions(c, rate, steps, ms_per_step, passes, decoded, decode_ms, peak_mem):
    """Each headline figure as a fraction of what HBM alone would allow: the
    step's algorithmic bytes (every kernel's byte model over the step's
    counters) at 8 TB/s is the step time floor; rays/s and ms per pass compare
    against it, blocks decoded/s against 8 TB/s over a decode's bytes per
    block, peak memory against the 288 GB of HBM."""
    names = ("k_block_ranges", "k_fine_grid", "k_coarse_grid", "k_iso_masks", "k_init_rays", "k_traverse", "k_dedupe",
             "k_mark", "k_assign_scatter", "k_decode", "k_raytrace", "k_finish", "k_compact")
    byts = sum(kernel_bytes(k, c, rate) or 0 for k in names) / max(steps, 1)
    t_floor_ms = byts / (HBM_PEAK_GBS * 1e9) * 1e3
    frac_t = t_floor_ms / ms_per_step if ms_per_step > 0 else None
    dec_bytes = 8 * rate + 268
    dec_rate = decoded / (decode_ms / 1e3) if decode_ms else None
    return {"bytes_per_step": round(byts), "step_ms_at_hbm_peak": round(t_floor_ms, 5),
            "rays_per_s_frac": round(frac_t, 5) if frac_t else None,
            "ms_per_pass_at_hbm_peak": round(t_floor_ms / max(passes, 1e-9), 5), "ms_per_pass_frac": round(frac_t, 5) if frac_t else None,
            "blocks_decoded_per_s_at_hbm_peak": round(HBM_PEAK_GBS * 1e9 / dec_bytes, 1),
            "blocks_decoded_per_s_frac": round(dec_rate / (HBM_PEAK_GBS * 1e9 / dec_bytes), 6) if dec_rate else None,
            "peak_mem_frac_of_hbm": round(peak_mem / 288e9, 5),
            "note": "fractions of the HBM-only bound: time at 8 TB/s for the step's algorithmic bytes over the measured "
                    "time; the decode rate over its own kernel time; peak memory over 288 GB"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    the workload (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel
    calibration), or None if there is none for this kernel or the kernel
    sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILES[workload]) as fh:
            kv = dict(line.strip().split("=", 1) for line in fh if "=" in line and not line.startswith("#"))
    except (OSError, KeyError):
        return None
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv[kernel + ".hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline_of(ktimes, counters, rate, workload):
    """Roofline of the dominant kernel (largest device time over the evented
    steps): algorithmic bytes per launch over its average launch time."""
    if not ktimes:
        return None
    dname, (dms, dn) = max(ktimes.items(), key=lambda kv: kv[1][0])
    byts = kernel_bytes(dname, counters, rate)
    if byts is None or dn <= 0 or dms <= 0:
        return None
    per_launch = byts / dn
    avg_s = dms / dn / 1e3
    ach = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 6), "traffic": measured_traffic(dname, workload), "kernel": dname,
            "bytes_per_launch": round(per_launch), "avg_launch_us": round(avg_s * 1e6, 2)}


def calibration_copy(mib):
    """One plain device-to-device copy of mib MiB: the kernel whose
    FETCH_SIZE/WRITE_SIZE counters calibrate the traffic figures."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy: {nbytes} bytes read, {nbytes} bytes written")


def mem_report(split):
    """Peak device memory split by kind (bytes), from spr_mem_split."""
    return {"peak_bytes": split["peak"], "at_peak": split["at_peak"], "kind_peak": split["kind_peak"]}


def _line(metric_value, ms_step, steps, warmup, workload_cfg, extra, dtype="f64"):
    out = {"metric": METRIC, "value": round(metric_value, 1), "unit": "rays/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": workload_cfg}
    out.update(extra)
    print(json.dumps(out), flush=True)


def _cores():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _counter_delta(c0, c1):
    d = {k: c1[k] - c0[k] for k in c1}
    d["max_active_blocks"] = c1["max_active_blocks"]
    return d


def _request(spr, vol, cam, iso, w, h, cap):
    """One render request: set-up (initial rays, isovalue masks) and passes
    to completion; returns its summary."""
    r = spr.Render(vol, cam, iso, w, h, spec_cap=cap)
    r.run()
    info = r.info()
    r.free()
    return info


def _evented(ctx, run):
    """Run `run()` with per-kernel HIP events on the library's stream; returns
    (kernel times, counter delta, wall ms)."""
    import torch
    ctx.profile(True, reset=True)
    c0 = ctx.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    return ctx.kernel_times(), _counter_delta(c0, ctx.counters()), (t1 - t0) * 1e3


# ------------------------------------------------------------- mixed batch --

def mix_leg(args, log_prefix="[bench]"):
    """The batched workload: 64 seeded requests over a pool of 8 volumes
    (blobs and Fourier fields, 128^3..1024^3, float32 or u8 levels, 2/4/8
    bits/value) at mixed image sizes; the autotuner picks the speculation cap
    and the raytrace tuning on a sample; then the 64 requests run as one
    graph-replayed batch and one at a time through the plain path with the
    same settings.  Both clocks include every request's set-up (render
    begin: rays, masks) and stop at the last pass; neither rebuilds grids.
    Each leg runs once untimed, then timed, on a warm cache."""
    import torch
    from paper_2309_10212_amd import autotune, spr
    from volgen import workloads
    t0 = time.perf_counter()
    pool = workloads.make_pool()
    reqs = workloads.make_requests(pool, 64)
    log(f"{log_prefix} pool of {len(pool)} volumes, {len(reqs)} requests ({time.perf_counter() - t0:.1f}s)")
    ctx = spr.Context(device=0, cache_bytes=4 * 10**9, spec_cap=16)
    vols = [ctx.load_volume(p.stream, p.dims, p.rate) for p in pool]
    best, table = autotune.autotune(ctx, vols, reqs, sample=8)
    log(f"{log_prefix} autotuned: {best}")
    for r in autotune.run_batch(ctx, vols, reqs, best.spec_cap, args.poll_every)[3]:
        r.free()
    dt_b, rays_b, passes_b, rs = autotune.run_batch(ctx, vols, reqs, best.spec_cap, args.poll_every)
    for r in rs:
        r.free()

    def plain():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rays = passes = 0
        for q in reqs:
            r = spr.Render(vols[q.vol], q.cam, q.iso, q.w, q.h, spec_cap=best.spec_cap)
            passes += r.run()
            rays += r.info()["rays_entered"]
            r.free()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, rays, passes
    plain()
    dt_p, rays_p, passes_p = plain()
    assert rays_p == rays_b, (rays_p, rays_b)
    split = ctx.mem_split()
    out = {"requests": len(reqs), "pool": [p.name for p in pool], "cache_bytes": 4 * 10**9,
           "batched_rays_per_s": round(rays_b / dt_b, 1), "plain_rays_per_s": round(rays_p / dt_p, 1),
           "vs_plain": round((rays_b / dt_b) / (rays_p / dt_p), 3),
           "batched_ms": round(dt_b * 1e3, 3), "plain_ms": round(dt_p * 1e3, 3),
           "batched_passes": passes_b, "plain_passes": passes_p, "rays_entered": rays_b,
           "timing": "both clocks from the first render set-up to the last pass, warm cache, no grid rebuild",
           "tuning": {"spec_cap": best.spec_cap, "pairs_per_wg": best.pairs_per_wg, "slot_tile": best.slot_tile},
           "autotune_table": [{"spec_cap": c.spec_cap, "pairs_per_wg": c.pairs_per_wg, "slot_tile": c.slot_tile,
                               "rays_per_s": round(c.rays_per_s, 1)} for c in table],
           "peak_mem": mem_report(split)}
    for v in vols:
        v.free()
    ctx.close()
    return out


# ------------------------------------------------------- RM-like (default) --

def rm_requests(n):
    """Request i of the RM-like workload: isovalue-major, 10 orbit views per
    isovalue (view i mod 10, isovalue (i div 10) mod 3)."""
    import volgen
    cams = [volgen.orbit_camera(*RM_DIMS, seed=RM_SEED, k=k, npos=10) for k in range(10)]
    return [(cams[i % 10], RM_ISOS[(i // 10) % 3], i % 10) for i in range(n)]


def rm_warm_requests(n):
    import volgen
    cams = [volgen.orbit_camera(*RM_DIMS, seed=RM_SEED, k=k, npos=10) for k in range(10)]
    return [(cams[(3 * i + 1) % 10], RM_WARM_ISOS[i % 2], (3 * i + 1) % 10) for i in range(n)]


def rm_cpu_baseline(args, stream, reqs):
    """The oracle's streamed march (blocks decoded on demand, the decoded
    volume is never materialised) on every 8th row and column of the timed
    requests, in order, until --cpu-seconds have passed (bounded sample)."""
    import numpy as np
    import oracle
    w, h = args.w, args.h
    ys, xs = np.meshgrid(np.arange(0, h, 8), np.arange(0, w, 8), indexing="ij")
    pix = (ys * w + xs).astype(np.uint32).ravel()
    entered = hits = done = 0
    t0 = time.perf_counter()
    for cam, iso, k in reqs:
        r = oracle.render_stream(stream, RM_DIMS, RM_RATE, cam, iso, w, h, pixels=pix)
        entered += int(r["entered"].sum())
        hits += int(np.isfinite(r["t"]).sum())
        done += 1
        if time.perf_counter() - t0 >= args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": round(entered / dt, 1), "unit": "rays/s", "cores": _cores(), "kind": "oracle",
            "sample": f"{done} of the timed requests, every 8th row and column ({len(pix)} pixels each, {entered} rays "
                      f"entered, {dt:.1f} s), the oracle's march over every dual cell with blocks decoded on demand",
            "render_s": round(dt, 3), "requests": done, "hits": hits}


def run_rm(args):
    """The headline line (see the module docstring)."""
    import numpy as np
    import torch
    import volgen
    from paper_2309_10212_amd import spr
    w, h, cap = args.w, args.h, 64
    t0 = time.perf_counter()
    stream = volgen.rm_encode(*RM_DIMS, RM_RATE, seed=RM_SEED)
    log(f"[bench] RM-like stream {stream.nbytes} B in {time.perf_counter() - t0:.1f}s")
    steps, warmup = args.steps, args.warmup
    reqs = rm_requests(steps)
    warm = rm_warm_requests(warmup)
    ctx = spr.Context(device=0, cache_bytes=2 * 10**9, spec_cap=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vol = ctx.load_volume(stream, RM_DIMS, RM_RATE)     # upload + grids (a0)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    vol.build_grids()
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - t0) * 1e3
    mem_load = ctx.mem_split(reset_peak=True)

    def fresh_volume():
        nonlocal vol
        vol.free()
        vol = ctx.load_volume(stream, RM_DIMS, RM_RATE)
        torch.cuda.synchronize()

    # warm-up on other isovalues (graph capture, allocator), then the cold
    # first view: the first timed request, alone, on a cache without its blocks
    for cam, iso, _ in warm:
        _request(spr, vol, cam, iso, w, h, cap)
    torch.cuda.synchronize()
    ctx.mem_split(reset_peak=True)
    c0 = ctx.counters()
    t0 = time.perf_counter()
    info0 = _request(spr, vol, *reqs[0][:2], w, h, cap)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1e3
    dcold = _counter_delta(c0, ctx.counters())
    mem_cold = ctx.mem_split()
    cold = {"ms": round(cold_ms, 4), "passes": info0["passes"], "rays_entered": info0["rays_entered"],
            "rays_per_s": round(info0["rays_entered"] / (cold_ms / 1e3), 1),
            "ms_per_pass": round(cold_ms / max(info0["passes"], 1), 4),
            "blocks_decoded": dcold["blocks_decoded"], "active_blocks_max": dcold["max_active_blocks"],
            "bcmc_blocks": info0["bcmc_blocks"],
            "bcmc_decoded_ratio": round(info0["bcmc_blocks"] / max(dcold["blocks_decoded"], 1), 2),
            "peak_mem": mem_report(mem_cold),
            "note": "the first timed request (isovalue 64, view 0) alone, after warm-up requests at other isovalues"}
    log(f"[bench] cold first view: {cold}")

    # timed region: the plain path, one request after another, graph-replayed
    # passes, no per-kernel events; the cache restarts from the same state
    fresh_volume()
    for cam, iso, _ in warm:
        _request(spr, vol, cam, iso, w, h, cap)
    if args.calib_copy_mib > 0:
        calibration_copy(args.calib_copy_mib)
    ctx.mem_split(reset_peak=True)
    c0 = ctx.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [_request(spr, vol, cam, iso, w, h, cap) for cam, iso, _ in reqs]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dc = _counter_delta(c0, ctx.counters())
    mem_steps = ctx.mem_split()
    rays = sum(i["rays_entered"] for i in infos)
    passes = sum(i["passes"] for i in infos)
    value = rays / el
    nb_vol = (RM_DIMS[0] // 4) * (RM_DIMS[1] // 4) * (RM_DIMS[2] // 4)
    nc_vol = ((RM_DIMS[0] // 4 + 3) // 4) * ((RM_DIMS[1] // 4 + 3) // 4) * ((RM_DIMS[2] // 4 + 3) // 4)
    # masks are built by the requests that found no kept set for their isovalue
    built = [i for i in infos if i["masks_built"]]
    extra_counts = {"load_blocks": 0, "load_coarse": 0, "mask_coarse": nc_vol * len(built),
                    "mask_blocks": 64 * sum(i["iso_coarse_cells"] for i in built),
                    "setup_pixels": w * h * steps}
    dc.update(extra_counts)
    log(f"[bench] plain: {steps} requests, {value / 1e6:.1f} M rays/s, {el * 1e3 / steps:.3f} ms per request, "
        f"{passes / steps:.2f} passes")

    # the same requests with per-ray speculation counts (plain path, the same
    # cache state): the policy changes passes and work, never the image
    per_ray = None
    if not args.no_per_ray:
        fresh_volume()
        for cam, iso, _ in warm:
            _request(spr, vol, cam, iso, w, h, cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pinfos = []
        for cam, iso, _ in reqs:
            r = spr.Render(vol, cam, iso, w, h, spec_cap=cap, policy=spr.SPEC_PER_RAY)
            r.run()
            pinfos.append(r.info())
            r.free()
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        prays = sum(i["rays_entered"] for i in pinfos)
        ppass = sum(i["passes"] for i in pinfos)
        assert prays == rays, (prays, rays)
        per_ray = {"rays_per_s": round(prays / pel, 1), "ms_per_step": round(pel * 1e3 / steps, 4),
                   "passes_per_step": ppass / steps, "ms_per_pass": round(pel * 1e3 / max(ppass, 1), 4),
                   "pairs_per_step": round(sum(i["pairs"] for i in pinfos) / steps, 1),
                   "uniform_pairs_per_step": round(sum(i["pairs"] for i in infos) / steps, 1),
                   "vs_uniform": round((prays / pel) / value, 3),
                   "rule": "n_i = min(64, 1 + floor((w*h - N_act) w_i / W)), w_i = 1 + floor(remaining path / 4)"}
        log(f"[bench] per-ray speculation: {per_ray}")

    # the same requests as one batch: one replayed pass advances all of them;
    # the clock starts before the first render set-up, as for the plain path
    batched = None
    if args.batch_reps > 0:
        brates = []
        for rep in range(args.batch_reps):
            fresh_volume()
            for cam, iso, _ in warm:
                _request(spr, vol, cam, iso, w, h, cap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = [spr.Render(vol, cam, iso, w, h, spec_cap=cap) for cam, iso, _ in reqs]
            b = spr.Batch(ctx, rs)
            npass = b.run(poll_every=args.poll_every)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rb = sum(r.info()["rays_entered"] for r in rs)
            b.free()
            for r in rs:
                r.free()
            assert rb == rays, (rb, rays)
            brates.append((rb / dt, dt, npass))
        bv, bdt, bpass = max(brates)
        batched = {"requests": steps, "reps": args.batch_reps, "rays_per_s": round(bv, 1),
                   "rays_per_s_all_reps": [round(x[0], 1) for x in brates],
                   "ms_per_batch": round(bdt * 1e3, 3), "passes": bpass, "ms_per_pass": round(bdt * 1e3 / max(bpass, 1), 4),
                   "plain_rays_per_s": round(value, 1), "vs_plain": round(bv / value, 3),
                   "timing": "from the first render set-up to the last pass, the cache in the same state as for the "
                             "plain leg (fresh volume, the same warm-up); best of reps"}
        log(f"[bench] batched: {batched}")

    # per-kernel times: the same steps again with HIP events around every
    # kernel (eager launches), from the same cache state
    ktimes, dcp, prof_ms = {}, dc, None
    if not args.no_profile:
        fresh_volume()
        for cam, iso, _ in warm:
            _request(spr, vol, cam, iso, w, h, cap)
        ktimes, dcp, prof_ms = _evented(ctx, lambda: [_request(spr, vol, cam, iso, w, h, cap) for cam, iso, _ in reqs])
        dcp.update(extra_counts)
        if dcp["blocks_decoded"] != dc["blocks_decoded"] or dcp["pairs"] != dc["pairs"]:
            log(f"[bench] note: the evented steps did other work (decoded {dcp['blocks_decoded']} vs "
                f"{dc['blocks_decoded']}, pairs {dcp['pairs']} vs {dc['pairs']})")
        log("[bench] device ms per step by kernel: " + ", ".join(
            f"{k} {ms / steps:.3f} ({nl})" for k, (ms, nl) in sorted(ktimes.items(), key=lambda kv: -kv[1][0])[:9]))
    dev_ms = sum(ktimes[k][0] for k in PASS_KERNELS if k in ktimes)
    dev_ms_all = sum(ms for ms, _ in ktimes.values())
    dec_ms = ktimes.get("k_decode", (0.0, 0))[0]
    roof = roofline_of(ktimes, dcp, RM_RATE, "rm")

    # load-path decode rate (every block once, k_block_ranges) from one evented grid build
    load_decode = None
    if not args.no_profile:
        lt, _, _ = _evented(ctx, vol.build_grids)
        lms = lt.get("k_block_ranges", (0.0, 0))[0]
        if lms > 0:
            load_decode = {"blocks": nb_vol, "ms": round(lms, 4), "blocks_per_s": round(nb_vol / (lms / 1e3), 1),
                           "frac_of_hbm_decode_bound": round(nb_vol / (lms / 1e3) / (HBM_PEAK_GBS * 1e9 / (8 * RM_RATE + 8)), 5),
                           "grid_ms": {k: round(v[0], 4) for k, v in lt.items()}}

    mix = None
    if not args.no_mix:
        mix = mix_leg(args)
        log(f"[bench] mixed workload: {mix['batched_rays_per_s'] / 1e6:.1f} M rays/s batched, "
            f"{mix['plain_rays_per_s'] / 1e6:.1f} M plain")

    cpu = None
    if not args.no_cpu:
        cpu = rm_cpu_baseline(args, stream, reqs)
        log(f"[bench] cpu baseline: {cpu}")

    bcmc = sum(i["bcmc_blocks"] for i in infos) / len(infos)
    ms_step = el * 1e3 / steps
    _line(value, ms_step, steps, warmup,
          {"workload": f"{RM_NAME}_cap64", "volume": "RM-like mixing layer 2048x2048x1920, levels 0..255 as float32, "
                                                   "2 bits/value (seed 3)",
           "image": f"{w}x{h}", "isovalues": list(RM_ISOS), "views": "10-position seeded orbit per isovalue",
           "spec_cap": cap, "cache_bytes": 2 * 10**9,
           "step": "one render request to completion (set-up + passes); grids built once at load"},
          {"ms_per_pass": round(el * 1e3 / max(passes, 1), 4), "passes_per_step": passes / steps,
           "device_ms_per_pass": round(dev_ms / max(passes, 1), 4) if ktimes else None,
           "device_ms_per_step": round(dev_ms_all / steps, 4) if ktimes else None,
           "evented_ms_per_step": round(prof_ms / steps, 4) if prof_ms is not None else None,
           "cold_first_view": cold,
           "blocks_decoded_per_s": round(dc["blocks_decoded"] / el, 1),
           "blocks_decoded_per_decode_s": round(dc["blocks_decoded"] / (dec_ms / 1e3), 1) if dec_ms > 0 else None,
           "load_ms": round(load_ms, 3), "upload_and_load_ms": round(upload_ms, 3), "load_path_decode": load_decode,
           "peak_mem": {"whole_run": mem_report(ctx.mem_split()), "after_load": mem_report(mem_load),
                        "timed_steps": mem_report(mem_steps)},
           "peak_mem_bytes": ctx.mem_split()["peak"],
           "counters": dc,
           "kernels_ms_per_launch": {k: round(ms / max(nl, 1), 5) for k, (ms, nl) in ktimes.items()},
           "roofline": roof,
           "hbm_roofline": hbm_fractions(dc, RM_RATE, steps, ms_step, passes / steps, dcp["blocks_decoded"], dec_ms,
                                         mem_steps["peak"]),
           "batched": batched,
           "batched_mix": mix,
           "per_ray_speculation": per_ray,
           "bcmc_proxy": {"blocks_per_request": round(bcmc, 1),
                          "decoded_blocks_per_request": round(dc["blocks_decoded"] / steps, 1),
                          "decoded_ratio": round(bcmc * steps / max(dc["blocks_decoded"], 1), 2),
                          "cold_first_view_ratio": cold["bcmc_decoded_ratio"],
                          "bytes": int(bcmc * 256), "cache_bytes_needed": int(dc["max_active_blocks"] * 256),
                          "note": "blocks whose fine range contains the isovalue (what decompressing every block that "
                                  "may hold the surface decodes) vs blocks decoded; the timed requests change isovalue "
                                  "every 10 views, so each isovalue's first view decodes its blocks"},
           "paper": {"ms_per_pass": 264.0, "s_per_request": 1.2, "passes_per_request_derived": 4.5,
                     "total_mem_bytes": 4.19e9,
                     "hardware": "RTX 3080 (12 GB), WebGPU compute shaders",
                     "data": "R-M 2048x2048x1920 uint8 as float32, zfp fixed rate (rate not stated), 1280x720",
                     "this_build": {"ms_per_pass": round(el * 1e3 / max(passes, 1), 4), "s_per_request": round(ms_step / 1e3, 6)},
                     "note": "context, not a target: other hardware, another codec and the paper's data set; this "
                             "line renders a synthetic RM-like stand-in at 2 bits/value"},
           "cpu_baseline": cpu})
    vol.free()
    ctx.close()


# ------------------------------------------------------- Fourier 512^3 ------

def make_inputs(args):
    import volgen
    n = args.n
    t0 = time.perf_counter()
    field = volgen.fourier(n, n, n, seed=2, nmode=64, kmax=24, period=float(n))
    iso = volgen.percentile_value(field, 0.6)
    stream = volgen.encode(field, args.rate)
    log(f"[bench] inputs: {n}^3 fourier, rate {args.rate}, iso {iso:.6g}, {stream.nbytes / 2**20:.1f} MiB "
        f"({time.perf_counter() - t0:.1f}s)")
    cams = [volgen.orbit_camera(n, n, n, seed=2, k=k, npos=10) for k in range(10)]
    return field, stream, iso, cams


def cpu_baseline(args, stream, iso, cams):
    """The oracle as it stands, timed on this host on the orbit of the workload
    (10 views at full resolution) after one whole-volume decode.  The orbit is
    repeated until the renders have taken --cpu-seconds (at most 100 times),
    a bounded sample."""
    import numpy as np
    import oracle
    n = args.n
    t0 = time.perf_counter()
    dec = oracle.decode_volume(stream, (n, n, n), args.rate)
    t_dec = time.perf_counter() - t0
    views = cams[: args.cpu_views]
    entered = hits = reps = 0
    t0 = time.perf_counter()
    while reps < 100:
        for cam in views:
            r = oracle.render(dec, cam, iso, args.w, args.h)
            entered += int(r["entered"].sum())
            hits += int(np.isfinite(r["t"]).sum())
        reps += 1
        if time.perf_counter() - t0 >= args.cpu_seconds:
            break
    t_r = time.perf_counter() - t0
    nblk = ((n + 3) // 4) ** 3
    return {"value": round(entered / t_r, 1), "unit": "rays/s", "cores": _cores(), "kind": "oracle",
            "sample": f"{reps} x {len(views)} orbit views at {args.w}x{args.h} ({entered} rays entered, "
                      f"{t_r:.1f} s), after one whole-volume decode timed separately",
            "render_s": round(t_r, 3), "decode_s": round(t_dec, 3), "decode_blocks_per_s": round(nblk / t_dec, 1),
            "hits": hits}


def run_fourier(args):
    """512^3 Fourier field at 4 bits/value, 1280x720, 60th-percentile
    isovalue, 10-position orbit, cache 512*10^6 B, speculation cap 16 (with
    a sweep of caps).  One step = one orbit view (set-up + passes); grids
    built once at load."""
    import torch
    from paper_2309_10212_amd import spr
    field, stream, iso, cams = make_inputs(args)
    del field
    n = args.n
    ctx = spr.Context(device=0, cache_bytes=args.cache_bytes, spec_cap=args.spec_cap)
    vol = ctx.load_volume(stream, (n, n, n), args.rate)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vol.build_grids()
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - t0) * 1e3

    def step(k, cap):
        return _request(spr, vol, cams[k % len(cams)], iso, args.w, args.h, cap)

    for i in range(args.warmup):
        step(i, args.spec_cap)
    if args.calib_copy_mib > 0:
        calibration_copy(args.calib_copy_mib)
    c0 = ctx.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(args.warmup + i, args.spec_cap) for i in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dc = _counter_delta(c0, ctx.counters())
    built = [i for i in infos if i["masks_built"]]
    dc.update({"load_blocks": 0, "load_coarse": 0, "setup_pixels": args.w * args.h * args.steps,
               "mask_blocks": 64 * sum(i["iso_coarse_cells"] for i in built),
               "mask_coarse": ((((n + 3) // 4) + 3) // 4) ** 3 * len(built)})
    ktimes, dcp, prof_ms = {}, dc, None
    if not args.no_profile:
        vol.free()
        vol = ctx.load_volume(stream, (n, n, n), args.rate)
        for i in range(args.warmup):
            step(i, args.spec_cap)
        ktimes, dcp, prof_ms = _evented(ctx, lambda: [step(args.warmup + i, args.spec_cap) for i in range(args.steps)])
        for k in ("load_blocks", "load_coarse", "setup_pixels", "mask_blocks", "mask_coarse"):
            dcp[k] = dc[k]
    rays = sum(i["rays_entered"] for i in infos)
    passes = sum(i["passes"] for i in infos)
    value = rays / el
    dec_ms = ktimes.get("k_decode", (0.0, 0))[0]
    roof = roofline_of(ktimes, dcp, args.rate, "fourier")
    sweep = []
    if args.sweep:
        for cap in [int(x) for x in args.sweep.split(",") if x]:
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            inf = [step(k, cap) for k in range(len(cams))]
            torch.cuda.synchronize()
            s1 = time.perf_counter()
            rr = sum(i["rays_entered"] for i in inf)
            pp = sum(i["passes"] for i in inf)
            sweep.append({"spec_cap": cap, "rays_per_s": round(rr / (s1 - s0)), "passes_per_view": pp / len(inf),
                          "ms_per_pass": round((s1 - s0) * 1e3 / pp, 4), "ms_per_view": round((s1 - s0) * 1e3 / len(inf), 3),
                          "utilization": round(sum(i["pairs"] for i in inf) / (pp * args.w * args.h), 4)})
            log(f"[bench] sweep cap {cap}: {sweep[-1]}")
    batched = None
    if args.batch_reps > 0:
        def batch_run():
            rs = [spr.Render(vol, cam, iso, args.w, args.h, spec_cap=args.spec_cap) for cam in cams]
            b = spr.Batch(ctx, rs)
            npass = b.run(poll_every=args.poll_every)
            infos_b = [r.info() for r in rs]
            b.free()
            for r in rs:
                r.free()
            return npass, infos_b

        def plain_run():
            return [step(k, args.spec_cap) for k in range(len(cams))]
        batch_run()
        plain_run()
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        tot_rays = tot_passes = 0
        for _ in range(args.batch_reps):
            npass, inf = batch_run()
            tot_rays += sum(i["rays_entered"] for i in inf)
            tot_passes += npass
        torch.cuda.synchronize()
        b1 = time.perf_counter()
        p_rays = 0
        for _ in range(args.batch_reps):
            p_rays += sum(i["rays_entered"] for i in plain_run())
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        brate, prate = tot_rays / (b1 - b0), p_rays / (p1 - b1)
        batched = {"requests": len(cams), "reps": args.batch_reps, "rays_per_s": round(brate, 1),
                   "plain_rays_per_s": round(prate, 1), "vs_plain": round(brate / prate, 3),
                   "ms_per_batch": round((b1 - b0) * 1e3 / args.batch_reps, 3),
                   "passes_per_batch": tot_passes / args.batch_reps,
                   "timing": "the 10 orbit views as one batch vs one at a time, both from render set-up to the last "
                             "pass, warm cache, no grid rebuild"}
        log(f"[bench] batched: {batched}")
    split = ctx.mem_split()
    cpu = None if args.no_cpu else cpu_baseline(args, stream, iso, cams)
    ms_step = el * 1e3 / args.steps
    _line(value, ms_step, args.steps, args.warmup,
          {"workload": f"fourier{n}_rate{args.rate}_{args.w}x{args.h}_cap{args.spec_cap}",
           "volume": f"{n}^3 float32, 64 Fourier modes |k|^-5/3 (seed 2), {args.rate} bits/value",
           "image": f"{args.w}x{args.h}", "isovalue": "60th percentile of the field",
           "spec_cap": args.spec_cap, "cache_bytes": args.cache_bytes,
           "step": "one orbit view to completion (set-up + passes); grids built once at load"},
          {"ms_per_pass": round(el * 1e3 / max(passes, 1), 4), "passes_per_step": passes / args.steps,
           "device_ms_per_pass": round(sum(ktimes[k][0] for k in PASS_KERNELS if k in ktimes) / max(passes, 1), 4)
           if ktimes else None,
           "evented_ms_per_step": round(prof_ms / args.steps, 4) if prof_ms is not None else None,
           "blocks_decoded_per_s": round(dc["blocks_decoded"] / el, 1),
           "blocks_decoded_per_decode_s": round(dc["blocks_decoded"] / (dec_ms / 1e3), 1) if dec_ms > 0 else None,
           "load_ms": round(load_ms, 4), "peak_mem": mem_report(split), "peak_mem_bytes": split["peak"],
           "counters": dc, "kernels_ms_per_launch": {k: round(ms / max(nl, 1), 5) for k, (ms, nl) in ktimes.items()},
           "roofline": roof,
           "hbm_roofline": hbm_fractions(dc, args.rate, args.steps, ms_step, passes / args.steps,
                                         dcp["blocks_decoded"], dec_ms, split["peak"]),
           "batched": batched, "sweep": sweep, "cpu_baseline": cpu})
    vol.free()
    ctx.close()


def run_batched(args):
    """The 64-request mixed workload on its own line (see mix_leg)."""
    m = mix_leg(args)
    _line(m["batched_rays_per_s"], m["batched_ms"], 1, 1,
          {"workload": "batched64_pool8_autotuned", "requests": m["requests"], "pool": m["pool"],
           "cache_bytes": m["cache_bytes"], "step": "the 64 requests as one batch, from the first render set-up to "
                                                    "the last pass"},
          {k: v for k, v in m.items() if k not in ("requests", "pool", "cache_bytes")} |
          {"roofline": None, "cpu_baseline": None})


def run_serving(args):
    """Serving: Poisson arrivals (lambda = 200/s over --serve-seconds, seed 7)
    of orbit-step (70%) and isovalue-change (30%) requests at 1280x720 or
    1920x1080 over three resident volumes (the 512^3 Fourier field at 4
    bits/value, a 1024^3 Fourier field, seed 4, at 4 bits/value, and the
    2048x2048x1920 RM-like volume at 2 bits/value), one shared 4*10^9-byte
    cache, continuous batching with admission by cache memory."""
    import torch
    import volgen
    from paper_2309_10212_amd import serve, spr
    from volgen import workloads
    t0 = time.perf_counter()
    f1 = volgen.fourier(512, 512, 512, seed=2, nmode=64, kmax=24, period=512.0)
    r1 = (volgen.percentile_value(f1, 0.1), volgen.percentile_value(f1, 0.9))
    s1 = volgen.encode(f1, 4)
    del f1
    f2 = volgen.fourier(1024, 1024, 1024, seed=4, nmode=64, kmax=24, period=1024.0)
    r2 = (volgen.percentile_value(f2, 0.1), volgen.percentile_value(f2, 0.9))
    s2 = volgen.encode(f2, 4)
    del f2
    s3 = volgen.rm_encode(2048, 2048, 1920, 2, seed=3)
    dims = [(512, 512, 512), (1024, 1024, 1024), (2048, 2048, 1920)]
    arr = workloads.serving_arrivals(dims, [r1, r2, (64.0, 192.0)], lam=200.0, span_s=args.serve_seconds, seed=7)
    log(f"[bench] serving inputs and {len(arr)} arrivals ({time.perf_counter() - t0:.1f}s)")
    ctx = spr.Context(device=0, cache_bytes=4 * 10**9, spec_cap=16)
    vols = [ctx.load_volume(s, d, r) for s, d, r in zip((s1, s2, s3), dims, (4, 4, 2))]
    torch.cuda.synchronize()
    srv = serve.Server(ctx, vols, cache_bytes=4 * 10**9, max_requests=32)
    # warm-up: a short stream before the measured one
    warm = workloads.serving_arrivals(dims, [r1, r2, (64.0, 192.0)], lam=200.0, span_s=1.0, seed=8)
    srv.run(warm)
    results, st = srv.run(arr)
    cur, peak = ctx.mem_stats()
    _line(st["rays_per_s"], st["makespan_s"] * 1e3, 1, 1,
          {"workload": f"serving_poisson200_{args.serve_seconds:g}s_3vol", "arrivals": len(arr), "lambda_per_s": 200.0,
           "volumes": ["fourier512_rate4", "fourier1024_rate4", "rm2048x2048x1920_rate2"], "cache_bytes": 4 * 10**9,
           "images": "1280x720 / 1920x1080 (50/50)", "mix": "70% orbit step, 30% isovalue change",
           "step": "the whole arrival stream, first arrival to last completion"},
          {"pass_latency_ms_p50": round(st["pass_latency_ms_p50"], 3), "pass_latency_ms_p99": round(st["pass_latency_ms_p99"], 3),
           "request_latency_ms_p50": round(st["request_latency_ms_p50"], 3), "max_concurrent": st["max_concurrent"],
           "batched_passes": st["passes"], "makespan_s": round(st["makespan_s"], 3),
           "peak_mem_bytes": peak, "roofline": None, "cpu_baseline": None})
    srv.close()
    for v in vols:
        v.free()
    ctx.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="timed requests (default: 3 isovalues x 10 views)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rm", choices=("rm", "fourier", "batched", "serving"),
                    help="rm (default: the headline line, 2048x2048x1920 RM-like), fourier (512^3 Fourier field), "
                         "batched (64 mixed requests, autotuned) or serving (Poisson arrivals, continuous batching)")
    ap.add_argument("--w", type=int, default=1280)
    ap.add_argument("--h", type=int, default=720)
    ap.add_argument("--n", type=int, default=512, help="fourier: samples per axis")
    ap.add_argument("--rate", type=int, default=4, help="fourier: bits per value")
    ap.add_argument("--spec-cap", type=int, default=16, help="fourier: speculation cap")
    ap.add_argument("--cache-bytes", type=int, default=512 * 10**6, help="fourier: cache capacity")
    ap.add_argument("--sweep", default="1,2,4,8,16", help="fourier: speculation caps for the sweep ('' = none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mix", action="store_true", help="rm: skip the 64-request mixed batched-vs-plain leg")
    ap.add_argument("--no-per-ray", action="store_true", help="rm: skip the per-ray speculation leg")
    ap.add_argument("--cpu-views", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="bound on the oracle's timed work (the sample stops after the request that crosses it)")
    ap.add_argument("--no-profile", action="store_true", help="no evented (per-kernel) rerun of the timed steps")
    ap.add_argument("--batch-reps", type=int, default=2, help="repetitions of the batched leg (0 = skip)")
    ap.add_argument("--poll-every", type=int, default=2)
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="length of the serving arrival stream")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, copy this many MiB device to device once (the plain copy "
                         "kernel that calibrates the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "libspr runs on exactly one GPU; --gpus N > 1 is not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    {"rm": run_rm, "fourier": run_fourier, "batched": run_batched, "serving": run_serving}[args.workload](args)


if __name__ == "__main__":
    main()
