#!/usr/bin/env python3
"""Benchmark of the whole hot path (Alg. 1: census, support matching, triangulation,
interpolation, validation/refinement, resampling) on one MI355X.

One step = one ``sm_solve`` of one 640x480 synthetic frame (20 slanted planes with
occlusions and untextured patches; 7x7 census, disparities 0-127, 3 iterations).
Frames are generated up front, uploaded once and stay resident in HBM; the timed
region covers exactly ``--steps`` solves, bracketed by device synchronisations.

Prints ONE JSON line. Besides frames/s it reports validated Mpx/s (frames whose
outputs were compared bit for bit with the CPU oracle), per-step latency
percentiles, per-kernel device time from HIP events recorded on the solve's stream
during the timed region, the roofline position of the dominant kernel, and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "VGA frames/sec + validated Mpx/s at 1 GPU; p50/p99 latency in 16-stream serving"

# MI355X peaks used for the roofline (published figures; integer VALU derived from
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz).
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 39.32 T int32 lane-ops/s

KERNEL_SOURCES = [os.path.join(ROOT, "paper_1511_00758_amd", "csrc", f)
                  for f in ("kernels.hip", "kernels.hpp", "star.hip", "star.hpp", "mesh_star.hpp", "predicates.hpp",
                            "raster.hpp")]


def progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_work(kernel, W, H, p, n_iters, launches, stats=None):
    """Algorithmic work of ONE launch of ``kernel`` on a W x H frame (average over the
    launches of one solve), as (bound, amount, unit_scale, unit, per_unit_note)."""
    npx = W * H
    if kernel == "mesh":
        # one tessellation (preparation + star kernel): the supports read (8 B each), the
        # triangles written (12 B each) and D_it, which the star kernel's workgroups write as
        # they rasterise their triangles (4 B per pixel: an upper bound, covered pixels only).
        # The bucket grid the preparation writes and the star kernel reads back is the
        # method's own overhead, not counted; the star kernel is bound by the latency of its
        # gathers, so the fraction of HBM peak is small
        if not stats:
            return None
        per = [8.0 * stats["n_support"][k] + 12.0 * stats["n_tris"][k] + 4.0 * npx for k in range(n_iters)]
        amount = sum(per) / len(per)
        return "hbm", amount, 1e9, "GB/s", (f"mean over tessellations 1..{n_iters}: 8 B x supports + "
                                            f"12 B x triangles + 4 B x {npx} px (D_it) = {amount / 1e3:.1f} kB")
    bits = p["census_w"] * p["census_h"] - 1
    if kernel == "census":
        # 2 images x (1 B read + 8 B census word written) -- but compute-bound:
        # 3 integer ops (compare, shift/select, or) per census bit per pixel per image
        return "alu", 2 * npx * 3 * bits, 1e12, "TOP/s", f"2 images x {npx} px x 3 ops x {bits} bits"
    if kernel == "validate":
        # per pixel: D_it 4 + cL 8 + cR 8 + Omega 1 + C_f 1 read; C_f 1 + D_f 4 written
        # (C_it is not stored by the solver); the last iteration also writes the 1 B mask
        per_px = 27.0 + 1.0 / n_iters
        return "hbm", npx * per_px, 1e9, "GB/s", f"{npx} px x {per_px:.2f} B"
    if kernel in ("nan_fill",):
        return "hbm", npx * 4.0, 1e9, "GB/s", f"{npx} px x 4 B"
    if kernel == "raster":
        return "hbm", npx * 4.0, 1e9, "GB/s", f"{npx} px x 4 B (upper bound: covered px only)"
    return None


def roofline_for(kernel, avg_us, W, H, p, n_iters, launches, traffic=None, stats=None):
    work = algorithmic_work(kernel, W, H, p, n_iters, launches, stats)
    if work is None or avg_us <= 0:
        return None
    bound, amount, scale, unit, note = work
    achieved = amount / (avg_us * 1e-6) / scale
    peak = PEAK_HBM_GBS if bound == "hbm" else PEAK_VALU_TOPS
    return {"kernel": kernel, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
            "avg_launch_us": round(avg_us, 3), "algorithmic_per_launch": note}


def load_traffic(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), only if taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def _cpu_worker(job):
    """One CPU-baseline job in a worker process that imports only the oracle and the
    scene generator, single-threaded. ("serial", seeds): every (config, frame) of the
    list solved one after another, each timed per stage; ("timed", cfg, frame): one frame,
    returning its start and end on the shared monotonic clock."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    import oracle
    import scenes
    if job[0] == "warm":
        time.sleep(0.3)
        return os.getpid()
    if job[0] == "timed":
        _, cfg, f = job
        sc = scenes.make_scene(cfg, scenes.seed_of(cfg, f))
        p = oracle.Params.from_dict(sc.params)
        t0 = time.perf_counter()
        oracle.solve(sc.left, sc.right, p)
        return t0, time.perf_counter(), os.getpid()
    out = []
    for cfg, f in job[1]:
        sc = scenes.make_scene(cfg, scenes.seed_of(cfg, f))
        p = oracle.Params.from_dict(sc.params)
        times = {}
        t0 = time.perf_counter()
        ref = oracle.solve(sc.left, sc.right, p, times=times)
        dt = time.perf_counter() - t0
        keep = (ref["D_f"], ref["C_f"], ref["mask"]) if cfg == 2 else None
        out.append((cfg, f, sc.left.shape, dt, times, keep))
    return out


def cpu_baseline(seeds_per_config=5, workers=None):
    """The oracle on the host cores, before any GPU work: (i) single-core latency per frame
    and per stage for >= 5 seeds of each single-frame workload (320x240, 640x480,
    1242x375), solved one after another in one worker process; (ii) throughput of N
    worker processes (N = host cores, at most 16) each solving a distinct 640x480 frame at
    once. Returns the record and the oracle outputs of 640x480 frames 0..seeds-1 (for the
    GPU parity check of the same frames)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    import platform
    nproc = os.cpu_count() or 1
    n = workers or min(nproc, 16)
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=1, mp_context=ctx) as ex:
        serial = ex.submit(_cpu_worker, ("serial", [(c, f) for c in (1, 2, 3) for f in range(seeds_per_config)])).result()
    single, refs = {}, {}
    for cfg in (1, 2, 3):
        rows = [r for r in serial if r[0] == cfg]
        ms = np.array([r[3] for r in rows]) * 1e3
        stages = {}
        for r in rows:
            for k, v in r[4].items():
                stages[k] = stages.get(k, 0.0) + v * 1e3 / len(rows)
        H, W = rows[0][2]
        single[f"{W}x{H}"] = {"frames": len(rows), "seeds": [1000 * cfg + r[1] for r in rows],
                              "ms_per_frame": {"mean": round(float(ms.mean()), 1), "p50": round(float(np.median(ms)), 1),
                                               "max": round(float(ms.max()), 1)},
                              "frames_per_s": round(1e3 / float(ms.mean()), 3),
                              "stage_ms_per_frame": {k: round(v, 1) for k, v in stages.items()}}
        if cfg == 2:
            refs = {r[1]: r[5] for r in rows}
    with cf.ProcessPoolExecutor(max_workers=n, mp_context=ctx) as ex:
        list(ex.map(_cpu_worker, [("warm",)] * (2 * n)))       # start and import in every worker
        spans = list(ex.map(_cpu_worker, [("timed", 2, 100 + i) for i in range(n)]))
    t0 = min(sp[0] for sp in spans)
    t1 = max(sp[1] for sp in spans)
    fps = n / (t1 - t0)
    rec = {"value": round(fps, 4), "unit": "frames/s", "cores": n, "kind": "oracle",
           "sample": (f"640x480 workload: {n} worker processes, one thread each, solving {n} distinct "
                      f"frames (seeds 2100..{2099 + n}) at once in {t1 - t0:.1f} s; single-core latencies "
                      f"below over {seeds_per_config} seeds of each single-frame workload"),
           "mpx_per_s": round(fps * 640 * 480 / 1e6, 4),
           "host": {"nproc": nproc, "workers": n, "cpu_model": model,
                    "processes_used": len({sp[2] for sp in spans})},
           "single_core": single,
           "context": "paper: ~120 Hz VGA (8.2 ms) at 1 iteration on one i7-3920XM thread (SSE census)"}
    return rec, refs


def roofline_probe(api, params, W=7680, H=4320, reps=20, dev="cuda:0"):
    """Interpolation and validation on one 7680x4320 frame (a working set far beyond
    the 256 MB Infinity Cache): a uniform-random texture shifted by 16 px, supports
    matched on the 10 px grid and triangulated once; each call timed with events."""
    import numpy as np
    import torch
    rng = np.random.default_rng(7)
    left = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    right = np.empty_like(left)
    right[:, :W - 16] = left[:, 16:]
    right[:, W - 16:] = rng.integers(0, 256, size=(H, 16), dtype=np.uint8)
    L = torch.from_numpy(left).to(dev)
    R = torch.from_numpy(right).to(dev)
    cL, om = api.census(L, params["census_w"], params["census_h"], params["grad_thr"])
    cR, _ = api.census(R, params["census_w"], params["census_h"], params["grad_thr"], with_omega=False)
    buf, n = api.match_support(cL, cR, om, params)
    n_s = int(n.item())
    S = api.supports_to_numpy(buf, n_s)
    tris = api.triangulate(S)
    T = torch.from_numpy(np.ascontiguousarray(tris, np.int32).reshape(-1)).to(dev)
    D = torch.empty((H, W), dtype=torch.float32, device=dev)
    lib = api._lib.load()
    stream = torch.cuda.current_stream()
    n_t = int(T.numel() // 3)

    def interp():
        api.check(lib.sm_interpolate(buf.data_ptr(), n_s, T.data_ptr(), n_t, W, H, D.data_ptr(),
                                     stream.cuda_stream))

    sz = 32
    n_cells = lib.sm_cells(W, H, sz)
    g = torch.empty(n_cells, dtype=torch.int64, device=dev)
    b = torch.empty(n_cells, dtype=torch.int64, device=dev)
    D_f = torch.zeros((H, W), dtype=torch.float32, device=dev)
    C_f = torch.empty((H, W), dtype=torch.uint8, device=dev)
    p = api.make_params(params)

    def valid():
        api.check(lib.sm_validate(cL.data_ptr(), cR.data_ptr(), om.data_ptr(), D.data_ptr(), W, H, p,
                                  sz, None, D_f.data_ptr(), C_f.data_ptr(), g.data_ptr(), b.data_ptr(),
                                  stream.cuda_stream))

    def fill_only():
        api.check(lib.sm_interpolate(buf.data_ptr(), n_s, T.data_ptr(), 0, W, H, D.data_ptr(),
                                     stream.cuda_stream))

    def timed(fn, before=None):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            if before is not None:
                before()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        return float(np.mean(ts))

    def entry(avg, per_px, kernel_name):
        gbs = W * H * per_px / (avg * 1e-6) / 1e9
        return {"avg_us": round(avg, 2), "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                "algorithmic_per_launch": f"{W}x{H} px x {per_px} B",
                "traffic": load_traffic(kernel_name, "probe_7680x4320") if kernel_name else None}

    t_fill = timed(fill_only)
    t_interp = timed(interp)  # leaves the interpolated D in place for the validation
    t_valid = timed(valid, before=lambda: C_f.fill_(params["t_hi"]))
    fast_prm = dict(params, support_mode=1)

    def fast():
        api.fast_candidates(L, fast_prm, stream=stream)

    t_fast = timed(fast)
    out = {"fast_candidates": entry(t_fast, 2.0, None),
           "interpolate": entry(t_interp, 4.0, None), "nan_fill": entry(t_fill, 4.0, "nan_fill"),
           "raster": entry(max(t_interp - t_fill, 1e-3), 4.0, "raster"),
           "validate": entry(t_valid, 27.0, "validate")}
    out["fast_candidates"]["note"] = ("sm_fast_candidates, 12 x 10 bins, <= 25 per bin: score "
                                      "(1 B read + 1 B written per px) + bin selection + compaction")
    out["interpolate"]["note"] = "sm_interpolate = NaN fill (4 B/px) + rasterisation"
    out["raster"]["note"] = ("rasteriser alone: sm_interpolate minus a call with no triangles "
                             "(NaN fill only); every pixel of this frame is covered")
    out["frame"] = f"{W}x{H}, {n_s} supports, {n_t} triangles, cells {sz}x{sz}"
    return out


def variant_runs(api, dframes, params, W, H, steps=100, warmup=10, dev="cuda:0"):
    """The paper variants on the 640x480 workload, plain per-frame path: FAST supports
    from 12 x 10 bins (threshold 16, at most 25 per bin) instead of the 10 px grid, and
    3-level cost evaluation, alone and together."""
    import numpy as np
    import torch
    out = {}
    for name, over in (("fast_supports", dict(support_mode=1)), ("levels3", dict(levels=3)),
                       ("fast_supports_levels3", dict(support_mode=1, levels=3))):
        prm = dict(params, **over)
        solver = api.Solver(W, H, prm, device=dev)
        for k in range(warmup):
            solver(*dframes[k % len(dframes)], stats=True, timing=True)
        torch.cuda.synchronize()
        acc, cnt, n_valid, n_sup = {}, {}, 0, 0
        t0 = time.perf_counter()
        for k in range(steps):
            st = solver(*dframes[k % len(dframes)], stats=True, timing=True).stats
            n_valid += st["n_valid"]
            n_sup += st["n_support"][0]
            for kname in ("fast", "validate", "match"):
                acc[kname] = acc.get(kname, 0.0) + st["stage_us"][kname]
                cnt[kname] = cnt.get(kname, 0) + st["stage_launches"][kname]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"frames_per_s": round(steps / dt, 2), "mpx_per_s": round(steps * W * H / dt / 1e6, 2),
                     "semi_dense_mpx_per_s": round(n_valid / dt / 1e6, 2),
                     "initial_supports_per_frame": round(n_sup / steps, 1),
                     "kernel_us_per_frame": {k: round(acc[k] / steps, 2) for k in acc if cnt[k]}}
    return out


def batched_runs(api, vga_frames, vga_params, workers=16, batches=12, dev="cuda:0"):
    """Throughput of sm_solve_batch (concurrent per-frame solves) and sm_solve_many (one
    launch per stage over the batch): (a) the 640x480 workload in batches of 64 frames,
    (b) the mixed batch of 64 pairs (16 each of 320x240, 640x480, 1242x375, 1280x720,
    disparity ranges cycling 64/128/192/256; two distinct scenes per size, cycled)."""
    import numpy as np
    import torch
    import scenes

    def run(frames, params_list, maxW, maxH, n_batches):
        bs = api.BatchSolver(workers, maxW, maxH, params_list, device=dev)
        outs = None
        bs(frames)  # warm-up (worker threads, staging)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(n_batches):
            outs, st, per = bs(frames, outputs=outs, stats=True)
            lat += [x[1] for x in per]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        npx = sum(int(f[0].numel()) for f in frames)
        lat = np.array(lat) / 1e3
        return {"frames_per_s": round(n_batches * len(frames) / dt, 1),
                "mpx_per_s": round(n_batches * npx / dt / 1e6, 2),
                "ms_per_batch": round(dt / n_batches * 1e3, 3),
                "frame_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                     "p99": round(float(np.percentile(lat, 99)), 3)},
                "frames_per_batch": len(frames), "workers": workers}

    d = [(torch.from_numpy(l).to(dev), torch.from_numpy(r).to(dev)) for (l, r) in vga_frames]
    vga = [(d[i % len(d)][0], d[i % len(d)][1], vga_params) for i in range(64)]
    out = {"vga_20planes_batch64": run(vga, [vga_params], 640, 480, batches)}
    sizes = ((320, 240), (640, 480), (1242, 375), (1280, 720))
    ranges = (64, 128, 192, 256)
    base = []
    for si, (W, H) in enumerate(sizes):
        for k in range(2):
            dr = ranges[(2 * si + k) % 4]
            sc = scenes.make_rect_scene(W, H, seed=4000 + 10 * si + k, dlo=2.0, dhi=0.9 * dr)
            prm = scenes.params_of(4, d_min=0, d_max=dr - 1)
            base.append((torch.from_numpy(sc.left).to(dev), torch.from_numpy(sc.right).to(dev), prm))
    mixed = [base[2 * (i % 4) + (i // 4) % 2] for i in range(64)]
    out["batch64_mixed"] = run(mixed, [b[2] for b in base], 1280, 720, batches)
    out["batch64_mixed"]["sizes"] = "16 each of 320x240, 640x480, 1242x375, 1280x720"

    def run_many(frames, n_batches):
        ms = api.ManySolver(workers, device=dev)
        outs = ms(frames)  # warm-up (workspace, staging, worker threads)
        torch.cuda.synchronize()
        acc = {}
        t0 = time.perf_counter()
        for _ in range(n_batches):
            outs, st = ms(frames, outputs=outs, stats=True, timing=True)
            for k, v in st["stage_us"].items():
                acc[k] = acc.get(k, 0.0) + v
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        npx = sum(int(f[0].numel()) for f in frames)
        return {"frames_per_s": round(n_batches * len(frames) / dt, 1),
                "mpx_per_s": round(n_batches * npx / dt / 1e6, 2),
                "ms_per_batch": round(dt / n_batches * 1e3, 3),
                "frames_per_batch": len(frames), "host_threads": workers,
                "us_per_batch": {k: round(v / n_batches, 1) for k, v in acc.items() if v > 0}}

    def run_graph(frames, n_batches):
        """The same batch captured once into a HIP graph and replayed (no stage timing)."""
        ms = api.ManySolver(workers, device=dev)
        outs, graph = ms.capture(frames)
        try:
            graph.run()  # warm-up replay
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n_batches):
                graph.run(stats=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            graph.close()
        npx = sum(int(f[0].numel()) for f in frames)
        return {"frames_per_s": round(n_batches * len(frames) / dt, 1),
                "mpx_per_s": round(n_batches * npx / dt / 1e6, 2),
                "ms_per_batch": round(dt / n_batches * 1e3, 3), "frames_per_batch": len(frames)}

    # stage-batched: one launch per stage over the 64 frames (sm_solve_many), eager with
    # stage timing, and captured into a HIP graph and replayed
    out["vga_20planes_batch64_stage_batched"] = run_many(vga, batches)
    out["batch64_mixed_stage_batched"] = run_many(mixed, batches)
    out["vga_20planes_batch64_graph"] = run_graph(vga, batches)
    out["batch64_mixed_graph"] = run_graph(mixed, batches)
    # the mixed batch again after sm_autotune on one frame of each size and disparity range
    # (matcher lanes per candidate, census rows, validation and raster shapes of that size)
    tuned = {}
    for (l, r, prm) in base:
        H_, W_ = l.shape
        key = f"{W_}x{H_} d0-{prm['d_max']}"
        if key not in tuned:
            tuned[key] = api.Solver(W_, H_, prm, device=dev).autotune(l, r)
    torch.cuda.synchronize()
    out["batch64_mixed_stage_batched_tuned"] = run_many(mixed, batches)
    out["batch64_mixed_stage_batched_tuned"]["autotune"] = tuned
    out["batch64_mixed_stage_batched_tuned"]["change_vs_untuned"] = round(
        out["batch64_mixed_stage_batched_tuned"]["frames_per_s"] / out["batch64_mixed_stage_batched"]["frames_per_s"],
        3)

    # 256 frames: one mesh workgroup per frame fills all 256 CUs; three frames of the
    # replayed batch are compared with the per-frame solver
    vga256 = [(d[i % len(d)][0], d[i % len(d)][1], vga_params) for i in range(256)]
    ms = api.ManySolver(workers, device=dev)
    outs, graph = ms.capture(vga256)
    try:
        graph.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(batches):
            graph.run(stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solo = api.Solver(640, 480, vga_params, device=dev)
        same = True
        for i in (0, 101, 255):
            r = solo(vga256[i][0], vga256[i][1])
            torch.cuda.synchronize()
            same = same and bool(torch.equal(r.D_f, outs[i][0]) and torch.equal(r.C_f, outs[i][1])
                                 and torch.equal(r.mask, outs[i][2]))
    finally:
        graph.close()
    out["vga_20planes_batch256_graph"] = {
        "frames_per_s": round(batches * 256 / dt, 1), "mpx_per_s": round(batches * 256 * 640 * 480 / dt / 1e6, 2),
        "ms_per_batch": round(dt / batches * 1e3, 3), "frames_per_batch": 256,
        "sampled_frames_equal_solo": same}
    return out


def serving_run(api, seconds=10.0, n_streams=16, lanes=2, max_batch=64, per_stream=8, budget_gb=48.0,
                dev="cuda:0"):
    """16 camera streams (640x480 / 1280x720 / 1920x1080 by stream id mod 3), Poisson
    arrivals at 30 Hz each, disparities 0-255, 3 iterations, replayed in real time
    through the continuous-batching server (latency), then all at once (capacity).
    Latency = completion - arrival, including the host-to-device upload of the pair.
    Beside it: each size solved alone on the plain per-frame path (sm_solve)."""
    import numpy as np
    import torch
    import scenes
    from paper_1511_00758_amd.serving import StereoServer, StreamSpec, replay

    sizes = ((640, 480), (1280, 720), (1920, 1080))
    prm = scenes.params_of(5)
    pairs = {}
    for si, (W, H) in enumerate(sizes):
        for k in range(2):
            sc = scenes.make_rect_scene(W, H, seed=5000 + 10 * si + k, dlo=2.0, dhi=240.0)
            pairs[(si, k)] = (torch.from_numpy(sc.left).pin_memory(),
                              torch.from_numpy(sc.right).pin_memory())
    specs = {s: StreamSpec(sizes[s % 3][0], sizes[s % 3][1], prm) for s in range(n_streams)}
    # per-frame path, each size alone (reference latency)
    solo = {}
    for si, (W, H) in enumerate(sizes):
        sv = api.Solver(W, H, prm, device=dev)
        l, r = (t.to(dev) for t in pairs[(si, 0)])
        sv(l, r)
        torch.cuda.synchronize()
        ts = []
        for _ in range(20):
            t0 = time.perf_counter()
            sv(l, r)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        solo[f"{W}x{H}"] = round(float(np.median(ts)), 3)
        del sv
    mix = [solo[f"{sizes[s % 3][0]}x{sizes[s % 3][1]}"] for s in range(n_streams)]
    counter = {s: 0 for s in specs}

    def frames_for(s):
        counter[s] += 1
        return pairs[(s % 3, (s // 3 + counter[s]) % 2)]

    out = {"streams": n_streams, "lanes": lanes, "max_batch": max_batch, "frames_per_stream": per_stream,
           "budget_gb": budget_gb,
           "rate_hz": 30.0, "simulated_s": seconds, "meshes": "device",
           "batching": "continuous: each free lane takes every admissible frame (sm_solve_many)",
           "per_frame_path": {"latency_ms_p50_alone": solo,
                              "capacity_frames_per_s": round(1e3 / float(np.mean(mix)), 1),
                              "note": "sm_solve one frame at a time; capacity = 1 / mean solo time over the stream mix"}}
    for mode, scale in (("realtime", 1.0), ("saturated", 0.0)):
        server = StereoServer(specs, budget_bytes=int(budget_gb * 2**30), device=dev, n_lanes=lanes,
                              max_batch=max_batch, frames_per_stream=per_stream)
        sched = scenes.stream_schedule(seed=11, n_streams=n_streams, rate_hz=30.0, seconds=seconds)
        done, wall = replay(server, sched, frames_for, time_scale=scale)
        warm = 0.1 * scale * seconds      # the first moments of the real-time run fill the lanes
        t_first = min(r.t_arrival for r in done)
        lat = np.array([r.latency for r in done if r.t_arrival - t_first >= warm]) * 1e3
        npx = sum(specs[r.stream].W * specs[r.stream].H for r in done)
        bs = np.array([b for (_, b, _) in server.batches])
        out[mode] = {"frames": len(done), "wall_s": round(wall, 3),
                     "frames_per_s": round(len(done) / wall, 1),
                     "mpx_per_s": round(npx / wall / 1e6, 1),
                     "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                    "p99": round(float(np.percentile(lat, 99)), 3)},
                     "batches": int(len(bs)), "frames_per_batch": {"mean": round(float(bs.mean()), 2),
                                                                   "max": int(bs.max())},
                     "evictions": server.adm.evictions}
    out["offered_frames_per_s"] = round(n_streams * 30.0, 1)
    return out


def calibrate_copy(mib):
    """A plain device copy of known size, for scaling the FETCH/WRITE counters."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda:0")
    a.fill_(1)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": mib << 20, "launches": 5}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--frames", type=int, default=8, help="distinct frames cycled")
    ap.add_argument("--cpu-frames", type=int, default=5,
                    help="oracle seeds per single-frame workload (single-core latency leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch-shape rules (no sm_autotune before timing)")
    ap.add_argument("--time-every", type=int, default=3, metavar="N",
                    help="time the dominant kernel with events on every N-th frame of the timed "
                         "region (default 3: every frame of the 8-frame cycle is sampled)")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not record per-kernel events in the timed region")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the 16-stream serving run")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched (sm_solve_batch) throughput runs")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the 7680x4320 interpolation/validation roofline probe")
    ap.add_argument("--time-all", action="store_true",
                    help="time every kernel of the solve with events (default: validate, raster and the mesh)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FAST-support / 3-level variants of the 640x480 workload")
    ap.add_argument("--probe-only", action="store_true",
                    help="only run the 7680x4320 roofline probe")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU: the hot path of one frame "
                          "fits one MI355X and frames/streams shard across GPUs without "
                          "collectives (see the design notes); run with --gpus 1"}))
        sys.exit(2)

    cpu, cpu_refs = None, {}
    if not args.no_cpu_baseline and not args.probe_only:
        # the oracle on the host cores first, before anything touches the GPU
        cpu, cpu_refs = cpu_baseline(seeds_per_config=args.cpu_frames)
        progress(f"cpu baseline: {cpu['value']} frames/s on {cpu['cores']} processes")

    import numpy as np
    import torch

    import scenes
    from paper_1511_00758_amd import api

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    dev = "cuda:0"
    cfg = 2
    params = scenes.params_of(cfg)
    if args.probe_only:
        print(json.dumps({"roofline_probe_7680x4320": roofline_probe(api, params)}))
        return
    W, H = scenes.CONFIGS[cfg]["W"], scenes.CONFIGS[cfg]["H"]
    frames = []
    for f in range(args.frames):
        sc = scenes.make_scene(cfg, scenes.seed_of(cfg, f))
        frames.append((sc.left, sc.right))
    dframes = [(torch.from_numpy(l).to(dev), torch.from_numpy(r).to(dev)) for (l, r) in frames]
    solver = api.Solver(W, H, params, device=dev)
    # launch shapes measured on the first frame (sm_autotune) for this size, used by every
    # later launch of the run (outputs do not depend on them)
    tuned = None if args.no_autotune else solver.autotune(*dframes[0])
    progress(f"autotune: {tuned}")
    # live timing of the dominant kernel (the mesh) inside the timed region, on every
    # --time-every-th frame (3: coprime to the 8 frames cycled, so every frame is sampled); an
    # event pair around a launch costs ~4 us of frame time, so validation and the raster are
    # timed in a pass of their own after it (--time-all times every kernel in the loop)
    timing = False if args.no_timing else (True if args.time_all else ("mesh",))
    every = 1 if args.time_all else max(1, args.time_every)

    for k in range(args.warmup):
        l, r = dframes[k % len(dframes)]
        solver(l, r, stats=True, timing=timing)
    torch.cuda.synchronize()

    acc_us = {}
    acc_n = {}
    lat = []
    n_valid = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        l, r = dframes[k % len(dframes)]
        ts = time.perf_counter()
        res = solver(l, r, stats=True, timing=timing if k % every == 0 else False)
        lat.append(time.perf_counter() - ts)
        st = res.stats
        n_valid += st["n_valid"]
        for name, us in st["stage_us"].items():
            acc_us[name] = acc_us.get(name, 0.0) + us
            acc_n[name] = acc_n.get(name, 0) + st["stage_launches"][name]
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    elapsed = t1 - t0
    fps = args.steps / elapsed
    progress(f"timed region: {args.steps} frames, {fps:.1f} frames/s")
    lat_ms = np.array(lat) * 1e3
    kernels = {}
    timed_steps = len(range(0, args.steps, every))
    for name in acc_us:
        if name in ("host_triangulate", "host_copies", "total"):
            continue
        if acc_n[name]:
            kernels[name] = {"avg_us": round(acc_us[name] / acc_n[name], 3),
                             "launches_per_step": round(acc_n[name] / timed_steps, 2),
                             "us_per_step": round(acc_us[name] / timed_steps, 3),
                             "timed": (f"in the timed region, on {timed_steps} of its {args.steps} frames"
                                       if timed_steps != args.steps else "in the timed region")}
    if timing and not args.time_all:
        side_us, side_n, side_steps = {}, {}, min(args.steps, 100)
        for k in range(side_steps):
            st2 = solver(*dframes[k % len(dframes)], stats=True, timing=("validate", "raster")).stats
            for name in ("validate", "raster"):
                side_us[name] = side_us.get(name, 0.0) + st2["stage_us"][name]
                side_n[name] = side_n.get(name, 0) + st2["stage_launches"][name]
        torch.cuda.synchronize()
        for name in side_us:
            if side_n[name]:
                kernels[name] = {"avg_us": round(side_us[name] / side_n[name], 3),
                                 "launches_per_step": round(side_n[name] / side_steps, 2),
                                 "us_per_step": round(side_us[name] / side_steps, 3),
                                 "timed": f"{side_steps} frames after the timed region"}
    host = {k: round(acc_us.get(k, 0.0) / args.steps, 1) for k in ("host_triangulate", "host_copies", "total")}
    roof = None
    roof_val = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["us_per_step"])
        roof = roofline_for(dom, kernels[dom]["avg_us"], W, H, params, params["n_iters"],
                            kernels[dom]["launches_per_step"],
                            traffic=load_traffic(dom, "vga_20planes"), stats=st)
        # the validation kernel, whose roofline the design targets, reported beside it
        if "validate" in kernels and dom != "validate":
            roof_val = roofline_for("validate", kernels["validate"]["avg_us"], W, H, params,
                                    params["n_iters"], kernels["validate"]["launches_per_step"],
                                    traffic=load_traffic("validate", "vga_20planes"))

    # the frames the oracle solved (640x480 seeds 2000..), solved again outside the timed
    # region and compared bit for bit
    validated = None
    for i, ref in sorted(cpu_refs.items()):
        if i >= len(dframes):
            continue
        rr = solver(dframes[i][0], dframes[i][1])
        torch.cuda.synchronize()
        D_f, C_f, mask = (rr.D_f.cpu().numpy(), rr.C_f.cpu().numpy(), rr.mask.cpu().numpy())
        ok = bool((C_f == ref[1]).all() and (mask.astype(bool) == ref[2]).all()
                  and (D_f.view(np.uint32) == ref[0].view(np.uint32)).all())
        validated = ok if validated is None else (validated and ok)
    probe = None if args.no_probe else roofline_probe(api, params)
    progress("roofline probe done")
    variants = None if args.no_variants else variant_runs(api, dframes, params, W, H)
    progress("paper variants done")
    batched = None if args.no_batch else batched_runs(api, frames, params)
    progress("batched runs done")
    serving = None if args.no_serve else serving_run(api, seconds=args.serve_seconds)
    progress("serving done")

    out = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u64 int + f32",
        "data": "synthetic",
        "config": {"workload": "vga_20planes: 640x480 pair, 20 slanted planes with occlusions "
                               "and ~5% untextured, 7x7 census, d 0-127, 3 iterations, "
                               "support grid 10 px, t_hi 12 / t_lo 6",
                   "frames_cycled": args.frames, "per_frame_path": "sm_solve, one stream"},
        "mpx_per_s": round(fps * W * H / 1e6, 3),
        "validated": validated,
        "validated_mpx_per_s": round(fps * W * H / 1e6, 3) if validated else None,
        "semi_dense_mpx_per_s": round(n_valid / elapsed / 1e6, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "max": round(float(lat_ms.max()), 4)},
        "kernels": kernels,
        "autotune": tuned,
        "host_us_per_step": host,
        "roofline": roof,
        "roofline_validate": roof_val,
        "roofline_probe_7680x4320": probe,
        "paper_variants": variants,
        "batched": batched,
        "serving_16_streams": serving,
        "cpu_baseline": cpu,
        "paper_context": "paper: ~120 Hz (8.2 ms) VGA, 1 iteration, one i7-3920XM thread; "
                         "19.2 ms at 2 iterations",
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
