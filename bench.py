#!/usr/bin/env python3
"""Throughput of the batched differentiable RGB-D-N rasterizer on one MI355X.

Workload C2: 200,000 voxel anchors x 10 Gaussians (2M Gaussians) over a
200 x 200 x 50 m synthetic city block, a batch of 8 views of uneven
resolution (960x540 .. 1920x1080) with per-view LoD.  One step is one fused
launch chain: anchor selection, decode + projection, tile binning, the
64-bit (tile | depth) sort, forward compositing of RGB / D / N / alpha with
the unbiased depth, the L1 loss of Eq. 8 against seeded targets, the
reverse-order backward raster and the projection / decoder adjoint.  Inputs
are resident in HBM before the timed region.

Prints one JSON line: fwd+bwd Mpixels/s (value), the batched vs per-view
speedup, the roofline of the dominant kernel (timed with HIP events on the
launch stream inside the timed region) and the FP64 oracle timed on a
bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# published MI355X peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# algorithmic work per list entry walked (pixel, splat), counted from the
# method's arithmetic, with a transcendental counted as one flop: forward =
# offsets, quadratic form, exponential, alpha, transmittance update and the
# 7-channel blend (26 + exp); backward = the recomputed alpha, the
# transmittance recovered by a reciprocal, the value / suffix terms and the
# 13 gradient terms (90 + exp + rcp)
FLOPS_FWD_PER_ENTRY = 27
FLOPS_BWD_PER_ENTRY = 92
SORT_BYTES_PER_ELEM_PASS = 16     # read + write of a 32-bit key and a 32-bit value


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--config", type=int, default=2)
    p.add_argument("--tile", type=str, default="16x16",
                   help="tile shape WxH (16x16 is the paper's patch), or 'auto' to time every "
                        "compiled shape with the autotuner and keep the fastest")
    p.add_argument("--no-per-view", action="store_true")
    p.add_argument("--no-graph", action="store_true",
                   help="skip the timing of the same step replayed from a captured hipGraph")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-tiles", type=int, default=4000)
    p.add_argument("--cpu-workers", type=int, default=0,
                   help="processes of the N-core oracle timing (0: the host's cores, at most 16)")
    p.add_argument("--configs", type=str, default="3,4",
                   help="further workloads timed after C2 (comma list of 3, 4; empty for none)")
    p.add_argument("--config-steps", type=int, default=10)
    p.add_argument("--no-ncc", action="store_true",
                   help="skip the timing of the batch geometric loss (Eq. 10)")
    p.add_argument("--ncc-patches", type=int, default=4096,
                   help="7x7 patches per view pair in the geometric-loss timing")
    p.add_argument("--ncc-only", action="store_true",
                   help="time only the geometric loss and print its JSON object")
    p.add_argument("--no-depth", action="store_true",
                   help="skip the timing of the depth-prior alignment and filter (Sec. 3.4)")
    p.add_argument("--depth-only", action="store_true",
                   help="time only the depth-prior steps and print their JSON object")
    p.add_argument("--no-tsdf", action="store_true",
                   help="skip the timing of the TSDF fusion (Sec. 4)")
    p.add_argument("--tsdf-only", action="store_true",
                   help="time only the TSDF fusion and print its JSON object")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="first run 3 plain device copies of MIB MiB (a known-traffic kernel "
                        "for scaling hardware byte counters)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_leg(args, wl, tile=None, steps=None, warmup=None, per_view=None, graph=None, count=True):
    """The fused step on workload wl: tile shape (WxH or 'auto'), `steps`
    timed steps after `warmup`, the same step replayed from a hipGraph, the
    per-view loop, peak HBM, and (count) one untimed counting step."""
    tile = args.tile if tile is None else tile
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    per_view = (not args.no_per_view) if per_view is None else per_view
    graph = (not args.no_graph) if graph is None else graph
    import numpy as np
    import torch

    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render

    dev = "cuda:0"
    sc = render.scene_from(wl.scene, dev)
    cat = lambda xs: torch.as_tensor(np.concatenate([x.ravel() for x in xs]), device=dev)  # noqa: E731
    tgt = dict(rgb=cat(wl.targets["rgb"]), depth=cat(wl.targets["depth"]),
               normal=cat(wl.targets["normal"]))
    w3 = (1.0, 1.0, 1.0)
    tune_ms = None
    if tile == "auto":
        rd = render.Renderer(0, (16, 16))
        (tw, th), tune_ms = rd.autotune(wl.views, sc, tgt, w3, reps=3)
        log(f"[bench] autotuned tile {tw}x{th}: " +
            ", ".join(f"{a}x{b} {m:.3f} ms" for (a, b), m in tune_ms.items()))
    else:
        tw, th = (int(x) for x in tile.split("x"))
        rd = render.Renderer(0, (tw, th))
    loss = torch.zeros(1, device=dev)
    # capacity discovery (grows the pair / row capacity on overflow)
    out, grads = rd.fwd_bwd_l1(wl.views, sc, tgt, w3, loss=loss)
    torch.cuda.synchronize()
    info0 = dict(rd.last_info)
    log(f"[bench] rows {info0['n_rows']} splats {info0['n_splats']} pairs {info0['n_pairs']} "
        f"loss {info0['loss']:.6f} workspace {rd.ws.numel() / 2**30:.2f} GiB")
    for _ in range(max(warmup, 1)):
        rd.fwd_bwd_l1(wl.views, sc, tgt, w3, out=out, grads=grads, loss=loss, check=False)
    torch.cuda.synchronize()
    log(f"[bench] warmup {warmup} done; capacities {rd.cap}, workspace {rd.ws.numel() / 2**30:.2f} GiB")
    torch.cuda.reset_peak_memory_stats()

    B.cgx_timing_enable(rd.ctx, 16 * steps + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rd.fwd_bwd_l1(wl.views, sc, tgt, w3, out=out, grads=grads, loss=loss, check=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    peak_bytes = torch.cuda.max_memory_allocated()      # the batched step's own peak
    phases = B.cgx_timing_read(rd.ctx)
    B.cgx_timing_enable(rd.ctx, 0)
    info = rd.info()      # raises if a capacity was exceeded inside the timed region
    # the work counts of the roofline: one more step, untimed, with the
    # raster kernels' counting variants
    if count:
        rd.count_work(True)
        rd.fwd_bwd_l1(wl.views, sc, tgt, w3, out=out, grads=grads, loss=loss, check=False)
        torch.cuda.synchronize()
        counts = rd.info()
        rd.count_work(False)
        for k in ("entries_fwd", "evals_fwd", "evals_bwd"):
            info[k] = counts[k]
    log(f"[bench] per step: list entries walked fwd {info['entries_fwd']} bwd {info['entries_bwd']}, "
        f"opacity evaluations fwd {info['evals_fwd']} bwd {info['evals_bwd']}")
    ms = (t1 - t0) / steps * 1e3
    log(f"[bench] timed {steps} steps: {ms:.3f} ms/step")
    for k, (t, c) in phases.items():
        if c:
            log(f"[bench]   {k:12s} {t / c:8.3f} ms x {c // steps} per step")

    # the same fused step replayed from a captured hipGraph (no phase events)
    graph_ms = None
    if graph:
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            g = B.cgx_graph_capture_fwd_bwd_l1(rd.ctx, wl.views, sc, rd.cap, rd.ws, tgt, w3, out,
                                               grads, loss, side)
        try:
            for _ in range(2):
                B.cgx_graph_launch(g, side)
            side.synchronize()
            t0g = time.perf_counter()
            for _ in range(steps):
                B.cgx_graph_launch(g, side)
            side.synchronize()
            graph_ms = (time.perf_counter() - t0g) / steps * 1e3
            rd.info()     # raises if a replay exceeded a capacity
        finally:
            B.cgx_graph_destroy(g)
        log(f"[bench] hipGraph replay: {graph_ms:.3f} ms/step")

    per_view_ms = None
    if per_view and len(wl.views) > 1:
        rv = render.Renderer(0, (tw, th))
        rv.cap = dict(rd.cap)
        offs = render.pixel_offsets(wl.views)
        singles = []
        for v, view in enumerate(wl.views):
            a, b = int(offs[v]), int(offs[v + 1])
            t1v = dict(rgb=tgt["rgb"][3 * a:3 * b], depth=tgt["depth"][a:b], normal=tgt["normal"][3 * a:3 * b])
            singles.append(([view], t1v))
        bufs = []
        for views1, t1v in singles:
            o1, g1 = rv.fwd_bwd_l1(views1, sc, t1v, w3, loss=loss)
            bufs.append((o1, g1))
        torch.cuda.synchronize()
        for _ in range(2):
            for (views1, t1v), (o1, g1) in zip(singles, bufs):
                rv.fwd_bwd_l1(views1, sc, t1v, w3, out=o1, grads=g1, loss=loss, check=False)
        torch.cuda.synchronize()
        reps = max(3, steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            for (views1, t1v), (o1, g1) in zip(singles, bufs):
                rv.fwd_bwd_l1(views1, sc, t1v, w3, out=o1, grads=g1, loss=loss, check=False)
        torch.cuda.synchronize()
        per_view_ms = (time.perf_counter() - t0) / reps * 1e3
        log(f"[bench] per-view loop: {per_view_ms:.3f} ms per batch ({len(wl.views)} calls)")
    return dict(ms=ms, info=info, phases=phases, per_view_ms=per_view_ms, graph_ms=graph_ms,
                peak_bytes=peak_bytes, tile=f"{tw}x{th}",
                tune_ms=({f"{a}x{b}": round(m, 4) for (a, b), m in tune_ms.items()}
                         if tune_ms else None))


def copy_calibration(mib):
    """Three device-to-device copies of `mib` MiB: each reads and writes
    exactly mib MiB, which calibrates FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * 2**20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {mib} MiB")
    del src, dst


PROFILE_BYTES = os.path.join(ROOT, "profiles", "c2_fused_step_hbm_bytes.md")
# the raster kernels and what decides their input (the pixel boxes)
KERNEL_SOURCES = ("paper_2503_23044_amd/csrc/k_raster.hip", "paper_2503_23044_amd/csrc/cgx_common.h",
                  "paper_2503_23044_amd/csrc/cgx_project.h")


def kernel_source_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` (e.g. 'k_raster_bwd<16, 16, false>') from the
    committed FETCH_SIZE / WRITE_SIZE summary, or None when there is none or
    it was taken from other raster sources than the ones built now."""
    if not os.path.exists(PROFILE_BYTES):
        return None
    digest = kernel_source_digest()
    with open(PROFILE_BYTES) as f:
        for line in f:
            m = re.match(r"traffic: kernel=(.+?) read_bytes=(\d+) write_bytes=(\d+) source=(\w+)", line.strip())
            if m and m.group(1) == kernel and m.group(4) == digest:
                return int(m.group(2)) + int(m.group(3))
    return None


def roofline(res, steps):
    info, ph = res["info"], res["phases"]
    cands = []
    t, c = ph["raster_bwd"]
    if c:
        d = t / c * 1e-3
        fl = info["entries_bwd"] * FLOPS_BWD_PER_ENTRY
        cands.append((t / steps, dict(kernel="raster_bwd", bound="alu", achieved=fl / d / 1e12,
                                      peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                                      work=f"{FLOPS_BWD_PER_ENTRY} flops x {info['entries_bwd']} "
                                           f"list entries walked backward")))
    t, c = ph["raster_fwd"]
    if c:
        d = t / c * 1e-3
        fl = info["entries_fwd"] * FLOPS_FWD_PER_ENTRY
        cands.append((t / steps, dict(kernel="raster_fwd", bound="alu", achieved=fl / d / 1e12,
                                      peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                                      work=f"{FLOPS_FWD_PER_ENTRY} flops x {info['entries_fwd']} "
                                           f"list entries walked forward")))
    t, c = ph["sort"]
    if c:
        # both sorts of a step: 4 passes over the visible splats' depth keys,
        # sort_passes over the pairs' tile ids; each pass reads and writes a
        # key and a value
        d = t / steps * 1e-3
        by = SORT_BYTES_PER_ELEM_PASS * (4 * info["n_visible"] + info["sort_passes"] * info["n_pairs"])
        cands.append((t / steps, dict(kernel="sort", bound="hbm", achieved=by / d / 1e9,
                                      peak=PEAK_HBM_GBS, unit="GB/s")))
    if not cands:
        return None
    cands.sort(key=lambda x: -x[0])
    r = cands[0][1]
    r["frac"] = r["achieved"] / r["peak"]
    tw, th = res["tile"].split("x")
    r["traffic"] = (profiled_traffic(f"k_{r['kernel']}<{tw}, {th}, false>")
                    if r["kernel"].startswith("raster") else None)
    return r


_ORACLE_JOB = None     # (splats, views, layout, sorted, view arrays, targets), inherited by fork


def _oracle_tiles(tiles):
    """Compositing + L1 + compositing adjoint of view 0 on the given tiles
    (one thread); the rest of the job comes from _ORACLE_JOB."""
    from threadpoolctl import threadpool_limits

    from oracle import raster as oras
    S, views, layout, srt, varr, targets = _ORACLE_JOB
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        imgs = oras.render_images([S], views, layout, srt, varr, keep_tiles=tiles)
        L, og = oras.l1_seed(imgs, targets)
        oras.composite_backward([S], views, imgs, og, varr)
        return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, n_sample_tiles, workers):
    """The FP64 oracle on a bounded sample of the workload: view 0 only;
    selection, decode, projection and sort of all of view 0, compositing and
    its adjoint on a seeded sample of view 0's tiles, the projection and
    decoder adjoint of all of view 0; the tile part is scaled to all of
    view 0's tiles.  Timed on one thread (BLAS pinned to 1), then with the
    tile part split over `workers` processes (forked before the GPU is
    touched, one thread each)."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import anchors as oanc
    from oracle import project as oprj
    from oracle import raster as oras

    views = wl.views[:1]
    sc = wl.scene
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        layout = oras.batch_layout(views, (16, 16))
        rows, offs = oanc.select(sc, views)
        D = oanc.decode(sc, views, rows)
        S = oprj.project(D["mu"], D["scales"], D["quats"], D["opacity"], views[0], (16, 16),
                         colour=D["rgb"])
        srt = oras.bin_and_sort([S], layout)
        t_fixed = time.perf_counter() - t0
        n_tiles = int(layout["tile_off"][-1])
        rng = np.random.default_rng(1234)
        sample = np.sort(rng.choice(n_tiles, min(n_sample_tiles, n_tiles), replace=False))
        varr = [oprj.view_arrays(views[0])]
        tg = {k: [wl.targets[k][0]] for k in ("rgb", "depth", "normal")}
        global _ORACLE_JOB
        _ORACLE_JOB = (S, views, layout, srt, varr, tg)
        t_tiles = _oracle_tiles(sample)
        t0 = time.perf_counter()
        imgs = oras.render_images([S], views, layout, srt, varr, keep_tiles=sample[:1])
        L, og = oras.l1_seed(imgs, tg)
        sg = oras.composite_backward([S], views, imgs, og, varr)
        pg = oprj.project_backward(S, sg[0])
        gparts = {k: pg[k] for k in ("mu", "scales", "quats", "opacity", "rgb")}
        oanc.decode_backward(sc, D, gparts)
        t_fixed += time.perf_counter() - t0
    px = int(views[0].width) * int(views[0].height)
    scale = n_tiles / len(sample)
    t_1 = t_fixed + t_tiles * scale
    # the tile part over `workers` processes: wall time of the pool
    shares = [sample[i::workers] for i in range(workers)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))         # the workers are up before the clock starts
        t0 = time.perf_counter()
        pool.map(_oracle_tiles, [sh for sh in shares if sh.size])
        t_par = time.perf_counter() - t0
    t_n = t_fixed + t_par * scale
    return dict(value=px / t_n / 1e6, unit="Mpixels/s", cores=workers, kind="oracle",
                value_1core=px / t_1 / 1e6, cpu=cpu_model(), cpu_count=os.cpu_count(),
                sample=(f"view 0 of C2 ({views[0].width}x{views[0].height}, {rows.shape[0]} rows): "
                        f"select/decode/project/sort and the projection+decoder adjoint in full "
                        f"({t_fixed:.1f} s, one thread), compositing + L1 + compositing adjoint on "
                        f"{len(sample)} of {n_tiles} tiles scaled to all tiles ({t_tiles:.1f} s on one "
                        f"thread, {t_par:.1f} s over {workers} processes); float64 NumPy"))


def config_leg(args, k):
    """Throughput of the fused step on workload C3 or C4 (batched vs per
    view, peak HBM).  C4 runs with the autotuned tile shape and reports its
    hipGraph replay."""
    import torch

    from synth import scenes
    t0 = time.perf_counter()
    wl = scenes.make(k)
    log(f"[bench] workload {wl.name}: {len(wl.views)} views, {wl.pixels} pixels "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    res = gpu_leg(args, wl, tile="auto" if k == 4 else args.tile, steps=args.config_steps, warmup=2,
                  per_view=True, graph=(k == 4), count=False)
    desc = {3: "C3: 600,000 voxel anchors x 10 Gaussians (6M), 4 views 3840x2160, per-view LoD, "
               "fused fwd+L1+bwd",
            4: "C4: 2,000,000 voxel anchors x 10 Gaussians (20M) over 1x1 km, 16 nadir/oblique views "
               "1600x1200, autotuned tile, fused fwd+L1+bwd"}[k]
    out = {"workload": desc, "views": len(wl.views), "pixels": wl.pixels, "tile": res["tile"],
           "ms_per_step": round(res["ms"], 4),
           "Mpixels_per_s": round(wl.pixels / (res["ms"] * 1e-3) / 1e6, 3),
           "per_view_ms": round(res["per_view_ms"], 4) if res["per_view_ms"] else None,
           "batched_vs_per_view": (round(res["per_view_ms"] / res["ms"], 3)
                                   if res["per_view_ms"] else None),
           "ms_per_step_graph": round(res["graph_ms"], 4) if res["graph_ms"] else None,
           "peak_hbm_gib": round(res["peak_bytes"] / 2**30, 3),
           "rows": res["info"]["n_rows"], "pairs": res["info"]["n_pairs"],
           "phases_ms": {p: round(t / max(args.config_steps, 1), 4)
                         for p, (t, c) in res["phases"].items() if c}}
    log(f"[bench] {wl.name}: {out['ms_per_step']} ms/step, {out['Mpixels_per_s']} Mpixels/s, "
        f"batched vs per-view {out['batched_vs_per_view']}, peak HBM {out['peak_hbm_gib']} GiB")
    del wl, res
    torch.cuda.empty_cache()
    return out


def ncc_leg(args):
    """Timing of the batch geometric loss (Eq. 10, cgx_ncc_loss) on the C2
    scene seen by 4 pairs of nearby 1920x1080 cameras: one forward render,
    then the loss and its RGB gradient over args.ncc_patches patches per
    pair, timed with HIP events over 20 launches."""
    import torch

    from paper_2503_23044_amd import render
    from synth import scenes

    wl = scenes.make_c2_pairs()
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene, "cuda:0")
    out = rd.forward(wl.views, sc)
    centres = torch.as_tensor(scenes.patch_centres(7, wl.views, args.ncc_patches), device="cuda:0")
    grad, loss = rd.ncc_loss(wl.views, out, centres)
    torch.cuda.synchronize()
    loss.zero_()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rd.ncc_loss(wl.views, out, centres, grad_rgb=grad, loss=loss)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    patches = len(wl.views) // 2 * args.ncc_patches
    log(f"[bench] geometric loss: {patches} patches in {ms * 1e3:.1f} us, loss {loss.item() / reps:.4f}")
    return {"workload": "C2 scene, 4 pairs of nearby 1920x1080 views, 7x7 patches",
            "patches": patches, "ms": round(ms, 4),
            "Mpatches_per_s": round(patches / (ms * 1e-3) / 1e6, 2),
            "loss": round(loss.item() / reps, 6)}


def depth_prior_leg(args):
    """Timing of the depth-prior steps (Sec. 3.4, Step 2): the per-view
    scale / shift of a pseudo depth against 1M sparse points
    (cgx_depth_prior_align) and the multi-view filter with tau_d = 1
    (cgx_depth_prior_filter) over 4 pairs of nearby 1920x1080 views, each
    timed with HIP events over 20 launches on the library's stream: the
    step as the renderer runs it (the filter aligns the raw prior on the
    fly), and, for reference, with the aligned image stored and re-read."""
    import torch

    import numpy as np

    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    from synth import scenes

    t0 = time.perf_counter()
    X = scenes.make_depth_prior()
    log(f"[bench] depth prior inputs generated in {time.perf_counter() - t0:.1f} s")
    rd = render.Renderer(0, (16, 16))
    prior = torch.from_numpy(np.concatenate(X.prior)).cuda()
    points = torch.from_numpy(X.points).cuda()
    filtered, aligned, st = rd.depth_prior(X.views, prior, points, X.nearby)
    torch.cuda.synchronize()
    reps = 20

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # the step as the renderer runs it: (s, t) only, then the filter aligning on the fly
    ms_a = timed(lambda: B.cgx_depth_prior_align(rd.ctx, X.views, prior, points, rd.depth_ws, st,
                                                 None))
    ms_f = timed(lambda: B.cgx_depth_prior_filter(rd.ctx, X.views, prior, X.nearby, 1.0, filtered,
                                                  scale_shift=st))
    # with the aligned image written and filtered from memory
    ms_a2 = timed(lambda: B.cgx_depth_prior_align(rd.ctx, X.views, prior, points, rd.depth_ws, st,
                                                  aligned))
    ms_f2 = timed(lambda: B.cgx_depth_prior_filter(rd.ctx, X.views, aligned, X.nearby, 1.0, filtered))
    px = sum(int(v.width) * int(v.height) for v in X.views)
    kept = float((filtered > 0).sum().item()) / max(float((aligned > 0).sum().item()), 1.0)
    log(f"[bench] depth prior: align {ms_a * 1e3:.1f} us, filter (aligning on the fly) "
        f"{ms_f * 1e3:.1f} us; with the aligned image stored {ms_a2 * 1e3:.1f} + {ms_f2 * 1e3:.1f} us; "
        f"{px} px, kept {kept:.3f}")
    return {"workload": "4 pairs of nearby 1920x1080 views over a box city, 1M sparse points",
            "pixels": px, "points": int(len(X.points)), "ms_align": round(ms_a, 4),
            "ms_filter": round(ms_f, 4), "ms": round(ms_a + ms_f, 4),
            "ms_with_aligned_image": round(ms_a2 + ms_f2, 4),
            "Mpixels_per_s": round(px / ((ms_a + ms_f) * 1e-3) / 1e6, 1), "kept": round(kept, 4)}


def tsdf_leg(args):
    """Timing of the TSDF fusion (Sec. 4, mesh reconstruction;
    cgx_tsdf_integrate): the z-depth and colour of 8 views over the box city
    fused into a 512 x 512 x 128 grid of 0.4 m voxels (truncation 2 m), timed
    with HIP events over 20 launches (each fuses all 8 views into the
    growing volume), with depth and colour interleaved into texels (the
    renderer's default) and, for reference, gathered from the planar
    images.  Two resolutions of the same cameras: 1920x1080 (a voxel spans
    about 4 pixels, so every gather pulls its own cache line) and 480x270
    (pixel footprint about one voxel)."""
    import numpy as np
    import torch

    from paper_2503_23044_amd import render
    from synth import scenes

    rd = render.Renderer(0, (16, 16))
    dims = (512, 512, 128)
    n = dims[0] * dims[1] * dims[2]
    res = {}
    for W, H in ((1920, 1080), (480, 270)):
        X = scenes.make_depth_prior(n_points=100, sizes=[(W, H)] * 8)
        rng = np.random.default_rng(60)
        depth = torch.from_numpy(np.concatenate(X.depth).astype(np.float32)).cuda()
        rgb = torch.from_numpy(np.concatenate([rng.uniform(0, 1, (3, int(v.width) * int(v.height)))
                                               .astype(np.float32).reshape(-1) for v in X.views])).cuda()
        vol = rd.tsdf_volume((-2.4, -2.4, -0.8), 0.4, dims, 2.0)
        rd.tsdf_integrate(X.views, depth, vol, rgb=rgb)
        torch.cuda.synchronize()
        reps = 20

        def timed(texels):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                rd.tsdf_integrate(X.views, depth, vol, rgb=rgb, texels=texels)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms = timed(True)
        ms_planar = timed(False)
        seen = float((vol["weight"] > 0).float().mean().item())
        log(f"[bench] tsdf fusion: 8 views of {W}x{H} into {n} voxels in {ms * 1e3:.1f} us with "
            f"interleaved texels, {ms_planar * 1e3:.1f} us from the planar images "
            f"({seen:.3f} of the voxels observed)")
        res[f"{W}x{H}"] = {"ms": round(ms, 4), "Gvoxel_views_per_s": round(n * 8 / (ms * 1e-3) / 1e9, 2),
                           "ms_planar": round(ms_planar, 4), "observed": round(seen, 4)}
        del vol, depth, rgb
    return {"workload": "8 views over a box city into a 512x512x128 grid of 0.4 m voxels",
            "voxels": n, "views": 8, **res}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.ncc_only:
        print(json.dumps({"ncc_loss": ncc_leg(args)}), flush=True)
        return
    if args.tsdf_only:
        if args.copy_calibration:
            copy_calibration(args.copy_calibration)
        print(json.dumps({"tsdf_fusion": tsdf_leg(args)}), flush=True)
        return
    if args.depth_only:
        if args.copy_calibration:
            copy_calibration(args.copy_calibration)
        print(json.dumps({"depth_prior": depth_prior_leg(args)}), flush=True)
        return
    from synth import scenes
    t0 = time.perf_counter()
    wl = scenes.make(args.config)
    cpu = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the worker processes are forked
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        t1 = time.perf_counter()
        cpu = cpu_baseline(wl, args.cpu_sample_tiles, workers)
        log(f"[bench] cpu baseline took {time.perf_counter() - t1:.1f} s: "
            f"{cpu['value_1core']:.4f} Mpixels/s on one thread, {cpu['value']:.4f} on {workers}")
    log(f"[bench] workload {wl.name}: {len(wl.views)} views, {wl.pixels} pixels "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    res = gpu_leg(args, wl)
    pixels = wl.pixels
    value = pixels / (res["ms"] * 1e-3) / 1e6
    line = {
        "metric": "fwd+bwd Mpixels/s, 2M Gaussians, batch-8 views; batched vs per-view speedup",
        "value": round(value, 3),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: 200,000 voxel anchors x 10 Gaussians (2M), 200x200x50 m city "
                               "block, 8 views 960x540..1920x1080, per-view LoD, fused fwd+L1+bwd",
                   "views": len(wl.views), "pixels": pixels, "tile": res["tile"],
                   "tile_autotune_ms": res["tune_ms"],
                   "rows": res["info"]["n_rows"], "pairs": res["info"]["n_pairs"]},
        "batched_vs_per_view": (round(res["per_view_ms"] / res["ms"], 3) if res["per_view_ms"] else None),
        "ms_per_step_graph": round(res["graph_ms"], 4) if res["graph_ms"] else None,
        "per_view_ms": (round(res["per_view_ms"], 4) if res["per_view_ms"] else None),
        "phases_ms": {k: round(t / max(args.steps, 1), 4) for k, (t, c) in res["phases"].items() if c},
        "peak_hbm_gib": round(res["peak_bytes"] / 2**30, 3),
        "roofline": roofline(res, args.steps),
    }
    if not args.no_ncc:
        line["ncc_loss"] = ncc_leg(args)
    if not args.no_depth:
        line["depth_prior"] = depth_prior_leg(args)
    if not args.no_tsdf:
        line["tsdf_fusion"] = tsdf_leg(args)
    extra = [int(c) for c in args.configs.split(",") if c.strip()]
    if extra and args.config == 2:
        del res
        line["configs"] = {f"C{k}": config_leg(args, k) for k in extra if k in (3, 4)}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
