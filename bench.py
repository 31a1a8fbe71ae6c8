"""Benchmark of the DPM scoring path on one MI355X.

One step = the whole workload once through the hot path: for every image (or
frame), projection, correlation of every level with every filter, distance
transform of every part map at the anchors, score assembly, and the
detection set (scores >= tau).  The default workload is the 256-frame stream
of 1920x1080 frames (51-level pyramids) with the 1080-filter bank (20 classes
x 6 components x (root + 8 parts)), tensor form in BF16 at rank 16.  The
frames share one pyramid shape, so one plan of `--chunk` frames serves every
chunk of the stream: a step enqueues, chunk after chunk, the scoring of the
chunk's frames (features read in place from the resident feature buffer)
into one reused score buffer, and the chunk's detections into a buffer of its
own.  Every input is resident in HBM before the timed region.

Also measured in the same run (one JSON line):
  * the launch strategies on one chunk (batched, per level, graph, overlap);
  * the direct FP32 path and the tensor form in FP32 / BF16 / FP8 operands
    and the per-filter CP form, on the first `--leg-images` frames;
  * the FP64 oracle on the host's cores (a process pool) on frame 0, with the
    GPU's score error against it (the oracle's own basis U_R);
  * the rank sweep R in {4, 8, 16, 32} on the 500x375 image with the same
    bank size: GPU throughput, its error against the oracle's tensor form at
    the same rank, and the truncation error of the tensor form against the
    oracle's direct scores.

Prints one JSON line.  --gpus N > 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "filter-response cells/s, tensor vs direct at stated error; % MFMA roofline"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP8_TFLOPS = 5000.0
PEAK_HBM_GBS = 8000.0
# score tolerance per mode; placements are compared where the oracle margin
# exceeds it.  FP8 has no stated target: 0.1 is a reporting margin only.
TOL = {"direct_fp32": 1e-4, "tensor_fp32": 1e-4, "tensor_bf16": 1e-2, "tensor_fp8": 1e-1}
SWEEP_RANKS = (4, 8, 16, 32)
MAX_POOL = 16            # worker processes of the oracle pool (the host's CPU share)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def _groups(pyramids, shapes, comps):
    """(level rows, level cols, [(h, w) of the filters run on it]) per level:
    roots on levels >= octave, parts one octave below."""
    roots = [c.root for c in comps]
    parts = sorted({p for c in comps for p in c.parts})
    for pyr in pyramids:
        L = len(pyr.levels)
        for l, lv in enumerate(pyr.levels):
            fs = []
            if l >= pyr.octave:
                fs += [shapes[k] for k in roots]
            if l + pyr.octave < L:
                fs += [shapes[k] for k in parts]
            yield lv.rows, lv.cols, fs


def corr_work(pyramids, shapes, comps, mode: str, rank: int):
    """Algorithmic flops and HBM bytes of one correlation launch over
    `pyramids` (all filters, all levels): 2*h*w*C flops per response (C = 32
    direct, R tensor); bytes = operand features read once per level + packed
    filters read once + FP32 responses written once."""
    C = 32 if mode == "direct_fp32" else rank
    esz = {"direct_fp32": 4, "tensor_fp32": 4, "tensor_bf16": 2, "tensor_fp8": 1}[mode]
    flops = resp = feat_bytes = 0
    for rows, cols, fs in _groups(pyramids, shapes, comps):
        used = False
        for (h, w) in fs:
            if rows >= h and cols >= w:
                n = (rows - h + 1) * (cols - w + 1)
                resp += n
                flops += 2 * n * h * w * C
                used = True
        if used:
            feat_bytes += rows * cols * C * esz
    filt_bytes = sum(h * w * C * esz for (h, w) in shapes)
    return flops, feat_bytes + filt_bytes + 4 * resp, resp


def mult_counts(pyramids, shapes, comps, rank: int, cp_rank: int) -> dict:
    """Multiplications per step of the three ways to correlate (Section 4's
    counting): direct h*w*32 per response; per-filter CP form R*(32 + h + w)
    per response (channel contraction, then 1-D correlations along x and y);
    shared feature-mode basis h*w*R per response plus 32*R per projected cell."""
    out = {"direct": 0, "cp": 0, "shared_basis": 0}
    for rows, cols, fs in _groups(pyramids, shapes, comps):
        used = False
        for (h, w) in fs:
            if rows >= h and cols >= w:
                n = (rows - h + 1) * (cols - w + 1)
                out["direct"] += n * h * w * 32
                out["cp"] += n * cp_rank * (32 + h + w)
                out["shared_basis"] += n * h * w * rank
                used = True
        if used:
            out["shared_basis"] += rows * cols * 32 * rank
    return out


def kernel_source_digest() -> str:
    """SHA-256 of the kernel sources; byte counters recorded for another
    digest describe other kernels and are not reported."""
    import hashlib
    h = hashlib.sha256()
    for name in ("dpmt_kernels.hip", "dpmt_internal.h"):
        with open(os.path.join(ROOT, "paper_1707_03268_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, mode: str, rank, tile_config) -> "int | None":
    """HBM bytes per launch of `kernel` measured with rocprofv3 FETCH_SIZE and
    WRITE_SIZE (scaled by a plain copy's counter reading), from the summary in
    profiles/, if it was taken on the current kernel sources with the same
    correlation tile configuration (tile_config None: any, for kernels that do
    not depend on it)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    want = [kernel, workload, mode, str(rank if mode != "direct_fp32" else 0),
            None if tile_config is None else str(tile_config), digest]
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 9 and t[0] == "traffic" and all(w is None or w == v for w, v in zip(want, t[1:7])):
                return int(float(t[7]) + float(t[8]))
    return None


def place_bytes(lay) -> int:
    """Algorithmic HBM bytes of one placement launch: every part and root
    response read once (FP32), every score (FP32) and placement offset pair
    (2 x int16) written once."""
    return 4 * lay.n_resp_part + 4 * lay.n_resp_root + 4 * lay.n_score + 2 * lay.n_offsets


# ----------------------------------------------------------------------------
# the workload as a stream of chunks that share one plan
# ----------------------------------------------------------------------------
def chunk_cells(wl, chunk: int):
    """Cells per chunk of `chunk` images, after checking that every chunk has
    the first chunk's pyramids shifted by a whole number of chunks (so one
    plan serves them all)."""
    n = len(wl.pyramids)
    if n % chunk:
        raise SystemExit(f"--chunk {chunk} does not divide the {n} images")
    first = wl.pyramids[chunk].levels[0].cell_offset if chunk < n else wl.total_cells
    for k in range(n // chunk):
        for i in range(chunk):
            a, b = wl.pyramids[i], wl.pyramids[k * chunk + i]
            if len(a.levels) != len(b.levels) or any(
                    (la.rows, la.cols, la.cell_offset + k * first) != (lb.rows, lb.cols, lb.cell_offset)
                    for la, lb in zip(a.levels, b.levels)):
                raise SystemExit("images of the chunks differ in shape: one plan cannot serve them")
    return first


class Stream:
    """A context planned for one chunk, the resident features of the whole
    workload, the reused score / offset buffers and the per-chunk detection
    buffers."""

    def __init__(self, torch, ctx, wl, feats, chunk: int, det_capacity: int):
        self.torch, self.ctx, self.wl, self.feats = torch, ctx, wl, feats
        self.chunk = chunk
        self.n_chunks = len(wl.pyramids) // chunk
        self.cells = chunk_cells(wl, chunk)
        self.lay = ctx.plan(wl.pyramids[:chunk])
        self.scores = torch.empty(max(self.lay.n_score, 1), dtype=torch.float32, device="cuda")
        self.offs = torch.empty(max(self.lay.n_offsets, 1), dtype=torch.int16, device="cuda")
        self.dets = torch.empty((self.n_chunks, det_capacity, 4), dtype=torch.int32, device="cuda")
        self.counts = torch.zeros((self.n_chunks, 1), dtype=torch.int64, device="cuda")
        self.tau = float("inf")

    def chunk_features(self, k: int):
        return self.feats[k * self.cells:(k + 1) * self.cells]

    def add_pipeline(self, ctx2) -> None:
        """A second context (same filters, decomposition and tile
        configuration, planned here for the same chunk) with its own score,
        offset and workspace buffers and its own stream: chunks then alternate
        between the two, so that one chunk's placement (VALU-bound) can run
        while the next chunk's correlation (MFMA- and store-bound) runs."""
        torch = self.torch
        lay2 = ctx2.plan(self.wl.pyramids[:self.chunk])
        assert lay2.n_score == self.lay.n_score and lay2.n_offsets == self.lay.n_offsets
        self.ctx2 = ctx2
        self.scores2 = torch.empty_like(self.scores)
        self.offs2 = torch.empty_like(self.offs)
        self.side = [torch.cuda.Stream(), torch.cuda.Stream()]     # default priority

    def step(self, mode: str, stream) -> None:
        if getattr(self, "ctx2", None) is None:
            for k in range(self.n_chunks):
                self.ctx.score_pyramid(mode, self.chunk_features(k), self.scores, self.offs, stream=stream)
                self.ctx.detect_into(self.scores, self.tau, self.dets[k], self.counts[k], stream=stream)
            return
        torch = self.torch
        start = torch.cuda.Event()
        start.record(stream)
        for s in self.side:
            s.wait_event(start)
        for k in range(self.n_chunks):
            c = k % 2
            ctx, sc, of = (self.ctx, self.scores, self.offs) if c == 0 else (self.ctx2, self.scores2, self.offs2)
            ctx.score_pyramid(mode, self.chunk_features(k), sc, of, stream=self.side[c])
            ctx.detect_into(sc, self.tau, self.dets[k], self.counts[k], stream=self.side[c])
        for s in self.side:
            done = torch.cuda.Event()
            done.record(s)
            stream.wait_event(done)

    def score_chunk(self, mode: str, k: int = 0) -> None:
        self.ctx.score_pyramid(mode, self.chunk_features(k), self.scores, self.offs)


def pick_tau(torch, scores, rate: float = 1e-4) -> float:
    """Detection threshold: the score exceeded by about `rate` of the finite
    scores (from every 16th score of one chunk)."""
    s = scores[::16]
    s = s[torch.isfinite(s)]
    if s.numel() == 0:
        return float("inf")
    k = max(1, int(rate * s.numel()))
    return float(torch.topk(s, k).values[-1].item())


def run_steps(torch, step, steps: int, warmup: int):
    """Warm up, then time exactly `steps` calls of step(stream) on torch's
    current stream with an event between consecutive steps.  Returns (mean
    ms, percentiles)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        step(stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        step(stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    pct = {"p10": float(np.percentile(per, 10)), "p50": float(np.percentile(per, 50)),
           "p90": float(np.percentile(per, 90))}
    return ms, pct


def stage_split(torch, ctx, step, steps: int):
    """Per-call stage times (HIP events the library records on the launch
    stream between its stages), averaged over the calls of `steps` steps; a
    pass of its own, since those events sit inside the calls."""
    step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    for _ in range(steps):
        step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    stages = ctx.stage_times()[0]
    ctx.set_profiling(False)
    return stages


def autotune(torch, ctx, mode, feats, lay):
    s_t = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
    o_t = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
    best, tms = ctx.autotune(mode, feats, s_t, o_t, reps=3)
    del s_t, o_t
    from paper_1707_03268_amd import tile_config_name
    return {"chosen": best, "name": tile_config_name(best),
            "median_ms": {tile_config_name(i): m for i, m in enumerate(tms) if m is not None}}


# ----------------------------------------------------------------------------
# FP64 oracle on a process pool (spawned workers, one BLAS thread each; the
# workers never touch the GPU)
# ----------------------------------------------------------------------------
_W: dict = {}


def _pool_init(config: int, n_images: int, bases: dict) -> None:
    try:
        from threadpoolctl import threadpool_limits
        _W["limit"] = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        pass
    import workloads
    preset = workloads.PRESETS[config]
    _W["wl"] = preset(n_images) if config in (4, 5) else preset()
    _W["bases"] = bases
    _W["cache"] = {}


def _oracle_task(task):
    """Score maps of one (image, root level, component) by the oracle: for
    each entry of `kinds`, 0 = direct correlation, R = tensor form with the
    basis bases[R].  Skipped (None) once `deadline` (wall clock) has passed."""
    image, level, comp, kinds, deadline = task
    if deadline is not None and time.time() > deadline:
        return None
    import oracle
    wl = _W["wl"]
    pyr = wl.pyramids[image]
    cache = _W["cache"]
    for l in (level, level - pyr.octave):
        if (image, l) not in cache:
            if len(cache) > 64:
                cache.clear()
            cache[(image, l)] = wl.level_features(image, l)
    Xr, Xp = cache[(image, level)], cache[(image, level - pyr.octave)]
    c = wl.bank.components[comp]
    out = {}
    t0 = time.time()
    for R in kinds:
        if R == 0:
            def resp(X, f):
                return oracle.correlate(X, f)
        else:
            U = _W["bases"][R]

            def resp(X, f):
                return oracle.tensor_response(X, f, U)
        rr = resp(Xr, wl.bank.filters[c.root])
        prs = [resp(Xp, wl.bank.filters[k]) for k in c.parts]
        sm = oracle.score_component(rr, prs, c.anchors, c.deform)
        out[R] = (sm.score, sm.offsets, sm.margin, int(rr.size + sum(p.size for p in prs)))
    return image, level, comp, t0, time.time(), out


def pool_size() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(MAX_POOL, n))


def run_oracle_pool(config, n_images, bases, tasks, workers):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_pool_init, initargs=(config, n_images, bases)) as pool:
        pool.map(_noop, range(workers), chunksize=1)      # workers started and initialised
        t_wall = time.time()
        res = [r for r in pool.imap_unordered(_oracle_task, tasks, chunksize=1) if r is not None]
        t_wall = time.time() - t_wall
    return res, t_wall


def _noop(_):
    return None


def compare_maps(results, kind, scores, offs, lay, tol, image_base=0):
    """GPU maps (host arrays of one plan) against the oracle results of
    `kind`: largest and p99.9 |score error| over finite oracle scores, and the
    placement agreement where the oracle's margin exceeds tol."""
    errs = []
    checked = total = bad = 0
    for image, level, comp, _, _, out in results:
        score, offsets, margin, _ = out[kind]
        k = lay.find(image - image_base, level, comp)
        Ho, Wo = score.shape
        g = scores[lay.map_score_off[k]:lay.map_score_off[k] + Ho * Wo].reshape(Ho, Wo)
        fin = np.isfinite(score)
        if fin.any():
            errs.append(np.abs(g[fin] - score[fin]))
        n_parts = offsets.shape[0]
        go = offs[lay.map_offs_off[k]:lay.map_offs_off[k] + Ho * Wo * n_parts * 2].reshape(n_parts, Ho, Wo, 2)
        chk = margin > tol
        total += chk.size
        checked += int(chk.sum())
        bad += int((chk[..., None] & (go != offsets)).any(-1).sum())
    e = np.concatenate(errs) if errs else np.zeros(1)
    return {"max_abs": float(e.max()), "p999_abs": float(np.quantile(e, 0.999)), "tolerance": tol,
            "argmax_checked": checked, "argmax_total": total, "argmax_mismatch": bad,
            "sample_maps": len(results)}


def oracle_diff(results, a, b):
    """Largest and p99.9 |s_a - s_b| between two oracle kinds on the same maps."""
    errs = []
    for *_, out in results:
        sa, sb = out[a][0], out[b][0]
        fin = np.isfinite(sa) & np.isfinite(sb)
        if fin.any():
            errs.append(np.abs(sa[fin] - sb[fin]))
    e = np.concatenate(errs) if errs else np.zeros(1)
    return {"max_abs": float(e.max()), "p999_abs": float(np.quantile(e, 0.999))}


def cpu_baseline(wl, mode, rank, budget_s, scores, offs, lay, workers):
    """The FP64 oracle (the headline's form: tensor at `rank` with the
    oracle's own basis, or direct) on image / frame 0, (root level,
    component) maps dealt to `workers` processes until `budget_s` of wall
    time; the GPU's score error on the maps it finished."""
    import oracle
    kind = 0 if mode == "direct_fp32" else rank
    bases = {} if kind == 0 else {rank: oracle.decompose(wl.bank.filters, rank).U}
    pyr = wl.pyramids[0]
    n_comp = len(wl.bank.components)
    order = list(range(0, n_comp, 7)) + [c for c in range(n_comp) if c % 7]
    tasks = [(0, l, c, (kind,), None) for l in range(pyr.octave, len(pyr.levels)) for c in order]
    n_img = len(wl.pyramids)
    # the deadline is set when the pool is up (spawned workers import numpy first)
    deadline_tasks = []
    res, wall = None, 0.0
    t_start = time.time()
    import multiprocessing as mp
    mctx = mp.get_context("spawn")
    with mctx.Pool(workers, initializer=_pool_init, initargs=(wl.config, n_img, bases)) as pool:
        pool.map(_noop, range(workers), chunksize=1)
        deadline = time.time() + budget_s
        deadline_tasks = [t[:4] + (deadline,) for t in tasks]
        t0 = time.time()
        res = [r for r in pool.imap_unordered(_oracle_task, deadline_tasks, chunksize=1) if r is not None]
        wall = time.time() - t0
    n_resp = sum(r[5][kind][3] for r in res)
    busy = sum(r[4] - r[3] for r in res)
    span = (max(r[4] for r in res) - min(r[3] for r in res)) if res else 0.0
    comps_done = len({r[2] for r in res})
    err = compare_maps(res, kind, scores, offs, lay, TOL[mode])
    form = "direct" if kind == 0 else f"tensor R={rank}, the oracle's own basis"
    return {
        "value": n_resp / max(span, 1e-9), "unit": "resp/s", "cores": workers, "kind": "oracle",
        "single_core_value": n_resp / max(busy, 1e-9),
        "sample": f"FP64 oracle ({form}) on {workers} worker processes with one BLAS thread each, "
                  f"{len(res)} of {len(tasks)} (root level, component) score maps of "
                  f"{'frame' if wl.config == 5 else 'image'} 0 ({comps_done} components, {n_resp} "
                  f"responses) in {span:.1f} s of wall time (pool up after {t0 - t_start:.1f} s)",
    }, err


# ----------------------------------------------------------------------------
# rank sweep on the 500x375 image with the 1080-filter bank
# ----------------------------------------------------------------------------
def rank_sweep(torch, workers, steps: int, n_comps: int = 24):
    import oracle
    import workloads
    from paper_1707_03268_amd import Context
    wl = workloads.config3()
    feats = workloads.features_device(wl, "cuda")
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    n_comp = len(wl.bank.components)
    comps = list(range(0, n_comp, max(1, n_comp // n_comps)))[:n_comps]
    pyr = wl.pyramids[0]
    bases = {}
    gaps = {}
    gpu = {}
    for R in SWEEP_RANKS:
        dec = oracle.decompose(wl.bank.filters, R)
        bases[R] = dec.U
        s = dec.sigma
        gaps[R] = float((s[R - 1] - s[R]) / s[0]) if R < len(s) else None
        ctx.decompose(R)
        lay = ctx.plan(wl.pyramids)
        autotune(torch, ctx, "tensor_bf16", feats, lay)
        sc = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
        of = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")

        def step(st):
            ctx.score_pyramid("tensor_bf16", feats, sc, of, stream=st)
        stages = stage_split(torch, ctx, step, 3)
        ms, _ = run_steps(torch, step, steps, 2)
        flops, _, _ = corr_work(wl.pyramids, wl.bank.shapes, wl.bank.components, "tensor_bf16", R)
        tf = flops / (stages["correlation"] * 1e-3) / 1e12
        gpu[R] = {"ms_per_step": ms, "value": lay.n_resp / (ms * 1e-3),
                  "correlation_tflops": tf, "correlation_frac_bf16_mfma": tf / PEAK_BF16_TFLOPS,
                  "scores": sc.cpu().numpy(), "offs": of.cpu().numpy(), "lay": lay}
        log(f"rank sweep R={R}: {ms:.3f} ms/step, correlation {tf:.0f} TFLOP/s")
    ctx.close()
    del feats
    tasks = [(0, l, c, (0,) + SWEEP_RANKS, None) for l in range(pyr.octave, len(pyr.levels)) for c in comps]
    t0 = time.time()
    res, _ = run_oracle_pool(3, 1, bases, tasks, workers)
    log(f"rank sweep oracle: {len(res)} maps in {time.time() - t0:.1f} s")
    out = {"workload": wl.name, "mode": "tensor_bf16",
           "sample": f"{len(comps)} of {n_comp} components on every root level ({len(res)} score maps), "
                     "oracle basis U_R from oracle.decompose", "ranks": {}}
    for R in SWEEP_RANKS:
        g = gpu[R]
        prec = compare_maps(res, R, g["scores"], g["offs"], g["lay"], TOL["tensor_bf16"])
        total = compare_maps(res, 0, g["scores"], g["offs"], g["lay"], TOL["tensor_bf16"])
        out["ranks"][str(R)] = {
            "ms_per_step": g["ms_per_step"], "value": g["value"],
            "correlation_tflops": g["correlation_tflops"],
            "correlation_frac_bf16_mfma": g["correlation_frac_bf16_mfma"],
            "spectral_gap_rel": gaps[R],
            "gpu_vs_oracle_tensor": prec,                       # precision error at this rank
            "oracle_tensor_vs_oracle_direct": oracle_diff(res, R, 0),   # truncation error
            "gpu_vs_oracle_direct": {"max_abs": total["max_abs"], "p999_abs": total["p999_abs"],
                                     "argmax_mismatch_above_margin": total["argmax_mismatch"],
                                     "argmax_checked": total["argmax_checked"]},
        }
    return out


# ----------------------------------------------------------------------------
def hog_leg(torch, ctx, wl, score_ms_per_image: float, reps: int = 10):
    """HOG feature pyramid of image 0 (a synthetic image of its size, every
    level of its pyramid), timed like the steps, beside the scoring time per
    image (the paper finds score estimation about 20x the feature extraction,
    Section 1)."""
    import workloads
    w, h = wl.image_sizes[0]
    pyr = wl.pyramids[0]
    base = pyr.levels[0].cell_offset
    levels = [(off - base, r, c, pr, pc, cell, inv)
              for (off, r, c, pr, pc, cell, inv) in workloads.hog_levels(pyr)]
    n = sum(r * c for _, r, c, *_ in levels)
    pixels = sum((r - 2 * pr) * cell * (c - 2 * pc) * cell for _, r, c, pr, pc, cell, _ in levels)
    img = torch.from_numpy(workloads.synthetic_image(0, w, h)).cuda()
    out = torch.empty((n, 32), dtype=torch.float32, device="cuda")
    ms, pct = run_steps(torch, lambda st: ctx.hog_pyramid(img, levels, out, stream=st), reps, 2)
    del out, img
    return {"image": f"{w}x{h}", "levels": len(levels), "cells": n, "resized_pixels": pixels,
            "ms_per_image": ms, "mpixels_per_s": pixels / (ms * 1e-3) / 1e6, **pct,
            "score_ms_per_image": score_ms_per_image,
            "score_over_features": score_ms_per_image / ms if ms > 0 else None}


def dt_methods(torch, reps: int = 10):
    """Single-map distance transform, window scans against lower envelopes,
    on a 1920x1080 frame's largest part map (277 x 497) and a 1024 x 1024
    map, with the workloads' deformation (0.05) and a weak one (0.001)."""
    from paper_1707_03268_amd import distance_transform
    out = {}
    rng = np.random.default_rng(0)
    for rows, cols in ((277, 497), (1024, 1024)):
        resp = torch.from_numpy(rng.standard_normal((rows, cols)).astype(np.float32)).cuda()
        D = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
        ay = torch.empty((rows, cols), dtype=torch.int32, device="cuda")
        ax = torch.empty_like(ay)
        for q in (0.05, 0.001):
            d = [0.02, q, -0.01, q]
            for method in ("window", "envelope"):
                ms, _ = run_steps(torch, lambda st: distance_transform(resp, d, D, ay, ax, stream=st, method=method),
                                  reps, 2)
                out[f"{rows}x{cols} d={q} {method}"] = ms
    return out


def legs(torch, wl, args, n_images, feats_all):
    """The other forms on the first n_images images / frames, in a context of
    their own: direct FP32, the tensor form in its three operand precisions
    (each autotuned) and the per-filter CP form with pruning."""
    import workloads
    from paper_1707_03268_amd import Context
    pyrs = wl.pyramids[:n_images]
    end = pyrs[-1].levels[-1].cell_offset + pyrs[-1].levels[-1].rows * pyrs[-1].levels[-1].cols
    feats = feats_all[:end]
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    ctx.decompose(args.rank)
    lay = ctx.plan(pyrs)
    sc = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
    of = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
    shapes, comps = wl.bank.shapes, wl.bank.components
    steps = max(2, min(args.steps, 5))

    def measure(mode, f=feats):
        def step(st):
            ctx.score_pyramid(mode, f, sc, of, stream=st)
        stages = stage_split(torch, ctx, step, 2)
        ms, _ = run_steps(torch, step, steps, 1)
        return ms, stages

    out = {"images": n_images, "resp_per_step": lay.n_resp}
    runs = {}
    for m in ("tensor_fp32", "tensor_bf16", "tensor_fp8"):
        if args.autotune:
            autotune(torch, ctx, m, feats, lay)
        ms, stages = measure(m)
        runs[m] = (ms, stages, sc.clone())
        log(f"legs {m}: {ms:.3f} ms/step, stages {stages}")
    ref = runs["tensor_fp32"][2]
    keep = torch.isfinite(ref)
    prec = {}
    for m, (ms, stages, msc) in runs.items():
        flops, _, _ = corr_work(pyrs, shapes, comps, m, args.rank)
        peak = {"tensor_bf16": PEAK_BF16_TFLOPS, "tensor_fp8": PEAK_FP8_TFLOPS}.get(m, PEAK_FP32_TFLOPS)
        tf = flops / (stages["correlation"] * 1e-3) / 1e12
        diff = (msc - ref).abs()[keep]
        prec[m] = {"value": lay.n_resp / (ms * 1e-3), "ms_per_step": ms,
                   "stages_ms": {k: round(v, 4) for k, v in stages.items()},
                   "tile_config": ctx.get_tile_config(m),
                   "correlation_tflops": tf, "correlation_peak_tflops": peak,
                   "correlation_frac_mfma": tf / peak,
                   "max_abs_score_diff_vs_tensor_fp32": float(diff.max()) if diff.numel() else 0.0,
                   "same_finite_pattern": bool(torch.equal(torch.isfinite(msc), keep))}
    out["precisions"] = prec
    del runs
    if not args.no_direct:
        dms, dstages = measure("direct_fp32")
        dflops, _, _ = corr_work(pyrs, shapes, comps, "direct_fp32", 32)
        tf = dflops / (dstages["correlation"] * 1e-3) / 1e12
        out["direct_fp32"] = {"value": lay.n_resp / (dms * 1e-3), "ms_per_step": dms,
                              "stages_ms": {k: round(v, 4) for k, v in dstages.items()},
                              "correlation_tflops": tf, "correlation_frac_fp32_mfma": tf / PEAK_FP32_TFLOPS}
        log(f"legs direct_fp32: {dms:.3f} ms/step")
    if args.cp_rank > 0:
        t0 = time.time()
        cp_err = ctx.decompose_cp(args.cp_rank, max_iters=60, tol=1e-9)
        als_s = time.time() - t0
        cms, cstages = measure("cp_fp32")
        mults = mult_counts(pyrs, shapes, comps, args.rank, args.cp_rank)
        ctf = 2 * mults["cp"] / (cstages["correlation"] * 1e-3) / 1e12
        cp = {"rank": args.cp_rank, "value": lay.n_resp / (cms * 1e-3), "ms_per_step": cms,
              "stages_ms": {k: round(v, 4) for k, v in cstages.items()},
              "als_seconds": als_s, "als_rel_err_mean": float(cp_err.mean()),
              "als_rel_err_max": float(cp_err.max()),
              "roofline": {"bound": "alu", "achieved": ctf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                           "frac": ctf / PEAK_FP32_TFLOPS, "kernel": "cp_corr_kernel",
                           "flops": 2 * mults["cp"]},
              "multiplies": mults,
              "formula1_gain_6x6_parts": 6 * 6 * 32 / (args.cp_rank * (6 + 6 + 32))}
        log(f"legs cp_fp32 R={args.cp_rank}: {cms:.3f} ms/step (ALS {als_s:.1f} s)")
        if args.plant > 0:
            # convolution shortening: objects planted into a host copy of these
            # images' features are the positives the thresholds are fitted on
            sub = workloads.Workload(wl.name, wl.config, pyrs, wl.bank, end, wl.feat_seed, wl.padded,
                                     wl.image_sizes[:n_images])
            host = feats.cpu().numpy()
            pfeat_host, pos = workloads.plant_objects(sub, host, args.plant)
            pfeat = torch.from_numpy(pfeat_host).cuda()
            ums, ustages = measure("cp_fp32", pfeat)
            uscores = sc.cpu().numpy()
            t0 = time.time()
            ctx.fit_thresholds(pfeat_host, pos, margin=1e-3)
            fit_s = time.time() - t0
            pms, pstages = measure("cp_fp32", pfeat)
            ps = sc.cpu().numpy()
            fin = np.isfinite(uscores)
            rejected = int((np.isneginf(ps) & fin).sum())
            kept = ~np.isneginf(ps)
            pos_ok = all(np.isfinite(ps[lay.map_score_off[lay.find(i, l, c)] + y * int(lay.map_cols[lay.find(i, l, c)]) + x])
                         for (i, l, c, y, x) in pos)
            cp["pruning"] = {"positives": len(pos),
                             "positive_rule": f"{args.plant} planted object(s) of every component per image",
                             "threshold_margin": 1e-3, "fit_seconds": fit_s,
                             "rejected_fraction": rejected / max(int(fin.sum()), 1),
                             "positives_kept": bool(pos_ok),
                             "survivors_equal_unpruned": bool(np.array_equal(ps[kept], uscores[kept])),
                             "unpruned_ms_per_step": ums,
                             "unpruned_stages_ms": {k: round(v, 4) for k, v in ustages.items()},
                             "ms_per_step": pms, "stages_ms": {k: round(v, 4) for k, v in pstages.items()},
                             "speedup_vs_unpruned": ums / pms}
            ctx.set_thresholds(None)
            del pfeat
            log(f"legs cp_fp32 planted: {ums:.3f} ms/step unpruned, {pms:.3f} pruned")
        out["cp_fp32"] = cp
    ctx.close()
    return out


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=5, help="workload preset 1..5")
    ap.add_argument("--images", type=int, default=0, help="images/frames for presets 4 and 5 (0: preset)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="images per plan of a stream of equally shaped images (0: 16 for preset 5, "
                         "else all images in one plan)")
    ap.add_argument("--mode", default="tensor_bf16", choices=list(TOL))
    ap.add_argument("--rank", type=int, default=16)
    ap.add_argument("--leg-images", type=int, default=0,
                    help="images / frames the other forms are timed on (0: 4 for preset 5, else all)")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="skip the other forms (direct FP32, FP32 / FP8 tensor, CP)")
    ap.add_argument("--no-direct", action="store_true", help="skip the direct FP32 comparison run")
    ap.add_argument("--cp-rank", type=int, default=6,
                    help="rank of the per-filter CP form timed for comparison (0: skip)")
    ap.add_argument("--plant", type=int, default=1,
                    help="objects of every component planted per image as positives for the CP form's pruning "
                         "thresholds (0: skip pruning)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle wall time (0: skip)")
    ap.add_argument("--rank-sweep", dest="rank_sweep", action="store_true", default=True)
    ap.add_argument("--no-rank-sweep", dest="rank_sweep", action="store_false",
                    help="skip the rank sweep R = 4, 8, 16, 32 on the 500x375 image")
    ap.add_argument("--launch", default="batched", choices=["batched", "per_level", "graph", "overlap"],
                    help="launch strategy of the timed steps")
    ap.add_argument("--no-compare-launch", dest="compare_launch", action="store_false",
                    help="skip timing every launch strategy on one chunk")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default correlation tile configuration instead of timing them all")
    ap.add_argument("--tile-config", type=int, default=None, help="correlation tile configuration index")
    ap.add_argument("--contexts", type=int, default=1, choices=[1, 2],
                    help="contexts the stream's chunks alternate between, each on its own stream")
    ap.add_argument("--no-dt-methods", dest="dt_methods", action="store_false",
                    help="skip timing the single-map transform's two methods")
    ap.add_argument("--no-hog", dest="hog", action="store_false",
                    help="skip timing the HOG feature pyramid of one image")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device three times (a known-size copy kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path has no "
              f"multi-GPU component in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_1707_03268_amd import Context, tile_config_name

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst
    preset = workloads.PRESETS[args.config]
    wl = preset(args.images) if (args.config in (4, 5) and args.images) else preset()
    n_img = len(wl.pyramids)
    chunk = args.chunk or (min(16, n_img) if args.config == 5 else n_img)
    log(f"workload: {wl.name}; {n_img // chunk} chunk(s) of {chunk}")
    t0 = time.time()
    feats = workloads.features_device(wl, "cuda")
    torch.cuda.synchronize()
    log(f"features: {feats.shape[0]} cells generated on the device in {time.time() - t0:.1f} s")
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    if args.mode != "direct_fp32":
        ctx.decompose(args.rank)
    S = Stream(torch, ctx, wl, feats, chunk, det_capacity=1 << 16)
    lay = S.lay
    n_resp = lay.n_resp * S.n_chunks
    log(f"plan: {lay.n_resp} responses per chunk, {n_resp} per step, {lay.n_maps} score maps per chunk, "
        f"workspace {lay.workspace_bytes / 2**30:.1f} GiB")

    tuning = None
    if args.autotune:
        tuning = autotune(torch, ctx, args.mode, S.chunk_features(0), lay)
        log(f"autotune: {tuning}")
    elif args.tile_config is not None:
        ctx.set_tile_config(args.mode, args.tile_config)
    S.score_chunk(args.mode, 0)
    S.tau = pick_tau(torch, S.scores)
    if args.contexts == 2 and S.n_chunks > 1:
        ctx2 = Context(0)
        ctx2.load_filters(wl.bank.filters, wl.bank.components)
        if args.mode != "direct_fp32":
            ctx2.decompose(args.rank)
        ctx2.set_tile_config(args.mode, ctx.get_tile_config(args.mode))
        S.add_pipeline(ctx2)
        log("pipeline: chunks alternate between two contexts on two streams")

    def step(st):
        S.step(args.mode, st)

    ctx.set_launch(args.launch)
    # the stage split runs the chunks one after another on one context (the
    # kernels alone), also when the timed steps alternate two contexts
    pipe, S.ctx2 = getattr(S, "ctx2", None), None
    stages = stage_split(torch, ctx, step, 1) if args.launch != "graph" else {}
    S.ctx2 = pipe
    ms, pct = run_steps(torch, step, args.steps, args.warmup)
    ctx.set_launch("batched")
    counts = S.counts.cpu().numpy().ravel()
    n_ctx = 2 if getattr(S, "ctx2", None) is not None else 1
    if n_ctx == 2:                                   # free the second workspace for the other legs
        S.ctx2.close()
        S.ctx2 = None
        del S.scores2, S.offs2
        torch.cuda.empty_cache()
    value = n_resp / (ms * 1e-3)
    log(f"{args.mode} ({args.launch}): {ms:.3f} ms/step, {value:.4g} resp/s, stages per chunk {stages}, "
        f"detections per step {int(counts.sum())} (tau {S.tau:.4g})")

    launches = None
    if args.compare_launch:
        launches = {"images": chunk}
        for launch in ("batched", "per_level", "graph", "overlap"):
            ctx.set_launch(launch)
            lms, lpct = run_steps(torch, lambda st: ctx.score_pyramid(args.mode, S.chunk_features(0), S.scores,
                                                                      S.offs, stream=st),
                                  max(2, min(args.steps, 10)), 1)
            launches[launch] = {"ms_per_step": lms, "resp_per_s": lay.n_resp / (lms * 1e-3), **lpct}
            log(f"launch {launch}: {lms:.3f} ms per chunk")
        ctx.set_launch("batched")

    hog = None
    if args.hog and wl.padded:
        hog = hog_leg(torch, ctx, wl, ms / n_img)
        log(f"hog: {hog}")
    dtm = dt_methods(torch) if args.dt_methods else None
    if dtm:
        log(f"distance transform methods (ms): {dtm}")

    # roofline of each kernel (per launch = per chunk); the headline object is the dominant one
    pyrs = wl.pyramids[:chunk]
    shapes, comps = wl.bank.shapes, wl.bank.components
    flops, cbytes, _ = corr_work(pyrs, shapes, comps, args.mode, args.rank)
    peak_mfma = {"tensor_bf16": PEAK_BF16_TFLOPS, "tensor_fp8": PEAK_FP8_TFLOPS}.get(args.mode, PEAK_FP32_TFLOPS)
    corr_ms = stages.get("correlation", float("nan"))
    ai = flops / cbytes
    corr = {"kernel": "corr_kernel", "ms": corr_ms, "tflops": flops / (corr_ms * 1e-3) / 1e12,
            "gbs": cbytes / (corr_ms * 1e-3) / 1e9, "flops": flops, "bytes": cbytes,
            "arith_intensity": ai}
    corr["frac_mfma"] = corr["tflops"] / peak_mfma
    corr["frac_attainable"] = corr["tflops"] / min(peak_mfma, ai * PEAK_HBM_GBS / 1e3)
    wtag = f"c{args.config}x{chunk}"
    rf_corr = {"bound": "mfma", "achieved": corr["tflops"], "peak": peak_mfma, "unit": "TFLOP/s",
               "frac": corr["frac_mfma"], "kernel": "corr_kernel", "flops": flops, "bytes": cbytes,
               "traffic": recorded_traffic("corr_kernel", wtag, args.mode, args.rank,
                                           ctx.get_tile_config(args.mode))}
    pbytes = place_bytes(lay)
    place_ms = stages.get("placement", float("nan"))
    pgbs = pbytes / (place_ms * 1e-3) / 1e9
    rf_place = {"bound": "hbm", "achieved": pgbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": pgbs / PEAK_HBM_GBS, "kernel": "place_kernel", "bytes": pbytes,
                "traffic": recorded_traffic("place_kernel", wtag, args.mode, args.rank, None)}
    roof = dict(rf_corr if not (place_ms > corr_ms) else rf_place)

    cpu = err = None
    if args.cpu_budget > 0:
        S.score_chunk(args.mode, 0)           # frame / image 0's maps for the comparison
        sc_host, of_host = S.scores.cpu().numpy(), S.offs.cpu().numpy()
        log("cpu baseline (oracle) ...")
        cpu, err = cpu_baseline(wl, args.mode, args.rank, args.cpu_budget, sc_host, of_host, lay, pool_size())
        del sc_host, of_host
        log(f"cpu baseline: {cpu}")
    leg = None
    if args.legs and args.mode != "direct_fp32":
        n_leg = args.leg_images or (min(4, n_img) if args.config == 5 else n_img)
        leg = legs(torch, wl, args, n_leg, feats)
    n_chunks, tau = S.n_chunks, S.tau
    sweep = None
    if args.rank_sweep and args.mode == "tensor_bf16":
        del S
        ctx.close()
        del feats
        torch.cuda.empty_cache()
        sweep = rank_sweep(torch, pool_size(), max(3, min(args.steps, 10)))

    dtype = {"tensor_bf16": "bf16", "tensor_fp32": "f32", "direct_fp32": "f32", "tensor_fp8": "fp8e4m3"}[args.mode]
    direct = (leg or {}).get("direct_fp32")
    out = {
        "metric": METRIC, "value": value, "unit": "resp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "mode": args.mode,
                   "rank": None if args.mode == "direct_fp32" else args.rank,
                   "images": n_img, "chunk": chunk, "resp_per_step": n_resp,
                   "score_maps_per_step": lay.n_maps * n_chunks, "detection_tau": tau},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms_per_chunk": {k: round(v, 4) for k, v in stages.items()},
        "step_ms_percentiles": pct,
        "detections_per_step": int(counts.sum()),
        "launch": args.launch,
        "contexts": n_ctx,
        "launch_strategies": launches,
        "tile_config": tuning if tuning else {"chosen": args.tile_config},
        "correlation": corr,
        "placement_roofline": rf_place,
        "legs": {k: v for k, v in (leg or {}).items() if k not in ("precisions", "direct_fp32", "cp_fp32")} or None,
        "direct_fp32": direct,
        "tensor_vs_direct": (leg["precisions"][args.mode]["value"] / direct["value"])
        if (leg and direct and args.mode in leg.get("precisions", {})) else None,
        "precisions": (leg or {}).get("precisions"),
        "cp_fp32": (leg or {}).get("cp_fp32"),
        "score_error_vs_oracle": err,
        "hog_features": hog,
        "distance_transform_ms": dtm,
        "rank_sweep": sweep,
        "paper_context": "the paper reports up to 4.5x fewer convolutions than DPM v5 at matched detection "
                         "quality, on hardware it does not state",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
