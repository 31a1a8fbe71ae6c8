"""Benchmark of the DPM scoring path on one MI355X.

One step = one dpmt_score_pyramid call over the whole batch: projection,
correlation of every level with every filter, distance transform of every
part map at the anchors, and score assembly.  Inputs are resident in HBM
before the timed region.  The default workload is the 500x375 image's
36-level pyramid with the 1080-filter bank (20 classes x 6 components x
(root + 8 parts)), tensor form in BF16 at rank 16, with the direct FP32 path
timed on the same workload for the tensor-vs-direct comparison.

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


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def corr_work(wl, mode: str, rank: int):
    """Algorithmic flops and HBM bytes of one correlation launch (all filters,
    all levels): 2*h*w*C flops per response (C = 32 direct, R tensor); bytes =
    operand features read once per level + packed filters read once + FP32
    responses written once."""
    shapes = wl.bank.shapes
    roots = [c.root for c in wl.bank.components]
    parts = sorted({p for c in wl.bank.components for p in c.parts})
    C = 32 if mode == "direct_fp32" else rank
    esz = {"direct_fp32": 4, "tensor_fp32": 4, "tensor_bf16": 2, "tensor_fp8": 1}[mode]
    flops = 0
    resp = 0
    feat_bytes = 0
    for pyr in wl.pyramids:
        L = len(pyr.levels)
        for l, lv in enumerate(pyr.levels):
            used = False
            for ks, ok in ((roots, l >= pyr.octave), (parts, l + pyr.octave < L)):
                if not ok:
                    continue
                for k in ks:
                    h, w = shapes[k]
                    if lv.rows >= h and lv.cols >= w:
                        n = (lv.rows - h + 1) * (lv.cols - w + 1)
                        resp += n
                        flops += 2 * n * h * w * C
                        used = True
            if used:
                feat_bytes += lv.rows * lv.cols * C * esz
    filt_bytes = sum(h * w * C * esz for (h, w) in shapes)
    return flops, feat_bytes + filt_bytes + 4 * resp, resp


def mult_counts(wl, rank: int, cp_rank: int) -> dict:
    """Multiplications per step of the three ways to correlate (Section 4's
    counting): direct h*w*32 per response; per-filter CP form R*(32 + h + w)
    per response (channel contraction, then 1-D correlations along x and y);
    shared feature-mode basis h*w*R per response plus 32*R per projected cell."""
    shapes = wl.bank.shapes
    roots = [c.root for c in wl.bank.components]
    parts = sorted({p for c in wl.bank.components for p in c.parts})
    out = {"direct": 0, "cp": 0, "shared_basis": 0}
    for pyr in wl.pyramids:
        L = len(pyr.levels)
        for l, lv in enumerate(pyr.levels):
            used = False
            for ks, ok in ((roots, l >= pyr.octave), (parts, l + pyr.octave < L)):
                if not ok:
                    continue
                for k in ks:
                    h, w = shapes[k]
                    if lv.rows >= h and lv.cols >= w:
                        n = (lv.rows - h + 1) * (lv.cols - w + 1)
                        out["direct"] += n * h * w * 32
                        out["cp"] += n * cp_rank * (32 + h + w)
                        out["shared_basis"] += n * h * w * rank
                        used = True
            if used:
                out["shared_basis"] += lv.rows * lv.cols * 32 * rank
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


def recorded_traffic(kernel: str, config: int, mode: str, rank, tile_config: int) -> "int | None":
    """HBM bytes per launch of `kernel` measured with rocprofv3 FETCH_SIZE and
    WRITE_SIZE (scaled by a plain copy's counter reading), from the summary in
    profiles/, if it was taken on the current kernel sources with the same
    correlation tile configuration (tile_config None: any, for kernels that do
    not depend on it)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    want = [kernel, f"c{config}", mode, str(rank if mode != "direct_fp32" else 0),
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


def run_mode(ctx, mode, feats, steps, warmup, torch, launch="batched", profile=False):
    """Warm up, then time exactly `steps` calls on torch's current stream with
    an event between consecutive calls.  With `profile` the library also
    records events between its stages, for the per-stage split (a run of its
    own: those events sit inside the timed calls).  Returns (mean ms,
    per-stage ms, step percentiles, scores, offsets)."""
    lay = ctx.layout
    scores = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
    offs = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
    stream = torch.cuda.current_stream()
    ctx.set_launch(launch)
    for _ in range(warmup):
        ctx.score_pyramid(mode, feats, scores, offs, stream=stream)
    torch.cuda.synchronize()
    ctx.set_profiling(profile)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        ctx.score_pyramid(mode, feats, scores, offs, stream=stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    pct = {"p10": float(np.percentile(per, 10)), "p50": float(np.percentile(per, 50)),
           "p90": float(np.percentile(per, 90))}
    stages = ctx.stage_times()[0] if profile else {}
    ctx.set_profiling(False)
    ctx.set_launch("batched")
    return ms, stages, pct, scores, offs


def measure(ctx, mode, feats, steps, warmup, torch, launch="batched"):
    """The stage split from a profiled pass, then the step time (with its
    percentiles and the outputs) from a pass with no events inside the calls."""
    _, stages, _, _, _ = run_mode(ctx, mode, feats, steps, warmup, torch, profile=True)
    ms, _, pct, scores, offs = run_mode(ctx, mode, feats, steps, warmup, torch, launch=launch)
    return ms, stages, pct, scores, offs


def cpu_baseline(wl, mode, U, budget_s, scores, offs, lay, torch):
    """The FP64 oracle on a bounded sample of the workload (whole components,
    every root level), single BLAS thread; also the GPU's score error on the
    same sample."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    s_cpu = scores.cpu().numpy()
    o_cpu = offs.cpu().numpy()
    cache = {}
    n_resp = 0
    n_maps = 0
    t_start = time.perf_counter()
    max_err = 0.0
    errs = []
    arg_checked = arg_total = arg_bad = 0
    comps = list(range(len(wl.bank.components)))
    # visit components spread over the classes, every root level of image 0
    order = comps[::7] + [c for c in comps if c % 7]
    pyr = wl.pyramids[0]
    resp_of = (lambda X, f: oracle.correlate(X, f)) if U is None else \
              (lambda X, f: oracle.tensor_response(X, f, U))
    tol = TOL[mode]
    comp_done = 0
    for ci in order:
        c = wl.bank.components[ci]
        for l in range(pyr.octave, len(pyr.levels)):
            for key in ((0, l), (0, l - pyr.octave)):
                if key not in cache:
                    cache[key] = wl.level_features(*key)
            Xr, Xp = cache[(0, l)], cache[(0, l - pyr.octave)]
            rr = resp_of(Xr, wl.bank.filters[c.root])
            prs = [resp_of(Xp, wl.bank.filters[k]) for k in c.parts]
            sm = oracle.score_component(rr, prs, c.anchors, c.deform)
            n_resp += rr.size + sum(p.size for p in prs)
            n_maps += 1
            k = lay.find(0, l, ci)
            Ho, Wo = sm.score.shape
            g = s_cpu[lay.map_score_off[k]:lay.map_score_off[k] + Ho * Wo].reshape(Ho, Wo)
            fin = np.isfinite(sm.score)
            if fin.any():
                e = np.abs(g[fin] - sm.score[fin])
                errs.append(e)
            go = o_cpu[lay.map_offs_off[k]:lay.map_offs_off[k] + Ho * Wo * len(c.parts) * 2]
            go = go.reshape(len(c.parts), Ho, Wo, 2)
            chk = sm.margin > tol
            arg_total += chk.size
            arg_checked += int(chk.sum())
            arg_bad += int((chk[..., None] & (go != sm.offsets)).any(-1).sum())
        comp_done += 1
        if time.perf_counter() - t_start > budget_s:
            break
    elapsed = time.perf_counter() - t_start
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    e = np.concatenate(errs) if errs else np.zeros(1)
    return {
        "value": n_resp / elapsed, "unit": "resp/s", "cores": 1, "kind": "oracle",
        "sample": f"FP64 oracle ({'direct' if U is None else 'tensor R=%d' % U.shape[1]}), "
                  f"{comp_done} of {len(comps)} components on every root level of image 0 "
                  f"({n_maps} score maps, {n_resp} responses, {elapsed:.1f} s), one BLAS thread",
    }, {
        "max_abs": float(e.max()), "p999_abs": float(np.quantile(e, 0.999)),
        "tolerance": tol, "argmax_checked": arg_checked, "argmax_total": arg_total,
        "argmax_mismatch": arg_bad, "sample_maps": n_maps,
    }


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, help="workload preset 1..5")
    ap.add_argument("--images", type=int, default=0, help="images/frames for presets 4 and 5 (0: preset)")
    ap.add_argument("--mode", default="tensor_bf16", choices=list(TOL))
    ap.add_argument("--rank", type=int, default=16)
    ap.add_argument("--no-direct", action="store_true", help="skip the direct FP32 comparison run")
    ap.add_argument("--no-precisions", dest="precisions", action="store_false",
                    help="skip the runs of the other tensor-form precisions (FP32, BF16, FP8)")
    ap.add_argument("--cp-rank", type=int, default=6,
                    help="rank of the per-filter CP form timed for comparison (0: skip)")
    ap.add_argument("--plant", type=int, default=1,
                    help="objects of every component planted per image as positives for the CP form's pruning "
                         "thresholds (0: skip pruning)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work (0: skip)")
    ap.add_argument("--launch", default="batched", choices=["batched", "per_level", "graph", "overlap"],
                    help="launch strategy of the timed steps")
    ap.add_argument("--compare-launch", action="store_true",
                    help="also time every launch strategy (batched, per level, graph)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default correlation tile configuration instead of timing them all")
    ap.add_argument("--tile-config", type=int, default=None, help="correlation tile configuration index")
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
    log(f"workload: {wl.name}")
    feats = torch.from_numpy(wl.features()).cuda()
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    U = None
    if args.mode != "direct_fp32":
        sigma, U = ctx.decompose(args.rank)
    lay = ctx.plan(wl.pyramids)
    log(f"plan: {lay.n_resp} responses/step, {lay.n_maps} score maps, workspace "
        f"{lay.workspace_bytes / 2**20:.0f} MiB")

    tuning = None
    if args.autotune:
        s_t = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
        o_t = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
        best, tms = ctx.autotune(args.mode, feats, s_t, o_t, reps=3)
        del s_t, o_t
        tuning = {"chosen": best, "name": tile_config_name(best),
                  "median_ms": {tile_config_name(i): m for i, m in enumerate(tms) if m is not None}}
        log(f"autotune: {tuning}")
    elif args.tile_config is not None:
        ctx.set_tile_config(args.mode, args.tile_config)

    # stage split from a profiled pass of the batched strategy (a graph launch
    # has none), then the timed steps with no events inside the calls
    ms, stages, pct, scores, offs = measure(ctx, args.mode, feats, args.steps, args.warmup, torch,
                                            launch=args.launch)
    value = lay.n_resp / (ms * 1e-3)
    log(f"{args.mode} ({args.launch}): {ms:.3f} ms/step, {value:.4g} resp/s, stages {stages}")

    launches = None
    if args.compare_launch:
        launches = {}
        for launch in ("batched", "per_level", "graph", "overlap"):
            lms, _, lpct, _, _ = run_mode(ctx, args.mode, feats, max(2, min(args.steps, 10)), 1,
                                          torch, launch=launch)
            launches[launch] = {"ms_per_step": lms, "resp_per_s": lay.n_resp / (lms * 1e-3), **lpct}
            log(f"launch {launch}: {lms:.3f} ms/step")

    direct = None
    if not args.no_direct and args.mode != "direct_fp32":
        dsteps = max(2, min(args.steps, 5))
        dms, dstages, _, _, _ = measure(ctx, "direct_fp32", feats, dsteps, 1, torch)
        dflops, dbytes, _ = corr_work(wl, "direct_fp32", 32)
        direct = {"value": lay.n_resp / (dms * 1e-3), "ms_per_step": dms,
                  "stages_ms": {k: round(v, 4) for k, v in dstages.items()},
                  "correlation_tflops": dflops / (dstages["correlation"] * 1e-3) / 1e12,
                  "correlation_frac_fp32_mfma": dflops / (dstages["correlation"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
        log(f"direct_fp32: {dms:.3f} ms/step")

    # the tensor form in its other operand precisions, each autotuned like the
    # headline; score differences against the FP32 tensor form (which the GPU
    # tests hold within 1e-4 of the FP64 oracle)
    precisions = None
    if args.precisions and args.mode != "direct_fp32":
        runs = {args.mode: (ms, stages, scores)}
        for m in ("tensor_fp32", "tensor_bf16", "tensor_fp8"):
            if m in runs:
                continue
            if args.autotune:
                s_t = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
                o_t = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
                ctx.autotune(m, feats, s_t, o_t, reps=3)
                del s_t, o_t
            mms, mstages, _, msc, _ = measure(ctx, m, feats, max(2, min(args.steps, 10)), args.warmup, torch)
            runs[m] = (mms, mstages, msc)
            log(f"{m}: {mms:.3f} ms/step, stages {mstages}")
        ref = runs["tensor_fp32"][2]
        keep = torch.isfinite(ref)
        precisions = {}
        for m in ("tensor_fp32", "tensor_bf16", "tensor_fp8"):
            mms, mstages, msc = runs[m]
            mflops, _, _ = corr_work(wl, m, args.rank)
            peak = {"tensor_bf16": PEAK_BF16_TFLOPS, "tensor_fp8": PEAK_FP8_TFLOPS}.get(m, PEAK_FP32_TFLOPS)
            tf = mflops / (mstages["correlation"] * 1e-3) / 1e12
            diff = (msc - ref).abs()[keep]
            precisions[m] = {"value": lay.n_resp / (mms * 1e-3), "ms_per_step": mms,
                             "stages_ms": {k: round(v, 4) for k, v in mstages.items()},
                             "tile_config": ctx.get_tile_config(m),
                             "correlation_tflops": tf, "correlation_peak_tflops": peak,
                             "correlation_frac_mfma": tf / peak,
                             "max_abs_score_diff_vs_tensor_fp32": float(diff.max()) if diff.numel() else 0.0,
                             "same_finite_pattern": bool(torch.equal(torch.isfinite(msc), keep))}

    cp = None
    if args.cp_rank > 0:
        t0 = time.time()
        cp_err = ctx.decompose_cp(args.cp_rank, max_iters=60, tol=1e-9)
        als_s = time.time() - t0
        cms, cstages, _, _, _ = measure(ctx, "cp_fp32", feats, max(2, min(args.steps, 5)), 1, torch)
        mults = mult_counts(wl, args.rank, args.cp_rank)
        ctf = 2 * mults["cp"] / (cstages["correlation"] * 1e-3) / 1e12
        cp = {"rank": args.cp_rank, "value": lay.n_resp / (cms * 1e-3), "ms_per_step": cms,
              "stages_ms": {k: round(v, 4) for k, v in cstages.items()},
              "als_seconds": als_s, "als_rel_err_mean": float(cp_err.mean()),
              "als_rel_err_max": float(cp_err.max()),
              "roofline": {"bound": "alu", "achieved": ctf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                           "frac": ctf / PEAK_FP32_TFLOPS, "kernel": "cp_corr_kernel",
                           "flops": 2 * mults["cp"],
                           "traffic": recorded_traffic("cp_corr_kernel", args.config, "cp_fp32",
                                                       args.cp_rank, 0)},
              "multiplies": mults,
              "formula1_gain_6x6_parts": 6 * 6 * 32 / (args.cp_rank * (6 + 6 + 32))}
        log(f"cp_fp32 R={args.cp_rank}: {cms:.3f} ms/step (ALS {als_s:.1f} s, mean rel err "
            f"{cp_err.mean():.3g}), stages {cstages}")
        if args.plant > 0:
            # convolution shortening: objects planted into a copy of the
            # features are the positives the thresholds are fitted on
            pfeat_host, pos = workloads.plant_objects(wl, wl.features(), args.plant)
            pfeat = torch.from_numpy(pfeat_host).cuda()
            ums, ustages, _, uscores, _ = measure(ctx, "cp_fp32", pfeat, max(2, min(args.steps, 5)), 1, torch)
            t0 = time.time()
            ctx.fit_thresholds(pfeat_host, pos, margin=1e-3)
            fit_s = time.time() - t0
            pms, pstages, _, pscores, _ = measure(ctx, "cp_fp32", pfeat, max(2, min(args.steps, 5)), 1, torch)
            us, ps = uscores.cpu().numpy(), pscores.cpu().numpy()
            fin = np.isfinite(us)
            rejected = int((np.isneginf(ps) & fin).sum())
            kept = ~np.isneginf(ps)
            pos_ok = all(np.isfinite(ps[lay.map_score_off[lay.find(i, l, c)] + y * int(lay.map_cols[lay.find(i, l, c)]) + x])
                         for (i, l, c, y, x) in pos)
            cp["pruning"] = {"positives": len(pos), "positive_rule": f"{args.plant} planted object(s) of every component per image",
                             "threshold_margin": 1e-3, "fit_seconds": fit_s,
                             "rejected_fraction": rejected / max(int(fin.sum()), 1),
                             "positives_kept": bool(pos_ok),
                             "survivors_equal_unpruned": bool(np.array_equal(ps[kept], us[kept])),
                             "unpruned_ms_per_step": ums,
                             "unpruned_stages_ms": {k: round(v, 4) for k, v in ustages.items()},
                             "ms_per_step": pms, "stages_ms": {k: round(v, 4) for k, v in pstages.items()},
                             "speedup_vs_unpruned": ums / pms}
            ctx.set_thresholds(None)
            del pfeat
            log(f"cp_fp32 on planted features: {ums:.3f} ms/step unpruned, {pms:.3f} pruned, "
                f"{100 * rejected / max(int(fin.sum()), 1):.1f}% rejected, positives kept {pos_ok}, "
                f"stages {pstages}")

    # roofline of each kernel; the headline object is the dominant one
    flops, cbytes, cresp = corr_work(wl, args.mode, args.rank)
    peak_mfma = {"tensor_bf16": PEAK_BF16_TFLOPS, "tensor_fp8": PEAK_FP8_TFLOPS}.get(args.mode, PEAK_FP32_TFLOPS)
    corr_ms = stages["correlation"]
    ai = flops / cbytes
    corr = {"kernel": "corr_kernel", "ms": corr_ms, "tflops": flops / (corr_ms * 1e-3) / 1e12,
            "gbs": cbytes / (corr_ms * 1e-3) / 1e9, "flops": flops, "bytes": cbytes,
            "arith_intensity": ai}
    corr["frac_mfma"] = corr["tflops"] / peak_mfma
    corr["frac_attainable"] = corr["tflops"] / min(peak_mfma, ai * PEAK_HBM_GBS / 1e3)
    # the correlation is priced against the MFMA peak of its operand type (the
    # target the tensor form is judged on), the placement against HBM
    rf_corr = {"bound": "mfma", "achieved": corr["tflops"], "peak": peak_mfma, "unit": "TFLOP/s",
               "frac": corr["frac_mfma"], "kernel": "corr_kernel", "bytes": cbytes,
               "traffic": recorded_traffic("corr_kernel", args.config, args.mode, args.rank,
                                           ctx.get_tile_config(args.mode))}
    pbytes = place_bytes(lay)
    place_ms = stages["placement"]
    pgbs = pbytes / (place_ms * 1e-3) / 1e9
    rf_place = {"bound": "hbm", "achieved": pgbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": pgbs / PEAK_HBM_GBS, "kernel": "place_kernel", "bytes": pbytes,
                "traffic": recorded_traffic("place_kernel", args.config, args.mode, args.rank, None)}
    roof = dict(rf_corr if corr_ms >= place_ms else rf_place)

    cpu = None
    err = None
    if args.cpu_budget > 0:
        log("cpu baseline (oracle) ...")
        cpu, err = cpu_baseline(wl, args.mode, U, args.cpu_budget, scores, offs, lay, torch)

    dtype = {"tensor_bf16": "bf16", "tensor_fp32": "f32", "direct_fp32": "f32", "tensor_fp8": "fp8e4m3"}[args.mode]
    out = {
        "metric": METRIC, "value": value, "unit": "resp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "mode": args.mode,
                   "rank": None if args.mode == "direct_fp32" else args.rank,
                   "resp_per_step": lay.n_resp, "score_maps": lay.n_maps},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "step_ms_percentiles": pct,
        "launch": args.launch,
        "launch_strategies": launches,
        "tile_config": tuning if tuning else {"chosen": ctx.get_tile_config(args.mode),
                                              "name": tile_config_name(ctx.get_tile_config(args.mode))},
        "correlation": corr,
        "placement_roofline": rf_place,
        "direct_fp32": direct,
        "tensor_vs_direct": (value / direct["value"]) if direct else None,
        "precisions": precisions,
        "cp_fp32": cp,
        "score_error_vs_oracle": err,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
