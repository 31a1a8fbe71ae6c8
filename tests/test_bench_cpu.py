"""CPU checks of bench.py: it refuses several GPUs, and the algorithmic work
it prices the kernels with counts what the plan lays out."""
import os
import subprocess
import sys

import numpy as np

import workloads
from paper_1707_03268_amd import Context

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr + r.stdout
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def _plan(wl):
    ctx = Context(device=-1)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    lay = ctx.plan(wl.pyramids)
    return ctx, lay


def test_work_counts_match_the_plan():
    for wl in (workloads.config1(), workloads.config2()):
        ctx, lay = _plan(wl)
        # every (filter, level) response the correlation writes, counted from shapes
        shapes, comps = wl.bank.shapes, wl.bank.components
        flops, nbytes, resp = bench.corr_work(wl.pyramids, shapes, comps, "direct_fp32", 32)
        assert resp == lay.n_resp
        want = 0
        for pyr in wl.pyramids:
            L = len(pyr.levels)
            for l, lv in enumerate(pyr.levels):
                for k, f in enumerate(wl.bank.filters):
                    is_root = any(c.root == k for c in wl.bank.components)
                    is_part = any(k in c.parts for c in wl.bank.components)
                    h, w = f.shape[:2]
                    n = max(lv.rows - h + 1, 0) * max(lv.cols - w + 1, 0)
                    uses = (is_root and l >= pyr.octave) + (is_part and l + pyr.octave < L)
                    want += uses * 2 * n * h * w * 32
        assert flops == want
        # the tensor form contracts R channels instead of 32
        tflops, _, tresp = bench.corr_work(wl.pyramids, shapes, comps, "tensor_bf16", 16)
        assert tresp == resp and tflops * 2 == flops
        # placement: every response read once, every score and offset pair written once
        assert bench.place_bytes(lay) == 4 * (lay.n_resp_part + lay.n_resp_root) + 4 * lay.n_score + 2 * lay.n_offsets
        assert lay.n_offsets == 2 * sum(int(lay.map_rows[k]) * int(lay.map_cols[k]) *
                                        len(wl.bank.components[int(lay.map_comp[k])].parts)
                                        for k in range(lay.n_maps))
        ctx.close()


def test_recorded_traffic_needs_the_current_kernels():
    """Traffic is reported only from a profile line taken on the current kernel
    sources, for the same kernel, workload, mode, rank and tile configuration."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    lines = [l.split() for l in open(path) if l.startswith("traffic ")]
    assert lines
    digest = bench.kernel_source_digest()
    for t in lines:
        got = bench.recorded_traffic(t[1], t[2], t[3], int(t[4]), int(t[5]))
        if t[6] == digest:
            assert got == int(float(t[7]) + float(t[8]))
        else:
            assert got is None
    assert bench.recorded_traffic("corr_kernel", "c5x16", "tensor_bf16", 16, 99) is None
    assert bench.recorded_traffic("no_such_kernel", "c5x16", "tensor_bf16", 16, None) is None


def test_stream_chunks_share_one_plan():
    """The 256-frame stream is scored as chunks of one plan: every chunk's
    pyramids are the first chunk's shifted by a whole chunk of cells, and the
    chunk plan's responses times the chunk count is the whole workload's."""
    wl = workloads.config5(8)
    cells = bench.chunk_cells(wl, 4)
    assert cells * 2 == wl.total_cells
    shapes, comps = wl.bank.shapes, wl.bank.components
    _, _, r_chunk = bench.corr_work(wl.pyramids[:4], shapes, comps, "tensor_bf16", 16)
    _, _, r_all = bench.corr_work(wl.pyramids, shapes, comps, "tensor_bf16", 16)
    assert 2 * r_chunk == r_all
    uneven = workloads.uneven_batch(4)
    import pytest
    with pytest.raises(SystemExit):
        bench.chunk_cells(uneven, 2)


def test_oracle_pool_task_matches_direct_call():
    """A pool task (as the CPU baseline and the rank sweep run it) returns the
    oracle's own score map for its (image, level, component)."""
    import oracle
    wl = workloads.config1()
    U = oracle.decompose(wl.bank.filters, 8).U
    bench._pool_init(1, 0, {8: U})
    img, lvl, comp, t0, t1, out = bench._oracle_task((0, 1, 0, (0, 8), None))
    assert (img, lvl, comp) == (0, 1, 0) and t1 >= t0
    c = wl.bank.components[0]
    X1, X0 = wl.level_features(0, 1), wl.level_features(0, 0)
    ref = oracle.score_component(oracle.correlate(X1, wl.bank.filters[c.root]),
                                 [oracle.correlate(X0, wl.bank.filters[k]) for k in c.parts],
                                 c.anchors, c.deform)
    assert np.array_equal(out[0][0], ref.score)
    assert out[0][3] == ref.score.size + sum(
        (X0.shape[0] - 5) * (X0.shape[1] - 5) for _ in c.parts)
    assert bench._oracle_task((0, 1, 0, (0,), 0.0)) is None      # past its deadline
