"""GPU tests of batching: a batch of images of uneven sizes against the FP64
oracle, and the launch strategies and correlation tile configurations against
each other.

Every strategy (one launch per stage, launches per level, a captured graph)
and every tile configuration runs the same kernels with each response
accumulated in the same order, so their scores and placements must be
bitwise equal; the autotuner's choice therefore cannot change results.
"""
import numpy as np
import pytest

import workloads

from _gpu_common import TOL, Cmp, compare_map, note, oracle_basis, oracle_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def batch():
    wl = workloads.uneven_batch()
    return wl, torch.from_numpy(wl.features()).cuda()


def _context(wl, rank):
    from paper_1707_03268_amd import Context
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    U = None
    if rank is not None:
        ctx.decompose(rank)
        U = oracle_basis(wl.bank.filters, rank)
    lay = ctx.plan(wl.pyramids)
    return ctx, lay, U


def _outputs(lay):
    scores = torch.full((max(lay.n_score, 1),), float("nan"), dtype=torch.float32, device="cuda")
    offs = torch.full((max(lay.n_offsets, 1),), -32768, dtype=torch.int16, device="cuda")
    return scores, offs


def _score(ctx, mode, feats, lay):
    scores, offs = _outputs(lay)
    ctx.score_pyramid(mode, feats, scores, offs)
    torch.cuda.synchronize()
    return scores.cpu().numpy(), offs.cpu().numpy()


@pytest.mark.parametrize("mode,rank,every", [("tensor_bf16", 16, 1), ("direct_fp32", None, 5)])
def test_uneven_batch_against_oracle(batch, mode, rank, every):
    """All images in one plan; every score map (every 5th for the slower
    direct oracle) compared with the oracle within the mode's tolerance,
    placements exact above the margin."""
    from _gpu_common import GpuRun
    wl, feats = batch
    note(f"uneven batch {mode} rank {rank}: {wl.image_sizes}")
    ctx, lay, U = _context(wl, rank)
    s, o = _score(ctx, mode, feats, lay)
    run = GpuRun(lay, s, o, None, U)
    cmp = Cmp()
    cache = {}
    for k in range(0, lay.n_maps, every):
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        if lay.map_rows[k] == 0 or lay.map_cols[k] == 0:
            continue
        sm = oracle_map(wl, img, lvl, comp, U, cache)
        compare_map(run, wl, img, lvl, comp, sm, TOL[mode], cmp)
        if k % 60 == 0:
            cache.clear()
    note(f"  {cmp.n_pos} positions, max |err| {cmp.max_err:.3g}, placements checked "
         f"{cmp.n_arg_checked}/{cmp.n_arg}")
    assert cmp.n_pos > 0
    ctx.close()


@pytest.mark.parametrize("mode,rank", [("tensor_bf16", 16), ("direct_fp32", None), ("tensor_fp8", 16)])
def test_launch_strategies_bitwise_equal(batch, mode, rank):
    wl, feats = batch
    note(f"launch strategies {mode}")
    ctx, lay, _ = _context(wl, rank)
    ref_s, ref_o = _score(ctx, mode, feats, lay)
    for launch in ("per_level", "overlap"):
        ctx.set_launch(launch)
        s, o = _score(ctx, mode, feats, lay)
        np.testing.assert_array_equal(s, ref_s, err_msg=launch)
        np.testing.assert_array_equal(o, ref_o, err_msg=launch)
    # graph: replayed several times with eager work in between, each replay checked
    ctx.set_launch("graph")
    scores, offs = _outputs(lay)
    for rep in range(3):
        scores.fill_(float("nan"))
        offs.fill_(-32768)
        ctx.score_pyramid(mode, feats, scores, offs)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(scores.cpu().numpy(), ref_s, err_msg=f"graph replay {rep}")
        np.testing.assert_array_equal(offs.cpu().numpy(), ref_o, err_msg=f"graph replay {rep}")
        junk = torch.randn(1 << 20, device="cuda")             # unrelated eager work
        junk.mul_(2.0).sum().item()
    # a new output buffer forces a new capture
    s2, o2 = _outputs(lay)
    ctx.score_pyramid(mode, feats, s2, o2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s2.cpu().numpy(), ref_s)
    ctx.set_launch("batched")
    ctx.close()


@pytest.mark.parametrize("mode,rank", [("tensor_bf16", 16), ("direct_fp32", None)])
def test_tile_configs_bitwise_equal(batch, mode, rank):
    from paper_1707_03268_amd import tile_config_count, tile_config_name
    wl, feats = batch
    ctx, lay, _ = _context(wl, rank)
    ref_s, ref_o = _score(ctx, mode, feats, lay)
    for cfg in range(1, tile_config_count()):
        note(f"tile config {cfg} ({tile_config_name(cfg)}) {mode}")
        ctx.set_tile_config(mode, cfg)
        assert ctx.get_tile_config(mode) == cfg
        s, o = _score(ctx, mode, feats, lay)
        np.testing.assert_array_equal(s, ref_s, err_msg=f"tile config {cfg}")
        np.testing.assert_array_equal(o, ref_o, err_msg=f"tile config {cfg}")
    ctx.close()


def test_autotune_picks_a_timed_config(batch):
    from paper_1707_03268_amd import tile_config_count
    wl, feats = batch
    note("autotune tensor_bf16")
    ctx, lay, _ = _context(wl, 16)
    ref_s, ref_o = _score(ctx, "tensor_bf16", feats, lay)
    scores, offs = _outputs(lay)
    best, ms = ctx.autotune("tensor_bf16", feats, scores, offs, reps=3)
    note(f"  best {best}, medians {ms}")
    assert 0 <= best < tile_config_count()
    assert ms[best] is not None and ms[best] == min(m for m in ms if m is not None)
    assert ctx.get_tile_config("tensor_bf16") == best
    s, o = _score(ctx, "tensor_bf16", feats, lay)
    np.testing.assert_array_equal(s, ref_s)
    np.testing.assert_array_equal(o, ref_o)
    ctx.close()


def _mixed_sizes_workload():
    """One 1920x1080 frame beside two small images, one class model: the
    frame's tallest score maps need several times the LDS of the small
    images' maps, so the batched placement runs as several launches whose LDS
    each run's own maps size (fewer workgroups per CU for the tall maps)."""
    sizes = [(1920, 1080), (320, 240), (400, 300)]
    pyrs, total = workloads.build_pyramids(sizes)
    bank = workloads.build_bank(5, 1)
    return workloads.Workload("mixed sizes: one 1920x1080 frame, two small images, 1 class", 5, pyrs,
                              bank, total, workloads.feature_seed(5), True, sizes)


def test_placement_runs_by_occupancy():
    from _gpu_common import GpuRun
    wl = _mixed_sizes_workload()
    note("placement runs by occupancy: batched vs per level, oracle on the tallest and a small map")
    feats = torch.from_numpy(wl.features()).cuda()
    ctx, lay, U = _context(wl, 16)
    ref_s, ref_o = _score(ctx, "tensor_bf16", feats, lay)
    for launch in ("per_level", "overlap"):
        ctx.set_launch(launch)
        s, o = _score(ctx, "tensor_bf16", feats, lay)
        np.testing.assert_array_equal(s, ref_s, err_msg=launch)
        np.testing.assert_array_equal(o, ref_o, err_msg=launch)
    ctx.set_launch("batched")
    run = GpuRun(lay, ref_s, ref_o, None, U)
    cmp, cache = Cmp(), {}
    oct0 = wl.pyramids[0].octave
    for img, level, comp in ((0, oct0, 0), (1, wl.pyramids[1].octave, 5)):
        sm = oracle_map(wl, img, level, comp, U, cache)
        compare_map(run, wl, img, level, comp, sm, TOL["tensor_bf16"], cmp)
    note(f"  {cmp.n_pos} positions, max |err| {cmp.max_err:.3g}")
    assert cmp.n_pos > 0
    ctx.close()
