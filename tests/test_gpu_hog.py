"""GPU tests of the HOG feature pyramid (dpmt_hog_pyramid) against the FP64
HOG oracle.  Both take the per-pixel channel and direction decisions in
float32 with the same rounding, so every cell is compared element by element
at a float32 accumulation tolerance; cells outside the levels must stay
untouched."""
import numpy as np
import pytest

import workloads
from oracle import hog

from _gpu_common import note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 2e-5          # float32 histograms, ratios and sums of at most 72 terms of <= 0.2


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ctx():
    from paper_1707_03268_amd import Context
    c = Context(0)
    yield c
    c.close()


def _gpu(ctx, img, levels, n_cells, fill=float("nan")):
    feats = torch.full((n_cells, 32), fill, dtype=torch.float32, device="cuda")
    ctx.hog_pyramid(torch.from_numpy(img).cuda(), levels, feats)
    torch.cuda.synchronize()
    return feats.cpu().numpy()


def _check_levels(img, levels, got, which=None):
    worst = 0.0
    for k, (off, rows, cols, pr, pc, cell, inv) in enumerate(levels):
        if which is not None and k not in which:
            continue
        want = hog.hog_level(img, hog.HogLevel(rows - 2 * pr, cols - 2 * pc, cell, inv, pr, pc))
        g = got[off:off + rows * cols].reshape(rows, cols, 32)
        assert np.isfinite(g).all(), f"level {k}: cells left unwritten"
        err = np.abs(g - want)
        worst = max(worst, float(err.max()))
        assert err.max() <= TOL, f"level {k} ({rows}x{cols}, cell {cell}, inv {inv:.4f}): max err {err.max():.3g}"
        np.testing.assert_array_equal(g[..., 31], want[..., 31])
    return worst


@pytest.mark.parametrize("size", [(500, 375), (333, 251)])
def test_pyramid_matches_the_oracle(ctx, size):
    w, h = size
    img = workloads.synthetic_image(11, w, h)
    pyrs, total = workloads.build_pyramids([(w, h)])
    levels = workloads.hog_levels(pyrs[0])
    note(f"HOG {w}x{h}: {len(levels)} levels, {total} cells")
    got = _gpu(ctx, img, levels, total)
    worst = _check_levels(img, levels, got)
    note(f"  max |err| {worst:.3g}")


def test_1080p_frame_sampled_levels(ctx):
    img = workloads.synthetic_image(12, 1920, 1080)
    pyrs, total = workloads.build_pyramids([(1920, 1080)])
    levels = workloads.hog_levels(pyrs[0])
    note(f"HOG 1920x1080: {len(levels)} levels, {total} cells")
    got = _gpu(ctx, img, levels, total)
    assert np.isfinite(got).all()
    _check_levels(img, levels, got, which={0, 5, 9, 10, 27, len(levels) - 1})


def test_batch_of_images_into_one_buffer(ctx):
    """Two images' pyramids in one packed buffer (as a plan of two images
    lays them out); each call writes its own image's levels only."""
    sizes = [(160, 120), (250, 190)]
    pyrs, total = workloads.build_pyramids(sizes)
    feats = torch.full((total, 32), float("nan"), dtype=torch.float32, device="cuda")
    imgs = [workloads.synthetic_image(20 + i, w, h) for i, (w, h) in enumerate(sizes)]
    ctx.hog_pyramid(torch.from_numpy(imgs[0]).cuda(), workloads.hog_levels(pyrs[0]), feats)
    torch.cuda.synchronize()
    first_end = pyrs[1].levels[0].cell_offset
    got = feats.cpu().numpy()
    assert np.isfinite(got[:first_end]).all() and np.isnan(got[first_end:]).all()
    ctx.hog_pyramid(torch.from_numpy(imgs[1]).cuda(), workloads.hog_levels(pyrs[1]), feats)
    torch.cuda.synchronize()
    got = feats.cpu().numpy()
    for i in range(2):
        _check_levels(imgs[i], workloads.hog_levels(pyrs[i]), got)


def test_odd_geometry_and_repeat_calls(ctx):
    """Hand-made levels: up- and down-sampling, a level of padding only, an
    interior smaller than one tile, no padding, a gap between levels; then the
    same call again (cached tables) and a different geometry (new tables),
    results bitwise equal to the first run."""
    img = workloads.synthetic_image(30, 97, 61)
    levels = [(0, 30, 40, 2, 3, 4, 0.5),        # upsampled 2x: the image repeats its edges beyond 2x its size
              (1200, 9, 14, 1, 1, 8, 1.0),
              (1400, 4, 6, 2, 3, 4, 1.0),       # padding only
              (1500, 5, 7, 0, 0, 4, 3.7),       # no padding, strong downsampling
              (1600, 23, 17, 0, 0, 8, 0.9)]
    n = 1600 + 23 * 17 + 5
    got = _gpu(ctx, img, levels, n)
    _check_levels(img, levels, got)
    gap = np.ones(n, bool)
    for off, rows, cols, *_ in levels:
        gap[off:off + rows * cols] = False
    assert np.isnan(got[gap]).all(), "cells outside the levels were written"
    again = _gpu(ctx, img, levels, n)
    np.testing.assert_array_equal(np.nan_to_num(again, nan=-1.0), np.nan_to_num(got, nan=-1.0))
    other = _gpu(ctx, img, levels[:2], n)
    np.testing.assert_array_equal(other[:1400], got[:1400])


def test_invalid_levels_are_rejected_before_any_write(ctx):
    img = torch.from_numpy(workloads.synthetic_image(31, 40, 30)).cuda()
    feats = torch.full((2000, 32), float("nan"), dtype=torch.float32, device="cuda")
    bad = [
        [(0, 10, 10, 1, 1, 5, 1.0)],                                   # cell not 4 or 8
        [(0, 10, 10, 6, 1, 4, 1.0)],                                   # padding wider than the level
        [(0, 10, 10, 1, 1, 4, 0.0)],                                   # inv_scale not > 0
        [(0, 10, 10, 1, 1, 4, float("inf"))],
        [(0, 10, 10, 1, 1, 4, 1.0), (50, 10, 10, 1, 1, 4, 1.0)],       # overlapping levels
        [(-1, 10, 10, 1, 1, 4, 1.0)],
    ]
    for levels in bad:
        with pytest.raises(RuntimeError):
            ctx.hog_pyramid(img, levels, feats)
    torch.cuda.synchronize()
    assert torch.isnan(feats).all()


def test_scores_from_images_end_to_end():
    """Algorithm 1 from pixels: the GPU's HOG pyramid of two images is scored
    on the GPU (BF16 tensor form) and compared with the oracle's scores of the
    oracle's HOG pyramid of the same images: scores within the BF16 tolerance
    plus what the features' float32 error can move them, placements equal
    above the margin, and the detection set at a threshold equal to the
    thresholding of the GPU's own scores."""
    import oracle
    from paper_1707_03268_amd import Context
    from _gpu_common import oracle_basis
    sizes = [(200, 150), (160, 136)]
    pyrs, total = workloads.build_pyramids(sizes)
    bank = workloads.build_bank(2, 1)
    imgs = [workloads.synthetic_image(40 + i, w, h) for i, (w, h) in enumerate(sizes)]
    note("scores from images: 2 images, 54 filters, HOG on the GPU")
    feats = torch.full((total, 32), float("nan"), dtype=torch.float32, device="cuda")
    ctx = Context(0)
    for img, pyr in zip(imgs, pyrs):
        ctx.hog_pyramid(torch.from_numpy(img).cuda(), workloads.hog_levels(pyr), feats)
    ctx.load_filters(bank.filters, bank.components)
    ctx.decompose(16)
    U = oracle_basis(bank.filters, 16)
    lay = ctx.plan(pyrs)
    scores = torch.empty(lay.n_score, dtype=torch.float32, device="cuda")
    offs = torch.empty(lay.n_offsets, dtype=torch.int16, device="cuda")
    ctx.score_pyramid("tensor_bf16", feats, scores, offs)
    torch.cuda.synchronize()
    s, o = scores.cpu().numpy(), offs.cpu().numpy()
    # the oracle's own HOG levels, scored by the oracle
    # the BF16 target, doubled because the HOG channels reach about twice the
    # synthetic features' range, plus the features' float32 error carried by 9
    # unit-norm filters of at most 8 x 15 x 32 taps: 9 * 2e-5 * sqrt(3840)
    tol = 2e-2 + 9 * 2e-5 * 3840 ** 0.5
    worst = 0.0
    checked = 0
    for i, (img, pyr) in enumerate(zip(imgs, pyrs)):
        levels = [hog.hog_level(img, hog.HogLevel(r - 2 * pr, c - 2 * pc, cell, inv, pr, pc))
                  for (_, r, c, pr, pc, cell, inv) in workloads.hog_levels(pyr)]
        ref = oracle.score_pyramid(levels, bank.filters, bank.components, pyr.octave, U)
        for (lvl, comp), sm in ref.items():
            k = lay.find(i, lvl, comp)
            Ho, Wo = int(lay.map_rows[k]), int(lay.map_cols[k])
            if Ho * Wo == 0:
                continue
            g = s[lay.map_score_off[k]:lay.map_score_off[k] + Ho * Wo].reshape(Ho, Wo)
            fin = np.isfinite(sm.score)
            assert np.array_equal(np.isfinite(g), fin)
            if fin.any():
                e = float(np.max(np.abs(g[fin] - sm.score[fin])))
                worst = max(worst, e)
                assert e <= tol, (i, lvl, comp, e)
            npart = len(bank.components[comp].parts)
            go = o[lay.map_offs_off[k]:lay.map_offs_off[k] + Ho * Wo * npart * 2].reshape(npart, Ho, Wo, 2)
            ok = sm.margin > tol
            checked += int(ok.sum())
            assert np.array_equal(go[ok], sm.offsets[ok]), (i, lvl, comp)
    note(f"  max |score err| {worst:.3g}, {checked} placements checked")
    assert checked > 0
    fin = s[np.isfinite(s)]
    tau = float(np.quantile(fin, 0.999))
    rec, sc, n = ctx.detect(scores, tau)
    assert n == int((fin >= tau).sum()) and n > 0
    ctx.close()
