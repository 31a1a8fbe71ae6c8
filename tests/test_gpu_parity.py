"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (absolute, per score and per response): 1e-4 for the FP32 modes,
1e-2 for BF16 (the stated target).  Placement offsets must match the oracle
exactly wherever the oracle's placement margin exceeds the same tolerance.
"""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_common import TOL, Cmp, compare_map, note, oracle_basis, oracle_map, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# ----------------------------------------------------------------- distance transform
DT_CASES = [(1, 1), (1, 17), (13, 1), (5, 7), (31, 64), (33, 65), (70, 93), (100, 142)]


@pytest.mark.parametrize("shape", DT_CASES)
def test_distance_transform_random(shape):
    from paper_1707_03268_amd import distance_transform
    rows, cols = shape
    note(f"DT random {shape}")
    rng = np.random.default_rng(rows * 1000 + cols)
    resp = rng.standard_normal((rows, cols)).astype(np.float32)
    d = np.array([rng.uniform(-0.3, 0.3), rng.uniform(0.01, 0.2), rng.uniform(-0.3, 0.3), rng.uniform(0.01, 0.2)], np.float32)
    D, ay, ax = distance_transform(torch.from_numpy(resp).cuda(), d)
    torch.cuda.synchronize()
    ref = oracle.distance_transform(resp, d)
    np.testing.assert_allclose(D.cpu().numpy(), ref.D, atol=2e-5, rtol=0)
    ok = ref.margin > 1e-4
    np.testing.assert_array_equal(ay.cpu().numpy()[ok], ref.arg_y[ok])
    np.testing.assert_array_equal(ax.cpu().numpy()[ok], ref.arg_x[ok])


@pytest.mark.parametrize("seed", range(3))
def test_distance_transform_integer_ties(seed):
    """Small-integer data and coefficients are exact in FP32: every value and
    every argmax (ties included) must equal the oracle's."""
    from paper_1707_03268_amd import distance_transform
    note(f"DT integer ties seed {seed}")
    rng = np.random.default_rng(50 + seed)
    rows, cols = 23, 37
    resp = rng.integers(-4, 5, size=(rows, cols)).astype(np.float32)
    d = np.array([rng.integers(-1, 2), 1, rng.integers(-1, 2), 1], np.float32)
    D, ay, ax = distance_transform(torch.from_numpy(resp).cuda(), d)
    torch.cuda.synchronize()
    ref = oracle.distance_transform(resp, d)
    np.testing.assert_array_equal(D.cpu().numpy(), ref.D)
    np.testing.assert_array_equal(ay.cpu().numpy(), ref.arg_y)
    np.testing.assert_array_equal(ax.cpu().numpy(), ref.arg_x)


@pytest.mark.parametrize("shape", DT_CASES)
def test_distance_transform_envelope_random(shape):
    """The lower-envelope method against the oracle, and against the window
    scans: the same maxima, the same maximisers wherever the oracle's margin
    exceeds the tolerance."""
    from paper_1707_03268_amd import distance_transform
    rows, cols = shape
    note(f"DT envelope random {shape}")
    rng = np.random.default_rng(rows * 1000 + cols + 7)
    resp = rng.standard_normal((rows, cols)).astype(np.float32)
    d = np.array([rng.uniform(-0.3, 0.3), rng.uniform(0.01, 0.2), rng.uniform(-0.3, 0.3), rng.uniform(0.01, 0.2)], np.float32)
    t = torch.from_numpy(resp).cuda()
    D, ay, ax = distance_transform(t, d, method="envelope")
    Dw, ayw, axw = distance_transform(t, d)
    torch.cuda.synchronize()
    ref = oracle.distance_transform(resp, d)
    np.testing.assert_allclose(D.cpu().numpy(), ref.D, atol=2e-5, rtol=0)
    ok = ref.margin > 1e-4
    np.testing.assert_array_equal(ay.cpu().numpy()[ok], ref.arg_y[ok])
    np.testing.assert_array_equal(ax.cpu().numpy()[ok], ref.arg_x[ok])
    np.testing.assert_array_equal(ay.cpu().numpy()[ok], ayw.cpu().numpy()[ok])
    np.testing.assert_allclose(D.cpu().numpy(), Dw.cpu().numpy(), atol=1e-6, rtol=0)


@pytest.mark.parametrize("seed", range(3))
def test_distance_transform_envelope_integer_ties(seed):
    """Exact FP32 data: every value and every maximiser, ties included, equal
    to the oracle's (the envelope keeps the smallest of tied candidates)."""
    from paper_1707_03268_amd import distance_transform
    note(f"DT envelope integer ties seed {seed}")
    rng = np.random.default_rng(60 + seed)
    rows, cols = 29, 41
    resp = rng.integers(-4, 5, size=(rows, cols)).astype(np.float32)
    d = np.array([rng.integers(-1, 2), rng.choice([0.25, 0.5, 1.0]), rng.integers(-1, 2), rng.choice([0.25, 1.0])], np.float32)
    D, ay, ax = distance_transform(torch.from_numpy(resp).cuda(), d, method="envelope")
    torch.cuda.synchronize()
    ref = oracle.distance_transform(resp, d)
    np.testing.assert_array_equal(D.cpu().numpy(), ref.D)
    np.testing.assert_array_equal(ay.cpu().numpy(), ref.arg_y)
    np.testing.assert_array_equal(ax.cpu().numpy(), ref.arg_x)


@pytest.mark.parametrize("dq", [0.001, 1e-5])
def test_distance_transform_weak_deformation_both_methods(dq):
    """Weak deformation (the windows grow to whole lines): both methods equal
    the oracle; -inf cells never win."""
    from paper_1707_03268_amd import distance_transform
    note(f"DT weak deformation {dq}")
    rng = np.random.default_rng(int(1 / dq))
    rows, cols = 96, 211
    resp = rng.standard_normal((rows, cols)).astype(np.float32)
    resp[rng.random((rows, cols)) < 0.05] = -np.inf
    d = np.array([0.002, dq, -0.001, dq], np.float32)
    ref = oracle.distance_transform(resp, d)
    ok = ref.margin > 1e-4
    t = torch.from_numpy(resp).cuda()
    for method in ("envelope", "window"):
        D, ay, ax = distance_transform(t, d, method=method)
        torch.cuda.synchronize()
        np.testing.assert_allclose(D.cpu().numpy(), ref.D, atol=2e-5, rtol=0, err_msg=method)
        np.testing.assert_array_equal(ay.cpu().numpy()[ok], ref.arg_y[ok], err_msg=method)
        np.testing.assert_array_equal(ax.cpu().numpy()[ok], ref.arg_x[ok], err_msg=method)


def test_distance_transform_pitched_input():
    from paper_1707_03268_amd import distance_transform
    note("DT pitched input")
    rng = np.random.default_rng(3)
    big = torch.from_numpy(rng.standard_normal((20, 40)).astype(np.float32)).cuda()
    view = big[:, 3:30]
    d = [0.05, 0.04, -0.02, 0.03]
    D, ay, ax = distance_transform(view, d)
    torch.cuda.synchronize()
    ref = oracle.distance_transform(view.cpu().numpy(), d)
    np.testing.assert_allclose(D.cpu().numpy(), ref.D, atol=2e-5)


# ----------------------------------------------------------------- responses
def _responses(wl, mode, rank, image, level):
    from paper_1707_03268_amd import Context
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    U = None
    if rank is not None:
        ctx.decompose(rank)
        U = oracle_basis(wl.bank.filters, rank)
    ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    out, n = ctx.level_responses(mode, feats, image, level)
    torch.cuda.synchronize()
    flat = out.cpu().numpy()
    ctx.close()
    return flat, U


@pytest.mark.parametrize("mode,rank", [("direct_fp32", None), ("tensor_fp32", 8), ("tensor_fp32", 16),
                                       ("tensor_fp32", 32), ("tensor_fp32", 5), ("tensor_bf16", 4),
                                       ("tensor_bf16", 8), ("tensor_bf16", 16), ("tensor_bf16", 32)])
def test_level_responses_c2(mode, rank):
    """Every filter of the 54-filter bank on a level of the 500x375 pyramid that
    spans several tiles with ragged edges (level 3: 79 x 109 cells)."""
    wl = workloads.config2()
    level = 3
    note(f"responses c2 level {level} {mode} R={rank}")
    flat, U = _responses(wl, mode, rank, 0, level)
    X = wl.level_features(0, level)
    tol = TOL[mode]
    off = 0
    worst = 0.0
    for k, f in enumerate(wl.bank.filters):
        ref = oracle.correlate(X, f) if U is None else oracle.tensor_response(X, f, U)
        got = flat[off:off + ref.size].reshape(ref.shape)
        off += ref.size
        err = np.max(np.abs(got - ref))
        worst = max(worst, err)
        assert err <= tol, f"filter {k}: max err {err:.3g} > {tol}"
    note(f"  worst response error {worst:.3g}")


# ----------------------------------------------------------------- end-to-end scores
def _check_all_maps(wl, run, mode, U, maps=None):
    cache = {}
    cmp = Cmp()
    lay = run.layout
    idx = range(lay.n_maps) if maps is None else maps
    for k in idx:
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        sm = oracle_map(wl, img, lvl, comp, U, cache)
        compare_map(run, wl, img, lvl, comp, sm, TOL[mode], cmp)
    note(f"  {mode}: {cmp.n_pos} positions, max |score err| {cmp.max_err:.3g}, "
         f"argmax checked {cmp.n_arg_checked}/{cmp.n_arg} (excluded below margin {cmp.n_arg_excluded})")
    return cmp


def test_c1_direct_full():
    wl = workloads.config1()
    note("c1 direct fp32 full")
    run = run_gpu(wl, "direct_fp32")
    _check_all_maps(wl, run, "direct_fp32", None)


@pytest.mark.parametrize("mode,rank", [("tensor_fp32", 8), ("tensor_fp32", 32), ("tensor_bf16", 8), ("tensor_bf16", 16)])
def test_c1_tensor_full(mode, rank):
    wl = workloads.config1()
    note(f"c1 {mode} R={rank} full")
    run = run_gpu(wl, mode, rank)
    _check_all_maps(wl, run, mode, run.basis)


def test_c2_direct_full():
    wl = workloads.config2()
    note("c2 direct fp32 full pyramid")
    run = run_gpu(wl, "direct_fp32")
    _check_all_maps(wl, run, "direct_fp32", None)


@pytest.mark.parametrize("rank", [4, 8, 16, 32])
def test_c2_bf16_full(rank):
    wl = workloads.config2()
    note(f"c2 tensor bf16 R={rank} full pyramid")
    run = run_gpu(wl, "tensor_bf16", rank)
    _check_all_maps(wl, run, "tensor_bf16", run.basis)


def test_c2_tensor_fp32_full():
    wl = workloads.config2()
    note("c2 tensor fp32 R=16 full pyramid")
    run = run_gpu(wl, "tensor_fp32", 16)
    _check_all_maps(wl, run, "tensor_fp32", run.basis)


def test_c3_sampled_bf16_r16():
    """The 1080-filter bank on the 500x375 pyramid in the launch configuration
    the benchmark times; oracle on a sample of maps (largest and smallest root
    levels, several classes and every root shape)."""
    wl = workloads.config3()
    note("c3 tensor bf16 R=16, sampled maps")
    run = run_gpu(wl, "tensor_bf16", 16)
    lay = run.layout
    want = []
    L = len(wl.pyramids[0].levels)
    for lvl in (10, 11, 23, L - 1):
        for comp in (0, 3, 5, 61, 119):
            want.append(lay.find(0, lvl, comp))
    _check_all_maps(wl, run, "tensor_bf16", run.basis, want)


def _sample_maps(wl, lay, images, comps):
    """Maps of the given images and components on the first, a middle and the
    last root level of each image (levels where the component has no map are
    skipped)."""
    want = []
    for i in images:
        L, o = len(wl.pyramids[i].levels), wl.pyramids[i].octave
        for lvl in sorted({o, (o + L - 1) // 2, L - 1}):
            for comp in comps:
                try:
                    want.append(lay.find(i, lvl, comp))
                except KeyError:
                    pass
    return want


def test_c4_sampled_bf16_r16():
    """The 64-image batch of uneven sizes (320x240 .. 1280x960 px) in one
    batched call; oracle on sampled maps of the first, last, largest and
    smallest images."""
    wl = workloads.config4()
    note("c4 tensor bf16 R=16, 64 images, sampled maps")
    run = run_gpu(wl, "tensor_bf16", 16)
    area = [w * h for (w, h) in wl.image_sizes]
    imgs = sorted({0, len(area) - 1, int(np.argmax(area)), int(np.argmin(area))})
    want = _sample_maps(wl, run.layout, imgs, (0, 61, 119))
    assert len(want) >= 24
    _check_all_maps(wl, run, "tensor_bf16", run.basis, want)


def test_c5_frames_sampled_bf16_r16():
    """Two 1920x1080 frames of the video workload (frame size and bank at full
    scale, fewer frames); oracle on sampled maps of both frames."""
    wl = workloads.config5(n_frames=2)
    note("c5 tensor bf16 R=16, 2 frames 1920x1080, sampled maps")
    run = run_gpu(wl, "tensor_bf16", 16)
    want = _sample_maps(wl, run.layout, (0, 1), (2, 60, 117))
    assert len(want) >= 12
    _check_all_maps(wl, run, "tensor_bf16", run.basis, want)


def test_c3_sampled_direct():
    wl = workloads.config3()
    note("c3 direct fp32, sampled maps")
    run = run_gpu(wl, "direct_fp32")
    lay = run.layout
    want = [lay.find(0, lvl, comp) for lvl in (10, 20, 35) for comp in (1, 58, 118)]
    _check_all_maps(wl, run, "direct_fp32", None, want)


def test_repeat_calls_bitwise_identical():
    """Two calls on the same inputs give bitwise identical outputs."""
    from paper_1707_03268_amd import Context
    wl = workloads.config2()
    note("determinism c2 bf16 R=8")
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    ctx.decompose(8)
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    outs = []
    for _ in range(2):
        s = torch.zeros(lay.n_score, dtype=torch.float32, device="cuda")
        o = torch.zeros(lay.n_offsets, dtype=torch.int16, device="cuda")
        ctx.score_pyramid("tensor_bf16", feats, s, o)
        torch.cuda.synchronize()
        outs.append((s.cpu().numpy(), o.cpu().numpy()))
    assert np.array_equal(outs[0][0].view(np.int32), outs[1][0].view(np.int32))
    assert np.array_equal(outs[0][1], outs[1][1])
    ctx.close()


# ----------------------------------------------------------------- FP8
@pytest.mark.parametrize("rank", [8, 16, 32])
def test_level_responses_c2_fp8_within_rounding_bound(rank):
    """FP8 responses of every filter on a ragged multi-tile level stay within
    the e4m3 rounding bound of the FP64 tensor response at the same rank."""
    from _gpu_common import fp8_channel_scales, fp8_response_bound
    wl = workloads.config2()
    level = 3
    note(f"responses c2 level {level} tensor_fp8 R={rank}")
    flat, U = _responses(wl, "tensor_fp8", rank, 0, level)
    X = wl.level_features(0, level).astype(np.float64)
    RP = 16 if rank <= 16 else 32
    s = fp8_channel_scales(np.abs(X).reshape(-1, 32).max(0), U, RP)
    off = 0
    worst = 0.0
    for k, f in enumerate(wl.bank.filters):
        ref = oracle.tensor_response(X, f, U)
        got = flat[off:off + ref.size].reshape(ref.shape)
        off += ref.size
        bound = fp8_response_bound(X, f, U, s)
        ratio = np.max(np.abs(got - ref) / bound)
        worst = max(worst, ratio)
        assert ratio <= 1.0, f"filter {k}: error exceeds the e4m3 rounding bound (ratio {ratio:.3g})"
    note(f"  worst error / bound {worst:.3g}")


def _check_fp8_maps(wl, run, rank, maps):
    """FP8 scores of `maps` against the FP64 tensor oracle: the distance
    transform is 1-Lipschitz, so a score errs by at most the root's response
    bound plus, per part, the largest response bound over its part map;
    placements must match where the oracle margin exceeds twice that part
    bound."""
    from _gpu_common import fp8_channel_scales, fp8_response_bound
    U = run.basis
    RP = 16 if rank <= 16 else 32
    feats = wl.features().astype(np.float64)
    s = fp8_channel_scales(np.abs(feats).max(0), U, RP)
    del feats
    lay = run.layout
    cache = {}
    worst = 0.0
    checked = total = 0
    for k in maps:
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        sm = oracle_map(wl, img, lvl, comp, U, cache)
        Ho, Wo = sm.score.shape
        if Ho * Wo == 0:
            continue
        c = wl.bank.components[comp]
        pyr = wl.pyramids[img]
        Xr, Xp = cache[(img, lvl)], cache[(img, lvl - pyr.octave)]
        tol = np.max(fp8_response_bound(Xr, wl.bank.filters[c.root], U, s))
        pb = [np.max(fp8_response_bound(Xp, wl.bank.filters[p], U, s)) for p in c.parts]
        tol += sum(pb)
        g = run.scores[lay.map_score_off[k]:lay.map_score_off[k] + Ho * Wo].reshape(Ho, Wo)
        fin = np.isfinite(sm.score)
        assert np.array_equal(np.isfinite(g), fin)
        if fin.any():
            err = np.max(np.abs(g[fin] - sm.score[fin]))
            worst = max(worst, err / tol)
            assert err <= tol, f"map {k}: score error {err:.3g} > propagated bound {tol:.3g}"
        go = run.offsets[lay.map_offs_off[k]:lay.map_offs_off[k] + Ho * Wo * len(c.parts) * 2]
        go = go.reshape(len(c.parts), Ho, Wo, 2)
        for i in range(len(c.parts)):
            chk = sm.margin[i] > 2 * pb[i]
            total += chk.size
            checked += int(chk.sum())
            assert np.array_equal(go[i][chk], sm.offsets[i][chk]), f"map {k} part {i}: placements differ"
    note(f"  worst score error / bound {worst:.3g}; placements checked {checked}/{total}")


@pytest.mark.parametrize("cfg,rank", [(1, 16), (2, 16)])
def test_scores_fp8_within_propagated_bound(cfg, rank):
    wl = workloads.PRESETS[cfg]()
    note(f"c{cfg} tensor_fp8 R={rank} scores")
    run = run_gpu(wl, "tensor_fp8", rank)
    lay = run.layout
    _check_fp8_maps(wl, run, rank, range(lay.n_maps) if cfg == 1 else range(0, lay.n_maps, 7))


class _ChannelGain:
    """A workload whose features are another's with channel l multiplied by
    gain[l] (different channel ranges, so different FP8 scales)."""

    def __init__(self, wl, gain):
        self._wl, self._gain = wl, np.asarray(gain, np.float32)

    def __getattr__(self, name):
        return getattr(self._wl, name)

    def features(self):
        return (self._wl.features() * self._gain).astype(np.float32)

    def level_features(self, image, level):
        return (self._wl.level_features(image, level) * self._gain).astype(np.float32)


def test_fp8_scales_follow_the_features():
    """The FP8 channel and filter scales are recomputed on every call: on one
    context, a second feature set with other channel ranges scores within its
    own propagated bound, and the first set then scores bitwise as before."""
    from paper_1707_03268_amd import Context
    wl = workloads.config1()
    wl_b = _ChannelGain(wl, np.linspace(0.25, 4.0, 32))
    note("FP8 scales per call, c1 R=16")
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    a1 = run_gpu(wl, "tensor_fp8", 16, ctx=ctx)
    b = run_gpu(wl_b, "tensor_fp8", 16, ctx=ctx, features=torch.from_numpy(wl_b.features()).cuda())
    a2 = run_gpu(wl, "tensor_fp8", 16, ctx=ctx)
    ctx.close()
    assert np.array_equal(a1.scores.view(np.int32), a2.scores.view(np.int32))
    assert np.array_equal(a1.offsets, a2.offsets)
    assert not np.array_equal(a1.scores, b.scores)
    _check_fp8_maps(wl_b, b, 16, range(b.layout.n_maps))


def test_c5_frames_fp8_within_propagated_bound():
    """FP8 e4m3 with per-channel scales on two full-size 1920x1080 frames of the
    video workload, sampled maps, against the propagated rounding bound."""
    wl = workloads.config5(n_frames=2)
    note("c5 tensor_fp8 R=16, 2 frames 1920x1080, sampled maps")
    run = run_gpu(wl, "tensor_fp8", 16)
    want = _sample_maps(wl, run.layout, (0, 1), (4, 77))
    assert len(want) >= 8
    _check_fp8_maps(wl, run, 16, want)
