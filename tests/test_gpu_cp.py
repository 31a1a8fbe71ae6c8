"""GPU parity of the per-filter CP form (Section 4): the decomposed
correlation (channel contraction, then 1-D correlations along x and y) and the
scores built on it, against the oracle's FP64 decomposed correlation with the
same factors.

The factors are the library's own ALS fit read back (or random factors loaded
through dpmt_load_cp), so the comparison isolates the GPU arithmetic: FP32
products and sums against FP64, well inside 1e-4 on these magnitudes.
"""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_common import Cmp, GpuRun, compare_map, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_CP = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cp_context(wl, ranks, factors=None):
    from paper_1707_03268_amd import Context
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    if factors is None:
        ctx.decompose_cp(ranks, max_iters=60, tol=1e-9)
    else:
        ctx.load_cp(ranks, factors)
    _, fac = ctx.get_cp(wl.bank.shapes)
    fac64 = [tuple(m.astype(np.float64) for m in abc) for abc in fac]
    ctx.plan(wl.pyramids)
    return ctx, fac64


def _check_level_responses(ctx, wl, fac64, feats, levels):
    worst = 0.0
    n = 0
    for (img, lvl) in levels:
        out, total = ctx.level_responses("cp_fp32", feats, img, lvl)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        X = wl.level_features(img, lvl).astype(np.float64)
        H, W = X.shape[:2]
        off = 0
        for k, (h, w) in enumerate(wl.bank.shapes):
            Ho, Wo = H - h + 1, W - w + 1
            if Ho <= 0 or Wo <= 0:
                continue
            want = oracle.cp_response(X, *fac64[k])
            g = got[off:off + Ho * Wo].reshape(Ho, Wo)
            off += Ho * Wo
            err = float(np.max(np.abs(g - want)))
            worst = max(worst, err)
            n += Ho * Wo
            assert err <= TOL_CP, f"image {img} level {lvl} filter {k} ({h}x{w}): max |err| {err:.3g}"
        assert off == total
    return worst, n


@pytest.mark.parametrize("R", [1, 5, 8])
def test_cp_level_responses_c1(R):
    """Every filter on both c1 levels (80x60 and 40x30 cells: several tiles,
    ragged tails in both directions); R = 5 leaves a partial batch of terms,
    R = 8 needs two."""
    wl = workloads.config1()
    note(f"cp level responses c1 R={R}")
    ctx, fac = _cp_context(wl, R)
    feats = torch.from_numpy(wl.features()).cuda()
    worst, n = _check_level_responses(ctx, wl, fac, feats, [(0, 0), (0, 1)])
    note(f"  {n} responses, max |err| {worst:.3g}")
    ctx.close()


def test_cp_random_factors_mixed_ranks_c2():
    """Factors loaded from outside with per-filter ranks across [1, 32] (all
    eight batches of terms, chunks whose filters differ in rank), on c2 levels
    from the largest down to ones smaller than a filter."""
    wl = workloads.config2()
    rng = np.random.default_rng(11)
    ranks = rng.integers(1, 33, size=len(wl.bank.filters))
    ranks[:3] = [32, 1, 17]
    fac = [(rng.standard_normal((h, R)) * 0.5, rng.standard_normal((w, R)) * 0.5,
            rng.standard_normal((32, R)) * 0.3) for (h, w), R in zip(wl.bank.shapes, ranks)]
    note(f"cp random factors c2, ranks {ranks.min()}..{ranks.max()}")
    ctx, fac64 = _cp_context(wl, ranks, fac)
    feats = torch.from_numpy(wl.features()).cuda()
    lv = wl.pyramids[0].levels
    picks = [0, 3, 17, len(lv) - 6, len(lv) - 1]
    worst, n = _check_level_responses(ctx, wl, fac64, feats, [(0, l) for l in picks])
    note(f"  {n} responses, max |err| {worst:.3g}")
    ctx.close()


def _oracle_cp_map(wl, fac, image, level, comp, cache):
    """Oracle score map of one (image, root level, component) with the CP
    form's decomposed correlation as the response, through the oracle's
    pyramid scoring."""
    from _gpu_common import _LazyLevels
    out = oracle.score_pyramid(_LazyLevels(wl, image, cache), wl.bank.filters, wl.bank.components,
                               wl.pyramids[image].octave, root_levels=[level], comps=[comp],
                               response=lambda X, k: oracle.cp_response(X, *fac[k]))
    return out[(level, comp)]


def _scores(ctx, lay, feats):
    scores = torch.full((max(lay.n_score, 1),), float("nan"), dtype=torch.float32, device="cuda")
    offs = torch.full((max(lay.n_offsets, 1),), -32768, dtype=torch.int16, device="cuda")
    ctx.score_pyramid("cp_fp32", feats, scores, offs)
    torch.cuda.synchronize()
    return scores.cpu().numpy(), offs.cpu().numpy()


@pytest.mark.parametrize("cfg,R,every", [(1, 6, 1), (2, 6, 3)])
def test_cp_scores_against_oracle(cfg, R, every):
    """Scores and placements of the CP mode (every map of c1, every third of
    c2) against the oracle's star-model scores over its CP responses."""
    wl = workloads.config1() if cfg == 1 else workloads.config2()
    note(f"cp scores c{cfg} R={R}")
    ctx, fac = _cp_context(wl, R)
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    s, o = _scores(ctx, lay, feats)
    run = GpuRun(lay, s, o, None, None)
    cmp = Cmp()
    cache = {}
    for k in range(0, lay.n_maps, every):
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        if lay.map_rows[k] == 0 or lay.map_cols[k] == 0:
            continue
        sm = _oracle_cp_map(wl, fac, img, lvl, comp, cache)
        compare_map(run, wl, img, lvl, comp, sm, TOL_CP, cmp)
    note(f"  {cmp.n_pos} positions, max |err| {cmp.max_err:.3g}, placements checked "
         f"{cmp.n_arg_checked}/{cmp.n_arg}")
    assert cmp.n_pos > 0
    ctx.close()


@pytest.mark.parametrize("S,T", [(8, 5), (6, 6)])
def test_cp_root_part_rank_pairs(S, T):
    """Section 5's (S, T) rank pairs: rank S for every root filter, T for every
    part filter (per-filter ranks), scored against the oracle on c2."""
    wl = workloads.config2()
    roots = {c.root for c in wl.bank.components}
    ranks = [S if k in roots else T for k in range(len(wl.bank.filters))]
    note(f"cp (S, T) = ({S}, {T}) scores c2")
    ctx, fac = _cp_context(wl, ranks)
    got_ranks, _ = ctx.get_cp(wl.bank.shapes)
    assert list(got_ranks) == ranks
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    s, o = _scores(ctx, lay, feats)
    run = GpuRun(lay, s, o, None, None)
    cmp = Cmp()
    cache = {}
    for k in range(0, lay.n_maps, 3):
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        if lay.map_rows[k] == 0 or lay.map_cols[k] == 0:
            continue
        sm = _oracle_cp_map(wl, fac, img, lvl, comp, cache)
        compare_map(run, wl, img, lvl, comp, sm, TOL_CP, cmp)
    note(f"  {cmp.n_pos} positions, max |err| {cmp.max_err:.3g}, placements checked "
         f"{cmp.n_arg_checked}/{cmp.n_arg}")
    assert cmp.n_pos > 0
    ctx.close()


@pytest.mark.parametrize("prune", [False, True])
def test_cp_launch_strategies_bitwise_equal(prune):
    wl = workloads.uneven_batch()
    note(f"cp launch strategies, pruning {prune}")
    ctx, _ = _cp_context(wl, 6)
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    if prune:
        ref_s, _ = _scores(ctx, lay, feats)
        pos = []
        for k in range(0, lay.n_maps, 4):
            n = int(lay.map_rows[k]) * int(lay.map_cols[k])
            if n == 0:
                continue
            m = ref_s[lay.map_score_off[k]:lay.map_score_off[k] + n]
            if not np.isfinite(m).any():
                continue
            i = int(np.argmax(m))
            pos.append((int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k]),
                        i // int(lay.map_cols[k]), i % int(lay.map_cols[k])))
        ctx.fit_thresholds(wl.features(), pos, margin=1e-3)
    ref_s, ref_o = _scores(ctx, lay, feats)
    assert np.isfinite(ref_s).any()
    if prune:
        assert np.isneginf(ref_s).sum() > 0
    for launch in ("per_level", "overlap", "graph", "graph"):
        ctx.set_launch(launch)
        s, o = _scores(ctx, lay, feats)
        np.testing.assert_array_equal(s, ref_s, err_msg=launch)
        np.testing.assert_array_equal(o, ref_o, err_msg=launch)
        torch.randn(1 << 18, device="cuda").mul_(2.0).sum().item()     # eager work between replays
    ctx.set_launch("batched")
    ctx.close()


def _oracle_thresholds(wl, fac, positives):
    """Per-filter thresholds (filter order) from positives (image, level,
    comp, y, x), in the oracle, less 1e-3; filters no positive covers get -inf."""
    parts_of = {k: [] for k in range(len(wl.bank.filters))}
    cache = {}

    def terms(img, lvl, k):
        key = (img, lvl, k)
        if key not in cache:
            cache[key] = oracle.cp_terms(wl.level_features(img, lvl).astype(np.float64), *fac[k])
        return cache[key]
    for (img, lvl, comp, y, x) in positives:
        c = wl.bank.components[comp]
        oct_ = wl.pyramids[img].octave
        parts_of[c.root].append(oracle.partial_sums(terms(img, lvl, c.root), y, x))
        for i, k in enumerate(c.parts):
            T = terms(img, lvl - oct_, k)
            ay, ax = 2 * y + int(c.anchors[i][0]), 2 * x + int(c.anchors[i][1])
            if ay < T.shape[1] and ax < T.shape[2]:
                parts_of[k].append(oracle.partial_sums(T, ay, ax))
    # lowered by 1e-3 so that FP32 partial sums decide every positive clearly
    return [oracle.fit_thresholds(ps) - 1e-3 if ps else np.full(fac[k][0].shape[1], -np.inf)
            for k, ps in parts_of.items()], terms


@pytest.mark.parametrize("cfg,every", [(1, 1), (2, 4)])
def test_cp_pruning_against_oracle(cfg, every):
    """Algorithm 1's early exit: thresholds fitted in the oracle on positives
    (each sampled map's best hypotheses, by the oracle's own CP scores), then
    the GPU's rejected set and surviving scores against the oracle's pruned
    maps, wherever every test of a hypothesis is decided by more than the
    tolerance.  Survivors keep their unpruned scores bit for bit."""
    wl = workloads.config1() if cfg == 1 else workloads.config2()
    note(f"cp pruning c{cfg}")
    ctx, fac = _cp_context(wl, 4)
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    free_s, free_o = _scores(ctx, lay, feats)
    maps = [k for k in range(0, lay.n_maps, every) if lay.map_rows[k] > 0 and lay.map_cols[k] > 0]
    cache = {}
    sms = {}
    positives = []
    for k in maps:
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        sm = _oracle_cp_map(wl, fac, img, lvl, comp, cache)
        sms[k] = sm
        fin = np.isfinite(sm.score)
        if fin.sum() >= 3:
            flat = np.where(fin, sm.score, -np.inf).ravel()
            for i in np.argsort(-flat)[:3]:
                positives.append((img, lvl, comp, int(i) // sm.score.shape[1], int(i) % sm.score.shape[1]))
    thr, terms = _oracle_thresholds(wl, fac, positives)
    ctx.set_thresholds(thr)
    s, o = _scores(ctx, lay, feats)
    n_cmp = n_pruned = n_skip = 0
    for k in maps:
        img, lvl, comp = int(lay.map_image[k]), int(lay.map_level[k]), int(lay.map_comp[k])
        c = wl.bank.components[comp]
        oct_ = wl.pyramids[img].octave
        sm = sms[k]
        pscore, pruned, margin = oracle.prune_component(
            sm.score, terms(img, lvl, c.root), [terms(img, lvl - oct_, q) for q in c.parts], c.anchors,
            thr[c.root], [thr[q] for q in c.parts])
        Ho, Wo = sm.score.shape
        n = Ho * Wo
        g = s[lay.map_score_off[k]:lay.map_score_off[k] + n].reshape(Ho, Wo)
        g0 = free_s[lay.map_score_off[k]:lay.map_score_off[k] + n].reshape(Ho, Wo)
        go = o[lay.map_offs_off[k]:lay.map_offs_off[k] + n * len(c.parts) * 2].reshape(len(c.parts), Ho, Wo, 2)
        decided = margin > TOL_CP
        n_skip += int((~decided).sum())
        gp = np.isneginf(g) & np.isfinite(g0)
        assert np.array_equal(gp[decided], (pruned & np.isfinite(sm.score))[decided]), f"map {k}: rejected sets differ"
        keep = ~np.isneginf(g)
        np.testing.assert_array_equal(g[keep], g0[keep])
        assert np.all(go[:, np.isneginf(g) & np.isfinite(g0)] == 0)
        n_cmp += int(decided.sum())
        n_pruned += int(gp.sum())
    for (img, lvl, comp, y, x) in positives:
        k = lay.find(img, lvl, comp)
        assert np.isfinite(s[lay.map_score_off[k] + y * int(lay.map_cols[k]) + x]), "a positive was rejected"
    note(f"  {n_cmp} decisions compared ({n_skip} near-ties skipped), {n_pruned} rejected, "
         f"{len(positives)} positives")
    assert n_pruned > 0
    ctx.set_thresholds(None)
    s2, _ = _scores(ctx, lay, feats)
    np.testing.assert_array_equal(s2, free_s)
    ctx.close()
