"""GPU parity on filter shapes outside the DPM defaults: 1x1 up to the
16 x 32 maximum, tall (> 8 rows) and wide filters, in every correlation
flavour.  These run the kernels' generic instances (the rolled filter-row
loop of the shift-GEMM for tall filters, the runtime-shape CP tile) that the
DPM-shaped workloads never reach."""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_common import TOL, note, oracle_basis

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(5, 7), (1, 1), (3, 5), (9, 4), (16, 32), (12, 20), (16, 1), (2, 32), (6, 6), (11, 13)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _odd_workload():
    rng = workloads.seed_rng(77, 1)
    q, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    basis = q[:, :8]
    filters = [workloads.draw_filter(rng, h, w, basis) for (h, w) in SHAPES]
    comps = [workloads.Component(0, [1, 2, 3], np.array([[0, 0], [3, 2], [1, 9]], np.int32),
                                 np.array([[0.02, 0.05, -0.01, 0.08]] * 3, np.float32)),
             workloads.Component(4, [5, 6, 7, 8, 9], np.array([[4, 10], [0, 31], [30, 0], [20, 25], [7, 3]],
                                                                np.int32),
                                 np.array([[0.05, 0.03, 0.02, 0.04]] * 5, np.float32))]
    levels = [workloads.Level(0, 70, 90), workloads.Level(70 * 90, 40, 50)]
    pyr = workloads.Pyramid(levels, octave=1)
    bank = workloads.Bank(filters, comps)
    return workloads.Workload("odd shapes", 77, [pyr], bank, 70 * 90 + 40 * 50,
                              workloads.feature_seed(77), False, [(90, 70)])


def _ctx(wl, mode, rank):
    from paper_1707_03268_amd import Context
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    ref = None
    if mode == "cp_fp32":
        ctx.decompose_cp(rank, max_iters=40)
        _, fac = ctx.get_cp(wl.bank.shapes)
        ref = [tuple(m.astype(np.float64) for m in abc) for abc in fac]
    elif mode != "direct_fp32":
        ctx.decompose(rank)
        ref = oracle_basis(wl.bank.filters, rank)
    ctx.plan(wl.pyramids)
    return ctx, ref


def _ref_response(mode, X, f, k, ref):
    if mode == "direct_fp32":
        return oracle.correlate(X, f)
    if mode == "cp_fp32":
        return oracle.cp_response(X, *ref[k])
    return oracle.tensor_response(X, f, ref)


@pytest.mark.parametrize("mode,rank", [("direct_fp32", None), ("tensor_fp32", 8), ("tensor_bf16", 16),
                                       ("cp_fp32", 3), ("cp_fp32", 7)])
def test_odd_shapes_level_responses(mode, rank):
    wl = _odd_workload()
    note(f"odd shapes responses {mode} R={rank}")
    ctx, ref = _ctx(wl, mode, rank)
    feats = torch.from_numpy(wl.features()).cuda()
    tol = TOL.get(mode, 1e-4)
    for level in (0, 1):
        out, total = ctx.level_responses(mode, feats, 0, level)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        X = wl.level_features(0, level).astype(np.float64)
        off = 0
        for k, f in enumerate(wl.bank.filters):
            Ho, Wo = X.shape[0] - f.shape[0] + 1, X.shape[1] - f.shape[1] + 1
            if Ho <= 0 or Wo <= 0:
                continue
            want = _ref_response(mode, X, f.astype(np.float64), k, ref)
            g = got[off:off + Ho * Wo].reshape(Ho, Wo)
            off += Ho * Wo
            err = float(np.max(np.abs(g - want)))
            assert err <= tol, f"level {level} filter {k} {f.shape[:2]}: max |err| {err:.3g} > {tol}"
        assert off == total
    ctx.close()


@pytest.mark.parametrize("mode,rank", [("direct_fp32", None), ("cp_fp32", 5)])
def test_odd_shapes_scores(mode, rank):
    """Score maps of both components (a 5x7 root with 1x1, 3x5 and 9x4 parts;
    the 16x32 root with 12x20, 16x1, 2x32, 6x6 and 11x13 parts)."""
    wl = _odd_workload()
    note(f"odd shapes scores {mode}")
    ctx, ref = _ctx(wl, mode, rank)
    lay = ctx.layout
    feats = torch.from_numpy(wl.features()).cuda()
    scores = torch.full((max(lay.n_score, 1),), float("nan"), dtype=torch.float32, device="cuda")
    offs = torch.full((max(lay.n_offsets, 1),), -32768, dtype=torch.int16, device="cuda")
    ctx.score_pyramid(mode, feats, scores, offs)
    torch.cuda.synchronize()
    s, o = scores.cpu().numpy(), offs.cpu().numpy()
    levels = [wl.level_features(0, 0).astype(np.float64), wl.level_features(0, 1).astype(np.float64)]
    tol = TOL.get(mode, 1e-4)
    maps = oracle.score_pyramid(levels, wl.bank.filters, wl.bank.components, 1,
                                response=lambda X, q: _ref_response(mode, X, wl.bank.filters[q].astype(np.float64), q, ref))
    for ci, c in enumerate(wl.bank.components):
        k = lay.find(0, 1, ci)
        Ho, Wo = int(lay.map_rows[k]), int(lay.map_cols[k])
        sm = maps[(1, ci)]
        assert sm.score.shape == (Ho, Wo)
        g = s[lay.map_score_off[k]:lay.map_score_off[k] + Ho * Wo].reshape(Ho, Wo)
        fin = np.isfinite(sm.score)
        assert np.array_equal(np.isfinite(g), fin)
        if fin.any():
            assert np.max(np.abs(g[fin] - sm.score[fin])) <= tol
        go = o[lay.map_offs_off[k]:lay.map_offs_off[k] + Ho * Wo * len(c.parts) * 2].reshape(len(c.parts), Ho, Wo, 2)
        check = sm.margin > tol
        assert not (check[..., None] & (go != sm.offsets)).any()
    ctx.close()


def _mixed_height_workload():
    """Filters of 6, 7, 8, 9 and 10 rows in one bank: the taller ones select
    the 16-row correlation instance, which still runs the 6- to 8-row groups
    through its unrolled, three-buffer staging (the LDS must hold three chunks
    of 8 rows as well as two of 10)."""
    rng = workloads.seed_rng(79, 1)
    q, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    basis = q[:, :8]
    shapes = [(10, 6), (8, 6), (8, 6), (7, 5), (6, 6), (8, 11), (10, 4), (9, 6), (8, 8)]
    filters = [workloads.draw_filter(rng, h, w, basis) for (h, w) in shapes]
    comps = [workloads.Component(0, [1, 2, 3, 4], np.array([[0, 0], [12, 6], [5, 7], [14, 3]], np.int32),
                                 np.array([[0.02, 0.05, -0.01, 0.08]] * 4, np.float32)),
             workloads.Component(5, [6, 7, 8], np.array([[3, 18], [7, 0], [8, 14]], np.int32),
                                 np.array([[0.05, 0.03, 0.02, 0.04]] * 3, np.float32))]
    levels = [workloads.Level(0, 66, 95), workloads.Level(66 * 95, 33, 47)]
    pyr = workloads.Pyramid(levels, octave=1)
    return workloads.Workload("mixed heights", 79, [pyr], workloads.Bank(filters, comps),
                              66 * 95 + 33 * 47, workloads.feature_seed(79), False, [(95, 66)])


@pytest.mark.parametrize("mode,rank", [("tensor_bf16", 8), ("tensor_fp32", 4), ("tensor_bf16", 16),
                                       ("direct_fp32", None)])
def test_mixed_heights_8_and_10_rows(mode, rank):
    """Responses of every filter on both levels and the score maps of both
    components, for a bank that mixes 8-row and 10-row filters, in the modes
    whose 16-byte planes take the 64-filter tiles with unrolled staging."""
    from _gpu_common import Cmp, compare_map, oracle_map, run_gpu
    wl = _mixed_height_workload()
    note(f"mixed 8/10-row bank {mode} R={rank}")
    ctx, ref = _ctx(wl, mode, rank)
    feats = torch.from_numpy(wl.features()).cuda()
    tol = TOL[mode]
    for level in (0, 1):
        out, total = ctx.level_responses(mode, feats, 0, level)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        X = wl.level_features(0, level).astype(np.float64)
        off = 0
        for k, f in enumerate(wl.bank.filters):
            Ho, Wo = X.shape[0] - f.shape[0] + 1, X.shape[1] - f.shape[1] + 1
            want = _ref_response(mode, X, f.astype(np.float64), k, ref)
            g = got[off:off + Ho * Wo].reshape(Ho, Wo)
            off += Ho * Wo
            err = float(np.max(np.abs(g - want)))
            assert err <= tol, f"level {level} filter {k} {f.shape[:2]}: max |err| {err:.3g} > {tol}"
        assert off == total
    ctx.close()
    run = run_gpu(wl, mode, rank)
    cmp = Cmp()
    for ci in range(len(wl.bank.components)):
        compare_map(run, wl, 0, 1, ci, oracle_map(wl, 0, 1, ci, run.basis, {}), tol, cmp)
    note(f"  {cmp.n_pos} positions, max |score err| {cmp.max_err:.3g}")


# ------------------------------------------------------------ placement limits
# (part level rows, cols, root level rows, cols): the widest part rows the
# placement stages (1976 responses, plus a 72-cell window span = 2048 floats),
# and the tallest score maps one placement block holds in its 160 KB of LDS.
LIMITS = [("widest", 40, 1981, 20, 990), ("tallest", 1011, 40, 505, 20)]


def _limit_workload(part_rows, part_cols, root_rows, root_cols):
    """One component (a 6x11 root, three 6x6 parts) on a two-level pyramid at
    one of the placement's limits.  The first part's quadratic terms are tiny,
    so that its windows span whole rows and columns: the staged row span and
    the cost tables reach the sizes the plan provisions for."""
    rng = workloads.seed_rng(78, 1)
    q, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    basis = q[:, :8]
    filters = [workloads.draw_filter(rng, 6, 11, basis)] + [workloads.draw_filter(rng, 6, 6, basis) for _ in range(3)]
    comps = [workloads.Component(0, [1, 2, 3], np.array([[0, 0], [4, 9], [6, 16]], np.int32),
                                 np.array([[0.0, 1e-6, 0.0, 1e-6], [0.05, 0.02, 0.02, 0.01],
                                           [0.0, 0.06, 0.01, 0.05]], np.float32))]
    levels = [workloads.Level(0, part_rows, part_cols),
              workloads.Level(part_rows * part_cols, root_rows, root_cols)]
    pyr = workloads.Pyramid(levels, octave=1)
    return workloads.Workload(f"placement limit {part_rows}x{part_cols}", 78, [pyr],
                              workloads.Bank(filters, comps), part_rows * part_cols + root_rows * root_cols,
                              workloads.feature_seed(78), False, [(part_cols, part_rows)])


@pytest.mark.parametrize("name,pr,pc,rr,rc", LIMITS)
@pytest.mark.parametrize("mode,rank", [("direct_fp32", None), ("tensor_bf16", 16)])
def test_placement_limits_scores(name, pr, pc, rr, rc, mode, rank):
    """The whole score map at the largest sizes dpmt_plan accepts."""
    from _gpu_common import Cmp, compare_map, oracle_map, run_gpu
    wl = _limit_workload(pr, pc, rr, rc)
    note(f"placement limit {name}: part level {pr}x{pc}, {mode}")
    run = run_gpu(wl, mode, rank)
    cmp = Cmp()
    sm = oracle_map(wl, 0, 1, 0, run.basis, {})
    compare_map(run, wl, 0, 1, 0, sm, TOL[mode], cmp)
    note(f"  {cmp.n_pos} positions, max |score err| {cmp.max_err:.3g}, argmax checked "
         f"{cmp.n_arg_checked}/{cmp.n_arg}")


# ------------------------------------------------- part maps taller than needed
def _tall_part_level_workload():
    """A part level far taller than its root level needs (60 rows of parts for
    a 7-row score map): the column pass's last groups of 4 window offsets then
    reach part rows below every target's window.  The first part (weak
    vertical deformation, anchor row 6, a filter 5x the norm of the others)
    has large row-pass values on those rows; the second (strong vertical
    deformation, anchor row 0) must not see them."""
    rng = workloads.seed_rng(79, 1)
    q, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    basis = q[:, :8]
    root = workloads.draw_filter(rng, 6, 11, basis)
    pa = 5.0 * workloads.draw_filter(rng, 6, 6, basis)
    pb = workloads.draw_filter(rng, 6, 6, basis)
    comps = [workloads.Component(0, [1, 2], np.array([[6, 3], [0, 8]], np.int32),
                                 np.array([[0.0, 0.05, 0.0, 1e-4], [0.01, 0.05, 0.0, 2.0]], np.float32))]
    levels = [workloads.Level(0, 60, 40), workloads.Level(60 * 40, 12, 20)]
    pyr = workloads.Pyramid(levels, octave=1)
    return workloads.Workload("tall part level", 79, [pyr], workloads.Bank([root, pa, pb], comps),
                              60 * 40 + 12 * 20, workloads.feature_seed(79), False, [(40, 60)])


@pytest.mark.parametrize("mode,rank", [("direct_fp32", None), ("tensor_fp32", 32)])
def test_part_level_taller_than_the_windows(mode, rank):
    from _gpu_common import Cmp, compare_map, oracle_map, run_gpu
    wl = _tall_part_level_workload()
    note(f"tall part level, {mode}")
    run = run_gpu(wl, mode, rank)
    cmp = Cmp()
    sm = oracle_map(wl, 0, 1, 0, run.basis, {})
    compare_map(run, wl, 0, 1, 0, sm, TOL[mode], cmp)
    assert cmp.n_pos == 7 * 10
