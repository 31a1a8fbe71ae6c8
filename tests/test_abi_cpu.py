"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, enforces its state machine and argument validation, and its host-side
FP64 decomposition and planning agree with the oracle.  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from paper_1707_03268_amd import Context, DpmtError, _abi

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "dpmt.h")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpmt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = _declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"


def test_status_strings():
    lib = _abi.load()
    for s in range(-6, 1):
        assert lib.dpmt_status_string(s)
    assert lib.dpmt_status_string(0) == b"ok"


def _tiny_bank():
    wl = workloads.config1()
    return wl, wl.bank.filters, wl.bank.components


def test_state_machine_host_only():
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    with pytest.raises(DpmtError) as e:
        ctx.decompose(4)
    assert e.value.status == _abi.DPMT_E_STATE
    with pytest.raises(DpmtError) as e:
        ctx.plan(wl.pyramids)
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.load_filters(fs, comps)
    lay = ctx.plan(wl.pyramids)
    assert lay.n_maps == 1
    # a host-only context plans but never scores
    lib = _abi.load()
    st = lib.dpmt_score_pyramid(ctx._h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None)
    assert st == _abi.DPMT_E_STATE
    # tensor mode before decompose
    ctx2 = Context(device=-1)
    ctx2.load_filters(fs, comps)
    ctx2.plan(wl.pyramids)
    st = lib.dpmt_score_pyramid(ctx2._h, _abi.TENSOR_BF16, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None)
    assert st == _abi.DPMT_E_STATE
    assert b"decompose" in lib.dpmt_last_error(ctx2._h)


@pytest.mark.parametrize("rank", [0, 33, -1])
def test_bad_rank(rank):
    _, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)
    with pytest.raises(DpmtError) as e:
        ctx.decompose(rank)
    assert e.value.status == _abi.DPMT_E_RANK


def _comp(root, parts, anchors, deform):
    class C:
        pass
    c = C()
    c.root, c.parts, c.anchors, c.deform = root, parts, np.array(anchors), np.array(deform, np.float32)
    return c


def test_validation_errors():
    rng = np.random.default_rng(0)
    fs = [rng.standard_normal((6, 11, 32)).astype(np.float32), rng.standard_normal((6, 6, 32)).astype(np.float32)]
    good = _comp(0, [1], [[0, 0]], [[0.1, 0.1, 0.1, 0.1]])
    ctx = Context(device=-1)
    ctx.load_filters(fs, [good])
    bad_cases = [
        ([_comp(0, [1], [[0, 0]], [[0.1, 0.0, 0.1, 0.1]])], "quadratic"),       # d_xx = 0
        ([_comp(0, [1], [[0, 0]], [[0.1, 0.1, 0.1, -0.2]])], "quadratic"),      # d_yy < 0
        ([_comp(0, [1], [[7, 0]], [[0.1, 0.1, 0.1, 0.1]])], "anchor"),          # v_y > 2*6-6
        ([_comp(0, [1], [[0, 17]], [[0.1, 0.1, 0.1, 0.1]])], "anchor"),         # v_x > 2*11-6
        ([_comp(0, [1], [[-1, 0]], [[0.1, 0.1, 0.1, 0.1]])], "anchor"),
        ([_comp(2, [1], [[0, 0]], [[0.1, 0.1, 0.1, 0.1]])], "root"),
        ([_comp(0, [5], [[0, 0]], [[0.1, 0.1, 0.1, 0.1]])], "part"),
        ([_comp(0, [1], [[0, 0]], [[np.nan, 0.1, 0.1, 0.1]])], "non-finite"),
    ]
    for comps, word in bad_cases:
        with pytest.raises(DpmtError) as e:
            ctx.load_filters(fs, comps)
        assert e.value.status == _abi.DPMT_E_INVALID
        assert word in str(e.value)
    nan_fs = [fs[0].copy(), fs[1]]
    nan_fs[0][1, 2, 3] = np.inf
    with pytest.raises(DpmtError) as e:
        ctx.load_filters(nan_fs, [good])
    assert e.value.status == _abi.DPMT_E_INVALID
    big = [rng.standard_normal((17, 6, 32)).astype(np.float32), fs[1]]
    with pytest.raises(DpmtError) as e:
        ctx.load_filters(big, [good])
    assert e.value.status == _abi.DPMT_E_UNSUPPORTED
    # the failed loads left the accepted bank in place
    ctx.decompose(8)


def test_plan_validation():
    _, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)

    class P:
        pass
    p = P()
    p.levels = [workloads.Level(0, 0, 5)]
    p.octave = 1
    with pytest.raises(DpmtError) as e:
        ctx.plan([p])
    assert e.value.status == _abi.DPMT_E_INVALID
    p.levels = [workloads.Level(0, 10, 10)]
    p.octave = 0
    with pytest.raises(DpmtError):
        ctx.plan([p])


def _one_component_bank():
    rng = np.random.default_rng(5)
    fs = [rng.standard_normal((6, 11, 32)).astype(np.float32), rng.standard_normal((6, 6, 32)).astype(np.float32)]
    comps = [workloads.Component(root=0, parts=[1], anchors=np.array([[2, 3]], np.int32),
                                 deform=np.array([[0.05, 0.05, 0.05, 0.05]], np.float32))]
    return fs, comps


def _two_level_pyramid(part_rows, part_cols, root_rows, root_cols):
    """Octave 1: parts on level 0, roots on level 1."""
    return workloads.Pyramid([workloads.Level(0, part_rows, part_cols),
                              workloads.Level(part_rows * part_cols, root_rows, root_cols)], octave=1)


def test_plan_size_limits():
    """The largest sizes plan; past them dpmt_plan fails with DPMT_E_UNSUPPORTED
    and names the limit, and the context still plans a valid batch afterwards."""
    fs, comps = _one_component_bank()
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)
    # part response rows of up to 1976 cells fit the placement's staging
    # (a row window spans the row plus 72 cells)
    lay = ctx.plan([_two_level_pyramid(40, 1981, 20, 990)])
    assert lay.n_maps == 1 and int(lay.map_cols[0]) == 990 - 11 + 1
    with pytest.raises(DpmtError) as e:
        ctx.plan([_two_level_pyramid(40, 1982, 20, 991)])
    assert e.value.status == _abi.DPMT_E_UNSUPPORTED and "wider" in str(e.value)
    # a placement block holds a whole strip of a score map in LDS (160 KB)
    ctx.plan([_two_level_pyramid(800, 40, 400, 20)])
    with pytest.raises(DpmtError) as e:
        ctx.plan([_two_level_pyramid(1400, 40, 700, 20)])
    assert e.value.status == _abi.DPMT_E_UNSUPPORTED and "tall" in str(e.value)
    # level sides beyond 16384 cells
    with pytest.raises(DpmtError) as e:
        ctx.plan([_two_level_pyramid(20, 16385, 10, 100)])
    assert e.value.status == _abi.DPMT_E_UNSUPPORTED
    lay = ctx.plan([_two_level_pyramid(60, 80, 30, 40)])
    assert lay.n_maps == 1
    ctx.close()


def test_null_pointer_rejected():
    lib = _abi.load()
    assert lib.dpmt_create(None, 0, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_load_filters(None, 1, None, None, 1, None) == _abi.DPMT_E_INVALID
    ctx = Context(device=-1)
    assert lib.dpmt_load_filters(ctx._h, 1, None, None, 1, None) == _abi.DPMT_E_INVALID
    d = (ctypes.c_float * 4)(0.1, 0.1, 0.1, 0.1)
    assert lib.dpmt_distance_transform(None, 4, 4, 4, d, None, None, None, None) == _abi.DPMT_E_INVALID
    bad = (ctypes.c_float * 4)(0.1, 0.0, 0.1, 0.1)
    assert lib.dpmt_distance_transform(ctypes.c_void_p(16), 4, 4, 4, bad, ctypes.c_void_p(16), None, None, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_distance_transform(ctypes.c_void_p(16), 4, 4, 3, d, ctypes.c_void_p(16), None, None, None) == _abi.DPMT_E_INVALID


# ------------------------------------------------------------ host-side parity
@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_decompose_matches_oracle(cfg):
    """The library's FP64 shared basis against the oracle's on every preset
    bank, the 1,080-filter banks of the larger workloads included."""
    wl = workloads.PRESETS[cfg]()
    ctx = Context(device=-1)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    for R in (1, 4, 8, 16, 32):
        sigma, U = ctx.decompose(R)
        dec = oracle.decompose(wl.bank.filters, R)
        assert dec.gap > 1e-9 or R < 32, "full rank always has a gap"
        np.testing.assert_allclose(sigma, dec.sigma, rtol=1e-10, atol=1e-12 * dec.sigma[0])
        if dec.gap > 1e-9:      # the subspace is unique only with a gap at R
            np.testing.assert_allclose(U @ U.T, dec.U @ dec.U.T, atol=1e-10)
        np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-12)
        # sign convention: largest-magnitude entry of every column positive
        idx = np.argmax(np.abs(U), axis=0)
        assert np.all(U[idx, np.arange(R)] > 0)


def test_plan_layout_matches_definition():
    wl = workloads.config2()
    ctx = Context(device=-1)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    lay = ctx.plan(wl.pyramids)
    cnt = workloads.count_responses(wl)
    assert lay.n_resp == cnt["total"] and lay.n_resp_root == cnt["root"] and lay.n_resp_part == cnt["part"]
    pyr = wl.pyramids[0]
    L = len(pyr.levels)
    assert lay.n_maps == (L - pyr.octave) * len(wl.bank.components)
    off = 0
    offs = 0
    for k in range(lay.n_maps):
        lv = pyr.levels[lay.map_level[k]]
        comp = wl.bank.components[lay.map_comp[k]]
        h0, w0 = wl.bank.filters[comp.root].shape[:2]
        assert lay.map_rows[k] == max(lv.rows - h0 + 1, 0)
        assert lay.map_cols[k] == max(lv.cols - w0 + 1, 0)
        assert lay.map_score_off[k] == off and lay.map_offs_off[k] == offs
        off += lay.map_rows[k] * lay.map_cols[k]
        offs += lay.map_rows[k] * lay.map_cols[k] * len(comp.parts) * 2
    assert lay.n_score == off and lay.n_offsets == offs
    assert lay.n_cells == wl.total_cells


def test_launch_strategy_and_tile_config_validation():
    from paper_1707_03268_amd import tile_config_count, tile_config_name
    lib = _abi.load()
    n = tile_config_count()
    assert n >= 2
    names = [tile_config_name(i) for i in range(n)]
    assert all(names) and len(set(names)) == n
    assert tile_config_name(-1) is None and tile_config_name(n) is None
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)
    for launch in ("batched", "per_level", "graph", "overlap"):
        ctx.set_launch(launch)
    with pytest.raises(DpmtError) as e:
        ctx.set_launch(4)
    assert e.value.status == _abi.DPMT_E_INVALID
    assert ctx.get_tile_config("tensor_bf16") == 0
    ctx.set_tile_config("tensor_bf16", n - 1)
    assert ctx.get_tile_config("tensor_bf16") == n - 1
    for bad in (-1, n):
        with pytest.raises(DpmtError) as e:
            ctx.set_tile_config("tensor_bf16", bad)
        assert e.value.status == _abi.DPMT_E_INVALID
    assert lib.dpmt_get_tile_config(None, 0) == -1
    # autotuning needs a device context
    ctx.plan(wl.pyramids)
    st = lib.dpmt_autotune(ctx._h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 3, None, None, None)
    assert st == _abi.DPMT_E_STATE
    ctx.close()


def test_tall_filters_restrict_tile_configs():
    """Filters taller than 8 rows are supported by the default tile only."""
    from paper_1707_03268_amd import tile_config_count
    rng = np.random.default_rng(0)
    fs = [rng.standard_normal((12, 5, 32)).astype(np.float32), rng.standard_normal((3, 3, 32)).astype(np.float32)]
    comps = [workloads.Component(root=0, parts=[1], anchors=np.array([[0, 0]], np.int32),
                                 deform=np.array([[0.05, 0.05, 0.05, 0.05]], np.float32))]
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)
    ctx.set_tile_config("direct_fp32", 0)
    rejected = 0
    for cfg in range(1, tile_config_count()):
        try:
            ctx.set_tile_config("direct_fp32", cfg)
        except DpmtError as e:
            assert e.status == _abi.DPMT_E_UNSUPPORTED
            rejected += 1
    assert rejected >= 1
    ctx.close()


def test_detect_validation():
    lib = _abi.load()
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    st = lib.dpmt_detect(ctx._h, ctypes.c_void_p(16), 0.0, None, 0, ctypes.c_void_p(16), None)
    assert st == _abi.DPMT_E_STATE                       # no plan
    ctx.load_filters(fs, comps)
    ctx.plan(wl.pyramids)
    st = lib.dpmt_detect(ctx._h, ctypes.c_void_p(16), 0.0, None, 0, ctypes.c_void_p(16), None)
    assert st == _abi.DPMT_E_STATE                       # host-only context
    assert lib.dpmt_detect(None, None, 0.0, None, 0, None, None) == _abi.DPMT_E_INVALID
    ctx.close()


# ------------------------------------------------------------ per-filter CP form
def test_cp_validation_host_only():
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    with pytest.raises(DpmtError) as e:
        ctx.decompose_cp(4)
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.load_filters(fs, comps)
    n = len(fs)
    for bad in (0, 33):
        with pytest.raises(DpmtError) as e:
            ctx.decompose_cp(bad)
        assert e.value.status == _abi.DPMT_E_RANK
    lib = _abi.load()
    r = np.full(n, 3, np.int32)
    rp = r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.dpmt_decompose_cp(ctx._h, rp, 0, 1e-6, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_decompose_cp(ctx._h, rp, 5, -1.0, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_decompose_cp(ctx._h, rp, 5, float("nan"), None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_decompose_cp(ctx._h, None, 5, 1e-6, None) == _abi.DPMT_E_INVALID
    with pytest.raises(DpmtError) as e:
        ctx.get_cp(wl.bank.shapes)
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.plan(wl.pyramids)
    # the CP mode without factors is out of order
    st = lib.dpmt_score_pyramid(ctx._h, _abi.CP_FP32, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None)
    assert st == _abi.DPMT_E_STATE
    # non-finite factors are refused, finite ones round-trip exactly
    rng = np.random.default_rng(0)
    fac = [(rng.standard_normal((h, 3)), rng.standard_normal((w, 3)), rng.standard_normal((32, 3)))
           for (h, w) in wl.bank.shapes]
    bad = [tuple(m.copy() for m in abc) for abc in fac]
    bad[2][1][0, 0] = np.inf
    with pytest.raises(DpmtError) as e:
        ctx.load_cp(3, bad)
    assert e.value.status == _abi.DPMT_E_INVALID
    ctx.load_cp(3, fac)
    ranks, got = ctx.get_cp(wl.bank.shapes)
    assert np.all(ranks == 3)
    for a, b in zip(fac, got):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.astype(np.float32), y)
    # only tile configuration 0 exists for the CP mode
    with pytest.raises(DpmtError) as e:
        ctx.set_tile_config("cp_fp32", 1)
    assert e.value.status == _abi.DPMT_E_UNSUPPORTED
    ctx.set_tile_config("cp_fp32", 0)
    assert ctx.get_tile_config("cp_fp32") == 0
    ctx.close()


def test_cp_als_matches_oracle_and_recovers_planted_rank():
    """The library's host ALS against the oracle's pins: a planted rank-R bank
    is fitted to rounding, and on the synthetic bank both reach the same error."""
    wl, fs, comps = _tiny_bank()
    rng = np.random.default_rng(3)
    planted = []
    for f in fs:
        h, w, _ = f.shape
        A, B, C = rng.standard_normal((h, 3)), rng.standard_normal((w, 3)), rng.standard_normal((32, 3))
        planted.append(oracle.cp_reconstruct(A, B, C).astype(np.float32))
    ctx = Context(device=-1)
    ctx.load_filters(planted, comps)
    err = ctx.decompose_cp(3, max_iters=3000, tol=1e-7)
    assert err.max() < 1e-6, err
    ranks, fac = ctx.get_cp(wl.bank.shapes)
    for f, (A, B, C) in zip(planted, fac):
        rec = oracle.cp_reconstruct(A.astype(np.float64), B.astype(np.float64), C.astype(np.float64))
        assert np.linalg.norm(rec - f) <= 1e-5 * np.linalg.norm(f)
    # the synthetic bank at ranks 2, 6 and 9 (beyond the 6-row mode)
    ctx.load_filters(fs, comps)
    for R in (2, 6, 9):
        err = ctx.decompose_cp(R, max_iters=200, tol=1e-12)
        for k in (0, 1, 4):
            f = fs[k].astype(np.float64)
            cp = oracle.cp_als(f, R, iters=200, eps=1e-12)
            e_or = cp.errors[-1] / np.linalg.norm(f)
            assert abs(err[k] - e_or) <= 0.02 * e_or + 1e-9, (R, k, err[k], e_or)
    ctx.close()


def test_select_ranks_matches_oracle():
    """The library's rank selection (binary search over ALS fits, Section 4
    criterion) against the oracle's on the c1 bank, at several e; the chosen
    fits become the CP factors."""
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    with pytest.raises(DpmtError) as e:
        ctx.select_ranks(1.0)
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.load_filters(fs, comps)
    for bad in (0, 33):
        with pytest.raises(DpmtError) as e:
            ctx.select_ranks(1.0, r_max=bad)
        assert e.value.status == _abi.DPMT_E_RANK
    with pytest.raises(DpmtError) as e:
        ctx.select_ranks(-1.0)
    assert e.value.status == _abi.DPMT_E_INVALID
    for e in (5.0, 40.0):
        ranks, err = ctx.select_ranks(e, r_max=12, max_iters=200)
        for k in range(len(fs)):
            want, _ = oracle.select_rank(fs[k].astype(np.float64), e, 12, iters=200)
            assert ranks[k] == want, (e, k, ranks[k], want)
        got_r, fac = ctx.get_cp(wl.bank.shapes)
        np.testing.assert_array_equal(got_r, ranks)
        for f, (A, B, C), rel in zip(fs, fac, err):
            rec = oracle.cp_reconstruct(A.astype(np.float64), B.astype(np.float64), C.astype(np.float64))
            assert abs(np.linalg.norm(rec - f) / np.linalg.norm(f) - rel) < 1e-5
    ctx.close()


def test_select_ranks_squared_bound_hand_case():
    """The hand-worked filter where Section 4's squared bound picks rank 2
    and an unsquared one would pick 1 (orthogonal terms of weights 1, 1/2, ...,
    1/32 on a 6x6x32 filter, e = 100): the library picks 2 as well."""
    f = np.zeros((6, 6, 32), np.float32)
    for j, w in enumerate([1, 1 / 2, 1 / 4, 1 / 8, 1 / 16, 1 / 32]):
        f[j, j, j] = w
    # a component needs a part: a 1x1 part rides along (rank 1 fits it exactly)
    part = np.zeros((1, 1, 32), np.float32)
    part[0, 0, 0] = 1.0
    comps = [workloads.Component(0, [1], np.zeros((1, 2), np.int32),
                                 np.array([[0.0, 0.1, 0.0, 0.1]], np.float32))]
    ctx = Context(device=-1)
    ctx.load_filters([f, part], comps)
    ranks, _ = ctx.select_ranks(100.0, r_max=6, max_iters=300)
    assert int(ranks[0]) == 2
    ctx.close()


def test_fit_thresholds_matches_oracle_and_validates():
    """The library's FP64 threshold fit (min over positives of the partial CP
    sums, root at the position, parts at their anchors) against the oracle."""
    wl, fs, comps = _tiny_bank()
    ctx = Context(device=-1)
    ctx.load_filters(fs, comps)
    with pytest.raises(DpmtError) as e:
        ctx.set_thresholds(np.zeros(4, np.float32))
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.decompose_cp(4, max_iters=30)
    X = wl.features()
    with pytest.raises(DpmtError) as e:                     # needs a plan
        ctx.fit_thresholds(X, [(0, 1, 0, 0, 0)])
    assert e.value.status == _abi.DPMT_E_STATE
    ctx.plan(wl.pyramids)
    ranks, fac = ctx.get_cp(wl.bank.shapes)
    fac64 = [tuple(m.astype(np.float64) for m in abc) for abc in fac]
    c = comps[0]
    Ho, Wo = 30 - 6 + 1, 40 - 11 + 1
    rng = np.random.default_rng(8)
    pos = [(0, 1, 0, int(rng.integers(0, Ho)), int(rng.integers(0, Wo))) for _ in range(9)]
    t = ctx.fit_thresholds(X, pos, margin=0.0)
    Xr = wl.level_features(0, 1).astype(np.float64)
    Xp = wl.level_features(0, 0).astype(np.float64)
    off = np.concatenate([[0], np.cumsum(ranks)])
    rt = oracle.cp_terms(Xr, *fac64[c.root])
    want = oracle.fit_thresholds([oracle.partial_sums(rt, y, x) for (_, _, _, y, x) in pos])
    np.testing.assert_allclose(t[off[c.root]:off[c.root + 1]], want, rtol=1e-6, atol=1e-6)
    for i, k in enumerate(c.parts):
        pt = oracle.cp_terms(Xp, *fac64[k])
        ps = [oracle.partial_sums(pt, 2 * y + c.anchors[i][0], 2 * x + c.anchors[i][1])
              for (_, _, _, y, x) in pos
              if 2 * y + c.anchors[i][0] < pt.shape[1] and 2 * x + c.anchors[i][1] < pt.shape[2]]
        got = t[off[k]:off[k + 1]]
        if ps:
            np.testing.assert_allclose(got, oracle.fit_thresholds(ps), rtol=1e-6, atol=1e-6)
        else:
            assert np.all(np.isneginf(got))
    # the margin is subtracted
    t2 = ctx.fit_thresholds(X, pos, margin=0.25)
    np.testing.assert_allclose(t2, t - 0.25, rtol=0, atol=1e-6)
    for bad in ([(0, 0, 0, 0, 0)], [(0, 1, 0, Ho, 0)], [(1, 1, 0, 0, 0)], [(0, 1, 1, 0, 0)]):
        with pytest.raises(DpmtError) as e:
            ctx.fit_thresholds(X, bad)
        assert e.value.status == _abi.DPMT_E_INVALID, bad
    with pytest.raises(DpmtError) as e:
        ctx.fit_thresholds(X, pos, margin=float("nan"))
    assert e.value.status == _abi.DPMT_E_INVALID
    bad = np.zeros(int(ranks.sum()), np.float32)
    bad[3] = np.nan
    with pytest.raises(DpmtError) as e:
        ctx.set_thresholds(bad)
    assert e.value.status == _abi.DPMT_E_INVALID
    ctx.set_thresholds(None)
    ctx.close()


def test_noalloc_distance_transform_limits_host_only():
    """The allocation-free transform rejects maps beyond its static scratch
    (either side > 16384, or more than 2^21 cells) before touching a device;
    dummy non-NULL pointers suffice since nothing is enqueued."""
    lib = _abi.load()
    d = (ctypes.c_float * 4)(0.0, 0.1, 0.0, 0.1)
    fake = ctypes.c_void_p(4096)
    for rows, cols in ((16385, 1), (1, 16385), (1449, 1449)):
        rc = lib.dpmt_distance_transform_noalloc(fake, rows, cols, cols, d, fake, None, None, None)
        assert rc == _abi.DPMT_E_UNSUPPORTED, (rows, cols, rc)
        assert b"allocation-free" in lib.dpmt_last_error(None)
    bad = (ctypes.c_float * 4)(0.0, 0.0, 0.0, 0.1)
    assert lib.dpmt_distance_transform_noalloc(fake, 4, 4, 4, bad, fake, None, None, None) == _abi.DPMT_E_INVALID
    assert _abi.DT_NOALLOC_MAX_CELLS == 1 << 21 and _abi.DT_NOALLOC_MAX_SIDE == 16384


def test_hog_arguments_host_only():
    """dpmt_hog_pyramid validates every argument before it needs a device:
    bad geometry is DPMT_E_INVALID (or DPMT_E_UNSUPPORTED past the size
    limits); valid arguments on a host-only context are DPMT_E_STATE."""
    lib = _abi.load()
    ctx = Context(device=-1)
    img, out = ctypes.c_void_p(16), ctypes.c_void_p(16)

    def call(levels, h=30, w=40, image=img, feats=out, handle=None):
        arr = (_abi.HogLevel * max(len(levels), 1))(*[_abi.HogLevel(*lv) for lv in levels])
        return lib.dpmt_hog_pyramid(ctx._h if handle is None else handle, image, h, w, len(levels), arr,
                                    feats, None)

    ok = [(0, 10, 12, 1, 2, 4, 1.0), (120, 6, 9, 3, 4, 8, 2.5)]
    assert call(ok) == _abi.DPMT_E_STATE
    assert b"host-only" in lib.dpmt_last_error(ctx._h)
    assert call([]) == _abi.DPMT_E_STATE
    assert ctypes.sizeof(_abi.HogLevel) == 32
    for bad in ([(0, 10, 12, 1, 2, 5, 1.0)],                        # cell
                [(0, 10, 12, 6, 2, 4, 1.0)],                        # padding rows
                [(0, 10, 12, 1, 7, 4, 1.0)],                        # padding cols
                [(0, 10, 12, -1, 2, 4, 1.0)],
                [(-5, 10, 12, 1, 2, 4, 1.0)],
                [(0, 10, 12, 1, 2, 4, 0.0)],
                [(0, 10, 12, 1, 2, 4, -2.0)],
                [(0, 10, 12, 1, 2, 4, float("nan"))],
                [(0, 10, 12, 1, 2, 4, 1.0), (119, 6, 9, 3, 4, 8, 2.5)]):   # overlap by one cell
        assert call(bad) == _abi.DPMT_E_INVALID, bad
    assert call(ok, h=0) == _abi.DPMT_E_INVALID
    assert call(ok, w=_abi.HOG_MAX_SIDE + 1) == _abi.DPMT_E_INVALID
    assert call(ok, image=None) == _abi.DPMT_E_INVALID
    assert call(ok, feats=None) == _abi.DPMT_E_INVALID
    assert call([(0, 16385, 12, 1, 2, 4, 1.0)]) == _abi.DPMT_E_UNSUPPORTED
    assert lib.dpmt_hog_pyramid(None, img, 30, 40, 0, None, out, None) == _abi.DPMT_E_INVALID


def test_distance_transform_method_validation():
    """An unknown method is DPMT_E_INVALID; the envelope method checks its
    arguments like the window method (no device needed to reject them)."""
    lib = _abi.load()
    d = (ctypes.c_float * 4)(0.0, 0.1, 0.0, 0.1)
    p = ctypes.c_void_p(16)
    assert lib.dpmt_distance_transform_method(p, 4, 4, 4, d, p, p, p, 7, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_distance_transform_method(p, 4, 4, 3, d, p, p, p, _abi.DT_ENVELOPE, None) == _abi.DPMT_E_INVALID
    bad = (ctypes.c_float * 4)(0.0, 0.0, 0.0, 0.1)
    assert lib.dpmt_distance_transform_method(p, 4, 4, 4, bad, p, p, p, _abi.DT_ENVELOPE, None) == _abi.DPMT_E_INVALID
    assert lib.dpmt_distance_transform_method(p, 4, 4, 4, d, p, p, None, _abi.DT_ENVELOPE, None) == _abi.DPMT_E_INVALID
