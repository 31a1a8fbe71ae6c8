"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to something fixed independently: a
hand-derived example (tests/golden), a textbook library routine, a closed
form, an invariant of the mathematics, or a direct search on tiny inputs.
All CPU-only.
"""
import json
import os

import numpy as np
from types import SimpleNamespace
import pytest
import scipy.signal

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- worked example
def test_worked_example_score_map():
    g = _load("worked_example.json")
    X0 = np.zeros((3, 4, 32))
    X0[:, :, 0] = np.array(g["root_level_ch0"])
    f0 = np.zeros((2, 2, 32))
    f0[:, :, 0] = np.array(g["root_filter_ch0"])
    X1 = np.zeros(tuple(g["part_level_shape"]) + (32,))
    for y, x, v in g["part_level_ch1_nonzero"]:
        X1[y, x, 1] = v
    f1 = np.zeros((1, 1, 32))
    f1[0, 0, 1] = g["part_filter_ch1"][0][0]
    rr = oracle.correlate(X0, f0)
    np.testing.assert_array_equal(rr, np.array(g["root_response"], float))
    pr = oracle.correlate(X1, f1)
    sm = oracle.score_component(rr, [pr], np.array([g["anchor"]]), np.array([g["deform"]], float))
    np.testing.assert_array_equal(sm.score, np.array(g["score"], float))
    np.testing.assert_array_equal(sm.D[0], np.array(g["D"], float))
    np.testing.assert_array_equal(sm.margin[0], np.array(g["margin"], float))
    place = np.array(g["placement"])
    Ho, Wo = rr.shape
    anchor_y = 2 * np.arange(Ho)[:, None] + g["anchor"][0]
    anchor_x = 2 * np.arange(Wo)[None, :] + g["anchor"][1]
    np.testing.assert_array_equal(sm.offsets[0, :, :, 0], place[:, :, 0] - anchor_y)
    np.testing.assert_array_equal(sm.offsets[0, :, :, 1], place[:, :, 1] - anchor_x)


def _pairing_case():
    g = _load("pyramid_pairing.json")
    levels = []
    for c0, c1 in zip(g["levels_ch0"], g["levels_ch1"]):
        X = np.zeros(np.array(c0).shape + (32,))
        X[:, :, 0] = np.array(c0)
        X[:, :, 1] = np.array(c1)
        levels.append(X)
    f_root = np.zeros((1, 1, 32))
    f_root[0, 0, 0] = 1.0
    f_part = np.zeros((1, 1, 32))
    f_part[0, 0, 1] = 1.0
    comp = SimpleNamespace(root=0, parts=[1], anchors=np.array([g["anchor"]]),
                           deform=np.array([g["deform"]], float))
    return g, levels, [f_root, f_part], [comp]


def test_score_pyramid_level_pairing_golden():
    """Root level l takes its parts from level l - octave (hand-worked
    three-level pyramid, tests/golden/pyramid_pairing.json)."""
    g, levels, filters, comps = _pairing_case()
    out = oracle.score_pyramid(levels, filters, comps, g["octave"])
    assert sorted(out) == [(1, 0), (2, 0)]
    np.testing.assert_array_equal(out[(1, 0)].score, np.array(g["score_level1"], float))
    np.testing.assert_array_equal(out[(2, 0)].score, np.array(g["score_level2"], float))
    np.testing.assert_array_equal(out[(1, 0)].offsets[0], np.array(g["offsets_level1"]))
    # a subset gives the same maps; a level below the octave is refused
    sub = oracle.score_pyramid(levels, filters, comps, g["octave"], root_levels=[2], comps=[0])
    np.testing.assert_array_equal(sub[(2, 0)].score, out[(2, 0)].score)
    with pytest.raises(ValueError):
        oracle.score_pyramid(levels, filters, comps, g["octave"], root_levels=[0])


def test_score_pyramid_worked_example_and_full_rank():
    """The worked example as a two-level pyramid (part level 6x8 = level 0,
    root level 3x4 = level 1, octave 1) gives its hand-derived score map, in
    the direct form and in the tensor form at full rank (U = I)."""
    g = _load("worked_example.json")
    X0 = np.zeros((3, 4, 32))
    X0[:, :, 0] = np.array(g["root_level_ch0"])
    X1 = np.zeros(tuple(g["part_level_shape"]) + (32,))
    for y, x, v in g["part_level_ch1_nonzero"]:
        X1[y, x, 1] = v
    f0 = np.zeros((2, 2, 32))
    f0[:, :, 0] = np.array(g["root_filter_ch0"])
    f1 = np.zeros((1, 1, 32))
    f1[0, 0, 1] = g["part_filter_ch1"][0][0]
    comp = SimpleNamespace(root=0, parts=[1], anchors=np.array([g["anchor"]]),
                           deform=np.array([g["deform"]], float))
    for U in (None, np.eye(32)):
        out = oracle.score_pyramid([X1, X0], [f0, f1], [comp], 1, U=U)
        np.testing.assert_array_equal(out[(1, 0)].score, np.array(g["score"], float))


def test_dt_1d_golden():
    for case in _load("dt_1d.json")["cases"]:
        resp = np.array([case["resp"]], float)
        r = oracle.distance_transform(resp, case["deform"])
        np.testing.assert_array_equal(r.D[0], np.array(case["D"], float))
        np.testing.assert_array_equal(r.arg_x[0], np.array(case["arg_x"]))
        np.testing.assert_array_equal(r.arg_y[0], np.zeros(len(case["D"]), int))
        np.testing.assert_array_equal(r.margin[0], np.array(case["margin"], float))


# ---------------------------------------------------------------- correlation
def test_correlate_matches_scipy_valid_correlation():
    rng = np.random.default_rng(0)
    for (H, W, h, w) in [(7, 9, 3, 2), (6, 11, 6, 11), (10, 8, 1, 1), (5, 5, 2, 4)]:
        X = rng.standard_normal((H, W, 32))
        f = rng.standard_normal((h, w, 32))
        ref = scipy.signal.correlate(X, f, mode="valid", method="direct")[:, :, 0]
        np.testing.assert_allclose(oracle.correlate(X, f), ref, rtol=1e-12, atol=1e-12)


def test_correlate_is_not_a_convolution():
    # A one-hot filter at tap (n, m) must read X[y+n, x+m]: a flipped
    # (convolution) implementation would read X[y+h-1-n, x+w-1-m].
    X = np.arange(5 * 6 * 32, dtype=float).reshape(5, 6, 32)
    f = np.zeros((2, 3, 32))
    f[0, 2, 4] = 1.0
    out = oracle.correlate(X, f)
    np.testing.assert_array_equal(out, X[0:4, 2:6, 4])


def test_correlate_linearity():
    rng = np.random.default_rng(1)
    X1, X2 = rng.standard_normal((2, 9, 12, 32))
    f1, f2 = rng.standard_normal((2, 4, 5, 32))
    a, b = 0.7, -1.3
    lhs = oracle.correlate(a * X1 + b * X2, f1)
    rhs = a * oracle.correlate(X1, f1) + b * oracle.correlate(X2, f1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    lhs = oracle.correlate(X1, a * f1 + b * f2)
    rhs = a * oracle.correlate(X1, f1) + b * oracle.correlate(X1, f2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_correlate_filter_larger_than_level_is_empty():
    assert oracle.correlate(np.zeros((4, 4, 32)), np.zeros((5, 2, 32))).shape == (0, 3)


# ---------------------------------------------------------------- decomposition
def _planted_bank(rng, sigmas, shapes):
    """Filters whose stacked cell vectors are A diag(sigmas) Q^T with A, Q orthonormal:
    the mode-3 singular values are exactly ``sigmas`` and the leading subspace is Q."""
    n_rows = sum(h * w for h, w in shapes)
    k = len(sigmas)
    A, _ = np.linalg.qr(rng.standard_normal((n_rows, k)))
    Q, _ = np.linalg.qr(rng.standard_normal((32, k)))
    M = A @ np.diag(sigmas) @ Q.T
    filters, r = [], 0
    for h, w in shapes:
        filters.append(M[r:r + h * w].reshape(h, w, 32))
        r += h * w
    return filters, Q


def test_decompose_recovers_planted_spectrum_and_subspace():
    rng = np.random.default_rng(2)
    sig = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    filters, Q = _planted_bank(rng, sig, [(6, 11), (6, 6), (7, 13), (6, 6), (8, 15)])
    for R in (1, 3, 6):
        dec = oracle.decompose(filters, R)
        np.testing.assert_allclose(dec.sigma[:6], sig, rtol=1e-10)
        np.testing.assert_allclose(dec.sigma[6:], 0.0, atol=1e-7)
        P = dec.U @ dec.U.T
        Pq = Q[:, :R] @ Q[:, :R].T
        np.testing.assert_allclose(P, Pq, atol=1e-10)


def test_decompose_orthonormal_and_eckart_young():
    wl = workloads.config2()
    fs = wl.bank.filters
    for R in (4, 8, 16, 32):
        dec = oracle.decompose(fs, R)
        np.testing.assert_allclose(dec.U.T @ dec.U, np.eye(R), atol=1e-12)
        P = dec.U @ dec.U.T
        resid = sum(np.sum((f.astype(np.float64) - f.astype(np.float64) @ P) ** 2) for f in fs)
        np.testing.assert_allclose(resid, np.sum(dec.sigma[R:] ** 2), rtol=1e-9, atol=1e-13)
        assert np.all(np.diff(dec.sigma) <= 1e-12)


def test_decompose_singular_values_of_unfolding():
    # the singular values of the stacked matrix, independently of the Gram route
    rng = np.random.default_rng(3)
    fs = [rng.standard_normal((h, w, 32)) for h, w in [(6, 6), (6, 11), (3, 4)]]
    dec = oracle.decompose(fs, 8)
    M = np.concatenate([f.reshape(-1, 32) for f in fs])
    sv = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(dec.sigma, sv, rtol=1e-10)


# ---------------------------------------------------------------- tensor form
def test_full_rank_tensor_form_reproduces_direct():
    wl = workloads.config1()
    X = wl.level_features(0, 1).astype(np.float64)
    dec = oracle.decompose(wl.bank.filters, 32)
    for f in wl.bank.filters:
        d = oracle.correlate(X, f)
        t = oracle.tensor_response(X, f, dec.U)
        np.testing.assert_allclose(t, d, rtol=0, atol=1e-10)


def test_tensor_form_closed_form_and_truncation_bound():
    wl = workloads.config1()
    X = wl.level_features(0, 1).astype(np.float64)
    for R in (2, 4, 8, 16):
        dec = oracle.decompose(wl.bank.filters, R)
        P = dec.U @ dec.U.T
        for f in wl.bank.filters[:3]:
            f64 = f.astype(np.float64)
            t = oracle.tensor_response(X, f, dec.U)
            np.testing.assert_allclose(t, oracle.correlate(X, f64 @ P), atol=1e-12)
            # |R_ten - R_dir| <= ||X window||_F ||f - f P||_F  (Cauchy-Schwarz)
            d = oracle.correlate(X, f)
            h, w, _ = f.shape
            wn = np.sqrt(oracle.correlate(X * X, np.ones((h, w, 32))))
            bound = wn * np.linalg.norm(f64 - f64 @ P)
            assert np.all(np.abs(t - d) <= bound + 1e-12)


# ---------------------------------------------------------------- distance transform
@pytest.mark.parametrize("seed", range(6))
def test_dt_separable_equals_2d_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    Hp, Wp = rng.integers(1, 7, size=2)
    if seed % 2 == 0:
        resp = rng.integers(-3, 4, size=(Hp, Wp)).astype(float)   # exact ties likely
        d = rng.integers(-1, 3, size=4).astype(float)
        d[1] = max(d[1], 1.0)
        d[3] = max(d[3], 1.0)
    else:
        resp = rng.standard_normal((Hp, Wp))
        d = np.array([rng.uniform(-0.5, 0.5), rng.uniform(0.01, 1), rng.uniform(-0.5, 0.5), rng.uniform(0.01, 1)])
    ty = np.arange(-1, Hp + 1)
    tx = np.arange(-2, Wp + 1)
    a = oracle.distance_transform(resp, d, ty, tx)
    b = oracle.distance_transform_2d_bruteforce(resp, d, ty, tx)
    np.testing.assert_array_equal(a.arg_y, b.arg_y)
    np.testing.assert_array_equal(a.arg_x, b.arg_x)
    np.testing.assert_allclose(a.D, b.D, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.margin, b.margin, rtol=0, atol=1e-12)


def test_dt_invariants():
    rng = np.random.default_rng(7)
    resp = rng.standard_normal((9, 13))
    d = np.array([0.05, 0.03, -0.02, 0.07])
    r = oracle.distance_transform(resp, d)
    # D >= resp (the target itself is a candidate with zero cost)
    assert np.all(r.D >= resp - 1e-15)
    # D equals the deformed score of its own argmax
    yy, xx = np.meshgrid(np.arange(9), np.arange(13), indexing="ij")
    dy, dx = r.arg_y - yy, r.arg_x - xx
    np.testing.assert_allclose(r.D, resp[r.arg_y, r.arg_x] - (d[0] * dx + d[1] * dx * dx + d[2] * dy + d[3] * dy * dy), atol=1e-14)
    # shift invariance: D(resp + c) = D(resp) + c, same argmax
    r2 = oracle.distance_transform(resp + 3.25, d)
    np.testing.assert_allclose(r2.D, r.D + 3.25, atol=1e-12)
    np.testing.assert_array_equal(r2.arg_y, r.arg_y)
    np.testing.assert_array_equal(r2.arg_x, r.arg_x)
    # 1-Lipschitz in the sup norm
    pert = resp + rng.uniform(-0.1, 0.1, resp.shape)
    r3 = oracle.distance_transform(pert, d)
    assert np.max(np.abs(r3.D - r.D)) <= np.max(np.abs(pert - resp)) + 1e-14
    # a huge quadratic cost pins every part to its anchor
    r4 = oracle.distance_transform(resp, [0, 1e9, 0, 1e9])
    np.testing.assert_array_equal(r4.D, resp)
    np.testing.assert_array_equal(r4.arg_y, yy)
    np.testing.assert_array_equal(r4.arg_x, xx)


def test_dt_targets_outside_give_neg_inf():
    resp = np.ones((3, 4))
    r = oracle.distance_transform(resp, [0, 1, 0, 1], np.array([-1, 0, 3]), np.array([0, 4]))
    assert np.isneginf(r.D[0]).all() and np.isneginf(r.D[2]).all() and np.isneginf(r.D[:, 1]).all()
    assert r.D[1, 0] == 1.0 and (r.arg_y[0] == -1).all()


# ---------------------------------------------------------------- assembly
def test_score_component_matches_bruteforce_assembly():
    rng = np.random.default_rng(11)
    root = rng.standard_normal((3, 4))
    parts = [rng.standard_normal((7, 9)) for _ in range(3)]
    anchors = np.array([[0, 0], [1, 2], [2, 1]])
    deform = rng.uniform(0.01, 0.5, size=(3, 4))
    sm = oracle.score_component(root, parts, anchors, deform)
    for y0 in range(3):
        for x0 in range(4):
            s = root[y0, x0]
            for i, pr in enumerate(parts):
                ty, tx = 2 * y0 + anchors[i, 0], 2 * x0 + anchors[i, 1]
                if not (0 <= ty < 7 and 0 <= tx < 9):
                    s = -np.inf
                    continue
                b = oracle.distance_transform_2d_bruteforce(pr, deform[i], [ty], [tx])
                s += b.D[0, 0]
                assert sm.offsets[i, y0, x0, 0] == b.arg_y[0, 0] - ty
                assert sm.offsets[i, y0, x0, 1] == b.arg_x[0, 0] - tx
            if np.isneginf(s):
                assert np.isneginf(sm.score[y0, x0])
            else:
                assert abs(sm.score[y0, x0] - s) < 1e-12


# ---------------------------------------------------------------- Section 4 accounting
def test_formula1_instance_from_section5():
    # rank 6, 8 parts of 8x8x32 and a 5x11x32 root: gain "beyond 7"
    direct = 8 * oracle.mults_direct(1, 1, 8, 8, 32) + oracle.mults_direct(1, 1, 5, 11, 32)
    cp = 8 * oracle.mults_cp(1, 1, 8, 8, 32, 6) + oracle.mults_cp(1, 1, 5, 11, 32, 6)
    assert direct / cp == pytest.approx(7.0, abs=1e-12)
    assert oracle.gain_formula1(8, 8, 32, 6) == pytest.approx(8 * 8 * 32 / (6 * 48))


def test_multiplication_counts_by_counting():
    # count the multiplications of the separable rank-R evaluation, one pass
    # per 1D factor over an N' x M' grid (borders ignored as in Section 4)
    Np, Mp, N, M, L, R = 5, 7, 3, 4, 6, 2
    count = 0
    for _r in range(R):
        count += Np * Mp * L      # feature-axis contraction with c_r
        count += Np * Mp * M      # x-direction 1D correlation with b_r
        count += Np * Mp * N      # y-direction 1D correlation with a_r
    assert count == oracle.mults_cp(Np, Mp, N, M, L, R)
    assert oracle.mults_direct(Np, Mp, N, M, L) == Np * Mp * N * M * L


def test_shared_basis_multiplication_count():
    """The shortened correlation of Section 4 over R projected channels: one
    multiplication per term of sum_{n,m,r} G[n,m,r] Z[y+n,x+m,r] at every
    output (counted by enumerating the terms), and at R = L it is exactly the
    direct count alpha."""
    import itertools
    Np, Mp, N, M, L, R = 3, 4, 2, 3, 5, 2
    terms = sum(1 for _ in itertools.product(range(Np), range(Mp), range(N), range(M), range(R)))
    assert terms == oracle.mults_shared_basis(Np, Mp, N, M, L, R)
    assert oracle.mults_shared_basis(Np, Mp, N, M, L, L) == oracle.mults_direct(Np, Mp, N, M, L)
    # the saving over direct is L / R, independent of the filter size
    assert oracle.mults_direct(7, 9, 6, 6, 32) / oracle.mults_shared_basis(7, 9, 6, 6, 32, 8) == 4.0


def test_detections_of_the_worked_example():
    """Algorithm 1's detection set on the hand-derived score map."""
    g = _load("worked_example.json")
    S = np.array(g["score"], float)
    assert oracle.detections([S], 5.0) == [(0, 0, 1, 10.0), (0, 0, 2, 5.0), (0, 1, 2, 5.0)]
    assert oracle.detections([S, S], 10.0) == [(0, 0, 1, 10.0), (1, 0, 1, 10.0)]
    assert oracle.detections([S], 10.5) == []
    assert oracle.detections([np.full((2, 2), -np.inf)], -1e30) == []


# ---------------------------------------------------------------- per-filter CP form
def _planted_cp(rng, N, M, L, R):
    return rng.standard_normal((N, R)), rng.standard_normal((M, R)), rng.standard_normal((L, R))


@pytest.mark.parametrize("R", [1, 2, 3])
def test_cp_als_recovers_planted_rank(R):
    """An exact rank-R tensor is fitted to rounding by rank-R ALS."""
    rng = np.random.default_rng(40 + R)
    A, B, C = _planted_cp(rng, 6, 6, 32, R)
    f = oracle.cp_reconstruct(A, B, C)
    cp = oracle.cp_als(f, R, iters=2000)
    rel = np.linalg.norm(f - oracle.cp_reconstruct(cp.A, cp.B, cp.C)) / np.linalg.norm(f)
    assert rel < 1e-8, rel


def test_cp_als_error_never_increases():
    """Every ALS micro-step is an exact least-squares minimisation, so the
    error after each cycle is non-increasing; more terms never fit worse."""
    rng = np.random.default_rng(5)
    f = rng.standard_normal((6, 6, 32))
    errs = {}
    for R in (1, 3, 6):
        cp = oracle.cp_als(f, R, iters=60)
        e = np.array(cp.errors)
        assert np.all(np.diff(e) <= 1e-12 * e[:-1] + 1e-14), R
        errs[R] = e[-1]
    assert errs[1] >= errs[3] >= errs[6]
    # terms beyond a mode's size (6 rows, 6 cols) still lower the error
    e8 = oracle.cp_als(f, 8, iters=60).errors[-1]
    assert e8 < errs[6] * 0.98, (e8, errs[6])
    # rank 1 with a planted rank-1 tensor is exact
    a, b, c = rng.standard_normal(6), rng.standard_normal(11), rng.standard_normal(32)
    f1 = np.einsum("n,m,l->nml", a, b, c)
    cp1 = oracle.cp_als(f1, 1)
    assert np.allclose(oracle.cp_reconstruct(cp1.A, cp1.B, cp1.C), f1, atol=1e-12)


def test_cp_response_is_correlation_with_reconstruction():
    """Closed form: the separable sum of 1-D correlations equals the direct
    correlation with the reconstructed filter (Section 4's identity)."""
    rng = np.random.default_rng(9)
    A, B, C = _planted_cp(rng, 5, 7, 32, 4)
    X = rng.uniform(0, 0.4, size=(19, 23, 32))
    got = oracle.cp_response(X, A, B, C)
    want = oracle.correlate(X, oracle.cp_reconstruct(A, B, C))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_cp_response_bruteforce_tiny():
    """The order of the 1-D passes by direct summation on a tiny input."""
    rng = np.random.default_rng(10)
    A, B, C = _planted_cp(rng, 2, 3, 32, 2)
    X = rng.standard_normal((4, 5, 32))
    got = oracle.cp_response(X, A, B, C)
    want = np.zeros((3, 3))
    for y in range(3):
        for x in range(3):
            for r in range(2):
                for n in range(2):
                    for m in range(3):
                        want[y, x] += A[n, r] * B[m, r] * float(np.dot(X[y + n, x + m], C[:, r]))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


# ------------------------------------------------------------ rank selection
def test_rank_bound_closed_form():
    # Section 4's bound e (r (N+M+L) / (N M L))^2 at e = 2, r = 6, N = M = 6,
    # L = 32: 2 (264 / 1152)^2 = 0.10503472222..., a literal worked by hand
    assert oracle.rank_bound(2.0, 6, 6, 6, 32) == pytest.approx(0.1050347222222222, rel=1e-14)
    # r = 1, N = M = 1, L = 2 -> e (4 / 2)^2 = 4 e
    assert oracle.rank_bound(0.5, 1, 1, 1, 2) == pytest.approx(2.0, rel=1e-15)
    # formula (1) of Section 4 is the inverse ratio without the square
    assert oracle.gain_formula1(6, 6, 32, 6) == pytest.approx(1152 / 264, rel=1e-15)


def _odeco(weights, N=6, M=6, L=32):
    """sum_j w_j e_j (x) e_j (x) e_j: orthogonal rank-1 terms, so the best
    rank-r approximation keeps the r largest and its error is the norm of the
    rest (no ALS subtlety)."""
    f = np.zeros((N, M, L))
    for j, w in enumerate(weights):
        f[j, j, j] = w
    return f


def test_select_rank_uses_the_squared_bound():
    """A filter where Section 4's squared bound and an unsquared one pick
    different ranks.  Weights (1, 1/2, 1/4, 1/8, 1/16, 1/32) on orthogonal
    terms of a 6x6x32 filter: errors after r terms are sqrt of the tail sums,
    0.5771, 0.2881, 0.1432 (r = 1..3).  With e = 100 the squared bound is
    100 (44 r / 1152)^2 = 0.1459 r^2: 0.146 (r = 1) < 0.577, 0.584 (r = 2) >
    0.288, so rank 2; the unsquared 100 (44 r / 1152) = 3.82 r accepts r = 1."""
    f = _odeco([1, 1 / 2, 1 / 4, 1 / 8, 1 / 16, 1 / 32])
    tail = [np.sqrt(sum(w * w for w in [1 / 2, 1 / 4, 1 / 8, 1 / 16, 1 / 32][r - 1:])) for r in (1, 2)]
    assert tail[0] == pytest.approx(0.5771, abs=1e-4) and tail[1] == pytest.approx(0.2881, abs=1e-4)
    r, errs = oracle.select_rank(f, 100.0, 6, iters=300)
    assert r == 2, (r, errs)
    # the binary search tried r = 3, 2, 1; their fits are the exact truncations
    assert errs[0] == pytest.approx(tail[0], rel=1e-9) and errs[1] == pytest.approx(tail[1], rel=1e-9)


def test_select_rank_finds_planted_rank():
    """A planted rank-3 filter: every fit below rank 3 leaves a large error,
    rank 3 fits to rounding, so the criterion picks exactly 3."""
    rng = np.random.default_rng(21)
    A, B, C = rng.standard_normal((6, 3)), rng.standard_normal((6, 3)), rng.standard_normal((32, 3))
    f = oracle.cp_reconstruct(A, B, C)
    f /= np.linalg.norm(f)
    r, errs = oracle.select_rank(f, 1.0, 16, iters=2000)
    assert r == 3, (r, errs)


def test_select_rank_extremes_and_linear_scan():
    """A huge e accepts rank 1, e = 0 accepts nothing (r_max); in between the
    binary search returns the same rank as a scan of every r (the error falls
    and the bound grows with r)."""
    wl = workloads.config1()
    f = wl.bank.filters[1].astype(np.float64)
    assert oracle.select_rank(f, 1e9, 12)[0] == 1
    assert oracle.select_rank(f, 0.0, 12)[0] == 12
    N, M, L = f.shape
    errs = [oracle.cp_als(f, r, iters=200, eps=1e-13).errors[-1] for r in range(1, 13)]
    for e in (5.0, 20.0, 80.0):
        scan = next((r for r in range(1, 13) if errs[r - 1] < oracle.rank_bound(e, r, N, M, L)), 12)
        assert oracle.select_rank(f, e, 12)[0] == scan, e


# ------------------------------------------------------- convolution shortening
def test_cp_terms_are_rank_one_correlations():
    """Each term equals the direct correlation with its rank-1 filter
    a_r (x) b_r (x) c_r, and the terms sum to the CP response."""
    rng = np.random.default_rng(31)
    A, B, C = rng.standard_normal((4, 3)), rng.standard_normal((5, 3)), rng.standard_normal((32, 3))
    X = rng.uniform(0, 0.4, size=(11, 13, 32))
    T = oracle.cp_terms(X, A, B, C)
    assert T.shape == (3, 8, 9)
    for r in range(3):
        f = np.einsum("n,m,l->nml", A[:, r], B[:, r], C[:, r])
        np.testing.assert_allclose(T[r], oracle.correlate(X, f), rtol=0, atol=1e-12)
    np.testing.assert_allclose(T.sum(0), oracle.cp_response(X, A, B, C), rtol=0, atol=1e-12)


def test_pruning_hand_example():
    """One hypothesis, a root of two terms with responses 1 and 2 (partial
    sums 1, 3) and no parts: strict comparison p_r < t_r."""
    terms = np.array([[[1.0]], [[2.0]]])
    score = np.array([[7.0]])
    cases = [([0.0, 4.0], True), ([2.0, 0.0], True), ([1.0, 3.0], False), ([-np.inf, -np.inf], False)]
    for t, want in cases:
        out, pruned, margin = oracle.prune_component(score, terms, [], np.zeros((0, 2)), np.array(t), [])
        assert bool(pruned[0, 0]) == want, t
        assert out[0, 0] == (-np.inf if want else 7.0)
    _, _, margin = oracle.prune_component(score, terms, [], np.zeros((0, 2)), np.array([0.5, 2.0]), [])
    assert margin[0, 0] == pytest.approx(0.5)


def test_pruning_keeps_positives_and_is_monotone():
    """Thresholds fitted on a set of positives never reject one of them
    (Section 4: the tightest such thresholds); raising every threshold only
    rejects more; -inf rejects nothing and +inf everything; a part is tested
    at its anchor only while the anchor is inside its map."""
    wl = workloads.config1()
    c = wl.bank.components[0]
    rng = np.random.default_rng(5)
    Xr, Xp = wl.level_features(0, 1).astype(np.float64), wl.level_features(0, 0).astype(np.float64)
    fac = {}
    for k in [c.root] + list(c.parts):
        cp = oracle.cp_als(wl.bank.filters[k].astype(np.float64), 4, iters=30)
        fac[k] = (cp.A, cp.B, cp.C)
    rt = oracle.cp_terms(Xr, *fac[c.root])
    pt = [oracle.cp_terms(Xp, *fac[k]) for k in c.parts]
    Ho, Wo = rt.shape[1:]
    score = rng.standard_normal((Ho, Wo))
    pos = [(int(rng.integers(0, Ho)), int(rng.integers(0, Wo))) for _ in range(12)]
    t_root = oracle.fit_thresholds([oracle.partial_sums(rt, y, x) for y, x in pos])
    t_parts = []
    for i, terms in enumerate(pt):
        ps = []
        for y, x in pos:
            ay, ax = 2 * y + c.anchors[i][0], 2 * x + c.anchors[i][1]
            if 0 <= ay < terms.shape[1] and 0 <= ax < terms.shape[2]:
                ps.append(oracle.partial_sums(terms, ay, ax))
        t_parts.append(oracle.fit_thresholds(ps) if ps else np.full(4, -np.inf))
    out, pruned, _ = oracle.prune_component(score, rt, pt, c.anchors, t_root, t_parts)
    for y, x in pos:
        assert not pruned[y, x]
    assert pruned.any() and not pruned.all()
    _, pruned_hi, _ = oracle.prune_component(score, rt, pt, c.anchors, t_root + 0.05,
                                            [t + 0.05 for t in t_parts])
    assert np.all(pruned_hi >= pruned) and pruned_hi.sum() > pruned.sum()
    _, none, _ = oracle.prune_component(score, rt, pt, c.anchors, np.full(4, -np.inf),
                                       [np.full(4, -np.inf)] * len(pt))
    assert not none.any()
    _, every, _ = oracle.prune_component(score, rt, pt, c.anchors, np.full(4, np.inf),
                                        [np.full(4, -np.inf)] * len(pt))
    assert every.all()
