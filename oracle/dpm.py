"""Plain FP64 CPU oracle of the DPM score-estimation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this module; only the tests, the smoke check and the benchmark's CPU
baseline leg call it.  It shares no code with the GPU path (the only common
import is the seeded input generator in ``workloads``, which holds none of the
method's arithmetic).

Every function works in float64 on numpy arrays, written for readability, not
speed.  Conventions (each one is a reading of the paper, see the notes):

* Feature level X: (H, W, 32), channel innermost.  Filter f: (h, w, 32).
* Correlation, not convolution (Section 4, the operator written as a small
  circle is a correlation), over valid placements only:
  resp(y, x) = sum_{n<h, m<w, l<32} f[n, m, l] * X[y+n, x+m, l],
  0 <= y <= H-h, 0 <= x <= W-w.
* Deformation feature psi = (dx, dx^2, dy, dy^2) with dx = x' - x_anchor,
  dy = y' - y_anchor; the cost d . psi is subtracted (Section 2, the score
  formula and the placement argmax).  Coefficient order d = (d_x, d_xx, d_y, d_yy).
* The part placement maximises over the whole part map, every position
  of it a candidate (Section 2, the placement argmax).  Exact ties go to the
  lexicographically smallest (y', x').
* Score (Section 2): s(p0) = resp_root(p0) + sum_i D_i(2*p0 + v_i); the parts
  live one octave below the root (twice the resolution), v_i is the anchor of
  part i.  No bias term.  An anchor outside the part map gives -inf.
* Tensor form: one feature-mode basis U_R (32 x R) shared by the whole bank,
  taken from the leading eigenvectors of the Gram matrix of the mode-3
  unfolding (the Frobenius-optimal truncation of Section 4's criterion applied
  to the feature mode); per-filter factors G_k = f_k x_3 U_R^T; projected
  features Z = X x_3 U_R^T; response = correlation of Z with G_k over R
  channels (Section 4, feature contraction first, then the spatial sums).

Parity status of each function is pinned by tests/test_oracle_pins.py.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

NEG_INF = -np.inf


# --------------------------------------------------------------------------
# O1: direct correlation  (Section 4, multiplication count alpha = N'M'NML)
# --------------------------------------------------------------------------
def correlate(X: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Valid-placement correlation of one level with one filter, float64.

    Sums taps in (n, m) order; the inner channel contraction is a library
    matrix-vector product.  Returns (H-h+1, W-w+1), or an empty array when the
    filter does not fit.
    """
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    H, W, C = X.shape
    h, w, C2 = f.shape
    assert C == C2
    Ho, Wo = H - h + 1, W - w + 1
    if Ho <= 0 or Wo <= 0:
        return np.zeros((max(Ho, 0), max(Wo, 0)))
    out = np.zeros((Ho, Wo))
    for n in range(h):
        for m in range(w):
            out += X[n:n + Ho, m:m + Wo, :] @ f[n, m, :]
    return out


# --------------------------------------------------------------------------
# O2: shared feature-mode basis (Section 4, Frobenius criterion)
# --------------------------------------------------------------------------
@dataclass
class Decomposition:
    sigma: np.ndarray       # (32,) singular values of the mode-3 unfolding, descending
    U: np.ndarray           # (32, R) leading feature-mode basis vectors
    rank: int

    @property
    def gap(self) -> float:
        """(sigma_R - sigma_{R+1}) / sigma_1; zero gap means U_R is not unique."""
        s = self.sigma
        nxt = s[self.rank] if self.rank < len(s) else 0.0
        return float((s[self.rank - 1] - nxt) / s[0])


def unfold_mode3(filters: Sequence[np.ndarray]) -> np.ndarray:
    """Rows = every cell vector f_k[n, m, :] of every filter (mode-3 unfolding, transposed)."""
    return np.concatenate([np.asarray(f, np.float64).reshape(-1, f.shape[2]) for f in filters], axis=0)


def decompose(filters: Sequence[np.ndarray], rank: int) -> Decomposition:
    """Leading ``rank`` eigenvectors of C = M^T M, M the mode-3 unfolding.

    The eigen-solve is the library symmetric eigensolver; eigenvalues are
    sorted in descending order and clipped at zero; sigma = sqrt(lambda).
    Sign convention: the largest-magnitude entry of each column is positive.
    """
    M = unfold_mode3(filters)
    C = M.T @ M
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam = np.clip(lam[order], 0.0, None)
    V = V[:, order]
    for j in range(V.shape[1]):
        i = np.argmax(np.abs(V[:, j]))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return Decomposition(np.sqrt(lam), V[:, :rank].copy(), rank)


def factor(f: np.ndarray, U: np.ndarray) -> np.ndarray:
    """G = f x_3 U^T: per-cell projection of the filter onto the basis, (h, w, R)."""
    return np.asarray(f, np.float64) @ U


def project(X: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Z = X x_3 U^T: per-cell projection of a feature level, (H, W, R)."""
    return np.asarray(X, np.float64) @ U


def tensor_response(X: np.ndarray, f: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Shortened correlation: feature contraction first (projection), then the
    spatial correlation over R channels with the factor G = f x_3 U^T."""
    return correlate(project(X, U), factor(f, U))


# --------------------------------------------------------------------------
# O4: generalized distance transform, brute force, separable
#     (Section 2, placement argmax over all part positions)
# --------------------------------------------------------------------------
@dataclass
class DTResult:
    D: np.ndarray        # best value  resp(y', x') - cost(y'-y, x'-x)
    arg_y: np.ndarray    # argmax y'  (-1 where the target is outside the map)
    arg_x: np.ndarray    # argmax x'
    margin: np.ndarray   # best minus the best value over positions != argmax


def _row_pass(resp: np.ndarray, d: np.ndarray, tx: np.ndarray):
    """For every row y' and target column x_t: max over x' of
    resp[y', x'] - (d_x (x'-x_t) + d_xx (x'-x_t)^2); first argmax; runner-up."""
    Hp, Wp = resp.shape
    dx = np.arange(Wp)[None, :] - tx[:, None]                    # (nT, Wp)
    cost = d[0] * dx + d[1] * dx * dx                            # (nT, Wp)
    V = resp[:, None, :] - cost[None, :, :]                       # (Hp, nT, Wp)
    arg = np.argmax(V, axis=2)                                   # first maximum
    best = np.take_along_axis(V, arg[..., None], axis=2)[..., 0]
    V2 = V.copy()
    np.put_along_axis(V2, arg[..., None], NEG_INF, axis=2)
    second = V2.max(axis=2) if Wp > 1 else np.full(best.shape, NEG_INF)
    return best, arg, second


def distance_transform(resp: np.ndarray, d: Sequence[float],
                       ty: Optional[np.ndarray] = None,
                       tx: Optional[np.ndarray] = None) -> DTResult:
    """D(y_t, x_t) = max_{y', x'} resp[y', x'] - d . (dx, dx^2, dy, dy^2),
    dx = x' - x_t, dy = y' - y_t, for targets on the grid ty x tx (default:
    every cell).  Row pass over x', then column pass over y', both brute force
    (quadratic per line).  Ties: smallest x' within a row, then smallest y'.
    Targets outside [0, Hp) x [0, Wp) give -inf with arg -1.
    """
    resp = np.asarray(resp, np.float64)
    d = np.asarray(d, np.float64)
    Hp, Wp = resp.shape
    ty = np.arange(Hp) if ty is None else np.asarray(ty, np.int64)
    tx = np.arange(Wp) if tx is None else np.asarray(tx, np.int64)
    nY, nX = len(ty), len(tx)
    D = np.full((nY, nX), NEG_INF)
    AY = np.full((nY, nX), -1, dtype=np.int64)
    AX = np.full((nY, nX), -1, dtype=np.int64)
    MG = np.full((nY, nX), np.inf)
    if Hp <= 0 or Wp <= 0 or nY == 0 or nX == 0:
        return DTResult(D, AY, AX, MG)
    okx = (tx >= 0) & (tx < Wp)
    oky = (ty >= 0) & (ty < Hp)
    if not okx.any() or not oky.any():
        return DTResult(D, AY, AX, MG)
    txv, tyv = tx[okx], ty[oky]
    rbest, rarg, rsecond = _row_pass(resp, d, txv)               # (Hp, nTx)
    dy = np.arange(Hp)[None, :] - tyv[:, None]                    # (nTy, Hp)
    cy = d[2] * dy + d[3] * dy * dy
    Vc = rbest.T[None, :, :] - cy[:, None, :]                     # (nTy, nTx, Hp)
    ay = np.argmax(Vc, axis=2)
    best = np.take_along_axis(Vc, ay[..., None], axis=2)[..., 0]
    Vc2 = Vc.copy()
    np.put_along_axis(Vc2, ay[..., None], NEG_INF, axis=2)
    other_rows = Vc2.max(axis=2) if Hp > 1 else np.full(best.shape, NEG_INF)
    # runner-up inside the winning row, with that row's vertical cost
    rs = rsecond.T[np.arange(len(txv))[None, :], ay]              # (nTy, nTx)
    cy_win = cy[np.arange(len(tyv))[:, None], ay]
    second = np.maximum(other_rows, rs - cy_win)
    ax = rarg.T[np.arange(len(txv))[None, :], ay]
    iy = np.nonzero(oky)[0]
    ix = np.nonzero(okx)[0]
    D[np.ix_(iy, ix)] = best
    AY[np.ix_(iy, ix)] = ay
    AX[np.ix_(iy, ix)] = ax
    MG[np.ix_(iy, ix)] = best - second
    return DTResult(D, AY, AX, MG)


def distance_transform_2d_bruteforce(resp: np.ndarray, d: Sequence[float],
                                     ty: Optional[np.ndarray] = None,
                                     tx: Optional[np.ndarray] = None) -> DTResult:
    """Same as ``distance_transform`` but by a direct search over all (y', x')
    for every target: pure Python loops, for tiny maps only."""
    resp = np.asarray(resp, np.float64)
    Hp, Wp = resp.shape
    ty = list(range(Hp)) if ty is None else list(ty)
    tx = list(range(Wp)) if tx is None else list(tx)
    D = np.full((len(ty), len(tx)), NEG_INF)
    AY = np.full((len(ty), len(tx)), -1, dtype=np.int64)
    AX = np.full((len(ty), len(tx)), -1, dtype=np.int64)
    MG = np.full((len(ty), len(tx)), np.inf)
    for a, yt in enumerate(ty):
        for b, xt in enumerate(tx):
            if not (0 <= yt < Hp and 0 <= xt < Wp):
                continue
            vals = []
            for yp in range(Hp):
                for xp in range(Wp):
                    ddx, ddy = xp - xt, yp - yt
                    c = d[0] * ddx + d[1] * ddx * ddx + d[2] * ddy + d[3] * ddy * ddy
                    vals.append((resp[yp, xp] - c, yp, xp))
            best = max(v[0] for v in vals)
            first = min((v for v in vals if v[0] == best), key=lambda v: (v[1], v[2]))
            rest = [v[0] for v in vals if (v[1], v[2]) != (first[1], first[2])]
            D[a, b] = best
            AY[a, b], AX[a, b] = first[1], first[2]
            MG[a, b] = best - (max(rest) if rest else NEG_INF)
    return DTResult(D, AY, AX, MG)


# --------------------------------------------------------------------------
# O5: star-model score (Section 2 score formula)
# --------------------------------------------------------------------------
@dataclass
class ScoreMap:
    score: np.ndarray          # (Ho, Wo) root-position scores, -inf where an anchor is outside
    offsets: np.ndarray        # (n_parts, Ho, Wo, 2) int (dy, dx) = placement - anchor
    margin: np.ndarray         # (n_parts, Ho, Wo) DT margin at the anchor
    root: np.ndarray           # (Ho, Wo) root response
    D: np.ndarray              # (n_parts, Ho, Wo) deformed part scores at the anchors


def score_component(root_resp: np.ndarray, part_resps: Sequence[np.ndarray],
                    anchors: np.ndarray, deform: np.ndarray) -> ScoreMap:
    """s(y0, x0) = root(y0, x0) + sum_i D_i(2 y0 + v_iy, 2 x0 + v_ix)."""
    Ho, Wo = root_resp.shape
    n = len(part_resps)
    score = np.array(root_resp, dtype=np.float64, copy=True)
    offs = np.zeros((n, Ho, Wo, 2), dtype=np.int64)
    marg = np.full((n, Ho, Wo), np.inf)
    Dall = np.full((n, Ho, Wo), NEG_INF)
    for i, resp in enumerate(part_resps):
        vy, vx = int(anchors[i][0]), int(anchors[i][1])
        ty = 2 * np.arange(Ho) + vy
        tx = 2 * np.arange(Wo) + vx
        r = distance_transform(resp, deform[i], ty, tx)
        score = score + r.D
        inside = r.arg_y >= 0
        offs[i, :, :, 0] = np.where(inside, r.arg_y - ty[:, None], 0)
        offs[i, :, :, 1] = np.where(inside, r.arg_x - tx[None, :], 0)
        marg[i] = r.margin
        Dall[i] = r.D
    return ScoreMap(score, offs, marg, np.asarray(root_resp, np.float64), Dall)


def score_pyramid(levels, filters: Sequence[np.ndarray], components, octave: int,
                  U: Optional[np.ndarray] = None, root_levels: Optional[Sequence[int]] = None,
                  comps: Optional[Sequence[int]] = None,
                  response: Optional[Callable[[np.ndarray, int], np.ndarray]] = None
                  ) -> Dict[Tuple[int, int], ScoreMap]:
    """Score maps of one image's pyramid: every component c at every root
    level l >= octave, with its root filter correlated on level l and its part
    filters on level l - octave (twice the resolution: the anchor of root
    position p0 is 2 p0 + v_i).

    ``levels``: anything indexable by level number with a length, each item an
    (H, W, 32) feature level (a list, or a lazy mapping).  ``components``:
    objects with ``root``, ``parts``, ``anchors``, ``deform``.  With ``U``
    given, every response is the shortened (tensor-form) correlation;
    otherwise direct.  ``response(X, k)``, when given, replaces both: the
    response map of filter k on level X (e.g. a CP form's decomposed
    correlation).  ``root_levels`` / ``comps`` restrict the output to a subset
    (default: all).  Returns {(root level, component index): ScoreMap}.
    """
    if response is not None:
        resp_of = lambda X, k: response(X, k)
    elif U is None:
        resp_of = lambda X, k: correlate(X, filters[k])
    else:
        resp_of = lambda X, k: tensor_response(X, filters[k], U)
    L = len(levels)
    lv_ids = range(octave, L) if root_levels is None else root_levels
    c_ids = range(len(components)) if comps is None else comps
    out: Dict[Tuple[int, int], ScoreMap] = {}
    for l in lv_ids:
        if not octave <= l < L:
            raise ValueError(f"root level {l} outside [{octave}, {L})")
        Xr, Xp = levels[l], levels[l - octave]
        for ci in c_ids:
            c = components[ci]
            rr = resp_of(Xr, c.root)
            prs = [resp_of(Xp, k) for k in c.parts]
            out[(l, ci)] = score_component(rr, prs, c.anchors, c.deform)
    return out


# --------------------------------------------------------------------------
# Section 4 accounting: multiplication counts and formula (1)
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# Per-filter CP form (Section 4): f ~ sum_r a_r (x) b_r (x) c_r, fitted by
# alternating least squares, and the decomposed correlation
# I o T = sum_r ((I o c_r) o b_r) o a_r  (feature contraction first, then the
# 1-D correlations along x with b_r and along y with a_r).
# --------------------------------------------------------------------------
@dataclass
class CPForm:
    A: np.ndarray            # (N, R) filter-row factors a_r
    B: np.ndarray            # (M, R) filter-column factors b_r
    C: np.ndarray            # (L, R) channel factors c_r
    errors: List[float]      # Frobenius error after each ALS cycle


def cp_reconstruct(A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """sum_r a_r (x) b_r (x) c_r as an (N, M, L) array."""
    return np.einsum("nr,mr,lr->nml", A, B, C)


def _leading_vectors(X: np.ndarray, R: int) -> np.ndarray:
    """R leading left singular vectors of X.  Columns beyond X's row count get
    fixed pseudo-random values: the paper does not say how ALS starts, and a
    zero column would stay zero under every update (its Gram rows vanish)."""
    U, _, _ = np.linalg.svd(X, full_matrices=True)
    n = X.shape[0]
    out = np.zeros((n, R))
    k = min(R, U.shape[1])
    out[:, :k] = U[:, :k]
    if R > k:
        out[:, k:] = np.random.default_rng([n, R]).uniform(-1.0, 1.0, size=(n, R - k))
    return out


def cp_als(f: np.ndarray, R: int, iters: int = 500, eps: float = 1e-13) -> CPForm:
    """Rank-R CP of an order-3 tensor by alternating least squares.

    One cycle solves, in turn, A = argmin ||f - CP(A, B, C)||_F, then B, then
    C, each an ordinary least-squares problem on the matching unfolding of f
    with a Khatri-Rao design matrix (numpy.linalg.lstsq).  Starts from the
    leading singular vectors of the three unfoldings.  Stops after `iters`
    cycles, when the error falls below eps * ||f||_F, or when a cycle no longer
    lowers it (relative change below 1e-12).
    """
    f = np.asarray(f, np.float64)
    N, M, L = f.shape
    X1 = f.reshape(N, M * L)                         # [n, m*L + l]
    X2 = f.transpose(1, 0, 2).reshape(M, N * L)      # [m, n*L + l]
    X3 = f.transpose(2, 0, 1).reshape(L, N * M)      # [l, n*M + m]
    A = _leading_vectors(X1, R)
    B = _leading_vectors(X2, R)
    C = _leading_vectors(X3, R)
    nf = np.linalg.norm(f)
    errors: List[float] = []

    def kr(P, Q):                                    # rows (p, q) -> P[p] * Q[q]
        return np.einsum("pr,qr->pqr", P, Q).reshape(P.shape[0] * Q.shape[0], -1)

    for _ in range(iters):
        A = np.linalg.lstsq(kr(B, C), X1.T, rcond=None)[0].T
        B = np.linalg.lstsq(kr(A, C), X2.T, rcond=None)[0].T
        C = np.linalg.lstsq(kr(A, B), X3.T, rcond=None)[0].T
        err = float(np.linalg.norm(f - cp_reconstruct(A, B, C)))
        errors.append(err)
        if err <= eps * nf:
            break
        if len(errors) > 1 and errors[-2] - err <= 1e-12 * max(errors[-2], 1e-300):
            break
    return CPForm(A, B, C, errors)


def cp_response(X: np.ndarray, A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Decomposed correlation of one level with a CP filter: per rank term,
    P = X o c_r (channel contraction), Q = P o b_r along x, S = Q o a_r along
    y; the terms are summed.  Valid placements only, as in correlate()."""
    X = np.asarray(X, np.float64)
    H, W, _ = X.shape
    N, R = A.shape
    M = B.shape[0]
    Ho, Wo = H - N + 1, W - M + 1
    if Ho <= 0 or Wo <= 0:
        return np.zeros((max(Ho, 0), max(Wo, 0)))
    out = np.zeros((Ho, Wo))
    for r in range(R):
        P = X @ C[:, r]                              # (H, W)
        Q = np.zeros((H, Wo))
        for m in range(M):
            Q += B[m, r] * P[:, m:m + Wo]
        S = np.zeros((Ho, Wo))
        for n in range(N):
            S += A[n, r] * Q[n:n + Ho, :]
        out += S
    return out


def cp_terms(X: np.ndarray, A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Response of each rank-1 term of a CP filter on its own, shape
    (R, Ho, Wo): term r is ((X o c_r) o_x b_r) o_y a_r; their sum over r is
    cp_response."""
    R = A.shape[1]
    return np.stack([cp_response(X, A[:, r:r + 1], B[:, r:r + 1], C[:, r:r + 1]) for r in range(R)])


# --------------------------------------------------------------------------
# Convolution shortening (Section 4 thresholds, Algorithm 1 early exit).
# A hypothesis is a root position p0 of one component on one root level.  For
# each of its filters (root at p0, part i at its anchor 2 p0 + v_i on the part
# level) the partial response after r terms is compared with t_r of that
# filter; falling below any of them rejects the hypothesis (score -inf).
# --------------------------------------------------------------------------
def partial_sums(terms: np.ndarray, y: int, x: int) -> np.ndarray:
    """p_r = sum of the first r terms' responses at (y, x), r = 1..R."""
    return np.cumsum(terms[:, y, x])


def fit_thresholds(partials: Sequence[np.ndarray]) -> np.ndarray:
    """t_r = min over the positives' partial sums p_r (Section 4: the tightest
    thresholds that reject no positive).  partials: one (R,) array per positive."""
    return np.min(np.stack(partials), axis=0)


def prune_component(score: np.ndarray, root_terms: np.ndarray, part_terms: Sequence[np.ndarray],
                    anchors: np.ndarray, t_root: np.ndarray, t_parts: Sequence[np.ndarray]):
    """Apply Algorithm 1's early exit to one score map.

    Returns (pruned score map, pruned mask, margin): margin[y0, x0] is the
    smallest |p_r - t_r| over every test the hypothesis went through (inf when
    none), so that callers comparing against another arithmetic can skip
    near-ties.  A part whose anchor is outside its map is not tested (the
    score is -inf already)."""
    Ho, Wo = score.shape
    pruned = np.zeros((Ho, Wo), bool)
    margin = np.full((Ho, Wo), np.inf)
    for y0 in range(Ho):
        for x0 in range(Wo):
            tests = [(root_terms, y0, x0, t_root)]
            for i, terms in enumerate(part_terms):
                ay, ax = 2 * y0 + int(anchors[i][0]), 2 * x0 + int(anchors[i][1])
                if 0 <= ay < terms.shape[1] and 0 <= ax < terms.shape[2]:
                    tests.append((terms, ay, ax, t_parts[i]))
            for terms, y, x, t in tests:
                p = partial_sums(terms, y, x)
                margin[y0, x0] = min(margin[y0, x0], float(np.min(np.abs(p - t))))
                if np.any(p < t):
                    pruned[y0, x0] = True
    out = np.where(pruned, -np.inf, score)
    return out, pruned, margin


def rank_bound(e: float, r: int, N: int, M: int, L: int) -> float:
    """Right-hand side of the rank criterion of Section 4:
    e * (r (N + M + L) / (N M L))^2."""
    return e * (r * (N + M + L) / (N * M * L)) ** 2


def select_rank(f: np.ndarray, e: float, r_max: int, iters: int = 200) -> Tuple[int, List[float]]:
    """Smallest r in [1, r_max] with ||f - CP(f, r)||_F < rank_bound(e, r, ...)
    (Section 4), by binary search over r (the error falls and the bound grows
    with r, so the predicate switches from false to true once); r_max when no
    r satisfies it.  Returns (r, Frobenius errors of the fits tried, by r)."""
    f = np.asarray(f, np.float64)
    N, M, L = f.shape
    tried = {}

    def ok(r):
        if r not in tried:
            cp = cp_als(f, r, iters=iters, eps=1e-13)
            tried[r] = cp.errors[-1]
        return tried[r] < rank_bound(e, r, N, M, L)

    lo, hi = 1, r_max
    while lo < hi:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid + 1
    return lo, [tried[r] for r in sorted(tried)]


# --------------------------------------------------------------------------
# Detection set (Algorithm 1: a hypothesis joins D when its score reaches tau)
# --------------------------------------------------------------------------
def detections(score_maps: Sequence[np.ndarray], tau: float) -> List[Tuple[int, int, int, float]]:
    """Every (map, y, x, score) with score >= tau, maps in the given order,
    positions row by row."""
    out = []
    for k, S in enumerate(score_maps):
        S = np.asarray(S)
        for y in range(S.shape[0]):
            for x in range(S.shape[1]):
                if S[y, x] >= tau:
                    out.append((k, y, x, float(S[y, x])))
    return out


def mults_direct(Np: int, Mp: int, N: int, M: int, L: int) -> int:
    """alpha = N' M' N M L multiplications for one filter on one image."""
    return Np * Mp * N * M * L


def mults_cp(Np: int, Mp: int, N: int, M: int, L: int, R: int) -> int:
    """R N' M' (L + M + N) multiplications for the rank-R separable form."""
    return R * Np * Mp * (L + M + N)


def gain_formula1(N: int, M: int, L: int, R: int) -> float:
    """Formula (1): N M L / (R (N + M + L)), speed and memory gain of rank R."""
    return N * M * L / (R * (N + M + L))


def mults_shared_basis(Np: int, Mp: int, N: int, M: int, L: int, R: int) -> int:
    """Shortened correlation over R projected channels: N' M' N M R per filter
    (the projection, N' M' L R per level, is shared by the whole bank)."""
    return Np * Mp * N * M * R
