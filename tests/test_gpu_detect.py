"""GPU tests of the detection set (Algorithm 1: keep every hypothesis whose
score reaches tau): the compaction is integer work, so the GPU list must equal
the thresholding of the GPU's own scores exactly, in (map, row, column) order;
against the FP64 oracle's scores it must agree wherever the score is farther
from tau than the mode's tolerance."""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_common import TOL, note, oracle_basis, oracle_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scored(wl, mode, rank):
    from paper_1707_03268_amd import Context
    ctx = Context(0)
    ctx.load_filters(wl.bank.filters, wl.bank.components)
    U = None
    if rank is not None:
        ctx.decompose(rank)
        U = oracle_basis(wl.bank.filters, rank)
    lay = ctx.plan(wl.pyramids)
    feats = torch.from_numpy(wl.features()).cuda()
    scores = torch.empty(max(lay.n_score, 1), dtype=torch.float32, device="cuda")
    offs = torch.empty(max(lay.n_offsets, 1), dtype=torch.int16, device="cuda")
    ctx.score_pyramid(mode, feats, scores, offs)
    torch.cuda.synchronize()
    return ctx, lay, scores, U


def _maps(lay, s):
    return [s[lay.map_score_off[k]:lay.map_score_off[k] + lay.map_rows[k] * lay.map_cols[k]]
            .reshape(lay.map_rows[k], lay.map_cols[k]) for k in range(lay.n_maps)]


def _host_list(lay, s, tau):
    maps = _maps(lay, s)
    if lay.n_score <= 600_000:
        return oracle.detections(maps, tau)
    # the same list, row-major per map, without a Python loop per position
    out = []
    for k, S in enumerate(maps):
        ys, xs = np.nonzero(S >= tau)
        out.extend((k, int(y), int(x), float(S[y, x])) for y, x in zip(ys, xs))
    return out


@pytest.mark.parametrize("wl_name", ["config2", "uneven_batch", "config3"])
def test_detections_equal_thresholded_scores(wl_name):
    wl = getattr(workloads, wl_name)()
    note(f"detect {wl.name}")
    ctx, lay, scores, _ = _scored(wl, "tensor_bf16", 16)
    s = scores.cpu().numpy()[:lay.n_score]
    # config3 has several thousand count blocks: the compaction's block
    # offsets then come from the two-level scan over segments of blocks
    note(f"  {lay.n_score} score positions")
    fin = s[np.isfinite(s)]
    for q in (0.5, 0.99, 0.9999):
        tau = float(np.quantile(fin, q))
        rec, sc, n = ctx.detect(scores, tau)
        want = _host_list(lay, s, tau)
        assert n == len(want), (q, n, len(want))
        got = [(int(a), int(b), int(c), float(d)) for (a, b, c, _), d in zip(rec.cpu().numpy(), sc.cpu().numpy())]
        assert got == want
    # capacity below the count: the first records, the full count
    tau = float(np.quantile(fin, 0.5))
    rec, sc, n = ctx.detect(scores, tau, capacity=7)
    assert n == len(_host_list(lay, s, tau)) and rec.shape[0] == 7
    assert [tuple(int(v) for v in r[:3]) for r in rec.cpu().numpy()] == [w[:3] for w in _host_list(lay, s, tau)[:7]]
    # nothing reaches a threshold above every score
    _, _, n = ctx.detect(scores, float(fin.max()) + 1.0)
    assert n == 0
    ctx.close()


def test_detections_agree_with_oracle_away_from_tau():
    wl = workloads.config1()
    note("detect vs oracle, config1")
    ctx, lay, scores, U = _scored(wl, "direct_fp32", None)
    sm = oracle_map(wl, 0, 1, 0, None, {})
    tau = float(np.median(sm.score[np.isfinite(sm.score)]))
    rec, sc, n = ctx.detect(scores, tau)
    got = {(int(r[1]), int(r[2])) for r in rec.cpu().numpy()}
    tol = TOL["direct_fp32"]
    for y in range(sm.score.shape[0]):
        for x in range(sm.score.shape[1]):
            v = sm.score[y, x]
            if abs(v - tau) > tol:
                assert ((y, x) in got) == (v >= tau), (y, x, v, tau)
    ctx.close()
