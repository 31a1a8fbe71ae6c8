"""Pins of the HOG oracle (oracle/hog.py) against facts fixed independently of
its code: closed forms on ramp images, symmetries of the gradient field,
shift and intensity-scale behaviour, the bounds the truncation implies, and
scalar brute force of its vectorised steps on tiny images."""
import math

import numpy as np
import pytest

from oracle import hog

A = hog.ALPHA


def _ramp(h, w, gx, gy, base=0):
    """uint8 image I(y, x) = base + gx x + gy y on all three channels."""
    y, x = np.mgrid[0:h, 0:w]
    v = base + gx * x + gy * y
    assert v.min() >= 0 and v.max() <= 255
    return np.repeat(v[..., None], 3, axis=2).astype(np.uint8)


def _noise_image(seed, h, w):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:h, 0:w]
    base = 128 + 60 * np.sin(x / 5.0 + rng.uniform(0, 6)) * np.cos(y / 7.0 + rng.uniform(0, 6))
    img = base[..., None] + rng.normal(0, 25, (h, w, 3))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def test_constant_image_has_no_gradient_features():
    img = np.full((40, 48, 3), 77, np.uint8)
    lv = hog.HogLevel(nr=9, nc=11, cell=4, inv_scale=1.0, pad_rows=2, pad_cols=3)
    f = hog.hog_level(img, lv)
    assert f.shape == (13, 17, 32)
    inner = f[2:11, 3:14]
    assert np.all(inner == 0.0)
    pad = np.ones((13, 17), bool)
    pad[2:11, 3:14] = False
    assert np.all(f[pad][:, :31] == 0.0) and np.all(f[pad][:, 31] == 1.0)


@pytest.mark.parametrize("cell", [4, 8])
def test_horizontal_ramp_closed_form(cell):
    """I = 3x: every pixel's gradient points along +x (direction 0), and every
    cell's ratios to its normalisers are at least 1/2, so each truncates to
    alpha: channels 0 and 18 are 4 * alpha / 2, texture channels alpha / sqrt(18),
    all others zero."""
    img = _ramp(8 * cell + 4, 80, 3, 0)
    lv = hog.HogLevel(nr=8, nc=80 // cell - 1, cell=cell, inv_scale=1.0)
    bins, mag = hog.pixel_votes(img, lv)
    assert np.all(bins == 0)
    assert np.all(mag[:, 1:] == 6.0) and np.all(mag[:, 0] == 3.0)   # the left edge repeats column 0
    f = hog.hog_level(img, lv)
    want = np.zeros(32)
    want[0] = want[18] = 4 * A / 2
    want[27:31] = A / math.sqrt(18.0)
    np.testing.assert_allclose(f, np.broadcast_to(want, f.shape), rtol=0, atol=1e-15)


def test_decreasing_ramp_votes_for_the_opposite_direction():
    img = _ramp(36, 60, -3, 0, base=200)
    lv = hog.HogLevel(nr=8, nc=13, cell=4, inv_scale=1.0)
    f = hog.hog_level(img, lv)
    assert np.allclose(f[..., 9], 4 * A / 2) and np.allclose(f[..., 18], 4 * A / 2)
    assert np.all(f[..., 0] == 0.0)


def test_vertical_ramp_ties_go_to_the_first_direction():
    """+y lies half-way between directions 4 (80 deg) and 5 (100 deg); their
    float32 sines are equal, so the projections tie and the first wins."""
    cos9, sin9 = hog.orientation_table()
    assert sin9[4] == sin9[5] and cos9[4] == -cos9[5]
    img = _ramp(80, 40, 0, 3)
    lv = hog.HogLevel(nr=18, nc=9, cell=4, inv_scale=1.0)
    bins, _ = hog.pixel_votes(img, lv)
    assert np.all(bins == 4)
    f = hog.hog_level(img, lv)
    assert np.allclose(f[..., 4], 4 * A / 2) and np.allclose(f[..., 18 + 4], 4 * A / 2)


def test_orientation_table_is_the_nine_directions():
    c, s = hog.orientation_table()
    assert c.dtype == np.float32 and s.dtype == np.float32
    for o in range(9):
        assert abs(float(c[o]) - math.cos(o * math.pi / 9)) <= 2 ** -24
        assert abs(float(s[o]) - math.sin(o * math.pi / 9)) <= 2 ** -24
    assert c[0] == 1.0 and s[0] == 0.0


@pytest.mark.parametrize("inv_scale", [1.0, 2.0])
def test_inverting_the_image_swaps_opposite_directions(inv_scale):
    """255 - I negates every gradient: contrast-sensitive bins o and o + 9 swap,
    the contrast-insensitive and texture channels stay.  Exact at inverse
    scales 1 and 2, where the float32 samples are exact."""
    img = _noise_image(5, 70, 90)
    lv = hog.HogLevel(nr=8, nc=10, cell=4, inv_scale=inv_scale, pad_rows=1, pad_cols=1)
    f = hog.hog_level(img, lv)
    g = hog.hog_level((255 - img).astype(np.uint8), lv)
    perm = [(o + 9) % 18 for o in range(18)]
    np.testing.assert_allclose(g[..., :18], f[..., perm], rtol=0, atol=1e-14)
    np.testing.assert_allclose(g[..., 18:], f[..., 18:], rtol=0, atol=1e-14)


def test_shift_by_one_cell_shifts_the_features():
    img = _noise_image(6, 60, 72)
    c = 4
    lv = hog.HogLevel(nr=10, nc=12, cell=c, inv_scale=1.0)
    f = hog.hog_level(img, lv)
    g = hog.hog_level(img[c:, c:], hog.HogLevel(nr=9, nc=11, cell=c, inv_scale=1.0))
    # cells two away from every border of both grids see the same pixels and neighbours
    np.testing.assert_allclose(g[2:-2, 2:-2], f[3:-2, 3:-2][:g.shape[0] - 4, :g.shape[1] - 4],
                               rtol=0, atol=1e-13)


def test_intensity_scale_leaves_features_almost_unchanged():
    img = (_noise_image(7, 50, 50) // 2).astype(np.uint8)
    lv = hog.HogLevel(nr=10, nc=10, cell=4, inv_scale=1.0)
    f = hog.hog_level(img, lv)
    g = hog.hog_level((2 * img.astype(np.int32)).astype(np.uint8), lv)
    np.testing.assert_array_equal(hog.pixel_votes(img, lv)[0], hog.pixel_votes(2 * img, lv)[0])
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-6)       # only eps breaks the invariance


def test_features_lie_within_the_truncation_bounds():
    img = _noise_image(8, 90, 120)
    for cell, k in ((4, 1.0), (4, 1.35), (8, 0.8)):
        lv = hog.HogLevel(nr=90 // cell - 1, nc=120 // cell - 1, cell=cell, inv_scale=k)
        f = hog.hog_level(img, lv)
        assert f.min() >= 0.0
        assert f[..., :27].max() <= 4 * A / 2 + 1e-15
        assert f[..., 27:31].max() <= 18 * A / math.sqrt(18.0) + 1e-12
        assert np.all(f[..., 31] == 0.0)
        # the insensitive channel is bounded by the sum of its two sensitive halves
        assert np.all(f[..., 18:27] <= f[..., :9] + f[..., 9:18] + 1e-12)


def _scalar_sample(img, y, x, k):
    """Step 1 for one resized pixel with numpy float32 scalars."""
    H, W, _ = img.shape
    f32 = np.float32

    def co(t, n):
        s = (f32(t) + f32(0.5)) * f32(k) - f32(0.5)
        s = min(max(s, f32(0.0)), f32(n - 1))
        i0 = int(math.floor(s))
        return i0, min(i0 + 1, n - 1), f32(s - f32(i0))

    y0, y1, fy = co(y, H)
    x0, x1, fx = co(x, W)
    out = []
    for ch in range(3):
        p = [[f32(img[a, b, ch]) for b in (x0, x1)] for a in (y0, y1)]
        top = (f32(1) - fx) * p[0][0] + fx * p[0][1]
        bot = (f32(1) - fx) * p[1][0] + fx * p[1][1]
        out.append((f32(1) - fy) * top + fy * bot)
    return out


@pytest.mark.parametrize("k", [1.0, 1.2599211, 0.75])
def test_pixel_votes_match_a_scalar_brute_force(k):
    img = _noise_image(9, 23, 29)
    lv = hog.HogLevel(nr=3, nc=4, cell=4, inv_scale=k)
    bins, mag = hog.pixel_votes(img, lv)
    cos9, sin9 = hog.orientation_table()
    f32 = np.float32
    for y in range(12):
        for x in range(16):
            P = {(dy, dx): _scalar_sample(img, y + dy, x + dx, k) for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0))}
            best, bx, by = f32(-1), None, None
            for ch in range(3):
                gx = P[(0, 1)][ch] - P[(0, -1)][ch]
                gy = P[(1, 0)][ch] - P[(-1, 0)][ch]
                m2 = gx * gx + gy * gy
                if m2 > best:
                    best, bx, by = m2, gx, gy
            dots = []
            for o in range(18):
                p = bx * cos9[o % 9] + by * sin9[o % 9]
                dots.append(p if o < 9 else -p)
            b = 0
            for o in range(1, 18):
                if dots[o] > dots[b]:
                    b = o
            assert bins[y, x] == b, (y, x)
            assert mag[y, x] == math.sqrt(float(bx) ** 2 + float(by) ** 2)


def test_cell_histograms_match_a_brute_force_over_pixels():
    """Each pixel's magnitude spread over the 4 surrounding cells by the
    product of its distances to their centres; summed cell by cell."""
    img = _noise_image(10, 40, 44)
    for cell in (4, 8):
        lv = hog.HogLevel(nr=40 // cell, nc=44 // cell, cell=cell, inv_scale=1.0)
        bins, mag = hog.pixel_votes(img, lv)
        want = np.zeros((lv.nr, lv.nc, 18))
        for i in range(lv.nr):
            for j in range(lv.nc):
                cy, cx = (i + 0.5) * cell, (j + 0.5) * cell       # cell centre in pixels
                for y in range(bins.shape[0]):
                    wy = 1.0 - abs(y + 0.5 - cy) / cell
                    if wy <= 0:
                        continue
                    for x in range(bins.shape[1]):
                        wx = 1.0 - abs(x + 0.5 - cx) / cell
                        if wx > 0:
                            want[i, j, bins[y, x]] += mag[y, x] * wy * wx
        np.testing.assert_allclose(hog.cell_histograms(bins, mag, lv), want, rtol=1e-12, atol=1e-9)


def test_normalisers_and_projection_by_hand():
    """A 2x2 grid with hand-set histograms: each cell's 4 blocks, the
    truncation, the two folds and the texture sums, written out cell by cell."""
    H = np.zeros((2, 2, 18))
    H[0, 0, 3] = 3.0
    H[0, 0, 12] = 1.0           # opposite of 3: folds into insensitive bin 3
    H[0, 1, 0] = 2.0
    H[1, 0, 17] = 0.5
    H[1, 1, 5] = 10.0
    E = {(0, 0): 16.0, (0, 1): 4.0, (1, 0): 0.25, (1, 1): 100.0}
    e = lambda i, j: E.get((i, j), 0.0)
    f = hog.cell_features(H)
    for i in range(2):
        for j in range(2):
            N = [math.sqrt(e(i, j) + e(i + a, j) + e(i, j + b) + e(i + a, j + b) + hog.EPS)
                 for a, b in ((-1, -1), (-1, 1), (1, -1), (1, 1))]
            for o in range(18):
                assert f[i, j, o] == pytest.approx(0.5 * sum(min(H[i, j, o] / n, A) for n in N), abs=1e-15)
            for o in range(9):
                d = H[i, j, o] + H[i, j, o + 9]
                assert f[i, j, 18 + o] == pytest.approx(0.5 * sum(min(d / n, A) for n in N), abs=1e-15)
            for k in range(4):
                t = sum(min(H[i, j, o] / N[k], A) for o in range(18))
                assert f[i, j, 27 + k] == pytest.approx(t / math.sqrt(18.0), abs=1e-15)
            assert f[i, j, 31] == 0.0
