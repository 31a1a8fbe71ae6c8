"""FP64 CPU oracle of the HOG feature pyramid (the feature map phi).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this module; only the tests, the smoke check and the benchmark's CPU
baseline leg call it.  It shares no code with the GPU path.

The paper scores a pyramid of HOG cells (Section 2, phi: "some variation of
HOG"), 32 values per cell (Section 5, L = 32), and leaves the variant open.
This oracle computes the 32-value variant of Felzenszwalb, Girshick,
McAllester and Ramanan (PAMI 2010, Section 6), written from that description:

1. Sampling.  A level of cell size c and inverse scale k samples the image at
   resized pixel (y, x) bilinearly at source position ((y+1/2) k - 1/2,
   (x+1/2) k - 1/2), clamped to the image (so rows and columns beyond the
   image repeat its edge).
2. Gradient.  Centred differences dx = I(y, x+1) - I(y, x-1), dy = I(y+1, x) -
   I(y-1, x) on each colour channel; the channel with the largest dx^2 + dy^2
   is kept (ties: the first channel).
3. Orientation.  The pixel votes for the direction among 18 (angles o pi / 9,
   o < 18) with the largest projection of (dx, dy); ties go to the smallest o.
   Directions o and o + 9 are opposite, so that projection is +p_o or -p_o
   with p_o = dx cos(o pi/9) + dy sin(o pi/9), o < 9.
4. Cells.  The vote has the gradient magnitude as weight and is spread
   bilinearly over the 4 cells whose centres surround the pixel: the pixel
   sits at cell coordinate ((y+1/2)/c - 1/2, (x+1/2)/c - 1/2).  Votes for
   cells outside the level's grid are dropped.  This gives the 18-bin
   contrast-sensitive histogram C of every cell and its 9-bin
   contrast-insensitive fold D_o = C_o + C_{o+9}.
5. Normalisation.  E = sum_o D_o^2 per cell (0 outside the grid).  Each cell
   has 4 normalisers, one per 2x2 block of cells that contains it,
   N_k = sqrt(E(i,j) + E(i+a,j) + E(i,j+b) + E(i+a,j+b) + eps) with
   (a, b) = (-1,-1), (-1,+1), (+1,-1), (+1,+1) for k = 0..3.
6. Truncation and projection.  T(v) = min(v, alpha), alpha = 0.2.
   channel o < 18:        1/2 * sum_k T(C_o / N_k)       (contrast-sensitive)
   channel 18 + o, o < 9: 1/2 * sum_k T(D_o / N_k)       (contrast-insensitive)
   channel 27 + k:        tau * sum_{o<18} T(C_o / N_k)  (texture), tau = 1/sqrt(18)
   channel 31:            0 inside the image, 1 in the padding band.
   eps = 1e-4.

alpha = 0.2 is the truncation the PAMI description gives; the factor 1/2,
tau and eps are this oracle's readings where that description is silent.

Steps 1-3 decide integers (a channel, a bin) from floating point, so they run
in float32 in a fixed order of operations, every product and sum rounded on
its own (no fused multiply-add): a kernel that does the same takes the same
decisions.  The orientation table is float32(cos(o pi/9)), float32(sin(o pi/9))
evaluated in float64.  Magnitudes, histograms and everything after them are
float64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

F32 = np.float32
ALPHA = 0.2
EPS = 1e-4
HALF = 0.5
TAU = 1.0 / np.sqrt(18.0)
N_BINS = 18
N_FEATURES = 32


@dataclass
class HogLevel:
    """Geometry of one pyramid level: an nr x nc grid of interior cells of
    cell size `cell` pixels, sampled at inverse scale `inv_scale`, with
    pad_rows / pad_cols padding cells on every side."""
    nr: int
    nc: int
    cell: int
    inv_scale: float
    pad_rows: int = 0
    pad_cols: int = 0


def orientation_table() -> Tuple[np.ndarray, np.ndarray]:
    """(cos, sin) of the 9 directions o pi / 9, o < 9, rounded to float32."""
    ang = np.arange(9, dtype=np.float64) * np.pi / 9.0
    return np.cos(ang).astype(F32), np.sin(ang).astype(F32)


def sample(img: np.ndarray, ys: np.ndarray, xs: np.ndarray, inv_scale: float) -> np.ndarray:
    """Step 1: float32 bilinear samples of the (H, W, 3) uint8 image at the
    resized pixel grid ys x xs (integers, any range); shape (len(ys), len(xs), 3)."""
    H, W, _ = img.shape
    k = F32(inv_scale)

    def coords(t, n):
        s = (np.asarray(t).astype(F32) + F32(0.5)) * k - F32(0.5)
        s = np.minimum(np.maximum(s, F32(0.0)), F32(n - 1))
        i0 = np.floor(s).astype(np.int64)
        f = s - i0.astype(F32)
        i1 = np.minimum(i0 + 1, n - 1)
        return i0, i1, f

    y0, y1, fy = coords(ys, H)
    x0, x1, fx = coords(xs, W)
    p = img.astype(F32)
    fy = fy[:, None, None]
    fx = fx[None, :, None]
    gy = F32(1.0) - fy
    gx = F32(1.0) - fx
    top = gx * p[y0][:, x0] + fx * p[y0][:, x1]
    bot = gx * p[y1][:, x0] + fx * p[y1][:, x1]
    return gy * top + fy * bot


def pixel_votes(img: np.ndarray, lv: HogLevel) -> Tuple[np.ndarray, np.ndarray]:
    """Steps 1-3 for the resized pixels 0 <= y < nr*cell, 0 <= x < nc*cell:
    (bin int64, magnitude float64), each of shape (nr*cell, nc*cell)."""
    Hr, Wr = lv.nr * lv.cell, lv.nc * lv.cell
    I = sample(img, np.arange(-1, Hr + 1), np.arange(-1, Wr + 1), lv.inv_scale)
    dx = I[1:-1, 2:, :] - I[1:-1, :-2, :]                      # float32, rounded once
    dy = I[2:, 1:-1, :] - I[:-2, 1:-1, :]
    m2 = dx * dx + dy * dy                                      # each product rounded, then the sum
    ch = np.argmax(m2, axis=2)                                  # first channel on ties
    gx = np.take_along_axis(dx, ch[..., None], axis=2)[..., 0]
    gy = np.take_along_axis(dy, ch[..., None], axis=2)[..., 0]
    u, v = orientation_table()
    p = gx[..., None] * u + gy[..., None] * v                   # (Hr, Wr, 9) float32
    dots = np.concatenate([p, -p], axis=2)                      # directions o and o + 9
    b = np.argmax(dots, axis=2)                                 # first direction on ties
    mag = np.sqrt(gx.astype(np.float64) ** 2 + gy.astype(np.float64) ** 2)
    return b.astype(np.int64), mag


def cell_histograms(bins: np.ndarray, mag: np.ndarray, lv: HogLevel) -> np.ndarray:
    """Step 4: the (nr, nc, 18) float64 histograms from the pixel votes."""
    c = lv.cell
    Hr, Wr = bins.shape
    hist = np.zeros((lv.nr + 2, lv.nc + 2, N_BINS))            # one spare cell on every side
    yp = (np.arange(Hr) + 0.5) / c - 0.5
    xp = (np.arange(Wr) + 0.5) / c - 0.5
    iy = np.floor(yp).astype(np.int64)
    ix = np.floor(xp).astype(np.int64)
    wy1 = yp - iy
    wx1 = xp - ix
    for a, wy in ((0, 1.0 - wy1), (1, wy1)):
        for b, wx in ((0, 1.0 - wx1), (1, wx1)):
            w = mag * wy[:, None] * wx[None, :]
            rows = (iy + a + 1)[:, None] + np.zeros_like(bins)
            cols = (ix + b + 1)[None, :] + np.zeros_like(bins)
            np.add.at(hist, (rows, cols, bins), w)
    return hist[1:-1, 1:-1]


def normalisers(hist: np.ndarray) -> np.ndarray:
    """Step 5: the (nr, nc, 4) block normalisers N_k."""
    D = hist[..., :9] + hist[..., 9:]
    E = np.zeros((hist.shape[0] + 2, hist.shape[1] + 2))
    E[1:-1, 1:-1] = (D * D).sum(axis=2)
    nr, nc = hist.shape[:2]
    out = np.empty((nr, nc, 4))
    for k, (a, b) in enumerate(((-1, -1), (-1, 1), (1, -1), (1, 1))):
        s = (E[1:-1, 1:-1] + E[1 + a:1 + a + nr, 1:-1] + E[1:-1, 1 + b:1 + b + nc]
             + E[1 + a:1 + a + nr, 1 + b:1 + b + nc])
        out[..., k] = np.sqrt(s + EPS)
    return out


def cell_features(hist: np.ndarray) -> np.ndarray:
    """Step 6: the (nr, nc, 32) features of the interior cells."""
    N = normalisers(hist)
    D = hist[..., :9] + hist[..., 9:]
    TC = np.minimum(hist[..., :, None] / N[..., None, :], ALPHA)   # (nr, nc, 18, 4)
    TD = np.minimum(D[..., :, None] / N[..., None, :], ALPHA)      # (nr, nc, 9, 4)
    out = np.zeros(hist.shape[:2] + (N_FEATURES,))
    out[..., :18] = HALF * TC.sum(axis=3)
    out[..., 18:27] = HALF * TD.sum(axis=3)
    out[..., 27:31] = TAU * TC.sum(axis=2)
    return out


def hog_level(img: np.ndarray, lv: HogLevel) -> np.ndarray:
    """One padded level, (nr + 2 pad_rows, nc + 2 pad_cols, 32) float64."""
    bins, mag = pixel_votes(img, lv)
    feat = cell_features(cell_histograms(bins, mag, lv))
    R, C = lv.nr + 2 * lv.pad_rows, lv.nc + 2 * lv.pad_cols
    out = np.zeros((R, C, N_FEATURES))
    out[..., 31] = 1.0
    out[lv.pad_rows:lv.pad_rows + lv.nr, lv.pad_cols:lv.pad_cols + lv.nc] = feat
    return out


def hog_pyramid(img: np.ndarray, levels: Sequence[HogLevel]) -> List[np.ndarray]:
    return [hog_level(img, lv) for lv in levels]
