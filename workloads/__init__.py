"""Seeded synthetic workloads of the paper's shapes.

This module only draws inputs: HOG-like feature pyramids, filter banks,
deformation coefficients and anchors, plus the five preset configurations.
It holds none of the scoring arithmetic (no correlation, no decomposition, no
distance transform), so the FP64 oracle and the GPU library can both be fed
from it without sharing any of the method's code.

Shapes follow the DPM setting the paper builds on (Section 2: a root filter,
n part filters at twice the resolution, deformation coefficients d_i, HOG
cells of L=32 features as in Section 5).  Value distributions are synthetic
stand-ins for trained models and real images, which are not available.

Seeds: ``numpy.random.default_rng(SeedSequence([1707, 3268, config, stream]))``
with stream 0 = image sizes, 1 = filters, 2 = deformations and anchors,
3 = the feature hash seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

N_CHANNELS = 32          # HOG feature length L (Section 5 uses L = 32)
OCTAVE = 10              # levels per octave; parts live one octave below the root
PAD_ROWS = 6             # pyramid padding, rows per side
PAD_COLS = 11            # pyramid padding, cols per side
CELL = 8                 # pixels per HOG cell

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


# --------------------------------------------------------------------------
# counter-based generator (SplitMix64, S. Vigna's published mixer)
# --------------------------------------------------------------------------
def splitmix64(x: np.ndarray) -> np.ndarray:
    """Stateless SplitMix64 output for counter values ``x`` (uint64 array).

    One step of the generator: add the golden-ratio increment, then the
    xor-shift-multiply finaliser with constants 0xbf58476d1ce4e5b9 and
    0x94d049bb133111eb and shifts 30, 27, 31.
    """
    z = np.asarray(x, dtype=np.uint64) + np.uint64(_GOLDEN)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def splitmix64_scalar(x: int) -> int:
    z = (x + _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def hash_uniform(seed: int, index: np.ndarray) -> np.ndarray:
    """u in [0, 1) with 24 random bits: (sm64(seed ^ sm64(index)) >> 40) * 2^-24."""
    with np.errstate(over="ignore"):
        inner = splitmix64(np.asarray(index, dtype=np.uint64))
        outer = splitmix64(inner ^ np.uint64(seed & _MASK))
    return (outer >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def seed_rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([1707, 3268, config, stream]))


def feature_seed(config: int) -> int:
    return int(np.random.SeedSequence([1707, 3268, config, 3]).generate_state(1, np.uint64)[0])


# --------------------------------------------------------------------------
# data classes
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Level:
    cell_offset: int      # first cell of this level in the packed HWC buffer
    rows: int             # padded rows
    cols: int             # padded cols


@dataclasses.dataclass
class Pyramid:
    levels: List[Level]
    octave: int = OCTAVE


@dataclasses.dataclass
class Component:
    root: int                     # filter index of the root
    parts: List[int]              # filter indices of the parts
    anchors: np.ndarray           # (n_parts, 2) int32 (v_y, v_x) on the part level
    deform: np.ndarray            # (n_parts, 4) float32 (d_x, d_xx, d_y, d_yy)


@dataclasses.dataclass
class Bank:
    filters: List[np.ndarray]     # each (h, w, 32) float32, HWC
    components: List[Component]

    @property
    def shapes(self) -> List[Tuple[int, int]]:
        return [(int(f.shape[0]), int(f.shape[1])) for f in self.filters]


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    pyramids: List[Pyramid]       # one per image
    bank: Bank
    total_cells: int              # cells in the packed feature buffer
    feat_seed: int
    padded: bool
    image_sizes: List[Tuple[int, int]]   # (width, height) in pixels, or level sizes for c1

    def features(self) -> np.ndarray:
        """The packed FP32 HWC feature buffer, shape (total_cells, 32)."""
        out = np.zeros((self.total_cells, N_CHANNELS), dtype=np.float32)
        for pyr in self.pyramids:
            for lv in pyr.levels:
                out[lv.cell_offset:lv.cell_offset + lv.rows * lv.cols] = \
                    level_values(lv, self.feat_seed, self.padded).reshape(-1, N_CHANNELS)
        return out

    def level_features(self, image: int, level: int) -> np.ndarray:
        return level_values(self.pyramids[image].levels[level], self.feat_seed, self.padded)


# --------------------------------------------------------------------------
# features
# --------------------------------------------------------------------------
def level_values(lv: Level, seed: int, padded: bool) -> np.ndarray:
    """One level's cells as a (rows, cols, 32) float32 array.

    Interior cells: channels 0-26 uniform [0, 0.2), 27-30 uniform [0, 0.4),
    channel 31 zero.  Padding cells (a band of PAD_ROWS rows and PAD_COLS cols
    on every side when ``padded``): channels 0-30 zero, channel 31 one.
    Values come from the counter hash of the global element index
    (cell_offset * 32 + cell * 32 + channel), so any level of the packed buffer
    can be regenerated on its own.
    """
    n = lv.rows * lv.cols
    idx = (np.arange(n * N_CHANNELS, dtype=np.uint64)
           + np.uint64(lv.cell_offset * N_CHANNELS))
    u = hash_uniform(seed, idx).astype(np.float32).reshape(lv.rows, lv.cols, N_CHANNELS)
    scale = np.full(N_CHANNELS, np.float32(0.2), dtype=np.float32)
    scale[27:31] = np.float32(0.4)
    scale[31] = np.float32(0.0)
    vals = u * scale
    if padded:
        interior = np.zeros((lv.rows, lv.cols), dtype=bool)
        interior[PAD_ROWS:lv.rows - PAD_ROWS, PAD_COLS:lv.cols - PAD_COLS] = True
        vals[~interior] = 0.0
        vals[~interior, 31] = 1.0
    return vals


def _i64(c: int) -> int:
    """A 64-bit constant as the signed value torch's int64 arithmetic uses."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _splitmix64_torch(z):
    """splitmix64 on a torch int64 tensor (two's-complement wrap-around, logical
    shifts by masking the arithmetic ones); the same bits as ``splitmix64``."""
    import torch  # noqa: F401

    def lsr(v, k):
        return (v >> k) & ((1 << (64 - k)) - 1)
    z = z + _i64(_GOLDEN)
    z = (z ^ lsr(z, 30)) * _i64(_M1)
    z = (z ^ lsr(z, 27)) * _i64(_M2)
    return z ^ lsr(z, 31)


def _image_cell_range(pyr: Pyramid) -> Tuple[int, int]:
    first = pyr.levels[0].cell_offset
    last = pyr.levels[-1]
    return first, last.cell_offset + last.rows * last.cols


def _padding_mask(pyr: Pyramid, padded: bool):
    """Boolean mask over an image's cells (relative to its first cell): True
    in the padding band of every level."""
    first, end = _image_cell_range(pyr)
    mask = np.zeros(end - first, dtype=bool)
    if padded:
        for lv in pyr.levels:
            m = np.ones((lv.rows, lv.cols), dtype=bool)
            m[PAD_ROWS:lv.rows - PAD_ROWS, PAD_COLS:lv.cols - PAD_COLS] = False
            mask[lv.cell_offset - first:lv.cell_offset - first + lv.rows * lv.cols] = m.ravel()
    return mask


def features_device(wl: "Workload", device, out=None, cell_base: int = 0, images=None):
    """The packed feature buffer generated on a torch device, bit for bit the
    values of ``Workload.features()`` (the same counter hash of the global
    element index, the same float32 scaling and padding), one image at a
    time, so that large batches need no host copy.  ``images`` (default all)
    selects a contiguous run of images; ``cell_base`` is the global cell index
    of ``out``'s first row (default 0: ``out`` holds the whole buffer).
    Returns ``out`` (allocated when None)."""
    import torch
    imgs = range(len(wl.pyramids)) if images is None else images
    if out is None:
        lo = _image_cell_range(wl.pyramids[imgs[0]])[0]
        hi = _image_cell_range(wl.pyramids[imgs[-1]])[1]
        out = torch.empty((hi - lo, N_CHANNELS), dtype=torch.float32, device=device)
        cell_base = lo
    scale = torch.full((N_CHANNELS,), 0.2, dtype=torch.float32, device=device)
    scale[27:31] = 0.4
    scale[31] = 0.0
    pad_row = torch.zeros(N_CHANNELS, dtype=torch.float32, device=device)
    pad_row[31] = 1.0
    seed = _i64(wl.feat_seed & _MASK)
    masks = {}
    for i in imgs:
        pyr = wl.pyramids[i]
        first, end = _image_cell_range(pyr)
        key = tuple((lv.cell_offset - first, lv.rows, lv.cols) for lv in pyr.levels)
        if key not in masks:
            masks[key] = torch.from_numpy(_padding_mask(pyr, wl.padded)).to(device)
        n = end - first
        idx = torch.arange(n * N_CHANNELS, dtype=torch.int64, device=device) + first * N_CHANNELS
        outer = _splitmix64_torch(_splitmix64_torch(idx) ^ seed)
        u = ((outer >> 40) & ((1 << 24) - 1)).to(torch.float32) * (2.0 ** -24)
        vals = u.view(n, N_CHANNELS) * scale
        vals[masks[key]] = pad_row
        out[first - cell_base:end - cell_base] = vals
        del idx, outer, u, vals
    return out


def pyramid_level_sizes(width: int, height: int) -> List[Tuple[int, int]]:
    """Unpadded (rows, cols) of every level: 10 levels per octave, level 0 at 2x.

    rows = floor(H * 2^(1 - l/10) / 8), cols likewise; stop once min < 8.
    """
    sizes = []
    lvl = 0
    while True:
        s = 2.0 ** (1.0 - lvl / OCTAVE)
        r = int(math.floor(height * s / CELL))
        c = int(math.floor(width * s / CELL))
        if min(r, c) < 8:
            break
        sizes.append((r, c))
        lvl += 1
    return sizes


def build_pyramids(image_sizes: Sequence[Tuple[int, int]]) -> Tuple[List[Pyramid], int]:
    pyrs = []
    off = 0
    for (w, h) in image_sizes:
        levels = []
        for (r, c) in pyramid_level_sizes(w, h):
            rows, cols = r + 2 * PAD_ROWS, c + 2 * PAD_COLS
            levels.append(Level(off, rows, cols))
            off += rows * cols
        pyrs.append(Pyramid(levels))
    return pyrs, off


def hog_levels(pyr: Pyramid, pad_rows: int = PAD_ROWS, pad_cols: int = PAD_COLS):
    """Geometry of a pyramid's levels for HOG extraction, one tuple
    (cell_offset, rows, cols, pad_rows, pad_cols, cell, inv_scale) per level.
    Level l of the first octave takes cells of 4 resized pixels on the image
    scaled by 2^(-l/10); later levels cells of CELL pixels on the image scaled
    by 2^(1 - l/10).  Both give the level's floor(side * 2^(1 - l/10) / CELL)
    interior cells (the image covers them: those cells span at most the
    resized image)."""
    out = []
    for l, lv in enumerate(pyr.levels):
        cell = CELL // 2 if l < pyr.octave else CELL
        inv = 2.0 ** (l / pyr.octave) if l < pyr.octave else 2.0 ** (l / pyr.octave - 1.0)
        out.append((lv.cell_offset, lv.rows, lv.cols, pad_rows, pad_cols, cell, inv))
    return out


def synthetic_image(seed: int, width: int, height: int, n_shapes: int = 24,
                    noise: float = 6.0) -> np.ndarray:
    """Seeded uint8 (height, width, 3) RGB test image: a smooth colour
    gradient, n_shapes filled ellipses and rotated rectangles of random
    colours and sizes, and Gaussian pixel noise, so that edges of every
    orientation and scale reach the HOG stage."""
    rng = np.random.default_rng(np.random.SeedSequence([1707, 3268, 99, seed]))
    y, x = np.mgrid[0:height, 0:width].astype(np.float32)
    c0, c1 = rng.uniform(40, 215, 3), rng.uniform(40, 215, 3)
    t = (x / max(width - 1, 1) * rng.uniform(0.2, 1.0) + y / max(height - 1, 1) * rng.uniform(0.2, 1.0))
    t = t / max(float(t.max()), 1e-6)
    img = c0[None, None, :] * (1.0 - t[..., None]) + c1[None, None, :] * t[..., None]
    for k in range(n_shapes):
        cx, cy = rng.uniform(0, width), rng.uniform(0, height)
        a, b = rng.uniform(0.03, 0.25) * width, rng.uniform(0.03, 0.25) * height
        th = rng.uniform(0, np.pi)
        u = (x - cx) * np.cos(th) + (y - cy) * np.sin(th)
        v = -(x - cx) * np.sin(th) + (y - cy) * np.cos(th)
        inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0 if k % 2 == 0 else (np.abs(u) <= a) & (np.abs(v) <= b)
        img[inside] = rng.uniform(0, 255, 3)
    img += rng.normal(0.0, noise, img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# filters, components
# --------------------------------------------------------------------------
def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v)


def draw_filter(rng: np.random.Generator, h: int, w: int, basis: np.ndarray,
                rank: int = 8, decay: float = 1.5, noise: float = 0.05) -> np.ndarray:
    """Rank-``rank`` sum of outer products plus Gaussian noise, unit Frobenius norm.

    f = sum_j j^-decay a_j (x) b_j (x) c_j + noise * E / ||E||, with a_j, b_j unit
    Gaussian vectors and c_j unit vectors in the span of the shared ``basis``.
    """
    f = np.zeros((h, w, N_CHANNELS), dtype=np.float64)
    for j in range(1, rank + 1):
        a = _unit(rng.standard_normal(h))
        b = _unit(rng.standard_normal(w))
        c = _unit(basis @ rng.standard_normal(basis.shape[1]))
        f += j ** (-decay) * np.einsum("i,j,k->ijk", a, b, c)
    e = rng.standard_normal((h, w, N_CHANNELS))
    f += noise * e / np.linalg.norm(e)
    f /= np.linalg.norm(f)
    return f.astype(np.float32)


ROOT_SHAPES = [(6, 11), (6, 11), (7, 13), (7, 13), (8, 15), (8, 15)]
PART_SHAPE = (6, 6)
N_PARTS = 8


def build_bank(config: int, n_classes: int, root_shapes=ROOT_SHAPES,
               part_shape=PART_SHAPE, n_parts=N_PARTS) -> Bank:
    """``n_classes`` class models; each has one component per root shape.

    Filter order: for each component, its root then its parts, so the parts of
    one component are consecutive filter indices.
    """
    rng_f = seed_rng(config, 1)
    rng_d = seed_rng(config, 2)
    q, _ = np.linalg.qr(rng_f.standard_normal((N_CHANNELS, N_CHANNELS)))
    basis = q[:, :8]
    filters: List[np.ndarray] = []
    comps: List[Component] = []
    for _cls in range(n_classes):
        for (h0, w0) in root_shapes:
            root = len(filters)
            filters.append(draw_filter(rng_f, h0, w0, basis))
            parts = []
            for _p in range(n_parts):
                parts.append(len(filters))
                filters.append(draw_filter(rng_f, part_shape[0], part_shape[1], basis))
            hp, wp = part_shape
            vy = rng_d.integers(0, 2 * h0 - hp + 1, size=n_parts)
            vx = rng_d.integers(0, 2 * w0 - wp + 1, size=n_parts)
            anchors = np.stack([vy, vx], axis=1).astype(np.int32)
            deform = rng_d.uniform(0.01, 0.1, size=(n_parts, 4)).astype(np.float32)
            comps.append(Component(root, parts, anchors, deform))
    return Bank(filters, comps)


# --------------------------------------------------------------------------
# presets
# --------------------------------------------------------------------------
def config1() -> Workload:
    """One root level of 40x30 cells and its 80x60 part level, no padding;
    one component: root 6x11 plus 8 parts 6x6."""
    levels = [Level(0, 60, 80), Level(60 * 80, 30, 40)]
    pyr = Pyramid(levels, octave=1)
    bank = build_bank(1, 1, root_shapes=[(6, 11)])
    return Workload("c1: one 40x30 root level + 80x60 part level, 1 component (9 filters)",
                    1, [pyr], bank, 60 * 80 + 30 * 40, feature_seed(1), False,
                    [(80, 60)])


def config2() -> Workload:
    pyrs, total = build_pyramids([(500, 375)])
    bank = build_bank(2, 1)
    return Workload("c2: 500x375 image, 36-level pyramid, 1 class (54 filters)",
                    2, pyrs, bank, total, feature_seed(2), True, [(500, 375)])


def config3() -> Workload:
    pyrs, total = build_pyramids([(500, 375)])
    bank = build_bank(3, 20)
    return Workload("c3: 500x375 image, 36-level pyramid, 20 classes (1080 filters)",
                    3, pyrs, bank, total, feature_seed(3), True, [(500, 375)])


def config4(n_images: int = 64) -> Workload:
    rng = seed_rng(4, 0)
    sizes = [(int(rng.integers(320, 1281)), int(rng.integers(240, 961))) for _ in range(n_images)]
    pyrs, total = build_pyramids(sizes)
    bank = build_bank(4, 20)
    return Workload(f"c4: {n_images} images 320x240..1280x960, full pyramids, 20 classes (1080 filters)",
                    4, pyrs, bank, total, feature_seed(4), True, sizes)


def config5(n_frames: int = 256) -> Workload:
    sizes = [(1920, 1080)] * n_frames
    pyrs, total = build_pyramids(sizes)
    bank = build_bank(5, 20)
    return Workload(f"c5: {n_frames} frames 1920x1080, 51-level pyramids, 20 classes (1080 filters)",
                    5, pyrs, bank, total, feature_seed(5), True, sizes)


def uneven_batch(n_images: int = 3, n_classes: int = 2, size_lo=(160, 120),
                 size_hi=(400, 300)) -> Workload:
    """A small batch in the shape of the 64-image workload: images of uneven
    sizes drawn uniformly from size_lo..size_hi (width, height), full padded
    pyramids, n_classes class models drawn like the 20-class bank."""
    rng = seed_rng(4, 3)
    sizes = [(int(rng.integers(size_lo[0], size_hi[0] + 1)), int(rng.integers(size_lo[1], size_hi[1] + 1)))
             for _ in range(n_images)]
    pyrs, total = build_pyramids(sizes)
    bank = build_bank(4, n_classes)
    return Workload(f"uneven batch: {n_images} images {size_lo[0]}x{size_lo[1]}..{size_hi[0]}x{size_hi[1]}, "
                    f"{n_classes} classes ({54 * n_classes} filters)", 4, pyrs, bank, total,
                    feature_seed(4), True, sizes)


PRESETS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def plant_objects(wl: Workload, features: np.ndarray, per_comp: int, seed: int = 0):
    """Synthetic positives: a copy of the packed features with ``per_comp``
    objects of every component planted into every image, and their
    hypotheses (image, root level, component, y, x).

    An object of component c at root position (y, x) of root level l writes
    the root filter's positive weights, scaled to a peak of 0.4 (the feature
    range), into the root window at (y, x), and each part filter's likewise
    into its window at the anchor (2y + v_y, 2x + v_x) of level l - octave.
    Root windows stay inside the unpadded interior, part windows inside their
    level; a root window avoids every window planted before it for up to 100
    draws, after which overlaps are allowed (a later object then overwrites
    part of an earlier one, which can only lower the thresholds fitted on
    them).  Only inputs are drawn here: no response is computed."""
    rng = seed_rng(wl.config, 10 + seed)
    out = features.copy()
    positives = []
    for img, pyr in enumerate(wl.pyramids):
        L = len(pyr.levels)
        used = [np.zeros((lv.rows, lv.cols), bool) for lv in pyr.levels]
        pr, pc = (PAD_ROWS, PAD_COLS) if wl.padded else (0, 0)
        for ci, c in enumerate(wl.bank.components):
            h0, w0 = wl.bank.shapes[c.root]
            for _ in range(per_comp):
                for _try in range(200):
                    l = int(rng.integers(pyr.octave, L))
                    lv, pl = pyr.levels[l], pyr.levels[l - pyr.octave]
                    ylo, yhi = pr, lv.rows - pr - h0
                    xlo, xhi = pc, lv.cols - pc - w0
                    if yhi < ylo or xhi < xlo:
                        continue
                    y, x = int(rng.integers(ylo, yhi + 1)), int(rng.integers(xlo, xhi + 1))
                    wins = [(l, y, x, wl.bank.filters[c.root])]
                    ok = True
                    for i, k in enumerate(c.parts):
                        ay, ax = 2 * y + int(c.anchors[i][0]), 2 * x + int(c.anchors[i][1])
                        f = wl.bank.filters[k]
                        if not (ay <= pl.rows - f.shape[0] and ax <= pl.cols - f.shape[1]):
                            ok = False
                            break
                        wins.append((l - pyr.octave, ay, ax, f))
                    if not ok or (_try < 100 and used[l][y:y + h0, x:x + w0].any()):
                        continue
                    for (ll, wy, wx, f) in wins:
                        L_ = pyr.levels[ll]
                        pat = np.maximum(f, 0.0)
                        pat = (0.4 / max(float(pat.max()), 1e-30)) * pat
                        view = out[L_.cell_offset:L_.cell_offset + L_.rows * L_.cols].reshape(
                            L_.rows, L_.cols, N_CHANNELS)
                        view[wy:wy + f.shape[0], wx:wx + f.shape[1], :] = pat.astype(np.float32)
                        used[ll][wy:wy + f.shape[0], wx:wx + f.shape[1]] = True
                    positives.append((img, l, ci, y, x))
                    break
    return out, positives


def count_responses(wl: Workload) -> dict:
    """Response cells the hot path computes: root filters on levels >= octave,
    part filters on the level one octave below, valid placements only."""
    shapes = wl.bank.shapes
    roots = [c.root for c in wl.bank.components]
    parts = sorted({p for c in wl.bank.components for p in c.parts})
    n_root = n_part = 0
    flops_direct = 0
    for pyr in wl.pyramids:
        L = len(pyr.levels)
        for l in range(pyr.octave, L):
            lv = pyr.levels[l]
            for k in roots:
                h, w = shapes[k]
                if lv.rows >= h and lv.cols >= w:
                    n = (lv.rows - h + 1) * (lv.cols - w + 1)
                    n_root += n
                    flops_direct += 2 * n * h * w * N_CHANNELS
            pl = pyr.levels[l - pyr.octave]
            for k in parts:
                h, w = shapes[k]
                if pl.rows >= h and pl.cols >= w:
                    n = (pl.rows - h + 1) * (pl.cols - w + 1)
                    n_part += n
                    flops_direct += 2 * n * h * w * N_CHANNELS
    return {"root": n_root, "part": n_part, "total": n_root + n_part,
            "flops_direct": flops_direct}
