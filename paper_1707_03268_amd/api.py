"""Python binding of libdpmt: argument marshalling over the C ABI.

Every step of the scoring path runs in the library's HIP kernels; this module
only converts numpy arrays and torch tensors into the pointers and structs the
C ABI takes.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_void_p
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _abi


class DpmtError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{message} (status {status})")


def _lib():
    return _abi.load()


def _check(status: int, ctx=None, what: str = "") -> None:
    if status != _abi.DPMT_OK:
        lib = _lib()
        detail = lib.dpmt_last_error(ctx)
        detail = detail.decode() if detail else ""
        name = lib.dpmt_status_string(status).decode()
        raise DpmtError(status, f"{what}: {name}: {detail}")


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, dtype, name: str) -> int:
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


@dataclass
class Layout:
    """Output layout of a plan (copied out of the context-owned dpmt_layout)."""
    n_score: int
    n_offsets: int
    n_maps: int
    map_image: np.ndarray
    map_level: np.ndarray
    map_comp: np.ndarray
    map_rows: np.ndarray
    map_cols: np.ndarray
    map_score_off: np.ndarray
    map_offs_off: np.ndarray
    n_cells: int
    n_resp: int
    n_resp_root: int
    n_resp_part: int
    workspace_bytes: int

    @staticmethod
    def from_c(lay: _abi.Layout) -> "Layout":
        n = lay.n_maps

        def arr(p, dt):
            return np.ctypeslib.as_array(p, shape=(n,)).astype(dt).copy() if n else np.zeros(0, dt)
        return Layout(lay.n_score, lay.n_offsets, n, arr(lay.map_image, np.int32),
                      arr(lay.map_level, np.int32), arr(lay.map_comp, np.int32),
                      arr(lay.map_rows, np.int32), arr(lay.map_cols, np.int32),
                      arr(lay.map_score_off, np.int64), arr(lay.map_offs_off, np.int64),
                      lay.n_cells, lay.n_resp, lay.n_resp_root, lay.n_resp_part,
                      lay.workspace_bytes)

    def find(self, image: int, level: int, comp: int) -> int:
        hit = np.nonzero((self.map_image == image) & (self.map_level == level) & (self.map_comp == comp))[0]
        if len(hit) != 1:
            raise KeyError((image, level, comp))
        return int(hit[0])


class Context:
    """A libdpmt context on one HIP device (``device=-1``: host-only, can load,
    decompose and plan but not score)."""

    def __init__(self, device: int = 0, stream=None):
        lib = _lib()
        h = c_void_p()
        sp = None
        if device >= 0 and stream is not None:
            sp = _stream_ptr(stream)
        _check(lib.dpmt_create(byref(h), int(device), sp), None, "dpmt_create")
        self._h = h
        self.device = device
        self.layout: Optional[Layout] = None
        self.n_filters = 0

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib().dpmt_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- bank
    def load_filters(self, filters: Sequence[np.ndarray], components) -> None:
        """filters: list of (h, w, 32) float32 arrays; components: objects with
        ``root``, ``parts``, ``anchors`` ((n, 2) int) and ``deform`` ((n, 4) float)."""
        shapes = (_abi.Shape * len(filters))()
        flat = []
        for k, f in enumerate(filters):
            f = np.asarray(f, dtype=np.float32)
            if f.ndim != 3 or f.shape[2] != 32:
                raise ValueError(f"filter {k} must be (h, w, 32)")
            shapes[k].h, shapes[k].w = f.shape[0], f.shape[1]
            flat.append(np.ascontiguousarray(f).ravel())
        weights = np.ascontiguousarray(np.concatenate(flat)) if flat else np.zeros(0, np.float32)
        comps = (_abi.Component * len(components))()
        keep = []
        for i, c in enumerate(components):
            parts = np.ascontiguousarray(np.asarray(c.parts, dtype=np.int32))
            anchors = np.ascontiguousarray(np.asarray(c.anchors, dtype=np.int32).reshape(-1, 2))
            deform = np.ascontiguousarray(np.asarray(c.deform, dtype=np.float32).reshape(-1, 4))
            keep += [parts, anchors, deform]
            comps[i].root = int(c.root)
            comps[i].n_parts = len(parts)
            comps[i].parts = parts.ctypes.data_as(POINTER(c_int32))
            comps[i].anchors = anchors.ctypes.data_as(POINTER(c_int32))
            comps[i].deform = deform.ctypes.data_as(POINTER(c_float))
        _check(_lib().dpmt_load_filters(self._h, len(filters), shapes,
                                        weights.ctypes.data_as(POINTER(c_float)),
                                        len(components), comps), self._h, "dpmt_load_filters")
        self.n_filters = len(filters)
        self.layout = None

    def decompose(self, rank: int):
        """Returns (sigma[32], U_R (32, rank)) in float64."""
        sigma = np.zeros(32, np.float64)
        basis = np.zeros((32, max(int(rank), 1)), np.float64)
        _check(_lib().dpmt_decompose(self._h, int(rank), sigma.ctypes.data_as(POINTER(c_double)),
                                     basis.ctypes.data_as(POINTER(c_double))), self._h,
               "dpmt_decompose")
        return sigma, basis

    # -------------------------------------------------- per-filter CP form
    def _ranks(self, ranks) -> np.ndarray:
        r = np.asarray(ranks, dtype=np.int32).reshape(-1)
        if r.size == 1 and self.n_filters > 1:
            r = np.full(self.n_filters, int(r[0]), np.int32)
        if r.size != self.n_filters and self.n_filters > 0:
            raise ValueError(f"need {self.n_filters} ranks, got {r.size}")
        return np.ascontiguousarray(r)

    def decompose_cp(self, ranks, max_iters: int = 100, tol: float = 1e-6) -> np.ndarray:
        """Fit every filter's rank-R_k CP form by ALS (FP64, on the host).
        ``ranks``: one rank for all filters or one per filter.  Returns the
        relative Frobenius error per filter."""
        r = self._ranks(ranks)
        err = np.zeros(self.n_filters, np.float64)
        _check(_lib().dpmt_decompose_cp(self._h, r.ctypes.data_as(POINTER(c_int32)), int(max_iters),
                                        float(tol), err.ctypes.data_as(POINTER(c_double))),
               self._h, "dpmt_decompose_cp")
        return err

    def select_ranks(self, e: float, r_max: int = 32, max_iters: int = 200):
        """Per-filter ranks by the Section 4 criterion (binary search), fitted
        and kept as the CP factors.  Returns (ranks, relative errors)."""
        ranks = np.zeros(max(self.n_filters, 1), np.int32)
        err = np.zeros(max(self.n_filters, 1), np.float64)
        _check(_lib().dpmt_select_ranks(self._h, float(e), int(r_max), int(max_iters),
                                        ranks.ctypes.data_as(POINTER(c_int32)),
                                        err.ctypes.data_as(POINTER(c_double))), self._h,
               "dpmt_select_ranks")
        return ranks[:self.n_filters], err[:self.n_filters]

    def load_cp(self, ranks, factors) -> None:
        """factors: per filter (A (h, R), B (w, R), C (32, R))."""
        r = self._ranks(ranks)
        flat = np.ascontiguousarray(np.concatenate(
            [np.asarray(m, np.float32).ravel() for abc in factors for m in abc]) if len(factors)
            else np.zeros(0, np.float32))
        _check(_lib().dpmt_load_cp(self._h, r.ctypes.data_as(POINTER(c_int32)),
                                   flat.ctypes.data_as(POINTER(c_float))), self._h, "dpmt_load_cp")

    def get_cp(self, shapes):
        """Current CP factors as (ranks, [(A, B, C)]) for filters of the given
        (h, w) shapes (float32 arrays)."""
        n = c_int64(0)
        _check(_lib().dpmt_get_cp(self._h, None, None, byref(n)), self._h, "dpmt_get_cp")
        ranks = np.zeros(self.n_filters, np.int32)
        flat = np.zeros(max(n.value, 1), np.float32)
        _check(_lib().dpmt_get_cp(self._h, ranks.ctypes.data_as(POINTER(c_int32)),
                                  flat.ctypes.data_as(POINTER(c_float)), byref(n)), self._h, "dpmt_get_cp")
        out, o = [], 0
        for (h, w), R in zip(shapes, ranks):
            A = flat[o:o + h * R].reshape(h, R); o += h * R
            B = flat[o:o + w * R].reshape(w, R); o += w * R
            C = flat[o:o + 32 * R].reshape(32, R); o += 32 * R
            out.append((A.copy(), B.copy(), C.copy()))
        return ranks, out

    # ------------------------------------------------ convolution shortening
    def set_thresholds(self, thresholds) -> None:
        """Per-filter thresholds t_1..t_R (list of arrays in filter order, or
        one flat array); None clears them."""
        if thresholds is None:
            _check(_lib().dpmt_set_thresholds(self._h, None), self._h, "dpmt_set_thresholds")
            return
        if not isinstance(thresholds, np.ndarray):
            thresholds = np.concatenate([np.asarray(t, np.float32).ravel() for t in thresholds])
        flat = np.ascontiguousarray(thresholds, dtype=np.float32)
        _check(_lib().dpmt_set_thresholds(self._h, flat.ctypes.data_as(POINTER(c_float))), self._h,
               "dpmt_set_thresholds")

    def fit_thresholds(self, features: np.ndarray, positives, margin: float = 1e-4) -> np.ndarray:
        """Thresholds from positives ((image, level, comp, y, x) tuples) over the
        host feature buffer; sets and returns them (flat, filter order)."""
        feats = np.ascontiguousarray(features, dtype=np.float32)
        hyp = (_abi.Hypothesis * max(len(positives), 1))()
        for i, g in enumerate(positives):
            hyp[i].image, hyp[i].level, hyp[i].comp, hyp[i].y, hyp[i].x = (int(v) for v in g)
        n = c_int64(0)
        _check(_lib().dpmt_get_cp(self._h, None, None, byref(n)), self._h, "dpmt_get_cp")
        ranks = np.zeros(max(self.n_filters, 1), np.int32)
        _check(_lib().dpmt_get_cp(self._h, ranks.ctypes.data_as(POINTER(c_int32)), None, byref(n)),
               self._h, "dpmt_get_cp")
        out = np.zeros(max(int(ranks[:self.n_filters].sum()), 1), np.float32)
        _check(_lib().dpmt_fit_thresholds(self._h, feats.ctypes.data_as(POINTER(c_float)), len(positives),
                                          hyp, float(margin), out.ctypes.data_as(POINTER(c_float))),
               self._h, "dpmt_fit_thresholds")
        return out[:int(ranks[:self.n_filters].sum())]

    def plan(self, pyramids) -> Layout:
        """pyramids: objects with ``levels`` (each with cell_offset, rows, cols) and ``octave``."""
        arrs = []
        pyrs = (_abi.PyramidDesc * len(pyramids))()
        for i, p in enumerate(pyramids):
            lv = (_abi.LevelDesc * len(p.levels))()
            for l, L in enumerate(p.levels):
                lv[l].cell_offset, lv[l].rows, lv[l].cols = int(L.cell_offset), int(L.rows), int(L.cols)
            arrs.append(lv)
            pyrs[i].n_levels = len(p.levels)
            pyrs[i].levels = ctypes.cast(lv, POINTER(_abi.LevelDesc))
            pyrs[i].octave = int(p.octave)
        out = POINTER(_abi.Layout)()
        _check(_lib().dpmt_plan(self._h, len(pyramids), pyrs, byref(out)), self._h, "dpmt_plan")
        self.layout = Layout.from_c(out.contents)
        return self.layout

    # -------------------------------------------------------------- scoring
    def score_pyramid(self, mode, features, scores, offsets=None, stream=None) -> None:
        """Enqueue the scoring of the planned batch on ``stream`` (default: torch's current)."""
        import torch
        m = _abi.MODES[mode] if isinstance(mode, str) else int(mode)
        _check(_lib().dpmt_score_pyramid(
            self._h, m, _dev_ptr(features, torch.float32, "features"),
            _dev_ptr(scores, torch.float32, "scores"),
            _dev_ptr(offsets, torch.int16, "offsets") if offsets is not None else None,
            _stream_ptr(stream)), self._h, "dpmt_score_pyramid")

    def level_responses(self, mode, features, image: int, level: int, out=None, stream=None):
        """Per-filter response maps of every filter on one level.  Returns
        (flat float32 tensor, [(offset, rows, cols) or None per filter])."""
        import torch
        m = _abi.MODES[mode] if isinstance(mode, str) else int(mode)
        n = c_int64(0)
        fp = _dev_ptr(features, torch.float32, "features")
        if out is None:
            _check(_lib().dpmt_level_responses(self._h, m, fp, int(image), int(level), None, 0,
                                               byref(n), _stream_ptr(stream)),
                   self._h, "dpmt_level_responses")
            out = torch.empty(max(n.value, 1), dtype=torch.float32, device=features.device)
        _check(_lib().dpmt_level_responses(self._h, m, fp, int(image), int(level),
                                           _dev_ptr(out, torch.float32, "out"), out.numel(),
                                           byref(n), _stream_ptr(stream)),
               self._h, "dpmt_level_responses")
        return out, n.value

    def detect(self, scores, tau: float, capacity: Optional[int] = None, stream=None):
        """Detection set (score >= tau) of the planned maps from ``scores``.
        Returns (records int32 tensor (n, 4) = (map, y, x, score bits),
        scores float32 tensor (n,), count) with n = min(count, capacity)."""
        import torch
        if capacity is None:
            capacity = max(self.layout.n_score, 1)
        rec = torch.empty((max(int(capacity), 1), 4), dtype=torch.int32, device=scores.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=scores.device)
        _check(_lib().dpmt_detect(self._h, _dev_ptr(scores, torch.float32, "scores"), float(tau),
                                  rec.data_ptr(), int(capacity), cnt.data_ptr(), _stream_ptr(stream)),
               self._h, "dpmt_detect")
        n = int(cnt.item())
        m = min(n, int(capacity))
        rec = rec[:m]
        return rec, rec[:, 3].contiguous().view(torch.float32), n

    def detect_into(self, scores, tau: float, records, count, stream=None) -> None:
        """Enqueue dpmt_detect into caller buffers without waiting: ``records``
        an int32 CUDA tensor of shape (capacity, 4), ``count`` an int64 CUDA
        tensor of at least one element (receives the full count)."""
        import torch
        if records.dim() != 2 or records.shape[1] != 4:
            raise ValueError("records must have shape (capacity, 4)")
        _check(_lib().dpmt_detect(self._h, _dev_ptr(scores, torch.float32, "scores"), float(tau),
                                  _dev_ptr(records, torch.int32, "records"), int(records.shape[0]),
                                  _dev_ptr(count, torch.int64, "count"), _stream_ptr(stream)),
               self._h, "dpmt_detect")

    # ------------------------------------------------------ HOG features
    def hog_pyramid(self, image, levels, features, stream=None) -> None:
        """Enqueue dpmt_hog_pyramid: ``image`` a uint8 CUDA tensor (H, W, 3),
        ``levels`` a sequence of (cell_offset, rows, cols, pad_rows, pad_cols,
        cell, inv_scale) tuples, ``features`` a float32 CUDA tensor holding
        every level's cells (32 floats per cell)."""
        import torch
        if image.dim() != 3 or image.shape[2] != 3:
            raise ValueError("image must have shape (H, W, 3)")
        n = len(levels)
        arr = (_abi.HogLevel * max(n, 1))()
        for k, lv in enumerate(levels):
            off, rows, cols, pr, pc, cell, inv = lv
            arr[k] = _abi.HogLevel(int(off), int(rows), int(cols), int(pr), int(pc), int(cell), float(inv))
        _check(_lib().dpmt_hog_pyramid(self._h, _dev_ptr(image, torch.uint8, "image"), int(image.shape[0]),
                                       int(image.shape[1]), n, arr,
                                       _dev_ptr(features, torch.float32, "features"), _stream_ptr(stream)),
               self._h, "dpmt_hog_pyramid")

    # ------------------------------------------------------ launch strategy
    def set_launch(self, launch) -> None:
        """'batched' (default), 'per_level' or 'graph' (see dpmt_launch)."""
        v = _abi.LAUNCHES[launch] if isinstance(launch, str) else int(launch)
        _check(_lib().dpmt_set_launch(self._h, v), self._h, "dpmt_set_launch")

    def set_tile_config(self, mode, config: int) -> None:
        m = _abi.MODES[mode] if isinstance(mode, str) else int(mode)
        _check(_lib().dpmt_set_tile_config(self._h, m, int(config)), self._h, "dpmt_set_tile_config")

    def get_tile_config(self, mode) -> int:
        m = _abi.MODES[mode] if isinstance(mode, str) else int(mode)
        return int(_lib().dpmt_get_tile_config(self._h, m))

    def autotune(self, mode, features, scores, offsets=None, reps: int = 5, stream=None):
        """Time every tile configuration on the planned batch and keep the
        fastest for ``mode``.  Returns (best index, [median ms or None])."""
        import torch
        m = _abi.MODES[mode] if isinstance(mode, str) else int(mode)
        n = tile_config_count()
        ms = (c_float * n)()
        best = c_int32(-1)
        _check(_lib().dpmt_autotune(
            self._h, m, _dev_ptr(features, torch.float32, "features"),
            _dev_ptr(scores, torch.float32, "scores"),
            _dev_ptr(offsets, torch.int16, "offsets") if offsets is not None else None,
            int(reps), ms, byref(best), _stream_ptr(stream)), self._h, "dpmt_autotune")
        return best.value, [ms[i] if ms[i] >= 0 else None for i in range(n)]

    def set_profiling(self, on: bool) -> None:
        _check(_lib().dpmt_set_profiling(self._h, 1 if on else 0), self._h, "dpmt_set_profiling")

    STAGES = ("projection", "correlation", "placement", "total")

    def stage_times(self):
        """Mean GPU milliseconds per profiled call of each stage, and the call count."""
        buf = (c_float * len(self.STAGES))()
        calls = c_int32(0)
        n = _lib().dpmt_stage_times(self._h, buf, len(self.STAGES), byref(calls))
        return {self.STAGES[i]: buf[i] for i in range(n)}, calls.value


def tile_config_count() -> int:
    return int(_lib().dpmt_tile_config_count())


def tile_config_name(config: int) -> Optional[str]:
    r = _lib().dpmt_tile_config_name(int(config))
    return r.decode() if r is not None else None


def distance_transform(resp, deform, out=None, arg_y=None, arg_x=None, stream=None, noalloc=False,
                       method: str = "window"):
    """Generalised distance transform of one 2D float32 CUDA map for every
    target cell; returns (D, arg_y, arg_x).  noalloc: call
    dpmt_distance_transform_noalloc (the library's static scratch, no
    allocation inside the call; outputs must then be given).  method:
    "window" (windowed scans) or "envelope" (lower envelopes, through
    dpmt_distance_transform_method)."""
    import torch
    if resp.dim() != 2:
        raise ValueError("resp must be 2D")
    rows, cols = resp.shape
    ld = resp.stride(0)
    if resp.stride(1) != 1:
        raise ValueError("resp rows must be contiguous")
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, device=resp.device)
    if arg_y is None:
        arg_y = torch.empty((rows, cols), dtype=torch.int32, device=resp.device)
    if arg_x is None:
        arg_x = torch.empty((rows, cols), dtype=torch.int32, device=resp.device)
    d = (c_float * 4)(*[float(v) for v in deform])
    if not resp.is_cuda or resp.dtype != torch.float32:
        raise TypeError("resp must be a float32 CUDA tensor")
    if method not in _abi.DT_METHODS:
        raise ValueError(f"method must be one of {sorted(_abi.DT_METHODS)}")
    ptrs = (c_void_p(resp.data_ptr()), rows, cols, ld, d, _dev_ptr(out, torch.float32, "out"),
            _dev_ptr(arg_y, torch.int32, "arg_y"), _dev_ptr(arg_x, torch.int32, "arg_x"))
    if method != "window":
        if noalloc:
            raise ValueError("the allocation-free transform uses windowed scans")
        _check(_lib().dpmt_distance_transform_method(*ptrs, _abi.DT_METHODS[method], _stream_ptr(stream)),
               None, "dpmt_distance_transform_method")
        return out, arg_y, arg_x
    fn = _lib().dpmt_distance_transform_noalloc if noalloc else _lib().dpmt_distance_transform
    _check(fn(*ptrs, _stream_ptr(stream)), None,
           "dpmt_distance_transform_noalloc" if noalloc else "dpmt_distance_transform")
    return out, arg_y, arg_x
