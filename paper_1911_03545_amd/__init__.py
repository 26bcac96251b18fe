"""MI355X (gfx950) binned pair counting -- Python binding of ``libpaircount.so``.

The library counts pairs of points in separation bins as defined by Sinha &
Garrison (Corrfunc, arXiv:1911.03545): DD(r), DD(rp, pi) / wp(rp) and
DD(theta) / DR(theta), autocorrelations and cross-correlations, periodic or
not, optionally weighted by the product of point weights.  Every step of the
computation runs in the library's HIP kernels; this module only marshals
arguments (NumPy arrays stay in host memory, torch CUDA tensors are passed by
device pointer) and converts status codes into exceptions.

The shared library is built in-tree with ``python -m paper_1911_03545_amd.build``.
There is no CPU fallback: without the library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaircount.so")

CF_OK, CF_EINVAL, CF_ERANGE, CF_ENOMEM, CF_EDEVICE, CF_EUNSUPPORTED, CF_EOVERFLOW = (
    0, -1, -2, -3, -4, -5, -6)
CF_F32, CF_F64 = 1, 2
CF_MEM_HOST, CF_MEM_DEVICE = 0, 1
CF_PREC_FP64, CF_PREC_FP32_RECHECK = 0, 1

STATUS_NAMES = {
    CF_OK: "CF_OK", CF_EINVAL: "CF_EINVAL", CF_ERANGE: "CF_ERANGE",
    CF_ENOMEM: "CF_ENOMEM", CF_EDEVICE: "CF_EDEVICE",
    CF_EUNSUPPORTED: "CF_EUNSUPPORTED", CF_EOVERFLOW: "CF_EOVERFLOW",
}

EXPORTED_SYMBOLS = (
    "cf_create", "cf_destroy", "cf_set_allocator", "cf_last_error", "cf_get_stats",
    "cf_default_options",
    "count_pairs_r", "count_pairs_r_ex", "count_pairs_r_noalloc", "count_pairs_rppi",
    "count_pairs_rppi_ex",
    "count_pairs_theta", "count_pairs_theta_ex", "count_pairs_rppi_batch",
    "count_pairs_rppi_batch_ex", "count_pairs_rppi_mocks", "count_pairs_rppi_mocks_ex",
    "cf_plan_grid", "cf_plan_grid_ex", "cf_plan_sky_grid", "cf_fp32_bands",
    "cf_fp32_bands_axes", "cf_fp32_bands_xy", "cf_fp32_pair_margin",
    "cf_fixed_sum",
)


class cf_catalog(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("wdtype", ctypes.c_int32), ("mem", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("w", ctypes.c_void_p)]


CF_WEIGHT_PRODUCT, CF_WEIGHT_SUM = 0, 1
WEIGHT_TYPES = {"product": CF_WEIGHT_PRODUCT, "sum": CF_WEIGHT_SUM}


class cf_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("slices_per_reach", ctypes.c_int32),
                ("chunk", ctypes.c_int32),
                ("output_on_device", ctypes.c_int32), ("theta_unit_vectors", ctypes.c_int32),
                ("collect_timing", ctypes.c_int32), ("hist_copies", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("weight_type", ctypes.c_int32), ("angular_grid", ctypes.c_int32),
                ("xy_refine", ctypes.c_int32), ("radec_on_device", ctypes.c_int32),
                ("flush_pairs", ctypes.c_int32), ("deterministic_weights", ctypes.c_int32),
                ("separation_form", ctypes.c_int32),
                ("ravg", ctypes.c_void_p)]


class cf_stats(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32 * 3), ("zreach", ctypes.c_int32),
                ("cell_width", ctypes.c_double * 3), ("n_blocks", ctypes.c_int64),
                ("n_items", ctypes.c_int64), ("candidate_pairs", ctypes.c_uint64),
                ("rechecks", ctypes.c_uint64),
                ("sweep_workgroups", ctypes.c_int32), ("hist_copies", ctypes.c_int32),
                ("t_prepare_ms", ctypes.c_float), ("t_grid_ms", ctypes.c_float),
                ("t_worklist_ms", ctypes.c_float), ("t_sweep_ms", ctypes.c_float),
                ("t_finalize_ms", ctypes.c_float),
                ("t_total_ms", ctypes.c_float),
                ("slices_per_reach", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("replayed", ctypes.c_int32), ("angular_grid", ctypes.c_int32),
                ("xy_refine", ctypes.c_int32), ("separation_form", ctypes.c_int32),
                ("flushes", ctypes.c_uint64)]


class cf_grid_plan(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("extent", ctypes.c_double * 3),
                ("inv_width", ctypes.c_double * 3), ("width", ctypes.c_double * 3),
                ("n", ctypes.c_int32 * 3), ("zreach", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("boxsize", ctypes.c_double), ("ncell", ctypes.c_int64)]


class cf_sky_band(ctypes.Structure):
    _fields_ = [("col0", ctypes.c_int32), ("nra", ctypes.c_int32),
                ("ra_scale", ctypes.c_double), ("dra", ctypes.c_double * 3)]


class cf_sky_plan(ctypes.Structure):
    _fields_ = [("nband", ctypes.c_int32), ("ncol", ctypes.c_int32),
                ("slices", ctypes.c_int32), ("zreach", ctypes.c_int32),
                ("dec_lo", ctypes.c_double), ("band_height", ctypes.c_double),
                ("inv_slice", ctypes.c_double), ("theta_reach", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class PairCountError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpaircount.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library with "
            "'python -m paper_1911_03545_amd.build' (there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes the library bind to that single runtime, so
    # both share one device context (loading the system runtime first leaves
    # torch without a usable GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    cat = ctypes.POINTER(cf_catalog)
    lib.cf_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.cf_create.restype = ctypes.c_int
    lib.cf_destroy.argtypes = [vp]
    lib.cf_destroy.restype = ctypes.c_int
    lib.cf_last_error.argtypes = [vp]
    lib.cf_last_error.restype = ctypes.c_char_p
    lib.cf_get_stats.argtypes = [vp, ctypes.POINTER(cf_stats)]
    lib.cf_get_stats.restype = ctypes.c_int
    lib.cf_default_options.argtypes = [ctypes.POINTER(cf_options)]
    lib.cf_default_options.restype = None
    for name in ("count_pairs_r", "count_pairs_r_ex", "count_pairs_r_noalloc"):
        f = getattr(lib, name)
        f.argtypes = [vp, cat, cat, vp, i32, dbl, ctypes.c_int, vp, vp] + (
            [] if name == "count_pairs_r" else [ctypes.POINTER(cf_options)])
        f.restype = ctypes.c_int
    for name in ("count_pairs_rppi", "count_pairs_rppi_ex"):
        f = getattr(lib, name)
        f.argtypes = [vp, cat, cat, vp, i32, dbl, i32, dbl, ctypes.c_int, vp, vp] + (
            [ctypes.POINTER(cf_options)] if name.endswith("_ex") else [])
        f.restype = ctypes.c_int
    for name in ("count_pairs_rppi_mocks", "count_pairs_rppi_mocks_ex"):
        f = getattr(lib, name)
        f.argtypes = [vp, cat, cat, vp, i32, dbl, i32, ctypes.c_int, vp, vp] + (
            [ctypes.POINTER(cf_options)] if name.endswith("_ex") else [])
        f.restype = ctypes.c_int
    for name in ("count_pairs_theta", "count_pairs_theta_ex"):
        f = getattr(lib, name)
        f.argtypes = [vp, cat, cat, vp, i32, ctypes.c_int, vp, vp] + (
            [ctypes.POINTER(cf_options)] if name.endswith("_ex") else [])
        f.restype = ctypes.c_int
    for name, ex in (("count_pairs_rppi_batch", False), ("count_pairs_rppi_batch_ex", True)):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i32, vp, i32, dbl, i32, dbl, ctypes.c_int, vp, vp] + (
            [ctypes.POINTER(cf_options)] if ex else [])
        f.restype = ctypes.c_int
    lib.cf_plan_grid.argtypes = [vp, vp, dbl, dbl, dbl, i32, ctypes.POINTER(cf_grid_plan)]
    lib.cf_plan_grid.restype = ctypes.c_int
    lib.cf_plan_grid_ex.argtypes = [vp, vp, dbl, dbl, dbl, i32, i32, i32,
                                    ctypes.POINTER(cf_grid_plan), vp, vp]
    lib.cf_plan_grid_ex.restype = ctypes.c_int
    lib.cf_set_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp]
    lib.cf_set_allocator.restype = ctypes.c_int
    lib.cf_plan_sky_grid.argtypes = [dbl, dbl, dbl, i32, i32, ctypes.POINTER(cf_sky_plan),
                                     vp, i32]
    lib.cf_plan_sky_grid.restype = ctypes.c_int
    lib.cf_fp32_bands.argtypes = [vp, i32, i32, dbl, vp, vp]
    lib.cf_fp32_bands.restype = ctypes.c_int
    lib.cf_fp32_bands_axes.argtypes = [vp, i32, i32, vp, dbl, vp, vp]
    lib.cf_fp32_bands_axes.restype = ctypes.c_int
    lib.cf_fp32_bands_xy.argtypes = [vp, i32, i32, vp, vp, dbl, vp, vp]
    lib.cf_fp32_bands_xy.restype = ctypes.c_int
    lib.cf_fp32_pair_margin.argtypes = [vp, i32, dbl, vp, vp]
    lib.cf_fp32_pair_margin.restype = ctypes.c_int
    lib.cf_fixed_sum.argtypes = [vp, ctypes.c_int64, i32, vp]
    lib.cf_fixed_sum.restype = ctypes.c_int
    _lib = lib
    return lib


def default_options(**overrides) -> cf_options:
    lib = load_library()
    o = cf_options()
    lib.cf_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v))
    return o


def plan_grid(lo, hi, boxsize: float, reach_xy: float, reach_z: float,
              slices_per_reach: int = 8) -> dict:
    """Host-only grid plan (no device needed)."""
    lib = load_library()
    lo_a = np.ascontiguousarray(lo if lo is not None else [0, 0, 0], dtype=np.float64)
    hi_a = np.ascontiguousarray(hi if hi is not None else [0, 0, 0], dtype=np.float64)
    p = cf_grid_plan()
    st = lib.cf_plan_grid(lo_a.ctypes.data, hi_a.ctypes.data, float(boxsize), float(reach_xy),
                          float(reach_z), int(slices_per_reach), ctypes.byref(p))
    if st != CF_OK:
        raise PairCountError(st, "cf_plan_grid failed")
    return {"n": list(p.n), "width": list(p.width), "extent": list(p.extent),
            "inv_width": list(p.inv_width), "lo": list(p.lo), "zreach": p.zreach,
            "periodic": p.periodic, "ncell": p.ncell}


def plan_grid_refined(lo, hi, boxsize: float, reach_xy: float, reach_z: float,
                      slices_per_reach: int = 32, xy_refine: int = 1, ball: bool = True) -> dict:
    """Host-only grid plan with x/y refinement; adds the per-offset z windows
    ``zro`` (5 x 5, -1: offset skipped) and the refinement used ``k``."""
    lib = load_library()
    lo_a = np.ascontiguousarray(lo if lo is not None else [0, 0, 0], dtype=np.float64)
    hi_a = np.ascontiguousarray(hi if hi is not None else [0, 0, 0], dtype=np.float64)
    p = cf_grid_plan()
    zro = np.zeros(25, dtype=np.int16)
    k = ctypes.c_int32(0)
    st = lib.cf_plan_grid_ex(lo_a.ctypes.data, hi_a.ctypes.data, float(boxsize),
                             float(reach_xy), float(reach_z), int(slices_per_reach),
                             int(xy_refine), int(bool(ball)), ctypes.byref(p), zro.ctypes.data,
                             ctypes.byref(k))
    if st != CF_OK:
        raise PairCountError(st, "cf_plan_grid_ex failed")
    return {"n": list(p.n), "width": list(p.width), "extent": list(p.extent),
            "inv_width": list(p.inv_width), "lo": list(p.lo), "zreach": p.zreach,
            "periodic": p.periodic, "ncell": p.ncell, "zro": zro.reshape(5, 5).copy(),
            "k": k.value}


def plan_sky_grid(chord_reach: float, zlo: float, zhi: float, slices: int = 16,
                  ra_refine: int = 1) -> dict:
    """Host-only angular grid plan (declination bands, right-ascension cells)."""
    lib = load_library()
    p = cf_sky_plan()
    bands = (cf_sky_band * 1024)()
    st = lib.cf_plan_sky_grid(float(chord_reach), float(zlo), float(zhi), int(slices),
                              int(ra_refine), ctypes.byref(p), ctypes.addressof(bands), 1024)
    if st != CF_OK:
        raise PairCountError(st, "cf_plan_sky_grid failed")
    out = {k: getattr(p, k) for k, _ in cf_sky_plan._fields_}
    out["col0"] = np.array([bands[k].col0 for k in range(p.nband)], dtype=np.int64)
    out["nra"] = np.array([bands[k].nra for k in range(p.nband)], dtype=np.int64)
    out["ra_scale"] = np.array([bands[k].ra_scale for k in range(p.nband)])
    out["dra"] = np.array([list(bands[k].dra) for k in range(p.nband)])
    return out


def fp32_bands(edges_sq, ndim: int, coord_scale: float):
    """Host-only float32 decision bands of squared (or line-of-sight) edges."""
    lib = load_library()
    e = np.ascontiguousarray(edges_sq, dtype=np.float64)
    lo = np.zeros(e.size, dtype=np.float32)
    hi = np.zeros(e.size, dtype=np.float32)
    st = lib.cf_fp32_bands(e.ctypes.data, e.size, int(ndim), float(coord_scale),
                           lo.ctypes.data, hi.ctypes.data)
    if st != CF_OK:
        raise PairCountError(st, "cf_fp32_bands failed")
    return lo, hi


def fp32_bands_axes(edges_sq, ndim: int, axis_eps, coord_scale: float):
    """Host-only float32 decision bands with a rounding bound per axis (the
    total error of the two float32 coordinates of that axis)."""
    lib = load_library()
    e = np.ascontiguousarray(edges_sq, dtype=np.float64)
    sc = np.ascontiguousarray(axis_eps, dtype=np.float64)
    if sc.size < ndim:
        raise ValueError("one bound per axis")
    lo = np.zeros(e.size, dtype=np.float32)
    hi = np.zeros(e.size, dtype=np.float32)
    st = lib.cf_fp32_bands_axes(e.ctypes.data, e.size, int(ndim), sc.ctypes.data,
                                float(coord_scale), lo.ctypes.data, hi.ctypes.data)
    if st != CF_OK:
        raise PairCountError(st, "cf_fp32_bands_axes failed")
    return lo, hi


def fp32_bands_xy(edges_sq, axis_eps, xy_max, coord_scale: float, ndim: int = 3):
    """Host-only float32 decision bands of a 3-D grid's sweep whose x and y
    are expanded (|a|^2 + |b|^2 - 2 a.b): squared r (ndim 3) or rp (ndim 2);
    xy_max = (a_x, a_y, b_x, b_y), the largest coordinate magnitudes of the
    lane and of the j point."""
    lib = load_library()
    e = np.ascontiguousarray(edges_sq, dtype=np.float64)
    sc = np.ascontiguousarray(axis_eps, dtype=np.float64)
    mx = np.ascontiguousarray(xy_max, dtype=np.float64)
    if sc.size < ndim or mx.size < 4:
        raise ValueError("one bound per axis and four magnitudes")
    lo = np.zeros(e.size, dtype=np.float32)
    hi = np.zeros(e.size, dtype=np.float32)
    st = lib.cf_fp32_bands_xy(e.ctypes.data, e.size, int(ndim), sc.ctypes.data, mx.ctypes.data,
                              float(coord_scale), lo.ctypes.data, hi.ctypes.data)
    if st != CF_OK:
        raise PairCountError(st, "cf_fp32_bands_xy failed")
    return lo, hi


def fp32_pair_margin(xy_max, fscale: float, ndim: int = 3):
    """Host-only (K, M) of the sweep's per-pair narrowing of the expanded
    bands (float32 values): a pair with magnitude term m narrows its band by
    K (M - m) in the coordinates scaled by fscale."""
    lib = load_library()
    mx = np.ascontiguousarray(xy_max, dtype=np.float64)
    if mx.size < 4:
        raise ValueError("four magnitudes")
    K = np.zeros(1, dtype=np.float32)
    M = np.zeros(1, dtype=np.float32)
    st = lib.cf_fp32_pair_margin(mx.ctypes.data, int(ndim), float(fscale), K.ctypes.data,
                                 M.ctypes.data)
    if st != CF_OK:
        raise PairCountError(st, "cf_fp32_pair_margin failed")
    return K[0], M[0]


def fixed_sum(values, q: int) -> float:
    """Host-only exact sum of multiples of 2^q through the fixed-point
    arithmetic of the deterministic weight sums, rounded once."""
    lib = load_library()
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = ctypes.c_double(0.0)
    st = lib.cf_fixed_sum(v.ctypes.data if v.size else None, v.size, int(q), ctypes.byref(out))
    if st != CF_OK:
        raise PairCountError(st, "cf_fixed_sum failed")
    return out.value


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Cat:
    """Marshal one catalogue; keeps referenced buffers alive."""

    def __init__(self, pts, w=None, two_columns: bool = False):
        self.keep = []
        if isinstance(pts, (tuple, list)):
            cols = list(pts)
        else:
            if _is_torch(pts):
                ncol = pts.shape[1]
                cols = [pts[:, k].contiguous() for k in range(ncol)]
            else:
                arr = np.asarray(pts)
                if arr.ndim != 2:
                    raise ValueError("positions must be (n, 3) or a tuple of columns")
                cols = [np.ascontiguousarray(arr[:, k]) for k in range(arr.shape[1])]
        need = 2 if two_columns else 3
        if len(cols) < need:
            raise ValueError(f"need {need} coordinate columns")
        c = cf_catalog()
        dev = _is_torch(cols[0]) and cols[0].is_cuda
        c.mem = CF_MEM_DEVICE if dev else CF_MEM_HOST
        ptrs = []
        dts = set()
        for col in cols[:3]:
            p, dt, n = self._ptr(col, dev)
            ptrs.append(p)
            dts.add(dt)
            c.n = n
        if len(dts) != 1:
            raise ValueError("coordinate columns must share one dtype")
        c.dtype = dts.pop()
        c.x, c.y = ptrs[0], ptrs[1]
        c.z = ptrs[2] if len(ptrs) > 2 else None
        if w is not None:
            if _is_torch(w) != dev:
                raise ValueError("weights must live where the coordinates live")
            p, dt, n = self._ptr(w, dev)
            if n != c.n:
                raise ValueError("weights and positions differ in length")
            c.w, c.wdtype = p, dt
        self.c = c

    def _ptr(self, col, dev):
        if dev:
            import torch
            if not col.is_contiguous():
                col = col.contiguous()
            if col.dtype == torch.float32:
                dt = CF_F32
            elif col.dtype == torch.float64:
                dt = CF_F64
            else:
                raise TypeError("coordinates must be float32 or float64")
            self.keep.append(col)
            return col.data_ptr(), dt, col.numel()
        a = np.asarray(col)
        if a.dtype == np.float32:
            dt = CF_F32
        elif a.dtype == np.float64:
            dt = CF_F64
        else:
            a = a.astype(np.float64)
            dt = CF_F64
        a = np.ascontiguousarray(a)
        self.keep.append(a)
        return a.ctypes.data, dt, a.size


class PairCounter:
    """A library context bound to one device and one HIP stream.

    ``stream``: a HIP stream handle (int) or a torch.cuda.Stream; by default
    torch's current stream on ``device`` when torch is importable, else the
    null stream.
    """

    def __init__(self, device: int = 0, stream=None):
        self._lib = load_library()
        handle = None
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    handle = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                handle = None
        elif hasattr(stream, "cuda_stream"):
            handle = stream.cuda_stream
        else:
            handle = int(stream)
        ctx = ctypes.c_void_p()
        st = self._lib.cf_create(int(device), handle, ctypes.byref(ctx))
        if st != CF_OK:
            msg = self._lib.cf_last_error(None)
            raise PairCountError(st, f"cf_create(device={device}): "
                                     f"{msg.decode() if msg else ''}")
        self._ctx = ctx
        self._device = int(device)
        self._stream_handle = handle
        self._alloc_cbs = None

    def set_allocator(self, alloc=None, free=None):
        """Route the context's device scratch through ``alloc(nbytes) -> int``
        (a device pointer, 256-byte aligned) and ``free(ptr)``; both None
        restores hipMalloc / hipFree."""
        if (alloc is None) != (free is None):
            raise ValueError("give both alloc and free, or neither")
        if alloc is None:
            st = self._lib.cf_set_allocator(self._ctx, ALLOC_FN(), FREE_FN(), None)
            self._check(st)
            self._alloc_cbs = None
            return
        a = ALLOC_FN(lambda n, user: int(alloc(int(n))) or None)
        f = FREE_FN(lambda p, user: free(int(p)))
        st = self._lib.cf_set_allocator(self._ctx, a, f, None)
        self._check(st)
        self._alloc_cbs = (a, f)   # kept alive while the library may call them

    def use_torch_allocator(self):
        """Take device scratch from torch's caching allocator on this
        context's device and stream (it then shows in
        torch.cuda.memory_allocated and is reused across contexts)."""
        import torch
        dev, stream = self._device, self._stream_handle or 0
        self.set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, stream),
                           torch.cuda.caching_allocator_delete)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.cf_destroy(self._ctx)
            self._ctx = None
        self._alloc_cbs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != CF_OK:
            msg = self._lib.cf_last_error(self._ctx)
            raise PairCountError(st, msg.decode() if msg else "")

    @staticmethod
    def _prec(precision):
        if precision in ("fp64", CF_PREC_FP64):
            return CF_PREC_FP64
        if precision in ("fp32", "fp32_recheck", CF_PREC_FP32_RECHECK):
            return CF_PREC_FP32_RECHECK
        raise ValueError(f"unknown precision {precision!r}")

    def _opts(self, options, weight_type=None, ravg=None, **fixed):
        """cf_options for a call (None: library defaults).  ``ravg`` is the
        float64 host array that receives the mean separations."""
        if options is None and weight_type is None and ravg is None and not fixed:
            return None
        if isinstance(options, cf_options):
            o = cf_options.from_buffer_copy(options)
        else:
            o = default_options(**(options or {}))
        for k, v in fixed.items():
            setattr(o, k, int(v))
        if weight_type is not None:
            if weight_type not in WEIGHT_TYPES:
                raise ValueError(f"unknown weight_type {weight_type!r}")
            o.weight_type = WEIGHT_TYPES[weight_type]
        o.ravg = None if ravg is None else ravg.ctypes.data
        self._last_opts = o   # keep alive for the call
        return ctypes.byref(o)

    @staticmethod
    def _result(counts, wsum, rv, shape):
        counts = counts.reshape(shape)
        if wsum is not None:
            wsum = wsum.reshape(shape)
        if rv is not None:
            return counts, wsum, rv.reshape(shape)
        return counts, wsum

    def count_r(self, d1, d2=None, edges=None, boxsize: float = 0.0, precision="fp64",
                w1=None, w2=None, options=None, weight_type=None, ravg=False):
        """DD(r): returns (counts uint64[nb], wsum float64[nb] or None), plus
        the mean separation per bin (float64[nb]) when ``ravg``."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        nb = e.size - 1
        c1 = _Cat(d1, w1)
        c2 = None if d2 is None else _Cat(d2, w2 if w2 is not None else None)
        counts = np.zeros(nb, dtype=np.uint64)
        wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
        rv = np.zeros(nb, dtype=np.float64) if ravg else None
        st = self._lib.count_pairs_r_ex(
            self._ctx, ctypes.byref(c1.c), None if c2 is None else ctypes.byref(c2.c),
            e.ctypes.data, nb, float(boxsize), self._prec(precision), counts.ctypes.data,
            None if wsum is None else wsum.ctypes.data, self._opts(options, weight_type, rv))
        self._check(st)
        return self._result(counts, wsum, rv, (nb,))

    def count_r_noalloc(self, d1, d2=None, edges=None, boxsize: float = 0.0,
                        precision="fp64", w1=None, w2=None, options=None, counts_out=None,
                        wsum_out=None):
        """DD(r) through count_pairs_r_noalloc (no device allocation: every
        buffer comes from the library's fixed per-GPU scratch).  With
        ``counts_out`` (and ``wsum_out``) torch CUDA tensors the outputs stay
        on the device (output_on_device) and are returned as given; otherwise
        returns host arrays like :meth:`count_r`."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        nb = e.size - 1
        c1 = _Cat(d1, w1)
        c2 = None if d2 is None else _Cat(d2, w2)
        fixed = {}
        if counts_out is not None:
            fixed["output_on_device"] = 1
            counts, cp = counts_out, counts_out.data_ptr()
            wsum = wsum_out
            wp = None if wsum_out is None else wsum_out.data_ptr()
        else:
            counts = np.zeros(nb, dtype=np.uint64)
            wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
            cp, wp = counts.ctypes.data, None if wsum is None else wsum.ctypes.data
        st = self._lib.count_pairs_r_noalloc(
            self._ctx, ctypes.byref(c1.c), None if c2 is None else ctypes.byref(c2.c),
            e.ctypes.data, nb, float(boxsize), self._prec(precision), cp, wp,
            self._opts(options, **fixed))
        self._check(st)
        return counts, wsum

    def count_rppi(self, d1, d2=None, rp_edges=None, pimax: float = 40.0, npi: int = 40,
                   boxsize: float = 0.0, precision="fp64", w1=None, w2=None, options=None,
                   weight_type=None, ravg=False):
        """DD(rp, pi): returns (counts uint64[nrp, npi], wsum or None), plus
        the mean rp per bin when ``ravg``."""
        e = np.ascontiguousarray(rp_edges, dtype=np.float64)
        nb = e.size - 1
        c1 = _Cat(d1, w1)
        c2 = None if d2 is None else _Cat(d2, w2)
        counts = np.zeros(nb * int(npi), dtype=np.uint64)
        wsum = np.zeros(nb * int(npi), dtype=np.float64) if w1 is not None else None
        rv = np.zeros(nb * int(npi), dtype=np.float64) if ravg else None
        st = self._lib.count_pairs_rppi_ex(
            self._ctx, ctypes.byref(c1.c), None if c2 is None else ctypes.byref(c2.c),
            e.ctypes.data, nb, float(pimax), int(npi), float(boxsize), self._prec(precision),
            counts.ctypes.data, None if wsum is None else wsum.ctypes.data,
            self._opts(options, weight_type, rv))
        self._check(st)
        return self._result(counts, wsum, rv, (nb, int(npi)))

    def count_rppi_batch(self, catalogues, rp_edges=None, pimax: float = 40.0, npi: int = 40,
                         boxsize: float = 0.0, precision="fp64", weights=None, options=None,
                         weight_type=None, ravg=False):
        """Batched DD(rp, pi) autocorrelations of several catalogues in one
        pass: returns (counts uint64[ncat, nrp, npi], wsum or None), plus the
        mean rp per bin when ``ravg``."""
        e = np.ascontiguousarray(rp_edges, dtype=np.float64)
        nb = e.size - 1
        ncat = len(catalogues)
        if weights is not None and len(weights) != ncat:
            raise ValueError("one weight array per catalogue")
        cats = [_Cat(p, None if weights is None else weights[k]) for k, p in enumerate(catalogues)]
        arr = (cf_catalog * max(ncat, 1))()
        for k, cc in enumerate(cats):
            arr[k] = cc.c
        counts = np.zeros(ncat * nb * int(npi), dtype=np.uint64)
        wsum = np.zeros(ncat * nb * int(npi), dtype=np.float64) if weights is not None else None
        rv = np.zeros(ncat * nb * int(npi), dtype=np.float64) if ravg else None
        st = self._lib.count_pairs_rppi_batch_ex(
            self._ctx, ctypes.cast(arr, ctypes.c_void_p), ncat, e.ctypes.data, nb, float(pimax),
            int(npi), float(boxsize), self._prec(precision), counts.ctypes.data,
            None if wsum is None else wsum.ctypes.data, self._opts(options, weight_type, rv))
        self._check(st)
        return self._result(counts, wsum, rv, (ncat, nb, int(npi)))

    def count_rppi_mocks(self, d1, d2=None, rp_edges=None, pimax: float = 40.0, npi: int = 40,
                         precision="fp64", w1=None, w2=None, options=None, weight_type=None,
                         ravg=False, cartesian=False):
        """On-sky DD(rp, pi) with the line of sight through each pair's
        midpoint.  d1, d2: columns (RA deg, DEC deg, distance), as an (n, 3)
        array or three arrays; with ``cartesian`` the columns are positions
        x, y, z.  Returns (counts uint64[nrp, npi], wsum or None), plus the
        mean rp per bin when ``ravg``."""
        e = np.ascontiguousarray(rp_edges, dtype=np.float64)
        nb = e.size - 1
        c1 = _Cat(d1, w1)
        c2 = None if d2 is None else _Cat(d2, w2)
        counts = np.zeros(nb * int(npi), dtype=np.uint64)
        wsum = np.zeros(nb * int(npi), dtype=np.float64) if w1 is not None else None
        rv = np.zeros(nb * int(npi), dtype=np.float64) if ravg else None
        fixed = {"theta_unit_vectors": 1} if cartesian else {}
        st = self._lib.count_pairs_rppi_mocks_ex(
            self._ctx, ctypes.byref(c1.c), None if c2 is None else ctypes.byref(c2.c),
            e.ctypes.data, nb, float(pimax), int(npi), self._prec(precision), counts.ctypes.data,
            None if wsum is None else wsum.ctypes.data,
            self._opts(options, weight_type, rv, **fixed))
        self._check(st)
        return self._result(counts, wsum, rv, (nb, int(npi)))

    def count_theta(self, ra1, dec1, ra2=None, dec2=None, theta_edges_deg=None,
                    precision="fp64", w1=None, w2=None, options=None, unit_vectors=None,
                    weight_type=None, ravg=False, angular_grid=None):
        """DD(theta)/DR(theta) from RA/DEC in degrees (or unit vectors when
        ``unit_vectors=(v1, v2)`` is given), plus the mean angle per bin in
        degrees when ``ravg``.  ``angular_grid``: None / 0 the default angular
        grid, n > 0 declination bands and right-ascension cells 1/n of the
        reach, -1 3-D cells on the unit vectors."""
        grid = {} if angular_grid is None else {"angular_grid": angular_grid}
        e = np.ascontiguousarray(theta_edges_deg, dtype=np.float64)
        nb = e.size - 1
        rv = np.zeros(nb, dtype=np.float64) if ravg else None
        if unit_vectors is not None:
            v1, v2 = unit_vectors
            c1 = _Cat(v1, w1)
            c2 = None if v2 is None else _Cat(v2, w2)
            optp = self._opts(options, weight_type, rv, theta_unit_vectors=1, **grid)
        else:
            c1 = _Cat((ra1, dec1), w1, two_columns=True)
            c2 = None if ra2 is None else _Cat((ra2, dec2), w2, two_columns=True)
            optp = self._opts(options, weight_type, rv, **grid)
        counts = np.zeros(nb, dtype=np.uint64)
        wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
        st = self._lib.count_pairs_theta_ex(
            self._ctx, ctypes.byref(c1.c), None if c2 is None else ctypes.byref(c2.c),
            e.ctypes.data, nb, self._prec(precision), counts.ctypes.data,
            None if wsum is None else wsum.ctypes.data, optp)
        self._check(st)
        return self._result(counts, wsum, rv, (nb,))

    def stats(self) -> dict:
        s = cf_stats()
        self._check(self._lib.cf_get_stats(self._ctx, ctypes.byref(s)))
        out = {}
        for name, _ in cf_stats._fields_:
            v = getattr(s, name)
            if hasattr(v, "__len__"):
                v = list(v)
            out[name] = v
        return out
