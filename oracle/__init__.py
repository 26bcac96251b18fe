"""CPU oracle for binned pair counting -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct binary64 brute-force pair counter written from
the paper (Sinha & Garrison, arXiv:1911.03545): Code 1's loop over all pairs,
Code 3's periodic wrap, squared-distance bins (section "Finding and updating the
histogram bins"), the separations of Appendix A and the self-pair rule of
Appendix B.  The arithmetic lives in ``paircount_oracle.c``; this module only
marshals arguments through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1911_03545_amd``), and the GPU library never imports it.

Pinning: every function here is checked in ``tests/test_oracle.py`` against
hand-enumerated golden counts (``tests/golden/``), exact rational arithmetic on
lattice inputs, analytic uniform-box expectations, invariants the paper fixes,
and Python's ``math.fsum`` for the exact weighted sums.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "paircount_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared"]

_lib = None


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    dp, up = ctypes.c_void_p, ctypes.c_void_p
    lib.oracle_count_r.argtypes = [i64, dp, dp, dp, dp, i64, dp, dp, dp, dp,
                                   ctypes.c_int, dp, i32, dbl, up, dp,
                                   ctypes.c_int]
    lib.oracle_count_r.restype = ctypes.c_int
    lib.oracle_count_rppi.argtypes = [i64, dp, dp, dp, dp, i64, dp, dp, dp, dp,
                                      ctypes.c_int, dp, i32, dbl, i32, dbl, up,
                                      dp, ctypes.c_int]
    lib.oracle_count_rppi.restype = ctypes.c_int
    lib.oracle_count_theta.argtypes = [i64, dp, dp, dp, i64, dp, dp, dp,
                                       ctypes.c_int, dp, i32, up, dp,
                                       ctypes.c_int]
    lib.oracle_count_theta.restype = ctypes.c_int
    lib.oracle_count_r_ex.argtypes = [i64, dp, dp, dp, dp, i64, dp, dp, dp, dp,
                                      ctypes.c_int, dp, i32, dbl, up, dp,
                                      ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_count_r_ex.restype = ctypes.c_int
    lib.oracle_count_rppi_ex.argtypes = [i64, dp, dp, dp, dp, i64, dp, dp, dp,
                                         dp, ctypes.c_int, dp, i32, dbl, i32,
                                         dbl, up, dp, ctypes.c_int, dp,
                                         ctypes.c_int]
    lib.oracle_count_rppi_ex.restype = ctypes.c_int
    lib.oracle_count_theta_ex.argtypes = [i64, dp, dp, dp, i64, dp, dp, dp,
                                          ctypes.c_int, dp, i32, up, dp,
                                          ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_count_theta_ex.restype = ctypes.c_int
    lib.oracle_count_rppi_mocks.argtypes = [i64, dp, dp, dp, dp, i64, dp, dp, dp,
                                            dp, ctypes.c_int, dp, i32, dbl, i32,
                                            up, dp, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_count_rppi_mocks.restype = ctypes.c_int
    lib.oracle_sky_to_cartesian.argtypes = [i64, dp, dp, dp, dp, dp, dp]
    lib.oracle_sky_to_cartesian.restype = ctypes.c_int
    lib.oracle_radec_to_unit.argtypes = [i64, dp, dp, dp, dp, dp]
    lib.oracle_radec_to_unit.restype = ctypes.c_int
    lib.oracle_theta_chord_edges.argtypes = [i32, dp, dp]
    lib.oracle_theta_chord_edges.restype = ctypes.c_int
    lib.oracle_pi_edges.argtypes = [dbl, i32, dp]
    lib.oracle_pi_edges.restype = ctypes.c_int
    lib.oracle_xsum.argtypes = [i64, dp]
    lib.oracle_xsum.restype = dbl
    lib.oracle_count_r_pruned.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, i64, dp, dp,
                                          dp, dp, ctypes.c_int, dp, i32, dbl, up, dp,
                                          ctypes.c_int, ctypes.c_int]
    lib.oracle_count_r_pruned.restype = ctypes.c_int
    lib.oracle_count_rppi_pruned.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, i64, dp,
                                             dp, dp, dp, ctypes.c_int, dp, i32, dbl, i32,
                                             dbl, up, dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_count_rppi_pruned.restype = ctypes.c_int
    lib.oracle_count_theta_uv_pruned.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, i64,
                                                 dp, dp, dp, dp, ctypes.c_int, dp, i32,
                                                 up, dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_count_theta_uv_pruned.restype = ctypes.c_int
    return lib


def load(path: str = _LIB, rebuild_if_missing: bool = True):
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        if not rebuild_if_missing:
            raise FileNotFoundError(path)
        build(out=path)
    lib = _bind(ctypes.CDLL(path))
    if path == _LIB:
        _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _f64(a):
    """Exact promotion to binary64 (float32 -> float64 widening is exact)."""
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _xyz(p):
    p = _f64(p)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("positions must be (n, 3)")
    return (np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
            np.ascontiguousarray(p[:, 2]))


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


WEIGHT_TYPES = {"product": 0, "sum": 1}


def _wtype(weight_type):
    if weight_type not in WEIGHT_TYPES:
        raise ValueError(f"unknown weight_type {weight_type!r}")
    return WEIGHT_TYPES[weight_type]


def count_r(d1, d2=None, edges=None, boxsize: float = 0.0, w1=None, w2=None,
            nthreads: int = 0, lib=None, weight_type: str = "product",
            ravg: bool = False):
    """DD(r) counts (uint64[nbins]) and weighted sums (float64[nbins] or None),
    plus the mean separation per bin (float64[nbins]) when ``ravg``.

    ``d2 is None`` selects the autocorrelation of d1 (== cross(d1, d1))."""
    lib = lib or load()
    edges = _f64(edges)
    nb = edges.size - 1
    x1, y1, z1 = _xyz(d1)
    auto = d2 is None
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(d2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb, dtype=np.uint64)
    wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
    rv = np.zeros(nb, dtype=np.float64) if ravg else None
    rc = lib.oracle_count_r_ex(x1.size, _ptr(x1), _ptr(y1), _ptr(z1), _ptr(ww1),
                               x2.size, _ptr(x2), _ptr(y2), _ptr(z2), _ptr(ww2),
                               int(auto), _ptr(edges), nb, float(boxsize),
                               counts.ctypes.data, _ptr(wsum), _wtype(weight_type),
                               _ptr(rv), int(nthreads))
    _check(rc, "oracle_count_r")
    return (counts, wsum, rv) if ravg else (counts, wsum)


def count_rppi(d1, d2=None, rp_edges=None, pimax: float = 40.0, npi: int = 40,
               boxsize: float = 0.0, w1=None, w2=None, nthreads: int = 0,
               lib=None, weight_type: str = "product", ravg: bool = False):
    """DD(rp, pi) counts as uint64[nrp, npi] (and weighted sums, and the mean
    rp per bin when ``ravg``)."""
    lib = lib or load()
    rp_edges = _f64(rp_edges)
    nb = rp_edges.size - 1
    x1, y1, z1 = _xyz(d1)
    auto = d2 is None
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(d2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb * npi, dtype=np.uint64)
    wsum = np.zeros(nb * npi, dtype=np.float64) if w1 is not None else None
    rv = np.zeros(nb * npi, dtype=np.float64) if ravg else None
    rc = lib.oracle_count_rppi_ex(x1.size, _ptr(x1), _ptr(y1), _ptr(z1),
                                  _ptr(ww1), x2.size, _ptr(x2), _ptr(y2),
                                  _ptr(z2), _ptr(ww2), int(auto), _ptr(rp_edges),
                                  nb, float(pimax), int(npi), float(boxsize),
                                  counts.ctypes.data, _ptr(wsum), _wtype(weight_type),
                                  _ptr(rv), int(nthreads))
    _check(rc, "oracle_count_rppi")
    counts = counts.reshape(nb, npi)
    if wsum is not None:
        wsum = wsum.reshape(nb, npi)
    if ravg:
        return counts, wsum, rv.reshape(nb, npi)
    return counts, wsum


def count_theta(ra1, dec1, ra2=None, dec2=None, theta_edges_deg=None,
                w1=None, w2=None, nthreads: int = 0, lib=None,
                weight_type: str = "product", ravg: bool = False):
    """DD(theta) / DR(theta) counts from RA/DEC in degrees (and the mean
    angle per bin in degrees when ``ravg``)."""
    lib = lib or load()
    te = _f64(theta_edges_deg)
    nb = te.size - 1
    a1, d1 = _f64(ra1), _f64(dec1)
    auto = ra2 is None
    a2, d2 = (a1, d1) if auto else (_f64(ra2), _f64(dec2))
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb, dtype=np.uint64)
    wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
    rv = np.zeros(nb, dtype=np.float64) if ravg else None
    rc = lib.oracle_count_theta_ex(a1.size, _ptr(a1), _ptr(d1), _ptr(ww1),
                                   a2.size, _ptr(a2), _ptr(d2), _ptr(ww2),
                                   int(auto), _ptr(te), nb, counts.ctypes.data,
                                   _ptr(wsum), _wtype(weight_type), _ptr(rv),
                                   int(nthreads))
    _check(rc, "oracle_count_theta")
    return (counts, wsum, rv) if ravg else (counts, wsum)


def count_rppi_mocks(d1, d2=None, rp_edges=None, pimax: float = 40.0, npi: int = 40,
                     w1=None, w2=None, nthreads: int = 0, lib=None,
                     weight_type: str = "product", ravg: bool = False):
    """On-sky DD(rp, pi) (line of sight through each pair's midpoint) of
    Cartesian positions (n, 3) from :func:`sky_to_cartesian`."""
    lib = lib or load()
    rp_edges = _f64(rp_edges)
    nb = rp_edges.size - 1
    x1, y1, z1 = _xyz(d1)
    auto = d2 is None
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(d2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb * npi, dtype=np.uint64)
    wsum = np.zeros(nb * npi, dtype=np.float64) if w1 is not None else None
    rv = np.zeros(nb * npi, dtype=np.float64) if ravg else None
    rc = lib.oracle_count_rppi_mocks(x1.size, _ptr(x1), _ptr(y1), _ptr(z1),
                                     _ptr(ww1), x2.size, _ptr(x2), _ptr(y2),
                                     _ptr(z2), _ptr(ww2), int(auto), _ptr(rp_edges),
                                     nb, float(pimax), int(npi), counts.ctypes.data,
                                     _ptr(wsum), _wtype(weight_type), _ptr(rv),
                                     int(nthreads))
    _check(rc, "oracle_count_rppi_mocks")
    counts = counts.reshape(nb, npi)
    if wsum is not None:
        wsum = wsum.reshape(nb, npi)
    if ravg:
        return counts, wsum, rv.reshape(nb, npi)
    return counts, wsum


def sky_to_cartesian(ra, dec, dist, lib=None):
    """(n, 3) positions D u from RA/DEC in degrees and distances D."""
    lib = lib or load()
    a, d, r = _f64(ra), _f64(dec), _f64(dist)
    out = np.zeros((3, a.size), dtype=np.float64)
    rc = lib.oracle_sky_to_cartesian(a.size, _ptr(a), _ptr(d), _ptr(r), out[0].ctypes.data,
                                     out[1].ctypes.data, out[2].ctypes.data)
    _check(rc, "oracle_sky_to_cartesian")
    return np.ascontiguousarray(out.T)


def radec_to_unit(ra, dec, lib=None):
    """(n, 3) unit vectors from RA/DEC in degrees."""
    lib = lib or load()
    a, d = _f64(ra), _f64(dec)
    out = np.zeros((3, a.size), dtype=np.float64)
    rc = lib.oracle_radec_to_unit(a.size, _ptr(a), _ptr(d), out[0].ctypes.data,
                                  out[1].ctypes.data, out[2].ctypes.data)
    _check(rc, "oracle_radec_to_unit")
    return np.ascontiguousarray(out.T)


def theta_chord_edges(theta_deg, lib=None):
    lib = lib or load()
    t = _f64(theta_deg)
    out = np.zeros_like(t)
    rc = lib.oracle_theta_chord_edges(t.size, _ptr(t), out.ctypes.data)
    _check(rc, "oracle_theta_chord_edges")
    return out


def pi_edges(pimax: float, npi: int, lib=None):
    lib = lib or load()
    q = np.zeros(int(npi) + 1, dtype=np.float64)
    rc = lib.oracle_pi_edges(float(pimax), int(npi), q.ctypes.data)
    _check(rc, "oracle_pi_edges")
    return q


def xsum(v, lib=None) -> float:
    lib = lib or load()
    v = _f64(v)
    return float(lib.oracle_xsum(v.size, _ptr(v)))


# --------------------------------------------------------------------------
# Exactly pruned variants: identical results to count_r / count_rppi /
# count_theta, visiting only pairs whose difference along one axis (with its
# periodic images) is within the reach plus a margin.  For reference counts
# of catalogues too large to enumerate.
# --------------------------------------------------------------------------
def count_r_pruned(d1, d2=None, edges=None, boxsize: float = 0.0, w1=None, w2=None,
                   axis: int = 2, nthreads: int = 0, lib=None,
                   weight_type: str = "product"):
    """DD(r) counts and weighted sums, pruned along ``axis``."""
    lib = lib or load()
    edges = _f64(edges)
    nb = edges.size - 1
    x1, y1, z1 = _xyz(d1)
    auto = d2 is None
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(d2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb, dtype=np.uint64)
    wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
    rc = lib.oracle_count_r_pruned(int(axis), x1.size, _ptr(x1), _ptr(y1), _ptr(z1),
                                   _ptr(ww1), x2.size, _ptr(x2), _ptr(y2), _ptr(z2),
                                   _ptr(ww2), int(auto), _ptr(edges), nb, float(boxsize),
                                   counts.ctypes.data, _ptr(wsum), _wtype(weight_type),
                                   int(nthreads))
    _check(rc, "oracle_count_r_pruned")
    return counts, wsum


def count_rppi_pruned(d1, d2=None, rp_edges=None, pimax: float = 40.0, npi: int = 40,
                      boxsize: float = 0.0, w1=None, w2=None, axis: int = 2,
                      nthreads: int = 0, lib=None, weight_type: str = "product"):
    """DD(rp, pi) counts uint64[nrp, npi] (and weighted sums), pruned along
    ``axis`` (the reach is pimax along z, the largest rp edge along x or y)."""
    lib = lib or load()
    rp_edges = _f64(rp_edges)
    nb = rp_edges.size - 1
    x1, y1, z1 = _xyz(d1)
    auto = d2 is None
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(d2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb * npi, dtype=np.uint64)
    wsum = np.zeros(nb * npi, dtype=np.float64) if w1 is not None else None
    rc = lib.oracle_count_rppi_pruned(int(axis), x1.size, _ptr(x1), _ptr(y1), _ptr(z1),
                                      _ptr(ww1), x2.size, _ptr(x2), _ptr(y2), _ptr(z2),
                                      _ptr(ww2), int(auto), _ptr(rp_edges), nb,
                                      float(pimax), int(npi), float(boxsize),
                                      counts.ctypes.data, _ptr(wsum), _wtype(weight_type),
                                      int(nthreads))
    _check(rc, "oracle_count_rppi_pruned")
    counts = counts.reshape(nb, npi)
    if wsum is not None:
        wsum = wsum.reshape(nb, npi)
    return counts, wsum


def count_theta_pruned(ra1, dec1, ra2=None, dec2=None, theta_edges_deg=None, w1=None,
                       w2=None, axis: int = 1, nthreads: int = 0, lib=None,
                       weight_type: str = "product"):
    """DD(theta) / DR(theta) from RA/DEC in degrees (converted like
    count_theta), pruned along one axis of the unit vectors."""
    lib = lib or load()
    te = _f64(theta_edges_deg)
    nb = te.size - 1
    v1 = radec_to_unit(ra1, dec1, lib=lib)
    auto = ra2 is None
    v2 = v1 if auto else radec_to_unit(ra2, dec2, lib=lib)
    x1, y1, z1 = _xyz(v1)
    x2, y2, z2 = (x1, y1, z1) if auto else _xyz(v2)
    ww1 = None if w1 is None else _f64(w1)
    ww2 = None if (w1 is None) else (ww1 if auto else _f64(w2))
    counts = np.zeros(nb, dtype=np.uint64)
    wsum = np.zeros(nb, dtype=np.float64) if w1 is not None else None
    rc = lib.oracle_count_theta_uv_pruned(int(axis), x1.size, _ptr(x1), _ptr(y1),
                                          _ptr(z1), _ptr(ww1), x2.size, _ptr(x2),
                                          _ptr(y2), _ptr(z2), _ptr(ww2), int(auto),
                                          _ptr(te), nb, counts.ctypes.data, _ptr(wsum),
                                          _wtype(weight_type), int(nthreads))
    _check(rc, "oracle_count_theta_uv_pruned")
    return counts, wsum
