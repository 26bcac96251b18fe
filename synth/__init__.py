"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays out arrays; it holds none of the
pair-counting arithmetic (no separations, no binning, no coordinate conversion
used by the method).  Every generator is a pure function of its arguments and a
seed: NumPy ``Generator(PCG64(seed))`` in float64 on the host.

Workload recipes (the paper's catalogues are not available, so these stand in):

* ``uniform_box``   -- points uniform in a periodic cube, as in the paper's
  analytic random-pair expectation (Appendix B).
* ``clustered_box`` -- half of the points uniform, half in equal-size Gaussian
  blobs (sigma = 2 by default) with uniform blob centres, wrapped into [0, L)
  and shuffled so that the input order carries no spatial information.  It
  stands in for the fiducial ~1.2 M galaxy mock in a 420 box (Benchmarks
  section) and the clustered halo catalogue of the code comparison.
* ``cap_radec``     -- RA/DEC points on a spherical cap, either uniform
  (cos(theta) uniform) or half uniform and half in tangent-plane Gaussian blobs;
  stands in for the paper's mock galaxies and randoms on the sky.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for",
    "uniform_box",
    "clustered_box",
    "uniform_weights",
    "log_edges",
    "cap_radec",
    "batch_sizes",
    "lattice_box",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_box(n: int, L: float, seed: int) -> np.ndarray:
    """(n, 3) float64 points uniform in [0, L)^3."""
    rng = rng_for(seed)
    return rng.uniform(0.0, L, size=(int(n), 3))


def clustered_box(n: int, L: float, seed: int, nblobs: int | None = None,
                  sigma: float = 2.0, frac: float = 0.5,
                  per_blob: int = 200) -> np.ndarray:
    """(n, 3) float64 clustered points in [0, L]^3.

    ``frac`` of the points are split evenly over ``nblobs`` Gaussian blobs
    (default n // per_blob blobs, i.e. per_blob/2 clustered points each at the
    default frac); the rest are uniform.  Positions are wrapped with a floating
    modulo, which may return exactly L for tiny negative inputs: the closed
    interval [0, L] is legal input.
    """
    rng = rng_for(seed)
    n = int(n)
    n_cl = int(round(n * frac))
    n_bg = n - n_cl
    if nblobs is None:
        nblobs = max(1, n // per_blob)
    bg = rng.uniform(0.0, L, size=(n_bg, 3))
    centres = rng.uniform(0.0, L, size=(nblobs, 3))
    owner = np.arange(n_cl) % nblobs
    cl = centres[owner] + rng.normal(0.0, sigma, size=(n_cl, 3))
    cl = np.mod(cl, L)
    pts = np.concatenate([bg, cl], axis=0)
    perm = rng.permutation(n)
    return np.ascontiguousarray(pts[perm])


def lattice_box(n: int, L: int, seed: int, denom: int = 1024) -> np.ndarray:
    """(n, 3) points on the lattice (1/denom)Z inside [0, L] (L an integer).

    With denom = 2^10 and L <= 2^11 every difference, square and sum of three
    squares is exact in binary64, so a float64 pair counter must agree with
    exact rational arithmetic on these inputs.
    """
    rng = rng_for(seed)
    k = rng.integers(0, int(L) * denom + 1, size=(int(n), 3))
    return k.astype(np.float64) / float(denom)


def uniform_weights(n: int, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """float32 weights uniform in [lo, hi)."""
    rng = rng_for(seed)
    return rng.uniform(lo, hi, size=int(n)).astype(np.float32)


def log_edges(lo: float, hi: float, nbins: int) -> np.ndarray:
    """nbins+1 logarithmically spaced edges from lo to hi (float64)."""
    return np.logspace(np.log10(lo), np.log10(hi), int(nbins) + 1)


def _cap_frame(ra0_deg: float, dec0_deg: float):
    """Orthonormal frame (e_centre, e_east, e_north) at a sky position."""
    a = np.deg2rad(ra0_deg)
    d = np.deg2rad(dec0_deg)
    c = np.array([np.cos(d) * np.cos(a), np.cos(d) * np.sin(a), np.sin(d)])
    east = np.array([-np.sin(a), np.cos(a), 0.0])
    north = np.cross(c, east)
    return c, east, north


def _to_radec(v: np.ndarray):
    ra = np.mod(np.rad2deg(np.arctan2(v[:, 1], v[:, 0])), 360.0)
    dec = np.rad2deg(np.arcsin(np.clip(v[:, 2], -1.0, 1.0)))
    return ra, dec


def _uniform_cap_vectors(rng, n, c, east, north, radius_rad):
    cos_t = rng.uniform(np.cos(radius_rad), 1.0, size=n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return (cos_t[:, None] * c[None, :]
            + (sin_t * np.cos(phi))[:, None] * east[None, :]
            + (sin_t * np.sin(phi))[:, None] * north[None, :])


def cap_radec(n: int, seed: int, radius_deg: float = 30.0, ra0_deg: float = 0.0,
              dec0_deg: float = 30.0, clustered: bool = False,
              nblobs: int = 10000, sigma_deg: float = 0.1, frac: float = 0.5):
    """RA, DEC (degrees, float64) of n points on a cap of angular radius
    ``radius_deg`` centred at (ra0, dec0).  With ``clustered`` half of the
    points sit in Gaussian blobs of tangent-plane width ``sigma_deg`` around
    uniform blob centres; blob points falling outside the cap are redrawn.
    The default centre makes the cap straddle the RA = 0/360 seam."""
    rng = rng_for(seed)
    n = int(n)
    c, east, north = _cap_frame(ra0_deg, dec0_deg)
    rad = np.deg2rad(radius_deg)
    if not clustered:
        v = _uniform_cap_vectors(rng, n, c, east, north, rad)
        return _to_radec(v)
    n_cl = int(round(n * frac))
    n_bg = n - n_cl
    bg = _uniform_cap_vectors(rng, n_bg, c, east, north, rad)
    centres = _uniform_cap_vectors(rng, nblobs, c, east, north, rad)
    # per-blob tangent basis
    ce = np.cross(np.array([0.0, 0.0, 1.0])[None, :], centres)
    norm = np.linalg.norm(ce, axis=1)
    ce[norm < 1e-12] = np.array([1.0, 0.0, 0.0])
    ce /= np.linalg.norm(ce, axis=1)[:, None]
    cn = np.cross(centres, ce)
    owner = np.arange(n_cl) % nblobs
    sig = np.deg2rad(sigma_deg)
    cos_rad = np.cos(rad)
    out = np.empty((n_cl, 3))
    todo = np.arange(n_cl)
    while todo.size:
        o = owner[todo]
        g = rng.normal(0.0, sig, size=(todo.size, 2))
        v = centres[o] + g[:, :1] * ce[o] + g[:, 1:] * cn[o]
        v /= np.linalg.norm(v, axis=1)[:, None]
        inside = v @ c >= cos_rad
        out[todo[inside]] = v[inside]
        todo = todo[~inside]
    v = np.concatenate([bg, out], axis=0)[rng.permutation(n)]
    return _to_radec(v)


def batch_sizes(ncat: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Catalogue sizes drawn uniformly from the integers [lo, hi]."""
    rng = rng_for(seed)
    return rng.integers(int(lo), int(hi) + 1, size=int(ncat))


def sky_mock(n: int, seed: int, radius_deg: float = 10.0, dmin: float = 500.0,
             dmax: float = 1500.0, clustered: bool = True, per_blob: int = 200,
             sigma: float = 2.0, frac: float = 0.5, ra0_deg: float = 0.0,
             dec0_deg: float = 30.0):
    """An on-sky catalogue: (RA deg, DEC deg, distance) columns as an (n, 3)
    float64 array.  Points fill the cone of angular radius ``radius_deg``
    around (ra0, dec0) between distances dmin and dmax uniformly in volume;
    with ``clustered`` a fraction ``frac`` of them sit in 3-D Gaussian blobs
    of width ``sigma`` (length units of the distances) around uniform
    centres, ``per_blob`` / 2 points each at the default fraction, redrawn
    until they fall inside the cone and the distance range."""
    rng = rng_for(seed)
    n = int(n)
    c, east, north = _cap_frame(ra0_deg, dec0_deg)
    rad = np.deg2rad(radius_deg)

    def uniform(m):
        u = _uniform_cap_vectors(rng, m, c, east, north, rad)
        d = np.cbrt(rng.uniform(dmin ** 3, dmax ** 3, size=m))
        return u * d[:, None]

    if not clustered:
        p = uniform(n)
    else:
        n_cl = int(round(n * frac))
        nblobs = max(1, (2 * n_cl) // max(per_blob, 1))
        centres = uniform(nblobs)
        owner = np.arange(n_cl) % nblobs
        out = np.empty((n_cl, 3))
        todo = np.arange(n_cl)
        cos_rad = np.cos(rad)
        while todo.size:
            v = centres[owner[todo]] + rng.normal(0.0, sigma, size=(todo.size, 3))
            d = np.linalg.norm(v, axis=1)
            ok = (d >= dmin) & (d <= dmax) & ((v @ c) >= cos_rad * d)
            out[todo[ok]] = v[ok]
            todo = todo[~ok]
        p = np.concatenate([uniform(n - n_cl), out], axis=0)[rng.permutation(n)]
    d = np.linalg.norm(p, axis=1)
    ra, dec = _to_radec(p / d[:, None])
    return np.stack([ra, dec, d], axis=1)
