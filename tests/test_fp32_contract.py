"""The float32 + binary64-recheck contract, validated on the CPU.

The float32 sweep may decide a pair only when its float32 separation lies
outside the decision band [lo_k, hi_k] of every squared edge E_k; inside a
band the pair is re-evaluated in binary64.  The bands come from a proven
bound B(s) on |s32 - s64| (cf_fp32_bands_axes).  These tests emulate the
sweep's float32 arithmetic exactly -- the column-local x and y frames of 3-D
grids, z in the domain frame, the periodic offset of the work item, the
coordinate scale (not a power of two), one float32 multiply and two fused
multiply-adds with a single rounding each -- on more than 10^8 pairs (random
pairs over the whole reach, periodic wraps, and adversarial pairs within a
few ulps of every edge), and check that

* the largest ratio |s32 - s64| / B(s64) is below 1 for the raw bound (the
  library adds a 1.25 safety factor on top), and is reported;
* no pair is decided the wrong way against any edge: s32 < lo_k implies
  s64 < E_k and s32 > hi_k implies s64 > E_k;

for DD(r) (3 axes), rp^2 (2 axes) and squared chords of unit vectors
(3 axes, no box).  The expanded forms of squared r and rp (x and y as |a|^2 +
|b|^2 - 2 a.b) are also checked with each band narrowed by the pair's own
magnitude term, computed in float32 as the sweep does before its binary64 recheck: no
wrong decision, and |s32 - s64| stays within the pair's own raw bound.  And
that the fixed-point line-of-sight coordinate of the
float32 DD(rp, pi) path stays within 1.5 quanta of the exact |dz|, below the
2-quanta margin inside which pi bins are re-decided in binary64.
"""
import math

import numpy as np
import pytest

import paper_1911_03545_amd as pc
import synth

U32 = 2.0 ** -24
SAFETY = 1.25


def fma32(a, b, c):
    """Fused multiply-add of float32 arrays with one rounding to float32.

    a * b is exact in binary64 (24 + 24 bits); p + c is computed in binary64
    with its exact residual (two-sum).  Rounding the binary64 sum to float32
    can only differ from rounding the exact sum when the binary64 sum sits
    exactly half-way between two float32 values while the residual is not
    zero; the result is then the float32 neighbour on the residual's side."""
    p = a.astype(np.float64) * b.astype(np.float64)
    c64 = c.astype(np.float64)
    r = p + c64
    bb = r - p
    err = (p - (r - bb)) + (c64 - bb)
    f = r.astype(np.float32)
    f64 = f.astype(np.float64)
    up = np.nextafter(f, np.float32(np.inf))
    dn = np.nextafter(f, np.float32(-np.inf))
    # r exactly half-way between f and its neighbour on r's side
    tie_hi = (r > f64) & (r - f64 == (up.astype(np.float64) - f64) / 2)
    tie_lo = (r < f64) & (f64 - r == (f64 - dn.astype(np.float64)) / 2)
    # the exact value is beyond the midpoint, away from f, on err's side
    f = np.where(tie_hi & (err > 0), up, f)
    f = np.where(tie_lo & (err < 0), dn, f)
    return f.astype(np.float32)


def test_fma32_emulation_exact():
    """The emulated fused multiply-add equals exact rational arithmetic
    rounded once (checked with Fraction on random and tie-prone inputs)."""
    from fractions import Fraction
    rng = synth.rng_for(900)
    a = rng.normal(size=4000).astype(np.float32)
    b = rng.normal(size=4000).astype(np.float32)
    c = (rng.normal(size=4000) * 10.0 ** rng.integers(-8, 8, 4000)).astype(np.float32)
    # products exactly half-way between two float32 values, plus addends that
    # are zero (a true tie), representable next to it, or far below binary64's
    # resolution there (the binary64 sum is the midpoint, the exact one not)
    a[:2000] = np.float32(1.0) + np.float32(2.0 ** -12)
    b[:2000] = np.float32(1.0) + np.float32(2.0 ** -12)
    c[:1000] = (np.float32(2.0 ** -30) * rng.integers(-4, 4, 1000)).astype(np.float32)
    c[1000:2000] = (np.float32(2.0 ** -62) * rng.integers(-4, 4, 1000)).astype(np.float32)
    got = fma32(a, b, c)
    for k in range(a.size):
        exact = Fraction(float(a[k])) * Fraction(float(b[k])) + Fraction(float(c[k]))
        want = np.float32(float(exact))     # float() rounds the rational once to binary64
        # binary64 rounding of the exact value cannot create a float32 tie
        # here except at the constructed midpoints: settle those exactly
        lo = np.float32(want)
        cands = [np.nextafter(lo, np.float32(-np.inf)), lo, np.nextafter(lo, np.float32(np.inf))]
        best = min(cands, key=lambda v: (abs(Fraction(float(v)) - exact),
                                         int(np.float32(v).view(np.int32)) & 1))
        assert got[k] == best, (k, a[k], b[k], c[k], got[k], best)


def plan(L, reach, k=1):
    return pc.plan_grid_refined(None, None, L, reach, reach, 32, k, True)


def frames(p, g, L):
    """Column centres of every point (as the gridding assigns columns)."""
    idx = []
    for a in range(2):
        i = np.floor((p[:, a] - g["lo"][a]) * g["inv_width"][a]).astype(np.int64)
        idx.append(np.clip(i, 0, g["n"][a] - 1))
    cx = g["lo"][0] + (idx[0] + 0.5) * g["width"][0]
    cy = g["lo"][1] + (idx[1] + 0.5) * g["width"][1]
    return cx, cy


def emulate_r(pi, pj, g, L, c, ndim):
    """float32 s of the sweep for pairs (pi, pj): x, y in the j column's
    frame with the periodic offset on the i point, z in the domain frame."""
    cx, cy = frames(pj, g, L)
    d = pi - pj
    D = np.where(d > L / 2, -L, np.where(d <= -L / 2, L, 0.0)) if L > 0 else np.zeros_like(d)
    ax = (((pi[:, 0] + D[:, 0]) - cx) * c).astype(np.float32)
    ay = (((pi[:, 1] + D[:, 1]) - cy) * c).astype(np.float32)
    bx = ((pj[:, 0] - cx) * c).astype(np.float32)
    by = ((pj[:, 1] - cy) * c).astype(np.float32)
    dx = ax - bx
    dy = ay - by
    t = dx * dx
    t = fma32(dy, dy, t)
    if ndim == 2:
        return t
    az = (((pi[:, 2] + D[:, 2]) - g["lo"][2]) * c).astype(np.float32)
    bz = ((pj[:, 2] - g["lo"][2]) * c).astype(np.float32)
    dz = az - bz
    return fma32(dz, dz, t)


def emulate_r_xy(pi, pj, g, L, c, ndim=3, parts=False):
    """float32 s of the expanded form: |b|^2 = fl(by by + fl(bx bx)) per j
    point, |a|^2 = fl(ay ay + fl(ax ax)) per lane, then fl(dz dz + |b|^2),
    fl(-2 ax bx + .), fl(-2 ay by + .) and fl(. + |a|^2) for r; for rp^2
    fl(|a|^2 + |b|^2), fl(-2 ax bx + .) and fl(-2 ay by + .) (the same frames
    as emulate_r)."""
    cx, cy = frames(pj, g, L)
    d = pi - pj
    D = np.where(d > L / 2, -L, np.where(d <= -L / 2, L, 0.0)) if L > 0 else np.zeros_like(d)
    ax = (((pi[:, 0] + D[:, 0]) - cx) * c).astype(np.float32)
    ay = (((pi[:, 1] + D[:, 1]) - cy) * c).astype(np.float32)
    bx = ((pj[:, 0] - cx) * c).astype(np.float32)
    by = ((pj[:, 1] - cy) * c).astype(np.float32)
    az = (((pi[:, 2] + D[:, 2]) - g["lo"][2]) * c).astype(np.float32)
    bz = ((pj[:, 2] - g["lo"][2]) * c).astype(np.float32)
    q = fma32(by, by, bx * bx)
    A = fma32(ay, ay, ax * ax)
    if ndim == 2:
        # rp^2: fl(A + |b|^2) first, then the two products
        t = fma32(np.float32(-2.0) * ax, bx, A + q)
        t = fma32(np.float32(-2.0) * ay, by, t)
        return (t, A, q) if parts else t
    dz = az - bz
    t = fma32(dz, dz, q)
    t = fma32(np.float32(-2.0) * ax, bx, t)
    t = fma32(np.float32(-2.0) * ay, by, t)
    return (t + A, A, q) if parts else t + A


def pair_narrowing(A, q, K, M, ndim=3):
    """The sweep's float32 per-pair narrowing of an expanded r band (scaled
    coordinates): m = fl(fl(11 q + fl(2.75 A)) (1 + 2^-18)) bounds 5 |b|^2 +
    2 |a|^2 + 4 |a| |b| from above (rp, ndim 2: fl(7 q + fl(4.375 A)) bounds
    4 |b|^2 + 4 |a|^2 + 2 |a| |b|), and D = fl(fl(K fl(M - m)) (1 - 2^-18))
    with the library's K and M (cf_fp32_pair_margin)."""
    f = np.float32
    if ndim == 3:
        m = fma32(f(11.0), q, f(2.75) * A) * f(1.0 + 2.0 ** -18)
    else:
        m = fma32(f(7.0), q, f(4.375) * A) * f(1.0 + 2.0 ** -18)
    return (K * (M - m)) * f(1.0 - 2.0 ** -18)


def expand_mag(xy_max, ndim):
    """The bands' magnitude term from the coordinates' maxima (a point may
    round a little outside its column)."""
    g = 1.0 + 2.0 ** -16
    ax, ay, bx, by = (v * g for v in xy_max)
    A, B, P = ax * ax + ay * ay, bx * bx + by * by, ax * bx + ay * by
    return 4 * A + 4 * B + 2 * P if ndim == 2 else 5 * B + 2 * A + 4 * P


def exact_s(pi, pj, L, ndim):
    """The binary64 definition: Code 3's wrap, ((dx^2 + dy^2) + dz^2)."""
    d = pi - pj
    if L > 0:
        d = np.where(d > 0.5 * L, d - L, d)
        d = np.where(d <= -0.5 * L, d + L, d)
    s = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    if ndim == 3:
        s = s + d[:, 2] * d[:, 2]
    return s


def draw_pairs(rng, n, L, reach, lo=0.0, hi=None, radial=None):
    """n pairs: i uniform in the box, j at a separation up to 1.05 reach in
    a random direction (or at the given radial distances), wrapped."""
    hi = L if hi is None else hi
    pi = rng.uniform(lo, hi, size=(n, 3))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    r = rng.uniform(0.0, 1.05 * reach, n) if radial is None else radial
    pj = pi + u * r[:, None]
    if L > 0:
        pj = np.mod(pj, L)
    else:
        pj = np.clip(pj, lo, hi)
    return pi, pj


def check_contract(pi, pj, g, L, c, ndim, edges, axis_eps, coord_scale, stats, xy_max=None,
                   count=True, narrow_scale=1.0):
    """xy_max given: the expanded form and its bands (cf_fp32_bands_xy);
    count: add the pairs to the in-band tallies (random pairs only);
    narrow_scale: multiplies the per-pair narrowing (1 as the sweep takes
    it; larger to check that a wrong narrowing is caught)."""
    s64 = exact_s(pi, pj, L, ndim)
    if xy_max is None:
        s32 = emulate_r(pi, pj, g, L, c, ndim).astype(np.float64) / (c * c)

        def bands(e2):
            return pc.fp32_bands_axes(e2, ndim, axis_eps, coord_scale)
    else:
        f32, A, q = emulate_r_xy(pi, pj, g, L, c, ndim, parts=True)
        s32 = f32.astype(np.float64) / (c * c)

        def bands(e2):
            return pc.fp32_bands_xy(e2, axis_eps, xy_max, coord_scale, ndim)
    E = edges * edges
    lo, hi = bands(E)
    for k in range(E.size):
        if E[k] == 0.0:
            continue
        below = s32 < lo[k]
        above = s32 > hi[k]
        assert np.all(s64[below] < E[k]), ("decided below but not", k)
        assert np.all(s64[above] > E[k]), ("decided above but not", k)
    tight = xy_max is not None
    if tight:
        # the narrowed bands, in the scaled coordinates as the sweep takes
        # them (bands scaled by c^2 and rounded outward, float32 differences)
        K, M = pc.fp32_pair_margin(xy_max, c, ndim)
        D = pair_narrowing(A, q, K, M, ndim) * np.float32(narrow_scale)
        c2 = c * c
        for k in range(E.size):
            if E[k] == 0.0:
                continue
            los = np.float32(lo[k] * c2)
            his = np.float32(hi[k] * c2)
            if float(los) > float(lo[k]) * c2:
                los = np.nextafter(los, np.float32(-np.inf))
            if float(his) < float(hi[k]) * c2:
                his = np.nextafter(his, np.float32(np.inf))
            inb = (s32 >= lo[k]) & (s32 <= hi[k])
            above = inb & ((f32 - his) > -D)
            below = inb & ((los - f32) > -D)
            stats["narrow_wrong"] += int((s64[above] <= E[k]).sum() + (s64[below] >= E[k]).sum())
            if count:
                stats["in_band"] += int(inb.sum())
                stats["narrowed_decided"] += int((above | below).sum())
    # the bound at each pair's own separation
    ok = s64 > 0
    blo, bhi = bands(s64[ok])
    half = np.minimum(s64[ok] - blo.astype(np.float64), bhi.astype(np.float64) - s64[ok])
    err = np.abs(s32[ok] - s64[ok])
    ratio_band = err / half
    stats["pairs"] += int(s64.size)
    stats["max_ratio_band"] = max(stats["max_ratio_band"], float(ratio_band.max()))
    stats["max_ratio_raw"] = max(stats["max_ratio_raw"], float((ratio_band * SAFETY).max()))
    if tight:
        # each pair's own raw bound: its band half width less its narrowing,
        # divided by the safety factor
        half_t = half - D[ok].astype(np.float64) / (c * c)
        ratio = np.where(half_t > 0, err / np.maximum(half_t, 1e-300) * SAFETY, np.inf)
        stats["max_ratio_pair_raw"] = max(stats["max_ratio_pair_raw"], float(ratio.max()))


def new_stats():
    return {"pairs": 0, "max_ratio_band": 0.0, "max_ratio_raw": 0.0, "in_band": 0,
            "narrowed_decided": 0, "max_ratio_pair_raw": 0.0, "narrow_wrong": 0}


def scale_for(edges, S, top=32766.0 / 32767.0):
    """A coordinate scale like the library's: the top band just below the
    top of the rounding key (not a power of two)."""
    E = edges[-1] ** 2
    lo, hi = pc.fp32_bands(np.array([E]), 3, S)
    return math.sqrt(top * (1.0 - 2.0 ** -16) / float(hi[0]))


@pytest.mark.parametrize("case", ["r_box420", "r_box1100_k2", "rp_box1000", "chord_open",
                                  "r_box420_xy", "r_box1100_k2_xy", "rp_box1000_xy",
                                  "chord_open_xy"])
def test_fp32_bound_holds_on_1e8_pairs(case):
    """The _xy cases: the expanded form of x and y (cf_options.separation_form
    2) against its own bands, fewer pairs (the bound's arithmetic is the
    same emulation checked above, with other magnitudes)."""
    rng = synth.rng_for(sum(map(ord, case)))
    xy = case.endswith("_xy")
    case = case[:-3] if xy else case
    stats = new_stats()
    if case == "r_box420":
        L, reach, k, ndim = 420.0, 25.0, 1, 3
        edges = synth.log_edges(0.1, 25.0, 20)
        npairs = 40_000_000
    elif case == "r_box1100_k2":
        L, reach, k, ndim = 1100.0, 50.0, 2, 3
        edges = synth.log_edges(0.1, 50.0, 25)
        npairs = 20_000_000
    elif case == "rp_box1000":
        L, reach, k, ndim = 1000.0, 25.0, 1, 2
        edges = synth.log_edges(0.1, 25.0, 20)
        npairs = 20_000_000
    else:   # unit vectors, 3-D chord grid, no box
        L, reach, k, ndim = 0.0, 2 * math.sin(math.radians(5.0)), 1, 3
        edges = 2 * np.sin(np.radians(synth.log_edges(0.01, 10.0, 20)) / 2)
        npairs = 20_000_000
    if L > 0:
        g = plan(L, reach, k)
        S = L
    else:
        g = pc.plan_grid_refined([-1.0, -1.0, -1.0], [1.0, 1.0, 1.0], 0.0, reach, reach, 32,
                                 k, True)
        S = 2.0
    # the library's per-axis rounding bounds for column-local x and y (the
    # lane within k + 1/2 widths of the j column's centre, the j point within
    # half a width, each rounded once) and box-frame z
    def frame_eps(a_max, b_max):
        return U32 * (a_max + b_max) * (1 + 2.0 ** -20) + 8 * 2.0 ** -53 * S
    kk = g["k"]
    axis_eps = [frame_eps((kk + 0.5) * g["width"][0], 0.5 * g["width"][0]),
                frame_eps((kk + 0.5) * g["width"][1], 0.5 * g["width"][1]),
                frame_eps(S + reach, S)]
    # the lane's largest |x|, |y| in the j column's frame, the j point's
    xy_max = ([(kk + 0.5) * g["width"][0], (kk + 0.5) * g["width"][1],
               0.5 * g["width"][0], 0.5 * g["width"][1]] if xy else None)
    if xy:
        npairs //= 2
    for c in (1.0, scale_for(edges, S)):
        done = 0
        while done < npairs // 2:
            n = 2_000_000
            if L > 0:
                pi, pj = draw_pairs(rng, n, L, reach)
            else:
                pi = rng.normal(size=(n, 3))
                pi /= np.linalg.norm(pi, axis=1)[:, None]
                pj = pi + rng.normal(size=(n, 3)) * (reach / 2)
                pj /= np.linalg.norm(pj, axis=1)[:, None]
            check_contract(pi, pj, g, L, c, ndim, edges, axis_eps, S, stats, xy_max)
            done += n
        # adversarial: separations within a few ulps of every edge
        e_rep = np.repeat(edges[edges > 0], 20000)
        jitter = e_rep * (1.0 + rng.integers(-8, 9, e_rep.size) * 2.0 ** -52)
        if L > 0:
            pi, pj = draw_pairs(rng, e_rep.size, L, reach, radial=jitter)
            check_contract(pi, pj, g, L, c, ndim, edges, axis_eps, S, stats, xy_max,
                           count=False)
    print(case, "expanded" if xy else "differences", stats)
    assert stats["pairs"] >= npairs
    assert stats["max_ratio_raw"] < 1.0, stats
    assert stats["max_ratio_band"] < 1.0 / SAFETY, stats
    if xy:
        assert stats["narrow_wrong"] == 0, stats
        assert stats["max_ratio_pair_raw"] < 1.0, stats
        # the narrowing decides most random pairs the expanded bands leave
        # open
        assert stats["narrowed_decided"] > 0.5 * stats["in_band"], stats


def test_fixed_point_pi_within_margin():
    """Fixed-point z of the float32 DD(rp, pi) path: Zq = round((z - lo)
    2^k / dpi) as an integer and the periodic offset round(L 2^k / dpi); the
    integer |Zq_i + D - Zq_j| differs from the exact |dz| 2^k / dpi by at most
    1.5 quanta (three roundings to an integer), inside the 2-quanta margin,
    at the benchmark's boxes and on pairs placed on the pi edges."""
    rng = synth.rng_for(901)
    worst = 0.0
    for L, pimax, npi in ((420.0, 40.0, 40), (1000.0, 40.0, 40), (1100.0, 40.0, 13)):
        dpi = pimax / npi
        # the library's choice: as many quanta per pi bin as keep every value
        # below 2^29
        k = 24
        while k >= 4 and math.ldexp(L / dpi, k) > 2.0 ** 29:
            k -= 1
        inv = math.ldexp(1.0, k) / dpi
        zq_L = round(L * inv)
        n = 4_000_000
        zi = rng.uniform(0.0, L, n)
        dz = rng.uniform(-pimax * 1.1, pimax * 1.1, n)
        # and differences exactly on the pi edges and one ulp beside them
        q = np.arange(npi + 1) * dpi
        on = np.repeat(q, 2000)
        on = on * (1.0 + rng.integers(-1, 2, on.size) * 2.0 ** -52)
        dz[: on.size] = on * np.where(rng.random(on.size) < 0.5, -1.0, 1.0)
        zj = np.mod(zi - dz, L)
        d = zi - zj
        D = np.where(d > L / 2, -L, np.where(d <= -L / 2, L, 0.0))
        Zi = np.rint(zi * inv).astype(np.int64)
        Zj = np.rint(zj * inv).astype(np.int64)
        Dq = np.where(D > 0, zq_L, np.where(D < 0, -zq_L, 0))
        got = np.abs(Zi + Dq - Zj).astype(np.float64)
        exact = np.abs(d + D) * inv
        err = np.abs(got - exact)
        worst = max(worst, float(err.max()))
    print("fixed-point pi: worst error", worst, "quanta")
    assert worst <= 1.5 + 1e-6


def test_wrong_narrowing_is_caught():
    """The per-pair narrowing check is not vacuous: the same pairs (random
    and within a few ulps of every edge, DD(r) in the expanded form) pass
    with the sweep's narrowing and fail -- wrong decisions, or an error
    beyond a pair's remaining bound -- with the narrowing a quarter larger."""
    rng = synth.rng_for(4242)
    L, reach = 420.0, 25.0
    edges = synth.log_edges(0.1, 25.0, 20)
    g = plan(L, reach, 1)
    kk, w = g["k"], g["width"]

    def frame_eps(a_max, b_max):
        return U32 * (a_max + b_max) * (1 + 2.0 ** -20) + 8 * 2.0 ** -53 * L
    axis_eps = [frame_eps((kk + 0.5) * w[0], 0.5 * w[0]),
                frame_eps((kk + 0.5) * w[1], 0.5 * w[1]), frame_eps(L + reach, L)]
    xy_max = [(kk + 0.5) * w[0], (kk + 0.5) * w[1], 0.5 * w[0], 0.5 * w[1]]
    c = scale_for(edges, L)
    pi, pj = draw_pairs(rng, 1_000_000, L, reach)
    e_rep = np.repeat(edges, 20000)
    jitter = e_rep * (1.0 + rng.integers(-8, 9, e_rep.size) * 2.0 ** -52)
    qi, qj = draw_pairs(rng, e_rep.size, L, reach, radial=jitter)
    got = {}
    for scale in (1.0, 1.25):
        st = new_stats()
        check_contract(pi, pj, g, L, c, 3, edges, axis_eps, L, st, xy_max, narrow_scale=scale)
        check_contract(qi, qj, g, L, c, 3, edges, axis_eps, L, st, xy_max, count=False,
                       narrow_scale=scale)
        got[scale] = st
    print(got)
    assert got[1.0]["narrow_wrong"] == 0 and got[1.0]["max_ratio_pair_raw"] < 1.0
    assert got[1.25]["narrow_wrong"] > 0


def test_pair_margin_constants():
    """The narrowing constants the library hands the sweep are the bound's,
    rounded down: K = 1.25 u (1 + 2^-20) and M = c^2 times the magnitude term
    of the largest coordinates, never above those values and at most a
    relative 2^-22 below them; bad arguments are refused."""
    rng = synth.rng_for(4343)
    for _ in range(200):
        ndim = int(rng.integers(2, 4))
        xy_max = rng.uniform(0.0, 50.0, 4)
        c = float(np.exp(rng.uniform(-6.0, 3.0)))
        K, M = pc.fp32_pair_margin(xy_max, c, ndim)
        exact_K = SAFETY * U32 * (1 + 2.0 ** -20)
        exact_M = expand_mag(xy_max, ndim) * c * c
        assert exact_K * (1 - 2.0 ** -22) <= float(K) <= exact_K, (K, exact_K)
        assert exact_M * (1 - 2.0 ** -22) <= float(M) <= exact_M, (ndim, xy_max, c, M, exact_M)
    with pytest.raises(pc.PairCountError):
        pc.fp32_pair_margin([1.0, 1.0, 1.0, -1.0], 1.0, 3)
    with pytest.raises(pc.PairCountError):
        pc.fp32_pair_margin([1.0, 1.0, 1.0, 1.0], 0.0, 3)
    with pytest.raises(pc.PairCountError):
        pc.fp32_pair_margin([1.0, 1.0, 1.0, 1.0], 1.0, 4)
