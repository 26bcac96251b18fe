"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every ``pin_*`` function takes a loaded oracle library and raises
``AssertionError`` when the oracle disagrees with the fact it checks.  The same
functions run against the real oracle (``test_oracle.py``) and against copies of
it with deliberately planted mistakes (``test_oracle_mutations.py``), which must
each be caught by at least one pin.

Sources of truth used here:
  * hand-enumerated counts in ``tests/golden/*.json`` (each cites the passage);
  * exact rational arithmetic (``fractions``) on lattice inputs, where binary64
    is exact, with the periodic separation taken as the minimum over images;
  * closed-form expectations for uniform random points (Appendix B);
  * invariants the paper fixes (auto == cross(D, D), doubling, self-pairs);
  * exact scaling by powers of two, bin-merge additivity, permutation
    invariance, and reductions of one statistic to another;
  * Python's ``math.fsum`` for exactly rounded sums.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# --------------------------------------------------------------------------
# hand enumeration
# --------------------------------------------------------------------------
def pin_golden_r_edges(lib):
    g = _golden("r_edge_inclusion.json")
    pts = np.array(g["points"], dtype=np.float64)
    w = np.array(g["weights"], dtype=np.float64)
    for case in g["cases"]:
        c, ws = oracle.count_r(pts, None, case["edges"], g["boxsize"], w1=w, lib=lib)
        assert c.tolist() == case["counts"], (c, case)
        assert ws.tolist() == case["wsum"], (ws, case)
        c2, ws2 = oracle.count_r(pts, pts, case["edges"], g["boxsize"], w1=w, w2=w, lib=lib)
        assert c2.tolist() == case["counts"], (c2, case)
        assert ws2.tolist() == case["wsum"], (ws2, case)


def pin_golden_r_periodic(lib):
    for name in ("r_periodic_wrap.json", "r_corner_wrap.json"):
        g = _golden(name)
        pts = np.array(g["points"], dtype=np.float64)
        for case in g["cases"]:
            c, _ = oracle.count_r(pts, None, case["edges"], case["boxsize"], lib=lib)
            assert c.tolist() == case["counts"], (name, c, case)
            c2, _ = oracle.count_r(pts, pts, case["edges"], case["boxsize"], lib=lib)
            assert c2.tolist() == case["counts"], (name, c2, case)


def pin_golden_rppi(lib):
    g = _golden("rppi_small.json")
    pts = np.array(g["points"], dtype=np.float64)
    for case in g["cases"]:
        c, _ = oracle.count_rppi(pts, None, case["rp_edges"], g["pimax"], g["npi"],
                                 g["boxsize"], lib=lib)
        assert c.tolist() == case["counts"], (c, case)
        c2, _ = oracle.count_rppi(pts, pts, case["rp_edges"], g["pimax"], g["npi"],
                                  g["boxsize"], lib=lib)
        assert c2.tolist() == case["counts"], (c2, case)


def pin_golden_theta(lib):
    g = _golden("theta_small.json")
    rd = np.array(g["radec"], dtype=np.float64)
    for case in g["cases"]:
        c, _ = oracle.count_theta(rd[:, 0], rd[:, 1], None, None,
                                  case["theta_edges"], lib=lib)
        assert c.tolist() == case["counts"], (c, case)
        c2, _ = oracle.count_theta(rd[:, 0], rd[:, 1], rd[:, 0], rd[:, 1],
                                   case["theta_edges"], lib=lib)
        assert c2.tolist() == case["counts"], (c2, case)


# --------------------------------------------------------------------------
# exact arithmetic on lattice inputs
# --------------------------------------------------------------------------
def _min_image_sq(d: Fraction, L: Fraction | None) -> Fraction:
    """Squared axis separation, minimised over periodic images."""
    if L is None:
        return d * d
    return min((d + m * L) ** 2 for m in (-1, 0, 1))


def _exact_counts_r(pts, edges, L, auto=True, pts2=None):
    Q = [[Fraction(float(v)) for v in p] for p in pts]
    Q2 = Q if pts2 is None else [[Fraction(float(v)) for v in p] for p in pts2]
    E = [Fraction(float(e) * float(e)) for e in edges]
    Lf = None if L <= 0 else Fraction(float(L))
    nb = len(edges) - 1
    out = [0] * nb
    for a in range(len(Q)):
        for b in range(len(Q2)):
            s = sum(_min_image_sq(Q[a][k] - Q2[b][k], Lf) for k in range(3))
            for k in range(nb):
                if E[k] <= s < E[k + 1]:
                    out[k] += 1
    return out


def pin_lattice_exact_r(lib):
    L = 64
    pts = synth.lattice_box(50, L, seed=11, denom=1024)
    # a few coincident points and points on the box faces
    pts[1] = pts[0]
    pts[2, 0] = L
    pts[3, 1] = 0.0
    edges = np.array([0.0, 1.5, 4.0, 9.25, 16.0, 21.0])
    for box in (float(L), 0.0):
        want = _exact_counts_r(pts, edges, box)
        got, _ = oracle.count_r(pts, None, edges, box, lib=lib)
        assert got.tolist() == want, (box, got, want)
    # cross-correlation between two different lattice sets
    pts2 = synth.lattice_box(30, L, seed=12, denom=1024)
    want = _exact_counts_r(pts, edges, float(L), pts2=pts2)
    got, _ = oracle.count_r(pts, pts2, edges, float(L), lib=lib)
    assert got.tolist() == want, (got, want)


def pin_lattice_exact_rppi(lib):
    L = 64
    pts = synth.lattice_box(45, L, seed=13, denom=1024)
    pts[1] = pts[0]
    pts[5, 2] = L
    rp_edges = [0.0, 2.0, 5.5, 12.0, 20.0]
    pimax, npi = 16.0, 8
    q = [Fraction(2 * p) for p in range(npi + 1)]
    E = [Fraction(e) ** 2 for e in rp_edges]
    Q = [[Fraction(float(v)) for v in p] for p in pts]
    for box in (float(L), 0.0):
        Lf = None if box <= 0 else Fraction(box)
        want = np.zeros((len(rp_edges) - 1, npi), dtype=np.int64)
        for a in range(len(Q)):
            for b in range(len(Q)):
                rp2 = _min_image_sq(Q[a][0] - Q[b][0], Lf) + _min_image_sq(Q[a][1] - Q[b][1], Lf)
                pi = _min_image_sq(Q[a][2] - Q[b][2], Lf)  # squared; compare squared
                for k in range(len(rp_edges) - 1):
                    if not (E[k] <= rp2 < E[k + 1]):
                        continue
                    for p in range(npi):
                        if q[p] ** 2 <= pi < q[p + 1] ** 2:
                            want[k, p] += 1
        got, _ = oracle.count_rppi(pts, None, rp_edges, pimax, npi, box, lib=lib)
        assert (got == want).all(), (box, got, want)


def pin_weighted_exact(lib):
    """Weighted sums equal the exactly rounded rational sum of products."""
    pts = synth.lattice_box(40, 32, seed=21, denom=1024)
    rng = synth.rng_for(22)
    w = rng.uniform(0.5, 1.5, size=40)   # full 53-bit mantissas
    w2 = rng.uniform(-1.0, 2.0, size=40)
    edges = [0.0, 3.0, 7.0, 12.0]
    E = [Fraction(e) ** 2 for e in edges]
    Q = [[Fraction(float(v)) for v in p] for p in pts]
    Lf = Fraction(32)
    for auto in (True, False):
        wb = w if auto else w2
        sums = [Fraction(0)] * 3
        cnt = [0] * 3
        for a in range(40):
            for b in range(40):
                s = sum(_min_image_sq(Q[a][k] - Q[b][k], Lf) for k in range(3))
                for k in range(3):
                    if E[k] <= s < E[k + 1]:
                        # each product is rounded to binary64, then summed exactly
                        sums[k] += Fraction(float(w[a]) * float(wb[b]))
                        cnt[k] += 1
        if auto:
            c, ws = oracle.count_r(pts, None, edges, 32.0, w1=w, lib=lib)
        else:
            c, ws = oracle.count_r(pts, pts, edges, 32.0, w1=w, w2=w2, lib=lib)
        assert c.tolist() == cnt, (auto, c, cnt)
        assert ws.tolist() == [float(x) for x in sums], (auto, ws, sums)


def pin_xsum_vs_fsum(lib):
    rng = synth.rng_for(31)
    cases = [
        rng.normal(size=1000),
        np.concatenate([rng.normal(size=500) * 1e16, rng.normal(size=500)]),
        np.array([1e100, 1.0, -1e100, 1e-100, 3.0, -2.0]),
        np.array([0.1] * 10),
        np.array([2.0 ** 53, 1.0, 1e-30]),   # half-way case broken by a tiny tail
        np.array([1.0, 2.0 ** -53, 2.0 ** -106]),
    ]
    for v in cases:
        assert oracle.xsum(v, lib=lib) == math.fsum(v.tolist())


# --------------------------------------------------------------------------
# invariants fixed by the paper and by the arithmetic
# --------------------------------------------------------------------------
def pin_auto_equals_cross(lib):
    pts = synth.clustered_box(600, 50.0, seed=41, nblobs=20, sigma=1.0)
    w = synth.uniform_weights(600, seed=42).astype(np.float64)
    for edges in (synth.log_edges(0.05, 12.0, 10), np.r_[0.0, synth.log_edges(0.05, 12.0, 10)]):
        for box in (50.0, 0.0):
            ca, wa = oracle.count_r(pts, None, edges, box, w1=w, lib=lib)
            cc, wc = oracle.count_r(pts, pts, edges, box, w1=w, w2=w, lib=lib)
            assert (ca == cc).all(), (box, ca, cc)
            assert (wa == wc).all(), (box, wa, wc)
            ra, _ = oracle.count_rppi(pts, None, edges, 12.0, 6, box, lib=lib)
            rc, _ = oracle.count_rppi(pts, pts, edges, 12.0, 6, box, lib=lib)
            assert (ra == rc).all()
    ra, dec = synth.cap_radec(400, seed=43, radius_deg=5.0, clustered=True,
                              nblobs=20, sigma_deg=0.2)
    te = synth.log_edges(0.01, 3.0, 8)
    ta, _ = oracle.count_theta(ra, dec, None, None, te, lib=lib)
    tc, _ = oracle.count_theta(ra, dec, ra, dec, te, lib=lib)
    assert (ta == tc).all(), (ta, tc)


def pin_pair_convention(lib):
    """Auto counts are ordered pairs: even, plus N self-pairs in bin 0 iff the
    first edge is zero (Appendix B)."""
    pts = synth.uniform_box(300, 20.0, seed=51)
    pts[7] = pts[3]            # a coincident pair
    e_pos = synth.log_edges(0.1, 5.0, 6)
    c, _ = oracle.count_r(pts, None, e_pos, 20.0, lib=lib)
    assert all(int(x) % 2 == 0 for x in c)
    e0 = np.r_[0.0, e_pos]
    c0, _ = oracle.count_r(pts, None, e0, 20.0, lib=lib)
    # the coincident pair (2 ordered) + 300 self-pairs land below e_pos[0]
    assert int(c0[0]) == 300 + 2
    assert (c0[1:] == c).all()
    n = 300
    assert int(c0.sum()) <= n * n


def pin_bin_merge_and_total(lib):
    pts = synth.clustered_box(700, 60.0, seed=61, nblobs=30, sigma=1.5)
    edges = synth.log_edges(0.2, 14.0, 12)
    c, _ = oracle.count_r(pts, None, edges, 60.0, lib=lib)
    merged = np.delete(edges, [3, 7, 8])
    cm, _ = oracle.count_r(pts, None, merged, 60.0, lib=lib)
    # removing edges 3, 7 and 8 merges bins (2, 3) and (6, 7, 8)
    want = [c[0], c[1], c[2] + c[3], c[4], c[5], c[6] + c[7] + c[8], c[9], c[10], c[11]]
    assert cm.tolist() == [int(x) for x in want], (cm, want)
    one, _ = oracle.count_r(pts, None, [edges[0], edges[-1]], 60.0, lib=lib)
    assert int(one[0]) == int(c.sum())


def pin_permutation_and_scaling(lib):
    pts = synth.clustered_box(500, 40.0, seed=71, nblobs=25, sigma=1.0)
    w = synth.uniform_weights(500, seed=72).astype(np.float64)
    edges = synth.log_edges(0.1, 9.0, 9)
    c, ws = oracle.count_r(pts, None, edges, 40.0, w1=w, lib=lib)
    perm = synth.rng_for(73).permutation(500)
    cp, wsp = oracle.count_r(pts[perm], None, edges, 40.0, w1=w[perm], lib=lib)
    assert (c == cp).all() and (ws == wsp).all()
    for m in (-3, 5):
        f = 2.0 ** m
        cs, wss = oracle.count_r(pts * f, None, edges * f, 40.0 * f, w1=w * f, lib=lib)
        assert (cs == c).all(), (m, cs, c)
        assert (wss == ws * f * f).all(), (m, wss, ws)
    ones = np.ones(500)
    c1, w1 = oracle.count_r(pts, None, edges, 40.0, w1=ones, lib=lib)
    assert (w1 == c1.astype(np.float64)).all()


def pin_periodic_interior(lib):
    """With every point inside a sub-box narrower than L/2 no wrap can trigger,
    so periodic and non-periodic counts agree exactly."""
    rng = synth.rng_for(81)
    pts = 30.0 + rng.uniform(0.0, 39.0, size=(500, 3))
    edges = synth.log_edges(0.5, 15.0, 8)
    a, _ = oracle.count_r(pts, None, edges, 100.0, lib=lib)
    b, _ = oracle.count_r(pts, None, edges, 0.0, lib=lib)
    assert (a == b).all()
    a, _ = oracle.count_rppi(pts, None, edges, 20.0, 5, 100.0, lib=lib)
    b, _ = oracle.count_rppi(pts, None, edges, 20.0, 5, 0.0, lib=lib)
    assert (a == b).all()


def pin_rppi_reductions(lib):
    """(1) With all z equal, pi = 0 and rp^2 is exactly the 3-D s, so DD(rp,pi)
    puts DD(r) into pi bin 0.  (2) With x = y = 0 on lattice inputs, rp = 0 and
    the pi histogram equals the r histogram over the pi edges."""
    pts = synth.clustered_box(500, 50.0, seed=91, nblobs=20, sigma=1.0)
    pts[:, 2] = 7.0
    edges = synth.log_edges(0.1, 12.0, 10)
    cr, _ = oracle.count_r(pts, None, edges, 50.0, lib=lib)
    cp, _ = oracle.count_rppi(pts, None, edges, 10.0, 5, 50.0, lib=lib)
    assert (cp[:, 0] == cr).all() and (cp[:, 1:] == 0).all()
    lat = synth.lattice_box(200, 64, seed=92)
    lat[:, 0] = 0.0
    lat[:, 1] = 0.0
    q = oracle.pi_edges(16.0, 8, lib=lib)
    assert q.tolist() == [2.0 * p for p in range(9)]
    cp, _ = oracle.count_rppi(lat, None, [0.0, 1.0], 16.0, 8, 64.0, lib=lib)
    cr, _ = oracle.count_r(lat, None, q, 64.0, lib=lib)
    assert (cp[0] == cr).all(), (cp, cr)


def pin_inclusion_r_in_rppi(lib):
    """r < R implies rp < R and pi < R, so counts inside the sphere never exceed
    counts inside the enclosing cylinder; the cylinder of half-height R has
    3/2 the sphere's volume, which the uniform counts must reflect."""
    pts = synth.uniform_box(2500, 50.0, seed=101)
    R = 6.0
    cr, _ = oracle.count_r(pts, None, [0.0, R], 50.0, lib=lib)
    cp, _ = oracle.count_rppi(pts, None, [0.0, R], R, 1, 50.0, lib=lib)
    assert int(cr[0]) <= int(cp[0, 0])
    ratio = (int(cp[0, 0]) - 2500) / (int(cr[0]) - 2500)
    assert abs(ratio - 1.5) < 0.1, ratio


def _zscores(got, expect):
    return (got.astype(np.float64) - expect) / np.sqrt(np.maximum(2.0 * expect, 1.0))


def pin_uniform_analytic(lib):
    """Appendix B: for N uniform points in a periodic box the expected ordered
    pair count in a shell is N (N-1) dV / V (variance ~ 2x the mean)."""
    N, L = 4000, 100.0
    pts = synth.uniform_box(N, L, seed=111)
    e = synth.log_edges(0.5, 20.0, 10)
    c, _ = oracle.count_r(pts, None, e, L, lib=lib)
    exp = N * (N - 1) * (4.0 / 3.0) * np.pi * (e[1:] ** 3 - e[:-1] ** 3) / L ** 3
    assert np.all(np.abs(_zscores(c, exp)) < 5), _zscores(c, exp)
    pimax, npi = 20.0, 5
    cp, _ = oracle.count_rppi(pts, None, e, pimax, npi, L, lib=lib)
    dpi = pimax / npi
    expp = (N * (N - 1) * np.pi * (e[1:] ** 2 - e[:-1] ** 2) * 2 * dpi / L ** 3)[:, None] \
        * np.ones(npi)[None, :]
    assert np.all(np.abs(_zscores(cp, expp)) < 5), _zscores(cp, expp)
    # full sphere: uniform directions, expected N(N-1)(cos t0 - cos t1)/2
    rng = synth.rng_for(112)
    v = rng.normal(size=(3000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    ra = np.mod(np.degrees(np.arctan2(v[:, 1], v[:, 0])), 360.0)
    dec = np.degrees(np.arcsin(v[:, 2]))
    te = np.array([1.0, 5.0, 20.0, 45.0, 90.0, 135.0, 179.0])
    ct, _ = oracle.count_theta(ra, dec, None, None, te, lib=lib)
    n = 3000
    expt = n * (n - 1) * (np.cos(np.radians(te[:-1])) - np.cos(np.radians(te[1:]))) / 2
    assert np.all(np.abs(_zscores(ct, expt)) < 5), _zscores(ct, expt)


def pin_theta_conversion(lib):
    """Unit vectors have unit norm, reproduce cos(theta) = v1.v2 of Appendix A,
    and chord edges satisfy c^2 = 2 - 2 cos(theta)."""
    rng = synth.rng_for(121)
    ra = rng.uniform(0, 360, 200)
    dec = rng.uniform(-90, 90, 200)
    v = oracle.radec_to_unit(ra, dec, lib=lib)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    # independent spherical law of cosines for the angle between two points
    a1, d1 = np.radians(ra[:100]), np.radians(dec[:100])
    a2, d2 = np.radians(ra[100:]), np.radians(dec[100:])
    cosang = np.sin(d1) * np.sin(d2) + np.cos(d1) * np.cos(d2) * np.cos(a1 - a2)
    dots = np.sum(v[:100] * v[100:], axis=1)
    assert np.allclose(dots, cosang, atol=1e-14)
    assert np.allclose(v[:, 2], np.sin(np.radians(dec)), atol=1e-15)
    assert np.allclose(np.arctan2(v[:, 1], v[:, 0]) % (2 * np.pi), np.radians(ra) % (2 * np.pi),
                       atol=1e-12)
    t = np.array([0.0, 0.01, 1.0, 10.0, 60.0, 90.0, 179.0])
    c = oracle.theta_chord_edges(t, lib=lib)
    # 2 - 2 cos(t) cancels for small t: allow its absolute rounding (~4e-16)
    assert np.allclose(c * c, 2.0 - 2.0 * np.cos(np.radians(t)), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# pair weight types and the mean separation per bin
# --------------------------------------------------------------------------
def _exact_chain_stats(x, z, w, edges, L, wtype, rp_edges_pi=None):
    """Exact per-bin count, weight sum and separation-weight sum over all
    ordered pairs (self-pairs included) of points (x_a, 2, z_a) whose pair
    separations are integers: r = |dx| with z constant, or rp = |dx| and
    pi = |dz| for the (rp, pi) case (rp_edges_pi = (pimax, npi))."""
    Lf = None if L <= 0 else Fraction(L)
    n = len(x)
    E = [Fraction(float(e) * float(e)) for e in edges]
    nb = len(edges) - 1
    npi = 1 if rp_edges_pi is None else rp_edges_pi[1]
    cnt = [[0] * npi for _ in range(nb)]
    ws = [[Fraction(0)] * npi for _ in range(nb)]
    rs = [[Fraction(0)] * npi for _ in range(nb)]
    for a in range(n):
        for b in range(n):
            dx2 = _min_image_sq(Fraction(x[a]) - Fraction(x[b]), Lf)
            d = Fraction(math.isqrt(int(dx2)))
            assert d * d == dx2
            p = 0
            if rp_edges_pi is not None:
                pimax, _ = rp_edges_pi
                dz = Fraction(math.isqrt(int(_min_image_sq(Fraction(z[a]) - Fraction(z[b]), Lf))))
                if dz >= pimax:
                    continue
                p = int(dz // (Fraction(pimax) / npi))
            for k in range(nb):
                if E[k] <= dx2 < E[k + 1]:
                    wab = Fraction(w[a]) * Fraction(w[b]) if wtype == "product" else \
                        Fraction(w[a]) + Fraction(w[b])
                    cnt[k][p] += 1
                    ws[k][p] += wab
                    rs[k][p] += d * wab
    return cnt, ws, rs


def pin_ravg_chain_r(lib):
    """Mean separation on a chain with integer separations: every sum is an
    integer, so the oracle's rounded quotient equals the exact rational mean
    rounded once; unit weights give the plain mean."""
    x = [0.5, 1.5, 2.5, 3.5, 5.5, 8.5, 13.5, 14.5]
    pts = np.array([[v, 2.0, 2.0] for v in x])
    w = np.array([1.0, 2.0, 3.0, 1.0, 4.0, 2.0, 5.0, 3.0])
    for edges in ([0.0, 1.5, 2.5, 6.5, 12.5], [0.5, 1.5, 4.5, 9.5]):
        for box in (32.0, 0.0):
            for wtype in ("product", "sum"):
                cnt, ws, rs = _exact_chain_stats(x, None, w, edges, box, wtype)
                c, gw, rv = oracle.count_r(pts, None, edges, box, w1=w, lib=lib,
                                           weight_type=wtype, ravg=True)
                assert c.tolist() == [v[0] for v in cnt], (edges, box, c, cnt)
                assert gw.tolist() == [float(v[0]) for v in ws], (edges, box, wtype, gw)
                want = [float(r[0] / q[0]) if q[0] else 0.0 for r, q in zip(rs, ws)]
                assert rv.tolist() == want, (edges, box, wtype, rv, want)
            one = np.ones(len(x))
            cnt, ws, rs = _exact_chain_stats(x, None, one, edges, box, "product")
            c, _, rv = oracle.count_r(pts, None, edges, box, lib=lib, ravg=True)
            want = [float(r[0] / k[0]) if k[0] else 0.0 for r, k in zip(rs, cnt)]
            assert rv.tolist() == want, (edges, box, rv, want)
            # cross-correlation of the chain with itself gives the same means
            _, _, rx = oracle.count_r(pts, pts.copy(), edges, box, lib=lib, ravg=True)
            assert rx.tolist() == want


def pin_ravg_chain_rppi(lib):
    """Mean rp per (rp, pi) bin on a chain with integer rp and pi."""
    x = [0.0, 1.0, 3.0, 4.0, 7.0, 11.0]
    z = [0.0, 2.0, 1.0, 5.0, 3.0, 9.0]
    pts = np.array([[a, 2.0, b] for a, b in zip(x, z)])
    w = np.array([2.0, 1.0, 3.0, 1.0, 2.0, 4.0])
    edges = [0.0, 1.5, 3.5, 8.5]
    pimax, npi = 8.0, 4
    for box in (24.0, 0.0):
        for wtype in ("product", "sum"):
            cnt, ws, rs = _exact_chain_stats(x, z, w, edges, box, wtype, (pimax, npi))
            c, gw, rv = oracle.count_rppi(pts, None, edges, pimax, npi, box, w1=w, lib=lib,
                                          weight_type=wtype, ravg=True)
            assert c.tolist() == cnt, (box, c, cnt)
            want = [[float(r / q) if q else 0.0 for r, q in zip(rr, qq)] for rr, qq in zip(rs, ws)]
            assert rv.tolist() == want, (box, wtype, rv, want)


def pin_ravg_theta_equator(lib):
    """Points on the equator: the angle of a pair is the difference of RA,
    so each bin's mean angle is a known rational (to the rounding of the
    trigonometric round trip, about 1e-15 relative)."""
    ra = np.array([0.0, 1.0, 2.5, 4.0, 7.0, 12.0])
    dec = np.zeros_like(ra)
    w = np.array([1.0, 3.0, 2.0, 2.0, 1.0, 4.0])
    edges = [0.5, 1.75, 3.25, 6.0, 13.0]
    for wtype in ("product", "sum"):
        c, gw, rv = oracle.count_theta(ra, dec, theta_edges_deg=edges, w1=w, lib=lib,
                                       weight_type=wtype, ravg=True)
        for k in range(len(edges) - 1):
            num = den = Fraction(0)
            n = 0
            for a in range(ra.size):
                for b in range(ra.size):
                    t = Fraction(abs(ra[a] - ra[b]))
                    if Fraction(edges[k]) <= t < Fraction(edges[k + 1]):
                        wab = Fraction(w[a]) * Fraction(w[b]) if wtype == "product" else \
                            Fraction(w[a]) + Fraction(w[b])
                        num += t * wab
                        den += wab
                        n += 1
            assert int(c[k]) == n, (k, c, n)
            want = float(num / den) if den else 0.0
            assert abs(rv[k] - want) <= 1e-13 * max(want, 1.0), (wtype, k, rv[k], want)


def pin_ravg_inside_bins(lib):
    """Each non-empty bin's mean separation lies inside the bin (positive
    weights), on clustered points, for r, rp and theta."""
    pts = synth.clustered_box(700, 30.0, seed=91, nblobs=6, sigma=1.5)
    w = synth.uniform_weights(700, seed=92)
    e = synth.log_edges(0.2, 6.0, 8)
    for box in (30.0, 0.0):
        c, _, rv = oracle.count_r(pts, None, e, box, w1=w, lib=lib, ravg=True)
        for k in range(e.size - 1):
            if c[k]:
                assert e[k] <= rv[k] <= e[k + 1], (box, k, rv[k])
        c, _, rv = oracle.count_rppi(pts, None, e, 5.0, 5, box, lib=lib, ravg=True)
        for k in range(e.size - 1):
            for p in range(5):
                if c[k, p]:
                    assert e[k] <= rv[k, p] <= e[k + 1], (box, k, p, rv[k, p])
    ra, dec = synth.cap_radec(600, seed=93, clustered=True)
    te = synth.log_edges(0.05, 8.0, 8)
    c, _, rv = oracle.count_theta(ra, dec, theta_edges_deg=te, lib=lib, ravg=True,
                                  w1=w[:600], weight_type="sum")
    for k in range(te.size - 1):
        if c[k]:
            assert te[k] * (1 - 1e-12) <= rv[k] <= te[k + 1] * (1 + 1e-12), (k, rv[k])


# --------------------------------------------------------------------------
# on-sky (rp, pi): line of sight through the pair's midpoint
# --------------------------------------------------------------------------
def _mocks_exact(P, rp_edges, pimax, npi):
    """Exact counts of all ordered pairs of integer positions P: with
    s = v1 - v2 and L = v1 + v2, pi^2 = (s.L)^2 / (L.L) and
    rp^2 = s.s - pi^2 as rationals, compared with squared edges."""
    E = [Fraction(float(e)) ** 2 for e in rp_edges]
    q = [(Fraction(pimax) * p / npi) ** 2 for p in range(npi + 1)]
    nb = len(rp_edges) - 1
    want = np.zeros((nb, npi), dtype=np.int64)
    for a in P:
        for b in P:
            s = [Fraction(int(a[k]) - int(b[k])) for k in range(3)]
            L = [Fraction(int(a[k]) + int(b[k])) for k in range(3)]
            sl = sum(s[k] * L[k] for k in range(3))
            ll = sum(L[k] * L[k] for k in range(3))
            ss = sum(s[k] * s[k] for k in range(3))
            pi2 = sl * sl / ll if ll else Fraction(0)
            rp2 = ss - pi2
            if pi2 >= q[npi]:
                continue
            for k in range(nb):
                if E[k] <= rp2 < E[k + 1]:
                    p = max(i for i in range(npi) if q[i] <= pi2)
                    want[k, p] += 1
    return want


def pin_mocks_lattice_exact(lib):
    """Integer positions: every intermediate of the definition is exact or
    decided far from its rounding, so the oracle must equal exact rational
    arithmetic (including pairs exactly on a pi edge, which are radial)."""
    rng = synth.rng_for(95)
    P = rng.integers(-6, 7, size=(60, 3)) + np.array([40, -25, 30])
    P[1] = P[0]                    # a coincident pair
    P[2] = 2 * P[3]                # a radial pair (same line of sight)
    rp_edges = [0.0, 1.25, 2.5, 4.75, 8.5]
    pimax, npi = 8.0, 8
    want = _mocks_exact(P, rp_edges, pimax, npi)
    got, _ = oracle.count_rppi_mocks(P.astype(np.float64), None, rp_edges, pimax, npi, lib=lib)
    assert (got == want).all(), (got, want)
    Q = rng.integers(-5, 6, size=(40, 3)) + np.array([38, -20, 33])
    wantx = _mocks_exact_cross(P, Q, rp_edges, pimax, npi)
    gotx, _ = oracle.count_rppi_mocks(P.astype(np.float64), Q.astype(np.float64), rp_edges,
                                      pimax, npi, lib=lib)
    assert (gotx == wantx).all(), (gotx, wantx)


def _mocks_exact_cross(P, Q, rp_edges, pimax, npi):
    both = _mocks_exact(np.concatenate([P, Q]), rp_edges, pimax, npi)
    return (both - _mocks_exact(P, rp_edges, pimax, npi) - _mocks_exact(Q, rp_edges, pimax, npi)) // 2


def pin_mocks_closed_forms(lib):
    """Points on one line of sight have rp = 0 and pi = |D1 - D2|; a pair
    mirrored across a line of sight has pi = 0 and rp = its full
    separation; the mean rp of a mirrored pair is that separation."""
    D = np.array([100.0, 103.0, 107.5, 111.0, 131.0])
    for axis in range(3):
        P = np.zeros((D.size, 3))
        P[:, axis] = D
        c, _ = oracle.count_rppi_mocks(P, None, [0.0, 0.5], 20.0, 20, lib=lib)
        want = np.zeros((1, 20), dtype=np.int64)
        want[0, 0] += D.size
        for a in range(D.size):
            for b in range(D.size):
                if a != b and abs(D[a] - D[b]) < 20.0:
                    want[0, int(abs(D[a] - D[b]))] += 1
        assert (c == want).all(), (axis, c, want)
    # two points at the same distance from the observer have s.L =
    # |v1|^2 - |v2|^2 = 0, so pi = 0 and rp = |s|; the two mirrored pairs
    # are 100 apart, far outside the bins
    M = np.array([[500.0, 3.0, -4.0], [500.0, -3.0, 4.0], [600.0, 6.0, 8.0],
                  [600.0, -6.0, -8.0]])
    c, _, rv = oracle.count_rppi_mocks(M, None, [1.0, 10.5, 20.5], 1.0, 1, lib=lib, ravg=True)
    assert c.tolist() == [[2], [2]], c
    assert rv[0, 0] == 10.0 and rv[1, 0] == 20.0, rv


def pin_mocks_symmetries(lib):
    """Exact symmetries: a quarter turn about any axis, swapping the two
    catalogues, and doubling every length (positions, edges, pimax)."""
    P = synth.cap_radec(300, seed=96, radius_deg=3.0)
    d = 400.0 + 60.0 * synth.rng_for(97).random(300)
    X = oracle.sky_to_cartesian(P[0], P[1], d, lib=lib)
    Y = oracle.sky_to_cartesian(*synth.cap_radec(200, seed=98, radius_deg=3.0),
                                420.0 + 30.0 * synth.rng_for(99).random(200), lib=lib)
    e = synth.log_edges(0.5, 12.0, 6)
    base, _ = oracle.count_rppi_mocks(X, Y, e, 15.0, 5, lib=lib)
    assert base.sum() > 0
    rot = X[:, [1, 0, 2]] * np.array([-1.0, 1.0, 1.0])
    roty = Y[:, [1, 0, 2]] * np.array([-1.0, 1.0, 1.0])
    assert (oracle.count_rppi_mocks(rot, roty, e, 15.0, 5, lib=lib)[0] == base).all()
    rot = X[:, [0, 2, 1]] * np.array([1.0, 1.0, -1.0])
    roty = Y[:, [0, 2, 1]] * np.array([1.0, 1.0, -1.0])
    assert (oracle.count_rppi_mocks(rot, roty, e, 15.0, 5, lib=lib)[0] == base).all()
    assert (oracle.count_rppi_mocks(Y, X, e, 15.0, 5, lib=lib)[0] == base).all()
    assert (oracle.count_rppi_mocks(2 * X, 2 * Y, 2 * e, 30.0, 5, lib=lib)[0] == base).all()


def pin_sky_to_cartesian(lib):
    ra = np.array([0.0, 90.0, 180.0, 0.0, 45.0])
    dec = np.array([0.0, 0.0, 0.0, 90.0, 0.0])
    D = np.array([10.0, 20.0, 30.0, 40.0, 50.0])
    v = oracle.sky_to_cartesian(ra, dec, D, lib=lib)
    want = np.array([[10, 0, 0], [0, 20, 0], [-30, 0, 0], [0, 0, 40],
                     [50 / math.sqrt(2), 50 / math.sqrt(2), 0]])
    assert np.allclose(v, want, rtol=0, atol=1e-13), v
    assert np.allclose(np.linalg.norm(v, axis=1), D, rtol=1e-15)


def pin_pi_edges_inexact_width(lib):
    """pi edges for a width pimax/npi that binary64 cannot hold (reading of
    Appendix A's linear pi bins): q_p is p times the rounded width, rounded
    once more, q_npi = pimax, and a bin is half-open.  The expected edges come
    from exact rational arithmetic (Fraction) rounded by Python's
    correctly-rounded conversion; pairs placed exactly on each edge and one
    ulp below it must land in the upper and lower bin respectively.  With
    pimax = 10 and npi = 9 the edge q_7 differs from the once-rounded 70/9,
    so the rounding order is visible; with pimax = 13 and npi = 23 the width
    times npi falls one ulp short of pimax, so the top edge must be pimax
    itself."""
    for pimax, npi in ((10.0, 9), (13.0, 23)):
        width = float(Fraction(pimax) / npi)
        want = [float(Fraction(p) * Fraction(width)) for p in range(npi)] + [pimax]
        if npi == 9:
            assert want[7] != float(Fraction(7) * Fraction(pimax) / npi)
        else:
            assert float(Fraction(npi) * Fraction(width)) != pimax
        q = oracle.pi_edges(pimax, npi, lib=lib)
        assert q.tolist() == want, (q, want)
        zs, expect = [], np.zeros(npi, dtype=np.int64)
        for p in range(1, npi + 1):
            on, below = want[p], math.nextafter(want[p], 0.0)
            zs += [on, below]
            if p < npi:
                expect[p] += 1
            expect[p - 1] += 1
        d1 = np.array([[1.0, 2.0, 0.0]])
        d2 = np.array([[1.0, 2.0, z] for z in zs])
        c, _ = oracle.count_rppi(d1, d2, [0.0, 1.0], pimax, npi, 0.0, lib=lib)
        assert c[0].tolist() == expect.tolist(), (pimax, npi, c, expect)
        c, _ = oracle.count_rppi(d2, d1, [0.0, 1.0], pimax, npi, 0.0, lib=lib)
        assert c[0].tolist() == expect.tolist(), (pimax, npi, c, expect)

def pin_pruned_equals_plain(lib):
    """The exactly pruned variants (one axis sorted, pairs beyond the reach
    along it skipped) give the plain oracle's counts and exactly rounded
    weighted sums bit for bit: periodic and open boxes, auto and cross,
    float32-valued inputs, lattice inputs with exact edge ties, every
    pruning axis, DD(rp, pi) with its pi reach along z, and DD(theta)."""
    pts = synth.clustered_box(2500, 60.0, seed=121, nblobs=40, sigma=1.5)
    w = synth.uniform_weights(2500, seed=122)
    e = synth.log_edges(0.2, 20.0, 9)
    for box in (60.0, 0.0):
        want = oracle.count_r(pts, None, e, box, w1=w, lib=lib)
        for ax in range(3):
            got = oracle.count_r_pruned(pts, None, e, box, w1=w, axis=ax, lib=lib)
            assert (got[0] == want[0]).all(), (box, ax, got[0], want[0])
            assert got[1].tolist() == want[1].tolist(), (box, ax)
        a, b = pts[:900], pts[900:]
        want = oracle.count_rppi(a, b, e, 14.0, 7, box, w1=w[:900], w2=w[900:], lib=lib)
        for ax in range(3):
            got = oracle.count_rppi_pruned(a, b, e, 14.0, 7, box, w1=w[:900], w2=w[900:],
                                           axis=ax, lib=lib)
            assert (got[0] == want[0]).all(), (box, ax)
            assert got[1].tolist() == want[1].tolist(), (box, ax)
    f32 = pts.astype(np.float32)
    assert (oracle.count_r_pruned(f32, None, e, 60.0, lib=lib)[0]
            == oracle.count_r(f32, None, e, 60.0, lib=lib)[0]).all()
    lat = synth.lattice_box(1500, 32, seed=123)
    el = [0.0, 1.0, 2.0, 3.0, 5.0, 8.0]
    for ax in range(3):
        assert (oracle.count_r_pruned(lat, None, el, 32.0, axis=ax, lib=lib)[0]
                == oracle.count_r(lat, None, el, 32.0, lib=lib)[0]).all()
        assert (oracle.count_rppi_pruned(lat, None, el, 4.0, 4, 32.0, axis=ax, lib=lib)[0]
                == oracle.count_rppi(lat, None, el, 4.0, 4, 32.0, lib=lib)[0]).all()
    ra, dec = synth.cap_radec(1500, seed=124, radius_deg=20.0, clustered=True,
                              nblobs=30, sigma_deg=0.5)
    ra2, dec2 = synth.cap_radec(700, seed=125, radius_deg=20.0)
    te = synth.log_edges(0.05, 8.0, 8)
    want = oracle.count_theta(ra, dec, None, None, te, lib=lib)[0]
    wantx = oracle.count_theta(ra, dec, ra2, dec2, te, lib=lib)[0]
    for ax in range(3):
        assert (oracle.count_theta_pruned(ra, dec, None, None, te, axis=ax, lib=lib)[0]
                == want).all(), ax
        assert (oracle.count_theta_pruned(ra, dec, ra2, dec2, te, axis=ax, lib=lib)[0]
                == wantx).all(), ax


ALL_PINS = [
    pin_golden_r_edges,
    pin_golden_r_periodic,
    pin_golden_rppi,
    pin_golden_theta,
    pin_lattice_exact_r,
    pin_lattice_exact_rppi,
    pin_weighted_exact,
    pin_xsum_vs_fsum,
    pin_auto_equals_cross,
    pin_pair_convention,
    pin_bin_merge_and_total,
    pin_permutation_and_scaling,
    pin_periodic_interior,
    pin_rppi_reductions,
    pin_inclusion_r_in_rppi,
    pin_uniform_analytic,
    pin_theta_conversion,
    pin_ravg_chain_r,
    pin_ravg_chain_rppi,
    pin_ravg_theta_equator,
    pin_ravg_inside_bins,
    pin_mocks_lattice_exact,
    pin_mocks_closed_forms,
    pin_mocks_symmetries,
    pin_sky_to_cartesian,
    pin_pi_edges_inexact_width,
    pin_pruned_equals_plain,
]
