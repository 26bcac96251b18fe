"""Host-only checks of the angular grid planner (declination bands and
right-ascension cells), no GPU needed.

The planner's promise: two unit vectors whose binary64 chord is below the
chord reach lie in cells the enumeration connects (same, neighbouring band;
right-ascension cell within the band pair's reach, round the circle) and at
most `zreach` declination slices apart.  The test assigns cells with the same
arithmetic the gridding kernel uses (atan2 of the components, floor, clamp)
and walks the neighbour enumeration the work-list kernel performs; the pairs
are drawn to stress the bounds: separations just under the reach, pairs along
a parallel (largest right-ascension difference) near the poles and band
edges, and pairs across the RA = 0 / 360 seam.
"""
import math

import numpy as np
import pytest

import paper_1911_03545_amd as pcm
import synth


def chord_of(theta_deg):
    return 2.0 * math.sin(0.5 * math.radians(theta_deg))


def cells(plan, v):
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    dec = np.arctan2(z, np.sqrt(x * x + y * y))
    ra = np.arctan2(y, x)
    ra = np.where(ra < 0.0, ra + 2.0 * np.pi, ra)
    S, nb = plan["slices"], plan["nband"]
    t = (dec - plan["dec_lo"]) * plan["inv_slice"]
    gs = np.where(t > 0.0, np.minimum(np.floor(np.where(t > 0, t, 0)), nb * S - 1), 0).astype(int)
    b = gs // S
    nra = plan["nra"][b]
    u = ra * plan["ra_scale"][b]
    a = np.where(u > 0.0, np.minimum(np.floor(np.where(u > 0, u, 0)), nra - 1), 0).astype(int)
    return b, a, gs


def neighbour_cells(plan, b, a):
    """Cells (band, RA cell) the cross-correlation enumeration visits."""
    out = set()
    for d in (-1, 0, 1):
        b2 = b + d
        if b2 < 0 or b2 >= plan["nband"]:
            continue
        n2 = int(plan["nra"][b2])
        D = plan["dra"][b][d + 1]
        ks = range(n2)
        if D < math.pi:
            x0 = (a / plan["ra_scale"][b] - D) * plan["ra_scale"][b2]
            x1 = ((a + 1) / plan["ra_scale"][b] + D) * plan["ra_scale"][b2]
            f0, f1 = math.floor(x0), math.floor(x1)
            if f1 - f0 + 1 < n2:
                ks = range(f0, f1 + 1)
        for k in ks:
            out.add((b2, k % n2))
    return out


def unit(v):
    return v / np.linalg.norm(v, axis=1)[:, None]


def stress_pairs(rng, theta_deg, zlo, zhi, n):
    """Pairs of unit vectors with chord below the reach, many near it."""
    th = math.radians(theta_deg)
    dlo, dhi = math.asin(zlo), math.asin(zhi)
    # first points: uniform in the declination range, plus points near the
    # range ends and near the poles
    dec = rng.uniform(dlo, dhi, n)
    dec[: n // 8] = np.clip(dhi - rng.uniform(0, min(th, dhi - dlo), n // 8), dlo, dhi)
    dec[n // 8: n // 4] = np.clip(dlo + rng.uniform(0, min(th, dhi - dlo), n // 8), dlo, dhi)
    ra = rng.uniform(0, 2 * np.pi, n)
    ra[n // 4: n // 3] = rng.uniform(0, 1e-6, n // 3 - n // 4)      # seam
    v1 = np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], 1)
    # second points: rotate towards a random tangent direction by rho * theta
    east = np.stack([-np.sin(ra), np.cos(ra), np.zeros(n)], 1)
    north = np.cross(v1, east)
    phi = rng.uniform(0, 2 * np.pi, n)
    phi[: n // 2] = rng.choice([0.0, np.pi], n // 2)                 # along a parallel
    rho = 1.0 - rng.uniform(0, 1e-3, n) ** 2
    ang = rho * th
    tdir = np.cos(phi)[:, None] * east + np.sin(phi)[:, None] * north
    v2 = np.cos(ang)[:, None] * v1 + np.sin(ang)[:, None] * tdir
    # along a parallel exactly: same declination, RA difference at the reach
    m = slice(n // 2, n // 2 + n // 8)
    cosd = np.cos(dec[m])
    s = math.sin(th / 2) / np.maximum(cosd, 1e-300)
    dra = np.where(s < 1, 2 * np.arcsin(np.minimum(s, 1.0)), np.pi) * (1 - 1e-9)
    sgn = rng.choice([-1.0, 1.0], dra.size)
    ra2 = ra[m] + sgn * dra
    v2[m] = np.stack([cosd * np.cos(ra2), cosd * np.sin(ra2), np.sin(dec[m])], 1)
    return v1, v2


def edge_pairs(plan, rng, theta_deg, zlo, zhi, per_band=400):
    """Pairs at the right-ascension reach itself: both points on the band's
    parallel furthest from the equator (where cos(dec) is smallest), the
    second one just past a cell boundary, so that any shortfall in the
    planned reach loses some of them; and pairs straddling a band edge."""
    th = math.radians(theta_deg)
    dlo, dhi = math.asin(zlo), math.asin(zhi)
    h = plan["band_height"]
    v1, v2 = [], []
    for b in range(plan["nband"]):
        d0 = plan["dec_lo"] + b * h
        d1 = d0 + h
        for dec in (d0 + 1e-12, d1 - 1e-12, d1 + 1e-12):
            if not (dlo <= dec <= dhi):
                continue
            r = math.sin(th / 2) / math.cos(dec)
            if r >= 1.0:
                continue
            dra = 2.0 * math.asin(r) * (1 - 1e-9)
            bb = min(b + (dec > d1), plan["nband"] - 1)
            n = int(plan["nra"][bb])
            k = rng.integers(0, n, per_band)
            ra2 = (k + rng.uniform(0, 1e-6, per_band)) * (2 * math.pi / n)
            sgn = rng.choice([-1.0, 1.0], per_band)
            ra1 = np.mod(ra2 - sgn * dra, 2 * math.pi)
            cd, sd = math.cos(dec), math.sin(dec)
            v1.append(np.stack([cd * np.cos(ra1), cd * np.sin(ra1), np.full(per_band, sd)], 1))
            v2.append(np.stack([cd * np.cos(ra2), cd * np.sin(ra2), np.full(per_band, sd)], 1))
    if not v1:
        return np.zeros((0, 3)), np.zeros((0, 3))
    return np.concatenate(v1), np.concatenate(v2)


CASES = [
    # theta_max (deg), z range, slices, ra_refine
    (10.0, (-1.0, 1.0), 16, 1),
    (10.0, (0.0, math.sin(math.radians(60))), 16, 2),
    (1.0, (0.9, 1.0), 8, 3),
    (0.05, (math.sin(math.radians(29)), math.sin(math.radians(31))), 16, 1),
    (30.0, (-1.0, 1.0), 4, 2),
    (89.0, (-1.0, 1.0), 1, 1),
    (120.0, (-0.5, 1.0), 16, 1),
    (180.0, (-1.0, 1.0), 16, 4),
]


@pytest.mark.parametrize("theta_deg,zr,slices,refine", CASES)
def test_sky_grid_completeness(theta_deg, zr, slices, refine):
    c = chord_of(theta_deg)
    plan = pcm.plan_sky_grid(c, zr[0], zr[1], slices, refine)
    nb, S = plan["nband"], plan["slices"]
    assert nb >= 1 and S >= 1 and 1 <= plan["zreach"] <= S
    assert plan["band_height"] >= plan["theta_reach"] > math.radians(theta_deg)
    assert np.all(np.diff(plan["col0"]) == plan["nra"][:-1]) and plan["col0"][0] == 0
    assert plan["ncol"] == int(plan["nra"].sum())
    rng = synth.rng_for(int(theta_deg * 1000) + slices)
    v1, v2 = stress_pairs(rng, theta_deg, zr[0], zr[1], 40000)
    e1, e2 = edge_pairs(plan, rng, theta_deg, zr[0], zr[1])
    v1, v2 = np.concatenate([v1, e1, e2]), np.concatenate([v2, e2, e1])
    # keep the pairs the counting criterion accepts (binary64 chord^2 below
    # the squared reach) whose points lie in the planned z range
    d = v1 - v2
    s = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    ok = (s < c * c) & (v1[:, 2] >= zr[0]) & (v1[:, 2] <= zr[1]) & \
         (v2[:, 2] >= zr[0]) & (v2[:, 2] <= zr[1])
    v1, v2 = v1[ok], v2[ok]
    assert v1.shape[0] > 1000
    b1, a1, g1 = cells(plan, v1)
    b2, a2, g2 = cells(plan, v2)
    assert np.all(np.abs(g1 - g2) <= plan["zreach"])
    cache = {}
    missing = 0
    for i in range(v1.shape[0]):
        key = (int(b1[i]), int(a1[i]))
        if key not in cache:
            cache[key] = neighbour_cells(plan, *key)
        missing += (int(b2[i]), int(a2[i])) not in cache[key]
    assert missing == 0


@pytest.mark.parametrize("theta_deg,zr,slices,refine", CASES)
def test_sky_grid_reach_follows_haversine(theta_deg, zr, slices, refine):
    """The right-ascension reach between two bands follows the paper's
    haversine relation at the bands' smallest cos(dec), sqrt(c_b c_b') (for
    one band the paper's binning equation): never below it, and within the
    planner's margins above it.  Cells are about 1/refine of the band's own
    reach wide."""
    plan = pcm.plan_sky_grid(chord_of(theta_deg), zr[0], zr[1], slices, refine)
    th = math.radians(theta_deg)
    h = plan["band_height"]
    nb = plan["nband"]

    def cmin(b):
        d0 = plan["dec_lo"] + b * h
        return max(0.0, math.cos(min(math.pi / 2, max(abs(d0), abs(d0 + h)))))

    for b in range(nb):
        for d in (-1, 0, 1):
            b2 = b + d
            if b2 < 0 or b2 >= nb:
                continue
            cc = math.sqrt(cmin(b) * cmin(b2))
            got = plan["dra"][b][d + 1]
            assert got == plan["dra"][b2][1 - d]          # symmetric
            r = math.sin(th / 2) / cc if cc > 0 else math.inf
            if r >= 1.0:
                assert got >= math.pi
                continue
            paper = 2.0 * math.asin(r)
            if got >= math.pi:
                # only margins can push a reach just under pi over it
                assert paper > math.pi * (1 - 1e-3)
                continue
            assert got >= paper
            # the planner widens the reach by 2^-19 in chord (inputs' norms)
            # and by relative margins of 2^-20; an angle 2^-18 larger bounds both
            r_up = math.sin((th + 2.0 ** -18) / 2) / cc
            assert r_up < 1.0 and got <= 2.0 * math.asin(r_up) * (1 + 1e-5)
        own = plan["dra"][b][1]
        if plan["nra"][b] > 1:
            width = 2 * math.pi / plan["nra"][b]
            assert width >= own / refine * (1 - 1e-12)
            assert width < 2 * own / refine + 1e-12 or plan["nra"][b] == 4096


def test_sky_grid_rejects_bad_input():
    with pytest.raises(pcm.PairCountError):
        pcm.plan_sky_grid(0.0, -1.0, 1.0)
    with pytest.raises(pcm.PairCountError):
        pcm.plan_sky_grid(0.1, 0.5, 0.2)
    with pytest.raises(pcm.PairCountError):
        pcm.plan_sky_grid(float("nan"), -1.0, 1.0)
