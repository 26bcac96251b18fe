"""The two forms of the float32 squared separation (needs an MI355X).

cf_options.separation_form 1 takes dx^2 + dy^2 + dz^2 (rp^2: dx^2 + dy^2)
from the coordinate differences; 2 expands x and y as |a|^2 + |b|^2 - 2 a.b
(one instruction fewer per pair, a larger absolute rounding bound folded into
the decision bands, each pair's band narrowed by its own magnitudes before
the binary64 recheck); 0 picks 2 for float32 DD(r), DD(rp, pi) (single and
batched) and chords of 3-D grids unless the bound would widen the smallest
edge's band by more than an eighth of it.
Both forms must give the oracle's counts exactly, whatever the workload:
clustered and uniform points, periodic and open boxes, auto- and
cross-correlations, weights, a first edge of zero, integer lattices with
pairs on the edges, edges one ulp apart, chords of unit vectors.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

WSUM_RTOL = 1e-12


@pytest.fixture(scope="module")
def pc():
    import paper_1911_03545_amd as m
    ctx = m.PairCounter(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def olib():
    return oracle.load()


def say(*a):
    print(*a, flush=True)


def form(f):
    return {"separation_form": f}


@pytest.mark.parametrize("box", [120.0, 0.0])
def test_forms_agree_with_oracle_clustered(pc, olib, box):
    say("separation forms clustered", box)
    pts = synth.clustered_box(30000, 120.0, seed=1201, nblobs=150, sigma=2.0)
    e = synth.log_edges(0.1, 10.0, 20)
    want, _ = oracle.count_r(pts, None, e, box, lib=olib)
    for f in (0, 1, 2):
        got, _ = pc.count_r(pts, None, e, box, "fp32", options=form(f))
        assert (got == want).all(), (f, got, want)
        used = pc.stats()["separation_form"]
        assert used == (1 if f == 1 else 2), (f, used)


def test_forms_cross_and_weights(pc, olib):
    say("separation forms cross/weights")
    L = 100.0
    x = synth.clustered_box(8000, L, seed=1202, nblobs=60, sigma=1.5)
    y = synth.uniform_box(12000, L, seed=1203)
    wx = synth.uniform_weights(8000, 1204)
    wy = synth.uniform_weights(12000, 1205)
    e = np.r_[0.0, synth.log_edges(0.2, 9.0, 12)]
    for box in (L, 0.0):
        want, ww = oracle.count_r(x, y, e, box, w1=wx, w2=wy, lib=olib)
        for f in (1, 2):
            got, gw = pc.count_r(x, y, e, box, "fp32", w1=wx, w2=wy, options=form(f))
            assert (got == want).all(), (box, f)
            np.testing.assert_allclose(gw, ww, rtol=WSUM_RTOL, atol=0)
            assert pc.stats()["separation_form"] == f
        # autocorrelation with weights, self-pairs in the first bin
        want, ww = oracle.count_r(x, None, e, box, w1=wx, lib=olib)
        got, gw = pc.count_r(x, None, e, box, "fp32", w1=wx, options=form(2))
        assert (got == want).all(), box
        np.testing.assert_allclose(gw, ww, rtol=WSUM_RTOL, atol=0)


def test_forms_lattice_ties_and_packed_edges(pc, olib):
    """Pairs exactly on the edges (integer lattice, integer squared edges)
    and edges a few ulps apart: the bands of both forms hand them to the
    binary64 recheck."""
    say("separation forms lattice")
    rng = synth.rng_for(1206)
    pts = rng.integers(0, 41, size=(6000, 3)).astype(np.float64)
    e = np.arange(0.0, 14.0)
    for box in (41.0, 0.0):
        want, _ = oracle.count_r(pts, None, e, box, lib=olib)
        for f in (1, 2):
            got, _ = pc.count_r(pts, None, e, box, "fp32", options=form(f))
            assert (got == want).all(), (box, f)
            assert pc.stats()["rechecks"] > 0
    lat = rng.integers(0, 24, size=(5000, 3)).astype(np.float64)
    base = np.sqrt(np.array([1.0, 2.0, 3.0, 4.0, 5.0]))
    e = np.unique(np.concatenate([base, np.nextafter(base, 0.0), np.nextafter(base, 9.0),
                                  base * (1 + 1e-9)]))
    want, _ = oracle.count_r(lat, None, e, 24.0, lib=olib)
    got, _ = pc.count_r(lat, None, e, 24.0, "fp32", options=form(2))
    assert (got == want).all()


def test_expanded_bands_narrowed_per_pair(pc, olib):
    """The expanded bands hold the rounding term of the largest magnitudes;
    the sweep first narrows a pair's band by its own, so the expanded form
    re-evaluates few more pairs in binary64 than the differences (here about
    1.15 times as many; about 2 times without the narrowing)."""
    say("separation forms per-pair narrowing")
    L = 250.0
    pts = synth.clustered_box(200000, L, seed=77, nblobs=1000, sigma=2.0)
    e = synth.log_edges(0.1, 15.0, 20)
    want, _ = oracle.count_r(pts, None, e, L, lib=olib)
    rq = {}
    for f in (1, 2):
        got, _ = pc.count_r(pts, None, e, L, "fp32", options=form(f))
        assert (got == want).all(), f
        rq[f] = pc.stats()["rechecks"]
    assert rq[1] > 0
    assert rq[2] <= 1.4 * rq[1], rq


def test_auto_keeps_differences_for_tiny_edges(pc, olib):
    """A first edge far below the column width: the expanded bound would
    swamp its band, so the default takes the differences; forcing the
    expanded form still counts exactly (more pairs go to the recheck)."""
    say("separation forms tiny edges")
    L = 60.0
    pts = synth.clustered_box(20000, L, seed=1207, nblobs=200, sigma=0.5)
    e = synth.log_edges(0.002, 6.0, 16)
    want, _ = oracle.count_r(pts, None, e, L, lib=olib)
    got, _ = pc.count_r(pts, None, e, L, "fp32")
    assert (got == want).all()
    assert pc.stats()["separation_form"] == 1
    r1 = pc.stats()["rechecks"]
    got, _ = pc.count_r(pts, None, e, L, "fp32", options=form(2))
    assert (got == want).all()
    assert pc.stats()["separation_form"] == 2
    assert pc.stats()["rechecks"] >= r1


def test_chords_of_unit_vectors(pc, olib):
    """theta on the 3-D chord grid (squared chords are the r statistic of
    unit vectors)."""
    say("separation forms chords")
    ra, dec = synth.cap_radec(20000, seed=1208, radius_deg=15.0, clustered=True)
    te = synth.log_edges(0.05, 5.0, 12)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    for f in (1, 2):
        got, _ = pc.count_theta(ra, dec, None, None, te, "fp32", angular_grid=-1,
                                options=form(f))
        assert (got == want).all(), f
        assert pc.stats()["separation_form"] == f


def test_mean_separation_keeps_differences(pc, olib):
    say("separation forms ravg")
    pts = synth.clustered_box(10000, 80.0, seed=1209, nblobs=80, sigma=1.5)
    e = synth.log_edges(0.1, 8.0, 10)
    want, _, _ = oracle.count_r(pts, None, e, 80.0, lib=olib, ravg=True)
    got, _, _ = pc.count_r(pts, None, e, 80.0, "fp32", ravg=True, options=form(2))
    assert (got == want).all()
    assert pc.stats()["separation_form"] == 1


def test_fp64_reports_no_form(pc):
    say("separation forms fp64")
    pts = synth.uniform_box(5000, 50.0, seed=1210)
    e = synth.log_edges(0.5, 5.0, 6)
    pc.count_r(pts, None, e, 50.0, "fp64", options=form(2))
    assert pc.stats()["separation_form"] == 0


@pytest.mark.parametrize("box", [150.0, 0.0])
def test_rppi_forms(pc, olib, box):
    """rp^2 expanded as fl(fl(|a|^2 + |b|^2) - 2 a_x b_x) - 2 a_y b_y, with
    the fixed-point pi test unchanged."""
    say("separation forms rppi", box)
    pts = synth.clustered_box(25000, 150.0, seed=1212, nblobs=120, sigma=2.0)
    e = synth.log_edges(0.2, 15.0, 14)
    want, _ = oracle.count_rppi(pts, None, e, 20.0, 20, box, lib=olib)
    for f in (0, 1, 2):
        got, _ = pc.count_rppi(pts, None, e, 20.0, 20, box, "fp32", options=form(f))
        assert (got == want).all(), (f, box)
        assert pc.stats()["separation_form"] == (1 if f == 1 else 2)
    # weighted cross-correlation, both forms
    y = synth.uniform_box(15000, 150.0, seed=1213)
    wx = synth.uniform_weights(25000, 1214)
    wy = synth.uniform_weights(15000, 1215)
    want, ww = oracle.count_rppi(pts, y, e, 20.0, 20, box, w1=wx, w2=wy, lib=olib)
    for f in (1, 2):
        got, gw = pc.count_rppi(pts, y, e, 20.0, 20, box, "fp32", w1=wx, w2=wy,
                                options=form(f))
        assert (got == want).all(), (f, box)
        np.testing.assert_allclose(gw, ww, rtol=WSUM_RTOL, atol=0)


def test_rppi_lattice_ties(pc, olib):
    """Integer lattice, integer rp^2 edges and integer pi edges: ties in
    both dimensions go to the binary64 recheck in both forms."""
    say("separation forms rppi lattice")
    rng = synth.rng_for(1216)
    pts = rng.integers(0, 30, size=(6000, 3)).astype(np.float64)
    e = np.sqrt(np.arange(1.0, 12.0))
    for box in (30.0, 0.0):
        want, _ = oracle.count_rppi(pts, None, e, 6.0, 6, box, lib=olib)
        for f in (1, 2):
            got, _ = pc.count_rppi(pts, None, e, 6.0, 6, box, "fp32", options=form(f))
            assert (got == want).all(), (box, f)


def test_batched_rppi_forms(pc, olib):
    say("separation forms batched")
    L = 200.0
    sizes = [9000, 300, 0, 4000, 1, 2500]
    cats = [synth.clustered_box(n, L, seed=1220 + k, nblobs=max(1, n // 200), sigma=2.0)
            for k, n in enumerate(sizes)]
    e = synth.log_edges(0.2, 18.0, 12)
    wants = [oracle.count_rppi(p, None, e, 25.0, 25, L, lib=olib)[0] for p in cats]
    for f in (0, 1, 2):
        got, _ = pc.count_rppi_batch(cats, e, 25.0, 25, L, "fp32", options=form(f))
        for k in range(len(cats)):
            assert (got[k] == wants[k]).all(), (f, k)
        # (the default follows the smallest edge's band, grids of sparse
        # catalogues have wide columns)
        assert pc.stats()["separation_form"] == f if f else pc.stats()["separation_form"] in (1, 2)


def test_invalid_form_refused(pc):
    import paper_1911_03545_amd as m
    pts = synth.uniform_box(1000, 20.0, seed=1211)
    with pytest.raises(m.PairCountError):
        pc.count_r(pts, None, synth.log_edges(0.5, 5.0, 4), 20.0, "fp32", options=form(3))
