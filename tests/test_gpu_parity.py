"""Parity of the HIP pair counter with the CPU oracle (needs an MI355X).

Integer counts must be bit-exact with the oracle; weighted sums must match the
oracle's exactly rounded sums to a relative error of 1e-12 (the GPU adds the
same binary64 products in a different order; with at most ~1e9 terms of one
sign the accumulated relative error stays below 1e-13).
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


def check_w(got, want):
    assert got is not None and want is not None
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= WSUM_RTOL), (rel.max(), got, want)


# ---------------------------------------------------------------- DD(r)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_uniform_box(pc, olib, prec):
    """N = 10^4 uniform in a periodic L = 100 box, 20 log bins in [0.1, 10]."""
    say("config 1", prec)
    pts = synth.uniform_box(10000, 100.0, seed=1)
    e = synth.log_edges(0.1, 10.0, 20)
    got, _ = pc.count_r(pts, None, e, 100.0, prec)
    want, _ = oracle.count_r(pts, None, e, 100.0, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("box", [80.0, 0.0])
def test_r_auto_clustered(pc, olib, prec, dtype, box):
    say("r auto clustered", prec, dtype, box)
    pts = synth.clustered_box(20000, 80.0, seed=3, nblobs=100, sigma=1.5).astype(dtype)
    e = synth.log_edges(0.05, 12.0, 15)
    got, _ = pc.count_r(pts, None, e, box, prec)
    want, _ = oracle.count_r(pts, None, e, box, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [60.0, 0.0])
def test_r_cross(pc, olib, prec, box):
    say("r cross", prec, box)
    a = synth.clustered_box(9000, 60.0, seed=5, nblobs=40)
    b = synth.uniform_box(7000, 60.0, seed=6)
    e = synth.log_edges(0.2, 15.0, 12)
    got, _ = pc.count_r(a, b, e, box, prec)
    want, _ = oracle.count_r(a, b, e, box, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_r_weighted_auto_and_cross(pc, olib, prec):
    say("r weighted", prec)
    a = synth.clustered_box(12000, 70.0, seed=7, nblobs=60)
    b = synth.uniform_box(5000, 70.0, seed=8)
    wa = synth.uniform_weights(12000, seed=9)
    wb = synth.uniform_weights(5000, seed=10)
    e = np.r_[0.0, synth.log_edges(0.1, 20.0, 10)]
    got, gw = pc.count_r(a, None, e, 70.0, prec, w1=wa)
    want, ww = oracle.count_r(a, None, e, 70.0, w1=wa, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)
    got, gw = pc.count_r(a, b, e, 0.0, prec, w1=wa, w2=wb)
    want, ww = oracle.count_r(a, b, e, 0.0, w1=wa, w2=wb, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_r_lattice_edge_ties(pc, olib, prec):
    """Integer coordinates and integer edges: very many pairs lie exactly on
    an edge, which the float32 pass must hand to the binary64 recheck."""
    say("r lattice ties", prec)
    rng = synth.rng_for(11)
    pts = rng.integers(0, 41, size=(6000, 3)).astype(np.float64)
    e = np.arange(0.0, 14.0)          # squared edges are exact integers
    for box in (41.0, 0.0):
        got, _ = pc.count_r(pts, None, e, box, prec)
        want, _ = oracle.count_r(pts, None, e, box, lib=olib)
        assert (got == want).all(), (box, got, want)
    if prec == "fp32":
        assert pc.stats()["rechecks"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_r_edges_one_ulp_apart(pc, olib, prec):
    """Edges packed within a few ulps of sqrt(1), sqrt(2), sqrt(3), 2 and
    sqrt(5) (each edge, its neighbours one ulp either side and one 1e-9
    above), on integer lattice points whose squared separations are exact
    integers, plus jittered points: float32 error bands of neighbouring edges
    overlap, so the table's multi-edge cells and the binary64 recheck decide
    every pair near them, and the counts between the packed edges come from
    the binary64 rounding of the squared edges alone.  DD(rp, pi) on the
    same rp edges with integer pi edges adds ties along the line of sight."""
    say("r edges one ulp apart", prec)
    rng = synth.rng_for(13)
    lat = rng.integers(0, 24, size=(5000, 3)).astype(np.float64)
    jit = lat[:2000] + rng.uniform(-1e-6, 1e-6, size=(2000, 3))
    pts = np.clip(np.r_[lat, jit], 0.0, 24.0)
    base = np.sqrt(np.array([1.0, 2.0, 3.0, 4.0, 5.0]))
    e = np.unique(np.concatenate([base, np.nextafter(base, 0.0), np.nextafter(base, 9.0),
                                  base * (1 + 1e-9)]))
    assert e.size == 20 and np.all(np.diff(e) > 0)
    for box in (24.0, 0.0):
        got, _ = pc.count_r(pts, None, e, box, prec)
        want, _ = oracle.count_r(pts, None, e, box, lib=olib)
        assert (got == want).all(), (box, got, want)
        assert want.sum() > 0
        if prec == "fp32":
            assert pc.stats()["rechecks"] > 0
        # the same rp edges with integer pi edges: ties in both dimensions
        got, _ = pc.count_rppi(pts, None, e, 5.0, 5, box, prec)
        want, _ = oracle.count_rppi(pts, None, e, 5.0, 5, box, lib=olib)
        assert (got == want).all(), (box, got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_r_points_on_faces_and_coincident(pc, olib, prec):
    say("r faces", prec)
    pts = synth.uniform_box(4000, 30.0, seed=12)
    pts[:300, 0] = 30.0                # exactly L (legal, closed box)
    pts[300:600, 1] = 0.0
    pts[600:700] = pts[700:800]        # coincident pairs
    pts[800:900, 2] = np.float64(np.float32(29.999999))
    e = np.r_[0.0, synth.log_edges(0.01, 9.0, 8)]
    got, _ = pc.count_r(pts, None, e, 30.0, prec)
    want, _ = oracle.count_r(pts, None, e, 30.0, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_r_minimal_grid_and_dense_cell(pc, olib, prec):
    """Three columns per axis (reach just under L/3) and a dense cluster
    whose cell holds a third of the points."""
    say("r minimal grid", prec)
    L = 30.0
    pts = synth.uniform_box(3000, L, seed=13)
    pts[:1000] = 15.0 + synth.rng_for(14).normal(0, 0.3, (1000, 3))
    e = synth.log_edges(0.05, 9.99, 10)
    got, _ = pc.count_r(pts, None, e, L, prec)
    want, _ = oracle.count_r(pts, None, e, L, lib=olib)
    assert (got == want).all(), (got, want)


def test_r_small_and_empty(pc, olib):
    say("r small/empty")
    e = np.array([0.0, 1.0, 2.0])
    z = np.zeros((0, 3))
    got, _ = pc.count_r(z, None, e, 10.0)
    assert got.tolist() == [0, 0]
    one = np.array([[1.0, 2.0, 3.0]])
    got, _ = pc.count_r(one, None, e, 10.0)
    assert got.tolist() == [1, 0]
    got, _ = pc.count_r(one, z, e, 10.0)
    assert got.tolist() == [0, 0]
    two = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 2.5]])
    for prec in ("fp64", "fp32"):
        got, _ = pc.count_r(two, None, e, 10.0, prec)
        want, _ = oracle.count_r(two, None, e, 10.0, lib=olib)
        assert (got == want).all()


def test_r_recheck_weighted_ties(pc, olib):
    """Pairs on edges with weights: the float32 pass hands them to the inline
    binary64 evaluation, which must add their weight products too."""
    say("r weighted ties")
    rng = synth.rng_for(15)
    pts = rng.integers(0, 31, size=(4000, 3)).astype(np.float64)
    w = synth.uniform_weights(4000, seed=151)
    e = np.arange(1.0, 10.0)
    got, gw = pc.count_r(pts, None, e, 31.0, "fp32", w1=w)
    assert pc.stats()["rechecks"] > 1000
    want, ww = oracle.count_r(pts, None, e, 31.0, w1=w, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


@pytest.mark.parametrize("chunk,spr", [(64, 1), (300, 3), (2048, 8), (100000, 20)])
def test_r_worklist_shapes(pc, olib, chunk, spr):
    """Work-item splitting and z-slice resolution do not change the counts."""
    say("r worklist", chunk, spr)
    pts = synth.clustered_box(8000, 50.0, seed=16, nblobs=50)
    e = synth.log_edges(0.1, 15.0, 9)
    want, _ = oracle.count_r(pts, None, e, 50.0, lib=olib)
    for prec in ("fp64", "fp32"):
        got, _ = pc.count_r(pts, None, e, 50.0, prec,
                            options={"chunk": chunk, "slices_per_reach": spr})
        assert (got == want).all(), (chunk, spr, prec)


def test_r_hist_replicas(pc, olib):
    say("r replicas")
    pts = synth.clustered_box(6000, 40.0, seed=17, nblobs=30)
    e = synth.log_edges(0.1, 12.0, 10)
    want, _ = oracle.count_r(pts, None, e, 40.0, lib=olib)
    for copies in (1, 2, 8, 32, 64):
        got, _ = pc.count_r(pts, None, e, 40.0, "fp32", options={"hist_copies": copies})
        assert (got == want).all(), copies


def test_r_torch_device_inputs(pc, olib):
    import torch
    say("r torch device inputs")
    pts = synth.clustered_box(10000, 60.0, seed=18, nblobs=40)
    w = synth.uniform_weights(10000, seed=19)
    e = synth.log_edges(0.1, 15.0, 12)
    t = torch.from_numpy(pts).cuda()
    cols = tuple(t[:, k].contiguous() for k in range(3))
    wt = torch.from_numpy(w).cuda()
    got, gw = pc.count_r(cols, None, e, 60.0, "fp32", w1=wt)
    want, ww = oracle.count_r(pts, None, e, 60.0, w1=w, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


# ---------------------------------------------------------------- DD(rp, pi)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [90.0, 0.0])
def test_rppi_auto(pc, olib, prec, box):
    say("rppi auto", prec, box)
    pts = synth.clustered_box(15000, 90.0, seed=21, nblobs=70, sigma=2.0)
    e = synth.log_edges(0.1, 25.0, 12)
    got, _ = pc.count_rppi(pts, None, e, 25.0, 25, box, prec)
    want, _ = oracle.count_rppi(pts, None, e, 25.0, 25, box, lib=olib)
    assert (got == want).all(), np.argwhere(got != want)[:5]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rppi_cross_weighted(pc, olib, prec):
    say("rppi cross weighted", prec)
    a = synth.clustered_box(8000, 100.0, seed=22, nblobs=40)
    b = synth.uniform_box(9000, 100.0, seed=23)
    wa = synth.uniform_weights(8000, seed=24)
    wb = synth.uniform_weights(9000, seed=25)
    e = np.r_[0.0, synth.log_edges(0.5, 30.0, 8)]
    got, gw = pc.count_rppi(a, b, e, 30.0, 15, 100.0, prec, w1=wa, w2=wb)
    want, ww = oracle.count_rppi(a, b, e, 30.0, 15, 100.0, w1=wa, w2=wb, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rppi_lattice_ties(pc, olib, prec):
    say("rppi lattice", prec)
    rng = synth.rng_for(26)
    pts = rng.integers(0, 40, size=(5000, 3)).astype(np.float64)
    e = np.arange(0.0, 11.0)
    got, _ = pc.count_rppi(pts, None, e, 12.0, 12, 40.0, prec)
    want, _ = oracle.count_rppi(pts, None, e, 12.0, 12, 40.0, lib=olib)
    assert (got == want).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rppi_noninteger_pi_bins(pc, olib, prec):
    say("rppi non-integer pi bins", prec)
    pts = synth.clustered_box(9000, 70.0, seed=27, nblobs=50)
    e = synth.log_edges(0.3, 20.0, 7)
    got, _ = pc.count_rppi(pts, None, e, 17.3, 7, 70.0, prec)
    want, _ = oracle.count_rppi(pts, None, e, 17.3, 7, 70.0, lib=olib)
    assert (got == want).all()


@pytest.mark.parametrize("box", [1000.0, 0.0])
def test_rppi_fine_pi_bins(pc, olib, box):
    """pi bins too fine for 2^4 fixed-point quanta each (box / dpi > 2^25):
    the float32 call sweeps in binary64 and must still match."""
    say("rppi fine pi bins", box)
    pts = synth.clustered_box(6000, 1000.0, seed=28, nblobs=30, sigma=0.002)
    e = synth.log_edges(0.001, 0.05, 6)
    got, _ = pc.count_rppi(pts, None, e, 0.002, 100, box, "fp32")
    want, _ = oracle.count_rppi(pts, None, e, 0.002, 100, box, lib=olib)
    assert want.sum() > 0
    assert (got == want).all()


# ---------------------------------------------------------------- DD(theta)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_theta_auto_cross(pc, olib, prec):
    say("theta", prec)
    ra, dec = synth.cap_radec(12000, seed=31, radius_deg=8.0, clustered=True,
                              nblobs=200, sigma_deg=0.1)
    rr, rd = synth.cap_radec(15000, seed=32, radius_deg=8.0)
    te = synth.log_edges(0.01, 3.0, 12)
    got, _ = pc.count_theta(ra, dec, None, None, te, prec)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    assert (got == want).all(), (got, want)
    got, _ = pc.count_theta(ra, dec, rr, rd, te, prec)
    want, _ = oracle.count_theta(ra, dec, rr, rd, te, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_theta_edges_one_ulp_apart(pc, olib, prec):
    """theta edges packed within an ulp of 0.5, 1, 1.5 and 2 degrees (each
    edge and its neighbours one ulp either side) on a half-degree RA/DEC grid
    (many separations of exactly those angles up to rounding) plus random cap
    points, converted on the host: counts equal the oracle's on the angular
    and the 3-D chord grid."""
    say("theta edges one ulp apart", prec)
    g = np.arange(0.0, 10.01, 0.5)
    gra, gdec = (a.ravel() for a in np.meshgrid(g, g - 5.0))
    ra, dec = synth.cap_radec(8000, seed=35, radius_deg=7.0, ra0_deg=5.0, dec0_deg=0.0)
    ra, dec = np.r_[gra, ra], np.r_[gdec, dec]
    base = np.array([0.5, 1.0, 1.5, 2.0])
    te = np.unique(np.concatenate([base, np.nextafter(base, 0.0), np.nextafter(base, 9.0)]))
    assert te.size == 12
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    assert want.sum() > 0
    for grid in (None, -1):
        got, _ = pc.count_theta(ra, dec, None, None, te, prec, angular_grid=grid)
        assert (got == want).all(), (grid, got, want)


def test_theta_unit_vectors_and_weights(pc, olib):
    say("theta unit vectors")
    ra, dec = synth.cap_radec(9000, seed=33, radius_deg=20.0, clustered=True,
                              nblobs=100, sigma_deg=0.3)
    w = synth.uniform_weights(9000, seed=34)
    te = np.r_[0.0, synth.log_edges(0.05, 10.0, 9)]
    v = oracle.radec_to_unit(ra, dec, lib=olib)
    want, ww = oracle.count_theta(ra, dec, None, None, te, w1=w, lib=olib)
    for prec in ("fp64", "fp32"):
        got, gw = pc.count_theta(None, None, theta_edges_deg=te, precision=prec, w1=w,
                                 unit_vectors=(v, None))
        assert (got == want).all(), prec
        check_w(gw, ww)


# ---------------------------------------------------------------- invariants
def test_auto_equals_cross_on_gpu(pc):
    say("auto == cross")
    pts = synth.clustered_box(30000, 100.0, seed=41, nblobs=150)
    e = np.r_[0.0, synth.log_edges(0.1, 20.0, 12)]
    for prec in ("fp64", "fp32"):
        a, _ = pc.count_r(pts, None, e, 100.0, prec)
        c, _ = pc.count_r(pts, pts, e, 100.0, prec)
        assert (a == c).all(), prec


def test_repeatable(pc):
    say("repeatable")
    pts = synth.clustered_box(30000, 100.0, seed=42, nblobs=150)
    e = synth.log_edges(0.1, 20.0, 12)
    first, _ = pc.count_r(pts, None, e, 100.0, "fp32")
    for _ in range(3):
        again, _ = pc.count_r(pts, None, e, 100.0, "fp32")
        assert (again == first).all()


# ---------------------------------------------------------------- errors
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fine_grid_gridding_paths(pc, olib, prec):
    """A grid of more columns (142 x 142 > 16384) than the two-level sort's
    LDS histogram holds is gridded by the one-atomic-per-point path; both
    paths must give the same exact counts (the coarse call uses the
    two-level sort)."""
    say("fine grid", prec)
    pts = synth.clustered_box(20000, 1000.0, seed=63, nblobs=100, sigma=2.0)
    e = synth.log_edges(0.5, 7.0, 8)
    got, _ = pc.count_r(pts, None, e, 1000.0, prec, options={"slices_per_reach": 1})
    assert pc.stats()["grid"][0] * pc.stats()["grid"][1] > 16384
    want, _ = oracle.count_r(pts, None, e, 1000.0, lib=olib)
    assert (got == want).all()
    e2 = synth.log_edges(0.5, 20.0, 8)
    got, _ = pc.count_r(pts, None, e2, 1000.0, prec)
    assert pc.stats()["grid"][0] * pc.stats()["grid"][1] <= 16384
    want, _ = oracle.count_r(pts, None, e2, 1000.0, lib=olib)
    assert (got == want).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bin_count_limits(pc, olib, prec):
    """The largest bin counts the library accepts: 1024 r bins (the edge
    limit), 64 x 64 = 4096 rp/pi bins (the total limit), 4 x 1024 (the pi
    limit), 2048 weighted bins and 1365 bins with the mean separation; one
    more bin is an error."""
    import paper_1911_03545_amd as m
    say("bin limits", prec)
    pts = synth.clustered_box(4000, 60.0, seed=61, nblobs=20)
    w = synth.uniform_weights(4000, seed=62)
    e = np.r_[0.0, synth.log_edges(0.02, 15.0, 1023)]
    got, _ = pc.count_r(pts, None, e, 60.0, prec)
    want, _ = oracle.count_r(pts, None, e, 60.0, lib=olib)
    assert (got == want).all()
    e64 = synth.log_edges(0.05, 15.0, 64)
    got, _ = pc.count_rppi(pts, None, e64, 16.0, 64, 60.0, prec)
    want, _ = oracle.count_rppi(pts, None, e64, 16.0, 64, 60.0, lib=olib)
    assert (got == want).all()
    e4 = synth.log_edges(0.5, 15.0, 4)
    got, _ = pc.count_rppi(pts, None, e4, 16.0, 1024, 60.0, prec)
    want, _ = oracle.count_rppi(pts, None, e4, 16.0, 1024, 60.0, lib=olib)
    assert (got == want).all()
    e32 = synth.log_edges(0.05, 15.0, 32)
    got, gw = pc.count_rppi(pts, None, e32, 16.0, 64, 60.0, prec, w1=w)
    want, ww = oracle.count_rppi(pts, None, e32, 16.0, 64, 60.0, w1=w, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)
    e21 = synth.log_edges(0.05, 15.0, 21)
    got, _, gr = pc.count_rppi(pts, None, e21, 16.0, 65, 60.0, prec, ravg=True)
    want, _, wr = oracle.count_rppi(pts, None, e21, 16.0, 65, 60.0, lib=olib, ravg=True)
    assert (got == want).all()
    if prec == "fp64":
        check_w(gr, wr)
    for args, kw in (((e64, 16.0, 65), {}), ((e32, 16.0, 65), {"w1": w}),
                     ((e21, 16.0, 66), {"ravg": True})):
        with pytest.raises(m.PairCountError) as ex:
            pc.count_rppi(pts, None, *args, 60.0, prec, **kw)
        assert ex.value.status == m.CF_EINVAL
    with pytest.raises(m.PairCountError):
        pc.count_r(pts, None, np.r_[0.0, synth.log_edges(0.02, 15.0, 1024)], 60.0, prec)


def test_error_codes(pc):
    import paper_1911_03545_amd as m
    say("errors")
    e = np.array([0.1, 1.0, 2.0])
    pts = synth.uniform_box(100, 10.0, seed=43)
    bad = pts.copy()
    bad[5, 1] = np.nan
    with pytest.raises(m.PairCountError) as ex:
        pc.count_r(bad, None, e, 10.0)
    assert ex.value.status == m.CF_EINVAL
    out = pts.copy()
    out[3, 0] = 10.5
    with pytest.raises(m.PairCountError) as ex:
        pc.count_r(out, None, e, 10.0)
    assert ex.value.status == m.CF_ERANGE
    with pytest.raises(m.PairCountError) as ex:
        pc.count_r(pts, None, np.array([0.1, 4.0]), 10.0)
    assert ex.value.status == m.CF_EUNSUPPORTED
    with pytest.raises(m.PairCountError) as ex:
        pc.count_r(pts, None, np.array([1.0, 0.5]), 10.0)
    assert ex.value.status == m.CF_EINVAL
    with pytest.raises(m.PairCountError) as ex:
        pc.count_theta(np.array([10.0, 400.0]), np.array([0.0, 0.0]), None, None,
                       np.array([0.1, 1.0]))
    assert ex.value.status == m.CF_ERANGE
    with pytest.raises(m.PairCountError) as ex:
        pc.count_theta(np.array([10.0, 20.0]), np.array([0.0, 0.0]), None, None,
                       np.array([0.1, 181.0]))
    assert ex.value.status == m.CF_ERANGE
    with pytest.raises(m.PairCountError) as ex:
        pc.count_r(pts, pts, e, 10.0, w1=np.ones(100))
    assert ex.value.status == m.CF_EINVAL
    for box in (float("nan"), float("inf")):
        with pytest.raises(m.PairCountError) as ex:
            pc.count_r(pts, None, e, box)
        assert ex.value.status == m.CF_EINVAL
    # the context stays usable after errors
    got, _ = pc.count_r(pts, None, e, 10.0)
    assert got.sum() > 0
