"""DD(theta) / DR(theta) on the angular grid (declination bands and
right-ascension cells) against the oracle (needs an MI355X).

The grid only decides which pairs are evaluated; every evaluated pair is
binned by the same chord^2 definition, so counts must equal the oracle's
bit for bit for any band / cell layout: full sky with both poles, a cap on
the RA = 0 / 360 seam, very large and very small angular reaches, points
exactly at the poles and on the seam, several right-ascension refinements and
slice counts, both precisions, weights and mean angles.  The 3-D chord grid
(angular_grid=-1) is checked alongside.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pc():
    import paper_1911_03545_amd as m
    ctx = m.PairCounter(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def olib():
    return oracle.load()


def rel_ok(got, want, rtol=RTOL):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= rtol), (rel.max(), got, want)


def full_sky(n, seed):
    rng = synth.rng_for(seed)
    ra = rng.uniform(0.0, 360.0, n)
    dec = np.rad2deg(np.arcsin(rng.uniform(-1.0, 1.0, n)))
    return ra, dec


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("refine", [1, 2])
def test_full_sky_auto_cross(pc, olib, prec, refine):
    say("angular grid full sky", prec, refine)
    ra, dec = full_sky(20000, 501)
    # poles and seam
    ra[:6] = [0.0, 360.0, 123.0, 0.0, 359.999999, 180.0]
    dec[:6] = [90.0, -90.0, 90.0, 0.0, 0.0, -90.0]
    r2, d2 = full_sky(15000, 502)
    te = synth.log_edges(0.1, 20.0, 10)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, None, None, te, prec, angular_grid=refine)
    assert (got == want).all(), (got, want)
    st = pc.stats()
    assert st["grid"][0] > 1
    want, _ = oracle.count_theta(ra, dec, r2, d2, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, r2, d2, te, prec, angular_grid=refine)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seam_cap_matches_chord_grid(pc, olib, prec):
    """A clustered 30-degree cap centred on the seam at DEC 30 (the angular
    statistic's benchmark shape, smaller): equal to the oracle and to the
    3-D chord grid, with fewer or comparable candidate pairs."""
    say("angular grid seam cap", prec)
    ra, dec = synth.cap_radec(30000, seed=503, radius_deg=30.0, clustered=True,
                              nblobs=300, sigma_deg=0.1)
    rr, rd = synth.cap_radec(40000, seed=504, radius_deg=30.0)
    te = synth.log_edges(0.01, 10.0, 20)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    for refine in (1, 2, 4):
        got, _ = pc.count_theta(ra, dec, None, None, te, prec, angular_grid=refine)
        assert (got == want).all(), (refine, got, want)
    chord, _ = pc.count_theta(ra, dec, None, None, te, prec, angular_grid=-1)
    assert (chord == want).all()
    default, _ = pc.count_theta(ra, dec, None, None, te, prec)
    assert (default == want).all() and pc.stats()["angular_grid"] == 16
    want, _ = oracle.count_theta(ra, dec, rr, rd, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, rr, rd, te, prec, angular_grid=2)
    assert (got == want).all()


@pytest.mark.parametrize("tmax", [90.0, 150.0, 180.0])
def test_large_reach(pc, olib, tmax):
    say("angular grid large reach", tmax)
    ra, dec = full_sky(3000, 505)
    te = np.linspace(0.0, tmax, 7)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    for prec in ("fp64", "fp32"):
        got, _ = pc.count_theta(ra, dec, None, None, te, prec, angular_grid=1)
        assert (got == want).all(), (prec, got, want)


@pytest.mark.parametrize("slices", [1, 3, 16, 64])
def test_small_reach_and_slices(pc, olib, slices):
    """Reach 0.05 degrees on a 2-degree cap (fine bands), and on the full
    sky (band and cell counts at their caps, so cells wider than needed)."""
    say("angular grid small reach", slices)
    ra, dec = synth.cap_radec(20000, seed=506, radius_deg=2.0, ra0_deg=200.0, dec0_deg=-60.0,
                              clustered=True, nblobs=50, sigma_deg=0.01)
    te = synth.log_edges(0.001, 0.05, 8)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, None, None, te, "fp32", angular_grid=2,
                            options={"slices_per_reach": slices})
    assert (got == want).all(), (got, want)
    ra, dec = full_sky(20000, 507)
    te = synth.log_edges(0.001, 0.01, 4)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, None, None, te, "fp64", angular_grid=1,
                            options={"slices_per_reach": slices})
    assert (got == want).all(), (got, want)


def test_weights_ravg_unit_vectors(pc, olib):
    say("angular grid weights, mean angle")
    ra, dec = synth.cap_radec(12000, seed=508, radius_deg=15.0, ra0_deg=10.0, dec0_deg=75.0,
                              clustered=True, nblobs=80, sigma_deg=0.2)
    w = synth.uniform_weights(12000, seed=509)
    te = np.r_[0.0, synth.log_edges(0.05, 8.0, 9)]
    v = oracle.radec_to_unit(ra, dec, lib=olib)
    for wtype in ("product", "sum"):
        want, ww, wr = oracle.count_theta(ra, dec, None, None, te, w1=w, lib=olib,
                                          weight_type=wtype, ravg=True)
        for prec in ("fp64", "fp32"):
            got, gw, gr = pc.count_theta(None, None, theta_edges_deg=te, precision=prec, w1=w,
                                         unit_vectors=(v, None), weight_type=wtype, ravg=True,
                                         angular_grid=3)
            assert (got == want).all(), (wtype, prec)
            rel_ok(gw, ww)
            rel_ok(gr, wr, 1e-9 if prec == "fp64" else 1e-5)


def test_float32_unit_vectors(pc):
    """float32 unit vectors (squared norm within ~1e-7 of 1) are accepted;
    counts equal those of the 3-D chord grid on the same vectors."""
    say("angular grid float32 unit vectors")
    ra, dec = full_sky(8000, 510)
    r = np.deg2rad
    v = np.stack([np.cos(r(dec)) * np.cos(r(ra)), np.cos(r(dec)) * np.sin(r(ra)),
                  np.sin(r(dec))], 1).astype(np.float32)
    te = synth.log_edges(0.5, 15.0, 6)
    for prec in ("fp64", "fp32"):
        got, _ = pc.count_theta(None, None, theta_edges_deg=te, precision=prec,
                                unit_vectors=(v, None), angular_grid=1)
        chord, _ = pc.count_theta(None, None, theta_edges_deg=te, precision=prec,
                                  unit_vectors=(v, None), angular_grid=-1)
        assert chord.sum() > 0 and (got == chord).all(), prec


def test_errors(pc):
    import paper_1911_03545_amd as m
    say("angular grid errors")
    v = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 1.0]])
    te = synth.log_edges(0.5, 15.0, 4)
    for grid in (None, 1):
        with pytest.raises(m.PairCountError):
            pc.count_theta(None, None, theta_edges_deg=te, unit_vectors=(v, None),
                           angular_grid=grid)
    # the chord grid takes any vectors
    pc.count_theta(None, None, theta_edges_deg=te, unit_vectors=(v, None), angular_grid=-1)
    with pytest.raises(m.PairCountError):
        pc.count_r(synth.uniform_box(100, 10.0, seed=1), None, synth.log_edges(0.1, 1.0, 3),
                   10.0, options={"angular_grid": 1})
    ra, dec = full_sky(100, 511)
    with pytest.raises(m.PairCountError):
        pc.count_theta(ra, dec, None, None, te, angular_grid=65)
    with pytest.raises(m.PairCountError):
        pc.count_theta(ra, dec, None, None, te, angular_grid=-2)


def test_cap_fullsize_equals_chord_grid(pc, olib):
    """2*10^6 clustered points on the 30-degree seam cap, 20 bins in
    [0.01, 10] degrees: the angular grid's counts equal the 3-D chord grid's
    (which evaluates more candidate pairs), and sampled cross counts of 256
    points equal the oracle's."""
    say("angular grid N=2e6")
    ra, dec = synth.cap_radec(2_000_000, seed=4, radius_deg=30.0, clustered=True)
    te = synth.log_edges(0.01, 10.0, 20)
    a, _ = pc.count_theta(ra, dec, None, None, te, "fp32", angular_grid=2)
    sa = pc.stats()
    c, _ = pc.count_theta(ra, dec, None, None, te, "fp32", angular_grid=-1)
    sc = pc.stats()
    say("candidates angular", sa["candidate_pairs"], "chord", sc["candidate_pairs"])
    assert (a == c).all()
    assert sa["candidate_pairs"] < sc["candidate_pairs"]
    idx = np.sort(synth.rng_for(512).choice(ra.size, size=256, replace=False))
    got, _ = pc.count_theta(ra[idx], dec[idx], ra, dec, te, "fp32", angular_grid=2)
    want, _ = oracle.count_theta(ra[idx], dec[idx], ra, dec, te, lib=olib)
    assert (got == want).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_radec_converted_on_host(pc, olib, prec):
    """RA/DEC converted on the host (the default) with the same C library as
    the oracle: counts equal the oracle's bit for bit, for host and
    device-resident float64 and float32 input."""
    import torch
    say("radec on host", prec)
    ra, dec = full_sky(60000, 513)
    rr, rd = synth.cap_radec(50000, seed=514, radius_deg=40.0, dec0_deg=60.0)
    te = synth.log_edges(0.02, 6.0, 12)
    opts = None
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, None, None, te, prec, options=opts)
    assert (got == want).all()
    dra, ddec = (torch.from_numpy(a).to("cuda:0") for a in (ra, dec))
    got, _ = pc.count_theta(dra, ddec, None, None, te, prec, options=opts)
    assert (got == want).all()
    want, _ = oracle.count_theta(ra, dec, rr, rd, te, lib=olib)
    got, _ = pc.count_theta(ra, dec, rr, rd, te, prec, options=opts)
    assert (got == want).all()
    r32, d32 = ra.astype(np.float32), dec.astype(np.float32)
    want, _ = oracle.count_theta(r32.astype(np.float64), d32.astype(np.float64), None, None, te,
                                 lib=olib)
    got, _ = pc.count_theta(r32, d32, None, None, te, prec, options=opts)
    assert (got == want).all()
    bad = dec.copy()
    bad[7] = 91.0
    import paper_1911_03545_amd as m
    with pytest.raises(m.PairCountError):
        pc.count_theta(ra, bad, None, None, te, prec, options=opts)
