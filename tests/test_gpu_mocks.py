"""On-sky DD(rp, pi) with the line of sight through each pair's midpoint
(needs an MI355X).

Exact parity uses Cartesian positions from the oracle's own sky conversion
(host libm), or RA/DEC/distance input, which the library converts on the host
with the same formula and library by default, so both sides start from
identical binary64 positions; counts must then be identical and weighted sums
/ mean rp within 1e-12 relative.  RA/DEC/distance converted on the device
(the opt-in cf_options.radec_on_device) goes through the device's
trigonometric functions, whose last-bit agreement with the host libm is not
pinned: there only the size of any count difference is bounded.
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


def cart(m, olib):
    return oracle.sky_to_cartesian(m[:, 0], m[:, 1], m[:, 2], lib=olib)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mocks_auto_cross(pc, olib, prec):
    say("mocks auto/cross", prec)
    m1 = synth.sky_mock(12000, seed=401, radius_deg=4.0, dmin=400.0, dmax=700.0)
    m2 = synth.sky_mock(8000, seed=402, radius_deg=4.0, dmin=400.0, dmax=700.0,
                        clustered=False)
    v1, v2 = cart(m1, olib), cart(m2, olib)
    e = np.r_[0.0, synth.log_edges(0.2, 20.0, 10)]
    got, _ = pc.count_rppi_mocks(v1, None, e, 25.0, 25, prec, cartesian=True)
    want, _ = oracle.count_rppi_mocks(v1, None, e, 25.0, 25, lib=olib)
    assert want.sum() > 0
    assert (got == want).all(), np.argwhere(got != want)[:5]
    got, _ = pc.count_rppi_mocks(v1, v2, e, 25.0, 25, prec, cartesian=True)
    want, _ = oracle.count_rppi_mocks(v1, v2, e, 25.0, 25, lib=olib)
    assert (got == want).all()


@pytest.mark.parametrize("wtype", ["product", "sum"])
def test_mocks_weighted_ravg(pc, olib, wtype):
    say("mocks weighted", wtype)
    m = synth.sky_mock(9000, seed=403, radius_deg=3.0, dmin=300.0, dmax=500.0)
    v = cart(m, olib)
    w = synth.uniform_weights(9000, seed=404)
    e = np.r_[0.0, synth.log_edges(0.3, 15.0, 8)]
    got, gw, gr = pc.count_rppi_mocks(v, None, e, 20.0, 10, "fp64", w1=w, cartesian=True,
                                      weight_type=wtype, ravg=True)
    want, ww, wr = oracle.count_rppi_mocks(v, None, e, 20.0, 10, w1=w, lib=olib,
                                           weight_type=wtype, ravg=True)
    assert (got == want).all()
    rel_ok(gw, ww)
    rel_ok(gr, wr)


def test_mocks_edge_cases(pc, olib):
    """Radial pairs (rp = 0, pi on integer edges), equal-distance pairs
    (pi = 0), points at the observer (L = 0), coincident points, and a
    catalogue smaller than one block."""
    say("mocks edge cases")
    pts = []
    for D in (100.0, 101.0, 103.0, 110.0):
        pts.append([D, 0.0, 0.0])
        pts.append([0.0, D, 0.0])
    pts += [[300.0, 3.0, -4.0], [300.0, -3.0, 4.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0],
            [0.5, 0.0, 0.0], [300.0, 3.0, -4.0]]
    v = np.array(pts)
    for e in ([0.0, 1.0, 5.0, 10.0, 10.5], [0.5, 3.0, 10.0]):
        got, _, gr = pc.count_rppi_mocks(v, None, e, 12.0, 12, "fp64", cartesian=True, ravg=True)
        want, _, wr = oracle.count_rppi_mocks(v, None, e, 12.0, 12, lib=olib, ravg=True)
        assert (got == want).all(), (e, got, want)
        rel_ok(gr, wr)


def test_mocks_default_and_device_conversion(pc, olib):
    """RA, DEC, distance input: the default host conversion gives the
    counts of the oracle's own conversion bit for bit (float64 and float32
    columns); the opt-in device conversion may differ only through last-bit
    trigonometric differences, whose count is reported and bounded."""
    say("mocks default and device conversion")
    m = synth.sky_mock(20000, seed=405, radius_deg=5.0, dmin=600.0, dmax=900.0)
    e = synth.log_edges(0.5, 25.0, 10)
    host, _ = pc.count_rppi_mocks(cart(m, olib), None, e, 30.0, 15, "fp64", cartesian=True)
    got, _ = pc.count_rppi_mocks(m, None, e, 30.0, 15, "fp64")
    assert (got == host).all()
    dev, _ = pc.count_rppi_mocks(m, None, e, 30.0, 15, "fp64", options={"radec_on_device": 1})
    diff = np.abs(dev.astype(np.int64) - host.astype(np.int64))
    say("mocks device-conversion differences:", int(diff.sum()), "of", int(host.sum()))
    assert diff.sum() <= 1e-6 * host.sum() + 16
    # three separate columns, float32 input
    cols = tuple(np.ascontiguousarray(m[:, k]).astype(np.float32) for k in range(3))
    h32 = oracle.sky_to_cartesian(*[c.astype(np.float64) for c in cols], lib=olib)
    w32, _ = pc.count_rppi_mocks(h32, None, e, 30.0, 15, "fp64", cartesian=True)
    c32, _ = pc.count_rppi_mocks(cols, None, e, 30.0, 15, "fp64")
    assert (c32 == w32).all()
    d32, _ = pc.count_rppi_mocks(cols, None, e, 30.0, 15, "fp64", options={"radec_on_device": 1})
    assert np.abs(d32.astype(np.int64) - w32.astype(np.int64)).sum() <= 1e-6 * w32.sum() + 16


def test_mocks_errors(pc):
    import paper_1911_03545_amd as m
    say("mocks errors")
    good = synth.sky_mock(100, seed=406)
    e = synth.log_edges(0.5, 5.0, 4)
    bad = good.copy()
    bad[3, 2] = -1.0      # negative distance
    with pytest.raises(m.PairCountError):
        pc.count_rppi_mocks(bad, None, e, 10.0, 10, "fp64")
    bad = good.copy()
    bad[5, 1] = 95.0      # DEC out of range
    with pytest.raises(m.PairCountError):
        pc.count_rppi_mocks(bad, None, e, 10.0, 10, "fp64")
    with pytest.raises(m.PairCountError):
        pc.count_rppi_mocks(good, None, e, 0.0, 10, "fp64")
    c, _ = pc.count_rppi_mocks(np.zeros((0, 3)), None, e, 10.0, 10, "fp64")
    assert c.sum() == 0


def test_mocks_fullsize_sampled(pc, olib):
    """10^6 clustered on-sky points (a 10-degree cone, distances 500-1500):
    sampled cross counts of 256 points against the whole catalogue equal
    the oracle's, and the autocorrelation equals the cross-correlation of
    the catalogue with itself."""
    say("mocks N=1e6")
    m = synth.sky_mock(1_000_000, seed=407)
    v = cart(m, olib)
    e = synth.log_edges(0.1, 25.0, 20)
    auto, _ = pc.count_rppi_mocks(v, None, e, 40.0, 40, "fp64", cartesian=True)
    cross, _ = pc.count_rppi_mocks(v, v.copy(), e, 40.0, 40, "fp64", cartesian=True)
    assert (auto == cross).all()
    idx = np.sort(synth.rng_for(408).choice(v.shape[0], size=256, replace=False))
    got, _ = pc.count_rppi_mocks(v[idx], v, e, 40.0, 40, "fp64", cartesian=True)
    want, _ = oracle.count_rppi_mocks(v[idx], v, e, 40.0, 40, lib=olib)
    assert (got == want).all()


def test_mocks_radec_converted_on_host(pc, olib):
    """RA/DEC/distance converted on the host (the default) with the oracle's
    C library: counts equal the oracle's on its own conversion bit for bit."""
    say("mocks radec on host")
    m = synth.sky_mock(40000, seed=409, radius_deg=6.0, dmin=500.0, dmax=900.0)
    e = synth.log_edges(0.3, 25.0, 12)
    want, _ = oracle.count_rppi_mocks(cart(m, olib), None, e, 30.0, 15, lib=olib)
    got, _ = pc.count_rppi_mocks(m, None, e, 30.0, 15, "fp64")
    assert (got == want).all()
    bad = m.copy()
    bad[3, 2] = -5.0
    import paper_1911_03545_amd as mm
    with pytest.raises(mm.PairCountError):
        pc.count_rppi_mocks(bad, None, e, 30.0, 15, "fp64")
