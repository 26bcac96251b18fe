"""x/y refinement of the 3-D grids (columns reach/k wide, (2k+1)^2
neighbour columns, z windows narrowed by the transverse distance when the
reach is a ball) against the oracle (needs an MI355X).

Refinement only changes which pairs are evaluated, so counts must equal the
oracle's bit for bit for every k: auto and cross, periodic and not, r, rp/pi
(no z narrowing), the on-sky statistic and angular chords, weights, a
lattice with exact edge ties, and a periodic box barely three reaches wide.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def opts(k, **kw):
    return dict(xy_refine=k, **kw)


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("box", [80.0, 0.0])
def test_r_auto_cross(pc, olib, k, box):
    say("refine r", k, box)
    a = synth.clustered_box(20000, 80.0, seed=71, nblobs=100, sigma=1.5)
    b = synth.uniform_box(9000, 80.0, seed=72)
    e = synth.log_edges(0.05, 12.0, 15)
    for prec in ("fp64", "fp32"):
        want, _ = oracle.count_r(a, None, e, box, lib=olib)
        got, _ = pc.count_r(a, None, e, box, prec, options=opts(k))
        assert (got == want).all(), (prec, got, want)
        st = pc.stats()
        assert st["xy_refine"] == k
        want, _ = oracle.count_r(a, b, e, box, lib=olib)
        got, _ = pc.count_r(a, b, e, box, prec, options=opts(k))
        assert (got == want).all(), (prec, got, want)


@pytest.mark.parametrize("k", [2, 4])
def test_r_lattice_ties_weighted(pc, olib, k):
    say("refine lattice", k)
    pts = synth.lattice_box(6000, 64, seed=73)
    w = synth.uniform_weights(6000, seed=74)
    e = np.array([0.0, 1.0, 2.0, 3.0, 5.0, 8.0, 13.0])
    want, ww = oracle.count_r(pts, None, e, 64.0, w1=w, lib=olib)
    for prec in ("fp64", "fp32"):
        got, gw = pc.count_r(pts, None, e, 64.0, prec, w1=w, options=opts(k))
        assert (got == want).all(), prec
        np.testing.assert_allclose(gw, ww, rtol=1e-12)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("box", [100.0, 0.0])
def test_rppi(pc, olib, k, box):
    say("refine rppi", k, box)
    a = synth.clustered_box(20000, 100.0, seed=75, nblobs=100)
    b = synth.uniform_box(8000, 100.0, seed=76)
    e = synth.log_edges(0.1, 15.0, 10)
    for prec in ("fp64", "fp32"):
        want, _ = oracle.count_rppi(a, None, e, 20.0, 20, box, lib=olib)
        got, _ = pc.count_rppi(a, None, e, 20.0, 20, box, prec, options=opts(k))
        assert (got == want).all(), prec
        want, _ = oracle.count_rppi(a, b, e, 20.0, 20, box, lib=olib)
        got, _ = pc.count_rppi(a, b, e, 20.0, 20, box, prec, options=opts(k))
        assert (got == want).all(), prec


def test_tight_box(pc, olib):
    """A periodic box just over three reaches wide (three columns at k = 1,
    twelve at k = 4): every refinement gives the oracle's counts."""
    say("refine tight box")
    pts = synth.uniform_box(5000, 31.0, seed=77)
    e = synth.log_edges(0.5, 10.0, 6)
    want, _ = oracle.count_r(pts, None, e, 31.0, lib=olib)
    for k in (1, 2, 3, 4):
        got, _ = pc.count_r(pts, None, e, 31.0, "fp32", options=opts(k))
        assert (got == want).all(), k
        assert pc.stats()["xy_refine"] == k


def test_mocks_and_theta_chord(pc, olib):
    say("refine mocks, theta chord grid")
    m = synth.sky_mock(9000, seed=78, radius_deg=4.0, dmin=400.0, dmax=700.0)
    v = oracle.sky_to_cartesian(m[:, 0], m[:, 1], m[:, 2], lib=olib)
    e = np.r_[0.0, synth.log_edges(0.2, 20.0, 10)]
    want, _ = oracle.count_rppi_mocks(v, None, e, 25.0, 25, lib=olib)
    for k in (2, 3):
        got, _ = pc.count_rppi_mocks(v, None, e, 25.0, 25, "fp64", cartesian=True,
                                     options=opts(k))
        assert (got == want).all(), k
    ra, dec = synth.cap_radec(15000, seed=79, radius_deg=10.0, clustered=True, nblobs=100,
                              sigma_deg=0.2)
    te = synth.log_edges(0.02, 3.0, 10)
    u = oracle.radec_to_unit(ra, dec, lib=olib)
    want, _ = oracle.count_theta(ra, dec, None, None, te, lib=olib)
    for k in (2, 3):
        got, _ = pc.count_theta(None, None, theta_edges_deg=te, precision="fp32",
                                unit_vectors=(u, None), angular_grid=-1, options=opts(k))
        assert (got == want).all(), k


def test_refine_errors(pc):
    import paper_1911_03545_amd as m
    pts = synth.uniform_box(100, 10.0, seed=1)
    e = synth.log_edges(0.1, 1.0, 3)
    for k in (-1, 5):
        with pytest.raises(m.PairCountError):
            pc.count_r(pts, None, e, 10.0, options=opts(k))
