"""Mean separation per bin and pair weight types on the GPU (needs an MI355X).

Counts must equal the oracle's bit for bit.  Weight sums and, in binary64
mode, mean separations must match the oracle's exactly rounded values to a
relative 1e-12 (only the order of accumulation differs).  In float32 mode
the mean is taken over the separations of the float32 evaluation; the bound
used below follows from its roundings: each float32 coordinate (relative to
the domain origin, magnitude <= C) is within u*C of the exact one, the
periodic offset within u*L, the subtraction adds u*|dx|, so each component
of the separation vector is within 5uC and its length within sqrt(3) * 5uC;
the float32 sum of squares and square root add 4u relative.  Hence
|r_f32 - r| <= 10 u C + 8 u r per pair, and the same for a weighted mean
with positive weights (u = 2^-24).  Angles: the same on unit vectors
(C = 2) for the chord, times d(theta)/d(chord) <= 1.01 below 16 degrees, in
degrees, plus the float32 arc sine.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
RTOL64 = 1e-12
R2D = 180.0 / math.pi


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


def rel_ok(got, want, rtol):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= rtol), (rel.max(), got, want)


def check_mean(got, want, prec, C, angle=False):
    if prec == "fp64":
        rel_ok(got, want, RTOL64)
        return
    if angle:
        tol = (10 * U32 * C + 8 * U32 * np.radians(want)) * 1.01 * R2D + 4 * U32 * want
    else:
        tol = 10 * U32 * C + 8 * U32 * want
    err = np.abs(got - want)
    assert np.all(err <= tol), (err.max(), (err / np.maximum(tol, 1e-300)).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [120.0, 0.0])
def test_ravg_r_unweighted(pc, olib, prec, box):
    say("ravg r", prec, box)
    pts = synth.clustered_box(12000, 120.0, seed=301, nblobs=60)
    e = np.r_[0.0, synth.log_edges(0.1, 15.0, 14)]
    got, gw, gr = pc.count_r(pts, None, e, box, prec, ravg=True)
    want, _, wr = oracle.count_r(pts, None, e, box, lib=olib, ravg=True)
    assert gw is None
    assert (got == want).all()
    check_mean(gr, wr, prec, 120.0)
    # cross-correlation against a second catalogue
    other = synth.uniform_box(7000, 120.0, seed=302)
    got, _, gr = pc.count_r(pts, other, e, box, prec, ravg=True)
    want, _, wr = oracle.count_r(pts, other, e, box, lib=olib, ravg=True)
    assert (got == want).all()
    check_mean(gr, wr, prec, 120.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wtype", ["product", "sum"])
def test_ravg_r_weighted(pc, olib, prec, wtype):
    say("ravg r weighted", prec, wtype)
    pts = synth.clustered_box(10000, 100.0, seed=303, nblobs=50)
    w = synth.uniform_weights(10000, seed=304)
    e = np.r_[0.0, synth.log_edges(0.2, 12.0, 10)]
    got, gw, gr = pc.count_r(pts, None, e, 100.0, prec, w1=w, weight_type=wtype, ravg=True)
    want, ww, wr = oracle.count_r(pts, None, e, 100.0, w1=w, lib=olib, weight_type=wtype,
                                  ravg=True)
    assert (got == want).all()
    rel_ok(gw, ww, RTOL64)
    check_mean(gr, wr, prec, 100.0)
    # weight sums alone (no mean) with summed pair weights
    got, gw = pc.count_r(pts, None, e, 100.0, prec, w1=w, weight_type=wtype)
    assert (got == want).all()
    rel_ok(gw, ww, RTOL64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [90.0, 0.0])
def test_ravg_rppi(pc, olib, prec, box):
    say("ravg rppi", prec, box)
    pts = synth.clustered_box(9000, 90.0, seed=305, nblobs=45)
    w = synth.uniform_weights(9000, seed=306)
    e = synth.log_edges(0.1, 20.0, 10)
    got, _, gr = pc.count_rppi(pts, None, e, 20.0, 10, box, prec, ravg=True)
    want, _, wr = oracle.count_rppi(pts, None, e, 20.0, 10, box, lib=olib, ravg=True)
    assert (got == want).all()
    check_mean(gr, wr, prec, 90.0)
    got, gw, gr = pc.count_rppi(pts, None, e, 20.0, 10, box, prec, w1=w, weight_type="sum",
                                ravg=True)
    want, ww, wr = oracle.count_rppi(pts, None, e, 20.0, 10, box, w1=w, lib=olib,
                                     weight_type="sum", ravg=True)
    assert (got == want).all()
    rel_ok(gw, ww, RTOL64)
    check_mean(gr, wr, prec, 90.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ravg_theta(pc, olib, prec):
    say("ravg theta", prec)
    ra, dec = synth.cap_radec(8000, seed=307, clustered=True)
    ra2, dec2 = synth.cap_radec(6000, seed=308)
    e = synth.log_edges(0.02, 8.0, 10)
    v = oracle.radec_to_unit(ra, dec, lib=olib)
    v2 = oracle.radec_to_unit(ra2, dec2, lib=olib)
    got, _, gr = pc.count_theta(None, None, theta_edges_deg=e, precision=prec,
                                unit_vectors=(v, None), ravg=True)
    want, _, wr = oracle.count_theta(ra, dec, theta_edges_deg=e, lib=olib, ravg=True)
    assert (got == want).all()
    check_mean(gr, wr, prec, 2.0, angle=True)
    w = synth.uniform_weights(8000, seed=309)
    w2 = synth.uniform_weights(6000, seed=310)
    got, gw, gr = pc.count_theta(None, None, theta_edges_deg=e, precision=prec, w1=w, w2=w2,
                                 unit_vectors=(v, v2), weight_type="sum", ravg=True)
    want, ww, wr = oracle.count_theta(ra, dec, ra2, dec2, theta_edges_deg=e, w1=w, w2=w2,
                                      lib=olib, weight_type="sum", ravg=True)
    assert (got == want).all()
    rel_ok(gw, ww, RTOL64)
    check_mean(gr, wr, prec, 2.0, angle=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ravg_batch(pc, olib, prec):
    say("ravg batch", prec)
    sizes = [3000, 0, 800, 5000, 1]
    cats = [synth.clustered_box(n, 150.0, seed=320 + k, nblobs=max(1, n // 200))
            if n else np.zeros((0, 3)) for k, n in enumerate(sizes)]
    ws = [synth.uniform_weights(n, seed=330 + k) for k, n in enumerate(sizes)]
    e = np.r_[0.0, synth.log_edges(0.2, 15.0, 8)]
    got, gw, gr = pc.count_rppi_batch(cats, e, 15.0, 5, 150.0, prec, weights=ws,
                                      weight_type="sum", ravg=True)
    for k, p in enumerate(cats):
        want, ww, wr = oracle.count_rppi(p, None, e, 15.0, 5, 150.0, w1=ws[k], lib=olib,
                                         weight_type="sum", ravg=True)
        assert (got[k] == want).all(), k
        rel_ok(gw[k], ww, RTOL64)
        check_mean(gr[k], wr, prec, 150.0)


def test_ravg_graph_replay(pc, olib):
    """Replays fill the mean-separation array passed to each call."""
    import torch
    say("ravg graph")
    n, L = 20000, 100.0
    cols = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    e = synth.log_edges(0.2, 10.0, 10)
    g = {"use_graph": 1}
    for rep in range(3):
        pts = synth.clustered_box(n, L, seed=340 + rep, nblobs=80)
        for k in range(3):
            cols[k].copy_(torch.from_numpy(np.ascontiguousarray(pts[:, k])))
        torch.cuda.synchronize()
        got, _, gr = pc.count_r(cols, None, e, L, "fp32", options=g, ravg=True)
        assert pc.stats()["replayed"] == (1 if rep > 0 else 0), rep
        want, _, wr = pc.count_r(cols, None, e, L, "fp32", ravg=True)
        assert (got == want).all(), rep
        # same pairs and separations; only the order of the sums may differ
        rel_ok(gr, wr, RTOL64)


def test_ravg_errors_and_empty(pc):
    import paper_1911_03545_amd as m
    say("ravg errors")
    pts = synth.uniform_box(100, 50.0, seed=350)
    e = synth.log_edges(0.5, 5.0, 4)
    with pytest.raises(m.PairCountError):
        pc.count_r(pts, None, e, 50.0, "fp32", weight_type="sum")
    with pytest.raises(ValueError):
        pc.count_r(pts, None, e, 50.0, "fp32", weight_type="max")
    c, _, r = pc.count_r(np.zeros((0, 3)), None, e, 50.0, "fp32", ravg=True)
    assert c.sum() == 0 and (r == 0).all()
    # a bin without pairs reports 0
    c, _, r = pc.count_r(pts[:2], None, [0.001, 0.002], 50.0, "fp64", ravg=True)
    assert c[0] == 0 and r[0] == 0.0
