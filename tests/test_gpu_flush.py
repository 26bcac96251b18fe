"""The overflow guard of the LDS histograms, forced from the host (needs an
MI355X).

Each wave keeps uint32 counters in LDS replicas and merges them into the
global uint64 bins before its pending pair evaluations could wrap a counter
(the per-thread histograms of section "Finding and updating the histogram
bins" and the OpenMP section, one per wavefront here).  At real sizes that
bound (2^31 evaluations per wave, 2^31 / waves for replicas shared by a
workgroup) is never reached, so cf_options.flush_pairs lowers it: every
variant of the sweep must then merge mid-sweep many times (cf_stats.flushes
> 0) and still give the oracle's counts bit for bit.  Covered: per-lane
replicas (unweighted DD(r)), shared replicas with weight sums (weighted
DD(r)), shared replicas with 2-D bins (DD(rp, pi)), private per-wave
replicas (batched calls), both precisions, and every point in one cell.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-12
THRESHOLDS = [1, 64, 4097]


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


@pytest.mark.parametrize("flush", THRESHOLDS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flush_r_unweighted(pc, olib, prec, flush):
    say("flush r unweighted", prec, flush)
    pts = synth.clustered_box(30000, 120.0, seed=601, nblobs=150, sigma=1.5)
    e = synth.log_edges(0.1, 12.0, 15)
    want, _ = oracle.count_r(pts, None, e, 120.0, lib=olib)
    got, _ = pc.count_r(pts, None, e, 120.0, prec, options={"flush_pairs": flush})
    assert (got == want).all()
    assert pc.stats()["flushes"] > 0
    x = pts[:7000]
    want, _ = oracle.count_r(x, pts, e, 120.0, lib=olib)
    got, _ = pc.count_r(x, pts, e, 120.0, prec, options={"flush_pairs": flush})
    assert (got == want).all()
    assert pc.stats()["flushes"] > 0


@pytest.mark.parametrize("flush", THRESHOLDS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flush_r_weighted(pc, olib, prec, flush):
    say("flush r weighted", prec, flush)
    pts = synth.clustered_box(25000, 110.0, seed=602, nblobs=120, sigma=1.5)
    w = synth.uniform_weights(25000, seed=603)
    e = np.r_[0.0, synth.log_edges(0.1, 11.0, 12)]
    want, ww = oracle.count_r(pts, None, e, 110.0, w1=w, lib=olib)
    got, gw = pc.count_r(pts, None, e, 110.0, prec, w1=w, options={"flush_pairs": flush})
    assert (got == want).all()
    rel_ok(gw, ww)
    assert pc.stats()["flushes"] > 0


@pytest.mark.parametrize("flush", THRESHOLDS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flush_rppi(pc, olib, prec, flush):
    say("flush rppi", prec, flush)
    pts = synth.clustered_box(25000, 130.0, seed=604, nblobs=120, sigma=1.5)
    e = synth.log_edges(0.1, 12.0, 10)
    want, _ = oracle.count_rppi(pts, None, e, 20.0, 20, 130.0, lib=olib)
    got, _ = pc.count_rppi(pts, None, e, 20.0, 20, 130.0, prec,
                           options={"flush_pairs": flush})
    assert (got == want).all()
    assert pc.stats()["flushes"] > 0


@pytest.mark.parametrize("flush", THRESHOLDS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flush_batched_private(pc, olib, prec, flush):
    say("flush batched", prec, flush)
    L = 150.0
    sizes = [9000, 300, 0, 6000, 1]
    cats = [synth.clustered_box(n, L, seed=610 + k, nblobs=max(1, n // 200), sigma=1.5)
            for k, n in enumerate(sizes)]
    e = synth.log_edges(0.2, 14.0, 9)
    got, _ = pc.count_rppi_batch(cats, e, 25.0, 25, L, prec, options={"flush_pairs": flush})
    assert pc.stats()["flushes"] > 0
    for k, p in enumerate(cats):
        want, _ = oracle.count_rppi(p, None, e, 25.0, 25, L, lib=olib)
        assert (got[k] == want).all(), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flush_one_cell(pc, olib, prec):
    """Every point in one cell: one column pair carries all the work, in
    items far larger than the bound, so each item is merged on its own."""
    say("flush one cell", prec)
    rng = synth.rng_for(620)
    pts = 40.0 + rng.uniform(0.0, 0.6, size=(6000, 3))
    w = synth.uniform_weights(6000, seed=621)
    e = np.r_[0.0, synth.log_edges(0.01, 1.5, 12)]
    want, ww = oracle.count_r(pts, None, e, 100.0, w1=w, lib=olib)
    for opts in ({"flush_pairs": 64}, {"flush_pairs": 64, "hist_copies": 1}):
        got, gw = pc.count_r(pts, None, e, 100.0, prec, w1=w, options=opts)
        assert (got == want).all()
        rel_ok(gw, ww)
        assert pc.stats()["flushes"] > 0
        got, _ = pc.count_r(pts, None, e, 100.0, prec, options=opts)
        assert (got == want).all()
    want, _ = oracle.count_rppi(pts, None, e, 1.0, 10, 100.0, lib=olib)
    got, _ = pc.count_rppi(pts, None, e, 1.0, 10, 100.0, prec, options={"flush_pairs": 64})
    assert (got == want).all()
    assert pc.stats()["flushes"] > 0


def test_flush_default_is_zero(pc):
    """At the default bound a modest call never merges mid-sweep."""
    pts = synth.uniform_box(20000, 100.0, seed=622)
    pc.count_r(pts, None, synth.log_edges(0.1, 10.0, 10), 100.0, "fp32")
    assert pc.stats()["flushes"] == 0
