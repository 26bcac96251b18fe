"""Exact fixed-point weight sums (cf_options.deterministic_weights; needs an
MI355X).

The paper accumulates weight_func(w_i, w_j) per pair into binary64 bins
(section 2.1 and the histogram update); with atomics the rounding of that
sum depends on the order of the adds.  With deterministic_weights the sweep
sums every binary64 pair weight exactly in 192-bit fixed point and rounds
once, so the result must equal the oracle's exactly rounded sum (Shewchuk
expansions, rounded once) bit for bit, in every run, for both precisions,
every statistic, both pair-weight types, mixed signs, self-pairs, mid-sweep
histogram merges and batched calls; weights too spread out for the grid are
refused with CF_EINVAL.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DET = {"deterministic_weights": 1}


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


def weights(kind, n, seed):
    rng = synth.rng_for(seed)
    if kind == "f32":        # float32 values in [0.5, 1.5)
        return synth.uniform_weights(n, seed)
    if kind == "f64":        # full 53-bit binary64 values spanning 2^10
        return np.exp2(rng.uniform(-5.0, 5.0, n))
    if kind == "signed":     # float32 magnitudes with both signs
        w = synth.uniform_weights(n, seed).astype(np.float64)
        return np.where(rng.random(n) < 0.4, -w, w)
    if kind == "dyadic":     # small dyadic rationals, many exact ties
        return rng.integers(1, 9, n) / 8.0
    raise ValueError(kind)


def same_bits(got, want):
    """Equal as binary64 values (zeros aside, equal values have equal bits)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    want = np.asarray(want, dtype=np.float64).ravel()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (bad[:8], got[bad[:8]], want[bad[:8]])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["f32", "f64", "signed", "dyadic"])
@pytest.mark.parametrize("wtype", ["product", "sum"])
def test_r_exact(pc, olib, prec, kind, wtype):
    say("det r", prec, kind, wtype)
    n = 24000
    pts = synth.clustered_box(n, 100.0, seed=701, nblobs=100, sigma=1.5)
    w = weights(kind, n, 702)
    # first edge zero: the self-pair weights join bin 0
    e = np.r_[0.0, synth.log_edges(0.1, 10.0, 14)]
    want, ww = oracle.count_r(pts, None, e, 100.0, w1=w, lib=olib, weight_type=wtype)
    got, gw = pc.count_r(pts, None, e, 100.0, prec, w1=w, options=DET, weight_type=wtype)
    assert (got == want).all()
    same_bits(gw, ww)
    # cross-correlation of a subset against all points, no periodic wrap
    x = pts[:5000]
    want, ww = oracle.count_r(x, pts, e, 0.0, w1=w[:5000], w2=w, lib=olib, weight_type=wtype)
    got, gw = pc.count_r(x, pts, e, 0.0, prec, w1=w[:5000], w2=w, options=DET,
                         weight_type=wtype)
    assert (got == want).all()
    same_bits(gw, ww)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_repeat_runs_identical(pc, prec):
    """The default binary64 sums may differ in the last bits between runs;
    the fixed-point sums never do."""
    say("det repeat", prec)
    n = 40000
    pts = synth.clustered_box(n, 120.0, seed=703, nblobs=150, sigma=1.5)
    w = weights("f64", n, 704)
    e = synth.log_edges(0.1, 12.0, 16)
    ref = None
    for _ in range(4):
        _, gw = pc.count_r(pts, None, e, 120.0, prec, w1=w, options=DET)
        if ref is None:
            ref = gw.copy()
        assert np.array_equal(gw.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wtype", ["product", "sum"])
def test_rppi_exact(pc, olib, prec, wtype):
    say("det rppi", prec, wtype)
    n = 20000
    pts = synth.clustered_box(n, 150.0, seed=705, nblobs=100, sigma=2.0)
    w = weights("f32", n, 706)
    e = synth.log_edges(0.2, 15.0, 12)
    want, ww = oracle.count_rppi(pts, None, e, 20.0, 20, 150.0, w1=w, lib=olib,
                                 weight_type=wtype)
    got, gw = pc.count_rppi(pts, None, e, 20.0, 20, 150.0, prec, w1=w, options=DET,
                            weight_type=wtype)
    assert (got == want).all()
    same_bits(gw, ww)


def test_theta_exact(pc, olib):
    say("det theta")
    ra, dec = synth.cap_radec(20000, seed=707, radius_deg=10.0, clustered=True)
    w = weights("f64", ra.size, 708)
    e = np.r_[0.0, np.logspace(-2, 0.3, 12)]
    want, ww = oracle.count_theta(ra, dec, None, None, e, w1=w, lib=olib)
    got, gw = pc.count_theta(ra, dec, None, None, e, "fp64", w1=w, options=DET)
    assert (got == want).all()
    same_bits(gw, ww)


def test_mocks_exact(pc, olib):
    say("det mocks")
    m = synth.sky_mock(15000, seed=709, radius_deg=4.0, dmin=400.0, dmax=700.0)
    # Cartesian positions from the oracle's own host conversion
    v = oracle.sky_to_cartesian(m[:, 0], m[:, 1], m[:, 2], lib=olib)
    w = weights("f32", m.shape[0], 710)
    e = synth.log_edges(0.5, 20.0, 10)
    for wtype in ("product", "sum"):
        want, ww = oracle.count_rppi_mocks(v, None, e, 20.0, 10, w1=w, lib=olib,
                                           weight_type=wtype)
        got, gw = pc.count_rppi_mocks(v, None, e, 20.0, 10, "fp64", w1=w, options=DET,
                                      cartesian=True, weight_type=wtype)
        assert (got == want).all()
        same_bits(gw, ww)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_exact(pc, olib, prec):
    """Private per-wave replicas, merged per catalogue."""
    say("det batch", prec)
    L = 150.0
    sizes = [7000, 400, 0, 5000, 1]
    cats = [synth.clustered_box(n, L, seed=711 + k, nblobs=max(1, n // 200), sigma=1.5)
            for k, n in enumerate(sizes)]
    ws = [weights("signed", n, 720 + k) for k, n in enumerate(sizes)]
    # (first rp edge zero: each catalogue's self-pair weights join its bin (0, 0))
    for e in (synth.log_edges(0.2, 14.0, 9), np.r_[0.0, synth.log_edges(0.2, 14.0, 8)]):
        for wtype in ("product", "sum"):
            got, gw = pc.count_rppi_batch(cats, e, 25.0, 25, L, prec, weights=ws, options=DET,
                                          weight_type=wtype)
            for k, p in enumerate(cats):
                want, ww = oracle.count_rppi(p, None, e, 25.0, 25, L, w1=ws[k], lib=olib,
                                             weight_type=wtype)
                assert (got[k] == want).all(), (k, wtype)
                same_bits(gw[k], ww)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("flush", [1, 97])
def test_exact_with_forced_merges(pc, olib, prec, flush):
    """Mid-sweep merges of the limb sums (cf_options.flush_pairs)."""
    say("det flush", prec, flush)
    n = 15000
    pts = synth.clustered_box(n, 90.0, seed=730, nblobs=80, sigma=1.5)
    w = weights("signed", n, 731)
    e = np.r_[0.0, synth.log_edges(0.1, 9.0, 10)]
    want, ww = oracle.count_r(pts, None, e, 90.0, w1=w, lib=olib)
    got, gw = pc.count_r(pts, None, e, 90.0, prec, w1=w,
                         options=dict(DET, flush_pairs=flush))
    assert (got == want).all()
    same_bits(gw, ww)
    assert pc.stats()["flushes"] > 0


def test_mean_separation_with_exact_weights(pc, olib):
    """The mean separation divides by the exact weight sum; its numerator
    stays a binary64 sum."""
    say("det ravg")
    n = 20000
    pts = synth.clustered_box(n, 100.0, seed=732, nblobs=100, sigma=1.5)
    w = weights("f32", n, 733)
    e = synth.log_edges(0.1, 10.0, 12)
    want, ww, wr = oracle.count_r(pts, None, e, 100.0, w1=w, lib=olib, ravg=True)
    got, gw, gr = pc.count_r(pts, None, e, 100.0, "fp64", w1=w, options=DET, ravg=True)
    assert (got == want).all()
    same_bits(gw, ww)
    np.testing.assert_allclose(gr, wr, rtol=1e-12, atol=0)


def test_one_cell_large_sums(pc, olib):
    """Every point in one cell: every pair of every block in a few large
    items, so the limb sums carry across words."""
    say("det one cell")
    rng = synth.rng_for(734)
    pts = 40.0 + rng.uniform(0.0, 0.6, size=(8000, 3))
    w = np.exp2(rng.uniform(-9.0, 9.0, 8000))
    e = np.r_[0.0, synth.log_edges(0.01, 1.5, 8)]
    want, ww = oracle.count_r(pts, None, e, 100.0, w1=w, lib=olib)
    for prec in ("fp64", "fp32"):
        got, gw = pc.count_r(pts, None, e, 100.0, prec, w1=w, options=DET)
        assert (got == want).all()
        same_bits(gw, ww)


def test_refuses_weights_without_a_grid(pc):
    import paper_1911_03545_amd as m
    pts = synth.uniform_box(2000, 50.0, seed=735)
    e = synth.log_edges(0.5, 5.0, 5)
    # products of binary64 weights spanning 2^80: no 2^95 window holds them
    w = np.exp2(synth.rng_for(736).uniform(-40.0, 40.0, 2000))
    with pytest.raises(m.PairCountError):
        pc.count_r(pts, None, e, 50.0, "fp64", w1=w, options=DET)
    # the same weights sum exactly with binary64 atomics (no option)
    pc.count_r(pts, None, e, 50.0, "fp64", w1=w)
    # and the context works on afterwards
    w2 = synth.uniform_weights(2000, 737)
    pc.count_r(pts, None, e, 50.0, "fp64", w1=w2, options=DET)
