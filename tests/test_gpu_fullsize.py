"""Parity at the full workload sizes (needs an MI355X).

At these sizes the GPU result is checked against:

* the oracle's full histograms, computed ahead of the tests by
  ``tests/golden/make_fullsize.py`` (the exactly pruned oracle, equal to the
  brute-force definition bit for bit) and stored in
  ``tests/golden/fullsize_*.json`` with the SHA-256 of their inputs, which the
  tests draw again and check; every auto (and cross) histogram of both
  precisions must equal them bit for bit, and weighted sums must lie within
  1e-12 of the exactly rounded sums (equal them bit for bit with
  deterministic_weights);
* sampled outputs the oracle computes on the spot: cross counts of a random
  subset S of the first catalogue against the whole second catalogue;
* properties that hold at any size: the float32+recheck path equals the
  binary64 path bit for bit, and the autocorrelation launch equals the
  cross-correlation of the catalogue with itself.

Workloads: clustered periodic boxes of 10^6 points (L = 420) and 4 x 10^6
weighted points (L = 1100), and a 30-degree cap with 2 x 10^6 clustered and
5 x 10^6 uniform RA/DEC points.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from golden import make_fullsize as recipes

pytestmark = pytest.mark.gpu


def golden(name, *inputs):
    """The stored oracle histograms of a workload, after checking that the
    inputs drawn here are the ones they were computed on."""
    path = recipes.path_of(name)
    assert os.path.exists(path), f"missing {path}: run tests/golden/make_fullsize.py"
    with open(path) as fh:
        g = json.load(fh)
    assert g["input_sha256"] == recipes.sha(*inputs), f"{name}: inputs differ from the golden's"
    g["counts"] = np.array(g["counts"], dtype=np.uint64)
    if "wsum_hex" in g:
        g["wsum"] = np.array([float.fromhex(v) for v in g["wsum_hex"]])
    return g

WSUM_RTOL = 1e-12
NSAMPLE = 384


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


def sample(n, k, seed):
    return np.sort(synth.rng_for(seed).choice(n, size=k, replace=False))


def check_w(got, want, rtol=WSUM_RTOL):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= rtol), (rel.max(), got, want)


# ---------------------------------------------------- 10^6 points, L = 420
@pytest.fixture(scope="module")
def box420():
    return recipes.box420(np.float64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_r_n1e6(pc, olib, box420, dtype):
    say("r N=1e6 L=420", dtype.__name__)
    pts = box420.astype(dtype)
    e = synth.log_edges(0.1, 25.0, 20)
    g = golden("r_n1e6_L420_" + ("f64" if dtype == np.float64 else "f32"), pts)
    assert (np.array(g["recipe"]["edges"]) == e).all()
    a32, _ = pc.count_r(pts, None, e, 420.0, "fp32")
    a64, _ = pc.count_r(pts, None, e, 420.0, "fp64")
    assert (a32 == g["counts"]).all(), (a32, g["counts"])
    assert (a64 == g["counts"]).all()
    x32, _ = pc.count_r(pts, pts.copy(), e, 420.0, "fp32")
    assert (a32 == x32).all()
    assert int(a32.sum()) % 2 == 0
    s = pts[sample(pts.shape[0], NSAMPLE, 11)]
    got, _ = pc.count_r(s, pts, e, 420.0, "fp32")
    want, _ = oracle.count_r(s, pts, e, 420.0, lib=olib)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_rppi_n1e6(pc, olib, box420, dtype):
    say("rppi N=1e6 L=420", dtype.__name__)
    pts = box420.astype(dtype)
    e = synth.log_edges(0.1, 25.0, 20)
    g = golden("rppi_n1e6_L420_" + ("f64" if dtype == np.float64 else "f32"), pts)
    a32, _ = pc.count_rppi(pts, None, e, 40.0, 40, 420.0, "fp32")
    a64, _ = pc.count_rppi(pts, None, e, 40.0, 40, 420.0, "fp64")
    assert (a32.ravel() == g["counts"]).all()
    assert (a64.ravel() == g["counts"]).all()
    x32, _ = pc.count_rppi(pts, pts.copy(), e, 40.0, 40, 420.0, "fp32")
    assert (a32 == x32).all()
    s = pts[sample(pts.shape[0], NSAMPLE, 12)]
    got, _ = pc.count_rppi(s, pts, e, 40.0, 40, 420.0, "fp32")
    want, _ = oracle.count_rppi(s, pts, e, 40.0, 40, 420.0, lib=olib)
    assert (got == want).all()


def test_r_ravg_n1e6(pc, olib, box420):
    """Mean separation per bin at full size: sampled cross means against the
    oracle (binary64: 1e-12 relative; float32: the float32 rounding bound,
    10 u C + 8 u r with C = 420), and the full autocorrelation's float32
    means within that bound of the binary64 ones."""
    say("ravg r N=1e6 L=420")
    u = 2.0 ** -24
    pts = box420
    e = synth.log_edges(0.1, 25.0, 20)
    a32, _, r32 = pc.count_r(pts, None, e, 420.0, "fp32", ravg=True)
    a64, _, r64 = pc.count_r(pts, None, e, 420.0, "fp64", ravg=True)
    assert (a32 == a64).all()
    assert np.all(np.abs(r32 - r64) <= 2 * (10 * u * 420.0 + 8 * u * r64))
    s = pts[sample(pts.shape[0], NSAMPLE, 17)]
    want, _, wr = oracle.count_r(s, pts, e, 420.0, lib=olib, ravg=True)
    got, _, gr = pc.count_r(s, pts, e, 420.0, "fp64", ravg=True)
    assert (got == want).all()
    check_w(gr, wr)
    got, _, gr = pc.count_r(s, pts, e, 420.0, "fp32", ravg=True)
    assert (got == want).all()
    assert np.all(np.abs(gr - wr) <= 10 * u * 420.0 + 8 * u * wr)


# ------------------------------------------- 4 x 10^6 weighted, L = 1100
@pytest.fixture(scope="module")
def box1100():
    return recipes.box1100()


def test_r_weighted_n4e6(pc, olib, box1100):
    say("weighted r N=4e6 L=1100")
    pts, w = box1100
    e = synth.log_edges(0.1, 50.0, 25)
    g = golden("r_w_n4e6_L1100", pts, w)
    c32, w32 = pc.count_r(pts, None, e, 1100.0, "fp32", w1=w)
    c64, w64 = pc.count_r(pts, None, e, 1100.0, "fp64", w1=w)
    assert (c32 == g["counts"]).all() and (c64 == g["counts"]).all()
    check_w(w32, g["wsum"])
    check_w(w64, g["wsum"])
    # exact fixed-point sums: the oracle's exactly rounded sums, bit for bit
    for prec in ("fp32", "fp64"):
        cd, wd = pc.count_r(pts, None, e, 1100.0, prec, w1=w,
                            options={"deterministic_weights": 1})
        assert (cd == g["counts"]).all()
        assert np.array_equal(wd, g["wsum"]), prec
    idx = sample(pts.shape[0], NSAMPLE, 13)
    got, gw = pc.count_r(pts[idx], pts, e, 1100.0, "fp32", w1=w[idx], w2=w)
    want, ww = oracle.count_r(pts[idx], pts, e, 1100.0, w1=w[idx], w2=w, lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


def test_rppi_weighted_n4e6(pc, olib, box1100):
    say("weighted rppi N=4e6 L=1100")
    pts, w = box1100
    e = synth.log_edges(0.1, 50.0, 25)
    g = golden("rppi_w_n4e6_L1100", pts, w)
    c32, w32 = pc.count_rppi(pts, None, e, 40.0, 40, 1100.0, "fp32", w1=w)
    c64, w64 = pc.count_rppi(pts, None, e, 40.0, 40, 1100.0, "fp64", w1=w)
    assert (c32.ravel() == g["counts"]).all() and (c64.ravel() == g["counts"]).all()
    check_w(w32.ravel(), g["wsum"])
    check_w(w64.ravel(), g["wsum"])
    for prec in ("fp32", "fp64"):
        cd, wd = pc.count_rppi(pts, None, e, 40.0, 40, 1100.0, prec, w1=w,
                               options={"deterministic_weights": 1})
        assert (cd.ravel() == g["counts"]).all()
        assert np.array_equal(wd.ravel(), g["wsum"]), prec
    idx = sample(pts.shape[0], NSAMPLE, 14)
    got, gw = pc.count_rppi(pts[idx], pts, e, 40.0, 40, 1100.0, "fp32", w1=w[idx], w2=w)
    want, ww = oracle.count_rppi(pts[idx], pts, e, 40.0, 40, 1100.0, w1=w[idx], w2=w,
                                 lib=olib)
    assert (got == want).all()
    check_w(gw, ww)


# ------------------------------------- theta on a 30-degree cap, 2e6 / 5e6
@pytest.fixture(scope="module")
def cap(olib):
    ra_d, dec_d = recipes.cap_d()
    ra_r, dec_r = recipes.cap_r(5_000_000)
    # unit vectors from the host conversion the oracle itself uses
    v_d = oracle.radec_to_unit(ra_d, dec_d, lib=olib)
    v_r = oracle.radec_to_unit(ra_r, dec_r, lib=olib)
    return (ra_d, dec_d, v_d), (ra_r, dec_r, v_r)


def test_theta_dd_n2e6(pc, olib, cap):
    say("theta DD N=2e6")
    (ra, dec, v), _ = cap
    e = synth.log_edges(0.01, 10.0, 20)
    g = golden("theta_dd_cap_n2e6", ra, dec)
    a32, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp32",
                            unit_vectors=(v, None))
    a64, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp64",
                            unit_vectors=(v, None))
    assert (a32 == g["counts"]).all() and (a64 == g["counts"]).all()
    x32, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp32",
                            unit_vectors=(v, v.copy()))
    assert (a32 == x32).all()
    idx = sample(ra.size, NSAMPLE, 15)
    got, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp32",
                            unit_vectors=(v[idx], v))
    want, _ = oracle.count_theta(ra[idx], dec[idx], ra, dec, e, lib=olib)
    assert (got == want).all()
    # RA/DEC input, converted on the host by default: identical counts
    r32, _ = pc.count_theta(ra, dec, theta_edges_deg=e, precision="fp32")
    assert (r32 == a32).all()
    # converted on the device (opt-in): parity across math libraries is not
    # pinned, so only the size of any difference is bounded and reported
    r32, _ = pc.count_theta(ra, dec, theta_edges_deg=e, precision="fp32",
                            options={"radec_on_device": 1})
    diff = np.abs(r32.astype(np.int64) - a32.astype(np.int64))
    say("theta DD device-conversion differences:", int(diff.sum()), "of", int(a32.sum()))
    assert diff.sum() <= 1e-9 * a32.sum() + 64


def test_theta_dr_n2e6_5e6(pc, olib, cap):
    say("theta DR N=2e6 x 5e6")
    (ra_d, dec_d, v_d), (ra_r, dec_r, v_r) = cap
    e = synth.log_edges(0.01, 10.0, 20)
    c32, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp32",
                            unit_vectors=(v_d, v_r))
    c64, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp64",
                            unit_vectors=(v_d, v_r))
    assert (c32 == c64).all()
    # the whole D against the first 5e5 randoms, against the stored oracle
    # histogram, from RA/DEC converted on the host (the default)
    k = 500_000
    g = golden("theta_dr_cap_n2e6_r5e5", ra_d, dec_d, ra_r[:k], dec_r[:k])
    for prec in ("fp32", "fp64"):
        got, _ = pc.count_theta(ra_d, dec_d, ra_r[:k], dec_r[:k], theta_edges_deg=e,
                                precision=prec)
        assert (got == g["counts"]).all(), prec
    idx = sample(ra_d.size, NSAMPLE // 2, 16)
    got, _ = pc.count_theta(None, None, theta_edges_deg=e, precision="fp32",
                            unit_vectors=(v_d[idx], v_r))
    want, _ = oracle.count_theta(ra_d[idx], dec_d[idx], ra_r, dec_r, e, lib=olib)
    assert (got == want).all()


# ------------------------- batched DD(rp, pi) with full-size mock catalogues
def test_batch_fullsize_catalogues(pc, olib):
    """Catalogues of the batched workload's sizes (2e5-2e6 clustered points,
    periodic L = 1000) in one batched, graph-replayed float32 call: every
    slice, and every single-catalogue binary64 call, equals the oracle's
    stored histogram, and sampled cross counts of the largest catalogue equal
    the oracle's."""
    import torch
    say("batch full-size catalogues")
    L = 1000.0
    pts = [recipes.batch_cat(k) for k in range(len(recipes.BATCH_SIZES))]
    gold = [golden(f"batch_L1000_c{k}", p) for k, p in enumerate(pts)]
    cols = [tuple(torch.from_numpy(np.ascontiguousarray(p[:, a])).cuda() for a in range(3))
            for p in pts]
    e = synth.log_edges(0.1, 25.0, 20)
    g = {"use_graph": 1}
    for _ in range(2):   # record, then replay
        got, _ = pc.count_rppi_batch(cols, e, 40.0, 40, L, "fp32", options=g)
    assert pc.stats()["replayed"] == 1
    for k, c in enumerate(cols):
        assert (got[k].ravel() == gold[k]["counts"]).all(), k
        one, _ = pc.count_rppi(c, None, e, 40.0, 40, L, "fp64")
        assert (one.ravel() == gold[k]["counts"]).all(), k
    big = pts[0]
    s = big[sample(big.shape[0], NSAMPLE // 2, 18)]
    gx, _ = pc.count_rppi(s, big, e, 40.0, 40, L, "fp32")
    want, _ = oracle.count_rppi(s, big, e, 40.0, 40, L, lib=olib)
    assert (gx == want).all()
