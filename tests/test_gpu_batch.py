"""Batched DD(rp, pi): one call over many catalogues (needs an MI355X).

Each catalogue's slice of a batched call must equal the oracle's counts of
that catalogue alone (bit-exact; weighted sums to the oracle's exactly
rounded sums within 1e-12), and the single-catalogue call on the GPU.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

WSUM_RTOL = 1e-12


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


def check_w(got, want):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= WSUM_RTOL), (rel.max(), got, want)


def catalogues(sizes, L, seed):
    return [synth.clustered_box(n, L, seed=seed + k, nblobs=max(1, n // 200), sigma=2.0)
            if n > 0 else np.zeros((0, 3)) for k, n in enumerate(sizes)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [200.0, 0.0])
def test_batch_matches_oracle(pc, olib, prec, box):
    say("batch", prec, box)
    cats = catalogues([3000, 0, 500, 12000, 1, 7000, 64, 65], 200.0, seed=500)
    e = synth.log_edges(0.1, 20.0, 12)
    got, _ = pc.count_rppi_batch(cats, e, 30.0, 15, box, prec)
    assert got.shape == (len(cats), 12, 15)
    for k, p in enumerate(cats):
        want, _ = oracle.count_rppi(p, None, e, 30.0, 15, box, lib=olib)
        assert (got[k] == want).all(), k
        one, _ = pc.count_rppi(p, None, e, 30.0, 15, box, prec)
        assert (got[k] == one).all(), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_weighted_self_pairs(pc, olib, prec):
    """Weighted batch with a zero first edge: each catalogue gets its own
    self-pairs (N_c) and sum of squared weights in bin 0."""
    say("batch weighted", prec)
    cats = catalogues([4000, 2500, 0, 6000], 150.0, seed=600)
    ws = [synth.uniform_weights(p.shape[0], seed=610 + k) for k, p in enumerate(cats)]
    e = np.concatenate([[0.0], synth.log_edges(0.2, 15.0, 10)])
    got, gw = pc.count_rppi_batch(cats, e, 20.0, 10, 150.0, prec, weights=ws)
    for k, p in enumerate(cats):
        want, ww = oracle.count_rppi(p, None, e, 20.0, 10, 150.0, w1=ws[k], lib=olib)
        assert (got[k] == want).all(), k
        check_w(gw[k], ww)


def test_batch_mixed_dtypes_and_devices(pc, olib):
    """float32 and float64 catalogues, host and device memory, in one batch."""
    import torch
    say("batch mixed")
    base = catalogues([5000, 3000, 4000], 120.0, seed=700)
    cats = [base[0].astype(np.float32),
            torch.from_numpy(base[1]).cuda(),
            torch.from_numpy(base[2].astype(np.float32)).cuda()]
    e = synth.log_edges(0.5, 12.0, 8)
    got, _ = pc.count_rppi_batch(cats, e, 12.0, 6, 120.0, "fp32")
    ref = [base[0].astype(np.float32), base[1], base[2].astype(np.float32)]
    for k, p in enumerate(ref):
        want, _ = oracle.count_rppi(p, None, e, 12.0, 6, 120.0, lib=olib)
        assert (got[k] == want).all(), k


def test_batch_many_small(pc, olib):
    """Many catalogues of uneven size (a miniature of the mock-catalogue
    workload): every slice exact, and fp32 == fp64."""
    say("batch many")
    sizes = synth.batch_sizes(40, 0, 3000, seed=5)
    cats = catalogues(list(sizes), 100.0, seed=800)
    e = synth.log_edges(0.1, 10.0, 10)
    g32, _ = pc.count_rppi_batch(cats, e, 15.0, 15, 100.0, "fp32")
    g64, _ = pc.count_rppi_batch(cats, e, 15.0, 15, 100.0, "fp64")
    assert (g32 == g64).all()
    for k in range(0, len(cats), 7):
        want, _ = oracle.count_rppi(cats[k], None, e, 15.0, 15, 100.0, lib=olib)
        assert (g32[k] == want).all(), k


def test_batch_thousands_of_tiny_catalogues(pc, olib):
    """5000 catalogues of 0-60 points (a quarter of them empty, a few with
    one point) in one call, both precisions and as a recorded graph: every
    slice equals the binary64 slice, every tenth the oracle's, and empty or
    single-point catalogues count nothing."""
    import torch
    say("batch 5000 tiny")
    rng = synth.rng_for(811)
    sizes = rng.integers(0, 61, 5000)
    sizes[rng.random(5000) < 0.25] = 0
    sizes[:3] = [1, 0, 1]
    cats = catalogues(list(sizes), 100.0, seed=20000)
    e = synth.log_edges(0.1, 12.0, 6)
    g64, _ = pc.count_rppi_batch(cats, e, 12.0, 6, 100.0, "fp64")
    g32, _ = pc.count_rppi_batch(cats, e, 12.0, 6, 100.0, "fp32")
    assert (g32 == g64).all()
    # device-resident columns, recorded and then replayed
    cols = [tuple(torch.from_numpy(np.ascontiguousarray(c[:, a])).cuda() for a in range(3))
            for c in cats]
    for rep in range(2):
        g32, _ = pc.count_rppi_batch(cols, e, 12.0, 6, 100.0, "fp32", options={"use_graph": 1})
        assert (g32 == g64).all()
    assert pc.stats()["replayed"] == 1
    assert g64.shape == (5000, 6, 6)
    assert not g64[sizes <= 1].any()
    for k in range(0, len(cats), 10):
        want, _ = oracle.count_rppi(cats[k], None, e, 12.0, 6, 100.0, lib=olib)
        assert (g64[k] == want).all(), (k, sizes[k])


def test_batch_errors(pc):
    import paper_1911_03545_amd as m
    say("batch errors")
    e = synth.log_edges(0.1, 10.0, 5)
    with pytest.raises(m.PairCountError):
        pc.count_rppi_batch([], e, 10.0, 5, 100.0, "fp32")
    cats = catalogues([100, 100], 100.0, seed=900)
    with pytest.raises(m.PairCountError):
        pc.count_rppi_batch(cats, e, 10.0, 5, 100.0, "fp32",
                            weights=[np.ones(100), None])
