"""Graph replay of repeated identical calls (needs an MI355X).

With cf_options.use_graph a call records its device work into a HIP graph
and later identical calls (same device buffers, sizes, bins and options)
replay it.  The data in the buffers may change between calls: every replay
is compared with an eager call on the same data, with other eager work in
between, and a replay whose new data needs more work items than the graph
holds must fall back to an eager call.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def olib():
    return oracle.load()


@pytest.fixture(scope="module")
def pc():
    import paper_1911_03545_amd as m
    ctx = m.PairCounter(0)
    yield ctx
    ctx.close()


def fill(cols, pts):
    import torch
    for k in range(3):
        cols[k].copy_(torch.from_numpy(np.ascontiguousarray(pts[:, k])))
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_graph_replay_r(pc, prec):
    import torch
    say("graph r", prec)
    n, L = 30000, 100.0
    cols = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    e = synth.log_edges(0.2, 10.0, 12)
    g = {"use_graph": 1}
    for rep in range(5):
        pts = synth.clustered_box(n, L, seed=40 + rep, nblobs=60)
        fill(cols, pts)
        got, _ = pc.count_r(cols, None, e, L, prec, options=g)
        want, _ = pc.count_r(cols, None, e, L, prec)
        assert (got == want).all(), rep
        # unrelated eager work between replays
        pc.count_r(pts[:500], None, e, L, prec)


def test_graph_replay_batch(pc):
    import torch
    say("graph batch")
    L = 120.0
    sizes = [5000, 2000, 8000, 1]
    cols = [[torch.empty(s, dtype=torch.float64, device="cuda") for _ in range(3)]
            for s in sizes]
    ws = [torch.empty(s, dtype=torch.float64, device="cuda") for s in sizes]
    e = synth.log_edges(0.1, 15.0, 10)
    g = {"use_graph": 1}
    for rep in range(4):
        for k, s in enumerate(sizes):
            fill(cols[k], synth.clustered_box(s, L, seed=100 * rep + k, nblobs=max(1, s // 100)))
            ws[k].copy_(torch.from_numpy(synth.uniform_weights(s, seed=7 * rep + k)
                                         .astype(np.float64)))
        torch.cuda.synchronize()
        got, gw = pc.count_rppi_batch(cols, e, 20.0, 10, L, "fp32", weights=ws, options=g)
        want, ww = pc.count_rppi_batch(cols, e, 20.0, 10, L, "fp32", weights=ws)
        assert (got == want).all(), rep
        den = np.maximum(np.abs(ww), 1e-300)
        assert np.all(np.abs(gw - ww) / den <= 1e-12), rep


def test_graph_item_overflow_falls_back(pc):
    """New data that needs far more work items than the recorded call
    (uniform -> one dense clump) must still give exact counts."""
    import torch
    say("graph overflow")
    n, L = 20000, 100.0
    cols = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    e = synth.log_edges(0.5, 10.0, 8)
    g = {"use_graph": 1}
    fill(cols, synth.uniform_box(n, L, seed=1))
    a, _ = pc.count_r(cols, None, e, L, "fp32", options=g)
    b, _ = pc.count_r(cols, None, e, L, "fp32")
    assert (a == b).all()
    rng = synth.rng_for(2)
    clump = np.clip(50.0 + rng.normal(0.0, 3.0, size=(n, 3)), 0.0, L)
    fill(cols, clump)
    for _ in range(2):
        a, _ = pc.count_r(cols, None, e, L, "fp32", options=g)
        b, _ = pc.count_r(cols, None, e, L, "fp32")
        assert (a == b).all()


def test_graph_switching_calls(pc):
    """Alternating two different graph calls re-records each time and stays
    exact; a host-memory call never records."""
    import torch
    say("graph switching")
    n, L = 15000, 80.0
    pts = synth.uniform_box(n, L, seed=9)
    cols = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).cuda() for k in range(3)]
    e1 = synth.log_edges(0.2, 8.0, 10)
    e2 = synth.log_edges(0.3, 12.0, 6)
    g = {"use_graph": 1}
    w1, _ = pc.count_r(cols, None, e1, L, "fp32")
    w2, _ = pc.count_r(cols, None, e2, L, "fp32")
    for _ in range(3):
        a, _ = pc.count_r(cols, None, e1, L, "fp32", options=g)
        b, _ = pc.count_r(cols, None, e2, L, "fp32", options=g)
        h, _ = pc.count_r(pts, None, e1, L, "fp32", options=g)
        assert (a == w1).all() and (b == w2).all() and (h == w1).all()


def test_autotune_same_counts(pc):
    """Autotuned calls (timing several grids on the live input on the first
    call of a workload class, then reusing the choice) give the same counts,
    also combined with graph replay."""
    import torch
    say("autotune")
    n, L = 40000, 150.0
    pts = synth.clustered_box(n, L, seed=21, nblobs=80)
    cols = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).cuda() for k in range(3)]
    e = synth.log_edges(0.1, 12.0, 10)
    want, _ = pc.count_rppi(cols, None, e, 20.0, 10, L, "fp32")
    for opts in ({"autotune": 1}, {"autotune": 1}, {"autotune": 1, "use_graph": 1},
                 {"autotune": 1, "use_graph": 1}):
        got, _ = pc.count_rppi(cols, None, e, 20.0, 10, L, "fp32", options=opts)
        assert (got == want).all()
        st = pc.stats()
        assert st["slices_per_reach"] in (2, 4, 8, 16, 32)
        assert st["chunk"] in (512, 1024, 2048, 4096, 8192)


def test_repeat_calls_item_overflow(pc, olib):
    """A repeat of the previous call's shape sizes its work list from the
    last call and keeps the count on the device; new data needing far more
    items (uniform -> one dense clump) must be redone and stay exact."""
    say("repeat overflow")
    n, L = 20000, 100.0
    e = synth.log_edges(0.5, 10.0, 8)
    uni = synth.uniform_box(n, L, seed=71)
    a, _ = pc.count_r(uni, None, e, L, "fp32")
    items_uni = pc.stats()["n_items"]
    b, _ = pc.count_r(uni, None, e, L, "fp32")
    assert (a == b).all() and pc.stats()["n_items"] == items_uni
    rng = synth.rng_for(72)
    clump = np.clip(50.0 + rng.normal(0.0, 3.0, size=(n, 3)), 0.0, L)
    want, _ = oracle.count_r(clump, None, e, L, lib=olib)
    for _ in range(2):
        got, _ = pc.count_r(clump, None, e, L, "fp32")
        assert (got == want).all()
        assert pc.stats()["n_items"] > items_uni
