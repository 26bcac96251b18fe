"""count_pairs_r_noalloc against count_pairs_r_ex (needs an MI355X).

The no-allocation entry point runs the same pipeline on buffers carved from
the library's fixed per-GPU scratch.  Its counts must equal those of the
ordinary entry point bit for bit (and its weighted sums agree to the
binary64 accumulation bound, 1e-12 relative), on two calls in a row with the
second input smaller than the first (the scratch keeps the first call's
contents), in both precisions, for host and device inputs and outputs; the
context's own buffers must be untouched by it; inputs beyond the fixed
scratch must be rejected with a clear error before any device work.
"""
import numpy as np
import pytest

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


def rel_ok(got, want, rtol=RTOL):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= rtol), (rel.max(), got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_ex_two_calls(pc, prec):
    say("noalloc two calls", prec)
    e = synth.log_edges(0.1, 25.0, 20)
    big = synth.clustered_box(400_000, 420.0, seed=701, nblobs=2000, sigma=2.0)
    small = synth.clustered_box(50_000, 300.0, seed=702, nblobs=250, sigma=2.0)
    for pts, L in ((big, 420.0), (small, 300.0)):
        want, _ = pc.count_r(pts, None, e, L, prec)
        got, _ = pc.count_r_noalloc(pts, None, e, L, prec)
        assert (got == want).all()
        assert want.sum() > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_device_inputs_outputs(pc, prec):
    import torch
    say("noalloc device io", prec)
    e = np.r_[0.0, synth.log_edges(0.1, 20.0, 15)]
    for n, L, seed in ((300_000, 400.0, 703), (20_000, 200.0, 704)):
        pts = synth.clustered_box(n, L, seed=seed, nblobs=n // 200, sigma=2.0)
        w = synth.uniform_weights(n, seed=seed + 100)
        cols = tuple(torch.from_numpy(np.ascontiguousarray(pts[:, k])).cuda() for k in range(3))
        wd = torch.from_numpy(w).cuda()
        want, ww = pc.count_r(cols, None, e, L, prec, w1=wd)
        co = torch.zeros(e.size - 1, dtype=torch.int64, device="cuda")
        wo = torch.zeros(e.size - 1, dtype=torch.float64, device="cuda")
        pc.count_r_noalloc(cols, None, e, L, prec, w1=wd, counts_out=co, wsum_out=wo)
        torch.cuda.synchronize()
        assert (co.cpu().numpy().astype(np.uint64) == want).all()
        rel_ok(wo.cpu().numpy(), ww)


def test_noalloc_cross_open_box_float32_input(pc):
    say("noalloc cross open box")
    e = synth.log_edges(0.2, 15.0, 12)
    a = synth.clustered_box(120_000, 250.0, seed=705, nblobs=600, sigma=2.0).astype(np.float32)
    b = synth.uniform_box(90_000, 250.0, seed=706).astype(np.float32)
    for x, y in ((a, b), (a[:30_000], b[:10_000])):
        for prec in ("fp32", "fp64"):
            want, _ = pc.count_r(x, y, e, 0.0, prec)
            got, _ = pc.count_r_noalloc(x, y, e, 0.0, prec)
            assert (got == want).all()


def test_noalloc_leaves_context_buffers(pc):
    """An ordinary call, a no-allocation call, and the ordinary call again
    (whose repeated shape reuses the context's buffers and work-list
    capacity) all agree."""
    say("noalloc interleaved")
    e = synth.log_edges(0.1, 20.0, 12)
    p = synth.clustered_box(200_000, 350.0, seed=707, nblobs=1000, sigma=2.0)
    q = synth.clustered_box(80_000, 350.0, seed=708, nblobs=400, sigma=2.0)
    first, _ = pc.count_r(p, None, e, 350.0, "fp32")
    mid, _ = pc.count_r_noalloc(q, None, e, 350.0, "fp32")
    again, _ = pc.count_r(p, None, e, 350.0, "fp32")
    assert (first == again).all()
    assert (mid == pc.count_r(q, None, e, 350.0, "fp32")[0]).all()


def test_noalloc_rejects_beyond_scratch(pc):
    import paper_1911_03545_amd as m
    say("noalloc limit")
    e = synth.log_edges(0.1, 10.0, 5)
    # (n, 3) zeros are never read: the size check comes before any device work
    big = np.zeros((2_000_000, 3))
    with pytest.raises(m.PairCountError) as err:
        pc.count_r_noalloc(big, None, e, 100.0, "fp32")
    assert err.value.status == m.CF_EINVAL
    assert "scratch" in str(err.value)
    with pytest.raises(m.PairCountError) as err:
        pc.count_r_noalloc(big[:10], None, e, 100.0, "fp32", options={"use_graph": 1})
    assert err.value.status == m.CF_EINVAL
    # the context still works afterwards
    p = synth.uniform_box(5000, 100.0, seed=709)
    assert (pc.count_r_noalloc(p, None, e, 100.0, "fp64")[0]
            == pc.count_r(p, None, e, 100.0, "fp64")[0]).all()
