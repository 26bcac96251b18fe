"""Device scratch from a registered allocator (cf_set_allocator), needs an
MI355X: torch's caching allocator, a recording allocator, a failing one, and
switching back to hipMalloc, each giving the oracle's counts."""
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
def data(olib):
    pts = synth.clustered_box(30000, 100.0, seed=91, nblobs=100)
    e = synth.log_edges(0.1, 12.0, 12)
    want, _ = oracle.count_r(pts, None, e, 100.0, lib=olib)
    return pts, e, want


def test_torch_caching_allocator(data):
    import torch
    import paper_1911_03545_amd as m
    say("torch allocator")
    pts, e, want = data
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    ctx = m.PairCounter(0)
    ctx.use_torch_allocator()
    for prec in ("fp64", "fp32"):
        got, _ = ctx.count_r(pts, None, e, 100.0, prec)
        assert (got == want).all(), prec
    held = torch.cuda.memory_allocated(0) - before
    assert held > 30000 * 40, held          # the gridded arrays at least
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before


def test_recording_and_failing_allocators(data):
    import torch
    import paper_1911_03545_amd as m
    say("recording allocator")
    pts, e, want = data
    live = {}

    def alloc(n):
        t = torch.empty(n + 256, dtype=torch.uint8, device="cuda:0")
        p = (t.data_ptr() + 255) // 256 * 256
        live[p] = t
        return p

    def free(p):
        del live[p]

    ctx = m.PairCounter(0)
    ctx.set_allocator(alloc, free)
    got, _ = ctx.count_r(pts, None, e, 100.0, "fp32")
    assert (got == want).all()
    assert len(live) > 10
    # back to hipMalloc: every recorded buffer is returned first
    ctx.set_allocator(None, None)
    assert not live
    got, _ = ctx.count_r(pts, None, e, 100.0, "fp32")
    assert (got == want).all()
    # an allocator that fails: CF_ENOMEM, and the context stays usable
    ctx.set_allocator(lambda n: 0, lambda p: None)
    with pytest.raises(m.PairCountError) as ex:
        ctx.count_r(pts, None, e, 100.0, "fp32")
    assert ex.value.status == m.CF_ENOMEM
    ctx.set_allocator(alloc, free)
    got, _ = ctx.count_r(pts, None, e, 100.0, "fp32")
    assert (got == want).all()
    ctx.close()
    assert not live
