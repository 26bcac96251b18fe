"""Reuse of the small per-call uploads (needs an MI355X).

A context keeps the catalogue descriptors and the bin description (with its
lookup table) that its last eager call left on the device, and skips their
copies when the next call's bytes are identical.  This checks, on one
context, that every call in a sequence that changes the bins, the statistic,
the catalogue and the precision, interleaved with graph records and
replays and with no-allocation calls (whose scratch is shared), still
counts exactly what the oracle counts.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_uploads_reused_and_invalidated():
    import paper_1911_03545_amd as m
    olib = oracle.load()
    L = 80.0
    p1 = synth.clustered_box(12000, L, seed=1301, nblobs=60, sigma=1.5)
    p2 = synth.uniform_box(9000, L, seed=1302)
    e1 = synth.log_edges(0.2, 8.0, 12)
    e2 = np.r_[0.0, synth.log_edges(0.5, 7.0, 9)]
    want = {}

    def ref(pts, e, kind):
        key = (id(pts), id(e), kind)
        if key not in want:
            if kind == "r":
                want[key] = oracle.count_r(pts, None, e, L, lib=olib)[0]
            else:
                want[key] = oracle.count_rppi(pts, None, e, 10.0, 10, L, lib=olib)[0]
        return want[key]

    seq = [("r", p1, e1, "fp32", None), ("r", p1, e1, "fp32", None),
           ("r", p1, e2, "fp32", None), ("r", p1, e1, "fp32", None),
           ("r", p2, e1, "fp32", None), ("r", p1, e1, "fp64", None),
           ("rppi", p1, e1, "fp32", None), ("r", p1, e1, "fp32", None),
           ("r", p1, e2, "fp32", {"use_graph": 1}), ("r", p1, e2, "fp32", {"use_graph": 1}),
           ("r", p1, e2, "fp32", {"use_graph": 1}), ("r", p1, e1, "fp32", None),
           ("noalloc", p2, e2, "fp32", None), ("r", p1, e1, "fp32", None),
           ("noalloc", p1, e1, "fp32", None), ("r", p2, e2, "fp32", None),
           ("r", p2, e2, "fp32", None)]
    with m.PairCounter(0) as pc:
        for n, (kind, pts, e, prec, opts) in enumerate(seq):
            say("upload cache step", n, kind, prec, opts)
            if kind == "rppi":
                got, _ = pc.count_rppi(pts, None, e, 10.0, 10, L, prec, options=opts)
                assert (got == ref(pts, e, "rppi")).all(), n
            elif kind == "noalloc":
                got, _ = pc.count_r_noalloc(pts, None, e, L, prec)
                assert (got == ref(pts, e, "r")).all(), n
            else:
                got, _ = pc.count_r(pts, None, e, L, prec, options=opts)
                assert (got == ref(pts, e, "r")).all(), n
