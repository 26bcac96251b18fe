"""The CPU oracle against its pins (no GPU needed)."""
import numpy as np
import pytest

import oracle
import synth
from oracle_pins import ALL_PINS


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin, lib):
    pin(lib)


def test_numpy_cross_check_no_fma(lib):
    """A vectorised NumPy evaluation of the same separations (one rounding per
    operation, no fused multiply-add) gives identical counts on random,
    non-lattice inputs; a contracted multiply-add in the oracle would move
    pairs across edges."""
    pts = synth.clustered_box(900, 30.0, seed=5, nblobs=40, sigma=0.7)
    edges = synth.log_edges(0.05, 9.0, 14)
    L = 30.0
    d = pts[:, None, :] - pts[None, :, :]
    d = np.where(d > 0.5 * L, d - L, d)
    d = np.where(d <= -0.5 * L, d + L, d)
    s = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    E = edges * edges
    k = np.searchsorted(E, s.ravel(), side="right") - 1
    k = k[(s.ravel() >= E[0]) & (s.ravel() < E[-1])]
    want = np.bincount(k, minlength=edges.size - 1)
    got, _ = oracle.count_r(pts, None, edges, L, lib=lib)
    assert (got == want).all()


def test_thread_count_invariance(lib):
    pts = synth.clustered_box(1500, 80.0, seed=6, nblobs=30, sigma=2.0)
    w = synth.uniform_weights(1500, seed=7)
    edges = synth.log_edges(0.1, 20.0, 12)
    a = oracle.count_r(pts, None, edges, 80.0, w1=w, nthreads=1, lib=lib)
    b = oracle.count_r(pts, None, edges, 80.0, w1=w, nthreads=4, lib=lib)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


def test_float32_promotion(lib):
    """float32 inputs are widened exactly: counting the float32 array equals
    counting its explicit float64 copy."""
    pts = synth.clustered_box(800, 50.0, seed=8, nblobs=30).astype(np.float32)
    edges = synth.log_edges(0.1, 10.0, 10)
    a, _ = oracle.count_r(pts, None, edges, 50.0, lib=lib)
    b, _ = oracle.count_r(pts.astype(np.float64), None, edges, 50.0, lib=lib)
    assert (a == b).all()


def test_invalid_arguments(lib):
    pts = synth.uniform_box(10, 10.0, seed=9)
    with pytest.raises(oracle.OracleError):
        oracle.count_r(pts, None, [1.0, 0.5], 10.0, lib=lib)
    with pytest.raises(oracle.OracleError):
        oracle.count_r(pts, None, [-1.0, 0.5], 10.0, lib=lib)
    with pytest.raises(oracle.OracleError):
        oracle.count_rppi(pts, None, [0.1, 1.0], -1.0, 4, 10.0, lib=lib)
    with pytest.raises(oracle.OracleError):
        oracle.count_theta([0.0, 400.0], [0.0, 0.0], None, None, [0.1, 1.0], lib=lib)


def test_empty_inputs(lib):
    e = np.zeros((0, 3))
    c, _ = oracle.count_r(e, None, [0.0, 1.0], 10.0, lib=lib)
    assert c.tolist() == [0]
    one = np.array([[1.0, 2.0, 3.0]])
    c, _ = oracle.count_r(one, None, [0.0, 1.0], 10.0, lib=lib)
    assert c.tolist() == [1]
    c, _ = oracle.count_r(one, None, [0.5, 1.0], 10.0, lib=lib)
    assert c.tolist() == [0]
