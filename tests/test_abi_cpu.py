"""C-ABI library: loads, exports the header's symbols, host-only planning.
No GPU is touched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1911_03545_amd as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paircount.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:cf_status|const char \*|void)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return pc.load_library()


def test_header_symbols_exported(lib):
    names = header_functions()
    assert len(names) >= 13, names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in paircount.h but not exported"
    assert sorted(names) == sorted(pc.EXPORTED_SYMBOLS)


def test_library_is_gfx950_code_object():
    data = open(pc.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_plan_grid_margin_rule(lib):
    # L / rmax = 10 exactly: the plain floor rule would give width == rmax;
    # the margin forces 9 columns (width 11.11 > 10).
    p = pc.plan_grid(None, None, 100.0, 10.0, 10.0)
    assert p["n"][0] == 9 and p["n"][1] == 9
    assert p["width"][0] > 10.0
    # generic: width always exceeds the reach by the margin
    rng = np.random.default_rng(0)
    for _ in range(200):
        L = rng.uniform(10, 2000)
        r = rng.uniform(L / 200, L / 3.2)
        p = pc.plan_grid(None, None, L, r, r)
        for a in range(2):
            n = p["n"][a]
            assert L / n >= r * (1 + 2 ** -28) + L * 2 ** -40
            assert n >= 3
            # one more column would be too narrow (or hits the cap)
            assert n == 1024 or L / (n + 1) < r * (1 + 2 ** -28) + L * 2 ** -40


def test_plan_grid_zreach_covers_reach(lib):
    rng = np.random.default_rng(1)
    for _ in range(200):
        L = rng.uniform(10, 2000)
        r = rng.uniform(L / 100, L / 3.5)
        spr = int(rng.integers(1, 16))
        p = pc.plan_grid(None, None, L, r, r, spr)
        wz = p["width"][2]
        # zreach slices on each side of any slice must cover a reach of r
        assert p["zreach"] * wz >= r or p["zreach"] == p["n"][2]
        assert p["zreach"] >= 1


def test_plan_grid_unsupported_periodic(lib):
    with pytest.raises(pc.PairCountError) as e:
        pc.plan_grid(None, None, 100.0, 40.0, 40.0)
    assert e.value.status == pc.CF_EUNSUPPORTED
    with pytest.raises(pc.PairCountError):
        pc.plan_grid(None, None, 100.0, 10.0, 34.0)   # pi reach above L/3


def test_plan_grid_rejects_nan_and_inf_box(lib):
    for box in (float("nan"), float("inf")):
        with pytest.raises(pc.PairCountError) as e:
            pc.plan_grid(None, None, box, 10.0, 10.0)
        assert e.value.status == pc.CF_EINVAL
        with pytest.raises(pc.PairCountError) as e:
            pc.plan_grid([0, 0, 0], [50, 50, 50], box, 10.0, 10.0)
        assert e.value.status == pc.CF_EINVAL
    # -inf is a non-positive box: no wrap, bounded by lo/hi
    assert pc.plan_grid([0, 0, 0], [50, 50, 50], float("-inf"), 10.0, 10.0)["periodic"] == 0


def test_plan_grid_nonperiodic(lib):
    p = pc.plan_grid([0, 0, 0], [5, 50, 500], 0.0, 10.0, 10.0)
    assert p["n"][0] == 1 and p["n"][1] == 4
    assert p["periodic"] == 0
    p = pc.plan_grid([1, 1, 1], [1, 1, 1], 0.0, 1.0, 1.0)   # zero extent
    assert p["n"] == [1, 1, 1]


def test_fp32_bands_bracket_edges(lib):
    edges = np.logspace(-1, np.log10(25), 21)
    E = edges * edges
    lo, hi = pc.fp32_bands(E, 3, 420.0)
    assert np.all(lo.astype(np.float64) < E) and np.all(hi.astype(np.float64) > E)
    assert np.all(np.diff(lo) > 0) and np.all(np.diff(hi) > 0)
    # width grows like sqrt(E) * L * 2^-24: a sanity range
    w = (hi.astype(np.float64) - lo.astype(np.float64))
    pred = 2 * 2 * np.sqrt(3) * edges * 6 * 2.0 ** -24 * 420
    assert np.all(w > pred) and np.all(w < 4 * pred + 1e-6)
    lo0, hi0 = pc.fp32_bands(np.array([0.0, 1.0]), 3, 100.0)
    assert lo0[0] == -1 and hi0[0] == -1


def test_fp32_bands_cover_emulated_error(lib):
    """Float32 separations evaluated the way the sweep does (per-axis
    float32 differences of box-frame float32 coordinates, fused multiply-adds
    emulated in binary64) stay inside the band of any edge they straddle."""
    rng = np.random.default_rng(2)
    L = 420.0
    n = 200000
    xi = rng.uniform(0, L, (n, 3))
    d = rng.normal(size=(n, 3))
    d *= (rng.uniform(0.05, 25.0, n) / np.linalg.norm(d, axis=1))[:, None]
    xj = np.mod(xi + d, L)
    # binary64 definition with Code 3's wrap
    dd = xi - xj
    dd = np.where(dd > L / 2, dd - L, dd)
    dd = np.where(dd <= -L / 2, dd + L, dd)
    s64 = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
    # float32 evaluation with the periodic offset per axis
    off = np.where(xi - xj > L / 2, -L, np.where(xi - xj <= -L / 2, L, 0.0)).astype(np.float32)
    A = (xi.astype(np.float32) + off).astype(np.float32)
    d32 = (A - xj.astype(np.float32)).astype(np.float32)
    t = (d32[:, 0].astype(np.float64) ** 2).astype(np.float32)
    t = (d32[:, 1].astype(np.float64) ** 2 + t.astype(np.float64)).astype(np.float32)
    s32 = (d32[:, 2].astype(np.float64) ** 2 + t.astype(np.float64)).astype(np.float32)
    E = np.sort(s64)[:: n // 50]
    lo, hi = pc.fp32_bands(E, 3, L)
    # for every pair and every edge: s32 below lo => s64 < E, above hi => s64 > E
    for k in range(E.size):
        below = s32 < lo[k]
        above = s32 > hi[k]
        assert np.all(s64[below] < E[k])
        assert np.all(s64[above] > E[k])


def test_options_layout_matches_library(lib):
    """The library's cf_default_options fills struct_size with its own
    sizeof(cf_options); the Python mirror must agree, with the output
    pointer last and 8-byte aligned."""
    o = pc.cf_options()
    lib.cf_default_options(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(pc.cf_options)
    assert pc.cf_options.ravg.offset == 64 and ctypes.sizeof(pc.cf_options) == 72
    assert o.weight_type == pc.CF_WEIGHT_PRODUCT and not o.ravg


def test_set_allocator_rejects_null_context(lib):
    """The allocator hook checks its context before touching any device."""
    st = lib.cf_set_allocator(None, pc.ALLOC_FN(), pc.FREE_FN(), None)
    assert st == pc.CF_EINVAL
