"""Seeded random configurations of every statistic and option against the
oracle (needs an MI355X).

Each case draws a statistic (DD(r), DD(rp, pi), DD(theta), on-sky DD(rp,
pi), batched DD(rp, pi)), auto or cross, periodic or not, float32 or
float64 inputs on the host or the device, weights (product or sum), the mean
separation, precision, slices per reach, work-item chunk, x/y or angular
refinement, the float32 separation form, RA/DEC input converted on the host or
unit vectors, and bin edges (log, linear, with e0 = 0 or not), with sizes the
oracle counts in well under a second.  Counts must equal the oracle's bit for
bit; weighted sums within 1e-12 relative; mean separations within 1e-9
relative in binary64, and in float32 within the bound 10u C + 8u r of the
float32 evaluation's separations (u = 2^-24, C the coordinate scale).  The
case seed and parameters are printed before each call.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

NCASES = 400
U32 = 2.0 ** -24
R2D = 180.0 / np.pi


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


def rel_ok(got, want, rtol):
    den = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(got - want) / den
    rel[(want == 0) & (got == 0)] = 0
    assert np.all(rel <= rtol), (rel.max(), got, want)


def check_mean(got, want, f32, C, angle=False):
    if not f32:
        rel_ok(got, want, 1e-9)
        return
    if angle:
        tol = (10 * U32 * C + 8 * U32 * np.radians(want)) * 1.01 * R2D + 4 * U32 * want
    else:
        tol = 10 * U32 * C + 8 * U32 * want
    err = np.abs(got - want)
    assert np.all(err <= tol), (err.max(), (err / np.maximum(tol, 1e-300)).max())


def edges_for(rng, lo, hi, nb):
    kind = rng.integers(0, 3)
    if kind == 0:
        e = synth.log_edges(lo, hi, nb)
    elif kind == 1:
        e = np.linspace(lo, hi, nb + 1)
    else:
        e = np.r_[0.0, synth.log_edges(lo, hi, nb - 1)]
    return e


def maybe_device(rng, a):
    """The array itself, a float32 copy, or a torch tensor on the GPU."""
    import torch
    k = rng.integers(0, 3)
    if k == 1:
        return a.astype(np.float32)
    if k == 2:
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return a


def on_device_like(pts, w):
    if w is None or not hasattr(pts, "cpu"):
        return w
    import torch
    return torch.from_numpy(np.ascontiguousarray(w)).to("cuda:0")


def host64(a):
    if hasattr(a, "cpu"):
        return a.cpu().numpy().astype(np.float64)
    return np.asarray(a, dtype=np.float64)


def options_for(rng, stat):
    o = {}
    if rng.random() < 0.5:
        o["slices_per_reach"] = int(rng.choice([1, 3, 8, 16, 32, 64]))
    if rng.random() < 0.5:
        o["chunk"] = int(rng.choice([64, 300, 1024, 4096]))
    if stat in ("r", "rppi", "mocks") and rng.random() < 0.5:
        o["xy_refine"] = int(rng.integers(1, 5))
    if stat == "theta":
        o["angular_grid"] = int(rng.choice([-1, 0, 1, 2, 8, 16, 32]))
    return o


@pytest.mark.parametrize("case", range(NCASES))
def test_random_config(pc, olib, case):
    rng = synth.rng_for(7000 + case)
    stat = ["r", "rppi", "theta", "mocks", "batch"][case % 5]
    auto = bool(rng.random() < 0.6) or stat == "batch"
    weighted = bool(rng.random() < 0.4)
    wtype = str(rng.choice(["product", "sum"])) if weighted else None
    ravg = bool(rng.random() < 0.3)
    prec = str(rng.choice(["fp64", "fp32"]))
    opts = options_for(rng, stat)
    # the float32 separation form (drawn from a stream of its own, so that
    # every other draw of the case stays as it was)
    form = int(synth.rng_for(9100 + case).integers(0, 3))
    if form:
        opts["separation_form"] = form
    n1 = int(rng.integers(0, 6000)) if rng.random() < 0.1 else int(rng.integers(500, 12000))
    n2 = int(rng.integers(300, 9000))
    say(f"case {case}: {stat} auto={auto} w={wtype} ravg={ravg} {prec} n1={n1} n2={n2} {opts}")
    scale = 2.0                      # coordinate scale of the float32 evaluation
    f32 = prec == "fp32" and stat != "mocks"   # on-sky pairs always run in binary64
    kw = {"weight_type": wtype} if weighted else {}
    if stat in ("r", "rppi"):
        L = float(rng.uniform(50.0, 200.0))
        periodic = bool(rng.random() < 0.6)
        box = L if periodic else 0.0
        a = synth.clustered_box(n1, L, seed=int(rng.integers(1 << 30)), nblobs=50, sigma=1.5)
        b = None if auto else synth.uniform_box(n2, L, seed=int(rng.integers(1 << 30)))
        w1 = synth.uniform_weights(n1, seed=int(rng.integers(1 << 30))) if weighted else None
        w2 = None if (auto or not weighted) else synth.uniform_weights(
            n2, seed=int(rng.integers(1 << 30)))
        scale = L
        rmax = float(rng.uniform(2.0, L / 3.2))
        e = edges_for(rng, rmax / 200.0, rmax, int(rng.integers(1, 25)))
        da = maybe_device(rng, a)
        db = None if b is None else maybe_device(rng, b)
        ha, hb = host64(da), (None if db is None else host64(db))
        # weights live where their catalogue's coordinates live
        dw1 = on_device_like(da, w1)
        dw2 = on_device_like(db, w2)
        if stat == "r":
            got = pc.count_r(da, db, e, box, prec, w1=dw1, w2=dw2, options=opts, ravg=ravg,
                             **kw)
            want = oracle.count_r(ha, hb, e, box, w1=w1, w2=w2, lib=olib, ravg=ravg,
                                  weight_type=wtype or "product")
        else:
            pimax = float(rng.uniform(1.0, L / 3.2))
            npi = int(rng.integers(1, 60))
            if ravg:   # the library's limit on bins with the mean separation
                npi = min(npi, 1365 // (e.size - 1))
            got = pc.count_rppi(da, db, e, pimax, npi, box, prec, w1=dw1, w2=dw2,
                                options=opts, ravg=ravg, **kw)
            want = oracle.count_rppi(ha, hb, e, pimax, npi, box, w1=w1, w2=w2, lib=olib,
                                     ravg=ravg, weight_type=wtype or "product")
    elif stat == "theta":
        radius = float(rng.uniform(2.0, 60.0))
        ra, dec = synth.cap_radec(n1, seed=int(rng.integers(1 << 30)), radius_deg=radius,
                                  ra0_deg=float(rng.uniform(0, 360)),
                                  dec0_deg=float(rng.uniform(-90, 90)), clustered=True,
                                  nblobs=50, sigma_deg=radius / 50)
        r2 = d2 = None
        if not auto:
            r2, d2 = synth.cap_radec(n2, seed=int(rng.integers(1 << 30)), radius_deg=radius)
        w1 = synth.uniform_weights(n1, seed=int(rng.integers(1 << 30))) if weighted else None
        w2 = None if (auto or not weighted) else synth.uniform_weights(
            n2, seed=int(rng.integers(1 << 30)))
        tmax = float(rng.uniform(0.05, min(2.0 * radius, 180.0)))
        te = edges_for(rng, tmax / 300.0, tmax, int(rng.integers(1, 25)))
        # unit vectors from the oracle's own conversion: exact parity
        v1 = oracle.radec_to_unit(ra, dec, lib=olib)
        v2 = None if auto else oracle.radec_to_unit(r2, d2, lib=olib)
        grid = opts.pop("angular_grid")
        if rng.random() < 0.5:
            # RA/DEC converted on the host (the default) with the oracle's
            # library
            got = pc.count_theta(ra, dec, r2, d2, te, prec, w1=w1, w2=w2, options=opts,
                                 ravg=ravg, angular_grid=grid, **kw)
        else:
            got = pc.count_theta(None, None, theta_edges_deg=te, precision=prec, w1=w1, w2=w2,
                                 unit_vectors=(v1, v2), options=opts, ravg=ravg,
                                 angular_grid=grid, **kw)
        want = oracle.count_theta(ra, dec, r2, d2, te, w1=w1, w2=w2, lib=olib, ravg=ravg,
                                  weight_type=wtype or "product")
    elif stat == "mocks":
        radius = float(rng.uniform(2.0, 8.0))
        m1 = synth.sky_mock(n1, seed=int(rng.integers(1 << 30)), radius_deg=radius,
                            dmin=300.0, dmax=600.0)
        v1 = oracle.sky_to_cartesian(m1[:, 0], m1[:, 1], m1[:, 2], lib=olib)
        v2 = None
        if not auto:
            m2 = synth.sky_mock(n2, seed=int(rng.integers(1 << 30)), radius_deg=radius,
                                dmin=300.0, dmax=600.0, clustered=False)
            v2 = oracle.sky_to_cartesian(m2[:, 0], m2[:, 1], m2[:, 2], lib=olib)
        w1 = synth.uniform_weights(n1, seed=int(rng.integers(1 << 30))) if weighted else None
        w2 = None if (auto or not weighted) else synth.uniform_weights(
            n2, seed=int(rng.integers(1 << 30)))
        e = edges_for(rng, 0.1, float(rng.uniform(5.0, 25.0)), int(rng.integers(1, 20)))
        pimax = float(rng.uniform(5.0, 40.0))
        npi = int(rng.integers(1, 40))
        if rng.random() < 0.5:
            got = pc.count_rppi_mocks(m1, None if auto else m2, e, pimax, npi, prec, w1=w1,
                                      w2=w2, options=opts, ravg=ravg, **kw)
        else:
            got = pc.count_rppi_mocks(v1, v2, e, pimax, npi, prec, w1=w1, w2=w2, options=opts,
                                      ravg=ravg, cartesian=True, **kw)
        want = oracle.count_rppi_mocks(v1, v2, e, pimax, npi, w1=w1, w2=w2, lib=olib,
                                       ravg=ravg, weight_type=wtype or "product")
    else:
        ncat = int(rng.integers(1, 9))
        L = float(rng.uniform(60.0, 200.0))
        scale = L
        cats = [synth.clustered_box(int(rng.integers(0, 4000)), L,
                                    seed=int(rng.integers(1 << 30)), nblobs=20)
                for _ in range(ncat)]
        ws = [synth.uniform_weights(c.shape[0], seed=int(rng.integers(1 << 30)))
              for c in cats] if weighted else None
        e = edges_for(rng, 0.2, float(rng.uniform(3.0, L / 3.5)), int(rng.integers(1, 15)))
        pimax = float(rng.uniform(2.0, L / 3.5))
        npi = int(rng.integers(1, 30))
        got = pc.count_rppi_batch(cats, e, pimax, npi, L, prec, weights=ws, options=opts,
                                  ravg=ravg, **kw)
        outs = [oracle.count_rppi(c, None, e, pimax, npi, L, w1=(ws[k] if ws else None),
                                  lib=olib, ravg=ravg, weight_type=wtype or "product")
                for k, c in enumerate(cats)]
        want = tuple(None if outs[0][i] is None else np.stack([o[i] for o in outs])
                     for i in range(len(outs[0])))
    assert (got[0] == want[0]).all(), (got[0], want[0])
    if weighted:
        rel_ok(got[1], want[1], 1e-12)
    if ravg:
        check_mean(got[2], want[2], f32, scale, angle=(stat == "theta"))
