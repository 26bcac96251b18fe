"""Write the full-size reference counts in tests/golden/fullsize_*.json.

Every value written here comes from the CPU oracle (``oracle/``, the exactly
pruned variants, which equal the plain brute-force definition bit for bit;
``pin_pruned_equals_plain`` checks that) on inputs drawn by ``synth``.  Each
file records how its input was drawn and the SHA-256 of the drawn arrays, so a
test that draws the input again can prove it counts the same points.

Workloads (the benchmark's configurations):

* ``r_n1e6_L420_{f64,f32}``, ``rppi_n1e6_L420_{f64,f32}``: 10^6 clustered
  points (5000 blobs, sigma 2) in a periodic box of side 420, 20 log bins in
  [0.1, 25]; DD(rp, pi) with pimax 40 in 40 bins; the float32 files count the
  float32 rounding of the same points.
* ``r_w_n4e6_L1100``, ``rppi_w_n4e6_L1100``: 4 x 10^6 clustered points
  (20 000 blobs) in a periodic box of side 1100, float32 weights uniform in
  [0.5, 1.5), 25 log bins in [0.1, 50], pimax 40 in 40 bins; counts and the
  exactly rounded weighted sums.
* ``theta_dd_cap_n2e6``: DD(theta) of 2 x 10^6 clustered RA/DEC points on a
  30-degree cap, 20 log bins in [0.01, 10] degrees; ``theta_dr_cap_n2e6_r5e5``:
  DR(theta) of the same points against the first 5 x 10^5 of the 5 x 10^6
  uniform points on the cap.
* ``batch_L1000_c{0,1,2}``: DD(rp, pi) of the batched workload's catalogue
  sizes 2 x 10^6, 2 x 10^5 and 1.1 x 10^6 (clustered, periodic side 1000).

Usage: ``python tests/golden/make_fullsize.py [name ...]`` (all by default;
about an hour on 8 cores).  Only the oracle and the input generators run.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CITE = ("Code 1 (brute-force pair counts), Code 3 (periodic wrap), Appendix A "
        "(separations, pi bins, angular chords), Appendix B (auto = cross(D, D))")


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ---- input recipes (also used by the GPU tests; synth only) -------------
def box420(dtype):
    p = synth.clustered_box(1_000_000, 420.0, seed=2, nblobs=5000, sigma=2.0)
    return p.astype(dtype)


def box1100():
    p = synth.clustered_box(4_000_000, 1100.0, seed=3, nblobs=20000, sigma=2.0)
    w = synth.uniform_weights(4_000_000, seed=33)
    return p, w


def cap_d():
    return synth.cap_radec(2_000_000, seed=4, clustered=True)


def cap_r(n=500_000):
    ra, dec = synth.cap_radec(5_000_000, seed=40)
    return ra[:n], dec[:n]


BATCH_SIZES = (2_000_000, 200_000, 1_100_000)


def batch_cat(k):
    n = BATCH_SIZES[k]
    return synth.clustered_box(n, 1000.0, seed=5000 + k, nblobs=n // 200, sigma=2.0)


def r_edges():
    return synth.log_edges(0.1, 25.0, 20)


def r_edges_w():
    return synth.log_edges(0.1, 50.0, 25)


def theta_edges():
    return synth.log_edges(0.01, 10.0, 20)


# ---- the reference counts -----------------------------------------------
def job(name):
    """(recipe description, input hash, result dict) of one workload."""
    if name in ("r_n1e6_L420_f64", "r_n1e6_L420_f32", "rppi_n1e6_L420_f64",
                "rppi_n1e6_L420_f32"):
        dtype = np.float64 if name.endswith("f64") else np.float32
        p = box420(dtype)
        e = r_edges()
        recipe = {"input": "clustered_box(1_000_000, 420.0, seed=2, nblobs=5000, sigma=2.0)"
                           + (".astype(float32)" if dtype == np.float32 else ""),
                  "boxsize": 420.0, "edges": e.tolist()}
        if name.startswith("r_"):
            c, _ = oracle.count_r_pruned(p, None, e, 420.0, axis=2)
            res = {"counts": c.tolist()}
        else:
            c, _ = oracle.count_rppi_pruned(p, None, e, 40.0, 40, 420.0, axis=0)
            recipe.update(pimax=40.0, npi=40)
            res = {"counts": c.ravel().tolist()}
        return recipe, sha(p), res
    if name in ("r_w_n4e6_L1100", "rppi_w_n4e6_L1100"):
        p, w = box1100()
        e = r_edges_w()
        recipe = {"input": "clustered_box(4_000_000, 1100.0, seed=3, nblobs=20000, sigma=2.0)",
                  "weights": "uniform_weights(4_000_000, seed=33)",
                  "boxsize": 1100.0, "edges": e.tolist()}
        if name.startswith("r_"):
            c, ws = oracle.count_r_pruned(p, None, e, 1100.0, w1=w, axis=2)
        else:
            c, ws = oracle.count_rppi_pruned(p, None, e, 40.0, 40, 1100.0, w1=w, axis=2)
            recipe.update(pimax=40.0, npi=40)
        res = {"counts": c.ravel().tolist(), "wsum_hex": [float(v).hex() for v in ws.ravel()]}
        return recipe, sha(p, w), res
    if name == "theta_dd_cap_n2e6":
        ra, dec = cap_d()
        e = theta_edges()
        c, _ = oracle.count_theta_pruned(ra, dec, None, None, e, axis=1)
        recipe = {"input": "cap_radec(2_000_000, seed=4, clustered=True)", "edges": e.tolist()}
        return recipe, sha(ra, dec), {"counts": c.tolist()}
    if name == "theta_dr_cap_n2e6_r5e5":
        ra, dec = cap_d()
        ra2, dec2 = cap_r()
        e = theta_edges()
        c, _ = oracle.count_theta_pruned(ra, dec, ra2, dec2, e, axis=1)
        recipe = {"input": "cap_radec(2_000_000, seed=4, clustered=True)",
                  "input2": "cap_radec(5_000_000, seed=40), first 500_000 points",
                  "edges": e.tolist()}
        return recipe, sha(ra, dec, ra2, dec2), {"counts": c.tolist()}
    if name.startswith("batch_L1000_c"):
        k = int(name[-1])
        p = batch_cat(k)
        e = r_edges()
        c, _ = oracle.count_rppi_pruned(p, None, e, 40.0, 40, 1000.0, axis=0)
        recipe = {"input": f"clustered_box({BATCH_SIZES[k]}, 1000.0, seed={5000 + k}, "
                           f"nblobs={BATCH_SIZES[k] // 200}, sigma=2.0)",
                  "boxsize": 1000.0, "edges": e.tolist(), "pimax": 40.0, "npi": 40}
        return recipe, sha(p), {"counts": c.ravel().tolist()}
    raise KeyError(name)


# cheapest first, so that partial runs leave usable files
NAMES = ["batch_L1000_c1", "r_n1e6_L420_f64", "r_n1e6_L420_f32", "rppi_n1e6_L420_f64",
         "rppi_n1e6_L420_f32", "batch_L1000_c2", "batch_L1000_c0", "theta_dr_cap_n2e6_r5e5",
         "theta_dd_cap_n2e6", "rppi_w_n4e6_L1100", "r_w_n4e6_L1100"]


def path_of(name):
    return os.path.join(HERE, f"fullsize_{name}.json")


def main(names):
    for name in names:
        t0 = time.time()
        recipe, digest, res = job(name)
        doc = {"workload": name, "cite": CITE,
               "oracle": "exactly pruned variant of the brute-force oracle",
               "recipe": recipe, "input_sha256": digest, **res,
               "oracle_seconds": round(time.time() - t0, 1)}
        tmp = path_of(name) + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(doc, fh)
        os.replace(tmp, path_of(name))
        print(f"{name}: {doc['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
