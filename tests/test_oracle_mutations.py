"""Each plausible mistake planted into a copy of the oracle must be caught by
at least one pin.  Mistakes are planted in the oracle source on the CPU only."""
import json
import os
import subprocess
import sys

import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "paircount_oracle.c")

# (name, exact text in the oracle, replacement)
MUTATIONS = [
    ("dropped_z_term", "s = (dx * dx + dy * dy) + dz * dz;", "s = (dx * dx + dy * dy);"),
    ("wrong_sign_dy", "double dy = yi - y2[j];", "double dy = yi + y2[j];"),
    ("wrong_array_z", "double dz = zi - z2[j];", "double dz = zi - y2[j];"),
    ("bottom_edge_exclusive", "if (s < E[0] || s >= E[nbins])\n                            continue;\n                        int k",
     "if (s <= E[0] || s >= E[nbins])\n                            continue;\n                        int k"),
    ("wrap_positive_side_missing", "if (d > half)", "if (d > L)"),
    ("wrap_wrong_direction", "d -= L;", "d += L;"),
    ("edge_inclusive_upper", "while (s < E[k])\n                            k--;\n                        bin = k;",
     "while (s <= E[k] && k > 0)\n                            k--;\n                        bin = k;"),
    ("top_edge_inclusive", "if (s < E[0] || s >= E[nbins])\n                            continue;\n                        int k",
     "if (s < E[0] || s > E[nbins])\n                            continue;\n                        int k"),
    ("unsquared_edges", "E[k] = edges[k] * edges[k];", "E[k] = edges[k];"),
    ("no_self_pairs", "counts[0] += (uint64_t)n1;", ""),
    ("no_doubling", "counts[b] *= 2u;", ""),
    ("auto_includes_diagonal", "autocorr ? i + 1 : 0", "autocorr ? i : 0"),
    ("pi_cut_inclusive", "pi >= pimax", "pi > pimax"),
    ("pi_bin_off_by_one", "while (pi < q[p])", "while (pi <= q[p] && p > 0)"),
    ("rp_uses_dz", "s = dx * dx + dy * dy;\n                            pi = fabs(dz);",
     "s = dx * dx + dz * dz;\n                            pi = fabs(dz);"),
    ("chord_not_halved", "2.0 * sin(0.5 * (theta_deg[k] * d2r))", "2.0 * sin(theta_deg[k] * d2r)"),
    ("radec_swapped_trig", "x[i] = cd * cos(a);", "x[i] = cd * sin(a);"),
    ("xsum_no_compensation", "double lo = y - (hi - x);", "double lo = 0.0 * (y - (hi - x));"),
    ("weight_transposed", "prod = pair_weight(wtype, w1[i], w2[j]);", "prod = pair_weight(wtype, w1[i], w1[j]);"),
    ("weights_not_doubled", "autocorr ? 2.0 * prod : prod", "prod"),
    ("self_weight_missing", "xacc_add(&total[0], pair_weight(wtype, w1[i], w1[i]));", "(void)0;"),
    ("self_weight_always_product", "xacc_add(&total[0], pair_weight(wtype, w1[i], w1[i]));",
     "xacc_add(&total[0], w1[i] * w1[i]);"),
    ("sum_weight_is_product", "return wtype == 1 ? a + b : a * b;", "return a * b;"),
    ("ravg_of_squared_separation", "const double c = sqrt(s);", "const double c = s;"),
    ("ravg_not_doubled", "xacc_add(&racc[bin], autocorr ? 2.0 * rw : rw);",
     "xacc_add(&racc[bin], rw);"),
    ("ravg_unweighted_numerator", "const double rw = separation_value(angle, s) * prod;",
     "const double rw = separation_value(angle, s);"),
    ("ravg_divides_by_count", "weighted ? xacc_value(&total[b]) : (double)counts[b]",
     "(double)counts[b]"),
    ("theta_mean_in_radians", "return (2.0 * asin(0.5 * c)) * (180.0 / M_PI);",
     "return 2.0 * asin(0.5 * c);"),
    ("mocks_pi_signed", "pi = ll > 0.0 ? fabs(sl) / sqrt(ll) : 0.0;",
     "pi = ll > 0.0 ? sl / sqrt(ll) : 0.0;"),
    ("mocks_los_from_difference", "const double lx = xi + x2[j], ly = yi + y2[j], lz = zi + z2[j];",
     "const double lx = xi - x2[j], ly = yi - y2[j], lz = zi - z2[j];"),
    ("mocks_pi_unnormalised", "fabs(sl) / sqrt(ll)", "fabs(sl) / ll"),
    ("mocks_rp_adds_pi", "s = fmax(ss - pi * pi, 0.0);", "s = fmax(ss + pi * pi, 0.0);"),
    ("mocks_sl_drops_z", "const double sl = (dx * lx + dy * ly) + dz * lz;",
     "const double sl = (dx * lx + dy * ly);"),
    ("mocks_ll_drops_y", "const double ll = (lx * lx + ly * ly) + lz * lz;",
     "const double ll = (lx * lx) + lz * lz;"),
    ("sky_distance_ignored", "x[i] = dist[i] * x[i];", "x[i] = x[i];"),
    ("pi_edges_rounded_once", "q[p] = (double)p * dpi;", "q[p] = (double)p * pimax / (double)npi;"),
    ("pi_top_edge_from_width", "q[npi] = pimax;", "q[npi] = (double)npi * dpi;"),
    ("prune_no_periodic_images", "const int nimg = L > 0.0 ? 3 : 1;", "const int nimg = 1;"),
    ("prune_half_reach", "(ki + shift[m]) + reach)", "(ki + shift[m]) + 0.5 * reach)"),
    ("prune_pi_reach_on_every_axis", "(mode == 1 && axis == 2) ? q[npi]", "(mode == 1) ? q[npi]"),
    ("prune_key_of_wrong_axis", "order[i].key = cols[axis][i];",
     "order[i].key = cols[(axis + 1) % 3][i];"),
    ("theta_mean_half_angle", "return (2.0 * asin(0.5 * c)) * (180.0 / M_PI);",
     "return asin(0.5 * c) * (180.0 / M_PI);"),
]


# Runs every pin against a mutated library in a child process: a planted
# mistake can make the oracle index outside its arrays, which must not take
# the test process down.  The child prints the names of the pins that fail.
_CHILD = """
import json, sys
sys.path[:0] = {paths!r}
import oracle
from oracle_pins import ALL_PINS
lib = oracle.load({so!r}, rebuild_if_missing=False)
print("PINS-START", len(ALL_PINS), flush=True)
failures = []
for pin in ALL_PINS:
    try:
        pin(lib)
    except AssertionError:
        failures.append(pin.__name__)
    except oracle.OracleError:
        failures.append(pin.__name__ + "(error)")
print(json.dumps(failures))
"""


def _run_pins(src_text, tmp_path):
    """Build `src_text` as an oracle library and run every pin against it in
    a child process.  Returns the list of failing pins, or ["<signal N>"] when
    the child died from a signal after the pins started (a planted mistake
    that makes the oracle index outside its arrays).  Any other abnormal exit
    (an import error, a pin that raises something unexpected, a child that
    never reached the pins) fails the test: it would prove nothing."""
    path = tmp_path / "mut.c"
    path.write_text(src_text)
    so = str(tmp_path / "libmut.so")
    oracle.build(src=str(path), out=so)
    here = os.path.dirname(os.path.abspath(__file__))
    paths = [here, os.path.dirname(here)]
    r = subprocess.run([sys.executable, "-c", _CHILD.format(paths=paths, so=so)],
                       capture_output=True, text=True, timeout=600)
    lines = r.stdout.strip().splitlines()
    started = any(line.startswith("PINS-START") for line in lines)
    assert started, ("child never started the pins", r.returncode, r.stderr[-2000:])
    if r.returncode < 0:
        return [f"<signal {-r.returncode}>"]
    assert r.returncode == 0, ("child failed outside the pins", r.returncode,
                               r.stderr[-2000:])
    return json.loads(lines[-1])


@pytest.mark.slow
def test_unmutated_oracle_passes_every_pin(tmp_path):
    """Control: the harness run on the oracle as committed reports no failing
    pin, so a failure reported for a mutant comes from its planted mistake."""
    src = open(SRC).read()
    assert _run_pins(src, tmp_path) == []


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation {name}: pattern not found"
    failures = _run_pins(src.replace(old, new, 1), tmp_path)
    print(name, "caught by", failures)
    assert failures, f"planted mistake {name} was not caught by any pin"
