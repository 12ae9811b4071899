"""The bench's held-out policy statistics (CPU only): Wilson intervals against
the values the paper prints (Sec. 4.3.1, tests/golden/wilson_cases.txt) and the
confusion / guard / margin bookkeeping on a hand-made run."""
import os

import pytest

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "wilson_cases.txt")


def _rows():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, n, _, lo, hi = line.split()[:5]
            rows.append((int(k), int(n), float(lo), float(hi)))
    return rows


@pytest.mark.parametrize("k,n,lo,hi", _rows())
def test_wilson_matches_printed_intervals(k, n, lo, hi):
    a, b = bench.wilson(k, n)
    assert round(100 * a, 1) == lo and round(100 * b, 1) == hi


def _att(rung, outcome, eta, accepted, its=50):
    return dict(rung=rung, outcome=outcome, true_eta=eta, accepted=accepted, iterations=its)


def test_policy_stats_bookkeeping():
    tau = 1e-6
    outs = [
        # predicted preserve, admissible: kept at rung 0 with 170 of 200 iterations
        dict(k0=0, rung=0, attempts=[_att(0, "PROJ_CONVERGED", 5e-7, True, 170)]),
        # predicted preserve, not admissible: projected convergence rejected, fallback to rung 1
        dict(k0=0, rung=1, attempts=[_att(0, "PROJ_CONVERGED", 3e-6, False),
                                     _att(1, "PROJ_CONVERGED", 4e-7, True)]),
        # predicted escalation, reference escalation
        dict(k0=2, rung=2, attempts=[_att(2, "PROJ_CONVERGED", 1e-7, True)]),
        # predicted escalation, but the original floor was admissible
        dict(k0=1, rung=1, attempts=[_att(1, "PROJ_CONVERGED", 2e-7, True)]),
        # nothing admissible
        dict(k0=3, rung=-1, attempts=[_att(3, "MAXIT", 2e-3, False, 200)]),
    ]
    labels = [0, 1, 2, 0, -1]
    st = bench.policy_stats(outs, labels, tau=tau, cap=200)
    assert st["reference"] == {"escalate": 3, "preserve": 2, "none_admissible": 1}
    assert st["confusion"] == {"TP": 2, "TN": 1, "FP": 1, "FN": 1}
    assert (st["sensitivity"]["k"], st["sensitivity"]["n"]) == (2, 3)
    assert (st["specificity"]["k"], st["specificity"]["n"]) == (1, 2)
    assert st["guard_fallbacks"] == 1
    assert (st["selected_meet_tolerance"]["k"], st["selected_meet_tolerance"]["n"]) == (4, 5)
    assert st["lowest_admissible_selected"] == 4
    assert st["projected_converged_rejected_by_guard"] == 1
    assert st["accepted_above_tolerance"] == 0
    assert st["preserve_margin"] == {"preserved": 1, "cap": 200, "max_iterations": 170, "at_least_80pct_of_cap": 1}
