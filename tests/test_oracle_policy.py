"""Pins of the oracle's probe features, rule and guarded ladder
(Sec. 3.4, Eq. trigger, Alg. floor_policy) and of its reporting statistics."""
import numpy as np
import pytest

from conftest import read_table
from oracle import policy, stats

RULE_ROWS = read_table("rule_cases.txt")


@pytest.mark.parametrize("row", RULE_ROWS, ids=[r[4][:40] for r in RULE_ROWS])
def test_rule_on_printed_features(row):
    r50, r100, t_high, expected = float(row[0]), row[1], float(row[2]), int(row[3])
    if r100 == "-":
        assert (r50 >= t_high) == bool(expected)
    else:
        assert policy.rule_fires(r50, float(r100), t_high=t_high) == bool(expected)


def test_rule_boundaries_inclusive():
    assert policy.rule_fires(1e-2, 1e-9)
    assert policy.rule_fires(1e-3, 1e-4 * 1.0) is False          # ratio 0.1
    assert policy.rule_fires(1e-4 / 0.6, 1e-4)                   # ratio exactly 0.6
    assert not policy.rule_fires(1e-3, 9.99e-5)


def test_probe_features_last_available_value():
    hist = np.array([1.0] + list(np.logspace(-1, -7, 30)))   # stops at k=30
    r50, r100 = policy.probe_features(hist, 30)
    assert r50 == r100 == hist[30]
    hist2 = np.logspace(0, -5, 101)
    assert policy.probe_features(hist2, 100) == (hist2[50], hist2[100])


class Mock:
    """Scripted solver: floor -> (iters, outcome, projected eta, true eta)."""

    def __init__(self, table):
        self.table = table
        self.calls = []

    def solve(self, floor):
        self.calls.append(floor)
        it, oc, proj, true = self.table[floor]
        return ("u", floor), it, oc, proj

    def true_eta(self, floor, u):
        assert u == ("u", floor)          # the solve's own iterate, never the probe's
        return self.table[floor][3]


RUNGS = [1e-9, 1e-6, 1e-4, 1e-3]


def test_preserve_then_guard_rejects_false_acceptance():
    m = Mock({1e-9: (85, 0, 8.1e-7, 1.45e-6),      # projected passes, true fails
              1e-6: (30, 0, 9e-7, 7e-7), 1e-4: (20, 0, 5e-7, 4e-7), 1e-3: (10, 0, 5e-7, 4e-7)})
    rung, u, att = policy.guarded_ladder(RUNGS, 0, m.solve, m.true_eta)
    assert rung == 1 and u == ("u", 1e-6)
    assert [a.accepted for a in att] == [False, True]
    assert att[0].proj_eta <= 1e-6 < att[0].true_eta


def test_escalation_skips_original_floor():
    m = Mock({f: (10, 0, 5e-7, 5e-7) for f in RUNGS})
    rung, u, att = policy.guarded_ladder(RUNGS, 1, m.solve, m.true_eta)
    assert rung == 1 and m.calls == [1e-6]


def test_no_admissible_floor():
    m = Mock({f: (200, 1, 1e-3, 1e-3) for f in RUNGS})
    rung, u, att = policy.guarded_ladder(RUNGS, 0, m.solve, m.true_eta)
    assert rung == -1 and u is None and len(att) == 4


def test_select_floor_never_returns_probe_iterate():
    m = Mock({f: (10, 0, 5e-7, 5e-7) for f in RUNGS})
    probe = lambda floor: (np.logspace(0, -1, 101), 100)      # r50 >= 1e-2: escalate
    out = policy.select_floor(RUNGS, probe, m.solve, m.true_eta)
    assert out["k0"] == 1 and out["rung"] == 1 and out["u"] == ("u", 1e-6)


def test_guard_is_inclusive():
    m = Mock({1e-9: (10, 0, 1e-6, 1e-6)})
    rung, _, _ = policy.guarded_ladder(RUNGS[:1], 0, m.solve, m.true_eta, tau=1e-6)
    assert rung == 0


WILSON_ROWS = read_table("wilson_cases.txt")


@pytest.mark.parametrize("row", WILSON_ROWS, ids=[r[5] for r in WILSON_ROWS])
def test_wilson_intervals_printed_in_paper(row):
    k, n = int(row[0]), int(row[1])
    point, lo, hi = float(row[2]), float(row[3]), float(row[4])
    a, b = stats.wilson(k, n)
    assert round(100 * k / n, 1) == point
    assert round(100 * a, 1) == lo and round(100 * b, 1) == hi


def test_confusion_counts_of_heldout_test():
    # TP/TN/FP/FN = 74/24/0/4 with 78 reference escalations
    pred = [1] * 74 + [0] * 24 + [0] * 4
    ref = [1] * 74 + [0] * 24 + [1] * 4
    assert stats.confusion(pred, ref) == (74, 24, 0, 4)


def test_reference_label_is_lowest_rung_passing_the_guard():
    """Reference label (Sec. 4.3.1 held-out reference): independent solves
    from the lowest rung up; the first one whose recomputed residual passes
    is the label, and no rung above it is solved."""
    m = Mock({1e-9: (200, 1, 3e-4, 3e-4), 1e-6: (85, 0, 8e-7, 2e-6),     # cap; projected-only pass
              1e-4: (40, 0, 9e-7, 9.9e-7), 1e-3: (20, 0, 5e-7, 4e-7)})
    assert policy.reference_label(RUNGS, m.solve, m.true_eta) == 2
    assert m.calls == [1e-9, 1e-6, 1e-4]


def test_reference_label_none_and_inclusive():
    m = Mock({f: (200, 1, 1e-3, 1e-3) for f in RUNGS})
    assert policy.reference_label(RUNGS, m.solve, m.true_eta) == -1 and m.calls == RUNGS
    m = Mock({f: (10, 0, 1e-6, 1e-6) for f in RUNGS})
    assert policy.reference_label(RUNGS, m.solve, m.true_eta, tau=1e-6) == 0


@pytest.mark.parametrize("passing", [[], [3], [2, 3], [1, 2, 3], [0, 1, 2, 3], [0, 3], [1, 3]])
def test_reference_label_equals_ladder_from_the_original_floor(passing):
    """The label is the rung the guarded ladder reaches from k0 = 0 (the rule
    quiet), so a rule that never escalates wrongly costs iterations only."""
    table = {f: (10, 0, 5e-7, 5e-7 if k in passing else 5e-6) for k, f in enumerate(RUNGS)}
    lab = policy.reference_label(RUNGS, Mock(table).solve, Mock(table).true_eta)
    m = Mock(table)
    rung, _, _ = policy.guarded_ladder(RUNGS, 0, m.solve, m.true_eta)
    assert lab == rung == (min(passing) if passing else -1)
