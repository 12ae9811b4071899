"""Probe features, the two-feature rule and the guarded floor ladder.

* Probe (Sec. 3.4): FGMRES at the original floor for at most 100 iterations;
  r50 = eta_{min(50, k_stop)}, r100 = eta_{min(100, k_stop)} taken from the
  recorded residual history (last available value if the probe stops early).
* Rule, Eq. (trigger): escalate iff r50 >= 1e-2 or (r100 >= 1e-4 and
  r100 / r50 >= 0.6).  Comparisons are inclusive.
* Guarded policy, Alg. (floor_policy): candidates are the ladder if the rule
  fires, else the original floor followed by the ladder; each candidate is
  solved independently (the probe iterate is never reused) and accepted only
  if the recomputed true residual is <= tau.  If no candidate passes, the
  answer is "no admissible floor in the tested ladder".

Rung convention: ``rungs`` is the ordered list whose first entry is the
original floor rho_0 (e.g. [1e-9, 1e-6, 1e-4, 1e-3]); the rule maps to a first
rung index k0 = 1 if it fires, else 0, and the ladder climbs from k0.
"""
import numpy as np


def probe_features(hist, k_stop):
    """(r50, r100) from a probe history hist[0..k_stop]."""
    r50 = float(hist[min(50, k_stop)])
    r100 = float(hist[min(100, k_stop)])
    return r50, r100


def rule_fires(r50, r100, t_high=1e-2, t_plateau=1e-4, t_ratio=0.6):
    """Eq. (trigger)."""
    return bool(r50 >= t_high or (r100 >= t_plateau and r100 / r50 >= t_ratio))


def first_rung(r50, r100, **thresholds):
    return 1 if rule_fires(r50, r100, **thresholds) else 0


class Attempt:
    def __init__(self, rung, floor, iters, outcome, proj_eta, true_eta, accepted):
        self.rung, self.floor, self.iters = rung, floor, iters
        self.outcome, self.proj_eta, self.true_eta = outcome, proj_eta, true_eta
        self.accepted = accepted


def guarded_ladder(rungs, k0, solve, true_eta, tau=1e-6):
    """Alg. (floor_policy) after the probe: climb rungs[k0:].

    solve(floor) -> (u, iters, outcome, proj_eta);  true_eta(floor, u) -> eta.
    Returns (accepted rung index or -1, u or None, attempts)."""
    attempts = []
    for r in range(k0, len(rungs)):
        u, iters, outcome, proj = solve(rungs[r])
        eta = true_eta(rungs[r], u)
        ok = bool(eta <= tau)
        attempts.append(Attempt(r, rungs[r], iters, outcome, proj, eta, ok))
        if ok:
            return r, u, attempts
    return -1, None, attempts


def select_floor(rungs, probe, solve, true_eta, tau=1e-6, selector=None):
    """Probe -> first rung (rule, or ``selector(r50, r100)``) -> guarded ladder."""
    hist, k_stop = probe(rungs[0])
    r50, r100 = probe_features(hist, k_stop)
    k0 = selector(r50, r100) if selector is not None else first_rung(r50, r100)
    rung, u, attempts = guarded_ladder(rungs, k0, solve, true_eta, tau)
    return dict(r50=r50, r100=r100, k_stop=k_stop, k0=k0, rung=rung, u=u,
                attempts=attempts)


def reference_label(rungs, solve, true_eta, tau=1e-6):
    """Lowest rung whose independent full solve passes the guard (-1 if none)."""
    for r, fl in enumerate(rungs):
        u, _, _, _ = solve(fl)
        if true_eta(fl, u) <= tau:
            return r
    return -1
