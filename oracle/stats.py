"""Reporting statistics (Sec. 4.3.1): Wilson 95% score interval for k/n."""
import math


def wilson(k, n, z=1.959963984540054):
    """Wilson score interval (lo, hi) for a binomial proportion k/n."""
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    den = 1.0 + z * z / n
    centre = (p + z * z / (2 * n)) / den
    half = z / den * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n))
    return (max(0.0, centre - half), min(1.0, centre + half))


def confusion(pred_escalate, ref_escalate):
    """TP/TN/FP/FN with escalation as the positive class."""
    tp = sum(1 for p, r in zip(pred_escalate, ref_escalate) if p and r)
    tn = sum(1 for p, r in zip(pred_escalate, ref_escalate) if not p and not r)
    fp = sum(1 for p, r in zip(pred_escalate, ref_escalate) if p and not r)
    fn = sum(1 for p, r in zip(pred_escalate, ref_escalate) if not p and r)
    return tp, tn, fp, fn
