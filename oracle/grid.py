"""Days a payoff expression can read, and the simulated grid (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Sec. 4 assumes a conservative horizon bound HOR; the Futhark backend
(Sec. 6.2) re-indexes the time indices an expression uses so that the
engine only simulates the days the payoff reads.  Here the set of readable
days is computed directly from the semantics of Fig. 3: a node under
enclosing loopifs is evaluated at every shift t0 the iteration can reach.
With the loopif reading (condition and first branch at t0 .. t0+n, second
branch only at t0+n), the reachable shifts of every node form one interval
[lo, hi], which this walk carries down the tree.

Reading taken where the paper is silent: the simulated slots are the
*sorted* unique days > 0 that any ``model`` node reads for a model asset;
day 0 is the spot and days < 0 are flat history (the spot), so neither is
simulated.  Parameter observables are constant in time and need no slot.
"""
from __future__ import annotations

from .il import tsem


def reads(e, delta, t0_lo=0, t0_hi=0):
    """Return (model_days, payoff_days).

    model_days: dict label -> set of days read by ``model`` nodes
    payoff_days: set of days at which ``payoff`` nodes discount
    """
    model_days: dict = {}
    payoff_days: set = set()

    def walk(x, lo, hi):
        k = x[0]
        if k == "model":
            base = tsem(x[2], delta)
            model_days.setdefault(x[1], set()).update(range(base + lo, base + hi + 1))
        elif k == "payoff":
            base = tsem(x[1], delta)
            payoff_days.update(range(base + lo, base + hi + 1))
        elif k == "loopif":
            n = tsem(x[4], delta)
            walk(x[1], lo, hi + n)
            walk(x[2], lo, hi + n)
            walk(x[3], lo + n, hi + n)
        elif k == "if":
            walk(x[1], lo, hi); walk(x[2], lo, hi); walk(x[3], lo, hi)
        elif k == "un":
            walk(x[2], lo, hi)
        elif k == "bin":
            walk(x[2], lo, hi); walk(x[3], lo, hi)

    walk(e, t0_lo, t0_hi)
    return model_days, payoff_days


def slots(e, delta, asset_labels, after=0):
    """Sorted unique days > after read for any model asset (the simulation
    grid; `after` is the last day of a given price history, else 0)."""
    md, _ = reads(e, delta)
    days = set()
    for lab in asset_labels:
        days |= {d for d in md.get(lab, ()) if d > after}
    return sorted(days)


def horizon(e, delta):
    """Largest day any node reads (0 if none)."""
    md, pd = reads(e, delta)
    hi = max(pd) if pd else 0
    for s in md.values():
        if s:
            hi = max(hi, max(s))
    return hi
