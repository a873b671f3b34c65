"""Windowed flow-rate convergence rule ("steady state"), plain Python.

TEST INFRASTRUCTURE ONLY (the test-suite, the smoke check and the benchmark's
CPU-baseline leg); the library never imports it.  It shares no code with the
GPU path.

The paper measures steady flows by their flow rate (Results, Fig. 3) without
stating when a run counts as steady; the rule used throughout is:

* the flow rate Q is sampled every `obs_every` steps, at t = 0, obs_every,
  2 obs_every, ... (sample k is the state at t = k obs_every, before that
  step's collision);
* consecutive samples form windows of W samples; each complete window has a
  mean Q_W;
* from the second window on, a window is "within eps" when
  |Q_W - Q_W(previous)| <= eps |Q_W|;
* the run has converged once m consecutive windows are within eps; the flag
  rises with the last sample of that m-th window and stays up.
"""
from __future__ import annotations

import math


def windowed_convergence(q, W: int, m: int, eps: float) -> dict:
    """Applies the rule to the samples q[0], q[1], ... in order.

    Returns ``first``: the index of the sample with which the flag rises
    (None if it never does); ``means``: the window means; ``ratios``: for
    each window after the first, |Q_W - Q_W(prev)| / (eps |Q_W|) (the
    decision is "within eps" when the ratio is <= 1, so ratios near 1 are
    decisions that rounding could flip).
    """
    if W < 1 or m < 1 or not eps >= 0:
        raise ValueError("need W >= 1, m >= 1, eps >= 0")
    means, ratios = [], []
    consec, first = 0, None
    for k in range(len(q) // W):
        mean = math.fsum(q[k * W:(k + 1) * W]) / W
        if means:
            diff = abs(mean - means[-1])
            lim = eps * abs(mean)
            ratios.append(diff / lim if lim > 0 else (0.0 if diff == 0 else math.inf))
            consec = consec + 1 if diff <= lim else 0
            if consec >= m and first is None:
                first = (k + 1) * W - 1
        means.append(mean)
    return {"first": first, "means": means, "ratios": ratios}


def run_to_convergence(o, obs_every: int, W: int, m: int, eps: float, max_steps: int) -> dict:
    """Steps an ``oracle.Oracle`` from its current state, sampling Q every
    obs_every steps, until the rule's flag rises or max_steps have passed.
    Returns the rule's result plus ``t_converged`` (the time of the sample
    with which the flag rose) and the samples."""
    q, t0 = [], o.t
    while True:
        q.append(o.observables()["Q"])
        r = windowed_convergence(q, W, m, eps)
        if r["first"] is not None or o.t - t0 >= max_steps:
            break
        o.step(obs_every)
    r["q"] = q
    r["t_converged"] = None if r["first"] is None else t0 + r["first"] * obs_every
    return r
