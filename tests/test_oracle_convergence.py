"""Pins of the windowed flow-rate convergence rule (oracle/convergence.py),
the steady-state criterion applied to the paper's observable Q (Results,
Fig. 3), against hand-worked sample sequences (no GPU)."""
import pytest

import oracle
import synth
from oracle.convergence import windowed_convergence, run_to_convergence


def _seq(means, spread):
    """Two samples per window, mean +- spread (so a rule that compared single
    samples instead of window means decides differently)."""
    out = []
    for mu in means:
        out += [mu - spread, mu + spread]
    return out


def test_rule_hand_worked():
    # eps = 0.01, W = 2, m = 2.  Window means 1.0, 1.05, 1.055, 1.06:
    # window 1 differs by 0.05 > 0.0105 (reset), window 2 by 0.005 <= 0.01055
    # (1 in a row), window 3 by 0.005 <= 0.0106 (2 in a row): the flag rises
    # with the last sample of window 3, sample index 7.
    r = windowed_convergence(_seq([1.0, 1.05, 1.055, 1.06], 0.2), W=2, m=2, eps=0.01)
    assert r["first"] == 7
    assert r["means"] == pytest.approx([1.0, 1.05, 1.055, 1.06], rel=1e-15)
    assert r["ratios"] == pytest.approx([0.05 / 0.0105, 0.005 / 0.01055, 0.005 / 0.0106], rel=1e-12)


def test_rule_resets_and_needs_m_in_a_row():
    # means 1, 1.001 (in), 1.1 (out: reset), 1.1 (in), 1.1 (in) -> m = 2 reached
    # at window 4: sample 9.  Without the reset it would fire at window 3
    # (sample 7); with "more than m" at window 5.
    r = windowed_convergence(_seq([1.0, 1.001, 1.1, 1.1, 1.1], 0.3), W=2, m=2, eps=0.01)
    assert r["first"] == 9
    # m = 3 is not reached within these five windows
    assert windowed_convergence(_seq([1.0, 1.001, 1.1, 1.1, 1.1], 0.3), W=2, m=3, eps=0.01)["first"] is None
    # the first window is never compared (nothing before it), and an
    # incomplete trailing window is not a window
    assert windowed_convergence([1.0, 1.0, 1.0, 1.0, 1.0], W=2, m=1, eps=0.0)["first"] == 3
    assert windowed_convergence([1.0, 1.0, 1.0], W=2, m=1, eps=0.0)["first"] is None


def test_rule_uses_relative_change():
    # the same absolute change is within eps at a large flow rate and not at
    # a small one
    assert windowed_convergence([100.0, 100.5], W=1, m=1, eps=0.01)["first"] == 1
    assert windowed_convergence([1.0, 1.5], W=1, m=1, eps=0.01)["first"] is None


def test_run_to_convergence_poiseuille():
    """Spin-up of a single-phase channel from rest: Q rises monotonically
    towards the Poiseuille flux, so the rule fires once the window means
    change by less than eps, by then within a few eps of the steady flux."""
    tau, F, ny = 1.0, 1e-6, 34
    case = synth.poiseuille_2d(nx=4, ny=ny, force=F, tau=tau)
    o = oracle.Oracle(oracle.Params(**case.params))
    o.init_fields(case.rho1, case.rho2)
    r = run_to_convergence(o, obs_every=10, W=50, m=3, eps=1e-3, max_steps=60000)
    assert r["t_converged"] is not None and r["t_converged"] % 10 == 0
    assert all(b > a for a, b in zip(r["means"], r["means"][1:]))  # monotone spin-up
    nu = (tau - 0.5) / 3
    q_steady = F * (ny - 2) ** 3 / (12 * nu)
    assert abs(r["means"][-1] - q_steady) <= 0.02 * q_steady
    assert r["ratios"][-1] <= 1 and r["ratios"][-4] > 1  # exactly m = 3 in a row at the end
