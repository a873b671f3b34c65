"""GPU test of the windowed flow-rate convergence flag against the oracle's
rule (oracle/convergence.py): the device flag must rise with exactly the
same recorded sample as the rule applied to the oracle's flow rates.

Q is sampled every obs_every steps at t = 0, obs_every, ... (the state before
that step's collision); with W samples per window the flag rises with the
last sample of the m-th consecutive window whose mean changed by at most eps
relative.  lb_step(t) runs the steps 0 .. t-1, so the flag must still be down
after lb_step up to the converging sample's time t_c and up after one more
step.  Each case is chosen so that no window decision of the oracle lies
within 2 % of the eps threshold (the GPU's Q differs from the oracle's by
~1e-6 relative, far inside that margin)."""
import numpy as np
import pytest

import oracle
import synth
import paper_2003_11069_amd as P
from oracle.convergence import run_to_convergence
from gpu_common import say

pytestmark = pytest.mark.gpu


def _cases():
    pois = synth.poiseuille_2d(nx=8, ny=34, force=1e-6, tau=1.0)
    spec = synth.channel_spec(7, Lx=128, Ly=40)
    drop = synth.channel_2d(spec)
    return {
        "poiseuille_8x34": (pois, dict(obs_every=10, W=50, m=3, eps=1e-3, cap=60000)),
        "droplet_channel_128x40": (drop, dict(obs_every=20, W=25, m=3, eps=2e-3, cap=40000)),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_convergence_flag_matches_oracle_rule(name):
    case, cv = CASES[name]
    say(f"[gpu] convergence flag vs oracle rule: {name} {cv}")
    o = oracle.Oracle(oracle.Params(**{k: v for k, v in case.params.items()
                                       if k in oracle.Params.__dataclass_fields__}))
    o.init_fields(case.rho1, case.rho2, case.u)
    r = run_to_convergence(o, cv["obs_every"], cv["W"], cv["m"], cv["eps"], cv["cap"])
    t_c = r["t_converged"]
    ratios = np.array(r["ratios"])
    say(f"  oracle: converged at t = {t_c} after {len(r['means'])} windows; "
        f"closest decision |ratio - 1| = {np.abs(ratios - 1).min():.3f}")
    assert t_c is not None
    assert np.abs(ratios - 1).min() > 0.02, "a window decision of this case is too close to eps"
    g = P.Lattice(P.Params.from_dict(case.params, obs_every=cv["obs_every"], conv_window=cv["W"],
                                     conv_m=cv["m"], conv_eps=cv["eps"]))
    g.init_fields(case.rho1, case.rho2, case.u)
    g.step(t_c)
    before = g.observables()
    g.step(1)
    after = g.observables()
    say(f"  gpu: flag before t_c {before['converged']}, after {after['converged']}; "
        f"Q_window {after['Q_window']:.9e} oracle {r['means'][-1]:.9e}")
    assert not before["converged"] and after["converged"]
    assert after["Q_window"] == pytest.approx(r["means"][-1], rel=1e-5)
