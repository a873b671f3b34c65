"""Flow-focuser droplet generation on the GPU against the FP64 oracle's
statistics (tests/golden/focuser_stats.json, written by
tests/golden/make_focuser_stats.py from the oracle): over steps
20,000-140,000 the number of main droplets crossing the measuring line, their
median volume V_d, nu and Q_d = nu V_d (Results, Fig. 3), and the mean
dispersed flux through that line.  The flow is laminar and the generation
periodic, so the statistics agree closely although the FP32 and FP64
trajectories are not identical."""
import json
import os

import pytest

from paper_2003_11069_amd import focuser
from gpu_common import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "focuser_stats.json")


def test_generation_statistics_match_the_oracle():
    ref = json.load(open(GOLDEN))
    cfg = ref["config"]
    say("[gpu] flow-focuser 433x98, 140k steps, droplet generation statistics")
    r = focuser.run(scale=cfg["scale"], phi=cfg["phi"], u_c=cfg["u_c"], A_s=cfg["A_s"], N_c=cfg["N_c"],
                    W_out=cfg["W_out"], steps=ref["steps"], t_skip=ref["skip"], every=ref["every"])
    say(f"  gpu: crossings {r['droplets_crossed']} V_d {r['V_d']} nu {r['nu']:.4e} Q_d {r['Q_d']:.4e} "
        f"flux {r['flux_xc_mean']:.5f}; oracle: {ref['crossings']} {ref['V_d']} {ref['nu']:.4e} "
        f"{ref['Q_d']:.4e} {ref['flux_xc_mean']:.5f}; {r['seconds']:.1f} s")
    assert r["x_c"] == ref["x_c"]
    assert abs(r["droplets_crossed"] - ref["crossings"]) <= 1
    assert r["V_d"] == pytest.approx(ref["V_d"], rel=0.05)
    assert r["Q_d"] == pytest.approx(ref["Q_d"], rel=0.1)
    assert r["flux_xc_mean"] == pytest.approx(ref["flux_xc_mean"], rel=0.01)
