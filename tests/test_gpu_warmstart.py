"""GPU test of what the learned warm start gains (steps to a steady flow
rate at equal 1 % flow-rate accuracy), trained and evaluated end to end with
the project's kernels: batched lattice Boltzmann runs generate the data set,
the U-Net trains on the BF16 MFMA forward/backward kernels, and held-out
channels run from the plain start and from the network's prediction.

Workload: 2-D wall-bounded channels 128 x 64 (62 fluid rows) from the
batched-sweep generator with large droplets (R 12..16, so one or two rows of
droplets, a flowing crystal), pressure gradient 3e-5..1e-4 and NCI strength
0.02..0.05 (near-contact number N_c = A h_min / sigma 3.6..9, no
coalescence).  In this regime the steady state is reproducible: the flow
rates of the plain start and of plain starts with a 1e-3 u_ref velocity
perturbation agree to 0.1 %.  (Across the generator's full range, where
droplets coalesce and rearrange, the steady flow rate depends on the start's
history by 1-2 %; there the warm start does not gain at 1 % accuracy.)

Metric (the flow rate is the paper's observable, Results / Fig. 3): Q_ref
is the mean over the plain start and three perturbed plain starts of each
run's mean windowed Q over the second half of 40,000 steps; t_1% is the first
window end (250-step windows) after which the windowed Q stays within 1 % of
Q_ref.  The test asserts the gain measured for the velocity warm start (the
network's predicted velocity field on the actual initial droplets): a lower
median t_1% than the plain start, and faster on most seeds.  The full warm
start (predicted phase and velocity) is reported.  Everything is seeded and
the kernels are deterministic, so the run reproduces exactly."""
import dataclasses
import json
import os

import numpy as np
import pytest

import synth
from paper_2003_11069_amd import warmstart as wsm, ws
from gpu_common import say

pytestmark = pytest.mark.gpu

CRYSTAL = dataclasses.replace(wsm.SMALL, G_range=(3e-5, 1e-4), A_range=(0.02, 0.05), R_range=(12, 16))


def test_warm_start_gain_at_one_percent():
    st = CRYSTAL
    say(f"[gpu] warm start: data set of 256 runs {st.W}x{st.H}")
    X, T, stats, glups, bad = wsm.generate(list(range(1000, 1256)), 40000, 256, say, st)
    assert not bad and len(X) == 256
    net = ws.UNet(ws.UNetConfig(levels=3, base=32, cin=3, cout=3, H=st.H, W=st.W, max_batch=16))
    net.set_params(synth.unet_params(3, 32, seed=0))
    say("[gpu] warm start: training (3 levels, 32 base channels, 60 epochs)")
    tr = wsm.train(net, X, T, epochs=60, batch=16, lr=1e-3, log=lambda m: None)
    say(f"  {tr['steps']} steps, last-batch loss of epochs 1 / 60: {tr['losses'][0]:.3e} / {tr['losses'][-1]:.3e}, "
        f"{tr['tflops']:.1f} TFLOP/s")
    say("[gpu] warm start: 64 held-out seeds, plain / warm / velocity-only / phase-only, 40000 steps")
    ev, _, _ = wsm.evaluate(net, list(range(5000, 5064)), 40000, 256, lambda m: None, st, n_ref=3)
    v = ev["variants"]
    summary = {k: {"t1_median": v[k]["t1"]["median"], "never": v[k]["t1"]["never"],
                   "better": v[k].get("frac_better_than_plain"), "worse": v[k].get("frac_worse_than_plain"),
                   "late_dev": round(v[k]["late_Q_abs_rel_dev_median"], 4)} for k in v}
    say(f"  reference spread (median) {ev['q_ref_spread_median']:.2e}; prediction {ev['prediction']}")
    say("  " + json.dumps(summary))
    os.makedirs("gpurun_out", exist_ok=True)
    with open("gpurun_out/warmstart_crystal_test.json", "w") as f:
        json.dump({"summary": summary, "eval": {k: ev[k] for k in ev if k != "per_seed"}}, f, indent=1)
    assert ev["n"] == 64
    assert ev["q_ref_spread_median"] < 2e-3  # a reproducible steady state
    plain, vel = v["plain"], v["velocity_only"]
    assert vel["t1"]["median"] <= 0.75 * plain["t1"]["median"]
    assert vel["frac_better_than_plain"] >= 0.6 and vel["frac_worse_than_plain"] <= 0.25
