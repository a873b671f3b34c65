"""Writes tests/golden/channel3d_long.json: the FP64 oracle's flow rates over
a long run of the 3-D droplet channel (synth.hex_channel_3d(): D3Q27
256 x 64 x 64, walls at y = 0 and 63, 272 jittered droplets of radius 7, body
force 1e-5 along x, NCI A = 0.005, h 2..4, tau = 1).

Q and Q_d (the flow rate and the dispersed-phase flow rate through a
cross-section, Results / Fig. 3) are sampled every 100 steps from step 5,000
to 10,000 (51 samples); the stored means over those samples are the
reference for the time-averaged flow rate of long chaotic runs.  Calls only
the oracle and the input generators; about half an hour on eight cores.

    python tests/golden/make_channel3d_long.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

T0, T1, EVERY = 5000, 10000, 100


def main():
    case = synth.hex_channel_3d()
    p = oracle.Params(**{k: v for k, v in case.params.items() if k in oracle.Params.__dataclass_fields__})
    o = oracle.Oracle(p)
    o.init_fields(case.rho1, case.rho2, case.u)
    m0 = o.observables()["mass"]
    start = time.time()
    o.step(T0)
    t, q, qd = [], [], []
    while True:
        ob = o.observables()
        t.append(o.t)
        q.append(ob["Q"])
        qd.append(ob["Q_d"])
        print(f"t={o.t} Q={ob['Q']:.9e} Q_d={ob['Q_d']:.9e} ({time.time() - start:.0f} s)", flush=True)
        if o.t >= T1:
            break
        o.step(EVERY)
    m1 = o.observables()["mass"]
    out = {"workload": "synth.hex_channel_3d()", "t0": T0, "t1": T1, "every": EVERY,
           "Q_mean": float(np.mean(q)), "Q_d_mean": float(np.mean(qd)),
           "Q_min": float(np.min(q)), "Q_max": float(np.max(q)),
           "mass_drift": [float(x) for x in (m1 - m0) / m0],
           "t": t, "Q": q, "Q_d": qd}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "channel3d_long.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("t", "Q", "Q_d")}))


if __name__ == "__main__":
    main()
