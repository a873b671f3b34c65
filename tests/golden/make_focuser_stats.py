"""Writes tests/golden/focuser_stats.json: droplet-generation statistics of
the flow-focuser (synth.flow_focuser_2d(scale=2, phi=0.25, u_c=0.004,
A_s=0.1, N_c=0.1, W_out=64)) from the FP64 oracle: droplet tables every 250
steps from step 20,000 to 140,000 (and over the first window, to 80,000),
reduced by oracle.analysis.generation_stats (V_d, nu, Q_d = nu V_d, Results /
Fig. 3), and the mean dispersed flux sum_y rho1 u_x through the measuring
column.  Calls only the oracle and the
input generators; about ten minutes on eight cores.

    python tests/golden/make_focuser_stats.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import analysis as A  # noqa: E402

CONFIG = dict(scale=2.0, phi=0.25, u_c=0.004, A_s=0.1, N_c=0.1, W_out=64)
STEPS, SKIP, EVERY = 140000, 20000, 250
EARLY = 80000  # end of the first window (steps 20,000-80,000)


def main():
    c = synth.flow_focuser_2d(**CONFIG)
    p = c.params
    nx, ny = p["nx"], p["ny"]
    o = oracle.Oracle(oracle.Params(**p))
    o.set_geometry(c.info["type"], c.rho1, c.rho2, c.u)
    o.init_fields(c.rho1, c.rho2, c.u)
    x0 = c.info["x_out0"]
    xc = x0 + (nx - x0) // 4
    o.step(SKIP)
    samples, flux = [], []
    while o.t < STEPS:
        o.step(EVERY)
        r1, r2, u = o.fields()
        m = A.dispersed_mask(r1, r2, nx, ny, 1, 0)
        lab, _ = A.components(m, (True, True, True))
        _, vols, cen = A.droplet_table(lab, nx, ny, 1, 0)
        keep = cen[:, 0] > x0
        samples.append((o.t, cen[keep, :2], vols[keep]))
        flux.append(float((r1.reshape(ny, nx)[:, xc] * u[0].reshape(ny, nx)[:, xc]).sum()))
    V_d, n, nu = A.generation_stats(samples, xc)
    early = [s for s in samples if s[0] <= EARLY]
    V_e, n_e, nu_e = A.generation_stats(early, xc)
    out = {"config": CONFIG, "steps": STEPS, "skip": SKIP, "every": EVERY, "x_c": int(xc),
           "V_d": V_d, "crossings": n, "nu": nu, "Q_d": nu * V_d, "flux_xc_mean": float(np.mean(flux)),
           "early_end": EARLY, "early_V_d": V_e, "early_crossings": n_e, "early_nu": nu_e,
           "early_flux_xc_mean": float(np.mean(flux[:len(early)]))}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "focuser_stats.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
