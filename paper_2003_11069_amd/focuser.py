"""Droplet generation in a flow-focuser (Results: Fig. 1 and the flow-rate
phase diagram of Fig. 3, Q_d = nu V_d).

Runs the device geometry of ``synth.flow_focuser_2d`` on the GPU library
(lb_set_geometry, lb_step) and measures, from lb_droplets samples taken every
``every`` steps after ``t_skip`` steps:

* V_d: the median volume of the main droplets (volume at least half the
  largest median, so satellites are excluded) downstream of the striction;
* nu: the generation frequency, the number of main droplets whose centroid
  crosses the line x_c (a quarter of the outlet channel downstream of the
  striction) per step; a droplet is followed between samples by the nearest
  earlier centroid at most one node ahead, 20 behind and 10 rows away;
* Q_d = nu V_d, beside the dispersed flux through x_c measured directly
  (the time average of sum_y rho1 u_x over that column) for comparison.

All arithmetic of the lattice runs in the library; this module only
schedules steps and reduces the sampled droplet tables.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import synth
from . import lb as _lb


def reduce_samples(samples, xc):
    """(V_d, crossings, nu) from droplet samples [(t, centroids[:, (x, y)],
    volumes)] taken at a fixed interval (see the module docstring)."""
    big = np.concatenate([v for _, _, v in samples]) if samples else np.zeros(0)
    v_main = 0.0
    if big.size:
        v_main = float(np.median(big[big >= 0.5 * np.percentile(big, 90)]))
    crossings = 0
    for (ta, ca, va), (tb, cb, vb) in zip(samples, samples[1:]):
        for (x, y), v in zip(cb, vb):
            if v < 0.5 * v_main or x < xc:
                continue
            # the same droplet one sample earlier: the nearest centroid at most
            # one node ahead and 20 behind, within 10 rows
            sel = (ca[:, 0] <= x + 1) & (ca[:, 0] > x - 20) & (np.abs(ca[:, 1] - y) < 10)
            if not sel.any():
                continue
            prev = ca[sel][np.argmin(np.hypot(ca[sel, 0] - x, ca[sel, 1] - y))]
            if prev[0] < xc:
                crossings += 1
    span = samples[-1][0] - samples[0][0] if len(samples) > 1 else 1
    return v_main, crossings, crossings / span


class _Run:
    """One flow-focuser handle and its samples (droplet tables and the flux
    through x_c), stepped by ``run`` alone or by ``sweep`` beside others."""

    def __init__(self, scale, phi, u_c, A_s, N_c, W_out, storage, stream=None):
        self.case = case = synth.flow_focuser_2d(scale=scale, phi=phi, u_c=u_c, A_s=A_s, N_c=N_c, W_out=W_out)
        p = case.params
        self.phi, self.nx, self.ny = phi, p["nx"], p["ny"]
        self.lat = _lb.Lattice(_lb.Params.from_dict(p, storage=_lb.STORAGE[storage]), stream=stream)
        self.lat.set_geometry(case.info["type"], case.rho1, case.rho2, case.u)
        self.lat.init_fields(case.rho1, case.rho2, case.u)
        self.x0 = case.info["x_out0"]
        self.xc = self.x0 + (self.nx - self.x0) // 4
        self.samples = []       # (t, centroids[:, (x, y)], volumes)
        self.flux = []

    def sample(self):
        d = self.lat.droplets(labels=False)
        cen, vol = d["centroids"], d["volumes"]
        keep = cen[:, 0] > self.x0
        self.samples.append((self.lat.t, cen[keep, :2].copy(), vol[keep].copy()))
        r1, r2, u = self.lat.fields()
        nx, ny, xc = self.nx, self.ny, self.xc
        self.flux.append(float((r1.reshape(ny, nx)[:, xc] * u[0].reshape(ny, nx)[:, xc]).sum()))

    def result(self, steps, t_skip, every, elapsed, keep_samples):
        info = self.case.info
        v_main, crossings, nu = reduce_samples(self.samples, self.xc)
        return {"nx": self.nx, "ny": self.ny, "fluid_nodes": int((info["type"] == synth.FLUID).sum()),
                "phi": self.phi, "u_c": info["u_c"], "u_d": info["u_d"],
                "steps": steps, "t_skip": t_skip, "every": every, "x_c": int(self.xc),
                "V_d": v_main, "droplets_crossed": crossings, "nu": nu, "Q_d": nu * v_main,
                "flux_xc_mean": float(np.mean(self.flux)) if self.flux else 0.0,
                "inlet_dispersed_flux": info["u_d"] * info["H"],
                "seconds": elapsed, "graphs": self.lat.graphs,
                "samples": self.samples if keep_samples else None,
                "flux_samples": self.flux if keep_samples else None}


def run(scale=2.0, phi=0.25, u_c=0.004, A_s=0.1, N_c=0.1, W_out=64, steps=60000, t_skip=20000,
        every=250, storage="fp32", keep_samples=False):
    r = _Run(scale, phi, u_c, A_s, N_c, W_out, storage)
    t0 = time.perf_counter()
    r.lat.step(t_skip)
    while r.lat.t < steps:
        r.lat.step(every)
        r.sample()
    return r.result(steps, t_skip, every, time.perf_counter() - t0, keep_samples)


def sweep(phis, scale=2.0, u_c=0.004, A_s=0.1, N_c=0.1, W_out=64, steps=60000, t_skip=20000, every=250,
          storage="fp32", keep_samples=False):
    """``run`` for every flow ratio in ``phis`` at once: one handle per phi,
    each on its own HIP stream (default priority), stepped in lockstep.  One
    focuser of this size keeps under one wave per SIMD busy, so the handles'
    kernels run side by side on the idle compute units; each handle's
    arithmetic is that of ``run`` (the same results, bit for bit).  Returns
    one result per phi, each with the wall time of the whole sweep."""
    streams, runs = [], []
    try:
        for phi in phis:
            streams.append(_lb.Stream())
            runs.append(_Run(scale, phi, u_c, A_s, N_c, W_out, storage, stream=streams[-1].handle))
        t0 = time.perf_counter()
        for r in runs:
            r.lat.step(t_skip)
        while runs[0].lat.t < steps:
            for r in runs:          # enqueue every handle's steps before the first sample waits
                r.lat.step(every)
            for r in runs:
                r.sample()
        elapsed = time.perf_counter() - t0
        return [r.result(steps, t_skip, every, elapsed, keep_samples) for r in runs]
    finally:  # handles before the streams they use
        for r in runs:
            r.lat.close()
        for st in streams:
            st.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--phi", type=float, nargs="+", default=[0.25])
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--skip", type=int, default=20000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--u-c", type=float, default=0.004)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--concurrent", action="store_true", help="all phi at once, one HIP stream each")
    a = ap.parse_args(argv)
    if a.concurrent:
        res = sweep(a.phi, u_c=a.u_c, steps=a.steps, t_skip=a.skip, every=a.every, storage=a.storage)
    else:
        res = (run(phi=phi, u_c=a.u_c, steps=a.steps, t_skip=a.skip, every=a.every, storage=a.storage)
               for phi in a.phi)
    for r in res:
        r.pop("samples"); r.pop("flux_samples")
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
