"""Learned warm start of the colour-gradient + NCI lattice Boltzmann channels.

A U-Net (``ws.UNet``: BF16 MFMA forward and backward kernels, Adam on FP32
master weights) is trained on steady states that the lattice Boltzmann
library itself produces.  It maps a channel's initial condition -- the
droplet-packed phase field psi0, the pressure-gradient plane and the NCI
strength plane -- to the predicted steady phase field and velocity field.
A run is then started from that prediction (phase clipped to [-1, 1] and
mass-corrected so that both component masses equal the plain start's,
populations at equilibrium with the predicted velocity) and stepped to the
same windowed flow-rate criterion as the plain start.

The method's own experiments (flow-rate measurements of droplet-packed
channels under a pressure gradient, Results section) motivate the workload:
2-D wall-bounded channels 256 x 128 (126 fluid rows) with a jittered
hexagonal droplet packing, packing fraction U[0.7, 0.9], pressure gradient
log-uniform in [1e-6, 1e-4], NCI strength U[0, 0.05], droplet radius
U{10..20}, relaxation time raised with the pressure gradient so that the
Poiseuille peak speed stays <= 0.05 (``synth.channel_spec``).

Metric: t_1% -- the first window end after which the windowed flow rate
stays within 1 % of Q_ref, the time average of the plain run's last windows
-- plus steps to the convergence criterion, for the plain and the warm start
on held-out seeds; velocity-only and phase-only warm starts are ablations.

Every lattice Boltzmann step and every network pass runs in the HIP library;
this module prepares inputs, moves data and keeps statistics.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import dataclasses
from dataclasses import dataclass

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from paper_2003_11069_amd import lb, ws  # noqa: E402

@dataclass(frozen=True)
class Setup:
    """Channel size, parameter ranges and convergence settings of a
    warm-start workload.  The channels come from the batched-sweep generator
    (synth.channel_spec) at a fixed size, its draws mapped onto the given
    ranges of pressure gradient, NCI strength and droplet radius."""
    H: int = 128          # image rows (y, walls at 0 and H-1)
    W: int = 256          # image columns (x, periodic)
    G_range: tuple = (1e-6, 1e-4)
    A_range: tuple = (0.0, 0.05)
    R_range: tuple = (10, 20)
    window: int = 500     # steps per flow-rate window
    obs_every: int = 10   # steps between flow-rate samples
    conv_m: int = 3
    conv_eps: float = 1e-4

    @property
    def conv(self) -> dict:
        return dict(obs_every=self.obs_every, conv_window=self.window // self.obs_every,
                    conv_m=self.conv_m, conv_eps=self.conv_eps)


FULL = Setup()                                         # the 256 x 128 workload
SMALL = Setup(H=64, W=128, R_range=(5, 10), window=250)  # the same geometry at half scale
H, W = FULL.H, FULL.W
WINDOW = FULL.window
CONV = FULL.conv
U_CLIP = 1.5     # bound on predicted |u_x|, |u_y| in units of u_ref


def make_case(seed: int, st: Setup = FULL):
    spec = synth.channel_spec(seed, Lx=st.W, Ly=st.H, G_range=st.G_range, A_range=st.A_range,
                              R_range=st.R_range)
    return spec, synth.channel_2d(spec)


def u_ref(spec) -> float:
    """Poiseuille centre-line speed G H^2 / (8 nu) over the fluid height."""
    nu = (spec.tau - 0.5) / 3.0
    h = spec.Ly - 2
    return spec.G_p * h * h / (8.0 * nu)


def net_input(spec, case) -> np.ndarray:
    """[H, W, 3] float32: psi0, (log10 G_p + 5), A_nci / 0.025 - 1."""
    H, W = spec.Ly, spec.Lx
    r1 = case.rho1.reshape(H, W)
    r2 = case.rho2.reshape(H, W)
    psi = np.where(r1 + r2 > 0, (r1 - r2) / np.maximum(r1 + r2, 1e-300), -1.0)
    psi[0, :] = psi[-1, :] = -1.0
    x = np.empty((H, W, 3), np.float32)
    x[..., 0] = psi
    x[..., 1] = math.log10(spec.G_p) + 5.0
    x[..., 2] = spec.A_nci / 0.025 - 1.0
    return x


def net_target(spec, rho1, rho2, u) -> np.ndarray:
    """[H, W, 3] float32: steady psi, u_x / u_ref, u_y / u_ref (walls: -1, 0, 0)."""
    H, W = spec.Ly, spec.Lx
    r1 = rho1.reshape(H, W)
    r2 = rho2.reshape(H, W)
    rho = r1 + r2
    psi = np.where(rho > 0, (r1 - r2) / np.where(rho > 0, rho, 1.0), -1.0)
    ur = u_ref(spec)
    t = np.empty((H, W, 3), np.float32)
    t[..., 0] = psi
    t[..., 1] = u[0].reshape(H, W) / ur
    t[..., 2] = u[1].reshape(H, W) / ur
    t[0] = t[-1] = 0.0
    t[0, :, 0] = t[-1, :, 0] = -1.0
    return t


def init_from_prediction(spec, case, pred: np.ndarray, phase=True, velocity=True):
    """Initial (rho1, rho2, u) of a warm start from a prediction [H, W, 3].

    Phase: psi clipped to [-1, 1], rho1 = (1 + psi)/2, rho2 = 1 - rho1 on
    fluid rows, then one component scaled (rho1 down, or rho2 down) so that
    the dispersed mass equals the plain start's; the total density stays 1,
    so the continuous mass matches too.  Velocity: u_ref times the predicted
    u / u_ref on fluid rows, each component clipped to [-U_CLIP, U_CLIP] (the
    steady speed never exceeds the Poiseuille centre-line speed by much; the
    clip keeps a poor prediction from starting an unstable run).  Unused
    parts come from the plain start."""
    H, W = spec.Ly, spec.Lx
    N = H * W
    pred = np.nan_to_num(pred, nan=0.0, posinf=0.0, neginf=0.0)
    fluid = np.zeros((H, W), bool)
    fluid[1:H - 1] = True
    fluid = fluid.ravel()
    if phase:
        psi = np.clip(pred[..., 0].astype(np.float64), -1.0, 1.0).ravel()
        r1 = 0.5 * (1.0 + psi)
        m_target = case.rho1[fluid].sum()
        m = r1[fluid].sum()
        if m > m_target:
            r1[fluid] *= m_target / m
        elif m < m_target:
            r2f = 1.0 - r1[fluid]
            r2f *= (fluid.sum() - m_target) / r2f.sum()
            r1[fluid] = 1.0 - r2f
        r1[~fluid] = 0.0
        r2 = np.where(fluid, 1.0 - r1, 0.0)
    else:
        r1, r2 = case.rho1.copy(), case.rho2.copy()
    u = None
    if velocity:
        ur = u_ref(spec)
        u = np.zeros((2, N))
        u[0] = (np.clip(pred[..., 1].astype(np.float64), -U_CLIP, U_CLIP) * ur).ravel()
        u[1] = (np.clip(pred[..., 2].astype(np.float64), -U_CLIP, U_CLIP) * ur).ravel()
        u[:, ~fluid] = 0.0
    return r1, r2, u


def perturbed_start(spec, case, amp=1e-3, noise_seed=0):
    """Plain start plus white-noise velocity of amplitude amp * u_ref."""
    H, W = spec.Ly, spec.Lx
    rng = np.random.Generator(np.random.PCG64(spec.seed + 7 + noise_seed))
    u = amp * u_ref(spec) * rng.uniform(-1.0, 1.0, (2, H * W))
    u[:, :W] = 0.0
    u[:, -W:] = 0.0
    return case.rho1.copy(), case.rho2.copy(), u


def run_channels(specs_cases, inits=None, cap=100_000, chunk=None, keep_fields=False,
                 mode=lb.LB_BATCH_LAUNCH, log=None, st: Setup = FULL, retire=True):
    """Steps the channels (one batch) to the convergence criterion or `cap`
    steps (to `cap` in every channel when retire is False).  Returns per
    channel: steps, converged, the windowed flow-rate history
    [(step, Q_window)], and final fields if keep_fields."""
    chunk = chunk or st.window
    conv = st.conv if retire else dict(st.conv, conv_m=2 ** 30)  # windows kept, never converged
    params = [lb.Params.from_dict(c.params, **conv) for _, c in specs_cases]
    b = lb.Batch(params)
    for k, (_, c) in enumerate(specs_cases):
        if inits is None or inits[k] is None:
            b.init_fields(k, c.rho1, c.rho2)
        else:
            r1, r2, u = inits[k]
            b.init_fields(k, r1, r2, u)
    n = len(params)
    hist = [[] for _ in range(n)]
    active = np.ones(n, bool)
    t, t0 = 0, time.perf_counter()
    while t < cap and active.any():
        b.step(chunk, mode, numeric_ok=True)  # non-finite runs are dropped below
        t += chunk
        for k in np.flatnonzero(active):
            inf = b.info(k)
            ob = b.observables(k)
            hist[k].append((inf["steps"], ob["Q_window"]))
            active[k] = inf["active"]
        if log and (t // chunk) % 20 == 0:
            log(f"    t={t} active {int(active.sum())}/{n} ({time.perf_counter() - t0:.1f} s)")
    out = []
    for k in range(n):
        ob = b.observables(k)
        r = {"steps": b.info(k)["steps"], "converged": bool(ob["converged"]), "hist": hist[k],
             "finite": not (ob["flags"] & 1) and ob["rc"] == 0 and math.isfinite(ob["Q"])}
        if keep_fields:
            r["fields"] = b.fields(k)
        out.append(r)
    lu = sum(r["steps"] * c.rho1.size for r, (_, c) in zip(out, specs_cases))
    b.close()
    return out, lu


def q_ref_of(hist, last=20) -> float:
    q = [v for _, v in hist[-last:]]
    return float(np.mean(q))


def q_final(hist, last=4) -> float:
    """Mean of the last windowed flow rates of a run."""
    return float(np.mean([v for _, v in hist[-last:]]))


def t_within(hist, q_ref: float, tol=0.01):
    """First window end after which every recorded windowed flow rate is
    within tol of q_ref (None if the last one is not)."""
    ok = [abs(v - q_ref) <= tol * abs(q_ref) for _, v in hist]
    if not ok or not ok[-1]:
        return None
    j = len(ok) - 1
    while j > 0 and ok[j - 1]:
        j -= 1
    return hist[j][0]


# --- dataset and training ------------------------------------------------------

def generate(seeds, cap, batch=256, log=print, st: Setup = FULL):
    """Plain runs to the convergence criterion; returns inputs, targets, stats."""
    X = np.empty((len(seeds), st.H, st.W, 3), np.float32)
    T = np.empty((len(seeds), st.H, st.W, 3), np.float32)
    stats, lu_total, t0 = [], 0, time.perf_counter()
    good = np.ones(len(seeds), bool)
    bad = []
    for s0 in range(0, len(seeds), batch):
        sc = [make_case(s, st) for s in seeds[s0:s0 + batch]]
        res, lu = run_channels(sc, cap=cap, keep_fields=True, log=log, st=st)
        lu_total += lu
        for k, ((spec, case), r) in enumerate(zip(sc, res)):
            X[s0 + k] = net_input(spec, case)
            T[s0 + k] = net_target(spec, *r["fields"])
            ok = r["finite"] and bool(np.isfinite(T[s0 + k]).all())
            good[s0 + k] = ok
            if not ok:
                bad.append(spec.as_dict())
            stats.append((r["steps"], r["converged"]))
        el = time.perf_counter() - t0
        log(f"  generated {s0 + len(sc)}/{len(seeds)}: {lu_total / el / 1e9:.2f} GLUPS, {el:.0f} s, "
            f"{len(bad)} non-finite so far")
    for sp in bad:
        log(f"  non-finite run: {sp}")
    return X[good], T[good], stats, lu_total / (time.perf_counter() - t0), bad


def augment(X, T, rng):
    """Random periodic shift along x and mirror in y (u_y changes sign): both
    map a channel's steady state to the steady state of the transformed
    channel (walls and force are symmetric under them)."""
    n, H, W = X.shape[:3]
    shift = rng.integers(0, W, n)
    flip = rng.uniform(size=n) < 0.5
    cols = (np.arange(W)[None, :] - shift[:, None]) % W            # [n, W]
    rows = np.where(flip[:, None], np.arange(H)[::-1][None, :], np.arange(H)[None, :])  # [n, H]
    idx = (np.arange(n)[:, None, None], rows[:, :, None], cols[:, None, :])
    X2, T2 = X[idx], T[idx]
    T2[flip, :, :, 2] *= -1.0
    return X2, T2


def train(net, X, T, epochs, batch, lr, seed=0, log=print):
    rng = np.random.default_rng(seed)
    H, W = X.shape[1:3]
    n = (len(X) // batch) * batch
    dX = ws.DeviceArray((n, H, W, 3))
    dT = ws.DeviceArray((n, H, W, 3))
    per = H * W * 3
    fwd, bwd = net.flops(batch)
    steps, t_gpu, losses = 0, 0.0, []
    total = epochs * (n // batch)
    for ep in range(epochs):
        perm = rng.permutation(len(X))[:n]
        xa, ta = augment(X[perm], T[perm], rng)
        dX.upload(xa)
        dT.upload(ta)
        ws.sync()
        t0 = time.perf_counter()
        ep_loss = []
        for i in range(n // batch):
            # cosine learning-rate decay over all steps
            lr_i = lr * 0.5 * (1 + math.cos(math.pi * steps / total))
            want = i == n // batch - 1
            l = net.train_step_ptr(dX.ptr(i * batch * per), dT.ptr(i * batch * per), batch, lr_i,
                                   want_loss=want)
            if want:
                ep_loss.append(l)
            steps += 1
        ws.sync()
        t_gpu += time.perf_counter() - t0
        losses.append(ep_loss[-1])
        log(f"  epoch {ep + 1}/{epochs}: loss {ep_loss[-1]:.4e}, "
            f"{(fwd + bwd) * steps / t_gpu / 1e12:.1f} TFLOP/s")
    dX.free()
    dT.free()
    return {"steps": steps, "seconds": t_gpu, "tflops": (fwd + bwd) * steps / t_gpu / 1e12, "losses": losses}


def predict(net, X, batch):
    H, W = X.shape[1:3]
    out = np.empty_like(X)
    dX = ws.DeviceArray((batch, H, W, 3))
    dY = ws.DeviceArray((batch, H, W, 3))
    for s in range(0, len(X), batch):
        b = min(batch, len(X) - s)
        dX.upload(X[s:s + b])
        net.forward_ptr(dX.ptr(), b, dY.ptr())
        out[s:s + b] = dY.download(b * H * W * 3).reshape(b, H, W, 3)
    dX.free()
    dY.free()
    return out


def _summary(ts, cap):
    a = np.array([cap if t is None else t for t in ts], float)
    return {"median": float(np.median(a)), "q25": float(np.percentile(a, 25)),
            "q75": float(np.percentile(a, 75)), "mean": float(a.mean()),
            "never": int(sum(t is None for t in ts))}


def late_mean(hist, frac=0.5) -> float:
    """Mean windowed flow rate over the last `frac` of a run's windows."""
    q = [v for _, v in hist]
    k = max(1, int(round(len(q) * frac)))
    return float(np.mean(q[-k:]))


def evaluate(net, seeds, cap, batch=200, log=print, st: Setup = FULL, n_ref=3):
    """Held-out evaluation of the warm start on the steps-to-steady metric.

    Every start runs `cap` steps (no early retirement).  The reference flow
    rate of a seed, Q_ref, is robust to the run-to-run spread of the method:
    the mean, over an ensemble of the plain start and n_ref plain starts with
    a velocity perturbation of 1e-3 u_ref (different noise each), of each
    run's mean windowed Q over the last half of the run; the ensemble's
    largest deviation from Q_ref is reported as the spread.  t_1% of a start
    is the first window end after which its windowed Q stays within 1 % of
    Q_ref to the end of the run (None: it is not within 1 % at the end).
    Variants: plain, warm (phase and velocity predicted), velocity only,
    phase only."""
    sc = [make_case(s, st) for s in seeds]
    X = np.stack([net_input(sp, c) for sp, c in sc])
    t0 = time.perf_counter()
    P = predict(net, X, 16)
    t_pred = time.perf_counter() - t0
    variants = {"plain": None, "warm": (True, True), "velocity_only": (False, True), "phase_only": (True, False)}
    for k in range(n_ref):
        variants[f"ref_{k}"] = ("noise", k)
    runs, acc = {}, []
    for name, v in variants.items():
        log(f"  eval {name}")
        res = []
        for s0 in range(0, len(sc), batch):
            part = sc[s0:s0 + batch]
            if v is None:
                inits = None
            elif v[0] == "noise":
                inits = [perturbed_start(sp, c, noise_seed=v[1]) for sp, c in part]
            else:
                inits = [init_from_prediction(sp, c, P[s0 + k], *v) for k, (sp, c) in enumerate(part)]
            r, _ = run_channels(part, inits, cap=cap, keep_fields=(v is None), log=None, st=st,
                                retire=False)
            if v is None:  # prediction accuracy against the plain end state
                for k, (sp, c) in enumerate(part):
                    tgt = net_target(sp, *r[k].pop("fields"))
                    pr = P[s0 + k]
                    du = pr[1:-1, :, 1:] - tgt[1:-1, :, 1:]
                    acc.append({"u_rel_l2": float(np.linalg.norm(du) / np.linalg.norm(tgt[1:-1, :, 1:])),
                                "q_pred_rel": float(pr[1:-1, :, 1].sum() / tgt[1:-1, :, 1].sum() - 1),
                                "psi_mae": float(np.abs(pr[1:-1, :, 0] - tgt[1:-1, :, 0]).mean())})
            res += r
        runs[name] = res
    ens = ["plain"] + [f"ref_{k}" for k in range(n_ref)]
    keep = [all(runs[e][i]["finite"] for e in ens) for i in range(len(sc))]
    excluded = [s for s, k in zip(seeds, keep) if not k]
    runs = {name: [r for r, k in zip(res, keep) if k] for name, res in runs.items()}
    acc = [a for a, k in zip(acc, keep) if k]
    late = np.array([[late_mean(runs[e][i]["hist"]) for e in ens] for i in range(len(runs["plain"]))])
    qref = late.mean(axis=1)
    spread = np.abs(late / qref[:, None] - 1).max(axis=1)
    out = {"n": len(qref), "excluded_nonfinite_seeds": excluded, "cap": cap, "n_ref": n_ref,
           "predict_seconds": t_pred, "q_ref_spread_median": float(np.median(spread)),
           "q_ref_spread_max": float(spread.max()), "variants": {}}
    seed_table, t1s = {}, {}
    for name in ["plain", "warm", "velocity_only", "phase_only"]:
        res = runs[name]
        t1 = [t_within(r["hist"], q) for r, q in zip(res, qref)]
        qf = [late_mean(r["hist"]) / q - 1 for r, q in zip(res, qref)]
        fin = [abs(x) for x in qf if math.isfinite(x)]
        out["variants"][name] = {"t1": _summary(t1, cap),
                                 "late_Q_abs_rel_dev_median": float(np.median(fin)) if fin else None,
                                 "nonfinite": int(sum(not r["finite"] for r in res))}
        t1s[name] = t1
        seed_table[name] = {"t1": [None if t is None else int(t) for t in t1],
                            "late_q_rel": [x if math.isfinite(x) else None for x in qf]}
    for name in ["warm", "velocity_only", "phase_only"]:
        a = [cap if t is None else t for t in t1s[name]]
        p = [cap if t is None else t for t in t1s["plain"]]
        out["variants"][name]["frac_worse_than_plain"] = float(np.mean([x > y for x, y in zip(a, p)]))
        out["variants"][name]["frac_better_than_plain"] = float(np.mean([x < y for x, y in zip(a, p)]))
        out["variants"][name]["median_speedup_t1"] = float(np.median([y / max(x, st.window)
                                                                      for x, y in zip(a, p)]))
    out["prediction"] = {k: float(np.median([a[k] for a in acc])) for k in acc[0]}
    out["prediction"]["q_pred_abs_rel_median"] = float(np.median([abs(a["q_pred_rel"]) for a in acc]))
    out["per_seed"] = seed_table
    out["per_seed_q_ref"] = qref.tolist()
    out["per_seed_spread"] = spread.tolist()
    out["seeds"] = [s for s, k in zip(seeds, keep) if k]
    hist = {name: [[v for _, v in r["hist"]] for r in res] for name, res in runs.items()}
    return out, P, hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", type=int, default=2000, help="training runs (seeds 1000...)")
    ap.add_argument("--eval", type=int, default=200, help="held-out runs (seeds 5000...)")
    ap.add_argument("--cap", type=int, default=100_000, help="step cap per run")
    ap.add_argument("--train-cap", type=int, default=None, help="step cap of the dataset runs")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--lb-batch", type=int, default=256, help="channels per batched LB launch")
    ap.add_argument("--out", default="gpurun_out/warmstart.json")
    ap.add_argument("--load-params", default=None, help="skip dataset and training; evaluate these weights")
    ap.add_argument("--small", action="store_true", help="128 x 64 channels, radii halved (test scale)")
    ap.add_argument("--n-ref", type=int, default=3, help="perturbed plain runs in the reference ensemble")
    ap.add_argument("--g-range", type=float, nargs=2, default=None, help="pressure-gradient range")
    ap.add_argument("--a-range", type=float, nargs=2, default=None, help="NCI-strength range")
    ap.add_argument("--r-range", type=int, nargs=2, default=None, help="droplet-radius range")
    ap.add_argument("--window", type=int, default=None, help="steps per flow-rate window")
    a = ap.parse_args(argv)
    st = SMALL if a.small else FULL
    over = {k: tuple(v) for k, v in (("G_range", a.g_range), ("A_range", a.a_range), ("R_range", a.r_range))
            if v is not None}
    if a.window:
        over["window"] = a.window
    if over:
        st = dataclasses.replace(st, **over)

    def log(msg):
        print(msg, flush=True)

    res = {"args": vars(a), "setup": dataclasses.asdict(st)}
    t_all = time.perf_counter()
    net = ws.UNet(ws.UNetConfig(levels=a.levels, base=a.base, cin=3, cout=3, H=st.H, W=st.W, max_batch=a.batch))
    if a.load_params:
        net.set_params(np.load(a.load_params))
        log(f"[warmstart] loaded {a.load_params}")
        ev, _, hist = evaluate(net, list(range(5000, 5000 + a.eval)), a.cap, a.lb_batch, log, st, a.n_ref)
        res["eval"] = ev
        _save(res, a.out)
        _save_hist(hist, a.out)
        log(json.dumps({"prediction": ev["prediction"], "variants": ev["variants"]}, indent=1))
        return 0
    log(f"[warmstart] dataset: {a.train} runs")
    X, T, stats, glups, bad = generate(list(range(1000, 1000 + a.train)), a.train_cap or a.cap, a.lb_batch, log,
                                       st)
    steps = np.array([s for s, _ in stats])
    res["dataset"] = {"runs": a.train, "used": int(len(X)), "nonfinite_runs": bad, "glups": glups / 1e9,
                      "steps_median": float(np.median(steps)),
                      "converged_frac": float(np.mean([c for _, c in stats]))}
    _save(res, a.out)
    log(f"[warmstart] train U-Net L={a.levels} base={a.base} on {len(X)} runs")
    net.set_params(synth.unet_params(a.levels, a.base, seed=0))
    res["train"] = train(net, X, T, a.epochs, a.batch, a.lr, log=log)
    del X, T
    np.save(os.path.splitext(a.out)[0] + "_params.npy", net.params())
    _save(res, a.out)
    log(f"[warmstart] evaluate on {a.eval} held-out seeds")
    ev, _, hist = evaluate(net, list(range(5000, 5000 + a.eval)), a.cap, a.lb_batch, log, st, a.n_ref)
    res["eval"] = ev
    _save_hist(hist, a.out)
    res["seconds"] = time.perf_counter() - t_all
    _save(res, a.out)
    log(json.dumps({"prediction": ev["prediction"], "variants": ev["variants"],
                    "q_ref_spread_median": ev["q_ref_spread_median"]}, indent=1))
    return 0


def _save_hist(hist, path):
    """Windowed flow-rate histories per variant and seed (npz, float64)."""
    arrays = {}
    for name, runs in hist.items():
        L = max(len(h) for h in runs)
        a = np.full((len(runs), L), np.nan)
        for i, h in enumerate(runs):
            a[i, :len(h)] = h
        arrays[name] = a
    np.savez_compressed(os.path.splitext(path)[0] + "_hist.npz", **arrays)


def _save(res, path):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
