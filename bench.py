#!/usr/bin/env python3
"""Throughput benchmark of the colour-gradient + NCI lattice Boltzmann step.

Workload (default): 3-D D3Q27 droplet-packed channel 256 x 64 x 64, walls at
y = 0 and 63, periodic x and z, 272 jittered droplets of radius 7 on a
hexagonal packing, body force 1e-5 along x, NCI on (A = 0.005, h_min = 2,
h_max = 4), tau = 1, FP32 deviation storage.  One step = k_phase + k_main over
the whole lattice; the state is resident in HBM before timing starts.

Prints ONE JSON line with MLUPS (fluid nodes), the roofline of the dominant
kernel (k_main) measured with HIP events on the library's stream, the
achievable-bandwidth reference of a plain copy kernel, and the FP64 oracle
timed on the host cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS/GPU + HBM roofline %; steps-to-steady-state plain vs learned warm start"
HBM_PEAK_GBPS = 8000.0
# bytes of the paper's two-population state read + written once per fluid
# node-update plus psi written and read once (FP32 populations)
def two_pop_bytes(dim: int, storage: str) -> int:
    """The paper's own state per fluid-node update: both components'
    populations read and written once in the storage precision, plus psi
    written and read once (4 B each)."""
    q = 9 if dim == 2 else 27
    e = 2 if storage in ("fp16", "bf16") else 4
    return 2 * 2 * q * e + 8


def main_kernel_bytes(dim: int, storage: str) -> int:
    """Compulsory HBM bytes per fluid node of one k_main launch in the
    library's layout: the Q stored deviations s_i read once, rho1 and psi read
    once, the full state (s_i, colour fraction a, colour vector B) written
    once."""
    Q = 9 if dim == 2 else 27
    s_b = 2 if storage in ("fp16", "bf16") else 4
    r_b = 8 if storage == "fp32" else 4
    rest_extra = 4 - s_b if storage in ("fp16", "bf16") else 0  # FP32 rest slot
    pops = Q * s_b + rest_extra
    return (pops + 2 * r_b) + (pops + r_b + 4 * dim)


def traffic_from_profile(name: str):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None
    when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*(\w+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    from paper_2003_11069_amd.profile_summary import kernel_source_hash
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def _oracle_steps_for(case, budget_s: float, max_steps: int = 1000):
    """Steps the FP64 oracle as it stands on the workload until ~budget_s;
    returns (steps, seconds) after one untimed first-touch step."""
    import oracle
    p = oracle.Params(**{k: v for k, v in case.params.items() if k in oracle.Params.__dataclass_fields__})
    o = oracle.Oracle(p)
    o.init_fields(case.rho1, case.rho2, case.u)
    o.step(1)  # first-touch of the arrays
    n, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= max_steps:
            return n, el


def host_cpu() -> dict:
    """Model name, physical cores and logical CPUs of the host (Linux
    /proc/cpuinfo), and the CPUs this process may run on."""
    model, cores, logical = "unknown", set(), 0
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"model": model, "physical_cores": len(cores) or None, "logical_cpus": logical or None,
            "usable_cpus": usable}


def cpu_baseline(case, budget_s: float):
    """The FP64 oracle as it stands on the host: all OpenMP threads in this
    process (~budget_s), and one thread in a child process (~budget_s/2)."""
    fluid = case.params["nx"] * (case.params["ny"] - 2 * case.params["walls_y"]) * case.params["nz"]
    n, el = _oracle_steps_for(case, budget_s)
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or host_cpu()["usable_cpus"]
    one = None
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json; sys.path.insert(0, %r); import bench, synth; "
            "print(json.dumps(bench._oracle_steps_for(synth.hex_channel_3d(), %r)))" % (ROOT, budget_s / 2))
    import subprocess
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode == 0:
        n1, el1 = json.loads(r.stdout.strip().splitlines()[-1])
        one = {"value": fluid * n1 / el1 / 1e6, "cores": 1, "sample": f"{n1} steps, {el1:.1f} s"}
    return {"value": fluid * n / el / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the same workload after 1 warm-up step, {el:.1f} s, "
                      f"{threads} OpenMP threads",
            "one_thread": one, "cpu": host_cpu()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16", "fp32_f32"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="channel3d", choices=["channel3d", "sweep", "unet", "analysis", "geometry",
                                                          "focuser", "oracle"])
    ap.add_argument("--batch", type=int, default=16, help="U-Net training batch (--workload unet)")
    ap.add_argument("--conv-algo", type=int, default=0, choices=[0, 1],
                    help="U-Net 3x3 convolutions: 0 direct kernels where the shape allows, 1 implicit GEMM only")
    ap.add_argument("--mode", default="auto", choices=["auto", "persistent", "launch"],
                    help="batched sweep: the autotuner's choice, or a fixed mode")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU domain decomposition is not built)"}))
        return 2

    import numpy as np
    import synth
    import paper_2003_11069_amd as P
    from paper_2003_11069_amd.lb import copy_probe

    if a.workload == "sweep":
        return bench_sweep(a)
    if a.workload == "unet":
        return bench_unet(a)
    if a.workload == "analysis":
        return bench_analysis(a)
    if a.workload == "geometry":
        return bench_geometry(a)
    if a.workload == "focuser":
        return bench_focuser(a)
    if a.workload == "oracle":
        return bench_oracle(a)
    case = synth.hex_channel_3d()
    prm = case.params
    dim = 3
    fluid = prm["nx"] * (prm["ny"] - 2) * prm["nz"]
    L = P.Lattice(P.Params.from_dict(prm, storage=P.STORAGE[a.storage]))
    L.init_fields(case.rho1, case.rho2, case.u)
    # one-time work outside the timed region: the step-replay graphs of both
    # ping-pong copies are captured and instantiated here, and the
    # achievable-bandwidth reference (a plain copy kernel) runs before the
    # steps, so the device is out of its idle clock state when timing starts
    tc = time.perf_counter()
    L.prepare()
    capture_ms = (time.perf_counter() - tc) * 1e3
    cp = copy_probe(1 << 30, iters=20)
    L.step(a.warmup)
    L.kernel_times()  # drains the stream
    t0 = time.perf_counter()
    dev_ms = L.step_timed(a.steps)  # HIP events on the library's stream around the K steps
    t1 = time.perf_counter()
    el = t1 - t0
    # per-kernel averages from HIP events between the kernels, in a separate
    # run of the same steps (events sit between the kernels, so no graphs)
    L.profile(True)
    L.step(min(a.steps, 500))
    kt = L.kernel_times()
    L.profile(False)
    ob = L.observables()
    mlups = fluid * a.steps / el / 1e6
    ms_step_dev = dev_ms / a.steps
    ms_main = kt["ms_main"] / max(kt["launches"], 1)
    ms_phase = kt["ms_phase"] / max(kt["launches"], 1)
    b_alg = two_pop_bytes(dim, a.storage)
    achieved = b_alg * fluid / (ms_step_dev * 1e-3) / 1e9
    achieved_wall = b_alg * fluid / (el / a.steps) / 1e9
    b_main = main_kernel_bytes(dim, a.storage)
    achieved_main = b_main * fluid / (ms_main * 1e-3) / 1e9
    tr_main = traffic_from_profile(f"k_main_d3q27_{a.storage}_channel256x64x64.txt")
    tr_phase = traffic_from_profile(f"k_phase_d3q27_{a.storage}_channel256x64x64.txt")
    traffic = tr_main + tr_phase if tr_main is not None and tr_phase is not None else None
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(el / a.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (seeded droplet packing)",
        "config": {"workload": "D3Q27 droplet channel 256x64x64, walls y, 272 droplets R=7, "
                               "body force 1e-5, NCI A=0.005 h 2..4, tau=1",
                   "lattice": "D3Q27", "nx": prm["nx"], "ny": prm["ny"], "nz": prm["nz"],
                   "fluid_nodes": fluid, "storage": a.storage,
                   "arithmetic": {"fp32": "fp32 per-direction update, fp64 moments/psi/NCI/colour fraction",
                                  "fp16": "fp32", "bf16": "fp32", "fp32_f32": "fp32"}[a.storage]},
        # the whole step (k_phase + k_main) against the per-node-update bytes
        # of the paper's two-population state read and written once plus psi
        # written and read once, timed by HIP events around the timed steps
        "roofline": {"bound": "hbm", "kernel": "step (k_phase + k_main)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "alg_bytes_per_node": b_alg, "units_per_launch": fluid,
                     "avg_ms": round(ms_step_dev, 5), "launches": a.steps,
                     "achieved_wall": round(achieved_wall, 1),
                     "frac_wall": round(achieved_wall / HBM_PEAK_GBPS, 4)},
        "step": {"k_phase_avg_ms": round(ms_phase, 5), "k_main_avg_ms": round(ms_main, 5),
                 "graphs": L.graphs, "graph_capture_ms": round(capture_ms, 2),
                 "k_main": {"layout_bytes_per_node": b_main, "achieved_GBps": round(achieved_main, 1),
                            "traffic": tr_main}},
        "copy_probe": {"GBps": round(cp["GBps"], 1), "frac_of_peak": round(cp["GBps"] / HBM_PEAK_GBPS, 4),
                       "step_frac_of_copy": round(achieved / cp["GBps"], 4)},
        "obs": {"Q": ob["Q"], "Q_d": ob["Q_d"], "umax": ob["umax"]},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def bench_oracle(a):
    """The FP64 oracle timed on the host cores on the three lattice workloads:
    the Laplace droplet (D2Q9 128 x 64, 2000 steps), the 3-D droplet channel
    (D3Q27 256 x 64 x 64: 200 steps on all OpenMP threads, and on one thread
    for ~30 s), and four channels of the batched sweep (2000 steps each).
    MLUPS count fluid nodes.  No GPU is used."""
    import subprocess
    import oracle
    import synth

    def run(case, steps):
        p = oracle.Params(**{k: v for k, v in case.params.items() if k in oracle.Params.__dataclass_fields__})
        o = oracle.Oracle(p)
        o.init_fields(case.rho1, case.rho2, case.u)
        t0 = time.perf_counter()
        o.step(steps)
        el = time.perf_counter() - t0
        fluid = p.nx * (p.ny - 2 * p.walls_y) * p.nz
        return {"nodes": fluid, "steps": steps, "seconds": round(el, 2), "MLUPS": round(fluid * steps / el / 1e6, 2)}

    out = {"metric": "oracle MLUPS (FP64, host)", "unit": "MLUPS", "cpu": host_cpu(),
           "omp_threads": int(os.environ.get("OMP_NUM_THREADS", 0)) or host_cpu()["usable_cpus"],
           "note": "lattices below 16384 nodes run on one thread"}
    out["laplace_d2q9_128x64_2000"] = run(synth.laplace_droplet(), 2000)
    out["channel_d3q27_256x64x64_200"] = run(synth.hex_channel_3d(), 200)
    code = ("import sys, json; sys.path.insert(0, %r); import bench, synth; "
            "print(json.dumps(bench._oracle_steps_for(synth.hex_channel_3d(), 30.0)))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, OMP_NUM_THREADS="1"),
                       capture_output=True, text=True, timeout=900)
    if r.returncode == 0:
        n1, el1 = json.loads(r.stdout.strip().splitlines()[-1])
        out["channel_d3q27_256x64x64_one_thread"] = {"steps": n1, "seconds": round(el1, 2),
                                                     "MLUPS": round(256 * 62 * 64 * n1 / el1 / 1e6, 3)}
    specs = synth.batch_specs(3, 64)[:4]
    out["sweep_channels_2000"] = [dict(run(synth.channel_2d(sp), 2000), Lx=sp.Lx, Ly=sp.Ly) for sp in specs]
    tot_lu = sum(c["nodes"] * c["steps"] for c in out["sweep_channels_2000"])
    tot_s = sum(c["seconds"] for c in out["sweep_channels_2000"])
    out["sweep_channels_MLUPS"] = round(tot_lu / tot_s / 1e6, 2)
    print(json.dumps(out), flush=True)
    return 0


def bench_sweep(a):
    """Batched sweep: 64 wall-bounded D2Q9 channels of uneven size (Lx 256..1024,
    Ly 64..160, hexagonal droplet packings, pressure gradient 1e-6..1e-4, NCI
    strength 0..0.05), stepped together in the mode and tile height the
    library's autotuner picks (its trial steps are real steps, taken before
    the timed region), or in a fixed mode (one persistent launch, or per-step
    batched launches).  Prints one JSON line (aggregate MLUPS over fluid
    nodes)."""
    import synth
    import paper_2003_11069_amd as P
    specs = synth.batch_specs(3, 64)
    cases = [synth.channel_2d(sp) for sp in specs]
    ps = [P.Params.from_dict(c.params, storage=P.STORAGE[a.storage]) for c in cases]
    b = P.Batch(ps)
    for k, c in enumerate(cases):
        b.init_fields(k, c.rho1, c.rho2)
    tuned = None
    if a.mode == "auto":
        tuned = b.tune(trial_steps=20)
        mode = P.LB_BATCH_AUTO
    else:
        mode = P.LB_BATCH_PERSISTENT if a.mode == "persistent" else P.LB_BATCH_LAUNCH
    fluid = sum(p.nx * (p.ny - 2) for p in ps)
    b.step(a.warmup, mode, numeric_ok=True)
    t0 = time.perf_counter()
    b.step(a.steps, mode, numeric_ok=True)  # synchronises at the end
    el = time.perf_counter() - t0
    # channels whose state went non-finite (observables evaluated after the
    # timed steps; the sweep's upper NCI range is not stable at every size)
    nonfinite = [k for k in range(len(ps)) if b.observables(k)["flags"] & 1]
    mlups = fluid * a.steps / el / 1e6
    bytes_node = main_kernel_bytes(2, a.storage) + (9 * (2 if a.storage in ("fp16", "bf16") else 4)
                                                    + (8 if a.storage == "fp32" else 4) * 3 + 8)
    out = {"metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(el / a.steps * 1e3, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32",
           "data": "synthetic (seeded channel sweep)",
           "config": {"workload": "64 D2Q9 channels, Lx 256..1024, Ly 64..160, seeded sweep",
                      "channels": len(ps), "fluid_nodes": fluid, "storage": a.storage, "mode": a.mode,
                      "tuned": tuned, "graphs": b.graphs, "nonfinite_channels": nonfinite},
           "step_bytes_per_node_measured_layout": bytes_node,
           "achieved_GBps_step": round(bytes_node * mlups * 1e6 / 1e9, 1)}
    print(json.dumps(out), flush=True)
    return 0


def bench_unet(a):
    """Training step of the warm-start U-Net (4 levels, 32 base channels,
    3 x 128 x 256 inputs and targets, batch --batch): forward, MSE, backward
    and Adam on BF16 MFMA kernels.  Prints one JSON line with the training
    throughput in TFLOP/s (2 FLOP per multiply-add of the convolutions)
    against the dense BF16 MFMA peak."""
    import synth
    from paper_2003_11069_amd import ws
    B, Hh, Ww = a.batch, 128, 256
    net = ws.UNet(ws.UNetConfig(levels=4, base=32, cin=3, cout=3, H=Hh, W=Ww, max_batch=B, conv_algo=a.conv_algo))
    net.set_params(synth.unet_params(4, 32, seed=1))
    x, t = synth.unet_batch(B, Hh, Ww, 3, 3, seed=2)
    dx, dt = ws.DeviceArray.from_host(x), ws.DeviceArray.from_host(t)
    fwd, bwd = net.flops(B)
    from paper_2003_11069_amd.lb import copy_probe
    cp = copy_probe(1 << 30, iters=3)  # the reference copy of a counter run
    for _ in range(a.warmup):
        net.train_step_ptr(dx.ptr(), dt.ptr(), B, 1e-4)
    ws.sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        net.train_step_ptr(dx.ptr(), dt.ptr(), B, 1e-4)
    ws.sync()
    el = time.perf_counter() - t0
    tflops = (fwd + bwd) * a.steps / el / 1e12
    out = {"metric": "U-Net training throughput (warm start)", "value": round(B * a.steps / el, 1),
           "unit": "samples/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": round(el / a.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded smooth fields)",
           "config": {"workload": "U-Net 4 levels, base 32, 3x128x256 -> 3x128x256, MSE + Adam",
                      "batch": B, "params": net.n_params, "gflop_per_sample_fwd": round(fwd / B / 1e9, 3),
                      "conv_algo": ["direct 3x3 where the shape allows", "implicit GEMM"][a.conv_algo]},
           "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": round(tflops / 2500.0, 4), "traffic": None},
           "copy_probe": {"GBps": round(cp["GBps"], 1)}}
    print(json.dumps(out), flush=True)
    return 0


def bench_geometry(a):
    """The 3-D benchmark channel with its wall rows given as solid nodes of a
    node-type geometry (lb_set_geometry): the GEOM kernels on the benchmark
    workload, to set their cost beside the built-in walls."""
    import numpy as np
    import synth
    import paper_2003_11069_amd as P
    case = synth.hex_channel_3d()
    prm = dict(case.params, walls_y=0)
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    t = np.zeros((nz, ny, nx), np.uint8)
    t[:, 0] = t[:, -1] = 1
    fluid = nx * (ny - 2) * nz
    L = P.Lattice(P.Params.from_dict(prm, storage=P.STORAGE[a.storage]))
    L.set_geometry(t.ravel(), case.rho1, case.rho2)
    L.init_fields(case.rho1, case.rho2)
    L.step(a.warmup)
    L.kernel_times()
    t0 = time.perf_counter()
    L.step(a.steps)
    L.kernel_times()
    el = time.perf_counter() - t0
    L.profile(True)
    L.step(min(a.steps, 500))
    kt = L.kernel_times()
    L.profile(False)
    mlups = fluid * a.steps / el / 1e6
    out = {"metric": "MLUPS with a node-type geometry", "value": round(mlups, 2), "unit": "MLUPS",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(el / a.steps * 1e3, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32",
           "data": "synthetic (seeded droplet packing)",
           "config": {"workload": "D3Q27 droplet channel 256x64x64, wall rows as solid nodes",
                      "fluid_nodes": fluid, "storage": a.storage},
           "step": {"k_phase_avg_ms": round(kt["ms_phase"] / max(kt["launches"], 1), 5),
                    "k_main_avg_ms": round(kt["ms_main"] / max(kt["launches"], 1), 5), "graphs": L.graphs}}
    print(json.dumps(out), flush=True)
    return 0


def bench_focuser(a):
    """Droplet generation in the 2-D flow-focuser (scale 2, phi 0.25):
    lattice throughput of the geometry step and the generation frequency,
    droplet volume and Q_d = nu V_d (see paper_2003_11069_amd.focuser)."""
    from paper_2003_11069_amd import focuser
    steps = max(a.steps, 40000)
    r = focuser.run(steps=steps, t_skip=min(20000, steps // 3), storage=a.storage)
    mlups = r["fluid_nodes"] * steps / r["seconds"] / 1e6
    out = {"metric": "flow-focuser droplet generation", "value": round(mlups, 2), "unit": "MLUPS",
           "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(r["seconds"] / steps * 1e3, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32",
           "data": "synthetic (flow-focuser geometry, inlet speeds)",
           "config": {"workload": f"D2Q9 flow-focuser {r['nx']}x{r['ny']}, phi {r['phi']}",
                      "storage": a.storage},
           "droplets": {k: r[k] for k in ("V_d", "nu", "Q_d", "droplets_crossed", "flux_xc_mean",
                                          "inlet_dispersed_flux", "x_c")},
           "note": "timed region includes the droplet sampling every 250 steps"}
    print(json.dumps(out), flush=True)
    return 0


def bench_analysis(a):
    """Droplet analysis and vorticity of the 3-D benchmark channel after
    --warmup steps: min(--steps, 50) calls of each, device time per call from
    events on the library's stream (FIELDS pass plus analysis kernels), and
    the host-inclusive time per call (copies of labels and tables included)."""
    import synth
    import paper_2003_11069_amd as P
    case = synth.hex_channel_3d()
    prm = case.params
    L = P.Lattice(P.Params.from_dict(prm, storage=P.STORAGE[a.storage]))
    L.init_fields(case.rho1, case.rho2, case.u)
    L.step(a.warmup)
    L.droplets()
    L.vorticity()
    n = max(1, min(a.steps, 50))
    dev_d = dev_w = 0.0
    t0 = time.perf_counter()
    for _ in range(n):
        d = L.droplets()
        dev_d += L.analysis_times()["ms_droplets"]
    t1 = time.perf_counter()
    for _ in range(n):
        L.vorticity()
        dev_w += L.analysis_times()["ms_vorticity"]
    t2 = time.perf_counter()
    N = L.N
    ms_d, ms_w = dev_d / n, dev_w / n
    out = {"metric": "droplet analysis throughput", "value": round(N / (ms_d * 1e-3) / 1e6, 1),
           "unit": "Mnodes/s", "n_gpus": 1, "steps": n, "warmup": a.warmup,
           "ms_per_step": round(ms_d, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded droplet packing)",
           "config": {"workload": "D3Q27 droplet channel 256x64x64 after the warm-up steps",
                      "nodes": N, "storage": a.storage},
           "droplets": {"count": d["count"], "dispersed": d["dispersed"], "rows": d["rows"],
                        "device_ms": round(ms_d, 4),
                        "host_ms": round((t1 - t0) / n * 1e3, 3)},
           "vorticity": {"device_ms": round(ms_w, 4), "host_ms": round((t2 - t1) / n * 1e3, 3),
                         "Mnodes_per_s": round(N / (ms_w * 1e-3) / 1e6, 1)}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
