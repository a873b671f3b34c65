"""GPU tests at the workloads' real sizes and over long runs.

* A dense emulsion channel whose flow rate keeps changing as droplets
  rearrange: the time-averaged flow rate of the FP32 path over 10,000 steps
  must match the FP64 oracle's within 1 %.
* The 3-D benchmark channel (256 x 64 x 64, 272 droplets): FP32 storage
  against the oracle after 200 steps at the 1e-5 bar; FP16 and BF16
  deviation storage against the same oracle run, within their stated error
  budgets.
* The same channel over 10,000 steps: time-averaged Q and Q_d over steps
  5,000-10,000 of the FP32, FP16 and BF16 paths against the FP64 oracle's
  (stored in tests/golden/channel3d_long.json by the oracle-only script
  tests/golden/make_channel3d_long.py), and the component mass drift."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
import paper_2003_11069_amd as P
from gpu_common import say, make_pair, fluid_mask, field_errors

pytestmark = pytest.mark.gpu


def _emulsion_case():
    spec = synth.channel_spec(11, Lx=160, Ly=64)
    spec.R = 9.0
    spec.A_nci = 0.01
    return synth.channel_2d(spec)


def test_long_run_time_averaged_flow_rate():
    case = _emulsion_case()
    say("[gpu] long run 10k steps, D2Q9 160x64 emulsion channel")
    o, g = make_pair(case)
    qo, qg, qdo, qdg = [], [], [], []
    for k in range(200):
        o.step(50)
        g.step(50)
        if k >= 79:  # from step 4000 on
            ob, gb = o.observables(), g.observables()
            qo.append(ob["Q"]); qg.append(gb["Q"])
            qdo.append(ob["Q_d"]); qdg.append(gb["Q_d"])
    qo, qg = np.array(qo), np.array(qg)
    rel = abs(qg.mean() - qo.mean()) / abs(qo.mean())
    rel_d = abs(np.mean(qdg) - np.mean(qdo)) / abs(np.mean(qdo))
    inst = np.abs(qg - qo).max() / np.abs(qo).max()
    say(f"  <Q> gpu {qg.mean():.6e} oracle {qo.mean():.6e} rel {rel:.2e}; <Q_d> rel {rel_d:.2e}; "
        f"max instantaneous rel {inst:.2e}; Q range {qo.min():.4e}..{qo.max():.4e}")
    assert qo.max() - qo.min() > 1e-3 * abs(qo.mean())  # the flow rate does change
    assert rel <= 1e-2 and rel_d <= 1e-2


@pytest.fixture(scope="module")
def config2_oracle_200():
    case = synth.hex_channel_3d()
    say("[gpu] oracle: 3-D benchmark channel, 200 steps (host, FP64)")
    o = oracle.Oracle(oracle.Params(**{k: v for k, v in case.params.items()
                                       if k in oracle.Params.__dataclass_fields__}))
    o.init_fields(case.rho1, case.rho2, case.u)
    o.step(200)
    return case, o


# error budgets of the 16-bit paths: about three times the errors measured
# on this workload (FP16: rho 1.4e-5, u 1.1e-3; BF16: rho 6.4e-5, u 2.1e-2)
@pytest.mark.parametrize("storage,tol_rho,tol_u", [("fp32", 1e-5, 1e-5), ("fp16", 4.2e-5, 3.3e-3),
                                                   ("bf16", 2e-4, 6.3e-2)])
def test_full_size_200_steps(config2_oracle_200, storage, tol_rho, tol_u):
    """FP32: the parity bar.  FP16/BF16: within the stated error budget."""
    case, o = config2_oracle_200
    g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[storage]))
    g.init_fields(case.rho1, case.rho2, case.u)
    m0 = g.observables()["mass"]
    g.step(200)
    e = field_errors(o, g, fluid_mask(case.params, case.N))
    m1 = g.observables()["mass"]
    say(f"  {storage}: {e} mass drift {(m1 - m0) / m0}")
    assert e["rho1"] <= tol_rho and e["rho2"] <= tol_rho and e["u"] <= tol_u


GOLD_LONG = os.path.join(os.path.dirname(__file__), "golden", "channel3d_long.json")

# budgets for the time-averaged flow rates against the oracle over steps
# 5,000-10,000: the 1 % bar for FP32 (measured 8.8e-9); 16-bit storage within
# about three times its measured error (FP16 3.3e-4, BF16 1.7e-2)
LONG_TOL = {"fp32": 1e-2, "fp16": 1e-3, "bf16": 5.2e-2}


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_full_size_time_averaged_flow_rate_vs_oracle(storage):
    ref = json.load(open(GOLD_LONG))
    case = synth.hex_channel_3d()
    say(f"[gpu] 3-D benchmark channel, 10k steps, {storage}, vs the oracle's stored flow rates")
    g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[storage]))
    g.init_fields(case.rho1, case.rho2, case.u)
    m0 = g.observables()["mass"]
    g.step(ref["t0"])
    q, qd = [], []
    while True:
        ob = g.observables()
        q.append(ob["Q"]); qd.append(ob["Q_d"])
        if g.t >= ref["t1"]:
            break
        g.step(ref["every"])
    m1 = g.observables()["mass"]
    assert len(q) == len(ref["Q"])
    rq = abs(np.mean(q) - ref["Q_mean"]) / abs(ref["Q_mean"])
    rqd = abs(np.mean(qd) - ref["Q_d_mean"]) / abs(ref["Q_d_mean"])
    inst = np.abs(np.array(q) - np.array(ref["Q"])).max() / np.abs(ref["Q"]).max()
    drift = (m1 - m0) / m0
    say(f"  {storage}: <Q> {np.mean(q):.6e} oracle {ref['Q_mean']:.6e} rel {rq:.2e}; <Q_d> rel {rqd:.2e}; "
        f"max instantaneous rel {inst:.2e}; mass drift {drift}")
    assert rq <= LONG_TOL[storage] and rqd <= LONG_TOL[storage]
    if storage == "fp32":
        assert abs(drift[0]) <= 1e-10
    else:
        assert np.abs(drift).max() <= 2e-4
