"""GPU tests at the workloads' real sizes and over long runs.

* A dense emulsion channel whose flow rate keeps changing as droplets
  rearrange: the time-averaged flow rate of the FP32 path over 10,000 steps
  must match the FP64 oracle's within 1 %.
* The 3-D benchmark channel (256 x 64 x 64, 272 droplets): FP32 storage
  against the oracle after 200 steps at the 1e-5 bar; FP16 and BF16
  deviation storage measured against the same oracle run.
* The same channel over 10,000 steps: time-averaged Q and Q_d of the FP16 and
  BF16 paths against the FP32 path (the oracle-matched reference for runs
  the oracle cannot do in test time), and the component mass drift."""
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


@pytest.mark.parametrize("storage,tol_rho,tol_u", [("fp32", 1e-5, 1e-5), ("fp16", 2e-3, 0.2),
                                                   ("bf16", 2e-2, 1.0)])
def test_full_size_200_steps(config2_oracle_200, storage, tol_rho, tol_u):
    """FP32: the parity bar.  FP16/BF16: measured, bounds are the error budget."""
    case, o = config2_oracle_200
    g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[storage]))
    g.init_fields(case.rho1, case.rho2, case.u)
    m0 = g.observables()["mass"]
    g.step(200)
    e = field_errors(o, g, fluid_mask(case.params, case.N))
    m1 = g.observables()["mass"]
    say(f"  {storage}: {e} mass drift {(m1 - m0) / m0}")
    assert e["rho1"] <= tol_rho and e["rho2"] <= tol_rho and e["u"] <= tol_u


def test_full_size_time_averaged_flow_rate_reduced_precision():
    case = synth.hex_channel_3d()
    say("[gpu] 3-D benchmark channel, 10k steps, FP32 / FP16 / BF16")
    res = {}
    for st in ("fp32", "fp16", "bf16"):
        g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[st]))
        g.init_fields(case.rho1, case.rho2, case.u)
        m0 = g.observables()["mass"]
        q, qd = [], []
        for k in range(100):
            g.step(100)
            if k >= 19:  # from step 2000 on
                ob = g.observables()
                q.append(ob["Q"]); qd.append(ob["Q_d"])
        m1 = g.observables()["mass"]
        res[st] = (np.mean(q), np.mean(qd), (m1 - m0) / m0)
        g.close()
    for st in ("fp16", "bf16"):
        rq = abs(res[st][0] - res["fp32"][0]) / abs(res["fp32"][0])
        rqd = abs(res[st][1] - res["fp32"][1]) / abs(res["fp32"][1])
        say(f"  {st}: <Q> rel {rq:.2e}, <Q_d> rel {rqd:.2e}, mass drift {res[st][2]}")
        assert rq <= 2e-2 and rqd <= 2e-2
    say(f"  fp32: <Q> {res['fp32'][0]:.6e} <Q_d> {res['fp32'][1]:.6e} mass drift {res['fp32'][2]}")
    assert abs(res["fp32"][2][0]) <= 1e-10
