"""GPU tests of the numeric guards: a NaN/Inf seen at a recorded step, and a
component mass drifting beyond mass_tol, surface as LB_ENUMERIC from
lb_step / lb_observables (single lattices) and from lb_batch_step (batches,
with the flagged channels named by lb_batch_flags).

The non-finite state is forced from the host with a finite but enormous body
force in a periodic box with NCI switched off (A = 0): every memory address
the kernels touch is then independent of the field values, so the NaNs only
travel through arithmetic."""
import numpy as np
import pytest

import synth
import paper_2003_11069_amd as P
from paper_2003_11069_amd.lb import LBError
from gpu_common import say

pytestmark = pytest.mark.gpu


def _box(force, **over):
    case = synth.random_fields(synth.base_params(lattice=0, nx=70, ny=30, A_nci=0.0, force=force), seed=3,
                               umax=0.0)
    p = P.Params.from_dict(case.params, **over)
    return case, p


def test_nan_surfaces_as_numeric_error():
    say("[gpu] flags: NaN from an enormous force")
    case, p = _box((1e300, 0.0, 0.0), obs_every=5)
    g = P.Lattice(p)
    g.init_fields(case.rho1, case.rho2, case.u)
    g.step(20)  # the blow-up is recorded at t = 5, 10, 15
    ob = g.observables()
    assert ob["rc"] == -4 and ob["flags"] & 1
    with pytest.raises(LBError) as e:
        g.step(1)
    assert e.value.code == -4
    # re-initialising clears the flags
    g.close()
    case2, p2 = _box((1e-6, 0.0, 0.0), obs_every=5)
    h = P.Lattice(p2)
    h.init_fields(case2.rho1, case2.rho2, case2.u)
    h.step(20)
    h.step(1)
    assert h.observables()["rc"] == 0


@pytest.mark.parametrize("storage,tol,flagged", [("fp32", 1e-6, False), ("fp16", 1e-15, True)])
def test_mass_drift_flag(storage, tol, flagged):
    """FP32 storage keeps the component masses to ~1e-12 (no flag at 1e-6);
    FP16 storage drifts by ~1e-6 over a few hundred steps (flag at 1e-15)."""
    say(f"[gpu] flags: mass drift, {storage}, tol {tol}")
    case = synth.channel_2d(synth.channel_spec(11, Lx=160, Ly=50))
    g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[storage], obs_every=10, mass_tol=tol))
    g.init_fields(case.rho1, case.rho2, case.u)
    g.step(200)
    ob = g.observables()
    say(f"  flags {ob['flags']} rc {ob['rc']}")
    assert bool(ob["flags"] & 2) == flagged and (ob["rc"] == -4) == flagged
    if flagged:
        with pytest.raises(LBError):
            g.step(1)
    else:
        g.step(1)


@pytest.mark.parametrize("mode", [P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT])
def test_batch_names_the_flagged_channel(mode):
    say(f"[gpu] flags: batch, mode {mode}")
    cases, ps = [], []
    for k, F in enumerate([1e-6, 1e300, 2e-6]):
        c, p = _box((F, 0.0, 0.0), obs_every=5)
        cases.append(c)
        ps.append(p)
    b = P.Batch(ps)
    for k, c in enumerate(cases):
        b.init_fields(k, c.rho1, c.rho2, c.u)
    with pytest.raises(LBError) as e:
        b.step(30, mode)
    assert e.value.code == -4
    assert list(np.flatnonzero(b.flags())) == [1]
    assert b.step(10, mode, numeric_ok=True) == [1]
    # the healthy channels stepped exactly like single lattices
    for k in (0, 2):
        g = P.Lattice(ps[k])
        g.init_fields(cases[k].rho1, cases[k].rho2, cases[k].u)
        g.step(40)
        for x, y in zip(b.fields(k), g.fields()):
            assert np.array_equal(x, y)
