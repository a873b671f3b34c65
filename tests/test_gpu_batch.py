"""GPU tests of batched stepping (lb_batch_*): many independent channels of
uneven size stepped by per-step batched launches (hipGraph) or by one
persistent launch with per-channel barriers.

Each channel must evolve exactly as the same lattice stepped alone (the tile
kernels are shared, so fields agree bit for bit), one channel is checked
against the FP64 oracle, and converged channels retire independently."""
import numpy as np
import pytest

import oracle
import synth
import paper_2003_11069_amd as P
from gpu_common import say, fluid_mask, field_errors

pytestmark = pytest.mark.gpu


def _specs():
    sizes = [(96, 20), (130, 37), (64, 50), (200, 24), (70, 33)]
    out = []
    for k, (lx, ly) in enumerate(sizes):
        spec = synth.channel_spec(100 + k, Lx=lx, Ly=ly)
        spec.R = 6.0 + k  # droplets that fit these short channels
        out.append(synth.channel_2d(spec))
    return out


CASES = _specs()


def _batch(cases, **over):
    ps = [P.Params.from_dict(c.params, **over) for c in cases]
    b = P.Batch(ps)
    for k, c in enumerate(cases):
        b.init_fields(k, c.rho1, c.rho2)
    return b, ps


@pytest.mark.parametrize("mode", [P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT])
def test_batch_matches_single_lattices(mode):
    say(f"[gpu] batch vs single, mode {mode}")
    b, ps = _batch(CASES)
    b.step(60, mode)
    b.step(41, mode)
    for k, c in enumerate(CASES):
        g = P.Lattice(ps[k])
        g.init_fields(c.rho1, c.rho2)
        g.step(101)
        assert b.info(k)["steps"] == 101
        fb = b.fields(k)
        fs = g.fields()
        for x, y in zip(fb, fs):
            assert np.array_equal(x, y), f"channel {k}"
    say(f"  graphs used: {b.graphs}")


def test_batch_channel_against_oracle():
    say("[gpu] batch channel vs oracle")
    b, ps = _batch(CASES)
    b.step(200, P.LB_BATCH_PERSISTENT)
    k = 1
    c = CASES[k]
    o = oracle.Oracle(oracle.Params(**c.params))
    o.init_fields(c.rho1, c.rho2)
    o.step(200)
    r1o, r2o, uo = o.fields()
    r1g, r2g, ug = b.fields(k)
    m = fluid_mask(c.params, c.N)
    e1 = np.abs(r1g - r1o)[m].max() / np.abs(r1o[m]).max()
    eu = np.abs(ug - uo)[:, m].max() / np.abs(uo[:, m]).max()
    say(f"  rho1 {e1:.2e} u {eu:.2e}")
    assert e1 <= 1e-5 and eu <= 1e-5


@pytest.mark.parametrize("mode", [P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT])
def test_batch_retirement(mode):
    """Single-phase channels of different heights reach the windowed flow-rate
    criterion at different times; each stops stepping on its own."""
    say(f"[gpu] batch retirement, mode {mode}")
    cases = [synth.poiseuille_2d(nx=16, ny=ny, force=1e-6) for ny in (12, 20, 34)]
    ps = [P.Params.from_dict(c.params, obs_every=5, conv_window=20, conv_m=3, conv_eps=1e-7)
          for c in cases]
    b = P.Batch(ps)
    for k, c in enumerate(cases):
        b.init_fields(k, c.rho1, c.rho2)
    for _ in range(30):
        b.step(2000, mode)
        if not any(b.info(k)["active"] for k in range(3)):
            break
    steps = [b.info(k)["steps"] for k in range(3)]
    say(f"  steps at retirement {steps}")
    assert not any(b.info(k)["active"] for k in range(3))
    assert steps[0] < steps[1] < steps[2]
    # a retired channel no longer changes
    before = b.fields(0)
    b.step(100, mode)
    after = b.fields(0)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    for k, c in enumerate(cases):
        ob = b.observables(k)
        assert ob["converged"]
        H = c.params["ny"] - 2
        nu = 0.5 / 3
        # flux of the discrete parabola over the H fluid rows (midpoint sum)
        q = 1e-6 * H ** 3 / (12 * nu) * (1 + 1 / (2 * H * H))
        assert ob["Q_window"] == pytest.approx(q, rel=1e-2)


def test_batch_tuner(tmp_path):
    """The autotuner's trial steps are real steps: after tuning, every channel
    equals a single lattice advanced by the same number of steps; the choice
    is cached per shape signature and reused."""
    say("[gpu] batch tuner")
    b, ps = _batch(CASES)
    cache = str(tmp_path / "tune.json")
    cfg = b.tune(trial_steps=4, cache=cache)
    say(f"  chosen {cfg}")
    b.step(10, P.LB_BATCH_AUTO)
    for k, c in enumerate(CASES):
        n = b.info(k)["steps"]
        g = P.Lattice(ps[k])
        g.init_fields(c.rho1, c.rho2)
        g.step(n)
        for x, y in zip(b.fields(k), g.fields()):
            assert np.array_equal(x, y), f"channel {k}"
    b2, _ = _batch(CASES)
    cfg2 = b2.tune(trial_steps=4, cache=cache)
    assert cfg2["cached"] and cfg2["mode"] == cfg["mode"] and cfg2["main_by"] == cfg["main_by"]


def test_sweep_full_size_sampled_channels():
    """The 64-channel sweep itself (Lx 256..1024, Ly 64..160): both batch
    modes step all channels 200 steps; they agree bit for bit, and the
    largest and the smallest channel match the FP64 oracle at the 1e-5 bar."""
    say("[gpu] full sweep, 64 channels, 200 steps")
    specs = synth.batch_specs(3, 64)
    cases = [synth.channel_2d(sp) for sp in specs]
    sizes = [c.params["nx"] * c.params["ny"] for c in cases]
    picks = [int(np.argmax(sizes)), int(np.argmin(sizes))]
    fields = {}
    for mode in (P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT):
        b, _ = _batch(cases)
        b.step(200, mode)
        fields[mode] = [b.fields(k) for k in picks]
        b.close()
    for fa, fb in zip(fields[P.LB_BATCH_LAUNCH], fields[P.LB_BATCH_PERSISTENT]):
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)
    for k, (r1g, r2g, ug) in zip(picks, fields[P.LB_BATCH_LAUNCH]):
        c = cases[k]
        o = oracle.Oracle(oracle.Params(**c.params))
        o.init_fields(c.rho1, c.rho2)
        o.step(200)
        r1o, r2o, uo = o.fields()
        m = fluid_mask(c.params, c.N)
        e1 = np.abs(r1g - r1o)[m].max() / np.abs(r1o[m]).max()
        e2 = np.abs(r2g - r2o)[m].max() / np.abs(r2o[m]).max()
        eu = np.abs(ug - uo)[:, m].max() / np.abs(uo[:, m]).max()
        say(f"  channel {k} {c.params['nx']}x{c.params['ny']}: rho1 {e1:.2e} rho2 {e2:.2e} u {eu:.2e}")
        assert e1 <= 1e-5 and e2 <= 1e-5 and eu <= 1e-5


# D3Q27 channels of uneven size (ragged tiles in every direction), walls in
# y or fully periodic, NCI active: the 3-D batch kernels (launch and
# persistent) against single lattices and the oracle
CASES_3D = [synth.random_fields(synth.base_params(lattice=1, nx=nx, ny=ny, nz=nz, walls_y=w, A_nci=0.01),
                                seed=30 + k)
            for k, (nx, ny, nz, w) in enumerate([(70, 21, 9, 1), (96, 13, 6, 0), (40, 30, 11, 1)])]


@pytest.mark.parametrize("mode", [P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT])
def test_batch_3d_matches_single_lattices(mode):
    say(f"[gpu] 3-D batch vs single, mode {mode}")
    b, ps = _batch(CASES_3D)
    b.step(23, mode)
    b.step(14, mode)
    for k, c in enumerate(CASES_3D):
        g = P.Lattice(ps[k])
        g.init_fields(c.rho1, c.rho2)
        g.step(37)
        for x, y in zip(b.fields(k), g.fields()):
            assert np.array_equal(x, y), f"channel {k}"


def test_batch_3d_channel_against_oracle():
    say("[gpu] 3-D batch channel vs oracle")
    b, ps = _batch(CASES_3D)
    b.step(100, P.LB_BATCH_PERSISTENT)
    for k in (0, 1):
        c = CASES_3D[k]
        o = oracle.Oracle(oracle.Params(**c.params))
        o.init_fields(c.rho1, c.rho2)
        o.step(100)
        r1o, r2o, uo = o.fields()
        r1g, r2g, ug = b.fields(k)
        m = fluid_mask(c.params, c.N)
        e1 = np.abs(r1g - r1o)[m].max() / np.abs(r1o[m]).max()
        e2 = np.abs(r2g - r2o)[m].max() / np.abs(r2o[m]).max()
        eu = np.abs(ug - uo)[:, m].max() / np.abs(uo[:, m]).max()
        say(f"  channel {k}: rho1 {e1:.2e} rho2 {e2:.2e} u {eu:.2e}")
        assert e1 <= 1e-5 and e2 <= 1e-5 and eu <= 1e-5


@pytest.mark.parametrize("mode", [P.LB_BATCH_LAUNCH, P.LB_BATCH_PERSISTENT])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_batch_16bit_matches_single_lattices(storage, dim, mode):
    """16-bit deviation storage: batched channels equal single lattices."""
    cases = CASES[:3] if dim == 2 else CASES_3D
    say(f"[gpu] {storage} batch vs single, {dim}-D, mode {mode}")
    b, ps = _batch(cases, storage=P.STORAGE[storage])
    b.step(29, mode)
    for k, c in enumerate(cases):
        g = P.Lattice(ps[k])
        g.init_fields(c.rho1, c.rho2)
        g.step(29)
        for x, y in zip(b.fields(k), g.fields()):
            assert np.array_equal(x, y), f"channel {k}"
