"""Host-side logic of the learned warm start (CPU only): network inputs and
targets, the mass-preserving initialisation from a prediction, the
augmentation symmetries, and the steps-to-steady metric."""
import math

import numpy as np
import pytest

from paper_2003_11069_amd import warmstart as wsm


@pytest.fixture(scope="module")
def case():
    return wsm.make_case(1000)


def _fluid():
    f = np.zeros((wsm.H, wsm.W), bool)
    f[1:-1] = True
    return f.ravel()


def test_inputs_and_targets(case):
    spec, c = case
    x = wsm.net_input(spec, c)
    assert x.shape == (wsm.H, wsm.W, 3) and x.dtype == np.float32
    assert np.all(x[0, :, 0] == -1) and np.all(x[-1, :, 0] == -1)
    assert -1 <= x[..., 0].min() and x[..., 0].max() <= 1
    assert x[0, 0, 1] == pytest.approx(math.log10(spec.G_p) + 5, rel=1e-6)
    assert x[0, 0, 2] == pytest.approx(spec.A_nci / 0.025 - 1, rel=1e-6)
    # Poiseuille reference speed of the fluid rows
    nu = (spec.tau - 0.5) / 3
    assert wsm.u_ref(spec) == pytest.approx(spec.G_p * 126 ** 2 / (8 * nu))
    u = np.zeros((2, wsm.H * wsm.W))
    u[0] = 0.5 * wsm.u_ref(spec)
    t = wsm.net_target(spec, c.rho1, c.rho2, u)
    assert np.allclose(t[1:-1, :, 1], 0.5) and np.all(t[0] == [-1, 0, 0])
    assert np.allclose(t[1:-1, :, 0], x[1:-1, :, 0], atol=1e-6)


@pytest.mark.parametrize("shift", [-0.4, 0.0, 0.3])
def test_warm_init_preserves_both_masses(case, shift):
    spec, c = case
    rng = np.random.default_rng(1)
    pred = np.zeros((wsm.H, wsm.W, 3), np.float32)
    pred[..., 0] = wsm.net_input(spec, c)[..., 0] + shift + 0.3 * rng.normal(size=(wsm.H, wsm.W))
    pred[..., 1] = 3.0 * rng.uniform(-1, 1, (wsm.H, wsm.W))  # partly beyond the clip
    r1, r2, u = wsm.init_from_prediction(spec, c, pred)
    f = _fluid()
    assert r1[f].sum() == pytest.approx(c.rho1[f].sum(), rel=1e-13)
    assert r2[f].sum() == pytest.approx(c.rho2[f].sum(), rel=1e-12)
    assert np.all(r1[f] >= 0) and np.all(r2[f] >= 0)
    assert np.allclose(r1[f] + r2[f], 1.0)
    assert np.all(r1[~f] == 0) and np.all(u[:, ~f] == 0)
    assert np.abs(u).max() <= wsm.U_CLIP * wsm.u_ref(spec) * (1 + 1e-12)


def test_ablation_variants_and_nan_guard(case):
    spec, c = case
    pred = np.full((wsm.H, wsm.W, 3), np.nan, np.float32)
    r1, r2, u = wsm.init_from_prediction(spec, c, pred, phase=False, velocity=True)
    assert np.array_equal(r1, c.rho1) and np.array_equal(r2, c.rho2) and np.all(u == 0)
    r1, r2, u = wsm.init_from_prediction(spec, c, np.zeros((wsm.H, wsm.W, 3), np.float32),
                                         phase=True, velocity=False)
    assert u is None and np.all(np.isfinite(r1))


def test_augmentation_is_a_symmetry_map():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(6, wsm.H, wsm.W, 3)).astype(np.float32)
    T = rng.normal(size=(6, wsm.H, wsm.W, 3)).astype(np.float32)
    X2, T2 = wsm.augment(X, T, np.random.default_rng(5))
    for i in range(6):
        # each sample is a periodic x-shift, possibly composed with a y-mirror
        # that flips the sign of u_y only
        found = False
        for flip in (False, True):
            x, t = X[i], T[i].copy()
            if flip:
                x, t = x[::-1], t[::-1].copy()
                t[..., 2] *= -1
            for s in range(wsm.W):
                if np.array_equal(np.roll(x, s, axis=1), X2[i]):
                    assert np.array_equal(np.roll(t, s, axis=1), T2[i])
                    found = True
                    break
            if found:
                break
        assert found


def test_steps_to_steady_metric():
    h = [(500, 1.0), (1000, 0.5), (1500, 0.995), (2000, 1.02), (2500, 1.004), (3000, 0.999)]
    assert wsm.t_within(h, 1.0) == 2500
    assert wsm.t_within(h[:4], 1.0) is None
    assert wsm.t_within([(500, 1.0)], 1.0) == 500
    assert wsm.t_within(h, 1.0, tol=0.03) == 1500
    assert wsm.q_ref_of(h, last=2) == pytest.approx((1.004 + 0.999) / 2)
    assert wsm.q_final(h, last=1) == 0.999
