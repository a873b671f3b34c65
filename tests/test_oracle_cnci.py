"""Pins of the oracle's continuous-NCI variant (nci_mode = 1): the contact
distance h at a closed-form crossing, agreement with the integer probe where
both sample the same nodes, continuity of F_rep under sub-lattice motion of a
film (where the integer probe jumps), the shifted A_h, and the qualitative
effect (NCI still keeps two droplets apart)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _p2(nx, ny, **kw):
    d = dict(lattice=0, nx=nx, ny=ny, nz=1, walls_y=0, A_nci=1.0, h_min=1.0, h_max=4.0)
    d.update(kw)
    return oracle.Params(**d)


def _film_1d(nx, ny, X0, k1, k2, c):
    """psi uniform in y, piecewise linear in x with its minimum c at node X0."""
    X = np.arange(nx, dtype=np.float64)
    prof = np.where(X <= X0, c + k1 * (X0 - X), c + k2 * (X - X0))
    return np.tile(prof, (ny, 1)).ravel()


@pytest.mark.parametrize("k1,k2", [(0.1, 0.25), (0.2, 0.3), (0.05, 0.4), (0.3, 0.3)])
def test_contact_distance_at_a_kinked_film(k1, k2):
    """From the node one spacing before the kink the ray runs down the left
    slope, passes the kink at distance 1 and climbs the right slope; psi is
    back at its starting level at distance 1 + k1/k2 (geometry of the
    piecewise-linear profile, which linear interpolation reproduces)."""
    nx, ny, X0 = 24, 4, 11
    psi = _film_1d(nx, ny, X0, k1, k2, -0.6)
    node = (X0 - 1) + nx * 2
    p = _p2(nx, ny, nci_mode=1)
    G, hit, Fr = oracle.node_nci(p, psi, node)
    # gradient of the left slope: G_x = 3 (w_1 + 2 w_2)(psi(x+1) - psi(x-1)) = -k1
    assert G[0] == pytest.approx(-k1, rel=1e-12) and abs(G[1]) < 1e-15
    h = 1.0 + k1 / k2
    Ah = oracle.A_h_shifted(h, 1.0, 1.0, 4.0)
    assert hit == 2
    assert Fr[0] == pytest.approx(-Ah * 0.5 * k1, rel=1e-12) and abs(Fr[1]) < 1e-15
    # the integer probe samples the same nodes here and reports step 2
    _, hit_r, _ = oracle.node_nci(_p2(nx, ny, nci_mode=0), psi, node)
    assert hit_r == 2


def test_axis_aligned_probe_agrees_with_the_integer_probe():
    """Along a lattice axis the interpolated samples are node values, so the
    step at which psi comes back equals the integer probe's hit."""
    rng = np.random.default_rng(3)
    nx, ny = 20, 3
    for _ in range(200):
        prof = np.tanh(2.0 * rng.uniform(-1, 1, nx))
        psi = np.tile(prof, (ny, 1)).ravel()
        node = int(rng.integers(0, nx)) + nx
        _, h1, F1 = oracle.node_nci(_p2(nx, ny, nci_mode=1), psi, node)
        _, h0, F0 = oracle.node_nci(_p2(nx, ny, nci_mode=0), psi, node)
        assert h1 == h0
        assert (np.abs(F1).max() == 0) == (np.abs(F0).max() == 0)


@pytest.mark.parametrize("angle", [0.0, 0.5, 0.9])
def test_force_is_continuous_in_the_film_position(angle):
    """A film of continuous phase between two dispersed regions, moved across
    the lattice in steps of 1/2000 of a spacing (direction at `angle` rad):
    the variant's F_rep at a fixed node changes by a small amount per step,
    the integer probe's jumps."""
    nx = ny = 24
    e = np.array([math.cos(angle), math.sin(angle)])
    Y, X = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    node = 10 + nx * 12
    out = {0: [], 1: []}
    for d in np.arange(0.0, 2.0, 0.0005):
        xi = (X - 10) * e[0] + (Y - 12) * e[1] - 1.3 - d  # film centred 1.3 + d ahead
        psi = np.maximum(np.tanh(1.2 * (np.abs(xi) - 1.0)), -1.0).ravel()
        for mode in (0, 1):
            _, _, Fr = oracle.node_nci(_p2(nx, ny, nci_mode=mode, A_nci=0.01, h_min=2.0), psi, node)
            out[mode].append(Fr[:2].copy())
    for mode in (0, 1):
        F = np.array(out[mode])
        jump = np.abs(np.diff(F, axis=0)).max()
        scale = np.abs(F).max()
        assert scale > 0
        if mode == 1:
            assert jump <= 0.02 * scale, (jump, scale)
        else:
            assert jump >= 0.05 * scale, (jump, scale)


def test_shifted_strength():
    A, hmin, hmax = 0.3, 2.0, 4.0
    assert oracle.A_h_shifted(1.0, A, hmin, hmax) == A
    assert oracle.A_h_shifted(hmin, A, hmin, hmax) == A
    assert oracle.A_h_shifted(hmin + 1e-9, A, hmin, hmax) == pytest.approx(A, rel=1e-8)
    assert oracle.A_h_shifted(hmax, A, hmin, hmax) == 0.0
    assert oracle.A_h_shifted(hmax - 1e-9, A, hmin, hmax) == pytest.approx(0.0, abs=1e-9)
    assert oracle.A_h_shifted(hmax + 0.1, A, hmin, hmax) == 0.0
    # strictly decreasing in between, and equal to the unshifted form minus a
    # constant, rescaled: A_h(h) = (A (hmin/h)^3 - A/8) / (7/8) for hmin/hmax = 1/2
    for h in (2.2, 2.9, 3.5):
        assert oracle.A_h_shifted(h, A, hmin, hmax) == pytest.approx(
            (oracle.A_h(h, A, hmin, hmax) - A / 8) / (7 / 8), rel=1e-12)
    # degenerate range: a step
    assert oracle.A_h_shifted(2.0, A, 2.0, 2.0) == A and oracle.A_h_shifted(2.1, A, 2.0, 2.0) == 0.0


def test_variant_keeps_droplets_apart():
    """As the integer probe (N_c ~ 3.6): two droplets 4 nodes apart stay
    separate; without NCI they merge (physics test of the same setup)."""
    nx, ny = 96, 48
    case = synth.two_droplets_2d(nx=nx, ny=ny, R=10, gap=4.0, A_nci=0.02)
    o = oracle.Oracle(oracle.Params(**case.params, nci_mode=1))
    o.init_fields(case.rho1, case.rho2)
    o.step(3000)
    r1, r2, _ = o.fields()
    from oracle import analysis as A
    m = A.dispersed_mask(r1, r2, nx, ny, 1, 0)
    _, n = A.components(m, (True, True, True))
    assert n == 2
