"""Pins of the oracle's density-ratio variant (rho_ratio = gamma > 0): the
component equilibrium's moments (closed form, both lattices), the reduction to
the equal-density model, exact conservation in a closed box, a uniform flow
as an exact steady state, and the pressure balance across a flat interface
(p_k = c_k^2 rho_k equal on both sides) reached from unbalanced densities."""
import numpy as np
import pytest

import oracle
import synth

W0 = {0: 4 / 9, 1: 8 / 27}


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("alpha", [0.2, 0.6, 0.85])
def test_component_equilibrium_moments(lat, alpha):
    c, w, _ = oracle.lattice(lat)
    rho = 0.7
    u = np.array([0.03, -0.02, 0.01 if lat == 1 else 0.0])
    e = oracle.equilibrium_k(lat, alpha, rho, u)
    cs2 = (1 - alpha) / (3 * (1 - W0[lat]))
    assert e.sum() == pytest.approx(rho, abs=1e-15)
    np.testing.assert_allclose(c.T @ e, rho * u, atol=1e-15)
    P = (c.T * e) @ c
    d = 2 if lat == 0 else 3
    np.testing.assert_allclose(P[:d, :d], rho * (cs2 * np.eye(d) + np.outer(u[:d], u[:d])), atol=1e-15)
    # the equal-density equilibrium is the case alpha = w_0
    np.testing.assert_allclose(oracle.equilibrium_k(lat, W0[lat], rho, u), oracle.equilibrium(lat, rho, u),
                               atol=1e-16)


def test_reduces_to_equal_densities():
    case = synth.two_droplets_2d(nx=64, ny=40, R=8, gap=3.0, jitter=0.4, seed=3, A_nci=0.01)
    a = oracle.Oracle(oracle.Params(**case.params))
    b = oracle.Oracle(oracle.Params(**case.params, rho_ratio=1.0, alpha1=4 / 9))
    for o in (a, b):
        o.init_fields(case.rho1, case.rho2)
        o.step(200)
    fa, fb = a.get_populations(), b.get_populations()
    assert max(np.abs(fa[0] - fb[0]).max(), np.abs(fa[1] - fb[1]).max()) <= 1e-13


def _slab(nx, ny, gamma, r1_in, r2_out, width):
    X = np.arange(nx)
    psi = np.tanh((width / 2 - np.abs(X - nx / 2)) / 2.0)
    psi = np.tile(psi, (ny, 1)).ravel()
    return r1_in * (1 + psi) / 2, r2_out * (1 - psi) / 2


@pytest.mark.parametrize("lat,gamma,alpha1", [(0, 2.0, 0.8), (0, 4.0, 0.9), (1, 3.0, 0.85)])
def test_closed_box_conserves_mass_and_momentum(lat, gamma, alpha1):
    p = synth.base_params(lattice=lat, nx=40, ny=24, nz=6 if lat else 1, A_nci=0.0)  # F_rep is external
    case = synth.random_fields(p, seed=2)
    o = oracle.Oracle(oracle.Params(**p, rho_ratio=gamma, alpha1=alpha1))
    o.init_fields(case.rho1, case.rho2 / gamma, case.u)
    ob0 = o.observables()
    o.step(300)
    ob1 = o.observables()
    np.testing.assert_allclose(ob1["mass"], ob0["mass"], rtol=1e-13)
    np.testing.assert_allclose(ob1["mom"], ob0["mom"], atol=1e-12)


@pytest.mark.parametrize("alpha,rho", [(0.8, 1.0), (0.6, 0.25)])
def test_uniform_flow_is_steady(alpha, rho):
    """One component at rest fraction alpha, uniform density and velocity."""
    nx, ny = 12, 8
    gamma = (1 - 0.6) / (1 - 0.8)
    p = synth.base_params(nx=nx, ny=ny, A_nci=0.0)
    o = oracle.Oracle(oracle.Params(**p, rho_ratio=gamma, alpha1=0.8))
    N = nx * ny
    u = np.zeros((2, N)); u[0] = 0.02; u[1] = 0.01
    comp1 = alpha == 0.8
    r1 = np.full(N, rho if comp1 else 0.0)
    r2 = np.full(N, 0.0 if comp1 else rho)
    o.init_fields(r1, r2, u)
    o.step(100)
    f1, f2 = o.get_populations()
    e = oracle.equilibrium_k(0, alpha, rho, (0.02, 0.01))
    f = f1 if comp1 else f2
    assert np.abs(f - e[:, None]).max() <= 1e-15


@pytest.mark.parametrize("gamma,alpha1", [(2.0, 0.8), (4.0, 0.9)])
def test_flat_interface_pressure_balance(gamma, alpha1):
    """A slab of component 1 in component 2, both started at density 1: the
    closed box relaxes (the slab's width adjusts) until the bulk pressures
    c_1^2 rho_1 and c_2^2 rho_2 agree, i.e. rho_1/rho_2 -> gamma."""
    nx, ny = 96, 4
    p = synth.base_params(nx=nx, ny=ny, A_nci=0.0)
    o = oracle.Oracle(oracle.Params(**p, rho_ratio=gamma, alpha1=alpha1))
    r1, r2 = _slab(nx, ny, gamma, 1.0, 1.0, 40)
    o.init_fields(r1, r2)
    o.step(20000)
    f1, f2, u = o.fields()
    a2 = 1 - gamma * (1 - alpha1)
    cs1, cs2 = (1 - alpha1) * 3 / 5, (1 - a2) * 3 / 5
    rho1_bulk = f1.reshape(ny, nx)[:, nx // 2].mean()
    rho2_bulk = f2.reshape(ny, nx)[:, 2].mean()
    assert cs1 * rho1_bulk == pytest.approx(cs2 * rho2_bulk, rel=1e-3)
    assert rho1_bulk / rho2_bulk == pytest.approx(gamma, rel=1e-3)
    assert np.abs(u).max() < 1e-4
