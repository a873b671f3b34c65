"""Pins of the FP64 oracle's time stepping against what the model fixes:
exact conservation laws, the Navier-Stokes (Poiseuille) limit, the Laplace law
with the perturbation operator's analytic surface tension, and the qualitative
NCI behaviour (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _oracle(case):
    o = oracle.Oracle(oracle.Params(**case.params))
    o.init_fields(case.rho1, case.rho2, case.u)
    return o


@pytest.mark.parametrize("lat,walls", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_component_mass_conserved(lat, walls):
    """Continuity (Eq. cont) per component: recolouring only redistributes
    colour, streaming and bounce-back move populations, so each M_k is
    constant to round-off."""
    p = synth.base_params(lattice=lat, nx=16, ny=12, nz=1 if lat == 0 else 10, walls_y=walls,
                          A_nci=0.02, force=(1e-4, 0, 0))
    case = synth.random_fields(p, seed=7)
    if walls:
        ny, nx = p["ny"], p["nx"]
        mask = np.zeros((p["nz"], ny, nx), bool)
        mask[:, 0] = mask[:, -1] = True
        case.rho1[mask.ravel()] = 0
        case.rho2[mask.ravel()] = 0
        case.rho2[mask.ravel()] = 1  # wall-row values are ignored by the oracle
    o = _oracle(case)
    m0 = o.observables()["mass"]
    o.step(300 if lat == 0 else 60)
    m1 = o.observables()["mass"]
    np.testing.assert_allclose(m1, m0, rtol=1e-12)


@pytest.mark.parametrize("lat", [0, 1])
def test_momentum_conserved_without_force(lat):
    """Navier-Stokes (Eq. Nav_stok) with no external force in a periodic box:
    total momentum is constant, including under a Galilean boost."""
    p = synth.base_params(lattice=lat, nx=20, ny=16, nz=1 if lat == 0 else 12, A_nci=0.0)
    case = synth.random_fields(p, seed=8, umax=0.0)
    d = 2 if lat == 0 else 3
    u0 = np.array([0.01, 0.005, -0.004][:d])
    case.u = np.repeat(u0[:, None], case.N, axis=1)
    o = _oracle(case)
    P0 = o.observables()["mom"]
    np.testing.assert_allclose(P0[:d], u0 * (case.rho1 + case.rho2).sum(), rtol=1e-13)
    o.step(200 if lat == 0 else 40)
    P1 = o.observables()["mom"]
    np.testing.assert_allclose(P1, P0, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("lat", [0, 1])
def test_momentum_budget_with_forces(lat):
    """Exact difference forcing adds exactly F per collision, so in a periodic
    box sum_x j(t+1) - sum_x j(t) = sum_x F(x,t) (body force + NCI)."""
    case = synth.two_droplets_2d(nx=48, ny=32, R=7, gap=1.0, A_nci=0.03, force=(2e-5, -1e-5, 0))
    if lat == 1:
        p = synth.base_params(lattice=1, nx=24, ny=24, nz=16, A_nci=0.03, force=(2e-5, -1e-5, 3e-6))
        case = synth.random_fields(p, seed=3)
    o = _oracle(case)
    d = 2 if lat == 0 else 3
    Fb = np.array(case.params["force"][:d])
    for _ in range(3):
        diag = o.diagnostics()
        Ftot = diag["Frep"][:d].sum(1) + Fb * (o.N)
        P0 = o.observables()["mom"][:d]
        o.step(1)
        diag1 = o.diagnostics()
        Ftot1 = diag1["Frep"][:d].sum(1) + Fb * (o.N)
        P1 = o.observables()["mom"][:d]
        # P = sum (j + F/2): P(t+1) - P(t) = F(t)/2 + F(t+1)/2
        np.testing.assert_allclose(P1 - P0, 0.5 * Ftot + 0.5 * Ftot1, rtol=1e-10, atol=1e-15)
    assert np.abs(diag["Frep"]).max() > 0 or lat == 1


def test_poiseuille_profile():
    """Single-phase channel (psi = 1 everywhere, so G = 0) driven by a body
    force with half-way bounce-back walls reaches the Navier-Stokes Poiseuille
    profile u(y) = F/(2 rho nu) (y - 1/2)(ny - 3/2 - y), nu = (tau - 1/2)/3;
    its bulk second difference is exactly -F/(rho nu)."""
    tau, F, ny = 1.0, 1e-6, 34
    case = synth.poiseuille_2d(nx=4, ny=ny, force=F, tau=tau)
    o = _oracle(case)
    o.step(40000)
    r1, r2, u = o.fields()
    ux = u[0].reshape(ny, 4)[:, 0]
    nu = (tau - 0.5) / 3
    y = np.arange(ny, dtype=float)
    ua = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    fl = slice(1, ny - 1)
    umax = ua[fl].max()
    assert np.abs(ux[fl] - ua[fl]).max() <= 5e-3 * umax
    # second difference on rows y = 2 .. ny-3 (all neighbours fluid)
    d2 = ux[3:ny - 1] - 2 * ux[2:ny - 2] + ux[1:ny - 3]
    np.testing.assert_allclose(d2, -F / nu, rtol=1e-6)


def _laplace(R, tau=1.0, steps=6000):
    case = synth.laplace_droplet(R=R, tau=tau)
    o = _oracle(case)
    o.step(steps)
    r1, r2, u = o.fields()
    rho = r1 + r2
    psi = (r1 - r2) / rho
    nx, ny = case.params["nx"], case.params["ny"]
    cx, cy = case.info["centre"]
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2).ravel()
    dp = (rho[r < R - 4].mean() - rho[r > R + 4].mean()) / 3.0
    R_eff = math.sqrt(((1 + psi) / 2).sum() / math.pi)
    return dp, R_eff, case.params


def test_laplace_law_config1():
    """Augmented Young-Laplace with pi = 0 for a static 2-D droplet:
    Delta p = sigma / R, sigma = 2 A_s tau / 9 from the perturbation
    operator's second moment (Chapman-Enskog; see DESIGN readings)."""
    dp, R_eff, p = _laplace(16.0)
    sigma = 2 * p["A_s"] * p["tau"] / 9
    assert dp * R_eff == pytest.approx(sigma, rel=0.03)


@pytest.mark.slow
def test_laplace_sweep_linear():
    """Delta p is linear in 1/R with slope sigma and ~zero intercept."""
    pts = [_laplace(R, steps=8000) for R in (12.0, 16.0, 20.0)]
    iR = np.array([1 / q[1] for q in pts])
    dp = np.array([q[0] for q in pts])
    A = np.vstack([iR, np.ones_like(iR)]).T
    (sl, ic), *_ = np.linalg.lstsq(A, dp, rcond=None)
    pred = A @ np.array([sl, ic])
    r2 = 1 - ((dp - pred) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    sigma = 2 * 0.05 / 9
    assert r2 >= 0.999
    assert sl == pytest.approx(sigma, rel=0.05)
    assert abs(ic) < 0.1 * dp.min()


def test_surface_tension_scales_with_tau():
    """sigma = 2 A_s tau / 9 is linear in tau at fixed A_s."""
    s = []
    for tau in (0.8, 1.5):
        dp, R_eff, p = _laplace(16.0, tau=tau)
        s.append(dp * R_eff / (2 * p["A_s"] * tau / 9))
    assert s[0] == pytest.approx(1.0, rel=0.08) and s[1] == pytest.approx(1.0, rel=0.08)


def _n_droplets(psi2d):
    from scipy import ndimage
    lab, n = ndimage.label(psi2d > 0)
    return n


@pytest.mark.slow
def test_nci_prevents_coalescence():
    """Near-contact number N_c = A dx / sigma (dx = h_min): with A = 0 two
    droplets whose surfaces are 4 nodes apart merge (capillarity wins,
    N_c << 1); at N_c ~ 3.6 the NCI force keeps the film open."""
    nx, ny = 96, 48
    n = {}
    for A in (0.0, 0.02):
        case = synth.two_droplets_2d(nx=nx, ny=ny, R=10, gap=4.0, A_nci=A)
        o = _oracle(case)
        o.step(3000)
        r1, r2, _ = o.fields()
        n[A] = _n_droplets(((r1 - r2) / (r1 + r2)).reshape(ny, nx))
    assert n[0.0] == 1 and n[0.02] == 2


def _viscous_profile(nu_rho, F):
    """Finite-volume solution of d/dy(rho nu du/dy) = -F on the fluid rows of a
    channel with half-way walls (harmonic face averages), given rho*nu per row."""
    n = len(nu_rho)
    A = np.zeros((n, n))
    for k in range(n):
        for j in (k - 1, k + 1):
            if 0 <= j < n:
                face = 2 * nu_rho[k] * nu_rho[j] / (nu_rho[k] + nu_rho[j])
                A[k, j] += face
                A[k, k] -= face
            else:  # wall half a spacing away
                A[k, k] -= 2 * nu_rho[k]
    return np.linalg.solve(A, -F * np.ones(n))


def test_two_layer_channel_flow():
    """Viscosity-ratio variant: two stratified fluids (nu2 = 3 nu1) driven by a
    body force reach the velocity profile of the viscous momentum balance
    d/dy(nu(y) du/dy) = -F, with nu(y) from the phase-weighted relaxation
    time of each row, and the flux of the sharp two-layer solution."""
    tau1, tau2, F = 1.0, 2.0, 1e-6
    case = synth.two_layer_channel(tau1=tau1, tau2=tau2, force=F)
    p = case.params
    o = oracle.Oracle(oracle.Params(**p))
    o.init_fields(case.rho1, case.rho2)
    o.step(20000)
    r1, r2, u = o.fields()
    ny, nx = p["ny"], p["nx"]
    r1 = r1.reshape(ny, nx)[1:-1, 0]
    r2 = r2.reshape(ny, nx)[1:-1, 0]
    ux = u[0].reshape(ny, nx)[1:-1, 0]
    rho = r1 + r2
    tau = 1.0 / ((r1 / rho) / tau1 + (r2 / rho) / tau2)
    ufd = _viscous_profile(rho * (tau - 0.5) / 3.0, F)
    err = np.abs(ux - ufd).max() / ufd.max()
    # sharp interface at eta_i between walls at eta = 0 and H
    H, eta_i = ny - 2, 16.0
    n1, n2 = (tau1 - 0.5) / 3, (tau2 - 0.5) / 3
    M = np.array([[eta_i, -(eta_i - H)], [n1, -n2]])
    A1, A2 = np.linalg.solve(M, [-F / (2 * n2) * (eta_i ** 2 - H ** 2) + F / (2 * n1) * eta_i ** 2, 0.0])
    eta = np.arange(H) + 0.5
    ush = np.where(eta < eta_i, -F / (2 * n1) * eta ** 2 + A1 * eta,
                   -F / (2 * n2) * (eta ** 2 - H ** 2) + A2 * (eta - H))
    assert err <= 0.03, err
    assert ux.sum() == pytest.approx(ush.sum(), rel=0.02)
    # a single viscosity (tau1 everywhere) would carry 1.8 times this flux
    assert ux.sum() < 0.6 * F * H ** 3 / (12 * n1)
