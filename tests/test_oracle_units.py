"""Pins of the FP64 oracle's single-node operators against closed forms,
hand-tabulated values and lattice identities (no GPU).

Each test names the passage of the Materials and Methods section it checks.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LATS = [oracle.D2Q9, oracle.D3Q27]


def _dim(lat):
    return 2 if lat == oracle.D2Q9 else 3


@pytest.mark.parametrize("lat", LATS)
def test_lattice_isotropy(lat):
    """D2Q9 / D3Q27 (Eq. CGLBE, b = 26): weights sum to 1, odd moments vanish,
    second moment c_s^2 delta with c_s^2 = 1/3, fourth moment isotropic."""
    c, w, opp = oracle.lattice(lat)
    Q = len(w)
    assert Q == (9 if lat == oracle.D2Q9 else 27)
    d = _dim(lat)
    cc = c[:, :d].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ cc).max() < 1e-16
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, cc, cc), np.eye(d) / 3, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, cc, cc, cc, cc)
    I = np.eye(d)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9
    np.testing.assert_allclose(m4, iso, atol=1e-16)
    assert (c[opp] == -c).all()
    # weights by speed class are the standard rationals
    sq = (c * c).sum(1)
    table = {oracle.D2Q9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36},
             oracle.D3Q27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}}[lat]
    for s, ws in table.items():
        assert np.allclose(w[sq == s], ws, rtol=0, atol=1e-17)


@pytest.mark.parametrize("lat", LATS)
def test_equilibrium_moments(lat):
    """Second-order equilibrium: zeroth, first and second moments are
    rho, rho u and rho (delta/3 + u u)."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = rng.uniform(0.2, 1.5)
        u = rng.uniform(-0.1, 0.1, d)
        E = oracle.equilibrium(lat, rho, u)
        cc = c[:, :d].astype(float)
        assert abs(E.sum() - rho) < 1e-15
        np.testing.assert_allclose(E @ cc, rho * u, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", E, cc, cc),
                                   rho * (np.eye(d) / 3 + np.outer(u, u)), atol=2e-16)


def _params(lat, **kw):
    p = oracle.Params(lattice=lat, nx=8, ny=8, nz=1 if lat == oracle.D2Q9 else 8)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("lat", LATS)
def test_exact_difference_forcing(lat):
    """Exact difference method: starting from equilibrium with no
    perturbation or recolouring, the collision adds exactly F to the
    momentum and leaves mass unchanged."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(2)
    p = _params(lat, A_s=0.0, beta=0.0, tau=0.8)
    rho1, rho2 = 0.7, 0.3
    u = rng.uniform(-0.05, 0.05, d)
    F = rng.uniform(-1e-3, 1e-3, d)
    f1 = oracle.equilibrium(lat, rho1, u)
    f2 = oracle.equilibrium(lat, rho2, u)
    o1, o2 = oracle.collide_node(p, f1, f2, np.zeros(3), F)
    cc = c[:, :d].astype(float)
    tot = o1 + o2
    assert abs(tot.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(tot @ cc, (rho1 + rho2) * u + F, atol=2e-15)


@pytest.mark.parametrize("lat", LATS)
def test_perturbation_moments(lat):
    """Perturbation (Omega2): zero mass and momentum, second moment
    (A_s/9)|G| G^ G^ (derived from the 4th-order isotropy of the lattice)."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(3)
    A_s = 0.07
    p = _params(lat, A_s=A_s, beta=0.0, tau=1.3)
    for _ in range(4):
        G = np.zeros(3)
        G[:d] = rng.normal(size=d) * 0.3
        rho, u = 1.02, rng.uniform(-0.02, 0.02, d)
        f = oracle.equilibrium(lat, rho, u)
        o1, o2 = oracle.collide_node(p, f, np.zeros_like(f), G, np.zeros(3))
        D = (o1 + o2) - f  # BGK term vanishes at equilibrium, F = 0
        cc = c[:, :d].astype(float)
        g = np.linalg.norm(G)
        Gh = G[:d] / g
        assert abs(D.sum()) < 2e-15
        assert np.abs(D @ cc).max() < 2e-15
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", D, cc, cc),
                                   A_s / 9 * g * np.outer(Gh, Gh), atol=2e-15)


KAPPA = {oracle.D2Q9: 2 / 9 + math.sqrt(2) / 18,
         oracle.D3Q27: 4 / 27 + 8 / (54 * math.sqrt(2)) + 8 / (216 * math.sqrt(3))}


@pytest.mark.parametrize("lat", LATS)
def test_recolouring(lat):
    """Recolouring (Omega3, Latva-Kokko form): component masses conserved,
    colour split sums to the total, and the colour flux differs from the
    passive share (rho1/rho) j' by beta kappa (rho1 rho2/rho) G^, with
    kappa = sum_i w_i c_ix^2/|c_i| worked by hand per lattice."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(4)
    beta = 0.6
    p = _params(lat, A_s=0.0, beta=beta, tau=1.0)  # tau = 1: f' = E(rho, u)
    for _ in range(4):
        f1 = rng.uniform(0.0, 0.1, len(w)) * w * 9
        f2 = rng.uniform(0.0, 0.1, len(w)) * w * 9
        G = np.zeros(3)
        G[:d] = rng.normal(size=d)
        o1, o2 = oracle.collide_node(p, f1, f2, G, np.zeros(3))
        r1, r2 = f1.sum(), f2.sum()
        rho = r1 + r2
        assert abs(o1.sum() - r1) < 1e-15 and abs(o2.sum() - r2) < 1e-15
        cc = c[:, :d].astype(float)
        j = (f1 + f2) @ cc
        fp = o1 + o2
        np.testing.assert_allclose(fp, oracle.equilibrium(lat, rho, j / rho), atol=2e-15)
        Gh = G[:d] / np.linalg.norm(G)
        flux = o1 @ cc - r1 / rho * (fp @ cc)
        np.testing.assert_allclose(flux, beta * KAPPA[lat] * r1 * r2 / rho * Gh, atol=1e-15)


@pytest.mark.parametrize("lat", LATS)
def test_bgk_relaxation(lat):
    """Standard relaxation (Omega1): the non-equilibrium second moment decays
    by exactly (1 - 1/tau) per collision, mass and momentum unchanged."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(5)
    tau = 0.73
    p = _params(lat, A_s=0.0, beta=0.0, tau=tau)
    f1 = w * (1 + rng.uniform(-0.1, 0.1, len(w)))
    f2 = np.zeros_like(f1)
    o1, o2 = oracle.collide_node(p, f1, f2, np.zeros(3), np.zeros(3))
    cc = c[:, :d].astype(float)
    rho = f1.sum()
    u = f1 @ cc / rho
    E = oracle.equilibrium(lat, rho, u)
    Pi = lambda f: np.einsum("i,ia,ib->ab", f, cc, cc)
    np.testing.assert_allclose(Pi(o1 + o2) - Pi(E), (1 - 1 / tau) * (Pi(f1) - Pi(E)), atol=1e-16)
    assert abs((o1 + o2).sum() - rho) < 1e-15
    np.testing.assert_allclose((o1 + o2) @ cc, rho * u, atol=1e-16)
    assert np.abs(o2).max() == 0.0  # single component stays single


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q27])
def test_two_tau_relaxation(lat):
    """Viscosity-ratio variant: with component relaxation times tau1, tau2 a
    node relaxes at the phase-weighted harmonic rate
    1/tau = (rho1/rho)/tau1 + (rho2/rho)/tau2 (mass fractions), and
    tau2 = tau1 is the single-tau collision."""
    c, w, _ = oracle.lattice(lat)
    d = _dim(lat)
    rng = np.random.default_rng(6)
    tau1, tau2 = 0.73, 1.9
    f1 = 0.3 * w * (1 + rng.uniform(-0.1, 0.1, len(w)))
    f2 = 0.7 * w * (1 + rng.uniform(-0.1, 0.1, len(w)))
    p = _params(lat, A_s=0.0, beta=0.0, tau=tau1, tau2=tau2)
    o1, o2 = oracle.collide_node(p, f1, f2, np.zeros(3), np.zeros(3))
    cc = c[:, :d].astype(float)
    f = f1 + f2
    rho = f.sum()
    u = f @ cc / rho
    E = oracle.equilibrium(lat, rho, u)
    Pi = lambda g: np.einsum("i,ia,ib->ab", g, cc, cc)
    omega = (f1.sum() / rho) / tau1 + (f2.sum() / rho) / tau2
    np.testing.assert_allclose(Pi(o1 + o2) - Pi(E), (1 - omega) * (Pi(f) - Pi(E)), atol=1e-16)
    assert abs(o1.sum() - f1.sum()) < 1e-15 and abs(o2.sum() - f2.sum()) < 1e-15
    p_same = _params(lat, A_s=0.0, beta=0.0, tau=tau1, tau2=tau1)
    p_one = _params(lat, A_s=0.0, beta=0.0, tau=tau1)
    for a, b in zip(oracle.collide_node(p_same, f1, f2, np.zeros(3), np.zeros(3)),
                    oracle.collide_node(p_one, f1, f2, np.zeros(3), np.zeros(3))):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-16)


def test_A_h_table():
    """A_h[h] against the hand-tabulated golden values (h_min=2, h_max=4)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "A_h_table.txt"))
    for h, a in tab:
        assert oracle.A_h(h, 1.0, 2.0, 4.0) == pytest.approx(a, rel=1e-15, abs=0)
    assert oracle.A_h(3.0, 0.005, 2.0, 4.0) == pytest.approx(0.005 * 8 / 27, rel=1e-15)


def _psi_box(lat, nx, ny, nz, fn):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return fn(x.astype(float), y.astype(float), z.astype(float)).ravel()


@pytest.mark.parametrize("lat", LATS)
def test_gradient_exact_on_quadratics(lat):
    """Isotropic second-order gradient G = 3 sum_i w_i c_i psi(x + c_i) is
    exact on linear and quadratic fields (central symmetric stencil)."""
    d = _dim(lat)
    nx = ny = 9
    nz = 1 if d == 2 else 9
    p = oracle.Params(lattice=lat, nx=nx, ny=ny, nz=nz, A_nci=0.0)
    a = np.array([0.3, -0.7, 0.2])
    H = np.array([[0.05, 0.01, -0.02], [0.01, -0.03, 0.04], [-0.02, 0.04, 0.02]])
    if d == 2:
        a[2] = 0
        H[2, :] = 0
        H[:, 2] = 0
    def fn(x, y, z):
        X = np.stack([x, y, z])
        return np.einsum("a...,ab,b...->...", X, H, X) + np.einsum("a,a...->...", a, X)
    psi = _psi_box(lat, nx, ny, nz, fn)
    x0 = np.array([4, 4, 4 if d == 3 else 0])
    node = x0[0] + nx * (x0[1] + ny * x0[2])
    G, hit, Fr = oracle.node_nci(p, psi, node)
    np.testing.assert_allclose(G, 2 * H @ x0 + a, atol=1e-14)


@pytest.mark.parametrize("lat", LATS)
def test_gradient_telescopes(lat):
    """For a 1-D monotone rise from -1 to +1 the central gradient telescopes:
    sum of |G| over the rise is exactly psi(+) - psi(-) = 2, so sum of
    delta_I = |G|/2 is 1 (the interface indicator of Eq. near_c has unit
    integral)."""
    d = _dim(lat)
    nx = 64
    ny = 4
    nz = 1 if d == 2 else 4
    p = oracle.Params(lattice=lat, nx=nx, ny=ny, nz=nz, A_nci=0.0)
    prof = np.full(nx, -1.0)
    prof[11:21] = np.tanh(np.linspace(-2.5, 2.5, 10)) * 0.99
    prof[21:41] = 1.0
    prof[41:51] = prof[11:21][::-1]
    psi = _psi_box(lat, nx, ny, nz, lambda x, y, z: prof[x.astype(int)])
    s = 0.0
    for x in range(0, 31):
        G, _, _ = oracle.node_nci(p, psi, x)
        s += np.linalg.norm(G)
    assert s == pytest.approx(2.0, abs=1e-14)


@pytest.mark.parametrize("lat", LATS)
def test_nci_film_golden(lat):
    """NCI probe and F_rep on hand-built 1-D films of width 1..6 against the
    hand-worked golden table."""
    d = _dim(lat)
    tab = np.loadtxt(os.path.join(GOLDEN, "nci_film.txt"))
    A = 0.01
    for w_film, h_exp, fx_exp in tab:
        w_film = int(w_film)
        nx = 40
        ny = 3
        nz = 1 if d == 2 else 3
        p = oracle.Params(lattice=lat, nx=nx, ny=ny, nz=nz, A_nci=A, h_min=2.0, h_max=4.0)
        prof = np.ones(nx)
        prof[10] = 0.0
        prof[11:11 + w_film] = -1.0
        prof[11 + w_film] = 0.0
        psi = _psi_box(lat, nx, ny, nz, lambda x, y, z: prof[x.astype(int)])
        node = 10 + nx * (1 + ny * (1 if d == 3 else 0))
        G, hit, Fr = oracle.node_nci(p, psi, node)
        assert hit == int(h_exp)
        assert Fr[0] == pytest.approx(fx_exp * A, rel=1e-14, abs=1e-18)
        assert Fr[1] == 0 and Fr[2] == 0


def test_nci_isolated_droplet_no_hit():
    """An isolated droplet has no facing interface: along the outward normal
    psi only decreases, so no interface node (|psi| < 0.9) gets a hit."""
    nx = ny = 64
    p = oracle.Params(lattice=oracle.D2Q9, nx=nx, ny=ny, nz=1, A_nci=0.01)
    psi = _psi_box(oracle.D2Q9, nx, ny, 1,
                   lambda x, y, z: np.tanh((12 - np.hypot(x - 31.3, y - 32.6)) / 2))
    n_band = 0
    for node in range(nx * ny):
        if abs(psi[node]) < 0.9:
            n_band += 1
            _, hit, Fr = oracle.node_nci(p, psi, node)
            assert hit == 0 and not Fr.any()
    assert n_band > 100


def test_nci_probe_stops_at_wall():
    """The probe does not cross a solid wall: the same column of psi gives a
    hit through the periodic boundary without walls and none with walls."""
    nx, ny = 5, 12
    prof = np.array([1.0, -1.0, -1.0, 0.0, 1, 1, 1, 1, 1, 1, 1, 1.0])
    psi = _psi_box(oracle.D2Q9, nx, ny, 1, lambda x, y, z: prof[y.astype(int)])
    node = 2 + nx * 3
    p = oracle.Params(lattice=oracle.D2Q9, nx=nx, ny=ny, nz=1, A_nci=0.01, walls_y=0)
    _, hit, _ = oracle.node_nci(p, psi, node)
    assert hit == 3  # periodic: y = 3 -> 2 -> 1 -> 0 (psi = 1 >= 0)
    p.walls_y = 1
    _, hit, Fr = oracle.node_nci(p, psi, node)
    assert hit == 0 and not Fr.any()
