"""Pins of the oracle's oblique NCI probe and of its observables (no GPU).

* The R-NCI probe on oblique normals against the hand-worked golden table
  tests/golden/nci_oblique.txt (Materials and Methods, Eq. near_c): normals
  at 45 degrees and atan(1/2) in 2-D, two diagonal directions in 3-D, the
  negative quadrant, the >= tie of the psi comparison, and an exact rounding
  tie of s*n at 0.5, which fixes the round-half-away-from-zero rule.
* The observables (mass, momentum, flow rate Q, dispersed flow rate Q_d,
  umax; the flow rate is the paper's observable, Results / Fig. 3) against
  closed forms: a uniformly forced periodic box, where exact-difference
  forcing makes the momentum grow by exactly F per step and the physical
  velocity is (t + 1/2) F / rho; the Poiseuille flux of a wall-bounded
  channel; the sharp split of a two-layer channel's flux.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oblique_cases():
    cases = []
    for line in open(os.path.join(GOLDEN, "nci_oblique.txt")):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        name, lat, ramp, over, h, ah, fr = [f.strip() for f in line.split("|")]
        ovr = []
        for tok in over.split():
            d, v = tok.split("=")
            ovr.append((tuple(int(x) for x in d.split(",")), float(v)))
        cases.append(dict(name=name, lat=int(lat), ramp=[int(x) for x in ramp.split()], over=ovr,
                          h=int(h), ah=float(ah), F=[float(x) for x in fr.split()]))
    return cases


OBLIQUE = _oblique_cases()


def _oblique_field(case):
    d3 = case["lat"] == 1
    L = 16
    nz = L if d3 else 1
    z, y, x = np.meshgrid(np.arange(nz), np.arange(L), np.arange(L), indexing="ij")
    x0 = (8, 8, 8 if d3 else 0)
    a, b, c = case["ramp"]
    psi = -(a * (x - x0[0]) + b * (y - x0[1]) + c * (z - x0[2])) / 8.0
    for (dx, dy, dz), v in case["over"]:
        psi[x0[2] + dz, x0[1] + dy, x0[0] + dx] = v
    node = x0[0] + L * (x0[1] + L * x0[2])
    p = oracle.Params(lattice=case["lat"], nx=L, ny=L, nz=nz, A_nci=0.01, h_min=2.0, h_max=4.0)
    return p, psi.ravel(), node


@pytest.mark.parametrize("case", OBLIQUE, ids=[c["name"] for c in OBLIQUE])
def test_nci_probe_oblique_golden(case):
    p, psi, node = _oblique_field(case)
    G, hit, Fr = oracle.node_nci(p, psi, node)
    if any(case["ramp"]):
        # the isotropic stencil is exact on a linear ramp
        np.testing.assert_allclose(G, -np.array(case["ramp"], float) / 8.0, rtol=0, atol=1e-16)
    assert hit == case["h"]
    assert oracle.A_h(float(hit), 1.0, 2.0, 4.0) == pytest.approx(case["ah"], rel=1e-15) if hit else True
    np.testing.assert_allclose(Fr / p.A_nci, case["F"], rtol=1e-13, atol=1e-18)


def test_rounding_tie_is_exact():
    """Precondition of the tie case: the oracle's gradient makes s*n_y hit
    0.5 exactly at s = 2 (FP64 norm and quotient as the probe forms them)."""
    case = next(c for c in OBLIQUE if c["name"] == "tie_hit2")
    p, psi, node = _oblique_field(case)
    G, _, _ = oracle.node_nci(p, psi, node)
    g = math.sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2])
    assert g == 0.5 and G[1] == -0.125
    assert 2 * (-G[1] / g) == 0.5


# --- observables ------------------------------------------------------------

def _uniform_box(lat, F):
    d3 = lat == 1
    nx, ny, nz = (6, 5, 4) if d3 else (7, 5, 1)
    N = nx * ny * nz
    p = oracle.Params(lattice=lat, nx=nx, ny=ny, nz=nz, walls_y=0, A_nci=0.01, force=tuple(F))
    o = oracle.Oracle(p)
    o.init_fields(np.full(N, 0.3), np.full(N, 0.7))
    return o, p


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q27])
def test_observables_uniform_forced_box(lat):
    """Uniform mixture (rho1 = 0.3, rho2 = 0.7, so psi is uniform, G = 0 and
    neither perturbation, recolouring nor NCI acts) at rest under a uniform
    force F: each step adds exactly F to every node's momentum, so after t
    steps u = (t + 1/2) F / rho (rho = 1), Q = (N/nx)(t + 1/2) F_x,
    Q_d = 0.3 Q, umax = (t + 1/2)|F|, momentum N (t + 1/2) F, masses 0.3 N and
    0.7 N."""
    F = np.array([2e-6, -1e-6, 5e-7 if lat == oracle.D3Q27 else 0.0])
    o, p = _uniform_box(lat, F)
    N = p.N
    for t in (0, 7):
        o.step(t - o.t)
        ob = o.observables()
        k = t + 0.5
        np.testing.assert_allclose(ob["mass"], [0.3 * N, 0.7 * N], rtol=1e-14)
        np.testing.assert_allclose(ob["mom"], N * k * F, rtol=1e-10, atol=1e-22)
        assert ob["Q"] == pytest.approx(N / p.nx * k * F[0], rel=1e-10)
        assert ob["Q_d"] == pytest.approx(0.3 * N / p.nx * k * F[0], rel=1e-10)
        assert ob["umax"] == pytest.approx(k * np.linalg.norm(F), rel=1e-10)
        # the same velocity node by node from the field call
        _, _, u = o.fields()
        np.testing.assert_allclose(u, np.repeat((k * F[:p.dim])[:, None], N, axis=1), rtol=1e-10)


def test_observables_poiseuille_flux_and_umax():
    """Single-phase channel with half-way bounce-back walls at steady state:
    Q (fluid nodes only, per unit length along x) equals the Poiseuille flux
    F H^3/(12 nu) of the fluid width H = ny - 2 within the walls' O(1 %) slip,
    umax equals max |u| of the field call exactly, Q_d = Q (no component 2)."""
    tau, F, ny, nx = 1.0, 1e-6, 34, 4
    case = synth.poiseuille_2d(nx=nx, ny=ny, force=F, tau=tau)
    o = oracle.Oracle(oracle.Params(**case.params))
    o.init_fields(case.rho1, case.rho2)
    o.step(40000)
    ob = o.observables()
    nu = (tau - 0.5) / 3
    H = ny - 2
    assert ob["Q"] == pytest.approx(F * H ** 3 / (12 * nu), rel=5e-3)
    assert ob["Q_d"] == pytest.approx(ob["Q"], rel=1e-12)
    r1, r2, u = o.fields()
    assert ob["umax"] == np.abs(u).max() or ob["umax"] == pytest.approx(np.sqrt((u ** 2).sum(0)).max(),
                                                                        rel=1e-15)
    # Q sums the fluid rows only: the same sum taken from the field call
    assert ob["Q"] == pytest.approx(u[0].sum() / nx, rel=1e-13)


def test_observables_two_layer_sharp_split():
    """Two stratified components of equal viscosity in a forced channel: the
    flat interface leaves the Poiseuille profile unchanged, so Q_d, the flux
    weighted by the colour fraction rho1/rho, equals the flux of the rows
    below the interface in the sharp-interface limit, and Q - Q_d the flux
    above it (within the diffuse interface's smoothing)."""
    tau, F, ny, nx, y_i = 1.0, 1e-6, 34, 4, 11.5
    case = synth.two_layer_channel(nx=nx, ny=ny, y_i=y_i, tau1=tau, tau2=0.0, force=F)
    o = oracle.Oracle(oracle.Params(**case.params))
    o.init_fields(case.rho1, case.rho2)
    o.step(30000)
    ob = o.observables()
    nu = (tau - 0.5) / 3
    y = np.arange(1, ny - 1, dtype=float)
    u_p = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    q_below = u_p[y < y_i].sum()
    q_above = u_p[y > y_i].sum()
    assert ob["Q"] == pytest.approx(q_below + q_above, rel=5e-3)
    assert ob["Q_d"] == pytest.approx(q_below, rel=2e-2)
    assert ob["Q"] - ob["Q_d"] == pytest.approx(q_above, rel=2e-2)
