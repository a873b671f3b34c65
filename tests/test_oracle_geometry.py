"""Pins of the oracle's node-type geometry (solid / inlet / outlet): the
mask form of a walled channel equals the built-in walls on a single-phase
flow, closed boxes with obstacles keep both component masses, a uniform flow
between a velocity inlet and a pressure outlet stays exactly uniform, the
inlet supplies its equilibrium, the steady flux is the same through every
cross-section and carries the inlet's velocity, solid
nodes carry the weighted mean psi of their non-solid neighbours, and the NCI
probe stops at a solid node."""
import numpy as np
import pytest

import oracle
import synth

W9 = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}  # D2Q9 weights by |c|^2


def _oracle(case, **over):
    d = dict(case.params)
    d.update(over)
    o = oracle.Oracle(oracle.Params(**{k: v for k, v in d.items() if k in oracle.Params.__dataclass_fields__}))
    if "type" in (case.info or {}):
        o.set_geometry(case.info["type"], case.rho1, case.rho2, case.u)
    o.init_fields(case.rho1, case.rho2, case.u)
    return o


def test_mask_walls_equal_builtin_walls_single_phase():
    case = synth.solid_wall_channel(nx=24, ny=34, force=1e-5)
    og = _oracle(case)
    ow = oracle.Oracle(oracle.Params(**{**case.params, "walls_y": 1}))
    ow.init_fields(case.rho1, case.rho2)
    og.step(400)
    ow.step(400)
    fg1, fg2 = og.get_populations()
    fw1, fw2 = ow.get_populations()
    fluid = case.info["type"] == synth.FLUID
    assert np.abs(fg1[:, fluid] - fw1[:, fluid]).max() <= 1e-15
    assert np.abs(fg2[:, fluid]).max() == 0
    r1, _, u = og.fields()
    assert u[0, fluid].max() > 1e-4  # the flow has developed


@pytest.mark.parametrize("lattice,nz", [(0, 1), (1, 6)])
def test_closed_box_with_obstacles_keeps_both_masses(lattice, nz):
    case = synth.obstacle_box(nx=40, ny=30, lattice=lattice, nz=nz)
    o = _oracle(case)
    m0 = o.observables()["mass"]
    o.step(300)
    m1 = o.observables()["mass"]
    np.testing.assert_allclose(m1, m0, rtol=1e-12)
    r1, r2, _ = o.fields()
    solid = case.info["type"] != synth.FLUID
    assert np.all(r1[solid] == 0) and np.all(r2[solid] == 0)


@pytest.mark.parametrize("rho1", [1.0, 0.0])
def test_uniform_flow_between_inlet_and_outlet_stays_uniform(rho1):
    """Periodic in y (no walls): inlet column with (rho, u), outlet column,
    the same uniform state inside -- an exact steady solution.  One component
    only: a uniform mixture has G = 0 only up to round-off, and the
    recolouring direction G/|G| is undefined there."""
    nx, ny, u0 = 30, 12, 0.02
    t = np.zeros((ny, nx), np.uint8)
    t[:, 0] = synth.INLET
    t[:, -1] = synth.OUTLET
    N = nx * ny
    r1 = np.full(N, rho1); r2 = np.full(N, 1.0 - rho1)
    u = np.zeros((2, N)); u[0] = u0; u[1] = -0.005
    case = synth.Case(synth.base_params(nx=nx, ny=ny, A_nci=0.0), r1, r2, u, {"type": t.ravel()})
    o = _oracle(case)
    o.step(200)
    f1, f2 = o.get_populations()
    fluid = t.ravel() == synth.FLUID
    e1 = oracle.equilibrium(0, rho1, (u0, -0.005))
    e2 = oracle.equilibrium(0, 1.0 - rho1, (u0, -0.005))
    assert np.abs(f1[:, fluid] - e1[:, None]).max() <= 1e-15
    assert np.abs(f2[:, fluid] - e2[:, None]).max() <= 1e-15


def test_inlet_supplies_its_equilibrium():
    """Velocity inlet: the equilibrium at the prescribed velocity and
    composition with the feeder's density (1 after the first collision)."""
    case = synth.inlet_outlet_channel(nx=20, ny=10, u_in=0.03, rho1_in=0.8, rho2_in=0.2)
    case.rho1[:] = 0.8
    case.rho2[:] = 0.2
    o = _oracle(case)
    o.step(1)
    f1, f2 = o.get_populations()
    c, w, _ = oracle.lattice(0)
    e1 = oracle.equilibrium(0, 0.8, (0.03, 0.0))
    # node (1, 5): directions with c_x = +1 come from the inlet column
    n = 1 + 20 * 5
    for i in range(9):
        if c[i][0] == 1:
            assert f1[i, n] == pytest.approx(e1[i], abs=1e-16)


def test_steady_flux_is_the_same_through_every_cross_section():
    case = synth.inlet_outlet_channel(nx=48, ny=26, u_in=0.01)
    o = _oracle(case)
    o.step(8000)
    r1, r2, u = o.fields()
    ny, nx = 26, 48
    jx = ((r1 + r2) * u[0]).reshape(ny, nx)
    flux = jx[1:-1, 1:-1].sum(axis=0)
    assert np.ptp(flux) <= 1e-6 * flux.mean()
    # the plug inlet delivers about its nominal flux; the profile downstream
    # is close to a parabola with zero slip at the solid rows
    assert flux.mean() == pytest.approx(0.01 * (ny - 2), rel=0.15)
    prof = jx[1:-1, nx - 6]
    y = np.arange(1, ny - 1) - (ny - 1) / 2
    par = (((ny - 2) / 2) ** 2 - y ** 2)
    par *= prof.sum() / par.sum()
    assert np.abs(prof - par).max() <= 0.05 * prof.max()


def test_solid_psi_is_the_weighted_mean_of_non_solid_neighbours():
    nx, ny = 12, 10
    rng = np.random.default_rng(4)
    t = np.zeros((ny, nx), np.uint8)
    t[5, 6] = synth.SOLID
    t[5, 7] = synth.SOLID        # a solid neighbour does not count
    t[4, 5] = synth.SOLID
    psi0 = rng.uniform(-0.9, 0.9, (ny, nx))
    r1, r2 = (1 + psi0.ravel()) / 2, (1 - psi0.ravel()) / 2
    case = synth.Case(synth.base_params(nx=nx, ny=ny, A_nci=0.0), r1, r2, None, {"type": t.ravel()})
    o = _oracle(case)
    psi = o.diagnostics()["psi"].reshape(ny, nx)
    sw = sp = 0.0
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == dy == 0 or t[5 + dy, 6 + dx] == synth.SOLID:
                continue
            w = W9[dx * dx + dy * dy]
            sw += w
            sp += w * psi0[5 + dy, 6 + dx]
    assert psi[5, 6] == pytest.approx(sp / sw, abs=1e-15)


def test_probe_stops_at_a_solid_node():
    """A continuous film with a dispersed region beyond: the probe from the
    film's edge hits the far interface, unless a solid node sits in its path."""
    nx, ny = 24, 6
    X = np.arange(nx)
    prof = np.where(X < 10, 0.9, np.where(X < 13, -0.9, 0.9)).astype(float)
    psi = np.tile(prof, (ny, 1))
    r1, r2 = (1 + psi.ravel()) / 2, (1 - psi.ravel()) / 2
    node = 9 + nx * 3
    free = synth.Case(synth.base_params(nx=nx, ny=ny, A_nci=0.02), r1, r2, None,
                      {"type": np.zeros(nx * ny, np.uint8)})
    assert _oracle(free).diagnostics()["hit"][node] > 0
    t = np.zeros((ny, nx), np.uint8)
    t[3, 11] = synth.SOLID
    blocked = synth.Case(free.params, r1, r2, None, {"type": t.ravel()})
    assert _oracle(blocked).diagnostics()["hit"][node] == 0


def test_invalid_masks_are_rejected():
    case = synth.inlet_outlet_channel(nx=20, ny=10)
    t = case.info["type"].reshape(10, 20).copy()
    t[3:6, 7:10] = synth.SOLID
    t[4, 8] = synth.INLET  # an inlet without a fluid neighbour along an axis
    o = oracle.Oracle(oracle.Params(**case.params))
    with pytest.raises(ValueError):
        o.set_geometry(t.ravel(), case.rho1, case.rho2, case.u)
    with pytest.raises(ValueError):
        oracle.Oracle(oracle.Params(**{**case.params, "walls_y": 1})).set_geometry(
            case.info["type"], case.rho1, case.rho2, case.u)
