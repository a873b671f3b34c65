"""GPU parity of the droplet analysis and the vorticity (lb_droplets,
lb_vorticity) against the analysis oracle.

Labels, counts, volumes and centroids are integer results or FP64 results of
exact integer sums, and the dispersed-phase decision is taken in FP64 on both
sides, so the library must match the oracle bit for bit on the same fields
(the fields the library itself reports).  The vorticity takes the same FP64
central differences on both sides and must match bit for bit too.  Against
the FP64 lattice oracle's own state the fields differ at the parity bar, so
the comparison there is of what that bar fixes: the vorticity within twice
the largest velocity difference (each component is a difference of two
half-differences of u), and the dispersed-phase masks equal except at nodes
whose psi is within the field error of 0."""
import numpy as np
import pytest

import synth
from oracle import analysis as A
import paper_2003_11069_amd as P
from gpu_common import say, make_pair

pytestmark = pytest.mark.gpu


def _periodic(p):
    return (True, not p["walls_y"], True)


def _oracle_of_fields(p, r1, r2):
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    m = A.dispersed_mask(r1, r2, nx, ny, nz, p["walls_y"])
    lab, n = A.components(m, _periodic(p))
    roots, vols, cen = A.droplet_table(lab, nx, ny, nz, p["walls_y"])
    return m, lab.ravel(), n, roots, vols, cen


def _check_droplets(g, p, tag):
    r1, r2, u = g.fields()
    d = g.droplets()
    m, lab, n, roots, vols, cen = _oracle_of_fields(p, r1, r2)
    rows = A.rows(cen[:, 1], vols, 2 if p["lattice"] == 0 else 3)
    say(f"  {tag}: {d['count']} droplets, {d['dispersed']} dispersed nodes, rows {d['rows']}; "
        f"oracle {n} / {int(m.sum())} / {rows}")
    assert d["count"] == n and d["dispersed"] == int(m.sum()) and d["rows"] == rows
    assert np.array_equal(d["labels"], lab.astype(np.int32))
    assert np.array_equal(d["roots"], roots) and np.array_equal(d["volumes"], vols)
    assert np.array_equal(d["centroids"], cen)
    return d


CASES = {
    "2d_channel_walls": lambda: synth.channel_2d(synth.channel_spec(0, Lx=300, Ly=100)),
    "2d_random_periodic_ragged": lambda: synth.random_fields(
        synth.base_params(nx=77, ny=45), seed=4),
    "3d_random_periodic_ragged": lambda: synth.random_fields(
        synth.base_params(lattice=1, nx=37, ny=23, nz=11), seed=5),
    "3d_random_walls": lambda: synth.random_fields(
        synth.base_params(lattice=1, nx=64, ny=20, nz=8, walls_y=1), seed=6),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("steps", [0, 60])
def test_droplets_bit_exact_on_library_fields(name, steps):
    case = CASES[name]()
    say(f"[gpu] droplets {name} after {steps} steps")
    g = P.Lattice(P.Params.from_dict(case.params))
    g.init_fields(case.rho1, case.rho2, case.u)
    g.step(steps)
    _check_droplets(g, case.params, name)
    g.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_droplets_full_size_3d_channel(storage):
    """The 3-D benchmark channel (256 x 64 x 64) at its initial state and after
    100 steps, in each storage format."""
    case = synth.hex_channel_3d()
    say(f"[gpu] droplets 3-D benchmark channel, {storage}")
    g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[storage]))
    g.init_fields(case.rho1, case.rho2)
    d0 = _check_droplets(g, case.params, "t=0")
    g.step(100)
    _check_droplets(g, case.params, "t=100")
    assert d0["count"] > 100
    g.close()


def test_droplets_degenerate_and_extreme():
    p = synth.base_params(nx=20, ny=14, walls_y=1)
    N = 20 * 14
    say("[gpu] droplets: no dispersed phase, all dispersed, checkerboard, cap")
    g = P.Lattice(P.Params.from_dict(p))
    g.init_fields(np.zeros(N), np.ones(N))
    d = g.droplets()
    assert d["count"] == 0 and d["dispersed"] == 0 and d["rows"] == 0 and np.all(d["labels"] == -1)
    g.init_fields(np.ones(N), np.zeros(N))
    d = _check_droplets(g, p, "all dispersed")
    assert d["count"] == 1 and d["dispersed"] == 20 * 12 and d["roots"][0] == 20
    g.close()
    # checkerboard on a periodic lattice: every dispersed node is its own droplet (N/2 of them)
    p = synth.base_params(nx=16, ny=10)
    N = 160
    x, y = np.arange(N) % 16, np.arange(N) // 16
    r1 = np.where((x + y) % 2 == 0, 0.7, 0.3)
    g = P.Lattice(P.Params.from_dict(p))
    g.init_fields(r1, 1.0 - r1)
    d = _check_droplets(g, p, "checkerboard")
    assert d["count"] == N // 2 and np.all(d["volumes"] == 1)
    # cap below the count lists the first droplets only
    d3 = g.droplets(labels=False, cap=3)
    assert d3["count"] == N // 2 and np.array_equal(d3["roots"], d["roots"][:3])
    assert d3["labels"] is None
    g.close()


def test_droplets_crossing_the_periodic_boundaries():
    """Droplets centred on the x and z faces of a periodic 3-D box: one label
    each, centroids on the faces."""
    p = synth.base_params(lattice=1, nx=40, ny=30, nz=24)
    cs = [(0.0, 15.0, 0.0), (20.0, 0.0, 12.0), (39.5, 29.5, 23.5)]
    psi = synth._droplet_psi((24, 30, 40), cs, [5.0, 5.0, 4.0], (True, True, True))
    r1, r2 = 0.5 * (1 + psi.ravel()), 0.5 * (1 - psi.ravel())
    say("[gpu] droplets across the periodic faces")
    g = P.Lattice(P.Params.from_dict(p))
    g.init_fields(r1, r2)
    d = _check_droplets(g, p, "periodic faces")
    assert d["count"] == 3
    g.close()


VORT = {
    "2d_channel_walls": CASES["2d_channel_walls"],
    "2d_random_periodic_ragged": CASES["2d_random_periodic_ragged"],
    "3d_random_walls": CASES["3d_random_walls"],
    "3d_random_periodic_ragged": CASES["3d_random_periodic_ragged"],
}


@pytest.mark.parametrize("name", list(VORT))
def test_vorticity_bit_exact_on_library_fields(name):
    case = VORT[name]()
    p = case.params
    say(f"[gpu] vorticity {name}")
    g = P.Lattice(P.Params.from_dict(p))
    g.init_fields(case.rho1, case.rho2, case.u)
    g.step(40)
    _, _, u = g.fields()
    w = g.vorticity()
    ref = A.vorticity(u, p["nx"], p["ny"], p["nz"], p["walls_y"])
    say(f"  max |omega| {np.abs(ref).max():.3e}, max diff {np.abs(w - ref).max():.1e}")
    assert np.array_equal(w, ref)
    g.close()


def test_vorticity_and_mask_against_the_lattice_oracle():
    """200 steps of the 2-D channel on both sides: vorticity within the bound
    set by the velocity difference; masks equal away from psi = 0."""
    case = synth.channel_2d(synth.channel_spec(0, Lx=300, Ly=100))
    p = case.params
    say("[gpu] vorticity and droplets vs the lattice oracle, 2-D channel 300x100, 200 steps")
    o, g = make_pair(case)
    o.step(200)
    g.step(200)
    r1o, r2o, uo = o.fields()
    r1g, r2g, ug = g.fields()
    wo = A.vorticity(uo, p["nx"], p["ny"], 1, 1)
    wg = g.vorticity()
    du = np.abs(ug - uo).max()
    dw = np.abs(wg - wo).max()
    say(f"  max |du| {du:.2e}, max |domega| {dw:.2e} (bound {2 * du:.2e}), max |omega| {np.abs(wo).max():.2e}")
    assert dw <= 2 * du * (1 + 1e-12) + 1e-18
    mo = A.dispersed_mask(r1o, r2o, p["nx"], p["ny"], 1, 1).ravel()
    d = g.droplets()
    mg = d["labels"] >= 0
    psi_o = (r1o - r2o) / np.where(r1o + r2o > 0, r1o + r2o, 1.0)
    e_psi = np.abs((r1g - r2g) / np.where(r1g + r2g > 0, r1g + r2g, 1.0) - psi_o).max()
    flips = np.nonzero(mg != mo)[0]
    say(f"  mask flips {len(flips)} (max |dpsi| {e_psi:.1e})")
    assert np.all(np.abs(psi_o[flips]) <= e_psi)
    if len(flips) == 0:
        lab, n = A.components(mo.reshape(1, p["ny"], p["nx"]), _periodic(p))
        assert np.array_equal(d["labels"], lab.ravel().astype(np.int32)) and d["count"] == n
