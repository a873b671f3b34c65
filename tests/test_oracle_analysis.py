"""Pins of the droplet-analysis oracle (CPU only): components against a
brute-force flood fill, periodic merging on hand-built masks, and the
discrete closed form of central-difference vorticity."""
import math
from collections import deque

import numpy as np
import pytest

from oracle import analysis as A


def _flood(mask, periodic):
    """Independent brute force: BFS with explicit neighbour wrapping."""
    nz, ny, nx = mask.shape
    lab = -np.ones(mask.shape, np.int64)
    dims = (nz, ny, nx)
    for start in range(mask.size):
        z, y, x = np.unravel_index(start, mask.shape)
        if not mask[z, y, x] or lab[z, y, x] >= 0:
            continue
        lab[z, y, x] = start
        q = deque([(z, y, x)])
        while q:
            c = q.popleft()
            for ax in range(3):
                for s in (-1, 1):
                    n = list(c)
                    n[ax] += s
                    if n[ax] < 0 or n[ax] >= dims[ax]:
                        if not periodic[ax] or dims[ax] < 2:
                            continue
                        n[ax] %= dims[ax]
                    n = tuple(n)
                    if mask[n] and lab[n] < 0:
                        lab[n] = start
                        q.append(n)
    return lab


@pytest.mark.parametrize("shape,periodic,seed", [((1, 9, 12), (True, True, True), 0),
                                                 ((1, 9, 12), (True, False, True), 1),
                                                 ((4, 5, 6), (True, True, True), 2),
                                                 ((4, 6, 5), (True, False, True), 3)])
def test_components_match_flood_fill(shape, periodic, seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        mask = rng.uniform(size=shape) < 0.45
        lab, n = A.components(mask, periodic)
        ref = _flood(mask, periodic)
        assert np.array_equal(lab, ref)
        assert n == len(np.unique(ref[ref >= 0]))


def test_periodic_merge_and_walls():
    m = np.zeros((1, 6, 10), bool)
    m[0, 2:4, 0:2] = True   # touches x = 0 ...
    m[0, 2:4, 8:10] = True  # ... and x = nx-1: one droplet through the boundary
    m[0, 0, 5] = m[0, 5, 5] = True  # rows 0 and ny-1: adjacent only if y is periodic
    lab, n = A.components(m, (True, True, True))
    assert n == 2 and lab[0, 2, 9] == lab[0, 2, 0] == 20 and lab[0, 5, 5] == lab[0, 0, 5] == 5
    lab, n = A.components(m, (True, False, True))
    assert n == 3
    assert A.droplet_sizes(lab) == {5: 1, 20: 8, 55: 1}


def test_vorticity_discrete_closed_form():
    nx, ny = 16, 12
    kx, ky = 2 * math.pi / nx, 2 * math.pi * 2 / ny
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    u = np.stack([np.sin(ky * y), np.sin(kx * x)]).reshape(2, -1)
    w = A.vorticity(u, nx, ny, 1, walls_y=0)
    ref = np.cos(kx * x) * math.sin(kx) - np.cos(ky * y) * math.sin(ky)
    np.testing.assert_allclose(w, ref.ravel(), atol=1e-14)
    # 3-D: u_x = sin(k z) gives omega_y = cos(k z) sin(k) only
    nz = 8
    k = 2 * math.pi / nz
    z = np.arange(nz)[:, None, None] * np.ones((1, 4, 5))
    u3 = np.zeros((3, nz * 4 * 5))
    u3[0] = np.sin(k * z).ravel()
    w3 = A.vorticity(u3, 5, 4, nz, walls_y=0)
    np.testing.assert_allclose(w3[1], (np.cos(k * z) * math.sin(k)).ravel(), atol=1e-14)
    assert np.abs(w3[0]).max() == 0 and np.abs(w3[2]).max() == 0


def test_vorticity_linear_shear_and_solid_rotation():
    # linear fields: the central difference is exact away from the wrap, so
    # shear u_x = a y gives omega_z = -a and solid rotation u = W x r gives 2 W
    nx, ny, nz = 7, 9, 8
    a = 0.3
    y = np.arange(ny)[None, :, None] * np.ones((nz, 1, nx))
    u = np.zeros((2, ny * nx))
    u[0] = (a * y[0]).ravel()
    w = A.vorticity(u, nx, ny, 1, walls_y=1).reshape(ny, nx)
    assert np.all(w[0] == 0) and np.all(w[-1] == 0)
    np.testing.assert_allclose(w[2:-2], -a, rtol=1e-14)
    # next to a wall the wall's u = 0 enters: (u(y+1) - 0) / 2
    np.testing.assert_allclose(w[1], -a * 2 / 2, rtol=1e-14)
    np.testing.assert_allclose(w[-2], -(0 - a * (ny - 3)) / 2, rtol=1e-14)
    Om = np.array([0.11, -0.07, 0.05])
    z, yy, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([x - 3.0, yy - 4.0, z - 3.5])
    U = np.cross(Om[:, None, None, None], r, axis=0)
    w3 = A.vorticity(U.reshape(3, -1), nx, ny, nz, walls_y=0).reshape(3, nz, ny, nx)
    inner = w3[:, 1:-1, 1:-1, 1:-1]
    np.testing.assert_allclose(inner, np.broadcast_to(2 * Om[:, None, None, None], inner.shape),
                               rtol=1e-13)


def test_dispersed_mask():
    nx, ny = 4, 5
    r1 = np.array([0.6, 0.4, 0.5, 0.0] * 5)
    r2 = np.array([0.4, 0.6, 0.5, 0.0] * 5)
    m = A.dispersed_mask(r1, r2, nx, ny, 1, walls_y=1)
    assert m.shape == (1, ny, nx)
    assert not m[0, 0].any() and not m[0, -1].any()
    assert np.array_equal(m[0, 1:-1], np.tile([True, False, False, False], (3, 1)))
    assert A.dispersed_mask(r1, r2, nx, ny, 1, walls_y=0)[0, 0, 0]


def _disks(shape, centres, R):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = np.zeros(shape, bool)
    for cx, cy, cz in centres:
        dx = (x - cx + nx / 2) % nx - nx / 2
        dz = (z - cz + nz / 2) % nz - nz / 2 if nz > 1 else 0
        m |= dx * dx + (y - cy) ** 2 + dz * dz <= R * R
    return m


def test_droplet_table_centroids_through_the_boundaries():
    nx, ny, nz = 20, 16, 16
    # a sphere centred on the x and z periodic faces, and one in the bulk
    # (both shorter than half of each period)
    m = _disks((nz, ny, nx), [(0.0, 7.0, 0.0), (10.0, 8.0, 6.0)], 3.2)
    lab, n = A.components(m, (True, False, True))
    roots, vols, cen = A.droplet_table(lab, nx, ny, nz, walls_y=1)
    assert n == 2 and vols.sum() == m.sum() and list(roots) == sorted(roots)
    # brute force: shift the lattice so that the droplet does not wrap, take
    # the plain mean, shift back; lattice spheres about a node are symmetric,
    # so the centroid is the centre itself
    for r, v, c, (sx, sz), ctr in zip(roots, vols, cen, [(10, 8), (0, 0)],
                                      [(0.0, 7.0, 0.0), (10.0, 8.0, 6.0)]):
        sh = np.roll(np.roll(lab, sx, axis=2), sz, axis=0)
        z, y, x = np.nonzero(sh == r)
        assert len(x) == v
        ref = ((x.mean() - sx) % nx, y.mean(), (z.mean() - sz) % nz)
        np.testing.assert_allclose(c, ref, atol=1e-12)
        np.testing.assert_allclose(c, ctr, atol=1e-12)


@pytest.mark.parametrize("n_rows", [1, 2, 3])
def test_rows_of_hexagonal_packings(n_rows):
    R, nx = 6.0, 120
    a = 2 * R + 3  # gap of 3 nodes between neighbours
    pitch = a * math.sqrt(3) / 2
    ny = int(2 * R + 4 + (n_rows - 1) * pitch + 2)
    cs = []
    for r in range(n_rows):
        for i in range(int(nx / a)):
            cs.append(((i + 0.5 * (r % 2)) * nx / int(nx / a), R + 2.5 + r * pitch, 0.0))
    m = _disks((1, ny, nx), cs, R)
    m[:, 0] = m[:, -1] = False
    lab, n = A.components(m, (True, False, True))
    assert n == len(cs)
    roots, vols, cen = A.droplet_table(lab, nx, ny, 1, walls_y=1)
    assert A.rows(cen[:, 1], vols, 2) == n_rows
    # debris below a quarter of the mean volume does not make a row
    m[0, ny // 2 + 1 if n_rows == 1 else 1, 3] = True
    lab, n2 = A.components(m, (True, False, True))
    roots, vols, cen = A.droplet_table(lab, nx, ny, 1, walls_y=1)
    assert A.rows(cen[:, 1], vols, 2) == n_rows


@pytest.mark.parametrize("seed,n_rows", [(0, 5), (2, 3), (3, 3), (4, 5)])
def test_rows_of_synthetic_channels(seed, n_rows):
    """Channels whose droplets do not touch: the count and the number of rows
    are those the generator placed."""
    import synth
    c = synth.channel_2d(synth.channel_spec(seed))
    p = c.params
    m = A.dispersed_mask(c.rho1, c.rho2, p["nx"], p["ny"], 1, 1)
    lab, n = A.components(m, (True, False, True))
    assert n == c.info["n_droplets"]
    roots, vols, cen = A.droplet_table(lab, p["nx"], p["ny"], 1, 1)
    assert A.rows(cen[:, 1], vols, 2) == n_rows


@pytest.mark.parametrize("period,speed", [(6600, 0.007), (2500, 0.015)])
def test_generation_stats_of_a_droplet_train(period, speed):
    """Main droplets born every `period` steps at the striction and moving at
    `speed`, each with a trailing satellite: nu = 1/period, V_d = the main
    volume."""
    rng = np.random.default_rng(3)
    x0, xc, L = 113, 190, 430
    samples = []
    for t in range(0, 150000, 250):
        births = np.arange(0, t + 1, period)
        x = x0 + 4 + speed * (t - births)
        x = x[x < L]
        y = 48.0 + rng.uniform(-1, 1, x.size)
        cen = np.concatenate([np.stack([x, y], 1), np.stack([x - 12, y], 1)])
        vol = np.concatenate([400 + rng.integers(-5, 6, x.size), np.full(x.size, 50)])
        keep = cen[:, 0] > x0
        samples.append((t, cen[keep], vol[keep]))
    V_d, n, nu = A.generation_stats(samples, xc)
    assert V_d == pytest.approx(400, abs=5)
    assert nu == pytest.approx(1 / period, rel=0.05)
