"""Droplet-level observables of a lattice state (FP64 / integer, CPU).

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's
droplet analysis; the GPU library never imports it.

The paper characterises its emulsions by droplets (their count, volumes and
arrangement) and by the vorticity of the flow (Results, Figs. 2-4).  Plain
definitions used here:

* dispersed phase: fluid nodes with psi = (rho1 - rho2)/(rho1 + rho2) > 0;
* droplets: connected components of the dispersed phase under face
  adjacency (4 neighbours in 2-D, 6 in 3-D), periodic in x and z, bounded
  by the wall rows in y (or periodic in y without walls);
* canonical label of a node: the smallest node index n = x + nx (y + ny z)
  in its droplet; -1 outside the dispersed phase;
* droplet table, in ascending order of canonical label: volume V_d (node
  count) and centroid.  Each node contributes its offset from the droplet's
  root node, taken in the periodic directions as the image in
  [-floor(L/2), L - 1 - floor(L/2)]; the centroid is root + (sum of
  offsets)/V, moved back into [0, L) (meaningful for droplets shorter than
  half the period);
* rows (hex-n, named by the number of droplet rows across the channel,
  Results): droplets of at least a quarter of the mean volume, sorted by
  centroid y; a gap in y larger than half the equivalent diameter of the
  median droplet starts a new row;
* droplet generation (a device with an outlet channel): from droplet tables
  sampled at a fixed interval, the main droplets are those of at least half
  the 90th-percentile volume and V_d is their median volume; nu counts the
  main droplets whose centroid passed the line x_c since the previous sample
  (the droplet being the nearest earlier centroid at most one node ahead, 20
  behind and 10 rows away), per step; Q_d = nu V_d (Results, Fig. 3);
* vorticity: omega = curl u by central differences over the node grid
  (periodic wrap in the periodic directions; wall rows hold u = 0).

Parity: pinned by a brute-force flood fill on small random masks, by
hand-built masks whose droplets cross the periodic boundaries, by the
exact central difference of linear shear and of solid rotation, and by the
discrete closed form for sinusoidal velocity fields.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage as ndi


def dispersed_mask(rho1, rho2, nx, ny, nz, walls_y):
    """Boolean mask [nz, ny, nx] of dispersed fluid nodes."""
    r1 = np.asarray(rho1, np.float64).reshape(nz, ny, nx)
    r2 = np.asarray(rho2, np.float64).reshape(nz, ny, nx)
    rho = r1 + r2
    with np.errstate(invalid="ignore", divide="ignore"):
        psi = np.where(rho > 0, (r1 - r2) / rho, -1.0)
    m = psi > 0
    if walls_y:
        m[:, 0, :] = False
        m[:, ny - 1, :] = False
    return m


def components(mask, periodic=(True, True, True)):
    """Canonical droplet labels of a [nz, ny, nx] mask; periodic flags are
    for (z, y, x).  Returns (labels [nz, ny, nx] int64, count)."""
    nz, ny, nx = mask.shape
    lab, n = ndi.label(mask, structure=ndi.generate_binary_structure(3, 1))
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    def union(a, b):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)

    # merge across each periodic boundary (the faces are adjacent)
    for axis, per in enumerate(periodic):
        if not per or mask.shape[axis] < 2:
            continue
        lo = np.take(lab, 0, axis=axis)
        hi = np.take(lab, mask.shape[axis] - 1, axis=axis)
        for a, b in zip(lo.ravel(), hi.ravel()):
            if a and b:
                union(int(a), int(b))
    roots = np.array([find(k) for k in range(n + 1)])
    merged = roots[lab]
    # canonical label: smallest node index of each merged component
    flat = merged.ravel()
    idx = np.arange(flat.size)
    out = np.full(flat.size, -1, np.int64)
    sel = flat > 0
    if sel.any():
        first = {}
        for i, r in zip(idx[sel], flat[sel]):
            if r not in first:
                first[r] = i  # idx is increasing, so the first hit is the minimum
        out[sel] = np.array([first[r] for r in flat[sel]])
    count = len(np.unique(out[out >= 0]))
    return out.reshape(mask.shape), count


def droplet_sizes(labels):
    """{canonical label: node count} of a label array."""
    lab = labels.ravel()
    lab = lab[lab >= 0]
    roots, counts = np.unique(lab, return_counts=True)
    return dict(zip(roots.tolist(), counts.tolist()))


def droplet_table(labels, nx, ny, nz, walls_y):
    """(roots, volumes, centroids [count, 3] as (x, y, z)) of a label array
    [nz, ny, nx], in ascending root order."""
    lab = np.asarray(labels).reshape(nz, ny, nx)
    roots = np.unique(lab[lab >= 0])
    vols = np.zeros(len(roots), np.int64)
    cen = np.zeros((len(roots), 3))
    z, y, x = np.nonzero(lab >= 0)
    r = lab[z, y, x]
    order = np.searchsorted(roots, r)
    coord = (x, y, z)
    L = (nx, ny, nz)
    per = (True, not walls_y, True)
    rc = (roots % nx, (roots // nx) % ny, roots // (nx * ny))
    np.add.at(vols, order, 1)
    for d in range(3):
        off = coord[d] - rc[d][order]
        if per[d]:
            h = L[d] // 2
            off = np.mod(off + h, L[d]) - h
        s = np.zeros(len(roots), np.int64)
        np.add.at(s, order, off)
        c = rc[d].astype(np.float64) + s.astype(np.float64) / vols.astype(np.float64)
        if per[d]:
            c = np.where(c < 0, c + L[d], np.where(c >= L[d], c - L[d], c))
        cen[:, d] = c
    return roots, vols, cen


def rows(centroid_y, volumes, dim):
    """Number of droplet rows across the channel (hex-n)."""
    v = np.asarray(volumes, np.float64)
    if len(v) == 0:
        return 0
    keep = v >= 0.25 * v.mean()
    y = np.sort(np.asarray(centroid_y, np.float64)[keep])
    vm = float(np.median(v[keep]))
    d_eq = 2.0 * (math.sqrt(vm / math.pi) if dim == 2 else (3.0 * vm / (4.0 * math.pi)) ** (1.0 / 3.0))
    return 1 + int(np.count_nonzero(np.diff(y) > 0.5 * d_eq))


def generation_stats(samples, xc):
    """(V_d, crossings, nu) from samples [(t, centroids [k, 2] as (x, y),
    volumes [k])] of the droplets downstream of a striction."""
    vols = [np.asarray(v, np.float64) for _, _, v in samples]
    allv = np.concatenate(vols) if vols else np.zeros(0)
    V_d = float(np.median(allv[allv >= 0.5 * np.percentile(allv, 90)])) if allv.size else 0.0
    n = 0
    for k in range(1, len(samples)):
        prev_c = np.asarray(samples[k - 1][1], np.float64)
        for (x, y), v in zip(np.asarray(samples[k][1], np.float64), samples[k][2]):
            if v < 0.5 * V_d or x < xc or prev_c.size == 0:
                continue
            near = (prev_c[:, 0] <= x + 1) & (prev_c[:, 0] > x - 20) & (np.abs(prev_c[:, 1] - y) < 10)
            if not near.any():
                continue
            cand = prev_c[near]
            j = int(np.argmin((cand[:, 0] - x) ** 2 + (cand[:, 1] - y) ** 2))
            n += int(cand[j, 0] < xc)
    span = samples[-1][0] - samples[0][0] if len(samples) > 1 else 1
    return V_d, n, n / span


def vorticity(u, nx, ny, nz, walls_y):
    """Central-difference curl of u (dim component-major blocks of N).
    2-D: [N] (omega_z); 3-D: [3, N].  Wall rows hold u = 0 and get 0."""
    dim = u.shape[0] if u.ndim == 2 else len(u) // (nx * ny * nz)
    U = np.asarray(u, np.float64).reshape(dim, nz, ny, nx).copy()
    if walls_y:
        U[:, :, 0, :] = 0.0
        U[:, :, ny - 1, :] = 0.0

    def d(f, axis):  # central difference along axis of [nz, ny, nx]; y without wrap at walls
        fp = np.roll(f, -1, axis=axis)
        fm = np.roll(f, 1, axis=axis)
        return 0.5 * (fp - fm)

    ux, uy = U[0], U[1]
    wz = d(uy, 2) - d(ux, 1)
    if dim == 2:
        if walls_y:
            wz[:, 0, :] = 0.0
            wz[:, ny - 1, :] = 0.0
        return wz.ravel()
    uz = U[2]
    wx = d(uz, 1) - d(uy, 0)
    wy = d(ux, 0) - d(uz, 2)
    w = np.stack([wx, wy, wz])
    if walls_y:
        w[:, :, 0, :] = 0.0
        w[:, :, ny - 1, :] = 0.0
    return w.reshape(3, -1)
