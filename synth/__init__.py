"""Seeded synthetic inputs: droplet geometries and channel parameters.

This module is the ONLY code shared by the GPU path's tests/benchmarks and the
oracle.  It builds initial component-density fields (rho1, rho2, u) and model
parameters; it contains none of the lattice Boltzmann arithmetic.

The paper's workloads (droplet-packed microchannels, flowing emulsions in a
flow-focuser outlet) come without lattice-unit geometry or data, so these
stand-ins follow the configurations used throughout this project:

* ``laplace_droplet``  -- one static droplet, 2-D periodic box (Laplace check)
* ``hex_channel_3d``   -- 3-D wall-bounded channel packed with spherical
  droplets on a jittered hexagonal lattice (x-y plane, stacked along z)
* ``channel_2d``       -- one 2-D wall-bounded channel with a hexagonal
  droplet packing, parameters drawn from ``batch_specs``
* ``two_droplets_2d``  -- two droplets separated by a thin film (NCI check)

All randomness is numpy PCG64 with the seed given.  Interfaces are initialised
with the profile psi0 = tanh((R - r)/2) and rho1 = (1 + psi0)/2,
rho2 = (1 - psi0)/2, where r is the distance to the nearest droplet centre
(periodic images in the periodic directions).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

SIGMA0 = 1.0 / 90.0  # surface tension held fixed across the sweep (lattice units)


def _profile(psi0: np.ndarray):
    return 0.5 * (1.0 + psi0), 0.5 * (1.0 - psi0)


def _droplet_psi(shape, centres, radii, periodic):
    """psi0 = max over droplets of tanh((R - r)/2); ``shape`` is (nz, ny, nx)
    (x fastest in memory), centres are (x, y, z) rows."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    psi = np.full(shape, -1.0)
    dims = (nx, ny, nz)
    for (cx, cy, cz), R in zip(centres, radii):
        d2 = np.zeros(shape)
        for a, (coord, cc) in enumerate(((x, cx), (y, cy), (z, cz))):
            d = coord - cc
            if periodic[a]:
                L = dims[a]
                d = d - L * np.round(d / L)
            d2 = d2 + d * d
        psi = np.maximum(psi, np.tanh((R - np.sqrt(d2)) / 2.0))
    return psi


@dataclass
class Case:
    """One workload: parameter dict (lb_params fields) and initial fields."""
    params: dict
    rho1: np.ndarray
    rho2: np.ndarray
    u: np.ndarray | None = None
    info: dict | None = None

    @property
    def N(self):
        return self.rho1.size


def base_params(**kw) -> dict:
    p = dict(lattice=0, nx=128, ny=64, nz=1, walls_y=0, tau=1.0, A_s=0.05, beta=0.7,
             A_nci=0.005, h_min=2.0, h_max=4.0, force=(0.0, 0.0, 0.0))
    p.update(kw)
    return p


def laplace_droplet(nx=128, ny=64, R=16.0, centre=None, **kw) -> Case:
    """One droplet of radius R centred in a periodic D2Q9 box."""
    cx, cy = centre if centre is not None else (nx // 2, ny // 2)
    psi = _droplet_psi((1, ny, nx), [(cx, cy, 0)], [R], (True, True, True))
    r1, r2 = _profile(psi.ravel())
    return Case(base_params(nx=nx, ny=ny, **kw), r1, r2, None, {"R": R, "centre": (cx, cy)})


def two_droplets_2d(nx=96, ny=48, R=10.0, gap=1.0, jitter=0.0, seed=0, **kw) -> Case:
    """Two droplets on the x axis whose surfaces are ``gap`` nodes apart."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 2 * R + gap
    cs = [(nx / 2 - d / 2, ny / 2, 0.0), (nx / 2 + d / 2, ny / 2, 0.0)]
    cs = [(x + jitter * rng.uniform(-1, 1), y + jitter * rng.uniform(-1, 1), 0.0) for x, y, _ in cs]
    psi = _droplet_psi((1, ny, nx), cs, [R, R], (True, True, True))
    r1, r2 = _profile(psi.ravel())
    return Case(base_params(nx=nx, ny=ny, **kw), r1, r2, None, {"centres": cs})


def _hex_rows(L_x, y_lo, y_hi, a):
    """Hexagonal lattice of centres in [0, L_x) x [y_lo, y_hi]: rows along x
    with spacing snapped so that an integer number fits the periodic length."""
    n_x = max(1, int(round(L_x / a)))
    a_x = L_x / n_x
    pitch = a_x * math.sqrt(3.0) / 2.0
    rows = []
    y = y_lo
    r = 0
    while y <= y_hi + 1e-9:
        off = 0.5 * a_x * (r % 2)
        rows.append([(off + a_x * i, y) for i in range(n_x)])
        y += pitch
        r += 1
    return rows, a_x, pitch


def hex_channel_3d(nx=256, ny=64, nz=64, R=7.0, frac=0.8, z_pitch=16.0, jitter=0.5, seed=2,
                   force=1e-5, **kw) -> Case:
    """Wall-bounded D3Q27 channel (walls at y=0, ny-1; periodic x, z) packed
    with spheres of radius R: hexagonal in the x-y plane at planar area
    fraction ``frac`` (spacing a from (2 pi/sqrt 3)(R/a)^2 = frac, snapped to
    the periodic length), layers along z at ``z_pitch``, uniform jitter of
    +-``jitter`` nodes per coordinate.  Centres stay >= R+1 from the walls."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = R * math.sqrt(2.0 * math.pi / (math.sqrt(3.0) * frac))
    rows, a_x, pitch = _hex_rows(nx, 1 + R + 1, ny - 2 - R - 1, a)
    n_layers = max(1, int(nz // z_pitch))
    centres = []
    for l in range(n_layers):
        zc = z_pitch / 2 + l * z_pitch
        for row in rows:
            for (xc, yc) in row:
                centres.append((xc + jitter * rng.uniform(-1, 1), yc + jitter * rng.uniform(-1, 1),
                                zc + jitter * rng.uniform(-1, 1)))
    psi = _droplet_psi((nz, ny, nx), centres, [R] * len(centres), (True, False, True))
    psi[:, 0, :] = -1.0
    psi[:, ny - 1, :] = -1.0
    r1, r2 = _profile(psi.ravel())
    p = base_params(lattice=1, nx=nx, ny=ny, nz=nz, walls_y=1, force=(force, 0.0, 0.0), **kw)
    vol = len(centres) * 4.0 / 3.0 * math.pi * R ** 3 / (nx * (ny - 2) * nz)
    return Case(p, r1, r2, None, {"n_droplets": len(centres), "a_x": a_x, "row_pitch": pitch,
                                  "volume_fraction": vol})


@dataclass
class ChannelSpec:
    """Parameters of one 2-D channel of the batched sweep."""
    seed: int
    Lx: int
    Ly: int
    phi_p: float
    G_p: float
    A_nci: float
    R: float
    tau: float
    A_s: float

    def as_dict(self):
        return asdict(self)


def channel_spec(seed: int, Lx=None, Ly=None, G_range=(1e-6, 1e-4), A_range=(0.0, 0.05),
                 R_range=(10, 20)) -> ChannelSpec:
    """Draw one channel: Lx ~ U{256..1024}, Ly ~ U{64..160}, packing
    phi_p ~ U[0.7, 0.9], pressure gradient G_p ~ logU[1e-6, 1e-4],
    A_nci ~ U[0, 0.05], droplet radius R ~ U{10..20} (other ranges map the
    same draws onto them).  tau is raised so that the Poiseuille peak speed
    3 G_p H^2 / (8 (tau - 1/2)) stays <= 0.05, and A_s = 9 sigma0 / (2 tau)
    keeps the surface tension at sigma0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lx = int(rng.integers(256, 1025))
    ly = int(rng.integers(64, 161))
    phi_p = float(rng.uniform(0.7, 0.9))
    ug = rng.uniform(-6, -4)
    ua = rng.uniform(0.0, 0.05)
    ur = int(rng.integers(10, 21))
    if tuple(G_range) == (1e-6, 1e-4):
        G_p = float(10 ** ug)
    else:
        lg = math.log10(G_range[0]), math.log10(G_range[1])
        G_p = float(10 ** (lg[0] + (lg[1] - lg[0]) * (ug + 6) / 2))
    A_nci = float(ua) if tuple(A_range) == (0.0, 0.05) else float(A_range[0] + (A_range[1] - A_range[0]) * ua / 0.05)
    R = float(R_range[0] + (ur - 10) * (R_range[1] - R_range[0]) // 10)
    Lx = lx if Lx is None else Lx
    Ly = ly if Ly is None else Ly
    H = Ly - 2
    tau = max(1.0, 0.5 + 3.0 * G_p * H * H / (8.0 * 0.05))
    A_s = 9.0 * SIGMA0 / (2.0 * tau)
    return ChannelSpec(seed, Lx, Ly, phi_p, G_p, A_nci, R, tau, A_s)


def batch_specs(master_seed=3, n=64):
    """Per-channel seeds drawn from the master seed, then ``channel_spec``."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    seeds = rng.integers(0, 2 ** 31 - 1, size=n)
    return [channel_spec(int(s)) for s in seeds]


def channel_2d(spec: ChannelSpec, jitter=0.5) -> Case:
    """Wall-bounded D2Q9 channel with a jittered hexagonal droplet packing."""
    rng = np.random.Generator(np.random.PCG64(spec.seed + 1))
    R = spec.R
    a = R * math.sqrt(2.0 * math.pi / (math.sqrt(3.0) * spec.phi_p))
    rows, a_x, pitch = _hex_rows(spec.Lx, 1 + R + 1, spec.Ly - 2 - R - 1, a)
    centres = []
    for row in rows:
        for (xc, yc) in row:
            centres.append((xc + jitter * rng.uniform(-1, 1), yc + jitter * rng.uniform(-1, 1), 0.0))
    psi = _droplet_psi((1, spec.Ly, spec.Lx), centres, [R] * len(centres), (True, False, True))
    psi[:, 0, :] = -1.0
    psi[:, spec.Ly - 1, :] = -1.0
    r1, r2 = _profile(psi.ravel())
    p = base_params(lattice=0, nx=spec.Lx, ny=spec.Ly, nz=1, walls_y=1, tau=spec.tau,
                    A_s=spec.A_s, A_nci=spec.A_nci, force=(spec.G_p, 0.0, 0.0))
    return Case(p, r1, r2, None, {"n_droplets": len(centres), "spec": spec.as_dict()})


def poiseuille_2d(nx=4, ny=34, force=1e-6, tau=1.0) -> Case:
    """Single-phase (rho1 = 1, rho2 = 0) wall-bounded channel at rest."""
    N = nx * ny
    r1 = np.ones(N)
    r2 = np.zeros(N)
    return Case(base_params(nx=nx, ny=ny, walls_y=1, tau=tau, force=(force, 0.0, 0.0)), r1, r2)


def random_fields(p: dict, seed=0, amp=0.05, umax=0.02) -> Case:
    """Smooth-ish random two-component fields (for invariant and parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    dim = 2 if p["lattice"] == 0 else 3
    psi = np.tanh(3.0 * rng.uniform(-1, 1, (nz, ny, nx)))
    rho = 1.0 + amp * rng.uniform(-1, 1, (nz, ny, nx))
    r1 = (rho * 0.5 * (1 + psi)).ravel()
    r2 = (rho * 0.5 * (1 - psi)).ravel()
    u = umax * rng.uniform(-1, 1, (dim, nx * ny * nz))
    return Case(dict(p), r1, r2, u)


# --- warm-start network inputs -----------------------------------------------

def unet_segments(levels: int, base: int):
    """(weight count, fan-in, bias count) of each layer of the warm-start U-Net
    in its flat parameter order: encoder levels 0..L-1 (two 3x3 convs each,
    input padded to 8 channels), decoder levels L-2..0 (2x2 up-sampling, two
    3x3 convs over [up | skip]), 1x1 head with 8 outputs."""
    C = [base << l for l in range(levels)]
    seg = []
    for l in range(levels):
        cin = 8 if l == 0 else C[l - 1]
        seg.append((C[l] * 9 * cin, 9 * cin, C[l]))
        seg.append((C[l] * 9 * C[l], 9 * C[l], C[l]))
    for l in range(levels - 2, -1, -1):
        seg.append((4 * C[l] * C[l + 1], C[l + 1], C[l]))
        seg.append((C[l] * 9 * 2 * C[l], 9 * 2 * C[l], C[l]))
        seg.append((C[l] * 9 * C[l], 9 * C[l], C[l]))
    seg.append((8 * base, base, 8))
    return seg


def unet_params(levels: int, base: int, seed: int = 0, bias: float = 0.05) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan-in); the head sqrt(1 / fan-in)) and
    small uniform biases, float32, flat parameter order of ``unet_segments``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    segs = unet_segments(levels, base)
    parts = []
    for k, (nw, fan, nb) in enumerate(segs):
        gain = 1.0 if k == len(segs) - 1 else 2.0
        parts.append(rng.normal(0.0, math.sqrt(gain / fan), nw))
        parts.append(rng.uniform(-bias, bias, nb))
    return np.concatenate(parts).astype(np.float32)


def unet_batch(B: int, H: int, W: int, cin: int, cout: int, seed: int = 0):
    """Smooth random inputs [B,H,W,cin] and targets [B,H,W,cout] (float32):
    sums of a few random Fourier modes plus white noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")

    def field(n, c):
        out = np.zeros((n, H, W, c))
        for b in range(n):
            for ch in range(c):
                for _ in range(4):
                    ky, kx = rng.integers(0, 4, 2)
                    ph = rng.uniform(0, 2 * np.pi)
                    out[b, :, :, ch] += rng.normal() * np.cos(2 * np.pi * (ky * yy / H + kx * xx / W) + ph)
        return out + 0.1 * rng.normal(size=out.shape)

    return field(B, cin).astype(np.float32), field(B, cout).astype(np.float32)


def unet_params_exact(levels: int, base: int, seed: int = 0) -> np.ndarray:
    """Parameters for which every network sum is exact in FP32: each output
    channel of each layer has one non-zero weight (+1 with probability 3/4,
    else -1) and a bias in {0, 1, 2, 3} / 16, so activations stay multiples of
    1/16 below 16 in magnitude (exact in bfloat16)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = [base << l for l in range(levels)]
    parts = []

    def layer(cout, taps, cin):
        w = np.zeros((cout, taps * cin))
        k = rng.integers(0, taps * cin, cout)
        w[np.arange(cout), k] = np.where(rng.uniform(size=cout) < 0.75, 1.0, -1.0)
        parts.append(w.ravel())
        parts.append(rng.integers(0, 4, cout) / 16.0)

    for l in range(levels):
        layer(C[l], 9, 8 if l == 0 else C[l - 1])
        layer(C[l], 9, C[l])
    for l in range(levels - 2, -1, -1):
        w = np.zeros((4, C[l], C[l + 1]))
        k = rng.integers(0, C[l + 1], (4, C[l]))
        for d in range(4):
            w[d, np.arange(C[l]), k[d]] = np.where(rng.uniform(size=C[l]) < 0.75, 1.0, -1.0)
        parts.append(w.ravel())
        parts.append(rng.integers(0, 4, C[l]) / 16.0)
        layer(C[l], 9, 2 * C[l])
        layer(C[l], 9, C[l])
    layer(8, 1, base)
    return np.concatenate(parts).astype(np.float32)


def unet_batch_exact(B: int, H: int, W: int, cin: int, cout: int, seed: int = 0):
    """Inputs and targets that are multiples of 1/16 in [-4, 4) (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(-64, 64, (B, H, W, cin)) / 16.0
    t = rng.integers(-64, 64, (B, H, W, cout)) / 16.0
    return x.astype(np.float32), t.astype(np.float32)


def two_layer_channel(nx=4, ny=34, y_i=16.5, tau1=1.0, tau2=2.0, force=1e-6, **kw) -> Case:
    """Wall-bounded D2Q9 channel with component 1 below the flat interface
    y = y_i and component 2 above it (tanh profile, width 2), each with its
    own relaxation time; uniform body force along x."""
    y = np.arange(ny, dtype=np.float64)
    psi = np.tanh((y_i - y) / 2.0)
    r1 = np.tile(((1 + psi) / 2)[:, None], (1, nx)).ravel()
    r2 = np.tile(((1 - psi) / 2)[:, None], (1, nx)).ravel()
    p = base_params(lattice=0, nx=nx, ny=ny, nz=1, walls_y=1, tau=tau1, tau2=tau2, A_nci=0.0,
                    force=(force, 0.0, 0.0), **kw)
    return Case(p, r1, r2)


# --- node-type geometries (fluid 0, solid 1, inlet 2, outlet 3) --------------
# Boundary conditions live in the library and the oracle; these only lay out
# the mask and the inlet values (carried in rho1, rho2, u at inlet nodes).

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3


def solid_wall_channel(nx=40, ny=34, force=1e-6, tau=1.0, two_phase=False, seed=0) -> Case:
    """Rows y = 0 and ny-1 solid on the periodic lattice (the walls_y channel
    expressed as a mask); single phase unless ``two_phase``."""
    t = np.zeros((ny, nx), np.uint8)
    t[0] = t[-1] = SOLID
    if two_phase:
        rng = np.random.Generator(np.random.PCG64(seed))
        psi = np.tanh(3.0 * rng.uniform(-1, 1, (ny, nx))).ravel()
        r1, r2 = _profile(psi)
    else:
        r1, r2 = np.ones(nx * ny), np.zeros(nx * ny)
    p = base_params(nx=nx, ny=ny, tau=tau, force=(force, 0.0, 0.0))
    return Case(p, r1, r2, None, {"type": t.ravel()})


def obstacle_box(nx=64, ny=48, lattice=0, nz=1, seed=1, A_nci=0.01) -> Case:
    """Closed periodic box with solid walls at y = 0, ny-1 and two solid
    blocks, random two-phase fields, no driving (mass must be conserved)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.zeros((nz, ny, nx), np.uint8)
    t[:, 0] = t[:, -1] = SOLID
    t[:, ny // 4:ny // 4 + 6, nx // 5:nx // 5 + 9] = SOLID
    t[:, ny // 2:ny // 2 + 10, (3 * nx) // 5:(3 * nx) // 5 + 5] = SOLID
    psi = np.tanh(3.0 * rng.uniform(-1, 1, (nz, ny, nx))).ravel()
    r1, r2 = _profile(psi)
    p = base_params(lattice=lattice, nx=nx, ny=ny, nz=nz, A_nci=A_nci)
    return Case(p, r1, r2, None, {"type": t.ravel()})


def inlet_outlet_channel(nx=48, ny=26, u_in=0.01, tau=1.0, rho1_in=1.0, rho2_in=0.0) -> Case:
    """Solid rows y = 0, ny-1; inlet column x = 0 with a plug velocity
    (u_in, 0); outlet column x = nx-1."""
    t = np.zeros((ny, nx), np.uint8)
    t[:, 0] = INLET
    t[:, -1] = OUTLET
    t[0] = t[-1] = SOLID
    N = nx * ny
    r1 = np.full(N, rho1_in)
    r2 = np.full(N, rho2_in)
    u = np.zeros((2, N))
    u[0, t.ravel() == INLET] = u_in
    p = base_params(nx=nx, ny=ny, tau=tau, A_nci=0.0)
    return Case(p, r1, r2, u, {"type": t.ravel(), "u_in": u_in})


def flow_focuser_2d(scale=1.0, phi=1.0, u_c=0.005, tau=1.0, A_s=0.05, N_c=0.1, h_min=2.0,
                    W_out=None, L_out=None) -> Case:
    """2-D flow-focuser (Fig. 1 layout): a horizontal dispersed-phase inlet
    channel of width H, two vertical continuous-phase inlet channels of width
    H entering from the bottom and top, a striction of width h = H/2, and an
    outlet channel (width ``W_out``, default 2h) ending in an outlet column.
    Lattice units at scale 1: H = 16 (the paper's 200 um), h = 8.  Inlet
    speeds u_c (continuous, both vertical inlets) and u_d = 2 phi u_c
    (dispersed); A = N_c sigma / h_min with sigma = 2 A_s tau / 9."""
    H = int(round(16 * scale))
    h = max(4, int(round(8 * scale)))
    W_out = 2 * h if W_out is None else W_out
    L_in = 2 * H                       # dispersed inlet channel length
    L_o = max(2, h)                    # striction length
    L_out = 10 * H if L_out is None else L_out
    ny = H + 2 * H + 2                 # vertical inlets (length H) above and below the junction
    ny = max(ny, W_out + 2)
    nx = 1 + L_in + H + L_o + L_out
    yc = ny // 2
    t = np.full((ny, nx), SOLID, np.uint8)
    y0, y1 = yc - H // 2, yc - H // 2 + H            # dispersed channel rows [y0, y1)
    xj = 1 + L_in                                    # junction columns [xj, xj + H)
    t[y0:y1, 0:xj] = FLUID
    t[1:ny - 1, xj:xj + H] = FLUID                   # vertical channels through the junction
    ho0 = yc - h // 2
    t[ho0:ho0 + h, xj + H:xj + H + L_o] = FLUID      # striction
    wo0 = yc - W_out // 2
    t[wo0:wo0 + W_out, xj + H + L_o:nx] = FLUID      # outlet channel
    t[y0:y1, 0] = INLET
    t[0, xj:xj + H] = INLET
    t[ny - 1, xj:xj + H] = INLET
    t[wo0:wo0 + W_out, nx - 1] = OUTLET
    N = nx * ny
    T = t.ravel()
    r1 = np.zeros((ny, nx)); r2 = np.ones((ny, nx))
    r1[y0:y1, 0:xj] = 1.0; r2[y0:y1, 0:xj] = 0.0     # dispersed phase fills its inlet channel
    u = np.zeros((2, ny, nx))
    u_d = 2.0 * phi * u_c
    u[0, y0:y1, 0] = u_d
    u[1, 0, xj:xj + H] = u_c
    u[1, ny - 1, xj:xj + H] = -u_c
    sigma = 2.0 * A_s * tau / 9.0
    p = base_params(nx=nx, ny=ny, tau=tau, A_s=A_s, A_nci=N_c * sigma / h_min, h_min=h_min)
    return Case(p, r1.ravel(), r2.ravel(), u.reshape(2, N),
                {"type": T, "H": H, "h": h, "W_out": W_out, "u_d": u_d, "u_c": u_c, "phi": phi,
                 "x_out0": xj + H + L_o, "junction": (xj, y0, y1)})
