"""GPU test of lb_get_fields_static, the allocation-free variant of
lb_get_fields (fields staged through the library's fixed per-device scratch
array): called through the C ABI, its output must equal lb_get_fields' bit
for bit on two calls in a row, the second on a smaller lattice (so the
scratch still holds the first call's larger contents), and a lattice whose
fields exceed the scratch is rejected before anything runs."""
import ctypes as C

import numpy as np
import pytest

import synth
import paper_2003_11069_amd as P
from gpu_common import say

pytestmark = pytest.mark.gpu


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _static_fields(g):
    lib = P.load_library()
    r1 = np.full(g.N, np.nan); r2 = np.full(g.N, np.nan); u = np.full(g.p.dim * g.N, np.nan)
    rc = lib.lb_get_fields_static(g.h, _dp(r1), _dp(r2), _dp(u))
    return rc, (r1, r2, u.reshape(g.p.dim, g.N))


def test_static_fields_equal_allocating_fields():
    c3 = synth.hex_channel_3d(nx=70, ny=21, nz=9, R=4.0, z_pitch=9.0, seed=4, force=2e-5)
    c2 = synth.two_droplets_2d(nx=64, ny=30, R=8, gap=3.0, jitter=0.4, seed=3, A_nci=0.02)
    for name, case, steps in (("3-D channel 70x21x9 (walls)", c3, 23), ("2-D box 64x30", c2, 11)):
        say(f"[gpu] lb_get_fields_static: {name}")
        g = P.Lattice(P.Params.from_dict(case.params))
        g.init_fields(case.rho1, case.rho2, case.u)
        g.step(steps)
        rc, got = _static_fields(g)
        assert rc == 0, P.load_library().lb_last_error()
        ref = g.fields()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        g.close()


def test_static_fields_reject_oversized_lattice():
    say("[gpu] lb_get_fields_static: oversized lattice rejected")
    p = P.Params(lattice=P.LB_D2Q9, nx=2048, ny=1025, nz=1)
    g = P.Lattice(p)
    N = p.nx * p.ny
    g.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    rc, _ = _static_fields(g)
    assert rc == -1 and b"static scratch" in P.load_library().lb_last_error()
