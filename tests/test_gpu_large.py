"""GPU parity on a lattice larger than one 32-bit byte offset can span.

The stored deviations of all Q directions take Q N sizeof(S) bytes; with a
64-bit base per direction only N sizeof(S) must stay below 4 GiB.  This
D3Q27 FP32 channel (384 x 256 x 416 = 40.9 M nodes, walls, body force) has
Q N 4 B = 4.42 GB, above 2^32 bytes, so directions beyond the 9th start past
the 4 GiB mark.  Three steps against the FP64 oracle at the 1e-5 bar (NCI
off: with random fields its discontinuous decisions would make single nodes
of a 40 M-node lattice flip, which is not what this test is about)."""
import numpy as np
import pytest

import synth
from gpu_common import say, make_pair, fluid_mask, field_errors

pytestmark = pytest.mark.gpu


def test_lattice_beyond_4GiB_of_state():
    p = synth.base_params(lattice=1, nx=384, ny=256, nz=416, walls_y=1, A_nci=0.0, force=(1e-5, 0.0, 0.0))
    N = p["nx"] * p["ny"] * p["nz"]
    assert 27 * N * 4 > 2 ** 32
    say(f"[gpu] large lattice D3Q27 {p['nx']}x{p['ny']}x{p['nz']} = {N} nodes, 3 steps (oracle on the host)")
    case = synth.random_fields(p, seed=77, umax=0.01)
    o, g = make_pair(case)
    o.step(3)
    g.step(3)
    e = field_errors(o, g, fluid_mask(case.params, case.N))
    say(f"  errors {e}")
    assert e["rho1"] <= 1e-5 and e["rho2"] <= 1e-5 and e["u"] <= 1e-5
