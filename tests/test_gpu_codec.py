"""GPU test of the 16-bit storage codec (populations stored as FP16/BF16
deviations s_i = f_i/w_i - 1 from the lattice weights, the rest direction in
FP32), through the C ABI.

Three handles take one step from the same explicit two-population state: FP32
storage with FP32 arithmetic, and FP16 / BF16 storage with the same FP32
arithmetic.  The stored deviations, read back with lb_get_populations, must
(i) lie on the 16-bit grid (decoding yields format values, so encoding them
again is the identity), and (ii) differ from the FP32-stored ones by at most
half an ulp of the 16-bit format at that value (round to nearest), with a
few FP32 ulps of slack for the two instantiations' own arithmetic."""
import numpy as np
import pytest

import synth
import paper_2003_11069_amd as P
from gpu_common import say, fluid_mask

pytestmark = pytest.mark.gpu


def _bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to BF16 (via FP32, round to nearest even)."""
    f = x.astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_ulp(x: np.ndarray) -> np.ndarray:
    e = np.floor(np.log2(np.maximum(np.abs(x), 2.0 ** -126)))
    return 2.0 ** (e - 7)


def _deviations(g, f1, f2):
    return (f1 + f2) / g.w[:, None] - 1.0


@pytest.mark.parametrize("lat", [0, 1])
def test_codec_round_trip(lat):
    say(f"[gpu] codec round trip, lattice {lat}")
    if lat == 0:
        case = synth.random_fields(synth.base_params(lattice=0, nx=150, ny=37, A_nci=0.01), seed=21,
                                   umax=0.05)
    else:
        case = synth.random_fields(synth.base_params(lattice=1, nx=70, ny=19, nz=11, A_nci=0.01), seed=22,
                                   umax=0.05)
    hs = {}
    for st in ("fp32_f32", "fp16", "bf16"):
        g = P.Lattice(P.Params.from_dict(case.params, storage=P.STORAGE[st]))
        g.init_fields(case.rho1, case.rho2, case.u)
        g.step(1)
        hs[st] = (g, _deviations(g, *g.populations()))
    g32, s32 = hs["fp32_f32"]
    rest = g32.Q // 2
    mov = np.arange(g32.Q) != rest
    mask = fluid_mask(case.params, case.N)
    for st, rnd, ulp in (("fp16", lambda v: np.float16(v).astype(np.float64),
                          lambda v: np.spacing(np.abs(np.float16(v))).astype(np.float64)),
                         ("bf16", _bf16_round, _bf16_ulp)):
        _, s16 = hs[st]
        a = s16[mov][:, mask]
        b = s32[mov][:, mask]
        # (i) on the 16-bit grid up to the FP64 rebuild's rounding
        on_grid = np.abs(a - rnd(a)).max()
        # (ii) within half an ulp of the FP32-stored deviation
        slack = 4 * np.spacing(np.abs(b).astype(np.float32)).astype(np.float64) + 1e-15
        excess = (np.abs(a - b) - (0.5 * ulp(b) + slack)).max()
        # the FP32 rest slot closes the node mass, so it moves by the weighted
        # sum of the other directions' storage roundings at the same node
        # (plus FP32 rounding).  The read-back values are post-streaming: the
        # value node x stored for direction i is read at x + c_i (periodic).
        w, c = g32.w, g32.c
        shp = (case.params["nz"], case.params["ny"], case.params["nx"])
        ds = np.abs(s16 - s32).reshape((g32.Q,) + shp)
        bound = np.zeros(shp)
        for i in np.flatnonzero(mov):
            bound += w[i] * np.roll(ds[i], shift=(-c[i][2], -c[i][1], -c[i][0]), axis=(0, 1, 2))
        bound = bound.ravel() / w[rest] + 1e-6
        er = (np.abs(s16[rest] - s32[rest]) - bound)[mask].max()
        say(f"  {st}: off-grid {on_grid:.2e}, max |s16 - s32| - ulp/2 {excess:.2e}, "
            f"max |ds| {np.abs(a - b).max():.2e}, rest excess over its bound {er:.2e}")
        assert on_grid <= 1e-13
        assert excess <= 0
        assert er <= 0
