"""GPU parity of the density-ratio variant (rho_ratio = gamma, alpha1)
against the FP64 oracle running the same variant: free runs of 200 steps on
droplets, a walled channel and a 3-D box (FP32 at the 1e-5 bar, FP16 within
its budget); the flat-interface pressure balance reached on the GPU; and the
equal-density case expressed through the variant equal to the default path."""
import numpy as np
import pytest

import synth
import paper_2003_11069_amd as P
from gpu_common import say, make_pair, fluid_mask, field_errors

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _ratio_case(case, gamma):
    """Component 2 at its reference density 1/gamma."""
    return synth.Case(dict(case.params), case.rho1, case.rho2 / gamma, case.u, case.info)


CASES = {
    "two_droplets_g2": (lambda: synth.two_droplets_2d(nx=100, ny=46, R=10, gap=3.0, jitter=0.4, seed=5,
                                                      A_nci=0.02), 2.0, 0.8),
    "channel_2d_g3": (lambda: synth.channel_2d(synth.channel_spec(11, Lx=160, Ly=50)), 3.0, 0.85),
    "periodic_3d_g2": (lambda: synth.random_fields(synth.base_params(lattice=1, nx=36, ny=20, nz=12,
                                                                     A_nci=0.01), seed=9), 2.0, 0.8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_free_run_parity_200(name):
    make, gamma, a1 = CASES[name]
    case = _ratio_case(make(), gamma)
    say(f"[gpu] density ratio {gamma}, alpha1 {a1}: {name}, 200 steps")
    o, g = make_pair(case, rho_ratio=gamma, alpha1=a1)
    o.step(200)
    g.step(200)
    e = field_errors(o, g, fluid_mask(case.params, case.N))
    say(f"  errors {e}")
    assert e["rho1"] <= TOL and e["rho2"] <= TOL and e["u"] <= TOL


def test_fp16_within_budget():
    """The deviations s = f/w - 1 of the lighter phase are about 1/gamma - 1
    rather than near 0, so FP16 storage rounds them more coarsely than at
    equal densities: the budget here is about three times the measured
    rho 3.4e-3, u 6.1e-2."""
    make, gamma, a1 = CASES["two_droplets_g2"]
    case = _ratio_case(make(), gamma)
    say("[gpu] density ratio 2, FP16 storage, 200 steps")
    o, g = make_pair(case, storage="fp16", rho_ratio=gamma, alpha1=a1)
    o.step(200)
    g.step(200)
    e = field_errors(o, g, fluid_mask(case.params, case.N))
    say(f"  errors {e}")
    assert e["rho1"] <= 1e-2 and e["rho2"] <= 1e-2 and e["u"] <= 0.18


@pytest.mark.parametrize("gamma,a1", [(2.0, 0.8), (4.0, 0.9)])
def test_flat_interface_pressure_balance(gamma, a1):
    nx, ny = 96, 4
    X = np.arange(nx)
    psi = np.tile(np.tanh((20 - np.abs(X - nx / 2)) / 2.0), (ny, 1)).ravel()
    r1, r2 = (1 + psi) / 2, (1 - psi) / 2
    say(f"[gpu] flat interface, density ratio {gamma}, 20000 steps")
    g = P.Lattice(P.Params.from_dict(synth.base_params(nx=nx, ny=ny, A_nci=0.0), rho_ratio=gamma, alpha1=a1))
    g.init_fields(r1, r2)
    g.step(20000)
    f1, f2, u = g.fields()
    ratio = f1.reshape(ny, nx)[:, nx // 2].mean() / f2.reshape(ny, nx)[:, 2].mean()
    say(f"  bulk density ratio {ratio:.6f}, max |u| {np.abs(u).max():.2e}")
    assert ratio == pytest.approx(gamma, rel=1e-3) and np.abs(u).max() < 1e-4


def test_equal_densities_through_the_variant():
    case = synth.two_droplets_2d(nx=64, ny=40, R=8, gap=3.0, jitter=0.4, seed=3, A_nci=0.01)
    say("[gpu] rho_ratio 1, alpha1 4/9 against the default path, 200 steps")
    a = P.Lattice(P.Params.from_dict(case.params))
    b = P.Lattice(P.Params.from_dict(case.params, rho_ratio=1.0, alpha1=4 / 9))
    for g in (a, b):
        g.init_fields(case.rho1, case.rho2)
        g.step(200)
    # psi is formed by a different expression (rounding 1e-16), which the FP32
    # collision carries to about 1e-9 in 200 steps
    for x, y in zip(a.fields(), b.fields()):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-7)
