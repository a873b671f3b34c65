"""Host-side reduction of the flow-focuser droplet samples (CPU only): a
synthetic train of droplets generated with a known period and speed, plus
satellites, gives the generation frequency and the main droplet volume."""
import numpy as np
import pytest

from paper_2003_11069_amd import focuser


@pytest.mark.parametrize("period,speed,every", [(6600, 0.007, 250), (3000, 0.012, 200)])
def test_generation_frequency_of_a_droplet_train(period, speed, every):
    rng = np.random.default_rng(2)
    x0, xc, L = 113, 200, 430
    samples = []
    for t in range(0, 200000, every):
        births = np.arange(0, t + 1, period)
        x = x0 + 5 + speed * (t - births)
        keep = x < L
        xs = x[keep]
        ys = 48.0 + rng.uniform(-1, 1, xs.size)
        vols = 425 + rng.integers(-8, 9, xs.size)
        # a satellite trailing each main droplet
        sx = xs - 12
        cen = np.concatenate([np.stack([xs, ys], 1), np.stack([sx, ys], 1)])
        vol = np.concatenate([vols, np.full(sx.size, 55)])
        sel = cen[:, 0] > x0
        samples.append((t, cen[sel], vol[sel]))
    v, n, nu = focuser.reduce_samples(samples, xc)
    assert v == pytest.approx(425, abs=8)
    assert nu == pytest.approx(1 / period, rel=0.05)
