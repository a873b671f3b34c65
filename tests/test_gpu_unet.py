"""GPU parity of the warm-start U-Net (BF16 MFMA kernels, FP32 accumulation)
against the FP64 oracle that rounds to BF16 at the same points.

Tolerance.  Both sides round every stored activation and backward operand to
BF16; they differ only in accumulation (FP32 on the GPU, FP64 in the oracle).
Where that difference crosses a BF16 rounding boundary the stored value moves
by one BF16 ulp (2^-8 relative), and in a deep network such flips cascade
until every rounding stage contributes noise of that order with random sign.
The relative L2 error of a result that has passed through n rounding stages
is therefore bounded by 2^-8 * sqrt(n): n = 1 + 5L - 3 stages for the output
(packed input, 2 convs per encoder level, up + 2 convs per decoder level) and
twice that for a parameter gradient (forward plus backward operands).  That
bound applies to the whole output and the whole gradient; a single small
layer sees the noise of only a few flips, so per-layer errors are allowed 4x.
Index and routing errors are excluded separately, bit for bit, by the
exact-arithmetic cases at the end of this file."""
import math

import numpy as np
import pytest

import synth
from oracle import unet as U
from paper_2003_11069_amd import ws
from gpu_common import say

pytestmark = pytest.mark.gpu


def _stages(L):
    return 1 + 2 * L + 3 * (L - 1)


def tol_out(L):
    return 2 ** -8 * math.sqrt(_stages(L))


def tol_grad(L):
    return 2 ** -8 * math.sqrt(2 * _stages(L))


def _net(L, base, H, W, B, cin=3, cout=3, seed=1):
    cfg = ws.UNetConfig(levels=L, base=base, cin=cin, cout=cout, H=H, W=W, max_batch=B)
    net = ws.UNet(cfg)
    ocfg = U.Config(levels=L, base=base, cin=cin, cout=cout, H=H, W=W)
    assert net.n_params == U.num_params(ocfg)
    p = synth.unet_params(L, base, seed=seed)
    net.set_params(p)
    return net, ocfg, p


def _layer_errors(ocfg, g_or, g_gpu):
    out, off = [], 0
    for name, _, ws_, nb in U.layer_shapes(ocfg):
        nw = int(np.prod(ws_))
        for lo, n, tag in [(off, nw, "W"), (off + nw, nb, "b")]:
            a, b = g_or[lo:lo + n], g_gpu[lo:lo + n].astype(np.float64)
            if name == "head":  # only the used outputs carry gradient
                a, b = (a.reshape(8, -1)[:ocfg.cout], b.reshape(8, -1)[:ocfg.cout])
            out.append((f"{name}.{tag}", np.linalg.norm(a - b) / np.linalg.norm(a)))
        off += nw + nb
    return out


def _grad_error(ocfg, g_or, g_gpu):
    """Relative L2 error of the whole gradient (used head outputs only)."""
    keep = np.ones(g_or.size, bool)
    off = g_or.size - 8 * ocfg.base - 8
    keep[off:off + 8 * ocfg.base] = np.repeat(np.arange(8) < ocfg.cout, ocfg.base)
    keep[-8:] = np.arange(8) < ocfg.cout
    a, b = g_or[keep], g_gpu[keep].astype(np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(a)


CASES = [
    # levels, base, H, W, batch   (ragged N = 8 and K = 72 / 216, non-square images)
    (2, 8, 16, 32, 3),
    (3, 24, 32, 32, 2),
    (2, 16, 16, 32, 3),
    # channel counts of 32 and 64 on whole 8 x 32 tiles: the direct 3x3 kernels
    # (level 2 of the second, 8 x 16, falls back to the implicit GEMM)
    (2, 32, 16, 64, 2),
    (3, 32, 32, 64, 2),
    # wide heads: the training head with 64 and 136 input channels (channel
    # tiles padded to 64 and 256; the latter needs more than 64 KB of LDS)
    (2, 64, 16, 32, 2),
    (2, 136, 16, 32, 1),
    # deep nets: five and six levels (direct kernels on the levels whose
    # images are whole tiles, the implicit GEMM below; one side-stream fork
    # per level)
    (5, 8, 128, 128, 1),
    (6, 8, 256, 256, 1),
]


@pytest.mark.parametrize("L,base,H,W,B", CASES)
def test_forward_and_gradients_match_oracle(L, base, H, W, B):
    say(f"[gpu] unet L={L} base={base} {H}x{W} batch {B}")
    net, ocfg, p = _net(L, base, H, W, B)
    x, t = synth.unet_batch(B, H, W, 3, 3, seed=11)
    y = net.forward(x)
    yo, _ = U.forward(ocfg, p.astype(np.float64), x.astype(np.float64))
    e_inf = np.abs(y - yo).max() / np.abs(yo).max()
    e_2 = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    loss = net.backward(x, t)
    lo, go = U.loss_and_grads(ocfg, p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    errs = _layer_errors(ocfg, go, net.grads())
    worst = max(errs, key=lambda e: e[1])
    e_g = _grad_error(ocfg, go, net.grads())
    say(f"  y rel Linf {e_inf:.2e} L2 {e_2:.2e}; loss {loss:.6e} vs {lo:.6e}; grad L2 {e_g:.2e}, "
        f"worst layer {worst[0]} {worst[1]:.2e} (tol {tol_grad(L):.2e})")
    assert e_2 <= tol_out(L) and e_inf <= 4 * tol_out(L)
    assert loss == pytest.approx(lo, rel=1e-3)
    assert e_g <= tol_grad(L)
    assert worst[1] <= 4 * tol_grad(L), errs
    g = net.grads()
    off = net.n_params - 8 * base - 8
    assert np.all(g[off:off + 8 * base].reshape(8, base)[3:] == 0) and np.all(g[-5:] == 0)


def test_full_size_network_matches_oracle():
    """The 4-level, 32-base network on 128 x 256 images (the warm-start
    shape), batch 2: all outputs and every layer's gradients."""
    L, base, H, W, B = 4, 32, 128, 256, 2
    say(f"[gpu] unet full size L={L} base={base} {H}x{W} batch {B}")
    net, ocfg, p = _net(L, base, H, W, B, seed=3)
    x, t = synth.unet_batch(B, H, W, 3, 3, seed=12)
    y = net.forward(x)
    loss = net.backward(x, t)
    lo, go = U.loss_and_grads(ocfg, p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    yo, _ = U.forward(ocfg, p.astype(np.float64), x.astype(np.float64))
    e_2 = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    errs = _layer_errors(ocfg, go, net.grads())
    worst = max(errs, key=lambda e: e[1])
    e_g = _grad_error(ocfg, go, net.grads())
    say(f"  y rel L2 {e_2:.2e} (tol {tol_out(L):.2e}); loss rel {abs(loss - lo) / lo:.2e}; "
        f"grad L2 {e_g:.2e}, worst layer {worst[0]} {worst[1]:.2e} (tol {tol_grad(L):.2e})")
    assert e_2 <= tol_out(L)
    assert loss == pytest.approx(lo, rel=1e-3)
    assert e_g <= tol_grad(L)
    assert worst[1] <= 4 * tol_grad(L), errs


def test_smaller_batch_and_determinism():
    """A batch below max_batch uses only its images; repeated backward passes
    give bit-identical gradients (fixed-order split reductions)."""
    net, ocfg, p = _net(2, 16, 16, 32, 4)
    x, t = synth.unet_batch(4, 16, 32, 3, 3, seed=13)
    y4 = net.forward(x)
    y2 = net.forward(x[:2])
    assert np.array_equal(y2, y4[:2])
    net.backward(x[:3], t[:3])
    g1 = net.grads()
    net.backward(x, t)
    net.backward(x[:3], t[:3])
    assert np.array_equal(g1, net.grads())
    with pytest.raises(ws.WSError):
        net.forward(np.zeros((5, 16, 32, 3), np.float32))


def test_one_training_step_matches_oracle():
    """ws_train_step = backward + Adam (t = 1): the loss equals the oracle's
    and the parameters move as the oracle's Adam step from the oracle's
    gradient wherever that gradient is not within the accumulation noise of
    zero (there the sign of a first Adam step is not determined)."""
    L, base, H, W, B = 2, 8, 16, 32, 3
    net, ocfg, p = _net(L, base, H, W, B)
    x, t = synth.unet_batch(B, H, W, 3, 3, seed=14)
    dx, dt = ws.DeviceArray.from_host(x), ws.DeviceArray.from_host(t)
    lr = 1e-3
    loss = net.train_step_ptr(dx.ptr(), dt.ptr(), B, lr, want_loss=True)
    lo, go = U.loss_and_grads(ocfg, p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    w_or, _, _ = U.adam(p.astype(np.float64), go, np.zeros_like(go), np.zeros_like(go), 1, lr)
    w = net.params().astype(np.float64)
    assert loss == pytest.approx(lo, rel=1e-3)
    firm = np.abs(go) > 1e-3 * np.abs(go).max()
    d = np.abs(w - w_or)
    say(f"  firm {firm.mean():.3f}; max |dw| firm {d[firm].max():.2e}, all {d.max():.2e}")
    assert np.all(d[firm] <= 2 ** -23 * np.abs(w_or[firm]) + 1e-4 * lr)
    assert np.all(d <= 2 * lr * (1 + 1e-6) + 2 ** -23 * np.abs(w_or))


def test_training_reduces_loss():
    L, base, H, W, B = 3, 16, 32, 64, 4
    net, ocfg, p = _net(L, base, H, W, B)
    x, t = synth.unet_batch(B, H, W, 3, 3, seed=15)
    dx, dt = ws.DeviceArray.from_host(x), ws.DeviceArray.from_host(t)
    l0 = net.backward_ptr(dx.ptr(), dt.ptr(), B)
    for _ in range(60):
        net.train_step_ptr(dx.ptr(), dt.ptr(), B, 2e-3)
    l1 = net.backward_ptr(dx.ptr(), dt.ptr(), B)
    say(f"  loss {l0:.4e} -> {l1:.4e}")
    assert l1 < 0.5 * l0


EXACT = [(2, 8, 16, 32, 2, 4), (3, 24, 32, 32, 2, 2), (2, 32, 16, 64, 2, 4), (3, 32, 32, 64, 1, 2),
         (4, 32, 128, 256, 1, 2), (2, 64, 16, 32, 2, 4), (5, 8, 128, 128, 1, 4)]


@pytest.mark.parametrize("L,base,H,W,B,cout", EXACT)
def test_exact_arithmetic_bit_identical(L, base, H, W, B, cout):
    """Sparse +-1 weights and 1/16-quantised biases, inputs and targets make
    every sum exact in FP32 and every stored value exact in BF16, and the
    batch size makes the loss normalisation a power of two: the GPU must then
    reproduce the oracle bit for bit (indexing, padding, skip routing, pool
    tie-breaking and the ReLU masks, free of rounding effects)."""
    say(f"[gpu] unet exact L={L} base={base} {H}x{W} batch {B} cout {cout}")
    cfg = ws.UNetConfig(levels=L, base=base, cin=3, cout=cout, H=H, W=W, max_batch=B)
    net = ws.UNet(cfg)
    ocfg = U.Config(levels=L, base=base, cin=3, cout=cout, H=H, W=W)
    p = synth.unet_params_exact(L, base, seed=1)
    net.set_params(p)
    x, t = synth.unet_batch_exact(B, H, W, 3, cout, seed=2)
    y = net.forward(x)
    loss = net.backward(x, t)
    g = net.grads()
    yo, _ = U.forward(ocfg, p.astype(np.float64), x.astype(np.float64))
    lo, go = U.loss_and_grads(ocfg, p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    bad_y = np.argwhere(y != yo)
    bad_g = np.flatnonzero(g != go)
    say(f"  y mismatches {len(bad_y)} of {y.size}; grad mismatches {len(bad_g)} of {g.size}; loss {loss} vs {lo}")
    if len(bad_y):
        say(f"  first y mismatches (b,y,x,c): {bad_y[:8].tolist()}")
    if len(bad_g):
        names, off = [], 0
        for name, _, ws_, nb in U.layer_shapes(ocfg):
            n = int(np.prod(ws_)) + nb
            k = np.count_nonzero((bad_g >= off) & (bad_g < off + n))
            if k:
                names.append(f"{name}:{k}")
            off += n
        say(f"  grad mismatches by layer: {names}")
    assert len(bad_y) == 0
    assert loss == lo
    assert len(bad_g) == 0


def test_direct_and_gemm_paths_agree_and_repeat():
    """conv_algo 0 (direct 3x3 kernels) and 1 (implicit GEMM only) compute the
    same network and differ only in FP32 summation order, so they agree to
    the accumulation-noise bound; the direct path repeats bit for bit, and a
    smaller batch uses only its images."""
    L, base, H, W, B = 2, 32, 16, 64, 3
    p = synth.unet_params(L, base, seed=3)
    x, t = synth.unet_batch(B, H, W, 3, 3, seed=16)
    res = {}
    for algo in (0, 1):
        net = ws.UNet(ws.UNetConfig(levels=L, base=base, cin=3, cout=3, H=H, W=W, max_batch=B, conv_algo=algo))
        net.set_params(p)
        y = net.forward(x)
        net.backward(x, t)
        res[algo] = (y, net.grads(), net)
    (y0, g0, net0), (y1, g1, _) = res[0], res[1]
    ey = np.linalg.norm(y0 - y1) / np.linalg.norm(y1)
    eg = np.linalg.norm(g0.astype(np.float64) - g1) / np.linalg.norm(g1)
    say(f"  direct vs implicit GEMM: y rel L2 {ey:.2e}, grad rel L2 {eg:.2e}")
    assert ey <= tol_out(L) and eg <= tol_grad(L)
    net0.backward(x, t)
    assert np.array_equal(net0.grads(), g0)
    assert np.array_equal(net0.forward(x[:2]), y0[:2])
