"""FP64 CPU oracle of the warm-start U-Net (forward, loss, backward, Adam).

TEST INFRASTRUCTURE ONLY.  The test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users; the GPU library never
imports it and it shares no code with the GPU path.

The lattice Boltzmann paper has no learned part: this network is the learned
warm start layered on top of the method (a U-Net mapping a channel's initial
phase field, pressure-gradient plane and NCI-strength plane to its steady
phase and velocity fields).  Its definition here is the plain one:

  conv KxK (zero padding K//2, stride 1):
      out[b,y,x,co] = bias[co] + sum_{ky,kx,ci} W[co,ky,kx,ci] in[b, y+ky-K//2, x+kx-K//2, ci]
  2x2 max pool, stride 2; gradient to the first maximum in window order
      (0,0), (0,1), (1,0), (1,1)
  2x2 stride-2 transposed conv:
      out[b, 2y+dy, 2x+dx, co] = bias[co] + sum_ci W[dy,dx,co,ci] in[b,y,x,ci]
  loss = mean over all outputs of (y - target)^2
  Adam with bias-corrected first and second moments.

Network (levels L, base C0, C_l = C0 * 2^l): per encoder level two 3x3
conv+ReLU then a pool (not at the bottom); per decoder level a transposed
conv, concatenation [up-sampled | encoder output], two 3x3 conv+ReLU; a 1x1
head without activation.  The input is zero-padded to 8 channels and the
head has 8 outputs of which the first `cout` are used.  The flat parameter
order is: encoder levels 0..L-1 (e1.W, e1.b, e2.W, e2.b), decoder levels
L-2..0 (up.W, up.b, d1.W, d1.b, d2.W, d2.b), head (W, b).

Precision.  With ``rounding=True`` values are rounded to bfloat16 (round to
nearest even) where the GPU stores BF16 -- the packed input, every weight,
every hidden layer output after bias and ReLU, and each backward operand
(output gradient times the ReLU mask) -- and everything else is FP64, so the
remaining GPU difference is FP32 accumulation, plus two roundings the GPU
adds on the pooling path (it stores the pooled gradient, and the sum of the
skip and pooled gradients, in BF16; here both stay FP64).  With
``rounding=False`` the network is plain FP64 (used for finite differences).

Parity: pinned by finite differences of the FP64 loss (all parameters and
layer kinds), by scipy's 2-D cross-correlation, by a Kronecker-product form
of the transposed conv, by reshape-max pooling, by torch's bfloat16
conversion and by the closed form of Adam under a constant gradient.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), as FP64."""
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.uint64).copy()
    drop = 52 - 7  # bfloat16 keeps 7 explicit mantissa bits
    lsb = (bits >> np.uint64(drop)) & np.uint64(1)
    bits = bits + np.uint64((1 << (drop - 1)) - 1) + lsb
    bits &= ~np.uint64((1 << drop) - 1)
    out = bits.view(np.float64)
    return np.where(np.isfinite(x), out, x)


@dataclass(frozen=True)
class Config:
    levels: int = 4
    base: int = 32
    cin: int = 3
    cout: int = 3
    H: int = 128
    W: int = 256


def layer_shapes(cfg: Config):
    """Ordered list of (name, kind, weight shape, bias length)."""
    L, C0 = cfg.levels, cfg.base
    C = [C0 << l for l in range(L)]
    out = []
    for l in range(L):
        cin = 8 if l == 0 else C[l - 1]
        out.append((f"e1.{l}", "conv", (C[l], 3, 3, cin), C[l]))
        out.append((f"e2.{l}", "conv", (C[l], 3, 3, C[l]), C[l]))
    for l in range(L - 2, -1, -1):
        out.append((f"up.{l}", "up", (2, 2, C[l], C[l + 1]), C[l]))
        out.append((f"d1.{l}", "conv", (C[l], 3, 3, 2 * C[l]), C[l]))
        out.append((f"d2.{l}", "conv", (C[l], 3, 3, C[l]), C[l]))
    out.append(("head", "conv", (8, 1, 1, C0), 8))
    return out


def num_params(cfg: Config) -> int:
    return sum(int(np.prod(w)) + b for _, _, w, b in layer_shapes(cfg))


def unpack(cfg: Config, flat: np.ndarray) -> dict:
    """Flat vector -> {name: (W, b)} views (FP64 copies)."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == num_params(cfg)
    d, off = {}, 0
    for name, _, ws, nb in layer_shapes(cfg):
        nw = int(np.prod(ws))
        d[name] = (flat[off:off + nw].reshape(ws), flat[off + nw:off + nw + nb])
        off += nw + nb
    return d


def pack(cfg: Config, grads: dict) -> np.ndarray:
    parts = []
    for name, _, ws, nb in layer_shapes(cfg):
        gw, gb = grads[name]
        parts += [np.asarray(gw).reshape(-1), np.asarray(gb).reshape(-1)]
    return np.concatenate(parts)


# --- layers (plain definitions) ---------------------------------------------

def conv_fwd(x, W, b):
    """x [B,H,W,Cin], W [Cout,K,K,Cin] -> pre-activation [B,H,W,Cout]."""
    Bn, H, Wd, _ = x.shape
    K = W.shape[1]
    r = K // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    out = np.zeros((Bn, H, Wd, W.shape[0]))
    for ky in range(K):
        for kx in range(K):
            out += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[:, ky, kx, :].T
    return out + b


def conv_bwd(x, W, dpre):
    """Gradients of conv_fwd: (dx, dW, db) for the pre-activation gradient dpre."""
    Bn, H, Wd, Cin = x.shape
    K = W.shape[1]
    r = K // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    g2 = dpre.reshape(-1, dpre.shape[-1])
    for ky in range(K):
        for kx in range(K):
            patch = xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, Cin)
            dW[:, ky, kx, :] = g2.T @ patch
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dpre @ W[:, ky, kx, :]
    dx = dxp[:, r:r + H, r:r + Wd, :]
    return dx, dW, g2.sum(axis=0)


def pool_fwd(x):
    """2x2 max pool; also returns the window index (2dy+dx) of the first max."""
    Bn, H, Wd, Cn = x.shape
    win = np.stack([x[:, dy::2, dx::2, :] for dy in (0, 1) for dx in (0, 1)], axis=0)
    return win.max(axis=0), win.argmax(axis=0)


def pool_bwd(dout, arg, shape):
    dx = np.zeros(shape)
    for d in range(4):
        dy, dxx = d >> 1, d & 1
        dx[:, dy::2, dxx::2, :] += np.where(arg == d, dout, 0.0)
    return dx


def up_fwd(x, W, b):
    """x [B,h,w,Cin], W [2,2,Cout,Cin] -> [B,2h,2w,Cout]."""
    Bn, h, w, _ = x.shape
    out = np.zeros((Bn, 2 * h, 2 * w, W.shape[2]))
    for dy in (0, 1):
        for dx in (0, 1):
            out[:, dy::2, dx::2, :] = x @ W[dy, dx].T + b
    return out


def up_bwd(x, W, dout):
    Cin = x.shape[-1]
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for dy in (0, 1):
        for dxx in (0, 1):
            g = dout[:, dy::2, dxx::2, :]
            dx += g @ W[dy, dxx]
            dW[dy, dxx] = g.reshape(-1, g.shape[-1]).T @ x.reshape(-1, Cin)
    return dx, dW, dout.reshape(-1, dout.shape[-1]).sum(axis=0)


# --- network ------------------------------------------------------------------

def _q(a, rounding):
    return bf16(a) if rounding else a


def forward(cfg: Config, params, x, rounding=True):
    """x [B,H,W,cin] -> (y [B,H,W,cout], cache for backward)."""
    L = cfg.levels
    P = unpack(cfg, params)
    Wq = {k: (_q(w, rounding), b) for k, (w, b) in P.items()}
    Bn = x.shape[0]
    x8 = np.zeros((Bn, cfg.H, cfg.W, 8))
    x8[..., :cfg.cin] = x
    x8 = _q(x8, rounding)
    c = {"x8": x8, "W": Wq}
    h = x8
    for l in range(L):
        if l > 0:
            h, c[f"arg{l}"] = pool_fwd(c[f"e{l - 1}"])
            c[f"pin{l}"] = h
        a1 = _q(np.maximum(conv_fwd(h, *Wq[f"e1.{l}"]), 0.0), rounding)
        a2 = _q(np.maximum(conv_fwd(a1, *Wq[f"e2.{l}"]), 0.0), rounding)
        c[f"ein{l}"], c[f"m{l}"], c[f"e{l}"] = h, a1, a2
    h = c[f"e{L - 1}"]
    for l in range(L - 2, -1, -1):
        u = _q(up_fwd(h, *Wq[f"up.{l}"]), rounding)
        cat = np.concatenate([u, c[f"e{l}"]], axis=-1)
        a1 = _q(np.maximum(conv_fwd(cat, *Wq[f"d1.{l}"]), 0.0), rounding)
        a2 = _q(np.maximum(conv_fwd(a1, *Wq[f"d2.{l}"]), 0.0), rounding)
        c[f"uin{l}"], c[f"cat{l}"], c[f"dm{l}"], c[f"dec{l}"] = h, cat, a1, a2
        h = a2
    y8 = conv_fwd(h, *Wq["head"])
    c["y8"] = y8
    return y8[..., :cfg.cout], c


def loss_and_grads(cfg: Config, params, x, target, rounding=True):
    """Mean-squared-error loss and its gradient (flat, parameter order)."""
    L = cfg.levels
    y, c = forward(cfg, params, x, rounding)
    Wq = c["W"]
    n = y.size
    loss = float(np.sum((y - target) ** 2) / n)
    dy8 = np.zeros_like(c["y8"])
    dy8[..., :cfg.cout] = 2.0 * (y - target) / n
    G = {}

    def relu_layer(name, inp, act, dout):
        dpre = _q(np.where(act > 0, dout, 0.0), rounding)
        dx, dW, db = conv_bwd(inp, Wq[name][0], dpre)
        G[name] = (dW, db)
        return dx

    dx, dW, db = conv_bwd(c["dec0"] if L > 1 else c[f"e{L - 1}"], Wq["head"][0], _q(dy8, rounding))
    G["head"] = (dW, db)
    dh = dx
    dskip = {}
    for l in range(0, L - 1):
        dm = relu_layer(f"d2.{l}", c[f"dm{l}"], c[f"dec{l}"], dh)
        dcat = relu_layer(f"d1.{l}", c[f"cat{l}"], c[f"dm{l}"], dm)
        Cl = cfg.base << l
        du, dskip[l] = dcat[..., :Cl], dcat[..., Cl:]
        dx, dW, db = up_bwd(c[f"uin{l}"], Wq[f"up.{l}"][0], _q(du, rounding))
        G[f"up.{l}"] = (dW, db)
        dh = dx  # gradient of the decoder output of level l+1 (or of the bottom)
    de = dh
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            de = dskip[l] + pool_bwd(dpool, c[f"arg{l + 1}"], c[f"e{l}"].shape)
        dm = relu_layer(f"e2.{l}", c[f"m{l}"], c[f"e{l}"], de)
        dpool = relu_layer(f"e1.{l}", c[f"ein{l}"], c[f"m{l}"], dm)
    return loss, pack(cfg, G)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam step (t = step number after this update, starting at 1)."""
    g = g + wd * w
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
