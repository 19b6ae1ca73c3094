"""Oracle: the paper's own U-Net layer set (Section 3.1, Table 2) as a second preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Table 2 fixes: 5 input and 2 output channels, depth 4, 32 channels per layer, PReLU activations,
8x8 convolutions with stride 2 and padding 3, batch normalisation and biases. It does not draw
the graph; the reading adopted here:

  * input: X as in unet.py (RMS-scaled Re v, Im v, c / c_ref, sigma_x, sigma_y), zero-padded at
    the bottom/right to a multiple of 2^depth (16);
  * encoder, l = 1..depth: E_l = prelu(down(E_{l-1})), E_0 = X, where down is the 8x8 stride-2
    padding-3 convolution (it halves each side), 32 channels;
  * decoder: U_{depth-1} = prelu(up(E_depth)); for l = depth-2 .. 0,
    U_l = prelu(up(concat[E_{l+1}, U_{l+1}])), where up is the 8x8 stride-2 padding-3 transposed
    convolution (it doubles each side), 32 channels; the skip part comes first in the concat;
  * head: 1x1 convolution to 2 channels, no activation; z = s (out_0 + i out_1), cropped.

Batch normalisation at inference is a per-channel affine map, which folds into the preceding
convolution's weight and bias; the parameters here are that folded inference form. PReLU has one
slope per layer (x for x > 0, a x otherwise). Each layer stores its weight (down / head:
[out, in, kh, kw]; up: [in, out, 8, 8]), its bias, then (down and up) its slope. With depth 4 the
network has 665,930 parameters; Table 2's graph is not drawn, and its quoted count of about 832 K
is not reproduced by this reading.

Definitions (cross-correlation, as in deep-learning libraries):
  down: y[o, i, j] = b[o] + sum_{c, a, e} W[o, c, a, e] x[c, 2 i + a - 3, 2 j + e - 3]
  up:   y[o, 2 i + a - 3, 2 j + e - 3] += W[c, o, a, e] x[c, i, j] (all i, j, a, e), then + b[o]
with x = 0 outside its grid and output positions outside the output grid dropped.
"""
from __future__ import annotations

import numpy as np

from . import helmholtz as hz
from .unet import pack_input

K8, S8, P8 = 8, 2, 3


def layer_specs(depth: int = 4, ch: int = 32, in_ch: int = 5, out_ch: int = 2):
    """[(name, kind, cin, cout)] with kind in {'down', 'up', 'conv1'}."""
    specs, cin = [], in_ch
    for l in range(1, depth + 1):
        specs.append((f"down{l}", "down", cin, ch))
        cin = ch
    specs.append((f"up{depth - 1}", "up", ch, ch))
    for l in range(depth - 2, -1, -1):
        specs.append((f"up{l}", "up", 2 * ch, ch))
    specs.append(("head", "conv1", ch, out_ch))
    return specs


def weight_shape(kind, cin, cout):
    return {"down": (cout, cin, K8, K8), "up": (cin, cout, K8, K8), "conv1": (cout, cin, 1, 1)}[kind]


def fan_in(kind, cin):
    return {"down": cin * K8 * K8, "up": cin * K8 * K8 // (S8 * S8), "conv1": cin}[kind]


def layer_len(kind, cin, cout):
    return int(np.prod(weight_shape(kind, cin, cout))) + cout + (kind != "conv1")


def param_count(specs) -> int:
    return sum(layer_len(k, ci, co) for _, k, ci, co in specs)


def unpack(theta, specs):
    """{name: (W, b, slope or None)} views of the flat vector."""
    out, off = {}, 0
    for name, kind, ci, co in specs:
        shp = weight_shape(kind, ci, co)
        nw = int(np.prod(shp))
        W = theta[off:off + nw].reshape(shp)
        b = theta[off + nw:off + nw + co]
        a = theta[off + nw + co] if kind != "conv1" else None
        out[name] = (W, b, a)
        off += layer_len(kind, ci, co)
    assert off == theta.size, (off, theta.size)
    return out


def init_theta(specs, rng: np.random.Generator, slope: float = 0.25) -> np.ndarray:
    """Seeded He-uniform weights and biases, PReLU slopes at the library default 0.25."""
    parts = []
    for _, kind, ci, co in specs:
        lim = np.sqrt(6.0 / fan_in(kind, ci))
        parts.append(rng.uniform(-lim, lim, int(np.prod(weight_shape(kind, ci, co)))))
        parts.append(rng.uniform(-1.0 / np.sqrt(fan_in(kind, ci)), 1.0 / np.sqrt(fan_in(kind, ci)), co))
        if kind != "conv1":
            parts.append(np.array([slope]))
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------- layers

def _mix(M, x):
    """sum_c M[o, c] x[b, c, h, w] -> [b, o, h, w] (a matrix product over the channel axis)."""
    return np.moveaxis(np.tensordot(M, x, axes=([1], [1])), 0, 1)


def _corr(g, x):
    """sum_{b, h, w} g[b, o, h, w] x[b, c, h, w] -> [o, c]."""
    return np.tensordot(g, x, axes=([0, 2, 3], [0, 2, 3]))


def down(x, W, b):
    """8x8 stride-2 padding-3 convolution of x [B, C, H, W] (H, W even) -> [B, O, H/2, W/2]."""
    B, C, H, Wd = x.shape
    Ho, Wo = (H + 2 * P8 - K8) // S8 + 1, (Wd + 2 * P8 - K8) // S8 + 1
    xp = np.zeros((B, C, H + 2 * P8, Wd + 2 * P8), x.dtype)
    xp[:, :, P8:P8 + H, P8:P8 + Wd] = x
    y = np.zeros((B, W.shape[0], Ho, Wo), x.dtype)
    for a in range(K8):
        for e in range(K8):
            y += _mix(W[:, :, a, e], xp[:, :, a:a + S8 * Ho:S8, e:e + S8 * Wo:S8])
    return y + b[None, :, None, None]


def down_backward(x, W, g):
    """Reverse mode of down: (dx, dW, db) for the output gradient g [B, O, H/2, W/2]."""
    B, C, H, Wd = x.shape
    Ho, Wo = g.shape[2], g.shape[3]
    xp = np.zeros((B, C, H + 2 * P8, Wd + 2 * P8), x.dtype)
    xp[:, :, P8:P8 + H, P8:P8 + Wd] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for a in range(K8):
        for e in range(K8):
            dW[:, :, a, e] = _corr(g, xp[:, :, a:a + S8 * Ho:S8, e:e + S8 * Wo:S8])
            dxp[:, :, a:a + S8 * Ho:S8, e:e + S8 * Wo:S8] += _mix(W[:, :, a, e].T, g)
    return dxp[:, :, P8:P8 + H, P8:P8 + Wd], dW, g.sum(axis=(0, 2, 3))


def up(x, W, b):
    """8x8 stride-2 padding-3 transposed convolution of x [B, C, H, W] -> [B, O, 2H, 2W]."""
    B, C, H, Wd = x.shape
    Ho, Wo = (H - 1) * S8 - 2 * P8 + K8, (Wd - 1) * S8 - 2 * P8 + K8
    # scatter into the uncropped output, then drop the padding rows/columns
    full = np.zeros((B, W.shape[1], (H - 1) * S8 + K8, (Wd - 1) * S8 + K8), x.dtype)
    for a in range(K8):
        for e in range(K8):
            full[:, :, a:a + S8 * H:S8, e:e + S8 * Wd:S8] += _mix(W[:, :, a, e].T, x)
    return full[:, :, P8:P8 + Ho, P8:P8 + Wo] + b[None, :, None, None]


def up_backward(x, W, g):
    """Reverse mode of up: (dx, dW, db) for the output gradient g [B, O, 2H, 2W]."""
    B, C, H, Wd = x.shape
    full = np.zeros((B, W.shape[1], (H - 1) * S8 + K8, (Wd - 1) * S8 + K8), x.dtype)
    full[:, :, P8:P8 + g.shape[2], P8:P8 + g.shape[3]] = g
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for a in range(K8):
        for e in range(K8):
            gs = full[:, :, a:a + S8 * H:S8, e:e + S8 * Wd:S8]
            dx += _mix(W[:, :, a, e], gs)
            dW[:, :, a, e] = _corr(x, gs)
    return dx, dW, g.sum(axis=(0, 2, 3))


def conv1(x, W, b):
    return _mix(W[:, :, 0, 0], x) + b[None, :, None, None]


def prelu(x, a):
    return np.where(x > 0, x, a * x)


def prelu_backward(s, a, g):
    """(ds, da) of y = prelu(s, a) for the output gradient g."""
    neg = s <= 0
    return np.where(neg, a * g, g), float(np.sum(np.where(neg, s * g, 0.0)))


def forward(theta, specs, X, act_round=None, keep=False):
    """Network output [B, 2, Hp, Wp] for the packed input X (act_round: optional rounding of
    every stored activation, as in unet.forward). keep: also return the cache for backward."""
    rnd = act_round if act_round is not None else (lambda t: t)
    P = unpack(np.asarray(theta, dtype=X.dtype), specs)
    depth = sum(1 for s in specs if s[1] == "down")
    cache = {}
    E = [rnd(X)]
    for l in range(1, depth + 1):
        W, b, a = P[f"down{l}"]
        s = down(E[-1], W, b)
        cache[f"down{l}"] = (E[-1], s)
        E.append(rnd(prelu(s, a)))
    W, b, a = P[f"up{depth - 1}"]
    s = up(E[depth], W, b)
    cache[f"up{depth - 1}"] = (E[depth], s)
    U = rnd(prelu(s, a))
    for l in range(depth - 2, -1, -1):
        W, b, a = P[f"up{l}"]
        xin = np.concatenate([E[l + 1], U], axis=1)
        s = up(xin, W, b)
        cache[f"up{l}"] = (xin, s)
        U = rnd(prelu(s, a))
    cache["head"] = (U, None)
    out = conv1(U, *P["head"][:2])
    return (out, cache) if keep else out


def backward(theta, specs, cache, gout):
    """Gradient of sum(gout * forward(theta, X)) with respect to theta (flat, the layout of
    unpack), from the cache of forward(keep=True)."""
    P = unpack(np.asarray(theta, dtype=gout.dtype), specs)
    depth = sum(1 for s in specs if s[1] == "down")
    grads = {}
    U = cache["head"][0]
    Wh = P["head"][0]
    grads["head"] = (_corr(gout, U)[:, :, None, None], gout.sum(axis=(0, 2, 3)), None)
    gU = _mix(Wh[:, :, 0, 0].T, gout)
    gE = {}
    for l in range(0, depth):               # up0, up1, ..., up(depth-1)
        W, b, a = P[f"up{l}"]
        xin, s = cache[f"up{l}"]
        gs, ga = prelu_backward(s, a, gU)
        gx, gW, gb = up_backward(xin, W, gs)
        grads[f"up{l}"] = (gW, gb, ga)
        if l < depth - 1:                   # input concat[E_{l+1}, U_{l+1}]
            ce = gx.shape[1] // 2
            gE[l + 1] = gx[:, :ce]
            gU = gx[:, ce:]
        else:                               # the deepest takes E_depth alone
            gE[depth] = gx
    g = gE[depth]
    for l in range(depth, 0, -1):           # down(depth), ..., down1
        W, b, a = P[f"down{l}"]
        xin, s = cache[f"down{l}"]
        gs, ga = prelu_backward(s, a, g)
        gx, gW, gb = down_backward(xin, W, gs)
        grads[f"down{l}"] = (gW, gb, ga)
        if l > 1:
            g = gx + gE[l - 1]
    parts = []
    for name, kind, ci, co in specs:
        gW, gb, ga = grads[name]
        parts.append(np.asarray(gW).ravel())
        parts.append(np.asarray(gb).ravel())
        if kind != "conv1":
            parts.append(np.array([ga]))
    return np.concatenate(parts)


def precond_apply(theta, specs, p: hz.Problem, v, dtype=np.float64, act_round=None):
    """Eq. (7) with this network: z = N_theta(v, c, sigma) for one complex field v [ny, nx]."""
    in_ch = specs[0][2]
    depth = sum(1 for s in specs if s[1] == "down")
    X, s = pack_input(v, p, in_ch, depth + 1, dtype)      # padded to a multiple of 2^depth
    if s == 0:
        return np.zeros((p.ny, p.nx), np.complex128)
    out = forward(np.asarray(theta, dtype=dtype), specs, X, act_round=act_round)
    return s * (out[0, 0, :p.ny, :p.nx].astype(np.float64) + 1j * out[0, 1, :p.ny, :p.nx].astype(np.float64))


def loss_and_grad(theta, specs, problems, rs, squared=False, dtype=np.float64, need_grad=True, ops=None):
    """Batch-mean physics-informed loss (eq. (12); unsquared unless squared) and its gradient with
    respect to theta for this network; problems share one grid size, rs [B, ny, nx] complex.
    ops: the operator module (op_apply, op_adjoint): helmholtz (the default, the finite-difference
    stencil) or spectral (the Fourier-differentiation form of Section 2.1).
    """
    ops = hz if ops is None else ops
    B = len(problems)
    in_ch = specs[0][2]
    depth = sum(1 for s in specs if s[1] == "down")
    theta = np.asarray(theta, dtype=dtype)
    Xs, ss = zip(*(pack_input(rs[b], problems[b], in_ch, depth + 1, dtype) for b in range(B)))
    out, cache = forward(theta, specs, np.concatenate(Xs), keep=True)
    gout = np.zeros_like(out)
    losses = np.empty(B)
    for b in range(B):
        p = problems[b]
        z = ss[b] * (out[b, 0, :p.ny, :p.nx].astype(np.float64) + 1j * out[b, 1, :p.ny, :p.nx].astype(np.float64))
        q = ops.op_apply(p, z) - rs[b]
        nq, nr = np.linalg.norm(q), np.linalg.norm(rs[b])
        if squared:
            losses[b] = nq * nq / (nr * nr)
            gq = 2.0 * q / (B * nr * nr)
        else:
            losses[b] = nq / nr
            gq = q / (B * nq * nr) if nq > 0 else np.zeros_like(q)
        gz = ops.op_adjoint(p, gq)
        gout[b, 0, :p.ny, :p.nx] = ss[b] * gz.real
        gout[b, 1, :p.ny, :p.nx] = ss[b] * gz.imag
    loss = float(losses.mean())
    if not need_grad:
        return loss, losses, None
    return loss, losses, backward(theta, specs, cache, gout.astype(dtype))
