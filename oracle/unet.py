"""Oracle: the U-Net neural operator, its reverse mode and the physics-informed loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps a complex field plus the problem's static fields to a complex
field (eq. (9), Section 3.1): the field is recast as real (Re, Im) channels,
optionally joined by the velocity and the complex PML damping, passed through an
encoder-decoder with skip connections, and read back as (Re, Im). Reading
adopted for the build (the paper's own layer hyper-parameters are in Table 2):

  * input scale s = ||v|| / sqrt(n); if s == 0 the output is 0;
  * X = [Re v / s, Im v / s] (+ [c / c_ref, sigma_x, sigma_y] when in_ch = 5),
    zero-padded at the bottom/right to a multiple of 2^(L-1);
  * encoder level l = 0..L-1: E_l = relu(conv3(relu(conv3(I_l)))), I_0 = X,
    I_l = avgpool2(E_{l-1}), C * 2^l channels;
  * decoder level l = L-2..0: U = convT2(D_{l+1}) (D_{L-1} = E_{L-1}),
    D_l = relu(conv3(relu(conv3(concat[E_l, U]))));
  * head: 1x1 conv to 2 channels, no activation; z = s (out_0 + i out_1), cropped.

conv3 is a 3x3 cross-correlation, stride 1, zero padding 1, with bias; convT2 a
2x2 stride-2 transposed convolution with bias; avgpool2 the mean of 2x2 blocks.

Parameters form one flat vector: layers in the order of ``layer_specs``, each
as its weight (conv: [out, in, kh, kw]; convT2: [in, out, 2, 2]) then its bias.

Loss (eq. (12) and (10)): per sample q = A N(r) - r and l = ||q|| / ||r||
(``squared=True`` gives the paper's ||q||^2 / ||r||^2); the cost is the batch mean.
Arrays are NCHW numpy arrays in float64 unless a dtype is given.
"""
from __future__ import annotations

import numpy as np

from . import helmholtz as hz


# --------------------------------------------------------------------------- architecture

def layer_specs(levels: int, base: int, in_ch: int, out_ch: int = 2):
    """[(name, kind, cin, cout)] with kind in {'conv3', 'convT2', 'conv1'}."""
    ch = [base * 2 ** l for l in range(levels)]
    specs, cin = [], in_ch
    for l in range(levels):
        specs.append((f"enc{l}a", "conv3", cin, ch[l]))
        specs.append((f"enc{l}b", "conv3", ch[l], ch[l]))
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        specs.append((f"up{l}", "convT2", ch[l + 1], ch[l]))
        specs.append((f"dec{l}a", "conv3", 2 * ch[l], ch[l]))
        specs.append((f"dec{l}b", "conv3", ch[l], ch[l]))
    specs.append(("head", "conv1", ch[0], out_ch))
    return specs


def weight_shape(kind, cin, cout):
    return {"conv3": (cout, cin, 3, 3), "convT2": (cin, cout, 2, 2), "conv1": (cout, cin, 1, 1)}[kind]


def fan_in(kind, cin):
    return {"conv3": 9 * cin, "convT2": cin, "conv1": cin}[kind]


def init_shapes(specs):
    """(weight_shape, fan_in, bias_len) per layer, for the seeded He-uniform generator."""
    return [(weight_shape(k, ci, co), fan_in(k, ci), co) for _, k, ci, co in specs]


def param_count(specs) -> int:
    return sum(int(np.prod(weight_shape(k, ci, co))) + co for _, k, ci, co in specs)


def unpack(theta, specs):
    """Split the flat vector into {name: (W, b)} views."""
    out, off = {}, 0
    for name, kind, ci, co in specs:
        shp = weight_shape(kind, ci, co)
        nw = int(np.prod(shp))
        out[name] = (theta[off:off + nw].reshape(shp), theta[off + nw:off + nw + co])
        off += nw + co
    assert off == theta.size, (off, theta.size)
    return out


# --------------------------------------------------------------------------- layers

def conv3(x, W, b):
    """out[b,o,y,x] = sum_{c,dy,dx} W[o,c,dy,dx] x[b,c,y+dy-1,x+dx-1] + b[o] (zero padding)."""
    B, C, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((W.shape[0], B, H, Wd), dtype=x.dtype)
    for dy in range(3):
        for dx in range(3):
            out += np.tensordot(W[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + Wd], axes=([1], [1]))
    return out.transpose(1, 0, 2, 3) + b[None, :, None, None]


def conv3_backward(x, W, g):
    """Gradients of conv3 w.r.t. its input, weight and bias given the output gradient g."""
    B, C, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            xs = xp[:, :, dy:dy + H, dx:dx + Wd]
            dW[:, :, dy, dx] = np.tensordot(g, xs, axes=([0, 2, 3], [0, 2, 3]))
            dxp[:, :, dy:dy + H, dx:dx + Wd] += np.tensordot(W[:, :, dy, dx], g, axes=([0], [1])).transpose(1, 0, 2, 3)
    db = g.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:H + 1, 1:Wd + 1], dW, db


def conv1(x, W, b):
    return np.tensordot(W[:, :, 0, 0], x, axes=([1], [1])).transpose(1, 0, 2, 3) + b[None, :, None, None]


def conv1_backward(x, W, g):
    dx = np.tensordot(W[:, :, 0, 0], g, axes=([0], [1])).transpose(1, 0, 2, 3)
    dW = np.tensordot(g, x, axes=([0, 2, 3], [0, 2, 3]))[:, :, None, None]
    return dx, dW, g.sum(axis=(0, 2, 3))


def convT2(x, W, b):
    """out[b,o,2y+p,2x+q] = sum_c x[b,c,y,x] W[c,o,p,q] + b[o]."""
    B, C, H, Wd = x.shape
    O = W.shape[1]
    out = np.empty((B, O, 2 * H, 2 * Wd), dtype=x.dtype)
    for p in range(2):
        for q in range(2):
            out[:, :, p::2, q::2] = np.tensordot(W[:, :, p, q], x, axes=([0], [1])).transpose(1, 0, 2, 3)
    return out + b[None, :, None, None]


def convT2_backward(x, W, g):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for p in range(2):
        for q in range(2):
            gs = g[:, :, p::2, q::2]
            dx += np.tensordot(W[:, :, p, q], gs, axes=([1], [1])).transpose(1, 0, 2, 3)
            dW[:, :, p, q] = np.tensordot(x, gs, axes=([0, 2, 3], [0, 2, 3]))
    return dx, dW, g.sum(axis=(0, 2, 3))


def avgpool2(x):
    return 0.25 * (x[:, :, 0::2, 0::2] + x[:, :, 1::2, 0::2] + x[:, :, 0::2, 1::2] + x[:, :, 1::2, 1::2])


def avgpool2_backward(g):
    B, C, H, W = g.shape
    dx = np.empty((B, C, 2 * H, 2 * W), dtype=g.dtype)
    for p in range(2):
        for q in range(2):
            dx[:, :, p::2, q::2] = 0.25 * g
    return dx


def relu(x):
    return np.maximum(x, 0)


# --------------------------------------------------------------------------- network

def bf16_activation(a):
    """Emulated BF16 activation storage: the value as an FP32 accumulator holds it, rounded to
    bfloat16 (8-bit significand) to nearest, ties to even; returned as float64. NaN stays NaN."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (((u + 0x7FFF + lsb) >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, r)


def forward(theta, specs, X, keep=False, act_round=None):
    """U-Net on an NCHW batch X. Returns out (and the activation cache when keep=True).

    act_round (optional, inference only): a rounding applied to every stored activation, to
    emulate a reduced-precision activation format: the network input, each 3x3 layer's output
    after ReLU and each transposed convolution's output. Pooling averages the encoder output
    before its rounding (the pooled value is then rounded)."""
    if act_round is not None and keep:
        raise ValueError("act_round is an inference-only emulation")
    q = act_round if act_round is not None else (lambda a: a)
    P = unpack(theta, specs)
    levels = sum(1 for s in specs if s[0].startswith("enc")) // 2
    cache = {}
    E, h = [], q(X)
    e_raw = None
    for l in range(levels):
        if l > 0:
            h = q(avgpool2(e_raw))
        Wa, ba = P[f"enc{l}a"]
        Wb, bb = P[f"enc{l}b"]
        a1 = conv3(h, Wa, ba)
        r1 = q(relu(a1))
        a2 = conv3(r1, Wb, bb)
        e_raw = relu(a2)
        if keep:
            cache[f"enc{l}"] = (h, a1, r1, a2)
        E.append(q(e_raw))
    D = E[-1]
    for l in range(levels - 2, -1, -1):
        Wu, bu = P[f"up{l}"]
        U = q(convT2(D, Wu, bu))
        cat = np.concatenate([E[l], U], axis=1)
        Wa, ba = P[f"dec{l}a"]
        Wb, bb = P[f"dec{l}b"]
        a1 = conv3(cat, Wa, ba)
        r1 = q(relu(a1))
        a2 = conv3(r1, Wb, bb)
        if keep:
            cache[f"dec{l}"] = (D, cat, a1, r1, a2)
        D = q(relu(a2))
    Wh, bh = P["head"]
    out = conv1(D, Wh, bh)
    if keep:
        cache["head"] = D
        cache["levels"] = levels
        return out, cache
    return out


def backward(theta, specs, cache, gout):
    """Reverse mode of ``forward``: returns (d theta flat, d X)."""
    P = unpack(theta, specs)
    grads = {}
    levels = cache["levels"]
    Wh, _ = P["head"]
    gD, dW, db = conv1_backward(cache["head"], Wh, gout)
    grads["head"] = (dW, db)
    gE = [None] * levels
    for l in range(0, levels - 1):
        D_in, cat, a1, r1, a2 = cache[f"dec{l}"]
        Wa, _ = P[f"dec{l}a"]
        Wb, _ = P[f"dec{l}b"]
        g = gD * (a2 > 0)
        gr1, dWb, dbb = conv3_backward(r1, Wb, g)
        g = gr1 * (a1 > 0)
        gcat, dWa, dba = conv3_backward(cat, Wa, g)
        grads[f"dec{l}b"] = (dWb, dbb)
        grads[f"dec{l}a"] = (dWa, dba)
        ce = gcat.shape[1] // 2
        gE[l] = gcat[:, :ce]
        Wu, _ = P[f"up{l}"]
        gD, dWu, dbu = convT2_backward(D_in, Wu, gcat[:, ce:])
        grads[f"up{l}"] = (dWu, dbu)
        # gD is now the gradient w.r.t. D_{l+1}; continue with the next (deeper) decoder level,
        # or with E_{L-1} once l + 1 == levels - 1
    # the loop above visits decoder levels from 0 upward, so gD is finally d E_{L-1}
    gE[levels - 1] = gD if gE[levels - 1] is None else gE[levels - 1] + gD
    gX = None
    gnext = None   # gradient flowing into E_l from level l+1 through the pooling
    for l in range(levels - 1, -1, -1):
        g = gE[l] if gnext is None else gE[l] + gnext
        h, a1, r1, a2 = cache[f"enc{l}"]
        Wa, _ = P[f"enc{l}a"]
        Wb, _ = P[f"enc{l}b"]
        g = g * (a2 > 0)
        gr1, dWb, dbb = conv3_backward(r1, Wb, g)
        g = gr1 * (a1 > 0)
        gh, dWa, dba = conv3_backward(h, Wa, g)
        grads[f"enc{l}b"] = (dWb, dbb)
        grads[f"enc{l}a"] = (dWa, dba)
        if l > 0:
            gnext = avgpool2_backward(gh)
        else:
            gX = gh
    flat = []
    for name, _, _, _ in specs:
        dW, db = grads[name]
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return np.concatenate(flat), gX


# --------------------------------------------------------------------------- preconditioner

def static_channels(p: hz.Problem):
    """[c / c_ref, sigma_x, sigma_y] at the nodes, [3, ny, nx] float64 (the 'complex sigma'
    input of Section 3.1 read as sigma_x + i sigma_y)."""
    sx, sy = p.sigma_nodes()
    return np.stack([p.c / p.c_ref, sx, sy])


def pad_multiple(levels: int) -> int:
    return 2 ** (levels - 1)


def pack_input(v, p: hz.Problem, in_ch: int, levels: int, dtype=np.float64):
    """(X [1, in_ch, Hp, Wp], s): the scaled, zero-padded network input for one field."""
    v = np.asarray(v, dtype=np.complex128).reshape(p.ny, p.nx)
    s = np.linalg.norm(v) / np.sqrt(v.size)
    m = pad_multiple(levels)
    Hp, Wp = -(-p.ny // m) * m, -(-p.nx // m) * m
    X = np.zeros((1, in_ch, Hp, Wp), dtype=dtype)
    if s > 0:
        X[0, 0, :p.ny, :p.nx] = v.real / s
        X[0, 1, :p.ny, :p.nx] = v.imag / s
    if in_ch == 5:
        X[0, 2:5, :p.ny, :p.nx] = static_channels(p)
    elif in_ch != 2:
        raise ValueError("in_ch must be 2 or 5")
    return X, s


def precond_apply(theta, specs, p: hz.Problem, v, dtype=np.float64, act_round=None):
    """Eq. (7): z = N_theta(v, c, sigma) for one complex field v [ny, nx] (act_round: see forward)."""
    in_ch = specs[0][2]
    levels = sum(1 for s in specs if s[0].startswith("enc")) // 2
    X, s = pack_input(v, p, in_ch, levels, dtype)
    if s == 0:
        return np.zeros((p.ny, p.nx), np.complex128)
    out = forward(np.asarray(theta, dtype=dtype), specs, X, act_round=act_round)
    return s * (out[0, 0, :p.ny, :p.nx].astype(np.float64) + 1j * out[0, 1, :p.ny, :p.nx].astype(np.float64))


def loss_and_grad(theta, specs, problems, rs, squared=False, dtype=np.float64, need_grad=True, ops=None):
    """Batch-mean physics-informed loss and its gradient w.r.t. theta.

    problems: list of B Problems sharing one grid size; rs: [B, ny, nx] complex residuals.
    Per sample q = A N(r) - r, l = ||q|| / ||r|| (or its square); loss = mean over samples.
    Returns (loss, per-sample losses, d loss / d theta or None).
    ops: the operator module (op_apply, op_adjoint): helmholtz (the default, the finite-difference
    stencil) or spectral (the Fourier-differentiation form of Section 2.1).
    """
    ops = hz if ops is None else ops
    B = len(problems)
    in_ch = specs[0][2]
    levels = sum(1 for s in specs if s[0].startswith("enc")) // 2
    theta = np.asarray(theta, dtype=dtype)
    Xs, ss = zip(*(pack_input(rs[b], problems[b], in_ch, levels, dtype) for b in range(B)))
    X = np.concatenate(Xs)
    out, cache = forward(theta, specs, X, keep=True)
    p0 = problems[0]
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
    g, _ = backward(theta, specs, cache, gout.astype(dtype))
    del p0
    return loss, losses, g
