"""Benchmark: solves/s of the BF16-network FGMRES on the single-solve workload (one MI355X).

Workload: 256^2 interior grid + 20-cell PML (296^2 nodes), skull-ring velocity with 1-3 rings
and 5% noise, 1-4 Gaussian sources, 4-level / 32-channel U-Net (BF16 operands, FP32
accumulation), FP32 Krylov basis, FGMRES restart 30, tol 1e-6 on the FP64 true residual. A step
is one full solve from x0 = 0 with every input resident on the GPU. The same solve with the
network in FP32 (the plain FP32 form) is timed beside it, and the dominant network layer is
timed alone with HIP events for the roofline. The oracle is timed on the host over a bounded
sample of iterations.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--roofline-only] [--only SECTION]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "unet_l4_c32_in5.npz")
M_RESTART, TOL, MAXIT = 30, 1e-6, 6000
LEVELS, BASE, IN_CH = 4, 32, 5
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


WEIGHTS8 = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "paper8_d4_c32_in5_D0.npz")
WEIGHTS_SPEC = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "unet_l4_c32_in5_spectral.npz")
WEIGHTS_L5 = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "unet_l5_c32_in5.npz")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "conv3_dominant_layer_296_bf16_traffic.txt")
GOLDEN_C2 = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2607_16906_amd", "csrc", f) for f in ("net_fwd.hip", "net_kernels.h")]


def note(msg):
    """One progress line on stderr per finished section (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_fingerprint():
    import hashlib
    h = hashlib.md5()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(layer, variant):
    """HBM bytes per launch of the dominant layer from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy of known size; one record per launch variant, records
    separated by blank lines), or None when no record matches the layer and variant or the kernel
    sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    recs, kv = [], {}
    for line in list(open(TRAFFIC_FILE)) + [""]:
        if not line.strip():
            if kv:
                recs.append(kv)
            kv = {}
        elif ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    fp = kernel_fingerprint()
    for kv in recs:
        try:
            if kv.get("source_md5") == fp and int(kv.get("layer", -1)) == layer and kv.get("variant") == variant:
                return float(kv["traffic_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def oracle_comparison(its, true_relres, run):
    """The solve against the FP64 oracle's solve of the same system, stored in the golden file
    (written by a script that calls only the oracle): iteration counts, the per-solve bar
    |d its| <= 2 + the oracle's own movement under BF16 activation storage, true residuals.
    None when the file is missing or was taken with other weights."""
    import hashlib
    try:
        with open(GOLDEN_C2) as f:
            g = json.load(f)
        with open(WEIGHTS, "rb") as f:
            if hashlib.md5(f.read()).hexdigest() != g["weights_md5"]:
                return None
    except OSError:
        return None
    ref = g["runs"][run]
    out = {"oracle_its": ref["its"], "d_its": its - ref["its"], "oracle_true_relres": ref["true_relres"],
           "true_relres": true_relres, "oracle": f"FP64 oracle FGMRES, {run.replace('_', ' ')}"}
    if run == "bf16_weights":
        q = g["runs"]["bf16_weights_bf16_activations"]["its"]
        out["oracle_its_bf16_activations"] = q
        out["bar"] = 2 + abs(q - ref["its"])
        out["within_bar"] = abs(its - ref["its"]) <= out["bar"]
    return out


def layer_flops(kind, cin, cout, H, W):
    """Algorithmic FLOPs of one layer launch on an H x W input (logical channels)."""
    if kind == 0:
        return 2.0 * 9 * cin * cout * H * W
    return 2.0 * cin * cout * 4 * H * W


def net_layers(levels, base, in_ch, Hp, Wp):
    """(index, kind, cin, cout, H, W) of every 3x3 / transposed layer, in parameter order."""
    out, i = [], 0
    cin = in_ch
    for l in range(levels):
        c = base << l
        out.append((i, 0, cin, c, Hp >> l, Wp >> l)); i += 1
        out.append((i, 0, c, c, Hp >> l, Wp >> l)); i += 1
        cin = c
    for l in range(levels - 2, -1, -1):
        c = base << l
        out.append((i, 1, 2 * c, c, Hp >> (l + 1), Wp >> (l + 1))); i += 1
        out.append((i, 0, 2 * c, c, Hp >> l, Wp >> l)); i += 1
        out.append((i, 0, c, c, Hp >> l, Wp >> l)); i += 1
    return out


def time_layers(net, Hp, Wp, reps, prec="bf16", only=-1, levels=LEVELS):
    """Per-layer average launch time (ms) with HIP events on the current stream, each layer with the
    launch variant the autotuner chose for it (the one the solve uses)."""
    import torch
    elem = {"bf16": torch.int16, "fp32": torch.float32}[prec]
    ws = torch.empty(4 * Hp * Wp * 32 * 4 + 256, dtype=torch.uint8, device="cuda")
    res = []
    for (i, kind, cin, cout, H, W) in net_layers(levels, BASE, IN_CH, Hp, Wp):
        if only >= 0 and i != only:
            continue
        _, cin_p, cout_p, cat_cp = net.layer_info(i)
        c0 = cat_cp if cat_cp else cin_p
        x0 = torch.zeros(H * W * c0, dtype=elem, device="cuda")
        x1 = torch.zeros(H * W * (cin_p - c0), dtype=elem, device="cuda") if cat_cp else None
        Ho, Wo = (H, W) if kind == 0 else (2 * H, 2 * W)
        y = torch.empty(Ho * Wo * cout_p, dtype=elem, device="cuda")
        for _ in range(3):
            net.layer_forward(i, x0, y, H=H, W=W, x1=x1, prec=prec, workspace=ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            net.layer_forward(i, x0, y, H=H, W=W, x1=x1, prec=prec, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res.append(dict(layer=i, kind=kind, cin=cin, cout=cout, H=H, W=W, ms=ms,
                        flops=layer_flops(kind, cin, cout, H, W)))
    return res


def time_stencil(hz, torch, nt, reps=50):
    """Average time (ms) of the FP32 stencil on an nt x nt homogeneous grid, HIP events."""
    c = np.full(nt * nt, 1500.0, np.float32)
    p = hz.Problem(c, nt - 32, nt - 32, 16, 2 * np.pi / 10)
    x = torch.randn(nt * nt, dtype=torch.complex64, device="cuda")
    for _ in range(3):
        p.apply(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y = p.apply(x)
    e1.record()
    torch.cuda.synchronize()
    del y
    return e0.elapsed_time(e1) / reps


def train_flops(levels, base, in_ch, Hp, Wp, batch):
    """Algorithmic FLOPs of one training step: forward, data gradients (all layers but the first)
    and weight gradients of every layer (the head and stencils are negligible)."""
    fwd = sum(layer_flops(k, ci, co, H, W) for (_, k, ci, co, H, W) in net_layers(levels, base, in_ch, Hp, Wp))
    first = layer_flops(0, in_ch, base, Hp, Wp)
    return batch * (3 * fwd - first)


def bench_training(hz, torch, steps=3, batch=64):
    """Training step of the physics-informed loss on 64 samples at 128^2 + 16 PML (BF16), from the
    seeded initial weights with Adam at lr 1e-3."""
    from synth import CFG_C3, COMP_WEIGHTS, H_10PPW, c3_batch, he_uniform, rng_for
    theta = he_uniform(hz.init_shapes(LEVELS, BASE, IN_CH), rng_for(CFG_C3, COMP_WEIGHTS, 0))
    cs, rs = c3_batch(batch=batch, step=0)
    probs = [hz.Problem(c.astype(np.float32).ravel(), 128, 128, 16, H_10PPW) for c in cs]
    net = hz.Net(LEVELS, BASE, IN_CH, theta)
    r = torch.from_numpy(rs.astype(np.complex64).reshape(batch, -1)).cuda()
    th = torch.from_numpy(theta.copy()).cuda()
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    ws = torch.empty(hz.train_workspace_bytes(net, probs[0], batch, "bf16"), dtype=torch.uint8, device="cuda")
    losses = []
    for step in range(1, steps + 2):
        if step == 2:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        loss, _, g = hz.loss_backward(net, probs, r, prec="bf16", workspace=ws)
        hz.adam_step(net, th, m, v, g, step, lr=1e-3, clip=1.0)
        losses.append(loss)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    fl = train_flops(LEVELS, BASE, IN_CH, 160, 160, batch)
    return {"workload": "training step, 64 x (128^2 + 16 PML), 4-level/32-ch U-Net, BF16 fwd/bwd, FP32 master, Adam",
            "ms_per_step": round(dt * 1e3, 2), "samples_per_s": round(batch / dt, 1),
            "tflops": round(fl / dt * 1e-12, 2), "loss_first": float(losses[0].item()),
            "loss_last": float(losses[-1].item())}


def bench_training_loop(hz, torch, S=1024, V=128, batch=32, epochs=2, nint=64, npml=16):
    """Epoch-based training (Section 3.4): a fixed D0-like set of S samples and V validation
    samples on the paper's training grid (64^2, here with 16 PML cells outside it), batch 32, Adam
    with clipping at 1, cosine schedule 1e-3 -> 1e-5 over the epochs, validation and best-epoch
    selection after each epoch; from the seeded initial weights. One untimed epoch first (it
    tunes the launch variants at this batch), then `epochs` timed epochs per precision."""
    from synth import CFG_C3, COMP_WEIGHTS, H_10PPW, VAL_FIRST, epoch_order, he_uniform, rng_for, training_set
    from paper_2607_16906_amd.train import Trainer, resident_set
    nt = nint + 2 * npml
    theta = he_uniform(hz.init_shapes(LEVELS, BASE, IN_CH), rng_for(CFG_C3, COMP_WEIGHTS, 0))
    c, b = training_set(S, nt, npml)
    vc, vb = training_set(V, nt, npml, first=VAL_FIRST)
    probs, r = resident_set(c, b, nint, npml, H_10PPW)
    vprobs, vr = resident_set(vc, vb, nint, npml, H_10PPW)
    out = {"workload": f"{S} training + {V} validation samples of the D0-like mixture, {nint}^2 + {npml} PML, "
                       f"batch {batch}, 4-level/32-ch U-Net, Adam, clip 1, cosine 1e-3 -> 1e-5, "
                       f"{epochs} timed epochs"}
    for prec in ("bf16", "fp32"):
        net = hz.Net(LEVELS, BASE, IN_CH, theta)
        tr = Trainer(net, probs, r, vprobs, vr, batch=batch, prec=prec)
        tr.fit(theta, [epoch_order(S, 0)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = tr.fit(theta, [epoch_order(S, e) for e in range(epochs)])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / epochs
        out[prec] = {"s_per_epoch": round(wall, 3), "train_samples_per_s": round(S / (res.step_ms * 1e-3 *
                                                                                     ((S + batch - 1) // batch)), 1),
                     "ms_per_step": round(res.step_ms, 2), "ms_validation": round(res.val_ms, 2),
                     "val_loss": [round(x, 5) for x in res.val_loss], "best_epoch": res.best_epoch}
        del tr, net
    return out


def paper8_flops(depth, ch, in_ch, Hp, Wp):
    """Algorithmic FLOPs of one forward of the paper's 8x8 stride-2 network on an Hp x Wp grid
    (logical channels; 64 taps down, 16 taps per output pixel up, the 1x1 head)."""
    fl = 0
    for l in range(1, depth + 1):
        fl += 2 * (Hp >> l) * (Wp >> l) * ch * (in_ch if l == 1 else ch) * 64
    for l in range(depth - 1, -1, -1):
        fl += 2 * (Hp >> l) * (Wp >> l) * ch * (ch if l == depth - 1 else 2 * ch) * 16
    return fl + 2 * Hp * Wp * 2 * ch


def bench_paper8(hz, torch, net3, reps=50):
    """The paper's own layer set (Table 2: depth 4, 32 channels, 8x8 stride-2, PReLU) as the
    preconditioner on the single-solve system (296^2): one application in BF16 and FP32 against the
    3x3 network's, and FGMRES with it (m = 30, tol 1e-6) with the weights the library's epoch loop
    trained for it on data set D0 (Table 4) at 128^2 + 16 PML (seeded He-uniform weights with
    slopes 0.25 when that file is absent)."""
    from paper_2607_16906_amd.train import init_theta_paper8
    from synth import H_10PPW, c2_system, rng_for
    trained = os.path.exists(WEIGHTS8)
    if trained:
        w8 = np.load(WEIGHTS8)
        theta8 = w8["theta"].astype(np.float32)
    else:
        theta8 = init_theta_paper8(4, 32, 5, rng_for(21, 2, 0))
    net8 = hz.Net(4, 32, 5, theta8, kind="paper8")
    s = c2_system(0)
    gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
    v = torch.from_numpy(s.b.ravel().astype(np.complex64)).cuda()
    Hp = (s.nt + 15) // 16 * 16
    out = {"workload": "one application on 296^2 (padded to 304^2); FGMRES(30) to 1e-6 on the single-solve system",
           "weights": (f"trained on the GPU on D0, {int(w8['epochs'])} epochs of {int(w8['step'])} steps, "
                       f"validation loss {float(w8['best_val']):.4f}") if trained else "seeded (untrained)",
           "params": net8.nparam, "gflop_per_apply": round(paper8_flops(4, 32, 5, Hp, Hp) * 1e-9, 3)}
    for tag, net in (("paper8", net8), ("unet3", net3)):
        for prec in ("bf16", "fp32"):
            net.autotune(gp, prec)
            for _ in range(3):
                net.apply(gp, v, prec=prec)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                net.apply(gp, v, prec=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out[f"{tag}_{prec}_apply_us"] = round(ms * 1e3, 1)
            if tag == "paper8":
                out[f"{tag}_{prec}_tflops"] = round(paper8_flops(4, 32, 5, Hp, Hp) / (ms * 1e-3) * 1e-12, 1)
    b = torch.from_numpy(s.b.ravel()).cuda()
    maxit = 3000 if trained else 60
    for prec in ("bf16", "fp32"):
        sfx = "" if prec == "bf16" else "_fp32_net"
        hz.fgmres(gp, b, net=net8, m=30, tol=1e-6, maxit=30, net_prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = hz.fgmres(gp, b, net=net8, m=30, tol=1e-6, maxit=maxit, net_prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["fgmres_ms_per_it" + sfx] = round(dt * 1e3 / max(info.its, 1), 3)
        out["fgmres_its" + sfx] = info.its
        out["fgmres_converged" + sfx] = info.status == 0
        out["fgmres_true_relres" + sfx] = float(f"{info.true_relres:.3e}")
        if info.status == 0:
            out["solves_per_s" + sfx] = round(1.0 / dt, 3)
    # at the training size (64^2 interior + 16 PML): iterations of both networks and of GMRES on
    # five seeded systems of the single-solve kind
    small = {"paper8": [], "unet3": [], "gmres": []}
    for sid in range(5):
        ss = c2_system(sid, nx=64, npml=16)
        gs = hz.Problem(ss.c.astype(np.float32).ravel(), ss.nx, ss.nx, ss.npml, H_10PPW)
        bs = torch.from_numpy(ss.b.ravel()).cuda()
        for tag, nn in (("paper8", net8), ("unet3", net3), ("gmres", None)):
            _, inf = hz.fgmres(gs, bs, net=nn, m=30, tol=1e-6, maxit=1000)
            small[tag].append(inf.its if inf.status == 0 else -inf.its)
    out["its_64_interior"] = small
    # at the paper network's training size (128^2 interior + 16 PML)
    mid = {"paper8": [], "unet3": []}
    for sid in range(2):
        ss = c2_system(sid, nx=128, npml=16)
        gs = hz.Problem(ss.c.astype(np.float32).ravel(), ss.nx, ss.nx, ss.npml, H_10PPW)
        bs = torch.from_numpy(ss.b.ravel()).cuda()
        for tag, nn in (("paper8", net8), ("unet3", net3)):
            _, inf = hz.fgmres(gs, bs, net=nn, m=30, tol=1e-6, maxit=2000)
            mid[tag].append(inf.its if inf.status == 0 else -inf.its)
    out["its_128_interior"] = mid
    out["its_64_interior_note"] = "FGMRES(30) to 1e-6, BF16 networks; negative: not converged"
    return out


def bench_train_then_solve(hz, torch, S=4096, V=256, batch=32, epochs=30, nint=64, npml=16):
    """The whole method on the GPU: train the 4-level / 32-channel network from the seeded initial
    weights with the epoch-based loop (BF16, S samples of the D0-like mixture at 64^2 + 16 PML,
    cosine 1e-3 -> 1e-5, clip 1, best epoch by validation loss), then solve the single-solve system
    (296^2, FGMRES(30), tol 1e-6) preconditioned by the saved epoch's weights. These weights live
    only in this run (the committed weights come from the oracle's training)."""
    from synth import CFG_C3, COMP_WEIGHTS, H_10PPW, VAL_FIRST, c2_system, epoch_order, he_uniform, rng_for, \
        training_set
    from paper_2607_16906_amd.train import Trainer, resident_set
    nt = nint + 2 * npml
    t0 = time.perf_counter()
    c, b = training_set(S, nt, npml)
    vc, vb = training_set(V, nt, npml, first=VAL_FIRST)
    probs, r = resident_set(c, b, nint, npml, H_10PPW)
    vprobs, vr = resident_set(vc, vb, nint, npml, H_10PPW)
    t_data = time.perf_counter() - t0
    theta0 = he_uniform(hz.init_shapes(LEVELS, BASE, IN_CH), rng_for(CFG_C3, COMP_WEIGHTS, 0))
    net = hz.Net(LEVELS, BASE, IN_CH, theta0)
    tr = Trainer(net, probs, r, vprobs, vr, batch=batch, prec="bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = tr.fit(theta0, [epoch_order(S, e) for e in range(epochs)])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    net.set_weights(res.theta_best)
    s = c2_system(0)
    gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
    bb = torch.from_numpy(s.b.ravel()).cuda()
    hz.fgmres(gp, bb, net=net, m=M_RESTART, tol=TOL, maxit=M_RESTART)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = hz.fgmres(gp, bb, net=net, m=M_RESTART, tol=TOL, maxit=3000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"train {epochs} epochs x {S} samples (+{V} validation) at {nint}^2 + {npml} PML, batch "
                        f"{batch}, BF16, from seeded weights; then FGMRES(30) to 1e-6 on the 296^2 system",
            "data_s": round(t_data, 2), "train_s": round(t_train, 2), "steps": len(res.train_loss),
            "ms_per_step": round(res.step_ms, 3), "best_epoch": res.best_epoch,
            "val_loss_first_best": [round(res.val_loss[0], 4), round(res.best_val, 4)],
            "its": info.its, "converged": info.status == 0, "true_relres": float(f"{info.true_relres:.3e}"),
            "solves_per_s": round(1.0 / dt, 3) if info.status == 0 else 0.0}


def bench_batched(hz, torch, net, nsys=128, maxit=MAXIT):
    """Ragged batch: the 128 systems of the batched-serving mix (128..512 interior + 16..32 PML, each
    with its own velocity and sources), BF16 network, FP32 Krylov vectors, FGMRES(30) to tol 1e-6,
    advanced together (systems leave the batch as they converge). Solves/s = systems solved per
    second of the whole batched solve."""
    from synth import H_10PPW, c4_sizes, c4_system
    sizes = c4_sizes(128)[:nsys]
    probs, bs = [], []
    for k, (nx, p) in enumerate(sizes):
        sy = c4_system(k, nx, p)
        probs.append(hz.Problem(sy.c.astype(np.float32).ravel(), nx, nx, p, H_10PPW))
        bs.append(torch.from_numpy(sy.b.ravel()).cuda())
    ws = torch.empty(hz.fgmres_batched_workspace_bytes(probs, net, M_RESTART, maxit, "c64", "bf16"),
                     dtype=torch.uint8, device="cuda")
    hz.fgmres_batched(probs, bs, net=net, m=M_RESTART, tol=TOL, maxit=M_RESTART, workspace=ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = hz.fgmres_batched(probs, bs, net=net, m=M_RESTART, tol=TOL, maxit=maxit, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    node_its = sum(i.its * p.n for i, p in zip(infos, probs))
    steps = max(i.its for i in infos)
    its = np.array([i.its for i in infos])
    conv = sum(1 for i in infos if i.status == 0 and i.true_relres <= TOL)
    # lower bound on the whole solve: every system's network FLOPs at the BF16 matrix peak plus its
    # algorithmic Krylov bytes (52n + 16nj at step j of a cycle) at the HBM peak
    q = 1 << (LEVELS - 1)
    net_fl = kry_b = 0.0
    for inf, p, (nx, pml) in zip(infos, probs, sizes):
        Hp = (nx + 2 * pml + q - 1) // q * q
        fl = sum(layer_flops(kind, ci, co, H, W) for (_, kind, ci, co, H, W) in net_layers(LEVELS, BASE, IN_CH, Hp, Hp))
        net_fl += inf.its * (fl + 2.0 * Hp * Hp * 2 * BASE)
        kry_b += sum(52.0 * p.n + 16.0 * p.n * (k % M_RESTART) for k in range(inf.its))
    bound_s = net_fl / (PEAK_BF16_TFLOPS * 1e12) + kry_b / (PEAK_HBM_GBS * 1e9)
    return {"workload": f"{nsys} systems of the batched-serving mix, BF16 U-Net, FP32 Krylov, FGMRES(30), tol 1e-6",
            "nodes_total": int(sum(p.n for p in probs)), "seconds": round(dt, 3),
            "converged": conv, "solves_per_s": round(conv / dt, 3),
            "its_min_median_max": [int(its.min()), int(np.median(its)), int(its.max())],
            "ms_per_step": round(dt / steps * 1e3, 2),
            "node_iterations_per_s": round(node_its / dt, 1),
            "max_true_relres": max(i.true_relres for i in infos),
            "network_tflop": round(net_fl * 1e-12, 2), "krylov_algorithmic_gb": round(kry_b * 1e-9, 1),
            "bound_s": round(bound_s, 3), "combined_frac": round(bound_s / dt, 4)}


def bench_spectral(hz, torch, net):
    """The paper's Fourier-differentiation operator (hz_grid.disc = spectral): one apply of A on
    the single-solve grid (296^2) and the large grid (1088^2) in FP32 and FP64 (HIP events; the
    kernel contracts each node's row and column with the per-axis matrices, 8 (nx + ny) FLOP per
    node), and the BF16-network FGMRES(30) solve of the single-solve system with that operator,
    bounded to 1000 iterations, with the network trained on the finite-difference operator (which
    does not precondition this one well) and with the one the library's epoch loop trained on
    the Fourier-differentiation operator itself (`solve_296_spectral_net`)."""
    from paper_2607_16906_amd.train import load_weights
    from synth import H_10PPW, c2_system, c5_system
    nets = [("solve_296", net)]
    if os.path.exists(WEIGHTS_SPEC):
        ws = np.load(WEIGHTS_SPEC)
        nets.append(("solve_296_spectral_net", hz.Net(int(ws["levels"]), int(ws["base"]), 5, load_weights(WEIGHTS_SPEC))))
    out = {"workload": "Fourier-differentiation operator: apply at 296^2 and 1088^2; FGMRES(30), BF16 U-Net, "
                       "FP32 Krylov, tol 1e-6 on the 256^2 + 20 PML system"}
    for name, sysf in (("296", c2_system), ("1088", c5_system)):
        s = sysf(0)
        gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW, disc="spectral")
        n = s.nt * s.nt
        flops = 8.0 * (2 * s.nt) * n
        for dt, tag in ((torch.complex64, "fp32"), (torch.complex128, "fp64")):
            x = torch.randn(n, dtype=dt, device="cuda")
            for _ in range(3):
                gp.apply(x)
            reps = 20 if name == "296" else 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                y = gp.apply(x)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out[f"apply_{name}_{tag}_us"] = round(ms * 1e3, 2)
            out[f"apply_{name}_{tag}_tflops"] = round(flops / ms * 1e-9, 2)
            del x, y
        if name == "296":
            b = torch.from_numpy(s.b.ravel()).cuda()
            for key, nn in nets:
                hz.fgmres(gp, b, net=nn, m=M_RESTART, tol=TOL, maxit=M_RESTART)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = hz.fgmres(gp, b, net=nn, m=M_RESTART, tol=TOL, maxit=1000)
                torch.cuda.synchronize()
                dtm = time.perf_counter() - t0
                out[key] = {"its": info.its, "converged": info.status == 0, "true_relres": info.true_relres,
                            "ms_per_solve": round(dtm * 1e3, 2), "solves_per_s": round(1.0 / dtm, 3),
                            "us_per_it": round(dtm * 1e6 / max(info.its, 1), 1)}
        del gp
    return out


def bench_appendix_b(hz, torch, net, nsys=5, nx=64, npml=16):
    """The paper's second synthetic workload at its solver settings (eta_b = 1e-12, maxit = 512
    without restart): constant speed with one or two +-1 point sources, four aligned or faulted
    layers with a smoothed source, at the paper's scale (64^2 interior, here with 16 PML cells
    outside it); nsys systems per kind, FGMRES with the BF16 network and plain GMRES, FP64 Krylov
    vectors (1e-12 is below FP32 resolution)."""
    from synth import APPB_KINDS, H_10PPW, appendix_b_system
    res = {"workload": f"{nsys} systems per kind, {nx}^2 + {npml} PML, m = 512 (no restart), maxit 512, "
                       "tol 1e-12, FP64 Krylov; FGMRES with the BF16 U-Net and GMRES", "kinds": {}}
    for kind in APPB_KINDS:
        rows = {"fgmres_its": [], "fgmres_ms": [], "fgmres_converged": 0, "fgmres_final_relres": [],
                "gmres_its": [], "gmres_ms": [], "gmres_converged": 0, "gmres_final_relres": []}
        for sid in range(nsys):
            s = appendix_b_system(kind, sid, nx=nx, npml=npml)
            gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
            b = torch.from_numpy(s.b.ravel()).cuda()
            for tag, nn in (("fgmres", net), ("gmres", None)):
                hz.fgmres(gp, b, net=nn, m=512, tol=1e-12, maxit=8, krylov="c128")   # graphs, tuning
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = hz.fgmres(gp, b, net=nn, m=512, tol=1e-12, maxit=512, krylov="c128")
                torch.cuda.synchronize()
                rows[f"{tag}_its"].append(info.its)
                rows[f"{tag}_ms"].append(round((time.perf_counter() - t0) * 1e3, 1))
                rows[f"{tag}_converged"] += int(info.status == 0)
                rows[f"{tag}_final_relres"].append(float(f"{info.true_relres:.3e}"))
            del gp
        res["kinds"][kind] = rows
    return res


RESTART_RUNS = [(m, "c64", "cgs2") for m in (10, 30, 50, 100, 200, 512)] + [
    (30, "c64", "dcgs2"), (100, "c64", "dcgs2"), (100, "c128", "cgs2"), (100, "c128", "dcgs2"),
    (512, "c128", "cgs2"), (512, "c128", "dcgs2")]


def bench_restart(hz, torch, net, runs=RESTART_RUNS):
    """Restart-length study on the single-solve workload (296^2, BF16 network, tol 1e-6), up to
    the paper's long-cycle regime (m = 512): iterations, solve time and time per iteration (the
    orthogonalisation grows with the basis), for CGS with one reorthogonalisation and the delayed
    (one-reduction) form, with FP32 or FP64 Krylov vectors. The one-reduction form is not run with
    FP32 vectors at m = 512: it loses orthogonality there and stalls near 4e-4."""
    from synth import H_10PPW, c2_system
    s = c2_system(0)
    gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
    b = torch.from_numpy(s.b.ravel()).cuda()
    rows = []
    for m, kr, ortho in runs:
        ws = torch.empty(hz.fgmres_workspace_bytes(gp, net, m, 3000, kr, "bf16", ortho), dtype=torch.uint8,
                         device="cuda")
        kw = dict(net=net, m=m, tol=TOL, maxit=3000, krylov=kr, workspace=ws, ortho=ortho)
        hz.fgmres(gp, b, **kw)   # warm-up (graphs, tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = hz.fgmres(gp, b, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows.append({"m": m, "krylov": kr, "ortho": ortho, "its": info.its, "cycles": info.cycles,
                     "converged": info.status == 0, "true_relres": info.true_relres,
                     "ms_per_solve": round(dt * 1e3, 2), "us_per_it": round(dt * 1e6 / max(info.its, 1), 1)})
        del ws
    return {"workload": "single solve, 256^2 interior + 20 PML, BF16 U-Net, tol 1e-6, FGMRES(m)", "runs": rows}


def bench_large(hz, torch, net4, maxit=12000, m=50):
    """Large single solve: 1024^2 interior + 32 PML (1088^2 nodes), FGMRES(50) to tol 1e-6 with the
    5-level / 32-channel BF16 network trained at 128^2 + 16 PML and applied fully convolutionally,
    FP32 Krylov vectors. Reports solves/s, the network's rate at this size, the HBM rate of the
    Krylov phase (stencil + Gram-Schmidt passes + Givens; the basis of m + 1 vectors of 9.5 MB no
    longer fits in the caches) and the checkpointed training step (loss and gradient) on 4 samples
    at this size."""
    from paper_2607_16906_amd.train import load_weights
    from synth import H_10PPW, c5_system
    s = c5_system(0)
    gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
    n = s.nt * s.nt
    net = hz.Net(5, BASE, IN_CH, load_weights(WEIGHTS_L5))
    Hp = (s.nt + 15) // 16 * 16
    net.autotune(gp, "bf16")
    layers = time_layers(net, Hp, Hp, reps=5, levels=5)
    net_ms = sum(r["ms"] for r in layers)
    net_flops = sum(r["flops"] for r in layers)
    dom = max(layers, key=lambda r: r["ms"])
    b = torch.from_numpy(s.b.ravel()).cuda()
    ws = torch.empty(hz.fgmres_workspace_bytes(gp, net, m, maxit, "c64", "bf16"), dtype=torch.uint8, device="cuda")

    def solve(mode, cap):
        net.set_fused_upsampling(mode)
        hz.fgmres(gp, b, net=net, m=m, tol=1e-6, maxit=m, workspace=ws)   # warm-up (one cycle)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = hz.fgmres(gp, b, net=net, m=m, tol=1e-6, maxit=cap, workspace=ws)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    # the phase split below subtracts the separately timed layers, so this solve runs them
    # separately; a bounded solve with the autotuned fused decoder form is timed beside it
    dt, info = solve(0, maxit)
    dt_f, info_f = solve(2, 200)
    ms_it = dt / max(info.its, 1) * 1e3
    # algorithmic bytes of step j, the least the step needs: the matvec (20n), one read of the
    # basis for the projections and one for the update (16nj), w and the new vector (32n):
    # 52n + 16nj; the implemented classical Gram-Schmidt with reorthogonalisation reads the basis
    # three times (52n + 24n (j + 1))
    steps = [k % m for k in range(info.its)]
    kbytes = sum(52 * n + 24 * n * (j + 1) for j in steps)
    abytes = sum(52 * n + 16 * n * j for j in steps)
    kry_s = max(dt - info.its * net_ms * 1e-3, 1e-9)
    # checkpointed training step (loss + gradient, BF16, recompute) on 4 samples of this size
    probs = [hz.Problem(c5_system(k).c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW) for k in range(4)]
    from synth import box_smoothed_noise, rng_for
    r = torch.from_numpy(np.stack([box_smoothed_noise(s.nt, rng_for(5, 3, k)).ravel() for k in range(4)])
                         .astype(np.complex64)).cuda()
    tws = torch.empty(hz.train_workspace_bytes(net, probs[0], 4, "bf16", recompute=True), dtype=torch.uint8,
                      device="cuda")
    hz.loss_backward(net, probs, r, prec="bf16", recompute=True, workspace=tws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        hz.loss_backward(net, probs, r, prec="bf16", recompute=True, workspace=tws)
    torch.cuda.synchronize()
    bwd_ms = (time.perf_counter() - t0) / 3 * 1e3
    conv = info.status == 0 and info.true_relres <= 1e-6
    return {"workload": "single solve, 1024^2 interior + 32 PML (1088^2), FGMRES(50) to tol 1e-6, BF16 5-level/32-ch "
                        "U-Net trained at 128^2 + 16 PML, FP32 Krylov",
            "nodes": n, "its": info.its, "converged": conv, "true_relres": info.true_relres,
            "solves_per_s": round(1.0 / dt, 4) if conv else 0.0, "seconds": round(dt, 3),
            "ms_per_it": round(ms_it, 3),
            "ms_per_it_fused_decoder": round(dt_f / max(info_f.its, 1) * 1e3, 3),
            "network_ms_per_apply": round(net_ms, 3), "network_tflops": round(net_flops / net_ms * 1e-9, 1),
            "network_mfma_frac": round(net_flops / net_ms * 1e-9 / PEAK_BF16_TFLOPS, 4),
            "dominant_layer": {"layer": dom["layer"], "shape": f"{dom['cin']}->{dom['cout']} ch on {dom['H']}x{dom['W']}",
                               "ms": round(dom["ms"], 4), "tflops": round(dom["flops"] / dom["ms"] * 1e-9, 1)},
            "krylov_ms_per_it": round(kry_s / max(info.its, 1) * 1e3, 3),
            "krylov_hbm_gbs": round(kbytes / kry_s / 1e9, 1),
            "krylov_hbm_frac": round(kbytes / kry_s / 1e9 / PEAK_HBM_GBS, 4),
            "krylov_algorithmic_hbm_gbs": round(abytes / kry_s / 1e9, 1),
            "krylov_algorithmic_hbm_frac": round(abytes / kry_s / 1e9 / PEAK_HBM_GBS, 4),
            "training_step_4x1088_checkpointed_ms": round(bwd_ms, 2)}


def cpu_baseline(system, theta, gpu_its, budget_s=20.0):
    """The FP64 oracle FGMRES on the same system and weights, timed over a bounded number of
    iterations and scaled to one solve of gpu_its iterations."""
    from oracle import fgmres as ofg
    from oracle import helmholtz as ohz
    from oracle import unet
    from synth import C_REF, H_10PPW
    op = ohz.Problem(system.c.astype(np.float32).astype(np.float64), system.npml, H_10PPW, 1.0, 2.0, C_REF)
    specs = unet.layer_specs(LEVELS, BASE, IN_CH)
    th = np.asarray(theta, np.float64)
    nt = system.nt
    A = lambda x: ohz.op_apply(op, x.reshape(nt, nt)).ravel()
    M = lambda v: unet.precond_apply(th, specs, op, v.reshape(nt, nt)).ravel()
    t0 = time.time()
    ofg.fgmres(A, M, system.b, m=M_RESTART, tol=TOL, maxit=1)
    t1 = time.time() - t0
    its = max(2, min(M_RESTART, int(budget_s / max(t1, 1e-3))))
    t0 = time.time()
    r = ofg.fgmres(A, M, system.b, m=M_RESTART, tol=TOL, maxit=its)
    dt = time.time() - t0
    per_it = dt / r.its
    return {"value": 1.0 / (per_it * gpu_its), "unit": "solves/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"{r.its} FP64 oracle FGMRES iterations ({dt:.1f} s, {per_it * 1e3:.0f} ms/it) on the same "
                      f"296^2 system and weights, scaled to the {gpu_its} iterations of the GPU solve"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--large-maxit", type=int, default=12000,
                    help="with --only large: cap on the large solve's iterations (a bounded run for the profiler)")
    ap.add_argument("--no-extra", action="store_true", help="skip the training and batched sections")
    ap.add_argument("--roofline-variant", default="",
                    help="with --roofline-only: pin the layer's launch variant 'tn,rows[,stages[,tiles]]'")
    ap.add_argument("--roofline-only", action="store_true", help="only the per-layer roofline timing")
    ap.add_argument("--roofline-layer", type=int, default=-1,
                    help="with --roofline-only: time this layer alone (for a profiler run of one kernel)")
    ap.add_argument("--roofline-grid", choices=["single", "large"], default="single",
                    help="with --roofline-only: the single-solve grid (296^2) or the large solve's (1088^2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --roofline-only: also copy 512 MiB with a plain device copy (counter calibration)")
    ap.add_argument("--only", choices=["training", "training_loop", "train_then_solve", "batched", "large",
                                       "restart", "spectral", "appendix_b", "paper8"],
                    default=None,
                    help="run one extra section alone and print its JSON (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the single-solve workload is measured on one MI355X; "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_16906_amd import hz
    from synth import H_10PPW, c2_system

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = np.load(WEIGHTS)
    theta = w["theta"].astype(np.float32)
    if args.only:
        if args.only == "training":
            res = bench_training(hz, torch, steps=2)
        elif args.only == "training_loop":
            res = bench_training_loop(hz, torch)
        elif args.only == "train_then_solve":
            res = bench_train_then_solve(hz, torch)
        else:
            net1 = hz.Net(LEVELS, BASE, IN_CH, theta)
            if args.only == "large":
                res = bench_large(hz, torch, net1, maxit=args.large_maxit)
            else:
                res = {"batched": bench_batched, "restart": bench_restart, "spectral": bench_spectral,
                       "appendix_b": bench_appendix_b, "paper8": bench_paper8}[args.only](hz, torch, net1)
        print(json.dumps({args.only: res}))
        return
    levels = LEVELS
    if args.roofline_only and args.roofline_grid == "large":
        # the large system with the 5-level network its solve uses
        from synth import c5_system
        s = c5_system(0)
        from paper_2607_16906_amd.train import load_weights
        levels = 5
        net = hz.Net(5, BASE, IN_CH, load_weights(WEIGHTS_L5))
    else:
        s = c2_system(0)
        net = hz.Net(LEVELS, BASE, IN_CH, theta)
    gp = hz.Problem(s.c.astype(np.float32).ravel(), s.nx, s.nx, s.npml, H_10PPW)
    q = 1 << (levels - 1)
    Hp = Wp = (s.nt + q - 1) // q * q
    net.autotune(gp, "bf16")
    if levels == LEVELS:
        net.autotune(gp, "fp32")

    if args.roofline_only and args.roofline_variant:
        # pin the launch variant (the profiler runs must time the launch the solve uses)
        vv = [int(t) for t in args.roofline_variant.split(",")]
        tn, rows, stages, tiles = vv[0], vv[1], (vv[2] if len(vv) > 2 else 1), (vv[3] if len(vv) > 3 else 1)
        lay = [r for r in net_layers(levels, BASE, IN_CH, Hp, Wp) if r[0] == args.roofline_layer][0]
        net.set_layer_variant(args.roofline_layer, lay[4], lay[5], tn, rows, stages, tiles)
    layers = time_layers(net, Hp, Wp, reps=50, only=args.roofline_layer if args.roofline_only else -1,
                         levels=levels)
    dom = max(layers, key=lambda r: r["ms"])
    tn, rows, stages, tiles = net.layer_variant(dom["layer"], dom["H"], dom["W"]) if dom["kind"] == 0 else (0, 0, 1, 1)
    variant = f"tn{tn} rows{rows}" + (f" stages{stages}" if stages > 1 else "") + (f" tiles{tiles}" if tiles > 1 else "")
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    net_ms = sum(r["ms"] for r in layers)
    net_flops = sum(r["flops"] for r in layers)
    kname = "k_conv3<PolBF16, ...> (3x3 layer, autotuned variant)" if dom["kind"] == 0 else "k_convT2<PolBF16>"
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": measured_traffic(dom["layer"], variant),
                "kernel": kname, "variant": variant, "layer": dom["layer"],
                "shape": f"{dom['cin']}->{dom['cout']} ch on {dom['H']}x{dom['W']}",
                "flops_per_launch": dom["flops"], "avg_launch_ms": round(dom["ms"], 5)}
    if args.roofline_only:
        if args.copy_calibration:
            src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"roofline": roofline, "layers": layers}))
        return

    b = torch.from_numpy(s.b.ravel()).cuda()
    ws = torch.empty(hz.fgmres_workspace_bytes(gp, net, M_RESTART, MAXIT, "c64", "fp32"), dtype=torch.uint8,
                     device="cuda")

    xbuf = torch.empty_like(b)

    def solve(prec):
        # fixed b, x and workspace: every solve after the first replays the kept cycle graphs
        return hz.fgmres(gp, b, net=net, m=M_RESTART, tol=TOL, maxit=MAXIT, krylov="c64", net_prec=prec,
                         workspace=ws, out=xbuf)

    for _ in range(args.warmup):
        x, info = solve("bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        x, info = solve("bf16")
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    its = infos[-1].its
    ok = all(i.status == 0 and i.true_relres <= TOL for i in infos)

    # the plain FP32 form: same solver and weights, network in FP32 on the matrix cores
    x32, i32 = solve("fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp32_steps):
        x32, i32 = solve("fp32")
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t0) / args.fp32_steps * 1e3

    st_ms = time_stencil(hz, torch, 296)
    big = 4096
    st_big = time_stencil(hz, torch, big, reps=20)

    out = {
        "metric": "solves/s to rel-res 1e-6: BF16-net FGMRES vs plain FP32 FGMRES; HBM GB/s",
        "value": round(args.steps / elapsed, 4) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "single solve, 256^2 interior + 20 PML (296^2), skull-ring velocity, 1-4 Gaussian "
                               "sources, 4-level/32-ch U-Net BF16, FP32 Krylov, FGMRES(30), tol 1e-6",
                   "nodes": s.nt * s.nt, "restart": M_RESTART, "tol": TOL,
                   "weights_step": int(w["step"])},
        "solve": {"its": its, "cycles": infos[-1].cycles, "true_relres": infos[-1].true_relres,
                  "converged": ok, "us_per_it": round(ms_step * 1e3 / max(its, 1), 1),
                  "phase_ms": {k: round(v, 3) for k, v in infos[-1].phase_ms.items()},
                  "vs_oracle": oracle_comparison(its, infos[-1].true_relres, "bf16_weights")},
        "fp32_form": {"value": round(1e3 / ms32, 4) if i32.status == 0 else 0.0, "unit": "solves/s",
                      "ms_per_solve": round(ms32, 3), "its": i32.its, "true_relres": i32.true_relres,
                      "vs_oracle": oracle_comparison(i32.its, i32.true_relres, "fp32_weights")},
        "speedup_bf16_vs_fp32": round(ms32 / ms_step, 3),
        "roofline": roofline,
        "network": {"ms_per_apply_layers": round(net_ms, 4), "tflops_layers": round(net_flops / net_ms * 1e-9, 2),
                    "gflop_per_apply": round(net_flops * 1e-9, 3),
                    "layer_us": [[r["layer"], "conv3" if r["kind"] == 0 else "convT2", r["cin"], r["cout"], r["H"],
                                  round(r["ms"] * 1e3, 2)] for r in layers]},
        "stencil": {"fp32_296_us": round(st_ms * 1e3, 2),
                    "fp32_296_gbs_in_cache": round(20 * 296 * 296 / (st_ms * 1e-3) / 1e9, 1),
                    f"fp32_{big}_us": round(st_big * 1e3, 2),
                    f"fp32_{big}_hbm_gbs": round(20 * big * big / (st_big * 1e-3) / 1e9, 1),
                    "hbm_frac": round(20 * big * big / (st_big * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
    }
    note(f"single solve: {out['value']} solves/s BF16, {out['fp32_form']['value']} FP32 form")
    if not args.no_extra:
        sections = [("training", lambda: bench_training(hz, torch)),
                    ("training_loop", lambda: bench_training_loop(hz, torch)),
                    ("train_then_solve", lambda: bench_train_then_solve(hz, torch)),
                    ("batched", lambda: bench_batched(hz, torch, net)),
                    ("large", lambda: bench_large(hz, torch, net)),
                    ("restart", lambda: bench_restart(hz, torch, net)),
                    ("spectral", lambda: bench_spectral(hz, torch, net)),
                    ("appendix_b", lambda: bench_appendix_b(hz, torch, net)),
                    ("paper8", lambda: bench_paper8(hz, torch, net))]
        for name, fn in sections:
            t0 = time.perf_counter()
            out[name] = fn()
            note(f"{name} done in {time.perf_counter() - t0:.1f} s")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, theta, its)
        note("cpu_baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
