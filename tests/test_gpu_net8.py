"""GPU parity of the paper's own network (NO_ARCH_PAPER8: 8x8 stride-2 layers, PReLU; Table 2)
against the oracle (oracle/unet8.py): each layer form in FP64, the whole preconditioner in FP64 /
FP32 / BF16 on ragged grids, and an FP64 FGMRES history with it as the preconditioner."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import fgmres as ofg
from oracle import helmholtz as ohz
from oracle import unet8
from synth import box_smoothed_noise, gaussian_sources, rng_for, skull_ring_velocity

from gpu_util import make_pair, rel, to_dev, to_np
from test_gpu_net import bf16_round


def nhwc(a, cp):
    """[C, H, W] -> [H, W, cp] zero-padded channels."""
    C, H, W = a.shape
    out = np.zeros((H, W, cp))
    out[:, :, :C] = a.transpose(1, 2, 0)
    return out


def net8(depth=4, in_ch=5, seed=0):
    from paper_2607_16906_amd import hz
    specs = unet8.layer_specs(depth, 32, in_ch)
    theta = unet8.init_theta(specs, rng_for(21, 2, seed))
    # a different PReLU slope in every layer (both signs of the negative branch)
    r = np.random.default_rng(100 + seed)
    off = 0
    for _, kind, ci, co in specs:
        off += unet8.layer_len(kind, ci, co)
        if kind != "conv1":
            theta[off - 1] = r.uniform(-0.3, 0.6)
    return specs, theta, hz.Net(depth, 32, in_ch, theta, kind="paper8")


def test_layers_fp64_match_oracle():
    specs, theta, net = net8()
    P = unet8.unpack(theta.astype(np.float64), specs)
    rng = np.random.default_rng(1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    # down1: 5 inputs padded to 8 channels, 2 samples, ragged sizes (H/2 x W/2 = 13 x 7)
    for (H, W) in ((26, 14), (64, 48)):
        x = rng.standard_normal((2, 5, H, W))
        y = torch.zeros((2, H // 2, W // 2, 32), dtype=torch.float64, device="cuda")
        net.layer_forward(0, dev(np.stack([nhwc(s, 8) for s in x])), y, H=H, W=W, batch=2, prec="fp64")
        W0, b0, a0 = P["down1"]
        ref = unet8.prelu(unet8.down(x, W0, b0), a0)
        assert rel(to_np(y).transpose(0, 3, 1, 2), ref) <= 1e-13
    # down2 (32 -> 32)
    x = rng.standard_normal((1, 32, 18, 30))
    y = torch.zeros((1, 9, 15, 32), dtype=torch.float64, device="cuda")
    net.layer_forward(1, dev(nhwc(x[0], 32)), y, H=18, W=30, prec="fp64")
    W1, b1, a1 = P["down2"]
    assert rel(to_np(y).transpose(0, 3, 1, 2), unet8.prelu(unet8.down(x, W1, b1), a1)) <= 1e-13
    # up3 (no concat) and up2 (concat: encoder part first), ragged 7 x 5 inputs
    for li, name, cin in ((4, "up3", 32), (5, "up2", 64)):
        x = rng.standard_normal((1, cin, 7, 5))
        y = torch.zeros((1, 14, 10, 32), dtype=torch.float64, device="cuda")
        if cin == 64:
            net.layer_forward(li, dev(nhwc(x[0, :32], 32)), y, H=7, W=5, x1=dev(nhwc(x[0, 32:], 32)), prec="fp64")
        else:
            net.layer_forward(li, dev(nhwc(x[0], 32)), y, H=7, W=5, prec="fp64")
        Wu, bu, au = P[name]
        assert rel(to_np(y).transpose(0, 3, 1, 2), unet8.prelu(unet8.up(x, Wu, bu), au)) <= 1e-13


@pytest.mark.parametrize("nt,p,depth,in_ch", [(74, 10, 4, 5), (45, 6, 3, 5), (16, 4, 4, 5), (296, 20, 4, 5),
                                               (30, 4, 1, 2), (70, 5, 5, 2)])
def test_precond_matches_oracle(nt, p, depth, in_ch):
    # grids padded to a multiple of 2^depth: 74 -> 80, 45 -> 48, 16 exact, 296 -> 304 (the
    # single-solve grid), 30 -> 30 (depth 1), 70 -> 96 (depth 5); two input channels (the field
    # alone) in the last two
    from paper_2607_16906_amd import hz
    specs, theta, net = net8(depth=depth, seed=depth, in_ch=in_ch)
    c = skull_ring_velocity(nt, p, rng_for(21, 0, nt), rings=2)
    op, gp = make_pair(c, p)
    v = box_smoothed_noise(nt, rng_for(21, 3, nt))
    ref = unet8.precond_apply(theta.astype(np.float64), specs, op, v)
    z64 = to_np(net.apply(gp, to_dev(v, torch.complex128), prec="fp64")).reshape(nt, nt)
    e64 = rel(z64, ref)
    z32 = to_np(net.apply(gp, to_dev(v, torch.complex64), prec="fp32")).reshape(nt, nt)
    e32 = rel(z32, ref)
    refb = unet8.precond_apply(bf16_round(theta), specs, op, v)
    zb = to_np(net.apply(gp, to_dev(v, torch.complex64), prec="bf16")).reshape(nt, nt)
    eb = rel(zb, refb)
    print(f"nt {nt}: fp64 {e64:.2e} fp32 {e32:.2e} bf16 {eb:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5 and eb <= 3e-2
    # a zero field gives a zero output
    z0 = net.apply(gp, torch.zeros(nt * nt, dtype=torch.complex128, device="cuda"), prec="fp64")
    assert torch.count_nonzero(z0).item() == 0


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_fgmres_fp64_with_paper_network_matches_oracle(ortho):
    from paper_2607_16906_amd import hz
    specs, theta, net = net8(seed=5)
    nt, p = 40, 6
    c = skull_ring_velocity(nt, p, rng_for(21, 0, 99), rings=1)
    b = gaussian_sources(nt, p, rng_for(21, 1, 99))
    op, gp = make_pair(c, p)
    M = lambda v: unet8.precond_apply(theta.astype(np.float64), specs, op, v.reshape(nt, nt)).ravel()
    A = lambda x: ohz.op_apply(op, x.reshape(nt, nt)).ravel()
    ref = ofg.fgmres(A, M, b, m=20, tol=1e-9, maxit=60)
    x, info = hz.fgmres(gp, to_dev(b, torch.complex128), net=net, m=20, tol=1e-9, maxit=60, krylov="c128",
                        net_prec="fp64", ortho=ortho)
    assert info.its == ref.its and info.status == ref.status
    h = np.array(ref.est_history)
    d = np.abs(info.hist - h)
    assert np.all(d <= 1e-10 * h + 1e-14), float(np.max(d / (1e-10 * h + 1e-14)))
    assert rel(to_np(x), ref.x) <= 1e-9


def test_paper_network_rejected_where_unsupported():
    from paper_2607_16906_amd import hz
    specs, theta, net = net8(depth=2)
    c = skull_ring_velocity(24, 4, rng_for(21, 0, 7), rings=1)
    _, gp = make_pair(c, 4)
    r = torch.zeros((1, gp.n), dtype=torch.complex64, device="cuda")
    with pytest.raises(hz.HzError):
        hz.loss_backward(net, [gp], r)
    with pytest.raises(hz.HzError):
        hz.fgmres_batched([gp], [r[0]], net=net, m=5, maxit=5)
    with pytest.raises(ValueError):
        hz.Net(4, 16, 5, np.zeros(10, np.float32), kind="paper8")


WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2607_16906_amd",
                           "weights")
# trained by the oracle's trainer (oracle/train_weights.py --arch paper8): may feed the oracle
WEIGHTS8 = os.path.join(WEIGHTS_DIR, "paper8_d4_c32_in5.npz")
# trained by the library's epoch loop on the GPU (train.py --arch paper8, data set D0): never fed
# to the oracle
WEIGHTS8_D0 = os.path.join(WEIGHTS_DIR, "paper8_d4_c32_in5_D0.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS8), reason="oracle-trained weights of the paper's network missing")
def test_trained_paper_network_fgmres_fp64_matches_oracle():
    # with the weights the oracle trained for this network: one FP64 FGMRES cycle of 30 steps on a
    # small grid against the oracle, step for step (the whole residual history, iteration count,
    # status and the cycle's solution); the network does not reach 1e-8 here, and over later
    # cycles of such a stagnating run rounding-level differences grow, as for the C1 system
    from paper_2607_16906_amd import hz
    w = np.load(WEIGHTS8)
    theta = w["theta"].astype(np.float32)
    specs = unet8.layer_specs(4, 32, 5)
    net = hz.Net(4, 32, 5, theta, kind="paper8")
    nt, p = 40, 8
    c = skull_ring_velocity(nt, p, rng_for(21, 0, 7), rings=1)
    b = gaussian_sources(nt, p, rng_for(21, 1, 7))
    op, gp = make_pair(c, p)
    M = lambda v: unet8.precond_apply(theta.astype(np.float64), specs, op, v.reshape(nt, nt)).ravel()
    A = lambda x: ohz.op_apply(op, x.reshape(nt, nt)).ravel()
    ref = ofg.fgmres(A, M, b, m=30, tol=1e-8, maxit=30)
    x, info = hz.fgmres(gp, to_dev(b, torch.complex128), net=net, m=30, tol=1e-8, maxit=30, krylov="c128",
                        net_prec="fp64")
    print(f"trained paper network, 40^2: oracle its {ref.its} (status {ref.status}), GPU its {info.its} "
          f"(status {info.status}), final estimate {ref.est_history[-1]:.3e}")
    assert info.status == ref.status and info.its == ref.its
    h = np.array(ref.est_history)
    d = np.abs(info.hist - h)
    assert np.all(d <= 1e-10 * h + 1e-14), float(np.max(d / (1e-10 * h + 1e-14)))
    assert rel(to_np(x), ref.x) <= 1e-8


@pytest.mark.skipif(not os.path.exists(WEIGHTS8_D0), reason="GPU-trained weights of the paper's network missing")
@pytest.mark.parametrize("sid", [0, 1])
def test_gpu_trained_paper_network_bf16_solve(sid):
    # the paper network trained on the GPU on data set D0 (Table 4) at 128^2 + 16 PML preconditions
    # BF16 FGMRES(30) on single-solve systems at the 64^2 + 16 PML size to 1e-6: converged, and the
    # true residual recomputed by the oracle's FP64 operator
    from paper_2607_16906_amd import hz
    from synth import c2_system
    w = np.load(WEIGHTS8_D0)
    net = hz.Net(4, 32, 5, w["theta"].astype(np.float32), kind="paper8")
    s = c2_system(sid, nx=64, npml=16)
    op, gp = make_pair(s.c, s.npml)
    x, info = hz.fgmres(gp, to_dev(s.b, torch.complex128), net=net, m=30, tol=1e-6, maxit=2000)
    xr = to_np(x).reshape(s.nt, s.nt)
    tr = np.linalg.norm(s.b - ohz.op_apply(op, xr)) / np.linalg.norm(s.b)
    print(f"GPU-trained paper network (D0), 96^2 BF16: its {info.its}, true relres {tr:.3e}")
    assert info.status == 0 and tr <= 1e-6 and abs(tr - info.true_relres) <= 1e-9
