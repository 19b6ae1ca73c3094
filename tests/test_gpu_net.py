"""GPU parity of the U-Net preconditioner (no_precond_apply) against the FP64 oracle in FP64,
FP32 and BF16 (the oracle then runs on the BF16-rounded weights)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import unet
from synth import box_smoothed_noise, c1_system, he_uniform, rng_for, skull_ring_velocity

from gpu_util import make_pair, rel, to_dev, to_np


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64 (test-side input preparation)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def setup(levels, base, in_ch, nx, p, seed=0):
    from paper_2607_16906_amd import hz
    nt = nx + 2 * p
    c = skull_ring_velocity(nt, p, rng_for(12, 0, seed), rings=2)
    op, gp = make_pair(c, p)
    specs = unet.layer_specs(levels, base, in_ch)
    theta = he_uniform(unet.init_shapes(specs), rng_for(12, 2, seed))
    net = hz.Net(levels, base, in_ch, theta)
    v = box_smoothed_noise(nt, rng_for(12, 3, seed)) + 0.3 * (
        np.random.default_rng(seed).standard_normal((nt, nt)))
    return op, gp, specs, theta, net, v


@pytest.mark.parametrize("levels,base,in_ch,nx,p", [(2, 16, 2, 64, 8), (3, 8, 5, 70, 8), (4, 8, 5, 40, 8),
                                                    (1, 8, 2, 21, 4)])
def test_net_fp64_matches_oracle(levels, base, in_ch, nx, p):
    op, gp, specs, theta, net, v = setup(levels, base, in_ch, nx, p)
    z = to_np(net.apply(gp, to_dev(v, torch.complex128), prec="fp64")).reshape(op.ny, op.nx)
    ref = unet.precond_apply(theta.astype(np.float64), specs, op, v)
    assert rel(z, ref) <= 1e-12


@pytest.mark.parametrize("levels,base,in_ch,nx,p", [(4, 32, 5, 88, 16), (2, 16, 2, 64, 8)])
def test_net_fp32_within_1e5(levels, base, in_ch, nx, p):
    op, gp, specs, theta, net, v = setup(levels, base, in_ch, nx, p, seed=1)
    z = to_np(net.apply(gp, to_dev(v, torch.complex64), prec="fp32")).reshape(op.ny, op.nx)
    ref = unet.precond_apply(theta.astype(np.float64), specs, op, v)
    assert rel(z, ref) <= 1e-5


@pytest.mark.parametrize("levels,base,in_ch,nx,p", [(4, 32, 5, 88, 16), (3, 16, 5, 50, 7)])
def test_net_bf16_normwise(levels, base, in_ch, nx, p):
    op, gp, specs, theta, net, v = setup(levels, base, in_ch, nx, p, seed=2)
    z = to_np(net.apply(gp, to_dev(v, torch.complex64), prec="bf16")).reshape(op.ny, op.nx)
    ref = unet.precond_apply(bf16_round(theta), specs, op, v)
    err = rel(z, ref)
    print(f"bf16 normwise error {err:.3e}")
    assert err <= 3e-2


def test_net_zero_input_and_scale():
    op, gp, specs, theta, net, v = setup(2, 16, 5, 30, 5, seed=3)
    zero = torch.zeros(gp.n, dtype=torch.complex64, device="cuda")
    assert torch.count_nonzero(net.apply(gp, zero, prec="fp32")).item() == 0
    z1 = net.apply(gp, to_dev(v, torch.complex128), prec="fp64")
    z2 = net.apply(gp, to_dev(3.0 * v, torch.complex128), prec="fp64")
    assert rel(to_np(z2), 3.0 * to_np(z1)) <= 1e-13


def test_net_bad_arch_rejected():
    from paper_2607_16906_amd import hz
    with pytest.raises(ValueError):
        hz.param_count(4, 12, 5)
    assert hz.param_count(4, 32, 5) == unet.param_count(unet.layer_specs(4, 32, 5))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 3e-2)])
def test_autotuned_variants_keep_parity(prec, tol):
    # the autotuner may pick other channel tiles, taller pixel tiles or a split of the input
    # channels (split-K with a separate reduction): the forward pass keeps its parity
    op, gp, specs, theta, net, v = setup(4, 32, 5, 120, 20, seed=5)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    vd = to_dev(v, dt)
    z0 = to_np(net.apply(gp, vd, prec=prec))
    net.autotune(gp, prec)
    z1 = to_np(net.apply(gp, vd, prec=prec)).reshape(op.ny, op.nx)
    th = bf16_round(theta) if prec == "bf16" else theta.astype(np.float64)
    ref = unet.precond_apply(th, specs, op, v)
    assert rel(z1, ref) <= tol
    assert rel(z1, z0.reshape(op.ny, op.nx)) <= (1e-13 if prec == "fp64" else tol)


def test_pinned_layer_variants_identical_bits():
    # every launch variant accumulates each output in the same order: pinning other channel tiles
    # and tile heights leaves the BF16 and FP32 outputs bit-identical
    from paper_2607_16906_amd import hz
    op, gp, specs, theta, net, v = setup(3, 16, 5, 60, 10, seed=6)
    Hp = (op.ny + 3) // 4 * 4
    convs = [i for i, s in enumerate(specs) if s[1] == "conv3"]
    level = {}
    for i, s in enumerate(specs):
        if s[0].startswith("enc"):
            level[i] = int(s[0][3])
        elif s[0].startswith("dec"):
            level[i] = int(s[0][3])
    for prec, dt in (("bf16", torch.complex64), ("fp32", torch.complex64)):
        vd = to_dev(v, dt)
        outs = []
        for tn0, rows in ((16, 8), (16, 16), (32, 8)):
            for i in convs:
                H = Hp >> level[i]
                tn = tn0 if specs[i][3] % tn0 == 0 else 16
                net.set_layer_variant(i, H, H, tn, rows, prec=prec)
                assert net.layer_variant(i, H, H, prec=prec) == (tn, rows, 1, 1)
            outs.append(net.apply(gp, vd, prec=prec))
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    with pytest.raises(hz.HzError):
        net.set_layer_variant(convs[0], Hp, Hp, 24, 8)
    with pytest.raises(hz.HzError):
        net.set_layer_variant(len(specs) - 1, Hp, Hp, 16, 8)   # the head is not a 3x3 layer
    with pytest.raises(hz.HzError):
        net.set_layer_variant(convs[0], Hp, Hp, 16, 8, stages=2, prec="fp32")   # BF16 only
    with pytest.raises(hz.HzError):
        net.set_layer_variant(convs[0], Hp, Hp, 16, 8, stages=3)
    i32 = next(i for i in convs if specs[i][3] % 32 == 0)
    with pytest.raises(hz.HzError):   # four stages of 32-channel, 16-row tiles do not fit in the LDS
        net.set_layer_variant(i32, Hp >> level[i32], Hp >> level[i32], 32, 16, stages=4)


@pytest.mark.parametrize("levels,base,nx,p", [(4, 32, 64, 8), (2, 96, 40, 8)])
def test_staged_chunks_identical_bits(levels, base, nx, p):
    # several input-channel chunks per LDS stage (one global-load latency per stage) compute the
    # chunks in the same order: BF16 outputs bit-identical to one chunk per stage, with chunk
    # counts that stages do not divide (96 / 192 channels: 3 or 6 chunks of 32; the decoder's two
    # input parts) and every channel tile and tile height
    from paper_2607_16906_amd import hz
    op, gp, specs, theta, net, v = setup(levels, base, 5, nx, p, seed=8)
    q = 1 << (levels - 1)
    Hp = (op.ny + q - 1) // q * q
    convs = [i for i, s in enumerate(specs) if s[1] == "conv3"]
    level = {i: int(s[0][3]) for i, s in enumerate(specs) if s[0][:3] in ("enc", "dec")}
    vd = to_dev(v, torch.complex64)
    net.set_fused_upsampling(0)

    used = [0]

    def run(tn0, rows, stages, tiles=1, inflight=1):
        nws = 0
        for i in convs:
            H = Hp >> level[i]
            tn = tn0 if specs[i][3] % tn0 == 0 else 16
            st, tl = stages, tiles
            if tl > 1:
                st = inflight
                while True:
                    try:
                        net.set_layer_variant(i, H, H, tn, rows, st, tl)
                        nws += 1
                        break
                    except hz.HzError:
                        if st == 2:
                            tl = 1
                            break
                        st -= 1
                if tl == 1:
                    st = stages
            if tl == 1:
                while st > 1:
                    try:
                        net.set_layer_variant(i, H, H, tn, rows, st)
                        break
                    except hz.HzError:
                        st //= 2
                if st == 1:
                    net.set_layer_variant(i, H, H, tn, rows, 1)
            assert net.layer_variant(i, H, H) == (tn, rows, st, tl)
        used[0] += nws
        return net.apply(gp, vd, prec="bf16")

    ref = run(16, 8, 1)
    for tn0, rows, stages in ((16, 8, 2), (16, 8, 4), (32, 8, 4), (16, 16, 4), (64, 16, 2), (32, 16, 2), (64, 8, 2)):
        out = run(tn0, rows, stages)
        assert torch.equal(out, ref), (tn0, rows, stages)
    # the weight-stationary form (all weights of the block's channels in LDS, several pixel tiles
    # per block; tile counts that do not divide the grid's tiles) where the layer qualifies, the
    # first layer (one k-group of 8 channels per tap) included
    for tn0, rows, tiles, inflight in ((16, 8, 2, 2), (32, 8, 3, 2), (64, 16, 4, 3), (32, 16, 7, 3), (16, 8, 64, 4),
                                       (32, 8, 8, 4), (16, 16, 5, 2), (32, 8, 1000, 4)):
        out = run(tn0, rows, 1, tiles, inflight)
        assert torch.equal(out, ref), (tn0, rows, tiles, inflight)
    # (in the 96-channel network, with 3 or 6 chunks per layer, only the first layer takes that
    # form: its input of one k-group per tap)
    assert used[0] > 0


@pytest.mark.parametrize("levels,base,nx,p", [(4, 32, 256, 20), (4, 32, 30, 6), (3, 64, 44, 10), (4, 32, 100, 14)])
def test_fused_upsampling_identical_bits(levels, base, nx, p):
    # the BF16 decoder with the transposed convolution computed inside the next 3x3 layer gives
    # the bits of the two separate layers (ragged tiles, both parities at the tile borders, the
    # image border, untuned and autotuned launch variants)
    from paper_2607_16906_amd import hz
    op, gp, specs, theta, net, v = setup(levels, base, 5, nx, p, seed=8)
    vd = to_dev(v, torch.complex64)
    for tune in (False, True):
        if tune:
            net.set_fused_upsampling(2)
            net.autotune(gp, "bf16")
        outs = []
        for mode in (1, 0, 2):   # always fused, never, the autotuner's choice
            net.set_fused_upsampling(mode)
            outs.append(net.apply(gp, vd, prec="bf16"))
        fused = outs[0]
        for o in outs[1:]:
            assert torch.equal(fused, o), (tune, rel(to_np(fused), to_np(o)))
    with pytest.raises(hz.HzError):
        net.set_fused_upsampling(3)
    # the oracle on the BF16-rounded weights, as for the unfused network
    ref = unet.precond_apply(bf16_round(theta), specs, op, v)
    assert rel(to_np(fused), ref) <= 3e-2
