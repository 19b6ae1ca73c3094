"""GPU parity of the epoch-based training loop (paper_2607_16906_amd.train) against the oracle's
loop (Section 3.4, Tables 3 and 5): per-step training losses, per-epoch validation losses, the
saved epoch and the parameters, on a fixed D0-like data set with a short last batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import helmholtz as ohz
from oracle import train_loop as otl
from oracle import unet
from synth import VAL_FIRST, epoch_order, he_uniform, rng_for, training_set

from gpu_util import make_pair, to_np
from test_gpu_net import bf16_round


def data(S, V, nint, p):
    nt = nint + 2 * p
    c, b = training_set(S, nt, p)
    vc, vb = training_set(V, nt, p, first=VAL_FIRST)
    b = b.astype(np.complex64)
    vb = vb.astype(np.complex64)
    tr = [make_pair(ci, p) for ci in c]
    va = [make_pair(ci, p) for ci in vc]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.reshape(len(a), -1))).cuda()
    return ([o for o, _ in tr], [g for _, g in tr], b, dev(b), [o for o, _ in va], [g for _, g in va], vb, dev(vb))


@pytest.mark.parametrize("squared,recompute", [(False, False), (True, True)])
def test_loop_matches_oracle_loop_fp32(squared, recompute):
    # the unsquared loss with full activations, and the paper's squared loss with activation
    # checkpointing
    from paper_2607_16906_amd import hz
    from paper_2607_16906_amd.train import Trainer
    levels, base, nint, p = 3, 8, 24, 4
    S, V, batch, epochs = 10, 3, 4, 3          # batches of 4, 4, 2
    otr, gtr, b, bd, ova, gva, vb, vbd = data(S, V, nint, p)
    specs = unet.layer_specs(levels, base, 5)
    theta0 = he_uniform(unet.init_shapes(specs), rng_for(42, 2, 0))
    orders = [epoch_order(S, e) for e in range(epochs)]
    net = hz.Net(levels, base, 5, theta0)
    tr = Trainer(net, gtr, bd, gva, vbd, batch=batch, prec="fp32", squared=squared, recompute=recompute)
    res = tr.fit(theta0, orders, lr0=1e-2, lr_min=1e-3, clip=1.0)
    ref = otl.train(theta0.astype(np.float64), specs, otr, b.astype(np.complex128), ova,
                    vb.astype(np.complex128), orders, batch=batch, lr0=1e-2, lr_min=1e-3, clip=1.0,
                    squared=squared)
    tl_err = np.max(np.abs(res.train_loss - ref.train_loss) / np.asarray(ref.train_loss))
    vl_err = np.max(np.abs(np.asarray(res.val_loss) - ref.val_loss) / np.asarray(ref.val_loss))
    moved = np.linalg.norm(ref.theta_last - theta0)
    th_err = np.linalg.norm(to_np(res.theta_last).astype(np.float64) - ref.theta_last) / moved
    print(f"train loss rel {tl_err:.2e}, val loss rel {vl_err:.2e}, theta rel to displacement {th_err:.2e}, "
          f"val {np.round(res.val_loss, 5)} vs {np.round(ref.val_loss, 5)}, best {res.best_epoch}/{ref.best_epoch}")
    assert len(res.train_loss) == epochs * 3
    assert np.allclose(res.lr, ref.lr, rtol=1e-15, atol=0)
    # the first step sees theta0 on both sides: the FP32 loss bar
    assert abs(res.train_loss[0] - ref.train_loss[0]) <= 1e-5 * ref.train_loss[0]
    # measured 1e-6 (losses) and 5e-6 (parameters): FP32 gradients move Adam's steps only slightly
    assert tl_err <= 2e-5 and vl_err <= 2e-5
    assert th_err <= 1e-4
    # the saved epoch: the GPU's own first minimum, and the oracle's unless the two are within
    # the loss tolerance of each other
    assert res.best_epoch == int(np.argmin(res.val_loss))
    gap = np.sort(ref.val_loss)
    if gap[1] - gap[0] > 4e-5 * gap[0]:
        assert res.best_epoch == ref.best_epoch
    # the saved parameters reproduce the saved validation loss
    net.set_weights(res.theta_best)
    assert abs(tr.validation_loss() - res.best_val) <= 1e-6 * res.best_val


def test_loss_only_pass_matches_loss_with_gradient():
    from paper_2607_16906_amd import hz
    _, gtr, _, bd, _, _, _, _ = data(6, 1, 24, 4)
    theta = he_uniform(unet.init_shapes(unet.layer_specs(3, 8, 5)), rng_for(42, 2, 1))
    net = hz.Net(3, 8, 5, theta)
    for prec in ("fp32", "bf16"):
        l1, p1, g1 = hz.loss_backward(net, gtr, bd, prec=prec)
        l2, p2, g2 = hz.loss_backward(net, gtr, bd, prec=prec, need_grad=False)
        assert g2 is None
        assert torch.equal(l1, l2) and torch.equal(p1, p2)


def test_trainer_rejects_bad_arguments():
    from paper_2607_16906_amd import hz
    from paper_2607_16906_amd.train import Trainer
    _, gtr, _, bd, _, gva, _, vbd = data(4, 2, 24, 4)
    theta = he_uniform(unet.init_shapes(unet.layer_specs(2, 8, 5)), rng_for(42, 2, 2))
    net = hz.Net(2, 8, 5, theta)
    with pytest.raises(ValueError):
        Trainer(net, gtr, bd[:3], gva, vbd)                       # one residual short
    with pytest.raises(ValueError):
        Trainer(net, gtr, bd.to(torch.complex128), gva, vbd.to(torch.complex128))
    tr = Trainer(net, gtr, bd, gva, vbd, batch=3)
    with pytest.raises(ValueError):
        tr.fit(theta, [np.array([0, 1, 1, 3])])                   # not a permutation
    with pytest.raises(ValueError):
        tr.fit(theta[:-1], [np.arange(4)])


def test_full_size_epoch_sampled():
    # the production network (4 levels, 32 channels) on the paper's training grid size: 64^2
    # interior + 16 PML, batch 32 with a short second batch, BF16 and FP32
    from paper_2607_16906_amd import hz
    from paper_2607_16906_amd.train import Trainer
    nint, p, S, V = 64, 16, 40, 6
    otr, gtr, b, bd, ova, gva, vb, vbd = data(S, V, nint, p)
    w = np.load("paper_2607_16906_amd/weights/unet_l4_c32_in5.npz")
    theta0 = w["theta"].astype(np.float32)
    specs = unet.layer_specs(4, 32, 5)
    net = hz.Net(4, 32, 5, theta0)
    def oracle_loss(i, prec):
        # per-sample loss ||A N(r) - r|| / ||r|| of the oracle; for the BF16 path with BF16-rounded
        # weights and BF16 activation storage (the trained network's loss is small, so the
        # rounding noise of z, amplified by A, shows in it)
        r = vb[i].astype(np.complex128)
        if prec == "fp32":
            return otl.mean_loss(theta0.astype(np.float64), specs, [ova[i]], r[None], 1)
        z = unet.precond_apply(bf16_round(theta0), specs, ova[i], r, act_round=unet.bf16_activation)
        return np.linalg.norm(ohz.op_apply(ova[i], z) - r) / np.linalg.norm(r)

    for prec, tol in (("fp32", 1e-5), ("bf16", 1e-2)):
        ref = [oracle_loss(i, prec) for i in (0, V - 1)]
        net.set_weights(theta0)
        tr = Trainer(net, gtr, bd, gva, vbd, batch=32, prec=prec)
        tr.validation_loss()
        per = to_np(tr.per[:V])
        print(prec, "per-sample losses", per[[0, V - 1]], "oracle", ref)
        for k, i in enumerate((0, V - 1)):
            assert abs(per[i] - ref[k]) <= tol * ref[k], (prec, i, per[i], ref[k])
        order = epoch_order(S, 0)
        res = tr.fit(theta0, [order], lr0=1e-4, lr_min=1e-4)
        # the first step's loss is that of the first batch at theta0 (same kernels, loss-only pass)
        net.set_weights(theta0)
        idx = order[:32]
        l0, _, _ = hz.loss_backward(net, [gtr[i] for i in idx], bd[torch.from_numpy(idx).cuda()], prec=prec,
                                    need_grad=False)
        assert res.train_loss[0] == float(to_np(l0)[0])
        assert len(res.train_loss) == 2 and np.all(np.isfinite(res.train_loss))
        assert np.isfinite(res.val_loss[0]) and res.best_epoch == 0
        print(f"{prec}: step {res.step_ms:.2f} ms, validation pass {res.val_ms:.2f} ms, val {res.val_loss[0]:.4f}")
