"""The allocation-free preconditioner entry point (no_precond_apply_noalloc) against the
workspace entry point (no_precond_apply) through the C ABI: bit-identical outputs on two calls in
a row, the second on a smaller grid (the scratch keeps the first call's contents), the FP32 and
BF16 forms, and a clear error for a grid whose scratch need exceeds the fixed size."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from synth import c2_system, gaussian_sources, rng_for, skull_ring_velocity

from gpu_util import make_pair, to_dev

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2607_16906_amd", "weights", "unet_l4_c32_in5.npz")


def _input(b, nt, seed):
    v = b.reshape(nt, nt) + 0.05 * np.random.default_rng(seed).standard_normal((nt, nt))
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("prec,dtype", [("bf16", torch.complex64), ("fp32", torch.complex64),
                                        ("bf16", torch.complex128)])
def test_noalloc_matches_workspace_entry(prec, dtype):
    from paper_2607_16906_amd import hz
    theta = np.load(WEIGHTS)["theta"].astype(np.float32)
    net = hz.Net(4, 32, 5, theta)
    big = c2_system(0)                                  # 296^2 nodes: the single-solve grid
    nts = 20
    small_c = skull_ring_velocity(nts, 4, rng_for(21, 0, 0), rings=1)
    small_b = gaussian_sources(nts, 4, rng_for(21, 1, 0))
    cases = [(big.c, big.npml, big.b, big.nt), (small_c, 4, small_b, nts)]
    for k, (c, p, b, nt) in enumerate(cases):
        _, gp = make_pair(c, p)
        v = to_dev(_input(b, nt, k), dtype)
        ref = net.apply(gp, v, prec=prec)
        z = torch.full_like(v, float("nan"))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        net.apply_noalloc(gp, v, z, prec=prec)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        print(f"{prec} {dtype} grid {nt}^2: max |diff| {(z - ref).abs().max().item():.3e}")
        assert torch.equal(z, ref), (prec, nt)


def test_noalloc_rejects_oversize_scratch():
    from paper_2607_16906_amd import hz
    theta = np.load(WEIGHTS)["theta"].astype(np.float32)
    net = hz.Net(4, 32, 5, theta)
    s = c2_system(0)
    _, gp = make_pair(s.c, s.npml)
    v = to_dev(_input(s.b, s.nt, 0), torch.complex128)
    z = torch.zeros_like(v)
    # the FP64 network at 296^2 needs about 180 MB of scratch, more than the fixed 128 MiB
    need = hz.load_library().no_workspace_size(net.handle, gp.handle, hz.NO_FP64)
    assert need > 128 << 20
    with pytest.raises(hz.HzError) as e:
        net.apply_noalloc(gp, v, z, prec="fp64")
    assert e.value.code == hz.HZ_ERR_WORKSPACE and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(z).item() == 0          # nothing was launched
