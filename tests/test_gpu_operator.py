"""GPU parity of the Helmholtz stencil (hz_op_apply) against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import helmholtz as ohz
from synth import c1_system, c2_system, rng_for, skull_ring_velocity

from gpu_util import make_pair, rel, to_dev, to_np


def rand_field(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("nx,p", [(70, 8), (64, 8), (5, 3), (130, 20)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_stencil_fp64_matches_oracle(nx, p, adjoint):
    nt = nx + 2 * p
    c = skull_ring_velocity(nt, p, rng_for(11, 0, nx), rings=2)
    op, gp = make_pair(c, p)
    u = rand_field((nt, nt), nx)
    y = to_np(gp.apply(to_dev(u, torch.complex128), adjoint=adjoint)).reshape(nt, nt)
    ref = ohz.op_adjoint(op, u) if adjoint else ohz.op_apply(op, u)
    # FP64 step: 1e-10 relative (the two sides differ only in rounding order)
    assert rel(y, ref) <= 1e-13
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("adjoint", [False, True])
def test_stencil_fp32_within_1e5(adjoint):
    s = c2_system(0, nx=100, npml=20)
    op, gp = make_pair(s.c, s.npml)
    nt = s.nt
    # smooth and rough inputs
    for u in (rand_field((nt, nt), 3), s.b):
        y = to_np(gp.apply(to_dev(u, torch.complex64), adjoint=adjoint)).reshape(nt, nt)
        ref = ohz.op_adjoint(op, u) if adjoint else ohz.op_apply(op, u)
        assert rel(y, ref) <= 1e-5


def test_stencil_c2_full_size_sampled():
    # the 296 x 296 grid of the single-solve workload, in the precision the solver uses
    s = c2_system(0)
    op, gp = make_pair(s.c, s.npml)
    u = rand_field((s.nt, s.nt), 5)
    y = to_np(gp.apply(to_dev(u, torch.complex64))).reshape(s.nt, s.nt)
    ref = ohz.op_apply(op, u)
    assert rel(y, ref) <= 1e-5


def test_stencil_rejects_bad_args():
    from paper_2607_16906_amd import hz
    s = c1_system(0)
    _, gp = make_pair(s.c, s.npml)
    x = torch.zeros(gp.n, dtype=torch.complex64, device="cuda")
    lib = hz.load_library()
    assert lib.hz_op_apply(gp.handle, 7, 0, hz._ptr(x), hz._ptr(x), None) == hz.HZ_ERR_ARG
    assert b"dtype" in lib.hz_last_error()
    with pytest.raises(ValueError):
        hz.Problem(np.ones(10, np.float32), 4, 4, 1, 0.6)
    bad = np.full((s.nt, s.nt), 1500.0, np.float32)
    bad[3, 4] = -1.0
    with pytest.raises(hz.HzError) as e:
        hz.Problem(bad.ravel(), s.nx, s.nx, s.npml, 0.6)
    assert e.value.code == hz.HZ_ERR_NONFINITE
