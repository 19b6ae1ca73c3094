"""The C-ABI library loads on the CPU and exports every function include/hz.h declares
(no compute call is made: that needs a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hz.h")
LIB = os.path.join(ROOT, "paper_2607_16906_amd", "libhzno.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z][a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("hz_op_apply", "no_precond_apply", "no_loss_backward", "fgmres_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_covers_the_header():
    from paper_2607_16906_amd import hz
    lib = hz.load_library()
    for n in declared_functions():
        assert hasattr(lib, n)
        assert n in hz.SIGNATURES, n
    # a pure host query needs no GPU
    assert hz.param_count(4, 32, 5) == 1_926_210
    assert lib.hz_last_error() == b""


def test_param_counts_of_both_network_kinds_on_the_cpu():
    # no_param_count is host logic: it needs no GPU
    from paper_2607_16906_amd import hz
    from oracle import unet, unet8
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    assert hz.param_count(4, 32, 5) == unet.param_count(unet.layer_specs(4, 32, 5))
    assert hz.param_count(4, 32, 5, "paper8") == unet8.param_count(unet8.layer_specs(4, 32, 5))
    assert hz.param_count(3, 32, 2, "paper8") == unet8.param_count(unet8.layer_specs(3, 32, 2))
    for bad in ((4, 16, 5, "paper8"), (6, 32, 5, "paper8"), (7, 32, 5, "unet3"), (4, 12, 5, "unet3")):
        with pytest.raises(ValueError):
            hz.param_count(*bad)


def test_training_loop_schedule_matches_torch_scheduler():
    # the GPU loop's host-side schedule: torch's CosineAnnealingLR stepped once per epoch
    import torch
    from paper_2607_16906_amd.train import cosine_lr
    for epochs in (1, 2, 7, 500):
        p = torch.nn.Parameter(torch.zeros(1))
        opt = torch.optim.SGD([p], lr=1e-3)
        sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=max(epochs - 1, 1), eta_min=1e-5)
        for e in range(epochs):
            assert abs(opt.param_groups[0]["lr"] - cosine_lr(e, epochs)) <= 1e-15
            opt.step()
            sch.step()
