"""Thin ctypes binding of the gfx950 library (include/hz.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels. PyTorch supplies device memory (torch tensors on ``cuda``) and the
current HIP stream. The library is loaded from the package directory; when it
is missing, or when no GPU is visible, every entry point raises.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhzno.so")

HZ_OK, HZ_NOT_CONVERGED = 0, 1
HZ_ERR_ARG, HZ_ERR_HIP, HZ_ERR_WORKSPACE, HZ_ERR_BREAKDOWN, HZ_ERR_NONFINITE = -1, -2, -3, -4, -5
HZ_C64, HZ_C128 = 0, 1
NO_BF16, NO_FP32, NO_FP64 = 0, 1, 2
PREC = {"bf16": NO_BF16, "fp32": NO_FP32, "fp64": NO_FP64}


class HzGrid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("npml", ct.c_int32),
                ("h", ct.c_double), ("omega", ct.c_double), ("sigma_max", ct.c_double), ("c_ref", ct.c_double),
                ("disc", ct.c_int32)]


class NoArch(ct.Structure):
    _fields_ = [("levels", ct.c_int32), ("base", ct.c_int32), ("in_ch", ct.c_int32), ("kind", ct.c_int32)]


class HzOpts(ct.Structure):
    _fields_ = [("m", ct.c_int32), ("maxit", ct.c_int32), ("tol", ct.c_double), ("krylov", ct.c_int),
                ("net_prec", ct.c_int), ("hist_host", ct.POINTER(ct.c_double)), ("hist_len", ct.c_int32),
                ("ortho", ct.c_int32)]


HZ_NPHASE = 4
PHASES = ("setup", "cycles", "build", "total")   # HZ_PHASE_* order


class HzInfo(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("its", ct.c_int32), ("cycles", ct.c_int32),
                ("est_relres", ct.c_double), ("true_relres", ct.c_double),
                ("phase_ms", ct.c_double * HZ_NPHASE)]


_P, _I, _SZ, _F = ct.c_void_p, ct.c_int, ct.c_size_t, ct.c_float
# name -> (restype, argtypes); the declarations of include/hz.h
SIGNATURES = {
    "hz_last_error": (ct.c_char_p, []),
    "hz_problem_create": (_I, [ct.POINTER(HzGrid), _P, _P, ct.POINTER(_P)]),
    "hz_problem_destroy": (_I, [_P]),
    "hz_problem_dims": (_I, [_P, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]),
    "hz_op_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "no_param_count": (ct.c_int64, [ct.POINTER(NoArch)]),
    "no_net_create": (_I, [ct.POINTER(NoArch), _P, _P, ct.POINTER(_P)]),
    "no_net_set_weights": (_I, [_P, _P, _P]),
    "no_net_destroy": (_I, [_P]),
    "no_workspace_size": (_SZ, [_P, _P, _I]),
    "no_precond_apply": (_I, [_P, _P, _I, _I, _P, _P, _P, _SZ, _P]),
    "no_precond_apply_noalloc": (_I, [_P, _P, _I, _I, _P, _P, _P]),
    "no_autotune": (_I, [_P, _P, _I, _P, _SZ, _P]),
    "no_layer_variant": (_I, [_P, _I, _I, _I, _I, _I, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                              ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]),
    "no_set_layer_variant": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _I]),
    "no_set_fused_upsampling": (_I, [_P, _I]),
    "no_layer_info": (_I, [_P, _I, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                           ct.POINTER(ct.c_int32)]),
    "no_layer_forward": (_I, [_P, _I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _SZ, _P]),
    "no_train_workspace_size": (_SZ, [_P, _P, _I, _I, _I]),
    "no_loss_backward": (_I, [_P, _I, _P, _P, _I, _I, _I, _P, _P, _P, _P, _SZ, _P]),
    "no_adam_workspace_size": (_SZ, [_P]),
    "no_adam_step": (_I, [_P, _P, _P, _P, _P, _I, _F, _F, _F, _F, _F, _P, _SZ, _P]),
    "fgmres_workspace_size": (_SZ, [_P, _P, ct.POINTER(HzOpts)]),
    "fgmres_solve": (_I, [_P, _P, ct.POINTER(HzOpts), _P, _P, _P, _SZ, ct.POINTER(HzInfo), _P]),
    "fgmres_batched_workspace_size": (_SZ, [_I, _P, _P, ct.POINTER(HzOpts)]),
    "fgmres_solve_batched": (_I, [_I, _P, _P, ct.POINTER(HzOpts), _P, _P, _P, _SZ, ct.POINTER(HzInfo), _P]),
}

_lib = None


class HzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load libhzno.so (no GPU needed to load it). Raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: run python -m paper_2607_16906_amd.build")
        lib = ct.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a visible GPU")
    return torch


def _stream():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ct.c_void_p(t.data_ptr())


def _check(rc, what):
    if rc < 0:
        raise HzError(rc, f"{what}: {load_library().hz_last_error().decode()}")
    return rc


def _ws(nbytes):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Problem:
    """One discrete Helmholtz system on the GPU (hz_problem_create)."""

    DISC = {"fd": 0, "spectral": 1}

    def __init__(self, c, nx: int, ny: int, npml: int, h: float, omega: float = 1.0,
                 sigma_max: float = 2.0, c_ref: float = 1500.0, disc: str = "fd"):
        """disc: "fd" (five-point finite differences) or "spectral" (Fourier differentiation)."""
        torch = _torch()
        lib = load_library()
        c = torch.as_tensor(c, dtype=torch.float32).to("cuda").contiguous()
        nxt, nyt = nx + 2 * npml, ny + 2 * npml
        if c.numel() != nxt * nyt:
            raise ValueError(f"velocity has {c.numel()} entries, grid needs {nxt * nyt}")
        self.grid = HzGrid(nx, ny, npml, h, omega, sigma_max, c_ref, self.DISC[disc])
        self.c = c
        self.nx, self.ny, self.npml = nx, ny, npml
        self.nxt, self.nyt, self.n = nxt, nyt, nxt * nyt
        h_ = ct.c_void_p()
        _check(lib.hz_problem_create(ct.byref(self.grid), _ptr(c), _stream(), ct.byref(h_)), "hz_problem_create")
        self.handle = h_

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.hz_problem_destroy(h)
            self.handle = None

    def apply(self, x, adjoint: bool = False):
        """y = A x (or A^H x) for a complex64/complex128 device vector of n entries."""
        torch = _torch()
        x = x.contiguous()
        dt = {torch.complex64: HZ_C64, torch.complex128: HZ_C128}[x.dtype]
        y = torch.empty_like(x)
        _check(load_library().hz_op_apply(self.handle, dt, int(adjoint), _ptr(x), _ptr(y), _stream()), "hz_op_apply")
        return y


class Net:
    """U-Net neural operator (no_net_create) holding its own repacked copies of theta."""

    KIND = {"unet3": 0, "paper8": 1}

    def __init__(self, levels: int, base: int, in_ch: int, theta, kind: str = "unet3"):
        """kind: "unet3" (3x3 / ReLU / doubling channels) or "paper8" (Table 2's 8x8 stride-2
        layers with PReLU; levels = depth, base = 32)."""
        torch = _torch()
        lib = load_library()
        self.arch = NoArch(levels, base, in_ch, self.KIND[kind])
        self.kind = kind
        self.nparam = param_count(levels, base, in_ch, kind)
        theta = torch.as_tensor(theta, dtype=torch.float32).to("cuda").contiguous()
        if theta.numel() != self.nparam:
            raise ValueError(f"theta has {theta.numel()} entries, the network needs {self.nparam}")
        self.theta = theta
        h_ = ct.c_void_p()
        _check(lib.no_net_create(ct.byref(self.arch), _ptr(theta), _stream(), ct.byref(h_)), "no_net_create")
        self.handle = h_

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.no_net_destroy(h)
            self.handle = None

    def set_weights(self, theta):
        torch = _torch()
        theta = torch.as_tensor(theta, dtype=torch.float32).to("cuda").contiguous()
        self.theta = theta
        _check(load_library().no_net_set_weights(self.handle, _ptr(theta), _stream()), "no_net_set_weights")

    def apply(self, problem: Problem, v, prec: str = "bf16"):
        """z = N(v, c, sigma) (no_precond_apply)."""
        torch = _torch()
        lib = load_library()
        v = v.contiguous()
        dt = {torch.complex64: HZ_C64, torch.complex128: HZ_C128}[v.dtype]
        z = torch.empty_like(v)
        nb = lib.no_workspace_size(self.handle, problem.handle, PREC[prec])
        ws = _ws(nb)
        _check(lib.no_precond_apply(self.handle, problem.handle, PREC[prec], dt, _ptr(v), _ptr(z), _ptr(ws),
                                    ct.c_size_t(ws.numel()), _stream()), "no_precond_apply")
        return z
    def apply_noalloc(self, problem: Problem, v, z, prec: str = "bf16"):
        """z = N(v, c, sigma) into the caller's z with the library's fixed scratch
        (no_precond_apply_noalloc): no device memory is allocated by this call."""
        torch = _torch()
        if not (v.is_contiguous() and z.is_contiguous()) or v.dtype != z.dtype or v.numel() != z.numel():
            raise ValueError("v and z must be contiguous device vectors of one complex type and size")
        dt = {torch.complex64: HZ_C64, torch.complex128: HZ_C128}[v.dtype]
        _check(load_library().no_precond_apply_noalloc(self.handle, problem.handle, PREC[prec], dt, _ptr(v), _ptr(z),
                                                       _stream()), "no_precond_apply_noalloc")
        return z

    def autotune(self, problem: Problem, prec: str = "bf16"):
        """Pick the fastest launch variant of every 3x3 layer at this problem's size (no_autotune)."""
        lib = load_library()
        ws = _ws(lib.no_workspace_size(self.handle, problem.handle, PREC[prec]))
        _check(lib.no_autotune(self.handle, problem.handle, PREC[prec], _ptr(ws), ct.c_size_t(ws.numel()), _stream()),
               "no_autotune")

    def layer_variant(self, layer: int, H: int, W: int, prec: str = "bf16", batch: int = 1):
        """(tn, rows, stages, tiles) launch variant of a 3x3 layer at this size (no_layer_variant)."""
        tn, rows, st, tl = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(load_library().no_layer_variant(self.handle, layer, PREC[prec], batch, H, W, ct.byref(tn),
                                               ct.byref(rows), ct.byref(st), ct.byref(tl)), "no_layer_variant")
        return tn.value, rows.value, st.value, tl.value

    def set_layer_variant(self, layer: int, H: int, W: int, tn: int, rows: int, stages: int = 1, tiles: int = 1,
                          prec: str = "bf16", batch: int = 1):
        """Pin the launch variant of a 3x3 layer at this size (no_set_layer_variant)."""
        _check(load_library().no_set_layer_variant(self.handle, layer, PREC[prec], batch, H, W, tn, rows, stages,
                                                   tiles), "no_set_layer_variant")

    def set_fused_upsampling(self, mode: int):
        """BF16 decoder: transposed convolution inside the next 3x3 layer: 0 never, 1 always,
        2 where autotuned faster (the default); the same result bits (no_set_fused_upsampling)."""
        _check(load_library().no_set_fused_upsampling(self.handle, int(mode)), "no_set_fused_upsampling")

    def layer_info(self, layer: int):
        """(kind, cin_p, cout_p, cat_cp) of one layer (no_layer_info)."""
        v = [ct.c_int32() for _ in range(4)]
        _check(load_library().no_layer_info(self.handle, layer, *[ct.byref(x) for x in v]), "no_layer_info")
        return tuple(x.value for x in v)

    def layer_forward(self, layer: int, x0, y, *, H: int, W: int, batch: int = 1, x1=None, pool=None,
                      prec: str = "bf16", workspace=None):
        """Run one layer on NHWC device tensors (no_layer_forward); asynchronous on the current stream."""
        ws = _ptr(workspace) if workspace is not None else None
        nb = ct.c_size_t(workspace.numel() if workspace is not None else 0)
        _check(load_library().no_layer_forward(self.handle, layer, PREC[prec], batch, H, W, _ptr(x0),
                                               _ptr(x1) if x1 is not None else None, _ptr(y),
                                               _ptr(pool) if pool is not None else None, ws, nb, _stream()),
               "no_layer_forward")


def init_shapes_paper8(depth: int, ch: int, in_ch: int):
    """(weight shape, fan-in, bias length) of every layer of the NO_ARCH_PAPER8 network in the flat
    parameter order of hz.h; each layer but the head is followed by one PReLU slope."""
    out = [((ch, in_ch, 8, 8), 64 * in_ch, ch)] + [((ch, ch, 8, 8), 64 * ch, ch)] * (depth - 1)
    out += [((ch, ch, 8, 8), 16 * ch, ch)] + [((2 * ch, ch, 8, 8), 32 * ch, ch)] * (depth - 1)
    return out + [((2, ch, 1, 1), ch, 2)]


def init_shapes(levels: int, base: int, in_ch: int):
    """(weight shape, fan-in, bias length) of every layer in the flat parameter order of hz.h
    (input for a seeded initialiser)."""
    out, cin = [], in_ch
    for l in range(levels):
        c = base << l
        out.append(((c, cin, 3, 3), 9 * cin, c))
        out.append(((c, c, 3, 3), 9 * c, c))
        cin = c
    for l in range(levels - 2, -1, -1):
        c = base << l
        out.append(((2 * c, c, 2, 2), 2 * c, c))
        out.append(((c, 2 * c, 3, 3), 18 * c, c))
        out.append(((c, c, 3, 3), 9 * c, c))
    out.append(((2, base, 1, 1), base, 2))
    return out


def param_count(levels: int, base: int, in_ch: int, kind: str = "unet3") -> int:
    n = load_library().no_param_count(ct.byref(NoArch(levels, base, in_ch, Net.KIND[kind])))
    if n < 0:
        raise ValueError("unsupported architecture")
    return int(n)


def loss_backward(net: Net, problems, r, *, squared: bool = False, prec: str = "bf16", workspace=None,
                  recompute: bool = False, need_grad: bool = True):
    """Physics-informed loss and its parameter gradient (no_loss_backward).

    problems: list of B Problems of one grid size; r: [B, n] complex64 device tensor.
    recompute: checkpoint activations (smaller workspace, bit-identical results).
    need_grad: False evaluates the loss alone (no reverse pass; grad is None).
    Returns (loss [1] float32, per-sample losses [B] float32, grad [nparam] float32).
    """
    torch = _torch()
    lib = load_library()
    B = len(problems)
    r = r.to(torch.complex64).contiguous()
    if r.numel() != B * problems[0].n:
        raise ValueError("r must hold batch x n entries")
    ptrs = (ct.c_void_p * B)(*[p.handle for p in problems])
    nb = lib.no_train_workspace_size(net.handle, problems[0].handle, B, PREC[prec], int(recompute))
    ws = workspace if workspace is not None and workspace.numel() >= nb else _ws(nb)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    per = torch.empty(B, dtype=torch.float32, device="cuda")
    grad = torch.empty(net.nparam, dtype=torch.float32, device="cuda") if need_grad else None
    _check(lib.no_loss_backward(net.handle, B, ptrs, _ptr(r), int(squared), int(recompute), PREC[prec],
                                _ptr(loss), _ptr(per), _ptr(grad) if need_grad else None, _ptr(ws),
                                ct.c_size_t(ws.numel()), _stream()),
           "no_loss_backward")
    return loss, per, grad


def train_workspace_bytes(net: Net, problem: Problem, batch: int, prec: str = "bf16",
                          recompute: bool = False) -> int:
    return int(load_library().no_train_workspace_size(net.handle, problem.handle, batch, PREC[prec],
                                                      int(recompute)))


def adam_step(net: Net, theta, m, v, grad, step: int, *, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, clip: float = 1.0):
    """One Adam step on the float32 master parameters in place; refreshes the network (no_adam_step)."""
    lib = load_library()
    ws = _ws(lib.no_adam_workspace_size(net.handle))
    _check(lib.no_adam_step(net.handle, _ptr(theta), _ptr(m), _ptr(v), _ptr(grad), int(step), lr, beta1, beta2, eps,
                            clip, _ptr(ws), ct.c_size_t(ws.numel()), _stream()), "no_adam_step")
    net.theta = theta


def _loss_function():
    torch = _torch()

    class NoLoss(torch.autograd.Function):
        """loss = mean_b ||A_b N_theta(r_b) - r_b|| / ||r_b|| with the library's hand-written reverse mode."""

        @staticmethod
        def forward(ctx, theta, net, problems, r, squared, prec, recompute):
            net.set_weights(theta.detach())
            loss, _, grad = loss_backward(net, problems, r, squared=squared, prec=prec, recompute=recompute)
            ctx.save_for_backward(grad)
            return loss[0]

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout * grad, None, None, None, None, None, None

    return NoLoss


def physics_loss(theta, net: Net, problems, r, squared: bool = False, prec: str = "bf16", recompute: bool = False):
    """Differentiable (w.r.t. theta) physics-informed loss, through torch.autograd."""
    return _loss_function().apply(theta, net, problems, r, squared, prec, recompute)


@dataclass
class SolveInfo:
    status: int
    its: int
    cycles: int
    est_relres: float
    true_relres: float
    hist: np.ndarray
    phase_ms: dict = None   # {"setup", "cycles", "build", "total"} in milliseconds


def _phases(info) -> dict:
    return {k: float(info.phase_ms[i]) for i, k in enumerate(PHASES)}


ORTHO = {"cgs2": 0, "dcgs2": 1}


def fgmres(problem: Problem, b, x0=None, *, net: Net | None = None, m: int = 30, tol: float = 1e-6,
           maxit: int = 300, krylov: str = "c64", net_prec: str = "bf16", workspace=None, ortho: str = "cgs2",
           out=None):
    """Solve A x = b (fgmres_solve). b: complex128 device vector; returns (x, SolveInfo).

    ortho: "cgs2" (classical Gram-Schmidt with one reorthogonalisation) or "dcgs2" (delayed
    reorthogonalisation, one reduction per step; needs a network).
    out: optional complex128 device vector of n entries that receives x (x0, or 0, is written into
    it first); repeated solves with the same b, out and workspace replay the library's kept cycle
    graphs."""
    torch = _torch()
    lib = load_library()
    b = b.to(torch.complex128).contiguous()
    if out is not None:
        if out.dtype != torch.complex128 or out.numel() != b.numel() or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must be a contiguous complex128 device vector of n entries")
        x = out
        if x0 is None:
            x.zero_()
        else:
            x.copy_(x0.reshape(x.shape))
    else:
        x = torch.zeros_like(b) if x0 is None else x0.to(torch.complex128).contiguous().clone()
    hist = np.zeros(maxit, np.float64)
    opts = HzOpts(m, maxit, tol, HZ_C64 if krylov == "c64" else HZ_C128, PREC[net_prec],
                  hist.ctypes.data_as(ct.POINTER(ct.c_double)), maxit, ORTHO[ortho])
    nh = net.handle if net is not None else None
    nb = lib.fgmres_workspace_size(problem.handle, nh, ct.byref(opts))
    if nb == 0:
        raise HzError(HZ_ERR_ARG, lib.hz_last_error().decode())
    ws = workspace if workspace is not None and workspace.numel() >= nb else _ws(nb)
    info = HzInfo()
    rc = lib.fgmres_solve(problem.handle, nh, ct.byref(opts), _ptr(b), _ptr(x), _ptr(ws), ct.c_size_t(ws.numel()),
                          ct.byref(info), _stream())
    if rc in (HZ_ERR_ARG, HZ_ERR_HIP, HZ_ERR_WORKSPACE):
        _check(rc, "fgmres_solve")
    return x, SolveInfo(info.status, info.its, info.cycles, info.est_relres, info.true_relres, hist[:info.its].copy(),
                        _phases(info))


def fgmres_batched(problems, bs, x0s=None, *, net: Net | None = None, m: int = 30, tol: float = 1e-6,
                   maxit: int = 300, krylov: str = "c64", net_prec: str = "bf16", workspace=None):
    """Solve many systems together (fgmres_solve_batched). bs: list of complex128 device vectors.

    Returns (list of x, list of SolveInfo without histories)."""
    torch = _torch()
    lib = load_library()
    nsys = len(problems)
    bs = [b.to(torch.complex128).contiguous() for b in bs]
    xs = [torch.zeros_like(b) if x0s is None else x0s[i].to(torch.complex128).contiguous().clone()
          for i, b in enumerate(bs)]
    opts = HzOpts(m, maxit, tol, HZ_C64 if krylov == "c64" else HZ_C128, PREC[net_prec], None, 0)
    probs = (ct.c_void_p * nsys)(*[p.handle for p in problems])
    nh = net.handle if net is not None else None
    nb = lib.fgmres_batched_workspace_size(nsys, probs, nh, ct.byref(opts))
    if nb == 0:
        raise HzError(HZ_ERR_ARG, lib.hz_last_error().decode())
    ws = workspace if workspace is not None and workspace.numel() >= nb else _ws(nb)
    bp = (ct.c_void_p * nsys)(*[b.data_ptr() for b in bs])
    xp = (ct.c_void_p * nsys)(*[x.data_ptr() for x in xs])
    infos = (HzInfo * nsys)()
    rc = lib.fgmres_solve_batched(nsys, probs, nh, ct.byref(opts), bp, xp, _ptr(ws), ct.c_size_t(ws.numel()), infos,
                                  _stream())
    if rc in (HZ_ERR_ARG, HZ_ERR_HIP, HZ_ERR_WORKSPACE):
        _check(rc, "fgmres_solve_batched")
    return xs, [SolveInfo(i.status, i.its, i.cycles, i.est_relres, i.true_relres, np.zeros(0), _phases(i))
                for i in infos]


def fgmres_batched_workspace_bytes(problems, net: Net | None, m: int, maxit: int, krylov: str = "c64",
                                   net_prec: str = "bf16") -> int:
    opts = HzOpts(m, maxit, 1e-6, HZ_C64 if krylov == "c64" else HZ_C128, PREC[net_prec], None, 0)
    probs = (ct.c_void_p * len(problems))(*[p.handle for p in problems])
    return int(load_library().fgmres_batched_workspace_size(len(problems), probs, net.handle if net else None,
                                                            ct.byref(opts)))


def fgmres_workspace_bytes(problem: Problem, net: Net | None, m: int, maxit: int, krylov: str = "c64",
                           net_prec: str = "bf16", ortho: str = "cgs2") -> int:
    opts = HzOpts(m, maxit, 1e-6, HZ_C64 if krylov == "c64" else HZ_C128, PREC[net_prec], None, 0, ORTHO[ortho])
    return int(load_library().fgmres_workspace_size(problem.handle, net.handle if net else None, ct.byref(opts)))
