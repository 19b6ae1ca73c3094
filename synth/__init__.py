"""Seeded synthetic inputs for the neural-operator-preconditioned Helmholtz solver.

This module is the only code shared by the CPU oracle and the GPU path. It
produces *inputs* only (velocity fields, source fields, training residuals,
network parameters, grid sizes) and holds none of the method's arithmetic:
no operator, no PML profile, no network, no Krylov step.

Units follow the paper's nondimensional setting (angular frequency 1,
velocities of order 1 after dividing by a reference speed, Section 2.1):
velocities are returned in m/s and the library divides by ``C_REF``.

Every generator draws from ``numpy.random.default_rng(SeedSequence([42, cfg,
comp, sys]))``; 42 is the paper's training seed (Table 3), ``cfg`` names the
workload, ``comp`` the component (``COMP_*``) and ``sys`` the system index.

Workloads stand in for the paper's datasets (idealized skulls and head-CT
slices, Sections 3.2 and 4.2): elliptical skull rings of fast bone-like
material on a water-like background, with point or Gaussian sources.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C_REF = 1500.0          # background speed of sound (m/s); c / C_REF is the nondimensional velocity
H_10PPW = 2.0 * math.pi / 10.0   # grid step giving 10 points per wavelength at c = C_REF, omega = 1

COMP_VELOCITY = 0
COMP_SOURCE = 1
COMP_WEIGHTS = 2
COMP_RESIDUAL = 3
COMP_SIZES = 4
COMP_ORDER = 7          # the per-epoch visiting order of a fixed training set

CFG_C1, CFG_C2, CFG_C3, CFG_C4, CFG_C5 = 1, 2, 3, 4, 5
CFG_APPB = 8            # the second synthetic workload (simplified spherical-wave and seismic settings)
CFG_TRAIN = 9           # epoch-based training on a fixed data set (Section 3.4)
CFG_TABLE4 = 10         # the six training data sets D0-D5 of Section 3.2 (Table 4)
VAL_FIRST = 10_000_000  # first stream index of validation samples (disjoint from training ones)


def rng_for(cfg: int, comp: int, sys: int = 0) -> np.random.Generator:
    """Counter-style seeding: one independent stream per (workload, component, system)."""
    return np.random.default_rng(np.random.SeedSequence([42, int(cfg), int(comp), int(sys)]))


# --------------------------------------------------------------------------- velocity fields

def skull_ring_velocity(nt: int, npml: int, rng: np.random.Generator, *, rings: int,
                        ring_speed=None, thickness: float = 4.0, noise: float = 0.05,
                        background: float = C_REF) -> np.ndarray:
    """Elliptical skull-like rings on a water background, with multiplicative noise.

    Returns c in m/s, float64 array [nt, nt] (row = y, column = x).
    Each ring: centre uniform in the central half of the interior, semi-axis
    a ~ U[0.25, 0.40] * N_int cells, b ~ U[0.6, 1.0] * a, angle ~ U[0, pi).
    A node is bone iff it lies inside the ellipse with semi-axes (a + t/2,
    b + t/2) and outside the one with semi-axes (a - t/2, b - t/2).
    Overlapping rings take the larger speed. ``ring_speed`` is a fixed speed or
    None for U[2500, 3000] m/s per ring. Finally c <- c * (1 + noise * xi),
    xi ~ N(0, 1) i.i.d. on every node (PML included).
    """
    nint = nt - 2 * npml
    c = np.full((nt, nt), float(background))
    jj, ii = np.meshgrid(np.arange(nt, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
    for _ in range(rings):
        cx = npml + nint * rng.uniform(0.25, 0.75)
        cy = npml + nint * rng.uniform(0.25, 0.75)
        a = rng.uniform(0.25, 0.40) * nint
        b = rng.uniform(0.6, 1.0) * a
        th = rng.uniform(0.0, math.pi)
        val = float(ring_speed) if ring_speed is not None else rng.uniform(2500.0, 3000.0)
        dx, dy = ii - cx, jj - cy
        u = dx * math.cos(th) + dy * math.sin(th)
        v = -dx * math.sin(th) + dy * math.cos(th)
        ao, bo = a + thickness / 2, b + thickness / 2
        ai, bi = max(a - thickness / 2, 1e-9), max(b - thickness / 2, 1e-9)
        outer = (u / ao) ** 2 + (v / bo) ** 2 <= 1.0
        inner = (u / ai) ** 2 + (v / bi) ** 2 < 1.0
        ring = outer & ~inner
        c = np.where(ring, np.maximum(c, val), c)
    c = c * (1.0 + noise * rng.standard_normal((nt, nt)))
    return c


def uniform_velocity(nt: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. nondimensional velocity U[1, 2] per node (paper's U([1,2]) class), in m/s."""
    return C_REF * rng.uniform(1.0, 2.0, (nt, nt))


def rand_constant_velocity(nt: int, rng: np.random.Generator) -> np.ndarray:
    """One constant nondimensional velocity U[1, 2] on every node (paper's randConstant)."""
    return np.full((nt, nt), C_REF * rng.uniform(1.0, 2.0))


def square_velocity(nt: int) -> np.ndarray:
    """Centred square at nondimensional speed 2 on background 1 (paper's square class).

    The square's side is half the grid.
    """
    c = np.full((nt, nt), C_REF)
    q = nt // 4
    c[q:nt - q, q:nt - q] = 2.0 * C_REF
    return c


def layered_velocity(nt: int, rng: np.random.Generator, *, layers: int = 4, faulted: bool = False,
                     lo: float = 1.0, hi: float = 2.0) -> np.ndarray:
    """Aligned horizontal layers over the whole grid, each at one nondimensional speed U[lo, hi]
    (the 4layered class of the paper's second synthetic workload); m/s.

    The layer boundaries are depths j drawn without repetition from [nt/8, 7 nt/8), at least
    nt/(4 layers) apart. faulted (4faulted): a vertical fault at column xf ~ U{nt/4 .. 3nt/4}; to
    its right every boundary is shifted down by s ~ U{nt/16 .. nt/8} rows (clipped to the grid)."""
    gap = max(1, nt // (4 * layers))
    while True:
        cuts = np.sort(rng.choice(np.arange(nt // 8, nt - nt // 8), size=layers - 1, replace=False))
        if np.all(np.diff(np.concatenate([[0], cuts, [nt]])) >= gap):
            break
    vals = C_REF * rng.uniform(lo, hi, layers)
    jj = np.arange(nt)[:, None]
    c = np.empty((nt, nt))
    if faulted:
        xf = int(rng.integers(nt // 4, 3 * nt // 4 + 1))
        sh = int(rng.integers(max(1, nt // 16), max(2, nt // 8) + 1))
        left = np.searchsorted(cuts, np.arange(nt), side="right")
        right = np.searchsorted(np.minimum(cuts + sh, nt), np.arange(nt), side="right")
        c[:, :xf] = vals[left][:, None]
        c[:, xf:] = vals[right][:, None]
    else:
        c[:] = vals[np.searchsorted(cuts, jj[:, 0], side="right")][:, None]
    return c


# --------------------------------------------------------------------------- sources

def _interior_node(nt: int, npml: int, rng: np.random.Generator, margin: int = 4):
    lo, hi = npml + margin, nt - 1 - npml - margin
    return int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))


def point_source(nt: int, npml: int, rng: np.random.Generator, amplitude: complex = 1.0) -> np.ndarray:
    """One point source at a random interior node at least 4 cells from the PML. complex128 [nt, nt]."""
    b = np.zeros((nt, nt), np.complex128)
    i, j = _interior_node(nt, npml, rng)
    b[j, i] = amplitude
    return b


def gaussian_sources(nt: int, npml: int, rng: np.random.Generator, *, nsrc=None,
                     width: float = 1.5) -> np.ndarray:
    """n_src ~ U{1..4} Gaussian blobs exp(-r^2 / (2 width^2)) (width in cells) with complex
    amplitudes rho * exp(i phi), rho ~ U[0.5, 1.5], phi ~ U[0, 2 pi). Centres are integer
    interior nodes at least 4 cells from the PML. complex128 [nt, nt]."""
    if nsrc is None:
        nsrc = int(rng.integers(1, 5))
    jj, ii = np.meshgrid(np.arange(nt, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
    b = np.zeros((nt, nt), np.complex128)
    for _ in range(nsrc):
        i, j = _interior_node(nt, npml, rng)
        amp = rng.uniform(0.5, 1.5) * np.exp(1j * rng.uniform(0.0, 2 * math.pi))
        b += amp * np.exp(-((ii - i) ** 2 + (jj - j) ** 2) / (2.0 * width * width))
    return b


def m_dirac_source(nt: int, npml: int, rng: np.random.Generator, m: int) -> np.ndarray:
    """m entries set to +1 or -1 (equally likely) at distinct random interior nodes at least 4
    cells from the PML, zero elsewhere (the paper's m-dirac class). complex128 [nt, nt]."""
    b = np.zeros((nt, nt), np.complex128)
    placed = 0
    while placed < m:
        i, j = _interior_node(nt, npml, rng)
        if b[j, i] != 0:
            continue
        b[j, i] = 1.0 if rng.uniform() < 0.5 else -1.0
        placed += 1
    return b


def box_smoothed_noise(nt: int, rng: np.random.Generator, box: int = 5) -> np.ndarray:
    """Complex Gaussian noise xi_re + i xi_im smoothed by a box x box mean with zero padding."""
    z = rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt))
    hw = box // 2
    zp = np.zeros((nt + 2 * hw, nt + 2 * hw), np.complex128)
    zp[hw:hw + nt, hw:hw + nt] = z
    out = np.zeros((nt, nt), np.complex128)
    for dj in range(box):
        for di in range(box):
            out += zp[dj:dj + nt, di:di + nt]
    return out / float(box * box)


def normal_source(nt: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. N(0,1) real and imaginary parts (paper's N(0,1) source class)."""
    return rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt))


def dirac_source(nt: int, rng: np.random.Generator, *, centred: bool = False, value: float = 60.0) -> np.ndarray:
    """Single spike of the given value (paper's dirac / dirac1 classes)."""
    b = np.zeros((nt, nt), np.complex128)
    if centred:
        b[nt // 2, nt // 2] = value
    else:
        b[int(rng.integers(0, nt)), int(rng.integers(0, nt))] = value
    return b


def dirac4_source(nt: int, value: float = 30.0) -> np.ndarray:
    """Four spikes at fixed nodes (quarter points of the grid), paper's dirac4 class."""
    b = np.zeros((nt, nt), np.complex128)
    for j in (nt // 4, 3 * nt // 4):
        for i in (nt // 4, 3 * nt // 4):
            b[j, i] = value
    return b


# --------------------------------------------------------------------------- network parameters

def he_uniform(shapes, rng: np.random.Generator) -> np.ndarray:
    """Flat float32 parameter vector from a list of (weight_shape, fan_in, bias_len).

    Weights ~ U[-sqrt(6/fan_in), sqrt(6/fan_in)], biases ~ U[-1/sqrt(fan_in), 1/sqrt(fan_in)];
    each layer contributes its weights (C order) followed by its bias.
    """
    parts = []
    for wshape, fan_in, blen in shapes:
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, int(np.prod(wshape))))
        blim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-blim, blim, int(blen)))
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------- workloads

@dataclass
class System:
    nx: int          # interior cells along x
    npml: int        # PML cells on each side
    c: np.ndarray    # velocity (m/s), float64 [nt, nt]
    b: np.ndarray    # source, complex128 [nt, nt]

    @property
    def nt(self) -> int:
        return self.nx + 2 * self.npml


def c1_system(sys: int = 0) -> System:
    """64^2 interior + 8 PML; one 2800 m/s ring, 5% noise; one unit point source."""
    nx, p = 64, 8
    c = skull_ring_velocity(nx + 2 * p, p, rng_for(CFG_C1, COMP_VELOCITY, sys), rings=1, ring_speed=2800.0)
    b = point_source(nx + 2 * p, p, rng_for(CFG_C1, COMP_SOURCE, sys))
    return System(nx, p, c, b)


def c2_system(sys: int = 0, nx: int = 256, npml: int = 20) -> System:
    """256^2 interior + 20 PML; 1-3 rings at 2500-3000 m/s, 5% noise; 1-4 Gaussian sources."""
    rv = rng_for(CFG_C2, COMP_VELOCITY, sys)
    rings = int(rv.integers(1, 4))
    c = skull_ring_velocity(nx + 2 * npml, npml, rv, rings=rings)
    b = gaussian_sources(nx + 2 * npml, npml, rng_for(CFG_C2, COMP_SOURCE, sys))
    return System(nx, npml, c, b)


def c4_sizes(nsys: int = 128):
    """Interior sizes ~ U{128,192,256,384,512}, PML ~ U{16..32}, one draw per system."""
    r = rng_for(CFG_C4, COMP_SIZES, 0)
    nxs = r.choice(np.array([128, 192, 256, 384, 512]), size=nsys)
    ps = r.integers(16, 33, size=nsys)
    return [(int(a), int(b)) for a, b in zip(nxs, ps)]


def c4_system(sys: int, nx: int, npml: int) -> System:
    rv = rng_for(CFG_C4, COMP_VELOCITY, sys)
    rings = int(rv.integers(1, 4))
    c = skull_ring_velocity(nx + 2 * npml, npml, rv, rings=rings)
    b = gaussian_sources(nx + 2 * npml, npml, rng_for(CFG_C4, COMP_SOURCE, sys))
    return System(nx, npml, c, b)


def c5_system(sys: int = 0) -> System:
    """1024^2 interior + 32 PML; 1-3 rings, 5% noise; 1-4 Gaussian sources."""
    nx, p = 1024, 32
    rv = rng_for(CFG_C5, COMP_VELOCITY, sys)
    rings = int(rv.integers(1, 4))
    c = skull_ring_velocity(nx + 2 * p, p, rv, rings=rings)
    b = gaussian_sources(nx + 2 * p, p, rng_for(CFG_C5, COMP_SOURCE, sys))
    return System(nx, p, c, b)


APPB_KINDS = ("gamma_dirac", "gamma_2dirac", "4layered", "4faulted")


def appendix_b_system(kind: str, sys: int = 0, nx: int = 256, npml: int = 20) -> System:
    """The paper's second synthetic workload (simplified spherical-wave and seismic settings):
    gamma_dirac / gamma_2dirac: one constant speed U[1, 2] (nondimensional) with 1 or 2 entries
    of +-1; 4layered / 4faulted: four aligned (or faulted) constant layers U[1, 2] with one
    smoothed unit point source (Gaussian, width 1.5 cells)."""
    nt = nx + 2 * npml
    k = APPB_KINDS.index(kind)
    rv = rng_for(CFG_APPB, COMP_VELOCITY, 100 * k + sys)
    rs = rng_for(CFG_APPB, COMP_SOURCE, 100 * k + sys)
    if kind in ("gamma_dirac", "gamma_2dirac"):
        c = rand_constant_velocity(nt, rv)
        b = m_dirac_source(nt, npml, rs, 1 if kind == "gamma_dirac" else 2)
    else:
        c = layered_velocity(nt, rv, layers=4, faulted=kind == "4faulted")
        i, j = _interior_node(nt, npml, rs)
        jj, ii = np.meshgrid(np.arange(nt, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
        b = np.exp(-((ii - i) ** 2 + (jj - j) ** 2) / (2.0 * 1.5 * 1.5)).astype(np.complex128)
    return System(nx, npml, c, b)


def c3_batch(batch: int = 64, nx: int = 128, npml: int = 16, step: int = 0):
    """Training batch: per sample a skull-ring velocity (1-3 rings) and a box-smoothed residual.

    Returns (c [B, nt, nt] float64 m/s, r [B, nt, nt] complex128).
    """
    nt = nx + 2 * npml
    cs = np.empty((batch, nt, nt))
    rs = np.empty((batch, nt, nt), np.complex128)
    for s in range(batch):
        sid = step * batch + s
        rv = rng_for(CFG_C3, COMP_VELOCITY, sid)
        cs[s] = skull_ring_velocity(nt, npml, rv, rings=int(rv.integers(1, 4)))
        rs[s] = box_smoothed_noise(nt, rng_for(CFG_C3, COMP_RESIDUAL, sid))
    return cs, rs


def mixed_training_sample(nt: int, npml: int, rng: np.random.Generator):
    """One (velocity, source) pair from a D0-like mixture (Table 4), with skull rings standing in
    for the idealized-skull class: velocity U([1,2]) or rings (1/2 each); source N(0,1), dirac,
    dirac1, dirac4, box-smoothed noise or Gaussian blobs."""
    if rng.uniform() < 0.5:
        c = uniform_velocity(nt, rng)
    else:
        c = skull_ring_velocity(nt, npml, rng, rings=int(rng.integers(1, 4)))
    u = rng.uniform()
    if u < 0.35:
        b = normal_source(nt, rng)
    elif u < 0.55:
        b = dirac_source(nt, rng)
    elif u < 0.60:
        b = dirac_source(nt, rng, centred=True)
    elif u < 0.65:
        b = dirac4_source(nt)
    elif u < 0.85:
        b = box_smoothed_noise(nt, rng)
    else:
        b = gaussian_sources(nt, npml, rng)
    return c, b


def training_set(count: int, nt: int, npml: int, *, first: int = 0):
    """A fixed data set of ``count`` (velocity, source) pairs from the D0-like mixture on one
    nt x nt grid (Section 3.4 trains on a fixed set of random samples per data set); sample i draws
    from stream ``first + i``. Validation sets use ``first = VAL_FIRST``.
    Returns (c [count, nt, nt] float64 in m/s, b [count, nt, nt] complex128)."""
    cs = np.empty((count, nt, nt), np.float64)
    bs = np.empty((count, nt, nt), np.complex128)
    for i in range(count):
        cs[i], bs[i] = mixed_training_sample(nt, npml, rng_for(CFG_TRAIN, COMP_SOURCE, first + i))
    return cs, bs


def epoch_order(count: int, epoch: int) -> np.ndarray:
    """The order in which epoch ``epoch`` visits a training set of ``count`` samples (a seeded
    permutation, drawn here so that the oracle and the GPU loop visit the same batches)."""
    return rng_for(CFG_TRAIN, COMP_ORDER, epoch).permutation(count)


# --------------------------------------------------------------------------- Table 4 data sets

# Section 3.2, Table 4: per data set, the source classes and the velocity classes with the
# probabilities they are drawn with. The idealized-skull class is stood in for by skull rings.
TABLE4 = {
    "D0": ((("normal", "dirac", "dirac1", "dirac4"), (0.6, 0.3, 0.05, 0.05)), (("uniform", "skull"), (0.5, 0.5))),
    "D1": ((("normal",), (1.0,)), (("uniform", "skull"), (0.5, 0.5))),
    "D2": ((("normal", "dirac", "dirac1", "dirac4"), (0.6, 0.3, 0.05, 0.05)),
           (("uniform", "skull", "rand_constant", "square"), (0.4, 0.4, 0.1, 0.1))),
    "D3": ((("normal",), (1.0,)), (("uniform", "skull", "rand_constant", "square"), (0.4, 0.4, 0.1, 0.1))),
    "D4": ((("normal",), (1.0,)), (("skull",), (1.0,))),
    "D5": ((("normal",), (1.0,)), (("uniform",), (1.0,))),
}


def table4_classes(dataset: str, rng: np.random.Generator):
    """(source class, velocity class) of one sample of data set D0..D5, drawn with Table 4's
    probabilities (source first, then velocity, one uniform draw each)."""
    (bk, bp), (ck, cp) = TABLE4[dataset]
    ub, uc = rng.uniform(), rng.uniform()
    b = bk[min(int(np.searchsorted(np.cumsum(bp), ub, side="right")), len(bk) - 1)]
    c = ck[min(int(np.searchsorted(np.cumsum(cp), uc, side="right")), len(ck) - 1)]
    return b, c


def table4_sample(dataset: str, nt: int, npml: int, rng: np.random.Generator):
    """One (velocity in m/s [nt, nt], source complex128 [nt, nt]) pair of data set D0..D5."""
    bkind, ckind = table4_classes(dataset, rng)
    if ckind == "uniform":
        c = uniform_velocity(nt, rng)
    elif ckind == "skull":
        c = skull_ring_velocity(nt, npml, rng, rings=int(rng.integers(1, 4)))
    elif ckind == "rand_constant":
        c = rand_constant_velocity(nt, rng)
    else:
        c = square_velocity(nt)
    if bkind == "normal":
        b = normal_source(nt, rng)
    elif bkind == "dirac":
        b = dirac_source(nt, rng)
    elif bkind == "dirac1":
        b = dirac_source(nt, rng, centred=True)
    else:
        b = dirac4_source(nt)
    return c, b


def table4_set(dataset: str, count: int, nt: int, npml: int, *, first: int = 0):
    """A fixed data set of ``count`` pairs of D0..D5 on one grid; sample i draws from stream
    ``first + i`` of the data set (validation sets use ``first = VAL_FIRST``).
    Returns (c [count, nt, nt] float64 in m/s, b [count, nt, nt] complex128)."""
    k = int(dataset[1])
    cs = np.empty((count, nt, nt), np.float64)
    bs = np.empty((count, nt, nt), np.complex128)
    for i in range(count):
        cs[i], bs[i] = table4_sample(dataset, nt, npml, rng_for(CFG_TABLE4, k, first + i))
    return cs, bs
