"""Write fgmres_counts.json: FP64 oracle FGMRES(30) iteration counts on twelve seeded systems, with
the network's stored activations exact and rounded to BF16.

Systems: interiors 40^2 + 8 PML and 64^2 + 16 PML, seeds 0-5 (skull-ring velocity with 1-3 rings,
1-4 Gaussian sources, generator stream 14 of synth); the committed 4-level / 32-channel network on
its BF16-rounded weights (eq. (7), eq. (9)); Algorithm 1 with restart 30 and the stopping rule of
eq. (13) at tol 1e-6. For each system the file holds the count with exact FP64 activations
("its") and with every stored activation rounded to BF16 ("its_bf16_act", the oracle's optional
diagnostic emulation). Their difference is how far a rounding-level change of the preconditioner
alone moves this nonlinear iteration's count on that system; it is never a parity reference.

Only oracle/ and synth/ are called. Usage: python tests/golden/make_fgmres_counts.py [--jobs 4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
WEIGHTS = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "unet_l4_c32_in5.npz")
OUT = os.path.join(HERE, "fgmres_counts.json")
SYSTEMS = [(40, 8, s) for s in range(6)] + [(64, 16, s) for s in range(6)]
M, TOL, MAXIT = 30, 1e-6, 600


def oracle_counts(nx: int, p: int, seed: int):
    """(its exact, its with BF16 activation storage, true relres of both) for one system."""
    sys.path.insert(0, ROOT)
    import numpy as np

    from oracle import fgmres as ofg
    from oracle import helmholtz as ohz
    from oracle import unet
    from synth import C_REF, H_10PPW, gaussian_sources, rng_for, skull_ring_velocity

    nt = nx + 2 * p
    c = skull_ring_velocity(nt, p, rng_for(14, 0, seed), rings=1 + seed % 3).astype(np.float32)
    b = gaussian_sources(nt, p, rng_for(14, 1, seed))
    op = ohz.Problem(c.astype(np.float64), p, H_10PPW, 1.0, 2.0, C_REF)
    theta = unet.bf16_activation(np.load(WEIGHTS)["theta"].astype(np.float32))
    specs = unet.layer_specs(4, 32, 5)
    A = lambda x: ohz.op_apply(op, x.reshape(op.ny, op.nx)).ravel()
    out = {}
    for key, act in (("its", None), ("its_bf16_act", unet.bf16_activation)):
        Mp = lambda v: unet.precond_apply(theta, specs, op, v.reshape(op.ny, op.nx), act_round=act).ravel()
        r = ofg.fgmres(A, Mp, b.ravel(), m=M, tol=TOL, maxit=MAXIT)
        out[key] = r.its
        out[key.replace("its", "true_relres")] = r.true_relres
        out[key.replace("its", "status")] = r.status
    return out


def _job(args):
    nx, p, seed = args
    return f"{nx}_{p}_{seed}", dict(nx=nx, npml=p, seed=seed, **oracle_counts(nx, p, seed))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    threads = max(1, (os.cpu_count() or 1) // a.jobs)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = str(threads)
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(a.jobs, mp_context=mp.get_context("spawn")) as ex:
        res = dict(ex.map(_job, SYSTEMS))
    doc = {
        "what": "FP64 oracle FGMRES iteration counts, network activations exact and rounded to BF16",
        "cite": "Algorithm 1 (flexible GMRES), eq. (7) and (9) (preconditioner), eq. (13) (stopping rule)",
        "m": M, "tol": TOL, "maxit": MAXIT, "generator_stream": 14,
        "systems": res,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    for k, r in res.items():
        print(k, r["its"], r["its_bf16_act"])


if __name__ == "__main__":
    main()
