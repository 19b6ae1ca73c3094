"""Write c2_oracle.json: the FP64 oracle's FGMRES(30) solve of the single-solve workload.

The system is synth.c2_system(0) (256^2 interior + 20 PML cells, skull-ring velocity, Gaussian
sources); the velocity is rounded to float32 first, as the library takes it. The preconditioner is
the committed 4-level / 32-channel network (eq. (7), eq. (9)); the Krylov method is Algorithm 1
with restart length 30 and the stopping rule of eq. (13) at tol 1e-6. Three oracle runs:

  bf16_weights      FP64 network on the BF16-rounded weights (the BF16 path's reference)
  fp32_weights      FP64 network on the float32 weights (the FP32 path's reference)
  bf16_weights_bf16_activations
                    as bf16_weights, with every stored activation rounded to BF16 as well
                    (a diagnostic of how far rounding alone moves the iteration count; never a
                    parity reference)

Only oracle/ and synth/ are called. Usage: python tests/golden/make_c2_oracle.py [--jobs 3]
(about 5 minutes per run on one core group).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
WEIGHTS = os.path.join(ROOT, "paper_2607_16906_amd", "weights", "unet_l4_c32_in5.npz")
OUT = os.path.join(HERE, "c2_oracle.json")
M, TOL, MAXIT = 30, 1e-6, 3000


def run(kind: str):
    sys.path.insert(0, ROOT)
    import numpy as np

    from oracle import fgmres as ofg
    from oracle import helmholtz as ohz
    from oracle import unet
    from synth import C_REF, H_10PPW, c2_system

    s = c2_system(0)
    c = s.c.astype(np.float32).astype(np.float64)
    op = ohz.Problem(c, s.npml, H_10PPW, 1.0, 2.0, C_REF)
    theta = np.load(WEIGHTS)["theta"].astype(np.float32)
    specs = unet.layer_specs(4, 32, 5)
    th = theta.astype(np.float64) if kind == "fp32_weights" else unet.bf16_activation(theta)
    act = unet.bf16_activation if kind == "bf16_weights_bf16_activations" else None
    A = lambda x: ohz.op_apply(op, x.reshape(op.ny, op.nx)).ravel()
    Mp = lambda v: unet.precond_apply(th, specs, op, v.reshape(op.ny, op.nx), act_round=act).ravel()
    t0 = time.time()
    r = ofg.fgmres(A, Mp, s.b.ravel(), m=M, tol=TOL, maxit=MAXIT)
    return kind, dict(its=r.its, cycles=r.cycles, status=r.status, true_relres=r.true_relres,
                      est_history=[float(e) for e in r.est_history],
                      true_history=[float(e) for e in r.true_history],
                      x_norm=float(np.linalg.norm(r.x)), seconds=round(time.time() - t0, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=3)
    a = ap.parse_args()
    kinds = ["bf16_weights", "fp32_weights", "bf16_weights_bf16_activations"]
    threads = max(1, (os.cpu_count() or 1) // a.jobs)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = str(threads)
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(a.jobs, mp_context=mp.get_context("spawn")) as ex:
        res = dict(ex.map(run, kinds))
    with open(WEIGHTS, "rb") as f:
        wsum = hashlib.md5(f.read()).hexdigest()
    doc = {
        "what": "FP64 oracle FGMRES on synth.c2_system(0) (256^2 interior + 20 PML), the committed "
                "4-level / 32-channel network, x0 = 0",
        "cite": "Algorithm 1 (flexible GMRES), eq. (7) and (9) (preconditioner), eq. (13) (stopping rule)",
        "m": M, "tol": TOL, "maxit": MAXIT, "weights_md5": wsum,
        "runs": res,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    for k, r in res.items():
        print(f"{k}: its {r['its']} cycles {r['cycles']} status {r['status']} "
              f"true relres {r['true_relres']:.3e} ({r['seconds']} s)")


if __name__ == "__main__":
    main()
