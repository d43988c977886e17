"""Writes c3_oracle_samples.npz: FP64 oracle trajectories of the 2 x 256 x 256, N = 1024,
sigma_o = 0.02 workload (all components observed through arctan), for the GPU parity tests
that cannot afford the oracle's run time on the test machine.

  implicit   linearly implicit likelihood step at the workload's K = 200, particles 0, 511,
             1023 of the 1024
  explicit   plain Euler-Maruyama (eq. 7) at the stable K = 2500 (dt = 1/K <= sigma_o^2),
             particles 0 and 1; the same run with the prior scaled by (1 + 1e-12) gives the
             stability gate (relative change of the result, must stay below 1e-9)

Only every STRIDE-th state component of each particle is stored (the GPU runs the whole
problem and is compared on those components).  Inputs are regenerated from the seeded
workload generator, so the file holds expected values only.  Calls only oracle/ and the
input generator:

    python tests/golden/make_c3_oracle.py        # about 25 min on 8 cores
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STRIDE = 32
IMPLICIT_ROWS = [0, 511, 1023]
EXPLICIT_ROWS = [0, 1]
EXPLICIT_K = 2500
OUT = os.path.join(HERE, "c3_oracle_samples.npz")


def _run(task):
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import ensf
    kind, scale = task
    p = workloads.config_problem(3)
    X = p.X.astype(np.float64) * scale
    t0 = time.time()
    with threadpool_limits(3):
        if kind == "implicit":
            Z = ensf.analysis(X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                              particle_ids=IMPLICIT_ROWS, lik_step="implicit",
                              chunk=len(IMPLICIT_ROWS))
        else:
            Z = ensf.analysis(X, p.obs_idx, p.obs_val, p.sigma_o, EXPLICIT_K, p.seed,
                              particle_ids=EXPLICIT_ROWS, chunk=len(EXPLICIT_ROWS))
    print(f"{kind} (scale {scale!r}) done in {time.time() - t0:.0f}s", flush=True)
    return Z


def main():
    tasks = [("implicit", 1.0), ("explicit", 1.0), ("explicit", 1.0 + 1e-12)]
    with ProcessPoolExecutor(max_workers=3) as ex:
        imp, exp, exp_pert = ex.map(_run, tasks)
    gate = float(np.linalg.norm(exp_pert - exp) / np.linalg.norm(exp))
    print(f"explicit K={EXPLICIT_K} sensitivity to a 1e-12 prior change: {gate:.2e}")
    np.savez_compressed(OUT, stride=STRIDE,
                        implicit_rows=np.array(IMPLICIT_ROWS), implicit_k=200,
                        implicit=imp[:, ::STRIDE],
                        explicit_rows=np.array(EXPLICIT_ROWS), explicit_k=EXPLICIT_K,
                        explicit=exp[:, ::STRIDE], explicit_gate=gate)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
