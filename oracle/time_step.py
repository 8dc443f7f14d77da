"""Wall time of one whole warm step of the CPU oracle on this host.

TEST INFRASTRUCTURE ONLY (see the package header): the CPU baseline that the
benchmark reports beside the device throughput.

A warm step is the step of an optimiser loop: from the converged
environment of the previous state, the state moves by
A <- A - 1e-3 |A| x / |x| along its preconditioned direction, the
environment is reconverged from the previous one (tolerance 1e-10), then the
K = 20 gradient and the 20-iteration CG run.  The cold preparation (first
convergence from the trace boundary, first gradient and direction) is timed
separately.  Prints one JSON record.

    python -m oracle.time_step d6chi72
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import torch

from . import ctmrg, gradient, metric


def main(name: str) -> dict:
    sys.path.insert(0, os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))))
    from paper_2511_09546_amd import inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    chi, K = w["chi"], w["grad_K"]
    t0 = time.perf_counter()
    env, it0, _ = ctmrg.converge(A, chi, w["tol"], w["n_iter"])
    e, g = gradient.grad_K(A, terms, env, chi, K)
    x, _, _, _ = metric.precondition(env, A, g.numpy(), w["delta"],
                                     w["cg_tol"], w["cg_maxiter"])
    t1 = time.perf_counter()
    x = x.numpy()
    A = A - 1e-3 * np.linalg.norm(A) / np.linalg.norm(x) * x
    t2 = time.perf_counter()
    env, it1, _ = ctmrg.converge(A, chi, w["tol"], w["n_iter"], env=env)
    t3 = time.perf_counter()
    e, g = gradient.grad_K(A, terms, env, chi, K)
    t4 = time.perf_counter()
    metric.precondition(env, A, g.numpy(), w["delta"], w["cg_tol"],
                        w["cg_maxiter"])
    t5 = time.perf_counter()
    return {"workload": name, "seconds": t5 - t2, "n_iter": it1,
            "phase_seconds": {"converge": t3 - t2, "grad": t4 - t3,
                              "precond": t5 - t4},
            "cold_preparation_seconds": t1 - t0, "cold_n_iter": it0,
            "cpu_count": os.cpu_count(),
            "torch_threads": torch.get_num_threads(),
            "command": f"python -m oracle.time_step {name}"}


if __name__ == "__main__":
    print(json.dumps(main(sys.argv[1] if len(sys.argv) > 1 else "d6chi72")),
          flush=True)
