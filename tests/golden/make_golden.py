"""Writes the oracle's expected values for the named workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators; the
device path is never involved.  Output: tests/golden/<workload>.json with the
iteration count, Delta, energy per site, gradient, preconditioned direction,
CG iteration count and residual, and the corner spectra.

    python tests/golden/make_golden.py d2chi8 d4chi32 [d6chi72 kitaev2x2]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import step  # noqa: E402
from paper_2511_09546_amd import inputs  # noqa: E402


def make(name: str) -> dict:
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    t0 = time.perf_counter()
    r = step.run_step(A, terms, w["chi"], w["tol"], w["n_iter"], w["grad_K"],
                      w["delta"], w["cg_tol"], w["cg_maxiter"])
    out = dict(workload=name, params=w, n_iter=r["n_iter"], delta=r["delta"],
               e=r["e"], g=r["g"].ravel().tolist(), x=r["x"].ravel().tolist(),
               cg_iter=r["cg_iter"], cg_resid=r["cg_resid"],
               breakdown=r["breakdown"],
               spectra=r["spectra"].reshape(-1).tolist(),
               spectra_shape=list(r["spectra"].shape),
               seconds=r["seconds"], total_seconds=time.perf_counter() - t0)
    return out


if __name__ == "__main__":
    for name in sys.argv[1:]:
        out = make(name)
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(name, out["n_iter"], out["delta"], out["e"], out["cg_iter"],
              out["cg_resid"], out["total_seconds"], flush=True)
