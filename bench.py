#!/usr/bin/env python3
"""Throughput of the preconditioned iPEPS step on one MI355X.

One step (the whole hot path on one state):
  ctm_converge      CTMRG to a corner-spectrum change < 1e-10 (FP64) or to
                    the rounding floor of the contraction arithmetic
  ipeps_energy_grad energy per site and dE/dA, K = 20 unrolled iterations
  precond_apply     x = (N_local + 1e-4 I)^-1 g, 20 CG iterations
  update            A <- A - 1e-3 |A| x/|x|, environment kept (warm start)
on the seeded 1x1, d=2, D=6, chi=72 J1-J2 (J2 = 0.5) state (synthetic
N(0,1) tensor, normalised to max|A| = 1).  The first warm-up step starts
from the trace boundary (cold); timed steps are warm, as in an optimiser.
A, g and x stay in device memory (device-pointer entry points); only
scalars cross PCIe inside the timed region.

The headline runs the dense contractions in FP32 on the matrix cores
(projector SVD, normalisation, traces and CG scalars stay FP64); the same
steps are then timed with BF16x3 contractions (three BF16 products of a
two-term split) and with every product in FP64 ("plain FP64"), and the
energies of the cold steps are compared with the FP64 one.

Prints one JSON line.  The roofline object reports the library's
matrix-core GEMM in the headline arithmetic (the dominant kernel):
algorithmic flops (2 M N K per launch) over the device time of its
launches, both recorded live with HIP events on the library's stream
during as many steps as the timed ones, run right after them (the events
cost about 6 % of a step, so the timed steps run without); its traffic is
the HBM bytes per launch from the
counter record under profiles/ (null when the kernel source has changed
since the counters were taken).  The cpu_baseline object times the CPU oracle on a
bounded sample of the same workload (one CTMRG iteration and one K=1
gradient step) and scales it to one step.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--prec fp32]
                    [--no-fp64] [--no-cpu-baseline] [--checkpoint]

Besides the contract fields the line reports the median and p10/p90 of the
timed steps with the mean time of each phase (step_ms), and for every
arithmetic the error of its cold step against the FP64 CPU oracle's stored
values for the same workload (error_vs_oracle: |de|, |dg|/|g|, |dx|/|x|).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("energy+grad+precond steps/s at D=6,χ=72 vs plain FP64; "
          "MFMA util; p50/p99 lat")
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def cpu_baseline(name, n_conv):
    """Oracle on the host: one CTMRG iteration from the trace boundary and
    one K=1 gradient step from that environment, scaled to a step of
    n_conv iterations + K gradient steps (+ the negligible CG)."""
    import torch
    from oracle import ctmrg, gradient
    from paper_2511_09546_amd import inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    env, _, _ = ctmrg.converge(A, w["chi"], 0.0, 1)
    t1 = time.perf_counter()
    gradient.grad_K(A, terms, env, w["chi"], 1)
    t2 = time.perf_counter()
    t_fwd, t_g1 = t1 - t0, t2 - t1
    t_step = n_conv * t_fwd + w["grad_K"] * t_g1
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"{name}: 1 CTMRG iteration ({t_fwd:.1f} s) + 1 "
                       f"K=1 gradient step ({t_g1:.1f} s) on the host, "
                       f"scaled to {n_conv} iterations + K={w['grad_K']} "
                       f"gradient steps = {t_step:.0f} s/step")}


def measured_traffic(prec):
    """HBM bytes per launch of the FP32 GEMM from the committed counter
    record (two rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, scaled
    by a plain copy), or None when the GEMM source changed since then."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", "gemm_fp32_d6chi72_traffic.json")
    src = os.path.join(ROOT, "paper_2511_09546_amd", "csrc", "gemm.hip")
    if prec != "fp32" or not os.path.exists(rec):
        return None
    r = json.load(open(rec))
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != r["gemm_source_sha256"]:
            return None
    return r["traffic_bytes_per_launch"]


def run(name, prec, steps, warmup, ckpt=0):
    """Warm-up and timed steps in one arithmetic; returns the measurements."""
    import torch
    from paper_2511_09546_amd import binding, inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    o = binding.default_opts()
    o.prec = {"fp64": binding.FP64, "fp32": binding.FP32,
              "bf16": binding.BF16}[prec]
    o.grad_checkpoint = ckpt
    ctx = binding.Context(A, w["chi"], opts=o)
    fam = {"fp64": binding.PROF_GEMM, "fp32": binding.PROF_GEMM32,
           "bf16": binding.PROF_GEMM16}[prec]

    # site tensor, gradient and direction stay resident in HBM: the step
    # uses the device-pointer entry points (torch provides the buffers)
    dA = torch.tensor(A, dtype=torch.float64, device="cuda:0")
    dg = torch.zeros_like(dA)
    dx = torch.zeros_like(dA)

    def step(A, keep=False):
        # every library call returns with its results written (the context
        # stream is synchronised), so host timers bracket the phases
        t0 = time.perf_counter()
        n_it, dl, ok = ctx.converge(w["tol"], w["n_iter"])
        t1 = time.perf_counter()
        e = ctx.energy_grad_dev(terms, dg.data_ptr())
        t2 = time.perf_counter()
        cg_it, res, brk = ctx.precond_dev(dg.data_ptr(), dx.data_ptr(),
                                          w["delta"], w["cg_tol"],
                                          w["cg_maxiter"])
        t3 = time.perf_counter()
        out = None
        if keep:  # the cold step's g and x, for the error against the oracle
            out = (dg.cpu().numpy().copy(), dx.cpu().numpy().copy())
        # optimiser stand-in of the benchmark loop (not part of the step's
        # method): a preconditioned descent move of 1e-3 |A|
        A.sub_(1e-3 * A.norm() / dx.norm() * dx)
        torch.cuda.synchronize()
        ctx.set_state_dev(A.data_ptr())
        return A, dict(ms=1e3 * (time.perf_counter() - t0), iters=n_it, e=e,
                       delta=dl, cg=cg_it, res=res,
                       phase_ms=[1e3 * (t1 - t0), 1e3 * (t2 - t1),
                                 1e3 * (t3 - t2)]), out

    A = dA
    infos = []
    cold = None
    for i in range(warmup):
        A, info, kept = step(A, keep=(i == 0))
        if i == 0:
            cold = (info["e"],) + kept
        infos.append(info)
        print(f"[{prec}] warmup {i}: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = []
    for i in range(steps):
        A, info, _ = step(A)
        timed.append(info)
        print(f"[{prec}] step {i}: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same number of steps again, continuing the trajectory, with HIP
    # events around every launch of the timed kernel families (the events
    # cost about 6 % of a step, so the steps above run without them)
    ctx.profile(True)
    t1 = time.perf_counter()
    for i in range(steps):
        A, info, _ = step(A)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    prof = {f: ctx.profile_read(f) for f in
            (fam, binding.PROF_JACOBI, binding.PROF_PERMUTE,
             binding.PROF_NET)}
    ctx.profile(False)
    stats = ctx.stats()
    ctx.close()
    return dict(elapsed=elapsed, timed=timed, infos=infos, prof=prof,
                fam=fam, stats=stats, cold=cold, elapsed_prof=elapsed_prof)


def step_summary(r):
    """Median, p10, p90 of the timed steps and the mean time per phase."""
    import numpy as np
    ms = np.array([t["ms"] for t in r["timed"]])
    ph = np.array([t["phase_ms"] for t in r["timed"]]).mean(axis=0)
    return {"p10_ms": float(np.percentile(ms, 10)),
            "p50_ms": float(np.percentile(ms, 50)),
            "p90_ms": float(np.percentile(ms, 90)),
            "phase_ms": {"ctm_converge": float(ph[0]),
                         "energy_grad": float(ph[1]),
                         "precond_apply": float(ph[2])}}


def oracle_error(name, cold):
    """Error of the cold step (trace boundary -> converge -> energy and
    gradient -> preconditioned direction, the protocol of the stored oracle
    values in tests/golden) against the FP64 CPU oracle's values."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if cold is None or not os.path.exists(path):
        return None
    gold = json.load(open(path))
    e, g, x = cold
    g_or = np.array(gold["g"]).reshape(g.shape)
    x_or = np.array(gold["x"]).reshape(x.shape)
    return {"e_abs": abs(e - gold["e"]),
            "e_rel": abs(e - gold["e"]) / abs(gold["e"]),
            "g_rel": float(np.linalg.norm(g - g_or) / np.linalg.norm(g_or)),
            "x_rel": float(np.linalg.norm(x - x_or) / np.linalg.norm(x_or)),
            "reference": f"tests/golden/{name}.json (oracle, FP64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="d6chi72")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16",
                                                       "fp64"])
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the plain FP64 and the other mixed runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--checkpoint", action="store_true",
                    help="checkpointed gradient (recompute each unrolled "
                         "iteration in the backward pass)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is "
              "not supported (independent states would shard across GPUs "
              "with no exchange; one state is not split)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_09546_amd import binding, inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    binding.load()
    name = args.workload
    w = inputs.WORKLOADS[name]

    ck = 1 if args.checkpoint else 0
    head = run(name, args.prec, args.steps, args.warmup, ck)
    base = other = None
    if args.prec != "fp64" and not args.no_fp64:
        oprec = "bf16" if args.prec == "fp32" else "fp32"
        other = (oprec, run(name, oprec, args.steps, args.warmup, ck))
        base = run(name, "fp64", args.steps, args.warmup, ck)

    timed, elapsed = head["timed"], head["elapsed"]
    n_g, t_g, fl_g, by_g = head["prof"][head["fam"]]
    _, t_jac, _, _ = head["prof"][binding.PROF_JACOBI]
    _, t_perm, _, _ = head["prof"][binding.PROF_PERMUTE]
    ms = sorted(t["ms"] for t in timed)
    p = lambda q: ms[min(len(ms) - 1, int(round(q * (len(ms) - 1))))]  # noqa
    achieved = fl_g / t_g / 1e12 if t_g > 0 else 0.0
    n_net, t_net, fl_net, _ = head["prof"][binding.PROF_NET]
    ach_net = fl_net / t_net / 1e12 if t_net > 0 else 0.0
    peak = PEAK_TFLOPS[args.prec]
    n_conv = int(round(sum(t["iters"] for t in timed) / len(timed)))
    value = args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 contractions, f64 SVD/CG",
                  "bf16": "bf16x3 contractions, f64 SVD/CG"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{name}: 1x1 iPEPS d={w['d']} D={w['D']} "
                               f"chi={w['chi']} J1-J2 J2={w['J2']}, warm "
                               "steps (env kept), CTMRG tol 1e-10 (FP32: its "
                               f"1e-7 floor), K={w['grad_K']}, CG 20 its, "
                               "delta 1e-4",
                   "D": w["D"], "chi": w["chi"], "d": w["d"],
                   "grad_K": w["grad_K"], "prec": args.prec,
                   "grad_checkpoint": ck},
        "p50_ms": p(0.5), "p99_ms": p(0.99),
        "step_ms": step_summary(head),
        "error_vs_oracle": oracle_error(name, head["cold"]),
        "ctm_iters_per_step": [t["iters"] for t in timed],
        "cold_step_ms": head["infos"][0]["ms"] if head["infos"] else None,
        "energy_per_site": timed[-1]["e"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(args.prec),
                     "kernel": f"{args.prec} matrix-core GEMM (gemm_kernel "
                               "and gemm_f32_lds_kernel, all tile shapes)",
                     "launches": n_g,
                     "avg_launch_us": 1e6 * t_g / max(n_g, 1),
                     "algorithmic_bytes_per_launch": by_g / max(n_g, 1),
                     "gemm_share_of_step": t_g / head["elapsed_prof"],
                     "measured_over": f"{args.steps} profiled steps after "
                                      "the timed ones",
                     # the same GEMM restricted to the launches of the
                     # tensor-network contractions (CTMRG moves, energy
                     # network, their reverse passes): no SVD or
                     # complement-solve products
                     "network_contractions": {
                         "achieved": ach_net, "frac": ach_net / peak,
                         "launches": n_net,
                         "share_of_gemm_time": t_net / max(t_g, 1e-30)}},
        "kernel_time_s": {"gemm": t_g, "jacobi": t_jac, "permute": t_perm},
        "svd_stats": head["stats"],
    }
    if base is not None:
        v64 = args.steps / base["elapsed"]
        e_b = base["infos"][0]["e"] if base["infos"] else None

        def ediff(r):
            e = r["infos"][0]["e"] if r["infos"] else None
            return abs(e - e_b) if e is not None and e_b is not None else None

        out["plain_fp64"] = {
            "value": v64, "ms_per_step": 1e3 * base["elapsed"] / args.steps,
            "speedup": value / v64,
            "step_ms": step_summary(base),
            "error_vs_oracle": oracle_error(name, base["cold"]),
            "ctm_iters_per_step": [t["iters"] for t in base["timed"]],
            "cold_step_energy_abs_diff": ediff(head)}
        oprec, o = other
        vo = args.steps / o["elapsed"]
        n_o, t_o, fl_o, _ = o["prof"][o["fam"]]
        out[f"{oprec}_contractions"] = {
            "value": vo, "ms_per_step": 1e3 * o["elapsed"] / args.steps,
            "speedup_vs_fp64": vo / v64,
            "step_ms": step_summary(o),
            "error_vs_oracle": oracle_error(name, o["cold"]),
            "ctm_iters_per_step": [t["iters"] for t in o["timed"]],
            "cold_step_energy_abs_diff_vs_fp64": ediff(o),
            "gemm_tflops": fl_o / t_o / 1e12 if t_o > 0 else 0.0}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name, n_conv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
