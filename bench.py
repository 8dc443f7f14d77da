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
steps are then timed with BF16x3 contractions, with every product in FP64
("plain FP64"), and shorter runs take single-pass BF16 contractions and the
BF16 -> FP32 precision ladder.  Every arithmetic reports the error of its
cold step against the FP64 oracle's stored values, its per-phase times and
its milliseconds per CTMRG iteration (the converge phases of different
arithmetics run different iteration counts: their floors differ).

Further legs: `serving` replays the seeded request stream (Poisson arrivals
at 20/s, D 3..6, chi 2D^2..3D^2; a prefix of --serve-requests requests) and
reports p50/p99 latency, throughput, the overlap of the request windows and how
many of a sample gave bitwise the results of the same request run alone;
`serving_sweep` replays a coupling sweep (8 states x 6 values of J2, one
state_key per state) and reports the same with the warm-start counts and
the CTMRG iterations of cold and warm requests;
`lbfgs` times iterations of the preconditioned L-BFGS on the same state;
`preconditioners` times one application of every preconditioner at the
converged state (local metric by CG and by GMRES(30), belief propagation,
one product with the full metric and its GMRES(30) solve) beside one
gradient evaluation.

The roofline object reports the dominant kernel, the FP32 matrix-core GEMM
with 128 x 144 tiles that carries the chi^2 D^8 products of the network
contractions (enlarged corners, renormalised edges, open corners of the
energy network, and their reverse passes): algorithmic flops (2 M N K per
launch) over the device time of its launches, both recorded live with HIP
events on the library's stream during as many steps as the timed ones, run
right after them (the events cost about 6 % of a step, so the timed steps
run without); its traffic is the HBM bytes per launch from the counter
record under profiles/ (null when the kernel source has changed since the
counters were taken).  Beside it: every GEMM launch of the network
contractions, and every GEMM launch of the step.  The cpu_baseline object times the CPU oracle on the host on a
bounded sample of the same workload (one CTMRG iteration, the energy network
with its backward, one unrolled iteration with its backward, one CG solve)
and composes one step from those phases; the wall time of the whole cold
oracle step that wrote the stored values (tests/golden) is reported beside
it, and so are one-core oracle times of the two small workloads (the whole
cold step of D=2, chi=8; a composed cold step of D=4, chi=32).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--prec fp32]
                    [--no-fp64] [--no-cpu-baseline] [--checkpoint]
                    [--serve-requests 128] [--no-lbfgs] [--no-precond]

Prints one JSON line.
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
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0,
               "bf16x1": 2500.0}


def cpu_baseline(name, n_conv):
    """The oracle on the host, phase by phase: one CTMRG iteration (from the
    trace boundary), the energy network and its backward (K = 0 gradient),
    one unrolled iteration with its backward (K = 1 minus K = 0) and one
    20-iteration CG solve; composed into one step of n_conv iterations and
    K unrolled iterations."""
    import numpy as np
    import torch
    from oracle import ctmrg, gradient, metric
    from paper_2511_09546_amd import inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    env, _, _ = ctmrg.converge(A, w["chi"], 0.0, 1)
    t1 = time.perf_counter()
    gradient.grad_K(A, terms, env, w["chi"], 0)
    t2 = time.perf_counter()
    _, g = gradient.grad_K(A, terms, env, w["chi"], 1)
    t3 = time.perf_counter()
    metric.precondition(env, A, g.numpy(), w["delta"], 0.0, w["cg_maxiter"])
    t4 = time.perf_counter()
    t_it, t_g0, t_g1, t_cg = t1 - t0, t2 - t1, t3 - t2, t4 - t3
    t_adj = max(t_g1 - t_g0, 0.0)
    K = w["grad_K"]
    t_step = n_conv * t_it + t_g0 + K * t_adj + t_cg
    out = {"value": 1.0 / t_step, "unit": "steps/s", "cores": threads,
           "kind": "oracle",
           "host_cpu_count": os.cpu_count(), "torch_threads": threads,
           "sample": (f"{name} on the host: 1 CTMRG iteration {t_it:.1f} s, "
                      f"energy network + backward {t_g0:.1f} s, 1 unrolled "
                      f"iteration + backward {t_g1:.1f} - {t_g0:.1f} s, "
                      f"CG {t_cg:.2f} s; one step = {n_conv} iterations + "
                      f"energy + K={K} unrolled iterations + CG = "
                      f"{t_step:.0f} s"),
           "sample_seconds": t4 - t0}
    gold = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if os.path.exists(gold):
        # the whole cold oracle step that wrote the stored values, timed
        # where they were written (not this host)
        g = json.load(open(gold))
        out["stored_cold_step_seconds"] = g.get("total_seconds")
    out["one_core_small"] = cpu_small_one_core()
    return out


def cpu_small_one_core():
    """The oracle on one host thread at the two small workloads: the whole
    cold step of d2chi8 (D=2, chi=8: its stored settings), and for d4chi32
    (D=4, chi=32) one CTMRG iteration, the energy network with its backward
    and one unrolled iteration with its backward, composed like the main
    sample into a cold step of its stored iteration count (seconds)."""
    import torch
    from oracle import ctmrg, gradient, metric, step
    from paper_2511_09546_amd import inputs
    keep = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        w = inputs.WORKLOADS["d2chi8"]
        A = inputs.workload_state("d2chi8")
        terms = inputs.workload_terms("d2chi8")
        t0 = time.perf_counter()
        step.run_step(A, terms, w["chi"], w["tol"], w["n_iter"], w["grad_K"],
                      w["delta"], w["cg_tol"], w["cg_maxiter"])
        t_small = time.perf_counter() - t0
        w = inputs.WORKLOADS["d4chi32"]
        A = inputs.workload_state("d4chi32")
        terms = inputs.workload_terms("d4chi32")
        t0 = time.perf_counter()
        env, _, _ = ctmrg.converge(A, w["chi"], 0.0, 1)
        t1 = time.perf_counter()
        gradient.grad_K(A, terms, env, w["chi"], 0)
        t2 = time.perf_counter()
        _, g = gradient.grad_K(A, terms, env, w["chi"], 1)
        t3 = time.perf_counter()
        metric.precondition(env, A, g.numpy(), w["delta"], 0.0,
                            w["cg_maxiter"])
        t4 = time.perf_counter()
        gold = json.load(open(os.path.join(ROOT, "tests", "golden",
                                           "d4chi32.json")))
        n_conv = int(gold["n_iter"])
        t_adj = max((t3 - t2) - (t2 - t1), 0.0)
        t_mid = (n_conv * (t1 - t0) + (t2 - t1) + w["grad_K"] * t_adj +
                 (t4 - t3))
    finally:
        torch.set_num_threads(keep)
    return {"cores": 1,
            "d2chi8_cold_step_s": t_small,
            "d4chi32_cold_step_s": t_mid,
            "d4chi32_sample": (f"1 CTMRG iteration {t1 - t0:.2f} s, energy "
                               f"network + backward {t2 - t1:.2f} s, 1 "
                               f"unrolled iteration + backward "
                               f"{t3 - t2:.2f} - {t2 - t1:.2f} s, CG "
                               f"{t4 - t3:.3f} s; {n_conv} iterations + "
                               f"energy + K={w['grad_K']} unrolled "
                               f"iterations + CG"),
            "sample_seconds": t_small + (t4 - t0)}


def measured_traffic(prec):
    """HBM bytes per launch of the 128 x 144-tile FP32 GEMM from the
    committed counter record (two rocprofv3 --pmc passes, FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy), or None when the GEMM source
    changed since then."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", "gemm_fp32_wide_d6chi72_traffic.json")
    src = os.path.join(ROOT, "paper_2511_09546_amd", "csrc", "gemm.hip")
    if prec != "fp32" or not os.path.exists(rec):
        return None
    r = json.load(open(rec))
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != r["gemm_source_sha256"]:
            return None
    return r["traffic_bytes_per_launch"]


PRECS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x1": 3}


def run(name, prec, steps, warmup, ckpt=0, ladder=0, profile=True):
    """Warm-up and timed steps in one arithmetic; returns the measurements."""
    import torch
    from paper_2511_09546_amd import binding, inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    o = binding.default_opts()
    o.prec = PRECS[prec]
    o.grad_checkpoint = ckpt
    o.ladder = ladder
    ctx = binding.Context(A, w["chi"], opts=o)
    fam = {"fp64": binding.PROF_GEMM, "fp32": binding.PROF_GEMM32,
           "bf16": binding.PROF_GEMM16,
           "bf16x1": binding.PROF_GEMM16}[prec]

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
        print(f"[{prec}{' ladder' if ladder else ''}] warmup {i}: {info}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = []
    for i in range(steps):
        A, info, _ = step(A)
        timed.append(info)
        print(f"[{prec}{' ladder' if ladder else ''}] step {i}: {info}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof, elapsed_prof = None, None
    if profile:
        # the same number of steps again, continuing the trajectory, with
        # HIP events around every launch of the timed kernel families (the
        # events cost about 6 % of a step, so the steps above run without)
        ctx.profile(True)
        t1 = time.perf_counter()
        for i in range(steps):
            A, info, _ = step(A)
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - t1
        prof = {f: ctx.profile_read(f) for f in
                (fam, binding.PROF_JACOBI, binding.PROF_PERMUTE,
                 binding.PROF_NET, binding.PROF_WIDE)}
        ctx.profile(False)
    stats = ctx.stats()
    ctx.close()
    return dict(elapsed=elapsed, timed=timed, infos=infos, prof=prof,
                fam=fam, stats=stats, cold=cold, elapsed_prof=elapsed_prof,
                steps=steps)


def step_summary(r):
    """Median, p10, p90 of the timed steps, the mean time per phase and the
    milliseconds per CTMRG iteration of the converge phase."""
    import numpy as np
    ms = np.array([t["ms"] for t in r["timed"]])
    ph = np.array([t["phase_ms"] for t in r["timed"]]).mean(axis=0)
    its = np.array([t["iters"] for t in r["timed"]], dtype=float)
    conv = np.array([t["phase_ms"][0] for t in r["timed"]])
    return {"p10_ms": float(np.percentile(ms, 10)),
            "p50_ms": float(np.percentile(ms, 50)),
            "p90_ms": float(np.percentile(ms, 90)),
            "phase_ms": {"ctm_converge": float(ph[0]),
                         "energy_grad": float(ph[1]),
                         "precond_apply": float(ph[2])},
            "ctm_iters_mean": float(its.mean()),
            "ms_per_ctm_iteration": float(conv.sum() / max(its.sum(), 1))}


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
            "g_max_rel": float(np.abs(g - g_or).max() / np.abs(g_or).max()),
            "x_max_rel": float(np.abs(x - x_or).max() / np.abs(x_or).max()),
            "reference": f"tests/golden/{name}.json (oracle, FP64)"}


def arith_record(r, name, base=None):
    """Throughput, per-phase times and error of one arithmetic's run."""
    v = r["steps"] / r["elapsed"]
    out = {"value": v, "ms_per_step": 1e3 * r["elapsed"] / r["steps"],
           "step_ms": step_summary(r),
           "error_vs_oracle": oracle_error(name, r["cold"]),
           "ctm_iters_per_step": [t["iters"] for t in r["timed"]]}
    if base is not None:
        sb, sr = step_summary(base), out["step_ms"]
        out["speedup_vs_fp64"] = v / (base["steps"] / base["elapsed"])
        # equal work: the K-step gradient and the 20-iteration CG do the
        # same iterations in every arithmetic; CTMRG per iteration
        out["speedup_vs_fp64_equal_work"] = {
            "energy_grad": sb["phase_ms"]["energy_grad"] /
            sr["phase_ms"]["energy_grad"],
            "precond_apply": sb["phase_ms"]["precond_apply"] /
            sr["phase_ms"]["precond_apply"],
            "per_ctm_iteration": sb["ms_per_ctm_iteration"] /
            sr["ms_per_ctm_iteration"]}
    if r["prof"] is not None:
        n, t, fl, _ = r["prof"][r["fam"]]
        out["gemm_tflops"] = fl / t / 1e12 if t > 0 else 0.0
    return out


def lbfgs_leg(name, prec, iters):
    """Iterations of the preconditioned L-BFGS (ipeps_lbfgs_step) on the
    workload's state: seconds and evaluations per iteration."""
    from paper_2511_09546_amd import binding, inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    o = binding.default_opts()
    o.prec = PRECS[prec]
    p = binding.lbfgs_default_params()
    rec = []
    with binding.Context(A, w["chi"], opts=o) as ctx:
        t0 = time.perf_counter()
        with binding.Lbfgs(ctx, terms, p) as opt:
            t1 = time.perf_counter()
            e0 = opt.e0
            for _ in range(iters):
                t = time.perf_counter()
                info = opt.step()
                info["seconds"] = time.perf_counter() - t
                rec.append(info)
                print(f"[lbfgs] {info}", file=sys.stderr, flush=True)
    secs = sum(r["seconds"] for r in rec)
    return {"workload": f"{name}, {prec} contractions, local-metric "
                        "preconditioned, m=200, Hager-Zhang, delta = |dE|",
            "first_evaluation_s": t1 - t0, "e0": e0,
            "energies": [r["e"] for r in rec],
            "evals_per_iteration": [r["n_evals"] for r in rec],
            "seconds_per_iteration": secs / max(len(rec), 1),
            "iterations": len(rec)}


def precond_leg(name, prec, gmres_m=30):
    """Seconds per application of every preconditioner at the workload's
    converged state, beside one energy-gradient evaluation: the local
    metric by CG (20 iterations) and by one GMRES cycle, the
    belief-propagation metric (messages converged from the trace message,
    then the closed-form solve), one product with the full metric, and the
    full metric by one GMRES cycle of gmres_m vectors."""
    from paper_2511_09546_amd import binding, inputs
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    o = binding.default_opts()
    o.prec = PRECS[prec]
    delta = w["delta"]
    out = {"workload": f"{name}, {prec} contractions, delta {delta}, "
                       f"K={w['grad_K']}", "gmres_m": gmres_m}

    def timed(key, f):
        t = time.perf_counter()
        r = f()
        out[key] = time.perf_counter() - t
        print(f"[precond] {key} {out[key]:.4f} s", file=sys.stderr,
              flush=True)
        return r

    with binding.Context(A, w["chi"], opts=o) as ctx:
        ctx.converge(w["tol"], w["n_iter"])
        _, g = timed("energy_grad_s", lambda: ctx.energy_grad(terms, True))
        timed("local_cg20_s", lambda: ctx.precond(g, delta, 0.0, 20))
        _, k, r = timed("local_gmres_s",
                        lambda: ctx.precond_gmres(g, delta, gmres_m))
        out["local_gmres_vectors"], out["local_gmres_resid"] = k, r
        timed("bp_converge_s", lambda: ctx.bp_converge(w["tol"], 500))
        timed("bp_apply_s", lambda: ctx.precond_bp(g, delta))
        timed("full_metric_product_s", lambda: ctx.metric_full(g))
        _, k, r = timed("full_gmres_s",
                        lambda: ctx.precond_full(g, delta, gmres_m))
        out["full_gmres_vectors"], out["full_gmres_resid"] = k, r
        out["peak_live_bytes"] = ctx.stats()["peak_live_bytes"]
    out["full_product_over_gradient"] = (out["full_metric_product_s"] /
                                         out["energy_grad_s"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="d6chi72")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16",
                                                       "fp64"])
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the plain FP64 and the other arithmetics")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--checkpoint", action="store_true",
                    help="checkpointed gradient (recompute each unrolled "
                         "iteration in the backward pass)")
    ap.add_argument("--serve-requests", type=int, default=128,
                    help="prefix of the seeded request stream to replay "
                         "(0: no serving leg)")
    ap.add_argument("--no-lbfgs", action="store_true")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the timing of every preconditioner")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is "
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
    base = None
    others = {}
    if args.prec != "fp64" and not args.no_fp64:
        base = run(name, "fp64", args.steps, args.warmup, ck, profile=False)
        oprec = "bf16" if args.prec == "fp32" else "fp32"
        others[oprec] = run(name, oprec, args.steps, args.warmup, ck)
        short = max(3, args.steps // 4)
        others["bf16x1"] = run(name, "bf16x1", short, args.warmup, ck,
                               profile=False)
        others["bf16_ladder"] = run(name, "bf16", short, args.warmup, ck,
                                    ladder=1, profile=False)

    timed, elapsed = head["timed"], head["elapsed"]
    n_g, t_g, fl_g, by_g = head["prof"][head["fam"]]
    n_w, t_w, fl_w, by_w = head["prof"][binding.PROF_WIDE]
    _, t_jac, _, _ = head["prof"][binding.PROF_JACOBI]
    _, t_perm, _, _ = head["prof"][binding.PROF_PERMUTE]
    ms = sorted(t["ms"] for t in timed)
    p = lambda q: ms[min(len(ms) - 1, int(round(q * (len(ms) - 1))))]  # noqa
    achieved = fl_g / t_g / 1e12 if t_g > 0 else 0.0
    ach_w = fl_w / t_w / 1e12 if t_w > 0 else 0.0
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
        # the dominant kernel: the 128 x 144-tile FP32 GEMM of the chi^2 D^8
        # network products (enlarged corners, renormalised edges, open
        # corners and their reverse passes), timed live with HIP events on
        # the library's stream; 2 M N K algorithmic flops per launch
        "roofline": {"bound": "mfma", "achieved": ach_w if n_w else achieved,
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": (ach_w if n_w else achieved) / peak,
                     "traffic": measured_traffic(args.prec),
                     "kernel": ("gemm_f32_lds_kernel, 128 x 144 tiles (FP32 "
                                "products of the chi^2 D^8 network "
                                "contractions)") if n_w else
                               f"{args.prec} matrix-core GEMM",
                     "launches": n_w,
                     "avg_launch_us": 1e6 * t_w / max(n_w, 1),
                     "algorithmic_flop_per_launch": fl_w / max(n_w, 1),
                     "algorithmic_bytes_per_launch": by_w / max(n_w, 1),
                     "share_of_step": t_w / head["elapsed_prof"],
                     "measured_over": f"{args.steps} profiled steps after "
                                      "the timed ones",
                     # every GEMM launch of the tensor-network contractions
                     # (all tile shapes; no SVD or complement-solve products)
                     "network_contractions": {
                         "achieved": ach_net, "frac": ach_net / peak,
                         "launches": n_net,
                         "share_of_gemm_time": t_net / max(t_g, 1e-30)},
                     # every matrix-core GEMM launch in the headline
                     # arithmetic, all shapes
                     "all_gemms": {
                         "achieved": achieved, "frac": achieved / peak,
                         "launches": n_g,
                         "avg_launch_us": 1e6 * t_g / max(n_g, 1),
                         "algorithmic_bytes_per_launch": by_g / max(n_g, 1),
                         "share_of_step": t_g / head["elapsed_prof"]}},
        "kernel_time_s": {"gemm": t_g, "jacobi": t_jac, "permute": t_perm},
        "svd_stats": head["stats"],
    }
    if base is not None:
        rb = arith_record(base, name)
        rb["cold_step_energy_abs_diff"] = (
            abs(head["infos"][0]["e"] - base["infos"][0]["e"])
            if head["infos"] and base["infos"] else None)
        hb = arith_record(head, name, base)
        rb["speedup"] = hb["speedup_vs_fp64"]
        rb["speedup_equal_work"] = hb["speedup_vs_fp64_equal_work"]
        out["plain_fp64"] = rb
        for k, r in others.items():
            out[f"{k}_contractions"] = arith_record(r, name, base)
    if args.serve_requests > 0:
        from paper_2511_09546_amd import serve
        out["serving"] = serve.replay(args.serve_requests, 20.0, 5,
                                      binding.FP32, 8, 230.0, check_solo=16)
        out["serving"]["prefix_of"] = 256
        # the warm-start variant: 8 states x 6 couplings, one state_key
        # per state
        out["serving_sweep"] = serve.replay(0, 20.0, 7, binding.FP32, 8,
                                            230.0, sweep=(8, 6))
    if not args.no_lbfgs:
        out["lbfgs"] = lbfgs_leg(name, args.prec, 3)
    if not args.no_precond:
        out["preconditioners"] = precond_leg(name, args.prec)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name, n_conv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
