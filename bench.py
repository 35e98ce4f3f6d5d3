#!/usr/bin/env python3
"""Throughput of the Born-rule probability path on one MI355X.

One step = one xf_probabilities call over the whole batch of the large-batch
workload: n = 100 modes (50 orbitals per spin), eta = 25 alpha + 25 beta,
three spin-restricted Haar rotation layers around two layers of 20 CPhase
gates each (k = 40, |theta| <= 0.05 uniform), t = 2^16 extent-sampled
trajectories for each of B = 10^5 output bitstrings at fixed (25, 25)
occupation; Raw Estimate in FP64, default evaluation (general determinant
lemma, two CPhase layers, one base per spin block).  Inputs are resident in
HBM before timing.

Prints one JSON line: value = sampled amplitude terms (bitstring x
trajectory) per second over the timed steps.  The call runs two stages, each
timed with the HIP events the library records on its stream: the sampler
(k_sample_entries) and the evaluation (k_gen_setup_wave + k_gen_eval, and
the fallback kernels: k_gen_setup for the bases the first left, k_gen_lu).
roofline: the sampler, the longest single kernel of the call (the
evaluation stage is split over the setup and pattern-pass kernels, each
shorter; see the kernel statistics in profiles/): achieved = the 32-bit
integer operations of the Philox4x32-10 blocks the sampling definition draws
(100 per block: per round two 32 x 32 -> 64-bit products, four XORs, two key
additions; counted on the device) over its time, against the chip's 32-bit
integer rate.  roofline_other_stage: the evaluation, achieved = its
algorithmic FP64 FLOPs (per bitstring and block the Gauss-Jordan inverse of
the base and the products X = M_B^-1 U and H = V X, per distinct flip
pattern an r x r elimination and the two-layer correction; counted on the
device) over its time, against the FP64 rate.  traffic = HBM bytes per
launch of the sampler from the committed rocprofv3 counters (null when its
sources have changed since).  cpu_baseline: the FP64 oracle on a bounded
sample of the same bitstrings, on all host threads and on one.  Extra keys:
the sampler's own rate; the mixed-precision run and both precisions' error
distributions against the stored oracle values of 1000 bitstrings of this
batch (with the terms' cancellation sum|w det| / |A|); the LUCJ workload
(n = 32), the exact-mode stress workload (n = 52, all 4096 terms; along the
term list's prefix tree, and again with every pattern's determinant on its
own), the forward and forward+adjoint time of the differentiation
workload (the backward taking the forward call's sampled patterns, and
drawing them again), and the latency of one exact outcome of random
extended-matchgate circuits with 16 CPhase layers (the paper's random
benchmark shape) for n = 8 to 36.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude terms/s (bitstring×Gaussian term) at stated rel err; fwd+bwd ms"
# 256 CUs x 2.4 GHz x 128 FP64 FLOP per clock per CU (vector FMA, and the
# FP64 matrix cores run at the same rate)
FP64_PEAK_TFLOPS = 78.6
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one 32-bit integer operation per
# lane and clock
INT32_PEAK_TOPS = 39.3
OPS_PER_PHILOX_BLOCK = 100
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sample_entries_large_batch.json")
# sources whose change invalidates the committed counters of the sampler
SAMPLER_SOURCES = ("sample_entries.h", "xf_device.h", "xf_internal.h", "k_lemma_gen.hip")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def sampler_source_hash() -> str:
    h = hashlib.sha256()
    for f in SAMPLER_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_12416_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of k_sample_entries from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size), or None if its sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("sources_sha256") != sampler_source_hash():
        return None
    return rec["bytes_per_launch"]


def timed_steps(plan, bits, mode, t, seed, out, steps, warmup):
    """Wall time of `steps` back-to-back calls (synchronised on both sides)."""
    import torch
    for _ in range(warmup):
        plan.probabilities(bits, mode, t, seed, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.probabilities(bits, mode, t, seed, out=out)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_split(plan, bits, mode, t, seed, out, steps):
    """Mean per-kernel times (sampler, evaluation) and per-call work over
    `steps` calls, from the HIP events the library records around its
    launches on the call's stream (read after each call, so this loop is
    kept apart from the timed one)."""
    sm, em = [], []
    for _ in range(steps):
        plan.probabilities(bits, mode, t, seed, out=out)
        wk = plan.last_work()
        sm.append(wk["sample_ms"])
        em.append(wk["eval_ms"])
    return float(np.mean(sm)), float(np.mean(em)), wk


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_oracle_rate(cfg: int, count: int, threads: int) -> dict:
    """The oracle on `count` bitstrings spread over workload `cfg`'s batch,
    in a child process with `threads` OpenMP threads."""
    code = (
        "import sys, time, json, numpy as np; sys.path.insert(0, %r)\n"
        "import oracle, workloads as W\n"
        "oracle.build(force=False)\n"
        "w = W.workload(%d)\n"
        "idx = np.linspace(0, w.B - 1, num=%d).astype(np.int64)\n"
        "t0 = time.perf_counter(); oracle.run_workload(w, index=idx); dt = time.perf_counter() - t0\n"
        "print(json.dumps({'seconds': dt, 'count': len(idx), 't': w.t}))\n" % (ROOT, cfg, count))
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(cfg: int, seconds: float) -> dict:
    """Oracle rate on all host threads and on one thread, each on a sample
    sized to take about `seconds` (calibrated on a few bitstrings)."""
    threads = host_threads()
    probe = cpu_oracle_rate(cfg, 4, threads)
    # the probe's 4 bitstrings ran side by side: one bitstring on one thread
    per1 = probe["seconds"] * min(threads, 4) / 4
    n_all = int(max(threads, min(4000, seconds * threads / max(per1, 1e-6))))
    full = cpu_oracle_rate(cfg, n_all, threads)
    n_one = int(max(2, min(200, seconds / max(per1, 1e-6))))
    one = cpu_oracle_rate(cfg, n_one, 1)
    t = full["t"]
    return {"value": full["count"] * t / full["seconds"], "unit": "terms/s", "cores": threads, "kind": "oracle",
            "sample": f"{full['count']} of the batch's bitstrings (evenly spread), all t={t} trajectories each, "
                      f"{full['seconds']:.1f} s on {threads} threads",
            "cpu": cpu_model(),
            "one_thread": {"value": one["count"] * t / one["seconds"], "unit": "terms/s",
                           "sample": f"{one['count']} bitstrings, {one['seconds']:.1f} s"}}


def err_stats(p, ref) -> dict:
    e = np.abs(p - ref) / np.where(ref > 0, ref, 1.0)
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "median": float(np.median(e)),
            "count": int(len(e))}


def run_headline(X, W, args, dev):
    import torch
    w = W.workload(5)
    log(f"workload: {w.name}")
    bits = X.bits_tensor(w.bits, dev)
    out = torch.empty(w.B, dtype=torch.float64, device=dev)
    res = {}
    for prec in ("fp64", "mixed"):
        plan = X.Plan(w.rot, w.pairs, w.layer, w.theta, w.input_bits, prec, device=0)
        steps = args.steps if prec == "fp64" else max(2, args.steps // 2)
        wall = timed_steps(plan, bits, "approx", w.t, w.seed, out, steps, args.warmup)
        sms, ems, wk = kernel_split(plan, bits, "approx", w.t, w.seed, out, max(2, steps // 2))
        res[prec] = dict(wall=wall, steps=steps, sample_ms=sms, eval_ms=ems, work=wk,
                         p=out.cpu().numpy().copy())
        log(f"{prec}: {steps} steps, {wall * 1e3 / steps:.3f} ms/step; sampler {sms:.3f} ms, "
            f"evaluation {ems:.3f} ms; {wk['determinants']} patterns, general={wk['general']}, "
            f"fp32 bases {wk['fp32_bases']}")
        plan.close()
    return w, res


def run_exact_stress(X, W, args, dev) -> int:
    """The exact stress workload alone (the command its kernel profile is
    taken with): ms per call, terms/s, the evaluation kernels' time."""
    import torch
    w = W.workload(3)
    bits = X.bits_tensor(w.bits, dev)
    out = torch.empty(w.B, dtype=torch.float64, device=dev)
    plan = X.Plan(w.rot, w.pairs, w.layer, w.theta, w.input_bits, "fp64", device=0)
    wall = timed_steps(plan, bits, w.mode, w.t, w.seed, out, args.steps, args.warmup)
    wk = plan.last_work()
    terms = w.B * (1 << w.k)
    print(json.dumps({"workload": w.name, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": wall * 1e3 / args.steps, "value": terms * args.steps / wall,
                      "unit": "terms/s", "dtype": "f64", "eval_ms_last_call": wk["eval_ms"],
                      "tree_bitstrings": wk["tree_bitstrings"], "flops_per_call": wk["flops"]}), flush=True)
    plan.close()
    return 0


def run_extras(X, W, args, dev):
    """Configs other than the headline: ms per call and terms/s."""
    import torch
    extra = {}
    for cfg, key in ((2, "lucj_n32"), (3, "exact_stress_n52")):
        w = W.workload(cfg)
        bits = X.bits_tensor(w.bits, dev)
        out = torch.empty(w.B, dtype=torch.float64, device=dev)
        plan = X.Plan(w.rot, w.pairs, w.layer, w.theta, w.input_bits, "fp64", device=0)
        steps = max(3, args.steps)
        wall = timed_steps(plan, bits, w.mode, w.t, w.seed, out, steps, args.warmup)
        terms = w.B * (w.t if w.mode == "approx" else (1 << w.k))
        wk = plan.last_work()
        ev = "general lemma" if wk["general"] else ("lemma" if wk["lemma"] else "LU")
        if wk["tree_bitstrings"]:
            ev += f", prefix tree ({wk['tree_bitstrings']} of {w.B} bitstrings)"
        extra[key] = {"workload": w.name, "ms_per_step": wall * 1e3 / steps, "value": terms * steps / wall,
                      "unit": "terms/s", "dtype": "f64", "evaluation": ev}
        log(f"{key}: {wall * 1e3 / steps:.3f} ms/step, {terms * steps / wall:.3e} terms/s ({ev})")
        if wk["tree_bitstrings"]:
            # the same call with every pattern's determinant on its own
            plan.set_evaluation("patterns")
            wall2 = timed_steps(plan, bits, w.mode, w.t, w.seed, out, steps, args.warmup)
            extra[key]["per_pattern_ms_per_step"] = wall2 * 1e3 / steps
            log(f"{key} per pattern: {wall2 * 1e3 / steps:.3f} ms/step")
        plan.close()
    # differentiation workload: forward (log p) and forward + adjoint
    w = W.workload(4)
    bits = X.bits_tensor(w.bits, dev)
    g = torch.full((w.B,), 1.0 / w.B, dtype=torch.float64, device=dev)
    out = torch.empty(w.B, dtype=torch.float64, device=dev)
    lp = torch.empty(w.B, dtype=torch.float64, device=dev)
    d = {"workload": w.name}
    rot = w.rot if w.rot is not None else X.spin_rotations(w.gens)
    for prec in ("fp64", "mixed"):
        plan = X.Plan(rot, w.pairs, w.layer, w.theta, w.input_bits, prec, device=0)
        steps = max(3, args.steps)
        for _ in range(args.warmup):
            plan.probabilities(bits, "approx", w.t, w.seed, out=out, logp=lp)
            plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.probabilities(bits, "approx", w.t, w.seed, out=out, logp=lp)
        torch.cuda.synchronize()
        fwd = (time.perf_counter() - t0) / steps
        fb = {}
        # the backward draws the samples again, then takes the forward call's
        for reuse in (False, True):
            plan.set_reuse_samples(reuse)
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.probabilities(bits, "approx", w.t, w.seed, out=out, logp=lp)
                plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
            torch.cuda.synchronize()
            fb[reuse] = (time.perf_counter() - t0) / steps
            assert plan.last_work()["backward_reused"] == reuse
        d[prec] = {"fwd_ms": fwd * 1e3, "fwd_bwd_ms": fb[True] * 1e3,
                   "fwd_bwd_terms_per_s": w.B * w.t / fb[True],
                   "fwd_bwd_ms_backward_resampling": fb[False] * 1e3,
                   "backward_lemma": bool(plan.last_work()["backward_lemma"])}
        log(f"differentiation {prec}: forward {fwd * 1e3:.3f} ms, forward+adjoint {fb[True] * 1e3:.3f} ms "
            f"({fb[False] * 1e3:.3f} ms with the backward drawing the samples again)")
        plan.close()
    extra["differentiation_n32"] = d
    # the paper's random-circuit benchmark shape (Sec. V-A): extended
    # matchgate circuits of n qubits, 16 CPhase gates and n - 1 matchgates
    # per layer; exact probability of one outcome near the input, per call
    lat = {}
    for n in (8, 16, 24, 32, 36):
        eta = n // 2
        gates, inp, _ = W.random_gate_circuit(85 + n, n, eta, 16, n - 1, theta_scale=1.0, max_bits=4)
        rot, pairs, layer, theta = X.circuit_from_gates(n, gates)
        one = X.bits_tensor(W.nearby_outcomes(7 + n, n, range(eta), 1, hops=4), dev)
        o1 = torch.empty(1, dtype=torch.float64, device=dev)
        plan = X.Plan(rot, pairs, layer, theta, inp, "fp64", device=0)
        for _ in range(3):
            plan.probabilities(one, "exact", out=o1)
        torch.cuda.synchronize()
        ts = []
        for _ in range(20):
            t0 = time.perf_counter()
            plan.probabilities(one, "exact", out=o1)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        lat[f"n{n}"] = float(np.median(ts)) * 1e3
        plan.close()
    extra["random_circuits_one_outcome_ms"] = {
        "workload": "random extended-matchgate circuits, 16 CPhase layers, n-1 matchgates per layer, "
                    "eta = n/2, exact probability of one outcome (median of 20 calls)", **lat}
    log("one outcome, 16 CPhase layers: " + ", ".join(f"{k} {v:.3f} ms" for k, v in lat.items()))
    return extra


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate wall time of each oracle baseline sample")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="after the timed region, a fill and a sum over this many MiB (the reference "
                         "kernels that scale the HBM byte counters)")
    ap.add_argument("--exact-stress", action="store_true",
                    help="only the exact-mode stress workload (n = 52, eta = 26, all 4096 terms of 4096 "
                         "bitstrings, along the term list's prefix tree): one JSON line of its own")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the path shards by "
              "bitstring with no communication, and no multi-GPU run is part of this measurement.",
              file=sys.stderr)
        return 2

    import torch
    import paper_2511_12416_amd as X
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.exact_stress:
        return run_exact_stress(X, W, args, dev)
    w, res = run_headline(X, W, args, dev)
    r = res["fp64"]
    terms = w.B * w.t
    value = terms * r["steps"] / r["wall"]
    flops = r["work"]["flops"]
    eval_tf = flops / (r["eval_ms"] * 1e-3) / 1e12
    int_ops = r["work"]["philox_blocks"] * OPS_PER_PHILOX_BLOCK
    samp_tops = int_ops / (r["sample_ms"] * 1e-3) / 1e12
    sampler_roof = {"bound": "alu", "achieved": samp_tops, "peak": INT32_PEAK_TOPS, "unit": "TOP/s",
                    "frac": samp_tops / INT32_PEAK_TOPS, "traffic": measured_traffic(),
                    "kernel": "k_sample_entries", "kernel_ms": r["sample_ms"], "ops_per_launch": int_ops,
                    "philox_blocks_per_launch": r["work"]["philox_blocks"],
                    "ops": "32-bit integer operations of the Philox4x32-10 blocks the sampling definition draws "
                           "(100 per block), counted on the device"}
    eval_roof = {"bound": "alu", "achieved": eval_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": eval_tf / FP64_PEAK_TFLOPS, "traffic": None,
                 "kernel": "k_gen_setup_wave + k_gen_eval (+ fallback kernels k_gen_setup, k_gen_lu)",
                 "kernel_ms": r["eval_ms"], "flops_per_launch": flops,
                 "flops": "algorithmic FP64 FLOPs counted on the device: per bitstring and block in-place "
                          "Gauss-Jordan of the m x m base (8 m^2 (m - 1) and the pivot steps), X = M_B^-1 U (8 m^2 kb), H = V X (8 kb^2 m), per distinct pattern and "
                          "block an r x r LU plus the two-layer correction"}
    # the sampler is one kernel; the evaluation stage is several (setup, pattern pass, fallbacks)
    dominant, other = sampler_roof, eval_roof

    # errors against the stored oracle values of 1000 bitstrings of this batch
    with open(os.path.join(ROOT, "tests", "golden", "config5_subset_oracle.json")) as f:
        gold = json.load(f)
    assert gold["workload"] == w.name and gold["t"] == w.t and gold["seed"] == w.seed
    gidx = np.asarray(gold["index"], dtype=np.int64)
    gref = np.asarray(gold["prob"])
    errors = {prec: err_stats(res[prec]["p"][gidx], gref) for prec in res}
    if "abs_sum" in gold:
        amp = np.hypot(np.asarray(gold["amp_re"]), np.asarray(gold["amp_im"]))
        kap = np.asarray(gold["abs_sum"]) / np.where(amp > 0, amp, np.inf)
        errors["cancellation_sum_abs_over_abs_sum"] = {"median": float(np.median(kap)),
                                                       "p99": float(np.quantile(kap, 0.99)),
                                                       "max": float(kap.max())}

    if args.calibrate_copy_mb > 0:
        # reference kernels of known traffic: a fill (writes nbytes) and a sum
        # (reads nbytes)
        nbytes = args.calibrate_copy_mb << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
        a.fill_(1.0)
        torch.cuda.synchronize()
        total = float(a.sum())
        torch.cuda.synchronize()
        log(f"calibration: fill of {nbytes} bytes, sum over {nbytes} bytes ({total:.0f})")
        del a
    extras = {} if args.no_extras else run_extras(X, W, args, dev)
    base = None if args.no_cpu else cpu_baseline(5, args.cpu_seconds)
    m = res["mixed"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / r["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "eta": w.eta, "k": w.k, "cphase_layers": 2, "t": w.t,
                   "B": w.B, "mode": "raw_estimate", "precision": "fp64",
                   "evaluation": "general determinant lemma, spin blocks", "parallelism": "single GPU"},
        "rel_err_vs_oracle": errors,
        "roofline": dominant,
        "roofline_other_stage": other,
        "kernels": {"k_sample_entries": {"ms": r["sample_ms"], "trajectories_per_s": terms / (r["sample_ms"] * 1e-3)},
                    "k_gen_eval": {"ms": r["eval_ms"],
                                   "patterns_per_s": r["work"]["determinants"] / (r["eval_ms"] * 1e-3),
                                   "patterns_per_step": r["work"]["determinants"]}},
        "mixed_precision": {"value": terms * m["steps"] / m["wall"], "unit": "terms/s",
                            "ms_per_step": m["wall"] * 1e3 / m["steps"], "eval_ms": m["eval_ms"],
                            "fp32_bases": m["work"]["fp32_bases"], "bases": 2 * w.B},
        "other_workloads": extras,
        "cpu_baseline": base,
        "device": torch.cuda.get_device_name(dev),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
