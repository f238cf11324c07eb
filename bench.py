"""Throughput of the RTU-grid ELBO step on one MI355X.

Workload (default): a 200x200 image with 4x4 sub-rays per pixel (640k rays),
a 64x64 RTU source grid, a 21x21 PSF and 32 reparameterised latent samples per
ELBO step; lens drawn uniformly (theta_E in [0.6, 1.6]", q in [0.5, 0.95],
phi in [0, pi), |gamma| < 0.08); synthetic arc-like data (see
paper_2606_30620_amd/synth.py).

One step = one whole ELBO step of the variational fit on the device: draw the
32 samples z = mu + exp(rho) eps (Philox), evaluate each sample's loss and its
gradient (masked-ray quantiles and CDF knots, GP source by FFT, ray shooting
and transform, bilinear interpolation, sub-ray sum, PSF, chi^2, and the full
adjoint chain), then the ELBO value and the Adam update.

value = fwd+adjoint sample evaluations per second (32 per step).

Serving (the metric's second part): 64 requests of the serving mix (image
64..300 px, 2..4 sub-rays, 32..128 source, 0..3 subhaloes; one sample per
step, 200 ELBO + Adam steps each).  First all requests arrive at once
(capacity), then Poisson arrivals at 0.8 x that capacity; the fleet
(continuous batching in shared launches) and sequential plain fits (one at a
time) serve the same trace; fits/s and p50/p99 latency (completion - arrival)
of both are reported under "serving".  Progress goes to stderr.

    python bench.py [--gpus 1] [--steps 40] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ELBO fwd+adjoint evals/s (200^2 img, 64^2 src); served fits/s + p99 latency"

# Algorithmic FP32 operations per sub-ray (SIE + external shear, no
# subhaloes), counted from the formulas of the method: add, sub, mul, compare
# = 1, fused multiply-add = 2, and each of sqrt, reciprocal, floor, atan,
# atanh = 1.  The forward is the lens equation (45), the knot interval (4),
# the Hermite CDF on both axes (42), the bilinear sample (23), the sub-ray sum
# and position (5); the adjoint recomputes the forward with the derivative
# factors (118 + 52) and adds the bilinear adjoint with the source scatter
# (26), the knot moments (16) and the lens vector-Jacobian product (67).
FLOP_PER_RAY_FWD = 118
FLOP_PER_RAY_ADJ = 279
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s of
# unpacked FP32.  The published 157.3 counts packed (2 x FP32) instructions,
# which this build disables; both are reported.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

KERNEL_OF_STAGE = {"rays_adj": "kf_rays_adj<true>", "rays_fwd": "kf_rays_fwd<false>", "psf_fwd": "kf_psf",
                   "psf_adj": "kf_psf", "prep": "kf_prep", "post": "kf_post", "sample": "kf_sample",
                   "adam": "kf_adam"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_30620_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for this kernel and workload or the kernels changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel + "|" + workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(problem, budget_s: float):
    """The FP64 oracle on the host: fwd + gradient of as many of the workload's
    samples as fit in about budget_s seconds."""
    import torch

    from oracle import rtu_oracle as O
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        O.loss_grad_problem(problem, n % problem.batch)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "evals/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n} evaluations (fwd + gradient, FP64) cycling over the {problem.batch} samples of "
                      f"one ELBO step of the same workload, {dt:.1f} s"}


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serving_bench(n: int, steps: int) -> dict:
    """Fleet vs sequential plain fits on the serving mix (see module docstring)."""
    from paper_2606_30620_amd import serve

    # warm-up (kernel loading) on a few short requests
    serve.serve_fleet(serve.make_requests(8, float("inf"), steps=10, first_id=900000))
    cap_reqs = serve.make_requests(n, float("inf"), steps=steps, first_id=0)
    cap = serve.serve_fleet(cap_reqs, keep_results=True)
    out_of_domain = sum(1 for r in cap.results.values() if r[3] & 8)
    note(f"serving capacity {cap.summary()}")
    rate = 0.8 * cap.fits_per_s
    reqs = serve.make_requests(n, rate, steps=steps, first_id=10000, seed=505)
    fleet = serve.serve_fleet(reqs)
    note(f"serving fleet on the Poisson trace {fleet.summary()}")
    seq = serve.serve_sequential(reqs)
    note(f"serving sequential on the same trace {seq.summary()}")
    return {"workload": f"{n} requests of the serving mix, {steps} ELBO + Adam steps each, 1 sample per step",
            "capacity_fits_per_s": round(cap.fits_per_s, 2), "arrival_rate_per_s": round(rate, 2),
            "fleet": fleet.summary(), "sequential": seq.summary(),
            "speedup_fits_per_s": round(fleet.fits_per_s / seq.fits_per_s, 2),
            "fits_leaving_parameter_domain": out_of_domain}


def light_bench(steps: int, warmup: int, n_gauss: int = 5) -> dict:
    """The C2 ELBO step with the paper's multi-Gaussian lens light (5 Gaussians,
    App. A) added to the model: throughput and stage times."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2606_30620_amd import _lib, api, synth
    S = 32
    geom = dataclasses.replace(synth.CONFIGS["C2"], n_gauss=n_gauss)
    problem = synth.make_problem("C2", batch=S, geom=geom)
    plan = api.plan_for_problem(problem, max_batch=S)
    nl = geom.n_lens
    mu = np.concatenate([problem.lens[0], problem.ps[0], problem.latent[0].reshape(-1)]).astype(np.float32)
    rho = np.full(mu.size, math.log(0.1), np.float32)
    rho[:nl] = math.log(0.01)
    rho[nl:nl + 4] = math.log(0.02)
    fit = _lib.Fit(plan, S, mu, rho, lr=1e-2, seed=203, max_steps=warmup + steps + 6)
    fit.step(warmup)
    plan.profile_begin(5)
    fit.step(5)
    stages = plan.profile_end()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    fit.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    note(f"lens light ({n_gauss} Gaussians): {ms:.4f} ms/step")
    return {"workload": f"C2 + {n_gauss} lens-light Gaussians", "evals_per_s": round(S * 1e3 / ms, 1),
            "ms_per_step": round(ms, 4), "steps": steps,
            "stage_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-light", action="store_true", help="skip the lens-light section")
    ap.add_argument("--serve-only", action="store_true", help="only the serving section (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="after the run, copy this many bytes device-to-device 3 times (a plain copy "
                         "kernel of known size, to scale the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "the path shards by samples or fits with one gradient all-reduce per step, "
              "which is not built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_30620_amd import _lib, api, synth

    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_steps)}), flush=True)
        return

    S = 32
    problem = synth.make_problem("C2", batch=S)
    g = problem.geom
    rays = g.n_img ** 2 * g.supersample ** 2
    plan = api.plan_for_problem(problem, max_batch=S)
    mu = np.concatenate([problem.lens[0], problem.ps[0], problem.latent[0].reshape(-1)]).astype(np.float32)
    rho = np.full(mu.size, math.log(0.1), np.float32)
    rho[:7] = math.log(0.01)          # keep sampled lenses physical (|e| < 1, theta_E > 0)
    rho[7:11] = math.log(0.02)
    fit = _lib.Fit(plan, S, mu, rho, lr=1e-2, seed=202, max_steps=args.warmup + 2 * args.steps + 1)
    stream = torch.cuda.current_stream()
    fit.step(args.warmup)
    torch.cuda.synchronize()
    note(f"warm-up done ({args.warmup} ELBO steps of {S} samples)")

    # stage times of every stage: a short run with events around each stage
    # (the events themselves cost time, so this run is not the timed one)
    n_prof = min(args.steps, 10)
    plan.profile_begin(n_prof)
    fit.step(n_prof)
    stages = plan.profile_end()
    per_launch = {k: v[0] / v[1] for k, v in stages.items() if v[1] > 0}
    dom = max(per_launch, key=per_launch.get)

    # the timed run: events only around the dominant stage (its kernel duration
    # for the roofline), and around the whole run
    plan.profile_begin(args.steps, stages=[dom])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fit.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    dom_stage = plan.profile_end()[dom]
    ms_step = ms / args.steps
    note(f"timed {args.steps} ELBO steps: {ms_step:.4f} ms/step")
    value = S * args.steps / (ms / 1e3)

    # dominant kernel and its roofline (ALU-bound: see the design doc)
    per_launch[dom] = dom_stage[0] / dom_stage[1]
    flops = {"rays_adj": FLOP_PER_RAY_ADJ, "rays_fwd": FLOP_PER_RAY_FWD}.get(dom)
    workload = "C2"
    roof = None
    if flops:
        achieved = flops * rays * S / (per_launch[dom] * 1e-3) / 1e12
        traffic = measured_traffic(KERNEL_OF_STAGE[dom], workload)
        roof = {"bound": "alu", "kernel": KERNEL_OF_STAGE[dom], "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic, "avg_launch_ms": round(per_launch[dom], 4),
                "flop_per_launch": flops * rays * S,
                "frac_of_packed_peak": round(achieved / PEAK_FP32_PACKED_TFLOPS, 4)}
    _, _, trace = fit.read()
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: 200x200 image, 4x4 sub-rays (640k rays/sample), 64x64 RTU source, "
                               "21x21 PSF, 32 latent samples per ELBO step, SIE+shear",
                   "samples_per_step": S, "rays_per_sample": rays, "elbo_steps_per_s": round(1e3 / ms_step, 2),
                   "stage_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
                   "elbo_last": float(trace[-1]) if trace.size else None},
        "roofline": roof,
    }
    if not args.no_serve:
        line["serving"] = serving_bench(args.serve_requests, args.serve_steps)
    if not args.no_light:
        line["lens_light"] = light_bench(20, 5)
    if args.calib_copy:
        src = torch.ones(args.calib_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu:
        note("oracle on the host (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(problem, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
