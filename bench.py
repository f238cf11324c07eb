"""Throughput of the RTU-grid ELBO step on one MI355X.

Headline workload (C2): a 200x200 image with 4x4 sub-rays per pixel (640k
rays), a 64x64 RTU source grid, a 21x21 PSF and 32 reparameterised latent
samples per ELBO step; lens drawn uniformly (theta_E in [0.6, 1.6]", q in
[0.5, 0.95], phi in [0, pi), |gamma| < 0.08); synthetic arc-like data (see
paper_2606_30620_amd/synth.py).

One step = one whole ELBO step of the variational fit on the device: draw the
32 samples z = mu + exp(rho) eps (Philox), evaluate each sample's loss and its
gradient (masked-ray quantiles and CDF knots, GP source by FFT, ray shooting
and transform, bilinear interpolation, sub-ray sum, PSF, chi^2, and the full
adjoint chain), then the ELBO value and the Adam update.

value = fwd+adjoint sample evaluations per second (32 per step).

Further sections of the JSON line:
* "c3": the substructure case (400x400, 3x3 sub-rays, 128x128 source, 31x31
  PSF, 9 truncated-NFW subhaloes, 32 samples per step): throughput and the
  roofline of its dominant kernel.
* "c4": the large single fit (512x512, 4x4 sub-rays, 256x256 source): 500 Adam
  iterations with 64 samples per launch against 500 with one sample per
  launch (wall time, ELBO trajectory), and the cost of one 64-sample step done
  as 64 single-sample evaluations.
* "serving": 1000 requests of the serving mix (image 64..300 px, 2..4
  sub-rays, 32..128 source, 0..3 subhaloes; one sample per step, 200 ELBO +
  Adam steps each).  First all at once (capacity), then Poisson arrivals at
  0.5, 0.8 and 0.95 x that capacity served by the fleet (continuous batching in
  shared launches), and the 0.5 trace served by sequential plain fits (one at
  a time); fits/s, p50/p99 latency (completion - arrival) and valid fits.
* "lens_light": C2 with the paper's 5 lens-light Gaussians.
* "cpu_baseline": the FP64 oracle on the host, single- and all-core.
Progress goes to stderr.

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
# Per truncated-NFW subhalo and sub-ray: the deflection (offset, radius,
# reciprocal, h(X) with its logarithm and atan/atanh polynomial, the radial
# factor) 47; the adjoint adds the deflection again and its vector-Jacobian
# product (h'(X), the four parameter terms) 87.
FLOP_PER_SUB_FWD = 47
FLOP_PER_SUB_ADJ = 87
# MI355X's published FP32 vector peak is 157.3 TFLOP/s (it counts packed
# two-wide FP32 instructions); 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
# = 78.6 TFLOP/s is the unpacked rate, which is what this build can issue
# (packed FP32 is disabled).  frac is against the published peak; the
# fraction of the unpacked rate is reported beside it.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

KERNEL_OF_STAGE = {"rays_adj": "kf_rays_adj<true, false>", "rays_fwd": "kf_rays_fwd<false>", "psf_fwd": "kf_psf",
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


def _cpu_info() -> dict:
    """CPU model, logical CPUs available to this process and physical cores."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "physical_cores": len(cores) or None}


def cpu_baseline(problem, budget_s: float):
    """The FP64 oracle on the host: median time of one fwd + gradient
    evaluation, cycling over the workload's samples, with one thread and with
    every thread torch uses; each run takes about budget_s / 2 seconds."""
    import torch

    from oracle import rtu_oracle as O

    def run(threads):
        old = torch.get_num_threads()
        torch.set_num_threads(threads)
        try:
            times = []
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < budget_s / 2 or len(times) < 3:
                t1 = time.perf_counter()
                O.loss_grad_problem(problem, len(times) % problem.batch)
                times.append(time.perf_counter() - t1)
            return float(np.median(times)), len(times)
        finally:
            torch.set_num_threads(old)

    import numpy as np
    info = _cpu_info()
    n_all = torch.get_num_threads()
    t_one, k_one = run(1)
    t_all, k_all = run(n_all)
    return {"value": round(1.0 / t_all, 3), "unit": "evals/s", "cores": n_all, "kind": "oracle",
            "single_core_evals_per_s": round(1.0 / t_one, 3), **info,
            "sample": f"C2 fwd + gradient evaluations (FP64 PyTorch on the CPU), cycling over the "
                      f"{problem.batch} samples of one ELBO step: median of {k_all} with {n_all} threads "
                      f"and of {k_one} with 1 thread"}


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _guide(problem, n_lens, lat_mean=True):
    import numpy as np
    lat = problem.latent[0].reshape(-1) if lat_mean else np.zeros(problem.latent[0].size)
    mu = np.concatenate([problem.lens[0], problem.ps[0], lat]).astype(np.float32)
    rho = np.full(mu.size, math.log(0.1), np.float32)
    rho[:n_lens] = math.log(0.01)          # keep sampled lenses physical (|e| < 1, theta_E > 0)
    rho[n_lens:n_lens + 4] = math.log(0.02)
    return mu, rho


def fit_bench(problem, S, steps, warmup, seed, workload, lr=1e-2, n_sub=0):
    """Timed ELBO steps of a fit of S samples per step: ms per step, stage
    times (a short profiled run), and the dominant stage's average launch time
    (events around that stage only in the timed run)."""
    import torch

    from paper_2606_30620_amd import _lib, api
    g = problem.geom
    plan = api.plan_for_problem(problem, max_batch=S)
    mu, rho = _guide(problem, g.n_lens)
    fit = _lib.Fit(plan, S, mu, rho, lr=lr, seed=seed, max_steps=warmup + 2 * steps + 1, n_sub=n_sub)
    stream = torch.cuda.current_stream()
    fit.step(warmup)
    torch.cuda.synchronize()
    n_prof = min(steps, 10)
    plan.profile_begin(n_prof)
    fit.step(n_prof)
    stages = plan.profile_end()
    per_launch = {k: v[0] / v[1] for k, v in stages.items() if v[1] > 0}
    dom = max(per_launch, key=per_launch.get)
    plan.profile_begin(steps, stages=[dom])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fit.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    dom_stage = plan.profile_end()[dom]
    per_launch[dom] = dom_stage[0] / dom_stage[1]
    _, _, trace = fit.read()
    # sub-rays on the grid in the last step's gradient pass, summed over its samples
    ongrid = sum(float(plan.debug_fetch(_lib.DBG_ONGRID, b)[0]) for b in range(S))
    note(f"{workload}: {ms / steps:.4f} ms/step")
    return {"ms_per_step": ms / steps, "stages": stages, "dominant": dom, "dom_ms": per_launch[dom],
            "elbo_last": float(trace[-1]) if trace.size else None, "status": fit.status_acc(),
            "ongrid": ongrid}


def roofline(dom, dom_ms, rays, S, n_sub, workload, ongrid, kernel=None):
    """The forward must shoot every sub-ray; the adjoint of a sub-ray off the
    zero-bordered source grid is zero, so its algorithmic work is that of the
    sub-rays on the grid (counted by the gradient pass).  The per-ray rate over
    all sub-rays is reported beside it."""
    flops = {"rays_adj": FLOP_PER_RAY_ADJ + FLOP_PER_SUB_ADJ * n_sub,
             "rays_fwd": FLOP_PER_RAY_FWD + FLOP_PER_SUB_FWD * n_sub}.get(dom)
    if not flops:
        return None
    units = ongrid if dom == "rays_adj" else rays * S
    achieved = flops * units / (dom_ms * 1e-3) / 1e12
    every = flops * rays * S / (dom_ms * 1e-3) / 1e12
    kernel = kernel or KERNEL_OF_STAGE[dom]
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": measured_traffic(kernel, workload), "avg_launch_ms": round(dom_ms, 4),
            "units": "sub-rays on the source grid" if dom == "rays_adj" else "sub-rays",
            "units_per_launch": int(units), "flop_per_unit": flops, "flop_per_launch": int(flops * units),
            "ongrid_fraction": round(ongrid / (rays * S), 4),
            "frac_of_unpacked_fp32": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
            "frac_counting_every_sub_ray": round(every / PEAK_FP32_TFLOPS, 4)}


def c3_bench(steps: int, warmup: int) -> dict:
    """C3: 400x400, 3x3 sub-rays, 128x128 source, 31x31 PSF, truncated-NFW
    subhaloes (seed 303: 9 of them), 32 samples per ELBO step."""
    from paper_2606_30620_amd import synth
    S = 32
    problem = synth.make_problem("C3", batch=S, seed=303)
    g = problem.geom
    ns = int(problem.n_sub[0])
    rays = g.n_img ** 2 * g.supersample ** 2
    r = fit_bench(problem, S, steps, warmup, 303, "C3", lr=1e-3, n_sub=ns)
    return {"workload": f"C3: 400x400 image, 3x3 sub-rays ({rays} rays/sample), 128x128 RTU source, 31x31 PSF, "
                        f"{ns} truncated NFW subhaloes, {S} latent samples per ELBO step",
            "evals_per_s": round(S * 1e3 / r["ms_per_step"], 1), "ms_per_step": round(r["ms_per_step"], 4),
            "steps": steps, "status_or": r["status"],
            "stage_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["stages"].items() if v[1]},
            "roofline": roofline(r["dominant"], r["dom_ms"], rays, S, ns, "C3", r["ongrid"],
                                 # 128 x 128 grid (d loss / d s in global memory), subhaloes
                                 kernel="kf_rays_adj_sub<false, false>" if r["dominant"] == "rays_adj" else None)}


def c4_bench(iters: int) -> dict:
    """C4: the 500-iteration Adam fit at 512x512 / 256x256 with 64 samples per
    launch against the plain one-sample-per-launch path: (a) the same fit with
    one sample per step, (b) one 64-sample step evaluated as 64 single-sample
    calls."""
    import numpy as np
    import torch

    from paper_2606_30620_amd import _lib, api, synth
    problem = synth.make_problem("C4", batch=64)
    g = problem.geom
    out = {"workload": "C4: 512x512 image, 4x4 sub-rays (4.2M rays/sample), 256x256 RTU source, 21x21 PSF, "
                       f"Matern n = 1.5; {iters} Adam iterations, lr 1e-3, latent guide mean 0",
           "iterations": iters}
    marks = sorted(set(list(range(0, iters, max(iters // 10, 1))) + [iters - 1]))
    for S in (64, 1):
        plan = api.plan_for_problem(problem, max_batch=S)
        mu, rho = _guide(problem, g.n_lens, lat_mean=False)
        fit = _lib.Fit(plan, S, mu, rho, lr=1e-3, seed=404, max_steps=iters + 2)
        fit.step(2)                                  # kernel loading
        torch.cuda.synchronize()
        fit2 = _lib.Fit(plan, S, mu, rho, lr=1e-3, seed=404, max_steps=iters)
        t0 = time.perf_counter()
        fit2.step(iters)
        _, _, trace = fit2.read()                    # synchronises
        wall = time.perf_counter() - t0
        st = fit2.status_acc()
        tail = trace[-50:]
        out[f"S{S}"] = {"samples_per_launch": S, "wall_s": round(wall, 3), "ms_per_iteration": round(1e3 * wall / iters, 4),
                        "sample_evals_per_s": round(S * iters / wall, 1), "status_or": st,
                        "elbo": {str(k): round(float(trace[k]), 2) for k in marks},
                        "elbo_last50_mean": round(float(np.mean(tail)), 2),
                        "elbo_last50_std": round(float(np.std(tail)), 2)}
        note(f"C4 fit, {S} samples per launch: {wall:.3f} s for {iters} iterations")
        del fit, fit2, plan
    # one 64-sample step's evaluations as 64 single-sample plain calls
    plan1 = api.plan_for_problem(problem, max_batch=1)
    lens, ps, lat, nsub = api.device_inputs(problem)
    outs = [api.evaluate(plan1, lens[:1], ps[:1], lat[:1], nsub[:1]) for _ in range(2)]   # warm
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        for s in range(64):
            api.evaluate(plan1, lens[s:s + 1], ps[s:s + 1], lat[s:s + 1], nsub[s:s + 1])
    torch.cuda.synchronize()
    ms64 = 1e3 * (time.perf_counter() - t0) / reps
    plan64 = api.plan_for_problem(problem, max_batch=64)
    api.evaluate(plan64, lens, ps, lat, nsub)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        api.evaluate(plan64, lens, ps, lat, nsub)
    torch.cuda.synchronize()
    msb = 1e3 * (time.perf_counter() - t0) / reps
    out["evaluations_of_64_samples"] = {"one_launch_ms": round(msb, 3), "64_single_sample_calls_ms": round(ms64, 3),
                                        "speedup": round(ms64 / msb, 2)}
    out["speedup_per_sample_eval"] = round(out["S64"]["sample_evals_per_s"] / out["S1"]["sample_evals_per_s"], 2)
    note(f"C4: 64 evaluations in one launch {msb:.2f} ms, as 64 single-sample calls {ms64:.2f} ms")
    return out


def serving_bench(n: int, steps: int, loads=(0.5, 0.8, 0.95), seq_load: float = 0.5) -> dict:
    """Fleet vs sequential plain fits on the serving mix (see module docstring)."""
    from paper_2606_30620_amd import _lib, serve

    # one fleet for every run, as a serving process keeps it: its arena, its
    # pinned staging pool and its work-list buffers are sized by a warm-up
    # burst of short requests (which also loads the kernels)
    fleet = _lib.Fleet(8 << 30, max_fits=512, sync_every=4)
    serve.serve_fleet(serve.make_requests(600, float("inf"), steps=5, first_id=900000), fleet=fleet)
    cap = serve.serve_fleet(serve.make_requests(n, float("inf"), steps=steps, first_id=0), fleet=fleet,
                            keep_results=True)
    note(f"serving capacity {cap.summary()}")
    out = {"workload": f"{n} requests of the serving mix, {steps} ELBO + Adam steps each, 1 sample per step, "
                       "subhalo scales fitted in log space",
           "capacity": cap.summary(), "capacity_fits_per_s": round(cap.fits_per_s, 2), "loads": {}}
    for lam in loads:
        rate = lam * cap.fits_per_s
        reqs = serve.make_requests(n, rate, steps=steps, first_id=10000, seed=505)
        res = serve.serve_fleet(reqs, fleet=fleet, keep_results=True)
        entry = {"arrival_rate_per_s": round(rate, 2), "fleet": res.summary()}
        note(f"serving fleet at {lam} x capacity {res.summary()}")
        if abs(lam - seq_load) < 1e-9:
            seq = serve.serve_sequential(reqs, keep_results=True)
            note(f"serving sequential on the same trace {seq.summary()}")
            entry["sequential"] = seq.summary()
            entry["speedup_fits_per_s"] = round(res.fits_per_s / seq.fits_per_s, 2)
        out["loads"][str(lam)] = entry
    return out


def light_bench(steps: int, warmup: int, n_gauss: int = 5) -> dict:
    """The C2 ELBO step with the paper's multi-Gaussian lens light (5 Gaussians,
    App. A) added to the model: throughput and stage times."""
    import dataclasses

    from paper_2606_30620_amd import synth
    S = 32
    geom = dataclasses.replace(synth.CONFIGS["C2"], n_gauss=n_gauss)
    problem = synth.make_problem("C2", batch=S, geom=geom)
    r = fit_bench(problem, S, steps, warmup, 203, f"C2 + {n_gauss} lens-light Gaussians")
    return {"workload": f"C2 + {n_gauss} lens-light Gaussians", "evals_per_s": round(S * 1e3 / r["ms_per_step"], 1),
            "ms_per_step": round(r["ms_per_step"], 4), "steps": steps,
            "stage_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["stages"].items() if v[1]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-light", action="store_true", help="skip the lens-light section")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the RTU vs uniform grid N_src sweep")
    ap.add_argument("--c4-iters", type=int, default=500)
    ap.add_argument("--serve-only", action="store_true", help="only the serving section (for profiling)")
    ap.add_argument("--c3-only", action="store_true", help="only the C3 section (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=1000)
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

    import torch

    from paper_2606_30620_amd import synth

    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_steps)}), flush=True)
        return
    if args.c3_only:
        print(json.dumps({"c3": c3_bench(args.steps, args.warmup)}), flush=True)
        return

    S = 32
    problem = synth.make_problem("C2", batch=S)
    g = problem.geom
    rays = g.n_img ** 2 * g.supersample ** 2
    r = fit_bench(problem, S, args.steps, args.warmup, 202, "C2")
    ms_step = r["ms_per_step"]
    value = S * 1e3 / ms_step
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: 200x200 image, 4x4 sub-rays (640k rays/sample), 64x64 RTU source, "
                               "21x21 PSF, 32 latent samples per ELBO step, SIE+shear",
                   "samples_per_step": S, "rays_per_sample": rays, "elbo_steps_per_s": round(1e3 / ms_step, 2),
                   "stage_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["stages"].items() if v[1]},
                   "elbo_last": r["elbo_last"]},
        "roofline": roofline(r["dominant"], r["dom_ms"], rays, S, 0, "C2", r["ongrid"]),
    }
    if not args.no_c3:
        line["c3"] = c3_bench(10, 3)
    if not args.no_c4:
        line["c4"] = c4_bench(args.c4_iters)
    if not args.no_serve:
        line["serving"] = serving_bench(args.serve_requests, args.serve_steps)
    if not args.no_light:
        line["lens_light"] = light_bench(20, 5)
    if not args.no_sweep:
        from paper_2606_30620_amd import sweep
        note("N_src sweep, RTU and uniform grids")
        line["nsrc_sweep"] = sweep.nsrc_sweep()
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
