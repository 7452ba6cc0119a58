#!/usr/bin/env python3
"""Benchmark of the GP-FVM hot path on one MI355X.

One step = one whole pass of the hot path for the 2D+time wave workload
(u_tt = div(c^2 grad u), c^2 piecewise constant per cell from a seeded smooth
bathymetry; 64 x 128 x 128 volumes + 16384 initial/boundary points):
assemble (closed-form factors, point-block Cholesky and inverse, Kronecker
plans), 200 early-terminated IterGP iterations with CG actions, and the
posterior mean and combined variance on the 8 x 128 x 128 grid of cell
centres.  This is the largest configuration that fits one GPU.  Inputs are
synthetic and seeded; host arrays are a few MB, so the step is device-bound.
The advection-diffusion 128 x 128 solve to 1e-8 (the launch-bound small
configuration), its coarse warm start and the serving trace are reported as
secondary blocks.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--c2-steps", type=int, default=20,
                    help="timed steps of the advection-diffusion 128x128 block (0 = skip)")
    ap.add_argument("--roofline-workload", choices=["advdiff", "wave", "heat2d"], default="wave",
                    help="with --roofline-only: wave 64x128x128 with 1 rhs, advdiff 128^2 or heat 64^3 with 64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mv-reps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the serving trace (0 = skip the serving measurement)")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-max-batch", type=int, default=16,
                    help="most requests of one operator solved together (1 = no batching)")
    ap.add_argument("--serve-rates", default="0.8",
                    help="comma-separated arrival rates as fractions of the saturated throughput")
    ap.add_argument("--serving-only", action="store_true", help="only the serving measurement")
    ap.add_argument("--serve-coarse", type=int, default=0,
                    help="also serve with every solve warm-started on a coarse scheme of at most this many "
                         "cells (0 = skip)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the volume-Gram matvec measurement (the command profiled under rocprofv3)")
    ap.add_argument("--extra-rooflines", action="store_true",
                    help="also measure the 64x128x128 wave volume matvec with one right-hand side and the "
                         "64^3 heat volume matvec with 64")
    ap.add_argument("--large-timing", action="store_true",
                    help="only time the wave 64x128x128 problem: assemble, 200 IterGP iterations, posterior")
    ap.add_argument("--c3-steps", type=int, default=2,
                    help="timed steps of the 2-D heat 64^3 block (assemble + 200 IterGP + posterior, float64 and "
                         "mixed; 0 = skip)")
    ap.add_argument("--sw-steps", type=int, default=1,
                    help="timed steps of the shallow-water system block (0: skip)")
    ap.add_argument("--sw-iters", type=int, default=1250,
                    help="IterGP iterations of the shallow-water block (the paper's CG budget)")
    ap.add_argument("--sw-only", action="store_true", help="only the shallow-water block (for profiling)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only the advection-diffusion block with its mixed-precision measurement (profiling)")
    ap.add_argument("--mixed-steps", type=int, default=5,
                    help="steps of the advection-diffusion solve on the mixed-precision path (0 = skip)")
    ap.add_argument("--coarse-steps", type=int, default=5,
                    help="steps of the same solve with the coarse-scheme warm start (8 x 8 fine cells per "
                         "coarse cell), reported beside the headline (0 = skip)")
    ap.add_argument("--copy-bytes", type=int, default=256 << 20,
                    help="size of the plain device copy run after the roofline measurement (the counter "
                         "calibration for FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def canonical_pp_flops(p):
    """Algorithmic flops of one volume-Gram matvec: the operator-term pairs
    merged into Kronecker products (orders add, signs (-1)^|alpha'|), terms
    that share every factor but the last spatial one summed into one product
    (2-D problems), then sum over products of sum_i 2 N N_i."""
    import numpy as np
    terms = {}
    for t1 in p.terms:
        for t2 in p.terms:
            m = tuple(a + b for a, b in zip(t1.alpha, t2.alpha))
            sgn = -1.0 if sum(t2.alpha) % 2 else 1.0
            key = (m, t1.cellwise, t2.cellwise)
            terms[key] = terms.get(key, 0.0) + t1.coef * t2.coef * sgn
    live = [k for k, v in terms.items() if v != 0.0]
    if p.d == 2:
        live = {(k[0][0], k[1], k[2]) for k in live}
    napp = len(live)
    nc = p.ncell
    N = int(np.prod(nc))
    return napp * sum(2.0 * N * n for n in nc), napp


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


WAVE_ITERS = 200
GOLDEN = os.path.join(ROOT, "tests", "golden", "wave2d_c4_itergp.json")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs a solve "
              "on a single device; sharding over several is a design note only).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2406_05020_amd as G
    import workloads as W

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.serving_only:
        rates = tuple(float(r) for r in args.serve_rates.split(","))
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_workers, rates, args.serve_coarse,
                                                    args.serve_max_batch)}), flush=True)
        return
    if args.large_timing:
        print(json.dumps(large_timing()), flush=True)
        return
    if args.roofline_only:
        wl = {"advdiff": (W.advdiff_c2, 64), "wave": (W.wave2d_c4, 1), "heat2d": (W.heat2d_c3, 64)}
        make, B = wl[args.roofline_workload]
        out = {"roofline": roofline_volume(make(), B=B, reps=args.mv_reps)}
        if args.extra_rooflines:
            out.update(extra_rooflines())
        out["copy_calibration"] = copy_calibration(args.copy_bytes)
        print(json.dumps(out), flush=True)
        return

    if args.mixed_only:
        print(json.dumps({"advdiff_128x128": c2_block(args, G, W, torch.cuda.current_stream())}), flush=True)
        return
    if args.sw_only:
        print(json.dumps({"shallow_water": sw_block(max(1, args.sw_steps), G, W, torch.cuda.current_stream(),
                                                    args.sw_iters)}), flush=True)
        return

    # ---- headline: wave 64x128x128 + 16384 points, assemble + 200 IterGP + posterior ----
    p = W.wave2d_c4()
    iters = WAVE_ITERS
    M = int(np.prod([len(a) for a in p.grid]))
    mean = torch.empty(M, dtype=torch.float64, device=dev)
    var = torch.empty(M, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    infos, phases = [], []

    def step():
        t0 = time.perf_counter()
        h = G.assemble(p, max_iter=iters, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        try:
            info = G.solve(h, tol=0.0, max_iter=iters, check_every=50, stream=stream.cuda_stream)
            t2 = time.perf_counter()
            G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
            t3 = time.perf_counter()
        finally:
            G.destroy(h)
        t4 = time.perf_counter()
        infos.append(info)
        phases.append((t1 - t0, t2 - t1, t3 - t2, t4 - t3))

    for k in range(args.warmup):
        step()
        note(f"warmup step {k + 1}/{args.warmup}: {sum(phases[-1]):.2f} s")
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        if (k + 1) % 5 == 0 or k + 1 == args.steps:
            note(f"timed step {k + 1}/{args.steps}: {lat[-1]:.2f} s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    info = infos[-1]
    err = oracle_error(mean, var, iters)

    # ---- the Gram matvec of this workload (one right-hand side), timed with HIP events ----
    rl = roofline_volume(p, B=1, reps=args.mv_reps)
    note("volume-Gram roofline measured")
    out = {
        "metric": "Gram matvec GFLOP/s + solves/s, p99 latency at 1e-4 rel error vs FP64 plain",
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded smooth bathymetry, Gaussian initial displacement)",
        "config": {"workload": "wave2d_64x128x128_cells_16384_pts_itergp200", "n_obs": int(p.n),
                   "n_pde": int(p.n_pde), "n_b": int(p.n_b), "itergp_iters": iters,
                   "grid": [len(a) for a in p.grid], "prec": "fp64"},
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "iters": info["iters"],
        "phase_ms_p50": {k: 1e3 * float(np.median([ph[j] for ph in phases[args.warmup:]]))
                         for j, k in enumerate(["assemble", "solve", "posterior", "destroy"])},
        "rel_res": info["rel_res"],
        "rel_res_full": info["rel_res_full"],
        "gram_matvec_gflops": rl["achieved"] * 1e3,
        "oracle_error": err,
    }
    out["roofline"] = rl
    if args.c2_steps > 0:
        out["advdiff_128x128"] = c2_block(args, G, W, stream)
        note("advection-diffusion block done")
    if args.c3_steps > 0:
        out["heat2d_64x64x64"] = c3_block(args.c3_steps, G, W, stream)
        note("heat 64^3 block done")
    if args.sw_steps > 0:
        out["shallow_water"] = sw_block(args.sw_steps, G, W, stream, args.sw_iters)
        note("shallow-water block done")
    if args.extra_rooflines:
        out.update(extra_rooflines())
    if args.serve_requests > 0:
        rates = tuple(float(r) for r in args.serve_rates.split(","))
        out["serving"] = serving_bench(args.serve_requests, args.serve_workers, rates, args.serve_coarse,
                                       args.serve_max_batch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_wave(p, iters, M)
    print(json.dumps(out), flush=True)


def oracle_error(mean, var, iters):
    """Error of the step's posterior against the oracle's values stored for
    the same IterGP iteration count (tests/golden, written by a script that
    calls only the oracle): L2-relative and max-abs / sf2 at the stored
    sample points of the grid."""
    import numpy as np
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        g = json.load(f)
    ref = g["stops"].get(str(iters))
    if ref is None:
        return None
    idx = np.asarray(g["idx"])
    m = mean.detach().cpu().numpy()[idx]
    v = var.detach().cpu().numpy()[idx]
    out = {"points": len(idx), "iters": iters}
    for name, got, r in (("mean", m, np.asarray(ref["mean"])), ("var", v, np.asarray(ref["var"]))):
        out[f"{name}_rel_l2"] = float(np.linalg.norm(got - r) / np.linalg.norm(r))
        out[f"{name}_max_abs"] = float(np.max(np.abs(got - r)))
    return out


def c2_block(args, G, W, stream):
    """Advection-diffusion 128 x 128 volumes + 256 initial points: assemble,
    IterGP-CG to 1e-8 and the posterior on the 128^2 grid per step, plus its
    64-rhs volume-Gram roofline and the coarse warm start."""
    import numpy as np
    import torch
    p = W.advdiff_c2()
    cap = 2048
    M = int(np.prod([len(a) for a in p.grid]))
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")
    infos, lat = [], []
    for k in range(args.c2_steps + 3):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        h = G.assemble(p, max_iter=cap, stream=stream.cuda_stream)
        try:
            info = G.solve(h, tol=1e-8, max_iter=cap, check_every=16, stream=stream.cuda_stream)
            G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
        finally:
            G.destroy(h)
        torch.cuda.synchronize()
        if k >= 3:
            lat.append(time.perf_counter() - s0)
            infos.append(info)
    info = infos[-1]
    out = {"workload": "advdiff_1d_128x128_cells_256_ic_cg1e-8", "solves_per_s": len(lat) / sum(lat),
           "p50_ms": _pctl(lat, 50), "p99_ms": _pctl(lat, 99), "steps": len(lat), "iters": info["iters"],
           "rel_res": info["rel_res"], "rel_res_full": info["rel_res_full"],
           "roofline_64rhs": roofline_volume(p, B=64, reps=args.mv_reps)}
    if args.coarse_steps > 0:
        out["coarse_warm_start"] = coarse_bench(p, (8, 8), args.coarse_steps, stream, mean, var)
    if args.mixed_steps > 0:
        out["mixed"] = mixed_bench(p, args.mixed_steps, stream, mean.cpu().numpy(), var.cpu().numpy(), info["iters"],
                                   args.mv_reps)
    return out


def c3_block(steps, G, W, stream, iters=200):
    """2-D heat on 64^3 volumes + 12288 initial/boundary points: assemble,
    200 IterGP iterations, posterior mean and combined variance on the
    16 x 64^2 grid, in float64 and on the mixed path (split-bfloat16 volume
    Gram in blocks of 32, each re-stabilised in float64).  The mixed result is
    compared with the float64 one of the same step."""
    import numpy as np
    import torch
    p = W.heat2d_c3()
    M = int(np.prod([len(a) for a in p.grid]))
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")
    out = {"workload": "heat2d_64x64x64_cells_12288_pts_itergp200", "n_pde": int(p.n_pde), "n_b": int(p.n_b),
           "itergp_iters": iters}
    res = {}
    for name, prec, tile in (("fp64", G.PREC_FP64, G.TILE_FP32), ("mixed_bf16x3", G.PREC_MIXED, G.TILE_BF16X3)):
        lat = []
        for k in range(steps + 1):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            h = G.assemble(p, max_iter=iters, tile=tile, stream=stream.cuda_stream)
            try:
                info = G.solve(h, prec=prec, tile=tile, tol=0.0, max_iter=iters, check_every=50, block=32,
                               stream=stream.cuda_stream)
                G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
            finally:
                G.destroy(h)
            torch.cuda.synchronize()
            if k > 0:
                lat.append(time.perf_counter() - s0)
        res[name] = (mean.cpu().numpy(), var.cpu().numpy())
        out[name] = {"solves_per_s": len(lat) / sum(lat), "ms_per_step": 1e3 * float(np.mean(lat)),
                     "rel_res": info["rel_res"], "iters": info["iters"]}
    (m64, v64), (mm, vm) = res["fp64"], res["mixed_bf16x3"]
    out["mixed_bf16x3"]["mean_rel_err_vs_fp64"] = float(np.linalg.norm(mm - m64) / np.linalg.norm(m64))
    out["mixed_bf16x3"]["var_rel_err_vs_fp64"] = float(np.linalg.norm(vm - v64) / np.linalg.norm(v64))
    return out


def sw_block(steps, G, W, stream, iters=1250):
    """The linearised shallow-water system at the paper's tsunami scale
    (20 x 90 x 170 cells, three equations on three outputs: 918 000 volume
    observations, 18 380 initial and radiation-boundary points): assemble,
    `iters` IterGP iterations with CG actions (the paper's budget before its
    targeted post-iterations), posterior mean and combined variance of h, u
    and v on the 4 x 90 x 170 grid of cell centres.  One untimed step of 50
    iterations first loads the kernels."""
    import numpy as np
    import torch
    p = W.shallow_water()
    M = int(np.prod([len(a) for a in p.grid]))
    mean = torch.empty(p.nout * M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(p.nout * M, dtype=torch.float64, device="cuda:0")
    out = {"workload": f"shallow_water_20x90x170_cells_3eq_{p.n_b}_pts_itergp{iters}", "n_pde": int(p.n_pde),
           "n_b": int(p.n_b), "n_obs": int(p.n), "itergp_iters": iters, "grid": [len(a) for a in p.grid],
           "outputs": p.nout,
           "paper_context": "about 15 min for 1250 + 500 targeted iterations on one A100 (the paper's tsunami; "
                            "GEBCO bathymetry, 936 672 observations)"}
    phases = []
    for k in range(steps + 1):
        n_it = 50 if k == 0 else iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = G.assemble(p, max_iter=n_it, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        try:
            info = G.solve(h, tol=0.0, max_iter=n_it, check_every=50, stream=stream.cuda_stream)
            t2 = time.perf_counter()
            G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
        finally:
            G.destroy(h)
        if k > 0:
            phases.append((t1 - t0, t2 - t1, t3 - t2))
        note(f"shallow-water step {k}/{steps}: {n_it} iterations, {t3 - t0:.2f} s")
    ph = np.median(np.asarray(phases), axis=0)
    v = var.cpu().numpy().reshape(p.nout, M)
    out.update({"s_per_step": float(np.sum(ph)), "phase_s": dict(zip(["assemble", "solve", "posterior"],
                                                                       [float(x) for x in ph])),
                "ms_per_iteration": 1e3 * float(ph[1]) / iters, "rel_res": info["rel_res"],
                "iters": info["iters"],
                "var_range": [[float(v[j].min()), float(v[j].max())] for j in range(p.nout)]})
    return out


def mixed_bench(p, steps, stream, mean64, var64, iters64, mv_reps):
    """The same step on the mixed-precision path: the volume Gram on the
    bfloat16 matrix cores (three bfloat16 slices per float32 operand) in
    blocks of 32 IterGP iterations, each re-stabilised in float64, to the same
    1e-8.  Errors against the float64 plain solve of the same step: the
    converged means, the combined variances (these differ by the unexplored
    part of the Krylov space, which the variance carries and the mean does
    not), and both at a fixed 120 iterations on either path.  Also the
    64-rhs volume matvec on the split-bfloat16 kernel."""
    import numpy as np
    import torch
    import paper_2406_05020_amd as G
    cap = 2048
    M = len(mean64)
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")

    def run(prec, k, tol):
        h = G.assemble(p, max_iter=k, tile=G.TILE_BF16X3, stream=stream.cuda_stream)
        try:
            info = G.solve(h, prec=prec, tile=G.TILE_BF16X3, tol=tol, max_iter=k, check_every=16,
                           stream=stream.cuda_stream)
            G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
        finally:
            G.destroy(h)
        torch.cuda.synchronize()
        return info

    lat = []
    for k in range(steps + 2):
        s0 = time.perf_counter()
        info = run(G.PREC_MIXED, cap, 1e-8)
        if k >= 2:
            lat.append(time.perf_counter() - s0)
    m, v = mean.cpu().numpy(), var.cpu().numpy()

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {"tile": "bf16x3", "block": 32, "solves_per_s": len(lat) / sum(lat), "p50_ms": _pctl(lat, 50),
           "p99_ms": _pctl(lat, 99), "iters": info["iters"], "fp64_iters": iters64, "blocks": info["outer"],
           "rel_res": info["rel_res"], "mean_rel_err_vs_fp64": rel(m, mean64), "var_rel_err_vs_fp64": rel(v, var64)}
    run(G.PREC_FP64, 120, 0.0)
    m64, v64 = mean.cpu().numpy(), var.cpu().numpy()
    run(G.PREC_MIXED, 120, 0.0)
    out["fixed120"] = {"mean_rel_err_vs_fp64": rel(mean.cpu().numpy(), m64),
                       "var_rel_err_vs_fp64": rel(var.cpu().numpy(), v64)}
    out["roofline_64rhs_bf16x3"] = roofline_volume(p, B=64, reps=mv_reps, prec=G.PREC_MIXED, tile=G.TILE_BF16X3)
    return out


# HBM bytes per launch of the volume-Gram GEMM stages: FETCH_SIZE + WRITE_SIZE
# (two rocprofv3 counter runs of `bench.py --roofline-only`), each divided by
# the ratio the same counter reads for the plain copy of known size that
# follows the measurement.  Each entry records the hash of the GEMM and plan
# sources it was measured with; once those change, traffic reads null until
# it is measured again.
VOLUME_GEMM_TRAFFIC = {
    # (workload, rhs): (bytes per launch, source hash); profiles/k_gemm_lds_wave64x128x128_volume_gram_1rhs.md
    ("wave2d_64x128x128", 1): (104.1e6, "9bdb9b1b46d25abb"),
}
TRAFFIC_SOURCES = ("kernels.hip", "plan.hip", "dense.hip", "common.h")


def gemm_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_05020_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def coarse_bench(p, coarsen, steps, stream, mean, var):
    """The same step (assemble, solve to 1e-8, posterior, destroy) with the
    coarse-scheme warm start: exact conditioning on the nested coarse volumes
    first, then CG.  One untimed step first."""
    import numpy as np
    import torch
    import paper_2406_05020_amd as G
    cap = 2048
    infos, lat = [], []
    for k in range(steps + 1):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        h = G.assemble(p, max_iter=cap, stream=stream.cuda_stream)
        try:
            info = G.solve(h, tol=1e-8, max_iter=cap, check_every=16, coarsen=coarsen, stream=stream.cuda_stream)
            G.posterior(h, p.grid, mean, var, stream=stream.cuda_stream)
        finally:
            G.destroy(h)
        torch.cuda.synchronize()
        if k > 0:
            lat.append(time.perf_counter() - s0)
            infos.append(info)
    info = infos[-1]
    return {"coarsen": list(coarsen), "solves_per_s": steps / sum(lat),
            "ms_per_step": 1e3 * float(np.mean(lat)), "coarse_dirs": info["coarse"],
            "cg_iters": info["iters"] - info["coarse"], "rel_res": info["rel_res"], "steps": steps}


def large_timing(iters=200):
    """Wave 64x128x128 cells + 16384 points: assemble, a fixed number of IterGP
    iterations, combined posterior on 8 x 128^2 points (wall clock, synchronised)."""
    import numpy as np
    import torch
    import paper_2406_05020_amd as G
    import workloads as W2
    p = W2.wave2d_c4()
    out = {"workload": p.name, "n_pde": int(p.n_pde), "n_b": int(p.n_b), "iters": iters}
    torch.cuda.synchronize()
    t = time.perf_counter()
    h = G.assemble(p, max_iter=iters)
    torch.cuda.synchronize()
    out["assemble_s"] = time.perf_counter() - t
    try:
        t = time.perf_counter()
        info = G.solve(h, tol=0.0, max_iter=iters, check_every=16)
        torch.cuda.synchronize()
        out["solve_s"] = time.perf_counter() - t
        out["rel_res"] = info["rel_res"]
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty_like(mean)
        t = time.perf_counter()
        G.posterior(h, p.grid, mean, var)
        torch.cuda.synchronize()
        out["posterior_s"] = time.perf_counter() - t
        out["grid_points"] = M
        v = var.cpu().numpy()
        out["var_min"], out["var_max"] = float(v.min()), float(v.max())
    finally:
        G.destroy(h)
    return out


def extra_rooflines():
    import workloads as W2
    return {"roofline_wave_1rhs": roofline_volume(W2.wave2d_c4(), B=1, reps=20),
            "roofline_heat3d_64rhs": roofline_volume(W2.heat2d_c3(), B=64, reps=5)}


def copy_calibration(nbytes):
    """A plain float64 device copy of `nbytes` (reads nbytes, writes nbytes),
    timed with HIP events; under the counter runs it calibrates FETCH_SIZE and
    WRITE_SIZE against known traffic."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"bytes_read": n * 8, "bytes_written": n * 8, "us": 1e3 * ms, "GB_s": 2 * n * 8 / (ms * 1e-3) / 1e9}


def roofline_volume(p, B, reps, prec=0, tile=0):
    """Volume-Gram matvec on B right-hand sides (its GEMM stages are the
    dominant kernel: k_gemm_lds<double, 64, 64> in float64, k_gemm_bf16s on
    the mixed path with split-bfloat16 tiles): HIP events on the stream it is
    launched on, around `reps` applications; per-launch time = time per
    application / launches.  The mixed path's roofline is the bfloat16 MFMA
    peak against the flops the slice products execute (six per canonical
    product)."""
    import torch
    import paper_2406_05020_amd as G
    stream = torch.cuda.current_stream()
    flops1, napp = canonical_pp_flops(p)
    h = G.assemble(p, max_iter=8, tile=tile, stream=stream.cuda_stream)
    try:
        x = torch.randn(p.n_pde * B, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            G.volume_matvec(h, x, y, nrhs=B, prec=prec, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            G.volume_matvec(h, x, y, nrhs=B, prec=prec, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        info = G.get_info(h)
    finally:
        G.destroy(h)
    launches = max(1, info["volume_launches"])
    alg = flops1 * B
    achieved = alg / (ms * 1e-3) / 1e12
    if prec == 0:
        ent = VOLUME_GEMM_TRAFFIC.get((p.name, B))
        traffic = ent[0] if (ent is not None and ent[1] == gemm_source_hash()) else None
        return {"bound": "mfma", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6,
                "traffic": traffic, "gemm_source_hash": gemm_source_hash(),
                "kernel": "k_gemm_lds<double,...> (volume-Gram mode products)",
                "workload": f"{p.name} volume Gram, {B} rhs", "alg_flops_per_launch": alg / launches,
                "launches_per_matvec": launches, "avg_launch_us": 1e3 * ms / launches,
                "executed_flops_per_matvec": info["volume_flops"], "kronecker_applications": napp}
    executed = 6.0 * alg / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved_executed": executed, "peak": 2500.0, "unit": "TFLOP/s",
            "frac": executed / 2500.0, "canonical_float32_equivalent": achieved,
            "kernel": "k_gemm_bf16s (split-bfloat16 slices, float32 accumulation)",
            "workload": f"{p.name} volume Gram, {B} rhs, mixed path", "ms_per_matvec": ms,
            "note": "time includes the float64<->float32 conversions of x and y around the plan"}


SERVE_TOL, SERVE_ITERS = 1e-6, 256


def _pctl(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) * 1e3


def serving_bench(n_req, workers, rates=(0.8,), coarse_cells=0, max_batch=16):
    """Continuous batching vs the plain per-request float64 solve (FIFO, one at
    a time) on the same Poisson arrival trace of 2-D heat requests with grids
    drawn from {16,32,48,64}^2 x {16,24,32} cells and GP-drawn initial data.
    Every solve: IterGP-CG to 1e-6 or 256 iterations, posterior on 8 time
    slices of the cell-centre grid.  Latency = completion - arrival.  The
    saturated throughput (all requests queued at t = 0) is measured first; each
    entry of `rates` is an arrival rate as a fraction of it.  With coarse_cells
    the served run is repeated with every solve warm-started on a coarse
    scheme of at most that many cells.  The top-level figures are those of the
    first rate."""
    import numpy as np
    import torch
    import paper_2406_05020_amd as G
    import workloads as W

    def note(msg):
        print(f"[serving] {msg}", file=sys.stderr, flush=True)

    probe = [W.heat2d_request(ns, nt, seed) for (_, ns, nt, seed) in W.serving_trace(n_req, 1.0, seed=5)]
    with G.Server(workers=workers, hbm_budget=96 << 30, prec=G.PREC_FP64, tol=SERVE_TOL,
                  max_iter=SERVE_ITERS, max_batch=max_batch) as S:
        t0 = time.perf_counter()
        tk = [S.submit(q) for q in probe]
        for t in tk:
            S.poll(t, wait=True)
        sat = n_req / (time.perf_counter() - t0)
    note(f"saturated {sat:.2f} solves/s")
    dev = torch.device("cuda:0")
    runs = []
    for frac in rates:
        rate = frac * sat
        trace = W.serving_trace(n_req, rate, seed=5)
        reqs = [(arr, W.heat2d_request(ns, nt, seed)) for (arr, ns, nt, seed) in trace]

        def served(coarse_cells):
            lat, conv, rres = [], [], []
            with G.Server(workers=workers, hbm_budget=96 << 30, prec=G.PREC_FP64, tol=SERVE_TOL,
                          max_iter=SERVE_ITERS, coarse_cells=coarse_cells, max_batch=max_batch) as S:
                start = time.perf_counter()
                tickets = []
                for arr, q in reqs:
                    now = time.perf_counter() - start
                    if arr > now:
                        time.sleep(arr - now)
                    tickets.append((arr, S.submit(q)))
                for arr, t in tickets:
                    _, res, _, _ = S.poll(t, wait=True)
                    conv.append(res["rc"] == G.OK)
                    rres.append(res["rel_res"])
                    # t_done comes from the library's std::chrono::steady_clock, the
                    # same CLOCK_MONOTONIC that time.perf_counter reads on Linux
                    lat.append(res["t_done"] - (start + arr))
                makespan = time.perf_counter() - start
                stats = S.stats()
            return lat, makespan, stats, conv, rres

        # continuous batching
        lat, makespan, stats, conv, rres = served(0)
        note(f"rate {frac:g}x: served {n_req / makespan:.2f} solves/s")
        coarse = {}
        if coarse_cells > 0:      # the same, each solve warm-started on a coarse scheme
            lat_c, makespan_c, _, _, _ = served(coarse_cells)
            note(f"rate {frac:g}x: served with the coarse warm start {n_req / makespan_c:.2f} solves/s")
            coarse = {"coarse_cells": coarse_cells, "coarse_solves_per_s": n_req / makespan_c,
                      "coarse_p50_ms": _pctl(lat_c, 50), "coarse_p99_ms": _pctl(lat_c, 99)}

        # plain float64 per-request solve, FIFO, one at a time, same arrivals
        lat_fifo = []
        start = time.perf_counter()
        for k, (arr, q) in enumerate(reqs):
            now = time.perf_counter() - start
            if arr > now:
                time.sleep(arr - now)
            h = G.assemble(q, max_iter=SERVE_ITERS)
            try:
                G.solve(h, tol=SERVE_TOL, max_iter=SERVE_ITERS, check_every=16)
                M = int(np.prod([len(a) for a in q.grid]))
                mean = torch.empty(M, dtype=torch.float64, device=dev)
                var = torch.empty(M, dtype=torch.float64, device=dev)
                G.posterior(h, q.grid, mean, var)
                torch.cuda.synchronize()
            finally:
                G.destroy(h)
            lat_fifo.append(time.perf_counter() - start - arr)
            if (k + 1) % 64 == 0:
                note(f"rate {frac:g}x: fifo {k + 1}/{n_req}")
        makespan_fifo = time.perf_counter() - start
        runs.append({
            "rate_fraction": frac, "arrival_rate_per_s": rate,
            "solves_per_s": n_req / makespan, "p50_ms": _pctl(lat, 50), "p99_ms": _pctl(lat, 99),
            "fifo_fp64_solves_per_s": n_req / makespan_fifo, "fifo_fp64_p50_ms": _pctl(lat_fifo, 50),
            "fifo_fp64_p99_ms": _pctl(lat_fifo, 99), "peak_in_flight": stats["peak_in_flight"],
            "peak_reserved_gb": stats["peak_reserved_bytes"] / 2 ** 30,
            "converged_fraction": float(np.mean(conv)), "rel_res_p50": float(np.median(rres)),
            "rel_res_max": float(np.max(rres)), **coarse,
        })
    out = {"requests": n_req, "workers": workers, "max_batch": max_batch, "saturated_solves_per_s": sat,
           **runs[0],
           "solve": f"fp64 IterGP-CG, tol {SERVE_TOL:g} or {SERVE_ITERS} iterations"}
    if len(runs) > 1:
        out["by_rate"] = runs
    return out


def cpu_baseline_wave(p, iters, n_grid, n_points=8):
    """The oracle timed on host cores on a bounded sample of the same step:
    its set-up (factors by quadrature, point Gram and LAPACK Cholesky, the
    volume-system right-hand side), one IterGP iteration after the first (four
    volume-system matvecs with the two-pass projection), and the posterior
    mean and combined variance at a few grid points.  Solves/s extrapolates:
    set-up + iters x the iteration + the grid x the per-point posterior."""
    import numpy as np
    from oracle import gpfvm_oracle as O
    from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    t0 = time.perf_counter()
    o = O.Oracle(p)
    S = SchurSystem(o)
    t1 = time.perf_counter()
    state = O.itergp(S, 1, passes=2)[:3]
    t2 = time.perf_counter()
    vp, D, eta, _ = O.itergp(S, 1, passes=2, init=state)
    t3 = time.perf_counter()
    X = o.grid_points(p.grid)
    idx = np.random.default_rng(0).choice(len(X), size=n_points, replace=False)
    two_stage_posterior(S, vp, X[idx], D, eta)
    t4 = time.perf_counter()
    setup, it, post = t1 - t0, t3 - t2, (t4 - t3) / n_points
    per_solve = setup + iters * it + n_grid * post
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle on {p.name}: set-up {setup:.1f}s (quadrature factors, point Gram, LAPACK "
                      f"Cholesky), the second IterGP iteration {it:.1f}s (x {iters}), posterior mean and "
                      f"combined variance at {n_points} grid points {post:.2f}s per point (x {n_grid}); "
                      f"float64 NumPy/SciPy, BLAS threads = {cores} host cores"}


if __name__ == "__main__":
    main()
