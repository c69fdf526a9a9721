#!/usr/bin/env python
"""Benchmark of the gfx950 Chebyshev filtered subspace iteration solver.

One step = one complete solve (Alg. 1 of the paper: Lanczos bounds, random
start block, step-0 QR, then filter -> condition estimate -> QR variant ->
Rayleigh-Ritz -> residuals -> locking until nev pairs converge) of a
synthetic planted-spectrum problem that is resident in HBM before timing.

Default workload (one GPU): complex Hermitian N = 20000, DFT-like spectrum
(5% of the eigenvalues clustered in [-2, -1], the rest in [-1, 50]),
nev = 1000, nex = 300, initial degree 20, optimised degrees in [10, 36],
tol 1e-10, FP64.

value = filter flops of the whole solve (8 N^2 per complex MatVec, 2 N^2 per
real one, summed over every column's degree: the paper's convention) /
time-to-solution, in TFLOP/s.
roofline: the filter kernel's executed flops (6 N^2 per complex MatVec, whose
products run as three real MFMA products; 2 N^2 per real one) / its device
time (HIP events recorded by the library around every filter phase on its
stream), against the MFMA peak of the filter's precision.
cpu_baseline: the CPU oracle's whole solve of the same matrix for the N = 1000
and N = 10000 workloads, its filter on a bounded sample of the same matrix for
the larger ones.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5]

c3 also solves the same matrix in plain FP64 and reports both
times-to-solution at the same tolerance.  c5 is the serving stream (Poisson
arrivals of 5-step correlated sequences, N log-uniform in [2000, 25000], FP32
filter): it prints p50/p99 latency and throughput at the specified arrival
rate (--c5-legs spec; every request arrives within seconds, so latency is
queueing and the run measures capacity) and, over the same requests with new
Poisson arrivals, at a sustainable rate (--c5-legs sus: --sus-rate, else 70%
of the capacity measured by the first leg).  --max-bypass 0 is strict FIFO
admission; --hbm-budget-gib caps the memory the scheduler may admit against.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3}  # MI355X dense MFMA TFLOP/s

WORKLOADS = {
    "c2": dict(name="complex Hermitian N=20000 DFT-like spectrum, nev=1000 nex=300, degrees 10-36, FP64",
               N=20000, cplx=True, family="dft", nev=1000, nex=300, degree=20, min_deg=10,
               max_deg=36, tol=1e-10, precision=0, seed=2),
    "c1": dict(name="real symmetric N=1000 uniform spectrum, nev=40 nex=20, FP64",
               N=1000, cplx=False, family="uniform", nev=40, nex=20, degree=20, min_deg=1,
               max_deg=36, tol=1e-10, precision=0, seed=1),
    "c3": dict(name="complex Hermitian N=30000 DFT-like spectrum, nev=1500 nex=400, FP32 filter / FP64 rest",
               N=30000, cplx=True, family="dft", nev=1500, nex=400, degree=20, min_deg=10,
               max_deg=36, tol=1e-10, precision=1, seed=3),
    "c5": dict(name="serving stream"),
    "c4": dict(name="real symmetric N=10000 ill-conditioning stress spectrum, nev=200 nex=100, degrees up to 60",
               N=10000, cplx=False, family="stress", nev=200, nex=100, degree=20, min_deg=1,
               max_deg=60, tol=1e-10, precision=0, seed=4),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the GEMM kernel source and its tuning constants."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2603_10514_amd", "csrc")
    src = open(os.path.join(csrc, "gemm.hpp")).read()
    src += "".join(l for l in open(os.path.join(csrc, "kernels.hip")) if l.startswith("#define CHASE_"))
    return hashlib.sha256(src.encode()).hexdigest()[:16]


PMC_SUMMARY = {"c2": "filter_gemm_c2_complex_n20000_pmc.md",
               "c3": "filter_gemm_c3_mixed_n30000_pmc.md",
               "c4": "filter_gemm_c4_real_n10000_pmc.md"}


def measured_traffic(workload):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per dispatch of the dominant
    filter kernel from the committed rocprofv3 summary, or None when there is
    none or the kernel changed since."""
    if workload not in PMC_SUMMARY:
        return None
    f = os.path.join(ROOT, "profiles", PMC_SUMMARY[workload])
    if not os.path.exists(f):
        return None
    vals = {}
    for line in open(f):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_dispatch", "kernel_source_sha"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_sha():
        return None
    return float(vals["traffic_bytes_per_dispatch"])


def cpu_baseline(H_dev, wl, cols, degree):
    """The oracle's filter (numpy, all host cores) on `cols` columns of the
    same matrix at a fixed degree: a bounded sample of the dominant phase."""
    import torch
    from oracle import filter as ofilter
    import synth
    t0 = time.perf_counter()
    H = np.ascontiguousarray(H_dev.T.cpu().numpy()).T  # column-major host copy
    log("cpu baseline: host copy of H in %.1f s" % (time.perf_counter() - t0))
    V = synth.start_block(wl["N"], cols, 99, wl["cplx"])
    lam_lo, lam_hi = -2.0, 50.0
    c, e = 0.5 * (0.0 + lam_hi), 0.5 * (lam_hi - 0.0)
    deg = np.full(cols, degree)
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    model, blas = host_description()
    t0 = time.perf_counter()
    ofilter.chebyshev_filter(H, V, deg, c, e, lam_lo)
    dt = time.perf_counter() - t0
    f = 8.0 if wl["cplx"] else 2.0
    flops = f * wl["N"] ** 2 * cols * degree
    del H
    return dict(value=flops / dt / 1e12, unit="TFLOP/s", cores=int(cores), kind="oracle",
                sample="oracle chebyshev_filter on %d columns x degree %d of the same N=%d matrix "
                       "(%.2f TFLOP in %.1f s); the filter is the dominant phase, so this bounds "
                       "the oracle's whole-solve throughput from above; host: %s, numpy BLAS %s"
                       % (cols, degree, wl["N"], flops / 1e12, dt, model, blas))


def cpu_baseline_solve(H_dev, wl):
    """The oracle's whole solve (numpy/scipy, all host cores) of the same
    matrix, for the workloads where it takes seconds: Lanczos bounds from four
    seeded runs and a seeded start block (not the library's, so the
    iteration count and MatVecs may differ slightly).  Rate in the bench's
    unit: filter flops of the solve (f N^2 per MatVec) per second."""
    from oracle import solver as osolver
    import synth
    N, nev, nex = wl["N"], wl["nev"], wl["nex"]
    H = np.ascontiguousarray(H_dev.T.cpu().numpy()).T  # column-major host copy
    V0 = synth.start_block(N, nev + nex, 99, wl["cplx"])
    lz = synth.lanczos_starts(N, 4, 98, wl["cplx"])
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    model, blas = host_description()
    t0 = time.perf_counter()
    r = osolver.chase_solve(H, nev, nex, wl["degree"], wl["tol"], V0=V0, lanczos_v0=lz,
                            min_deg=wl["min_deg"], max_deg=wl["max_deg"])
    dt = time.perf_counter() - t0
    f = 8.0 if wl["cplx"] else 2.0
    flops = f * float(N) ** 2 * r.matvecs
    del H
    return dict(value=flops / dt / 1e12, unit="TFLOP/s", cores=int(cores), kind="oracle",
                sample="oracle chase_solve, the whole solve of the same N=%d matrix (%d iterations, "
                       "%d MatVecs, %d of %d pairs converged) in %.2f s; host: %s, numpy BLAS %s"
                       % (N, r.iters, r.matvecs, r.converged, nev, dt, model, blas),
                time_to_solution_s=dt)


def host_description():
    """(CPU model, BLAS library of numpy) of the host running the oracle."""
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas = "%s %s" % (info[0].get("internal_api", "?"), info[0].get("version", "?"))
    except Exception:
        pass
    return model, blas


def qr_timing(N=20000, L=1300, reps=3):
    """The QR step alone on a block of the bench workload's shape: median
    time of chase_qr_factor per variant after one warm-up (the entry point's
    copies of the block in and out, 2 x 0.4 GB, included)."""
    import torch
    import paper_2603_10514_amd as P
    import synth
    dev = torch.device("cuda:0")
    X0 = synth.start_block_torch(N, L, 7, True, dev)
    res = {}
    for variant in ["householder", "chol2", "shifted"]:
        ts = []
        for rep in range(reps + 1):
            X = X0.T.contiguous().T.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.chase_qr_factor(X, variant)
            torch.cuda.synchronize()
            if rep:
                ts.append(time.perf_counter() - t0)
        res[variant] = float(np.median(ts)) * 1e3
        log("qr %s %dx%d complex: %.2f ms" % (variant, N, L, res[variant]))
    print(json.dumps({"qr_ms": res, "N": N, "L": L, "dtype": "complex128", "reps": reps}),
          flush=True)


def serving(args):
    import torch
    from paper_2603_10514_amd import serve
    dev = torch.device("cuda:0")
    legs = args.c5_legs.split(",")
    t0 = time.perf_counter()
    reqs = serve.make_stream(args.requests, args.rate, 2000, 25000, 5, dev, progress=log)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the generator's temporaries: back to the device
    log("generated %d request inputs in %.1f s" % (len(reqs), time.perf_counter() - t0))
    budget = int(args.hbm_budget_gib * serve.GIB) if args.hbm_budget_gib else None
    srv = serve.Server(n_slots=args.slots, N_max=25000, device=dev, hbm_budget=budget,
                       max_bypass=args.max_bypass)

    def summary(done, wall):
        st = serve.latency_stats(done)
        flops = sum(8.0 * r.N ** 2 * sum(i["matvecs"] for i in r.infos) for r in done)
        ok = all(all(x == 0 for x in r.status) for r in done)
        err = max(float(np.max(np.abs(r.evals[0] - r.lam[:r.nev]))) / float(np.max(np.abs(r.lam)))
                  for r in done)
        err_pe = max(float(np.max(np.abs(r.evals[0] - r.lam[:r.nev]) / np.abs(r.lam[:r.nev])))
                     for r in done)
        maxres = max(float(np.max(x)) for r in done for x in r.resid)
        big = max(done, key=lambda r: r.N)
        return dict(p50_s=st["p50"], p99_s=st["p99"], mean_s=st["mean"], max_s=st["max"],
                    samples=len(done), makespan_s=wall, throughput_req_s=len(done) / wall,
                    filter_tflops_aggregate=flops / wall / 1e12, all_converged=ok,
                    max_eig_err_rel_step0=err, max_eig_err_rel_per_eigenvalue_step0=err_pe,
                    max_resid=maxres, requests=len(done),
                    bypass_events=sum(r.bypassed for r in done),
                    wait_s_mean=float(np.mean([r.t_admit - r.arrival for r in done])),
                    largest_request={"N": big.N, "latency_s": big.t_done - big.arrival,
                                     "wait_s": big.t_admit - big.arrival},
                    peak_admitted_gib=srv.peak_used / serve.GIB)

    out = {
        "metric": "ChASE serving p50/p99 latency (continuous batching, warm-started sequences)",
        "value": None, "unit": "s", "n_gpus": 1, "steps": len(reqs), "warmup": 0,
        "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "complex64 filter / complex128 rest",
        "data": "synthetic",
        "config": {"workload": "Poisson arrivals of 5-step correlated complex Hermitian sequences "
                               "H_{j+1} = H_j + 1e-3 E, N log-uniform in [2000, 25000], nev = 5% N, "
                               "nex = max(20, 1.5% N), FP32 filter, HBM admission",
                   "rate_per_s": args.rate, "requests": args.requests, "slots": args.slots,
                   "max_bypass": args.max_bypass,
                   "hbm_budget_gib": srv.budget / serve.GIB,
                   "hbm_budget_capped": bool(budget)},
    }
    cap = None
    if "spec" in legs:
        t0 = time.perf_counter()
        done = srv.run(reqs, progress=log)
        wall = time.perf_counter() - t0
        spec = summary(done, wall)
        log("as specified (%.1f/s): %s" % (args.rate, spec))
        out["as_specified"] = spec
        out["value"] = spec["p99_s"]
        out["ms_per_step"] = spec["makespan_s"] / len(done) * 1e3
        cap = spec["throughput_req_s"]
    if "sus" in legs:
        rate2 = args.sus_rate if args.sus_rate else (0.7 * cap if cap else None)
        if rate2 is None:
            raise SystemExit("--c5-legs sus needs --sus-rate or the spec leg first")
        rng = np.random.default_rng(6)
        t = 0.0
        fresh = []
        for r in reqs:
            t += rng.exponential(1.0 / rate2)
            fresh.append(serve.Request(rid=r.rid, arrival=t, N=r.N, nev=r.nev, nex=r.nex, H0=r.H0,
                                       lam=r.lam, steps=r.steps, eps=r.eps, seed=r.seed))
        srv.peak_used = 0
        t0 = time.perf_counter()
        done2 = srv.run(fresh, progress=log)
        wall2 = time.perf_counter() - t0
        sus = summary(done2, wall2)
        sus["rate_per_s"] = rate2
        sus["rate_basis"] = "given" if args.sus_rate else "0.7 x capacity of the spec leg"
        log("sustainable (%.3f/s): %s" % (rate2, sus))
        out["sustainable"] = sus
        if out["value"] is None:
            out["value"] = sus["p99_s"]
            out["ms_per_step"] = sus["makespan_s"] / len(done2) * 1e3
    srv.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=192)
    ap.add_argument("--cpu-degree", type=int, default=20)
    ap.add_argument("--requests", type=int, default=50)
    ap.add_argument("--c5-legs", default="spec,sus",
                    help="c5: comma list of spec (the specified rate) and sus (sustainable rate)")
    ap.add_argument("--sus-rate", type=float, default=None)
    ap.add_argument("--max-bypass", type=int, default=4,
                    help="c5: times a waiting request may be overtaken (0: strict FIFO)")
    ap.add_argument("--hbm-budget-gib", type=float, default=None,
                    help="c5: admission budget for request data (default: free HBM - 16 GiB)")
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-mixed-pair", action="store_true",
                    help="default workload: skip the untimed mixed-vs-FP64 solve pair of the "
                         "N = 30000 workload that runs after the timed steps")
    ap.add_argument("--cache-dir", default=None,
                    help="save the generated matrix here, or load it if already saved")
    ap.add_argument("--generate-only", action="store_true")
    ap.add_argument("--mixed-switch", type=float, default=None,
                    help="mixed form: switch the filter to FP64 below this residual / ||H||")
    ap.add_argument("--mixed-buffer32", type=int, default=1, choices=[0, 1],
                    help="mixed form, after the switch to FP64: 1 keeps the nex buffer "
                         "columns in the FP32 filter, 0 moves the whole block to FP64")
    ap.add_argument("--qr-policy", default="auto",
                    choices=["auto", "chol1", "chol2", "shifted", "householder"],
                    help="force one QR variant every iteration (Table 3 compares "
                         "Householder QR with the estimate-driven choice)")
    ap.add_argument("--qr-timing", action="store_true",
                    help="instead of a solve: time chase_qr_factor (Householder, CholeskyQR2, "
                         "shifted CholeskyQR2) on a Gaussian 20000 x 1300 complex block")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        serving(args)
        return
    if args.qr_timing:
        qr_timing()
        return

    import torch
    import paper_2603_10514_amd as P
    import synth

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    N, nev, nex = wl["N"], wl["nev"], wl["nex"]
    L = nev + nex
    t0 = time.perf_counter()
    cache = os.path.join(args.cache_dir, "H_%s.npy" % args.workload) if args.cache_dir else None
    if cache and os.path.exists(cache) and os.path.exists(cache + ".lam.npy"):
        # the same seeded matrix, generated by an earlier run of this script
        Hn = np.load(cache, mmap_mode="r")  # row-major H^T == column-major H
        H = torch.from_numpy(np.ascontiguousarray(Hn)).to(dev).T
        lam = np.load(cache + ".lam.npy")
        del Hn
        log("loaded H (N=%d) from %s in %.1f s" % (N, cache, time.perf_counter() - t0))
    else:
        H, lam = synth.planted_torch(N, wl["family"], wl["seed"], wl["cplx"], dev)
        torch.cuda.synchronize()
        log("generated H (N=%d, %s) in %.1f s" % (N, "complex" if wl["cplx"] else "real",
                                                    time.perf_counter() - t0))
        if cache:
            os.makedirs(args.cache_dir, exist_ok=True)
            np.save(cache, H.T.contiguous().cpu().numpy())
            np.save(cache + ".lam.npy", lam)
            log("saved H to %s" % cache)
    if args.generate_only:
        return
    dt = torch.complex128 if wl["cplx"] else torch.float64
    evecs = P.colmajor_empty(N, L, dt, dev)
    opts = dict(min_deg=wl["min_deg"], max_deg=wl["max_deg"], precision=wl["precision"],
                qr_policy=args.qr_policy)
    if args.mixed_switch is not None:
        opts["mixed_switch"] = args.mixed_switch
    if wl["precision"]:
        opts["mixed_buffer32"] = args.mixed_buffer32

    def one(step):
        return P.chase_solve(H, nev, nex, wl["degree"], wl["tol"], evecs=evecs, seed=1000 + step,
                             **opts)

    for w in range(args.warmup):
        r = one(-1 - w)
        log("warmup %d: %.2f s, iters %d, matvecs %d" % (w, r["info"]["t_total"],
                                                          r["info"]["iters"], r["info"]["matvecs"]))
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        results.append(one(s))
        log("step %d: %.2f s" % (s, results[-1]["info"]["t_total"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    f = 8.0 if wl["cplx"] else 2.0
    matvecs = sum(r["info"]["matvecs"] for r in results)
    flops = f * float(N) ** 2 * matvecs
    t_filter = sum(r["info"]["t_filter"] for r in results)
    launches = sum(r["info"]["filter_launches"] for r in results)
    fp32_iters = sum(r["info"]["filter_fp32_iters"] for r in results)
    iters = sum(r["info"]["iters"] for r in results)
    # per-precision filter rates; the roofline entry is the kernel with the
    # larger share of filter time (FP32 and FP64 flops are never mixed)
    mv32 = sum(r["info"]["matvecs_fp32"] for r in results)
    t32 = sum(r["info"]["t_filter_fp32"] for r in results)
    mv64, t64 = matvecs - mv32, t_filter - t32
    # executed flops per MatVec: complex products run as three real MFMA
    # products (6 N^2 per complex MatVec), real ones as one (2 N^2); the
    # paper's convention counts 8 N^2 per complex MatVec
    fx = 6.0 if wl["cplx"] else 2.0
    if t32 > t64:
        prec, kflops, ktime = "f32", fx * float(N) ** 2 * mv32, t32
    else:
        prec, kflops, ktime = "f64", fx * float(N) ** 2 * mv64, t64
    achieved = kflops / ktime / 1e12
    achieved_conv = achieved * f / fx
    # per-step roofline: step i with l'_i active columns cannot take less
    # than max(fx N^2 l'_i / peak, s (N^2 + 3 N l'_i) / HBM), executed flops
    # the FP64 part of an iteration is its first ncols - ncols_fp32 columns,
    # the FP32 part the rest; algorithmic bytes of a step: s (N^2 + 3 N l')
    t_star = 0.0
    alg_bytes = {"f64": 0.0, "f32": 0.0}
    for r in results:
        for x in r["log"]:
            d_all = np.asarray(x["degrees"])
            n32 = int(x["ncols_fp32"])
            for part, d in (("f64", d_all[:d_all.size - n32]), ("f32", d_all[d_all.size - n32:])):
                if d.size == 0:
                    continue
                pk = PEAK[part] * 1e12
                bpe = (16.0 if wl["cplx"] else 8.0) / (2.0 if part == "f32" else 1.0)
                for i in range(1, int(d.max()) + 1):
                    lp = float(np.sum(d >= i))
                    b = bpe * (float(N) ** 2 + 3.0 * N * lp)
                    alg_bytes[part] += b
                    t_star += max(fx * float(N) ** 2 * lp / pk, b / 8e12)
    launches32 = sum(r["info"]["filter_launches_fp32"] for r in results)
    klaunches = launches32 if prec == "f32" else launches - launches32
    scale = float(np.max(np.abs(lam)))
    eig_err = max(float(np.max(np.abs(r["evals"] - lam[:nev]))) / scale for r in results)
    # per eigenvalue: max_i |lambda_i - planted_i| / |planted_i|
    eig_err_each = max(float(np.max(np.abs(r["evals"] - lam[:nev]) / np.abs(lam[:nev])))
                       for r in results)
    max_res = max(float(np.max(r["resid"])) for r in results)
    status_ok = all(r["status"] == P.CHASE_OK for r in results)
    phases = {k: sum(r["info"][k] for r in results) / len(results)
              for k in ("t_filter", "t_qr", "t_rr", "t_resid", "t_lanczos")}
    variants = [[x["variant"] for x in r["log"]] for r in results]

    out = {
        "metric": "ChASE time-to-solution & filter TFLOP/s",
        "value": flops / wall / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128" if wl["cplx"] else "float64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "N": N, "nev": nev, "nex": nex,
                   "degree": wl["degree"], "min_deg": wl["min_deg"], "max_deg": wl["max_deg"],
                   "tol": wl["tol"], "precision": "mixed" if wl["precision"] else "fp64",
                   "qr_policy": args.qr_policy,
                   **({"mixed_buffer32": args.mixed_buffer32} if wl["precision"] else {})},
        "time_to_solution_s": wall / args.steps,
        "filter_tflops": flops / t_filter / 1e12,
        "filter_tflops_basis": "%d N^2 flops per MatVec (the paper's convention)" % int(f),
        "filter_frac_of_per_step_roofline": t_star / t_filter,
        "matvecs_per_solve": matvecs / args.steps,
        "iters_per_solve": iters / args.steps,
        "phase_s_per_solve": phases,
        "qr_variants": variants[0],
        "max_eig_err_rel": eig_err,
        "max_eig_err_rel_per_eigenvalue": eig_err_each,
        "max_resid": max_res,
        "converged": status_ok,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[prec],
                     "flops_basis": "executed MFMA flops: %s N^2 per MatVec (%s)" % (
                         int(fx), "three real products per complex product" if wl["cplx"]
                         else "one real product"),
                     "achieved_paper_convention": achieved_conv,
                     "paper_convention": "%d N^2 flops per MatVec" % int(f),
                     "traffic": measured_traffic(args.workload),
                     "traffic_unit": "bytes per filter dispatch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     # s (N^2 + 3 N l') per degree step (H once; X, X_prev and the
                     # output once), summed over this kernel's steps, per dispatch
                     "algorithmic_bytes_per_dispatch": alg_bytes[prec] / max(klaunches, 1),
                     "kernel": "filter GEMM (gemm_kernel, EPI_FILTER, %s)" % prec,
                     "launches": klaunches, "avg_launch_ms": ktime / max(klaunches, 1) * 1e3,
                     "executed_flops_per_launch": kflops / max(klaunches, 1)},
    }
    if wl["precision"] == 1:
        r32 = f * float(N) ** 2 * mv32 / max(t32, 1e-12) / 1e12
        r64 = f * float(N) ** 2 * mv64 / max(t64, 1e-12) / 1e12
        # fractions of peak on executed flops (fx per MatVec), rates in the
        # paper's convention (f per MatVec)
        out["mixed"] = {"fp32_filter_tflops": r32,
                        "fp32_frac_of_peak": r32 * fx / f / PEAK["f32"],
                        "fp64_filter_tflops": r64,
                        "fp64_frac_of_peak": r64 * fx / f / PEAK["f64"],
                        "fp32_matvec_share": mv32 / max(matvecs, 1),
                        "fp32_filter_time_share": t32 / max(t_filter, 1e-12),
                        "fp32_iters_per_solve": fp32_iters / args.steps}
        if not args.no_fp64_compare:
            s64 = P.chase_solve(H, nev, nex, wl["degree"], wl["tol"], evecs=evecs, seed=1000,
                                min_deg=wl["min_deg"], max_deg=wl["max_deg"], precision=0)
            out["mixed"]["fp64_time_to_solution_s"] = s64["info"]["t_total"]
            out["mixed"]["fp64_max_eig_err_rel"] = float(np.max(np.abs(s64["evals"] - lam[:nev]))) / scale
            out["mixed"]["mixed_vs_fp64_speedup"] = s64["info"]["t_total"] / (wall / args.steps)
            out["mixed"]["max_abs_eig_diff_mixed_vs_fp64_rel"] = float(
                np.max(np.abs(results[0]["evals"] - s64["evals"]))) / scale
            log("fp64 comparison: %.2f s" % s64["info"]["t_total"])
    if args.workload == "c4":
        # untimed diagnostic solve: estimate vs exact kappa_2 (SVD of a host
        # copy of [Y, filtered]) and the QR variant, per iteration
        rd = P.chase_solve(H, nev, nex, wl["degree"], wl["tol"], evecs=evecs, seed=1000,
                           exact_cond=True, **opts)
        out["cond_log"] = [{"iter": x["iter"], "locked": x["locked"], "cond_est": x["cond_est"],
                            "cond_exact": x["cond_exact"], "variant": x["variant"],
                            "deg_max": x["deg_max"]} for x in rd["log"]]
    if not args.no_cpu_baseline:
        if args.workload in ("c1", "c4"):  # whole oracle solve: about 0.6 s and 20 s
            out["cpu_baseline"] = cpu_baseline_solve(H, wl)
        else:
            out["cpu_baseline"] = cpu_baseline(H, wl, args.cpu_cols, args.cpu_degree)
    if args.workload == "c2" and not args.no_mixed_pair:
        del H, evecs
        torch.cuda.empty_cache()
        out["mixed_vs_fp64_n30000"] = mixed_pair()
    print(json.dumps(out), flush=True)


def mixed_pair():
    """Untimed: one solve of the N = 30000 workload with the FP32 filter and
    one in plain FP64 on the same matrix and start block (a child process,
    after the timed steps), reported beside the default workload's line."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "c3", "--steps", "1",
           "--warmup", "0", "--no-cpu-baseline"]
    log("mixed-vs-FP64 pair (N = 30000): " + " ".join(cmd[2:]))
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                           timeout=480)
    except subprocess.TimeoutExpired:
        return {"error": "timed out"}
    sys.stderr.write(r.stderr[-2000:])
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": "exit status %d" % r.returncode}
    d = json.loads(lines[-1])
    m = d.get("mixed", {})
    return {"workload": d["config"]["workload"], "tol": d["config"]["tol"],
            "mixed_time_to_solution_s": d["time_to_solution_s"],
            "fp64_time_to_solution_s": m.get("fp64_time_to_solution_s"),
            "mixed_vs_fp64_speedup": m.get("mixed_vs_fp64_speedup"),
            "mixed_max_eig_err_rel": d["max_eig_err_rel"],
            "mixed_max_eig_err_rel_per_eigenvalue": d["max_eig_err_rel_per_eigenvalue"],
            "fp64_max_eig_err_rel": m.get("fp64_max_eig_err_rel"),
            "max_abs_eig_diff_mixed_vs_fp64_rel": m.get("max_abs_eig_diff_mixed_vs_fp64_rel"),
            "mixed_max_resid": d["max_resid"], "mixed_converged": d["converged"],
            "fp32_filter_frac_of_fp32_peak": m.get("fp32_frac_of_peak"),
            "fp64_filter_frac_of_fp64_peak": m.get("fp64_frac_of_peak"),
            "fp32_matvec_share": m.get("fp32_matvec_share"),
            "iters": d["iters_per_solve"], "matvecs": d["matvecs_per_solve"]}


if __name__ == "__main__":
    main()
