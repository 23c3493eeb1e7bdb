#!/usr/bin/env python3
"""Throughput of the variance-reduced EM hot path on one MI355X.

Workload (default): SVREM on a 256 x 256 image (2 mm pixels), 252 views x
344 bins, 21 interleaved subsets, 1e6 counts with a 10% uniform background,
quadratic 8-neighbour penalty with beta = 1e-2, alpha = 0.7, eta = 1, FP32
weights.  Seeded synthetic data (ellipse phantom, Poisson counts).

One step = one SVREM outer loop: an anchor pass over all subsets followed by
eta*Ns subset updates, which the paper's accounting counts as eta + 1 epochs.
``value`` is epochs per second with all inputs resident in HBM.

The dominant kernel's duration is measured with HIP events recorded by the
library on the stream its kernels run on, over a second pass of the same
steps (events between kernels would perturb the step time of the first).

``python bench.py [--gpus 1] [--steps K] [--warmup W]``
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SVREM epochs/s + projector HBM GB/s (256², 21 subsets); p50/p99 recon latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("kernels.h", "phases.h", "persist.hip", "proj.hip", "update.hip", "penalty.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def settle_gc():
    """Collects garbage and moves every object alive now (modules, the set-up's
    data) out of the collector's generations (gc.freeze), so that a full
    collection inside a timed region scans only what the region itself
    creates.  With torch and numpy loaded a full collection otherwise takes
    35-45 ms, as long as 150 headline steps, and whether one lands in the
    region depends on how many objects the process has made before it."""
    import gc
    gc.collect()
    gc.freeze()


def kernel_source_hash():
    """Hash of the kernel sources and the device compile flags: a profile taken
    under another hash describes other machine code."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_03172_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    from paper_2106_03172_amd import build as _build
    h.update(" ".join(_build.FLAGS).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_kind, wtype):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel_kind}_{wtype}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel-source-hash:\s*([0-9a-f]+)", txt)
    m_val = re.search(r"hbm-bytes-per-launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def algorithmic_bytes(kind, A_info, nnz_t_mean, M, Mt_mean, N, Ns, wb):
    """Bytes each launch of a kernel must move at minimum;
    ``ib`` index bytes (2 or 4) and ``wb`` weight bytes per non-zero."""
    ib = A_info.index_bytes
    if kind == "forward":  # index + weight stream, row pointers, image, g, w, ratio
        return nnz_t_mean * (ib + wb) + 4 * (Mt_mean + 1) + 4 * N + 12 * Mt_mean
    if kind == "update":   # transposed stream, pointers, ratio, per-pixel SVREM state, tiled iterate copy
        return nnz_t_mean * (ib + wb) + 4 * (N + 1) + 4 * Mt_mean + 48 * N
    if kind == "anchor_forward":
        return A_info.nnz * (ib + wb) + 4 * (M + 1) + 4 * N + 12 * M
    if kind == "anchor_table":  # all transposed rows, their pointers, ratio, f, table write
        return A_info.nnz * (ib + wb) + 4 * (Ns * N + 1) + 4 * M + 4 * N + 4 * Ns * N
    if kind == "anchor_sum":    # table read, s_anc and s_hat writes, then the fused SVREM update
        return 4 * Ns * N + 8 * N + 48 * N
    raise ValueError(kind)


def epoch_bytes(A_info, nnz_t_mean, M, Mt_mean, N, Ns, wb, per):
    """Algorithmic bytes of one persistent epoch kernel: one anchor pass and
    ``per`` subset iterations (forward + fused update)."""
    args = (A_info, nnz_t_mean, M, Mt_mean, N, Ns, wb)
    return (algorithmic_bytes("anchor_forward", *args) + algorithmic_bytes("anchor_table", *args)
            + algorithmic_bytes("anchor_sum", *args)
            + per * (algorithmic_bytes("forward", *args) + algorithmic_bytes("update", *args)))


def cpu_baseline(P, beta, alpha, eta, seconds, label="256x256 / 252x344 / 21-subset", max_loops=200):
    """The FP64 oracle (as it stands) on the same workload, for ~``seconds``."""
    import numpy as np

    import datagen
    import oracle
    log("cpu baseline: building the oracle model")
    Ao = oracle.system_matrix(P.geom, P.mu)
    m = oracle.Model(Ao, P.g, P.w, P.geom, P.n_subsets, beta=beta)
    f0 = oracle.osem_epoch(m, np.ones((1, P.geom.n_pixels)), range(P.n_subsets))
    alg = oracle.SVREM(m, f0, alpha, eta)
    per = eta * P.n_subsets
    loops = 0
    c0, t0 = time.process_time(), time.perf_counter()
    while True:
        alg.run(datagen.make_order(P.n_subsets, per, seed=9000 + loops))
        loops += 1
        el = time.perf_counter() - t0
        if el >= seconds or loops >= max_loops:
            break
    cpu = time.process_time() - c0
    cores = max(1, int(round(cpu / el)))
    log(f"cpu baseline: {loops} outer loops in {el:.1f} s")
    return {"value": loops * (eta + 1) / el, "unit": "epochs/s", "cores": cores, "kind": "oracle",
            "sample": f"{loops} SVREM outer loops (anchor + {per} subset updates each) of the same "
                      f"{label} workload, FP64 NumPy+SciPy, {el:.1f} s wall"}


def bench_convergence(args):
    """Convergence curves (Sec. 5.1) on a stand-in for the paper's brain slice:
    114 x 114 (2 mm), 180 views 1 degree apart x 154 bins, 30 subsets, 1e6
    counts, log cosh penalty with the paper's delta = 0.01 and beta = 60.  All
    methods start from one OSEM epoch.  f* is a long SVREM run (its last
    relative change is reported); Delta(f) = ||f - f*|| / ||f*||.  Then the
    SVREM sweeps of Fig. 3 (alpha, eta and the number of subsets)."""
    import torch

    import datagen
    import paper_2106_03172_amd as pkg
    from paper_2106_03172_amd import convergence as cv
    beta, pen, delta = 60.0, "logcosh", 0.01
    P = datagen.make_problem(114, 114, 2.0, 180, 154, 2.0, 30, 1e6, attenuation=False, seed=7)
    A = pkg.SystemMatrix(P.geom, 30, pkg.SVR_W_F32)
    t0 = time.perf_counter()
    ref_m = cv.Method("SVREM", "svrem", dict(alpha=0.7, eta=1, beta=beta, penalty=pen, delta=delta))
    f_ref, ref_epochs, ref_change = cv.reference_image(A, P.g, P.w, ref_m, max_epochs=3000, tol=1e-7)
    log(f"reference: {ref_epochs:.0f} epochs, last relative change {ref_change:.1e} "
        f"({time.perf_counter() - t0:.1f} s)")
    methods = cv.paper_methods(beta, pen, delta)
    curves = cv.compare(A, P.g, P.w, methods, args.epochs, f_ref=f_ref)
    sweeps = []
    for alpha in (0.3, 0.7, 1.0, 1.4):
        sweeps.append(("alpha", alpha, 30, cv.Method(f"SVREM alpha={alpha}", "svrem",
                                                     dict(alpha=alpha, eta=1, beta=beta, penalty=pen, delta=delta))))
    for eta in (2, 3):
        sweeps.append(("eta", eta, 30, cv.Method(f"SVREM eta={eta}", "svrem",
                                                 dict(alpha=0.7, eta=eta, beta=beta, penalty=pen, delta=delta))))
    for ns in (15, 45):
        sweeps.append(("n_subsets", ns, ns, cv.Method(f"SVREM Ns={ns}", "svrem",
                                                      dict(alpha=0.7, eta=1, beta=beta, penalty=pen, delta=delta))))
    sweep_curves = []
    mats = {30: A}
    for kind, val, ns, m in sweeps:
        if ns not in mats:
            mats[ns] = pkg.SystemMatrix(P.geom, ns, pkg.SVR_W_F32)
        sweep_curves.append((kind, val, cv.run_method(mats[ns], P.g, P.w, m, args.epochs, f_ref, seed=900 + len(
            sweep_curves))))
    torch.cuda.synchronize()

    def summary(c):
        at = {}
        for e_mark in (10, 25, 50):
            vals = [d for e, d in zip(c.epochs, c.delta) if e <= e_mark]
            at[str(e_mark)] = round(vals[-1], 6) if vals else None
        return {"delta_at_epochs": at, "epochs_to_1e-2": c.epochs_to(1e-2), "epochs_to_1e-3": c.epochs_to(1e-3),
                "final_phi": c.phi[-1] if c.phi else None, "status": c.status,
                "seconds": round(sum(c.seconds), 4)}
    out = {"workload": "convergence",
           "problem": "114x114 (2 mm), 180 views x 154 bins, 30 subsets, 1e6 counts, 10% background, "
                      "log cosh delta=0.01 beta=60; every method starts from one OSEM epoch",
           "reference": {"method": "SVREM alpha=0.7 eta=1", "epochs": ref_epochs, "last_change": ref_change},
           "methods": {c.name: summary(c) for c in curves},
           "sweeps": [{"param": k, "value": v, **summary(c)} for k, v, c in sweep_curves]}
    print(json.dumps(out), flush=True)
    if args.curves_out:
        with open(args.curves_out, "w") as fh:
            fh.write(cv.to_json(curves + [c for _, _, c in sweep_curves]))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--wtype", choices=("f32", "f16", "bf16"), default="f32")
    ap.add_argument("--counts", type=float, default=1e6)
    ap.add_argument("--beta", type=float, default=1e-2)
    ap.add_argument("--alpha", type=float, default=0.7)
    ap.add_argument("--eta", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the size-based run lengths instead of autotuning them (a profiled run uses this so "
                         "that its kernels do not depend on timings taken under the profiler)")
    ap.add_argument("--workload", choices=("headline", "multislice", "serve", "serve-scanner", "serve-compare", "copy",
                                           "convergence", "algos", "small", "projectors", "precision"),
                    default="headline",
                        help="headline: the JSON line below; multislice / serve / serve-compare / convergence / "
                         "algos / small: supplementary measurements")
    ap.add_argument("--epochs", type=float, default=50, help="convergence: epochs per curve")
    ap.add_argument("--curves-out", default="", help="convergence: write every curve as JSON to this file")
    ap.add_argument("--requests", type=int, default=200, help="serve: number of requests")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="headline: requests of the serving stream for the p50/p99 latency and the batched "
                         "FP32/BF16/FP16 comparison in the JSON line (0: skip)")
    ap.add_argument("--fwd-natural-order", action="store_true",
                    help="per-subset forward passes take their rows in order instead of one bin band per XCD")
    ap.add_argument("--persistent", action="store_true",
                    help="one persistent cooperative kernel per epoch call instead of one kernel per phase")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} (WORLD_SIZE={world}) is not supported: "
              "the reconstruction path runs on one GPU and would shard across GPUs only by whole requests "
              "or slice slabs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2106_03172_amd as pkg

    torch.cuda.set_device(0)
    if args.workload == "multislice":
        return bench_multislice(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "serve-compare":
        return bench_serve_compare(args)
    if args.workload == "serve-scanner":
        return bench_serve_scanner(args)
    if args.workload == "convergence":
        return bench_convergence(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "algos":
        return bench_algos(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "projectors":
        return bench_projectors(args)
    if args.workload == "precision":
        return bench_precision(args)
    wt = {"f32": pkg.SVR_W_F32, "f16": pkg.SVR_W_F16, "bf16": pkg.SVR_W_BF16}[args.wtype]
    wb = 4 if args.wtype == "f32" else 2
    cfg = dict(datagen.CONFIG_HEADLINE)
    cfg["counts"] = args.counts
    P = datagen.make_problem(**cfg)
    Ns, N, M = P.n_subsets, P.geom.n_pixels, P.geom.n_rays
    log("building the system matrix on the device")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    A = pkg.SystemMatrix(P.geom, Ns, wt)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    inf, per_subset = A.info()
    log(f"nnz = {inf.nnz}, build {build_s:.3f} s")
    if args.no_tune:
        tuning = A.tuning()
        log(f"size-based run lengths: forward {tuning[0]}, anchor table {tuning[1]}")
    else:
        tuning = A.tune()
        log(f"autotuned run lengths: forward {tuning[0]} rows/wavefront ({tuning[2]:.1f} us), "
            f"anchor table {tuning[1]} rows/group ({tuning[3]:.1f} us); per-subset batch widths "
            f"{A.batch_widths()}")

    if args.fwd_natural_order:
        A.set_tuning(tuning[0], tuning[1], fwd_natural_order=1)
    f0 = np.ones((1, N), dtype=np.float32)
    flags = pkg.binding.FLAG_PERSISTENT_EPOCH if args.persistent else 0
    R = pkg.Recon(A, P.g, P.w, f0, pkg.params("svrem", alpha=args.alpha, eta=args.eta, beta=args.beta,
                                                flags=flags))
    R.osem_epoch(list(range(Ns)))
    per = args.eta * Ns
    total = args.warmup + 2 * args.steps
    orders = [datagen.make_order(Ns, per, seed=100 + i) for i in range(total)]

    settle_gc()
    for i in range(args.warmup):
        R.svrem_epoch(orders[i])
    torch.cuda.synchronize()
    log("timed region")
    t0 = time.perf_counter()
    for i in range(args.steps):
        R.svrem_epoch(orders[args.warmup + i])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    epochs_per_step = args.eta + 1
    value = args.steps * epochs_per_step / el
    log(f"{value:.1f} epochs/s ({1e3 * el / args.steps:.3f} ms per step)")

    # second pass with per-kernel HIP events
    R.set_profiling(True)
    used = []
    for i in range(args.steps):
        o = orders[args.warmup + args.steps + i]
        used.extend(int(t) for t in o)
        R.svrem_epoch(o)
    kt = R.kernel_times()
    R.set_profiling(False)
    phi = R.objective()
    nnz_t_mean = float(np.mean([per_subset[t] for t in used]))
    rows_t = [(len(range(t, P.geom.n_views, Ns)) * P.geom.n_bins) for t in range(Ns)]
    Mt_mean = float(np.mean([rows_t[t] for t in used]))
    kernels = {}
    for name, (n, ms) in kt.items():
        if n == 0:
            continue
        avg_s = ms / n / 1e3
        if name == "epoch":
            b = epoch_bytes(inf, nnz_t_mean, M, Mt_mean, N, Ns, wb, per)
        else:
            b = algorithmic_bytes(name, inf, nnz_t_mean, M, Mt_mean, N, Ns, wb)
        kernels[name] = {"launches": n, "avg_us": avg_s * 1e6, "share": 0.0,
                         "algorithmic_bytes": b, "gbs": b / avg_s / 1e9}
    tot_ms = sum(v[1] for v in kt.values())
    for name, (n, ms) in kt.items():
        if name in kernels:
            kernels[name]["share"] = ms / tot_ms
    dom = max(kernels, key=lambda k: kernels[k]["share"])
    d = kernels[dom]
    traffic = traffic_from_profile(dom, args.wtype)
    roofline = {"bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_us": round(d["avg_us"], 3), "bytes_per_launch": int(d["algorithmic_bytes"]),
                "duration": "mean of HIP events attached to each dispatch of the kernel on the library's stream, "
                            "over a second pass of the timed steps"}

    # standalone projectors over the whole matrix
    x = torch.rand(1, N, device="cuda")
    y = torch.rand(1, M, device="cuda")
    yo = torch.empty(1, M, device="cuda")
    xo = torch.empty(1, N, device="cuda")
    for _ in range(3):
        A.project(x, -1, yo)
        A.backproject(y, -1, xo)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 20
    ev[0].record()
    for _ in range(reps):
        A.project(x, -1, yo)
    ev[1].record()
    for _ in range(reps):
        A.backproject(y, -1, xo)
    ev[2].record()
    torch.cuda.synchronize()
    fwd_s = ev[0].elapsed_time(ev[1]) / reps / 1e3
    bwd_s = ev[1].elapsed_time(ev[2]) / reps / 1e3
    ib = inf.index_bytes
    fwd_b = inf.nnz * (ib + wb) + 4 * (M + 1) + 4 * N + 4 * M
    bwd_b = inf.nnz * (ib + wb) + 4 * (Ns * N + 1) + 4 * N + 12 * M
    projector = {"forward_gbs": round(fwd_b / fwd_s / 1e9, 1), "back_gbs": round(bwd_b / bwd_s / 1e9, 1),
                 "forward_us": round(fwd_s * 1e6, 2), "back_us": round(bwd_s * 1e6, 2),
                 "matrix_mb": round(inf.nnz * (ib + wb) / 1e6, 1), "index_bytes": ib}
    # one subset (t = 0): the calls take natural-order sinograms, so the back-projection call
    # also permutes the whole sinogram into subset order (8M bytes)
    nnz0 = int(np.asarray(per_subset)[0])
    M0 = ((P.geom.n_views + Ns - 1) // Ns) * P.geom.n_bins  # views v = 0 (mod Ns)
    reps = 50
    ev[0].record()
    for _ in range(reps):
        A.project(x, 0, yo)
    ev[1].record()
    for _ in range(reps):
        A.backproject(y, 0, xo)
    ev[2].record()
    torch.cuda.synchronize()
    f0_s = ev[0].elapsed_time(ev[1]) / reps / 1e3
    b0_s = ev[1].elapsed_time(ev[2]) / reps / 1e3
    f0_b = nnz0 * (ib + wb) + 4 * (M0 + 1) + 4 * N + 4 * M0
    b0_b = nnz0 * (ib + wb) + 4 * (N + 1) + 4 * N + 8 * M + 4 * M0
    projector["subset0"] = {"forward_us": round(f0_s * 1e6, 2), "back_us": round(b0_s * 1e6, 2),
                            "forward_gbs": round(f0_b / f0_s / 1e9, 1), "back_gbs": round(b0_b / b0_s / 1e9, 1),
                            "rows": M0, "nnz": nnz0}

    serving = compare = None
    if args.serve_requests > 0:
        specs, sdata = _serving_data(args.serve_requests)
        serving = serve_latency(specs, sdata, args.alpha)
        log(f"serving: p50 {serving['p50_ms']} ms, p99 {serving['p99_ms']} ms, {serving['achieved_rps']} requests/s")
        compare = serve_compare(specs, sdata, args.alpha)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P, args.beta, args.alpha, args.eta, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "epochs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SVREM 256x256 (2 mm), 252 views x 344 bins, 21 interleaved subsets, "
                               f"counts {args.counts:.0e}, 10% background, quadratic 8-neighbour beta={args.beta}, "
                               f"alpha={args.alpha}, eta={args.eta}; {args.wtype} weights and FP32 iterate, "
                               f"FP64 products, sums and statistics",
                   "arithmetic": {"weights": args.wtype, "iterate": "f32", "tables": "f32",
                                  "products_and_sums": "f64", "statistics_and_objective": "f64"},
                   "epochs_per_step": epochs_per_step, "nnz": int(inf.nnz), "build_s": round(build_s, 4),
                   "tuning": {"fwd_pairs_per_wave": tuning[0], "bp_rows_per_group": tuning[1],
                              "fwd_row_order": "natural" if args.fwd_natural_order else "xcd_bin_bands",
                              "subset_batch_widths": dict(zip(("forward", "update"), A.batch_widths()))},
                   "objective_after": phi, "parallelism": "single GPU",
                   "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                               for k, v in kernels.items()},
                   "projector": projector, "kernel_source_hash": kernel_source_hash(),
                   "serving": serving, "serve_compare": compare},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_algos(args):
    """Every update rule of the library on the headline workload (256 x 256,
    252 x 344, 21 subsets, 1e6 counts, quadratic beta = 0.01), one after another
    on one matrix: subset iterations per second and epochs per second in the
    paper's accounting (Sec. 5.1: a pass over the data, i.e. Ns subset updates
    or one anchor / table fill, counts one epoch).  SVREM alpha = 0.7, eta = 1;
    SVRG alpha = 2, eta = 2 and SAGA alpha = 2 with the frozen preconditioner
    f0 / A^T 1 (Sec. 5.1, Theorem 1); SGA, BSREM (a_k = 1/(0.001 k + 1)) and SEM with
    the decaying step; OSEM unpenalised.  Each figure is the median of five
    timed blocks of --steps epoch calls.  Also the wall time of one objective
    evaluation (svr_objective, which synchronises) on the SVREM recon."""
    import numpy as np
    import torch

    import datagen
    import paper_2106_03172_amd as pkg
    P = datagen.make_problem(**datagen.CONFIG_HEADLINE)
    Ns, N = P.n_subsets, P.geom.n_pixels
    A = pkg.SystemMatrix(P.geom, Ns, pkg.SVR_W_F32)
    A.tune()
    cases = [("osem", dict(), 1), ("svrem", dict(alpha=0.7, eta=1, beta=1e-2), 1),
             ("svrg", dict(alpha=2.0, eta=2, beta=1e-2), 2), ("saga", dict(alpha=2.0, beta=1e-2), 1),
             ("sga", dict(alpha=1.0, beta=1e-2), 1), ("bsrem", dict(alpha=1.0, beta=1e-2), 1),
             ("sem", dict(alpha=1.0, beta=1e-2), 1)]
    calls = max(1, args.steps)
    reps = 5  # the median of five timed blocks of `calls` epoch calls
    out = {}
    for algo, kw, eta in cases:
        R = pkg.Recon(A, P.g, P.w, np.ones((1, N), np.float32), pkg.params(algo, **kw))
        R.osem_epoch(list(range(Ns)))
        per = eta * Ns  # iterations per call: one anchor period for SVREM / SVRG
        orders = [datagen.make_order(Ns, per, seed=4000 + i) for i in range(calls * reps + 5)]
        for i in range(5):
            R.epoch(algo, orders[i])
        times = []
        settle_gc()
        for r in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(calls):
                R.epoch(algo, orders[5 + r * calls + i])
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        el = sorted(times)[reps // 2]
        anchors = 1 if algo in ("svrem", "svrg") else 0  # one anchor pass per call
        epochs = calls * (eta + anchors)
        out[algo] = {"iterations_per_s": round(calls * per / el, 1), "epochs_per_s": round(epochs / el, 1),
                     "ms_per_call": round(el / calls * 1e3, 4), "iterations_per_call": per,
                     "epochs_per_call": eta + anchors}
        log(f"{algo}: {out[algo]}")
        if algo == "svrem":  # the objective (whole forward + log terms + penalty, FP64 sums; synchronises)
            for _ in range(3):
                R.objective()
            t0 = time.perf_counter()
            for _ in range(50):
                R.objective()
            objective_ms = (time.perf_counter() - t0) / 50 * 1e3
        R.close()
    print(json.dumps({"workload": "algos", "metric": "subset iterations/s and epochs/s per update rule",
                      "config": "SVREM 256x256 (2 mm), 252 views x 344 bins, 21 subsets, counts 1e6, FP32 weights",
                      "calls": calls, "repetitions": reps, "results": out,
                      "objective_ms_per_call": round(objective_ms, 4)}), flush=True)


def bench_small(args):
    """The small configuration (64 x 64 at 4 mm, 60 views x 95 bins, 6 subsets,
    attenuation, 1e5 counts): OSEM and SVREM (alpha = 0.7, eta = 1, beta = 0.01)
    epochs/s on the GPU and in the FP64 oracle on one host core, and their
    ratio.  At this size every kernel is a few wavefronts, so the GPU figure is
    the dispatch rate of the dependent launches."""
    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_2106_03172_amd as pkg
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    Ns, N = P.n_subsets, P.geom.n_pixels
    A = pkg.SystemMatrix(P.geom, Ns, pkg.SVR_W_F32, mu=P.mu)
    calls = max(1, args.steps)
    cyc = list(range(Ns))
    out = {}
    # GPU: OSEM epochs (Ns iterations each), then SVREM calls (anchor + Ns iterations = 2 epochs)
    R = pkg.Recon(A, P.g, P.w, np.ones((1, N), np.float32), pkg.params("svrem", alpha=0.7, eta=1, beta=1e-2))
    for _ in range(5):
        R.osem_epoch(cyc)
    settle_gc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        R.osem_epoch(cyc)
    torch.cuda.synchronize()
    out["osem_gpu_epochs_per_s"] = calls / (time.perf_counter() - t0)
    orders = [datagen.make_order(Ns, Ns, seed=500 + i) for i in range(calls + 5)]
    for i in range(5):
        R.svrem_epoch(orders[i])
    settle_gc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(calls):
        R.svrem_epoch(orders[5 + i])
    torch.cuda.synchronize()
    out["svrem_gpu_epochs_per_s"] = 2 * calls / (time.perf_counter() - t0)
    # oracle (FP64, one core): OSEM epochs, then SVREM outer loops
    Ao = oracle.system_matrix(P.geom, P.mu)
    m = oracle.Model(Ao, P.g, P.w, P.geom, Ns)
    f = np.ones((1, N))
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
        f = oracle.osem_epoch(m, f, cyc)
        n += 1
    out["osem_oracle_epochs_per_s"] = n / (time.perf_counter() - t0)
    cpu = cpu_baseline(P, 1e-2, 0.7, 1, min(args.cpu_seconds, 5.0), label="64x64 / 60x95 / 6-subset",
                       max_loops=100000)
    out["svrem_oracle_epochs_per_s"] = cpu["value"]
    out["oracle_cores"] = cpu["cores"]
    out["svrem_gpu_over_oracle"] = out["svrem_gpu_epochs_per_s"] / out["svrem_oracle_epochs_per_s"]
    out["osem_gpu_over_oracle"] = out["osem_gpu_epochs_per_s"] / out["osem_oracle_epochs_per_s"]
    print(json.dumps({"workload": "small", "metric": "OSEM and SVREM epochs/s, GPU and FP64 oracle",
                      "config": "64x64 (4 mm), 60 views x 95 bins, 6 subsets, attenuation, counts 1e5",
                      "calls": calls, **{k: round(v, 2) for k, v in out.items()}}), flush=True)


def bench_projectors(args):
    """The whole-matrix projector calls (svr_project / svr_backproject over every
    subset) and the subset-0 calls on the largest single-image serving size,
    384 x 384 (2 mm), 400 views x 518 bins, 21 subsets: 75 M non-zeros with
    32-bit indices, 602 MB per layout, so neither layout fits the 256 MB
    Infinity Cache and the streams come from HBM.  Algorithmic bytes: index and
    weight of every non-zero, row pointers, the input read once and the output
    written once (plus the input permutation or tiling the call performs)."""
    import numpy as np
    import torch

    import datagen
    import paper_2106_03172_amd as pkg
    geom = datagen.Geometry(384, 384, 2.0, 400, 518, 2.0)
    Ns, N, M = 21, geom.n_pixels, geom.n_rays
    wt = {"f32": pkg.SVR_W_F32, "f16": pkg.SVR_W_F16, "bf16": pkg.SVR_W_BF16}[args.wtype]
    wb = 4 if args.wtype == "f32" else 2
    A = pkg.SystemMatrix(geom, Ns, wt)
    inf, per_subset = A.info()
    ib = inf.index_bytes
    x = torch.rand(1, N, device="cuda")
    y = torch.rand(1, M, device="cuda")
    yo = torch.empty(1, M, device="cuda")
    xo = torch.empty(1, N, device="cuda")
    reps = max(1, args.steps)
    out = {"workload": "projectors", "config": "384x384 (2 mm), 400 views x 518 bins, 21 subsets",
           "nnz": int(inf.nnz), "index_bytes": ib, "wtype": args.wtype,
           "layout_mb": round(inf.nnz * (ib + wb) / 1e6, 1)}
    for label, subset in (("all", -1), ("subset0", 0)):
        for _ in range(3):
            A.project(x, subset, yo)
            A.backproject(y, subset, xo)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(reps):
            A.project(x, subset, yo)
        ev[1].record()
        for _ in range(reps):
            A.backproject(y, subset, xo)
        ev[2].record()
        torch.cuda.synchronize()
        f_s = ev[0].elapsed_time(ev[1]) / reps / 1e3
        b_s = ev[1].elapsed_time(ev[2]) / reps / 1e3
        nnz = inf.nnz if subset < 0 else int(np.asarray(per_subset)[0])
        rows = M if subset < 0 else ((geom.n_views + Ns - 1) // Ns) * geom.n_bins
        f_b = nnz * (ib + wb) + 4 * (rows + 1) + 4 * N + 4 * rows
        b_b = nnz * (ib + wb) + 4 * ((Ns if subset < 0 else 1) * N + 1) + 4 * N + 8 * M + 4 * rows
        out[label] = {"forward_us": round(f_s * 1e6, 2), "back_us": round(b_s * 1e6, 2),
                      "forward_gbs": round(f_b / f_s / 1e9, 1), "back_gbs": round(b_b / b_s / 1e9, 1),
                      "forward_bytes": int(f_b), "back_bytes": int(b_b)}
        log(f"{label}: {out[label]}")
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """The precision sweep of the headline problem (256 x 256, 252 x 344, 21
    subsets, counts 1e6, beta 1e-2): for FP32, FP16 and BF16 weights, SVREM
    epochs/s (alpha 0.7, eta 1), the whole-matrix projector kernels' GB/s
    (forward and back-projection calls over all subsets, algorithmic bytes of
    the stored weight type) and, after 50 epochs, the relative L2 error of the
    iterate and the relative error of the objective against the FP64 oracle
    run with the exact lengths on the same subset sequence."""
    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_2106_03172_amd as pkg
    P = datagen.make_problem(**datagen.CONFIG_HEADLINE)
    Ns, N, M = P.n_subsets, P.geom.n_pixels, P.geom.n_rays
    beta, calls = 1e-2, 25
    orders = [datagen.make_order(Ns, Ns, seed=3000 + 100 * c) for c in range(calls)]
    log("oracle: 50 epochs of SVREM in FP64")
    Ao = oracle.system_matrix(P.geom)
    m = oracle.Model(Ao, P.g, P.w, P.geom, Ns, beta=beta)
    alg = oracle.SVREM(m, oracle.osem_epoch(m, np.ones((1, N)), range(Ns)), 0.7, 1)
    for o in orders:
        alg.run(o)
    f_or, phi_or = alg.f, m.objective(alg.f)
    out = {"workload": "precision", "config": "SVREM 256x256 (2 mm), 252 views x 344 bins, 21 subsets, counts 1e6, "
                                              "beta 1e-2, alpha 0.7, eta 1; 50 epochs against the FP64 oracle",
           "results": {}}
    for name, wt, wb in (("f32", pkg.SVR_W_F32, 4), ("f16", pkg.SVR_W_F16, 2), ("bf16", pkg.SVR_W_BF16, 2)):
        A = pkg.SystemMatrix(P.geom, Ns, wt)
        A.tune()
        inf, _ = A.info()
        R = pkg.Recon(A, P.g, P.w, np.ones((1, N), np.float32), pkg.params("svrem", alpha=0.7, eta=1, beta=beta))
        R.osem_epoch(list(range(Ns)))
        for o in orders:
            R.svrem_epoch(o)
        fg = R.image().cpu().numpy()
        err = float(np.linalg.norm(fg - f_or) / np.linalg.norm(f_or))
        phi_err = abs(R.objective() - phi_or) / abs(phi_or)
        steps = max(1, args.steps)
        extra = [datagen.make_order(Ns, Ns, seed=8000 + i) for i in range(steps + 5)]
        for o in extra[:5]:
            R.svrem_epoch(o)
        settle_gc()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for o in extra[5:]:
            R.svrem_epoch(o)
        torch.cuda.synchronize()
        eps = 2 * steps / (time.perf_counter() - t0)
        x = torch.rand(1, N, device="cuda")
        y = torch.rand(1, M, device="cuda")
        yo, xo = torch.empty(1, M, device="cuda"), torch.empty(1, N, device="cuda")
        for _ in range(3):
            A.project(x, -1, yo)
            A.backproject(y, -1, xo)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(20):
            A.project(x, -1, yo)
        ev[1].record()
        for _ in range(20):
            A.backproject(y, -1, xo)
        ev[2].record()
        torch.cuda.synchronize()
        ib = inf.index_bytes
        f_s, b_s = ev[0].elapsed_time(ev[1]) / 20e3, ev[1].elapsed_time(ev[2]) / 20e3
        f_b = inf.nnz * (ib + wb) + 4 * (M + 1) + 4 * N + 4 * M
        b_b = inf.nnz * (ib + wb) + 4 * (Ns * N + 1) + 4 * N + 12 * M
        out["results"][name] = {"iterate_rel_l2": err, "objective_rel": phi_err, "svrem_epochs_per_s": round(eps, 1),
                                "projector_forward_gbs": round(f_b / f_s / 1e9, 1),
                                "projector_back_gbs": round(b_b / b_s / 1e9, 1),
                                "projector_forward_us": round(f_s * 1e6, 2), "projector_back_us": round(b_s * 1e6, 2),
                                "matrix_mb": round(inf.nnz * (ib + wb) / 1e6, 1)}
        log(f"{name}: {out['results'][name]}")
        R.close()
        A.close()
    print(json.dumps(out), flush=True)


def bench_copy(args):
    """A plain device copy of a known size (256 MiB read + 256 MiB written per
    launch): the calibration run for the HBM byte counters of rocprofv3."""
    import torch
    n = 64 << 20  # floats
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(max(1, args.steps)):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": max(1, args.steps)}), flush=True)


def bench_multislice(args):
    """SVREM on a stack of 127 slices of 285 x 285 (2.5 mm) sharing one 2D matrix
    (344 views x 435 bins, 21 subsets), in-plane 8-neighbour + 2 axial quadratic
    penalty, one sparse-times-dense product per subset and phase."""
    import numpy as np
    import torch

    import datagen
    import paper_2106_03172_amd as pkg
    cfg = datagen.CONFIG_MULTISLICE
    wt = {"f32": pkg.SVR_W_F32, "f16": pkg.SVR_W_F16, "bf16": pkg.SVR_W_BF16}[args.wtype]
    wb = 4 if args.wtype == "f32" else 2
    log("generating the 127-slice stack")
    P = datagen.make_multislice_problem(cfg["nx"], cfg["ny"], cfg["pixel_mm"], cfg["n_views"], cfg["n_bins"],
                                        cfg["bin_mm"], cfg["n_subsets"], cfg["counts"], n_slices=cfg["n_slices"],
                                        seed=cfg["seed"])
    Ns, S, N, M = cfg["n_subsets"], cfg["n_slices"], P.geom.n_pixels, P.geom.n_rays
    A = pkg.SystemMatrix(P.geom, Ns, wt)
    inf, per_subset = A.info()
    prm = pkg.params("svrem", alpha=args.alpha, eta=args.eta, beta=args.beta,
                     flags=pkg.binding.FLAG_AXIAL_PENALTY)
    R = pkg.Recon(A, P.g, P.w, np.ones((S, N), dtype=np.float32), prm)
    R.osem_epoch(list(range(Ns)))
    per = args.eta * Ns
    steps = max(1, args.steps)
    orders = [datagen.make_order(Ns, per, seed=700 + i) for i in range(args.warmup + 2 * steps)]
    for i in range(args.warmup):
        R.svrem_epoch(orders[i])
    settle_gc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        R.svrem_epoch(orders[args.warmup + i])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    R.set_profiling(True)
    used = []
    for i in range(steps):
        o = orders[args.warmup + steps + i]
        used.extend(int(t) for t in o)
        R.svrem_epoch(o)
    kt = R.kernel_times()
    R.set_profiling(False)
    nnz_t = float(np.mean([per_subset[t] for t in used]))
    Mt = float(np.mean([len(range(t, P.geom.n_views, Ns)) * P.geom.n_bins for t in used]))
    # algorithmic bytes: the matrix rows once, the image or ratio block once, data, state
    ib = inf.index_bytes
    byts = {"forward": nnz_t * (ib + wb) + 4 * (Mt + 1) + 4 * N * S + 12 * Mt * S,
            "update": nnz_t * (ib + wb) + 4 * (N + 1) + 4 * Mt * S + 8 * N + 36 * N * S,
            "anchor_forward": inf.nnz * (ib + wb) + 4 * (M + 1) + 4 * N * S + 12 * M * S,
            "anchor_table": inf.nnz * (ib + wb) + 4 * (Ns * N + 1) + 4 * M * S + 4 * N * S + 4 * Ns * N * S,
            "anchor_sum": 4 * Ns * N * S + 8 * N * S}
    kernels = {}
    tot = sum(v[1] for v in kt.values())
    for name, (n, ms) in kt.items():
        if n:
            avg = ms / n / 1e3
            kernels[name] = {"launches": n, "avg_us": round(avg * 1e6, 2), "share": round(ms / tot, 3),
                             "gbs": round(byts[name] / avg / 1e9, 1)}
    value = steps * (args.eta + 1) / el
    print(json.dumps({"workload": "multislice", "metric": "SVREM stack epochs/s (127 x 285^2, 344x435, 21 subsets)",
                      "value": round(value, 3), "slice_epochs_per_s": round(value * S, 1), "unit": "epochs/s",
                      "ms_per_step": round(1e3 * el / steps, 3), "steps": steps, "wtype": args.wtype,
                      "nnz": int(inf.nnz), "kernels": kernels, "objective_after": R.objective()}), flush=True)


def _serving_data(n):
    """The first ``n`` requests of the seeded serving stream (sizes from
    {128, 192, 256, 384}^2, views in [120, 400], bins 1.35 N, subsets in
    {8, 14, 21}, counts log-uniform in [1e5, 1e7], SVREM 30 epochs)."""
    import datagen
    specs = datagen.serving_requests(n, 1.0, seed=0)
    log(f"generating {n} requests")
    data = [datagen.make_problem(r["nx"], r["ny"], r["pixel_mm"], r["n_views"], r["n_bins"], r["bin_mm"],
                                 r["n_subsets"], r["counts"], seed=r["seed"]) for r in specs]
    return specs, data


def serve_latency(specs, data, alpha, share=True, rate=None):
    """Continuous batching with Poisson arrivals: capacity from all requests at
    once (the second of two such runs), then a Poisson stream at ``rate``
    (default 0.8 of the capacity); latency from arrival to completion.
    ``share``: requests of one geometry share a matrix.  One server serves
    the three runs, as a long-lived service would: the device blocks it keeps
    carry over from run to run, its matrices do not (each run starts by
    dropping the idle ones), so every run builds the matrices it needs."""
    import numpy as np

    import paper_2106_03172_amd as pkg
    n = len(data)
    prm = pkg.params("svrem", alpha=alpha, eta=1, beta=1e-3)
    budget = 64 << 30
    S = pkg.Server(budget, max_slots=16, n_streams=8, share_matrices=share)

    def run(arrivals):
        S.trim(drop_matrices=True, keep_bytes=budget)
        order = np.argsort(arrivals)
        done, owner = {}, {}  # owner: pending ticket -> request index
        nxt = 0
        settle_gc()
        t0 = time.perf_counter()
        while len(done) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                P = data[i]
                owner[S.submit(P.geom, P.n_subsets, P.g, P.w, prm, specs[i]["epochs"], 1000 + i)] = i
                nxt += 1
            if owner:
                S.step(1)
            elif nxt < n:
                time.sleep(max(0.0, arrivals[order[nxt]] - (time.perf_counter() - t0)))
            for t in S.done():
                i = owner.pop(t)
                res = S.poll(t)
                done[i] = (time.perf_counter() - t0 - arrivals[i], res)
        total = time.perf_counter() - t0
        return done, total

    run(np.zeros(n))  # warm-up: code objects, allocator pools
    done, total = run(np.zeros(n))
    capacity = n / total
    log(f"capacity {capacity:.2f} requests/s (all {n} at t=0, {total:.2f} s)")
    if rate is None:
        rate = 0.8 * capacity
    gaps = np.random.Generator(np.random.PCG64(4001)).exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps)
    done, total = run(arrivals)
    S.close()
    lat = np.array([done[i][0] for i in range(n)]) * 1e3
    ok = all(done[i][1]["status"] == 0 for i in range(n))
    return {"requests": n, "capacity_rps": round(capacity, 3), "offered_rps": round(rate, 3),
            "achieved_rps": round(n / total, 3), "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2), "mean_ms": round(float(lat.mean()), 2),
            "all_ok": ok, "epochs_per_request": specs[0]["epochs"]}


def serve_compare(specs, data, alpha):
    """The same requests (SVREM, 30 epochs each, the subset sequence of each
    request from its seed) four ways: the plain per-request path (FP32
    weights; build the matrix, one OSEM epoch, the SVREM epochs, one request
    after the other, through SystemMatrix / Recon), and the continuous-batching
    server with every request submitted at once: each request's epochs on one
    of 8 streams (FP32), and the subset iterations batched into one launch per
    phase (FP32, BF16 and FP16 weights).  SVREM epochs/s of each and, over the
    requests, the relative L2 difference of each result from the per-request
    FP32 one (the GPU tests pin every weight type against the FP64 oracle).
    The server forms run on two long-lived servers (per-stream and batched),
    each warmed by one untimed pass and cleared of its idle matrices before
    every pass, so every pass builds its matrices."""
    import numpy as np
    import torch

    import paper_2106_03172_amd as pkg
    n = len(data)
    prm = pkg.params("svrem", alpha=alpha, eta=1, beta=1e-3)
    epochs = [int(r["epochs"]) for r in specs]
    total_epochs = sum(epochs)

    def per_request():
        out = []
        settle_gc()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, P in enumerate(data):
            A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
            R = pkg.Recon(A, P.g, P.w, np.ones((1, P.geom.n_pixels), np.float32), prm)
            R.osem_epoch(list(range(P.n_subsets)))
            R.svrem_epoch(np.concatenate(pkg.splitmix64_orders(1000 + i, P.n_subsets, epochs[i])))
            out.append(R.image().cpu().numpy()[0])
            R.close()
            A.close()
        return out, time.perf_counter() - t0

    budget = 64 << 30
    servers = {b: pkg.Server(budget, max_slots=16, n_streams=8, batch=b) for b in (False, True)}

    def served(wtype, batch=True):
        S = servers[batch]
        S.trim(drop_matrices=True, keep_bytes=budget)
        settle_gc()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, epochs[i], 1000 + i, wtype=wtype)
                   for i, P in enumerate(data)]
        res = {}
        index = {t: i for i, t in enumerate(tickets)}
        while len(res) < n:
            S.step(1)
            for t in S.done():
                res[index[t]] = S.poll(t)
        total = time.perf_counter() - t0
        assert all(res[i]["status"] == 0 for i in range(n))
        return [res[i]["f"] for i in range(n)], total

    per_request()  # warm-up: code objects, allocator pools
    f_req, t_req = per_request()
    log(f"per-request FP32: {t_req:.3f} s")
    served(pkg.SVR_W_F32, batch=False)  # warm-ups
    served(pkg.SVR_W_F32)
    f32_str, t_str = served(pkg.SVR_W_F32, batch=False)
    f32_srv, t_f32 = served(pkg.SVR_W_F32)
    f_bf, t_bf = served(pkg.SVR_W_BF16)
    f_h, t_h = served(pkg.SVR_W_F16)
    for S in servers.values():
        S.close()
    log(f"8 streams FP32 {t_str:.3f} s, batched FP32 {t_f32:.3f} s, BF16 {t_bf:.3f} s, FP16 {t_h:.3f} s")

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    def entry(t, f=None):
        e = {"seconds": round(t, 4), "epochs_per_s": round(total_epochs / t, 1)}
        if f is not None:
            d = [rel(f[i], f_req[i]) for i in range(n)]
            e.update(max_rel_diff_vs_f32=float(max(d)), median_rel_diff_vs_f32=float(np.median(d)))
        return e
    return {"requests": n, "epochs": total_epochs, "per_request_f32": entry(t_req),
            "streams_f32": entry(t_str, f32_str), "batched_f32": entry(t_f32, f32_srv),
            "batched_bf16": entry(t_bf, f_bf), "batched_f16": entry(t_h, f_h),
            "speedup_bf16_batched_vs_f32_per_request": round(t_req / t_bf, 3),
            "speedup_f16_batched_vs_f32_per_request": round(t_req / t_h, 3)}


def bench_serve(args):
    """p50/p99 latency of --requests serving requests with Poisson arrivals."""
    specs, data = _serving_data(args.requests)
    out = serve_latency(specs, data, args.alpha)
    print(json.dumps({"workload": "serve", "metric": "p50/p99 recon latency and requests/s (Poisson arrivals)",
                      **out}), flush=True)


def bench_serve_scanner(args):
    """Requests from one scanner (one geometry, different data): capacity and
    Poisson-arrival latency with the requests sharing one matrix and with each
    building its own, both at 0.8 of the latter's capacity."""
    import datagen
    specs = datagen.scanner_requests(args.requests)
    log(f"generating {len(specs)} requests of one geometry")
    data = [datagen.make_problem(r["nx"], r["ny"], r["pixel_mm"], r["n_views"], r["n_bins"], r["bin_mm"],
                                 r["n_subsets"], r["counts"], seed=r["seed"]) for r in specs]
    own = serve_latency(specs, data, args.alpha, share=False)
    shared = serve_latency(specs, data, args.alpha, share=True, rate=own["offered_rps"])
    print(json.dumps({"workload": "serve-scanner",
                      "metric": "p50/p99 recon latency and requests/s, one scanner geometry (256^2, 252 x 344, "
                                "21 subsets), shared matrix against one matrix per request",
                      "shared": shared, "own_matrix": own,
                      "capacity_ratio": round(shared["capacity_rps"] / own["capacity_rps"], 3)}), flush=True)


def bench_serve_compare(args):
    """Batched FP32 / BF16 / FP16 serving against the plain FP32 per-request path."""
    specs, data = _serving_data(min(args.requests, 64))
    out = serve_compare(specs, data, args.alpha)
    print(json.dumps({"workload": "serve-compare", "metric": "SVREM epochs/s over a set of serving requests",
                      **out}), flush=True)


if __name__ == "__main__":
    main()
