"""Benchmark: time to a 1e-10 relative residual and achieved HBM bandwidth of
the matrix-powers + Gram phase, adaptive s-step CG on one MI355X.

Workload: 3-D 7-point Dirichlet Poisson on a 256^3 grid (N = 16,777,216,
nnz = 117,047,296, FP64 CSR, two-sided diagonal scaling), b = A x* with
x* ~ U(-1, 1) (seed 102), x0 = 0, sigma = 10, tol = 1e-10.  One step is one
complete solve (all of the hot path: setup, every outer loop's matrix
powers, Gram, controller, recovery and convergence checks) with A, b and
x0 resident in HBM.  The Newton basis and the plain HSCG comparator are
timed on the same GPU and reported beside it; the CPU oracle is timed on a
bounded sample on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--size 256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0        # MI355X HBM3E, vendor figure


COUNTER_FILE = os.path.join(ROOT, "profiles", "hbm_counters_poisson3d_256.txt")
KERNEL_SOURCES = ["kernels.hip", "device.hpp", "launch.hpp", "ctl.hpp"]


def measured_traffic(kernel: str):
    """HBM bytes per launch of the sweep kernel ``kernel`` (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated) from the committed counter summary of the
    256^3 workload, or None when the kernel sources no longer hash to the
    ones that were measured."""
    import hashlib
    try:
        text = open(COUNTER_FILE).read()
    except OSError:
        return None
    csrc = os.path.join(ROOT, "paper_1908_04081_amd", "csrc")
    digest = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                     for f in KERNEL_SOURCES)).hexdigest()[:16]
    if f"ctl.hpp): {digest}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"traffic {kernel} per launch (bytes):"):
            return int(line.split(":")[1])
    return None


def matrix_bytes(A, fmt: str) -> int:
    """|A|, the bytes one read of the matrix moves in the storage the kernels
    use: CSR 12 nnz + 4 (n + 1) (FP64 values, int32 columns and row
    pointers); diagonal storage 8 nd n (FP64 values, nd diagonals of n
    positions, no indices)."""
    n = A.shape[0]
    if fmt == "dia":
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.indptr))
        nd = int(np.unique(A.indices.astype(np.int64) - rows).size)
        return 8 * nd * n
    return 12 * int(A.nnz) + 4 * (n + 1)


def mpk_bytes(n: int, abytes: int, s: int, chebyshev: bool):
    """Algorithmic HBM bytes of one outer loop's matrix powers + Gram (s
    levels), and of one two-chain sweep at level >= 2, for a matrix read of
    ``abytes`` = |A| (matrix_bytes).

    Sweep l (1 <= l < s): |A| + read level l-1 pairs (16 n) + write level l
    pairs (16 n) + for l >= 2 with a mu term (Chebyshev) read level l-2 pairs
    (16 n).  Last sweep + Gram: |A| + read the s pair levels (16 s n) + write
    P_s (8 n)."""
    A = abytes
    sweep_ge2 = A + (48 if chebyshev else 32) * n
    sweep1 = A + 32 * n
    last = A + 16 * s * n + 8 * n
    total = sweep1 + (s - 2) * sweep_ge2 + last if s >= 2 else last
    return total, sweep_ge2, sweep1, last


def time_solves(run, warmup, steps, torch):
    """``warmup`` untimed calls of ``run()``, then ``steps`` timed ones, the
    device synchronized before and after each; returns the per-call wall
    times and the last call's result."""
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    times, res = [], None
    for _ in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    return times, res


def summary(times, info, extra=None):
    d = {"s_median": round(float(np.median(times)), 5), "s_min": round(min(times), 5),
         "s_mean": round(float(np.mean(times)), 5), "runs": len(times),
         "outer_iters": info["outer_iters"], "total_iters": info["total_iters"],
         "outcome": info["outcome_name"], "relres_true": info["relres_true"]}
    if extra:
        d.update(extra)
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-compare", action="store_true", help="skip Newton and HSCG runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-system batched workload")
    ap.add_argument("--no-grad", action="store_true", help="skip the differentiable workload")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the table of the paper's comparison methods")
    ap.add_argument("--no-diffusion", action="store_true",
                    help="skip the 160^3 27-point diffusion workload")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 64x64 Poisson workload (GPU and oracle times)")
    ap.add_argument("--no-probe", action="store_true", help="skip the bandwidth probes")
    ap.add_argument("--format", choices=["auto", "csr", "dia"], default="auto",
                    help="storage of A for the matrix-powers kernels (assg_set_format)")
    ap.add_argument("--sizes", type=str, default="",
                    help="only a size sweep of the 7-point workload, e.g. 32,64,128 (sides)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (its path on one GPU's share of the "
              "rows; sharding across GPUs is not built); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1908_04081_amd as L
    import spd_problems as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sizes:
        print(json.dumps({"size_sweep": bench_sizes(L, P, torch, [int(v) for v in
                                                                  args.sizes.split(",")],
                                                    args.warmup, args.steps)}))
        return
    ceilings = None if args.no_probe else bandwidth_ceilings(torch, dev)
    t0 = time.perf_counter()
    pr = P.make_config("poisson3d_256", size=args.size)
    n, nnz = pr.n, pr.A.nnz
    print(f"[bench] generated {pr.name} n={n} nnz={nnz} in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    A = L.csr_to_device(pr.A, dev)
    b = torch.from_numpy(pr.b).to(dev)
    x = torch.zeros_like(b)
    h = L.assg_create()
    L.assg_set_format(h, args.format)
    L.assg_analyze(h, A)
    fmt = L.assg_get_format(h)
    abytes = matrix_bytes(pr.A, fmt)
    sweep_kernel = "k_sweep_dia" if fmt == "dia" else "k_sweep"
    sigma, tol = 10, 1e-10
    max_iters = 200000

    def solve(basis, timing=False):
        x.zero_()
        opts = L.assg_default_opts(s_max=sigma, s_init=sigma, growth=sigma, tol=tol, basis=basis,
                                   max_iters=max_iters, time_kernels=1 if timing else 0)
        return L.assg_solve(h, A, b, x, opts)

    def hscg():
        x.zero_()
        return L.assg_hscg_solve(h, A, b, x, tol, max_iters)

    # ---- the headline: adaptive s-step CG, Chebyshev basis, production path
    # (outer loops replayed from the captured graph); exactly --steps timed
    # solves between two device synchronizations
    for _ in range(args.warmup):
        solve("chebyshev")
    torch.cuda.synchronize()
    per, last = [], None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        last = solve("chebyshev")
        per.append(last["solve_ms"] * 1e-3)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    xg = x.cpu().numpy()
    relres = float(np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b))
    print(f"[bench] chebyshev: {ms_step:.1f} ms/solve outer={last['outer_iters']} "
          f"iters={last['total_iters']} relres(host)={relres:.3e} {last['outcome_name']}",
          file=sys.stderr, flush=True)

    extra = {}
    methods = {"chebyshev": {"s_median_device": round(float(np.median(per)), 5),
                             "s_min_device": round(min(per), 5), "s_mean_wall": round(ms_step * 1e-3, 5),
                             "runs": args.steps, "outer_iters": last["outer_iters"],
                             "total_iters": last["total_iters"], "outcome": last["outcome_name"],
                             "relres_true": last["relres_true"]}}
    if not args.no_compare:
        # Newton basis and plain HSCG, the same protocol (warm-up, then timed
        # solves on the production path; median and min)
        tn, inf_n = time_solves(lambda: solve("newton"), args.warmup, args.steps, torch)
        th, inf_h = time_solves(hscg, args.warmup, args.steps, torch)
        tc, inf_c = time_solves(lambda: solve("chebyshev"), 0, args.steps, torch)
        methods["chebyshev_wall"] = summary(tc, inf_c)
        methods["newton"] = summary(tn, inf_n)
        methods["hscg"] = summary(th, inf_h)
        extra["speedup_vs_hscg"] = {
            "chebyshev": round(float(np.median(th)) / float(np.median(tc)), 3),
            "newton": round(float(np.median(th)) / float(np.median(tn)), 3),
            "basis": "median wall time of --steps solves each, same warm-up"}
        print(f"[bench] median wall: chebyshev {np.median(tc)*1e3:.1f} ms, newton "
              f"{np.median(tn)*1e3:.1f} ms, hscg {np.median(th)*1e3:.1f} ms",
              file=sys.stderr, flush=True)
    extra["methods"] = methods

    # ---- per-kernel times: a separate solve with HIP events around every
    # matrix-powers launch on the library's stream (same kernels, launched
    # one by one instead of from the graph; bit-identical iterates)
    kt = solve("chebyshev", timing=True)
    tot_b, sweep_b, sweep1_b, last_b = mpk_bytes(n, abytes, sigma, True)
    sweep_avg_ms = kt["sweep_ms"] / max(kt["sweep_launches"], 1)
    achieved = sweep_b / (sweep_avg_ms * 1e-3) / 1e9
    lastg_avg_ms = kt["last_gram_ms"] / max(kt["last_gram_launches"], 1)
    mpk_time_ms = (kt["sweep_ms"] + kt["sweep1_ms"] + kt["last_gram_ms"]) / \
        max(kt["last_gram_launches"], 1)      # per outer loop
    mpk_gbps = tot_b / (mpk_time_ms * 1e-3) / 1e9
    if not args.no_compare:
        kn = solve("newton", timing=True)
        _, sweep_nb, _, _ = mpk_bytes(n, abytes, sigma, False)
        nav = kn["sweep_ms"] / max(kn["sweep_launches"], 1)
        methods["newton"]["sweep_avg_ms"] = round(nav, 4)
        methods["newton"]["sweep_GBps"] = round(sweep_nb / (nav * 1e-3) / 1e9, 1)

    if not args.no_compare and fmt != "csr":
        # the same three methods with the CSR storage forced (A read as it is
        # handed over), the same protocol, on a handle of its own
        h2 = L.assg_create()
        L.assg_set_format(h2, "csr")
        L.assg_analyze(h2, A)

        def solve_csr(basis):
            x.zero_()
            return L.assg_solve(h2, A, b, x, L.assg_default_opts(
                s_max=sigma, s_init=sigma, growth=sigma, tol=tol, basis=basis,
                max_iters=max_iters))

        def hscg_csr():
            x.zero_()
            return L.assg_hscg_solve(h2, A, b, x, tol, max_iters)

        tc2, ic2 = time_solves(lambda: solve_csr("chebyshev"), args.warmup, args.steps, torch)
        tn2, in2 = time_solves(lambda: solve_csr("newton"), args.warmup, args.steps, torch)
        th2, ih2 = time_solves(hscg_csr, args.warmup, args.steps, torch)
        extra["csr_storage"] = {
            "format": L.assg_get_format(h2), "matrix_bytes": matrix_bytes(pr.A, "csr"),
            "chebyshev": summary(tc2, ic2), "newton": summary(tn2, in2),
            "hscg": summary(th2, ih2),
            "speedup_vs_hscg": {
                "chebyshev": round(float(np.median(th2)) / float(np.median(tc2)), 3),
                "newton": round(float(np.median(th2)) / float(np.median(tn2)), 3)}}
        print(f"[bench] CSR storage, median wall: chebyshev {np.median(tc2)*1e3:.1f} ms, newton "
              f"{np.median(tn2)*1e3:.1f} ms, hscg {np.median(th2)*1e3:.1f} ms",
              file=sys.stderr, flush=True)
        L.assg_destroy(h2)

    if not args.no_small:
        extra["poisson2d_64"] = bench_small(L, P, torch, args.warmup, args.steps)
    if not args.no_diffusion:
        extra["diffusion27_160"] = bench_diffusion(L, P, torch, args.warmup, args.steps)
    if not args.no_variants:
        extra["variants"] = bench_variants(L, P, torch)
    if not args.no_batch:
        extra["batched"] = bench_batch(L, P, torch)
    if not args.no_grad:
        extra["differentiable"] = bench_grad(L, P, torch)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pr, sigma, tol, last["outer_iters"])

    out = {
        "metric": "time-to-1e-10 rel. residual; achieved HBM GB/s of matrix-powers+Gram",
        "value": round(ms_step * 1e-3, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"poisson3d_{args.size}: 3-D 7-point Poisson {args.size}^3, scaled, "
                        "b = A x*, x* ~ U(-1,1) seed 102, x0 = 0",
            "n": n, "nnz": nnz, "method": "improved adaptive s-step CG", "basis": "chebyshev",
            "s_max": sigma, "tol": tol, "format": fmt, "matrix_bytes": abytes,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{sweep_kernel} (two-chain matrix-powers level, levels >= 2)",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": measured_traffic(sweep_kernel) if args.size == 256 else None,
            "bytes_per_launch": sweep_b,
            "avg_launch_ms": round(sweep_avg_ms, 5),
            "launches": kt["sweep_launches"],
            "timing": "HIP events on the library's stream around each launch, in a separate "
                      "solve of the same workload with time_kernels=1",
        },
        "mpk_gram": {
            "GBps": round(mpk_gbps, 1), "frac": round(mpk_gbps / PEAK_HBM_GBPS, 4),
            "bytes_per_outer_loop": tot_b, "ms_per_outer_loop": round(mpk_time_ms, 4),
            "last_gram_avg_ms": round(lastg_avg_ms, 4),
            "last_gram_GBps": round(last_b / (lastg_avg_ms * 1e-3) / 1e9, 1),
            "last_gram_frac": round(last_b / (lastg_avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
            "sweep1_avg_ms": round(kt["sweep1_ms"] / max(kt["sweep1_launches"], 1), 4),
        },
        "ceilings": ceilings,
        "solve": {"outer_iters": last["outer_iters"], "total_iters": last["total_iters"],
                  "relres_true": relres, "outcome": last["outcome_name"],
                  "device_solve_ms": round(last["solve_ms"], 3)},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))
    L.assg_destroy(h)


def bench_sizes(L, P, torch, sides, warmup, steps):
    """The 7-point Poisson workload (same recipe, b = A x*, tol 1e-10,
    sigma = 10) at other grid sides: adaptive s-step CG with both bases and
    HSCG, each warm-up then --steps timed solves on the production path
    (median wall time)."""
    rows = []
    for side in sides:
        pr = P.make_config("poisson3d_256", size=side)
        A = L.csr_to_device(pr.A)
        b = torch.from_numpy(pr.b).cuda()
        x = torch.zeros_like(b)
        h = L.assg_create()
        L.assg_analyze(h, A)
        row = {"side": side, "n": pr.n, "format": L.assg_get_format(h)}
        for m in ("chebyshev", "newton", "hscg"):
            def run(m=m):
                x.zero_()
                if m == "hscg":
                    return L.assg_hscg_solve(h, A, b, x, 1e-10, 0)
                return L.assg_solve(h, A, b, x, L.assg_default_opts(s_max=10, tol=1e-10, basis=m))
            t, inf = time_solves(run, warmup, steps, torch)
            row[m + "_ms"] = round(1e3 * float(np.median(t)), 3)
            row[m + "_outer"] = inf["outer_iters"]
            row[m + "_iters"] = inf["total_iters"]
        row["chebyshev_speedup"] = round(row["hscg_ms"] / row["chebyshev_ms"], 3)
        row["newton_speedup"] = round(row["hscg_ms"] / row["newton_ms"], 3)
        L.assg_destroy(h)
        print(f"[bench] {side}^3: chebyshev {row['chebyshev_ms']} ms, newton {row['newton_ms']} ms, "
              f"hscg {row['hscg_ms']} ms", file=sys.stderr, flush=True)
        rows.append(row)
    return rows


def bandwidth_ceilings(torch, dev):
    """Measured ceilings of this GPU (project-written probe kernels, HIP
    events): a streaming read and a streaming copy of 1 GiB, and repeated
    ordinary reads of a 128 MiB buffer (served by the 256 MB Infinity Cache
    after the first pass)."""
    from paper_1908_04081_amd import bwprobe
    big = torch.ones(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
    dst = torch.empty_like(big)
    read_nt, ms_r = bwprobe.read_gbps(big, nontemporal=True)
    read_t, _ = bwprobe.read_gbps(big, nontemporal=False)
    copy, ms_c = bwprobe.copy_gbps(big, dst)
    del dst
    # ordinary loads of buffers of growing size read again and again: the
    # 4 MB L2 of each XCD (every workgroup index lands on the same XCD on
    # every pass), the 256 MB Infinity Cache, then HBM
    reread = {}
    for mib in (8, 32, 64, 128, 192, 512):
        part = big[: mib << 17]
        reread[str(mib)], _ = bwprobe.read_gbps(part, nontemporal=False, iters=50)
        reread[str(mib)] = round(reread[str(mib)], 1)
    del big
    out = {"stream_read_1GiB_GBps": round(read_nt, 1), "read_1GiB_cached_loads_GBps": round(read_t, 1),
           "stream_copy_1GiB_GBps": round(copy, 1), "reread_GBps_by_MiB": reread,
           "peak_GBps": PEAK_HBM_GBPS,
           "note": "paper_1908_04081_amd/bwprobe kernels; copy counts read + write bytes"}
    print(f"[bench] ceilings: {out}", file=sys.stderr, flush=True)
    return out


def bench_small(L, P, torch, warmup, steps):
    """64 x 64 Poisson (N = 4,096), Chebyshev, sigma = 10, tol 1e-10: GPU
    s-step and GPU HSCG (warm-up, then timed solves; median and min), and the
    oracle's adaptive s-step CG and HSCG to the same tolerance on the host,
    three times each."""
    import oracle as O
    pr = P.make_config("poisson2d_64")
    A = L.csr_to_device(pr.A)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    h = L.assg_create()
    L.assg_analyze(h, A)
    fmt = L.assg_get_format(h)
    opts = L.assg_default_opts(s_max=10, tol=1e-10, basis="chebyshev")

    def ss():
        x.zero_()
        return L.assg_solve(h, A, b, x, opts)

    def hs():
        x.zero_()
        return L.assg_hscg_solve(h, A, b, x, 1e-10, 0)

    k = max(steps, 5)
    ts, i_s = time_solves(ss, max(warmup, 1), k, torch)
    th, i_h = time_solves(hs, max(warmup, 1), k, torch)
    L.assg_destroy(h)
    to, th_o = [], []
    for _ in range(3):
        t = time.perf_counter()
        _, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis="chebyshev",
                                    record=False)
        to.append(time.perf_counter() - t)
        t = time.perf_counter()
        _, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
        th_o.append(time.perf_counter() - t)
    out = {"n": pr.n, "nnz": int(pr.A.nnz), "format": fmt, "gpu_sstep": summary(ts, i_s), "gpu_hscg": summary(th, i_h),
           "oracle_sstep": {"s_median": round(float(np.median(to)), 4), "s_min": round(min(to), 4),
                            "runs": 3, "outer_iters": io["outer"], "total_iters": io["iters"]},
           "oracle_hscg": {"s_median": round(float(np.median(th_o)), 4), "s_min": round(min(th_o), 4),
                           "runs": 3, "iters": ih["iters"]},
           "speedup_vs_gpu_hscg": round(float(np.median(th)) / float(np.median(ts)), 3)}
    print(f"[bench] poisson2d_64: gpu s-step {np.median(ts)*1e3:.2f} ms, gpu hscg "
          f"{np.median(th)*1e3:.2f} ms, oracle s-step {np.median(to)*1e3:.0f} ms",
          file=sys.stderr, flush=True)
    return out


def bench_variants(L, P, torch):
    """The layout of the paper's tables (Section 5) on synthetic matrices:
    for eps* in {the relative residual HSCG attains, 1e-6} and s = sigma in
    {5, 10, 15}, outer loops (total iterations) of fixed s-step CG, the old
    adaptive method (monomial basis, c = 1), Algorithm 5 with the Newton and
    the Chebyshev basis, and HSCG; "-" marks breakdown or divergence and
    "- [r]" a run that stopped at relative residual r above eps*."""
    mats = {"poisson2d_64 (N=4096, scaled)": P.make_config("poisson2d_64"),
            "diffusion27_16 (N=4096, lognormal sigma=2, scaled)":
                P.make_config("diffusion27_160", size=16)}
    h = L.assg_create()
    tables = {}
    for label, pr in mats.items():
        A = L.csr_to_device(pr.A)
        L.assg_analyze(h, A)
        b = torch.from_numpy(pr.b).cuda()
        x = torch.zeros_like(b)
        x.zero_()
        hs = L.assg_hscg_solve(h, A, b, x, 1e-15, 20 * pr.n)
        attain = float(f"{max(hs['relres_true'], 1e-15) * 1.1:.1e}")
        rows = []
        for tol in (attain, 1e-6):
            x.zero_()
            hc = L.assg_hscg_solve(h, A, b, x, tol, 20 * pr.n)
            for sigma in (5, 10, 15):
                cells = {}
                for col, variant, basis in (("fixed", "fixed", "monomial"),
                                            ("old adaptive", "old", "monomial"),
                                            ("impr. Newton", "improved", "newton"),
                                            ("impr. Chebyshev", "improved", "chebyshev")):
                    x.zero_()
                    i = L.assg_solve(h, A, b, x, L.assg_default_opts(
                        s_max=sigma, s_init=sigma, growth=sigma, tol=tol, basis=basis,
                        variant=variant, max_outer=5000, max_iters=20 * pr.n))
                    if i["outcome"] == L.CONVERGED:
                        cells[col] = f"{i['outer_iters']} ({i['total_iters']})"
                    elif i["outcome"] in (L.BREAKDOWN, L.DIVERGED) or not \
                            (i["relres_true"] < 1.0):
                        cells[col] = "-"
                    else:
                        cells[col] = f"- [{i['relres_true']:.0e}]"
                cells["HSCG"] = (str(hc["total_iters"]) if hc["outcome"] == L.CONVERGED
                                 else f"- [{hc['relres_true']:.0e}]")
                rows.append({"eps": tol, "s": sigma, **cells})
        tables[label] = rows
    L.assg_destroy(h)
    for label, rows in tables.items():
        print(f"[bench] {label}", file=sys.stderr)
        for r in rows:
            print("[bench]   " + "  ".join(f"{k}={v}" for k, v in r.items()), file=sys.stderr)
    return tables


def bench_diffusion(L, P, torch, warmup, steps):
    """27-point lognormal (sigma = 2) diffusion on 160^3, Jacobi-scaled, b ~
    N(0, 1), sigma = 10, tol 1e-10: both bases and HSCG, each warm-up then
    --steps timed solves (median and min)."""
    pr = P.make_config("diffusion27_160")
    A = L.csr_to_device(pr.A)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    h = L.assg_create()
    L.assg_analyze(h, A)
    out = {"n": pr.n, "nnz": int(pr.A.nnz), "format": L.assg_get_format(h)}
    for basis in ("chebyshev", "newton", "hscg"):
        def run(basis=basis):
            x.zero_()
            if basis == "hscg":
                return L.assg_hscg_solve(h, A, b, x, 1e-10, 0)
            return L.assg_solve(h, A, b, x, L.assg_default_opts(s_max=10, tol=1e-10, basis=basis))
        t, inf = time_solves(run, warmup, steps, torch)
        out[basis] = summary(t, inf)
    out["speedup_vs_hscg"] = round(out["hscg"]["s_median"] / out["chebyshev"]["s_median"], 3)
    L.assg_destroy(h)
    print(f"[bench] diffusion27_160: chebyshev {out['chebyshev']['s_median']*1e3:.1f} ms, newton "
          f"{out['newton']['s_median']*1e3:.1f} ms, hscg {out['hscg']['s_median']*1e3:.1f} ms",
          file=sys.stderr, flush=True)
    return out


def bench_batch(L, P, torch):
    """64 shifted 2D Poisson systems (sides 32..512): one batched solve
    (every kernel launch covers all systems, outer loops replayed from a
    captured graph) against the same systems solved one after another with
    the single solve and with HSCG on the same GPU."""
    probs = P.make_batch()
    As = [L.csr_to_device(pr.A) for pr in probs]
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    h = L.assg_create()
    t0 = time.perf_counter()
    L.assg_batch_analyze(h, As)
    t_an = time.perf_counter() - t0
    opts = L.assg_default_opts(s_max=10, tol=1e-10, basis="chebyshev")

    def batch():
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        inf = L.assg_batch_solve(h, As, bs, xs, opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t, inf

    batch()
    t_batch, infos = min((batch() for _ in range(3)), key=lambda r: r[0])
    worst = max(float(np.linalg.norm(pr.b - pr.A @ x.cpu().numpy()) / np.linalg.norm(pr.b))
                for pr, x in zip(probs, xs))
    hs = L.assg_create()

    def sequential(hscg):
        tot = 0.0
        for A, b, x in zip(As, bs, xs):
            L.assg_analyze(hs, A)
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            if hscg:
                L.assg_hscg_solve(hs, A, b, x, 1e-10, 0)
            else:
                L.assg_solve(hs, A, b, x, opts)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t
        return tot

    sequential(False)
    t_seq = sequential(False)
    t_hscg = sequential(True)
    tune = L.assg_batch_tuning(h)
    L.assg_destroy(h)
    L.assg_destroy(hs)
    out = {
        "systems": len(probs), "rows": int(sum(pr.n for pr in probs)),
        "nnz": int(sum(pr.A.nnz for pr in probs)),
        "batch_solve_s": round(t_batch, 4),
        "sequential_sstep_s": round(t_seq, 4), "sequential_hscg_s": round(t_hscg, 4),
        "speedup_vs_sequential_sstep": round(t_seq / t_batch, 2),
        "speedup_vs_sequential_hscg": round(t_hscg / t_batch, 2),
        "all_converged": all(i["outcome"] == L.CONVERGED for i in infos),
        "max_outer": max(i["outer_iters"] for i in infos),
        "worst_relres_host": worst, "analyze_s": round(t_an, 3), "tuning": tune,
    }
    print(f"[bench] batch of {len(probs)}: {t_batch*1e3:.1f} ms (sequential s-step "
          f"{t_seq*1e3:.1f} ms, HSCG {t_hscg*1e3:.1f} ms)", file=sys.stderr, flush=True)
    return out


def bench_grad(L, P, torch):
    """Differentiable workload: varcoef7 128^3, L = ||x - t||^2, gradients in b
    and in A's values from the forward and adjoint solves at tol 1e-12, with
    the basis growth factor f = sigma (Section 5's choice) and f = 2 (fewer
    levels built when (3.2) keeps s~ small, which it does for the adjoint
    right-hand side: its residual norm climbs above ||b|| early on).  Also
    the relative residual plain HSCG attains on the adjoint right-hand side
    at tol 1e-12, and the adjoint's outer loops with s~ = 1."""
    import warnings

    from paper_1908_04081_amd import autograd as AG
    pr = P.make_config("varcoef7_128")
    n = pr.n
    pat = L.csr_to_device(pr.A)
    h = L.assg_create()
    L.assg_analyze(h, pat)
    t = torch.from_numpy(P.rhs_normal(n, 2105)).cuda()
    b0 = torch.from_numpy(pr.b).cuda()

    def run(growth):
        val = pat.val.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = AG.solve(pat, val, b, handle=h, tol=1e-12, s_max=10, basis="chebyshev",
                     growth=growth, record_trace=1)
        loss = ((x - t) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", AG.SolveStagnated)
            loss.backward()
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, x.detach()

    out = {"workload": "varcoef7_128 (N=2,097,152), tol 1e-12, sigma = 10, Chebyshev",
           "format": L.assg_get_format(h)}
    for growth in (10, 2):
        run(growth)
        fwd, bwd, x = run(growth)
        fi, ai = AG.last_info["forward"], AG.last_info["adjoint"]
        tr = L.assg_get_trace(h)                      # the adjoint solve's loops
        out[f"f={growth}"] = {
            "forward_s": round(fwd, 4), "backward_s": round(bwd, 4),
            "backward_over_forward": round(bwd / fwd, 2),
            "forward_outer": fi["outer_iters"], "forward_iters": fi["total_iters"],
            "forward_outcome": fi["outcome_name"], "forward_relres": fi["relres_true"],
            "adjoint_outer": ai["outer_iters"], "adjoint_iters": ai["total_iters"],
            "adjoint_outcome": ai["outcome_name"], "adjoint_relres": ai["relres_true"],
            "adjoint_loops_stilde_1": sum(1 for r in tr if r["stilde"] == 1),
            "adjoint_max_rho_m": max(r["rho_m"] for r in tr),
            "adjoint_levels_built": sum(r["sbar"] for r in tr)}
        print(f"[bench] differentiable f={growth}: forward {fwd*1e3:.1f} ms, backward "
              f"{bwd*1e3:.1f} ms", file=sys.stderr, flush=True)
    g = (2.0 * (x - t)).contiguous()
    lam = torch.zeros_like(g)
    hi = L.assg_hscg_solve(h, pat, g, lam, 1e-12, 0)
    out["hscg_on_adjoint_rhs"] = {"outcome": hi["outcome_name"], "relres": hi["relres_true"],
                                  "iters": hi["total_iters"]}
    L.assg_destroy(h)
    return out


def cpu_baseline(pr, sigma, tol, gpu_outer):
    """The oracle (unchanged) on a bounded sample of the same workload: its
    first outer loops on the full problem, timed on the host with every
    library thread pool held to one thread (SciPy's CSR product is
    single-threaded anyway), scaled by the outer-loop count of a full
    solve."""
    import contextlib

    import oracle as O
    try:
        from threadpoolctl import threadpool_limits
        one_thread = threadpool_limits(limits=1)
    except Exception:
        one_thread = contextlib.nullcontext()
    loops = 1
    with one_thread:
        t0, c0 = time.perf_counter(), time.process_time()
        _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=sigma, tol=tol, basis="chebyshev",
                                      max_outer=loops)
        dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    per_loop = dt / max(info["outer"], 1)
    return {
        "value": round(per_loop * gpu_outer, 2),
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {info['outer']} outer loop(s) of the oracle's adaptive s-step CG on the "
                  f"same {pr.n}-row problem ({dt:.1f} s wall, {cpu:.1f} s CPU, {per_loop:.2f} s "
                  f"per loop; each loop builds the full sigma={sigma} basis), scaled by the GPU "
                  f"solve's {gpu_outer} outer loops; BLAS and OpenMP pools held to one thread",
        "host_cpus": os.cpu_count(),
    }


if __name__ == "__main__":
    main()
