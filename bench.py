"""Benchmark of the SIVF hot path on one MI355X.

A step is one Lloyd iteration (assignment step + update step, Alg. 1 around
Alg. 4 / Alg. 5) of the whole path on the headline workload: N = 8,000,000
L2-normalised sparse rows, D = 140,000 terms, nnz/row ~ Poisson(90), Zipf(1.1)
term ids, lognormal values (seeded synthetic stand-in for the paper's 8M
PubMed subset), k = 10,000 seeded initial centroids.  The timed region is
iterations 1..K of a fresh run from the seeded initial state (default K = 30,
the run length of this workload; W untimed warmup iterations are run first on
a separate run from the same state).

Reported value: assignment-step object-centroid mult-adds per second with FP32
postings (sum of posting mult-adds over the timed iterations divided by the
summed assignment-step time, HIP events on the library's stream), plus s/iter,
the same for BF16 postings (identical trajectory), the walk kernel's roofline
figures and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
POSTING_BYTES = {"fp32": 6, "bf16": 4}  # 2-byte centroid id + value
WALK_KERNEL = "k_walk_fast<false, false>"   # FP32 postings, SIVF filter
# counter-based HBM traffic of the walk, written from the rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs; used only while the kernel sources still hash the same
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "walk_8m_k10k_hbm_traffic.md")
WALK_SOURCES = ["paper_2103_16141_amd/csrc/k_assign.hip", "paper_2103_16141_amd/csrc/internal.h",
                "paper_2103_16141_amd/csrc/wave.h"]


def walk_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per walk launch from the committed counter profile, or None
    when the profile is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("TRAFFIC_JSON "):
                    rec = json.loads(line[len("TRAFFIC_JSON "):])
                    if rec.get("walk_source_hash") == walk_source_hash():
                        return rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def measured_copy_gbs(gib=1, reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time), HIP events."""
    import torch
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def run_soft(reps=3):
    """Differentiation form at its own shape (N = 262,144, D = 100,000,
    Poisson(100), k = 4,096 dense centroids, tau = 0.05): forward (lse + loss)
    and backward (dC, dX) timed with HIP events on the library's stream."""
    import torch

    import synth
    from paper_2103_16141_amd.api import Context, DeviceCsr
    corpus, ids, w = synth.workload("soft-262k")
    C = torch.from_numpy(synth.dense_centroids(corpus, ids, noise=1e-3, seed=2103 + 5)).cuda()
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    ctx = Context(0)
    tau = 0.05
    lse, _ = ctx.soft_assign_fwd(X, C, tau)
    ctx.soft_assign_bwd(X, C, tau, lse, 1.0)   # warm: the backward's transposes and CSC
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, bwd = [], []
    for _ in range(reps):
        ev[0].record()
        lse, loss = ctx.soft_assign_fwd(X, C, tau)
        ev[1].record()
        dC, dX = ctx.soft_assign_bwd(X, C, tau, lse, 1.0)
        ev[2].record()
        torch.cuda.synchronize()
        fwd.append(ev[0].elapsed_time(ev[1]))
        bwd.append(ev[1].elapsed_time(ev[2]))
    ctx.close()
    k = C.shape[0]
    ma = corpus.nnz * k   # mult-adds of one S = X C^T pass
    f, b = min(fwd), min(bwd)
    out = dict(workload="soft-assignment loss, N=%d, D=%d, nnz=%d, k=%d dense centroids, tau=%g"
                        % (corpus.n, corpus.d, corpus.nnz, k, tau),
               fwd_ms=f, bwd_ms=b, s_pass_multadds=ma, fwd_multadds_per_s=ma / (f * 1e-3),
               bwd_multadds_per_s=3 * ma / (b * 1e-3), loss=loss)
    del C, X, dC, dX, lse
    torch.cuda.empty_cache()
    return out


def copy_calibration(gib=1):
    """A plain device-to-device copy of a known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters (one kernel launch per copy)."""
    import torch
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "launches": 3}), flush=True)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(stat, nnz, n, n_tiles, posting):
    """Minimal bytes the walk must move for one launch: every posting once per
    (object, posting) pair at its minimal encoding, the CSR rows (4-byte column
    + 4-byte value), two 8-byte segment offsets per (object term, tile), and
    row pointer / previous assignment / own similarity per object."""
    return stat["multadds"] * POSTING_BYTES[posting] + nnz * (8 + 16 * n_tiles) + 12 * n


def run_lloyd_timed(ctx, X, k, ids, steps, warmup, posting):
    import torch
    from paper_2103_16141_amd.api import Lloyd

    if warmup > 0:
        Lw = Lloyd(ctx, X, k, ids)
        for _ in range(warmup):
            Lw.assign()
            Lw.update()
        Lw.ivf.free()
        del Lw
    torch.cuda.synchronize()
    L = Lloyd(ctx, X, k, ids)
    sizes = L.ivf.sizes()
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(1, steps + 1):
        st = L.assign()
        up = L.update()
        st["t_update_ms"] = up["t_update_ms"]
        stats.append(st)
        log("%s iter %d: M=%.3e walk %.1f ms assign %.1f ms update %.1f ms moved %d inv %d icp %d rescored %d/%d "
            "full %d head rows %d relaxed %d"
            % (posting, r, st["multadds"], st["t_walk_ms"], st["t_assign_ms"], st["t_update_ms"], st["moved"],
               st["n_invariant"], st["icp_objects"], st["rescored_objects"], st["rescored_candidates"],
               st["full_rescored"], st["head_rows"], st["relaxed_objects"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assign_a = L.a.clone()
    L.ivf.free()
    return stats, wall, sizes, assign_a


def summarize(stats, wall, sizes, nnz, n, posting):
    M = sum(s["multadds"] for s in stats)
    t_assign = sum(s["t_assign_ms"] for s in stats) / 1e3
    t_walk = sum(s["t_walk_ms"] for s in stats) / 1e3
    t_update = sum(s["t_update_ms"] for s in stats) / 1e3
    bytes_ = sum(algorithmic_bytes(s, nnz, n, sizes["n_tiles"], posting) for s in stats)
    return dict(multadds=M, multadds_per_s=M / t_assign, s_per_iter=wall / len(stats),
                assign_s=t_assign, walk_s=t_walk, update_s=t_update,
                walk_multadds_per_s=M / t_walk, walk_algorithmic_gbs=bytes_ / t_walk / 1e9,
                iter1_multadds_per_s=stats[0]["multadds"] / (stats[0]["t_assign_ms"] / 1e3),
                rescored_objects=sum(s["rescored_objects"] for s in stats),
                full_rescored=sum(s["full_rescored"] for s in stats),
                walk_avg_ms=1e3 * t_walk / len(stats))


def cpu_baseline(corpus, ids, k, budget_s=15.0):
    """FP64 oracle assignment (iteration 1, against the seeded initial centroids)
    on a bounded sample of objects, in posting mult-adds per second."""
    import numpy as np

    import oracle

    cents = oracle.init_centroids(corpus, ids)
    _, per_row = oracle.multadds(corpus, oracle.build_ivf(cents, None), per_row=True)
    rng = np.random.default_rng(0)
    m, rows_done, total_m, total_t = 256, 0, 0, 0.0
    while total_t < budget_s:
        rows = np.sort(rng.choice(corpus.n, m, replace=False))
        t0 = time.perf_counter()
        oracle.assign(corpus, cents, rows=rows)
        dt = time.perf_counter() - t0
        total_m += int(per_row[rows].sum())
        total_t += dt
        rows_done += m
        if dt < budget_s / 8:
            m *= 2
    return dict(value=total_m / total_t, unit="mult-adds/s", cores=oracle.num_threads(), kind="oracle",
                sample="%d uniformly drawn objects of the same workload at iteration 1 (FP64 inner products "
                       "against the %d seeded initial centroids), %.1f s of CPU work" % (rows_done, k, total_t))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--n", type=int, default=None, help="override N (smaller runs for development)")
    ap.add_argument("--skip-bf16", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--k-tile", type=int, default=0, help="centroids per LDS tile (0 = automatic)")
    ap.add_argument("--head-density", type=float, default=None,
                    help="dense head rows for terms held by at least this fraction of centroids (default: library's)")
    ap.add_argument("--tiles-per-launch", type=int, default=None,
                    help="centroid tiles per walk launch (default: library's, one tile per launch)")
    ap.add_argument("--skip-soft", action="store_true", help="skip the differentiation-form timing")
    ap.add_argument("--filter", default="sivf", choices=["sivf", "ivf", "cbicp", "relaxed"],
                    help="ICP realisation: structured file (SIVF), none (IVF), per-posting test (IVF-CBICP), "
                         "SIVF with relaxed ICP")
    ap.add_argument("--workload", default="8m-f32", help="synthetic workload name (8m-f32, 8m-bf16-k20k, 1m-f32)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 3 copies of 1 GiB (counter calibration for the traffic figure)")
    ap.add_argument("--print-walk-hash", action="store_true", help="print the walk kernel source hash and exit")
    args = ap.parse_args()
    if args.print_walk_hash:
        print(walk_source_hash())
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one GPU per run).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2103_16141_amd import _native
    from paper_2103_16141_amd.api import Context, DeviceCsr

    _native.load()
    over = {} if args.n is None else {"n": args.n}
    t0 = time.perf_counter()
    corpus, ids, w = synth.workload(args.workload, **over)
    log("corpus N=%d D=%d nnz=%d generated in %.1f s (%d threads)" % (corpus.n, corpus.d, corpus.nnz,
                                                                    time.perf_counter() - t0, synth.num_threads()))
    dev = torch.device("cuda", 0)
    X = DeviceCsr.from_corpus(corpus, dev)
    torch.cuda.synchronize()
    k = w["k"]

    ctx32 = Context(0, posting_dtype="fp32", k_tile=args.k_tile, head_density=args.head_density,
                    tiles_per_launch=args.tiles_per_launch, filter_mode=args.filter)
    st32, wall32, sizes, a32 = run_lloyd_timed(ctx32, X, k, ids, args.steps, args.warmup, "fp32")
    s32 = summarize(st32, wall32, sizes, corpus.nnz, corpus.n, "fp32")
    ctx32.close()
    out_bf16 = None
    if not args.skip_bf16:
        ctx16 = Context(0, posting_dtype="bf16", k_tile=args.k_tile, head_density=args.head_density,
                    tiles_per_launch=args.tiles_per_launch, filter_mode=args.filter)
        st16, wall16, sizes16, a16 = run_lloyd_timed(ctx16, X, k, ids, args.steps, args.warmup, "bf16")
        s16 = summarize(st16, wall16, sizes16, corpus.nnz, corpus.n, "bf16")
        ctx16.close()
        same = bool(torch.equal(a32, a16)) and [s["multadds"] for s in st32] == [s["multadds"] for s in st16]
        out_bf16 = dict(value=s16["multadds_per_s"], s_per_iter=s16["s_per_iter"], walk_avg_ms=s16["walk_avg_ms"],
                        rescored_objects=s16["rescored_objects"], full_rescored=s16["full_rescored"],
                        identical_trajectory=same, vs_fp32=s16["multadds_per_s"] / s32["multadds_per_s"])

    soft = None
    if not args.skip_soft and args.n is None:
        del X
        torch.cuda.empty_cache()
        soft = run_soft()
        log("soft form: fwd %.2f ms, bwd %.2f ms" % (soft["fwd_ms"], soft["bwd_ms"]))
    copy_gbs = measured_copy_gbs()

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(corpus, ids, k, args.cpu_budget)

    achieved = s32["walk_algorithmic_gbs"]
    # the walk is one kernel launch per group of tiles_per_launch centroid tiles
    tpl = max(1, args.tiles_per_launch or 1)
    launches = len(st32) * ((sizes["n_tiles"] + tpl - 1) // tpl)
    launch_ms = s32["walk_s"] * 1e3 / launches
    line = {
        "metric": "assign-step object-centroid mult-adds/s + s/iter at N=8M,k=10k; BF16 vs FP32",
        "value": s32["multadds_per_s"],
        "unit": "mult-adds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * s32["s_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Lloyd iterations 1..K, N=%d, D=%d, nnz/row~Poisson(%d), Zipf(%.1f) terms, "
                               "lognormal values, L2-normalised rows, k=%d seeded initial objects"
                               % (corpus.n, corpus.d, w["lam"], w["zipf_s"], k),
                   "n": corpus.n, "d": corpus.d, "k": k, "nnz": corpus.nnz, "k_tile": sizes["k_tile"],
                   "n_tiles": sizes["n_tiles"],
                   "filter": {"sivf": "SIVF (ICP via structured file)", "ivf": "IVF (no ICP)",
                              "cbicp": "IVF-CBICP (ICP by per-posting flag test)",
                              "relaxed": "SIVF with relaxed ICP"}[args.filter]},
        "s_per_iter": s32["s_per_iter"],
        "iter1_multadds_per_s": s32["iter1_multadds_per_s"],
        "assign_s": s32["assign_s"], "update_s": s32["update_s"],
        "multadds_total": s32["multadds"],
        "bf16": out_bf16,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": WALK_KERNEL, "launches": launches, "launch_avg_ms": launch_ms,
                     "algorithmic_bytes_per_launch": achieved * 1e9 * launch_ms * 1e-3,
                     "walk_avg_ms_per_iter": s32["walk_avg_ms"], "measured_copy_gbs": copy_gbs},
        "soft": soft,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
