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
N_CU, CLOCK_GHZ = 256, 2.4   # MI355X compute units and peak engine clock
POSTING_BYTES = {"fp32": 6, "bf16": 4}  # 2-byte centroid id + value
WALK_KERNEL = "k_walk_fast<false, false>"   # FP32 postings, SIVF filter
# bytes the walk's L2 sends toward memory, from calibrated rocprofv3 --pmc
# runs; used only while the kernel sources still hash the same
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "walk_8m_k10k_dram_traffic.md")
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
    """DRAM-side bytes per walk launch from the committed counter profile
    (record of the profile's TRAFFIC_JSON line), or None when the profile is
    missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("TRAFFIC_JSON "):
                    rec = json.loads(line[len("TRAFFIC_JSON "):])
                    if rec.get("walk_source_hash") == walk_source_hash():
                        return rec
    except (OSError, ValueError, KeyError):
        pass
    return None


PROBE_CASES = [
    # name, kind (0 loads, 1 LDS read, 2 LDS write), bytes per lane, region, window, stride
    ("l1_b32", 0, 4, 4 << 10, 4 << 10, 4 << 10),
    ("l1_b64", 0, 8, 8 << 10, 8 << 10, 8 << 10),
    ("l1_b128", 0, 16, 16 << 10, 16 << 10, 16 << 10),
    ("l2_b128", 0, 16, 2 << 20, 256 << 10, 16 << 10),
    ("mall_b128", 0, 16, 64 << 20, 8 << 20, 256 << 10),
    ("lds_read_b128", 1, 16, 0, 0, 0),
    ("lds_write_b128", 2, 16, 0, 0, 0),
]


def run_probe(reps=3):
    """Data rates of one compute unit's vector loads (from regions resident in
    L1, L2, the memory-side cache and HBM) and of its LDS, from the kernels of
    libsivf_probe.so: bytes per shader clock per CU, the shader clock from
    s_memtime against the 100 MHz s_memrealtime, and GB/s over the device."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2103_16141_amd", "libsivf_probe.so"))
    c_u32, vp = ctypes.c_uint32, ctypes.c_void_p
    lib.sivf_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, vp, c_u32, c_u32, c_u32, ctypes.c_int, ctypes.c_int,
                                   vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_ulonglong)]
    lib.sivf_probe_run.restype = ctypes.c_int
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    need = max(c[3] + c[4] for c in PROBE_CASES)
    buf = torch.ones(need, dtype=torch.uint8, device="cuda")
    scratch = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for name, kind, width, region, window, stride in PROBE_CASES:
        blocks = n_cu * 8
        rounds = 8192 if (kind or region <= (16 << 10)) else 2048
        nbytes = ctypes.c_double()
        clk = (ctypes.c_ulonglong * 2)()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lib.sivf_probe_run(kind, width, ctypes.c_void_p(buf.data_ptr()), region, window, stride, blocks,
                                    rounds, ctypes.c_void_p(scratch.data_ptr()), ctypes.c_void_p(stream.cuda_stream),
                                    ctypes.byref(nbytes), clk)
            e1.record(stream)
            torch.cuda.synchronize()
            if rc != 0:
                raise RuntimeError("probe %s failed (%d)" % (name, rc))
            ms = e0.elapsed_time(e1)
            ghz = clk[0] / (clk[1] / 1e8) / 1e9 if clk[1] else float("nan")
            rec = dict(gbs=nbytes.value / (ms * 1e-3) / 1e9, ms=ms, shader_ghz=ghz)
            if best is None or rec["gbs"] > best["gbs"]:
                best = rec
        best["bytes_per_clk_cu"] = best["gbs"] * 1e9 / n_cu / (best["shader_ghz"] * 1e9)
        out[name] = best
        log("probe %s: %.0f GB/s, %.1f B/clk/CU at %.2f GHz" % (name, best["gbs"], best["bytes_per_clk_cu"],
                                                                 best["shader_ghz"]))
    del buf, scratch
    torch.cuda.empty_cache()
    return out


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
    loaded = sum(s["walk_bytes"] for s in stats)
    wide = sum(s["walk_wide_bytes"] for s in stats)
    return dict(multadds=M, multadds_per_s=M / t_assign, s_per_iter=wall / len(stats),
                assign_s=t_assign, walk_s=t_walk, update_s=t_update,
                walk_multadds_per_s=M / t_walk, walk_algorithmic_gbs=bytes_ / t_walk / 1e9,
                walk_loaded_bytes=loaded, walk_wide_bytes=wide, walk_data_gbs=loaded / t_walk / 1e9,
                walk_launches=sum(s["walk_launches"] for s in stats),
                iter1_multadds_per_s=stats[0]["multadds"] / (stats[0]["t_assign_ms"] / 1e3),
                rescored_objects=sum(s["rescored_objects"] for s in stats),
                full_rescored=sum(s["full_rescored"] for s in stats),
                walk_avg_ms=1e3 * t_walk / len(stats))


def cpu_baseline(corpus, ids, k, budget_s=15.0):
    """FP64 oracle assignment (iteration 1, against the seeded initial centroids)
    on a bounded sample of objects, in posting mult-adds per second: credited
    with the same count M as the GPU (the structured file's postings of the
    objects' terms), so it compares with the GPU's iteration-1 rate; the
    oracle itself multiplies every term by all k centroids (dense FP64)."""
    import numpy as np

    import oracle

    cents = oracle.init_centroids(corpus, ids)
    _, per_row = oracle.multadds(corpus, oracle.build_ivf(cents, None), per_row=True)
    rng = np.random.default_rng(0)
    m, rows_done, total_m, total_t, total_terms = 256, 0, 0, 0.0, 0
    lens = np.diff(corpus.row_ptr)
    while total_t < budget_s:
        rows = np.sort(rng.choice(corpus.n, m, replace=False))
        t0 = time.perf_counter()
        oracle.assign(corpus, cents, rows=rows)
        dt = time.perf_counter() - t0
        total_terms += int(lens[rows].sum())
        total_m += int(per_row[rows].sum())
        total_t += dt
        rows_done += m
        if dt < budget_s / 8:
            m *= 2
    return dict(value=total_m / total_t, unit="mult-adds/s", cores=oracle.num_threads(), kind="oracle",
                sample="%d uniformly drawn objects of the same workload at iteration 1 (FP64 inner products "
                       "against the %d seeded initial centroids), %.1f s of CPU work" % (rows_done, k, total_t),
                compare_with="iter1_multadds_per_s (the GPU's rate at the same iteration and count)",
                dense_fp64_multadds_per_s=total_terms * k / total_t)


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
    ap.add_argument("--soft-only", action="store_true", help="only time the differentiation form and print it")
    ap.add_argument("--filter", default="sivf", choices=["sivf", "ivf", "cbicp", "relaxed"],
                    help="ICP realisation: structured file (SIVF), none (IVF), per-posting test (IVF-CBICP), "
                         "SIVF with relaxed ICP")
    ap.add_argument("--workload", default="8m-f32", help="synthetic workload name (8m-f32, 8m-bf16-k20k, 1m-f32)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 3 copies of 1 GiB (counter calibration for the traffic figure)")
    ap.add_argument("--print-walk-hash", action="store_true", help="print the walk kernel source hash and exit")
    ap.add_argument("--probe", action="store_true", help="only run the data-rate probes and print them")
    ap.add_argument("--skip-probe", action="store_true", help="skip the data-rate probes (roofline peak)")
    args = ap.parse_args()
    if args.print_walk_hash:
        print(walk_source_hash())
        return
    if args.probe:
        print(json.dumps(run_probe()), flush=True)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.soft_only:
        print(json.dumps(run_soft()), flush=True)
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
    probe = None if args.skip_probe else run_probe()

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(corpus, ids, k, args.cpu_budget)

    # the walk is one kernel launch per group of tiles_per_launch centroid tiles
    launches = s32["walk_launches"]
    launch_ms = s32["walk_s"] * 1e3 / launches
    # Roofline of the walk: the vector memory data path.  Its peak is what the
    # walk's own mix of loads could move per launch at the probed per-CU rates
    # (16-byte loads at the L1-resident b128 rate, 4- and 8-byte loads at the
    # b64 rate), over 256 CUs at the 2.4 GHz peak clock; achieved = the bytes
    # the walk's vector loads request (counted by the kernel) over its launch
    # time.
    achieved = s32["walk_data_gbs"]
    peak = peak16 = None
    if probe:
        r16 = probe["l1_b128"]["bytes_per_clk_cu"] * N_CU * CLOCK_GHZ
        r8 = probe["l1_b64"]["bytes_per_clk_cu"] * N_CU * CLOCK_GHZ
        wide, narrow = s32["walk_wide_bytes"], s32["walk_loaded_bytes"] - s32["walk_wide_bytes"]
        peak = (wide + narrow) / (wide / r16 + narrow / r8)
        peak16 = r16
    if out_bf16 is not None:
        # the BF16 walk against the same data-path roof, for its own load mix
        # (16-byte head-row loads, 8-byte id and value loads of the lists)
        out_bf16["walk_requested_gbs"] = s16["walk_data_gbs"]
        out_bf16["wide_load_fraction"] = s16["walk_wide_bytes"] / s16["walk_loaded_bytes"]
        if probe:
            w16, n16 = s16["walk_wide_bytes"], s16["walk_loaded_bytes"] - s16["walk_wide_bytes"]
            out_bf16["vmem_peak_gbs"] = (w16 + n16) / (w16 / r16 + n16 / r8)
            out_bf16["vmem_frac"] = s16["walk_data_gbs"] / out_bf16["vmem_peak_gbs"]
    traffic = measured_traffic()
    dram = None
    if traffic:
        # bytes the L2 sent toward memory per launch (reads + writes), from
        # calibrated counters; memory-side-cache hits are included
        tb = traffic["l2_to_memory_bytes_per_launch"]
        dram_gbs = tb / (traffic["launch_ms"] * 1e-3) / 1e9
        dram = dict(bytes_per_launch=tb, read_bytes_per_launch=traffic["read_bytes_per_launch"],
                    write_bytes_per_launch=traffic["write_bytes_per_launch"], gbs=dram_gbs,
                    frac_of_measured_copy=dram_gbs / copy_gbs, frac_of_hbm_peak=dram_gbs / HBM_PEAK_GBS,
                    includes_memory_side_cache_hits=traffic["includes_memory_side_cache_hits"],
                    counter_launch_ms=traffic["launch_ms"], profile=os.path.relpath(TRAFFIC_PROFILE, ROOT))
    roofline = {"bound": "vmem", "achieved": achieved, "peak": peak, "unit": "GB/s",
                "frac": achieved / peak if peak else None,
                "traffic": traffic["l2_to_memory_bytes_per_launch"] if traffic else None,
                "kernel": WALK_KERNEL, "launches": launches, "launch_avg_ms": launch_ms,
                "bytes_per_launch": s32["walk_loaded_bytes"] / launches,
                "wide_load_fraction": s32["walk_wide_bytes"] / s32["walk_loaded_bytes"],
                "peak_basis": "walk's load mix at the probed L1 rates (b128 for 16-byte loads, b64 for 4-/8-byte "
                              "loads) x %d CUs x %.1f GHz" % (N_CU, CLOCK_GHZ),
                "peak_all_16byte_loads": peak16,
                "dram": dram,
                "algorithmic_gbs": s32["walk_algorithmic_gbs"],
                "algorithmic_frac_of_hbm_peak": s32["walk_algorithmic_gbs"] / HBM_PEAK_GBS,
                "walk_avg_ms_per_iter": s32["walk_avg_ms"], "measured_copy_gbs": copy_gbs, "probe": probe}
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
        "roofline": roofline,
        "soft": soft,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
