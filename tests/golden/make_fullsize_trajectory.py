"""Write the FP64 oracle's full-size Lloyd trajectory as hashes.

    python tests/golden/make_fullsize_trajectory.py 8m-f32 --iters 3
    python tests/golden/make_fullsize_trajectory.py 8m-bf16-k20k --iters 2

Calls only ``oracle`` and ``synth``: the corpus and the initial objects come
from the seeded generator, the trajectory from the oracle's plain FP64 Lloyd
loop (Alg. 1 with the ICP bookkeeping of Alg. 4/5).  For every iteration r it
records SHA-256 digests of a^[r] (int32) and lambda^[r] (uint8), the moved
count, the SIVF posting mult-add count M, the number of objects in the ICP
branch, the FP64 objective sum_i rho_{i,a_i} (summed exactly) and, after the
update, the digest of the FP64 centroids mu^[r] as CSR (int64 row pointers,
int32 columns, float64 values, little endian).  The GPU test regenerates the
corpus, checks its digest first, runs the same iterations on the device and
compares every digest: a bit-exact check of all N objects and every centroid
value without storing gigabytes of expected values.

The file is rewritten after every iteration, so a long run leaves a usable
prefix.  --state DIR saves the oracle's state after each update (centroids,
a, own similarities, flags) and --resume continues from the last one saved,
so the run can be split over several sessions; a resumed run appends to the
existing file's iterations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        assert a.dtype.byteorder in ("<", "=", "|")
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()


def corpus_digest(corpus) -> str:
    return digest(corpus.row_ptr, corpus.col, corpus.val)


def centroid_digest(c: oracle.Centroids) -> str:
    return digest(np.asarray(c.ptr, np.int64), np.asarray(c.col, np.int32), np.asarray(c.val, np.float64))


def golden_path(name: str) -> str:
    return os.path.join(HERE, "fullsize_%s.json" % name)


def save_state(state_dir, st: oracle.LloydState):
    os.makedirs(state_dir, exist_ok=True)
    tmp = os.path.join(state_dir, "state.tmp.npz")
    np.savez(tmp, r=st.r, k=st.cents.k, d=st.cents.d, ptr=st.cents.ptr, col=st.cents.col, val=st.cents.val,
             a=st.a, own=st.own, lam=st.lam)
    os.replace(tmp, os.path.join(state_dir, "state.npz"))


def load_state(state_dir) -> oracle.LloydState:
    z = np.load(os.path.join(state_dir, "state.npz"))
    c = oracle.Centroids(int(z["k"]), int(z["d"]), z["ptr"], z["col"], z["val"])
    return oracle.LloydState(int(z["r"]), c, z["a"], z["own"], z["lam"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--iters", type=int, required=True, help="last iteration to record")
    ap.add_argument("--state", default=None, help="directory for the oracle state after each update")
    ap.add_argument("--resume", action="store_true", help="continue from the state in --state")
    args = ap.parse_args()

    t0 = time.perf_counter()
    corpus, ids, w = synth.workload(args.workload)
    k = w["k"]
    out = golden_path(args.workload)
    rec = dict(workload=args.workload, n=corpus.n, d=corpus.d, nnz=corpus.nnz, k=k, lam=w["lam"],
               zipf_s=w["zipf_s"], data_seed=16141 + w["c"], init_seed=2103 + w["c"],
               corpus_sha256=corpus_digest(corpus), init_ids_sha256=digest(np.asarray(ids, np.int32)),
               oracle_threads=oracle.num_threads(), filter="SIVF (ICP)", iterations=[])
    print("corpus %d x %d, nnz %d, generated and hashed in %.1f s" % (corpus.n, corpus.d, corpus.nnz,
                                                                      time.perf_counter() - t0), flush=True)
    start = None
    if args.resume:
        with open(out) as fh:
            old = json.load(fh)
        assert old["corpus_sha256"] == rec["corpus_sha256"], "the saved run used another corpus"
        start = load_state(args.state)
        rec["iterations"] = [it for it in old["iterations"] if it["r"] <= start.r]
        assert rec["iterations"][-1]["centroids_sha256"] == centroid_digest(start.cents)
        print("resuming after iteration %d" % start.r, flush=True)

    tick = [time.perf_counter()]

    def on_iter(info):
        r = info["r"]
        a, lam, own = info["a"], info["lam"], info["own"]
        it = dict(r=r, a_sha256=digest(a), lam_sha256=digest(lam), moved=int(info["moved"]),
                  multadds=int(info["multadds"]), icp_objects=int((info["branch"] == 1).sum()) if r >= 2 else 0,
                  n_invariant=int(lam.sum()), objective=math.fsum(own.tolist()))
        if info["cents"] is not None:
            c = info["cents"]
            it["centroids_sha256"] = centroid_digest(c)
            it["centroid_nnz"] = int(c.ptr[-1])
            if args.state:
                save_state(args.state, oracle.LloydState(r, c, a, own, lam))
        now = time.perf_counter()
        it["oracle_seconds"] = round(now - tick[0], 1)
        tick[0] = now
        rec["iterations"].append(it)
        tmp = out + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        os.replace(tmp, out)
        print("iteration %d: moved %d, M %d, icp %d, invariant %d, %.0f s" % (
            r, it["moved"], it["multadds"], it["icp_objects"], it["n_invariant"], it["oracle_seconds"]), flush=True)

    oracle.lloyd(corpus, k, ids, args.iters, icp=True, start=start, on_iter=on_iter)


if __name__ == "__main__":
    main()
