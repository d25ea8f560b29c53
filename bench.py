#!/usr/bin/env python3
"""Throughput of the cascade vector-set search on one MI355X.

Workload (default "scale"): 1,000,000 synthetic sets with sizes uniform in
5-100 (52.5M vectors), d = 384, 10,000 topics; FlyHash L = 4096, s = 16,
wta_k = 64; A = 3, M = 1, T = 1000; 1,024 subset queries; top-10.  Data is
drawn on the GPU by paper_2412_03301_amd.synth and stays resident in HBM.

One step = one bvs_search call over the whole query batch: query
conversion and encoding, query sketches, second-layer scores of every set,
top-T selection, exact Hausdorff re-rank and top-k.  The timed region holds
exactly `--steps` steps bracketed by device synchronisation.

Also reported: recall@10 against the exact GPU brute force (on a sample of
the queries), the brute-force throughput on that sample, per-stage times
from HIP events recorded by the library on its stream, the roofline of the
dominant kernel, and the CPU oracle timed on a bounded sample.
Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "queries/sec at recall@10>=0.95 on 1M sets vs GPU brute-force Hausdorff"
HBM_PEAK_GBS = 8000.0
# Integer VALU lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Dense int8 matrix-core peak of MI355X (TOP/s), the brute force's roof.
INT8_PEAK_TOPS = 5000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scale", choices=["scale", "tiny", "batched", "precision", "learned", "full", "metrics",
                                                       "trends"])
    ap.add_argument("--train-epochs", type=int, default=1)
    ap.add_argument("--train-batch", type=int, default=256)
    ap.add_argument("--train-lr", type=float, default=3e-4)
    ap.add_argument("--train-tau", type=float, default=0.01)
    ap.add_argument("--train-margin", type=float, default=64.0)
    ap.add_argument("--mine-queries", type=int, default=None)
    ap.add_argument("--train-sets", type=int, default=None)
    ap.add_argument("--sweep-t", default="500,1000,2000")
    ap.add_argument("--margin", type=float, default=0.02, help="precision workload: re-check margin")
    ap.add_argument("--form", default="fp8", choices=["fp8", "bf16"], help="precision workload: reported form")
    ap.add_argument("--per-query-sample", type=int, default=1024,
                    help="batched workload: queries searched one call each for the comparison")
    ap.add_argument("--n-sets", type=int, default=None, help="override the set count (for quick runs)")
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--top-t", type=int, default=None)
    ap.add_argument("--brute-queries", type=int, default=256)
    ap.add_argument("--op-sweep", default="100,200,300,500,1000",
                    help="scale workload: T values for the recall/throughput operating points ('' to skip)")
    ap.add_argument("--bf16-brute", type=int, default=16,
                    help="scale workload: queries of the bfloat16 brute force (0 to skip)")
    ap.add_argument("--cpu-sample-sets", type=int, default=1000)
    ap.add_argument("--cpu-sample-queries", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brute", action="store_true")
    ap.add_argument("--full-queries", type=int, default=64,
                    help="full workload: queries per step of the full scan (Alg. 2)")
    ap.add_argument("--streams", type=int, default=2,
                    help="scale workload: host threads searching at once on their own streams (1 to skip)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration runs)")
    return ap.parse_args()


def source_sha(*paths):
    """First 16 hex digits of the SHA-256 of the files' contents, in order."""
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_file, kernel_prefix):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel source (the summary lists the files it hashed);
    else None."""
    p = os.path.join(ROOT, "profiles", f"pmc_{kernel_prefix}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        files = [os.path.join(ROOT, f) for f in d.get("sources", [os.path.relpath(kernel_file, ROOT)])]
        if d.get("source_sha") != source_sha(*files):
            return None
        return d.get("hbm_bytes_per_launch")
    except Exception:
        return None


_CPU = {}


def _cpu_query(i):
    """One query of the oracle on the slice (runs in a pool worker; the
    slice index is inherited from the parent).  Returns the seconds spent in
    query encoding, in the filter steps and in the exact re-rank, and the
    vectors of the slice's F2 that the re-rank measured."""
    import numpy as np

    from oracle import filter as flt
    from oracle import flyhash, hausdorff, search

    st = _CPU
    cfg, ix = st["cfg"], st["ix"]
    Q = st["q"][st["q_off"][i]:st["q_off"][i + 1]].astype(np.float64)
    t0 = time.perf_counter()
    HQ = flyhash.codes(Q, ix.idx, cfg["wta_k"])
    C_Q, S_Q = flt.query_sketches(HQ)
    P = flt.top_positions(C_Q, cfg["A"])
    t1 = time.perf_counter()
    member = flt.first_filter(ix.C, P, cfg["M"])
    scores = flt.hamming(S_Q, ix.B)
    f2, _ = flt.second_filter(member, scores, cfg["top_t"])
    t2 = time.perf_counter()
    h2 = np.array([hausdorff.hausdorff_sq(Q, ix.members(j)) for j in f2])
    search.rank_by_distance(f2, h2, cfg["k"])
    t3 = time.perf_counter()
    vec = int(sum(ix.offsets[j + 1] - ix.offsets[j] for j in f2))
    return t1 - t0, t2 - t1, t3 - t2, vec


def cpu_baseline(db_cpu, offsets, q_cpu, q_off, cfg, n_sets_full, sample_sets, sample_queries, f2_vectors):
    """The oracle as it stands, on the host cores: a slice of the first
    sample_sets sets (same generator and parameters) and sample_queries
    queries spread over a process pool with one worker per core (one BLAS
    thread each).  Per query: encoding as measured; the filter steps (linear
    in the set count) scaled from the slice to the full set count; the exact
    re-rank scaled from its time per vector on the slice's F2 to the number
    of vectors in that query's F2 on the full database (f2_vectors, from the
    GPU's F2).  Throughput = workers / mean scaled seconds per query."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import prng, search

    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    n_s = min(sample_sets, len(offsets) - 1)
    X = db_cpu[: offsets[n_s]].astype(np.float64)
    off = offsets[: n_s + 1]
    idx = prng.projection_rows(cfg["seed"], cfg["dim"], cfg["code_bits"], cfg["fan_in"])
    t0 = time.perf_counter()
    with threadpool_limits(cores):
        ix = search.build_index(X, off, idx, cfg["wta_k"])
    build_s = time.perf_counter() - t0
    _CPU.update(cfg=cfg, ix=ix, q=q_cpu, q_off=q_off)
    nq = min(sample_queries, len(q_off) - 1, len(f2_vectors))
    t0 = time.perf_counter()
    with threadpool_limits(1):
        with mp.get_context("fork").Pool(cores) as pool:
            res = pool.map(_cpu_query, range(nq), chunksize=1)
    wall = time.perf_counter() - t0
    per_q = []
    for i, (te, tf, tr, vec) in enumerate(res):
        per_q.append(te + tf * n_sets_full / n_s + tr / max(1, vec) * float(f2_vectors[i]))
    return {
        "value": cores / (sum(per_q) / len(per_q)),
        "unit": "queries/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle search of {nq} queries against the first {n_s} sets of the workload (slice index built "
                   f"in {build_s:.1f} s, untimed), in a pool of {cores} worker processes with one BLAS thread each "
                   f"({wall:.1f} s wall); per query the filter steps are scaled by {n_sets_full}/{n_s} and the "
                   f"exact re-rank from its time per vector to the {np.mean(f2_vectors[:nq]):.0f} vectors (mean) "
                   f"of that query's F2 on the full database; throughput = workers / mean scaled time"),
        "mean_s_per_query": {"encode": float(np.mean([r[0] for r in res])),
                             "filter_scaled": float(np.mean([r[1] * n_sets_full / n_s for r in res])),
                             "rerank_scaled": float(np.mean([r[2] / max(1, r[3]) * float(f2_vectors[i])
                                                             for i, r in enumerate(res)]))},
    }


def concurrent_streams(ix, q, q_off, k, steps, ref_ids, streams):
    """The same batch searched by several host threads at once, each on its
    own stream and workspace (a server keeping several batches in flight on
    one GPU): total queries over the wall time, outside the headline's timed
    steps, with every thread's results checked against the single stream's."""
    import threading

    import numpy as np
    import torch

    n_q, NQ = len(q_off) - 1, int(q_off[-1])
    runs = []
    for i in range(streams):
        st = torch.cuda.Stream()
        ws = ix.search_workspace(n_q, NQ)
        out = (torch.empty(n_q, k, dtype=torch.int32, device=q.device),
               torch.empty(n_q, k, dtype=torch.float32, device=q.device),
               torch.empty(n_q, dtype=torch.int32, device=q.device))
        ix.search(q, q_off, k, ws=ws, out=out, stream=st)
        runs.append((st, ws, out))
    torch.cuda.synchronize()

    def worker(i):
        st, ws, out = runs[i]
        for _ in range(steps):
            ix.search(q, q_off, k, ws=ws, out=out, stream=st)
        st.synchronize()

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(streams)]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    same = all(np.array_equal(r[2][0].cpu().numpy().view(np.uint32), ref_ids) for r in runs)
    qps = streams * steps * n_q / el
    log(f"{streams} concurrent streams: {qps:.0f} q/s; identical results {same}")
    return {"streams": streams, "qps": qps, "steps_per_stream": steps, "identical_results": bool(same),
            "note": "host threads each searching the batch on their own stream and workspace; not the headline value"}


def f2_vectors_per_query(ix, q, q_off, db_offsets):
    """Vectors in each query's F2 (sum of the member sets' sizes), from the
    GPU's candidate lists (outside any timed region)."""
    import numpy as np
    ids, _, cnt = ix.candidates(q, q_off)
    ids = ids.cpu().numpy().view(np.uint32)
    cnt = cnt.cpu().numpy()
    sizes = np.diff(np.asarray(db_offsets, dtype=np.int64))
    return np.array([int(sizes[ids[i, :cnt[i]].astype(np.int64)].sum()) for i in range(len(cnt))], dtype=np.int64)


def sketch_rows(ix, q, q_off):
    """Sum over the queries of |S_Q|: the tile rows the bit-sliced filter
    adds for every set (computed outside the timed region)."""
    import numpy as np
    _, sq, _ = ix.query_sketch(q, q_off)
    return float(np.unpackbits(sq.cpu().numpy().view(np.uint8)).sum())


def rooflines(per_step, work, L, dim_padded, rerank_kernel, rerank_file, n_sets=None, counted=True):
    """Roofline of the dominant stage (filter or re-rank) from its
    algorithmic work per launch and its measured time per launch.  counted:
    the committed counter summaries were taken on this workload (the 1M-set,
    d = 384 one); otherwise traffic is null."""
    csrc = os.path.join(ROOT, "paper_2412_03301_amd", "csrc")
    dominant = max(("filter", "rerank"), key=lambda s2: per_step.get(s2, 0.0))
    # exact passes read both planes and the norm; the screen reads the high
    # plane and the 8-byte screening pair
    scr_vec = work.get("rerank_screen_vectors", 0.0)
    rer_bytes = work["rerank_vectors"] * (dim_padded * 2 + 4) + scr_vec * (dim_padded + 8)
    if dominant == "filter" and n_sets and work.get("sketch_rows"):
        # bit-sliced counting: every query adds its |S_Q| tile rows for every
        # set; one 3:2 carry-save compression (two 3-input logic ops) per
        # row and 32-bit word of 32 sets
        words = -(-n_sets // 32)
        ops = work["sketch_rows"] * words * 2
        ach = ops / (per_step["filter"] / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": ALU_PEAK_TOPS, "unit": "Tops/s", "frac": ach / ALU_PEAK_TOPS,
                "kernel": "k_filter_sliced<4,9>",
                "algorithmic": f"{work['sketch_rows']:.4g} query rows x {words} words x 2 int32 ops per launch",
                "traffic": traffic_from_profiles(os.path.join(csrc, "k_sliced.hip"), "k_filter_sliced")
                if counted else None}
    else:
        ach = rer_bytes / (per_step["rerank"] / 1e3) / 1e9
        # with the screen, the stage is the screen kernel (high planes of the
        # candidates after the first 64) and the exact kernel's launches; the
        # persistent batched kernel screens inside itself
        label = rerank_kernel
        if scr_vec:
            label = (f"{rerank_kernel} (re-rank stage, first-tile screen inside the kernel)"
                     if rerank_kernel == "k_haus_queue" else f"k_haus_screen + {rerank_kernel} (re-rank stage)")
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "kernel": label,
                "algorithmic": (f"{rer_bytes:.4g} bytes per step, all re-rank launches (vectors read in full "
                                f"x (2 dp + 4) + vectors screened x (dp + 8))"),
                "traffic": traffic_from_profiles(os.path.join(csrc, rerank_file), rerank_kernel)
                if counted else None}
    rerank_roof = {"achieved_gbs": rer_bytes / (per_step["rerank"] / 1e3) / 1e9 if per_step.get("rerank") else None,
                   "vectors_read": work["rerank_vectors"], "vectors_screened": scr_vec,
                   "candidates": work["rerank_candidates"], "abandoned": work["rerank_abandoned"],
                   "screened_out": work.get("rerank_screened", 0.0)}
    return roof, rerank_roof


def bf16_bruteforce(ix, q, q_off, k, nq, truth, n_vec):
    """Brute force through the bfloat16 copy of the vectors on the matrix
    cores (approximate Hausdorff values of every set, then the k smallest):
    throughput and recall against the exact brute force."""
    import numpy as np
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbytes = ix.attach_lowp("bf16")
    torch.cuda.synchronize()
    attach_s = time.perf_counter() - t0
    n = ix.n_sets
    qb = q[: int(q_off[nq])].contiguous()
    ob = q_off[: nq + 1]
    ids = torch.arange(n, dtype=torch.int32, device=q.device).repeat(nq, 1)
    ix.hausdorff_lowp(qb[: int(ob[1])].contiguous(), ob[:2], ids[:1], "bf16")   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h2 = ix.hausdorff_lowp(qb, ob, ids, "bf16")
    top = torch.topk(h2, k, dim=1, largest=False, sorted=True).indices
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    top = top.cpu().numpy()
    recall = float(np.mean([len(set(top[i].tolist()) & set(truth[i].tolist())) / k for i in range(nq)]))
    qsz = np.diff(ob).astype(np.float64)
    flops = float((2.0 * qsz * n_vec * ix.dim_padded).sum())
    del h2, ids
    ix.__dict__.get("_lowp", {}).pop("bf16", None)
    torch.cuda.empty_cache()
    return {"qps": nq / el, "queries": nq, "recall_at_10": recall, "kernel": "k_haus_lp<bf16> over every set + topk",
            "attach_s": attach_s, "copy_bytes": nbytes,
            "roofline": {"bound": "mfma", "achieved": flops / el / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": flops / el / 1e12 / 2500.0,
                         "algorithmic": f"{flops:.4g} bf16 flops (2 m_q N dp) over {nq} queries"}}


def stage_rooflines(per_step, work, w, n_q, NQ, ix):
    """HBM and ALU figures of the filter and the query encode beside the
    re-rank's: the filter streams the position-major bitmap planes of every
    set once per step (L x ld / 8 bytes) and does 2 int32 ops per query row
    and 32-set word; the encode reads 2 dp bytes and writes L / 8 per query
    vector and does L s adds and about 30 L compares of its threshold search."""
    L, s = w["code_bits"], w["fan_in"]
    out = {}
    if per_step.get("filter"):
        t = per_step["filter"] / 1e3
        words = -(-w["n_sets"] // 32)
        ops = work["sketch_rows"] * words * 2
        byts = L * ix.ld / 8 + 2 * ix.ld
        out["filter"] = {"kernel": "k_filter_sliced", "alu_achieved_tops": ops / t / 1e12,
                         "alu_frac": ops / t / 1e12 / ALU_PEAK_TOPS, "hbm_gbs": byts / t / 1e9,
                         "hbm_frac": byts / t / 1e9 / HBM_PEAK_GBS,
                         "note": (f"{ops:.4g} int32 ops ({work['sketch_rows']:.4g} query rows x {words} words x 2) "
                                  f"and {byts:.4g} bytes of bitmap planes per step; the kernel is bound by VALU "
                                  f"issue, not HBM")}
    if per_step.get("encode"):
        t = per_step["encode"] / 1e3
        byts = NQ * (2 * ix.dim_padded + L / 8)
        ops = NQ * (L * s + 30 * L)
        out["encode"] = {"kernel": "k_encode_vectors", "hbm_gbs": byts / t / 1e9, "hbm_frac": byts / t / 1e9 / HBM_PEAK_GBS,
                         "alu_achieved_tops": ops / t / 1e12, "alu_frac": ops / t / 1e12 / ALU_PEAK_TOPS,
                         "note": f"{NQ} query vectors: {byts:.4g} bytes and about {ops:.4g} int32 ops per step"}
    return out


def operating_points(ix, q, q_off, k, truth, nb, args, w):
    """Throughput and recall@10 (first nb queries, against the exact brute
    force) at each T of --op-sweep; the cheapest T reaching 0.95."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs
    n_q = len(q_off) - 1
    NQ = int(q_off[-1])
    rows = []
    for T in [int(x) for x in args.op_sweep.split(",") if x]:
        ix.set_search_params(3, 1, T)
        ws = ix.search_workspace(n_q, NQ)
        out = (torch.empty(n_q, k, dtype=torch.int32, device=q.device),
               torch.empty(n_q, k, dtype=torch.float32, device=q.device),
               torch.empty(n_q, dtype=torch.int32, device=q.device))
        ix.search(q, q_off, k, ws=ws, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ix.search(q, q_off, k, ws=ws, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ids = out[0].cpu().numpy().view(np.uint32)
        rec = float(np.mean([len(set(ids[i].tolist()) & set(truth[i].tolist())) / k for i in range(nb)]))
        # stage times of one more call (the dense fallback shows up as its own stage)
        bvs.profile_enable(True)
        ix.search(q, q_off, k, ws=ws, out=out)
        torch.cuda.synchronize()
        st = {nm: round(ms, 4) for nm, (ms, c) in bvs.profile_read().items() if c}
        bvs.profile_enable(False)
        rows.append({"top_t": T, "qps": n_q * args.steps / el, "recall_at_10": rec, "stages_ms": st})
        log(f"T={T}: {rows[-1]['qps']:.0f} q/s, recall@10 {rec:.4f}; stages {st}")
        del ws, out
    ok = [r for r in rows if r["recall_at_10"] >= 0.95]
    best = max(ok, key=lambda r: r["qps"]) if ok else None
    return {"rows": rows, "recall_queries": nb, "cheapest_at_0.95": best}


def brute_recall(ix, q, q_off, ids, k, nb):
    """Recall@k of `ids` against the exact brute force on the first nb
    queries, and the brute-force throughput on them."""
    import numpy as np
    import torch
    qb = q[: int(q_off[nb])].contiguous()
    ob = q_off[: nb + 1]
    bws = ix.brute_workspace(nb, int(ob[-1]))
    ix.bruteforce(q[: int(q_off[2])].contiguous(), q_off[:3], k)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bids, _, _ = ix.bruteforce(qb, ob, k, ws=bws)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    bids = bids.cpu().numpy().view(np.uint32)
    recall = float(np.mean([len(set(ids[i].tolist()) & set(bids[i].tolist())) / k for i in range(nb)]))
    return recall, nb / bt


def batched(args, w, cfg, ix, q, q_off, n_vec, build_s, cpu_db, db_offsets):
    """Uneven query batch through the batched entry points: one hipGraph
    replay per step (persistent re-rank inside), autotuned re-rank shape,
    compared with one search call per query and with one multi-launch
    search call over the whole batch."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs

    dev = q.device
    n_q, k = w["n_queries"], w["k"]
    NQ = int(q_off[-1])
    sizes = np.diff(q_off)
    log(f"batched: {n_q} queries, sizes {sizes.min()}-{sizes.max()} (mean {sizes.mean():.1f})")
    t0 = time.perf_counter()
    b = bvs.Batch(ix, q, q_off, k, graph=True)
    info = b.info()
    log(f"plan bound in {time.perf_counter() - t0:.2f} s: lds_rows={info['lds_rows']} waves={info['waves']} "
        f"blocks={info['blocks']} tried={info['tried']}")
    for i in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    st = b.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(st)
    for i in range(args.steps):
        lib_status = bvs.lib().bvs_batch_launch(b._h, bvs._stream(st))
        bvs.check(lib_status)
    ev1.record(st)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t_wall
    gpu_ms = ev0.elapsed_time(ev1)
    b.status()
    elapsed_s = max(wall_s, gpu_ms / 1e3)
    qps = n_q * args.steps / elapsed_s
    log(f"timed {args.steps} graph replays: {gpu_ms:.2f} ms (wall {wall_s * 1e3:.2f} ms) -> {qps:.0f} q/s")
    ids = b.ids.cpu().numpy().view(np.uint32)

    # stage times and work: the same plan shape launched eagerly with events
    phases = info["waves"] == 0   # the tuner chose the phase sequence by size class
    e = bvs.Batch(ix, q, q_off, k, lds_rows=info["lds_rows"], waves=info["waves"], graph=False, phases=phases)
    e.run()
    bvs.profile_enable(True)
    for i in range(args.steps):
        e.run()
    stages = bvs.profile_read()
    bvs.profile_enable(False, counters=True)
    e.run()
    work = dict(bvs.profile_counters())
    bvs.profile_enable(False)
    same = np.array_equal(e.ids.cpu().numpy(), b.ids.cpu().numpy())
    e.close()
    per_step = {name: ms / max(1, calls) for name, (ms, calls) in stages.items() if calls}

    # one multi-launch search call over the whole batch
    ws = ix.search_workspace(n_q, NQ)
    out = (torch.empty(n_q, k, dtype=torch.int32, device=dev), torch.empty(n_q, k, dtype=torch.float32, device=dev),
           torch.empty(n_q, dtype=torch.int32, device=dev))
    ix.search(q, q_off, k, ws=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ix.search(q, q_off, k, ws=ws, out=out)
    torch.cuda.synchronize()
    call_qps = n_q * args.steps / (time.perf_counter() - t0)
    same_call = np.array_equal(out[0].cpu().numpy(), b.ids.cpu().numpy())
    del ws

    # one search call per query (each call: its own launches and host sync)
    nper = min(args.per_query_sample, n_q)
    ws1 = ix.search_workspace(1, int(sizes.max()))
    out1 = (torch.empty(1, k, dtype=torch.int32, device=dev), torch.empty(1, k, dtype=torch.float32, device=dev),
            torch.empty(1, dtype=torch.int32, device=dev))
    qs = [q[int(q_off[i]):int(q_off[i + 1])].contiguous() for i in range(nper)]
    ix.search(qs[0], [0, qs[0].shape[0]], k, ws=ws1, out=out1)
    mism = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nper):
        ix.search(qs[i], [0, qs[i].shape[0]], k, ws=ws1, out=out1)
    torch.cuda.synchronize()
    per_query_qps = nper / (time.perf_counter() - t0)
    for i in range(0, nper, max(1, nper // 16)):
        ix.search(qs[i], [0, qs[i].shape[0]], k, ws=ws1, out=out1)
        mism += int(not np.array_equal(out1[0].cpu().numpy()[0].view(np.uint32), ids[i]))
    log(f"per-query calls: {per_query_qps:.0f} q/s on {nper}; one search call: {call_qps:.0f} q/s; "
        f"identical results: eager {same}, call {same_call}, per-query mismatches {mism}")

    recall = brute_qps = None
    if not args.no_brute:
        nb = min(args.brute_queries, n_q)
        recall, brute_qps = brute_recall(ix, q, q_off, ids, k, nb)
        log(f"brute force on {nb} queries: {brute_qps:.1f} q/s; recall@10 {recall:.4f}")

    work["sketch_rows"] = sketch_rows(ix, q, q_off)
    roof, rerank_roof = rooflines(per_step, work, w["code_bits"], ix.dim_padded,
                                  "k_haus_cand" if phases else "k_haus_queue", "k_haus.hip" if phases else "k_batch.hip",
                                  w["n_sets"], counted=False)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        ncq = min(args.cpu_sample_queries, len(q_off) - 1)
        qc = q[: int(q_off[ncq])].cpu().numpy()
        f2v = f2_vectors_per_query(ix, q[: int(q_off[ncq])].contiguous(), q_off[: ncq + 1], db_offsets)
        cpu = cpu_baseline(cpu_db, db_offsets, qc, q_off, cfg, w["n_sets"], args.cpu_sample_sets, ncq, f2v)
    L = w["code_bits"]
    return {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "exact int16 grid values as int8 hi/lo planes (4 int8 MFMA products, int32 accumulation)",
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                         f"{w['n_topics']} topics; FlyHash L={L}, s={w['fan_in']}, wta_k={w['wta_k']}; "
                         f"A=3, M=1, T={w['top_t']}; {n_q} fresh-entity queries of 1-{w['max_query']} vectors "
                         f"(log-uniform) per step, one hipGraph replay; top-{k}"),
            "n_sets": w["n_sets"], "n_vectors": n_vec, "n_queries": n_q, "query_vectors": NQ,
        },
        "batch_plan": {k2: info[k2] for k2 in ("lds_rows", "waves", "blocks", "from_cache", "graph", "tried")},
        "per_query_calls_qps": per_query_qps,
        "per_query_sample": nper,
        "single_call_qps": call_qps,
        "identical_to_single_call": bool(same_call and same and mism == 0),
        "recall_at_10": recall,
        "recall_sample_queries": None if args.no_brute else min(args.brute_queries, n_q),
        "bruteforce_qps": brute_qps,
        "speedup_vs_bruteforce": (qps / brute_qps) if brute_qps else None,
        "stages_ms_per_step": per_step,
        "work_per_step": work,
        "rerank": rerank_roof,
        "index_build_s": build_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def precision(args, w, cfg, ix, q, q_off, n_vec, build_s, cpu_db, db_offsets):
    """The exact re-rank against the BF16 and FP8 E4M3 re-rank with the exact
    re-check within a margin: throughput, recall@10 against brute force,
    agreement with the exact cascade, and the error of the approximate
    values against the exact (float64-equal) distances."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs

    dev = q.device
    n_q, k = w["n_queries"], w["k"]
    NQ = int(q_off[-1])
    attach_s = {}
    for fmt in ("bf16", "fp8"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nb = ix.attach_lowp(fmt)
        torch.cuda.synchronize()
        attach_s[fmt] = time.perf_counter() - t0
        log(f"attached {fmt} copy ({nb / 2**30:.1f} GiB) in {attach_s[fmt]:.2f} s")

    ws = ix.lowp_workspace(n_q, NQ)
    outs, rows = {}, {}

    def run(mode):
        if mode == "exact":
            return ix.search(q, q_off, k, ws=ws, out=outs["exact"])
        return ix.search_lowp(q, q_off, k, mode, margin=args.margin, ws=ws, out=outs[mode])

    for mode in ("exact", "bf16", "fp8"):
        outs[mode] = (torch.empty(n_q, k, dtype=torch.int32, device=dev),
                      torch.empty(n_q, k, dtype=torch.float32, device=dev),
                      torch.empty(n_q, dtype=torch.int32, device=dev)) + \
            (() if mode == "exact" else (torch.empty(n_q, dtype=torch.int32, device=dev),))
        for i in range(args.warmup):
            run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            run(mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # stage times from as many steps again with the per-stage events on
        bvs.profile_enable(True)
        for i in range(args.steps):
            run(mode)
        torch.cuda.synchronize()
        stages = bvs.profile_read()
        bvs.profile_enable(False)
        rows[mode] = {"qps": n_q * args.steps / el, "ms_per_step": el * 1e3 / args.steps,
                      "stages_ms_per_step": {nm: ms / max(1, c) for nm, (ms, c) in stages.items() if c}}
        # work counters of one more call (outside the timed region)
        bvs.profile_enable(False, counters=True)
        run(mode)
        torch.cuda.synchronize()
        rows[mode]["work"] = dict(bvs.profile_counters())
        bvs.profile_enable(False)
        log(f"{mode}: {rows[mode]['qps']:.0f} q/s ({rows[mode]['ms_per_step']:.2f} ms/step)")

    exact_ids = outs["exact"][0].cpu().numpy().view(np.uint32)
    exact_dist = outs["exact"][1].cpu().numpy()
    for mode in ("bf16", "fp8"):
        ids = outs[mode][0].cpu().numpy().view(np.uint32)
        rows[mode]["identical_to_exact"] = float(np.mean([np.array_equal(ids[i], exact_ids[i]) for i in range(n_q)]))
        rows[mode]["rechecked_mean"] = float(outs[mode][3].float().mean().item())
        # approximate values of the exact top-10 against their exact distances
        ah = ix.hausdorff_lowp(q, q_off, outs["exact"][0], mode).cpu().numpy().astype(np.float64)
        d_true = exact_dist.astype(np.float64)
        rel = np.abs(np.sqrt(np.maximum(ah, 0)) - d_true) / np.maximum(d_true, 1e-12)
        rows[mode]["approx_rel_err"] = {"mean": float(rel.mean()), "p99": float(np.quantile(rel, 0.99)),
                                        "max": float(rel.max()),
                                        "per_query_max_mean": float(rel.max(axis=1).mean())}
        dd = np.abs(outs[mode][1].cpu().numpy().astype(np.float64) - d_true)
        same = ids == exact_ids
        rows[mode]["reported_rel_err_where_same_id"] = float((dd[same] / np.maximum(d_true[same], 1e-12)).max())

    recall = brute_qps = None
    if not args.no_brute:
        nb = min(args.brute_queries, n_q)
        for mode in ("exact", "bf16", "fp8"):
            ids = outs[mode][0].cpu().numpy().view(np.uint32)
            r, bq = brute_recall(ix, q, q_off, ids, k, nb)
            rows[mode]["recall_at_10"] = r
            brute_qps = bq
        log(f"brute force {brute_qps:.1f} q/s; recall exact {rows['exact']['recall_at_10']:.4f} "
            f"bf16 {rows['bf16']['recall_at_10']:.4f} fp8 {rows['fp8']['recall_at_10']:.4f}")

    # float64 oracle on the host for a few queries: exact distances of the
    # reported results and the oracle's own approximate values
    from oracle import hausdorff, lowp
    from paper_2412_03301_amd import synth
    host = {}
    nh = 4
    offs = np.asarray(db_offsets)
    want = set()
    for mode in ("bf16", "fp8"):
        want |= set(outs[mode][0][:nh].cpu().numpy().view(np.uint32).reshape(-1).tolist())
    sets = synth.redraw_sets(w["n_sets"], w["size_lo"], w["size_hi"], w["dim"], w["n_topics"], sorted(want),
                             seed=0, device=dev)
    for mode in ("bf16", "fp8"):
        ids = outs[mode][0].cpu().numpy().view(np.uint32)
        errs, aerrs = [], []
        for i in range(nh):
            Q = q[int(q_off[i]):int(q_off[i + 1])].cpu().numpy().astype(np.float64)
            for t in range(k):
                j = int(ids[i, t])
                V = sets[j].astype(np.float64)
                h2 = hausdorff.hausdorff_sq(Q, V)
                errs.append(abs(float(outs[mode][1][i, t]) - np.sqrt(h2)) / np.sqrt(h2))
                aerrs.append(abs(np.sqrt(lowp.approx_hausdorff_sq(Q, V, mode)) - np.sqrt(h2)) / np.sqrt(h2))
        host[mode] = {"queries": nh, "reported_max_rel_err": float(max(errs)),
                      "approx_max_rel_err": float(max(aerrs))}
    # the line reports the form under test; the exact re-rank is listed beside it
    best = args.form
    st = rows[best]["stages_ms_per_step"]
    work = {"filter_pairs": 0.0, "rerank_vectors": 0.0, "rerank_candidates": 0.0, "rerank_abandoned": 0.0}
    roof = None
    if best != "exact":
        # approximate re-rank: the candidate rows it read (a device work
        # counter; abandoned candidates count only the tiles they read), at
        # row_bytes + 4 bytes each
        vec = float(rows[best]["work"]["lowp_vectors"])
        rb = 2 * ix.dim_padded if best == "bf16" else -(-ix.dim_padded // 128) * 128
        byts = vec * (rb + 4)
        ach = byts / (st["approx"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "kernel": f"k_haus_lp ({best})", "stage": "approx (query encode, approximate values, selection)",
                "algorithmic": f"{byts:.4g} bytes per step ({vec:.4g} candidate vectors read x {rb + 4} B)",
                "traffic": None}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        ncq = min(args.cpu_sample_queries, len(q_off) - 1)
        qc = q[: int(q_off[ncq])].cpu().numpy()
        f2v = f2_vectors_per_query(ix, q[: int(q_off[ncq])].contiguous(), q_off[: ncq + 1], db_offsets)
        cpu = cpu_baseline(cpu_db, db_offsets, qc, q_off, cfg, w["n_sets"], args.cpu_sample_sets, ncq, f2v)
    L = w["code_bits"]
    return {
        "metric": METRIC,
        "value": rows[best]["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rows[best]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"exact": "exact int16 grid values as int8 hi/lo planes", "bf16": "bf16",
                  "fp8": "fp8-e4m3"}[best],
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                         f"{w['n_topics']} topics; FlyHash L={L}, s={w['fan_in']}, wta_k={w['wta_k']}; "
                         f"A=3, M=1, T={w['top_t']}; {n_q} subset queries per step; top-{k}; re-rank in "
                         f"{best} with exact re-check within {args.margin:.0%} of the k-th distance"),
            "n_sets": w["n_sets"], "n_vectors": n_vec, "n_queries": n_q, "query_vectors": NQ,
        },
        "forms": rows,
        "margin": args.margin,
        "host_oracle_check": host,
        "attach_s": attach_s,
        "bruteforce_qps": brute_qps,
        "speedup_vs_bruteforce": (rows[best]["qps"] / brute_qps) if brute_qps else None,
        "recall_sample_queries": None if args.no_brute else min(args.brute_queries, n_q),
        "index_build_s": build_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def learned_bench(args, w, cfg, dev):
    """Learned projection: mine triplets with the exact brute force on a
    separate training corpus, train the network with the library's trainer,
    then search the evaluation database with the learned index and with the
    random FlyHash index over a sweep of T (recall@10 against brute force and
    throughput for each), keeping the random projection if the learned one
    does not reach its recall."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs, synth

    d, L, k_wta, H = w["dim"], w["code_bits"], w["wta_k"], w["hidden"]
    n_tr = args.train_sets or w["train_sets"]
    n_mine = args.mine_queries or w["mine_queries"]
    n_neg = w["negatives"]
    k = w["k"]
    t_start = time.perf_counter()
    log(f"training corpus: {n_tr} sets (d={d}, seed {w['train_seed']})")
    tdb = synth.make_database(n_tr, w["size_lo"], w["size_hi"], d, w["n_topics"], seed=w["train_seed"], device=dev)
    tq, tq_off, _ = synth.make_subset_queries(tdb, n_mine, seed=w["train_seed"] + 1)
    tq = tq.contiguous()
    p_tr = bvs.Params.make(dim=d, code_bits=L, fan_in=w["fan_in"], wta_k=k_wta, top_t=w["top_t"], seed=0)
    tix = bvs.Index(p_tr, tdb.vectors, tdb.offsets)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pos = np.zeros((n_mine, 10), np.int64)
    ch = 2048
    for c0 in range(0, n_mine, ch):
        c1 = min(n_mine, c0 + ch)
        qc = tq[int(tq_off[c0]):int(tq_off[c1])].contiguous()
        ids, _, _ = tix.bruteforce(qc, tq_off[c0:c1 + 1] - tq_off[c0], 10)
        pos[c0:c1] = ids.cpu().numpy().view(np.uint32)
    mine_s = time.perf_counter() - t0
    log(f"mined the exact top-10 of {n_mine} training queries in {mine_s:.1f} s")
    del tix
    torch.cuda.empty_cache()
    rng = np.random.default_rng(w["train_seed"] + 2)
    neg = rng.integers(0, n_tr, size=(n_mine, n_neg))
    qid = n_tr + np.arange(n_mine)
    trip = np.stack([np.repeat(qid, 10 * n_neg), np.repeat(pos.reshape(-1), n_neg), np.tile(neg, (1, 10)).reshape(-1)],
                    axis=1).astype(np.uint32)
    coll = torch.cat([tdb.vectors, tq]).contiguous()
    coll_off = np.concatenate([tdb.offsets, tdb.offsets[-1] + tq_off[1:]])
    del tdb
    weights = bvs.mlp_weights(d, H, L, seed=w["train_seed"] + 3)
    tc = bvs.TrainConfig(d, H, L, k_wta, args.train_batch, args.train_epochs, args.train_lr, args.train_tau,
                         args.train_margin, 0, w["train_seed"] + 4)
    max_rows = args.train_batch * 3 * int(np.diff(coll_off).max())
    trainer = bvs.Trainer(tc, coll, coll_off, max_rows)
    loss0, _ = trainer.gradients(weights, trip[: args.train_batch])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = trainer.train(weights, trip)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss1, _ = trainer.gradients(weights, trip[: args.train_batch])
    log(f"trained on {len(trip)} triplets in {train_s:.1f} s: epoch losses {losses}, first batch {loss0:.2f} -> "
        f"{loss1:.2f}")
    del trainer, coll
    torch.cuda.empty_cache()

    log(f"evaluation corpus: {w['n_sets']} sets (d={d}, seed 0)")
    db = synth.make_database(w["n_sets"], w["size_lo"], w["size_hi"], d, w["n_topics"], seed=0, device=dev)
    q, q_off, _ = synth.make_subset_queries(db, w["n_queries"], seed=1)
    q = q.contiguous()
    n_q = w["n_queries"]
    NQ = int(q_off[-1])
    nb = min(args.brute_queries, n_q)
    truth = None
    rows = []
    out = (torch.empty(n_q, k, dtype=torch.int32, device=dev), torch.empty(n_q, k, dtype=torch.float32, device=dev),
           torch.empty(n_q, dtype=torch.int32, device=dev))
    counters = None
    for form in ("random", "learned"):
        for T in [int(x) for x in args.sweep_t.split(",")]:
            p = bvs.Params.make(dim=d, code_bits=L, fan_in=w["fan_in"], wta_k=k_wta, top_t=T, seed=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ix = bvs.Index(p, db.vectors, db.offsets, mlp=(H, weights) if form == "learned" else None)
            torch.cuda.synchronize()
            build_s = time.perf_counter() - t0
            ws = ix.search_workspace(n_q, NQ)
            for i in range(args.warmup):
                ix.search(q, q_off, k, ws=ws, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                ix.search(q, q_off, k, ws=ws, out=out)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            # stage times from as many steps again with the per-stage events on
            bvs.profile_enable(True)
            for i in range(args.steps):
                ix.search(q, q_off, k, ws=ws, out=out)
            torch.cuda.synchronize()
            st = {nm: ms / max(1, c) for nm, (ms, c) in bvs.profile_read().items() if c}
            bvs.profile_enable(False)
            if form == "learned" and T == w["top_t"]:
                bvs.profile_enable(False, counters=True)
                ix.search(q, q_off, k, ws=ws, out=out)
                counters = dict(bvs.profile_counters())
                counters["sketch_rows"] = sketch_rows(ix, q, q_off)
                bvs.profile_enable(False)
            ids = out[0].cpu().numpy().view(np.uint32)
            if truth is None:
                qb = q[: int(q_off[nb])].contiguous()
                t1 = time.perf_counter()
                bids, _, _ = ix.bruteforce(qb, q_off[: nb + 1], k)
                torch.cuda.synchronize()
                brute_qps = nb / (time.perf_counter() - t1)
                truth = bids.cpu().numpy().view(np.uint32)
            recall = float(np.mean([len(set(ids[i].tolist()) & set(truth[i].tolist())) / k for i in range(nb)]))
            rows.append({"form": form, "top_t": T, "qps": n_q * args.steps / el, "recall_at_10": recall,
                         "ms_per_step": el * 1e3 / args.steps, "build_s": build_s, "stages_ms_per_step": st})
            log(f"{form} T={T}: {rows[-1]['qps']:.0f} q/s, recall@10 {recall:.4f} (build {build_s:.1f} s)")
            del ix, ws
            torch.cuda.empty_cache()
    at_t = {r["form"]: r for r in rows if r["top_t"] == w["top_t"]}
    keep = "learned" if at_t["learned"]["recall_at_10"] >= at_t["random"]["recall_at_10"] else "random"
    best = at_t[keep]
    roof = None
    if counters is not None and keep == "learned":
        work = {k2: float(v) for k2, v in counters.items()}
        roof, _ = rooflines(best["stages_ms_per_step"], work, L, -(-d // 64) * 64, "k_haus_cand", "k_haus.hip",
                            w["n_sets"], counted=False)
    return {
        "metric": METRIC,
        "value": best["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 projection network; exact int16 grid values as int8 hi/lo planes in the re-rank",
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={d}, {w['n_topics']} topics; "
                         f"learned projection {d}->{H} relu->{L}, WTA k={k_wta}; A=3, M=1, T={w['top_t']}; "
                         f"{n_q} subset queries per step; top-{k}; projection in use: {keep}"),
            "n_sets": w["n_sets"], "n_queries": n_q, "query_vectors": NQ,
        },
        "projection_in_use": keep,
        "training": {"corpus_sets": n_tr, "mined_queries": n_mine, "triplets": int(len(trip)), "mine_s": mine_s,
                     "train_s": train_s, "epoch_losses": losses, "first_batch_loss_before_after": [loss0, loss1],
                     "batch_triplets": args.train_batch, "lr": args.train_lr, "tau": args.train_tau,
                     "margin": args.train_margin, "hidden": H},
        "sweep": rows,
        "bruteforce_qps": brute_qps,
        "recall_sample_queries": nb,
        "roofline": roof,
        "cpu_baseline": None,
        "total_s": time.perf_counter() - t_start,
    }


def full_scan(args, w, ix, q, q_off, n_vec, build_s):
    """The full-scan search of Alg. 2 on the scale database: Haus^H of the
    query codes to every set, the first c = T sets, exact re-rank; compared
    with the cascade (Alg. 6) and the exact brute force on the same queries."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs

    dev = q.device
    k = w["k"]
    n_q = min(args.full_queries, w["n_queries"])
    qf = q[: int(q_off[n_q])].contiguous()
    of = q_off[: n_q + 1]
    NQ = int(of[-1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbytes = ix.attach_codes()
    torch.cuda.synchronize()
    attach_s = time.perf_counter() - t0
    log(f"attached sparse codes ({nbytes / 2**30:.1f} GiB) in {attach_s:.2f} s")
    ws = ix.full_workspace(n_q, NQ)
    out = ix._outs(n_q, k)
    for i in range(args.warmup):
        ix.search_full(qf, of, k, ws=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ix.search_full(qf, of, k, ws=ws, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    qps = n_q * args.steps / el
    bvs.profile_enable(True)
    for i in range(args.steps):
        ix.search_full(qf, of, k, ws=ws, out=out)
    torch.cuda.synchronize()
    per_step = {nm: ms / max(1, c) for nm, (ms, c) in bvs.profile_read().items() if c}
    bvs.profile_enable(False)
    ids = out[0].cpu().numpy().view(np.uint32)
    log(f"full scan: {qps:.1f} q/s on {n_q} queries per step; stages {per_step}")
    # the cascade on the same queries
    wsc = ix.search_workspace(n_q, NQ)
    outc = ix._outs(n_q, k)
    ix.search(qf, of, k, ws=wsc, out=outc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ix.search(qf, of, k, ws=wsc, out=outc)
    torch.cuda.synchronize()
    cascade_qps = n_q * args.steps / (time.perf_counter() - t0)
    cids = outc[0].cpu().numpy().view(np.uint32)
    recall = recall_c = brute_qps = None
    if not args.no_brute:
        recall, brute_qps = brute_recall(ix, q, q_off, ids, k, n_q)
        bids = ix.bruteforce(qf, of, k)[0].cpu().numpy().view(np.uint32)
        recall_c = float(np.mean([len(set(cids[i].tolist()) & set(bids[i].tolist())) / k for i in range(n_q)]))
        log(f"recall@10: full scan {recall:.4f}, cascade {recall_c:.4f}; brute force {brute_qps:.1f} q/s")
    # scan work: every database vector against every query; positions are
    # read from HBM once per (query, set) pair
    L, K = w["code_bits"], w["wta_k"]
    KP = -(-K // 8) * 8
    scan_ms = per_step.get("fullscan")
    scan_bytes = n_vec * KP * 2 * n_q
    groups = (np.minimum(np.diff(of), 256) + 63) // 64
    # one table lookup and one 64-slot carry-save step (3 ops on each of 2
    # words) per code position, per vector and group of 64 query vectors
    ops = float(n_vec) * K * 7 * float(groups.sum())
    roof = None
    if scan_ms:
        ach_gbs = scan_bytes / (scan_ms / 1e3) / 1e9
        ach_ops = ops / (scan_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": ach_ops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": ach_ops / ALU_PEAK_TOPS, "kernel": "k_full_scan<7,1> (full-scan stage)",
                "algorithmic": (f"{ops:.4g} int32 ops per step: n_vectors x wta_k x 7 (one LDS lookup, 6 carry-save "
                                f"ops) x query groups of 64"),
                "hbm_gbs": ach_gbs, "hbm_frac": ach_gbs / HBM_PEAK_GBS, "hbm_bytes_per_step": scan_bytes,
                "traffic": None}
    return {
        "metric": "queries/sec of the full-scan search (Alg. 2) on 1M sets",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bit-sliced counts; exact integer re-rank",
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                         f"{w['n_topics']} topics; FlyHash L={L}, s={w['fan_in']}, wta_k={K}; c=T={w['top_t']}; "
                         f"{n_q} subset queries per step; top-{k}"),
            "n_sets": w["n_sets"], "n_vectors": n_vec, "n_queries": n_q, "query_vectors": NQ,
        },
        "recall_at_10": recall,
        "cascade_recall_at_10": recall_c,
        "cascade_qps_same_queries": cascade_qps,
        "bruteforce_qps": brute_qps,
        "speedup_vs_bruteforce": (qps / brute_qps) if brute_qps else None,
        "stages_ms_per_step": per_step,
        "codes_attach_s": attach_s,
        "codes_bytes": nbytes,
        "index_build_s": build_s,
        "roofline": roof,
        "cpu_baseline": None,
    }


def metrics_bench(args, w, ix, q, q_off, n_vec, build_s):
    """The cascade re-ranked by MeanMin (query to set) and by Min distance
    (Sec. 3.2) beside Hausdorff: throughput of the whole search, recall@10
    against the exact brute force by the same measure, and that brute
    force's throughput."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs

    k = w["k"]
    n_q = w["n_queries"]
    NQ = int(q_off[-1])
    nb = min(args.brute_queries, n_q)
    ws = ix.search_workspace(n_q, NQ)
    rows = {}
    for metric in ("hausdorff", "meanmin", "min"):
        out = (torch.empty(n_q, k, dtype=torch.int32, device=q.device),
               torch.empty(n_q, k, dtype=torch.float32, device=q.device),
               torch.empty(n_q, dtype=torch.int32, device=q.device))
        for i in range(args.warmup):
            ix.search_metric(q, q_off, k, metric, ws=ws, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ix.search_metric(q, q_off, k, metric, ws=ws, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        bvs.profile_enable(True)
        for i in range(args.steps):
            ix.search_metric(q, q_off, k, metric, ws=ws, out=out)
        torch.cuda.synchronize()
        per_step = {nm: ms / max(1, c) for nm, (ms, c) in bvs.profile_read().items() if c}
        bvs.profile_enable(False)
        ids = out[0].cpu().numpy().view(np.uint32)
        row = {"qps": n_q * args.steps / el, "ms_per_step": el * 1e3 / args.steps, "stages_ms_per_step": per_step}
        if not args.no_brute:
            qb, ob = q[: int(q_off[nb])].contiguous(), q_off[: nb + 1]
            bws = ix.brute_workspace(nb, int(ob[-1]))
            ix.bruteforce_metric(q[: int(q_off[2])].contiguous(), q_off[:3], k, metric)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bids = ix.bruteforce_metric(qb, ob, k, metric, ws=bws)[0]
            torch.cuda.synchronize()
            row["bruteforce_qps"] = nb / (time.perf_counter() - t0)
            bids = bids.cpu().numpy().view(np.uint32)
            row["recall_at_10"] = float(np.mean([len(set(ids[i].tolist()) & set(bids[i].tolist())) / k
                                                 for i in range(nb)]))
            row["speedup_vs_bruteforce"] = row["qps"] / row["bruteforce_qps"]
            del bws
        rows[metric] = row
        log(f"{metric}: {row['qps']:.0f} q/s, recall@10 {row.get('recall_at_10')}, brute {row.get('bruteforce_qps')}")
    mm = rows["meanmin"]
    return {
        "metric": "queries/sec of the cascade re-ranked by MeanMin on 1M sets (recall@10 against the MeanMin brute force)",
        "value": mm["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mm["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "exact int16 grid values as int8 hi/lo planes; MeanMin summed in f64, ranked in f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                         f"{w['n_topics']} topics; FlyHash L={w['code_bits']}, s={w['fan_in']}, wta_k={w['wta_k']}; "
                         f"A=3, M=1, T={w['top_t']}; {n_q} subset queries per step; top-{k}; re-rank by MeanMin, "
                         f"Min and Hausdorff"),
            "n_sets": w["n_sets"], "n_vectors": n_vec, "n_queries": n_q, "query_vectors": NQ,
        },
        "recall_at_10": mm.get("recall_at_10"),
        "recall_sample_queries": None if args.no_brute else nb,
        "by_metric": rows,
        "index_build_s": build_s,
        "roofline": None,
        "cpu_baseline": None,
    }


def trends_bench(args, w, dev):
    """The paper's parameter study (Sec. 6.3) on the scale generator: recall
    at 3, 5 and 10 against the exact brute force and throughput while
    sweeping the winner-take-all count k_wta and the Bloom filter size L
    (index rebuilt), the lists accessed A, the minimum count M and the
    candidate count T (search-time parameters of the same index)."""
    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs, synth

    t_start = time.perf_counter()
    db = synth.make_database(w["n_sets"], w["size_lo"], w["size_hi"], w["dim"], w["n_topics"], seed=0, device=dev)
    q, q_off, _ = synth.make_subset_queries(db, w["n_queries"], seed=1)
    q = q.contiguous()
    n_q = w["n_queries"]
    NQ = int(q_off[-1])
    k = 10

    def build(L, wta):
        p = bvs.Params.make(dim=w["dim"], code_bits=L, fan_in=w["fan_in"], wta_k=wta, access_lists=3, min_count=1,
                            top_t=1000, seed=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ix = bvs.Index(p, db.vectors, db.offsets)
        torch.cuda.synchronize()
        return ix, time.perf_counter() - t0

    ix, _ = build(4096, 64)
    truth = ix.bruteforce(q, q_off, k)[0].cpu().numpy().view(np.uint32)
    log(f"ground truth of {n_q} queries by brute force")

    def measure(ix, A, M, T, label, first_layer="bitmaps"):
        ix.set_search_params(A, M, T)
        ix.set_first_layer(first_layer)
        ws = ix.search_workspace(n_q, NQ)
        out = (torch.empty(n_q, k, dtype=torch.int32, device=q.device),
               torch.empty(n_q, k, dtype=torch.float32, device=q.device),
               torch.empty(n_q, dtype=torch.int32, device=q.device))
        for i in range(max(1, args.warmup)):
            ix.search(q, q_off, k, ws=ws, out=out)
        torch.cuda.synchronize()
        bvs.profile_enable(True)
        t0 = time.perf_counter()
        for i in range(args.steps):
            ix.search(q, q_off, k, ws=ws, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = {nm: ms / max(1, c) for nm, (ms, c) in bvs.profile_read().items() if c}
        bvs.profile_enable(False)
        ids = out[0].cpu().numpy().view(np.uint32)
        rec = {f"recall_at_{r}": float(np.mean([len(set(ids[i, :r].tolist()) & set(truth[i, :r].tolist())) / r
                                                for i in range(n_q)])) for r in (3, 5, 10)}
        f1 = None
        _, _, cnt = ix.candidates(q[: int(q_off[8])].contiguous(), q_off[:9])
        ix.set_first_layer("bitmaps")
        row = {"label": label, "A": A, "M": M, "T": T, "first_layer": first_layer, "qps": n_q * args.steps / el, **rec,
               "first_layer_ms": st.get("cutoff", 0.0) + st.get("filter", 0.0) + st.get("select", 0.0)
               + st.get("fallback", 0.0) + st.get("lists", 0.0), "rerank_ms": st.get("rerank"),
               "f2_count_mean_first8": float(cnt.float().mean().item())}
        del ws, out, f1
        log(f"{label} A={A} M={M} T={T} {first_layer}: {row['qps']:.0f} q/s, recall@3/5/10 {rec['recall_at_3']:.3f} "
            f"{rec['recall_at_5']:.3f} {rec['recall_at_10']:.3f}")
        return row

    rows = []
    for L in (1024, 2048, 4096):
        for wta in (16, 32, 48, 64):
            del ix
            torch.cuda.empty_cache()
            ix, bs = build(L, wta)
            r = measure(ix, 3, 1, 1000, f"L={L} k_wta={wta}")
            r.update(L=L, k_wta=wta, build_s=bs)
            rows.append(r)
            if wta == 64 and L in (1024, 4096):
                for A in (1, 2):
                    r = measure(ix, A, 1, 1000, f"L={L} k_wta=64")
                    r.update(L=L, k_wta=64)
                    rows.append(r)
                r = measure(ix, 3, 2, 1000, f"L={L} k_wta=64")
                r.update(L=L, k_wta=64)
                rows.append(r)
                for T in (200, 500, 2000, 4000):
                    r = measure(ix, 3, 1, T, f"L={L} k_wta=64")
                    r.update(L=L, k_wta=64)
                    rows.append(r)
                # the first layer from inverted lists (Def. 9, Alg. 4) against bitmaps / count columns
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lb = ix.attach_lists()
                torch.cuda.synchronize()
                attach_s = time.perf_counter() - t0
                log(f"L={L}: inverted lists {lb / 2**30:.2f} GiB built in {attach_s:.2f} s")
                for A, M in ((3, 1), (3, 2), (1, 1), (1, 2), (1, 3)):
                    for fl in (("bitmaps", "lists") if (A, M) in ((1, 2), (1, 3)) else ("lists",)):
                        r = measure(ix, A, M, 1000, f"L={L} k_wta=64", first_layer=fl)
                        r.update(L=L, k_wta=64, lists_bytes=lb, lists_build_s=attach_s)
                        rows.append(r)
    return {
        "metric": "recall@3/5/10 and queries/sec across the parameter study (Sec. 6.3) on 1M sets",
        "value": None,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(1, args.warmup),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "exact int16 grid values as int8 hi/lo planes",
        "data": "synthetic",
        "config": {"workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                                f"{w['n_topics']} topics; s={w['fan_in']}; {n_q} subset queries; recall against "
                                f"the exact brute force"),
                   "n_sets": w["n_sets"], "n_queries": n_q},
        "rows": rows,
        "total_s": time.perf_counter() - t_start,
        "roofline": None,
        "cpu_baseline": None,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the search runs on a single MI355X "
              "(sharding across GPUs is described in the design notes, not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_03301_amd import bvs, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bvs.lib()

    w = dict(synth.WORKLOADS[args.workload])
    if args.n_sets:
        w["n_sets"] = args.n_sets
    if args.queries:
        w["n_queries"] = args.queries
    if args.top_t:
        w["top_t"] = args.top_t
    cfg = dict(seed=0, dim=w["dim"], code_bits=w["code_bits"], fan_in=w["fan_in"], wta_k=w["wta_k"], A=3, M=1,
               top_t=w["top_t"], k=w["k"])

    if args.workload == "learned":
        print(json.dumps(learned_bench(args, w, cfg, dev)), flush=True)
        return
    if args.workload == "trends":
        print(json.dumps(trends_bench(args, w, dev)), flush=True)
        return

    log(f"generating {w['n_sets']} sets (d={w['dim']}) on the GPU")
    t0 = time.perf_counter()
    db = synth.make_database(w["n_sets"], w["size_lo"], w["size_hi"], w["dim"], w["n_topics"], seed=0, device=dev)
    if args.workload == "batched":
        q, q_off = synth.make_fresh_queries(w["n_queries"], w["max_query"], w["dim"], w["n_topics"], db_seed=0,
                                            seed=1, device=dev)
    else:
        q, q_off, _ = synth.make_subset_queries(db, w["n_queries"], seed=1)
    q = q.contiguous()
    torch.cuda.synchronize()
    n_vec = int(db.offsets[-1])
    log(f"generated {n_vec} vectors in {time.perf_counter() - t0:.1f} s; {w['n_queries']} queries "
        f"({int(q_off[-1])} vectors)")
    cpu_db = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample_sets, w["n_sets"])
        cpu_db = db.vectors[: int(db.offsets[n_s])].cpu().numpy()

    p = bvs.Params.make(dim=w["dim"], code_bits=w["code_bits"], fan_in=w["fan_in"], wta_k=w["wta_k"],
                        access_lists=3, min_count=1, top_t=w["top_t"], seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = bvs.Index(p, db.vectors, db.offsets)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"index built in {build_s:.2f} s ({ix.mem.numel() / 2**30:.1f} GiB)")
    db.vectors = None
    torch.cuda.empty_cache()

    if args.workload == "batched":
        res = batched(args, w, cfg, ix, q, q_off, n_vec, build_s, cpu_db, db.offsets)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "precision":
        res = precision(args, w, cfg, ix, q, q_off, n_vec, build_s, cpu_db, db.offsets)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "full":
        print(json.dumps(full_scan(args, w, ix, q, q_off, n_vec, build_s)), flush=True)
        return
    if args.workload == "metrics":
        print(json.dumps(metrics_bench(args, w, ix, q, q_off, n_vec, build_s)), flush=True)
        return

    n_q = w["n_queries"]
    k = w["k"]
    NQ = int(q_off[-1])
    ws = ix.search_workspace(n_q, NQ)
    out = (torch.empty(n_q, k, dtype=torch.int32, device=dev), torch.empty(n_q, k, dtype=torch.float32, device=dev),
           torch.empty(n_q, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        ix.search(q, q_off, k, ws=ws, out=out)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        ix.search(q, q_off, k, ws=ws, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t_wall
    gpu_ms = ev0.elapsed_time(ev1)
    # stage times from the same number of steps with the per-stage events on
    # (outside the timed region: the events add a little time of their own)
    bvs.profile_enable(True)
    for i in range(args.steps):
        ix.search(q, q_off, k, ws=ws, out=out)
    torch.cuda.synchronize()
    stages = bvs.profile_read()
    # work counters from one more (untimed) step: the counted work is the
    # same every step for a fixed batch
    bvs.profile_enable(False, counters=True)
    ix.search(q, q_off, k, ws=ws, out=out)
    counters = {k2: v * args.steps for k2, v in bvs.profile_counters().items()}
    bvs.profile_enable(False)
    log(f"timed {args.steps} steps: {gpu_ms:.2f} ms (wall {wall_s * 1e3:.2f} ms)")
    elapsed_s = max(wall_s, gpu_ms / 1e3)
    qps = n_q * args.steps / elapsed_s
    ids = out[0].cpu().numpy().view(np.uint32)
    concurrent = concurrent_streams(ix, q, q_off, k, args.steps, ids, args.streams) if args.streams > 1 else None

    f2v_all = f2_vectors_per_query(ix, q, q_off, db.offsets)
    f2_vectors = float(f2v_all.sum())
    f2_ids, _, f2_cnt = ix.candidates(q, q_off)
    f1_note = float(f2_cnt.float().mean().item())

    # First-layer selectivity on a few queries (diagnostic, outside the timed region).
    cnt_view, _ = ix.sketch_views()
    _, _, pos = ix.query_sketch(q[: int(q_off[16])].contiguous(), q_off[:17])
    f1_frac = float(np.mean([((cnt_view[pos[i].long()] > 0).any(0)[: w["n_sets"]]).float().mean().item()
                             for i in range(16)]))
    log(f"mean first-layer fraction {f1_frac:.4f}; F2 holds {f2_vectors / n_q:.1f} vectors per query")

    recall = brute_qps = truth = brute = None
    nb = min(args.brute_queries, n_q)
    if not args.no_brute:
        recall, brute_qps = brute_recall(ix, q, q_off, ids, k, nb)
        truth = ix.bruteforce(q[: int(q_off[nb])].contiguous(), q_off[: nb + 1], k)[0].cpu().numpy().view(np.uint32)
        log(f"brute force on {nb} queries: {brute_qps:.1f} q/s; recall@10 {recall:.4f}")
        # exact brute force: 2 m_q N dp multiply-adds per query, each as four
        # int8 matrix-core products (hi/lo split)
        qsz = np.diff(q_off[: nb + 1]).astype(np.float64)
        ops = float((2.0 * qsz * n_vec * ix.dim_padded * 4).sum())
        t_b = nb / brute_qps
        brute = {"qps": brute_qps, "queries": nb, "kernel": "k_haus_all",
                 "roofline": {"bound": "mfma", "achieved": ops / t_b / 1e12, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                              "frac": ops / t_b / 1e12 / INT8_PEAK_TOPS,
                              "algorithmic": f"{ops:.4g} int8 ops (2 m_q N dp x 4 products) over {nb} queries"}}
        if args.bf16_brute:
            brute["bf16"] = bf16_bruteforce(ix, q, q_off, k, min(args.bf16_brute, nb), truth, n_vec)
            log(f"bf16 brute force: {brute['bf16']['qps']:.1f} q/s, recall@10 {brute['bf16']['recall_at_10']:.4f}")

    per_step = {name: ms / max(1, calls) for name, (ms, calls) in stages.items() if calls}
    work = {k2: v / args.steps for k2, v in counters.items()}
    L = w["code_bits"]
    work["sketch_rows"] = sketch_rows(ix, q, q_off)
    work["f2_vectors"] = f2_vectors
    _, rerank_roof = rooflines(per_step, work, L, ix.dim_padded, "k_haus_cand", "k_haus.hip", w["n_sets"])
    # the re-rank against its algorithmic bytes: every vector of every F2
    # set, d int16 elements
    alg_bytes = f2_vectors * w["dim"] * 2
    rr_s = per_step["rerank"] / 1e3
    roof = {"bound": "hbm", "achieved": alg_bytes / rr_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg_bytes / rr_s / 1e9 / HBM_PEAK_GBS,
            "kernel": "k_haus_screen + k_haus_cand (re-rank stage)",
            "algorithmic": (f"{alg_bytes:.4g} bytes per step: the {f2_vectors:.4g} vectors of all F2 sets "
                            f"({f2_vectors / n_q:.1f} per query) x d = {w['dim']} int16 elements"),
            "post_pruning": {"bytes": rerank_roof["achieved_gbs"] * rr_s * 1e9,
                             "achieved": rerank_roof["achieved_gbs"],
                             "frac": rerank_roof["achieved_gbs"] / HBM_PEAK_GBS,
                             "note": "bytes the kernels read after abandoning and screening: vectors read in full "
                                     "x (2 dp + 4) + first-tile rows screened x (dp + 8)"},
            "traffic": traffic_from_profiles(os.path.join(ROOT, "paper_2412_03301_amd", "csrc", "k_haus.hip"),
                                             "k_haus_cand")}
    other_roofs = stage_rooflines(per_step, work, w, n_q, NQ, ix)

    sweep = None
    if args.op_sweep and truth is not None:
        sweep = operating_points(ix, q, q_off, k, truth, nb, args, w)
        ix.set_search_params(3, 1, w["top_t"])

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        ncq = min(args.cpu_sample_queries, len(q_off) - 1)
        qc = q[: int(q_off[ncq])].cpu().numpy()
        cpu = cpu_baseline(cpu_db, db.offsets, qc, q_off, cfg, w["n_sets"], args.cpu_sample_sets, ncq,
                           f2v_all[:ncq])

    if args.copy_probe_mb:
        a = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    res = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "exact int16 grid values as int8 hi/lo planes (4 int8 MFMA products, int32 accumulation)",
        "data": "synthetic",
        "config": {
            "workload": (f"{w['n_sets']} sets, sizes {w['size_lo']}-{w['size_hi']}, d={w['dim']}, "
                         f"{w['n_topics']} topics; FlyHash L={L}, s={w['fan_in']}, wta_k={w['wta_k']}; "
                         f"A=3, M=1, T={w['top_t']}; {n_q} subset queries per step; top-{k}"),
            "n_sets": w["n_sets"], "n_vectors": n_vec, "n_queries": n_q, "query_vectors": NQ,
        },
        "recall_at_10": recall,
        "recall_sample_queries": None if args.no_brute else nb,
        "bruteforce_qps": brute_qps,
        "speedup_vs_bruteforce": (qps / brute_qps) if brute_qps else None,
        "operating_point": sweep,
        "bruteforce": brute,
        "stages_ms_per_step": per_step,
        "stage_rooflines": other_roofs,
        "work_per_step": work,
        "rerank": rerank_roof,
        "mean_f2_size": f1_note,
        "mean_f2_vectors": f2_vectors / n_q,
        "mean_f1_fraction": f1_frac,
        "index_build_s": build_s,
        "concurrent": concurrent,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
