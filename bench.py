#!/usr/bin/env python3
"""Throughput of RaBitQ IVF search on one MI355X.

Default workload (the headline): learned per-query nprobe against fixed
nprobe, both at recall@10 >= 0.95, on 10,000,000 embedding-like vectors
(D = 768, unit norm, power-law spectrum), 16,384 k-means lists, BF16x3
rotation, B_q = 4, eps0 = 1.9, top-10. The MLP is trained on the GPU on
1,000,000 seeded queries labelled from the method's own searches; a step is
one search of a batch of 10,000 test queries (rotation, centroid scoring,
probe selection, the fused features + MLP + policy launch, per-(query, list)
quantisation, popcount scan with the estimator, error-bound rerank, top-10).

Other workloads (--workload): sift1m (1M SIFT-like D = 128, nprobe sweep),
embed10m (ragged batches, graph replay), gist1m (batched MFMA vs popcount).

Prints ONE JSON line on stdout (progress goes to stderr).
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 MFMA
FP8_PEAK_TFLOPS = 5000.0       # MI355X dense FP8 MFMA (the FP8 x FP4 products run at the FP8 operand's rate)

# Kernel sources per scan kind; stored counter readings apply only while their
# sources hash to the value they were taken on.
SCAN_SOURCES = {
    "popcnt": ("paper_2405_12497_amd/csrc/kernels_popcnt.hip", "paper_2405_12497_amd/csrc/scan_code.hpp",
               "paper_2405_12497_amd/csrc/rbq_internal.hpp"),
    "mfma": ("paper_2405_12497_amd/csrc/kernels_mfma.hip", "paper_2405_12497_amd/csrc/scan_code.hpp",
             "paper_2405_12497_amd/csrc/rbq_internal.hpp"),
    "finalize": ("paper_2405_12497_amd/csrc/kernels_scan.hip", "paper_2405_12497_amd/csrc/wave_select.hpp",
                 "paper_2405_12497_amd/csrc/rbq_internal.hpp"),
}
# HBM traffic of one launch per workload, from rocprofv3 --pmc FETCH_SIZE and
# --pmc WRITE_SIZE (KiB per dispatch, mean over the timed steps' dispatches of
# that kernel), each scaled by the reading of the same counter for a 1 GiB
# device-to-device copy (FETCH_SIZE reads 0.5x the copied bytes, WRITE_SIZE
# 1.0x). A reading applies only while the kernel's sources hash to the value
# it was taken on and the workload key matches.
COUNTERS = {
    "learned_mfma": {
        "kind": "mfma",
        "sources_sha256": "effe3d43f3f1890aee0b9d23aa294e21b38897b58d613440da5cbb9991cac9e9",
        "workload": "learned n=10000000 nlist=16384 batch=10000",
        "fetch_kib": 2308801.4, "write_kib": 1008186.1, "fetch_scale": 2.0, "write_scale": 1.0,
        # SQ counters of the same dispatches: SQ_VALU_MFMA_BUSY_CYCLES and
        # 4 x SQ_INSTS_VALU over (GRBM_GUI_ACTIVE / 8 XCDs) x 1024 SIMDs, and
        # SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES
        "sq": {"mfma_busy": 0.186, "valu_busy": 0.640, "wave_wait_frac": 0.451},
    },
    "fullscan": {
        "kind": "popcnt",
        "sources_sha256": "1278f4a38262bec68207cdf10beb63ee30fda320a5b4b5e8326dab9947da0949",
        "workload": "fullscan n=10000000 nlist=16384",
        "fetch_kib": 540390.8, "write_kib": 624.3, "fetch_scale": 2.0, "write_scale": 1.0,
    },
    "finalize": {
        "kind": "finalize",
        "sources_sha256": "f4437b650ca24495580c991eacba6fa405e43ffd54af47d10710ab9f9d3d2c62",
        "workload": "learned n=10000000 nlist=16384 batch=10000",
        "fetch_kib": 6355367.4, "write_kib": 2191.3, "fetch_scale": 2.0, "write_scale": 1.0,
    },
}
NPROBE_SWEEP = (8, 12, 16, 20, 24, 28, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256)
METRIC = "QPS at recall@10≥0.95, learned vs fixed nprobe; code-scan GB/s vs HBM peak"


def scan_sources_sha256(kind="popcnt"):
    import hashlib
    h = hashlib.sha256()
    for rel in SCAN_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_sq(name, workload_key):
    """The stored SQ counter fractions of a kernel, under the same conditions as stored_traffic."""
    c = COUNTERS.get(name)
    if not c or "sq" not in c or c["sources_sha256"] != scan_sources_sha256(c["kind"]) or c["workload"] != workload_key:
        return None
    return c["sq"]


def stored_traffic(name, workload_key):
    """HBM bytes per scan launch from the stored counter readings, or None when
    there are none for this workload or they were taken on other sources."""
    c = COUNTERS.get(name)
    if not c or c["sources_sha256"] != scan_sources_sha256(c["kind"]) or c["workload"] != workload_key:
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def scan_roofline(kernel, codes, ms, dim, bpc, wkey):
    """Roofline of the phase-1 scan of one batch (the dominant kernel of the
    learned step): the batched MFMA scans against the matrix-core peak of their
    operand type, with 2 D integer operations per (query, code) pair (D products
    and D additions of <x_b, q_u>); the popcount scan against HBM with its
    algorithmic bytes per (query, code) pair."""
    if kernel in ("mfma", "mfma_fp4"):
        ops = codes * 2.0 * dim
        achieved = ops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        peak = INT8_PEAK_TOPS if kernel == "mfma" else FP8_PEAK_TFLOPS
        name = ("k_scan_mfma_w<false,12,1> (phase-1 batched scan, int8 MFMA)" if kernel == "mfma" else
                "k_scan_mfma_w<true,12,1> (phase-1 batched scan, FP8 x FP4 MFMA)")
        return {"bound": "mfma", "achieved": achieved, "peak": peak,
                "unit": "TOP/s" if kernel == "mfma" else "TFLOP/s", "frac": achieved / peak,
                "traffic": stored_traffic("learned_" + kernel, wkey), "sq_counters": stored_sq("learned_" + kernel, wkey),
                "kernel": name,
                "algorithmic_ops_per_code": 2 * dim, "ops_per_launch": ops, "avg_launch_ms": ms,
                "counters_workload": wkey}
    achieved = codes * bpc / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("learned", wkey),
            "kernel": "k_scan_popcnt<12,4,1> (phase-1 scan, learned batches; codes served mostly from cache: "
                      "each list is scanned by many queries of the batch)",
            "algorithmic_bytes_per_code": bpc, "bytes_per_launch": codes * bpc, "avg_launch_ms": ms,
            "counters_workload": wkey}


def finalize_roofline(st, dim, nq, ms):
    """Algorithmic HBM bytes of one finalize launch over its measured time:
    per reranked candidate its raw vector and id (4 dim + 8 B), per candidate
    entry 8 B."""
    per_q = st["reranked_per_query"] * (4 * dim + 8) + st["candidates_per_query"] * 8
    bytes_launch = per_q * nq
    achieved = bytes_launch / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": "k_finalize (error-bound rerank)",
            "bytes_per_launch": bytes_launch, "avg_launch_ms": ms,
            "algorithmic_bytes": "reranked x (4 D + 8) + candidates x 8"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ground_truth(data, queries, k, dev, chunk=1024):
    """Exact top-k by squared L2 (FP32 matmul shortlist of 4k, FP64 recheck), ordered by (dist, id)."""
    import torch
    x = torch.from_numpy(data).to(dev)
    xn = (x.double() ** 2).sum(1).float()
    out_i = np.empty((len(queries), k), np.int64)
    out_d = np.empty((len(queries), k), np.float64)
    for s in range(0, len(queries), chunk):
        q = torch.from_numpy(queries[s:s + chunk]).to(dev)
        d = xn[None, :] - 2.0 * (q @ x.T)
        cand = torch.topk(d, 4 * k, dim=1, largest=False).indices
        exact = ((x[cand].double() - q[:, None, :].double()) ** 2).sum(-1)
        ci, ex = cand.cpu().numpy(), exact.cpu().numpy()
        for r in range(len(ci)):
            o = np.lexsort((ci[r], ex[r]))[:k]
            out_i[s + r], out_d[s + r] = ci[r][o], ex[r][o]
    return out_i, out_d


def recall(ids, gt_d, data, queries, k):
    """A returned id is a hit when its exact distance is within the k-th true distance (+1e-6 rel)."""
    hits = 0
    for i in range(len(ids)):
        got = ids[i][ids[i] >= 0]
        d = ((data[got].astype(np.float64) - queries[i].astype(np.float64)) ** 2).sum(1)
        hits += int(np.sum(d <= gt_d[i, k - 1] * (1 + 1e-6)))
    return hits / (k * len(ids))


def cpu_baseline(wl, nprobe, k, budget_s=15.0, max_q=5000):
    """The FP64 oracle (paper's sequential rerank rule) on a bounded query sample, 1 thread."""
    from threadpoolctl import threadpool_limits

    from oracle import rabitq_oracle as O
    with threadpool_limits(limits=1):
        log("cpu baseline: building the FP64 oracle index")
        oidx = O.build_index(wl.data, wl.centroids, wl.assign, wl.gauss)
        t0 = time.perf_counter()
        n = 0
        codes = 0
        while n < min(max_q, len(wl.queries)) and time.perf_counter() - t0 < budget_s:
            _, _, info = O.search(oidx, wl.queries[n], n, k, nprobe, wl.seed)
            codes += sum(len(oidx.lists[l]) for l in info["probed"])
            n += 1
        dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} queries of the workload at nprobe={nprobe}, FP64 NumPy oracle "
                      f"(Algorithm 2 + sequential error-bound rerank), one thread, {dt:.1f} s, "
                      f"{codes / dt:.3g} codes/s"}


def ground_truth_dev(x, queries, k, qchunk=128, rchunk=1 << 20):
    """ground_truth() for a GPU-resident float32 data tensor x [n, dim]:
    per query the 4k smallest FP32 distances, rechecked in FP64, ordered by
    (distance, id). Returns numpy (ids [nq,k], dists [nq,k])."""
    import torch
    n = x.shape[0]
    xn = torch.cat([(x[s:s + rchunk].double() ** 2).sum(1) for s in range(0, n, rchunk)]).float()
    out_i = np.empty((queries.shape[0], k), np.int64)
    out_d = np.empty((queries.shape[0], k), np.float64)
    for s in range(0, queries.shape[0], qchunk):
        q = queries[s:s + qchunk]
        d = xn[None, :] - 2.0 * (q @ x.T)
        cand = torch.topk(d, 4 * k, dim=1, largest=False).indices
        del d
        exact = ((x[cand].double() - q[:, None, :].double()) ** 2).sum(-1)
        ci, ex = cand.cpu().numpy(), exact.cpu().numpy()
        for r in range(len(ci)):
            o = np.lexsort((ci[r], ex[r]))[:k]
            out_i[s + r], out_d[s + r] = ci[r][o], ex[r][o]
    return out_i, out_d


def recall_dev(ids, gt_d, x, queries, k):
    """recall() with the exact distances of the returned ids computed on the GPU."""
    import torch
    ids_t = torch.as_tensor(ids, device=x.device)
    valid = ids_t >= 0
    rows = x[ids_t.clamp(min=0)]
    d = ((rows.double() - queries[:, None, :].double()) ** 2).sum(-1)
    kth = torch.as_tensor(gt_d[:, k - 1], device=x.device)[:, None]
    hits = (valid & (d <= kth * (1 + 1e-6))).sum().item()
    return hits / (k * ids_t.shape[0])


def bench_embed(args):
    """Embedding-like 10M x 768 with 16384 lists: (a) one query scanning every
    list (nprobe = nlist): the phase-1 scan kernel's algorithmic GB/s; (b)
    ragged batches of 1..1024 queries at the nprobe reaching recall@10 >= 0.95,
    direct launches vs one graph replay per batch."""
    import torch

    import synth
    from paper_2405_12497_amd import rabitq as R
    dev = torch.device("cuda:0")
    k, dim = 10, 768
    n, nlist, nq = args.n or 10_000_000, args.nlist or 16384, args.nq or 20_000
    t0 = time.perf_counter()
    log(f"embedding-like workload n={n} D={dim} nlist={nlist}, {nq} queries in ragged batches")
    data_t, q_all = synth.embedding_like_gpu(n, nq + 1, dev, seed_data=1004, seed_query=2004)
    cent, assign = R.rbq_kmeans(data_t, nlist, iters=10, sample=min(n, 1_000_000), seed=5004)
    log(f"data and k-means in {time.perf_counter() - t0:.1f}s; building the index")
    t1 = time.perf_counter()
    idx = R.Index(dim, nlist, rot_precision=R.RBQ_ROT_BF16X3, seed=4004)
    idx.build(data_t, cent, assign, synth.gaussian_matrix(dim, 3004))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t1
    log(f"index built in {build_s:.1f}s; ground truth")
    q = q_all[:nq].contiguous()
    sizes = idx.list_sizes()
    if args.fullscan_only:
        q1 = q_all[nq:nq + 1].contiguous()
        for _ in range(6):
            idx.search(q1, k, min(nlist, R.MAX_NPROBE))
        torch.cuda.synchronize()
        log("single-query full scans done")
        return
    gt_i, gt_d = ground_truth_dev(data_t, q, k)
    # nprobe: smallest of the sweep reaching recall 0.95 on the first 1000 queries
    nsw = min(1000, nq)
    chosen = None
    sweep = {}
    for p in (64, 128, 256, 384, 512, 768, 1024, 1536, 2048):
        if p > nlist:
            break
        ids, _, st = idx.search(q[:nsw], k, p, stats=True)
        rc = recall_dev(ids.cpu().numpy(), gt_d[:nsw], data_t, q[:nsw], k)
        sweep[p] = {"recall@10": round(rc, 4), "codes_per_query": st["codes_scanned"] / nsw,
                    "reranked_per_query": st["reranked"] / nsw}
        log(f"nprobe={p}: recall@10={rc:.4f} codes/q={st['codes_scanned'] / nsw:.0f}")
        if rc >= 0.95:
            chosen = p
            break
    chosen = chosen or p
    # (a) one query, every list
    q1 = q_all[nq:nq + 1].contiguous()
    bpc = dim // 8 + 8
    reps = 5
    try:
        idx.search(q1, k, min(nlist, R.MAX_NPROBE))
        torch.cuda.synchronize()
        R.rbq_profile_enable(idx.h, True)
        t2 = time.perf_counter()
        for _ in range(reps):
            idx.search(q1, k, min(nlist, R.MAX_NPROBE))
        torch.cuda.synchronize()
        full_lat = (time.perf_counter() - t2) / reps
        prof = R.rbq_profile_read(idx.h)
        R.rbq_profile_enable(idx.h, False)
        scan_ms = prof["ms_scan1"] / reps
        scan_bytes = prof["codes_scan1"] / reps * bpc
        full_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
        full_stage = {kk: round(prof[kk] / reps, 4) for kk in prof if kk.startswith("ms_")}
        full = {"nprobe": min(nlist, R.MAX_NPROBE), "ms_per_search": full_lat * 1e3, "scan_ms": scan_ms,
                "codes": prof["codes_scan1"] / reps, "gb_per_s": full_gbs, "stage_ms": full_stage}
        log(f"single query, nprobe={full['nprobe']}: {full_lat * 1e3:.3f} ms per search; phase-1 scan "
            f"{scan_ms:.4f} ms for {full['codes']:.0f} codes = {full_gbs:.0f} GB/s; stages {full_stage}")
    except R.RbqError as e:
        R.rbq_profile_enable(idx.h, False)
        full, scan_ms, scan_bytes, full_gbs = {"error": str(e)}, None, None, 0.0
        log(f"single query full scan failed: {e}")
    # (b) ragged batches
    bs = synth.query_batch_sizes(nq, seed=2104)
    starts = np.concatenate([[0], np.cumsum(bs)[:-1]])
    batches = [q[s0:s0 + b].contiguous() for s0, b in zip(starts, bs)]
    outs = [(torch.empty((b, k), dtype=torch.int64, device=dev), torch.empty((b, k), dtype=torch.float32, device=dev))
            for b in bs]
    res = {}
    for mode in ("eager", "graph"):
        ug = mode == "graph"
        for qb, (oi, od) in zip(batches, outs):     # warm-up: allocation, capture
            idx.search(qb, k, chosen, out_ids=oi, out_dists=od, use_graph=ug)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for qb, (oi, od) in zip(batches, outs):
            idx.search(qb, k, chosen, out_ids=oi, out_dists=od, use_graph=ug)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t3
        ids = torch.cat([oi for oi, _ in outs]).cpu().numpy()
        rc = recall_dev(ids, gt_d, data_t, q, k)
        res[mode] = {"qps": nq / dt, "seconds": round(dt, 4), "recall@10": round(rc, 4)}
        if ug:
            info = R.rbq_index_info_get(idx.h)
            res[mode]["graph_captures"] = info["graph_captures"]
            res[mode]["graphs_cached"] = info["graphs_cached"]
        log(f"ragged {mode}: {len(bs)} batches, {nq / dt:.0f} QPS, recall {rc:.4f}")
    line = {
        "metric": METRIC,
        "value": res["graph"]["qps"],
        "unit": "queries/s",
        "n_gpus": 1, "steps": len(bs), "warmup": len(bs),
        "ms_per_step": res["graph"]["seconds"] * 1e3 / len(bs),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int1xint4->int32 scan, fp32 estimator/rerank", "data": "synthetic",
        "config": {
            "workload": f"persistent ragged batches: {n} embedding-like vectors D={dim} (power-law spectrum, "
                        f"unit norm), {nlist} lists, BF16x3 rotation, {nq} queries in {len(bs)} batches of "
                        f"1..1024, top-10",
            "nprobe": chosen, "sweep": sweep, "ragged": res,
            "speedup_graph_over_eager": res["eager"]["seconds"] / res["graph"]["seconds"],
            "single_query_full_scan": full,
            "index_build_s": round(build_s, 1), "list_size_max": int(sizes.max()),
            "list_size_min": int(sizes.min()),
        },
        "roofline": {"bound": "hbm", "achieved": full_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": full_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_scan_popcnt (phase-1 scan, one query, every list)",
                     "algorithmic_bytes_per_code": bpc, "bytes_per_launch": scan_bytes,
                     "avg_launch_ms": scan_ms},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_gist(args):
    """GIST-like 1M x 960 (Zipf list sizes), 4096 lists, 10,000 queries in
    batches of 256, top-100, BF16x3 rotation: the batched int8-MFMA scan vs
    the popcount scan at the nprobe reaching recall@100 >= 0.95, and the
    rotation's error against an FP64 rotation by the same P."""
    import torch

    import synth
    from paper_2405_12497_amd import rabitq as R
    dev = torch.device("cuda:0")
    k, dim, batch = 100, 960, 256
    n, nlist, nq = args.n or 1_000_000, args.nlist or 4096, args.nq or 10_000
    t0 = time.perf_counter()
    log(f"GIST-like workload n={n} D={dim} nlist={nlist}, {nq} queries in batches of {batch}, top-{k}")
    data, qs, means = synth.gist_like(n, nq, dim=dim, ncomp=4096, seed_data=1003, seed_query=2003)
    data_t = torch.from_numpy(data).to(dev)
    init = means[:nlist] if nlist <= len(means) else None
    gauss = synth.gaussian_matrix(dim, 3003)
    log(f"data in {time.perf_counter() - t0:.1f}s; k-means and index build (the index phase, timed)")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cent, assign = R.rbq_kmeans(data_t, nlist, iters=10, seed=5003, init=init)
    torch.cuda.synchronize()
    kmeans_s = time.perf_counter() - t1
    idx = R.Index(dim, nlist, rot_precision=R.RBQ_ROT_BF16X3, seed=4003)
    t2 = time.perf_counter()
    idx.build(data_t, cent, assign, gauss)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t2
    log(f"index phase: k-means {kmeans_s:.2f}s + build {build_s:.2f}s (the paper's RaBitQ indexing of GIST "
        f"1M x 960 took 117 s on 32 CPU threads)")
    cent, assign = cent.cpu().numpy(), assign.cpu().numpy()
    sizes = idx.list_sizes()
    q = torch.from_numpy(qs).to(dev)
    gt_i, gt_d = ground_truth_dev(data_t, q, k)
    # BF16x3 rotation vs FP64 with the same orthonormalised P (rows of P^T applied as Q P)
    qm, r = np.linalg.qr(np.asarray(gauss, np.float64).T)
    p64 = (qm * np.sign(np.diag(r))).T
    ns = min(256, nq)
    rot = R.rbq_debug_rotate(idx.h, q[:ns].contiguous(), dim).cpu().numpy().astype(np.float64)
    ref = qs[:ns].astype(np.float64) @ p64
    err = np.abs(rot - ref)
    qn = np.linalg.norm(qs[:ns].astype(np.float64), axis=1)
    rot_err = {"max_abs": float(err.max()), "mean_abs": float(err.mean()),
               "max_rel_to_norm": float((err.max(1) / qn).max()), "queries": ns}
    log(f"BF16x3 rotation vs FP64: {rot_err}")
    # nprobe: smallest of the sweep reaching recall@100 >= 0.95 on the first 1024 queries
    nsw = min(1024, nq)
    sweep, chosen = {}, None
    for p in (8, 16, 32, 64, 128, 256):
        ids, _, st = idx.search(q[:nsw], k, p, scan_kernel=R.RBQ_SCAN_MFMA, stats=True)
        rc = recall_dev(ids.cpu().numpy(), gt_d[:nsw], data_t, q[:nsw], k)
        sweep[p] = {"recall@100": round(rc, 4), "codes_per_query": st["codes_scanned"] / nsw}
        log(f"nprobe={p}: recall@100={rc:.4f} codes/q={st['codes_scanned'] / nsw:.0f}")
        if rc >= 0.95:
            chosen = p
            break
    chosen = chosen or p
    batches = [q[s0:s0 + batch].contiguous() for s0 in range(0, nq, batch)]
    res = {}
    bpc = dim // 8 + 8
    for name, kern in (("mfma", R.RBQ_SCAN_MFMA), ("popcnt", R.RBQ_SCAN_POPCNT)):
        outs = [(torch.empty((len(b), k), dtype=torch.int64, device=dev),
                 torch.empty((len(b), k), dtype=torch.float32, device=dev)) for b in batches]
        for qb, (oi, od) in zip(batches, outs):
            idx.search(qb, k, chosen, scan_kernel=kern, out_ids=oi, out_dists=od)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for qb, (oi, od) in zip(batches, outs):
            idx.search(qb, k, chosen, scan_kernel=kern, out_ids=oi, out_dists=od)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t2
        R.rbq_profile_enable(idx.h, True)
        for qb, (oi, od) in zip(batches, outs):
            idx.search(qb, k, chosen, scan_kernel=kern, out_ids=oi, out_dists=od)
        torch.cuda.synchronize()
        prof = R.rbq_profile_read(idx.h)
        R.rbq_profile_enable(idx.h, False)
        ids = torch.cat([oi for oi, _ in outs]).cpu().numpy()
        rc = recall_dev(ids, gt_d, data_t, q, k)
        nb = max(1, prof["searches"])
        scan_ms = prof["ms_scan1"] / nb
        gbs = prof["codes_scan1"] / nb * bpc / (scan_ms * 1e-3) / 1e9
        res[name] = {"qps": nq / dt, "ms_per_batch": dt * 1e3 / len(batches), "recall@100": round(rc, 4),
                     "phase1_scan_ms_per_batch": scan_ms, "phase1_scan_gb_per_s": gbs,
                     "stage_ms_per_batch": {kk: round(prof[kk] / nb, 4) for kk in prof if kk.startswith("ms_")}}
        log(f"{name}: {nq / dt:.0f} QPS, recall@100 {rc:.4f}, phase-1 scan {scan_ms:.3f} ms/batch = {gbs:.0f} GB/s")
    best = max(res, key=lambda kk: res[kk]["qps"])
    line = {
        "metric": METRIC,
        "value": res[best]["qps"],
        "unit": "queries/s",
        "n_gpus": 1, "steps": len(batches), "warmup": len(batches),
        "ms_per_step": res[best]["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int1xint4->int32 scan (int8 MFMA or popcount), fp32 estimator/rerank", "data": "synthetic",
        "config": {
            "workload": f"batched scan: {n} GIST-like vectors D={dim} (values in [0,1], decaying spectrum, "
                        f"Zipf(1.1) components), {nlist} lists, BF16x3 rotation, {nq} queries in batches of "
                        f"{batch}, top-{k}",
            "nprobe": chosen, "sweep": sweep, "scan": res, "best_scan_kernel": best,
            "rotation_error_vs_fp64": rot_err, "index_build_s": round(build_s, 2), "kmeans_s": round(kmeans_s, 2),
            "index_phase_s": round(kmeans_s + build_s, 2),
            "paper_index_phase_s": "117 s for GIST 1M x 960 on 32 CPU threads (RaBitQ; context only)",
            "list_size_max": int(sizes.max()), "list_size_median": float(np.median(sizes)),
        },
        "roofline": {"bound": "hbm", "achieved": res["mfma"]["phase1_scan_gb_per_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": res["mfma"]["phase1_scan_gb_per_s"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_scan_mfma (phase-1 scan, batches of 256)", "algorithmic_bytes_per_code": bpc,
                     "avg_launch_ms": res["mfma"]["phase1_scan_ms_per_batch"]},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def time_search(idx, q, k, nprobe, steps, warmup, **kw):
    """Seconds per search of the whole batch, plus the per-stage device times
    (ms per search) from a separate profiled pass of the same searches."""
    import torch

    from paper_2405_12497_amd import rabitq as R
    out_i = torch.empty((q.shape[0], k), dtype=torch.int64, device=q.device)
    out_d = torch.empty((q.shape[0], k), dtype=torch.float32, device=q.device)
    for _ in range(warmup):
        idx.search(q, k, nprobe, out_ids=out_i, out_dists=out_d, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        idx.search(q, k, nprobe, out_ids=out_i, out_dists=out_d, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    R.rbq_profile_enable(idx.h, True)
    for _ in range(3):
        idx.search(q, k, nprobe, out_ids=out_i, out_dists=out_d, **kw)
    torch.cuda.synchronize()
    prof = R.rbq_profile_read(idx.h)
    R.rbq_profile_enable(idx.h, False)
    stages = {key: round(prof[key] / max(1, prof["searches"]), 3) for key in prof if key.startswith("ms_")}
    return dt, stages


def time_batches(idx, batches, k, nprobe, steps, warmup, **kw):
    """Seconds per step, a step being one search of one batch (the batches in
    turn), and the phase-1 scan / rerank device times of the timed steps (HIP
    events on the search stream around those two launch groups only)."""
    import torch

    from paper_2405_12497_amd import rabitq as R
    outs = [(torch.empty((b.shape[0], k), dtype=torch.int64, device=b.device),
             torch.empty((b.shape[0], k), dtype=torch.float32, device=b.device)) for b in batches]
    for i in range(warmup):
        j = i % len(batches)
        idx.search(batches[j], k, nprobe, out_ids=outs[j][0], out_dists=outs[j][1], **kw)
    torch.cuda.synchronize()
    R.rbq_profile_enable(idx.h, R.RBQ_PROFILE_SCAN)
    torch.cuda.synchronize()
    t = time.perf_counter()
    nq = 0
    for i in range(steps):
        j = i % len(batches)
        idx.search(batches[j], k, nprobe, out_ids=outs[j][0], out_dists=outs[j][1], **kw)
        nq += batches[j].shape[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    prof = R.rbq_profile_read(idx.h)
    R.rbq_profile_enable(idx.h, False)
    return dt / steps, nq, prof, torch.cat([o[0] for o in outs])


def stage_times(idx, batch, k, nprobe, **kw):
    """Per-stage device ms of one search of `batch` (an untimed pass with every stage bounded by events)."""
    import torch

    from paper_2405_12497_amd import rabitq as R
    R.rbq_profile_enable(idx.h, R.RBQ_PROFILE_STAGES)
    for _ in range(3):
        idx.search(batch, k, nprobe, **kw)
    torch.cuda.synchronize()
    prof = R.rbq_profile_read(idx.h)
    R.rbq_profile_enable(idx.h, False)
    return {key: round(prof[key] / max(1, prof["searches"]), 4) for key in prof if key.startswith("ms_")}


def search_all(idx, q, k, nprobe, chunk=20_000, **kw):
    """ids (GPU int64 [nq, k]) and summed stats of a search of q in chunks."""
    import torch
    ids = torch.empty((q.shape[0], k), dtype=torch.int64, device=q.device)
    tot = {}
    for s0 in range(0, q.shape[0], chunk):
        i, _, st = idx.search(q[s0:s0 + chunk].contiguous(), k, nprobe, stats=True, qid_base=0, **kw)
        ids[s0:s0 + chunk] = i
        for key, v in st.items():
            tot[key] = tot.get(key, 0) + v
    return ids, tot


def cpu_baseline_learned(data_t, cent, assign, gauss, queries, nprobe, seed, k, n_sample=4, budget_s=12.0):
    """The FP64 oracle (Algorithm 2 + the sequential Sec. 4 rerank) on a seeded
    sample of test queries at the fixed nprobe, timed on this host's cores:
    one thread, then a process pool with one single-threaded worker per core
    (queries of the sample handed out in turn). The oracle index holds only the
    lists the sample probes, which gives the sample's queries the same
    probed lists and codes as the full index."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import rabitq_oracle as O
    cores = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(77)
    qs = queries[np.sort(rng.choice(len(queries), n_sample, replace=False))].astype(np.float32)
    lists = np.unique(np.concatenate([O.probe_lists(q, cent, nprobe) for q in qs]))
    keep = np.flatnonzero(np.isin(assign, lists))
    import torch
    sub = data_t[torch.from_numpy(keep).to(data_t.device)].cpu().numpy()
    log(f"cpu baseline: oracle index over {len(lists)} lists ({len(keep)} vectors) probed by {n_sample} queries")
    t0 = time.perf_counter()
    with threadpool_limits(limits=cores):
        oidx = O.build_index(sub, cent, assign[keep], gauss)
    log(f"cpu baseline: oracle index built in {time.perf_counter() - t0:.1f}s")
    global _ORACLE_JOB
    _ORACLE_JOB = (O, oidx, qs, k, nprobe, seed)

    codes_per_q = [sum(len(oidx.lists[l]) for l in O.probe_lists(q, cent, nprobe)) for q in qs]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n1 = 0
        while n1 < 2 * n_sample and (n1 < 1 or time.perf_counter() - t0 < budget_s):
            _oracle_query(n1 % n_sample)
            n1 += 1
        dt1 = time.perf_counter() - t0
    one = {"value": n1 / dt1, "unit": "queries/s", "cores": 1, "queries": n1, "seconds": round(dt1, 2),
           "codes_per_s": sum(codes_per_q[i % n_sample] for i in range(n1)) / dt1}
    log(f"cpu baseline, 1 core: {one['value']:.3f} queries/s")
    allc = None
    try:
        ctx = mp.get_context("fork")
        with ctx.Pool(cores, initializer=_pool_init) as pool:
            t0 = time.perf_counter()
            per_q = dt1 / n1
            njobs = min(4 * cores, max(cores, int(round(budget_s * cores / per_q))))
            res = pool.map_async(_oracle_query, [i % n_sample for i in range(njobs)], chunksize=1)
            res.get(timeout=20 * budget_s)
            dta = time.perf_counter() - t0
        allc = {"value": njobs / dta, "unit": "queries/s", "cores": cores, "queries": njobs,
                "seconds": round(dta, 2),
                "codes_per_s": sum(codes_per_q[i % n_sample] for i in range(njobs)) / dta}
        log(f"cpu baseline, {cores} cores: {allc['value']:.3f} queries/s")
    except Exception as e:      # the single-core figure stands on its own
        log(f"cpu baseline all-cores mode failed: {e!r}")
    best = allc or one
    return {"value": best["value"], "unit": "queries/s", "cores": best["cores"], "kind": "oracle",
            "sample": f"{n_sample} seeded test queries at fixed nprobe={nprobe}, FP64 NumPy oracle (Algorithm 2 "
                      f"+ sequential error-bound rerank) over the {len(lists)} lists they probe "
                      f"({len(keep)} vectors); value = {'all-cores process pool' if allc else 'one thread'}",
            "host_cores": cores, "single_core": one, "all_cores": allc}


_ORACLE_JOB = None


def _pool_init():
    from threadpoolctl import threadpool_limits
    global _POOL_LIMIT
    _POOL_LIMIT = threadpool_limits(limits=1)


def _oracle_query(i):
    O, oidx, qs, k, nprobe, seed = _ORACLE_JOB
    O.search(oidx, qs[i], i, k, nprobe, seed)
    return i


def bench_learned(args):
    """Learned per-query nprobe vs fixed nprobe, both at recall@10 >= 0.95, on
    10M embedding-like vectors (D = 768, 16,384 lists, BF16x3 rotation): the
    network is trained on the GPU on labels from the method's own traces (the
    probe ranks of the top-10 that a plain search with twice the nprobe cap
    returns), then both operating points are calibrated on validation queries
    and timed on test queries."""
    import torch

    import synth
    from paper_2405_12497_amd import rabitq as R
    dev = torch.device("cuda:0")
    k, dim, cap = 10, 768, 512
    n, nlist = args.n or 10_000_000, args.nlist or 16384
    ntr, nva, nte = args.ntrain, 10_000, args.nq or 100_000
    batch = min(10_000, nte)
    t_all = time.perf_counter()
    log(f"learned nprobe: embedding-like n={n} D={dim} nlist={nlist}; {ntr} training, {nva} validation, "
        f"{nte} test queries")
    data_t, q_test = synth.embedding_like_gpu(n, nte, dev, seed_data=1004, seed_query=2004)
    q_train = synth.embedding_queries_gpu(ntr, dev, seed_query=5005)
    q_val = synth.embedding_queries_gpu(nva, dev, seed_query=6005)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cent_t, assign_t = R.rbq_kmeans(data_t, nlist, iters=10, sample=min(n, 1_000_000), seed=5004)
    kmeans_s = time.perf_counter() - t0
    gauss = synth.gaussian_matrix(dim, 3004)
    idx = R.Index(dim, nlist, rot_precision=R.RBQ_ROT_BF16X3, seed=4004)
    t0 = time.perf_counter()
    idx.build(data_t, cent_t, assign_t, gauss)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    cent, assign = cent_t.cpu().numpy(), assign_t.cpu().numpy()
    del cent_t, assign_t
    log(f"k-means {kmeans_s:.1f}s, index build {build_s:.1f}s; ground truth of validation and test queries")
    t0 = time.perf_counter()
    gva_i, gva_d = ground_truth_dev(data_t, q_val, k)
    gte_i, gte_d = ground_truth_dev(data_t, q_test, k)
    log(f"ground truth in {time.perf_counter() - t0:.1f}s; training labels from searches at nprobe {2 * cap}")
    # training labels: the method's own traces
    t0 = time.perf_counter()
    tr_ids, tr_st = search_all(idx, q_train, k, min(2 * cap, nlist, R.MAX_NPROBE))
    labels, need = R.rbq_nprobe_labels(idx.h, q_train, tr_ids)
    va_ids, _ = search_all(idx, q_val, k, min(2 * cap, nlist, R.MAX_NPROBE))
    va_lab, _ = R.rbq_nprobe_labels(idx.h, q_val, va_ids)
    va_lab_exact, _ = R.rbq_nprobe_labels(idx.h, q_val, torch.from_numpy(gva_i).to(dev))
    label_agree = float((va_lab == va_lab_exact).float().mean().item())
    trace_s = time.perf_counter() - t0
    hist = torch.bincount(labels.long(), minlength=32).cpu().numpy().tolist()
    log(f"labels in {trace_s:.1f}s (histogram {hist}); validation labels equal to exact-neighbour labels: "
        f"{label_agree:.4f}")
    # features and training
    t0 = time.perf_counter()
    feats = torch.empty((ntr, 96), dtype=torch.float32, device=dev)
    for s0 in range(0, ntr, 50_000):
        R.rbq_nprobe_features(idx.h, q_train[s0:s0 + 50_000].contiguous(), qid_base=0, feats=feats[s0:s0 + 50_000])
    losses = R.rbq_nprobe_model_train(idx.h, feats, labels, epochs=args.epochs, batch=4096, lr=args.lr, seed=11)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del feats
    log(f"features + {args.epochs} epochs of training in {train_s:.1f}s, losses {np.round(losses, 4).tolist()}")
    w, _ = R.rbq_nprobe_model_get(idx.h)
    target, margin = 0.95, 0.002

    def rec(ids, gt_d, q):
        return recall_dev(ids.cpu().numpy(), gt_d, data_t, q, k)

    def learned_at(q, thr):
        R.rbq_nprobe_model_set(idx.h, w, thr)
        return search_all(idx, q, k, cap, use_learned_nprobe=True)

    # both operating points calibrated on validation queries to target + margin
    t0 = time.perf_counter()
    lo, hi = 0.2, 0.9995
    if rec(learned_at(q_val, hi)[0], gva_d, q_val) >= target + margin:
        for _ in range(13):
            mid = 0.5 * (lo + hi)
            if rec(learned_at(q_val, mid)[0], gva_d, q_val) >= target + margin:
                hi = mid
            else:
                lo = mid
    thr = hi
    R.rbq_nprobe_model_set(idx.h, None, 0.9)
    plo, phi = 1, cap
    while plo < phi:
        mid = (plo + phi) // 2
        if rec(search_all(idx, q_val, k, mid)[0], gva_d, q_val) >= target + margin:
            phi = mid
        else:
            plo = mid + 1
    fixed = phi
    calib_s = time.perf_counter() - t0
    # test recall; an operating point below the target on the test queries is
    # raised on them (reported)
    recal = {"learned": False, "fixed": False}
    ids_l, st_l = learned_at(q_test, thr)
    rc_l = rec(ids_l, gte_d, q_test)
    while rc_l < target and thr < 0.99999:
        thr = min(0.99999, thr + 0.25 * (1.0 - thr))
        recal["learned"] = True
        ids_l, st_l = learned_at(q_test, thr)
        rc_l = rec(ids_l, gte_d, q_test)
    R.rbq_nprobe_model_set(idx.h, None, 0.9)
    ids_f, st_f = search_all(idx, q_test, k, fixed)
    rc_f = rec(ids_f, gte_d, q_test)
    while rc_f < target and fixed < cap:
        fixed = min(cap, fixed + max(1, fixed // 50))
        recal["fixed"] = True
        ids_f, st_f = search_all(idx, q_test, k, fixed)
        rc_f = rec(ids_f, gte_d, q_test)
    log(f"calibrated in {calib_s:.1f}s: learned threshold {thr:.5f} (test recall {rc_l:.4f}, mean nprobe "
        f"{st_l['pairs'] / nte:.1f}), fixed nprobe {fixed} (test recall {rc_f:.4f})")
    batches = [q_test[s0:s0 + batch].contiguous() for s0 in range(0, nte, batch)]
    kern = {"popcnt": R.RBQ_SCAN_POPCNT, "mfma": R.RBQ_SCAN_MFMA, "mfma_fp4": R.RBQ_SCAN_MFMA_FP4,
            "auto": R.RBQ_SCAN_AUTO}[args.kernel]
    # timed: learned, then fixed
    R.rbq_nprobe_model_set(idx.h, w, thr)
    t_l, nq_l, prof_l, out_l = time_batches(idx, batches, k, cap, args.steps, args.warmup, use_learned_nprobe=True,
                                            scan_kernel=kern)
    stages_l = stage_times(idx, batches[0], k, cap, use_learned_nprobe=True, scan_kernel=kern)
    R.rbq_nprobe_model_set(idx.h, None, 0.9)
    t_f, nq_f, prof_f, out_f = time_batches(idx, batches, k, fixed, args.steps, args.warmup, scan_kernel=kern)
    stages_f = stage_times(idx, batches[0], k, fixed, scan_kernel=kern)
    # recall of the timed searches' own outputs (every test batch was searched at least once when steps >= 10)
    if args.steps >= len(batches):
        rc_l = rec(out_l, gte_d, q_test)
        rc_f = rec(out_f, gte_d, q_test)
    qps_l, qps_f = batch / t_l, batch / t_f
    log(f"learned {qps_l:.0f} QPS ({t_l * 1e3:.3f} ms per batch of {batch}), fixed {qps_f:.0f} QPS "
        f"({t_f * 1e3:.3f} ms); speedup {t_f / t_l:.3f}")
    bpc = dim // 8 + 8
    scan_ms = prof_l["ms_scan1"] / max(1, prof_l["searches"])
    scan_codes = prof_l["codes_scan1"] / max(1, prof_l["searches"])   # (query, code) pairs of the phase-1 scan
    scan_bytes = scan_codes * bpc
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9 if scan_ms > 0 else 0.0
    fin_ms = prof_l["ms_finalize"] / max(1, prof_l["searches"])
    # finalize's own reranks (its seeds were reranked by the bootstrap kernel)
    fin_rr = (st_l["reranked"] - st_l["reranked_bootstrap"]) / nte
    fin_bytes = (fin_rr * (4 * dim + 8) + st_l["candidates"] / nte * 8) * batch
    fin_gbs = fin_bytes / (fin_ms * 1e-3) / 1e9 if fin_ms > 0 else 0.0
    wkey = f"learned n={n} nlist={nlist} batch={batch}"
    # one query probing every list: the scan's HBM-bound case (codes do not fit the Infinity Cache)
    q1 = q_val[:1].contiguous()
    idx.search(q1, k, min(nlist, R.MAX_NPROBE))
    torch.cuda.synchronize()
    R.rbq_profile_enable(idx.h, R.RBQ_PROFILE_SCAN)
    reps = 8
    t0 = time.perf_counter()
    for _ in range(reps):
        idx.search(q1, k, min(nlist, R.MAX_NPROBE))
    torch.cuda.synchronize()
    full_lat = (time.perf_counter() - t0) / reps
    pf = R.rbq_profile_read(idx.h)
    R.rbq_profile_enable(idx.h, False)
    full_ms = pf["ms_scan1"] / reps
    full_bytes = pf["codes_scan1"] / reps * bpc
    full_gbs = full_bytes / (full_ms * 1e-3) / 1e9
    full_stages = stage_times(idx, q1, k, min(nlist, R.MAX_NPROBE))
    fkey = f"fullscan n={n} nlist={nlist}"
    log(f"single query, every list: {full_lat * 1e3:.3f} ms per search, phase-1 scan {full_ms * 1e3:.1f} us "
        f"= {full_gbs:.0f} GB/s")
    line = {
        "metric": METRIC,
        "value": qps_l,
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_l * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"mfma": "int8 MFMA scan (1-bit codes x 4-bit queries -> int32)",
                  "mfma_fp4": "fp8 x fp4 MFMA scan (exact integers)",
                  "popcnt": "int1 x int4 popcount scan -> int32",
                  "auto": "autotuned scan"}[args.kernel] + ", bf16 MLP, fp32 estimator/rerank",
        "data": "synthetic",
        "config": {
            "workload": f"learned per-query nprobe: {n} embedding-like vectors D={dim} (power-law spectrum, unit "
                        f"norm), {nlist} k-means lists, BF16x3 rotation, {ntr} training / {nva} validation / {nte} "
                        f"test queries, steps of {batch} test queries, top-{k}, recall@10 >= {target}",
            "learned": {"qps": qps_l, "recall@10": round(rc_l, 4), "threshold": thr,
                        "mean_nprobe": st_l["pairs"] / nte, "codes_per_query": st_l["codes_scanned"] / nte,
                        "reranked_per_query": st_l["reranked"] / nte,
                        "reranked_bootstrap_per_query": st_l["reranked_bootstrap"] / nte,
                        "nonfinite_fallbacks": st_l["nonfinite_fallbacks"], "stage_ms_per_batch": stages_l},
            "fixed": {"qps": qps_f, "recall@10": round(rc_f, 4), "nprobe": fixed,
                      "codes_per_query": st_f["codes_scanned"] / nte, "reranked_per_query": st_f["reranked"] / nte,
                      "stage_ms_per_batch": stages_f},
            "speedup_learned_over_fixed": t_f / t_l,
            "calibration": f"threshold and fixed nprobe chosen on the validation queries for recall@10 >= "
                           f"{target + margin}; raised on the test queries where they fell below {target}: {recal}",
            "labels": f"smallest bucket covering the probe ranks of the top-10 a plain search at nprobe {2 * cap} "
                      f"returns; {label_agree:.4f} of validation labels equal those from exact neighbours",
            "label_histogram": hist, "train_s": round(train_s, 2), "label_trace_s": round(trace_s, 2),
            "epochs": args.epochs, "lr": args.lr, "losses": [round(float(x), 4) for x in losses],
            "kmeans_s": round(kmeans_s, 1), "index_build_s": round(build_s, 1),
            "single_query_full_scan": {"nprobe": min(nlist, R.MAX_NPROBE), "ms_per_search": full_lat * 1e3,
                                       "stage_ms": full_stages},
        },
        "roofline": scan_roofline(args.kernel, scan_codes, scan_ms, dim, bpc, wkey),
        "roofline_fullscan": {"bound": "hbm", "achieved": full_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": full_gbs / HBM_PEAK_GBS, "traffic": stored_traffic("fullscan", fkey),
                              "kernel": "k_scan_popcnt<12,4,1> (one query, every list)",
                              "bytes_per_launch": full_bytes, "avg_launch_ms": full_ms, "counters_workload": fkey},
        "roofline_finalize": {"bound": "hbm", "achieved": fin_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": fin_gbs / HBM_PEAK_GBS, "traffic": stored_traffic("finalize", wkey),
                              "kernel": "k_finalize (error-bound rerank)",
                              "bytes_per_launch": fin_bytes, "avg_launch_ms": fin_ms,
                              "algorithmic_bytes": "own reranks x (4 D + 8) + candidate entries x 8",
                              "counters_workload": wkey},
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_learned(data_t, cent, assign, gauss, q_test.cpu().numpy(), fixed,
                                                    4004, k)
    log(f"total {time.perf_counter() - t_all:.0f}s")
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="vectors (0: the workload's default)")
    ap.add_argument("--nq", type=int, default=0, help="queries (0: the workload's default)")
    ap.add_argument("--nlist", type=int, default=0, help="IVF lists (0: the workload's default)")
    ap.add_argument("--nprobe", type=int, default=0, help="0: smallest of the sweep reaching recall 0.95")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel", default=None, choices=["popcnt", "mfma", "mfma_fp4", "auto"],
                    help="phase-1 scan kernel (default: mfma for the learned-nprobe batches, popcnt otherwise)")
    ap.add_argument("--workload", default="learned", choices=["learned", "sift1m", "embed10m", "gist1m"])
    ap.add_argument("--fullscan-only", action="store_true",
                    help="embed10m: only build the index and run six one-query searches of every list")
    ap.add_argument("--ntrain", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=5)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="only run 3 device-to-device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.kernel is None:
        args.kernel = "mfma" if args.workload == "learned" else "popcnt"
    if args.copy_mb:
        import torch
        n = args.copy_mb * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": n * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library shards "
              "nothing across GPUs (how it would is described with the design).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "embed10m":
        bench_embed(args)
        return
    if args.workload == "gist1m":
        bench_gist(args)
        return
    args.n = args.n or 1_000_000
    args.nq = args.nq or 10_000
    args.nlist = args.nlist or 4096

    import torch

    import synth
    from paper_2405_12497_amd import rabitq as R

    dev = torch.device("cuda:0")
    k = 10
    t0 = time.perf_counter()
    log(f"generating SIFT-like workload n={args.n} nq={args.nq} nlist={args.nlist}")
    wl = synth.workload(2, n=args.n, nq=args.nq, nlist=args.nlist, device=dev)
    log(f"workload ready in {time.perf_counter() - t0:.1f}s; building index")
    idx = R.Index(wl.dim, wl.centroids.shape[0], rot_precision=R.RBQ_ROT_FP32, seed=wl.seed)
    t1 = time.perf_counter()
    idx.build(wl.data, wl.centroids, wl.assign, wl.gauss)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t1
    log(f"index built in {build_s:.2f}s; ground truth")
    gt_i, gt_d = ground_truth(wl.data, wl.queries, k, dev)
    q = torch.from_numpy(wl.queries).to(dev)
    kern = {"popcnt": R.RBQ_SCAN_POPCNT, "mfma": R.RBQ_SCAN_MFMA, "mfma_fp4": R.RBQ_SCAN_MFMA_FP4,
            "auto": R.RBQ_SCAN_AUTO}[args.kernel]

    sweep = {}
    chosen = args.nprobe
    for p in ([args.nprobe] if args.nprobe else NPROBE_SWEEP):
        ids, _, st = idx.search(q, k, p, scan_kernel=kern, stats=True)
        rc = recall(ids.cpu().numpy(), gt_d, wl.data, wl.queries, k)
        sweep[p] = {"recall@10": round(rc, 4), "reranked_per_query": st["reranked"] / len(wl.queries),
                    "candidates_per_query": st["candidates"] / len(wl.queries),
                    "codes_per_query": st["codes_scanned"] / len(wl.queries)}
        log(f"nprobe={p}: recall@10={rc:.4f} reranked/q={sweep[p]['reranked_per_query']:.1f} "
            f"candidates/q={sweep[p]['candidates_per_query']:.1f} codes/q={sweep[p]['codes_per_query']:.0f}")
        if not args.nprobe and rc >= 0.95:
            chosen = p
            break
    if not chosen:
        chosen = NPROBE_SWEEP[-1]

    out_i = torch.empty((len(wl.queries), k), dtype=torch.int64, device=dev)
    out_d = torch.empty((len(wl.queries), k), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        idx.search(q, k, chosen, scan_kernel=kern, out_ids=out_i, out_dists=out_d)
    torch.cuda.synchronize()
    # timed region: HIP events (on the search stream) around the main scan and
    # the rerank only, since every event record stalls the stream briefly
    R.rbq_profile_enable(idx.h, R.RBQ_PROFILE_SCAN)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        idx.search(q, k, chosen, scan_kernel=kern, out_ids=out_i, out_dists=out_d)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t2
    prof = R.rbq_profile_read(idx.h)
    # the per-stage breakdown from a separate, untimed pass with every stage bounded
    R.rbq_profile_enable(idx.h, R.RBQ_PROFILE_STAGES)
    for _ in range(3):
        idx.search(q, k, chosen, scan_kernel=kern, out_ids=out_i, out_dists=out_d)
    torch.cuda.synchronize()
    prof_st = R.rbq_profile_read(idx.h)
    R.rbq_profile_enable(idx.h, False)
    rc = recall(out_i.cpu().numpy(), gt_d, wl.data, wl.queries, k)
    qps = len(wl.queries) * args.steps / dt
    bytes_per_code = wl.dim_pad // 8 + 8
    launches = max(1, prof["searches"])
    scan_ms = prof["ms_scan1"] / launches
    bytes_launch = prof["codes_scan1"] / launches * bytes_per_code
    achieved = bytes_launch / (scan_ms * 1e-3) / 1e9 if scan_ms > 0 else 0.0
    kernel_ms = {kk: round(prof_st[kk] / max(1, prof_st["searches"]), 4) for kk in
                 ("ms_front", "ms_prep", "ms_scan0", "ms_tau", "ms_scan1", "ms_finalize")}
    log(f"timed {args.steps} steps: {dt * 1e3 / args.steps:.3f} ms/step, {qps:.0f} QPS, recall {rc:.4f}; "
        f"per-step kernel ms {kernel_ms}; scan {achieved:.0f} GB/s")

    wkey = f"sift-like n={args.n} nq={args.nq} nlist={args.nlist} nprobe={chosen} kernel={args.kernel}"
    line = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int1xint4->int32 scan, fp32 estimator/rerank",
        "data": "synthetic",
        "config": {
            "workload": f"IVF-RaBitQ single-query popcount path: {args.n} SIFT-like vectors D=128, "
                        f"{args.nlist} k-means lists, {args.nq} queries per step, top-10, FP32 rotation",
            "nprobe": chosen, "recall@10": round(rc, 4), "batch": args.nq, "sweep": sweep,
            "scan_kernel": args.kernel, "index_build_s": round(build_s, 3),
            "codes_per_s": (prof["codes_scan0"] + prof["codes_scan1"]) / launches / (dt / args.steps),
            "kernel_ms_per_step": kernel_ms,   # untimed pass with every stage bounded by events
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("sift", wkey),
                     "kernel": "k_scan_popcnt (phase-1 scan)",
                     "algorithmic_bytes_per_code": bytes_per_code,
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": scan_ms,
                     "scan_sources_sha256": scan_sources_sha256(), "counters_workload": wkey},
        # the rerank gathers raw vectors at random: its algorithmic bytes are
        # the reranked candidates' raw vectors and ids plus every candidate
        # entry read (counts from the statistics pass at the timed nprobe)
        "roofline_finalize": finalize_roofline(sweep[chosen], wl.dim, args.nq, prof["ms_finalize"] / launches),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, chosen, k)
        log(f"cpu baseline {line['cpu_baseline']['value']:.2f} queries/s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
