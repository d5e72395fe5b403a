"""Benchmark of batched Seismic query processing on one MI355X.

A step is one seismic_search_batch call over one batch of synthetic queries
(all hot-path steps: query cut, summary scoring, block ordering, pruned block
evaluation, top-k).  The workload defaults to the 8.8M-document index
(lambda 6000, beta 400, gamma 0.4) with 7000-query batches of uniform [5, 200]
nonzeros, query_cut 10, k 10.

Prints one JSON line.  value = queries per second over the timed steps at
the fastest swept heap_factor whose Recall@10 (against GPU exact top-k) is at
least the target; the inputs are resident in HBM before timing starts.
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

# heap_factor sweep, most pruning first (Algorithm 2 skip rule r * hf < heap.min):
# the first point reaching the recall target is the fastest one that does.
HF_SWEEP = (0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.25, 1.5, 2.0)

WORKLOADS = {
    # name: docs, queries, query law, lambda, beta, gamma, cut, heap factors swept
    # k100: the (query_cut, heap_factor) reaching Recall@100 0.95 on this
    # workload (found by the operating-point search with --k 100), timed as a
    # fixed point beside the k = 10 sweep
    "msmarco-8.8M": dict(n_docs=8_841_823, n_queries=7000, qlaw="uniform", lam=6000, beta=400, gamma=0.4,
                         cut=10, hfs=HF_SWEEP, k100=(20, 1.125)),
    "1M": dict(n_docs=1_000_000, n_queries=10_000, qlaw="poisson", lam=3000, beta=150, gamma=0.4,
               cut=10, hfs=HF_SWEEP),
    "100k": dict(n_docs=100_000, n_queries=1000, qlaw="poisson", lam=1000, beta=50, gamma=0.4,
                 cut=10, hfs=HF_SWEEP),
    # the scale study's collection shape (138M passages, 127 / 44 nonzeros per
    # document / query, lambda 6e4), generated straight into HBM and indexed
    # there: it does not fit the host's memory alongside its index
    "msmarco-v2-138M": dict(n_docs=138_000_000, n_queries=3903, qlaw="poisson", qmean=44.0, dmean=127.0,
                            lam=60000, beta=400, gamma=0.4, cut=10, hfs=(0.1, 0.15, 0.2) + HF_SWEEP,
                            device_build=True, hot_hf=0.3),
}

PEAK_HBM_GBS = 8000.0

# Sources of the search kernel: a traffic figure taken from rocprofv3 counters
# is reported only while these files are unchanged since the counters were read.
KERNEL_SOURCES = ("paper_2509_24815_amd/csrc/search.hip", "paper_2509_24815_amd/csrc/device_common.h",
                  "paper_2509_24815_amd/csrc/search_kernels.h")


def kernel_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, cut: int, hf: float, k: int):
    """HBM-side bytes per launch from a committed rocprofv3 summary of this
    workload and operating point (profiles/k_search_<workload>_*traffic.md:
    request-size-resolved read and write counters), or None when there is
    none or the kernel has changed since it was taken."""
    import glob
    want = f"{workload} query_cut {cut} heap_factor {hf} k {k}"
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"k_search_{workload}_*traffic.md"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith((" ", "|", "#")):
                    key, val = line.split(":", 1)
                    kv[key.strip()] = val.strip()
        try:
            if kv.get("workload") == want and kv.get("source_sha256") == kernel_sha():
                return float(kv["traffic_bytes_per_launch"].split()[0])
        except (KeyError, ValueError):
            continue
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def alg_bytes(counters: np.ndarray, q_nnz: np.ndarray, k: int) -> np.ndarray:
    """Algorithmic HBM bytes per query of one search (layout of the library):
    query row 8 + 4 n_q; per visited list 8 (list offsets); per block of a
    visited list 16 (summary offset, m, delta) + 3 per summary entry (u16
    term + u8 code); per evaluated block 8 (posting offsets) + per document
    4 (posting) + 16 (row offsets) + 4 per nonzero; results 8 k."""
    c = counters.astype(np.float64)
    return (8 + 4 * q_nnz + 8 * c[:, 7] + 16 * c[:, 1] + 3 * c[:, 0] + 8 * c[:, 2] + 20 * c[:, 3]
            + 4 * c[:, 4] + 8 * k)


def scope_bytes(counters: np.ndarray, q_nnz: np.ndarray, k: int, distinct_docs=None, distinct_nnz=None) -> np.ndarray:
    """Algorithmic bytes per query by the hot-path scope's formula: 4 n_q
    (query) + per block of a visited list 3 per summary entry + 20 (header)
    + 4 per posting of an evaluated block + per distinct scored document 8
    (row offset) + 4 per nonzero + 8 k (results).  distinct_docs /
    distinct_nnz [nq]: the distinct documents of each query's evaluated
    blocks and their nonzeros; without them every document of an evaluated
    block is counted (an upper bound)."""
    c = counters.astype(np.float64)
    d = c[:, 3] if distinct_docs is None else np.asarray(distinct_docs, np.float64)
    z = c[:, 4] if distinct_nnz is None else np.asarray(distinct_nnz, np.float64)
    return 4 * q_nnz + 3 * c[:, 0] + 20 * c[:, 1] + 4 * c[:, 3] + 8 * d + 4 * z + 8 * k


def evaluated_blocks(S: dict, qs, list_term: np.ndarray, prefix: np.ndarray):
    """(query, block) pairs a batch evaluated, recovered from its trace: the
    i-th visited list of query q evaluated the first prefix[q, i] blocks in
    the order of Algorithm 2 (summary score desc, block asc); the scores are
    recomputed from the index exactly (fp64 sums of fp16 x grid values,
    rounded to fp32)."""
    import scipy.sparse as sp
    nq = qs.n_rows
    lo = S["list_off"].astype(np.int64)
    so = S["blk_sum_off"].astype(np.int64)
    terms = list_term.astype(np.int64)
    valid = list_term != 0xFFFFFFFF
    Q = sp.csr_matrix((qs.values().astype(np.float64), qs.terms(), qs.row_ptr.astype(np.int64)),
                      shape=(nq, qs.dim))
    qi, ci = np.nonzero(valid & (prefix > 0))
    order = np.argsort(terms[qi, ci], kind="stable")
    qi, ci = qi[order], ci[order]
    ts = terms[qi, ci]
    starts = np.concatenate([[0], np.flatnonzero(np.diff(ts)) + 1, [len(ts)]])
    out_q, out_b = [], []
    for g0, g1 in zip(starts[:-1], starts[1:]):
        if g1 <= g0:
            continue
        t = int(ts[g0])
        b0, b1 = int(lo[t]), int(lo[t + 1])
        nb = b1 - b0
        lens = np.diff(so[b0:b1 + 1])
        row = np.repeat(np.arange(nb), lens)
        s0, s1 = int(so[b0]), int(so[b1])
        vals = (S["blk_m"][b0 + row].astype(np.float64)
                + S["sum_code"][s0:s1].astype(np.float64) * S["blk_delta"][b0 + row].astype(np.float64))
        M = sp.csr_matrix((vals, S["sum_term"][s0:s1].astype(np.int64), np.concatenate([[0], np.cumsum(lens)])),
                          shape=(nb, qs.dim))
        R = (M @ Q[qi[g0:g1]].T).toarray().astype(np.float32)
        ordr = np.argsort(-R, axis=0, kind="stable")  # score desc, block asc on ties
        p = prefix[qi[g0:g1], ci[g0:g1]].astype(np.int64)
        take = np.arange(nb)[:, None] < p[None, :]
        blocks = b0 + ordr  # [nb, group]
        cols = np.broadcast_to(qi[g0:g1][None, :], blocks.shape)
        out_b.append(blocks[take])
        out_q.append(cols[take])
    if not out_q:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(out_q).astype(np.int64), np.concatenate(out_b).astype(np.int64)


def trace_bytes(S: dict, qs, list_term: np.ndarray, prefix: np.ndarray, k: int):
    """(compulsory bytes of the batch, distinct documents [nq], their
    nonzeros [nq]).  Compulsory: what the batch must read at least once,
    however many of its queries share it -- the queries and results, every
    summary entry and block header of each distinct visited list, and each
    distinct evaluated block's posting offsets, postings, row offsets and
    rows (layout of the library)."""
    nq = qs.n_rows
    q_nnz = np.diff(qs.row_ptr.astype(np.int64))
    lo = S["list_off"].astype(np.int64)
    so = S["blk_sum_off"].astype(np.int64)
    po = S["blk_post_off"].astype(np.int64)
    doc_len = np.diff(S["row_ptr"].astype(np.int64))
    valid = list_term != 0xFFFFFFFF
    ut = np.unique(list_term[valid].astype(np.int64))
    total = float((8 + 4 * q_nnz).sum() + 8 * k * nq)
    total += float((8 + 16 * (lo[ut + 1] - lo[ut]) + 3 * (so[lo[ut + 1]] - so[lo[ut]])).sum())
    pq, pb = evaluated_blocks(S, qs, list_term, prefix)
    eb = np.unique(pb)
    n_docs = po[eb + 1] - po[eb]
    first = np.repeat(po[eb] - np.concatenate([[0], np.cumsum(n_docs)[:-1]]), n_docs)
    posts = S["postings"][np.arange(int(n_docs.sum())) + first]
    total += float(8 * len(eb) + 20 * n_docs.sum() + 4 * doc_len[posts].sum())
    # per query: the distinct documents of its evaluated blocks
    cnt = po[pb + 1] - po[pb]
    firsts = np.repeat(po[pb] - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
    docs = S["postings"][np.arange(int(cnt.sum())) + firsts].astype(np.int64)
    owner = np.repeat(pq, cnt)
    key = np.unique(owner * int(S["n_docs"]) + docs)
    kq, kd = key // int(S["n_docs"]), key % int(S["n_docs"])
    distinct = np.bincount(kq, minlength=nq)
    distinct_nnz = np.bincount(kq, weights=doc_len[kd].astype(np.float64), minlength=nq)
    return total, distinct, distinct_nnz


def device_collection(torch, synth, n_docs, mean, chunk=2_000_000):
    """The document stream's rows 0 .. n_docs - 1 generated on the host in
    chunks (the next chunk drawn while the last one is copied) into device
    tensors: row_ptr int64 [n_docs + 1], words int32 [nnz]."""
    from concurrent.futures import ThreadPoolExecutor
    dev = torch.device("cuda", 0)
    counts = synth.row_counts(n_docs, seed=0, mean=mean, lo=10, hi=400)
    rp = np.zeros(n_docs + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    del counts
    nnz = int(rp[-1])
    log(f"[bench] {n_docs} documents, {nnz} nonzeros ({nnz * 4 / 1e9:.1f} GB of words)")
    rp_dev = torch.from_numpy(rp).to(dev)
    w_dev = torch.empty(nnz, dtype=torch.int32, device=dev)
    starts = list(range(0, n_docs, chunk))

    def gen(r0):
        return synth.generate(min(chunk, n_docs - r0), seed=0, mean=mean, lo=10, hi=400, row0=r0)

    t0 = time.time()
    with ThreadPoolExecutor(1) as ex:
        fut = ex.submit(gen, starts[0])
        for i, r0 in enumerate(starts):
            part = fut.result()
            if i + 1 < len(starts):
                fut = ex.submit(gen, starts[i + 1])
            a = int(rp[r0])
            assert part.nnz == int(rp[r0 + part.n_rows]) - a
            w_dev[a:a + part.nnz].copy_(torch.from_numpy(part.words.view(np.int32)))
            if i % 10 == 9 or i + 1 == len(starts):
                log(f"[bench] generated {r0 + part.n_rows} documents ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return rp_dev, w_dev, nnz


def lone_query_latency(binding, ix, q_rp, q_w, dim, n_rows, k, cut, hf, stream, n=64, reps=3):
    """Device time of single-query searches (HIP events on the launch
    stream): n queries spread over the batch, each searched alone `reps`
    times after a warm-up, in a new workspace's shape for one query (the
    wide schedule) and in the query-major shape (512 threads, window 16)."""
    import torch
    out = {"queries": n}
    picks = np.linspace(0, n_rows - 1, n).astype(np.int64)
    ids = torch.empty((1, k), dtype=torch.int32, device=q_w.device)
    sc = torch.empty((1, k), dtype=torch.float32, device=q_w.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, shape in (("wide", None), ("query_major", (512, 0, 16, 0))):
        ws = binding.seismic_workspace_create(ix.handle, 1, k)
        try:
            if shape:
                binding.seismic_workspace_set_config(ws, *shape)
            ts = []
            for i in picks:
                q = binding.device_csr(q_rp[int(i):int(i) + 2], q_w, dim)  # one row, absolute offsets
                binding.seismic_search_batch(ix.handle, ws, q, k, cut, hf, ids, sc, stream=stream)
                e0.record(stream)
                for _ in range(reps):
                    binding.seismic_search_batch(ix.handle, ws, q, k, cut, hf, ids, sc, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) / reps)
            ts = np.asarray(ts)
            out[name] = {"launch": binding.seismic_workspace_get_config(ws, 1),
                         "p50_ms": round(float(np.percentile(ts, 50)), 3),
                         "p99_ms": round(float(np.percentile(ts, 99)), 3), "mean_ms": round(float(ts.mean()), 3)}
        finally:
            binding.seismic_workspace_free(ws)
    return out


def batch_latency(binding, ix, q_rp, q_w, dim, n_rows, k, cut, hf, stream, sizes=(1, 8, 32, 64, 128), n_batches=12):
    """Device time of small batches in a new workspace's shapes (the wide
    schedule up to 64 queries, query-major above): for each size, n_batches
    batches of consecutive queries spread over the batch, each timed with
    HIP events on the launch stream after a warm-up of the same batch."""
    import torch
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for n in sizes:
        ws = binding.seismic_workspace_create(ix.handle, n, k)
        try:
            ids = torch.empty((n, k), dtype=torch.int32, device=q_w.device)
            sc = torch.empty((n, k), dtype=torch.float32, device=q_w.device)
            ts = []
            for s0 in np.linspace(0, n_rows - n, n_batches).astype(np.int64):
                q = binding.device_csr(q_rp[int(s0):int(s0) + n + 1], q_w, dim)
                binding.seismic_search_batch(ix.handle, ws, q, k, cut, hf, ids, sc, stream=stream)
                e0.record(stream)
                binding.seismic_search_batch(ix.handle, ws, q, k, cut, hf, ids, sc, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            out[str(n)] = {"mean_ms": round(float(np.mean(ts)), 3), "schedule": binding.seismic_workspace_get_config(ws, n)}
        finally:
            binding.seismic_workspace_free(ws)
    return out


def serve_run(binding, ix, qs, rate, seconds, k, cut, hf, probe, tau, max_batch=1024, slots=4):
    """Open-loop Poisson arrivals at `rate` queries/s for `seconds` (queries
    cycle through the batch), served by the library's serving loop.
    Latency = completion - arrival."""
    n = int(rate * seconds)
    rows = np.arange(n) % qs.n_rows
    sub = qs.subset(rows)
    arrivals = 0.2 + np.cumsum(np.random.default_rng(4).exponential(1.0 / rate, n))
    sv = binding.seismic_server_create(ix.handle, k, cut, hf, max_batch=max_batch, n_slots=slots, probe=probe,
                                       probe_tau=tau)
    try:
        t0 = binding.seismic_server_clock(sv)
        first = binding.seismic_server_submit_batch(sv, binding.host_csr(sub.row_ptr, sub.words, sub.dim),
                                                    t0 + arrivals)
        binding.seismic_server_wait_all(sv, 600.0)
        _, _, lat = binding.seismic_server_results(sv, first, n, k)
        st = binding.seismic_server_stats(sv)
    finally:
        binding.seismic_server_free(sv)
    span = float(np.max(arrivals + lat) - arrivals[0])
    return {"offered_qps": rate, "queries": n, "sustained_qps": round(n / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "batches": st["batches"], "mean_batch": round(n / max(st["batches"], 1), 1),
            "max_inflight": st["max_inflight"], "slots": slots, "max_batch": max_batch}


def grid_1m_leg():
    """The 1M-document configuration's query_cut x heap_factor grid (10k
    Poisson(43) queries, k 10), run by this script in a child process; its
    progress goes to stderr."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--workload", "1M", "--grid", "5,10,20x0.7,0.8,0.9",
           "--no-serve", "--knn", "0", "--probe", "none", "--cpu-seconds", "0", "--no-k100", "--no-unique",
           "--steps", "5", "--warmup", "1"]
    log("[bench] 1M grid: " + " ".join(cmd[2:]))
    t0 = time.time()
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
        if r.returncode != 0:
            return {"error": f"exit status {r.returncode}"}
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError) as e:
        return {"error": f"{type(e).__name__}: {e}"}
    grid = [[p["query_cut"], p["hf"], p["recall"], round(p["qps"]), p["layout_frac"]] for p in d["config"]["grid"] or []]
    return {"qps": d["value"], "recall_at_10": d["config"]["recall_at_10"], "ms_per_step": d["ms_per_step"],
            "workload": d["config"]["workload"], "frac": d["roofline"]["frac"],
            "layout_frac": d["roofline"]["layout_frac"],
            "grid_fields": ["query_cut", "heap_factor", "recall_at_10", "qps", "layout_frac"], "grid": grid,
            "seconds": round(time.time() - t0, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="msmarco-8.8M", choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--recall", type=float, default=0.95)
    ap.add_argument("--hf", type=float, default=None, help="skip the sweep and use this heap_factor")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline budget (0 = skip)")
    ap.add_argument("--cpu-exact-queries", type=int, default=32,
                    help="queries of the CPU exact brute-force baseline (0 = skip)")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--profile-copy", action="store_true", help="also run a plain copy for counter calibration")
    ap.add_argument("--index-cache", default=None, help="load the index from this file if present, else build and save")
    ap.add_argument("--plain-rows", action="store_true", help="search the forward rows in place (no block-major copies)")
    ap.add_argument("--hot-sample", type=int, default=2000,
                    help="device-built index: queries of a held-out sample whose most evaluated lists get block-major "
                         "copies (0 = none)")
    ap.add_argument("--hot-reserve-gb", type=float, default=8.0,
                    help="device memory left free by the hot-list copies")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--schedule", type=int, default=None,
                    help="fix the launch shape to 256 threads, 3 per CU, window 8 and this schedule (0 query-major, "
                         "1 list-major) instead of autotuning")
    ap.add_argument("--host-build", action="store_true",
                    help="build the index on the host (default: the GPU build, byte-identical)")
    ap.add_argument("--alpha", type=float, default=0.0,
                    help="proportional list caps ceil(alpha |L_i|) at build time (0 = fixed lambda)")
    ap.add_argument("--query-mass", type=float, default=0.0,
                    help="search with the alpha_q-MSS query cut of this mass fraction instead of query_cut")
    ap.add_argument("--cuts", default="",
                    help="query_cut values of the operating-point search, e.g. '10,15,20,30' (default: the workload's "
                         "cut for k <= 10, else 10,15,20,30)")
    ap.add_argument("--grid", default="", help="also sweep query_cut x heap_factor, e.g. '5,10,20x0.7,0.8,0.9'")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-grid-1m", action="store_true",
                    help="skip the 1M configuration's query_cut x heap_factor grid (run with the 8.8M default)")
    ap.add_argument("--no-k100", action="store_true",
                    help="skip the fixed k = 100 operating point (timed only in runs without --hf)")
    ap.add_argument("--lone-only", action="store_true",
                    help="measure only the lone-query latency (at --hf, default 0.75) and print it as one JSON line")
    ap.add_argument("--knn", type=int, default=20, help="kappa of the kappa-NN graph for the refined form (0 = skip)")
    ap.add_argument("--knn-cut", type=int, default=10, help="query_cut of the graph-building searches")
    ap.add_argument("--knn-hf", type=float, default=0.5, help="heap_factor of the graph-building searches")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window per serving rate")
    ap.add_argument("--n-docs", type=int, default=0, help="override the workload's document count")
    ap.add_argument("--no-unique", action="store_true", help="skip the compulsory (unique) bytes of the batch")
    ap.add_argument("--locality", action="store_true",
                    help="also time the batch reordered so that queries sharing their first lists run together")
    ap.add_argument("--probe", default="train",
                    help="learned block probe evaluated beside the heap_factor rule: 'train' trains it in this run on "
                         "the GPU (1M-document index, 500k samples), a path loads saved weights, '' or none skips it")
    ap.add_argument("--probe-epochs", type=int, default=200)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2509_24815_amd import Index, binding, hot_list_order

    for lib in (synth._LIB_PATH, binding.LIB_PATH):
        if not os.path.exists(lib):
            import __graft_entry__
            __graft_entry__.build()
            break
    binding.load()
    W = WORKLOADS[args.workload]
    k = args.k
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    n_docs = args.n_docs or W["n_docs"]
    on_device = W.get("device_build", False)
    t0 = time.time()
    hbm = None
    if on_device:
        # collection and index live only in HBM: no host oracle, graph, probe or serving legs
        args.cpu_seconds, args.knn, args.probe, args.no_serve = 0.0, 0, "", True
        log(f"[bench] workload {args.workload}: generating {n_docs} docs into HBM (host cores: {os.cpu_count()})")
        rp_dev, w_dev, doc_nnz = device_collection(torch, synth, n_docs, W["dmean"])
        qs = synth.generate(W["n_queries"], seed=0, stream=synth.STREAM_QUERIES, law=W["qlaw"], mean=W["qmean"],
                            lo=1, hi=400)
        log(f"[bench] generated {doc_nnz} doc nonzeros, {qs.nnz} query nonzeros ({time.time() - t0:.1f} s)")
        docs = None
        t1 = time.time()
        ix = Index.build_device(binding.device_csr(rp_dev, w_dev, synth.DIM), W["lam"], W["beta"], W["gamma"],
                                seed=0, verbose=True, alpha=args.alpha)
        build_s = time.time() - t1
        log(f"[bench] index built on the device in {build_s:.1f} s")
        del rp_dev, w_dev
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info()
        hbm = {"index_resident_gb": round((total - free) / 1e9, 1), "device_total_gb": round(total / 1e9, 1)}
        info = ix.info()
        log(f"[bench] index: {info}; HBM in use {hbm}")
        layout = "rows"
    else:
        log(f"[bench] workload {args.workload}: generating {n_docs} docs (host cores: {os.cpu_count()})")
        docs = synth.docs(n_docs, seed=0)
        qs = synth.queries(W["n_queries"], seed=0, law=W["qlaw"])
        log(f"[bench] generated {docs.nnz} doc nonzeros, {qs.nnz} query nonzeros ({time.time() - t0:.1f} s)")
        t1 = time.time()
        cache = args.index_cache
        if cache and os.path.exists(cache):
            ix = Index.load(cache)
            build_s = None
            log(f"[bench] index loaded from {cache} in {time.time() - t1:.1f} s")
        else:
            builder = Index.build if args.host_build else Index.build_gpu
            ix = builder(docs, W["lam"], W["beta"], W["gamma"], seed=0, n_threads=args.threads, verbose=True,
                         alpha=args.alpha)
            build_s = time.time() - t1
            log(f"[bench] index built in {build_s:.1f} s")
            if cache:
                ix.save(cache)
                log(f"[bench] index saved to {cache}")
        info = ix.info()
        log(f"[bench] index: {info}")
        t1 = time.time()
        layout = "block_rows"
        try:
            ix.upload(0, block_rows=not args.plain_rows)
            layout = "rows" if args.plain_rows else "block_rows"
        except Exception as e:  # not enough HBM for the block-major copies
            log(f"[bench] block-major rows unavailable ({e}); plain rows")
            ix.close()
            ix = Index.load(cache) if cache and os.path.exists(cache) else \
                Index.build(docs, W["lam"], W["beta"], W["gamma"], seed=0, n_threads=args.threads, alpha=args.alpha)
            ix.upload(0)
            layout = "rows"
        log(f"[bench] index resident in HBM ({layout}, {time.time() - t1:.1f} s)")

    q_rp = torch.from_numpy(qs.row_ptr.astype(np.int64)).to(dev)
    q_w = torch.from_numpy(qs.words.view(np.int32)).to(dev)
    qcsr = binding.device_csr(q_rp, q_w, qs.dim)
    nq = qs.n_rows
    q_nnz = np.diff(qs.row_ptr.astype(np.int64))
    ws = binding.seismic_workspace_create(ix.handle, nq, max(k, 100))
    binding.seismic_workspace_set_config(ws, 256, 0, 8)
    if args.schedule is not None:
        binding.seismic_workspace_set_config(ws, 256, 3, 8, args.schedule)
        args.no_autotune = True
    out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    out_sc = torch.empty((nq, k), dtype=torch.float32, device=dev)
    if args.query_mass > 0:
        cuts = [0]
    elif args.cuts:
        cuts = [int(c) for c in args.cuts.split(",")]
    else:
        cuts = [W["cut"]] if k <= 10 else [W["cut"], 15, 20, 30]
    cut = cuts[0]
    if args.lone_only:
        hf = args.hf if args.hf is not None else 0.75
        lone = lone_query_latency(binding, ix, q_rp, q_w, qs.dim, nq, k, cut, hf, stream)
        print(json.dumps({"lone_query_latency": lone, "workload": args.workload, "query_cut": cut, "k": k,
                          "heap_factor": hf}), flush=True)
        return
    qmass = args.query_mass
    grid_cuts = sorted({int(c) for c in args.grid.split("x")[0].split(",")}) if args.grid else []
    prefix = torch.zeros((nq, max([c or binding.MAX_QUERY_NNZ for c in cuts] + grid_cuts)), dtype=torch.int16,
                         device=dev)
    counters = torch.zeros((nq, 8), dtype=torch.int64, device=dev)

    # ground truth
    t2 = time.time()
    ex_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    ex_sc = torch.empty((nq, k), dtype=torch.float32, device=dev)
    binding.exact_topk(ix.handle, qcsr, k, ex_ids, ex_sc, stream)
    torch.cuda.synchronize()
    exact_s = time.time() - t2
    log(f"[bench] exact top-{k} of {nq} queries on the GPU: {exact_s:.2f} s")
    ex = ex_ids.cpu().numpy().view(np.uint32)
    ex_s = ex_sc.cpu().numpy()

    hot = None
    if on_device and not args.plain_rows and args.hot_sample > 0:
        # the index reads its rows in place (copies of every list would not
        # fit): block-major copies of the lists that a held-out sample of
        # queries evaluates most, in the memory left once exact search's
        # inverted index is freed
        t3 = time.time()
        ix.release_exact()
        sample = synth.generate(args.hot_sample, seed=1, stream=synth.STREAM_QUERIES, law=W["qlaw"],
                                mean=W["qmean"], lo=1, hi=400)
        s_rp = torch.from_numpy(sample.row_ptr.astype(np.int64)).to(dev)
        s_w = torch.from_numpy(sample.words.view(np.int32)).to(dev)
        hf_s = args.hf if args.hf is not None else W.get("hot_hf", 0.3)
        _, _, s_pre, _, _, s_term = ix.search(binding.device_csr(s_rp, s_w, sample.dim), k, cut, hf_s, trace=True,
                                              prefix_stride=max(cut, 1))
        torch.cuda.synchronize()
        s_pre = s_pre.cpu().numpy().astype(np.uint16).astype(np.int64)
        s_term = s_term.cpu().numpy().astype(np.int64)
        order = hot_list_order(s_pre, s_term)
        del s_rp, s_w
        torch.cuda.empty_cache()

        def batch_ms():  # the timed batch at the sample's heap_factor, the workspace's launch shape
            for _ in range(2):
                binding.seismic_search_batch(ix.handle, ws, qcsr, k, cut, hf_s, out_ids, out_sc, None, 0, None, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                binding.seismic_search_batch(ix.handle, ws, qcsr, k, cut, hf_s, out_ids, out_sc, None, 0, None, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.steps, out_ids.cpu().numpy().copy(), out_sc.cpu().numpy().copy()

        before_ms, before_ids, before_sc = batch_ms()
        free, total = torch.cuda.mem_get_info()
        budget = max(0, int(free - args.hot_reserve_gb * 1e9))
        t4 = time.time()
        n_cp, used = ix.copy_lists(order, budget)
        copy_s = time.time() - t4
        after_ms, after_ids, after_sc = batch_ms()
        # the timed batch's own evaluated blocks that lie in copied lists
        _, _, b_pre, _, _, b_term = ix.search(qcsr, k, cut, hf_s, trace=True, prefix_stride=max(cut, 1))
        torch.cuda.synchronize()
        b_pre = b_pre.cpu().numpy().astype(np.uint16).astype(np.int64)
        b_term = b_term.cpu().numpy().astype(np.int64)
        copied = np.zeros(qs.dim, dtype=bool)
        copied[order[:n_cp]] = True
        m = s_pre > 0
        cover = float(s_pre[m][copied[s_term[m]]].sum() / max(1, s_pre[m].sum()))
        mb = b_pre > 0
        cover_b = float(b_pre[mb][copied[b_term[mb]]].sum() / max(1, b_pre[mb].sum()))
        free, total = torch.cuda.mem_get_info()
        hot = {"lists_copied": n_cp, "lists_evaluated_by_sample": int(len(order)), "copies_gb": round(used / 1e9, 1),
               "sample_queries": args.hot_sample, "sample_heap_factor": hf_s,
               "sample_blocks_in_copied_lists": round(cover, 4), "batch_blocks_in_copied_lists": round(cover_b, 4),
               "copy_s": round(copy_s, 2), "step_s": round(time.time() - t3, 1),
               "hbm_in_use_gb": round((total - free) / 1e9, 1),
               "batch_ms_rows_in_place": round(before_ms, 3), "batch_ms_with_copies": round(after_ms, 3),
               "same_results": bool(np.array_equal(before_ids, after_ids) and np.array_equal(before_sc, after_sc))}
        layout = "rows in place + block-major copies of hot lists"
        log(f"[bench] hot-list copies: {hot}")

    def recall_of(ids_np, sc_np, truth=None):
        t_ids, t_sc = (ex, ex_s) if truth is None else truth
        strict, tie = [], []
        for a, b, bs, asc in zip(ids_np, t_ids, t_sc, sc_np):
            valid = b != 0xFFFFFFFF
            n = int(valid.sum())
            if n == 0:
                continue
            strict.append(len(set(a[a != 0xFFFFFFFF]) & set(b[valid])) / n)
            kth = bs[valid][-1]
            tie.append(min(n, int((asc[a != 0xFFFFFFFF] >= kth).sum())) / n)
        return float(np.mean(strict)), float(np.mean(tie))

    def run(hf, with_stats, probe=None, tau=0.0, c=None, flags=0):
        c = cut if c is None else c
        binding.seismic_search_batch(ix.handle, ws, qcsr, k, c, hf, out_ids, out_sc,
                                     prefix if with_stats else None, prefix.shape[1] if with_stats else 0,
                                     counters if with_stats else None, stream, probe=probe, probe_tau=tau,
                                     flags=flags, query_mass=qmass)

    def measure(hf, probe=None, tau=0.0, c=None, flags=0):
        run(hf, True, probe, tau, c, flags)
        torch.cuda.synchronize()
        cnt = counters.cpu().numpy()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(2):
            run(hf, False, probe, tau, c, flags)
        ev[1].record(stream)
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) / 2e3
        rs, rt = recall_of(out_ids.cpu().numpy().view(np.uint32), out_sc.cpu().numpy())
        return dict(recall=round(rs, 4), recall_tie_aware=round(rt, 4), qps=round(nq / dt, 1),
                    docs_evaluated=float(cnt[:, 3].mean()), blocks_evaluated=float(cnt[:, 2].mean()),
                    layout_gbs=round(float(alg_bytes(cnt, q_nnz, k).sum()) / dt / 1e9, 1))

    def search_grid(values, key, fn, bisections=3):
        """Walk values from most to least pruning; stop at the first point
        that reaches the recall target, then bisect between it and the
        previous point (up to `bisections` times) for the most pruning value
        that still reaches it (recall is deterministic, so the choice is
        too).  Returns (chosen value, points)."""
        pts, chosen, prev = [], None, None
        for v in values:
            pt = dict({key: v}, **fn(v))
            pts.append(pt)
            log(f"[bench] sweep {pt}")
            if pt["recall"] >= args.recall:
                chosen = v
                break
            prev = v
        lo, hi = prev, chosen
        for _ in range(bisections if chosen is not None and prev is not None else 0):
            mid = round((lo + hi) / 2, 4)
            if mid in (lo, hi):
                break
            pt = dict({key: mid}, **fn(mid))
            pts.append(pt)
            log(f"[bench] sweep {pt}")
            if pt["recall"] >= args.recall:
                hi = chosen = mid
            else:
                lo = mid
        return chosen, pts

    # operating point: for each query_cut, sweep heap_factor (Alg. 2 skip rule
    # r * hf < heap.min: larger hf prunes less) up to the first point that
    # reaches the recall target; keep the fastest (cut, hf) that does
    best, cut_points = None, []
    for c in cuts:
        cut = c
        if args.hf:
            sweep = [dict(hf=args.hf, **measure(args.hf))]
            log(f"[bench] sweep query_cut {c}: {sweep[0]}")
            ch = args.hf if sweep[0]["recall"] >= args.recall else None
        else:
            ch, sweep = search_grid(list(W["hfs"]), "hf", measure)
        if ch is not None:
            pt = next(p for p in sweep if p["hf"] == ch)
            cut_points.append(dict(query_cut=c, **pt))
            if best is None or pt["qps"] > best[2]["qps"]:
                best = (c, ch, pt)
        else:
            top = max(sweep, key=lambda p: p["recall"])
            cut_points.append(dict(query_cut=c, reached_target=False, **top))
            log(f"[bench] query_cut {c}: no swept heap_factor reached Recall@{k} {args.recall} "
                f"(best {top['recall']} at hf {top['hf']})")
    if best is None:
        c, ch = max(((p["query_cut"], p["hf"], p["recall"]) for p in cut_points), key=lambda x: x[2])[:2]
        best = (c, ch, next(p for p in cut_points if p["query_cut"] == c))
        log(f"[bench] no (query_cut, heap_factor) reached Recall@{k} {args.recall}; using the best ({c}, {ch})")
    cut, chosen, point = best
    if len(cuts) > 1:
        log(f"[bench] operating points per query_cut: {cut_points}; chosen query_cut {cut}, heap_factor {chosen}")

    # algorithmic bytes of the chosen point
    run(chosen, True)
    torch.cuda.synchronize()
    cnt = counters.cpu().numpy()
    plain_prefix = prefix.cpu().numpy().view(np.uint16)[:, :max(cut, 1)].copy()
    layout_bytes = float(alg_bytes(cnt, q_nnz, k).sum())

    # launch shape for this batch: the library's autotuner times every shape
    tuned = binding.seismic_workspace_get_config(ws, nq) if args.schedule is not None else None
    if not args.no_autotune:
        tt = time.time()
        res = binding.seismic_autotune(ix.handle, ws, qcsr, k, cut, chosen, out_ids, out_sc, reps=2, stream=stream)
        tuned = binding.seismic_workspace_get_config(ws, nq)
        log(f"[bench] autotuned over {len(res)} shapes in {time.time() - tt:.1f} s: {tuned} "
            f"({min(r[1] for r in res):.3f} ms; worst {max(r[1] for r in res):.3f} ms)")
        for sched in sorted({r[0].get("schedule", 0) for r in res}):
            best_s = min((r for r in res if r[0].get("schedule", 0) == sched), key=lambda r: r[1])
            log(f"[bench]   schedule {sched}: best {best_s[0]} {best_s[1]:.3f} ms")

    if tuned is not None:  # workgroups per CU that actually stay resident in that shape
        tuned["resident_per_cu"] = binding.seismic_workspace_resident_per_cu(ws, nq, k)

    # timed steps
    for _ in range(args.warmup):
        run(chosen, False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = time.time()
    ev0.record(stream)
    for _ in range(args.steps):
        run(chosen, False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - ts
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    qps = nq * args.steps / (gpu_ms / 1e3)
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, {qps:.0f} QPS, wall {wall:.2f} s, "
        f"{layout_bytes / (ms_per_step / 1e3) / 1e9:.1f} GB/s by the library layout's bytes")

    plain_ids = out_ids.cpu().numpy().view(np.uint32).copy()  # results of the timed steps
    plain_sc = out_sc.cpu().numpy().copy()

    locality = None
    if args.locality:
        # queries sorted by their first two visited lists (largest entries,
        # value desc then term asc): concurrent queries share lists and blocks
        keys = []
        for q in range(nq):
            t, v = qs.row(q)
            o = np.lexsort((t, -v.astype(np.float64)))[:2]
            keys.append((int(t[o[0]]) if len(o) else -1, int(t[o[1]]) if len(o) > 1 else -1))
        perm = sorted(range(nq), key=lambda q: keys[q])
        pq = qs.subset(perm)
        prp = torch.from_numpy(pq.row_ptr.astype(np.int64)).to(dev)
        pw_ = torch.from_numpy(pq.words.view(np.int32)).to(dev)
        pcsr = binding.device_csr(prp, pw_, pq.dim)
        for _ in range(args.warmup):
            binding.seismic_search_batch(ix.handle, ws, pcsr, k, cut, chosen, out_ids, out_sc, None, 0, None, stream,
                                         query_mass=qmass)
        torch.cuda.synchronize()
        o0, o1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        o0.record(stream)
        for _ in range(args.steps):
            binding.seismic_search_batch(ix.handle, ws, pcsr, k, cut, chosen, out_ids, out_sc, None, 0, None, stream,
                                         query_mass=qmass)
        o1.record(stream)
        torch.cuda.synchronize()
        oms = o0.elapsed_time(o1) / args.steps
        same = bool(np.array_equal(out_ids.cpu().numpy().view(np.uint32), plain_ids[perm]))
        locality = {"ms_per_step": round(oms, 4), "qps": round(nq / (oms / 1e3), 1),
                    "vs_batch_order": round(ms_per_step / oms, 4), "same_results": same}
        log(f"[bench] locality order {locality}")

    # the batch's trace at the chosen point: compulsory bytes (lower bound of
    # the traffic) and each query's distinct scored documents (the scope
    # formula's row term)
    serialized, unique, distinct, distinct_nnz = None, None, None, None
    if not on_device and not args.no_unique:
        tu = time.time()
        from paper_2509_24815_amd import indexfile
        serialized = ix.serialize()
        stride = cut or binding.MAX_QUERY_NNZ
        _, _, pref_t, _, _, term_t = ix.search(qcsr, k, cut, chosen, trace=True, prefix_stride=stride,
                                               query_mass=qmass)
        unique, distinct, distinct_nnz = trace_bytes(indexfile.sections(serialized), qs,
                                                     term_t.cpu().numpy().view(np.uint32),
                                                     pref_t.cpu().numpy().view(np.uint16), k)
        log(f"[bench] compulsory bytes of the batch: {unique:.4e} ({unique / layout_bytes:.3f} of the "
            f"layout's algorithmic bytes); distinct scored documents per query {distinct.mean():.0f} of "
            f"{cnt[:, 3].mean():.0f} evaluated ({time.time() - tu:.1f} s)")
    bytes_per_launch = float(scope_bytes(cnt, q_nnz, k, distinct, distinct_nnz).sum())
    achieved = bytes_per_launch / (ms_per_step / 1e3) / 1e9
    log(f"[bench] algorithmic bytes per launch: {bytes_per_launch:.4e} by the scope formula"
        + ("" if distinct is not None else " (every document of an evaluated block counted)")
        + f", {layout_bytes:.4e} by the library layout; {achieved:.1f} GB/s")

    # query_cut x heap_factor grid (same batch, autotuned shape)
    grid = None
    if args.grid:
        hf_list = [float(x) for x in args.grid.split("x")[1].split(",")]
        grid = []
        for c in grid_cuts:
            for hf in hf_list:
                pt = dict(query_cut=c, hf=hf, **measure(hf, c=c))
                pt["layout_frac"] = round(pt["layout_gbs"] / PEAK_HBM_GBS, 4)
                grid.append(pt)
                log(f"[bench] grid {pt}")

    # learned block probe (lists that start with a full heap), heap_factor rule
    # elsewhere: trained here on the GPU by the library's kernels on a
    # separate 1M-document index and probe-training queries, or loaded
    learned, probe_src, probe_train = None, None, None
    if args.probe == "train":
        from paper_2509_24815_amd import train_probe
        tt = time.time()
        weights, probe_train = train_probe.train_probe(epochs=args.probe_epochs, log=log)
        probe_train = {key: v for key, v in probe_train.items() if key != "loss_history"}
        probe_train["total_s"] = round(time.time() - tt, 1)
        probe_src = "trained in this run"
        log(f"[bench] probe trained: {probe_train}")
    elif args.probe not in ("", "none"):
        if not os.path.exists(args.probe):
            raise SystemExit(f"--probe {args.probe}: no such file (use 'train', a saved probe, or none)")
        from paper_2509_24815_amd import probe as P
        weights = P.load(args.probe)
        probe_src = os.path.relpath(args.probe, ROOT)
    if probe_src is not None:
        from paper_2509_24815_amd import probe as P
        pw = P.to_device(weights, dev)
        taus = [2.0, 1.5, 1.0, 0.75, 0.5, 0.25, 0.0, -0.25, -0.5, -1.0, -1.5, -2.0, -3.0]
        tau, lpts = search_grid(taus, "tau", lambda t: measure(chosen, pw, t))
        if tau is not None:
            lp = next(p for p in lpts if p["tau"] == tau)
            for _ in range(args.warmup):
                run(chosen, False, pw, tau)
            torch.cuda.synchronize()
            l0, l1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            l0.record(stream)
            for _ in range(args.steps):
                run(chosen, False, pw, tau)
            l1.record(stream)
            torch.cuda.synchronize()
            lms = l0.elapsed_time(l1) / args.steps
            learned = {"probe": probe_src, "tau": tau, "heap_factor_fallback": chosen,
                       f"recall_at_{k}": lp["recall"], "qps": round(nq / (lms / 1e3), 1), "ms_per_step": round(lms, 4),
                       "docs_evaluated": round(lp["docs_evaluated"], 1),
                       "qps_vs_heap_factor_rule": round(lms and ms_per_step / lms, 4),
                       "docs_vs_heap_factor_rule": round(lp["docs_evaluated"] / point["docs_evaluated"], 4),
                       "training": probe_train}
        else:
            learned = {"probe": probe_src, "reached_target": False, "training": probe_train}
        log(f"[bench] learned probe {learned}; sweep {lpts}")

    # refined form: kappa-NN graph built on the GPU with the method itself,
    # then the refinement step after every search
    refined = None
    if args.knn > 0 and k * args.knn <= 256:
        tb = time.time()
        binding.seismic_knn_build(ix.handle, args.knn, args.knn_cut, args.knn_hf)
        knn_s = time.time() - tb
        log(f"[bench] kappa-NN graph (kappa {args.knn}, cut {args.knn_cut}, hf {args.knn_hf}) built in {knn_s:.1f} s")
        best = None
        rpts = []
        for c in sorted({max(1, cut // 2), cut}):
            ch, pts = search_grid([0.1, 0.2] + list(W["hfs"]), "hf",
                                  lambda h: measure(h, c=c, flags=binding.SEARCH_KNN))
            for p_ in pts:
                p_["query_cut"] = c
            rpts += pts
            if ch is not None:
                pt = next(p_ for p_ in pts if p_["hf"] == ch)
                if best is None or pt["qps"] > best["qps"]:
                    best = pt
        if best is not None:
            c, h = best["query_cut"], best["hf"]
            for _ in range(args.warmup):
                run(h, False, c=c, flags=binding.SEARCH_KNN)
            torch.cuda.synchronize()
            r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            r0.record(stream)
            for _ in range(args.steps):
                run(h, False, c=c, flags=binding.SEARCH_KNN)
            r1.record(stream)
            torch.cuda.synchronize()
            rms = r0.elapsed_time(r1) / args.steps
            refined = {"kappa": args.knn, "graph_build_s": round(knn_s, 1),
                       "graph_search": {"query_cut": args.knn_cut, "heap_factor": args.knn_hf},
                       "query_cut": c, "heap_factor": h, f"recall_at_{k}": best["recall"],
                       "qps": round(nq / (rms / 1e3), 1), "ms_per_step": round(rms, 4),
                       "docs_evaluated": best["docs_evaluated"],
                       "qps_vs_heap_factor_rule": round(ms_per_step / rms, 4)}
        else:
            refined = {"kappa": args.knn, "graph_build_s": round(knn_s, 1), "reached_target": False}
        log(f"[bench] refined sweep {rpts}")
        # both additions together: learned probe for the traversal, then refinement
        if learned and learned.get("tau") is not None:
            taus = [2.0, 1.5, 1.0, 0.75, 0.5, 0.25, 0.0, -0.25, -0.5, -1.0]
            t2, lpts2 = search_grid(taus, "tau", lambda t: measure(chosen, pw, t, flags=binding.SEARCH_KNN))
            both = {"tau": t2, "heap_factor_fallback": chosen}
            log(f"[bench] learned + refined sweep {lpts2}")
            if t2 is not None:
                lp2 = next(p_ for p_ in lpts2 if p_["tau"] == t2)
                for _ in range(args.warmup):
                    run(chosen, False, pw, t2, flags=binding.SEARCH_KNN)
                torch.cuda.synchronize()
                b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                b0.record(stream)
                for _ in range(args.steps):
                    run(chosen, False, pw, t2, flags=binding.SEARCH_KNN)
                b1.record(stream)
                torch.cuda.synchronize()
                bms = b0.elapsed_time(b1) / args.steps
                both.update({f"recall_at_{k}": lp2["recall"], "qps": round(nq / (bms / 1e3), 1),
                             "ms_per_step": round(bms, 4), "docs_evaluated": lp2["docs_evaluated"],
                             "qps_vs_heap_factor_rule": round(ms_per_step / bms, 4)})
            refined["with_learned_probe"] = both
        log(f"[bench] refined {refined}")

    # the workload's k = 100 operating point, fixed (no sweep), in the launch
    # shape its traffic profile was taken in; ground truth: exact top-100.
    # Part of the default run only (not of runs fixing --hf)
    k100 = None
    if W.get("k100") and k == 10 and args.hf is None and not (args.no_k100 or args.alpha or qmass):
        c100, h100 = W["k100"]
        tx = time.time()
        t_ids = torch.empty((nq, 100), dtype=torch.int32, device=dev)
        t_sc = torch.empty((nq, 100), dtype=torch.float32, device=dev)
        binding.exact_topk(ix.handle, qcsr, 100, t_ids, t_sc, stream)
        torch.cuda.synchronize()
        truth = (t_ids.cpu().numpy().view(np.uint32), t_sc.cpu().numpy())
        log(f"[bench] exact top-100 of {nq} queries on the GPU: {time.time() - tx:.2f} s")
        o_ids = torch.empty((nq, 100), dtype=torch.int32, device=dev)
        o_sc = torch.empty((nq, 100), dtype=torch.float32, device=dev)
        pre = torch.zeros((nq, c100), dtype=torch.int16, device=dev)
        binding.seismic_workspace_set_config(ws, 256, 3, 8, 0)

        def run100(stats):
            binding.seismic_search_batch(ix.handle, ws, qcsr, 100, c100, h100, o_ids, o_sc,
                                         pre if stats else None, c100 if stats else 0,
                                         counters if stats else None, stream)
        run100(True)
        torch.cuda.synchronize()
        c_np = counters.cpu().numpy()
        rs, _ = recall_of(o_ids.cpu().numpy().view(np.uint32), o_sc.cpu().numpy(), truth)
        for _ in range(args.warmup):
            run100(False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            run100(False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms100 = e0.elapsed_time(e1) / args.steps
        lb100 = float(alg_bytes(c_np, q_nnz, 100).sum())
        tr100 = measured_traffic(args.workload, c100, h100, 100)
        k100 = {"query_cut": c100, "heap_factor": h100, "recall_at_100": round(rs, 4),
                "qps": round(nq / (ms100 / 1e3), 1), "ms_per_step": round(ms100, 4),
                "docs_evaluated": round(float(c_np[:, 3].mean()), 1),
                "launch": {"threads": 256, "blocks_per_cu": 3, "window": 8, "schedule": 0,
                           "resident_per_cu": binding.seismic_workspace_resident_per_cu(ws, nq, 100)},
                "layout_bytes_per_launch": lb100,
                "layout_frac": round(lb100 / (ms100 / 1e3) / 1e9 / PEAK_HBM_GBS, 4), "traffic": tr100,
                "traffic_frac": None if tr100 is None else round(tr100 / (ms100 / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        log(f"[bench] k = 100 point {k100}")
        del t_ids, t_sc, o_ids, o_sc, pre

    # lone-query latency (device time), then the serving loop: Poisson
    # arrivals, continuous batching over 4 slots
    serving = None
    lone = None
    small = None
    if not args.no_serve:
        lone = lone_query_latency(binding, ix, q_rp, q_w, qs.dim, nq, k, cut, chosen, stream)
        log(f"[bench] lone-query latency {lone}")
        small = batch_latency(binding, ix, q_rp, q_w, qs.dim, nq, k, cut, chosen, stream)
        log(f"[bench] small-batch latency {small}")
        serving = {}
        rates = (5000.0, 20000.0, 50000.0)
        forms = [("heap_factor_rule", None, 0.0)]
        if learned and learned.get("tau") is not None:
            forms.append(("learned_probe", pw, learned["tau"]))
        for name, pr, tau in forms:
            rows = []
            for rate in rates:
                rows.append(serve_run(binding, ix, qs, rate, args.serve_seconds, k, cut, chosen, pr, tau))
                log(f"[bench] serving {name} {rows[-1]}")
            serving[name] = rows

    if args.profile_copy:
        # counter calibration: kernels of known traffic next to the search
        # in the same profile -- a plain copy (2^28 bytes read and written,
        # streaming), and a gather of 2^22 random 64-byte rows out of a 4 GiB
        # table (2^28 bytes read in scattered 64-byte segments, written
        # contiguously; the 32 MB of row indices are read too)
        n = 1 << 28
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        for _ in range(3):
            b.copy_(a)
        del a, b
        table = torch.zeros((1 << 26, 16), dtype=torch.int32, device=dev)
        rows = torch.randint(0, 1 << 26, (1 << 22,), dtype=torch.int64, device=dev,
                             generator=torch.Generator(device=dev).manual_seed(5))
        for _ in range(3):
            torch.index_select(table, 0, rows)
        torch.cuda.synchronize()
        del table, rows
        log(f"[bench] counter calibration: 3 copies of {n} bytes, 3 gathers of {1 << 22} random 64-byte rows")

    # CPU baseline: the oracle on a bounded sample of the same queries, and
    # the oracle's exact brute force on a few of them
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        oracle.build() if not os.path.exists(oracle._LIB_PATH) else None
        log("[bench] CPU baseline: the serialized index for the oracle")
        buf = serialized if serialized is not None else ix.serialize()
        ref = oracle.Index(buf)
        threads = os.cpu_count() or 1
        pilot = qs.subset(range(min(nq, 4 * threads)))
        tp = time.time()
        ref.pruned_search(pilot, k, cut, chosen, nthreads=threads, c_cap=max(cut, 1))
        per_q = (time.time() - tp) / pilot.n_rows
        n_sample = int(max(threads, min(nq, args.cpu_seconds / max(per_q, 1e-9))))
        sample = qs.subset(range(n_sample))
        tc = time.time()
        r = ref.pruned_search(sample, k, cut, chosen, nthreads=threads, c_cap=max(cut, 1))
        cpu_s = time.time() - tc
        # a query matches when its ids, scores and per-list evaluated prefixes all equal the GPU's
        same = ((r["ids"] == plain_ids[:n_sample]).all(axis=1) & (r["scores"] == plain_sc[:n_sample]).all(axis=1)
                & (r["prefix"][:, :plain_prefix.shape[1]] == plain_prefix[:n_sample]).all(axis=1))
        # the paper's protocol: one thread, mean latency per query
        one = qs.subset(range(min(nq, max(8, int(3.0 / max(per_q * threads, 1e-9))))))
        t1 = time.time()
        ref.pruned_search(one, k, cut, chosen, nthreads=1, c_cap=max(cut, 1))
        st_ms = (time.time() - t1) / one.n_rows * 1e3
        cpu = {"value": round(n_sample / cpu_s, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"first {n_sample} of the {nq} queries, heap_factor {chosen}, {cpu_s:.1f} s",
               "gpu_match_fraction": float(same.mean()), "gpu_match": "ids, scores and evaluated prefixes",
               "single_thread_ms_per_query": round(st_ms, 3), "single_thread_sample": one.n_rows}
        if docs is not None and args.cpu_exact_queries > 0:
            # exact search by brute force over every document: the exact-search CPU baseline
            ne = min(nq, args.cpu_exact_queries)
            te = time.time()
            e_ids, e_sc = oracle.exact_topk(docs, qs.subset(range(ne)), k, threads)
            ex_s_cpu = time.time() - te
            cpu["exact"] = {"value": round(ne / ex_s_cpu, 2), "unit": "queries/s", "queries": ne,
                            "seconds": round(ex_s_cpu, 1),
                            "gpu_exact_match_fraction": float(((e_ids == ex[:ne]).all(axis=1)
                                                               & (e_sc == ex_s[:ne]).all(axis=1)).mean()),
                            "gpu_exact_qps": round(nq / exact_s, 1)}
        log(f"[bench] CPU baseline {cpu}")
        del ref, buf

    traffic = measured_traffic(args.workload, cut, chosen, k) if not (args.alpha or qmass) else None
    step_s = ms_per_step / 1e3
    # one compact line per form of the method measured in this run
    forms = {"heap_factor_rule": {"qps": round(qps, 1), f"recall_at_{k}": point["recall"], "heap_factor": chosen,
                                  "ms_per_step": round(ms_per_step, 4),
                                  "docs_evaluated": round(point["docs_evaluated"], 1)},
             "launch": tuned}
    if learned:
        forms["learned_probe"] = {key: learned.get(key) for key in
                                  ("qps", f"recall_at_{k}", "tau", "heap_factor_fallback", "docs_evaluated",
                                   "qps_vs_heap_factor_rule", "probe", "training")}
    if refined:
        forms["knn_refined"] = {key: refined.get(key) for key in
                                ("qps", f"recall_at_{k}", "kappa", "query_cut", "heap_factor", "graph_build_s",
                                 "qps_vs_heap_factor_rule")}
        both = refined.get("with_learned_probe")
        if both:
            forms["learned_probe_knn_refined"] = {key: both.get(key) for key in
                                                  ("qps", f"recall_at_{k}", "tau", "qps_vs_heap_factor_rule")}
    if k100:
        forms["k100"] = k100
    if lone:
        forms["lone_query"] = {name: {"p50_ms": v["p50_ms"], "p99_ms": v["p99_ms"]}
                               for name, v in lone.items() if isinstance(v, dict)}
    if small:
        forms["batch_ms"] = {n: v["mean_ms"] for n, v in small.items()}
    if serving:
        forms["serving"] = {name: [{"offered_qps": r_["offered_qps"], "sustained_qps": r_["sustained_qps"],
                                    "p50_ms": r_["p50_ms"], "p99_ms": r_["p99_ms"]} for r_ in rows]
                            for name, rows in serving.items()}
    if args.workload == "msmarco-8.8M" and args.hf is None and not args.no_grid_1m:
        forms["grid_1M"] = grid_1m_leg()
    out = {
        "metric": "QPS at Recall@10>=0.95 (1 GPU, 8.8M docs); p50/p99 query latency",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16xf16->f64 accumulate, f32 out",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n_docs} docs, {nq}-query batch ({W['qlaw']} nnz), "
                               f"lambda {W['lam']}, beta {W['beta']}, gamma {W['gamma']}, "
                               + (f"alpha {args.alpha}, " if args.alpha else "")
                               + (f"query_mass {qmass}, " if qmass else f"query_cut {cut}, ")
                               + f"k {k}, heap_factor {chosen}",
                   f"recall_at_{k}": point["recall"], "recall_target": args.recall,
                   "index_build_s": None if build_s is None else round(build_s, 1),
                   "index_build": "cached" if build_s is None else
                   ("device-resident" if on_device else "host" if args.host_build else "gpu"),
                   "hbm": hbm, "exact_topk_s": round(exact_s, 2), "layout": layout, "launch": tuned,
                   "grid": grid, "locality_order": locality, "hot_copies": hot},
        "forms": forms,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "traffic_frac": None if traffic is None else round(traffic / step_s / 1e9 / PEAK_HBM_GBS, 4),
                     "alg_bytes_per_launch": bytes_per_launch,
                     "alg_bytes": "scope formula, distinct scored documents" if distinct is not None
                     else "scope formula, every document of an evaluated block",
                     "layout_bytes_per_launch": layout_bytes,
                     "layout_frac": round(layout_bytes / step_s / 1e9 / PEAK_HBM_GBS, 4),
                     "unique_bytes_per_launch": unique,
                     "unique_frac": None if unique is None else round(unique / step_s / 1e9 / PEAK_HBM_GBS, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
