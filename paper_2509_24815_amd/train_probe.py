"""Train the learned block probe on a synthetic collection, on the GPU.

    python -m paper_2509_24815_amd.train_probe --docs 1000000 --lam 3000 --beta 150 \\
        --queries 600 --pairs 500000 --out paper_2509_24815_amd/probes/probe_1m.npy

Builds (or loads, with --index-cache) the index (GPU build unless
--host-build; byte-identical either way), draws training queries from
the generator's probe-training stream, traces a plain search (query_cut,
heap_factor) to find each cut list's starting heap minimum, labels every
block of the lists that start with a full heap by exact top-k (does it hold
one of the query's exact top-10 documents), keeps a random subset of
--pairs samples and trains with the library's kernels.  Prints one JSON line
with the training summary.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def train_probe(docs: int = 1_000_000, lam: int = 3000, beta: int = 150, gamma: float = 0.4, queries: int = 600,
                qlaw: str = "uniform", pairs: int = 500_000, cut: int = 10, hf: float = 0.8, epochs: int = 200,
                batch: int = 8192, lr: float = 3e-3, neg_weight_per_doc: float = 0.5, seed: int = 0,
                index_cache: str | None = None, gpu_build: bool = True, log=None):
    """Builds (or loads) the training index, collects samples and trains the
    probe with the library's kernels.  Returns (bf16 weights, summary)."""
    import torch
    import synth
    from paper_2509_24815_amd import Index
    from paper_2509_24815_amd import probe as P
    from paper_2509_24815_amd.binding import device_csr

    log = log or (lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.set_device(0)
    t0 = time.time()
    if index_cache and os.path.exists(index_cache):
        ix = Index.load(index_cache)
        log(f"[train] index loaded from {index_cache}")
    else:
        log(f"[train] generating {docs} documents and building the index")
        d = synth.docs(docs, seed=seed)
        builder = Index.build_gpu if gpu_build else Index.build
        ix = builder(d, lam=lam, beta=beta, gamma=gamma, seed=seed)
        del d
        if index_cache:
            ix.save(index_cache)
    build_s = time.time() - t0
    try:
        ix.upload(0, block_rows=True)
        qs = synth.queries(queries, seed=seed, law=qlaw, stream=synth.STREAM_PROBE_QUERIES)
        rp = torch.from_numpy(qs.row_ptr.astype("int64")).cuda()
        w = torch.from_numpy(qs.words.view("int32").copy()).cuda()
        q = device_csr(rp, w, qs.dim)
        t1 = time.time()
        feat, label, idx = P.collect(ix, q, qs.n_rows, 10, cut, hf, exact_k=10)
        torch.cuda.synchronize()
        collect_s = time.time() - t1
        n_all = int(idx.numel())
        if n_all > pairs:
            g = torch.Generator(device=idx.device)
            g.manual_seed(seed)
            idx = idx[torch.randperm(n_all, generator=g, device=idx.device)[:pairs]].contiguous()
        n_pos = int((label[idx.long()] == 1).sum())
        log(f"[train] {n_all} samples collected in {collect_s:.1f} s; training on {idx.numel()} ({n_pos} positive)")
        t2 = time.time()
        weights, hist = P.train(feat, label, idx, epochs=epochs, batch=batch, lr=lr,
                                neg_weight_per_doc=neg_weight_per_doc, seed=seed, log=log)
        torch.cuda.synchronize()
        train_s = time.time() - t2
    finally:
        ix.close()
    summary = {"docs": docs, "lambda": lam, "beta": beta, "queries": queries, "query_law": qlaw,
               "traced_heap_factor": hf, "samples_collected": n_all, "samples_used": int(idx.numel()),
               "positives": n_pos, "epochs": epochs, "batch": batch, "lr": lr,
               "neg_weight_per_doc": neg_weight_per_doc, "loss_history": hist,
               "index_build_s": round(build_s, 1), "collect_s": round(collect_s, 2), "train_s": round(train_s, 2)}
    return weights, summary


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--docs", type=int, default=1_000_000)
    ap.add_argument("--lam", type=int, default=3000)
    ap.add_argument("--beta", type=int, default=150)
    ap.add_argument("--gamma", type=float, default=0.4)
    ap.add_argument("--queries", type=int, default=600)
    ap.add_argument("--qlaw", default="uniform", choices=("uniform", "poisson"))
    ap.add_argument("--pairs", type=int, default=500_000)
    ap.add_argument("--cut", type=int, default=10)
    ap.add_argument("--hf", type=float, default=0.8, help="heap_factor of the traced plain search")
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--neg-weight-per-doc", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--index-cache", default=None)
    ap.add_argument("--host-build", action="store_true")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    sys.path.insert(0, ROOT)
    from paper_2509_24815_amd import probe as P
    weights, summary = train_probe(args.docs, args.lam, args.beta, args.gamma, args.queries, args.qlaw, args.pairs,
                                   args.cut, args.hf, args.epochs, args.batch, args.lr, args.neg_weight_per_doc,
                                   args.seed, args.index_cache, gpu_build=not args.host_build)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    P.save(args.out, weights)
    print(json.dumps(dict({"out": args.out}, **summary)), flush=True)


if __name__ == "__main__":
    main()
