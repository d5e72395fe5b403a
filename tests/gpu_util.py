"""Helpers shared by the GPU tests: device placement of CSR inputs and the
comparison of GPU results with the oracle."""
import numpy as np

from paper_2509_24815_amd import binding


def to_device_csr(csr):
    import torch
    rp = torch.from_numpy(csr.row_ptr.astype(np.int64)).cuda()
    w = torch.from_numpy(csr.words.view(np.int32).copy() if csr.nnz else np.zeros(1, dtype=np.int32)).cuda()
    if csr.nnz == 0:
        w = w[:0]
    return binding.device_csr(rp, w, csr.dim)


def as_u32(t):
    return t.cpu().numpy().view(np.uint32)


def compare_with_oracle(gpu, ref, k, cut_cap):
    """gpu = (ids, scores, prefix, counters) torch; ref = oracle dict.
    Returns the number of mismatching queries (and prints the first)."""
    ids, sc, pref, cnt = gpu
    g_ids = as_u32(ids)
    g_sc = sc.cpu().numpy()
    g_pref = pref.cpu().numpy().view(np.uint16)[:, :cut_cap]
    g_cnt = cnt.cpu().numpy().view(np.uint64)
    bad = []
    for q in range(g_ids.shape[0]):
        same = (np.array_equal(g_ids[q], ref["ids"][q]) and np.array_equal(g_sc[q], ref["scores"][q])
                and np.array_equal(g_pref[q], ref["prefix"][q][:cut_cap])
                and np.array_equal(g_cnt[q][[0, 1, 2, 3, 4, 5, 7]], ref["counters"][q][[0, 1, 2, 3, 4, 5, 7]]))
        if not same:
            bad.append(q)
    if bad:
        q = bad[0]
        print(f"first mismatch q={q}: gpu ids {g_ids[q]} oracle {ref['ids'][q]}")
        print(f"  gpu scores {g_sc[q]} oracle {ref['scores'][q]}")
        print(f"  gpu prefix {g_pref[q]} oracle {ref['prefix'][q][:cut_cap]}")
        print(f"  gpu counters {g_cnt[q]} oracle {ref['counters'][q]}")
    return bad
