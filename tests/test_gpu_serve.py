"""GPU tests of the serving loop through the C ABI: results of queries
served in mixed, overlapping batches equal the oracle's and the results of
the same queries searched alone; admission, latency and error handling."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def idx():
    import torch
    _log("[serve] building a 30k-document index (lambda 600, beta 30)")
    docs = synth.docs(30_000, seed=4)
    qs = synth.queries(800, seed=4, law="uniform")
    ix = Index.build(docs, lam=600, beta=30, gamma=0.4, seed=4)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, ix, ref


def _arrivals(n, rate, seed, lead=0.05):
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return lead + np.cumsum(gaps)


@pytest.mark.parametrize("rate,max_batch,slots", [(20000.0, 64, 4), (200000.0, 256, 2)])
def test_served_results_equal_alone_and_oracle(idx, rate, max_batch, slots):
    docs, qs, ix, ref = idx
    _log(f"[serve] {qs.n_rows} queries at {rate:.0f}/s, batches of <= {max_batch}, {slots} slots")
    sv = binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=max_batch, n_slots=slots)
    try:
        t0 = binding.seismic_server_clock(sv)
        first = binding.seismic_server_submit_batch(sv, binding.host_csr(qs.row_ptr, qs.words, qs.dim),
                                                    t0 + _arrivals(qs.n_rows, rate, 1))
        binding.seismic_server_wait_all(sv, 120.0)
        ids, sc, lat = binding.seismic_server_results(sv, first, qs.n_rows, 10)
        st = binding.seismic_server_stats(sv)
    finally:
        binding.seismic_server_free(sv)
    _log(f"  stats {st}; latency p50 {np.percentile(lat, 50) * 1e3:.3f} ms, p99 {np.percentile(lat, 99) * 1e3:.3f} ms")
    assert st["submitted"] == st["completed"] == qs.n_rows
    assert st["batches"] > 1 and st["max_inflight"] <= slots * max_batch
    assert st["max_busy_slots"] <= slots
    if rate >= 100000.0:
        # arrivals far faster than one batch completes: batches overlapped on the device
        assert st["max_busy_slots"] >= 2, st
    assert (lat > 0).all()
    r = ref.pruned_search(qs, 10, 10, 0.8, c_cap=10)
    assert np.array_equal(ids, r["ids"]) and np.array_equal(sc, r["scores"])
    # the same queries alone, one search call each
    for i in range(0, qs.n_rows, 40):
        a_ids, a_sc = ix.search(to_device_csr(qs.subset([i])), 10, 10, 0.8)
        assert np.array_equal(as_u32(a_ids)[0], ids[i]) and np.array_equal(a_sc.cpu().numpy()[0], sc[i])


def test_served_learned_probe_equals_batch_search(idx):
    docs, qs, ix, ref = idx
    rng = np.random.default_rng(5)
    p = np.zeros(512, np.float32)
    p[:449] = rng.normal(0, 0.5, 449)
    p[320:384] = np.abs(p[320:384])
    w = P.to_device(P.bf16_bits(p))
    sv = binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=100, n_slots=3, probe=w, probe_tau=0.0)
    try:
        t0 = binding.seismic_server_clock(sv)
        first = binding.seismic_server_submit_batch(sv, binding.host_csr(qs.row_ptr, qs.words, qs.dim),
                                                    t0 + _arrivals(qs.n_rows, 50000.0, 2))
        binding.seismic_server_wait_all(sv, 120.0)
        ids, sc, _ = binding.seismic_server_results(sv, first, qs.n_rows, 10)
    finally:
        binding.seismic_server_free(sv)
    b_ids, b_sc = ix.search(to_device_csr(qs), 10, 10, 0.8, probe=w, probe_tau=0.0)
    assert np.array_equal(ids, as_u32(b_ids)) and np.array_equal(sc, b_sc.cpu().numpy())


def test_server_submit_poll_and_errors(idx):
    docs, qs, ix, ref = idx
    sv = binding.seismic_server_create(ix.handle, 5, 10, 0.8, max_batch=8, n_slots=2)
    try:
        tickets = [binding.seismic_server_submit(sv, qs.words[qs.row_ptr[i]:qs.row_ptr[i + 1]]) for i in range(20)]
        assert tickets == list(range(20))
        binding.seismic_server_wait_all(sv, 60.0)
        r = ref.pruned_search(qs.subset(range(20)), 5, 10, 0.8, c_cap=10)
        for i, t in enumerate(tickets):
            got = binding.seismic_server_poll(sv, t, 5)
            assert got is not None and np.array_equal(got[0], r["ids"][i]) and got[2] > 0
        bad = np.array([7 | (0x3C00 << 16), 5 | (0x3C00 << 16)], dtype=np.uint32)  # unsorted
        with pytest.raises(SeismicError):
            binding.seismic_server_submit(sv, bad)
        with pytest.raises(SeismicError):
            binding.seismic_server_submit(sv, bad[:1], not_before=-1.0)  # not_before decreased
        empty = binding.seismic_server_submit(sv, np.zeros(0, np.uint32), not_before=1e9 * 0)
        binding.seismic_server_wait_all(sv, 60.0)
        ids, sc, _ = binding.seismic_server_poll(sv, empty, 5)
        assert (ids == 0xFFFFFFFF).all() and np.isneginf(sc).all()
    finally:
        binding.seismic_server_free(sv)
    with pytest.raises(SeismicError):
        binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=8, n_slots=0)


def _max_reservation(ix, k, cut):
    """One query's largest scratch reservation (the header's formula)."""
    return 4 * binding.MAX_QUERY_NNZ + 16 * k + 8 * cut * ix.info()["max_blocks_per_list"]


def test_admission_defers_and_never_drops(idx):
    """Host-forced admission failures and a scratch budget of three queries:
    queries wait in the queue (deferred) and are all served, in order, with
    the oracle's results; the reserved scratch never exceeds the budget."""
    docs, qs, ix, ref = idx
    n = 200
    sub = qs.subset(range(n))
    budget = 3 * _max_reservation(ix, 10, 10)
    _log(f"[serve] {n} queries, 7 injected admission failures, scratch budget {budget} bytes")
    sv = binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=64, n_slots=4, scratch_bytes=budget,
                                       inject_admission_failures=7)
    try:
        first = binding.seismic_server_submit_batch(sv, binding.host_csr(sub.row_ptr, sub.words, sub.dim))
        binding.seismic_server_wait_all(sv, 120.0)
        ids, sc, lat = binding.seismic_server_results(sv, first, n, 10)
        st = binding.seismic_server_stats(sv)
    finally:
        binding.seismic_server_free(sv)
    _log(f"  stats {st}")
    assert st["completed"] == n and st["deferred_admissions"] >= 7
    assert 0 < st["peak_scratch_bytes"] <= budget
    # every reservation holds at least the result, top-k and block-order parts
    least = 16 * 10 + 8 * 10 * ix.info()["max_blocks_per_list"]
    assert st["max_inflight"] <= budget // least
    r = ref.pruned_search(sub, 10, 10, 0.8, c_cap=10)
    assert np.array_equal(ids, r["ids"]) and np.array_equal(sc, r["scores"])
    with pytest.raises(SeismicError):  # a budget below one query's reservation
        binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=8, n_slots=1,
                                      scratch_bytes=_max_reservation(ix, 10, 10) - 1)


def test_release_keeps_the_store_bounded(idx):
    """Waves of queries served and released: the server holds no request
    after each release, released tickets are refused, later tickets keep
    counting and their results are still right."""
    docs, qs, ix, ref = idx
    sv = binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=64, n_slots=2)
    try:
        for wave in range(4):
            rows = range(wave * 100, wave * 100 + 100)
            sub = qs.subset(rows)
            first = binding.seismic_server_submit_batch(sv, binding.host_csr(sub.row_ptr, sub.words, sub.dim))
            assert first == wave * 100
            binding.seismic_server_wait_all(sv, 60.0)
            ids, sc, _ = binding.seismic_server_results(sv, first, 100, 10)
            r = ref.pruned_search(sub, 10, 10, 0.8, c_cap=10)
            assert np.array_equal(ids, r["ids"]) and np.array_equal(sc, r["scores"])
            assert binding.seismic_server_stats(sv)["held"] == 100
            assert binding.seismic_server_release(sv, first + 100) == first + 100
            assert binding.seismic_server_stats(sv)["held"] == 0
            with pytest.raises(SeismicError):
                binding.seismic_server_poll(sv, first, 10)
        with pytest.raises(SeismicError):
            binding.seismic_server_release(sv, 10**6)  # beyond the last ticket
        assert binding.seismic_server_stats(sv)["completed"] == 400
    finally:
        binding.seismic_server_free(sv)
