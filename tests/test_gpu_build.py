"""GPU index build through the C ABI: byte for byte the host builder's
index, over fixed and proportional caps, tiny and tie-heavy collections, and
accepted by the oracle's structure check; the device-resident build (rows
already on the device, index left there) gives the same bytes, searches as
the oracle does, and refuses invalid rows."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _same(docs, **kw):
    h = Index.build(docs, seed=kw.get("seed", 0), **{k: v for k, v in kw.items() if k != "seed"})
    g = Index.build_gpu(docs, seed=kw.get("seed", 0), verbose=True, **{k: v for k, v in kw.items() if k != "seed"})
    hb, gb = h.serialize(), g.serialize()
    assert hb.size == gb.size
    if not np.array_equal(hb, gb):
        diff = np.nonzero(hb != gb)[0]
        raise AssertionError(f"{diff.size} bytes differ, first at {diff[0]}")
    return g


@pytest.mark.parametrize("n,lam,beta,gamma,alpha", [
    (20000, 500, 25, 0.4, 0.0),
    (30000, 300, 10, 1.0, 0.0),
    (30000, 300, 10, 0.05, 0.0),
    (50000, 2000, 80, 0.7, 0.3),
    (5000, 100000, 10, 0.4, 0.0),     # nothing truncated
    (40000, 150, 150, 0.4, 0.0),      # a block per document in full lists
])
def test_gpu_build_equals_host_build(n, lam, beta, gamma, alpha):
    _log(f"[gpu build] n={n} lambda={lam} beta={beta} gamma={gamma} alpha={alpha}")
    docs = synth.docs(n, seed=n % 101)
    g = _same(docs, lam=lam, beta=beta, gamma=gamma, alpha=alpha, seed=7)
    assert oracle.Index(g.serialize()).check(clustering=True, term_stride=5) == ""


def test_gpu_build_ties_and_tiny_collections():
    # every value equal: ties at every selection and summary boundary
    rows = [{t: 1.0 for t in range(i % 7, 60 + i % 13, 1 + i % 3)} for i in range(3000)]
    docs = synth.make_csr(rows, dim=128)
    _same(docs, lam=200, beta=20, gamma=0.5)
    # a handful of documents, some columns with a single entry
    small = synth.make_csr([{0: 2.0, 5: 1.0}, {5: 3.0}, {1: 0.5, 5: 0.5}, {7: 1.0}], dim=16)
    _same(small, lam=2, beta=2, gamma=0.4)


def _on_device(docs):
    import torch
    torch.cuda.set_device(0)
    return to_device_csr(docs)


@pytest.mark.parametrize("n,lam,beta,gamma,alpha", [
    (20000, 500, 25, 0.4, 0.0),
    (50000, 2000, 80, 0.7, 0.3),
    (40000, 150, 150, 0.4, 0.0),      # a block per document in full lists
    (40000, 3000, 200, 0.4, 0.0),     # several documents chunks per column
])
def test_device_build_equals_host_build(n, lam, beta, gamma, alpha):
    """Built from device rows and left on the device: the same bytes as
    the host build, and the same search results as the oracle on them."""
    _log(f"[device build] n={n} lambda={lam} beta={beta} gamma={gamma} alpha={alpha}")
    docs = synth.docs(n, seed=n % 89)
    h = Index.build(docs, lam=lam, beta=beta, gamma=gamma, alpha=alpha, seed=5)
    dv = Index.build_device(_on_device(docs), lam=lam, beta=beta, gamma=gamma, alpha=alpha, seed=5)
    info = dv.info()
    assert info["on_device"] == 1 and info["nnz"] == docs.nnz and info["n_docs"] == n
    hb, db = h.serialize(), dv.serialize()
    assert hb.size == db.size
    if not np.array_equal(hb, db):
        diff = np.nonzero(hb != db)[0]
        raise AssertionError(f"{diff.size} bytes differ, first at {diff[0]}")
    ref = oracle.Index(hb)
    qs = synth.queries(150, seed=n % 13)
    r = ref.pruned_search(qs, 10, 10, 0.8, c_cap=10)
    gpu = dv.search(to_device_csr(qs), 10, 10, 0.8, stats=True, prefix_stride=10)
    assert not compare_with_oracle(gpu, r, 10, 10)
    e_ids, e_sc = dv.exact(to_device_csr(qs), 10)  # column lists built on the device
    o_ids, o_sc = oracle.exact_topk(docs, qs, 10)
    assert np.array_equal(as_u32(e_ids), o_ids) and np.array_equal(e_sc.cpu().numpy(), o_sc)


def test_device_build_edges_and_errors():
    import torch
    # a handful of documents, some columns with a single entry, an empty row
    small = synth.make_csr([{0: 2.0, 5: 1.0}, {}, {5: 3.0}, {1: 0.5, 5: 0.5}, {7: 1.0}], dim=16)
    h = Index.build(small, lam=2, beta=2, gamma=0.4)
    dv = Index.build_device(_on_device(small), lam=2, beta=2, gamma=0.4)
    assert np.array_equal(h.serialize(), dv.serialize())
    with pytest.raises(SeismicError) as e:
        dv.upload(0)
    assert e.value.code == binding.ESTATE
    # invalid rows are refused on the device before anything reads them
    good = synth.docs(300, seed=2)
    for name, mutate in [("unsorted", lambda w, rp: w.__setitem__(slice(int(rp[3]), int(rp[3]) + 2),
                                                                 w[int(rp[3]):int(rp[3]) + 2][::-1].copy())),
                         ("term >= dim", lambda w, rp: w.__setitem__(int(rp[5]), np.uint32(0x3C00FFFF))),
                         ("zero value", lambda w, rp: w.__setitem__(int(rp[7]), w[int(rp[7])] & np.uint32(0xFFFF)))]:
        w = good.words.copy()
        mutate(w, good.row_ptr)
        bad = synth.CSR(good.row_ptr.copy(), w, good.dim)
        _log(f"[device build] invalid rows: {name}")
        with pytest.raises(SeismicError) as e:
            Index.build_device(_on_device(bad), lam=100, beta=10, gamma=0.4)
        assert e.value.code == binding.EINVAL
    rp = torch.from_numpy(good.row_ptr.astype(np.int64)).cuda()
    words = torch.from_numpy(good.words.view(np.int32)).cuda()
    short = binding.device_csr(rp, words[:-1], good.dim)  # row_ptr ends past nnz
    with pytest.raises(SeismicError) as e:
        Index.build_device(short, lam=100, beta=10, gamma=0.4)
    assert e.value.code == binding.EINVAL


def test_gpu_builds_refuse_lists_beyond_their_capacity():
    # term 0 in every document: its list gets 1025 blocks, one more than the
    # GPU build handles; neither GPU entry point falls back silently
    rows = [{0: 0.02, d + 1: 1.0 + (d % 7) * 0.25} for d in range(3000)]
    docs = synth.make_csr(rows, dim=3001)
    with pytest.raises(SeismicError) as e:
        Index.build_gpu(docs, lam=3000, beta=1025, gamma=0.4)
    assert e.value.code == binding.EINVAL
    with pytest.raises(SeismicError) as e:
        Index.build_device(_on_device(docs), lam=3000, beta=1025, gamma=0.4)
    assert e.value.code == binding.EINVAL
    assert Index.build(docs, lam=3000, beta=1025, gamma=0.4).info()["max_blocks_per_list"] == 1025
