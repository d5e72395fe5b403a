"""Host-side tests of libseismic: exported symbols, the index builder checked
by the oracle, the serialized format and error paths.  No GPU needed."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding, hot_list_order

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seismic.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared_functions()
    assert "seismic_search_batch" in names and "exact_topk" in names and "seismic_build_index" in names
    for n in names:
        assert hasattr(lib, n), n


@pytest.fixture(scope="module")
def small():
    docs = synth.generate(6000, seed=11, stream=0, mean=40.0, lo=5, hi=120, dim=2000)
    ix = Index.build(docs, lam=150, beta=12, gamma=0.4, seed=3, n_threads=4)
    return docs, ix


def test_build_matches_indexing_algorithm(small):
    """Every list, block, centroid assignment, summary and code re-derived by
    the oracle from the forward index."""
    docs, ix = small
    o = oracle.Index(ix.serialize())
    info = ix.info()
    assert o.n_docs == docs.n_rows and o.nnz == docs.nnz and o.n_blocks == info["n_blocks"]
    assert o.check(clustering=True) == ""


def test_build_is_deterministic_and_thread_independent(small):
    docs, ix = small
    other = Index.build(docs, lam=150, beta=12, gamma=0.4, seed=3, n_threads=1)
    assert np.array_equal(ix.serialize(), other.serialize())
    reseeded = Index.build(docs, lam=150, beta=12, gamma=0.4, seed=4, n_threads=4)
    assert not np.array_equal(ix.serialize(), reseeded.serialize())


def test_save_load_roundtrip(small, tmp_path):
    _, ix = small
    p = str(tmp_path / "ix.bin")
    ix.save(p)
    back = Index.load(p)
    assert np.array_equal(back.serialize(), ix.serialize())
    assert oracle.Index(p).n_blocks == ix.info()["n_blocks"]


def test_corrupt_index_is_rejected(small, tmp_path):
    _, ix = small
    buf = ix.serialize()
    p = str(tmp_path / "trunc.bin")
    buf[: len(buf) // 2].tofile(p)
    with pytest.raises(SeismicError) as e:
        Index.load(p)
    assert e.value.code == binding.EFORMAT
    bad = buf.copy()
    bad[0] = ord("X")
    p2 = str(tmp_path / "magic.bin")
    bad.tofile(p2)
    with pytest.raises(SeismicError) as e:
        Index.load(p2)
    assert e.value.code == binding.EFORMAT
    with pytest.raises(SeismicError) as e:
        Index.load(str(tmp_path / "missing.bin"))
    assert e.value.code == binding.EIO


def test_invalid_build_inputs():
    docs = synth.make_csr([{3: 1.0, 1: 2.0}], dim=8)  # make_csr sorts terms
    Index.build(docs, 10, 2, 0.5)
    w = docs.words.copy()
    w[[0, 1]] = w[[1, 0]]  # unsorted terms
    with pytest.raises(SeismicError) as e:
        binding.seismic_build_index(docs.row_ptr, w, 8, 10, 2, 0.5)
    assert e.value.code == binding.EINVAL
    w = docs.words.copy()
    w[0] = (w[0] & 0xFFFF)  # zero value
    with pytest.raises(SeismicError):
        binding.seismic_build_index(docs.row_ptr, w, 8, 10, 2, 0.5)
    with pytest.raises(SeismicError):
        binding.seismic_build_index(docs.row_ptr, docs.words, 2, 10, 2, 0.5)  # term >= dim
    for lam, beta, gamma in ((0, 2, 0.5), (10, 0, 0.5), (10, 2, 0.0), (10, 2, 1.5)):
        with pytest.raises(SeismicError) as e:
            binding.seismic_build_index(docs.row_ptr, docs.words, 8, lam, beta, gamma)
        assert e.value.code == binding.EINVAL


def test_search_requires_device_index(small):
    _, ix = small
    with pytest.raises(SeismicError) as e:
        binding.seismic_workspace_create(ix.handle, 10, 10)
    assert e.value.code == binding.ESTATE
    with pytest.raises(SeismicError) as e:  # block-major copies need the resident index
        ix.copy_lists([0, 1], 1 << 40)
    assert e.value.code == binding.ESTATE
    ix.release_exact()  # nothing to free: no error


def test_hot_list_order():
    # prefix[q, i] blocks of list term[q, i] evaluated; zero prefixes (lists
    # never evaluated, unused positions with any term) do not count
    prefix = np.array([[3, 1, 0], [2, 0, 0], [1, 4, 0]], dtype=np.int16)
    term = np.array([[7, 2, 9], [2, 5, 11], [4, 7, 30000]], dtype=np.int32)
    # totals: 7 -> 7, 2 -> 3, 4 -> 1; ties broken by smaller term id
    assert hot_list_order(prefix, term).tolist() == [7, 2, 4]
    assert hot_list_order(np.array([[1, 1]]), np.array([[9, 3]])).tolist() == [3, 9]
    assert hot_list_order(np.zeros((2, 2)), np.ones((2, 2))).size == 0
    # prefixes above 2^15 arrive as negative int16
    assert hot_list_order(np.array([[-1, 5]], dtype=np.int16), np.array([[1, 2]])).tolist() == [1, 2]


def test_empty_and_degenerate_collections():
    docs = synth.make_csr([{}, {5: 1.0}, {}], dim=16)
    ix = Index.build(docs, 1, 1, 1.0)
    info = ix.info()
    assert info["n_blocks"] == 1 and info["n_postings"] == 1
    assert oracle.Index(ix.serialize()).check() == ""


def test_proportional_caps_reproduce_fig3_and_pass_the_check():
    """Set alpha-MSS in its proportional form (Section 3.4): with alpha 0.4
    each column keeps its ceil(0.4 |L_i|) largest values.  The library's
    build of the Figure "set-sketch" matrix keeps the figure's values
    (column 7 of the figure is defective, ties may break either way), and
    the oracle's structure check accepts it."""
    from tests.test_oracle_sketch import _read_fig3
    before, after = _read_fig3()
    rows = [{int(c): float(v) for c, v in enumerate(r) if v} for r in before]
    docs = synth.make_csr(rows, dim=8)
    ix = Index.build(docs, lam=1000, beta=1, gamma=1.0, seed=0, alpha=0.4)
    ref = oracle.Index(ix.serialize())
    assert ref.check() == ""
    S = ref.sections()
    for c in range(8):
        b0, b1 = int(S["list_off"][c]), int(S["list_off"][c + 1])
        kept = sorted(int(d) for d in S["postings"][S["blk_post_off"][b0]:S["blk_post_off"][b1]])
        nz = np.nonzero(before[:, c])[0]
        assert len(kept) == math.ceil(0.4 * len(nz) - 1e-12)
        if c == 6:
            continue
        assert sorted(before[kept, c]) == sorted(after[:, c][np.nonzero(after[:, c])[0]]), f"column {c + 1}"


def test_proportional_caps_random_collection():
    docs = synth.docs(3000, seed=31)
    ix = Index.build(docs, lam=400, beta=20, gamma=0.4, seed=3, alpha=0.3)
    ref = oracle.Index(ix.serialize())
    assert ref.check(clustering=True) == ""
    # caps: min(lambda, ceil(0.3 n)) per column
    S = ref.sections()
    counts = np.bincount((docs.words & 0xFFFF).astype(np.int64), minlength=docs.dim)
    for t in np.nonzero(counts)[0][::37]:
        b0, b1 = int(S["list_off"][t]), int(S["list_off"][t + 1])
        n = int(S["blk_post_off"][b1] - S["blk_post_off"][b0])
        assert n == min(400, max(1, math.ceil(0.3 * int(counts[t]))))
    with pytest.raises(SeismicError):
        Index.build(docs, lam=400, beta=20, gamma=0.4, alpha=1.5)
