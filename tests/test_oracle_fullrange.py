"""Pins of the oracle outside the value range where its sums are exact:
documents and queries with fp16 values over the whole positive range
(subnormals and values above 64 included).  There fp64 sums are rounded, so
scores are checked against exact rational arithmetic within the tolerance
the method's results are held to (1e-5 relative), and ties closer than that
are counted, not asserted."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_check import _bound_inputs, _bound_violations
from tests import tiny_index

REL = 1e-5


def _exact_scores(docs, q_terms, q_vals):
    """Exact <q, d> of every document as Fractions."""
    qd = {int(t): Fraction(float(v)) for t, v in zip(q_terms, q_vals)}
    out = []
    for d in range(docs.n_rows):
        t, v = docs.row(d)
        out.append(sum((qd[int(a)] * Fraction(float(b)) for a, b in zip(t, v) if int(a) in qd), Fraction(0)))
    return out


@pytest.fixture(scope="module")
def wide():
    docs = synth.wide_values(synth.generate(1500, seed=9, stream=0, mean=30.0, lo=2, hi=80, dim=300), seed=9)
    qs = synth.wide_values(synth.generate(40, seed=9, stream=1, mean=12.0, lo=1, hi=40, dim=300), seed=10)
    return docs, qs


def test_inputs_span_the_fp16_range(wide):
    docs, qs = wide
    v = docs.values().astype(np.float64)
    assert v.min() < 2.0 ** -14 and v.max() > 2.0 ** 10  # subnormals and large values
    assert not oracle.value_range_ok(docs) and not oracle.value_range_ok(qs)


def test_exact_topk_against_rationals(wide):
    """Every score the oracle returns is the exact inner product within one
    fp32 rounding (plus the fp64 sum's error), and its top-k is the exact
    top-k by rational arithmetic except where two scores are within 1e-5."""
    docs, qs = wide
    k = 10
    ids, sc = oracle.exact_topk(docs, qs, k)
    worst, near = 0.0, 0
    for q in range(qs.n_rows):
        t, v = qs.row(q)
        ex = _exact_scores(docs, t, v)
        for j in range(k):
            if ids[q, j] == 0xFFFFFFFF:
                continue
            e = ex[int(ids[q, j])]
            worst = max(worst, abs(float(Fraction(float(sc[q, j])) - e) / e))
        order = sorted((d for d in range(docs.n_rows) if ex[d] > 0), key=lambda d: (-ex[d], d))[:k]
        if list(ids[q][ids[q] != 0xFFFFFFFF]) != order:
            # allowed only where the exact scores at the differing places are within REL
            got = [ex[int(d)] for d in ids[q] if d != 0xFFFFFFFF]
            want = [ex[d] for d in order]
            assert len(got) == len(want)
            for a, b in zip(got, want):
                assert abs(a - b) <= REL * max(a, b), (q, float(a), float(b))
            near += 1
    print(f"max relative score error {worst:.3e}; queries with a near-tie swap {near}")
    assert worst <= 2.0 ** -23


def test_summary_bounds_at_full_range(wide):
    """The summary bounds hold for wide-range blocks too (with one
    rounding's slack): r_j <= <q, phi(B_j)> and the gap bounds."""
    from paper_2509_24815_amd import Index
    docs, qs = wide
    buf = Index.build(docs, lam=120, beta=12, gamma=0.4, seed=2).serialize()
    ref = oracle.Index(buf)
    assert ref.check(clustering=True) == ""
    ix = tiny_index.read(buf)
    rows = tiny_index._rows(ix["docs"])
    cache = {}
    n = 0
    for qi in range(qs.n_rows):
        qt, qv = qs.row(qi)
        qmax = float(qv.astype(np.float64).max())
        for t in qt[:4]:
            t = int(t)
            if t not in ix["lists"]:
                continue
            r, _ = ref.summary_scores(qt, qv, t)
            phi_dot, phi_s_dot, phi_l1, delta, q_sum, _ = _bound_inputs(ix, qt, qv, t, cache, rows)
            assert _bound_violations(r, phi_dot, phi_s_dot, qmax, phi_l1, delta, q_sum, 0.4) == []
            n += len(r)
    ref.close()
    assert n > 100
