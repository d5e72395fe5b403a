"""Pins of the oracle's learned block probe (not part of the paper, so there
is no published value to compare with): the quantizers against an
independent integer bf16 rounding and hand-worked boundaries, the logit
against an independent numpy forward pass, the backward pass against finite
differences, Adam's first step against its closed form, and the traversal
rule against hand-traced indexes and against the plain rule in its special
cases."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests.indexfile import write_index

H, IN = mlp.H, mlp.IN


def bits(x):
    return mlp.float_to_bf16_bits(np.asarray(x, dtype=np.float32))


def probe_words(W1=None, b1=None, w2=None, b2=0.0):
    p = mlp.pack(np.zeros((H, IN)) if W1 is None else W1, np.zeros(H) if b1 is None else b1,
                 np.zeros(H) if w2 is None else w2, b2)
    return bits(p)


# ---------------------------------------------------------------- quantizers

def test_bf16_rounding_two_ways():
    """frexp/rint rounding equals integer rounding of the fp32 bit pattern."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.lognormal(0, 3, 20000), [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 255.5, 2.0 ** -8]])
    x = x.astype(np.float32).astype(np.float64)
    a = mlp.bf16_round(x)
    b = mlp.bf16_bits_to_float(bits(x))
    assert np.array_equal(a, b)
    assert mlp.bf16_round(1 + 2 ** -8) == 1.0                        # tie -> even
    assert mlp.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6            # tie -> even (up)
    assert mlp.bf16_round(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7     # above the tie


def test_oracle_quantizers_match_their_definition():
    xs = np.array([0.0, -1.0, 2.0 ** -9, 2.0 ** -8 * (1 - 2 ** -10), 2.0 ** -8, 0.3, 15.9, 16.0, 17.0,
                   200.0, 255.0, 300.0, 1 + 2 ** -8])
    f = oracle.probe_quantize(xs, 0)
    b03 = float(mlp.bf16_round(0.3))
    assert list(f) == [0.0, 0.0, 0.0, 2.0 ** -8, 2.0 ** -8, b03, 15.875, 16.0, 16.0, 16.0, 16.0, 16.0, 1.0]
    h = oracle.probe_quantize(xs, 1)
    assert list(h) == [0.0, 0.0, 0.0, 2.0 ** -8, 2.0 ** -8, b03, 15.875, 16.0, 17.0, 200.0, 255.0, 256.0, 1.0]
    assert np.array_equal(mlp.quantize_hidden(xs), h)
    w = np.array([0x7FC0, 0x3900, 0x3980, 0x3F80, 0x4180, 0x4200, 0xC200, 0xB980, 0x8000], dtype=np.float64)
    s = oracle.probe_quantize(w, 2)
    assert list(s) == [0.0, 0.0, 2.0 ** -12, 1.0, 16.0, 16.0, -16.0, -(2.0 ** -12), 0.0]
    assert np.array_equal(mlp.sanitize(mlp.bf16_bits_to_float(w.astype(np.uint16))), s)


# --------------------------------------------------------------------- logit

def _numpy_features(r, h0, nd, nq, ci):
    def q(x):
        y = np.where(x > 0, mlp.bf16_round(np.where(x > 0, x, 1.0)), 0.0)
        y = np.where(y < 2.0 ** -8, 0.0, y)
        return np.minimum(y, 16.0)
    r = r.astype(np.float64)
    return np.stack([q(r / 16.0), q(r / h0.astype(np.float64)), q(nd / 64.0), q(nq / 64.0), q(ci / 8.0)], 1)


def test_logit_matches_numpy_forward_exactly():
    rng = np.random.default_rng(1)
    n = 5000
    r = rng.lognormal(1.5, 1.0, n).astype(np.float32)
    h0 = rng.lognormal(2.5, 0.5, n).astype(np.float32)
    nd = rng.integers(1, 3000, n).astype(np.uint32)
    nq = rng.integers(1, 400, n).astype(np.int32)
    ci = rng.integers(0, 20, n).astype(np.int32)
    raw = np.concatenate([rng.normal(0, 0.7, H * IN + 2 * H + 1), np.zeros(512 - mlp.N_USED)])
    raw[:7] = [40.0, -40.0, 1e-5, -1e-5, np.nan, 2.0 ** -12, 0.0]  # clamp / flush cases
    pw = bits(raw)
    feat, z = oracle.probe_eval(pw, r, h0, nd, nq, ci)
    f_np = _numpy_features(r, h0, nd, nq, ci)
    assert np.array_equal(feat, f_np)
    W1, b1, w2, b2 = mlp.unpack(mlp.sanitize(mlp.bf16_bits_to_float(pw)))
    z_np = mlp.quantize_hidden(f_np @ W1.T + b1) @ w2 + b2
    assert np.array_equal(z, z_np)  # both sums are exact in fp64
    assert (z > 0).any() and (z < 0).any()


def test_logit_special_cases():
    """Zero weights give z = b2; a single path gives z = q(f_i) * w + b2."""
    one = np.zeros(H)
    one[0] = 1.0
    for b2 in (0.5, -3.0):
        _, z = oracle.probe_eval(probe_words(b2=b2), [5.0], 2.0, 10, 7, 3)
        assert z[0] == b2
    for i, expect in enumerate([5.0 / 16, mlp.bf16_round(5.0 / 3.0), 2.0 ** -3 * 1.25, 7 / 64, 3 / 8]):
        W1 = np.zeros((H, IN))
        W1[0, i] = 1.0
        _, z = oracle.probe_eval(probe_words(W1=W1, w2=one, b2=-0.25), [5.0], 3.0, 10, 7, 3)
        assert z[0] == mlp.bf16_round(expect) - 0.25


# ------------------------------------------------------------ backward / Adam

def _random_problem(seed, n=64):
    rng = np.random.default_rng(seed)
    p = np.zeros(512)
    p[:mlp.N_USED] = rng.normal(0, 0.5, mlp.N_USED)
    f = rng.uniform(0.05, 3.0, (n, IN))
    y = rng.integers(0, 2, n).astype(np.uint8)
    y[:3] = 255  # not samples
    wt = rng.uniform(0.5, 3.0, n)
    return p, f, y, wt


def _fd_grad(p, f, y, wt, eps=1e-6):
    fd = np.zeros(512)
    for j in range(mlp.N_USED):
        e = np.zeros(512)
        e[j] = eps
        fd[j] = (mlp.loss_only(p + e, f, y, wt) - mlp.loss_only(p - e, f, y, wt)) / (2 * eps)
    return fd


def test_backward_matches_finite_differences():
    p, f, y, wt = _random_problem(2)
    W1, b1, _, _ = mlp.unpack(p)
    a = f @ W1.T + b1
    assert np.min(np.abs(a)) > 1e-4  # no sample sits on a ReLU kink
    loss, g, s, n = mlp.forward_backward(p, f, y, wt, quantize=False)
    assert n == 61 and np.isclose(loss, mlp.loss_only(p, f, y, wt))
    fd = _fd_grad(p, f, y, wt)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7)
    assert (g[mlp.N_USED:] == 0).all() and (s >= np.abs(g) - 1e-12).all()


def test_finite_differences_catch_a_planted_mistake():
    """The same check rejects a gradient whose ReLU mask was dropped."""
    p, f, y, wt = _random_problem(3)
    _, g, _, _ = mlp.forward_backward(p, f, y, wt, quantize=False)
    W1, b1, w2, b2 = mlp.unpack(p)
    valid = y != 255
    z = np.maximum(f @ W1.T + b1, 0) @ w2 + b2
    dz = wt * (mlp.sigmoid(z) - (y == 1))
    wrong = g.copy()
    wrong[H * IN:H * IN + H] = (dz[valid][:, None] * w2[None, :]).sum(0)  # mask dropped
    fd = _fd_grad(p, f, y, wt)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7)
    assert not np.allclose(wrong, fd, rtol=1e-5, atol=1e-7)


def test_quantized_forward_gradient_is_straight_through():
    """With hidden rounding the gradient is the smooth formula evaluated at
    the rounded activations; when every activation is a bf16 value below 256
    rounding changes nothing and both coincide."""
    rng = np.random.default_rng(4)
    p = np.zeros(512)
    p[0:IN] = 1.0                                   # unit 0: a = sum of the features
    p[H * IN + H:H * IN + 2 * H] = 0.5
    f = np.round(rng.uniform(0.5, 2.0, (32, IN)) * 4) / 4   # quarters: sums below 16 are bf16 values
    y = rng.integers(0, 2, 32).astype(np.uint8)
    wt = np.ones(32)
    l0, g0, _, _ = mlp.forward_backward(p, f, y, wt, quantize=False)
    l1, g1, _, _ = mlp.forward_backward(p, f, y, wt, quantize=True)
    assert l0 == l1 and np.array_equal(g0, g1)
    p[0:IN] = 1.0 + 2 ** -7                         # now a is not a bf16 value: h is rounded
    l2, g2, _, _ = mlp.forward_backward(p, f, y, wt, quantize=True)
    l3, _, _, _ = mlp.forward_backward(p, f, y, wt, quantize=False)
    assert l2 != l3


def test_adam_first_step_closed_form():
    """First Adam step: m_hat = g and v_hat = g^2, so the update is
    -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    g = np.zeros(512)
    g[:mlp.N_USED] = rng.normal(0, 1, mlp.N_USED)
    w0 = np.zeros(512)
    w0[:mlp.N_USED] = rng.normal(0, 1, mlp.N_USED)
    w, m, v = mlp.adam(w0, np.zeros(512), np.zeros(512), g * 10, 10, 1, lr=0.01)
    assert np.allclose(w - w0, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ----------------------------------------------------------------- traversal

def _counterexample():
    """k = 1; cut order (a, b).  List a: X1 (r 10, doc score 5), X2 (r 6,
    doc 11); list b: Z (r 10.5, doc 12), one document, n_q = 2."""
    a, b = 0, 1
    docs = synth.make_csr([{a: 2.5}, {a: 5.5}, {b: 12.0}], dim=4)
    lists = {
        a: [dict(docs=[0], summary=[(a, 0)], m=5.0, delta=0.0),
            dict(docs=[1], summary=[(a, 0)], m=3.0, delta=0.0)],
        b: [dict(docs=[2], summary=[(b, 0)], m=10.5, delta=0.0)],
    }
    qs = synth.make_csr([{a: 2.0, b: 1.0}], dim=4)
    return oracle.Index(write_index(docs, lists, dim=4)), qs


def _single_path(i, w, b2, b1=0.0):
    W1 = np.zeros((H, IN))
    W1[0, i] = w
    bb = np.zeros(H)
    bb[0] = b1
    w2 = np.zeros(H)
    w2[0] = 1.0
    return probe_words(W1=W1, b1=bb, w2=w2, b2=b2)


@pytest.mark.parametrize("feature,w,b2,b1,tau,evaluates", [
    # f1 = q(10.5 / 11) = 244/256 (rounded down from 0.95454...); list b starts with heap min 11
    (1, 1.0, -0.9375, 0.0, 0.0, True),
    (1, 1.0, -244 / 256, 0.0, 0.0, True),          # z = 0 >= tau: evaluated
    (1, 1.0, -245 / 256, 0.0, 0.0, False),
    # f0 = 10.5 / 16
    (0, 1.0, -0.65625, 0.0, 0.0, True),
    (0, 1.0, -169 / 256, 0.0, 0.0, False),
    # f2 = 1 document / 64; a stored weight of 32 acts as 16
    (2, 16.0, -0.25, 0.0, 0.0, True),
    (2, 32.0, -0.375, 0.0, 0.0, False),
    # f3 = n_q / 64 = 2 / 64
    (3, 8.0, -0.25, 0.0, 0.0, True),
    (3, 8.0, -66 / 256, 0.0, 0.0, False),
    # f4 = cut rank 1 / 8
    (4, 2.0, -0.25, 0.0, 0.0, True),
    (4, 2.0, -0.25, 0.0, 2.0 ** -20, False),
    # hidden rounding: a = 1 + 2^-8 rounds to 1 (tie to even), so z = 0 < 2^-20
    (2, 0.25, -1.0, 1.0, 2.0 ** -20, False),
    (2, 0.25, -1.0, 1.0, 0.0, True),
])
def test_hand_traced_learned_list(feature, w, b2, b1, tau, evaluates):
    """List a starts with an empty heap: the heap_factor rule (hf 1) evaluates
    X1 then X2 (6 >= 5), heap min 11.  List b starts with a full heap, so the
    probe decides Z with features (10.5/16, q(10.5/11), 1/64, 2/64, 1/8)."""
    ix, qs = _counterexample()
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0, probe=_single_path(feature, w, b2, b1), tau=tau)
    assert list(r["hmin"][0]) == [-1.0, 11.0]
    if evaluates:
        assert r["ids"][0, 0] == 2 and r["scores"][0, 0] == 12.0 and list(r["prefix"][0]) == [2, 1]
    else:
        assert r["ids"][0, 0] == 1 and r["scores"][0, 0] == 11.0 and list(r["prefix"][0]) == [2, 0]
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["prune_tests"] == 1 + 1  # X2 by the plain rule, Z by the probe


def test_learned_list_ignores_heap_factor():
    """Once the probe owns a list, heap_factor plays no part in it: with
    hf 0.01 the plain rule would skip Z (10.5 * 0.01 < 11)."""
    ix, qs = _counterexample()
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0, probe=probe_words(b2=1.0), tau=0.0)
    assert r["ids"][0, 0] == 2
    r0 = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0)
    assert r0["ids"][0, 0] == 1  # plain rule: Z skipped


@pytest.fixture(scope="module")
def small():
    docs = synth.docs(4000, seed=5)
    qs = synth.queries(120, seed=5)
    from paper_2509_24815_amd import Index  # host build only, no GPU
    ix = Index.build(docs, lam=400, beta=20, gamma=0.4, seed=1)
    return docs, qs, oracle.Index(ix.serialize())


def test_keep_all_probe_equals_no_pruning(small):
    """A probe that keeps every block, with no pruning in the lists it does
    not own (hf = +inf), is exhaustive over the cut lists."""
    docs, qs, ref = small
    a = ref.pruned_search(qs, 10, 10, float("inf"), c_cap=10)
    b = ref.pruned_search(qs, 10, 10, float("inf"), c_cap=10, probe=probe_words(b2=1.0), tau=0.0)
    assert (b["hmin"] >= 0).sum() > 500  # most lists were owned by the probe
    for key in ("ids", "scores", "prefix"):
        assert np.array_equal(a[key], b[key])


def test_stop_all_probe_equals_cut_before_first_full_list(small):
    """A probe that rejects every block ends the search at the first list
    that starts with a full heap: the result is the plain search with the
    cut shortened to that list."""
    docs, qs, ref = small
    b = ref.pruned_search(qs, 10, 10, 0.8, c_cap=10, probe=probe_words(b2=-1.0), tau=0.0)
    checked = 0
    for i in range(qs.n_rows):
        full = np.nonzero(b["hmin"][i] >= 0)[0]
        c = int(full[0]) if len(full) else 10
        if c == 0:
            continue
        sub = qs.subset([i])
        a = ref.pruned_search(sub, 10, c, 0.8, c_cap=10)
        assert np.array_equal(a["ids"][0], b["ids"][i]) and np.array_equal(a["scores"][0], b["scores"][i])
        assert (b["prefix"][i][c:] == 0).all()
        checked += len(full) > 0
    assert checked > 50
