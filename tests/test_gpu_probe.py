"""GPU tests of the learned block probe through the C ABI: learned search,
sample collection, gradients and Adam against the CPU oracle, and what a
trained probe gains over the heap_factor rule."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from paper_2509_24815_amd import Index, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


def _log(msg):
    print(msg, flush=True)


def random_probe(seed, scale=0.6):
    rng = np.random.default_rng(seed)
    p = np.zeros(512, dtype=np.float32)
    p[:mlp.N_USED] = rng.normal(0, scale, mlp.N_USED)
    p[320:384] = np.abs(p[320:384])           # b1 > 0: units active on non-negative features
    p[:3] = [40.0, 1e-5, np.nan]              # clamp, flush and NaN cases of the stored weights
    return mlp.float_to_bf16_bits(p)


@pytest.fixture(scope="module")
def small():
    import torch
    _log("[probe] building a 30k-document index (lambda 600, beta 30)")
    docs = synth.docs(30_000, seed=3)
    qs = synth.queries(200, seed=3)
    ix = Index.build(docs, lam=600, beta=30, gamma=0.4, seed=2)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, ix, ref


@pytest.mark.parametrize("tau", [-2.0, 0.0, 0.5, 3.0])
def test_learned_search_parity(small, tau):
    docs, qs, ix, ref = small
    w = random_probe(7)
    _log(f"[probe parity] tau={tau}")
    r = ref.pruned_search(qs, 10, 10, 0.8, c_cap=10, probe=w, tau=tau)
    ids, sc, pref, cnt, hmin, term = ix.search(to_device_csr(qs), 10, 10, 0.8, trace=True, prefix_stride=10,
                                               probe=P.to_device(w), probe_tau=tau)
    assert not compare_with_oracle((ids, sc, pref, cnt), r, 10, 10)
    assert np.array_equal(hmin.cpu().numpy(), r["hmin"])
    owned = r["hmin"] >= 0
    _log(f"  lists owned by the probe: {owned.sum()}, blocks evaluated {r['counters'][:, 2].sum()}")


def test_learned_search_tau_extremes(small):
    """tau -> -inf evaluates every block of probe-owned lists, tau -> +inf
    none of them."""
    docs, qs, ix, ref = small
    w = P.to_device(random_probe(8))
    base = ix.search(to_device_csr(qs), 10, 10, 0.8, stats=True, prefix_stride=10)
    lo = ix.search(to_device_csr(qs), 10, 10, 0.8, stats=True, prefix_stride=10, probe=w, probe_tau=-1e300)
    hi = ix.search(to_device_csr(qs), 10, 10, 0.8, stats=True, prefix_stride=10, probe=w, probe_tau=1e300)
    e_lo = lo[3].cpu().numpy()[:, 2].sum()
    e_base = base[3].cpu().numpy()[:, 2].sum()
    e_hi = hi[3].cpu().numpy()[:, 2].sum()
    assert e_hi < e_base < e_lo
    r = ref.pruned_search(qs, 10, 10, 0.8, c_cap=10, probe=random_probe(8), tau=-1e300)
    assert not compare_with_oracle(lo, r, 10, 10)


def _cut_terms(qs, i, cut):
    t, v = qs.row(i)
    order = sorted(range(len(t)), key=lambda j: (-float(v[j]), int(t[j])))
    return [int(t[j]) for j in order[:cut]]


def test_collect_matches_oracle(small):
    """Features and labels of every (query, list, block) sample against
    values computed from the serialized index and the oracle."""
    import torch
    docs, qs, ix, ref = small
    sub = qs.subset(range(60))
    q = to_device_csr(sub)
    feat, label, idx = P.collect(ix, q, 60, 10, 10, 0.8, exact_k=10)
    torch.cuda.synchronize()
    _, _, _, _, hmin, term = ix.search(q, 10, 10, 0.8, trace=True, prefix_stride=10)
    r = ref.pruned_search(sub, 10, 10, 0.8, c_cap=10)
    e_ids, _ = oracle.exact_topk(docs, sub, 10)
    S = ref.sections()
    mb = ix.info()["max_blocks_per_list"]
    g_feat = feat.cpu().numpy().view(np.uint16)
    g_lab = label.cpu().numpy()
    g_term = term.cpu().numpy().view(np.uint32)
    n_samples = 0
    for i in range(60):
        cut = _cut_terms(sub, i, 10)
        assert list(g_term[i][:len(cut)]) == cut and (g_term[i][len(cut):] == 0xFFFFFFFF).all()
        tq, vq = sub.row(i)
        qd = dict(zip([int(x) for x in tq], [float(x) for x in vq]))
        for ci in range(10):
            slot0 = (i * 10 + ci) * mb
            if ci >= len(cut) or r["hmin"][i, ci] < 0:
                assert (g_lab[slot0:slot0 + mb] == 255).all()
                continue
            t = cut[ci]
            b0, b1 = int(S["list_off"][t]), int(S["list_off"][t + 1])
            rs, nds = [], []
            for b in range(b0, b1):
                e0, e1 = int(S["blk_sum_off"][b]), int(S["blk_sum_off"][b + 1])
                A = sum(qd.get(int(x), 0.0) for x in S["sum_term"][e0:e1])
                B = sum(qd.get(int(x), 0.0) * int(c) for x, c in zip(S["sum_term"][e0:e1], S["sum_code"][e0:e1]))
                rs.append(np.float32(float(S["blk_m"][b]) * A + float(S["blk_delta"][b]) * B))
                p0, p1 = int(S["blk_post_off"][b]), int(S["blk_post_off"][b + 1])
                nds.append(p1 - p0)
                lab = int(bool(set(S["postings"][p0:p1].tolist()) & set(e_ids[i].tolist())))
                assert g_lab[slot0 + b - b0] == lab
            f, _ = oracle.probe_eval(np.zeros(512, np.uint16), np.array(rs, np.float32), r["hmin"][i, ci],
                                     np.array(nds), len(tq), ci)
            got = mlp.bf16_bits_to_float(g_feat[slot0:slot0 + (b1 - b0), :5])
            assert np.array_equal(got, f), (i, ci)
            assert (g_feat[slot0:slot0 + (b1 - b0), 5:] == 0).all()
            assert (g_lab[slot0 + (b1 - b0):slot0 + mb] == 255).all()
            n_samples += b1 - b0
    assert n_samples == idx.numel() and n_samples > 1000
    _log(f"  {n_samples} samples, {int((label == 1).sum())} positive")


def _grad_problem(seed, n):
    rng = np.random.default_rng(seed)
    raw = np.stack([rng.lognormal(0, 1, n), rng.lognormal(0, 0.5, n), rng.integers(1, 200, n) / 64,
                    rng.integers(1, 200, n) / 64, rng.integers(0, 10, n) / 8], 1)
    f = oracle.probe_quantize(raw.reshape(-1), 0).reshape(n, 5)
    fb = np.zeros((n, 8), np.uint16)
    fb[:, :5] = mlp.float_to_bf16_bits(f)
    lab = (rng.random(n) < 0.2).astype(np.uint8)
    lab[rng.random(n) < 0.1] = 255
    return f, fb, lab


@pytest.mark.parametrize("n,seed", [(3000, 0), (256, 1), (4096, 2)])
def test_grad_matches_oracle(n, seed):
    """Gradient sum of the GPU kernels against the fp64 oracle, element by
    element within the fp32 summation bound (terms + 4 quarters + partials
    + a few roundings per term) times the sum of |terms|."""
    import torch
    f, fb, lab = _grad_problem(seed, n)
    rng = np.random.default_rng(seed + 10)
    order = rng.permutation(n)[: n - n // 7].astype(np.int32)  # a shuffled subset
    w = random_probe(seed + 20, 0.4)
    pw, nw, nwd = 3.0, 0.5, 0.25
    tr = binding.seismic_probe_trainer_create(0, 4096)
    grad = torch.empty(512, dtype=torch.float32, device="cuda")
    stats = torch.empty(4, dtype=torch.float32, device="cuda")
    binding.seismic_probe_grad(tr, torch.from_numpy(fb.view(np.int16)).cuda(), torch.from_numpy(lab).cuda(),
                               torch.from_numpy(order).cuda(), len(order), P.to_device(w), grad, stats, pw, nw, nwd)
    torch.cuda.synchronize()
    binding.seismic_probe_trainer_free(tr)
    fo, lo = f[order], lab[order]
    wt = np.where(lo == 1, pw, nw + nwd * fo[:, 2])
    params = mlp.sanitize(mlp.bf16_bits_to_float(w))
    loss, g_ref, s_ref, cnt = mlp.forward_backward(params, fo, lo, wt, quantize=True)
    g = grad.cpu().numpy().astype(np.float64)
    st = stats.cpu().numpy().astype(np.float64)
    groups = (len(order) + 255) // 256
    bound = (64 + 4 + groups + 8) * U * s_ref + 1e-30
    err = np.abs(g - g_ref)
    _log(f"[grad n={n}] max err / bound = {np.max(err / bound):.3f}; max |g| {np.max(np.abs(g_ref)):.3g}")
    assert (err <= bound).all()
    assert st[1] == cnt and st[2] == int((lo == 1).sum())
    assert abs(st[0] - loss) <= (256 + groups + 16) * U * loss
    assert abs(st[3] - wt[lo != 255].sum()) <= (256 + groups) * U * wt.sum()


def test_adam_matches_oracle():
    import torch
    rng = np.random.default_rng(3)
    master = np.zeros(512, np.float32)
    master[:mlp.N_USED] = rng.normal(0, 0.5, mlp.N_USED)
    g = np.zeros(512, np.float32)
    g[:mlp.N_USED] = rng.normal(0, 3, mlp.N_USED)
    stats = np.array([0, 37, 5, 37], np.float32)
    m_ref, v_ref, w_ref = np.zeros(512), np.zeros(512), master.astype(np.float64)
    dm = torch.from_numpy(master.copy()).cuda()
    dmm = torch.zeros(512, device="cuda")
    dv = torch.zeros(512, device="cuda")
    wout = torch.empty(512, dtype=torch.int16, device="cuda")
    dg = torch.from_numpy(g).cuda()
    ds = torch.from_numpy(stats).cuda()
    lr = 0.01
    for step in (1, 2, 3):
        binding.seismic_probe_adam(dg, ds, dm, dmm, dv, step, wout, lr=lr)
        w_ref, m_ref, v_ref = mlp.adam(w_ref, m_ref, v_ref, g.astype(np.float64), 37, step, lr)
    torch.cuda.synchronize()
    got = dm.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - w_ref) <= 1e-6 * np.abs(w_ref) + 1e-4 * lr)
    bits = wout.cpu().numpy().view(np.uint16)
    assert np.array_equal(bits, mlp.float_to_bf16_bits(dm.cpu().numpy()))
    assert (bits[mlp.N_USED:] == 0).all()


def test_trained_probe_gain(small):
    """Train on samples of one query set, evaluate on another: the loss
    falls, and the learned rule is compared with the heap_factor rule by
    documents scored at equal or better Recall@10 (reported)."""
    import torch
    docs, qs, ix, ref = small
    train_q = synth.queries(400, seed=3, stream=synth.STREAM_PROBE_QUERIES)
    feat, label, idx = P.collect(ix, to_device_csr(train_q), 400, 10, 10, 1.0, exact_k=10)
    w, hist = P.train(feat, label, idx, epochs=8, batch=4096, lr=3e-3, neg_weight_per_doc=0.5, log=_log)
    assert hist[-1] < hist[0]
    qd = to_device_csr(qs)
    e_ids, _ = ix.exact(qd, 10)
    ex = as_u32(e_ids)

    def point(**kw):
        ids, _, _, cnt = ix.search(qd, 10, 10, kw.pop("hf"), stats=True, prefix_stride=10, **kw)
        got = as_u32(ids)
        rec = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(got, ex)])
        return rec, float(cnt.cpu().numpy()[:, 3].mean())

    plain = [(hf,) + point(hf=hf) for hf in (0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0)]
    learned = [(tau,) + point(hf=1.0, probe=w, probe_tau=tau) for tau in (-3, -2, -1, -0.5, 0, 0.5, 1, 2)]
    for p in plain:
        _log(f"  plain hf={p[0]}: recall {p[1]:.4f}, docs {p[2]:.0f}")
    for p in learned:
        _log(f"  learned tau={p[0]}: recall {p[1]:.4f}, docs {p[2]:.0f}")
    recalls = [p[1] for p in learned]
    assert recalls[0] >= recalls[-1]  # lower tau evaluates more

    def cheapest(points, target):
        ok = [p[2] for p in points if p[1] >= target]
        return min(ok) if ok else float("inf")

    for target in (0.93, 0.95):
        a, b = cheapest(plain, target), cheapest(learned, target)
        _log(f"  Recall@10 >= {target}: plain {a:.0f} docs/query, learned {b:.0f} ({100 * (1 - b / a):.1f}% fewer)")
    # the trained probe reaches Recall@10 >= 0.95 scoring fewer documents than the heap_factor rule
    assert cheapest(learned, 0.95) < cheapest(plain, 0.95)
