"""Pins of the oracle's sketching and quantization routines against the
paper's worked example and against properties fixed by the definitions."""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig3_set_mss.txt")


def _read_fig3():
    mats = {}
    cur = None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("before", "after"):
            cur = line
            mats[cur] = []
            continue
        mats[cur].append([float(x) for x in line.split()])
    return np.array(mats["before"]), np.array(mats["after"])


def test_fig3_set_alpha_mss_columns():
    """Set alpha-MSS worked example (Figure "set-sketch"): per column keep
    ceil(0.4 |L_i|) largest values.  Column 7 of the figure is defective."""
    before, after = _read_fig3()
    alpha = 0.4
    for c in range(before.shape[1]):
        col = before[:, c]
        nz = np.nonzero(col)[0]
        lam = math.ceil(alpha * len(nz) - 1e-12)
        keep = oracle.column_keep(nz.astype(np.uint32), col[nz].astype(np.float16), lam)
        assert keep.sum() == lam
        kept_vals = sorted(col[nz][keep])
        if c == 6:
            # printed figure keeps only 2 of 6; the definition keeps 3
            assert np.count_nonzero(after[:, c]) == 2
            continue
        paper_kept = after[:, c][np.nonzero(after[:, c])[0]]
        assert sorted(paper_kept) == kept_vals, f"column {c + 1}"
        # the oracle's choice is the id-ascending tie-break of a valid choice
        dropped = col[nz][~keep]
        if len(dropped):
            assert min(kept_vals) >= dropped.max()


def test_column_keep_is_top_lambda_with_id_tiebreak():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = int(rng.integers(1, 60))
        ids = rng.choice(10_000, size=n, replace=False).astype(np.uint32)
        vals = rng.choice([0.25, 0.5, 1.0, 1.5, 2.0], size=n).astype(np.float16)
        lam = int(rng.integers(1, 70))
        keep = oracle.column_keep(ids, vals, lam)
        order = sorted(range(n), key=lambda i: (-float(vals[i]), int(ids[i])))
        expect = np.zeros(n, dtype=bool)
        expect[order[:min(n, lam)]] = True
        assert np.array_equal(keep, expect)


def _rand_half(rng, n, lo=-6, hi=6):
    v = np.exp2(rng.uniform(lo, hi, size=n)).astype(np.float16)
    return v


def test_alpha_mss_definition_properties():
    """alpha-MSS (Definition "alpha-mass subvector sketch"): the kept entries
    are the largest ones, their mass reaches alpha of the total, and no
    shorter prefix does."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        n = int(rng.integers(1, 300))
        ids = rng.choice(30522, size=n, replace=False).astype(np.uint32)
        v = _rand_half(rng, n)
        alpha = float(rng.uniform(0.01, 1.0))
        keep = oracle.alpha_mss(ids, v, alpha)
        vv = v.astype(np.float64)
        total = vv.sum()
        kept = vv[keep]
        assert kept.sum() >= alpha * total
        if (~keep).any():
            assert kept.min() >= vv[~keep].max()
        # minimality: dropping the smallest kept entry falls short
        if keep.sum() > 1:
            assert kept.sum() - kept.min() < alpha * total
    # alpha = 1 keeps everything
    v = _rand_half(rng, 40)
    assert oracle.alpha_mss(np.arange(40, dtype=np.uint32), v, 1.0).all()


def test_alpha_mss_error_bound_theorem():
    """Theorem "alpha-mss-bound": <u,v> - <u~,v~> <= (1-a)|u|(1-b)|v| +
    |u_I|(1-b)|v| + |v_I|(1-a)|u| for an a-MSS of u and a b-MSS of v."""
    rng = np.random.default_rng(3)
    d = 400
    for _ in range(300):
        nu, nv = int(rng.integers(1, 120)), int(rng.integers(1, 120))
        iu = rng.choice(d, size=nu, replace=False)
        iv = rng.choice(d, size=nv, replace=False)
        u = np.zeros(d); v = np.zeros(d)
        u[iu] = _rand_half(rng, nu).astype(np.float64)
        v[iv] = _rand_half(rng, nv).astype(np.float64)
        u /= 2 * u.sum(); v /= 2 * v.sum()  # inside the l1 ball
        u = u.astype(np.float16).astype(np.float64); v = v.astype(np.float16).astype(np.float64)
        a, b = float(rng.uniform(0.05, 1)), float(rng.uniform(0.05, 1))
        ku = oracle.alpha_mss(iu.astype(np.uint32), u[iu].astype(np.float16), a)
        kv = oracle.alpha_mss(iv.astype(np.uint32), v[iv].astype(np.float16), b)
        ut = np.zeros(d); vt = np.zeros(d)
        ut[iu[ku]] = u[iu[ku]]; vt[iv[kv]] = v[iv[kv]]
        inter = (u != 0) & (v != 0)
        lhs = u @ v - ut @ vt
        rhs = ((1 - a) * u.sum() * (1 - b) * v.sum() + u[inter].sum() * (1 - b) * v.sum()
               + v[inter].sum() * (1 - a) * u.sum())
        assert lhs <= rhs + 1e-15


def test_quantize_properties():
    """u8 scalar quantization (Section 4.1.3): codes index 256 equal
    sub-intervals above m; reconstruction m + code*size is the left end of
    the sub-interval holding the value."""
    rng = np.random.default_rng(4)
    for _ in range(300):
        n = int(rng.integers(1, 400))
        v = _rand_half(rng, n, -6, 6)
        m, delta, codes = oracle.quantize(v)
        vv = v.astype(np.float64)
        grid = 2.0 ** -14
        assert m <= vv.min() < m + grid
        assert math.fmod(m, grid) == 0 and math.fmod(delta, grid) == 0
        assert 256 * delta >= vv.max() - m
        assert delta < (vv.max() - m) / 256 + grid
        deq = m + codes.astype(np.float64) * delta
        assert (deq <= vv).all()
        assert (vv - deq <= delta).all()
        assert codes.max() <= 255
        if delta > 0:
            assert (vv - deq < delta).all() or codes.max() == 255


def test_quantize_degenerate_range():
    v = np.array([0.5, 0.5, 0.5], dtype=np.float16)  # on the 2^-14 grid
    m, delta, codes = oracle.quantize(v)
    assert m == 0.5 and delta == 0.0 and (codes == 0).all()
    v = np.array([0.3], dtype=np.float16)  # off the grid: size one grid step
    m, delta, codes = oracle.quantize(v)
    assert m <= float(v[0]) < m + 2 ** -14 and codes[0] == 0
