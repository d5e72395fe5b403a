"""The seeded input generator: Philox-4x32-10 against the known-answer
vectors published with the generator (Salmon et al., SC'11, Random123),
the fp16 rounding against NumPy's, row slices that concatenate to the whole
stream, and the row law's shape."""
import numpy as np

import synth


def test_philox_known_answers():
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                               [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_half_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    xs = list(np.exp(rng.uniform(np.log(1e-9), np.log(65000.0), 20000)))
    for e in range(-26, 16):  # every binade, with exact ties and their neighbours
        for m in range(0, 2048, 61):
            b = (1024 + m) * 2.0 ** (e - 10)
            xs += [b, b * (1 + 2.0 ** -11), b * (1 - 2.0 ** -12), np.nextafter(b, 0.0), np.nextafter(b, 1e9)]
    xs += [2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 65504.0, 65519.99]
    with np.errstate(over="ignore"):  # past 65520 both give +inf
        want = np.array(xs, dtype=np.float64).astype(np.float16).view(np.uint16)
    for x, w in zip(xs, want):
        assert synth.half_from_double(float(x)) == int(w), x
    assert synth.half_from_double(65520.0) == 0x7C00
    assert synth.half_from_double(0.0) == 0


def test_row_slices_concatenate():
    whole = synth.generate(3000, seed=3, mean=127.0)
    cuts = [0, 1, 1234, 2999, 3000]
    for a, b in zip(cuts, cuts[1:]):
        part = synth.generate(b - a, seed=3, mean=127.0, row0=a)
        lo, hi = int(whole.row_ptr[a]), int(whole.row_ptr[b])
        assert np.array_equal(part.words, whole.words[lo:hi])
        assert np.array_equal(part.row_ptr, whole.row_ptr[a:b + 1] - whole.row_ptr[a])


def test_row_counts_match_rows():
    whole = synth.generate(2000, seed=4, mean=127.0)
    c = synth.row_counts(1500, seed=4, mean=127.0, row0=500)
    assert np.array_equal(c.astype(np.uint64), np.diff(whole.row_ptr)[500:])


def test_row_law_shape():
    d = synth.docs(4000, seed=1)
    lens = np.diff(d.row_ptr.astype(np.int64))
    assert lens.min() >= 10 and lens.max() <= 400 and abs(lens.mean() - 120) < 1.5
    v = d.values().astype(np.float64)
    assert v.min() >= 2.0 ** -6 and v.max() <= 2.0 ** 6
    assert abs(np.log(v).std() - 0.6) < 0.02
    for i in range(0, 4000, 97):
        t, _ = d.row(i)
        assert np.all(np.diff(t) > 0)  # distinct, ascending
    # heavy head: the first terms are in every document, document frequency
    # falls with rank, the last 522 terms hold a fraction of a percent
    df = np.bincount(d.terms(), minlength=synth.DIM)
    assert df[0] == df[1] == 4000
    assert df[10] > df[100] > df[1000] > df[10000] > 0
    assert df[30000:].sum() < 0.002 * d.nnz
    q = synth.queries(3000, seed=1, law="uniform")
    ql = np.diff(q.row_ptr.astype(np.int64))
    assert ql.min() >= 5 and ql.max() <= 200
