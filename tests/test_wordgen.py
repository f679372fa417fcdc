"""The seeded generator: determinism and the statistics it is meant to have."""
import numpy as np

from paper_1411_5283_amd import wordgen


def test_deterministic_per_seed():
    a = wordgen.config(1, 0.2)
    b = wordgen.config(1, 0.2)
    assert np.array_equal(a.chars, b.chars) and np.array_equal(a.offsets, b.offsets)
    c = wordgen.single(7000, 5000, 1.0, 16, seed=1)
    assert not np.array_equal(a.offsets, c.offsets)


def test_config1_shape():
    wl = wordgen.config(1)
    lens = np.diff(wl.offsets.astype(np.int64))
    assert wl.n == 35_000 and lens.min() >= 1 and lens.max() <= 16
    assert set(np.unique(wl.chars)) <= set(range(ord("a"), ord("z") + 1))
    text_bytes = int(wl.offsets[-1]) + wl.n          # one separator per word
    assert 150_000 < text_bytes < 230_000             # the paper's 190 KB text


def test_length_law_and_zipf():
    rng = np.random.Generator(np.random.PCG64(3))
    v = wordgen.make_vocabulary(rng, 200_000, 16, 1.0)
    lens = np.diff(v.offsets)
    assert abs(lens.mean() - 4.43) < 0.03
    p = np.bincount(lens, minlength=17)[1:7] / lens.shape[0]
    assert np.allclose(p, [0.132, 0.168, 0.161, 0.136, 0.109, 0.083], atol=0.005)
    tok = wordgen.draw_tokens(rng, v, 400_000)
    top = np.bincount(tok).max() / tok.shape[0]
    h = (np.arange(1, 200_001, dtype=np.float64) ** -1.0).sum()
    assert abs(top - 1.0 / h) < 0.01


def test_batch_docs():
    wl = wordgen.config(3, 0.02)
    sizes = np.diff(wl.doc_offsets.astype(np.int64))
    assert wl.n_docs == 82 and sizes.min() >= 100 and sizes.max() <= 50_000
    assert int(wl.doc_offsets[-1]) == wl.n


def test_serving_requests():
    reqs = list(wordgen.serving_requests(20, scale=0.01))
    assert len(reqs) == 20 and all(r.n >= 10 for r in reqs)
