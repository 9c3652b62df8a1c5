"""The seeded input generator: determinism, distinct coordinates, index ranges and
the Zipf head mass."""
import hashlib

import numpy as np

from paper_1902_03317_amd import synth


def _digest(coo):
    h = hashlib.sha256()
    h.update(coo.inds.tobytes())
    h.update(coo.vals.tobytes())
    return h.hexdigest()


def test_deterministic_and_distinct():
    spec = synth.CONFIGS[2].scaled(200_000, dims=(5000, 4000, 3000))
    a, b = synth.make_coo(spec), synth.make_coo(spec)
    assert _digest(a) == _digest(b)
    assert a.inds.dtype == np.uint32 and a.inds.shape == (3, 200_000)
    for k, d in enumerate(spec.dims):
        assert int(a.inds[k].max()) < d
    keys = (a.inds[0].astype(np.int64) * 4000 + a.inds[1]) * 3000 + a.inds[2]
    assert np.unique(keys).size == 200_000
    assert np.all((a.vals >= 0) & (a.vals < 1))
    c = synth.make_coo(spec.scaled(200_000, seed=spec.seed + 1))
    assert _digest(c) != _digest(a)


def test_two_word_keys_for_huge_cell_counts():
    """1e6 x 1e6 x 1e5 x 1e3 x 1e2 has ~1e22 cells: keys span two uint64 words."""
    spec = synth.CONFIGS[5].scaled(300_000)
    assert len(synth._pack_words(spec.dims)) == 2
    coo = synth.make_coo(spec)
    t = np.stack([coo.inds[k] for k in range(5)], axis=1)
    assert np.unique(t, axis=0).shape[0] == 300_000
    assert np.all(coo.vals > 0)


def test_zipf_head_mass():
    """Without dedup the rank-1 index of a Zipf(1.1) mode over 50K appears with
    probability 1/H(50K, 1.1) (about 0.139), within 5 binomial sigmas."""
    n = 400_000
    spec = synth.TensorSpec("z", (50_000, 7), n, 4, (1.1, None), "uniform", False, 77)
    coo = synth.make_coo(spec)
    p1 = 1.0 / np.sum(np.arange(1, 50_001, dtype=np.float64) ** -1.1)
    top = np.bincount(coo.inds[0]).max()
    assert abs(top - n * p1) <= 5 * np.sqrt(n * p1 * (1 - p1))


def test_zipf_sampler_exact_inverse_cdf():
    s = synth._ZipfSampler(1000, 1.2)
    u = np.random.default_rng(3).random(200_000)
    assert np.array_equal(s.ranks(u), np.minimum(np.searchsorted(s.cdf, u, side="right"), 999))


def test_uniform_small_workload():
    spec = synth.CONFIGS[1]
    coo = synth.make_coo(spec)
    assert coo.dims == (100, 80, 60) and coo.nnz == 20_000
    keys = (coo.inds[0].astype(np.int64) * 80 + coo.inds[1]) * 60 + coo.inds[2]
    assert np.unique(keys).size == 20_000
    f = synth.make_factors(spec)
    assert [x.shape for x in f] == [(100, 16), (80, 16), (60, 16)] and f[0].dtype == np.float32
