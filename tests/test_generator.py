"""Pins for the seeded Kronecker input generator (kronecker/).

The exact Graph500 generator is not available, so the generator is pinned by
its own definition: the published SplitMix64 output vector, exact tuple counts
and ranges (Section 2.1 sizes), determinism, the initiator's quadrant
frequencies at every level, and the relabel being a bijection.
"""
import numpy as np
import pytest

import kronecker as K


def test_splitmix64_published_vector():
    # SplitMix64 (Steele, Lea, Flood 2014) seeded with 1234567: the first five
    # outputs of the reference implementation.
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert [K.splitmix64_at(1234567, c) for c in range(5)] == expect
    lib = K._load_host()
    assert [lib.kron_splitmix64_at(1234567, c) for c in range(5)] == expect


@pytest.mark.parametrize("scale,ef", [(1, 16), (5, 1), (10, 16), (13, 8)])
def test_counts_and_range(scale, ef):
    e = K.edges_host(scale, ef)
    assert e.shape == (ef * (1 << scale), 2)
    assert e.dtype == np.int64
    assert e.min() >= 0 and e.max() < (1 << scale)


def test_deterministic_and_seeded():
    a = K.edges_host(12)
    b = K.edges_host(12)
    c = K.edges_host(12, seed=K.graph_seed(12) + 1)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_ranges_compose():
    full = K.edges_host(11)
    parts = [K.edges_host(11, start=s, stop=min(s + 5000, full.shape[0]))
             for s in range(0, full.shape[0], 5000)]
    assert np.array_equal(full, np.concatenate(parts))


@pytest.mark.parametrize("scale", [12, 15])
def test_quadrant_frequencies_every_level(scale):
    raw = K.edges_host(scale, relabel=False)
    m = raw.shape[0]
    probs = np.array([0.57, 0.19, 0.19, 0.05])
    sigma = np.sqrt(probs * (1 - probs) / m)
    for k in range(scale):
        bit = scale - 1 - k
        rb = (raw[:, 0] >> bit) & 1
        cb = (raw[:, 1] >> bit) & 1
        freq = np.array([np.mean((rb == 0) & (cb == 0)), np.mean((rb == 0) & (cb == 1)),
                         np.mean((rb == 1) & (cb == 0)), np.mean((rb == 1) & (cb == 1))])
        assert np.all(np.abs(freq - probs) < 5 * sigma), (k, freq)


@pytest.mark.parametrize("scale", list(range(1, 17)))
def test_relabel_is_bijection(scale):
    p = K.relabel_host(scale, K.graph_seed(scale), np.arange(1 << scale))
    assert np.array_equal(np.sort(p), np.arange(1 << scale))


def test_relabel_applied_to_raw_tuples():
    scale = 12
    raw = K.edges_host(scale, relabel=False)
    lab = K.edges_host(scale)
    assert np.array_equal(K.relabel_host(scale, K.graph_seed(scale), raw.ravel()),
                          lab.ravel())


def test_relabel_destroys_locality():
    # Vertex 0 of the raw tuples is the highest-degree vertex; after relabelling
    # it lands elsewhere and the degree sequence is a permutation.
    scale = 12
    raw = K.edges_host(scale, relabel=False)
    lab = K.edges_host(scale)
    n = 1 << scale
    d_raw = np.bincount(raw.ravel(), minlength=n)
    d_lab = np.bincount(lab.ravel(), minlength=n)
    assert np.array_equal(np.sort(d_raw), np.sort(d_lab))
    assert d_raw.argmax() == 0
    assert not np.array_equal(d_raw, d_lab)


def test_nonisolated_mask():
    scale = 11
    n = 1 << scale
    e = K.edges_host(scale)
    mask = K.nonisolated_host(e, n)
    nl = e[e[:, 0] != e[:, 1]]
    expect = np.zeros(n, np.uint8)
    expect[nl.ravel()] = 1
    assert np.array_equal(mask, expect)
    with pytest.raises(ValueError):
        K.nonisolated_host(np.array([[0, n]]), n)


def test_select_roots():
    scale = 10
    n = 1 << scale
    e = K.edges_host(scale)
    mask = K.nonisolated_host(e, n)
    roots = K.select_roots(mask, 64, K.root_seed(scale))
    assert len(set(roots)) == 64
    assert all(mask[r] for r in roots)
    assert roots == K.select_roots(mask, 64, K.root_seed(scale))
    with pytest.raises(ValueError):
        K.select_roots(np.zeros(8, np.uint8), 1, 1)


def test_weights_definition_range_and_frequencies():
    # weight of tuple i = 1 + (splitmix64_at(splitmix64_at(seed, 3), i) mod 255)
    scale = 12
    w = K.weights_host(scale)
    assert w.dtype == np.uint8 and w.shape == (K.num_tuples(scale),)
    base = K.splitmix64_at(K.graph_seed(scale), 3)
    for i in (0, 1, 2, 1000, len(w) - 1):
        assert int(w[i]) == 1 + K.splitmix64_at(base, i) % 255
    assert w.min() >= 1 and w.max() <= 255
    # a window of the list equals the same tuples of the whole list
    assert np.array_equal(K.weights_host(scale, start=100, stop=900), w[100:900])
    # every value 1..255 within 5 sigma of uniform
    cnt = np.bincount(w, minlength=256)[1:]
    exp = len(w) / 255
    assert np.all(np.abs(cnt - exp) < 5 * np.sqrt(exp))
    # another seed gives other weights
    assert not np.array_equal(K.weights_host(scale, seed=7)[:64], w[:64])
