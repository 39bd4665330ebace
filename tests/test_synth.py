"""Seeded input generators: determinism and the moments the workloads promise."""

import numpy as np

from paper_2101_05012_amd import synth


def test_model_shape_and_ranges():
    m = synth.pore_model(6)
    assert m.level_mean.shape == (4096,) and m.level_mean.dtype == np.float32
    assert 60 <= m.level_mean.min() and m.level_mean.max() <= 130
    assert 1 <= m.level_stdv.min() and m.level_stdv.max() <= 3
    m2 = synth.pore_model(6)
    assert np.array_equal(m.level_mean, m2.level_mean)


def test_kmer_ranks_base4():
    bases = np.array([0, 1, 2, 3, 3, 0], np.uint8)  # ACGTTA
    r = synth.kmer_ranks(bases, 3)
    assert r.tolist() == [0 * 16 + 1 * 4 + 2, 1 * 16 + 2 * 4 + 3, 2 * 16 + 3 * 4 + 3, 3 * 16 + 3 * 4 + 0]


def test_read_is_independent_of_batch_position():
    m = synth.pore_model(6)
    a = synth.workload_batch("plain-4000-lognormal5kb", m, read_ids=[5, 6, 7])
    b = synth.workload_batch("plain-4000-lognormal5kb", m, read_ids=[7, 99, 5])
    ra, rb = a.read(2), b.read(0)
    assert np.array_equal(ra.events, rb.events) and np.array_equal(ra.ranks, rb.ranks)
    assert a.read(0).scale == b.read(2).scale


def test_event_moments_64x1kb():
    m = synth.pore_model(6)
    b = synth.workload_batch("plain-64x1kb", m)
    ne = np.diff(b.event_offset).astype(np.float64)
    nk = np.diff(b.kmer_offset).astype(np.float64)
    assert np.all(nk == 995)
    epk = ne.sum() / nk.sum()
    assert abs(epk - 0.95 * 1.8) < 0.03
    assert 0.9 <= b.scale.min() and b.scale.max() <= 1.1
    assert -5 <= b.shift.min() and b.shift.max() <= 5
    assert b.events.shape == (int(ne.sum()), 3)


def test_length_distributions():
    L1 = synth.workload_lengths("plain-4000-lognormal5kb", range(4000))
    assert L1.min() >= 200 and L1.max() <= 100_000
    assert 4500 < np.median(L1) < 5500
    L2 = synth.workload_lengths("uneven-20000", range(4000))
    long = L2 >= 20_000
    assert 0.27 < long.mean() < 0.33
    assert L2[~long].min() >= 500 and L2[~long].max() <= 5000
    L4 = synth.workload_lengths("ultralong-200", range(200))
    assert L4.min() >= 200_000 and L4.max() <= 1_000_000


def test_noiseless_batch():
    m = synth.pore_model(6)
    b = synth.noiseless_batch(2, 100, m)
    rd = b.read(0)
    assert np.array_equal(rd.events[:, 0], m.level_mean[rd.ranks])
    assert rd.scale == 1 and rd.shift == 0


def test_serving_arrivals_rate():
    t = synth.serving_arrivals(n_channels=512, duration_s=20.0)
    rate = len(t) / 20.0
    expected = 512 * 400.0 / (8000.0 * np.exp(0.5))
    assert abs(rate - expected) < 0.15 * expected
    assert np.all(np.diff(t) >= 0)
