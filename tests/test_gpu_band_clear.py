"""Slot clearing of interior bands (abea_launch_t.band_clear): clearing every
slot outside the band and clearing only the two slots beside it give the
same bits in every launch form, and the oracle's results; the automatic
choice resolves as documented; invalid choices are refused."""

import sys

import numpy as np
import pytest

from paper_2101_05012_amd import abea, synth

pytestmark = pytest.mark.gpu

WINDOW, EDGES, AUTO = abea.ABEA_CLEAR_WINDOW, abea.ABEA_CLEAR_EDGES, abea.ABEA_CLEAR_AUTO


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def m6():
    return synth.pore_model(6)


@pytest.fixture(scope="module")
def om6(oracle_mod, m6):
    return oracle_mod.Model(m6.level_mean, m6.level_stdv)


def same(a, b):
    assert np.array_equal(a.status, b.status)
    assert np.array_equal(a.cells, b.cells)
    assert np.array_equal(a.log_likelihood.view(np.uint32), b.log_likelihood.view(np.uint32))
    assert np.array_equal(a.pair_offset, b.pair_offset)
    assert np.array_equal(a.pairs, b.pairs)


def _batch(m, rng):
    """Log-normal reads (long enough for many interior bands), short reads
    around the band width, an empty read, a read with a bad rank and one
    noiseless read."""
    main = synth.workload_batch("plain-4000-lognormal5kb", m, read_ids=range(600, 660))
    reads = [main.read(i) for i in range(main.n_reads)]
    nmodel = m.level_mean.shape[0]
    reads.append(synth.Read(np.zeros((0, 3), np.float32), np.array([1, 2, 3], np.uint32), np.float32(1), np.float32(0)))
    bad = rng.integers(0, nmodel, 300).astype(np.uint32)
    bad[5] = nmodel
    reads.append(synth.Read(np.array([[90, 1, 0]] * 400, np.float32), bad, np.float32(1), np.float32(0)))
    for L in (20, 65, 129, 257, 600, 3000):
        reads.append(synth.gen_read(rng, L, m))
    reads.append(synth.gen_read(rng, 2000, m, noiseless=True))
    order = rng.permutation(len(reads))
    return synth.make_batch([reads[i] for i in order])


@pytest.mark.parametrize("W", [64, 100, 112, 113, 120, 121, 126, 128, 200, 248, 250, 252])
def test_window_and_edges_identical_and_match_oracle(oracle_mod, m6, om6, W):
    """Band widths at two and four slots per lane, on both sides of the
    one-refill/two-refill limit; every launch form with both clearings."""
    cpl = abea.min_cells_per_lane(W)
    if cpl not in (2, 4):
        pytest.skip(f"W={W} uses {cpl} slots per lane")
    rng = np.random.default_rng(4000 + W)
    b = _batch(m6, rng)
    base = None
    for workers in (0, abea.ABEA_WORKERS_SPLIT, 16):
        for clear in (WINDOW, EDGES):
            say(f"gpu: band_clear={clear} W={W} cpl={cpl} workers={workers} n={b.n_reads}")
            al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=W, workers=workers, band_clear=clear)
            g = al.align(b)
            assert al.plan_info()["band_clear"] == clear
            al.close()
            if base is None:
                base = g
                o = oracle_mod.align_batch(b, om6, W, n_threads=8)
                for r in range(b.n_reads):
                    assert g.status[r] == o.status[r], r
                    if o.status[r] != 0:
                        continue
                    assert int(g.cells[r]) == int(o.cells[r]), r
                    assert g.log_likelihood[r] == o.score[r], r
                    assert np.array_equal(g.read_pairs(r), o.read_pairs(r)), r
                assert set(g.status.tolist()) >= {0, 1, 3}
            else:
                same(base, g)


def test_edges_with_explicit_slot_counts(m6):
    """Edge clearing at four slots per lane for a width that needs two, in the
    fused and pooled forms, against the default."""
    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(2000, 2064))
    ref = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, band_clear=WINDOW).align(b)
    for workers in (0, 8):
        say(f"gpu: edges cpl=4 W=100 workers={workers}")
        al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=workers, cells_per_lane=4, band_clear=EDGES)
        same(ref, al.align(b))
        al.close()


def test_auto_choice(m6):
    """Auto: edges at four slots per lane; at two, edges once the launch has
    at least two wavefronts per SIMD (8 per CU), else window; never at one or
    eight slots per lane."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    small = synth.workload_batch("plain-64x1kb", m6, read_ids=range(16))

    def resolved(W, batch, **kw):
        al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=W, **kw)
        al.align(batch)
        c = al.plan_info()["band_clear"]
        al.close()
        return c

    say(f"gpu: auto choice, {cus} CUs")
    assert resolved(100, small) == WINDOW
    assert resolved(250, small) == EDGES
    assert resolved(40, small) == WINDOW
    assert resolved(100, small, cells_per_lane=8) == WINDOW
    # enough reads for two wavefronts per SIMD: tiny reads keep this fast
    rng = np.random.default_rng(3)
    many = synth.make_batch([synth.gen_read(rng, 12, m6) for _ in range(8 * cus)])
    assert resolved(100, many) == EDGES
    assert resolved(100, many, workers=8 * cus - 1) == WINDOW
    assert resolved(100, many, band_clear=WINDOW) == WINDOW


def test_invalid_choices_refused(m6):
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    for bad in (3, -1, 7):
        with pytest.raises(abea.AbeaError) as ei:
            al.set_launch(band_clear=bad)
        assert ei.value.code == abea.ABEA_E_INVAL
    with pytest.raises(abea.AbeaError) as ei:
        al.set_launch(cells_per_lane=8, band_clear=EDGES)
    assert ei.value.code == abea.ABEA_E_INVAL and "cells_per_lane" in str(ei.value)
    al.close()
    narrow = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=40)
    with pytest.raises(abea.AbeaError):
        narrow.set_launch(band_clear=EDGES)
    narrow.close()


@pytest.mark.parametrize("clear", [WINDOW, EDGES])
def test_graph_keeps_the_clearing_form(m6, clear):
    """A captured batch records the clearing form it was planned with
    (abea_graph_info) and its replays equal the eager call of the other form."""
    import torch

    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(3000, 3096))
    other = EDGES if clear == WINDOW else WINDOW
    ref_al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=16, band_clear=other)
    ref = ref_al.align(b)
    ref_al.close()
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=16, band_clear=clear)
    db = abea.to_device(b)
    dr = abea.DeviceResult.empty(db)
    say(f"gpu: graph with band_clear={clear}")
    g = al.graph(db, dr)
    assert g.info()["band_clear"] == clear
    st = torch.cuda.Stream()
    for _ in range(3):
        dr.log_likelihood.fill_(0.0)
        dr.pairs.fill_(-1)
        g.launch(st)
        st.synchronize()
        same(ref, dr.to_host(b.n_reads))
    g.close()
    al.close()
