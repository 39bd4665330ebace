"""Trim states on the GPU (ABEA_F_TRIM; the trim paragraph after Alg. 5.3)
against the oracle's trim reading (ORACLE_TRIM):
* every read of the 4000-read workload with open-pore and adaptor events at
  its ends, in the plain benchmark's launch form and one wavefront per read;
* edge cases at many band widths in every launch form (split kernels, fused,
  pool), including tiny reads, reads of open-pore events only and noiseless
  reads between open-pore events;
* the split kernels in parts, captured graphs, the no-allocation call and the
  serving loop give the same bits.
"""

import sys

import numpy as np
import pytest

import parity_util
from paper_2101_05012_amd import abea, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def m6():
    return synth.pore_model(6)


@pytest.fixture(scope="module")
def om6(oracle_mod, m6):
    return oracle_mod.Model(m6.level_mean, m6.level_stdv)


def digests(h):
    return parity_util.result_digests(h.pairs, h.pair_offset, h.status, h.cells, h.log_likelihood)


def oracle_digests_of(O, om, batch, W):
    return parity_util.oracle_result_digests(O.align_batch(batch, om, W, n_threads=16, flags=O.TRIM))


def same(a, b):
    assert np.array_equal(a.status, b.status)
    assert np.array_equal(a.cells, b.cells)
    assert np.array_equal(a.log_likelihood.view(np.uint32), b.log_likelihood.view(np.uint32))
    assert np.array_equal(a.pair_offset, b.pair_offset)
    assert np.array_equal(a.pairs, b.pairs)


@pytest.fixture(scope="module")
def ends4000(m6):
    return synth.workload_batch("plain-4000-lognormal5kb-ends", m6)


@pytest.mark.parametrize("workers,clear", [(320, abea.ABEA_CLEAR_EDGES), (0, abea.ABEA_CLEAR_AUTO)])
def test_ends_4000_every_read(oracle_mod, om6, m6, ends4000, workers, clear):
    import torch

    b = ends4000
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, trim=True, workers=workers, band_clear=clear)
    db = abea.to_device(b)
    dr = abea.DeviceResult.empty(db)
    say(f"gpu: trim, 4000 reads with open-pore ends, workers={workers}")
    al.align_device(db, dr)
    torch.cuda.synchronize()
    h = dr.to_host(b.n_reads)
    al.close()
    parity_util.check_acceptance(f"trim ends-4000 workers={workers}", digests(h),
                                 oracle_digests_of(oracle_mod, om6, b, 100), say)
    # the trimmed alignments leave the leading open-pore events out
    first = h.pairs[h.pair_offset[:-1].astype(np.int64), 0]
    ev0 = b.events[b.event_offset[:-1].astype(np.int64), 0]
    assert np.mean(first[ev0 > 150.0] > 0) > 0.99


def _edge_batch(m, rng):
    reads = []
    for L in (6, 7, 8, 9, 20, 64, 65, 129, 300):
        reads.append(synth.gen_read(rng, L, m, ends=True))
    reads.append(synth.gen_read(rng, 200, m))  # no end events
    # open-pore events only
    op = np.zeros((12, 3), np.float32)
    op[:, 0] = rng.normal(synth.OPEN_PORE_MEAN, synth.OPEN_PORE_SD, 12)
    op[:, 1] = 1.0
    reads.append(synth.Read(op, rng.integers(0, 4096, 30).astype(np.uint32), np.float32(1), np.float32(0)))
    # a single event and a single k-mer
    reads.append(synth.Read(np.array([[80, 1, 0]], np.float32), np.array([7], np.uint32), np.float32(1),
                            np.float32(0)))
    # a noiseless read between open-pore events
    nl = synth.gen_read(rng, 400, m, noiseless=True)
    pad = np.zeros((9, 3), np.float32)
    pad[:, 0] = synth.OPEN_PORE_MEAN
    reads.append(synth.Read(np.concatenate([pad, nl.events, pad[:4]]), nl.ranks, nl.scale, nl.shift))
    return synth.make_batch(reads)


@pytest.mark.parametrize("W", [2, 3, 17, 64, 100, 129, 200, 250, 512])
def test_trim_edge_cases_every_form(oracle_mod, om6, m6, W):
    rng = np.random.default_rng(4000 + W)
    b = _edge_batch(m6, rng)
    ref = oracle_digests_of(oracle_mod, om6, b, W)
    out = []
    for workers in (abea.ABEA_WORKERS_SPLIT, 0, 3):
        al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=W, trim=True, workers=workers)
        say(f"gpu: trim edge batch W={W} workers={workers}")
        g = al.align(b)
        al.close()
        parity_util.check_acceptance(f"trim edge W={W} workers={workers}", digests(g), ref, say)
        out.append(g)
    same(out[0], out[1])
    same(out[1], out[2])
    if W >= 64:  # the noiseless read between open-pore events: exactly the read's own events
        r = b.n_reads - 1
        n_k = b.n_kmers(r)
        assert np.array_equal(out[1].read_pairs(r), np.stack([9 + np.arange(n_k), np.arange(n_k)], 1))


def test_trim_in_parts_graph_and_noalloc_same_bits(m6, ends4000):
    import torch

    b = ends4000.subset(range(300))
    ref_al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, trim=True)
    ref = ref_al.align(b)
    # split kernels in parts under a trace budget
    G = 32 // abea.min_cells_per_lane(100)
    nb = np.diff(b.event_offset.astype(np.int64)) + np.diff(b.kmer_offset.astype(np.int64)) - 1
    budget = int((((nb + G - 1) // G) * 512).sum() // 3)
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, trim=True, workers=abea.ABEA_WORKERS_SPLIT,
                      arena_bytes=budget)
    say("gpu: trim, split kernels in parts")
    same(al.align(b), ref)
    assert al.plan_info()["parts"] >= 3
    al.close()
    # captured graph, replayed twice
    db = abea.to_device(b)
    dr = abea.DeviceResult.empty(db)
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, trim=True, workers=64)
    g = al.graph(db, dr)
    st = torch.cuda.Stream()
    say("gpu: trim, graph")
    g.launch(st)
    g.launch(st)
    st.synchronize()
    same(dr.to_host(b.n_reads), ref)
    g.close()
    # the no-allocation call
    dr2 = abea.DeviceResult.empty(db)
    say("gpu: trim, no-allocation call")
    ref_al.align_device_noalloc(db, dr2, st)
    st.synchronize()
    same(dr2.to_host(b.n_reads), ref)
    al.close()
    ref_al.close()


def test_trim_serving_matches_alone(m6, ends4000):
    from paper_2101_05012_amd import serving

    b = ends4000.subset(range(120))
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, trim=True)
    alone = [al.align(b.subset([i])) for i in range(b.n_reads)]
    srv = abea.Server(al, slots=3, max_batch_reads=16)
    say("gpu: trim, serving")
    res = serving.run(srv, b, np.sort(np.random.default_rng(5).uniform(0, 0.03, b.n_reads)), keep_pairs=True)
    c = res["completions"]
    for r in range(b.n_reads):
        assert c[r]["status"] == alone[r].status[0]
        assert np.float32(c[r]["log_likelihood"]).view(np.uint32) == alone[r].log_likelihood[0:1].view(np.uint32)[0]
        assert np.array_equal(res["pairs"][r], alone[r].read_pairs(0))
    srv.close()
    al.close()
