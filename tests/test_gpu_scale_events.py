"""Events scaled to the model (ABEA_F_SCALE_EVENTS; per-read scaling
paragraph after Alg. 5.3): the HIP path against the oracle's scaled-events
switch, bit for bit, in every launch form and through the serving loop."""

import sys

import numpy as np
import pytest

from paper_2101_05012_amd import abea, serving, synth

from test_gpu_parity import _edge_batch, check_parity

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


def test_64x1kb_scaled_events_bit_exact(oracle_mod, m6, om6):
    b = synth.workload_batch("plain-64x1kb", m6)
    say("gpu: scale-events 64 reads of 1 kb W=100")
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, scale_events=True)
    g = al.align(b)
    al.close()
    check_parity(b, g, oracle_mod, om6, 100, flags=oracle_mod.SCALE_EVENTS)
    assert np.all(g.status == 0)
    # the mode changes the result: the events, not the model, carry the scaling
    o_model = oracle_mod.align_batch(b, om6, 100, n_threads=8)
    assert not np.array_equal(g.log_likelihood, o_model.score)


@pytest.mark.parametrize("W", [17, 100, 129, 250])
@pytest.mark.parametrize("workers", [-1, 0, 3])
def test_edge_cases_scaled_events_every_form(oracle_mod, m6, om6, W, workers):
    rng = np.random.default_rng(3000 + W)
    b = _edge_batch(m6, rng)
    say(f"gpu: scale-events edge batch W={W} workers={workers} n={b.n_reads}")
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=W, scale_events=True, workers=workers)
    g = al.align(b)
    al.close()
    check_parity(b, g, oracle_mod, om6, W, flags=oracle_mod.SCALE_EVENTS)
    assert g.status[0] == abea.READ_EMPTY and g.status[3] == abea.READ_BAD_RANK


def test_4000_lognormal_scaled_events_device_api_sampled(oracle_mod, m6, om6):
    """The 4000-read workload in the benchmark's launch form (device API,
    320-wavefront pool, edge clearing); the oracle checks the 8 longest reads
    and 24 others."""
    import torch

    b = synth.workload_batch("plain-4000-lognormal5kb", m6)
    say("gpu: scale-events 4000 log-normal reads device API, 320 workers, edge clearing")
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, scale_events=True, workers=320,
                      band_clear=abea.ABEA_CLEAR_EDGES)
    db = abea.to_device(b)
    dr = abea.DeviceResult.empty(db)
    al.align_device(db, dr)
    torch.cuda.synchronize()
    g = dr.to_host(b.n_reads)
    assert al.plan_info()["band_clear"] == abea.ABEA_CLEAR_EDGES
    al.close()
    assert np.all(g.status == 0)
    L = np.diff(b.kmer_offset)
    longest = list(np.argsort(-L, kind="stable")[:8])
    others = list(np.random.default_rng(6).choice(b.n_reads, 24, replace=False))
    idx = sorted(set(int(x) for x in longest + others))
    check_parity(b, g, oracle_mod, om6, 100, idx=idx, flags=oracle_mod.SCALE_EVENTS)


def test_serving_scaled_events_matches_oracle(oracle_mod, m6, om6):
    b = synth.workload_batch("serving-lognormal8kb", m6, read_ids=range(40))
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, scale_events=True)
    srv = abea.Server(al, slots=4, max_batch_reads=16)
    say("gpu: scale-events serving 40 reads")
    arr = np.sort(np.random.default_rng(8).uniform(0.0, 0.05, b.n_reads))
    res = serving.run(srv, b, arr, compression=1.0, keep_pairs=True, timeout_s=120)
    srv.close()
    al.close()
    o = oracle_mod.align_batch(b, om6, 100, n_threads=8, flags=oracle_mod.SCALE_EVENTS)
    c = res["completions"]
    assert c.shape[0] == b.n_reads
    for r in range(b.n_reads):
        assert c[r]["status"] == o.status[r], r
        assert np.float32(c[r]["log_likelihood"]) == o.score[r], r
        assert c[r]["cells"] == o.cells[r], r
        assert np.array_equal(res["pairs"][r], o.read_pairs(r)), r
