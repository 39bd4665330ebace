"""Every read of the full-size workloads, in the launch forms the benchmark
times, against the CPU oracle (Alg. 5.1-5.3).

* plain-4000-lognormal5kb (W = 100): a pool of 320 wavefronts per batch with
  edge clearing, four contexts in flight over one device-resident batch;
  every read against the oracle run here (8.75 G cells).
* uneven-20000 (W = 100 and W = 200): the whole job as one captured graph of
  the persistent kernel, in the autotuned form of each width.
* ultralong-200 (W = 100 and 250 with k = 6; W = 250 with k = 9 under an
  8 GB trace budget, so that reads wait in the device queue for a trace
  slot).
The oracle's results for the last two (about 770 G cells) are per-read
digests written by ``tests/golden/oracle_digests.py``; a few reads of each
are re-run through the oracle here to show the digests are current.  Each
test asserts the acceptance rule and prints the identical fraction and the
smallest decision margin (``parity_util``).
"""

import gc
import sys

import numpy as np
import pytest

import oracle_digests
import parity_util
from paper_2101_05012_amd import abea, autotune, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_device():
    import torch

    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def digests_for(name, batch):
    ref = oracle_digests.load(name)
    assert np.array_equal(ref["n_events"], np.diff(batch.event_offset.astype(np.int64))), name
    assert np.array_equal(ref["n_kmers"], np.diff(batch.kmer_offset.astype(np.int64))), name
    return ref


def recheck_digests(O, model, batch, W, ref, idx):
    """The live oracle on reads idx gives the stored digests."""
    om = O.Model(model.level_mean, model.level_stdv)
    live = parity_util.oracle_result_digests(O.align_batch(batch.subset(idx), om, W, n_threads=16))
    for f in ("status", "cells", "path_len", "score_bits", "pairs_digest"):
        assert np.array_equal(live[f], ref[f][idx]), (f, idx)


def freshness_sample(batch, rng, n_rand=4):
    L = np.diff(batch.kmer_offset.astype(np.int64))
    order = np.argsort(-L, kind="stable")
    idx = {int(order[0]), int(order[-1])} | set(int(i) for i in rng.choice(batch.n_reads, n_rand, replace=False))
    return sorted(idx)


def host_digests(h):
    return parity_util.result_digests(h.pairs, h.pair_offset, h.status, h.cells, h.log_likelihood)


@pytest.fixture(scope="module")
def uneven():
    say("gpu: generating uneven-20000")
    return synth.workload_batch_parallel("uneven-20000", k=6)


@pytest.mark.parametrize("W,cpl,wpg,wps", [(100, 2, 4, 4), (200, 4, 4, 3)])
def test_uneven_20000_every_read(oracle_mod, uneven, W, cpl, wpg, wps):
    import torch

    name = f"uneven-20000_w{W}_k6"
    model = synth.pore_model(6)
    ref = digests_for(name, uneven)
    launch = autotune.Launch(cells_per_lane=cpl, waves_per_group=wpg, waves_per_simd=wps, batches=1)
    job = autotune.Job(uneven, 1, 0)
    al = autotune.make_aligner(model, 6, W, launch, 0, 0)
    run = autotune.GraphRun(al, job)
    assert run.info[0]["workers"] < uneven.n_reads
    st = torch.cuda.Stream()
    say(f"gpu: {name} graph replay, {run.info[0]}")
    run.launch(st)
    run.launch(st)  # a replay recomputes every output
    st.synchronize()
    h = run.results[0].to_host(uneven.n_reads)
    run.close()
    al.close()
    del run, job
    free_device()
    po = h.pair_offset.astype(np.int64)
    assert po[0] == 0 and np.all(np.diff(po) > 0) and po[-1] == len(h.pairs)
    say(f"gpu: {name} digests of {uneven.n_reads} reads")
    parity_util.check_acceptance(name, host_digests(h), ref, say)
    del h
    idx = freshness_sample(uneven, np.random.default_rng(W))
    say(f"gpu: {name} live oracle on reads {idx}")
    recheck_digests(oracle_mod, model, uneven, W, ref, idx)


@pytest.fixture(scope="module")
def ultralong6():
    say("gpu: generating ultralong-200 k=6")
    return synth.workload_batch_parallel("ultralong-200", k=6)


@pytest.mark.parametrize("W,cpl", [(100, 2), (250, 4)])
def test_ultralong_200_k6_every_read(oracle_mod, ultralong6, W, cpl):
    import torch

    name = f"ultralong-200_w{W}_k6"
    model = synth.pore_model(6)
    ref = digests_for(name, ultralong6)
    launch = autotune.Launch(cells_per_lane=cpl, waves_per_group=1, waves_per_simd=4, batches=1)
    job = autotune.Job(ultralong6, 1, 0)
    al = autotune.make_aligner(model, 6, W, launch, 0, 0)
    run = autotune.GraphRun(al, job)
    st = torch.cuda.Stream()
    say(f"gpu: {name} graph replay, {run.info[0]}")
    run.launch(st)
    st.synchronize()
    h = run.results[0].to_host(ultralong6.n_reads)
    run.close()
    al.close()
    del run, job
    free_device()
    parity_util.check_acceptance(name, host_digests(h), ref, say)
    idx = freshness_sample(ultralong6, np.random.default_rng(W), n_rand=1)
    say(f"gpu: {name} live oracle on reads {idx}")
    recheck_digests(oracle_mod, model, ultralong6, W, ref, idx)


def test_ultralong_200_w250_k9_under_trace_budget_every_read(oracle_mod):
    import torch

    name = "ultralong-200_w250_k9"
    model = synth.pore_model(9)
    say("gpu: generating ultralong-200 k=9")
    batch = synth.workload_batch_parallel("ultralong-200", k=9)
    ref = digests_for(name, batch)
    launch = autotune.Launch(cells_per_lane=4, waves_per_group=1, waves_per_simd=4, batches=1)
    job = autotune.Job(batch, 1, 0)
    al = autotune.make_aligner(model, 9, 250, launch, 0, 8_000_000_000)
    run = autotune.GraphRun(al, job)
    info = run.info[0]
    assert 0 < info["workers"] < batch.n_reads and info["trace_bytes"] <= 8_000_000_000
    st = torch.cuda.Stream()
    say(f"gpu: {name} graph replay, {info}")
    run.launch(st)
    st.synchronize()
    h = run.results[0].to_host(batch.n_reads)
    run.close()
    al.close()
    del run, job
    free_device()
    parity_util.check_acceptance(name, host_digests(h), ref, say)
    idx = freshness_sample(batch, np.random.default_rng(9), n_rand=1)
    say(f"gpu: {name} live oracle on reads {idx}")
    recheck_digests(oracle_mod, model, batch, 250, ref, idx)


def test_plain_4000_bench_launch_in_flight_every_read(oracle_mod):
    """plain-4000-lognormal5kb (W = 100) in the launch form of the plain
    benchmark: a pool of 320 wavefronts per batch with edge clearing, four
    contexts in flight on their own streams over one device-resident batch.
    Every context equals the window-clearing form bit for bit, and every read
    meets the acceptance rule against the oracle."""
    import torch

    model = synth.pore_model(6)
    b = synth.workload_batch("plain-4000-lognormal5kb", model)
    db = abea.to_device(b, 0)
    ref_al = abea.Aligner(model.level_mean, model.level_stdv, 6, W=100, workers=320,
                          band_clear=abea.ABEA_CLEAR_WINDOW)
    ref_dr = abea.DeviceResult.empty(db, 0)
    ref_al.align_device(db, ref_dr)
    torch.cuda.synchronize()
    ref = ref_dr.to_host(b.n_reads)
    slots = []
    for _ in range(4):
        al = abea.Aligner(model.level_mean, model.level_stdv, 6, W=100, workers=320,
                          band_clear=abea.ABEA_CLEAR_EDGES)
        slots.append((al, abea.DeviceResult.empty(db, 0), torch.cuda.Stream(0)))
    say("gpu: plain-4000 bench launch, 4 contexts in flight, edges vs window")
    for _ in range(2):
        for al, dr, st in slots:
            al.align_device(db, dr, st)
    torch.cuda.synchronize()
    for al, dr, _ in slots:
        info = al.plan_info()
        assert info["workers"] == 320 and info["band_clear"] == abea.ABEA_CLEAR_EDGES
        g = dr.to_host(b.n_reads)
        assert np.array_equal(g.status, ref.status)
        assert np.array_equal(g.cells, ref.cells)
        assert np.array_equal(g.log_likelihood.view(np.uint32), ref.log_likelihood.view(np.uint32))
        assert np.array_equal(g.pair_offset, ref.pair_offset)
        assert np.array_equal(g.pairs, ref.pairs)
        al.close()
    ref_al.close()
    say("gpu: plain-4000 oracle on all 4000 reads")
    om = oracle_mod.Model(model.level_mean, model.level_stdv)
    ores = oracle_mod.align_batch(b, om, 100, n_threads=16)
    parity_util.check_acceptance("plain-4000-lognormal5kb_w100_k6", host_digests(ref),
                                 parity_util.oracle_result_digests(ores), say)
