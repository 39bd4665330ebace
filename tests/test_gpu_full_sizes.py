"""Full-size workloads in the launch form the benchmark times, checked on
sampled reads against the CPU oracle (bit-exact scores and pairs).

* uneven-20000 (W = 100): the whole job as one captured graph of the
  persistent kernel (pool of 4 wavefronts per SIMD, 4 reads per workgroup).
* ultralong-200 (W = 250, k = 9): the persistent kernel under an 8 GB trace
  budget (fewer workers than reads, so reads come from the work queue).
"""

import sys

import numpy as np
import pytest

from paper_2101_05012_amd import abea, autotune, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sampled_parity(O, model, batch, W, res_by_read, idx):
    om = O.Model(model.level_mean, model.level_stdv)
    sub = batch.subset(idx)
    o = O.align_batch(sub, om, W, n_threads=16)
    for t, r in enumerate(idx):
        status, ll, cells, pairs = res_by_read(r)
        assert status == o.status[t], r
        assert cells == int(o.cells[t]), r
        if o.status[t] != 0:
            continue
        assert np.float32(ll) == o.score[t], (r, ll, o.score[t])
        assert np.array_equal(pairs, o.read_pairs(t)), r


def pick(batch, rng, n_long, n_short, n_rand):
    L = np.diff(batch.kmer_offset.astype(np.int64))
    order = np.argsort(-L, kind="stable")
    idx = set(order[:n_long].tolist()) | set(order[-n_short:].tolist())
    idx |= set(rng.choice(batch.n_reads, n_rand, replace=False).tolist())
    return sorted(int(i) for i in idx)


def test_uneven_20000_persistent_graph(oracle_mod):
    import torch

    model = synth.pore_model(6)
    say("gpu: generating uneven-20000")
    batch = synth.workload_batch_parallel("uneven-20000", k=6)
    launch = autotune.Launch(cells_per_lane=2, waves_per_group=4, waves_per_simd=4, batches=1)
    job = autotune.Job(batch, 1, 0)
    al = autotune.make_aligner(model, 6, 100, launch, 0, 0)
    run = autotune.GraphRun(al, job)
    assert run.info[0]["workers"] < batch.n_reads
    st = torch.cuda.Stream()
    say("gpu: uneven-20000 graph replay")
    run.launch(st)
    st.synchronize()
    h = run.results[0].to_host(batch.n_reads)
    run.close()
    al.close()
    assert np.all(h.status == 0)
    po = h.pair_offset.astype(np.int64)
    assert po[0] == 0 and np.all(np.diff(po) > 0)
    idx = pick(batch, np.random.default_rng(21), 3, 2, 10)
    say(f"gpu: uneven-20000 oracle on {len(idx)} reads")
    sampled_parity(oracle_mod, model, batch, 100,
                   lambda r: (h.status[r], h.log_likelihood[r], int(h.cells[r]), h.read_pairs(r)), idx)


def test_ultralong_w250_k9_under_trace_budget(oracle_mod):
    import torch

    model = synth.pore_model(9)
    say("gpu: generating ultralong-200 k=9")
    batch = synth.workload_batch_parallel("ultralong-200", k=9)
    al = abea.Aligner(model.level_mean, model.level_stdv, 9, W=250, arena_bytes=8_000_000_000,
                      workers=4 * autotune.resident_simds(0))
    db = abea.to_device(batch)
    dr = abea.DeviceResult.empty(db)
    say("gpu: ultralong-200 W=250 k=9")
    al.align_device(db, dr)
    torch.cuda.synchronize()
    info = al.plan_info()
    assert 0 < info["workers"] < batch.n_reads and info["trace_bytes"] <= 8_000_000_000
    h = dr.to_host(batch.n_reads)
    al.close()
    assert np.all(h.status == 0)
    idx = pick(batch, np.random.default_rng(22), 1, 1, 1)
    say(f"gpu: ultralong oracle on {len(idx)} reads")
    sampled_parity(oracle_mod, model, batch, 250,
                   lambda r: (h.status[r], h.log_likelihood[r], int(h.cells[r]), h.read_pairs(r)), idx)


def test_plain_4000_bench_launch_in_flight(oracle_mod):
    """plain-4000-lognormal5kb (W = 100) in the launch form the default bench
    times: a pool of 320 wavefronts per batch with edge clearing, several
    batches in flight on their own streams over one device-resident batch.
    Every context's result equals the window-clearing form's bit for bit; 10
    longest, 10 shortest and 40 other reads match the oracle."""
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
    assert np.all(ref.status == 0)
    slots = []
    for j in range(4):
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
    idx = pick(b, np.random.default_rng(11), 10, 10, 40)
    say(f"gpu: plain-4000 oracle on {len(idx)} sampled reads")
    sampled_parity(oracle_mod, model, b, 100,
                   lambda r: (int(ref.status[r]), ref.log_likelihood[r], int(ref.cells[r]), ref.read_pairs(r)), idx)
