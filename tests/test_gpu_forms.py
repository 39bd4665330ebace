"""Launch forms of the HIP path (split kernels, fused kernel, persistent pool
with a device work queue and trace admission, captured graphs): every form
must give the same bits as every other and as the CPU oracle."""

import sys

import numpy as np
import pytest

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


def same(a: abea.HostResult, b: abea.HostResult):
    assert np.array_equal(a.status, b.status)
    assert np.array_equal(a.cells, b.cells)
    assert np.array_equal(a.log_likelihood.view(np.uint32), b.log_likelihood.view(np.uint32))
    assert np.array_equal(a.pair_offset, b.pair_offset)
    assert np.array_equal(a.pairs, b.pairs)


def oracle_check(O, om, batch, g, W, idx):
    sub = batch.subset(idx)
    o = O.align_batch(sub, om, W, n_threads=8)
    for t, r in enumerate(idx):
        assert g.status[r] == o.status[t], r
        if o.status[t] != 0:
            continue
        assert g.log_likelihood[r] == o.score[t], r
        assert np.array_equal(g.read_pairs(r), o.read_pairs(t)), r


def _edge_reads(m, rng):
    reads = []
    nmodel = m.level_mean.shape[0]
    reads.append(synth.Read(np.zeros((0, 3), np.float32), np.array([1, 2, 3], np.uint32), np.float32(1), np.float32(0)))
    reads.append(synth.Read(np.array([[80, 1, 0]] * 500, np.float32), np.zeros(0, np.uint32), np.float32(1), np.float32(0)))
    bad = rng.integers(0, nmodel, 300).astype(np.uint32)
    bad[11] = nmodel
    reads.append(synth.Read(np.array([[90, 1, 0]] * 400, np.float32), bad, np.float32(1), np.float32(0)))
    for L in (7, 20, 64, 65, 300, 1000, 2500, 6000):
        reads.append(synth.gen_read(rng, L, m))
    return synth.make_batch(reads)


def test_forms_identical_on_mixed_batch(oracle_mod, m6, om6):
    """200 reads of the 4000-read log-normal workload plus edge reads: the
    split kernels, the fused kernel and persistent pools of 1, 7 and 64
    workers agree bit for bit, and with the oracle."""
    rng = np.random.default_rng(77)
    main = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(200, 400))
    edge = _edge_reads(m6, rng)
    reads = [main.read(i) for i in range(main.n_reads)] + [edge.read(i) for i in range(edge.n_reads)]
    order = rng.permutation(len(reads))
    b = synth.make_batch([reads[i] for i in order])
    base = None
    for workers in (abea.ABEA_WORKERS_SPLIT, 0, 1, 7, 64):
        say(f"gpu: forms workers={workers} n={b.n_reads}")
        al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=workers)
        g = al.align(b)
        info = al.plan_info()
        if workers > 0:
            assert info["workers"] == workers
        elif workers == 0:
            assert info["workers"] == b.n_reads
        else:
            assert info["workers"] == 0
        al.close()
        if base is None:
            base = g
            L = np.diff(b.kmer_offset.astype(np.int64))
            idx = sorted(set(np.argsort(-L, kind="stable")[:6].tolist() + rng.choice(b.n_reads, 40, replace=False).tolist()))
            idx = sorted(set(idx) | set(np.nonzero(g.status != 0)[0].tolist()))
            oracle_check(oracle_mod, om6, b, g, 100, idx)
            assert set(g.status.tolist()) == {0, 1, 3}
        else:
            same(base, g)


@pytest.mark.parametrize("wpg,cpl", [(2, 0), (4, 0), (1, 4), (2, 8)])
def test_group_shapes_and_slot_counts(m6, wpg, cpl):
    """Waves per workgroup and slots per lane change the schedule only."""
    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(1000, 1096))
    ref = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100).align(b)
    say(f"gpu: wpg={wpg} cpl={cpl}")
    for workers in (0, 16):
        al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=workers,
                          waves_per_group=wpg, cells_per_lane=cpl)
        same(ref, al.align(b))
        al.close()


def test_trace_admission_limits_workers(m6):
    """A trace budget smaller than the batch's trace admits fewer workers (the
    split kernels run in parts); the results do not change; a budget below
    the longest read's trace is an error that names it."""
    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(0, 128))
    full = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    ref = full.align(b)
    total = full.plan_info()["trace_bytes"]
    budget = total // 6
    say(f"gpu: admission budget={budget} of {total}")
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, arena_bytes=budget)
    g = al.align(b)
    info = al.plan_info()
    assert 0 < info["workers"] < b.n_reads
    assert info["trace_bytes"] <= budget
    same(ref, g)
    tiny = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, arena_bytes=4096)
    with pytest.raises(abea.AbeaError) as ei:
        tiny.align(b)
    assert ei.value.code == abea.ABEA_E_NOMEM and "longest read" in str(ei.value)
    split = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, arena_bytes=budget, workers=abea.ABEA_WORKERS_SPLIT)
    same(ref, split.align(b))
    sinfo = split.plan_info()
    assert sinfo["parts"] >= 2 and sinfo["trace_bytes"] <= budget
    for a in (full, al, tiny, split):
        a.close()


@pytest.mark.parametrize("workers", [0, 48])
def test_graph_replays_match_eager(m6, workers):
    """A captured batch replayed several times, with eager work and
    synchronisation between replays: every replay equals the eager call."""
    import torch

    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(2000, 2160))
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=workers)
    db = abea.to_device(b)
    dr_e = abea.DeviceResult.empty(db)
    al.align_device(db, dr_e)
    torch.cuda.synchronize()
    eager = dr_e.to_host(b.n_reads)
    dr_g = abea.DeviceResult.empty(db)
    say(f"gpu: graph capture workers={workers}")
    g = al.graph(db, dr_g)
    if workers:
        assert g.info()["workers"] == workers
    st = torch.cuda.Stream()
    for rep in range(4):
        dr_g.log_likelihood.fill_(0.0)
        dr_g.pairs.fill_(-1)
        dr_g.pair_offset.fill_(0)
        g.launch(st)
        st.synchronize()
        same(eager, dr_g.to_host(b.n_reads))
        # eager work on the same context between replays
        al.align_device(db, dr_e)
        torch.cuda.synchronize()
        same(eager, dr_e.to_host(b.n_reads))
    g.close()
    al.close()


def test_two_graphs_concurrently(m6):
    """Two captured batches on two streams at once: each equals its eager
    result."""
    import torch

    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, workers=32)
    parts = [synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(3000 + 80 * j, 3080 + 80 * j)) for j in range(2)]
    eager = [al.align(p) for p in parts]
    dbs = [abea.to_device(p) for p in parts]
    drs = [abea.DeviceResult.empty(d) for d in dbs]
    gs = [al.graph(d, r) for d, r in zip(dbs, drs)]
    sts = [torch.cuda.Stream(), torch.cuda.Stream()]
    say("gpu: two graphs")
    for rep in range(2):
        for g, s in zip(gs, sts):
            g.launch(s)
        torch.cuda.synchronize()
        for j in range(2):
            same(eager[j], drs[j].to_host(parts[j].n_reads))
    for g in gs:
        g.close()
    al.close()


@pytest.mark.parametrize("workers", [-1, 0])
def test_kernel_timings(m6, workers):
    """abea_get_timings: every stage of the last call has a device time; the
    band (split) or fused kernel's interval lies inside the call's wall time;
    the fused form has no separate backtrack; a context made without
    ABEA_F_TIMING refuses."""
    import time

    import torch

    b = synth.workload_batch("plain-4000-lognormal5kb", m6, read_ids=range(0, 400))
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, timing=True, workers=workers)
    db = abea.to_device(b)
    dr = abea.DeviceResult.empty(db)
    say(f"gpu: timings workers={workers}")
    al.align_device(db, dr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    al.align_device(db, dr)
    ms = al.timings()
    wall = (time.perf_counter() - t0) * 1e3
    al.close()
    assert ms.shape == (4,) and np.all(np.isfinite(ms)) and np.all(ms >= 0)
    assert ms[0] > 0 and ms[1] > 0 and ms[3] > 0
    assert ms[1] <= wall
    if workers == -1:
        assert ms[2] > 0  # the split backtrack kernel
    else:
        assert ms[2] < 0.5 * ms[1]  # nothing between the fused kernel's end and the next event
    plain = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    plain.align(b.subset(range(4)))
    with pytest.raises(abea.AbeaError):
        plain.timings()
    plain.close()
