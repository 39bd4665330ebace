"""The serving loop (continuous batching): every read's result equals the
read aligned alone, whatever micro-batch it ran in; admission keeps the
traceback memory on the device within the budget; every submitted read comes
back exactly once."""

import sys

import numpy as np
import pytest

from paper_2101_05012_amd import abea, serving, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def m6():
    return synth.pore_model(6)


@pytest.fixture(scope="module")
def reads(m6):
    return synth.workload_batch("serving-lognormal8kb", m6, read_ids=range(160))


@pytest.fixture(scope="module")
def alone(m6, reads, oracle_mod):
    """Each read aligned alone by the library, and those results checked
    against the oracle (acceptance rule), so that the mix is compared with
    oracle-checked results."""
    import parity_util

    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    out = [al.align(reads.subset([i])) for i in range(reads.n_reads)]
    al.close()
    om = oracle_mod.Model(m6.level_mean, m6.level_stdv)
    ores = oracle_mod.align_batch(reads, om, 100, n_threads=16)
    po = np.zeros(reads.n_reads + 1, np.uint64)
    po[1:] = np.cumsum([len(a.pairs) for a in out])
    got = parity_util.result_digests(np.concatenate([a.pairs for a in out]), po,
                                     np.array([a.status[0] for a in out]), np.array([a.cells[0] for a in out]),
                                     np.array([a.log_likelihood[0] for a in out], np.float32))
    parity_util.check_acceptance("serving-lognormal8kb alone", got, parity_util.oracle_result_digests(ores), say)
    return out


def arrivals(n, span_s, seed):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, span_s, n))
    return t


def check_against_alone(res, alone, n):
    c = res["completions"]
    assert c.shape[0] == n
    assert np.array_equal(c["tag"], np.arange(n, dtype=np.uint64))
    for r in range(n):
        a = alone[r]
        rec = c[r]
        assert rec["status"] == a.status[0], r
        assert np.float32(rec["log_likelihood"]).view(np.uint32) == a.log_likelihood[0:1].view(np.uint32)[0], r
        assert rec["cells"] == a.cells[0], r
        assert np.array_equal(res["pairs"][r], a.read_pairs(0)), r
    assert np.all(c["t_done_ns"] >= c["t_admit_ns"]) and np.all(c["t_admit_ns"] >= c["t_arrival_ns"])


def test_results_same_alone_and_in_the_mix(m6, reads, alone):
    """160 log-normal (median 8 kb) reads arriving over 40 ms into 3 slots of
    at most 12 reads: they overlap on the device in several micro-batches."""
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    srv = abea.Server(al, slots=3, max_batch_reads=12)
    say("gpu: serving mix")
    res = serving.run(srv, reads, arrivals(reads.n_reads, 0.04, 1), compression=1.0, keep_pairs=True)
    check_against_alone(res, alone, reads.n_reads)
    st = res["stats"]
    assert st["micro_batches"] >= reads.n_reads // 12
    assert st["completed"] == reads.n_reads and st["pending"] == 0 and st["inflight_reads"] == 0
    srv.close()
    al.close()


def test_trace_budget_bounds_device_memory(m6, reads, alone):
    """A budget of about three of the largest reads: admission waits for
    memory, results do not change."""
    nb = np.diff(reads.event_offset.astype(np.int64)) + np.diff(reads.kmer_offset.astype(np.int64)) - 1
    G = 32 // abea.min_cells_per_lane(100)
    need = ((nb + G - 1) // G) * 512
    budget = int(3 * need.max())
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    srv = abea.Server(al, slots=4, max_batch_reads=64, trace_budget_bytes=budget)
    say(f"gpu: serving budget {budget}")
    res = serving.run(srv, reads, arrivals(reads.n_reads, 0.005, 2), compression=1.0, keep_pairs=True)
    check_against_alone(res, alone, reads.n_reads)
    st = res["stats"]
    assert 0 < st["max_inflight_trace_bytes"] <= budget
    assert st["max_inflight_reads"] < reads.n_reads
    srv.close()
    al.close()


def test_oversize_read_is_refused(m6, reads):
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    L = np.diff(reads.kmer_offset.astype(np.int64))
    big = int(np.argmax(L))
    srv = abea.Server(al, slots=1, max_batch_reads=4, max_batch_events=1 << 20, max_batch_kmers=int(L[big]) - 1)
    with pytest.raises(abea.AbeaError) as ei:
        srv.submit(reads, big, big + 1, [big])
    assert ei.value.code == abea.ABEA_E_CAPACITY
    assert srv.stats()["submitted"] == 0
    # the server still serves reads that fit
    small = int(np.argmin(L))
    srv.submit(reads, small, small + 1, [small])
    got = 0
    for _ in range(500):
        c, _ = srv.poll(timeout_us=10000)
        got += c.shape[0]
        if got:
            break
    assert got == 1
    srv.close()
    al.close()


def _collect(srv, n, timeout_s=60.0):
    import time

    got, pairs = [], {}
    deadline = time.monotonic() + timeout_s
    while sum(c.shape[0] for c in got) < n:
        assert time.monotonic() < deadline, "serving: results missing"
        c, p = srv.poll(timeout_us=5000)
        if c.shape[0]:
            got.append(c)
            for rec in c:
                pairs[int(rec["tag"])] = p[int(rec["pair_offset"]): int(rec["pair_offset"]) + int(rec["n_pairs"])]
    c = np.concatenate(got)
    return c[np.argsort(c["tag"])], pairs


def _check_unrun(rec):
    assert rec["n_pairs"] == 0 and rec["cells"] == 0
    assert np.isneginf(rec["log_likelihood"])
    assert rec["t_done_ns"] >= rec["t_admit_ns"] >= rec["t_arrival_ns"]


def test_cancel_queued_reads(m6, reads, alone):
    """120 reads submitted at once to one slot of four reads: cancelling the
    odd tags right away cancels those still queued; they come back as
    cancelled with no pairs, every other read as if aligned alone, each read
    exactly once."""
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    srv = abea.Server(al, slots=1, max_batch_reads=4)
    n = 120
    say("gpu: serving cancel")
    srv.submit(reads, 0, n, np.arange(n, dtype=np.uint64))
    k = srv.cancel(np.arange(1, n, 2, dtype=np.uint64))
    c, pairs = _collect(srv, n)
    assert np.array_equal(c["tag"], np.arange(n, dtype=np.uint64))
    cancelled = c["status"] == abea.READ_CANCELLED
    assert 0 < k == int(cancelled.sum())
    assert np.all(c["tag"][cancelled] % 2 == 1)
    for r in range(n):
        if cancelled[r]:
            _check_unrun(c[r])
        else:
            assert c[r]["status"] == alone[r].status[0]
            assert np.float32(c[r]["log_likelihood"]).view(np.uint32) == alone[r].log_likelihood[0:1].view(np.uint32)[0]
            assert np.array_equal(pairs[r], alone[r].read_pairs(0))
    st = srv.stats()
    assert st["cancelled"] == k and st["completed"] == n and st["pending"] == 0
    # cancelling what is no longer queued cancels nothing
    assert srv.cancel(np.arange(n, dtype=np.uint64)) == 0
    srv.close()
    al.close()


def test_queue_timeout(m6, reads, alone):
    """100 reads submitted at once to one slot of two reads with a 50 ms
    queue limit (counted from the arrival stamp, which precedes the submit
    call's own copying): the reads the slot cannot reach in time complete as
    timed out, the others as if aligned alone, each read exactly once."""
    limit = 50_000_000
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    srv = abea.Server(al, slots=1, max_batch_reads=2, max_queue_wait_ns=limit)
    n = 100
    say("gpu: serving queue timeout")
    srv.submit(reads, 0, n, np.arange(n, dtype=np.uint64))
    c, pairs = _collect(srv, n)
    assert np.array_equal(c["tag"], np.arange(n, dtype=np.uint64))
    out = c["status"] == abea.READ_TIMED_OUT
    assert out.sum() > 0 and (~out).sum() > 0
    for r in range(n):
        if out[r]:
            _check_unrun(c[r])
            assert c[r]["t_admit_ns"] - c[r]["t_arrival_ns"] >= limit
        else:
            assert np.float32(c[r]["log_likelihood"]).view(np.uint32) == alone[r].log_likelihood[0:1].view(np.uint32)[0]
            assert np.array_equal(pairs[r], alone[r].read_pairs(0))
    st = srv.stats()
    assert st["timed_out"] == int(out.sum()) and st["completed"] == n and st["pending"] == 0
    srv.close()
    al.close()
