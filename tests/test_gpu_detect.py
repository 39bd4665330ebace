"""Event detection on the GPU (abea_detect_events*) against the CPU oracle
(oracle/event_oracle.c), read by read and event by event.

Change points are integers decided in float32 by the same operations on both
sides, so event boundaries and durations must be identical; means are double
arithmetic rounded once to float and must be identical too; stdv takes a
double square root, so it is allowed one float32 ulp and the number of
inexact ones is printed (expected 0)."""

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
def aligner(m6):
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100)
    yield al
    al.close()


def edge_reads(m6):
    """Degenerate and boundary cases: empty, one sample, shorter than the
    windows, constant (one event spanning many tiles), exactly one tile and
    one tile plus one sample, noiseless steps, a spike, int16 extremes, a long
    read whose change-free middle spans several tiles."""
    rng = np.random.default_rng(42)
    T = 1024
    out = []

    def rr(x, off=0.0, sc=0.17):
        return synth.RawRead(np.ascontiguousarray(x, np.int16), np.zeros(0, np.uint32), np.float32(off),
                             np.float32(sc), np.float32(1), np.float32(0), np.zeros(0, np.int64))

    out.append(rr(np.zeros(0)))
    out.append(rr(np.array([321])))
    out.append(rr(np.array([100, 900, 100, 900, 100])))
    out.append(rr(np.full(5 * T + 17, 612)))
    for n in (T, T + 1, 2 * T - 1):
        out.append(rr(np.round(rng.normal(600, 30, n))))
    lens = rng.integers(16, 60, 200)
    out.append(rr(np.repeat(rng.integers(300, 900, 200), lens), 3.5, 0.171))
    spike = np.full(300, 500)
    spike[150] = 32767
    out.append(rr(spike))
    out.append(rr(rng.integers(-32768, 32768, 3000)))
    out.append(rr(np.concatenate([np.round(rng.normal(700, 20, 1500)), np.full(4 * T + 3, 455),
                                  np.round(rng.normal(400, 20, 900))])))
    out.append(rr(np.zeros(0)))
    for L in (50, 400, 3000):
        out.append(synth.gen_raw_read(np.random.default_rng([43, L]), L, m6))
    return synth.make_raw_batch(out)


def oracle_events(oracle_mod, rb, params=None, threads=16):
    return oracle_mod.ed_batch(rb, params, n_threads=threads)


def gpu_events_device(al, rb, params=None, cap=None):
    import torch

    d = abea.raw_to_device(rb)
    cap = d.n_samples if cap is None else cap
    ev = torch.full((max(cap, 1), 3), -7.0, dtype=torch.float32, device="cuda")
    eo = torch.zeros(rb.n_reads + 1, dtype=torch.int64, device="cuda")
    al.detect_events_device(d, ev, eo, params, event_capacity=cap)
    torch.cuda.synchronize()
    eo_h = eo.cpu().numpy().view(np.uint64)
    return ev.cpu().numpy(), eo_h


def compare(tag, got_ev, got_eo, want_ev, want_eo):
    assert np.array_equal(got_eo, want_eo), f"{tag}: event offsets differ"
    m = int(want_eo[-1])
    g, w = got_ev[:m], want_ev[:m]
    assert np.array_equal(g[:, 2], w[:, 2]), f"{tag}: durations (event boundaries) differ"
    assert np.array_equal(g[:, 0].view(np.uint32), w[:, 0].view(np.uint32)), f"{tag}: means differ"
    gs, ws = g[:, 1].view(np.int32).astype(np.int64), w[:, 1].view(np.int32).astype(np.int64)
    d = np.abs(gs - ws)
    say(f"{tag}: {m} events, stdv bit-identical {int((d == 0).sum())}, off by one ulp {int((d == 1).sum())}")
    assert int(d.max(initial=0)) <= 1, f"{tag}: stdv differs by more than one ulp"


def test_edge_cases_device(aligner, m6, oracle_mod):
    rb = edge_reads(m6)
    say("gpu: detect edge cases (device API)")
    ev, eo = gpu_events_device(aligner, rb)
    want_ev, want_eo = oracle_events(oracle_mod, rb)
    compare("edge", ev, eo, want_ev, want_eo)
    # the constant read is one event over all its tiles; the empty reads none
    assert int(eo[1] - eo[0]) == 0 and int(eo[4] - eo[3]) == 1


def test_raw_workload_device_and_host(aligner, oracle_mod):
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(300))
    say(f"gpu: detect raw-4000 first 300 reads ({int(rb.sample_offset[-1])} samples)")
    want_ev, want_eo = oracle_events(oracle_mod, rb)
    ev, eo = gpu_events_device(aligner, rb)
    compare("raw300 device", ev, eo, want_ev, want_eo)
    hev, heo = aligner.detect_events(rb)
    compare("raw300 host", hev, heo, want_ev, want_eo)


@pytest.mark.parametrize("params", [(2, 2, 0.0, 0.0), (4, 12, 2.5, 3.0), (16, 16, 1.0, 9.0), (2, 16, 1.2, 6.0)])
def test_other_detectors(aligner, oracle_mod, m6, params):
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(300, 340))
    rb2 = edge_reads(m6)
    say(f"gpu: detect with windows/thresholds {params}")
    for tag, b in (("raw", rb), ("edge", rb2)):
        pa = abea.detect_params(*params)
        po = oracle_mod.ed_params(params[0], params[2], params[1], params[3])
        ev, eo = gpu_events_device(aligner, b, pa)
        want_ev, want_eo = oracle_events(oracle_mod, b, po)
        compare(f"{tag} {params}", ev, eo, want_ev, want_eo)


def test_long_events_wide_variance(aligner, oracle_mod):
    """Events far longer than a tile and than the 2^16 samples below which the
    events' variance is taken in 64 bits: full-range uniform noise under
    thresholds no finite statistic of two-sample windows reaches in practice
    (t^2 above 10^6), so each read is one event or very few; at 300000 samples
    len * Q - S^2 exceeds 2^64, the 128-bit path's rounding with a sticky
    bit."""
    rng = np.random.default_rng(44)

    def rr(x):
        return synth.RawRead(np.ascontiguousarray(x, np.int16), np.zeros(0, np.uint32), np.float32(2.0),
                             np.float32(0.17), np.float32(1), np.float32(0), np.zeros(0, np.int64))

    rb = synth.make_raw_batch([rr(rng.integers(-32768, 32768, n)) for n in (70000, 300000)])
    params = (2, 2, 1000.0, 1000.0)
    say(f"gpu: detect two long full-range reads with {params}")
    pa = abea.detect_params(*params)
    po = oracle_mod.ed_params(params[0], params[2], params[1], params[3])
    want_ev, want_eo = oracle_events(oracle_mod, rb, po)
    ev, eo = gpu_events_device(aligner, rb, pa)
    compare("long events", ev, eo, want_ev, want_eo)
    dur = want_ev[: int(want_eo[-1]), 2]
    assert (dur > 65536).sum() >= 2, dur
    # the longest event of the second read: len * Q - S^2 above 2^64
    k0, k1 = int(want_eo[1]), int(want_eo[2])
    j = k0 + int(np.argmax(dur[k0:k1]))
    start = int(dur[k0:j].sum())
    x = rb.raw[int(rb.sample_offset[1]) + start: int(rb.sample_offset[1]) + start + int(dur[j])].astype(np.int64)
    n, S, Q = len(x), int(x.sum()), int((x * x).sum())
    assert n * Q - S * S >= 2 ** 64


def test_capacity(aligner, oracle_mod):
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(20))
    want_ev, want_eo = oracle_events(oracle_mod, rb)
    total = int(want_eo[-1])
    say("gpu: detect capacity")
    # device API: events beyond the capacity are not written; the total is reported
    ev, eo = gpu_events_device(aligner, rb, cap=total - 5)
    assert np.array_equal(eo, want_eo)
    assert np.array_equal(ev[: total - 5, 2], want_ev[: total - 5, 2])
    # host API: ABEA_E_CAPACITY with nothing written, exactly enough succeeds
    with pytest.raises(abea.AbeaError) as ei:
        aligner.detect_events(rb, event_capacity=total - 1)
    assert ei.value.code == abea.ABEA_E_CAPACITY
    hev, heo = aligner.detect_events(rb, event_capacity=total)
    compare("capacity exact", hev, heo, want_ev, want_eo)


def test_bad_arguments(aligner):
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(2))
    for params in ((1, 8, 1.5, 5.0), (3, 17, 1.5, 5.0), (8, 3, 1.5, 5.0), (3, 8, -1.0, 5.0),
                   (3, 8, 1.5, float("inf"))):
        with pytest.raises(abea.AbeaError) as ei:
            aligner.detect_events(rb, abea.detect_params(*params))
        assert ei.value.code == abea.ABEA_E_INVAL, params
    bad = synth.RawBatch(rb.raw, rb.sample_offset[::-1].copy(), rb.ranks, rb.kmer_offset, rb.offset, rb.pa_scale,
                         rb.scale, rb.shift, rb.dwell)
    with pytest.raises(abea.AbeaError) as ei:
        aligner.detect_events(bad)
    assert ei.value.code == abea.ABEA_E_INVAL


def test_detected_events_align_like_the_oracle(aligner, m6, oracle_mod):
    """Raw signal to alignment: the GPU's events aligned on the GPU equal the
    oracle's events aligned by the oracle (pairs, score, status)."""
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(400, 440))
    say("gpu: detect then align")
    ev, eo = aligner.detect_events(rb)
    b = synth.Batch(ev, eo, rb.ranks, rb.kmer_offset, rb.scale, rb.shift)
    got = aligner.align(b)
    want_ev, want_eo = oracle_events(oracle_mod, rb)
    ob = synth.Batch(want_ev, want_eo, rb.ranks, rb.kmer_offset, rb.scale, rb.shift)
    om = oracle_mod.Model(m6.level_mean, m6.level_stdv)
    ores = oracle_mod.align_batch(ob, om, 100, n_threads=16)
    ok = 0
    for r in range(rb.n_reads):
        assert got.status[r] == ores.status[r], r
        assert np.float32(got.log_likelihood[r]).view(np.uint32) == np.float32(ores.score[r]).view(np.uint32), r
        assert np.array_equal(got.read_pairs(r), ores.read_pairs(r)), r
        ok += int(got.status[r] == abea.READ_OK)
    assert ok >= rb.n_reads - 1


def test_whole_raw_workload(aligner, oracle_mod):
    """All 4000 reads of raw-4000-lognormal5kb (293 M samples) in one device
    call, in the launch form the benchmark times, against the oracle on 16
    threads: every read's events identical."""
    import os

    from paper_2101_05012_amd import synth as S

    rb = S.workload_raw_batch("raw-4000-lognormal5kb")
    say(f"gpu: detect whole raw-4000 ({int(rb.sample_offset[-1])} samples)")
    want_ev, want_eo = oracle_events(oracle_mod, rb, threads=min(16, os.cpu_count() or 1))
    ev, eo = gpu_events_device(aligner, rb)
    compare("raw-4000 whole", ev, eo, want_ev, want_eo)
    ratio = float(want_eo[-1]) / float(rb.kmer_offset[-1])
    say(f"raw-4000: {ratio:.3f} events per k-mer")
    assert 1.5 <= ratio <= 2.0


def test_detect_timings(m6):
    """abea_get_detect_timings after a timed call: both streaming kernels'
    dispatch times are positive and lie within the batch's time."""
    al = abea.Aligner(m6.level_mean, m6.level_stdv, 6, W=100, timing=True)
    rb = synth.workload_raw_batch("raw-4000-lognormal5kb", read_ids=range(100))
    say("gpu: detect timings")
    with pytest.raises(abea.AbeaError):
        al.detect_timings()  # no detection call yet
    al.detect_events(rb)
    t = al.detect_timings()
    assert t[0] > 0 and t[1] > 0 and t[2] >= t[0] + t[1] - 1e-3, t
    al.close()
