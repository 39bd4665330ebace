"""The stored per-read oracle digests of the full workloads are current: they
cover every read of each workload with the generator's read sizes, and the
live oracle reproduces them on a few reads of each.  (The digests are
written by ``tests/golden/oracle_digests.py``, which calls only the oracle
and the input generator.)"""

import numpy as np
import pytest

import oracle_digests
import parity_util
from paper_2101_05012_amd import synth


@pytest.mark.parametrize("name", sorted(oracle_digests.CASES))
def test_digests_cover_every_read_and_match_the_live_oracle(oracle_mod, name):
    workload, W, k = oracle_digests.CASES[name]
    ref = oracle_digests.load(name)
    n = synth.WORKLOADS[workload]["n_reads"]
    for f in oracle_digests.FIELDS:
        assert ref[f].shape == (n,), (f, ref[f].shape)
    L = synth.workload_lengths(workload, range(n))
    assert np.array_equal(ref["n_kmers"], L - k + 1)
    assert np.all(ref["status"] == 0)
    assert np.all(ref["path_len"] >= ref["n_events"]) and np.all(ref["path_len"] <= ref["n_events"] + ref["n_kmers"] - 1)
    # the live oracle on the three shortest reads, and the median one if short
    order = np.argsort(L, kind="stable")
    idx = {int(i) for i in order[:3]}
    if L[order[n // 2]] < 30000:
        idx.add(int(order[n // 2]))
    idx = sorted(idx)
    model = synth.pore_model(k)
    b = synth.workload_batch(workload, model, read_ids=idx)
    om = oracle_mod.Model(model.level_mean, model.level_stdv)
    live = parity_util.oracle_result_digests(oracle_mod.align_batch(b, om, W, n_threads=4))
    for f in ("status", "cells", "path_len", "score_bits", "pairs_digest", "min_margin"):
        assert np.array_equal(live[f], ref[f][idx]), (f, idx)
    assert np.array_equal(np.diff(b.event_offset.astype(np.int64)), ref["n_events"][idx])


def test_acceptance_rule_flags_a_changed_read():
    """check_acceptance fails on a changed path, on a changed score beyond the
    relative tolerance, and on a status change; it passes identical digests."""
    rng = np.random.default_rng(0)
    n = 2000
    ref = {
        "status": np.zeros(n, np.int8),
        "cells": rng.integers(1000, 9000, n),
        "path_len": rng.integers(100, 900, n),
        "score_bits": (-rng.uniform(100, 5000, n)).astype(np.float32).view(np.uint32),
        "pairs_digest": rng.integers(0, 2**63, n, dtype=np.int64).astype(np.uint64),
        "min_margin": rng.uniform(0.01, 1.0, n),
    }
    got = {f: v.copy() for f, v in ref.items() if f != "min_margin"}
    parity_util.check_acceptance("same", got, ref, say=lambda *a: None)
    g1 = {f: v.copy() for f, v in got.items()}
    g1["pairs_digest"][7] ^= np.uint64(1)
    with pytest.raises(AssertionError):
        parity_util.check_acceptance("pairs", g1, ref, say=lambda *a: None)
    g2 = {f: v.copy() for f, v in got.items()}
    s = g2["score_bits"].view(np.float32)
    s[3] = s[3] * np.float32(1.0001)
    with pytest.raises(AssertionError):
        parity_util.check_acceptance("score", g2, ref, say=lambda *a: None)
    g3 = {f: v.copy() for f, v in got.items()}
    g3["status"][5] = 2
    with pytest.raises(AssertionError):
        parity_util.check_acceptance("status", g3, ref, say=lambda *a: None)
    # a read below the margin may differ, within 0.1% of the reads
    ref4 = {f: v.copy() for f, v in ref.items()}
    ref4["min_margin"][11] = 0.0
    g4 = {f: v.copy() for f, v in got.items()}
    g4["pairs_digest"][11] ^= np.uint64(1)
    st = parity_util.check_acceptance("tie", g4, ref4, say=lambda *a: None)
    assert st["identical"] == n - 1
