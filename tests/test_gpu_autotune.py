"""The launch-form autotuner (persistent kernel, device work queue, captured
graphs): on a small mixed-length job it measures every candidate, picks a
valid form, and the chosen form gives the default form's bits, which match
the oracle."""

import sys

import numpy as np
import pytest

import parity_util
from paper_2101_05012_amd import abea, autotune, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("W", [100, 200])
def test_autotune_picks_a_valid_form_with_the_default_bits(oracle_mod, W):
    import torch

    model = synth.pore_model(6)
    # 300 reads of the uneven job: about 90 of 20..200 kb, the rest 0.5..5 kb
    batch = synth.workload_batch("uneven-20000", model, read_ids=range(300))
    say(f"gpu: autotune W={W} on {batch.n_reads} reads")
    tuned = autotune.autotune(model, 6, W, batch, 0, reps=1, log=say, batch_counts=(1, 2))
    best = tuned["best"]
    minc = abea.min_cells_per_lane(W)
    assert best.cells_per_lane in (minc, 2 * minc)
    assert best.waves_per_group in (1, 2, 4)
    assert best.waves_per_simd in (1, 2, 3, 4, 8)
    assert best.batches in (1, 2)
    assert tuned["best_ms"] == min(r["ms"] for r in tuned["table"] if r["launch"] == best.as_dict())
    assert len(tuned["table"]) >= 8 and all(r["ms"] > 0 for r in tuned["table"])

    # the chosen form, replayed, against the default one-launch form
    job = autotune.Job(batch, best.batches, 0)
    al = autotune.make_aligner(model, 6, W, best, 0, 0)
    run = autotune.GraphRun(al, job)
    st = torch.cuda.Stream()
    run.launch(st)
    st.synchronize()
    hosts = [r.to_host(p.n_reads) for p, r in zip(job.parts, run.results)]
    run.close()
    al.close()
    # the default form (one fused wavefront per read, one launch) on the job's
    # reads in the same order as its batches
    ref_al = abea.Aligner(model.level_mean, model.level_stdv, 6, W=W)
    d = ref_al.align(job.host)
    ref_al.close()
    pos = 0
    for h in hosts:
        n = h.status.shape[0]
        assert np.array_equal(h.status, d.status[pos:pos + n])
        assert np.array_equal(h.log_likelihood.view(np.uint32), d.log_likelihood[pos:pos + n].view(np.uint32))
        for r in range(n):
            assert np.array_equal(h.read_pairs(r), d.read_pairs(pos + r))
        pos += n
    assert pos == batch.n_reads
    om = oracle_mod.Model(model.level_mean, model.level_stdv)
    ores = oracle_mod.align_batch(job.host, om, W, n_threads=16)
    parity_util.check_acceptance(f"autotune W={W}", parity_util.result_digests(
        d.pairs, d.pair_offset, d.status, d.cells, d.log_likelihood), parity_util.oracle_result_digests(ores), say)
