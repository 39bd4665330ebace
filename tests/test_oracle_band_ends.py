"""The move rule's both -inf case (Alg. 5.1: the band alternates when both
end cells are -inf) never arises from a band that lies wholly inside the
table.  Each cell of such a band has its up neighbour (or, for the last
cell after a k-mer move, its left neighbour) inside the previous band, so by
induction every cell of the band, its two end cells included, is finite.
The band fill relies on this: in interior bands (every cell in the table)
it decides the move by one compare of the end cells, without the
alternation.  Checked here with the oracle's count of such bands and of
their -inf end cells, over the read shapes of the workloads, with and
without trim, at the band widths of the two- and four-slot launch forms,
and on reads whose events ignore the model or stop early."""

import numpy as np
import pytest

from paper_2101_05012_amd import synth


@pytest.fixture(scope="module")
def m6():
    return synth.pore_model(6)


def _reads(m6):
    out = []
    for wl, ids in (("plain-4000-lognormal5kb", range(0, 4000, 400)), ("plain-4000-lognormal5kb-ends", range(8))):
        b = synth.workload_batch(wl, m6, read_ids=ids)
        out += [b.read(i) for i in range(b.n_reads)]
    rng = np.random.default_rng(31)
    for _ in range(12):
        r = synth.gen_read(rng, int(rng.integers(300, 2500)), m6)
        ev = r.events.copy()
        ev[:, 0] = rng.uniform(0.0, 300.0, ev.shape[0]).astype(np.float32)  # events ignore the model
        if rng.random() < 0.5:
            ev = ev[: max(1, ev.shape[0] // 3)]  # the read stops early
        out.append(synth.Read(ev, r.ranks, r.scale, r.shift))
    return out


@pytest.mark.parametrize("W", [64, 100, 113, 126, 200, 250])
def test_bands_inside_the_table_have_finite_end_cells(oracle_mod, m6, W):
    om = oracle_mod.Model(m6.level_mean, m6.level_stdv)
    bands = 0
    for rd in _reads(m6):
        for flags in (0, oracle_mod.TRIM):
            res = oracle_mod.align(rd.events[:, 0], rd.ranks, om, rd.scale, rd.shift, W, flags=flags)
            bands += res.in_table_bands
            assert res.in_table_inf_ends == 0, (W, flags, res.in_table_bands)
    assert bands > 10000
