"""CPU check of the band fill's two ways of clearing the slots outside a band
(abea_launch_t.band_clear), on a slot-ring model of the wavefront's band fill.

The model keeps one band as N > W + 1 slots, k-mer kv in slot kv mod N, and
every slot computes a score each band, as the kernel does.
* Window clearing sets every slot outside the band's cells in the table to
  -inf.
* Edge clearing does that only in bands with a cell outside the table.  In
  the other bands it clears just k-mers K - 1 and K + W, and the remaining
  slots outside the band keep whatever they computed.  The model makes that
  NaN or huge on purpose.

Pinned:
* the window model reproduces the oracle (score, status and k-mer moves,
  bit for bit);
* the edge model gives the window model's scores and trace codes in every
  band cell, bit for bit.
So no slot outside a band beyond the two cleared ones reaches a cell in one.
"""

import numpy as np
import pytest

from paper_2101_05012_amd import synth

NEG_INF = np.float32(-np.inf)


def model_fill(x, ranks, mean, c, h, lp, W, N, edges, rng, clear_below=True, clear_above=True):
    """Band fill of one read (scale 1, shift 0) on an N-slot ring; returns the
    terminal score, the k-mer move count and, per band, the in-band scores and
    trace codes (1 = D, 2 = U, 3 = L) keyed by k-mer."""
    n_e, n_k = len(x), len(ranks)
    lp_skip, lp_stay, lp_step = (np.float32(v) for v in lp)
    half = W // 2
    S2 = np.full(N, NEG_INF, np.float32)  # band 0: only the origin, k-mer -1
    S2[(-1) % N] = np.float32(0.0)
    S1 = np.full(N, NEG_INF, np.float32)  # band 1: all -inf
    K1 = -half
    last = n_e + n_k
    moves = 0
    cells = {}
    slots = np.arange(N)
    for i in range(2, last + 1):
        lo, hi = S1[K1 % N], S1[(K1 + W - 1) % N]
        if lo == NEG_INF and hi == NEG_INF:
            kmove = i % 2 == 1
        else:
            kmove = bool(lo < hi)
        K = K1 + 1 if kmove else K1
        moves += int(kmove)
        kv = K + ((slots - K) % N)  # every slot's k-mer, labelled from K
        # kv is in [K, K + N): slots above the band hold k-mers not yet in it
        e = i - 2 - kv
        intab = (e >= 0) & (e < n_e) & (kv >= 0) & (kv < n_k)
        inband = kv <= K + W - 1
        em = np.empty(N, np.float32)
        # outside the table: stale or garbage parameters, NaN or huge
        em[:] = rng.choice(np.array([np.nan, 3e38, -3e38, 0.0], np.float32), N)
        ok = np.nonzero(intab)[0]
        if ok.size:
            r = ranks[kv[ok]]
            d = x[e[ok]] - mean[r]
            t = d * d
            u = t * h[r]
            em[ok] = c[r] - u
        up = S1
        left = np.roll(S1, 1)  # slot s - 1 of band i-1
        diag = np.roll(S2, 1)  # slot s - 1 of band i-2
        with np.errstate(invalid="ignore", over="ignore"):
            sd = (diag + lp_step) + em
            su = (up + lp_stay) + em
            sl = left + lp_skip
            mu = su > sd
            s1 = np.where(mu, su, sd)
            ml = sl > s1
            sv = np.where(ml, sl, s1)
        code = np.where(ml, 3, np.where(mu, 2, 1))
        window = intab & inband
        interior = bool(window.sum() == W)
        nv = sv.copy()
        if edges and interior:
            if clear_below:
                nv[(K - 1) % N] = NEG_INF
            if clear_above:
                nv[(K + W) % N] = NEG_INF
        else:
            nv[~window] = NEG_INF
        for s in np.nonzero(window)[0]:
            cells[(i, int(kv[s]))] = (nv[s].view(np.uint32), int(code[s]))
        S2, S1, K1 = S1, nv, K
    score = S1[(n_k - 1) % N] if K1 <= n_k - 1 <= K1 + W - 1 else NEG_INF
    return np.float32(score), moves, cells


@pytest.mark.parametrize("W,N", [(8, 16), (9, 16), (14, 16), (20, 32), (31, 32)])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_edge_clearing_equals_window_clearing(oracle_mod, W, N, seed):
    rng = np.random.default_rng(seed * 100 + W)
    model = synth.pore_model(4, seed=seed)
    om = oracle_mod.Model(model.level_mean, model.level_stdv)
    read = synth.gen_read(rng, int(rng.integers(60, 160)), model)
    x = read.events[:, 0].astype(np.float32)
    x = (x - read.shift) / read.scale  # events brought to the model: scale 1, shift 0 below
    x = x.astype(np.float32)
    lp = oracle_mod.transitions(len(x), len(read.ranks))
    o = oracle_mod.align(x, read.ranks, om, 1.0, 0.0, W)
    sw, mw, cw = model_fill(x, read.ranks, om.level_mean, om.c, om.h, lp, W, N, False, rng)
    se, me, ce = model_fill(x, read.ranks, om.level_mean, om.c, om.h, lp, W, N, True, rng)
    # the window model is the oracle's band fill
    assert mw == o.kmer_moves
    if o.status == 0:
        assert sw.view(np.uint32) == np.float32(o.score).view(np.uint32)
    else:
        assert sw == NEG_INF
    # edge clearing changes nothing a band cell sees
    assert me == mw
    assert se.view(np.uint32) == sw.view(np.uint32)
    assert ce == cw


def _read(seed, W):
    rng = np.random.default_rng(seed * 100 + W)
    model = synth.pore_model(4, seed=seed)
    read = synth.gen_read(rng, int(rng.integers(60, 160)), model)
    x = ((read.events[:, 0].astype(np.float32) - read.shift) / read.scale).astype(np.float32)
    return rng, model, read, x


@pytest.mark.parametrize("drop", ["below", "above"])
def test_clearing_one_edge_slot_is_not_enough(oracle_mod, drop):
    """Planted on the model: leaving either slot beside the band uncleared
    changes band cells (so the test above would catch a kernel that did)."""
    W, N = 8, 16
    changed = 0
    for seed in (1, 2, 3):
        rng, model, read, x = _read(seed, W)
        om = oracle_mod.Model(model.level_mean, model.level_stdv)
        lp = oracle_mod.transitions(len(x), len(read.ranks))
        sw, mw, cw = model_fill(x, read.ranks, om.level_mean, om.c, om.h, lp, W, N, False, rng)
        se, me, ce = model_fill(x, read.ranks, om.level_mean, om.c, om.h, lp, W, N, True, rng,
                                clear_below=(drop != "below"), clear_above=(drop != "above"))
        changed += int(ce != cw or me != mw or se.view(np.uint32) != sw.view(np.uint32))
    assert changed == 3
