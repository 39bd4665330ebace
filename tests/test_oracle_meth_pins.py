"""Pins of the methylation-scoring oracle (oracle/meth_oracle.c).

The thesis (Ch. 5 §5.2.2) sends the aligned events through HMM profiling to
call methylation but gives no algorithm; the reading (sites, windows, a
best-path profile with the alignment's cell score under two models, their
difference) is the oracle's.  Each pin is chosen so that a plausible mistake
fails it:

* M1 identical models give LLR 0 at every site; swapping the models negates
  every LLR bit for bit;
* M2 the profile equals the best float32 path sum over every monotone path
  (brute force) on tiny windows: a wrong move constant, a missing emission,
  a wrong start fail;
* M3 a one-k-mer window is the closed form (origin step, then stays);
* M4 the sites are exactly the k-mers starting with C, G (decoded from the
  ranks independently), each with the events from the first paired with the
  window's first k-mer to the last paired with the site's own;
* M5 on the synthetic methylation workload the LLR's sign tells methylated
  reads from unmethylated ones (at least 95% of sites, every read by its sum).
"""

import itertools

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_05012_amd import synth

F = np.float32


@pytest.fixture(scope="module")
def models():
    m = synth.pore_model(6)
    mm = synth.methylated_model(m)
    return m, mm, orc.Model(m.level_mean, m.level_stdv), orc.Model(mm.level_mean, mm.level_stdv)


@pytest.fixture(scope="module")
def aligned(models):
    m, mm, Mu, Mm = models
    b = synth.workload_batch("meth-4000-lognormal5kb", m, read_ids=range(120))
    res = orc.align_batch(b, Mu, 100, n_threads=8)
    po = np.zeros(b.n_reads + 1, np.uint64)
    po[1:] = np.cumsum(res.path_len)
    pairs = np.concatenate([res.read_pairs(r) for r in range(b.n_reads)])
    return b, pairs, po, res.status


def test_m1_identical_models_and_swap(models, aligned):
    m, mm, Mu, Mm = models
    b, pairs, po, st = aligned
    llr0, n0 = orc.meth_batch(b, 6, Mu, Mu, pairs, po, st, n_threads=8)
    sites = n0 > 0
    assert sites.sum() > 1000
    assert np.all(llr0[sites] == 0.0) and np.all(np.isnan(llr0[~sites]))
    llr, n = orc.meth_batch(b, 6, Mu, Mm, pairs, po, st, n_threads=8)
    llr_s, n_s = orc.meth_batch(b, 6, Mm, Mu, pairs, po, st, n_threads=8)
    assert np.array_equal(n, n_s) and np.array_equal(n, n0)
    assert np.array_equal(llr_s[sites].view(np.uint32), (-llr[sites]).view(np.uint32))


def brute_profile(x, mu, c, h, lp):
    """Best float32 path sum over every monotone path from the virtual origin
    through (0, 0) to (m-1, n-1): D and U moves add the move constant then the
    emission, L moves only the skip constant, in path order."""
    lp_skip, lp_stay, lp_step = F(lp[0]), F(lp[1]), F(lp[2])
    m, n = len(x), len(mu)

    def em(e, j):
        d = F(x[e]) - F(mu[j])
        return F(c[j]) - F(F(d * d) * F(h[j]))

    best = F(-np.inf)
    # a path: the sequence of moves after the first cell (entered from the
    # origin by D); a D move advances both indices, so paths have between
    # max(m, n) - 1 and m + n - 2 moves
    all_moves = itertools.chain.from_iterable(
        itertools.product("DUL", repeat=L) for L in range(max(m, n) - 1, m + n - 1))
    for moves in all_moves:
        e = j = 0
        s = F(F(F(0.0) + lp_step) + em(0, 0))
        ok = True
        for mv in moves:
            if mv == "D":
                e, j = e + 1, j + 1
            elif mv == "U":
                e += 1
            else:
                j += 1
            if e >= m or j >= n:
                ok = False
                break
            if mv == "D":
                s = F(F(s + lp_step) + em(e, j))
            elif mv == "U":
                s = F(F(s + lp_stay) + em(e, j))
            else:
                s = F(s + lp_skip)
        if ok and e == m - 1 and j == n - 1 and s > best:
            best = s
    return best


def test_m2_profile_is_the_best_path(models):
    m, mm, Mu, Mm = models
    rng = np.random.default_rng(21)
    for trial in range(60):
        mev = int(rng.integers(1, 5))
        nk = int(rng.integers(1, 4))
        ranks = rng.integers(0, 4096, nk)
        mu = m.level_mean[ranks] * F(rng.uniform(0.9, 1.1)) + F(rng.uniform(-5, 5))
        x = (mu[np.minimum(np.arange(mev) * nk // max(mev, 1), nk - 1)] + rng.normal(0, 2, mev)).astype(F)
        lp = orc.transitions(int(rng.integers(1, 40)), int(rng.integers(1, 40)))
        sg, c, h = m.level_stdv[ranks], Mu.c[ranks], Mu.h[ranks]
        got = orc.meth_profile(x, mu, sg, c, h, lp)
        want = brute_profile(x, mu, c, h, lp)
        assert got.view(np.uint32) == want.view(np.uint32), (trial, got, want)


def test_m3_one_kmer_window_closed_form(models):
    m, mm, Mu, Mm = models
    rng = np.random.default_rng(22)
    for trial in range(40):
        r = int(rng.integers(0, 4096))
        mev = int(rng.integers(1, 12))
        mu = np.array([m.level_mean[r]], F)
        x = (mu[0] + rng.normal(0, 2, mev)).astype(F)
        lp = orc.transitions(30, 20)
        c, h = F(Mu.c[r]), F(Mu.h[r])

        def em(v):
            d = F(v) - mu[0]
            return c - F(F(d * d) * h)

        want = F(F(F(0.0) + F(lp[2])) + em(x[0]))
        for v in x[1:]:
            want = F(F(want + F(lp[1])) + em(v))
        got = orc.meth_profile(x, mu, m.level_stdv[[r]], [c], [h], lp)
        assert got.view(np.uint32) == want.view(np.uint32)


def test_m4_sites_and_event_ranges(models, aligned):
    m, mm, Mu, Mm = models
    b, pairs, po, st = aligned
    llr, nev = orc.meth_batch(b, 6, Mu, Mm, pairs, po, st, n_threads=8)
    k = 6
    for r in range(b.n_reads):
        k0, k1 = int(b.kmer_offset[r]), int(b.kmer_offset[r + 1])
        rk = b.ranks[k0:k1].astype(np.int64)
        digits = np.stack([(rk >> (2 * (k - 1 - t))) & 3 for t in range(k)], 1)
        is_site = (digits[:, 0] == 1) & (digits[:, 1] == 2)
        assert np.array_equal(nev[k0:k1] > 0, is_site & (st[r] == 0)), r
        pr = pairs[int(po[r]):int(po[r + 1])]
        for i in np.nonzero(is_site)[0][:20]:
            j0 = max(0, i - k + 1)
            e0 = pr[pr[:, 1] == j0, 0].min()
            e1 = pr[pr[:, 1] == i, 0].max()
            assert nev[k0 + i] == e1 - e0 + 1, (r, i)


def test_m5_separates_methylated_reads(models, aligned):
    m, mm, Mu, Mm = models
    b, pairs, po, st = aligned
    llr, nev = orc.meth_batch(b, 6, Mu, Mm, pairs, po, st, n_threads=8)
    right = total = 0
    for r in range(b.n_reads):
        meth = synth.read_is_methylated("meth-4000-lognormal5kb", r, m)
        k0, k1 = int(b.kmer_offset[r]), int(b.kmer_offset[r + 1])
        v = llr[k0:k1][nev[k0:k1] > 0]
        if v.size == 0:
            continue
        right += int(((v > 0) if meth else (v < 0)).sum())
        total += v.size
        assert (v.sum() > 0) == meth, r
    assert right / total >= 0.95, right / total
