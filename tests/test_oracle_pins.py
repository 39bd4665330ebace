"""Pins of the CPU oracle against what the thesis and the mathematics fix.

Each test names the passage it checks (thesis Ch. 5).  None of them re-runs
the oracle's own formula to check itself: they use closed forms, a printed
worked example, brute force over every path on tiny inputs, an unbanded DP
written independently here, textbook Gaussian densities from scipy, exact
rational arithmetic, and invariants of the alignment.
"""

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from paper_2101_05012_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32
NINF = F32(-np.inf)


# ---------------------------------------------------------------- helpers

def round_f32(q: Fraction) -> np.float32:
    """Exact round-to-nearest-even of a rational to float32."""
    x = F32(float(q))
    cands = [np.nextafter(x, F32(-np.inf)), x, np.nextafter(x, F32(np.inf))]
    best = None
    for c in cands:
        err = abs(Fraction(float(c)) - q)
        key = (err, int(np.array(c, np.float32).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return F32(best[1])


def fma_f32(a, b, c) -> np.float32:
    return round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def em_f32(x, mu, c, h) -> np.float32:
    d = F32(F32(x) - F32(mu))
    t = F32(d * d)
    u = F32(t * F32(h))
    return F32(F32(c) - u)


def lp_consts(O, n_e, n_k):
    lp = O.transitions(n_e, n_k)
    return F32(lp[0]), F32(lp[1]), F32(lp[2])


def tiny_read(rng, n_e, n_k, model, scale=None, shift=None):
    ranks = rng.integers(0, model.level_mean.shape[0], n_k).astype(np.uint32)
    sc = F32(rng.uniform(0.9, 1.1)) if scale is None else F32(scale)
    sh = F32(rng.uniform(-5, 5)) if shift is None else F32(shift)
    # events drawn around the k-mers in order so that good paths exist
    owner = np.sort(rng.integers(0, n_k, n_e))
    x = np.array(
        [rng.normal(model.level_mean[ranks[o]] * sc + sh, model.level_stdv[ranks[o]]) for o in owner],
        np.float32,
    )
    return x, ranks, sc, sh


def brute_force(x, ranks, M, sc, sh, lp):
    """Best float32 path score over every monotone path from the origin to
    (n_e-1, n_k-1), summing in path order; returns (score, paths attaining it)."""
    lp_skip, lp_stay, lp_step = lp
    n_e, n_k = len(x), len(ranks)
    mu = [fma_f32(M.level_mean[r], sc, sh) for r in ranks]
    em = [[em_f32(x[e], mu[k], M.c[ranks[k]], M.h[ranks[k]]) for k in range(n_k)] for e in range(n_e)]
    best = [NINF, []]

    def rec(e, k, acc, path):
        if e == n_e - 1 and k == n_k - 1:
            if acc > best[0]:
                best[0], best[1] = acc, [list(path)]
            elif acc == best[0]:
                best[1].append(list(path))
            return
        if e + 1 < n_e and k + 1 < n_k:
            path.append((e + 1, k + 1))
            rec(e + 1, k + 1, F32(F32(acc + lp_step) + em[e + 1][k + 1]), path)
            path.pop()
        if e + 1 < n_e:
            path.append((e + 1, k))
            rec(e + 1, k, F32(F32(acc + lp_stay) + em[e + 1][k]), path)
            path.pop()
        if k + 1 < n_k:
            path.append((e, k + 1))
            rec(e, k + 1, F32(acc + lp_skip), path)
            path.pop()

    # the first cell is entered from the origin (-1, -1) by a diagonal step
    rec(0, 0, F32(F32(F32(0.0) + lp_step) + em[0][0]), [(0, 0)])
    return best[0], best[1]


def full_dp(x, ranks, M, sc, sh, lp):
    """Unbanded DP over the whole table (same recurrence and tie-break as the
    cell computation of Alg. 5.2), written independently of the oracle."""
    lp_skip, lp_stay, lp_step = lp
    n_e, n_k = len(x), len(ranks)
    S = np.full((n_e + 1, n_k + 1), NINF, np.float32)  # S[e+1, k+1]
    T = np.zeros((n_e + 1, n_k + 1), np.uint8)
    S[0, 0] = F32(0)
    for e in range(n_e):
        for k in range(n_k):
            r = ranks[k]
            mu = fma_f32(M.level_mean[r], sc, sh)
            em = em_f32(x[e], mu, M.c[r], M.h[r])
            sd = F32(F32(S[e, k] + lp_step) + em)
            su = F32(F32(S[e, k + 1] + lp_stay) + em)
            sl = F32(S[e + 1, k] + lp_skip)
            s, d = sd, 1
            if su > s:
                s, d = su, 2
            if sl > s:
                s, d = sl, 3
            S[e + 1, k + 1] = s
            T[e + 1, k + 1] = d
    e, k, path = n_e - 1, n_k - 1, []
    while e >= 0 and k >= 0:
        path.append((e, k))
        d = T[e + 1, k + 1]
        if d == 1:
            e, k = e - 1, k - 1
        elif d == 2:
            e -= 1
        else:
            k -= 1
    return S[n_e, n_k], path[::-1]


@pytest.fixture(scope="module")
def model6(oracle_mod):
    m = synth.pore_model(6)
    return oracle_mod.Model(m.level_mean, m.level_stdv)


@pytest.fixture(scope="module")
def model2(oracle_mod):
    m = synth.pore_model(2)
    return oracle_mod.Model(m.level_mean, m.level_stdv)


# ---------------------------------------------------------------- P1 constants

@pytest.mark.parametrize("n_e,n_k", [(100, 100), (171, 100), (180, 100), (200, 100), (250, 100), (1701, 995), (7, 5)])
def test_transition_constants_closed_form(oracle_mod, n_e, n_k):
    """Alg. 5.2 constants: lp_skip = ln(1e-10); lp_stay = ln(1 - 1/(epk+1))
    which equals ln(epk) - ln(epk+1); the three transition probabilities sum
    to one by construction of lp_step."""
    lp_skip, lp_stay, lp_step = lp_consts(oracle_mod, n_e, n_k)
    epk = n_e / n_k
    assert lp_skip == F32(-23.025850929940457)  # ln(1e-10) = -10 ln 10
    assert abs(float(lp_stay) - (math.log(epk) - math.log1p(epk))) <= 2 * np.spacing(abs(lp_stay))
    total = math.exp(float(lp_skip)) + math.exp(float(lp_stay)) + math.exp(float(lp_step))
    assert abs(total - 1.0) < 4e-7
    # probabilities of staying grows with events per k-mer
    assert lp_stay < 0 and lp_step < 0 and lp_skip < lp_stay


def test_transition_constants_one_event_per_kmer(oracle_mod):
    """epk = 1: staying and stepping are equally likely (1/2 each, minus the
    skip mass)."""
    lp_skip, lp_stay, lp_step = lp_consts(oracle_mod, 50, 50)
    assert lp_stay == F32(math.log(0.5))
    assert lp_step == F32(math.log(0.5))


def test_transition_constants_use_events_over_kmers(oracle_mod):
    """A transposed ratio (k-mers per event) would give different stay
    probabilities for n_e != n_k."""
    a = lp_consts(oracle_mod, 171, 100)[1]
    b = lp_consts(oracle_mod, 100, 171)[1]
    assert a != b
    assert a == F32(math.log(171 / 271))


# ---------------------------------------------------------------- P2 band limits

def _golden_limits():
    rows = []
    with open(os.path.join(GOLDEN, "band_limits_footnote.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, *vals = line.split()
            rows.append((name, *map(int, vals)))
    return rows


@pytest.mark.parametrize("row", _golden_limits(), ids=lambda r: r[0])
def test_band_limits_footnote(oracle_mod, row):
    """First footnote of Alg. 5.1: limits inside the bands of the worked
    example (13 events, 6 k-mers, W = 3)."""
    _, E, K, n_e, n_k, W, lo, hi = row
    assert oracle_mod.band_limits(E, K, n_e, n_k, W) == (lo, hi)


def test_band_limits_footnote_rest_of_bands(oracle_mod):
    """The footnote also says every band between b1 and b16 has limits
    [0, 2]; some sequence of single-step moves from b1 = (1, 0) to
    b16 = (13, 3) achieves that, and the end-band lower-lefts are unique."""
    n_e, n_k, W = 13, 6, 3
    reach = {(1, 0)}
    for _ in range(2, 16):
        nxt = set()
        for E, K in reach:
            for cand in ((E + 1, K), (E, K + 1)):
                if oracle_mod.band_limits(*cand, n_e, n_k, W) == (0, 2):
                    nxt.add(cand)
        reach = nxt
    assert any(((E + 1, K) == (13, 3) or (E, K + 1) == (13, 3)) for E, K in reach)
    # uniqueness of the last two lower-lefts given the footnote's limits
    ok17 = [(E, 17 - E) for E in range(0, 20) if oracle_mod.band_limits(E, 17 - E, n_e, n_k, W) == (1, 1)
            and 0 <= E - 12 < W]
    assert ok17 == [(13, 4)]
    ok16 = [p for p in ((12, 4), (13, 3)) if oracle_mod.band_limits(*p, n_e, n_k, W) == (1, 2)]
    assert ok16 == [(13, 3)]


# ---------------------------------------------------------------- P3 emission

@pytest.mark.parametrize("form", [0, 1])
def test_emission_is_gaussian_log_density(oracle_mod, model6, form):
    """Alg. 5.3: ln(1/sqrt(2 pi)) - ln(sigma) - z^2/2 is the log of the normal
    density; compare with scipy in double precision."""
    rng = np.random.default_rng(11)
    idx = rng.integers(0, model6.n, 4000)
    for r in idx[:4000]:
        sigma = model6.level_stdv[r]
        mu = F32(rng.uniform(55, 135))
        x = F32(mu + rng.normal(0, 3 * sigma))
        em = oracle_mod.emission(x, mu, sigma, model6.c[r], model6.h[r], form)
        ref = stats.norm.logpdf(float(x), float(mu), float(sigma))
        tol = 4 * np.spacing(F32(max(1.0, abs(ref))))
        assert abs(float(em) - ref) <= tol, (x, mu, sigma, em, ref)


def test_emission_at_mean_is_constant_term(oracle_mod, model6):
    for r in range(0, model6.n, 97):
        mu = F32(100.0)
        assert oracle_mod.emission(mu, mu, model6.level_stdv[r], model6.c[r], model6.h[r]) == model6.c[r]
        assert abs(float(model6.c[r]) - stats.norm.logpdf(0.0, 0.0, float(model6.level_stdv[r]))) < 1e-6


# ---------------------------------------------------------------- P4 brute force

@pytest.mark.parametrize("seed", range(40))
def test_banded_score_equals_best_path_by_brute_force(oracle_mod, model2, seed):
    """Max-plus recurrence of Alg. 5.2 on tiny reads with a band covering the
    whole table: the oracle's score is bit-identical to the best float32 path
    sum over every monotone path (rounding is monotone, so the DP maximum is
    the maximum path sum), and its path is one of the best paths."""
    rng = np.random.default_rng(seed)
    n_e = int(rng.integers(1, 8))
    n_k = int(rng.integers(1, 6))
    x, ranks, sc, sh = tiny_read(rng, n_e, n_k, model2)
    W = 2 * (n_e + n_k) + 4
    res = oracle_mod.align(x, ranks, model2, sc, sh, W)
    lp = lp_consts(oracle_mod, n_e, n_k)
    best, paths = brute_force(x, ranks, model2, sc, sh, lp)
    assert res.status == 0
    assert res.score == best
    assert [tuple(p) for p in res.pairs.tolist()] in [list(map(tuple, p)) for p in paths]


def test_brute_force_catches_planted_mistakes(oracle_mod, model2):
    """A dropped term or a wrong index planted in the oracle changes its score
    on tiny reads, so the brute-force pin would fail."""
    caught = {oracle_mod.PLANT_DROP_UP_EMISSION: 0, oracle_mod.PLANT_EVENT_OFF_BY_ONE: 0}
    for seed in range(40):
        rng = np.random.default_rng(seed)
        n_e, n_k = int(rng.integers(2, 8)), int(rng.integers(2, 6))
        x, ranks, sc, sh = tiny_read(rng, n_e, n_k, model2)
        W = 2 * (n_e + n_k) + 4
        best, _ = brute_force(x, ranks, model2, sc, sh, lp_consts(oracle_mod, n_e, n_k))
        for flag in caught:
            if oracle_mod.align(x, ranks, model2, sc, sh, W, flags=flag).score != best:
                caught[flag] += 1
    assert all(v > 0 for v in caught.values()), caught


# ---------------------------------------------------------------- P5 full DP

@pytest.mark.parametrize("seed", range(12))
def test_banded_equals_unbanded_dp_when_band_covers_table(oracle_mod, model6, seed):
    rng = np.random.default_rng(100 + seed)
    n_e = int(rng.integers(5, 40))
    n_k = int(rng.integers(3, 25))
    x, ranks, sc, sh = tiny_read(rng, n_e, n_k, model6)
    W = 2 * (n_e + n_k) + 4
    res = oracle_mod.align(x, ranks, model6, sc, sh, W, want_trace=True)
    # explicit coverage check: every table cell lies in its anti-diagonal band
    for e in range(n_e):
        for k in range(n_k):
            E, K = res.ll[e + k + 2]
            j = E - e
            assert 0 <= j < W and K + j == k
    score, path = full_dp(x, ranks, model6, sc, sh, lp_consts(oracle_mod, n_e, n_k))
    assert res.score == score
    assert [tuple(p) for p in res.pairs.tolist()] == path
    assert res.cells == n_e * n_k


# ---------------------------------------------------------------- P6 noiseless

@pytest.mark.parametrize("L", [6, 7, 50, 300, 1000, 4000])
def test_noiseless_reads_align_on_the_diagonal(oracle_mod, L):
    """One event per k-mer with the event mean equal to the k-mer level: the
    best alignment is the diagonal (any other step costs at least
    -lp_skip - (lp_stay - lp_step) - |ln sigma - ln sigma'| > 0), and the
    adaptive band has to follow it for the whole read at W = 100."""
    m = synth.pore_model(6)
    M = oracle_mod.Model(m.level_mean, m.level_stdv)
    b = synth.noiseless_batch(3, L, m, seed=L)
    for i in range(b.n_reads):
        rd = b.read(i)
        res = oracle_mod.align(rd.events, rd.ranks, M, 1.0, 0.0, 100)
        n = rd.ranks.shape[0]
        assert res.status == 0
        assert np.array_equal(res.pairs, np.stack([np.arange(n), np.arange(n)], 1))
        lp_skip, lp_stay, lp_step = lp_consts(oracle_mod, n, n)
        acc = F32(0)
        for kk in range(n):
            acc = F32(F32(acc + lp_step) + M.c[rd.ranks[kk]])
        assert res.score == acc


def test_noiseless_catches_reversed_band_rule(oracle_mod):
    """The band-move direction is the reading least fixed by the text; moving
    the band away from the better end (the planted mistake) loses the
    diagonal on noiseless reads."""
    m = synth.pore_model(6)
    M = oracle_mod.Model(m.level_mean, m.level_stdv)
    b = synth.noiseless_batch(3, 1000, m, seed=5)
    lost = 0
    for i in range(b.n_reads):
        rd = b.read(i)
        n = rd.ranks.shape[0]
        res = oracle_mod.align(rd.events, rd.ranks, M, 1.0, 0.0, 100, flags=oracle_mod.PLANT_SK_REVERSED)
        diag = np.stack([np.arange(n), np.arange(n)], 1)
        if res.status != 0 or not np.array_equal(res.pairs, diag):
            lost += 1
    assert lost == b.n_reads


# ---------------------------------------------------------------- P7 path invariants

def rescore(pairs, x, ranks, M, sc, sh, lp, dtype):
    lp_skip, lp_stay, lp_step = (dtype(v) for v in lp)
    acc = dtype(0)
    pe, pk = -1, -1
    for e, k in pairs:
        r = ranks[k]
        if dtype is F32:
            em = em_f32(x[e], fma_f32(M.level_mean[r], sc, sh), M.c[r], M.h[r])
        else:
            em = stats.norm.logpdf(float(x[e]), float(M.level_mean[r]) * float(sc) + float(sh), float(M.level_stdv[r]))
        if (e - pe, k - pk) == (1, 1):
            acc = dtype(dtype(acc + lp_step) + em)
        elif (e - pe, k - pk) == (1, 0):
            acc = dtype(dtype(acc + lp_stay) + em)
        else:
            acc = dtype(acc + lp_skip)
        pe, pk = e, k
    return acc


def test_path_invariants_64x1kb(oracle_mod, model6):
    b = synth.workload_batch("plain-64x1kb", synth.pore_model(6), read_ids=range(16))
    for i in range(b.n_reads):
        rd = b.read(i)
        x = rd.events[:, 0]
        res = oracle_mod.align(rd.events, rd.ranks, model6, rd.scale, rd.shift, 100)
        n_e, n_k = len(x), len(rd.ranks)
        assert res.status == 0
        p = res.pairs
        assert tuple(p[0]) == (0, 0) and tuple(p[-1]) == (n_e - 1, n_k - 1)
        steps = {tuple(s) for s in np.diff(p, axis=0).tolist()}
        assert steps <= {(1, 1), (1, 0), (0, 1)}
        assert set(p[:, 0].tolist()) == set(range(n_e))
        assert set(p[:, 1].tolist()) == set(range(n_k))
        lp = lp_consts(oracle_mod, n_e, n_k)
        pl = [tuple(v) for v in p.tolist()]
        assert rescore(pl, x, rd.ranks, model6, rd.scale, rd.shift, lp, F32) == res.score
        dbl = rescore(pl, x, rd.ranks, model6, rd.scale, rd.shift, lp, float)
        # float32 summation error bound: two roundings per path step, each at
        # most half an ulp of the running score (|running| <= |final|)
        bound = len(pl) * float(np.spacing(F32(abs(res.score)))) + 1e-3
        assert abs(dbl - float(res.score)) <= bound
        assert res.cells > 0 and res.cells <= 100 * (n_e + n_k - 1)


# ---------------------------------------------------------------- P8 scaling

def test_model_scaling_is_a_single_rounding_fma(oracle_mod, model6):
    """Read-model scaling (paragraph after Alg. 5.3): mu = mean*scale + shift
    with one rounding.  Aligning with (scale, shift) equals aligning against a
    model whose means were scaled exactly here, with scale 1 and shift 0."""
    b = synth.workload_batch("plain-64x1kb", synth.pore_model(6), read_ids=range(3))
    for i in range(b.n_reads):
        rd = b.read(i)
        used = np.unique(rd.ranks)
        lm2 = model6.level_mean.copy()
        for r in used:
            lm2[r] = fma_f32(model6.level_mean[r], rd.scale, rd.shift)
        M2 = oracle_mod.Model(lm2, model6.level_stdv)
        a = oracle_mod.align(rd.events, rd.ranks, model6, rd.scale, rd.shift, 100)
        c = oracle_mod.align(rd.events, rd.ranks, M2, 1.0, 0.0, 100)
        assert a.score == c.score and np.array_equal(a.pairs, c.pairs)


# ---------------------------------------------------------------- special cases

def test_empty_and_bad_rank(oracle_mod, model6):
    x = np.array([80.0, 81.0], np.float32)
    assert oracle_mod.align(x[:0], np.array([1, 2], np.uint32), model6, 1, 0, 100).status == oracle_mod.READ_EMPTY
    assert oracle_mod.align(x, np.array([], np.uint32), model6, 1, 0, 100).status == oracle_mod.READ_EMPTY
    r = oracle_mod.align(x, np.array([1, 4096], np.uint32), model6, 1, 0, 100)
    assert r.status == oracle_mod.READ_BAD_RANK and r.score == NINF and len(r.pairs) == 0


def test_single_cell_read(oracle_mod, model6):
    x = np.array([90.0], np.float32)
    rk = np.array([17], np.uint32)
    res = oracle_mod.align(x, rk, model6, 1.0, 0.0, 100)
    lp_skip, lp_stay, lp_step = lp_consts(oracle_mod, 1, 1)
    assert res.status == 0 and res.pairs.tolist() == [[0, 0]]
    assert res.score == F32(F32(F32(0) + lp_step) + em_f32(90.0, model6.level_mean[17], model6.c[17], model6.h[17]))
    assert res.cells == 1


def test_band_follows_table_edges_on_fuzzed_reads(oracle_mod):
    """The band-move rule never loses the terminal cell, even with W = 2 or 3
    and unrelated events: when one end cell of a band leaves the table its
    score is -inf and the rule moves the band back towards the other end.
    (The BAND_LOST status exists for robustness; no input found reaches it.)"""
    m = synth.pore_model(2)
    M = oracle_mod.Model(m.level_mean, m.level_stdv)
    for seed in range(1500):
        rng = np.random.default_rng(seed)
        n_k, n_e, W = int(rng.integers(1, 12)), int(rng.integers(1, 12)), int(rng.integers(2, 4))
        rk = rng.integers(0, 16, n_k).astype(np.uint32)
        x = rng.uniform(60, 130, n_e).astype(np.float32)
        r = oracle_mod.align(x, rk, M, 1.0, 0.0, W)
        assert r.status == oracle_mod.READ_OK
        assert tuple(r.pairs[-1]) == (n_e - 1, n_k - 1)


# ---------------------------------------------------------------- P9 forms

def test_literal_and_canonical_emission_forms_agree(oracle_mod, model6):
    """The canonical emission (multiply by 0.5/sigma^2) and the literal one
    (divide by sigma, then square and halve) are the same function up to a few
    ulp; alignments agree except on reads whose decisions hinge on an exact
    float32 tie, and scores agree to 1e-5 relative."""
    m = synth.pore_model(6)
    b = synth.workload_batch("plain-64x1kb", m, read_ids=range(64, 464))
    nt = max(1, min(8, os.cpu_count() or 1))
    r0 = oracle_mod.align_batch(b, model6, 100, n_threads=nt, flags=0)
    r1 = oracle_mod.align_batch(b, model6, 100, n_threads=nt, flags=oracle_mod.FORM_LITERAL)
    assert np.array_equal(r0.status, r1.status)
    ok = r0.status == 0
    rel = np.abs(r0.score[ok].astype(np.float64) - r1.score[ok]) / np.abs(r0.score[ok].astype(np.float64))
    assert rel.max() <= 1e-5
    same = sum(np.array_equal(r0.read_pairs(i), r1.read_pairs(i)) for i in range(b.n_reads))
    assert same >= 0.999 * b.n_reads


def test_batch_driver_matches_single_read_calls(oracle_mod, model6):
    b = synth.workload_batch("plain-64x1kb", synth.pore_model(6), read_ids=range(8))
    rb = oracle_mod.align_batch(b, model6, 100, n_threads=3)
    for i in range(b.n_reads):
        rd = b.read(i)
        r = oracle_mod.align(rd.events, rd.ranks, model6, rd.scale, rd.shift, 100)
        assert rb.status[i] == r.status and rb.score[i] == r.score and rb.cells[i] == r.cells
        assert np.array_equal(rb.read_pairs(i), r.pairs)


# ---------------------------------------------------------------- P9 events scaled to the model

def scaled_events_f32(x, sc, sh):
    """x' = (x - shift) / scale, each operation rounded to float32 (numpy's
    float32 arithmetic is IEEE round-to-nearest-even)."""
    x = np.asarray(x, np.float32)
    return (x - F32(sh)) / F32(sc)


@pytest.mark.parametrize("seed", range(4))
def test_scale_events_single_cell_is_gaussian_of_scaled_event(oracle_mod, model6, seed):
    """Paragraph after Alg. 5.3, events scaled to the model: a one-event,
    one-k-mer read scores lp_step + ln N((x - shift)/scale; mu, sigma) with the
    model level unscaled.  Reference in double precision from scipy; a shift
    added instead of subtracted, a product instead of a quotient, or a model
    level still scaled moves the score far outside the tolerance."""
    rng = np.random.default_rng(500 + seed)
    lp_step = float(oracle_mod.transitions(1, 1)[2])
    for _ in range(300):
        r = int(rng.integers(0, model6.n))
        sc = F32(rng.uniform(0.8, 1.25))
        sh = F32(rng.choice([-1, 1]) * rng.uniform(1.0, 5.0))
        mu = float(model6.level_mean[r])
        sigma = float(model6.level_stdv[r])
        x = F32((mu + rng.normal(0, 2 * sigma)) * float(sc) + float(sh))
        res = oracle_mod.align(np.array([x], np.float32), np.array([r], np.uint32), model6, sc, sh, 100,
                               flags=oracle_mod.SCALE_EVENTS)
        assert res.status == 0 and res.pairs.tolist() == [[0, 0]]
        xp = (float(x) - float(sh)) / float(sc)
        ref = lp_step + stats.norm.logpdf(xp, mu, sigma)
        # float32 rounding of x', of the emission's four operations and of the two adds
        tol = 8 * float(np.spacing(F32(max(1.0, abs(ref))))) + abs(xp - mu) / sigma ** 2 * abs(xp) * 2.0 ** -22
        assert abs(float(res.score) - ref) <= tol, (x, sc, sh, r, res.score, ref)


@pytest.mark.parametrize("shift", [0.0, 3.0, -4.5])
def test_scale_events_at_unit_scale_equals_model_scaling_exactly(oracle_mod, shift):
    """With scale 1 both modes compare x - (m + shift) and (x - shift) - m.
    On inputs where both are exact (model levels and events on a 1/64 grid)
    they are the same number, so the two modes give identical alignments."""
    rng = np.random.default_rng(77)
    n_model = 4 ** 4
    lm = (rng.integers(60 * 64, 130 * 64, n_model) / 64.0).astype(np.float32)
    ls = rng.uniform(1.0, 3.0, n_model).astype(np.float32)
    M = oracle_mod.Model(lm, ls)
    for _ in range(6):
        n_k = int(rng.integers(50, 200))
        ranks = rng.integers(0, n_model, n_k).astype(np.uint32)
        owner = np.sort(rng.integers(0, n_k, int(1.7 * n_k)))
        x = (lm[ranks[owner]] + rng.integers(-3 * 64, 3 * 64, owner.size) / 64.0 + shift).astype(np.float32)
        a = oracle_mod.align(x, ranks, M, 1.0, shift, 100)
        b = oracle_mod.align(x, ranks, M, 1.0, shift, 100, flags=oracle_mod.SCALE_EVENTS)
        assert a.status == b.status == 0
        assert a.score == b.score and np.array_equal(a.pairs, b.pairs) and a.cells == b.cells


@pytest.mark.parametrize("seed", range(20))
def test_scale_events_banded_score_equals_best_path_by_brute_force(oracle_mod, model2, seed):
    """The max-plus recurrence over scaled events: with a band covering the
    table the oracle's score is the best float32 path sum over every path,
    and its path is one of the best."""
    rng = np.random.default_rng(900 + seed)
    n_e = int(rng.integers(1, 8))
    n_k = int(rng.integers(1, 6))
    x, ranks, sc, sh = tiny_read(rng, n_e, n_k, model2)
    W = 2 * (n_e + n_k) + 4
    res = oracle_mod.align(x, ranks, model2, sc, sh, W, flags=oracle_mod.SCALE_EVENTS)
    lp = lp_consts(oracle_mod, n_e, n_k)
    # scaled events against the unscaled model: scale 1 and shift 0 in the helper
    best, paths = brute_force(scaled_events_f32(x, sc, sh), ranks, model2, 1.0, 0.0, lp)
    assert res.status == 0
    assert res.score == best
    assert [tuple(p) for p in res.pairs.tolist()] in [list(map(tuple, p)) for p in paths]
