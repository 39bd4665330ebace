"""Seeded synthetic ABEA inputs: pore models, reads, events and batches.

This module only draws random numbers and lays them out; it holds none of the
alignment's arithmetic, so both the HIP path and the CPU oracle can take their
inputs from it.

The workloads stand in for the nanopore datasets the thesis measures on
(Ch. 5, Table "Information of the datasets": NA12878 D_small, D_ligation,
D_rapid), which are not available here.  What is drawn, and why:

* Pore model over all 4^k k-mers (Ch. 5 §5.2.1, figure "an example
  pore-model"): level_mean ~ U(60, 130) pA, level_stdv ~ U(1, 3), float32.
  The k-mer rank is the base-4 number of the k-mer (A=0, C=1, G=2, T=3, first
  base most significant).
* A read is a uniform i.i.d. ACGT reference of length L; it has n_k = L-k+1
  k-mers.  Per read, scale ~ U(0.9, 1.1) and shift ~ U(-5, 5) (the per-read
  read-model scaling paragraph after Alg. 5.3).
* Events: each k-mer position is skipped (0 events) with probability 0.05,
  otherwise it emits Geometric(p=1/1.8) events on {1, 2, ...} (mean 1.8), so
  there are about 1.71 events per k-mer (over-segmentation, §5.2.3: "usually
  by a factor 1.5-2").  Each event has mean ~ N(level_mean*scale + shift,
  level_stdv), stdv ~ U(0.5, 3), duration ~ Exp(mean 2.5 ms), all float32.
  Only the mean is read by the alignment (Alg. 5.3).

Raw signal (the input of event detection, Ch. 5 §5.2.2 "Methylation
calling"; sampling figures of the "Nanopore sequencing and the raw signal"
paragraph): the current is sampled at 4000 Hz while the strand moves at about
450 bases/s, so a k-mer dwells about 8.9 samples on average.  Each k-mer's
dwell is round(Gamma(shape 2, mean 8.89)), at least 1 sample (the speed
varies: the signal warps in time).  Each sample is
level_mean*scale + shift + N(0, level_stdv) pA, digitised as
round(pA / pa_scale - offset) into int16 with, per read,
pa_scale = U(1380, 1420) pA / 8192 levels and offset ~ U(-20, 20): the
reading back to pA is (raw + offset) * pa_scale.

Methylation (row f3 of the scope; Ch. 5 §5.2.2 names HMM profiling of the
aligned events as the step after the alignment): a synthetic methylated pore
model equals the pore model except that every k-mer containing the
dinucleotide CG has its level shifted by +-U(2, 5) pA (seeded per k); a read
of a methylation workload is methylated with probability 1/2, and then the
events of its CG-containing k-mers are drawn from the methylated levels.

Every read draws from its own stream ``default_rng([workload_seed, read_id])``,
so a read's bytes do not depend on which batch it is in or where.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

MODEL_SEED_BASE = 1000
WORKLOAD_SEED_BASE = 2026_0000

SKIP_PROB = 0.05
EVENTS_PER_KMER_MEAN = 1.8

# Events outside the molecule (the trim paragraph after Alg. 5.3): open-pore
# current before and after the read, and adaptor events between the leading
# open pore and the read.  Open-pore current is far above every k-mer level
# of the model (60..130 pA); adaptor events take arbitrary levels in the
# model's range.
OPEN_PORE_MEAN, OPEN_PORE_SD = 220.0, 4.0
MAX_OPEN_PORE_EVENTS = 30
MAX_ADAPTOR_EVENTS = 10

# Workload shapes.  W is the band width, k the k-mer length.
WORKLOADS = {
    "plain-64x1kb": dict(seed_index=0, n_reads=64, W=100, k=6, lengths="fixed1000"),
    "plain-4000-lognormal5kb": dict(seed_index=1, n_reads=4000, W=100, k=6, lengths="lognormal5k"),
    "uneven-20000": dict(seed_index=2, n_reads=20000, W=100, k=6, lengths="mixed"),
    "serving-lognormal8kb": dict(seed_index=3, n_reads=None, W=100, k=6, lengths="lognormal8k"),
    "ultralong-200": dict(seed_index=4, n_reads=200, W=100, k=6, lengths="ultralong"),
    # the 4000-read log-normal lengths with open-pore and adaptor events at
    # the read ends
    "plain-4000-lognormal5kb-ends": dict(seed_index=5, n_reads=4000, W=100, k=6, lengths="lognormal5k",
                                         ends=True),
    # plain-4000's length mix, each read methylated with probability 1/2
    "meth-4000-lognormal5kb": dict(seed_index=7, n_reads=4000, W=100, k=6, lengths="lognormal5k", meth=True),
    # raw signal of reads of the same length mix (event detection's input)
    "raw-4000-lognormal5kb": dict(seed_index=6, n_reads=4000, W=100, k=6, lengths="lognormal5k", raw=True),
    # raw signal again, each read methylated with probability 1/2: the input of
    # the whole pipeline (event detection, alignment, methylation scoring)
    "pipeline-4000-lognormal5kb": dict(seed_index=8, n_reads=4000, W=100, k=6, lengths="lognormal5k", raw=True,
                                       meth=True),
}

SAMPLE_RATE_HZ = 4000.0
BASES_PER_S = 450.0
DWELL_GAMMA_SHAPE = 2.0
RAW_DIGITISATION = 8192.0
RAW_RANGE_PA = (1380.0, 1420.0)
RAW_OFFSET = (-20.0, 20.0)


@dataclasses.dataclass
class PoreModel:
    k: int
    level_mean: np.ndarray  # float32 [4^k]
    level_stdv: np.ndarray  # float32 [4^k]


@dataclasses.dataclass
class Read:
    events: np.ndarray  # float32 [n_e, 3] = (mean, stdv, duration)
    ranks: np.ndarray  # uint32 [n_k]
    scale: np.float32
    shift: np.float32


@dataclasses.dataclass
class Batch:
    """Concatenated reads with exclusive prefix-sum offsets (the serialised
    batch layout of Ch. 5 §5.4.2.1, Alg. 5.9)."""

    events: np.ndarray  # float32 [sum n_e, 3]
    event_offset: np.ndarray  # uint64 [n+1]
    ranks: np.ndarray  # uint32 [sum n_k]
    kmer_offset: np.ndarray  # uint64 [n+1]
    scale: np.ndarray  # float32 [n]
    shift: np.ndarray  # float32 [n]

    @property
    def n_reads(self) -> int:
        return int(self.scale.shape[0])

    def n_events(self, i: int) -> int:
        return int(self.event_offset[i + 1] - self.event_offset[i])

    def n_kmers(self, i: int) -> int:
        return int(self.kmer_offset[i + 1] - self.kmer_offset[i])

    def read(self, i: int) -> Read:
        e0, e1 = int(self.event_offset[i]), int(self.event_offset[i + 1])
        k0, k1 = int(self.kmer_offset[i]), int(self.kmer_offset[i + 1])
        return Read(self.events[e0:e1], self.ranks[k0:k1], self.scale[i], self.shift[i])

    def subset(self, idx: Sequence[int]) -> "Batch":
        return make_batch([self.read(int(i)) for i in idx])


def kmer_has_cpg(ranks: np.ndarray, k: int) -> np.ndarray:
    """True for each rank whose k-mer contains the dinucleotide CG (C = 1,
    G = 2; the first base is the most significant digit)."""
    r = np.asarray(ranks, np.int64)
    out = np.zeros(r.shape, bool)
    for t in range(k - 1):
        b0 = (r >> (2 * (k - 1 - t))) & 3
        b1 = (r >> (2 * (k - 2 - t))) & 3
        out |= (b0 == 1) & (b1 == 2)
    return out


def methylated_model(model: PoreModel, seed: Optional[int] = None) -> PoreModel:
    """The pore model with every CG-containing k-mer's level shifted by
    +-U(2, 5) pA; level_stdv unchanged."""
    k = model.k
    rng = np.random.default_rng(MODEL_SEED_BASE + 100 + k if seed is None else seed)
    n = 4**k
    shift = rng.uniform(2.0, 5.0, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    cpg = kmer_has_cpg(np.arange(n), k)
    lm = (model.level_mean.astype(np.float64) + np.where(cpg, shift, 0.0)).astype(np.float32)
    return PoreModel(k, lm, model.level_stdv.copy())


def pore_model(k: int, seed: Optional[int] = None) -> PoreModel:
    rng = np.random.default_rng(MODEL_SEED_BASE + k if seed is None else seed)
    n = 4**k
    lm = rng.uniform(60.0, 130.0, n).astype(np.float32)
    ls = rng.uniform(1.0, 3.0, n).astype(np.float32)
    return PoreModel(k, lm, ls)


def kmer_ranks(bases: np.ndarray, k: int) -> np.ndarray:
    """Rank of every k-mer of a base array (values 0..3), first base most
    significant."""
    L = bases.shape[0]
    n = L - k + 1
    if n <= 0:
        return np.zeros(0, np.uint32)
    r = np.zeros(n, np.uint64)
    for t in range(k):
        r = r * np.uint64(4) + bases[t : t + n].astype(np.uint64)
    return r.astype(np.uint32)


def draw_length(rng: np.random.Generator, kind: str) -> int:
    if kind == "fixed1000":
        return 1000
    if kind == "lognormal5k":
        return int(np.clip(round(math.exp(rng.normal(math.log(5000.0), 1.0))), 200, 100_000))
    if kind == "lognormal8k":
        return int(np.clip(round(math.exp(rng.normal(math.log(8000.0), 1.0))), 200, 1_000_000))
    if kind == "mixed":
        if rng.random() < 0.7:
            return int(rng.integers(500, 5001))
        return int(rng.integers(20_000, 200_001))
    if kind == "ultralong":
        return int(rng.integers(200_000, 1_000_001))
    raise ValueError(kind)


def gen_read(
    rng: np.random.Generator,
    L: int,
    model: PoreModel,
    noiseless: bool = False,
    ends: bool = False,
    meth_model: Optional[PoreModel] = None,
) -> Read:
    """Draw one read of reference length L (see the module docstring).

    ``noiseless``: one event per k-mer, scale 1, shift 0 and every event mean
    equal to the model level of its k-mer, so the model levels need no scaling.
    ``meth_model``: with probability 1/2 (drawn after the event counts) the
    event means come from its levels (a methylated read).
    ``ends``: the read is preceded by U{0..30} open-pore events and U{0..10}
    adaptor events and followed by U{0..30} open-pore events (drawn after
    everything else, so the read's own events are those without ``ends``).
    """
    k = model.k
    bases = rng.integers(0, 4, L).astype(np.uint8)
    ranks = kmer_ranks(bases, k)
    n_k = ranks.shape[0]
    if noiseless:
        ev = np.zeros((n_k, 3), np.float32)
        ev[:, 0] = model.level_mean[ranks]
        ev[:, 1] = 1.0
        ev[:, 2] = 0.0025
        return Read(ev, ranks, np.float32(1.0), np.float32(0.0))
    scale = np.float32(rng.uniform(0.9, 1.1))
    shift = np.float32(rng.uniform(-5.0, 5.0))
    skipped = rng.random(n_k) < SKIP_PROB
    cnt = rng.geometric(1.0 / EVENTS_PER_KMER_MEAN, n_k)
    cnt[skipped] = 0
    r_ev = np.repeat(ranks, cnt)
    n_e = r_ev.shape[0]
    levels = model.level_mean
    if meth_model is not None and rng.random() < 0.5:
        levels = meth_model.level_mean  # a methylated read: CG k-mers at the methylated levels
    loc = levels[r_ev].astype(np.float64) * float(scale) + float(shift)
    ev = np.empty((n_e, 3), np.float32)
    ev[:, 0] = rng.normal(loc, model.level_stdv[r_ev].astype(np.float64))
    ev[:, 1] = rng.uniform(0.5, 3.0, n_e)
    ev[:, 2] = rng.exponential(0.0025, n_e)
    if ends:
        ev = np.concatenate([end_events(rng, True), ev, end_events(rng, False)])
    return Read(ev, ranks, scale, shift)


def end_events(rng: np.random.Generator, leading: bool) -> np.ndarray:
    """Events outside the molecule: open pore (and, before the read, adaptor
    events after it), as [n, 3] float32 (mean, stdv, duration)."""
    n_open = int(rng.integers(0, MAX_OPEN_PORE_EVENTS + 1))
    n_adapt = int(rng.integers(0, MAX_ADAPTOR_EVENTS + 1)) if leading else 0
    n = n_open + n_adapt
    ev = np.empty((n, 3), np.float32)
    ev[:n_open, 0] = rng.normal(OPEN_PORE_MEAN, OPEN_PORE_SD, n_open)
    ev[n_open:, 0] = rng.uniform(60.0, 130.0, n_adapt)
    ev[:, 1] = rng.uniform(0.5, 3.0, n)
    ev[:, 2] = rng.exponential(0.0025, n)
    return ev


@dataclasses.dataclass
class RawRead:
    raw: np.ndarray  # int16 [n_samples]
    ranks: np.ndarray  # uint32 [n_k]
    offset: np.float32  # pA = (raw + offset) * pa_scale
    pa_scale: np.float32
    scale: np.float32  # model scaling of the alignment (mu' = level_mean * scale + shift)
    shift: np.float32
    dwell: np.ndarray  # int64 [n_k]: samples of each k-mer (ground truth)
    methylated: bool = False  # drawn from the methylated levels (ground truth)


@dataclasses.dataclass
class RawBatch:
    """Concatenated raw reads with exclusive prefix-sum offsets."""

    raw: np.ndarray  # int16 [sum n]
    sample_offset: np.ndarray  # uint64 [n+1]
    ranks: np.ndarray  # uint32 [sum n_k]
    kmer_offset: np.ndarray  # uint64 [n+1]
    offset: np.ndarray  # float32 [n]
    pa_scale: np.ndarray  # float32 [n]
    scale: np.ndarray  # float32 [n]
    shift: np.ndarray  # float32 [n]
    dwell: np.ndarray  # int64 [sum n_k]
    methylated: Optional[np.ndarray] = None  # bool [n]

    @property
    def n_reads(self) -> int:
        return int(self.offset.shape[0])

    def read_raw(self, i: int) -> np.ndarray:
        return self.raw[int(self.sample_offset[i]) : int(self.sample_offset[i + 1])]

    def read_ranks(self, i: int) -> np.ndarray:
        return self.ranks[int(self.kmer_offset[i]) : int(self.kmer_offset[i + 1])]


def gen_raw_read(rng: np.random.Generator, L: int, model: PoreModel, noiseless: bool = False,
                 meth_model: Optional[PoreModel] = None) -> RawRead:
    """Raw signal of one read of reference length L (see the module
    docstring).  ``noiseless``: every sample is exactly its k-mer's level.
    ``meth_model``: with probability 1/2 (drawn after everything else) the
    levels come from it (a methylated read); the draw is kept in
    ``RawRead.methylated``."""
    k = model.k
    bases = rng.integers(0, 4, L).astype(np.uint8)
    ranks = kmer_ranks(bases, k)
    n_k = ranks.shape[0]
    scale = np.float32(rng.uniform(0.9, 1.1))
    shift = np.float32(rng.uniform(-5.0, 5.0))
    mean_dwell = SAMPLE_RATE_HZ / BASES_PER_S
    dwell = np.maximum(1, np.round(rng.gamma(DWELL_GAMMA_SHAPE, mean_dwell / DWELL_GAMMA_SHAPE, n_k))).astype(
        np.int64)
    r = np.repeat(ranks, dwell)
    noise = None if noiseless else rng.normal(0.0, 1.0, r.shape[0])
    pa_scale = np.float32(rng.uniform(*RAW_RANGE_PA) / RAW_DIGITISATION)
    offset = np.float32(rng.uniform(*RAW_OFFSET))
    methylated = bool(meth_model is not None and rng.random() < 0.5)
    levels = meth_model.level_mean if methylated else model.level_mean
    pa = levels[r].astype(np.float64) * float(scale) + float(shift)
    if noise is not None:
        pa = pa + noise * model.level_stdv[r].astype(np.float64)
    raw = np.clip(np.round(pa / float(pa_scale) - float(offset)), -32768, 32767).astype(np.int16)
    return RawRead(raw, ranks, offset, pa_scale, scale, shift, dwell, methylated)


def make_raw_batch(reads: Sequence[RawRead]) -> RawBatch:
    n = len(reads)
    ns = np.array([r.raw.shape[0] for r in reads], np.uint64)
    nk = np.array([r.ranks.shape[0] for r in reads], np.uint64)
    so = np.zeros(n + 1, np.uint64)
    ko = np.zeros(n + 1, np.uint64)
    np.cumsum(ns, out=so[1:])
    np.cumsum(nk, out=ko[1:])

    def cat(xs, dt):
        return np.ascontiguousarray(np.concatenate(xs) if n else np.zeros(0, dt), dt)

    return RawBatch(
        cat([r.raw for r in reads], np.int16), so, cat([r.ranks for r in reads], np.uint32), ko,
        np.array([r.offset for r in reads], np.float32), np.array([r.pa_scale for r in reads], np.float32),
        np.array([r.scale for r in reads], np.float32), np.array([r.shift for r in reads], np.float32),
        cat([r.dwell for r in reads], np.int64),
        np.array([r.methylated for r in reads], bool),
    )


def workload_raw_batch(workload: str, model: Optional[PoreModel] = None,
                       read_ids: Optional[Sequence[int]] = None) -> RawBatch:
    """Raw reads of a raw-signal workload; read ``i`` is identical whatever
    batch it is in."""
    cfg = WORKLOADS[workload]
    assert cfg.get("raw"), workload
    if model is None:
        model = pore_model(cfg["k"])
    if read_ids is None:
        read_ids = range(cfg["n_reads"])
    mm = methylated_model(model) if cfg.get("meth") else None
    out = []
    for i in read_ids:
        rng = read_rng(workload, int(i))
        out.append(gen_raw_read(rng, draw_length(rng, cfg["lengths"]), model, meth_model=mm))
    return make_raw_batch(out)


def make_batch(reads: Sequence[Read]) -> Batch:
    n = len(reads)
    ne = np.array([r.events.shape[0] for r in reads], np.uint64)
    nk = np.array([r.ranks.shape[0] for r in reads], np.uint64)
    eo = np.zeros(n + 1, np.uint64)
    ko = np.zeros(n + 1, np.uint64)
    np.cumsum(ne, out=eo[1:])
    np.cumsum(nk, out=ko[1:])
    ev = np.concatenate([r.events for r in reads]) if n else np.zeros((0, 3), np.float32)
    rk = np.concatenate([r.ranks for r in reads]) if n else np.zeros(0, np.uint32)
    return Batch(
        np.ascontiguousarray(ev, np.float32).reshape(-1, 3),
        eo,
        np.ascontiguousarray(rk, np.uint32),
        ko,
        np.array([r.scale for r in reads], np.float32),
        np.array([r.shift for r in reads], np.float32),
    )


def workload_seed(workload: str) -> int:
    return WORKLOAD_SEED_BASE + WORKLOADS[workload]["seed_index"]


def read_rng(workload: str, read_id: int) -> np.random.Generator:
    return np.random.default_rng([workload_seed(workload), read_id])


def workload_read(workload: str, read_id: int, model: PoreModel) -> Read:
    """Read ``read_id`` of a workload; identical whatever batch it is in."""
    rng = read_rng(workload, read_id)
    cfg = WORKLOADS[workload]
    L = draw_length(rng, cfg["lengths"])
    mm = methylated_model(model) if cfg.get("meth") else None
    return gen_read(rng, L, model, ends=cfg.get("ends", False), meth_model=mm)


def workload_batch(
    workload: str,
    model: Optional[PoreModel] = None,
    read_ids: Optional[Sequence[int]] = None,
) -> Batch:
    cfg = WORKLOADS[workload]
    if model is None:
        model = pore_model(cfg["k"])
    if read_ids is None:
        read_ids = range(cfg["n_reads"])
    return make_batch([workload_read(workload, int(i), model) for i in read_ids])


def _workload_chunk(args):
    """Generate reads ``ids`` of a workload into a shared-memory block of its
    own (returned by name, so that the arrays need not be pickled)."""
    from multiprocessing import shared_memory

    workload, ids, k = args
    model = pore_model(k)
    b = make_batch([workload_read(workload, int(i), model) for i in ids])
    parts = [
        b.events,
        np.diff(b.event_offset).astype(np.uint64),
        b.ranks,
        np.diff(b.kmer_offset).astype(np.uint64),
        b.scale,
        b.shift,
    ]
    total = sum(p.nbytes for p in parts)
    shm = shared_memory.SharedMemory(create=True, size=max(total, 1))
    meta = []
    off = 0
    for p in parts:
        dst = np.ndarray(p.shape, p.dtype, buffer=shm.buf, offset=off)
        dst[...] = p
        meta.append((p.shape, p.dtype.str, off))
        off += p.nbytes
    del dst
    name = shm.name
    # the parent unlinks the block; keep this process's resource tracker
    # from removing it when the worker exits
    from multiprocessing import resource_tracker

    resource_tracker.unregister(shm._name, "shared_memory")
    shm.close()
    return name, meta


def workload_batch_parallel(
    workload: str,
    k: Optional[int] = None,
    read_ids: Optional[Sequence[int]] = None,
    workers: Optional[int] = None,
    chunk: int = 100,
) -> Batch:
    """workload_batch over a process pool (same bytes: every read has its own
    random stream); for the large workloads.  The pore model is the seeded
    one of k (``pore_model(k)``)."""
    import multiprocessing as mp
    import os
    from multiprocessing import shared_memory

    cfg = WORKLOADS[workload]
    k = cfg["k"] if k is None else k
    ids = list(range(cfg["n_reads"]) if read_ids is None else read_ids)
    workers = workers or min(16, os.cpu_count() or 1)
    jobs = [(workload, ids[j : j + chunk], k) for j in range(0, len(ids), chunk)]
    with mp.get_context("fork").Pool(max(1, workers)) as pool:
        results = pool.map(_workload_chunk, jobs, chunksize=1)
    blocks = []
    try:
        views = []
        for name, meta in results:
            shm = shared_memory.SharedMemory(name=name)
            blocks.append(shm)
            views.append([np.ndarray(s, np.dtype(d), buffer=shm.buf, offset=o) for s, d, o in meta])
        n = len(ids)
        ne = np.concatenate([v[1] for v in views]) if views else np.zeros(0, np.uint64)
        nk = np.concatenate([v[3] for v in views]) if views else np.zeros(0, np.uint64)
        eo = np.zeros(n + 1, np.uint64)
        ko = np.zeros(n + 1, np.uint64)
        np.cumsum(ne, out=eo[1:])
        np.cumsum(nk, out=ko[1:])
        ev = np.empty((int(eo[-1]), 3), np.float32)
        rk = np.empty(int(ko[-1]), np.uint32)
        e0 = k0 = 0
        for v in views:
            ev[e0 : e0 + v[0].shape[0]] = v[0]
            rk[k0 : k0 + v[2].shape[0]] = v[2]
            e0 += v[0].shape[0]
            k0 += v[2].shape[0]
        sc = np.concatenate([v[4] for v in views]) if views else np.zeros(0, np.float32)
        sh = np.concatenate([v[5] for v in views]) if views else np.zeros(0, np.float32)
        del views, v
    finally:
        for shm in blocks:
            shm.close()
            shm.unlink()
    return Batch(ev, eo, rk, ko, sc, sh)


def read_is_methylated(workload: str, read_id: int, model: PoreModel) -> bool:
    """Whether read ``read_id`` of a methylation workload was drawn
    methylated (replays its stream up to that draw)."""
    rng = read_rng(workload, read_id)
    L = draw_length(rng, WORKLOADS[workload]["lengths"])
    rng.integers(0, 4, L)
    n_k = max(L - model.k + 1, 0)
    rng.uniform(0.9, 1.1)
    rng.uniform(-5.0, 5.0)
    rng.random(n_k)
    rng.geometric(1.0 / EVENTS_PER_KMER_MEAN, n_k)
    return bool(rng.random() < 0.5)


def workload_lengths(workload: str, read_ids: Sequence[int]) -> np.ndarray:
    """Reference lengths only (cheap: draws the first number of each stream)."""
    kind = WORKLOADS[workload]["lengths"]
    return np.array([draw_length(read_rng(workload, int(i)), kind) for i in read_ids], np.int64)


def noiseless_batch(n_reads: int, L: int, model: PoreModel, seed: int = 7) -> Batch:
    return make_batch(
        [gen_read(np.random.default_rng([seed, i]), L, model, noiseless=True) for i in range(n_reads)]
    )


def serving_arrivals(
    n_channels: int = 512,
    bases_per_s: float = 400.0,
    duration_s: float = 10.0,
    mean_len: Optional[float] = None,
    seed: int = WORKLOAD_SEED_BASE + WORKLOADS["serving-lognormal8kb"]["seed_index"],
) -> np.ndarray:
    """Arrival times (s) of reads from ``n_channels`` independent Poisson
    channels, each delivering ``bases_per_s`` on average (a simulated
    sequencer).  The expected read length of the serving workload
    (log-normal, median 8 kb, sigma 1, clipped) sets the per-channel rate."""
    if mean_len is None:
        mean_len = 8000.0 * math.exp(0.5)
    rate = bases_per_s / mean_len
    rng = np.random.default_rng(seed)
    times = []
    for _ in range(n_channels):
        t = rng.exponential(1.0 / rate)
        while t < duration_s:
            times.append(t)
            t += rng.exponential(1.0 / rate)
    return np.sort(np.array(times, np.float64))
