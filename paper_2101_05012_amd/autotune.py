"""Launch-form autotuner and batch runner for the persistent alignment kernel.

A *job* is a set of reads already in device memory.  It is split into ``nb``
length-interleaved batches, each captured once as a HIP graph
(``abea_graph_create``) that runs one persistent fused kernel: a pool of
wavefronts takes the batch's reads, longest first, from a device work queue
(Ch. 5 §5.4.3 fights the same length imbalance with CPU off-load; §5.4.2.2
bounds memory with pre-allocation).  Replaying the graphs is one pass over
the job.

The tuner measures whole passes and picks, by coordinate descent:
  * cells (band slots) per lane: the smallest that fits W, or twice that;
  * wavefronts (reads) per workgroup: 1, 2 or 4;
  * pool size in wavefronts per SIMD (capped by residency and by the trace
    budget, i.e. admission by traceback bytes);
  * batches per job (reads per persistent launch).
Every candidate gives the same bits; only time differs.  All compute runs in
libabea.so; this module only builds graphs and times them with HIP events.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import abea


@dataclasses.dataclass
class Launch:
    cells_per_lane: int = 0
    waves_per_group: int = 1
    waves_per_simd: int = 4
    batches: int = 1

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


def interleave_order(lengths: np.ndarray, nb: int) -> List[np.ndarray]:
    """Split read indices into nb batches with the same length mix: sort by
    length (longest first) and deal the reads round robin."""
    order = np.argsort(-np.asarray(lengths), kind="stable")
    return [np.sort(order[j::nb]) for j in range(nb)]


def slice_device_batch(db: abea.DeviceBatch, lo: int, hi: int) -> abea.DeviceBatch:
    """Reads [lo, hi) of a device batch as a batch of its own (views)."""
    e0, e1 = int(db.event_offset[lo]), int(db.event_offset[hi])
    k0, k1 = int(db.kmer_offset[lo]), int(db.kmer_offset[hi])
    return abea.DeviceBatch(
        hi - lo,
        db.events[e0:e1],
        db.ranks[k0:k1],
        db.scale[lo:hi],
        db.shift[lo:hi],
        (db.event_offset[lo : hi + 1] - np.uint64(e0)).astype(np.uint64),
        (db.kmer_offset[lo : hi + 1] - np.uint64(k0)).astype(np.uint64),
    )


class Job:
    """A device-resident job, pre-split into nb interleaved batches: the host
    batch is permuted once so that every batch is a contiguous range."""

    def __init__(self, batch, nb: int, device: int = 0):
        L = np.diff(batch.event_offset.astype(np.int64)) + np.diff(batch.kmer_offset.astype(np.int64))
        parts = interleave_order(L, nb)
        perm = np.concatenate(parts)
        self.perm = perm
        self.bounds = np.cumsum([0] + [len(p) for p in parts])
        self.host = batch.subset(perm) if nb > 1 else batch
        self.device = device
        self.db = abea.to_device(self.host, device)
        self.parts = [slice_device_batch(self.db, int(self.bounds[j]), int(self.bounds[j + 1])) for j in range(nb)]
        self.cells = None

    @property
    def n_reads(self) -> int:
        return self.db.n_reads


class GraphRun:
    """The job's batches captured as graphs with one launch form."""

    def __init__(self, aligner: abea.Aligner, job: Job):
        self.job = job
        self.results = [abea.DeviceResult.empty(p, job.device) for p in job.parts]
        self.graphs = [aligner.graph(p, r) for p, r in zip(job.parts, self.results)]
        self.info = [g.info() for g in self.graphs]

    def launch(self, stream) -> None:
        for g in self.graphs:
            g.launch(stream)

    def close(self) -> None:
        for g in self.graphs:
            g.close()
        self.graphs = []


def time_passes(fn, stream, reps: int) -> float:
    """Mean milliseconds of fn(stream) over reps passes (HIP events on the
    stream the work is launched on)."""
    import torch

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        fn(stream)
    ev1.record(stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / reps


def resident_simds(device: int = 0) -> int:
    import torch

    return 4 * torch.cuda.get_device_properties(device).multi_processor_count


def make_aligner(model, k: int, W: int, launch: Launch, device: int, arena_bytes: int) -> abea.Aligner:
    workers = max(1, launch.waves_per_simd * resident_simds(device))
    return abea.Aligner(
        model.level_mean, model.level_stdv, k, W=W, device=device, arena_bytes=arena_bytes,
        workers=workers, waves_per_group=launch.waves_per_group, cells_per_lane=launch.cells_per_lane,
    )


def measure(model, k, W, batch, launch: Launch, device=0, arena_bytes=0, reps=2, jobs: Optional[dict] = None,
            log=print) -> dict:
    """Time whole passes of the job in the given launch form."""
    import torch

    if jobs is not None and launch.batches in jobs:
        job = jobs[launch.batches]
    else:
        job = Job(batch, launch.batches, device)
        if jobs is not None:
            jobs[launch.batches] = job
    al = make_aligner(model, k, W, launch, device, arena_bytes)
    run = GraphRun(al, job)
    st = torch.cuda.Stream(device)
    time_passes(run.launch, st, 1)  # warm-up pass
    ms = time_passes(run.launch, st, reps)
    out = {
        "launch": launch.as_dict(),
        "ms": ms,
        "workers": [i["workers"] for i in run.info],
        "trace_gb": sum(i["trace_bytes"] for i in run.info) / 1e9,
        "cells_per_lane": run.info[0]["cells_per_lane"],
    }
    log(f"autotune: {out}")
    run.close()
    al.close()
    del run
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def autotune(model, k: int, W: int, batch, device: int = 0, arena_bytes: int = 0, reps: int = 2,
             log=print, batch_counts: Sequence[int] = (1, 2, 4)) -> Dict:
    """Coordinate descent over the launch form on the job itself."""
    jobs: dict = {}
    table = []
    best = Launch()

    def run(c: Launch) -> float:
        r = measure(model, k, W, batch, c, device, arena_bytes, reps, jobs, log)
        table.append(r)
        return r["ms"]

    # 1. slots per lane x reads per workgroup
    minc = abea.min_cells_per_lane(W)
    cands = [(c, wpg) for c in (minc, 2 * minc) if c <= 16 for wpg in (1, 2, 4)]
    res = {cw: run(dataclasses.replace(best, cells_per_lane=cw[0], waves_per_group=cw[1])) for cw in cands}
    cw = min(res, key=res.get)
    best = dataclasses.replace(best, cells_per_lane=cw[0], waves_per_group=cw[1])
    best_ms = res[cw]
    # 2. pool size
    for wps in (1, 2, 3, 8):
        c = dataclasses.replace(best, waves_per_simd=wps)
        ms = run(c)
        if ms < best_ms:
            best, best_ms = c, ms
    # 3. batches per job
    for nb in batch_counts:
        if nb == best.batches:
            continue
        c = dataclasses.replace(best, batches=nb)
        ms = run(c)
        if ms < best_ms:
            best, best_ms = c, ms
    for j in jobs.values():
        del j.db
    jobs.clear()
    return {"best": best, "best_ms": best_ms, "table": table}
