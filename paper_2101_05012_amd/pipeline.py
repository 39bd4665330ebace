"""Methylation calling on one GPU, the thesis's three steps of Ch. 5 §5.2.2
("Methylation calling": event detection, signal-space alignment, HMM
profiling) as library calls on one stream:

  abea_detect_events_device  raw samples -> events (and per-read event offsets)
  abea_align_batch_device    events + k-mer ranks -> alignment pairs
  abea_methylation_device    aligned events -> LLR per CpG site

The event offsets come back to the host between the first two calls (the
alignment plans its batch from host offsets).  Orchestration only: every
step runs in the HIP library.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import abea


@dataclasses.dataclass
class PipelineResult:
    event_offset: np.ndarray  # host uint64 [n+1]
    events: object  # torch float32 [cap, 3]
    dres: abea.DeviceResult
    llr: object  # torch float32 [K]
    n_ev: object  # torch int32 [K]
    ms: dict  # stage times (HIP events on the stream)


def start(al: abea.Aligner, draw: abea.DeviceRawBatch, kmer_offset: np.ndarray, bufs: dict, params=None,
          stream=None) -> None:
    """Enqueue the event detection of a raw batch on ``stream`` (output
    tensors kept in ``bufs``)."""
    import torch

    dev = draw.samples.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    n = draw.n_reads
    K = int(kmer_offset[-1])
    if bufs.get("ev") is None or bufs["ev"].shape[0] < max(draw.n_samples, 1):
        bufs["ev"] = torch.empty((max(draw.n_samples, 1), 3), dtype=torch.float32, device=dev)
        bufs["eo"] = torch.empty(n + 1, dtype=torch.int64, device=dev)
        bufs["llr"] = torch.empty(max(K, 1), dtype=torch.float32, device=dev)
        bufs["nev"] = torch.empty(max(K, 1), dtype=torch.int32, device=dev)
    al.detect_events_device(draw, bufs["ev"], bufs["eo"], params, stream=st)
    ev = bufs.get("detected")
    if ev is None:
        ev = bufs["detected"] = torch.cuda.Event()
    ev.record(st)


def ready(bufs: dict) -> bool:
    """True once the detection that ``start`` enqueued with ``bufs`` has run
    (``finish`` then waits for nothing but the offsets' copy)."""
    return bufs["detected"].query()


def run_in_flight(n_slots: int, n_batches: int, start_fn, finish_fn, slot_bufs: list, poll_s: float = 20e-6) -> list:
    """Batches 0 .. n_batches-1 over n_slots slots (a context and a stream
    each): ``start_fn(slot, b)`` enqueues batch b's detection on the slot
    (with ``start``), ``finish_fn(slot, b)`` its alignment and scoring (with
    ``finish``) and returns what is kept of it.  A batch is finished as soon
    as its detection has run, in whatever order the slots get there, and the
    slot's next batch is enqueued behind it at once: a slot whose detection
    waits behind its previous batch's longest read holds back no other slot.
    Returns finish_fn's results in batch order."""
    import time

    results = [None] * n_batches
    busy = [None] * n_slots  # the batch whose detection each slot holds
    nxt = 0
    for i in range(min(n_slots, n_batches)):
        start_fn(i, nxt)
        busy[i] = nxt
        nxt += 1
    done = 0
    while done < n_batches:
        moved = False
        for i in range(n_slots):
            b = busy[i]
            if b is None or not ready(slot_bufs[i]):
                continue
            results[b] = finish_fn(i, b)
            done += 1
            busy[i] = None
            moved = True
            if nxt < n_batches:
                start_fn(i, nxt)
                busy[i] = nxt
                nxt += 1
        if not moved:
            time.sleep(poll_s)
    return results


def finish(al: abea.Aligner, draw: abea.DeviceRawBatch, ranks, kmer_offset: np.ndarray, scale, shift, bufs: dict,
           stream=None) -> PipelineResult:
    """After ``start`` on the same stream: the event offsets to the host (a
    wait for that stream only), then the alignment and the scoring enqueued
    on the stream."""
    import torch

    dev = draw.samples.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    n = draw.n_reads
    K = int(kmer_offset[-1])
    with torch.cuda.stream(st):
        eo_h = bufs["eo"].to("cpu").numpy().view(np.uint64).copy()
    db = abea.DeviceBatch(n, bufs["ev"], ranks, scale, shift, eo_h, np.ascontiguousarray(kmer_offset, np.uint64))
    if bufs.get("dres") is None or bufs["dres"].capacity < db.capacity:
        bufs["dres"] = abea.DeviceResult.empty(db, dev.index or 0)
    d = bufs["dres"]
    dres = abea.DeviceResult(d.pairs, db.capacity, d.pair_offset, d.log_likelihood, d.status, d.cells)
    al.align_device(db, dres, stream=st)
    al.methylation_device(db, dres, bufs["llr"], bufs["nev"], stream=st)
    return PipelineResult(eo_h, bufs["ev"], dres, bufs["llr"][:K], bufs["nev"][:K], {})


def call_methylation(al: abea.Aligner, draw: abea.DeviceRawBatch, ranks, kmer_offset: np.ndarray, scale, shift,
                     params=None, stream=None, bufs: Optional[dict] = None) -> PipelineResult:
    """Raw reads on the device to per-site LLRs.  ``ranks`` (torch int32, the
    uint32 ranks), ``scale``, ``shift`` are device tensors; ``kmer_offset`` a
    host array.  ``bufs`` (optional) keeps the output tensors between calls."""
    import torch

    dev = draw.samples.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    n = draw.n_reads
    K = int(kmer_offset[-1])
    bufs = {} if bufs is None else bufs
    if bufs.get("ev") is None or bufs["ev"].shape[0] < max(draw.n_samples, 1):
        bufs["ev"] = torch.empty((max(draw.n_samples, 1), 3), dtype=torch.float32, device=dev)
        bufs["eo"] = torch.empty(n + 1, dtype=torch.int64, device=dev)
        bufs["llr"] = torch.empty(max(K, 1), dtype=torch.float32, device=dev)
        bufs["nev"] = torch.empty(max(K, 1), dtype=torch.int32, device=dev)
    ev, eo, llr, nev = bufs["ev"], bufs["eo"], bufs["llr"], bufs["nev"]
    t = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t[0].record(st)
    al.detect_events_device(draw, ev, eo, params, stream=st)
    t[1].record(st)
    eo_h = eo.to("cpu", non_blocking=False).numpy().view(np.uint64).copy()
    db = abea.DeviceBatch(n, ev, ranks, scale, shift, eo_h, np.ascontiguousarray(kmer_offset, np.uint64))
    if bufs.get("dres") is None or bufs["dres"].capacity < db.capacity:
        bufs["dres"] = abea.DeviceResult.empty(db, dev.index or 0)
    dres = bufs["dres"]
    dres = abea.DeviceResult(dres.pairs, db.capacity, dres.pair_offset, dres.log_likelihood, dres.status, dres.cells)
    t2 = torch.cuda.Event(enable_timing=True)
    t2.record(st)
    al.align_device(db, dres, stream=st)
    t[2].record(st)
    al.methylation_device(db, dres, llr, nev, stream=st)
    t[3].record(st)
    t[3].synchronize()
    ms = {"detect": t[0].elapsed_time(t[1]), "offsets_to_host": t[1].elapsed_time(t2),
          "align": t2.elapsed_time(t[2]), "methylation": t[2].elapsed_time(t[3]), "total": t[0].elapsed_time(t[3])}
    return PipelineResult(eo_h, ev, dres, llr[:K], nev[:K], ms)
