"""Throughput benchmark of the ABEA hot path on one MI355X.

A step is one pass of the whole path over one batch (job) of synthetic reads
already resident in HBM:
  * per-read constants and batch plan;
  * k-parameter prep;
  * band fill;
  * backtrack;
  * pair compaction.

The default workload is the largest single-GPU job, uneven-20000-w100:
20000 reads, 70% 500 b..5 kb and 30% 20..200 kb (W = 100, k = 6), run as a
captured graph of the persistent kernel (device work queue, admission by
traceback bytes) in the launch form the autotuner chose for it.  Beside it,
in the same line:
  * the plain per-batch kernel on the same reads (5 batches of 4000, one
    launch each, one wavefront per read);
  * a short serving level (reads of the 512-channel sequencer replayed 1000x
    faster than real time) with p50/p99 latency;
  * abea_align_batch on host buffers (the first 4000 reads of the job);
  * the oracle on the host's cores.

Other workloads (``--workload``):
  uneven-20000-w200: the same reads at W = 200 (``--tune`` autotunes the
      launch form of either width).
  plain-4000-lognormal5kb: 4000 log-normal reads (median 5 kb, clipped
      200 b..100 kb, W = 100), one kernel launch per batch.  `--inflight P`
      keeps P batches in flight on P streams (default 16, on 16 hardware
      queues): a batch lasts as long as its longest read, and the batches in
      flight overlap those tails.  Each launch runs a pool of 320 fused
      wavefronts that take the batch's reads from a device work queue; the
      16 pools together ask for the chip's 5120 resident wave slots.
  ultralong-200-*: 200 reads of 200 kb..1 Mb (W = 100 or 250, k = 6 or 9).
      The persistent kernel under a trace budget, and the backtrack's
      throughput.
  raw-4000-lognormal5kb: event detection (the step before the alignment)
      on the raw signal of 4000 log-normal reads, 4 kHz samples at 450
      bases/s (293 M int16 samples); value in G samples/s, roofline on HBM.
  meth-4000-lognormal5kb: methylation scoring (the step after the
      alignment) of the CpG sites of 4000 aligned reads, half of them
      methylated; value in M sites/s, roofline on the FP32 issue ceiling.
  pipeline-4000-lognormal5kb: the whole methylation call on one GPU, raw
      signal of 4000 reads (half methylated) to events, alignment and per-site
      LLRs; value in G samples/s, with each stage's time.
  serving-512ch: reads arrive from 512 simulated channels (Poisson, 400
      bases/s each, log-normal lengths with median 8 kb) into the library's
      continuous-batching server.  The replay is sped up 1x..10000x; each
      level reports p50/p99 per-read latency, reads/s and GCUPS.  The plain
      batched kernel runs beside it on the same reads.

Prints one JSON line.  ``value`` is whole-job GCUPS (DP cells filled inside
the table per second, the same cell count as the CPU oracle's).  The line
also carries:
  * reads/s;
  * per-kernel times;
  * the fused or band kernel's fraction of the FP32 VALU roofline;
  * the CPU oracle timed on the host's cores on a sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ABEA GCUPS + reads/s on 1 MI355X; p50/p99 per-read latency in serving mode"

# Algorithmic FP32 work of one DP cell (Alg. 5.2 + 5.3): emission 4 (sub,
# mul, mul, sub), three moves 5 adds, arg-max 2 compare/selects.
OPS_PER_CELL = 11
# Plain (non-packed, non-fused) FP32 VALU peak of MI355X: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz.  The cell's arithmetic cannot use FMA (its rounding
# order is fixed) nor packed FP32, so this is its issue ceiling.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# MI355X's published FP32 vector peak (counts an FMA as two flops and packed
# FP32 as two lanes).
FP32_VECTOR_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "plain-4000-lognormal5kb": dict(kind="plain", source="plain-4000-lognormal5kb", W=100, k=6),
    "plain-64x1kb": dict(kind="plain", source="plain-64x1kb", W=100, k=6),
    # the same 4000 reads with the events scaled to the model instead
    "plain-4000-lognormal5kb-scale-events": dict(kind="plain", source="plain-4000-lognormal5kb", W=100, k=6, scale_events=True),
    # reads with open-pore and adaptor events at both ends, aligned with trim states
    "plain-4000-lognormal5kb-ends-trim": dict(kind="plain", source="plain-4000-lognormal5kb-ends", W=100, k=6,
                                              trim=True),
    # launch: the autotuner's choice (cells per lane, reads per workgroup,
    # pool wavefronts per SIMD, batches per job)
    "uneven-20000-w100": dict(kind="persistent", source="uneven-20000", W=100, k=6, plain_batches=5,
                              launch=(2, 4, 4, 1), extras=True),
    "uneven-20000-w200": dict(kind="persistent", source="uneven-20000", W=200, k=6, plain_batches=5,
                              launch=(4, 4, 3, 1)),
    "ultralong-200-w100": dict(kind="persistent", source="ultralong-200", W=100, k=6, plain_batches=1,
                               launch=(2, 1, 4, 1)),
    "ultralong-200-w250": dict(kind="persistent", source="ultralong-200", W=250, k=6, plain_batches=1,
                               launch=(4, 1, 4, 1)),
    "ultralong-200-w250-k9": dict(kind="persistent", source="ultralong-200", W=250, k=9, plain_batches=1,
                                  launch=(4, 1, 4, 1)),
    "serving-512ch": dict(kind="serving", source="serving-lognormal8kb", W=100, k=6),
    # event detection: the raw signal of 4000 log-normal reads (4 kHz samples,
    # 450 bases/s) cut into events on the GPU
    "raw-4000-lognormal5kb": dict(kind="detect", source="raw-4000-lognormal5kb", W=100, k=6),
    # methylation scoring: the CpG sites of 4000 aligned reads, half of them
    # methylated, under a methylated and an unmethylated model
    "meth-4000-lognormal5kb": dict(kind="meth", source="meth-4000-lognormal5kb", W=100, k=6),
    # the three steps of methylation calling on one GPU: raw signal of 4000
    # reads (half methylated) to events, alignment and per-site LLRs
    "pipeline-4000-lognormal5kb": dict(kind="pipeline", source="pipeline-4000-lognormal5kb", W=100, k=6),
}

HBM_PEAK_GBS = 8000.0
# HBM bytes of one k_ed_events launch (the slower detection kernel), from
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE with the same calibration factors
# as ALIGN_TRAFFIC_BYTES; null for a workload without a measurement of the
# current kernels.
DETECT_TRAFFIC_BYTES = {"raw-4000-lognormal5kb": 1.5632e9}

# serving: (time compression, reads) per load level; x1 is real time for 512
# channels at 400 bases/s each
SERVING_LEVELS = [(1, 300), (10, 1000), (100, 4000), (1000, 20000), (3000, 30000), (10000, 30000)]

# HBM bytes of one fused-kernel launch (k_align), from two rocprofv3 --pmc
# runs (FETCH_SIZE x 1.99989, WRITE_SIZE x 1.0: the factors a 1 GiB device
# copy needs to read its known size), by workload; a workload without a
# measurement of the current kernel reports null.
ALIGN_TRAFFIC_BYTES = {"uneven-20000-w100": 150.22e9, "plain-4000-lognormal5kb": 6.806e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(batch, model, W, idx, what, scale_events=False, trim=False):
    """The oracle on the host's cores (up to 16 threads) over reads idx."""
    from oracle import oracle as O

    flags = (O.SCALE_EVENTS if scale_events else 0) | (O.TRIM if trim else 0)
    cores = min(16, os.cpu_count() or 1)
    sub = batch.subset(idx)
    om = O.Model(model.level_mean, model.level_stdv)
    t0 = time.perf_counter()
    res = O.align_batch(sub, om, W, n_threads=cores, flags=flags)
    dt = time.perf_counter() - t0
    cells = int(res.cells.sum())
    # one thread on the first reads of the same sample (about 0.25 G cells)
    per = np.cumsum(res.cells.astype(np.int64))
    n1 = max(1, int(np.searchsorted(per, min(250_000_000, int(per[-1]) if per.size else 0)) + 1))
    n1 = min(n1, len(idx))
    sub1 = batch.subset(list(idx)[:n1])
    t1 = time.perf_counter()
    r1 = O.align_batch(sub1, om, W, n_threads=1, flags=flags)
    dt1 = time.perf_counter() - t1
    c1 = int(r1.cells.sum())
    return {
        "value": round(cells / dt / 1e9, 4),
        "unit": "GCUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{what}: {len(idx)} reads, {cells / 1e9:.2f} Gcells, {dt:.2f} s",
        "one_thread": {"value": round(c1 / dt1 / 1e9, 4), "unit": "GCUPS",
                       "sample": f"the first {n1} reads of that sample, {c1 / 1e9:.2f} Gcells, {dt1:.2f} s"},
        "host_cpu": host_cpu(),
    }


def host_cpu() -> str:
    """Model name of the host CPU and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return f"{model}, {n} logical CPUs available"


def band_slots(batch, W) -> int:
    """W x computed bands (2 .. n_e + n_k) over the batch: the band-slot count
    (cells of every band whether inside the table or not)."""
    ne = np.diff(batch.event_offset.astype(np.int64))
    nk = np.diff(batch.kmer_offset.astype(np.int64))
    ok = (ne > 0) & (nk > 0)
    return int(W * (ne[ok] + nk[ok] - 1).sum())


def host_api_rate(al, batch, cells, reps=3):
    """abea_align_batch with inputs and outputs in host memory (copies over
    PCIe both ways inside the call), result buffers allocated once."""
    import ctypes

    from paper_2101_05012_amd import abea

    n = batch.n_reads
    ev = np.ascontiguousarray(batch.events, np.float32)
    eo = np.ascontiguousarray(batch.event_offset, np.uint64)
    ko = np.ascontiguousarray(batch.kmer_offset, np.uint64)
    rk = np.ascontiguousarray(batch.ranks, np.uint32)
    sc = np.ascontiguousarray(batch.scale, np.float32)
    sh = np.ascontiguousarray(batch.shift, np.float32)
    cap = abea.pair_capacity(eo, ko)
    pairs = np.ones((max(cap, 1), 2), np.int32)  # touched: no page faults inside the timed calls
    po = np.zeros(n + 1, np.uint64)
    ll = np.zeros(n, np.float32)
    st = np.zeros(n, np.int32)
    ce = np.zeros(n, np.uint64)
    b = abea.abea_batch_t(n, ev.ctypes.data, eo.ctypes.data, rk.ctypes.data, ko.ctypes.data, sc.ctypes.data,
                          sh.ctypes.data)
    r = abea.abea_result_t(pairs.ctypes.data, cap, po.ctypes.data, ll.ctypes.data, st.ctypes.data, ce.ctypes.data)
    call = lambda: al._check(abea.lib().abea_align_batch(al.handle, ctypes.byref(b), ctypes.byref(r)),  # noqa: E731
                             "abea_align_batch")
    call()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    dt = (time.perf_counter() - t0) / reps
    return {"gcups": round(cells / dt / 1e9, 3), "ms_per_batch": round(dt * 1e3, 3),
            "reads_per_s": round(n / dt, 1), "calls": reps,
            "what": "abea_align_batch, host buffers, PCIe both ways, one batch at a time"}


def sample_reads(batch, W, target_cells: float):
    """Every s-th read, s chosen so that the sample has about target_cells."""
    n = batch.n_reads
    per = (np.diff(batch.event_offset.astype(np.float64)) + np.diff(batch.kmer_offset.astype(np.float64))) * W
    stride = max(1, int(np.ceil(per.sum() / target_cells)))
    return list(range(0, n, stride))


def roofline(cells, kernel_ms, kernel_name, workload=None, job_gcups=None):
    """The kernel's algorithmic FP32 work (11 ops per cell) over its average
    launch duration, against the FP32 issue ceiling of non-fused, non-packed
    lane operations (``peak``) and against the published FP32 vector peak;
    with ``job_gcups``, the same over the whole job's wall time."""
    achieved = cells * OPS_PER_CELL / (kernel_ms / 1e3) / 1e12
    out = {
        "bound": "alu",
        "kernel": kernel_name,
        "achieved": round(achieved, 3),
        "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "TFLOP/s",
        "frac": round(achieved / VALU_PEAK_TOPS, 4),
        "traffic": ALIGN_TRAFFIC_BYTES.get(workload) if kernel_name == "k_align" else None,
        "fp32_vector_peak": FP32_VECTOR_PEAK_TFLOPS,
        "frac_of_fp32_vector_peak": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
    }
    if job_gcups is not None:
        job = job_gcups * OPS_PER_CELL / 1e3
        out.update({"achieved_job": round(job, 3), "frac_job": round(job / VALU_PEAK_TOPS, 4),
                    "frac_job_of_fp32_vector_peak": round(job / FP32_VECTOR_PEAK_TFLOPS, 4)})
    return out


def base_line(args, value, ms_step, workload, cfg_extra):
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, **cfg_extra},
    }


# --------------------------------------------------------------- plain form


def bench_plain(args, wl):
    import torch

    from paper_2101_05012_amd import abea, synth

    W, k = wl["W"], wl["k"]
    log(f"bench: generating workload {args.workload}")
    model = synth.pore_model(k)
    batch = synth.workload_batch(wl["source"], model)
    n = batch.n_reads
    dev = 0
    torch.cuda.set_device(dev)
    P = max(1, args.inflight)
    # edge clearing exists at 2 and 4 slots per lane; other widths take the automatic choice
    # slot clearing: by default edges when the batches in flight together hold
    # at least two wavefronts per SIMD (the library sees one launch at a time),
    # else the library's own choice; edges exist at 2 and 4 slots per lane
    band_clear = args.band_clear
    if band_clear < 0:
        simds = 4 * torch.cuda.get_device_properties(dev).multi_processor_count
        per_launch = n if args.workers <= 0 else min(n, args.workers)
        band_clear = abea.ABEA_CLEAR_EDGES if P * per_launch >= 2 * simds else abea.ABEA_CLEAR_AUTO
    if band_clear == abea.ABEA_CLEAR_EDGES and abea.min_cells_per_lane(W) not in (2, 4):
        band_clear = abea.ABEA_CLEAR_AUTO
    db = abea.to_device(batch, dev)  # inputs resident in HBM, shared by all slots
    slots = []
    for _ in range(P):
        al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev, timing=True,
                          workers=args.workers, waves_per_group=args.wpg, band_clear=band_clear,
                          scale_events=wl.get("scale_events", False), trim=wl.get("trim", False))
        slots.append((al, abea.DeviceResult.empty(db, dev), torch.cuda.Stream(dev)))
    torch.cuda.synchronize()

    def run(steps, kt=None):
        """Issue `steps` batches round-robin over the slots; before a slot is
        reused its previous batch must be finished (its kernel times are read
        then), so at most P batches are in flight."""
        pending = [False] * P
        for t in range(steps):
            si = t % P
            al, dr, st = slots[si]
            if pending[si]:
                ms = al.timings()  # waits for this slot's previous batch
                if kt is not None:
                    kt += ms
            al.align_device(db, dr, st)
            pending[si] = True
        for si in range(P):
            if pending[si]:
                ms = slots[si][0].timings()
                if kt is not None:
                    kt += ms

    # every context makes its first call (buffer allocation, staging) before
    # the timed region, whatever --warmup says
    warm = max(args.warmup, P)
    log(f"bench: warmup {warm} batches ({P} contexts)")
    run(warm)
    torch.cuda.synchronize()
    dr0 = slots[0][1]
    cells_per_step = int(dr0.cells[:n].sum().item())
    status = dr0.status[:n].cpu().numpy()

    log(f"bench: timing {args.steps} steps, {P} in flight")
    kt = np.zeros(4, np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps, kt)  # per-kernel HIP-event times on each launch stream
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("bench: timed region done")
    plan = slots[0][0].plan_info()
    host = host_api_rate(slots[0][0], batch, cells_per_step) if args.host_api else None
    for al, _, _ in slots:
        al.close()

    ms_step = dt / args.steps * 1e3
    gcups = cells_per_step * args.steps / dt / 1e9
    kms = kt / args.steps
    fused = plan["workers"] > 0
    kname = "k_align" if fused else "k_band"
    out = base_line(args, gcups, ms_step, args.workload, {
        "n_reads": n,
        "bandwidth": W,
        "k": k,
        "cells_per_step": cells_per_step,
        "parallelism": "one wavefront per read",
        "launch": "fused band+backtrack, one launch per batch" if fused else "band and backtrack kernels",
        "batches_in_flight": P,
        "alignment_launch": {"workers": args.workers} if args.workers > 0 else "one wavefront per read",
        "warmup_batches": warm,
        "band_clear": {1: "window", 2: "edges"}.get(plan.get("band_clear"), "?"),
        "per_read_scaling": "events to the model" if wl.get("scale_events") else "model to the events",
        "trim_states": bool(wl.get("trim", False)),
    })
    out.update({
        "reads_per_s": round(n * args.steps / dt, 1),
        "band_slot_gcups": round(band_slots(batch, W) * args.steps / dt / 1e9, 3),
        "kernel_gcups": round(cells_per_step / (kms.sum() / 1e3) / 1e9, 3),
        "kernel_ms": {
            "prep": round(float(kms[0]), 4),
            "align" if fused else "band": round(float(kms[1]), 4),
            "backtrack": round(float(kms[2]), 4),
            "compact": round(float(kms[3]), 4),
        },
        "reads_ok": int((status == 0).sum()),
        **({"host_api": host} if host else {}),
        # per launch (launches overlap), and over the whole job's time
        "roofline": roofline(cells_per_step, float(kms[1]), kname, args.workload, job_gcups=gcups),
    })
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        idx = list(range(min(args.cpu_sample_reads, n)))
        out["cpu_baseline"] = cpu_baseline(batch, model, W, idx, f"reads 0..{len(idx) - 1} of the same workload",
                                           scale_events=wl.get("scale_events", False), trim=wl.get("trim", False))
    return out


# ---------------------------------------------------------- persistent form


def bench_persistent(args, wl):
    import torch

    from paper_2101_05012_amd import abea, autotune, synth

    W, k = wl["W"], wl["k"]
    dev = 0
    torch.cuda.set_device(dev)
    log(f"bench: generating workload {args.workload}")
    t0 = time.perf_counter()
    model = synth.pore_model(k)
    ids = None
    if args.max_reads > 0:
        ids = range(min(args.max_reads, synth.WORKLOADS[wl["source"]]["n_reads"]))
    batch = synth.workload_batch_parallel(wl["source"], k=k, read_ids=ids)
    n = batch.n_reads
    log(f"bench: generated {n} reads, {int(batch.kmer_offset[-1]) / 1e6:.1f} M k-mers in "
        f"{time.perf_counter() - t0:.1f} s")
    arena = int(args.trace_budget_gb * 1e9) if args.trace_budget_gb > 0 else 0

    if args.tune:
        log("bench: autotuning the launch form")
        tuned = autotune.autotune(model, k, W, batch, dev, arena_bytes=arena, reps=1, log=log)
        launch = tuned["best"]
        tune_report = {"best": launch.as_dict(), "candidates": [
            {**r["launch"], "ms": round(r["ms"], 2), "workers": r["workers"]} for r in tuned["table"]]}
    else:
        dc, dw, dp, db_ = wl["launch"]
        launch = autotune.Launch(cells_per_lane=args.cpl if args.cpl >= 0 else dc,
                                 waves_per_group=args.wpg if args.wpg > 0 else dw,
                                 waves_per_simd=args.wps if args.wps > 0 else dp,
                                 batches=args.nb if args.nb > 0 else db_)
        tune_report = None

    # persistent form: the job as nb captured graphs
    job = autotune.Job(batch, launch.batches, dev)
    al = autotune.make_aligner(model, k, W, launch, dev, arena)
    run = autotune.GraphRun(al, job)
    st = torch.cuda.Stream(dev)
    log(f"bench: persistent {launch.as_dict()} workers {[i['workers'] for i in run.info]}")
    autotune.time_passes(run.launch, st, max(1, args.warmup))
    cells = int(sum(int(r.cells[: p.n_reads].sum().item()) for r, p in zip(run.results, job.parts)))
    status = np.concatenate([r.status[: p.n_reads].cpu().numpy() for r, p in zip(run.results, job.parts)])
    log(f"bench: timing {args.steps} passes")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run.launch(st)
    st.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = run.info
    run.close()
    al.close()
    del run
    torch.cuda.empty_cache()

    # kernel times of the first batch in the same form, eager, HIP events on
    # the launch stream
    log("bench: kernel times")
    al_t = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev, timing=True,
                        arena_bytes=arena,
                        workers=max(1, launch.waves_per_simd * autotune.resident_simds(dev)),
                        waves_per_group=launch.waves_per_group, cells_per_lane=launch.cells_per_lane)
    p0 = job.parts[0]
    r0 = abea.DeviceResult.empty(p0, dev)
    al_t.align_device(p0, r0, st)
    kms0 = [float(x) for x in al_t.timings()]
    cells0 = int(r0.cells[: p0.n_reads].sum().item())
    al_t.close()
    del r0
    torch.cuda.empty_cache()

    # plain per-batch form on the same reads: fused kernel, one wavefront per
    # read, one launch per batch, batches one after the other
    log("bench: plain per-batch form")
    nbp = wl["plain_batches"]
    jobp = autotune.Job(batch, nbp, dev) if nbp != launch.batches else job
    alp = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
    resp = [abea.DeviceResult.empty(p, dev) for p in jobp.parts]

    def plain_pass(stream):
        for p, r in zip(jobp.parts, resp):
            alp.align_device(p, r, stream)

    autotune.time_passes(plain_pass, st, 1)
    plain_ms = autotune.time_passes(plain_pass, st, max(1, min(args.steps, 3)))
    alp.close()
    del resp
    torch.cuda.empty_cache()

    ms_step = dt / args.steps * 1e3
    gcups = cells * args.steps / dt / 1e9
    out = base_line(args, gcups, ms_step, args.workload, {
        "n_reads": n,
        "bandwidth": W,
        "k": k,
        "cells_per_step": cells,
        "parallelism": "persistent pool of wavefronts, device work queue, HIP graphs",
        "launch": launch.as_dict(),
        "workers": [i["workers"] for i in info],
        "trace_gb": round(sum(i["trace_bytes"] for i in info) / 1e9, 3),
        "trace_budget_gb": args.trace_budget_gb,
        "reads_used": "all" if args.max_reads <= 0 else f"first {n}",
    })
    out.update({
        "reads_per_s": round(n * args.steps / dt, 1),
        "band_slot_gcups": round(band_slots(batch, W) * args.steps / dt / 1e9, 3),
        "reads_ok": int((status == 0).sum()),
        "plain_per_batch": {
            "batches": nbp,
            "ms_per_step": round(plain_ms, 3),
            "gcups": round(cells / (plain_ms / 1e3) / 1e9, 3),
        },
        "kernel_ms_batch0": {"prep": round(float(kms0[0]), 4), "align": round(float(kms0[1]), 4),
                             "compact": round(float(kms0[3]), 4)},
        # per launch: batch 0 run eagerly in the same form; job: the timed passes
        "roofline": roofline(cells0, float(kms0[1]), "k_align", args.workload,
                             job_gcups=gcups if launch.batches == 1 else None),
    })
    if wl.get("extras") and not args.no_extras:
        log("bench: event detection (raw-4000-lognormal5kb)")
        out["event_detection"] = detect_summary(detect_run(args, WORKLOADS["raw-4000-lognormal5kb"], dev,
                                                           steps=10, warmup=2))
        log("bench: methylation scoring (meth-4000-lognormal5kb)")
        ma = argparse.Namespace(steps=10, warmup=2, no_cpu_baseline=True, workload="meth-4000-lognormal5kb")
        mo = bench_meth(ma, WORKLOADS["meth-4000-lognormal5kb"])
        out["methylation"] = {"workload": "meth-4000-lognormal5kb", "sites": mo["config"]["sites_per_step"],
                              "ms_per_call": mo["ms_per_step"], "m_sites_per_s": mo["value"],
                              "kernel_ms": mo["kernel_ms"], "alignment_ms": mo["alignment_ms"],
                              "sites_right_sign": mo["sites_right_sign"], "roofline": mo["roofline"]}
        log("bench: host-buffer API on the first 4000 reads")
        sub = batch.subset(range(min(4000, n)))
        alh = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
        sub_cells = int(alh.align(sub).cells.sum())
        out["host_api"] = {**host_api_rate(alh, sub, sub_cells),
                           "reads": sub.n_reads, "what": "abea_align_batch on the first 4000 reads of the job: "
                           "host buffers through the pinned staging ring, PCIe both ways, one batch at a time"}
        alh.close()
        del sub
        out["serving"] = serving_level(args, dev)
        # ultra-long reads: the longest reads' serial chains set the pass
        log("bench: ultra-long reads (ultralong-200-w100)")
        ua = argparse.Namespace(**vars(args))
        ua.workload, ua.steps, ua.warmup = "ultralong-200-w100", 2, 1
        ua.no_extras, ua.no_cpu_baseline, ua.tune, ua.backtrack_probe = True, True, False, False
        ua.cpl, ua.wpg, ua.wps, ua.nb, ua.max_reads, ua.trace_budget_gb = -1, 0, 0, 0, 0, 0.0
        uo = bench_persistent(ua, WORKLOADS["ultralong-200-w100"])
        # the same job at W = 200 in its tuned form
        log("bench: uneven-20000-w200")
        wa = argparse.Namespace(**vars(ua))
        wa.workload = "uneven-20000-w200"
        wo = bench_persistent(wa, WORKLOADS["uneven-20000-w200"])
        out["uneven_w200"] = {"workload": "uneven-20000-w200", "gcups": wo["value"], "ms_per_pass": wo["ms_per_step"],
                              "reads_per_s": wo.get("reads_per_s"), "reads_ok": wo.get("reads_ok"),
                              "launch": wo["config"]["launch"], "steps": wa.steps, "roofline": wo["roofline"]}
        # the raw-signal pipeline: detection, alignment and scoring in flight
        log("bench: raw-signal pipeline (pipeline-4000-lognormal5kb)")
        pa = argparse.Namespace(workload="pipeline-4000-lognormal5kb", steps=64, warmup=2, inflight=16,
                                workers=320, no_cpu_baseline=True)
        po_ = bench_pipeline(pa, WORKLOADS["pipeline-4000-lognormal5kb"])
        out["pipeline"] = {"workload": "pipeline-4000-lognormal5kb", "g_samples_per_s": po_["value"],
                           "ms_per_batch": po_["ms_per_step"], "batches": po_["steps"],
                           "batches_in_flight": po_["batches_in_flight"], "reads_per_s": po_["reads_per_s"],
                           "one_batch_alone_ms": po_["one_batch_alone"]["ms"],
                           "sites_right_sign": po_["sites_right_sign"]}
        out["ultralong"] = {"workload": "ultralong-200-w100", "gcups": uo["value"], "ms_per_pass": uo["ms_per_step"],
                            "reads_per_s": uo.get("reads_per_s"), "reads_ok": uo.get("reads_ok"),
                            "steps": ua.steps, "roofline": uo["roofline"]}
    if tune_report:
        out["autotune"] = tune_report
    if args.backtrack_probe:
        log("bench: backtrack probe")
        out["backtrack"] = backtrack_probe(model, k, W, job, dev, st)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        idx = sample_reads(batch, W, args.cpu_sample_gcells * 1e9)
        stride = idx[1] - idx[0] if len(idx) > 1 else 1
        out["cpu_baseline"] = cpu_baseline(batch, model, W, idx, f"every {stride}-th read of the same workload")
    return out


# ------------------------------------------------------------ event detection


def detect_run(args, wl, dev, steps, warmup):
    """Event detection of a whole raw workload resident in HBM: ``warmup``
    untimed passes, then ``steps`` timed passes (HIP events on the launch
    stream around them), and one timed pass's kernel times from the
    library's own dispatch events."""
    import torch

    from paper_2101_05012_amd import abea, synth

    model = synth.pore_model(wl["k"])
    t0 = time.perf_counter()
    rb = synth.workload_raw_batch(wl["source"], model)
    S = int(rb.sample_offset[-1])
    log(f"bench: {rb.n_reads} raw reads, {S} samples, generated in {time.perf_counter() - t0:.1f} s")
    al = abea.Aligner(model.level_mean, model.level_stdv, wl["k"], W=wl["W"], device=dev, timing=True)
    d = abea.raw_to_device(rb, dev)
    ev = torch.empty((max(S, 1), 3), dtype=torch.float32, device=f"cuda:{dev}")
    eo = torch.empty(rb.n_reads + 1, dtype=torch.int64, device=f"cuda:{dev}")
    st = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        al.detect_events_device(d, ev, eo, stream=st)
    torch.cuda.synchronize()
    kms = al.detect_timings()  # the last warmup pass, alone on the stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        al.detect_events_device(d, ev, eo, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    n_ev = int(eo[-1].item())
    al.close()
    return {"rb": rb, "S": S, "n_events": n_ev, "ms": ms, "kernel_ms": [float(x) for x in kms],
            "steps": steps, "warmup": warmup}


def detect_roofline(r, workload):
    """HBM roofline of the slower of the two streaming kernels, on their
    algorithmic bytes: k_ed_detect reads 2 B per sample; k_ed_events reads
    2 B per sample and writes one 12-byte event record per event."""
    S, E = r["S"], r["n_events"]
    det_ms, ev_ms = r["kernel_ms"][0], r["kernel_ms"][1]
    by = {"k_ed_detect": (2.0 * S, det_ms), "k_ed_events": (2.0 * S + 12.0 * E, ev_ms)}
    name = max(by, key=lambda k: by[k][1])
    nbytes, kms = by[name]
    gbs = nbytes / (kms / 1e3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": DETECT_TRAFFIC_BYTES.get(workload),
            "algorithmic_bytes": nbytes,
            "achieved_job": round((2.0 * S + 12.0 * E) / (r["ms"] / 1e3) / 1e9, 1)}


def detect_summary(r):
    return {"workload": "raw-4000-lognormal5kb", "samples": r["S"], "events": r["n_events"],
            "ms_per_pass": round(r["ms"], 4), "gsamples_per_s": round(r["S"] / r["ms"] / 1e6, 2),
            "events_per_kmer": round(r["n_events"] / float(r["rb"].kmer_offset[-1]), 3),
            "kernel_ms": {"k_ed_detect": round(r["kernel_ms"][0], 4), "k_ed_events": round(r["kernel_ms"][1], 4),
                          "pass": round(r["kernel_ms"][2], 4)},
            "roofline": detect_roofline(r, "raw-4000-lognormal5kb")}


def bench_detect(args, wl):
    dev = 0
    r = detect_run(args, wl, dev, args.steps, args.warmup)
    S, ms = r["S"], r["ms"]
    out = {
        "metric": "event detection throughput (raw samples cut into events per second) on 1 MI355X",
        "value": round(S / ms / 1e6, 3),
        "unit": "G samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_reads": r["rb"].n_reads, "samples_per_step": S,
                   "detector": "windows 3 and 8 samples, t thresholds 1.5 and 5.0"},
        "events_per_step": r["n_events"],
        "events_per_kmer": round(r["n_events"] / float(r["rb"].kmer_offset[-1]), 3),
        "kernel_ms": {"k_ed_detect": round(r["kernel_ms"][0], 4), "k_ed_events": round(r["kernel_ms"][1], 4),
                      "pass": round(r["kernel_ms"][2], 4)},
        "roofline": detect_roofline(r, args.workload),
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        cores = min(16, os.cpu_count() or 1)
        log("bench: cpu baseline (oracle)")
        t0 = time.perf_counter()
        O.ed_batch(r["rb"], n_threads=cores)
        dt = time.perf_counter() - t0
        sub = r["rb"]
        n1 = 200
        from paper_2101_05012_amd import synth

        one = synth.make_raw_batch([synth.RawRead(sub.read_raw(i), sub.read_ranks(i), sub.offset[i],
                                                  sub.pa_scale[i], sub.scale[i], sub.shift[i],
                                                  np.zeros(0, np.int64)) for i in range(n1)])
        t1 = time.perf_counter()
        O.ed_batch(one, n_threads=1)
        dt1 = time.perf_counter() - t1
        s1 = int(one.sample_offset[-1])
        out["cpu_baseline"] = {
            "value": round(S / dt / 1e9, 4), "unit": "G samples/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole workload: {S} samples, {dt:.2f} s",
            "one_thread": {"value": round(s1 / dt1 / 1e9, 4), "unit": "G samples/s",
                           "sample": f"the first {n1} reads, {s1} samples, {dt1:.2f} s"},
            "host_cpu": host_cpu(),
        }
    return out


# ------------------------------------------------------ methylation scoring


def bench_meth(args, wl):
    """Methylation scores of a whole aligned batch resident in HBM: the
    batch is aligned once (not timed), then ``steps`` timed calls of
    abea_methylation_device (HIP events on the launch stream) and one call's
    kernel times from the library's dispatch events."""
    import torch

    from paper_2101_05012_amd import abea, synth

    dev = 0
    k, W = wl["k"], wl["W"]
    model = synth.pore_model(k)
    mm = synth.methylated_model(model)
    t0 = time.perf_counter()
    batch = synth.workload_batch_parallel(wl["source"], k)
    log(f"bench: {batch.n_reads} reads generated in {time.perf_counter() - t0:.1f} s")
    al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev, timing=True)
    al.set_methylated_model(mm.level_mean, mm.level_stdv)
    db = abea.to_device(batch, dev)
    dr = abea.DeviceResult.empty(db, dev)
    st = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    al.align_device(db, dr, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    align_ms = e0.elapsed_time(e1)
    K = int(batch.kmer_offset[-1])
    llr = torch.empty(K, dtype=torch.float32, device=f"cuda:{dev}")
    nev = torch.empty(K, dtype=torch.int32, device=f"cuda:{dev}")
    for _ in range(args.warmup):
        al.methylation_device(db, dr, llr, nev, stream=st)
    torch.cuda.synchronize()
    kms = al.meth_timings()
    e0.record(st)
    for _ in range(args.steps):
        al.methylation_device(db, dr, llr, nev, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nv = nev.cpu().numpy()
    lv = llr.cpu().numpy()
    sites = nv > 0
    n_sites = int(sites.sum())
    # window cells: events x k-mers of each site's window (the k-mers holding its C)
    ko = batch.kmer_offset.astype(np.int64)
    local = np.arange(K, dtype=np.int64) - np.repeat(ko[:-1], np.diff(ko))
    nk = np.minimum(local, k - 1) + 1
    cells = int((nv[sites].astype(np.int64) * nk[sites]).sum())
    ops = cells * 2 * OPS_PER_CELL  # two models, the alignment's 11 FP32 ops per cell
    llr_ms = float(kms[1])
    achieved = ops / (llr_ms / 1e3) / 1e12
    meth = np.array([synth.read_is_methylated(wl["source"], r, model) for r in range(batch.n_reads)])
    read_of = np.repeat(np.arange(batch.n_reads), np.diff(ko))
    right = np.where(meth[read_of[sites]], lv[sites] > 0, lv[sites] < 0)
    out = {
        "metric": "methylation scoring throughput (CpG sites of aligned reads scored per second) on 1 MI355X",
        "value": round(n_sites / ms / 1e3, 3),
        "unit": "M sites/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_reads": batch.n_reads, "k": k, "sites_per_step": n_sites,
                   "window_cells_per_step": cells},
        "kernel_ms": {"k_meth_bounds+sites": round(float(kms[0]), 4), "k_meth_llr": round(llr_ms, 4)},
        "alignment_ms": round(align_ms, 3),
        "sites_right_sign": round(float(right.mean()), 4),
        "roofline": {"bound": "alu", "kernel": "k_meth_llr", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": None, "ops_per_window_cell": 2 * OPS_PER_CELL},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        cores = min(16, os.cpu_count() or 1)
        log("bench: cpu baseline (oracle alignment, then the timed oracle scoring)")
        Mu = O.Model(model.level_mean, model.level_stdv)
        Mm = O.Model(mm.level_mean, mm.level_stdv)
        res = O.align_batch(batch, Mu, W, n_threads=cores)
        po = np.zeros(batch.n_reads + 1, np.uint64)
        po[1:] = np.cumsum(np.where(res.status == 0, res.path_len, 0))
        pairs = np.concatenate([res.read_pairs(r) for r in range(batch.n_reads) if res.status[r] == 0])
        t1 = time.perf_counter()
        O.meth_batch(batch, k, Mu, Mm, pairs, po, res.status, n_threads=cores)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(n_sites / dt / 1e6, 3), "unit": "M sites/s", "cores": cores,
                               "kind": "oracle", "sample": f"the whole workload's {n_sites} sites, {dt:.2f} s",
                               "host_cpu": host_cpu()}
    al.close()
    return out


# ------------------------------------------------ the whole methylation call


def bench_pipeline(args, wl):
    """Raw signal resident in HBM to per-site LLRs (event detection,
    alignment, methylation scoring on one stream; the event offsets go to
    the host between the first two, as the alignment plans from host
    offsets).  ``steps`` timed calls after ``warmup`` untimed ones."""
    import torch

    from paper_2101_05012_amd import abea, pipeline, synth

    dev = 0
    k, W = wl["k"], wl["W"]
    model = synth.pore_model(k)
    mm = synth.methylated_model(model)
    t0 = time.perf_counter()
    rb = synth.workload_raw_batch(wl["source"], model)
    log(f"bench: {rb.n_reads} raw reads generated in {time.perf_counter() - t0:.1f} s")
    al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
    al.set_methylated_model(mm.level_mean, mm.level_stdv)
    draw = abea.raw_to_device(rb, dev)
    ranks = torch.from_numpy(rb.ranks.view(np.int32)).to(f"cuda:{dev}")
    scale = torch.from_numpy(rb.scale).to(f"cuda:{dev}")
    shift = torch.from_numpy(rb.shift).to(f"cuda:{dev}")
    st = torch.cuda.current_stream(dev)
    bufs = {}
    for _ in range(args.warmup):
        pipeline.call_methylation(al, draw, ranks, rb.kmer_offset, scale, shift, stream=st, bufs=bufs)
    t1 = time.perf_counter()
    stages = []
    alone_steps = min(args.steps, 10)
    for _ in range(alone_steps):
        res = pipeline.call_methylation(al, draw, ranks, rb.kmer_offset, scale, shift, stream=st, bufs=bufs)
        stages.append(res.ms)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t1) / alone_steps * 1e3
    S = int(rb.sample_offset[-1])
    nev = res.n_ev.cpu().numpy()
    llr = res.llr.cpu().numpy()
    sites = nev > 0
    ko = rb.kmer_offset.astype(np.int64)
    read_of = np.repeat(np.arange(rb.n_reads), np.diff(ko))
    right = np.where(rb.methylated[read_of[sites]], llr[sites] > 0, llr[sites] < 0)
    cells = int(res.dres.cells[: rb.n_reads].sum().item())
    med = {key: round(float(np.median([s_[key] for s_ in stages])), 4) for key in stages[0]}
    # throughput: P batches in flight, each on its own context and stream
    # (the same reads; inputs shared read-only), so that one batch's longest
    # reads overlap the others' work
    P = max(1, args.inflight)
    als = [al]
    for _ in range(P - 1):
        a2 = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
        a2.set_methylated_model(mm.level_mean, mm.level_stdv)
        als.append(a2)
    # in flight, each alignment launch as a pool of --workers wavefronts (the
    # plain workload's form: 16 pools of 320 fill the chip's resident slots)
    if args.workers > 0:
        clear = abea.ABEA_CLEAR_EDGES if abea.min_cells_per_lane(W) in (2, 4) else abea.ABEA_CLEAR_AUTO
        for a2 in als:
            a2.set_launch(workers=args.workers, waves_per_group=1, band_clear=clear)
    streams = [torch.cuda.Stream(dev) for _ in range(P)]
    pbufs = [{} for _ in range(P)]

    def start_fn(i, b):
        pipeline.start(als[i], draw, rb.kmer_offset, pbufs[i], stream=streams[i])

    def finish_fn(i, b):
        pipeline.finish(als[i], draw, ranks, rb.kmer_offset, scale, shift, pbufs[i], stream=streams[i])

    # every slot warmed (its buffers sized, its first plans made)
    pipeline.run_in_flight(P, P, start_fn, finish_fn, pbufs)
    torch.cuda.synchronize()
    # steps batches (at least one per slot) through the slots, each finished
    # as soon as its detection has run and the slot refilled at once
    n_batches = max(P, args.steps)
    t3 = time.perf_counter()
    pipeline.run_in_flight(P, n_batches, start_fn, finish_fn, pbufs)
    torch.cuda.synchronize()
    flight_ms = (time.perf_counter() - t3) / n_batches * 1e3
    for a2 in als[1:]:
        a2.close()
    out = {
        "metric": "methylation calling from raw signal (event detection + alignment + site scoring) on 1 MI355X",
        "value": round(S / flight_ms / 1e6, 3),
        "unit": "G samples/s",
        "n_gpus": 1,
        "steps": n_batches,
        "warmup": args.warmup,
        "ms_per_step": round(flight_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_reads": rb.n_reads, "samples_per_step": S,
                   "events_per_step": int(res.event_offset[-1]), "sites_per_step": int(sites.sum()),
                   "alignment_cells_per_step": cells, "W": W, "k": k},
        "reads_per_s": round(rb.n_reads / flight_ms * 1e3, 1),
        "batches_in_flight": P,
        "alignment_launch": {"workers": args.workers} if args.workers > 0 else "one wavefront per read",
        "one_batch_alone": {"ms": round(wall_ms, 3), "g_samples_per_s": round(S / wall_ms / 1e6, 3),
                            "stage_ms_median": med},
        "alignment_gcups_alone": round(cells / (med["align"] / 1e3) / 1e9, 1),
        "sites_right_sign": round(float(right.mean()), 4),
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        cores = min(16, os.cpu_count() or 1)
        log("bench: cpu baseline (the three oracles chained)")
        Mu = O.Model(model.level_mean, model.level_stdv)
        Mm = O.Model(mm.level_mean, mm.level_stdv)
        t2 = time.perf_counter()
        ev, eo = O.ed_batch(rb, n_threads=cores)
        b = synth.Batch(ev, eo, rb.ranks, rb.kmer_offset, rb.scale, rb.shift)
        ores = O.align_batch(b, Mu, W, n_threads=cores)
        po = np.zeros(b.n_reads + 1, np.uint64)
        po[1:] = np.cumsum(np.where(ores.status == 0, ores.path_len, 0))
        pairs = np.concatenate([ores.read_pairs(r) for r in range(b.n_reads) if ores.status[r] == 0])
        O.meth_batch(b, k, Mu, Mm, pairs, po, ores.status, n_threads=cores)
        dt = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": round(S / dt / 1e9, 4), "unit": "G samples/s", "cores": cores,
                               "kind": "oracle", "sample": f"the whole workload: {S} samples, {dt:.2f} s",
                               "host_cpu": host_cpu()}
    al.close()
    return out


def backtrack_probe(model, k, W, job, dev, st):
    """The backtrack alone (split kernels, first batch): path steps per second
    and trace bytes walked per second."""
    from paper_2101_05012_amd import abea

    al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev, timing=True,
                      workers=abea.ABEA_WORKERS_SPLIT)
    p0 = job.parts[0]
    r0 = abea.DeviceResult.empty(p0, dev)
    al.align_device(p0, r0, st)
    ms = [float(x) for x in al.timings()]
    info = al.plan_info()
    steps = int(r0.pair_offset[-1].item())
    al.close()
    return {
        "band_ms": round(float(ms[1]), 3),
        "backtrack_ms": round(float(ms[2]), 3),
        "path_steps": steps,
        "msteps_per_s": round(steps / (ms[2] / 1e3) / 1e6, 2),
        "trace_gb": round(info["trace_bytes"] / 1e9, 3),
        "trace_gb_per_s": round(info["trace_bytes"] / (ms[2] / 1e3) / 1e9, 2),
    }


# ------------------------------------------------------------------ serving


def serving_level(args, dev):
    """One load level of the serving loop (reads of the 512-channel
    sequencer, replayed `compression` times faster than real time), beside
    the plain batched kernel on the same reads."""
    import torch

    from paper_2101_05012_amd import abea, serving, synth

    comp, n = (int(x) for x in args.serving_level.split(":"))
    W, k = 100, 6
    model = synth.pore_model(k)
    batch = synth.workload_batch_parallel("serving-lognormal8kb", k=k, read_ids=range(n))
    arr = synth.serving_arrivals(duration_s=60.0)
    while arr.shape[0] < n:
        arr = synth.serving_arrivals(duration_s=2 * arr[-1])
    arr = arr[:n]
    al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
    srv = abea.Server(al, slots=args.slots, max_batch_reads=args.batch_reads, trace_budget_bytes=32_000_000_000,
                      host_staging_bytes=int(args.host_staging_gb * (1 << 30)))
    log(f"bench: serving x{comp} {n} reads")
    res = serving.run(srv, batch, arr, compression=float(comp), submitters=args.submitters)
    srv.close()
    s = serving.summarize(res, batch, float(comp), arr)
    db = abea.to_device(batch, dev)
    dr = abea.DeviceResult.empty(db, dev)
    st = torch.cuda.Stream(dev)
    al.align_device(db, dr, st)
    st.synchronize()
    cells = int(dr.cells[:n].sum().item())
    t0 = time.perf_counter()
    for _ in range(3):
        al.align_device(db, dr, st)
    st.synchronize()
    plain_s = (time.perf_counter() - t0) / 3
    al.close()
    keep = ("compression", "reads", "offered_reads_per_s", "reads_per_s", "gcups", "latency_ms",
            "admission_wait_ms", "micro_batches", "span_s", "reads_ok")
    return {"workload": "serving-512ch", "slots": args.slots, "max_batch_reads": args.batch_reads,
            **{key: s[key] for key in keep},
            "plain_batched_same_reads": {"s": round(plain_s, 4), "gcups": round(cells / plain_s / 1e9, 3),
                                         "reads_per_s": round(n / plain_s, 1)}}


def bench_serving(args, wl):
    import torch

    from paper_2101_05012_amd import abea, serving, synth

    W, k = wl["W"], wl["k"]
    dev = 0
    torch.cuda.set_device(dev)
    levels = SERVING_LEVELS if not args.levels else [tuple(int(x) for x in s.split(":")) for s in args.levels.split(",")]
    n_max = max(n for _, n in levels)
    log(f"bench: generating {n_max} serving reads")
    t0 = time.perf_counter()
    model = synth.pore_model(k)
    batch = synth.workload_batch_parallel(wl["source"], k=k, read_ids=range(n_max))
    # arrival times of the simulated sequencer (first n_max reads)
    dur = 60.0
    arr = synth.serving_arrivals(duration_s=dur)
    while arr.shape[0] < n_max:
        dur *= 2
        arr = synth.serving_arrivals(duration_s=dur)
    arr = arr[:n_max]
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s; real-time rate {n_max / arr[-1]:.1f} reads/s")
    al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev)
    budget = int(args.trace_budget_gb * 1e9) if args.trace_budget_gb > 0 else 32_000_000_000
    out_levels = []
    for comp, n in levels:
        sub = batch.subset(range(n)) if n < batch.n_reads else batch
        srv = abea.Server(al, slots=args.slots, max_batch_reads=args.batch_reads, trace_budget_bytes=budget,
                          host_staging_bytes=int(args.host_staging_gb * (1 << 30)))
        log(f"bench: serving x{comp} {n} reads")
        res = serving.run(srv, sub, arr[:n], compression=float(comp), submitters=args.submitters)
        srv.close()
        s = serving.summarize(res, sub, float(comp), arr[:n])
        log(f"bench: {s}")
        out_levels.append(s)
    # the plain batched kernel on the same reads (largest level, inputs in HBM)
    n = levels[-1][1]
    sub = batch.subset(range(n)) if n < batch.n_reads else batch
    db = abea.to_device(sub, dev)
    dr = abea.DeviceResult.empty(db, dev)
    st = torch.cuda.Stream(dev)
    al.align_device(db, dr, st)
    st.synchronize()
    cells = int(dr.cells[:n].sum().item())
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        al.align_device(db, dr, st)
    st.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    al.close()
    best = max(out_levels, key=lambda s: s["gcups"])
    out = base_line(args, best["gcups"], 1e3 * best["reads"] / best["reads_per_s"], args.workload, {
        "reads_max": n_max,
        "bandwidth": W,
        "k": k,
        "parallelism": "continuous batching: micro-batches on several streams, one wavefront per read",
        "slots": args.slots,
        "max_batch_reads": args.batch_reads,
        "submitters": args.submitters,
        "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
        "host_staging_gb": args.host_staging_gb,
        "trace_budget_gb": budget / 1e9,
        "value_is": "GCUPS of the load level with the highest throughput",
    })
    out.update({
        "reads_per_s": best["reads_per_s"],
        "latency_ms": best["latency_ms"],
        "levels": out_levels,
        "plain_batched": {"reads": n, "s": round(plain_s, 4), "gcups": round(cells / plain_s / 1e9, 3),
                          "reads_per_s": round(n / plain_s, 1)},
    })
    return out


def copy_calibration(mb: int) -> None:
    """One plain device-to-device copy of `mb` MiB (a torch copy kernel), so
    that a counter run of this program also measures what FETCH_SIZE and
    WRITE_SIZE report for a known number of bytes."""
    import torch

    n = mb * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"bench: copy calibration {mb} MiB read + {mb} MiB written")
    del src, dst
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 batches for the plain workloads, 10 passes for the persistent ones)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 16 batches for the plain workloads, 1 pass for the persistent ones)")
    ap.add_argument("--workload", default="uneven-20000-w100", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-reads", type=int, default=1000)
    ap.add_argument("--cpu-sample-gcells", type=float, default=20.0,
                    help="persistent workloads: oracle sample size in Gcells")
    ap.add_argument(
        "--inflight",
        type=int,
        default=16,
        help="plain workloads: batches in flight, each with its own context and stream, so one "
        "batch's longest reads overlap the next batch's work (1 = one batch after the other)",
    )
    ap.add_argument(
        "--workers",
        type=int,
        default=320,
        help="plain workloads: wavefronts of each batch's launch: -1 split band/backtrack kernels, 0 one "
        "fused wavefront per read, >0 a pool of that many fused wavefronts taking the batch's reads from "
        "a device work queue (still one launch per batch); the default 320 x 16 batches in flight fills "
        "the 5120 resident wave slots",
    )
    ap.add_argument("--wpg", type=int, default=0,
                    help="wavefronts (reads) per workgroup of the fused kernel (default: 1 for the plain "
                         "workloads, the tuned form for the persistent ones)")
    ap.add_argument("--band-clear", type=int, default=-1, choices=(-1, 0, 1, 2),
                    help="plain workloads: slot clearing of interior bands, 0 the library's choice, 1 window, "
                         "2 edges; -1 (default) edges when the batches in flight hold two wavefronts per SIMD, "
                         "else the library's choice")
    ap.add_argument("--tune", action="store_true", help="persistent workloads: autotune the launch form")
    ap.add_argument("--cpl", type=int, default=-1,
                    help="persistent: cells per lane (0 = smallest; default: the workload's tuned form)")
    ap.add_argument("--wps", type=int, default=0, help="persistent: pool wavefronts per SIMD (default: tuned)")
    ap.add_argument("--nb", type=int, default=0, help="persistent: batches (graphs) per job (default: tuned)")
    ap.add_argument("--trace-budget-gb", type=float, default=0.0,
                    help="persistent: traceback memory budget per batch (0 = the library's default, 0.9 of "
                         "the device memory free when the context is created)")
    ap.add_argument("--serving-level", default="1000:5000",
                    help="default workload: the serving load level in the line, compression:reads")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: leave out the serving level and the host-buffer rate")
    ap.add_argument("--max-reads", type=int, default=0,
                    help="persistent: only the first N reads of the workload (quick runs; 0 = all)")
    ap.add_argument("--slots", type=int, default=16, help="serving: micro-batches on the device at once")
    ap.add_argument("--batch-reads", type=int, default=256, help="serving: reads per micro-batch")
    ap.add_argument("--submitters", type=int, default=8, help="serving: sequencer threads handing reads to the server")
    ap.add_argument("--host-staging-gb", type=float, default=6.0,
                    help="serving: pinned host arena for queued reads (GiB)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32), so that batches or "
                    "serving micro-batches on different streams run side by side")
    ap.add_argument("--levels", default="", help="serving: compression:reads,... (default: the full sweep)")
    ap.add_argument("--host-api", action="store_true",
                    help="plain: also time abea_align_batch on host buffers (PCIe both ways), after the timed region")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--backtrack-probe", action="store_true", help="persistent: time the backtrack alone")
    args = ap.parse_args()
    if args.gpus != 1:
        print(
            f"bench.py runs on one GPU: the alignment of a read never spans devices, so the benchmark "
            f"measures one GPU's share (asked for --gpus {args.gpus})",
            file=sys.stderr,
        )
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    # plain: enough batches that the drain of the last ones in flight is a
    # small part of the timed region; persistent: whole passes of the job
    if args.steps is None:
        args.steps = {"plain": 200, "detect": 20, "meth": 20, "pipeline": 64}.get(wl["kind"], 10)
    if args.warmup is None:
        args.warmup = {"plain": 16, "detect": 3, "meth": 3, "pipeline": 2}.get(wl["kind"], 1)
    if args.wpg <= 0 and wl["kind"] != "persistent":
        args.wpg = 1
    if 0 < args.hw_queues <= 32:
        # read by the HIP runtime when it starts, i.e. before torch touches the GPU
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.copy_calibration_mb > 0:
        copy_calibration(args.copy_calibration_mb)
    if wl["kind"] == "plain":
        out = bench_plain(args, wl)
    elif wl["kind"] == "detect":
        out = bench_detect(args, wl)
    elif wl["kind"] == "meth":
        out = bench_meth(args, wl)
    elif wl["kind"] == "pipeline":
        out = bench_pipeline(args, wl)
    elif wl["kind"] == "serving":
        out = bench_serving(args, wl)
    else:
        out = bench_persistent(args, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
