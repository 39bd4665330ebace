"""Throughput benchmark of the ABEA hot path on one MI355X.

A step is one pass of the whole path (per-read constants and batch plan,
k-parameter prep, band fill, backtrack, pair compaction) over one batch of
synthetic reads already resident in HBM.  The default workload is the
4000-read log-normal batch (median 5 kb, clipped 200 b..100 kb, W = 100,
k = 6), aligned with one launch per kernel per batch.

Prints one JSON line.  ``value`` is whole-job GCUPS (DP cells filled inside
the table per second, the same cell count as the CPU oracle's); the line also
carries reads/s, per-kernel times, the band kernel's fraction of the FP32
VALU roofline and the CPU oracle timed on the host's cores on a sample of the
same workload.
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
# 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "plain-4000-lognormal5kb": dict(config=1, W=100, k=6),
    "plain-64x1kb": dict(config=0, W=100, k=6),
}

# HBM traffic of one band-kernel launch on the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a copy-kernel
# calibration; None until measured for the current kernel.
BAND_TRAFFIC_BYTES = None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(batch, model, W, n_reads_sample):
    from oracle import oracle as O

    cores = min(16, os.cpu_count() or 1)
    sub = batch.subset(range(n_reads_sample))
    om = O.Model(model.level_mean, model.level_stdv)
    t0 = time.perf_counter()
    res = O.align_batch(sub, om, W, n_threads=cores)
    dt = time.perf_counter() - t0
    cells = int(res.cells.sum())
    return {
        "value": cells / dt / 1e9,
        "unit": "GCUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"reads 0..{n_reads_sample - 1} of the same workload, {cells / 1e9:.2f} Gcells, {dt:.2f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain-4000-lognormal5kb", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-reads", type=int, default=1000)
    ap.add_argument(
        "--inflight",
        type=int,
        default=3,
        help="batches in flight: each has its own context and stream, so one batch's longest "
        "reads overlap the next batch's work (1 = strictly one batch after the other)",
    )
    ap.add_argument(
        "--workers",
        type=int,
        default=0,
        help="launch form: -1 split band/backtrack kernels, 0 one fused wavefront per read, "
        ">0 a persistent pool of that many wavefronts with a device work queue",
    )
    ap.add_argument("--wpg", type=int, default=1, help="wavefronts (reads) per workgroup of the fused kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(
            f"bench.py runs on one GPU: the alignment of a read never spans devices and this build "
            f"measures one GPU's share (asked for --gpus {args.gpus})",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    from paper_2101_05012_amd import abea, synth

    wl = WORKLOADS[args.workload]
    W, k = wl["W"], wl["k"]
    log(f"bench: generating workload {args.workload}")
    model = synth.pore_model(k)
    batch = synth.config_batch(wl["config"], model)
    n = batch.n_reads
    dev = 0
    torch.cuda.set_device(dev)
    P = max(1, args.inflight)
    db = abea.to_device(batch, dev)  # inputs resident in HBM, shared by all slots
    slots = []
    for _ in range(P):
        al = abea.Aligner(model.level_mean, model.level_stdv, k, W=W, device=dev, timing=True,
                          workers=args.workers, waves_per_group=args.wpg)
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

    log(f"bench: warmup {args.warmup}")
    run(args.warmup)
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
    for al, _, _ in slots:
        al.close()

    ms_step = dt / args.steps * 1e3
    gcups = cells_per_step * args.steps / dt / 1e9
    kms = kt / args.steps
    band_s = kms[1] / 1e3
    achieved = cells_per_step * OPS_PER_CELL / band_s / 1e12
    out = {
        "metric": METRIC,
        "value": round(gcups, 3),
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
        "config": {
            "workload": args.workload,
            "n_reads": n,
            "bandwidth": W,
            "k": k,
            "cells_per_step": cells_per_step,
            "parallelism": "one wavefront per read",
            "batches_in_flight": P,
        },
        "reads_per_s": round(n * args.steps / dt, 1),
        "kernel_gcups": round(cells_per_step / (kms.sum() / 1e3) / 1e9, 3),
        "kernel_ms": {
            "prep": round(float(kms[0]), 4),
            "band": round(float(kms[1]), 4),
            "backtrack": round(float(kms[2]), 4),
            "compact": round(float(kms[3]), 4),
        },
        "reads_ok": int((status == 0).sum()),
        "roofline": {
            "bound": "alu",
            "kernel": "k_band",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": BAND_TRAFFIC_BYTES,
        },
    }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(batch, model, W, min(args.cpu_sample_reads, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
