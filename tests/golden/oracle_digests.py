"""Per-read oracle results of whole workloads, stored as digests.

The CPU oracle (``oracle/``) is run over every read of a workload and, per
read, the following is kept:
  * status;
  * in-table cell count;
  * path length;
  * float32 log-likelihood (its bits);
  * smallest decision margin (band moves and path cells; oracle_stats_t);
  * an 8-byte BLAKE2b digest of the read's (event, k-mer) pairs as
    little-endian int32.
The GPU parity tests compare every read of the same workload, aligned by the
HIP library in the launch form the benchmark times, against these digests.
The workloads are too large for the oracle to run inside a GPU test (about
770 G cells in all).

Only this script writes the files, and it calls nothing but the oracle and
the seeded input generator: no expected value comes from the HIP path.

    python tests/golden/oracle_digests.py [--threads N] [case ...]
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# name -> (synthetic workload, band width W, k-mer length k)
CASES = {
    "uneven-20000_w100_k6": ("uneven-20000", 100, 6),
    "uneven-20000_w200_k6": ("uneven-20000", 200, 6),
    "ultralong-200_w100_k6": ("ultralong-200", 100, 6),
    "ultralong-200_w250_k6": ("ultralong-200", 250, 6),
    "ultralong-200_w250_k9": ("ultralong-200", 250, 9),
}

FIELDS = ("status", "cells", "path_len", "score_bits", "min_margin", "pairs_digest", "n_events", "n_kmers")


def digest_pairs(pairs: np.ndarray) -> int:
    """8-byte BLAKE2b of an [n, 2] pair array as little-endian int32."""
    a = np.ascontiguousarray(pairs, dtype="<i4")
    return int.from_bytes(hashlib.blake2b(a.tobytes(), digest_size=8).digest(), "little")


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def load(name: str) -> dict:
    with np.load(path(name), allow_pickle=False) as z:
        return {f: z[f] for f in FIELDS}


def batch_for(name: str):
    from paper_2101_05012_amd import synth

    workload, W, k = CASES[name]
    return synth.workload_batch_parallel(workload, k=k), W, k


def compute(name: str, threads: int, batch=None, log=print) -> dict:
    from oracle import oracle as O
    from paper_2101_05012_amd import synth

    workload, W, k = CASES[name]
    if batch is None:
        batch, _, _ = batch_for(name)
    m = synth.pore_model(k)
    om = O.Model(m.level_mean, m.level_stdv)
    n = batch.n_reads
    t0 = time.perf_counter()
    # reads in chunks of 1000, which bounds the pair buffer of one oracle call
    out = {f: np.zeros(n, dt) for f, dt in zip(FIELDS, (np.int8, np.int64, np.int64, np.uint32, np.float64,
                                                       np.uint64, np.int64, np.int64))}
    step = 1000
    for lo in range(0, n, step):
        idx = list(range(lo, min(n, lo + step)))
        sub = batch.subset(idx)
        r = O.align_batch(sub, om, W, n_threads=threads)
        for t, i in enumerate(idx):
            out["status"][i] = r.status[t]
            out["cells"][i] = r.cells[t]
            out["path_len"][i] = r.path_len[t]
            out["score_bits"][i] = np.float32(r.score[t]).view(np.uint32)
            out["min_margin"][i] = r.min_margin[t]
            out["pairs_digest"][i] = digest_pairs(r.read_pairs(t))
            out["n_events"][i] = batch.n_events(i)
            out["n_kmers"][i] = batch.n_kmers(i)
        log(f"{name}: {idx[-1] + 1}/{n} reads, {time.perf_counter() - t0:.0f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for name in args.cases:
        t0 = time.perf_counter()
        d = compute(name, args.threads)
        np.savez_compressed(path(name), **d)
        print(f"{name}: wrote {path(name)} in {time.perf_counter() - t0:.0f} s; "
              f"{int(d['cells'].sum()) / 1e9:.1f} G cells", flush=True)


if __name__ == "__main__":
    main()
