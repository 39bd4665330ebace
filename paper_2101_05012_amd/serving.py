"""Simulated sequencer driving the library's serving loop.

Reads of a host batch arrive at given times (seconds from the start, sorted,
read i at arrivals[i]), replayed ``compression`` times faster than real time.
A submitter thread hands every read to the server at its arrival instant,
stamped with that instant (so queueing in Python counts as latency).  The
calling thread collects the results.  Latency = result in host memory -
arrival.  All alignment runs in libabea.so; this module only paces
submissions and does the book-keeping.
"""

from __future__ import annotations

import threading
import time
from typing import Dict, Optional

import numpy as np

from . import abea


def run(server: abea.Server, batch, arrivals_s: np.ndarray, compression: float = 1.0,
        keep_pairs: bool = False, tick_s: float = 0.0005, timeout_s: float = 600.0,
        submitters: int = 4) -> Dict:
    n = batch.n_reads
    arrivals_s = np.asarray(arrivals_s, np.float64)
    assert arrivals_s.shape[0] == n and np.all(np.diff(arrivals_s) >= 0)
    t0 = abea.now_ns() + 2_000_000  # start 2 ms from now
    target = t0 + (arrivals_s / compression * 1e9).astype(np.int64)
    submitted = np.zeros(n, np.int64)  # when each read's submit call returned
    call_ns = []  # per submitter: time spent inside submit calls
    err = []

    def submitter(mine: np.ndarray):
        """Hand reads `mine` (sorted) to the server at their arrival times;
        several submitters share the copying of arriving reads."""
        spent = 0
        try:
            i = 0
            m = mine.shape[0]
            tm = target[mine]
            while i < m:
                now = abea.now_ns()
                r = int(mine[i])
                if target[r] > now:
                    wait = (target[r] - now) / 1e9
                    time.sleep(min(wait, tick_s) if wait > tick_s else max(wait, 0.0))
                    continue
                j = int(np.searchsorted(tm, now, side="right"))
                j = max(j, i + 1)
                # runs of consecutive read indices go in one call
                while i < j:
                    a = int(mine[i])
                    b = i + 1
                    while b < j and int(mine[b]) == int(mine[b - 1]) + 1:
                        b += 1
                    last = int(mine[b - 1])
                    c0 = abea.now_ns()
                    server.submit(batch, a, last + 1, np.arange(a, last + 1, dtype=np.uint64), target[a:last + 1])
                    c1 = abea.now_ns()
                    spent += c1 - c0
                    submitted[a : last + 1] = c1
                    i = b
        except Exception as e:  # surfaced by the collector
            err.append(e)
        call_ns.append(spent)

    T = max(1, min(int(submitters), n))
    if T == 1:
        parts = [np.arange(n)]
    else:
        # contiguous blocks of 64 reads dealt round robin: a submitter that
        # is behind hands a whole run of due reads over in one call
        blk = np.arange(n) // 64
        parts = [np.nonzero(blk % T == t)[0] for t in range(T)]
    threads = [threading.Thread(target=submitter, args=(p,), daemon=True) for p in parts]
    for th in threads:
        th.start()
    comps = []
    pairs: Optional[dict] = {} if keep_pairs else None
    got = 0
    deadline = time.monotonic() + timeout_s
    while got < n:
        if err:
            raise err[0]
        if time.monotonic() > deadline:
            raise TimeoutError(f"serving: {got} of {n} reads finished")
        c, p = server.poll(max_out=4096, timeout_us=2000, want_pairs=keep_pairs)
        if c.shape[0] == 0:
            continue
        comps.append(c)
        got += c.shape[0]
        if keep_pairs:
            for rec in c:
                o = int(rec["pair_offset"])
                pairs[int(rec["tag"])] = p[o : o + int(rec["n_pairs"])]
    for th in threads:
        th.join()
    if err:
        raise err[0]
    comp = np.concatenate(comps)
    comp = comp[np.argsort(comp["tag"])]
    return {"completions": comp, "pairs": pairs, "t0": t0, "stats": server.stats(),
            "submit_lag_ns": submitted - target, "submit_call_ns": call_ns}


def summarize(res: Dict, batch, compression: float, arrivals_s: np.ndarray) -> Dict:
    c = res["completions"]
    n = c.shape[0]
    lat_ms = (c["t_done_ns"] - c["t_arrival_ns"]) / 1e6
    wait_ms = (c["t_admit_ns"] - c["t_arrival_ns"]) / 1e6
    span_s = (c["t_done_ns"].max() - c["t_arrival_ns"].min()) / 1e9
    cells = int(c["cells"].sum())
    L = np.diff(batch.kmer_offset.astype(np.int64))
    long = L > np.median(L)
    # completions are sorted by tag = read index, so L lines up with them
    Lr = L[c["tag"].astype(np.int64)]
    dec = np.minimum(9, (np.argsort(np.argsort(Lr, kind="stable"), kind="stable") * 10) // max(1, n))
    bases = int(L.sum())
    offered = n / (arrivals_s[-1] / compression) if arrivals_s[-1] > 0 else float("inf")
    pct = lambda a, q: round(float(np.percentile(a, q)), 3) if a.size else None  # noqa: E731
    st = res["stats"]
    return {
        "compression": compression,
        "reads": n,
        "offered_reads_per_s": round(offered, 1),
        "offered_kbases_per_s": round(offered * bases / n / 1e3, 1),
        "reads_per_s": round(n / span_s, 1),
        "gcups": round(cells / span_s / 1e9, 3),
        "latency_ms": {"p50": pct(lat_ms, 50), "p99": pct(lat_ms, 99), "max": round(float(lat_ms.max()), 3)},
        "latency_ms_reads_below_median_length": {"p50": pct(lat_ms[~long], 50), "p99": pct(lat_ms[~long], 99)},
        "latency_ms_reads_above_median_length": {"p50": pct(lat_ms[long], 50), "p99": pct(lat_ms[long], 99)},
        # by decile of read length (shortest tenth first)
        "latency_ms_by_length_decile": [
            {"p50": pct(lat_ms[m], 50), "p99": pct(lat_ms[m], 99),
             "kb": [round(float(Lr[m].min()) / 1e3, 1), round(float(Lr[m].max()) / 1e3, 1)]}
            for m in (dec == q for q in range(10)) if m.any()
        ],
        "admission_wait_ms": {"p50": pct(wait_ms, 50), "p99": pct(wait_ms, 99)},
        # arrival -> the submit call returned (the simulated sequencer's own lag)
        "submit_lag_ms": {"p50": pct(res["submit_lag_ns"] / 1e6, 50), "p99": pct(res["submit_lag_ns"] / 1e6, 99)},
        "submit_calls_s": round(sum(res["submit_call_ns"]) / 1e9, 3),
        "submit_in_library_s": round(st["submit_ns"] / 1e9, 3),
        "submit_copy_s": round(st["submit_copy_ns"] / 1e9, 3),
        "pageable_reads": st["pageable_reads"],
        "micro_batches": st["micro_batches"],
        "max_inflight_reads": st["max_inflight_reads"],
        "max_inflight_trace_mb": round(st["max_inflight_trace_bytes"] / 1e6, 1),
        "server_thread_s": {"enqueue": round(st["enqueue_ns"] / 1e9, 3), "device": round(st["device_ns"] / 1e9, 3),
                            "harvest": round(st["harvest_ns"] / 1e9, 3)},
        "span_s": round(span_s, 3),
        "reads_ok": int((c["status"] == 0).sum()),
    }
