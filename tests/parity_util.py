"""Whole-workload parity helpers: per-read digests of a result and the
acceptance rule.

The acceptance rule for the alignment against the oracle:
  * every read has the oracle's status and in-table cell count;
  * the pairs are bit-identical on every read whose decision margins (band
    moves and path cells, the oracle's min_margin) all exceed 1e-3, and on at
    least 99.9% of all reads;
  * the path score's relative error is at most 1e-5 on every aligned read.
Both sides round every float32 operation the same way, so the expected
outcome is 100% identical reads; the rule is what is asserted, the identical
fraction is printed.
"""

from __future__ import annotations

import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.join(HERE, "golden") not in sys.path:
    sys.path.insert(0, os.path.join(HERE, "golden"))

import oracle_digests  # noqa: E402

MARGIN = 1e-3
MIN_IDENTICAL = 0.999
SCORE_REL = 1e-5


def result_digests(pairs: np.ndarray, pair_offset: np.ndarray, status, cells, log_likelihood,
                   threads: int = 16) -> dict:
    """Per-read digests of a result laid out as the library returns it
    (pairs of read r at pair_offset[r] .. pair_offset[r+1])."""
    po = np.asarray(pair_offset, np.int64)
    n = po.shape[0] - 1
    pairs = np.ascontiguousarray(pairs, dtype="<i4")

    def dig(r):
        return oracle_digests.digest_pairs(pairs[po[r]: po[r + 1]])

    with ThreadPoolExecutor(max(1, threads)) as ex:  # hashlib releases the GIL on large buffers
        d = np.fromiter(ex.map(dig, range(n), chunksize=64), np.uint64, count=n)
    return {
        "status": np.asarray(status).astype(np.int8),
        "cells": np.asarray(cells).astype(np.int64),
        "path_len": np.diff(po),
        "score_bits": np.asarray(log_likelihood, np.float32).view(np.uint32),
        "pairs_digest": d,
    }


def oracle_result_digests(ores) -> dict:
    """Digests of a live oracle batch result (oracle.BatchResult)."""
    n = ores.status.shape[0]
    return {
        "status": ores.status.astype(np.int8),
        "cells": ores.cells.astype(np.int64),
        "path_len": ores.path_len.astype(np.int64),
        "score_bits": ores.score.astype(np.float32).view(np.uint32),
        "min_margin": ores.min_margin,
        "pairs_digest": np.array([oracle_digests.digest_pairs(ores.read_pairs(t)) for t in range(n)], np.uint64),
    }


def check_acceptance(name: str, got: dict, ref: dict, say=print) -> dict:
    """Assert the acceptance rule for `got` against the oracle's `ref`
    (digests of the same reads in the same order) and report it."""
    n = ref["status"].shape[0]
    assert got["status"].shape[0] == n, (name, got["status"].shape, n)
    bad_status = np.nonzero(got["status"] != ref["status"])[0]
    assert bad_status.size == 0, (name, "status differs", bad_status[:10])
    ok = ref["status"] == 0
    bad_cells = np.nonzero(ok & (got["cells"] != ref["cells"]))[0]
    assert bad_cells.size == 0, (name, "cells differ", bad_cells[:10])
    ident = ok & (got["path_len"] == ref["path_len"]) & (got["pairs_digest"] == ref["pairs_digest"]) & (
        got["score_bits"] == ref["score_bits"])
    ident |= ~ok
    gs = got["score_bits"].view(np.float32).astype(np.float64)
    rs = ref["score_bits"].view(np.float32).astype(np.float64)
    rel = np.zeros(n)
    rel[ok] = np.abs(gs[ok] - rs[ok]) / np.maximum(np.abs(rs[ok]), 1e-30)
    margin = ref["min_margin"]
    wide = ok & (margin > MARGIN)
    frac = float(ident.mean()) if n else 1.0
    stats = {
        "reads": int(n),
        "aligned": int(ok.sum()),
        "identical": int(ident.sum()),
        "identical_frac": frac,
        "reads_margin_above_1e-3": int(wide.sum()),
        "min_margin": float(margin[ok].min()) if ok.any() else float("inf"),
        "max_score_rel_err": float(rel.max()) if n else 0.0,
    }
    say(f"parity {name}: {stats}")
    not_ident_wide = np.nonzero(wide & ~ident)[0]
    assert not_ident_wide.size == 0, (name, "pairs differ on reads with margins above 1e-3", not_ident_wide[:10])
    assert frac >= MIN_IDENTICAL, (name, "identical fraction", frac, np.nonzero(~ident)[0][:10])
    assert stats["max_score_rel_err"] <= SCORE_REL, (name, "score relative error", stats["max_score_rel_err"])
    return stats
