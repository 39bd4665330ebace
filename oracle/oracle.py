"""ctypes front-end of the CPU ABEA oracle -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It builds ``oracle/liboracle.so`` from
``abea_oracle.c`` with gcc when the library is missing.  Nothing here is shared
with the HIP library.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "abea_oracle.c")
SRCS = [SRC, os.path.join(HERE, "event_oracle.c"), os.path.join(HERE, "meth_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

READ_OK, READ_EMPTY, READ_BAND_LOST, READ_BAD_RANK = 0, 1, 2, 3
STATUS_NAMES = {0: "ok", 1: "empty", 2: "band_lost", 3: "bad_rank"}

FORM_LITERAL = 1
PLANT_SK_REVERSED = 2
PLANT_DROP_UP_EMISSION = 4
PLANT_EVENT_OFF_BY_ONE = 8
SCALE_EVENTS = 16  # events scaled to the model: x' = (x - shift) / scale, model levels unscaled
TRIM = 32  # trim states: leading and trailing events may be left unaligned at ln(1/100) each
PLANT_TRIM_NO_TAIL = 64
PLANT_TRIM_SKIP_IN = 128

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-pthread"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no fused multiply-add except the
    explicit fmaf of the model scaling)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in SRCS):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, *SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Stats(ctypes.Structure):
    _fields_ = [
        ("cells", ctypes.c_int64),
        ("n_bands", ctypes.c_int64),
        ("kmer_moves", ctypes.c_int64),
        ("path_len", ctypes.c_int64),
        ("min_margin", ctypes.c_double),
        ("min_move_margin", ctypes.c_double),
        ("in_table_bands", ctypes.c_int64),
        ("in_table_inf_ends", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, u32, f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_float
        L.oracle_transitions.argtypes = [i64, i64, P]
        L.oracle_transitions.restype = None
        L.oracle_model_terms.argtypes = [i64, P, P, P]
        L.oracle_model_terms.restype = None
        L.oracle_emission.argtypes = [f32, f32, f32, f32, f32, u32]
        L.oracle_emission.restype = f32
        L.oracle_band_limits.argtypes = [i64, i64, i64, i64, i32, P, P]
        L.oracle_band_limits.restype = None
        L.oracle_align.argtypes = [P, i64, i64, P, i64, P, P, P, P, i64, f32, f32, i32, u32,
                                   P, P, P, P, P]
        L.oracle_align.restype = ctypes.c_int
        L.oracle_align_batch.argtypes = [i32, P, i64, P, P, P, P, P, P, P, P, P, i64, i32, u32, i32,
                                         P, P, P, P, P, P, P]
        L.oracle_align_batch.restype = ctypes.c_int
        L.oracle_ed_stat.argtypes = [P, i64, i32, i64]
        L.oracle_ed_stat.restype = f32
        L.oracle_ed_stats.argtypes = [P, i64, f32, f32, P]
        L.oracle_ed_stats.restype = None
        L.oracle_ed_change_points.argtypes = [P, i64, P, P]
        L.oracle_ed_change_points.restype = i64
        L.oracle_ed_read.argtypes = [P, i64, f32, f32, P, P]
        L.oracle_ed_read.restype = i64
        L.oracle_ed_batch.argtypes = [i32, P, P, P, P, P, i32, P, P]
        L.oracle_ed_batch.restype = ctypes.c_int
        L.oracle_meth_is_site.argtypes = [u32, i32]
        L.oracle_meth_is_site.restype = ctypes.c_int
        L.oracle_meth_profile.argtypes = [P, i64, P, P, P, P, i64, P, u32]
        L.oracle_meth_profile.restype = f32
        L.oracle_meth_read.argtypes = [P, i64, i64, P, i64, i32, P, P, f32, f32, u32, P, i64, P, P]
        L.oracle_meth_read.restype = ctypes.c_int
        L.oracle_meth_batch.argtypes = [i32, P, i64, P, P, P, i32, P, P, P, P, u32, P, P, P, i32, P, P]
        L.oracle_meth_batch.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def transitions(n_events: int, n_kmers: int) -> np.ndarray:
    out = np.zeros(3, np.float32)
    lib().oracle_transitions(n_events, n_kmers, _p(out))
    return out


def model_terms(level_stdv: np.ndarray):
    s = np.ascontiguousarray(level_stdv, np.float32)
    c = np.zeros_like(s)
    h = np.zeros_like(s)
    lib().oracle_model_terms(s.shape[0], _p(s), _p(c), _p(h))
    return c, h


def emission(x, mu, sigma, c, h, flags: int = 0) -> np.float32:
    return np.float32(lib().oracle_emission(float(x), float(mu), float(sigma), float(c), float(h), flags))


def band_limits(E: int, K: int, n_e: int, n_k: int, W: int):
    lo = np.zeros(1, np.int64)
    hi = np.zeros(1, np.int64)
    lib().oracle_band_limits(E, K, n_e, n_k, W, _p(lo), _p(hi))
    return int(lo[0]), int(hi[0])


@dataclasses.dataclass
class Result:
    status: int
    score: np.float32
    pairs: np.ndarray  # int32 [n, 2] (event_idx, kmer_idx)
    cells: int
    n_bands: int
    kmer_moves: int
    min_margin: float
    min_move_margin: float
    trace: Optional[np.ndarray] = None  # uint8 [n_bands, W]
    ll: Optional[np.ndarray] = None  # int64 [n_bands, 2]
    in_table_bands: int = 0  # bands whose W cells all lie in the table
    in_table_inf_ends: int = 0  # of those, bands with an end cell at -inf


class Model:
    """Pore model with its emission terms, prepared once."""

    def __init__(self, level_mean: np.ndarray, level_stdv: np.ndarray):
        self.level_mean = np.ascontiguousarray(level_mean, np.float32)
        self.level_stdv = np.ascontiguousarray(level_stdv, np.float32)
        self.c, self.h = model_terms(self.level_stdv)

    @property
    def n(self) -> int:
        return int(self.level_mean.shape[0])


def align(
    event_mean: np.ndarray,
    ranks: np.ndarray,
    model: Model,
    scale: float,
    shift: float,
    W: int,
    flags: int = 0,
    want_trace: bool = False,
) -> Result:
    """Align one read.  ``event_mean`` is a float32 vector (or an [n, 3] event
    table whose first column is the mean)."""
    ev = np.ascontiguousarray(event_mean, np.float32)
    stride = 1 if ev.ndim == 1 else ev.shape[1]
    n_e = ev.shape[0]
    rk = np.ascontiguousarray(ranks, np.uint32)
    n_k = rk.shape[0]
    pairs = np.zeros((n_e + n_k + 1, 2), np.int32)
    score = np.zeros(1, np.float32)
    st = _Stats()
    nb = n_e + n_k + 1
    trace = np.zeros((nb, W), np.uint8) if want_trace else None
    ll = np.zeros((nb, 2), np.int64) if want_trace else None
    s = lib().oracle_align(
        _p(ev), stride, n_e, _p(rk), n_k, _p(model.level_mean), _p(model.level_stdv),
        _p(model.c), _p(model.h), model.n, float(np.float32(scale)), float(np.float32(shift)),
        W, flags, _p(pairs), _p(score), ctypes.byref(st),
        _p(trace) if want_trace else None, _p(ll) if want_trace else None,
    )
    if s < 0:
        raise RuntimeError(f"oracle_align error {s}")
    return Result(
        s, score[0], pairs[: st.path_len].copy(), st.cells, st.n_bands, st.kmer_moves,
        st.min_margin, st.min_move_margin, trace, ll, st.in_table_bands, st.in_table_inf_ends,
    )


@dataclasses.dataclass
class BatchResult:
    status: np.ndarray
    score: np.ndarray
    path_len: np.ndarray
    cells: np.ndarray
    pair_slot: np.ndarray
    pairs: np.ndarray  # int32 [capacity, 2]
    min_margin: np.ndarray  # float64 [n]: smallest band-move or path-cell decision margin

    def read_pairs(self, r: int) -> np.ndarray:
        s = int(self.pair_slot[r])
        return self.pairs[s : s + int(self.path_len[r])]


def align_batch(batch, model: Model, W: int, n_threads: int = 1, flags: int = 0) -> BatchResult:
    """Align a synthetic batch (``paper_2101_05012_amd.synth.Batch``) on
    ``n_threads`` host threads."""
    n = batch.n_reads
    ev = np.ascontiguousarray(batch.events, np.float32)
    sizes = np.diff(batch.event_offset) + np.diff(batch.kmer_offset)
    slot = np.zeros(n + 1, np.uint64)
    np.cumsum(sizes, out=slot[1:])
    pairs = np.zeros((int(slot[-1]) + 1, 2), np.int32)
    path_len = np.zeros(n, np.int64)
    score = np.zeros(n, np.float32)
    status = np.zeros(n, np.int32)
    cells = np.zeros(n, np.int64)
    margin = np.zeros(n, np.float64)
    eo = np.ascontiguousarray(batch.event_offset, np.uint64)
    ko = np.ascontiguousarray(batch.kmer_offset, np.uint64)
    rk = np.ascontiguousarray(batch.ranks, np.uint32)
    sc = np.ascontiguousarray(batch.scale, np.float32)
    sh = np.ascontiguousarray(batch.shift, np.float32)
    err = lib().oracle_align_batch(
        n, _p(ev), 3, _p(eo), _p(rk), _p(ko), _p(sc), _p(sh),
        _p(model.level_mean), _p(model.level_stdv), _p(model.c), _p(model.h), model.n,
        W, flags, n_threads, _p(slot), _p(pairs), _p(path_len), _p(score), _p(status), _p(cells),
        _p(margin),
    )
    if err < 0:
        raise RuntimeError(f"oracle_align_batch error {err}")
    return BatchResult(status, score, path_len, cells, slot[:-1], pairs, margin)


# ---- event detection (event_oracle.c) ----------------------------------------


class EdParams(ctypes.Structure):
    """Detector parameters: a short and a long window (samples) with their t
    thresholds."""

    _fields_ = [("w_short", ctypes.c_int32), ("w_long", ctypes.c_int32),
                ("t_short", ctypes.c_float), ("t_long", ctypes.c_float)]


def ed_params(w_short: int = 3, t_short: float = 1.5, w_long: int = 8, t_long: float = 5.0) -> EdParams:
    return EdParams(w_short, w_long, t_short, t_long)


def _raw(x) -> np.ndarray:
    return np.ascontiguousarray(x, np.int16)


def ed_stat(x, w: int, i: int) -> np.float32:
    """T(i) of the detector with window w (-1 where undefined)."""
    x = _raw(x)
    return np.float32(lib().oracle_ed_stat(_p(x), x.shape[0], w, i))


def ed_stats(x, offset: float, pa_scale: float) -> np.ndarray:
    """{mean, stdv, duration} of one event's samples."""
    x = _raw(x)
    out = np.zeros(3, np.float32)
    lib().oracle_ed_stats(_p(x), x.shape[0], float(np.float32(offset)), float(np.float32(pa_scale)), _p(out))
    return out


def ed_change_points(x, params: Optional[EdParams] = None) -> np.ndarray:
    """Sample indices where events start (besides sample 0)."""
    x = _raw(x)
    cp = np.zeros(x.shape[0] + 1, np.uint8)
    m = lib().oracle_ed_change_points(_p(x), x.shape[0], ctypes.byref(params or ed_params()), _p(cp))
    if m < 0:
        raise RuntimeError("oracle_ed_change_points failed")
    return np.nonzero(cp)[0].astype(np.int64)


def ed_read(x, offset: float, pa_scale: float, params: Optional[EdParams] = None) -> np.ndarray:
    """Events of one read as float32 [m, 3] (mean, stdv, duration)."""
    x = _raw(x)
    ev = np.zeros((max(x.shape[0], 1), 3), np.float32)
    m = lib().oracle_ed_read(_p(x), x.shape[0], float(np.float32(offset)), float(np.float32(pa_scale)),
                             ctypes.byref(params or ed_params()), _p(ev))
    if m < 0:
        raise RuntimeError("oracle_ed_read failed")
    return ev[:m].copy()


def ed_batch(raw_batch, params: Optional[EdParams] = None, n_threads: int = 1):
    """Events of a raw batch (``paper_2101_05012_amd.synth.RawBatch``):
    (events float32 [m, 3], event_offset uint64 [n+1])."""
    n = raw_batch.n_reads
    raw = _raw(raw_batch.raw)
    so = np.ascontiguousarray(raw_batch.sample_offset, np.uint64)
    off = np.ascontiguousarray(raw_batch.offset, np.float32)
    sc = np.ascontiguousarray(raw_batch.pa_scale, np.float32)
    ev = np.zeros((max(int(so[-1]) if n else 0, 1), 3), np.float32)
    cnt = np.zeros(max(n, 1), np.int64)
    err = lib().oracle_ed_batch(n, _p(raw), _p(so), _p(off), _p(sc), ctypes.byref(params or ed_params()),
                                n_threads, _p(ev), _p(cnt))
    if err < 0:
        raise RuntimeError("oracle_ed_batch failed")
    eo = np.zeros(n + 1, np.uint64)
    np.cumsum(cnt[:n], out=eo[1:])
    out = np.zeros((int(eo[-1]), 3), np.float32)
    for r in range(n):
        a = int(so[r])
        out[int(eo[r]):int(eo[r + 1])] = ev[a:a + int(cnt[r])]
    return out, eo


# ---- methylation scoring (meth_oracle.c) ----------------------------------------


class _MethModel(ctypes.Structure):
    _fields_ = [("level_mean", ctypes.c_void_p), ("level_stdv", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("h", ctypes.c_void_p)]


def _meth_struct(model: Model) -> _MethModel:
    return _MethModel(model.level_mean.ctypes.data, model.level_stdv.ctypes.data, model.c.ctypes.data,
                      model.h.ctypes.data)


def meth_is_site(rank: int, k: int) -> bool:
    return bool(lib().oracle_meth_is_site(int(rank), int(k)))


def meth_profile(x, mu, sigma, c, h, lp, flags: int = 0) -> np.float32:
    """Best-path score of events x through a window of k-mers."""
    x = np.ascontiguousarray(x, np.float32)
    arrs = [np.ascontiguousarray(a, np.float32) for a in (mu, sigma, c, h)]
    lpa = np.ascontiguousarray(lp, np.float32)
    return np.float32(lib().oracle_meth_profile(_p(x), x.shape[0], *[_p(a) for a in arrs], arrs[0].shape[0],
                                                _p(lpa), flags))


def meth_read(event_mean, ranks, k: int, model_u: Model, model_m: Model, scale, shift, pairs, flags: int = 0):
    """One read: (llr float32 [n_k], n_ev int32 [n_k]); NaN / 0 off the sites."""
    ev = np.ascontiguousarray(event_mean, np.float32)
    stride = 1 if ev.ndim == 1 else ev.shape[1]
    rk = np.ascontiguousarray(ranks, np.uint32)
    pr = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    llr = np.zeros(rk.shape[0], np.float32)
    nev = np.zeros(rk.shape[0], np.int32)
    mu, mm = _meth_struct(model_u), _meth_struct(model_m)
    rc = lib().oracle_meth_read(_p(ev), stride, ev.shape[0], _p(rk), rk.shape[0], k, ctypes.byref(mu),
                                ctypes.byref(mm), float(np.float32(scale)), float(np.float32(shift)), flags,
                                _p(pr), pr.shape[0], _p(llr), _p(nev))
    if rc < 0:
        raise RuntimeError("oracle_meth_read failed")
    return llr, nev


def meth_batch(batch, k: int, model_u: Model, model_m: Model, pairs, pair_offset, status, n_threads: int = 1,
               flags: int = 0):
    """A batch (``synth.Batch``) with its alignment (pairs int32 [P, 2] in
    path order per read, pair_offset [n+1], status [n]): (llr, n_ev) per
    k-mer of the batch."""
    n = batch.n_reads
    ev = np.ascontiguousarray(batch.events, np.float32)
    eo = np.ascontiguousarray(batch.event_offset, np.uint64)
    ko = np.ascontiguousarray(batch.kmer_offset, np.uint64)
    rk = np.ascontiguousarray(batch.ranks, np.uint32)
    sc = np.ascontiguousarray(batch.scale, np.float32)
    sh = np.ascontiguousarray(batch.shift, np.float32)
    pr = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    po = np.ascontiguousarray(pair_offset, np.uint64)
    st = np.ascontiguousarray(status, np.int32)
    K = int(ko[-1]) if n else 0
    llr = np.zeros(max(K, 1), np.float32)
    nev = np.zeros(max(K, 1), np.int32)
    mu, mm = _meth_struct(model_u), _meth_struct(model_m)
    rc = lib().oracle_meth_batch(n, _p(ev), 3, _p(eo), _p(rk), _p(ko), k, ctypes.byref(mu), ctypes.byref(mm),
                                 _p(sc), _p(sh), flags, _p(pr), _p(po), _p(st), n_threads, _p(llr), _p(nev))
    if rc < 0:
        raise RuntimeError("oracle_meth_batch failed")
    return llr[:K], nev[:K]
