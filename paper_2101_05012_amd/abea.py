"""Python binding of libabea.so (include/abea.h): argument marshalling only.

Every step of the alignment runs in the HIP library; this module converts
numpy arrays / torch tensors to the C structs and back.  PyTorch is used only
to hold device memory and to name a stream.  If the library is not built the
import of the binding fails loudly: there is no fallback.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabea.so")

ABEA_OK = 0
ABEA_E_INVAL = -1
ABEA_E_NOMEM = -2
ABEA_E_HIP = -3
ABEA_E_CAPACITY = -4
ABEA_E_UNSUPPORTED = -5

READ_OK, READ_EMPTY, READ_BAND_LOST, READ_BAD_RANK = 0, 1, 2, 3
READ_CANCELLED, READ_TIMED_OUT = 4, 5  # serving: completed without running
ABEA_MAX_BANDWIDTH = 512
ABEA_MAX_K = 12
ABEA_F_TIMING = 1
ABEA_F_SCALE_EVENTS = 2  # events scaled to the model: (x - shift) / scale
ABEA_F_TRIM = 4  # trim states: events at either end may stay unaligned at ln(1/100) each
ABEA_WORKERS_SPLIT = -1
ABEA_CLEAR_AUTO = 0  # band_clear: the library chooses
ABEA_CLEAR_WINDOW = 1  # every slot outside the band's cells, every band
ABEA_CLEAR_EDGES = 2  # interior bands: only the two slots beside the band
ABEA_ARENA_AUTO = 0  # arena_bytes: 0.9 of the device memory free at abea_create
ABEA_ARENA_UNBOUNDED = (1 << 64) - 1  # arena_bytes: no trace budget
ABEA_HOST_STAGING_CHUNK = 32 << 20
ABEA_NOALLOC_SCRATCH_BYTES = 256 << 20  # the fixed device scratch of abea_align_batch_device_noalloc
ABEA_NOALLOC_MAX_READS = 16384
ABEA_DETECT_MAX_WINDOW = 16
DETECT_DEFAULT = (3, 8, 1.5, 5.0)  # window_short, window_long, threshold_short, threshold_long

EXPORTED = (
    "abea_create",
    "abea_align_batch",
    "abea_align_batch_device",
    "abea_align_batch_device_noalloc",
    "abea_detect_events",
    "abea_detect_events_device",
    "abea_get_detect_timings",
    "abea_set_methylated_model",
    "abea_methylation_device",
    "abea_get_meth_timings",
    "abea_get_timings",
    "abea_set_launch",
    "abea_cells_per_lane",
    "abea_get_plan_info",
    "abea_graph_create",
    "abea_graph_launch",
    "abea_graph_info",
    "abea_graph_destroy",
    "abea_server_now_ns",
    "abea_server_create",
    "abea_server_submit",
    "abea_server_cancel",
    "abea_server_poll",
    "abea_server_stats",
    "abea_server_destroy",
    "abea_destroy",
    "abea_strerror",
    "abea_last_error",
)


class AbeaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class abea_event_t(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_float), ("stdv", ctypes.c_float), ("duration", ctypes.c_float)]


class abea_pair_t(ctypes.Structure):
    _fields_ = [("event_idx", ctypes.c_int32), ("kmer_idx", ctypes.c_int32)]


class abea_model_t(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("level_mean", ctypes.c_void_p), ("level_stdv", ctypes.c_void_p)]


class abea_config_t(ctypes.Structure):
    _fields_ = [
        ("bandwidth", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("arena_bytes", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
    ]


class abea_batch_t(ctypes.Structure):
    _fields_ = [
        ("n_reads", ctypes.c_int32),
        ("events", ctypes.c_void_p),
        ("event_offset", ctypes.c_void_p),
        ("kmer_rank", ctypes.c_void_p),
        ("kmer_offset", ctypes.c_void_p),
        ("scale", ctypes.c_void_p),
        ("shift", ctypes.c_void_p),
    ]


class abea_result_t(ctypes.Structure):
    _fields_ = [
        ("pairs", ctypes.c_void_p),
        ("pair_capacity", ctypes.c_uint64),
        ("pair_offset", ctypes.c_void_p),
        ("log_likelihood", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("cells", ctypes.c_void_p),
    ]


class abea_detect_params_t(ctypes.Structure):
    _fields_ = [
        ("window_short", ctypes.c_int32),
        ("window_long", ctypes.c_int32),
        ("threshold_short", ctypes.c_float),
        ("threshold_long", ctypes.c_float),
    ]


def detect_params(window_short: int = DETECT_DEFAULT[0], window_long: int = DETECT_DEFAULT[1],
                  threshold_short: float = DETECT_DEFAULT[2], threshold_long: float = DETECT_DEFAULT[3]):
    return abea_detect_params_t(int(window_short), int(window_long), float(threshold_short), float(threshold_long))


class abea_raw_batch_t(ctypes.Structure):
    _fields_ = [
        ("n_reads", ctypes.c_int32),
        ("samples", ctypes.c_void_p),
        ("sample_offset", ctypes.c_void_p),
        ("offset", ctypes.c_void_p),
        ("pa_scale", ctypes.c_void_p),
    ]


class abea_launch_t(ctypes.Structure):
    _fields_ = [
        ("workers", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("cells_per_lane", ctypes.c_int32),
        ("band_clear", ctypes.c_int32),
    ]


class abea_plan_info_t(ctypes.Structure):
    _fields_ = [
        ("n_reads", ctypes.c_int32),
        ("workers", ctypes.c_int32),
        ("cells_per_lane", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("trace_bytes", ctypes.c_uint64),
        ("scratch_bytes", ctypes.c_uint64),
        ("band_clear", ctypes.c_int32),
        ("parts", ctypes.c_int32),
        ("trace_budget", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class abea_server_config_t(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32),
        ("max_batch_reads", ctypes.c_int32),
        ("max_batch_events", ctypes.c_uint64),
        ("max_batch_kmers", ctypes.c_uint64),
        ("trace_budget_bytes", ctypes.c_uint64),
        ("host_staging_bytes", ctypes.c_uint64),
        ("max_queue_wait_ns", ctypes.c_int64),
    ]


class abea_completion_t(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("log_likelihood", ctypes.c_float),
        ("cells", ctypes.c_uint64),
        ("pair_offset", ctypes.c_uint64),
        ("n_pairs", ctypes.c_uint64),
        ("t_arrival_ns", ctypes.c_int64),
        ("t_admit_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64),
    ]


COMPLETION_DTYPE = np.dtype(
    [
        ("tag", np.uint64),
        ("status", np.int32),
        ("log_likelihood", np.float32),
        ("cells", np.uint64),
        ("pair_offset", np.uint64),
        ("n_pairs", np.uint64),
        ("t_arrival_ns", np.int64),
        ("t_admit_ns", np.int64),
        ("t_done_ns", np.int64),
    ]
)


class abea_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("pending", ctypes.c_uint64),
        ("micro_batches", ctypes.c_uint64),
        ("inflight_reads", ctypes.c_uint64),
        ("max_inflight_reads", ctypes.c_uint64),
        ("inflight_trace_bytes", ctypes.c_uint64),
        ("max_inflight_trace_bytes", ctypes.c_uint64),
        ("error", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("enqueue_ns", ctypes.c_uint64),
        ("device_ns", ctypes.c_uint64),
        ("harvest_ns", ctypes.c_uint64),
        ("submit_ns", ctypes.c_uint64),
        ("submit_copy_ns", ctypes.c_uint64),
        ("pageable_reads", ctypes.c_uint64),
        ("cancelled", ctypes.c_uint64),
        ("timed_out", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "reserved"}


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch bundles its own libamdhip64 with
        # the same SONAME as the system one.  Loading torch first makes the
        # library bind to that copy instead of bringing a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                "(the HIP library is the only implementation)"
            )
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.abea_create.argtypes = [ctypes.POINTER(abea_config_t), ctypes.POINTER(abea_model_t), ctypes.POINTER(P)]
        L.abea_create.restype = ctypes.c_int
        L.abea_align_batch.argtypes = [P, ctypes.POINTER(abea_batch_t), ctypes.POINTER(abea_result_t)]
        L.abea_align_batch.restype = ctypes.c_int
        L.abea_align_batch_device.argtypes = [P, ctypes.POINTER(abea_batch_t), ctypes.POINTER(abea_result_t), P]
        L.abea_align_batch_device.restype = ctypes.c_int
        L.abea_align_batch_device_noalloc.argtypes = [P, ctypes.POINTER(abea_batch_t), ctypes.POINTER(abea_result_t),
                                                      P]
        L.abea_align_batch_device_noalloc.restype = ctypes.c_int
        L.abea_detect_events.argtypes = [P, ctypes.POINTER(abea_raw_batch_t), ctypes.POINTER(abea_detect_params_t),
                                         P, ctypes.c_uint64, P]
        L.abea_detect_events.restype = ctypes.c_int
        L.abea_detect_events_device.argtypes = [P, ctypes.POINTER(abea_raw_batch_t),
                                                ctypes.POINTER(abea_detect_params_t), P, ctypes.c_uint64, P, P]
        L.abea_detect_events_device.restype = ctypes.c_int
        L.abea_set_methylated_model.argtypes = [P, ctypes.POINTER(abea_model_t)]
        L.abea_set_methylated_model.restype = ctypes.c_int
        L.abea_methylation_device.argtypes = [P, ctypes.POINTER(abea_batch_t), ctypes.POINTER(abea_result_t), P, P, P]
        L.abea_methylation_device.restype = ctypes.c_int
        L.abea_get_meth_timings.argtypes = [P, P, ctypes.c_int]
        L.abea_get_meth_timings.restype = ctypes.c_int
        L.abea_get_detect_timings.argtypes = [P, P, ctypes.c_int]
        L.abea_get_detect_timings.restype = ctypes.c_int
        L.abea_get_timings.argtypes = [P, P, ctypes.c_int]
        L.abea_get_timings.restype = ctypes.c_int
        L.abea_set_launch.argtypes = [P, ctypes.POINTER(abea_launch_t)]
        L.abea_set_launch.restype = ctypes.c_int
        L.abea_cells_per_lane.argtypes = [ctypes.c_int32]
        L.abea_cells_per_lane.restype = ctypes.c_int
        L.abea_get_plan_info.argtypes = [P, ctypes.POINTER(abea_plan_info_t)]
        L.abea_get_plan_info.restype = ctypes.c_int
        L.abea_graph_create.argtypes = [P, ctypes.POINTER(abea_batch_t), ctypes.POINTER(abea_result_t), ctypes.POINTER(P)]
        L.abea_graph_create.restype = ctypes.c_int
        L.abea_graph_launch.argtypes = [P, P]
        L.abea_graph_launch.restype = ctypes.c_int
        L.abea_graph_info.argtypes = [P, ctypes.POINTER(abea_plan_info_t)]
        L.abea_graph_info.restype = ctypes.c_int
        L.abea_graph_destroy.argtypes = [P]
        L.abea_graph_destroy.restype = None
        L.abea_server_now_ns.argtypes = []
        L.abea_server_now_ns.restype = ctypes.c_int64
        L.abea_server_create.argtypes = [P, ctypes.POINTER(abea_server_config_t), ctypes.POINTER(P)]
        L.abea_server_create.restype = ctypes.c_int
        L.abea_server_submit.argtypes = [P, ctypes.POINTER(abea_batch_t), P, P]
        L.abea_server_submit.restype = ctypes.c_int
        L.abea_server_cancel.argtypes = [P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.abea_server_cancel.restype = ctypes.c_int
        L.abea_server_poll.argtypes = [P, P, ctypes.c_int, P, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int)]
        L.abea_server_poll.restype = ctypes.c_int
        L.abea_server_stats.argtypes = [P, ctypes.POINTER(abea_server_stats_t)]
        L.abea_server_stats.restype = ctypes.c_int
        L.abea_server_destroy.argtypes = [P]
        L.abea_server_destroy.restype = None
        L.abea_destroy.argtypes = [P]
        L.abea_destroy.restype = None
        L.abea_strerror.argtypes = [ctypes.c_int]
        L.abea_strerror.restype = ctypes.c_char_p
        L.abea_last_error.argtypes = [P]
        L.abea_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor


@dataclasses.dataclass
class HostResult:
    pairs: np.ndarray  # int32 [total, 2]
    pair_offset: np.ndarray  # uint64 [n+1]
    log_likelihood: np.ndarray  # float32 [n]
    status: np.ndarray  # int32 [n]
    cells: np.ndarray  # uint64 [n]

    def read_pairs(self, r: int) -> np.ndarray:
        return self.pairs[int(self.pair_offset[r]) : int(self.pair_offset[r + 1])]


def min_cells_per_lane(W: int) -> int:
    """Band slots per lane the library uses for band width W."""
    c = lib().abea_cells_per_lane(int(W))
    if c <= 0:
        raise ValueError(f"band width {W} out of range")
    return c


def pair_capacity(event_offset: np.ndarray, kmer_offset: np.ndarray) -> int:
    ne = np.diff(np.asarray(event_offset, np.int64))
    nk = np.diff(np.asarray(kmer_offset, np.int64))
    return int(np.where((ne > 0) & (nk > 0), ne + nk - 1, 0).sum())


class Aligner:
    """One library context (pore model on the device, band width W)."""

    def __init__(
        self,
        level_mean,
        level_stdv,
        k: int,
        W: int = 100,
        device: int = 0,
        timing: bool = False,
        arena_bytes: int = 0,
        workers: int = 0,
        waves_per_group: int = 1,
        cells_per_lane: int = 0,
        scale_events: bool = False,
        band_clear: int = ABEA_CLEAR_AUTO,
        trim: bool = False,
    ):
        self._lm = np.ascontiguousarray(level_mean, np.float32)
        self._ls = np.ascontiguousarray(level_stdv, np.float32)
        flags = ((ABEA_F_TIMING if timing else 0) | (ABEA_F_SCALE_EVENTS if scale_events else 0)
                 | (ABEA_F_TRIM if trim else 0))
        cfg = abea_config_t(W, device, int(arena_bytes), flags)
        mdl = abea_model_t(k, self._lm.ctypes.data, self._ls.ctypes.data)
        h = ctypes.c_void_p()
        rc = lib().abea_create(ctypes.byref(cfg), ctypes.byref(mdl), ctypes.byref(h))
        if rc != ABEA_OK:
            raise AbeaError(rc, "abea_create: " + lib().abea_strerror(rc).decode())
        self.handle = h
        self.W = W
        self.k = k
        self.device = device
        if (workers, waves_per_group, cells_per_lane, band_clear) != (0, 1, 0, ABEA_CLEAR_AUTO):
            self.set_launch(workers, waves_per_group, cells_per_lane, band_clear)

    def set_launch(self, workers: int = 0, waves_per_group: int = 1, cells_per_lane: int = 0,
                   band_clear: int = ABEA_CLEAR_AUTO) -> None:
        """Launch form (abea_set_launch): workers -1 split kernels, 0 one fused
        wavefront per read, > 0 a persistent pool with a device work queue;
        band_clear one of ABEA_CLEAR_*."""
        L = abea_launch_t(int(workers), int(waves_per_group), int(cells_per_lane), int(band_clear))
        self._check(lib().abea_set_launch(self.handle, ctypes.byref(L)), "abea_set_launch")

    def plan_info(self) -> dict:
        info = abea_plan_info_t()
        self._check(lib().abea_get_plan_info(self.handle, ctypes.byref(info)), "abea_get_plan_info")
        return info.as_dict()

    def graph(self, dbatch: "DeviceBatch", dres: "DeviceResult") -> "Graph":
        """Capture the batch's kernels into a HIP graph (abea_graph_create)."""
        b, r = _dev_structs(dbatch, dres)
        g = ctypes.c_void_p()
        self._check(lib().abea_graph_create(self.handle, ctypes.byref(b), ctypes.byref(r), ctypes.byref(g)),
                    "abea_graph_create")
        return Graph(self, g, dbatch, dres)

    def _check(self, rc: int, what: str):
        if rc != ABEA_OK:
            msg = lib().abea_last_error(self.handle).decode()
            raise AbeaError(rc, f"{what}: {lib().abea_strerror(rc).decode()}: {msg}")

    def align(self, batch) -> HostResult:
        """Host-memory batch (``synth.Batch``-like) through abea_align_batch."""
        n = batch.n_reads
        ev = np.ascontiguousarray(batch.events, np.float32)
        eo = np.ascontiguousarray(batch.event_offset, np.uint64)
        ko = np.ascontiguousarray(batch.kmer_offset, np.uint64)
        rk = np.ascontiguousarray(batch.ranks, np.uint32)
        sc = np.ascontiguousarray(batch.scale, np.float32)
        sh = np.ascontiguousarray(batch.shift, np.float32)
        cap = pair_capacity(eo, ko)
        pairs = np.zeros((max(cap, 1), 2), np.int32)
        po = np.zeros(n + 1, np.uint64)
        ll = np.zeros(n, np.float32)
        st = np.zeros(n, np.int32)
        cells = np.zeros(n, np.uint64)
        b = abea_batch_t(n, _ptr(ev), _ptr(eo), _ptr(rk), _ptr(ko), _ptr(sc), _ptr(sh))
        r = abea_result_t(_ptr(pairs), cap, _ptr(po), _ptr(ll), _ptr(st), _ptr(cells))
        self._check(lib().abea_align_batch(self.handle, ctypes.byref(b), ctypes.byref(r)), "abea_align_batch")
        return HostResult(pairs[: int(po[-1])], po, ll, st, cells)

    def align_device(self, dbatch: "DeviceBatch", dres: "DeviceResult", stream=None) -> None:
        """Device-resident batch through abea_align_batch_device (asynchronous
        on ``stream``: a torch.cuda.Stream, a raw hipStream_t int, or None for
        torch's current stream)."""
        b, r = _dev_structs(dbatch, dres)
        self._check(
            lib().abea_align_batch_device(self.handle, ctypes.byref(b), ctypes.byref(r),
                                          ctypes.c_void_p(_stream_ptr(stream, self.device))),
            "abea_align_batch_device",
        )

    def align_device_noalloc(self, dbatch: "DeviceBatch", dres: "DeviceResult", stream=None) -> None:
        """The same through abea_align_batch_device_noalloc: no allocation,
        intermediate buffers in the library's fixed per-device scratch."""
        b, r = _dev_structs(dbatch, dres)
        self._check(
            lib().abea_align_batch_device_noalloc(self.handle, ctypes.byref(b), ctypes.byref(r),
                                                  ctypes.c_void_p(_stream_ptr(stream, self.device))),
            "abea_align_batch_device_noalloc",
        )

    def detect_events(self, raw_batch, params=None, event_capacity: Optional[int] = None):
        """Event detection of a host raw batch (``synth.RawBatch``-like) through
        abea_detect_events: (events float32 [m, 3], event_offset uint64 [n+1])."""
        n = raw_batch.n_reads
        x = np.ascontiguousarray(raw_batch.raw, np.int16)
        so = np.ascontiguousarray(raw_batch.sample_offset, np.uint64)
        off = np.ascontiguousarray(raw_batch.offset, np.float32)
        sc = np.ascontiguousarray(raw_batch.pa_scale, np.float32)
        cap = int(so[-1]) if event_capacity is None else int(event_capacity)
        ev = np.zeros((max(cap, 1), 3), np.float32)
        eo = np.zeros(n + 1, np.uint64)
        b = abea_raw_batch_t(n, _ptr(x), _ptr(so), _ptr(off), _ptr(sc))
        p = params if params is not None else detect_params()
        self._check(lib().abea_detect_events(self.handle, ctypes.byref(b), ctypes.byref(p), _ptr(ev), cap, _ptr(eo)),
                    "abea_detect_events")
        return ev[: int(eo[-1])], eo

    def detect_events_device(self, draw: "DeviceRawBatch", events, event_offset, params=None,
                             event_capacity: Optional[int] = None, stream=None) -> None:
        """Device raw batch through abea_detect_events_device (asynchronous):
        ``events`` a torch float32 [cap, 3] and ``event_offset`` a torch int64
        [n+1] on the device."""
        cap = int(events.shape[0]) if event_capacity is None else int(event_capacity)
        b = abea_raw_batch_t(draw.n_reads, _ptr(draw.samples), _ptr(draw.sample_offset), _ptr(draw.offset),
                             _ptr(draw.pa_scale))
        p = params if params is not None else detect_params()
        self._check(
            lib().abea_detect_events_device(self.handle, ctypes.byref(b), ctypes.byref(p), _ptr(events), cap,
                                            _ptr(event_offset), ctypes.c_void_p(_stream_ptr(stream, self.device))),
            "abea_detect_events_device",
        )

    def set_methylated_model(self, level_mean, level_stdv) -> None:
        """The methylated pore model (abea_set_methylated_model); same k."""
        self._mlm = np.ascontiguousarray(level_mean, np.float32)
        self._mls = np.ascontiguousarray(level_stdv, np.float32)
        mdl = abea_model_t(self.k, self._mlm.ctypes.data, self._mls.ctypes.data)
        self._check(lib().abea_set_methylated_model(self.handle, ctypes.byref(mdl)), "abea_set_methylated_model")

    def methylation_device(self, dbatch: "DeviceBatch", dres: "DeviceResult", llr, n_events=None, stream=None) -> None:
        """Methylation LLR per k-mer of an aligned device batch
        (abea_methylation_device): ``llr`` a torch float32 [total k-mers],
        ``n_events`` a torch int32 [total k-mers] or None."""
        b, r = _dev_structs(dbatch, dres)
        self._check(
            lib().abea_methylation_device(self.handle, ctypes.byref(b), ctypes.byref(r), _ptr(llr), _ptr(n_events),
                                          ctypes.c_void_p(_stream_ptr(stream, self.device))),
            "abea_methylation_device",
        )

    def meth_timings(self) -> np.ndarray:
        """Milliseconds of [per-read kernel, per-site kernel] of the last
        methylation call (the context needs timing=True)."""
        out = np.zeros(2, np.float32)
        self._check(lib().abea_get_meth_timings(self.handle, _ptr(out), 2), "abea_get_meth_timings")
        return out

    def detect_timings(self) -> np.ndarray:
        """Milliseconds of [change-point kernel, event kernel, whole batch] of
        the last detection call (the context needs timing=True)."""
        out = np.zeros(3, np.float32)
        self._check(lib().abea_get_detect_timings(self.handle, _ptr(out), 3), "abea_get_detect_timings")
        return out

    def timings(self) -> np.ndarray:
        """Milliseconds of [prep, band, backtrack, compaction] of the last call."""
        out = np.zeros(4, np.float32)
        self._check(lib().abea_get_timings(self.handle, _ptr(out), 4), "abea_get_timings")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().abea_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream, device: int) -> int:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream(device)
    return stream if isinstance(stream, int) else int(stream.cuda_stream)


def _dev_structs(dbatch: "DeviceBatch", dres: "DeviceResult"):
    b = abea_batch_t(
        dbatch.n_reads, _ptr(dbatch.events), _ptr(dbatch.event_offset), _ptr(dbatch.ranks),
        _ptr(dbatch.kmer_offset), _ptr(dbatch.scale), _ptr(dbatch.shift),
    )
    r = abea_result_t(
        _ptr(dres.pairs), dres.capacity, _ptr(dres.pair_offset), _ptr(dres.log_likelihood),
        _ptr(dres.status), _ptr(dres.cells),
    )
    return b, r


class Graph:
    """A captured batch (abea_graph_*): replay with ``launch(stream)``."""

    def __init__(self, aligner: Aligner, handle, dbatch, dres):
        self.aligner = aligner
        self.handle = handle
        self.dbatch = dbatch  # keeps the device buffers alive
        self.dres = dres

    def launch(self, stream=None) -> None:
        rc = lib().abea_graph_launch(self.handle, ctypes.c_void_p(_stream_ptr(stream, self.aligner.device)))
        self.aligner._check(rc, "abea_graph_launch")

    def info(self) -> dict:
        info = abea_plan_info_t()
        self.aligner._check(lib().abea_graph_info(self.handle, ctypes.byref(info)), "abea_graph_info")
        return info.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().abea_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class DeviceBatch:
    n_reads: int
    events: object  # torch float32 [N, 3] on the device
    ranks: object  # torch int32 [K] (uint32 bits) on the device
    scale: object
    shift: object
    event_offset: np.ndarray  # host uint64 [n+1]
    kmer_offset: np.ndarray  # host uint64 [n+1]

    @property
    def capacity(self) -> int:
        return pair_capacity(self.event_offset, self.kmer_offset)


def to_device(batch, device: int = 0) -> DeviceBatch:
    import torch

    dev = torch.device("cuda", device)
    return DeviceBatch(
        batch.n_reads,
        torch.from_numpy(np.ascontiguousarray(batch.events, np.float32)).to(dev),
        torch.from_numpy(np.ascontiguousarray(batch.ranks, np.uint32).view(np.int32)).to(dev),
        torch.from_numpy(np.ascontiguousarray(batch.scale, np.float32)).to(dev),
        torch.from_numpy(np.ascontiguousarray(batch.shift, np.float32)).to(dev),
        np.ascontiguousarray(batch.event_offset, np.uint64),
        np.ascontiguousarray(batch.kmer_offset, np.uint64),
    )


@dataclasses.dataclass
class DeviceRawBatch:
    n_reads: int
    samples: object  # torch int16 [S] on the device
    offset: object  # torch float32 [n]
    pa_scale: object  # torch float32 [n]
    sample_offset: np.ndarray  # host uint64 [n+1]

    @property
    def n_samples(self) -> int:
        return int(self.sample_offset[-1])


def raw_to_device(raw_batch, device: int = 0) -> DeviceRawBatch:
    import torch

    dev = torch.device("cuda", device)
    return DeviceRawBatch(
        raw_batch.n_reads,
        torch.from_numpy(np.ascontiguousarray(raw_batch.raw, np.int16)).to(dev),
        torch.from_numpy(np.ascontiguousarray(raw_batch.offset, np.float32)).to(dev),
        torch.from_numpy(np.ascontiguousarray(raw_batch.pa_scale, np.float32)).to(dev),
        np.ascontiguousarray(raw_batch.sample_offset, np.uint64),
    )


@dataclasses.dataclass
class DeviceResult:
    pairs: object  # torch int32 [cap, 2]
    capacity: int
    pair_offset: object  # torch int64 [n+1] (uint64 bits)
    log_likelihood: object  # torch float32 [n]
    status: object  # torch int32 [n]
    cells: object  # torch int64 [n] (uint64 bits)

    @staticmethod
    def empty(dbatch: DeviceBatch, device: int = 0) -> "DeviceResult":
        import torch

        dev = torch.device("cuda", device)
        cap = dbatch.capacity
        n = dbatch.n_reads
        return DeviceResult(
            torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev),
            cap,
            torch.empty(n + 1, dtype=torch.int64, device=dev),
            torch.empty(max(n, 1), dtype=torch.float32, device=dev),
            torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            torch.empty(max(n, 1), dtype=torch.int64, device=dev),
        )

    def to_host(self, n: int) -> HostResult:
        po = self.pair_offset.cpu().numpy().view(np.uint64)
        total = int(po[-1])
        return HostResult(
            self.pairs[:total].cpu().numpy(),
            po,
            self.log_likelihood[:n].cpu().numpy(),
            self.status[:n].cpu().numpy(),
            self.cells[:n].cpu().numpy().view(np.uint64),
        )


def now_ns() -> int:
    """The serving loop's clock (steady, nanoseconds)."""
    return int(lib().abea_server_now_ns())


class Server:
    """Continuous-batching serving loop of the library (abea_server_*)."""

    def __init__(self, aligner: Aligner, slots: int = 4, max_batch_reads: int = 1024,
                 max_batch_events: int = 1 << 24, max_batch_kmers: int = 1 << 23, trace_budget_bytes: int = 0,
                 host_staging_bytes: int = 0, max_queue_wait_ns: int = 0):
        self.aligner = aligner
        cfg = abea_server_config_t(int(slots), int(max_batch_reads), int(max_batch_events), int(max_batch_kmers),
                                   int(trace_budget_bytes), int(host_staging_bytes), int(max_queue_wait_ns))
        h = ctypes.c_void_p()
        aligner._check(lib().abea_server_create(aligner.handle, ctypes.byref(cfg), ctypes.byref(h)),
                       "abea_server_create")
        self.handle = h
        self._out = np.zeros(0, COMPLETION_DTYPE)
        self._pairs = np.zeros((0, 2), np.int32)

    def submit(self, batch, lo: int, hi: int, tags, arrival_ns=None) -> None:
        """Queue reads [lo, hi) of a host batch (``synth.Batch``-like)."""
        eo = batch.event_offset
        ko = batch.kmer_offset
        e0, e1 = int(eo[lo]), int(eo[hi])
        k0, k1 = int(ko[lo]), int(ko[hi])
        ev = np.ascontiguousarray(batch.events[e0:e1], np.float32)
        rk = np.ascontiguousarray(batch.ranks[k0:k1], np.uint32)
        eor = np.ascontiguousarray(eo[lo : hi + 1] - eo[lo], np.uint64)
        kor = np.ascontiguousarray(ko[lo : hi + 1] - ko[lo], np.uint64)
        sc = np.ascontiguousarray(batch.scale[lo:hi], np.float32)
        sh = np.ascontiguousarray(batch.shift[lo:hi], np.float32)
        tg = np.ascontiguousarray(tags, np.uint64)
        at = None if arrival_ns is None else np.ascontiguousarray(arrival_ns, np.int64)
        b = abea_batch_t(hi - lo, _ptr(ev), _ptr(eor), _ptr(rk), _ptr(kor), _ptr(sc), _ptr(sh))
        self.aligner._check(lib().abea_server_submit(self.handle, ctypes.byref(b), _ptr(tg), _ptr(at)),
                            "abea_server_submit")

    def cancel(self, tags) -> int:
        """Cancel the queued reads with these tags (abea_server_cancel); returns
        how many were still queued and are now cancelled."""
        tg = np.ascontiguousarray(tags, np.uint64)
        k = ctypes.c_int(0)
        self.aligner._check(lib().abea_server_cancel(self.handle, _ptr(tg), int(tg.shape[0]), ctypes.byref(k)),
                            "abea_server_cancel")
        return k.value

    def poll(self, max_out: int = 4096, timeout_us: int = 1000, pair_capacity: int = 1 << 22, want_pairs: bool = True):
        """Finished reads: (completions structured array, pairs int32 [total, 2]
        or None when want_pairs is False)."""
        if self._out.shape[0] < max_out:
            self._out = np.zeros(max_out, COMPLETION_DTYPE)
        if want_pairs and self._pairs.shape[0] < pair_capacity:
            self._pairs = np.zeros((pair_capacity, 2), np.int32)
        n = ctypes.c_int(0)
        pp, cap = (_ptr(self._pairs), int(self._pairs.shape[0])) if want_pairs else (None, 0)
        rc = lib().abea_server_poll(self.handle, _ptr(self._out), int(max_out), pp, cap, int(timeout_us),
                                    ctypes.byref(n))
        if rc == ABEA_E_CAPACITY:  # the next result is larger: grow and retry
            self._pairs = np.zeros((self._pairs.shape[0] * 4, 2), np.int32)
            return self.poll(max_out, timeout_us, self._pairs.shape[0], want_pairs)
        self.aligner._check(rc, "abea_server_poll")
        k = n.value
        comp = self._out[:k].copy()
        if not want_pairs:
            return comp, None
        total = int((comp["n_pairs"]).sum()) if k else 0
        return comp, self._pairs[:total].copy()

    def stats(self) -> dict:
        st = abea_server_stats_t()
        self.aligner._check(lib().abea_server_stats(self.handle, ctypes.byref(st)), "abea_server_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().abea_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
