/*
 * abea_host.cpp -- host runtime of libabea.so: context, batch planning,
 * device buffers and the C ABI of include/abea.h.
 *
 * Planning follows the thesis's batch flow (Ch. 5 §5.4, Alg. 5.4: copy in,
 * align on the GPU, copy out) and its serialised layout (§5.4.2.1, Alg. 5.9:
 * per-read offsets are exclusive prefix sums).  Instead of the thesis's
 * heuristic pre-allocation with CPU overflow (§5.4.2.2, Alg. 5.10) every
 * buffer is sized exactly from the batch (a band costs W/4 bytes of trace,
 * far less than the W*5 bytes of score+trace the thesis stores), grown on
 * demand and kept for the next batch.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"
#include "abea_runtime.h"

using namespace abea;

static_assert(NOALLOC_SCRATCH_BYTES == ABEA_NOALLOC_SCRATCH_BYTES, "one size of the fixed scratch");

struct abea_graph {
  abea_ctx *ctx = nullptr;
  abea_rt::Work work;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace abea_rt {

int fail(abea_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int ensure(abea_ctx *ctx, Work *w, DevBuf &b, size_t bytes, hipStream_t st) {
  if (bytes == 0) bytes = 256;
  if (bytes <= b.cap) return ABEA_OK;
  const size_t rounded = (bytes + (2u << 20) - 1) & ~size_t((2u << 20) - 1);
  hipError_t e;
  if (w && ctx->pools) {
    /* stream-ordered growth: the old buffer is released on `st` once w's last
     * batch is done with it (same stream: stream order; another stream: a
     * device-side wait on that batch's event), and the new one is allocated
     * on `st` */
    if (b.p) {
      if (w->done_pending && w->last_stream != st) HIP_TRY(ctx, hipStreamWaitEvent(st, w->done, 0));
      if (b.pooled) {
        HIP_TRY(ctx, hipFreeAsync(b.p, st));
      } else {
        const int rc = work_wait(ctx, *w);
        if (rc) return rc;
        HIP_TRY(ctx, hipFree(b.p));
      }
      b.p = nullptr;
      b.cap = 0;
    }
    e = hipMallocAsync(&b.p, rounded, st);
    b.pooled = true;
  } else {
    /* a set-up buffer (no queued work uses it), or a device without memory
     * pools: wait for w's own last batch only */
    if (w && b.p) {
      const int rc = work_wait(ctx, *w);
      if (rc) return rc;
    }
    if (b.p) HIP_TRY(ctx, hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    e = hipMalloc(&b.p, rounded);
    b.pooled = false;
  }
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, ABEA_E_NOMEM, "device allocation of %zu bytes failed: %s", rounded, hipGetErrorString(e));
  }
  b.cap = rounded;
  return ABEA_OK;
}

void free_buf(DevBuf &b, hipStream_t st) {
  if (b.borrowed) {
    b = DevBuf();
    return;
  }
  if (b.p) {
    if (b.pooled)
      (void)hipFreeAsync(b.p, st);
    else
      (void)hipFree(b.p);
  }
  b.p = nullptr;
  b.cap = 0;
  b.pooled = false;
}

int work_init(abea_ctx *ctx, Work &w) {
  HIP_TRY(ctx, hipEventCreateWithFlags(&w.staging_done, hipEventDisableTiming));
  HIP_TRY(ctx, hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
  for (auto &ev : w.tev) HIP_TRY(ctx, hipEventCreate(&ev));
  return ABEA_OK;
}

int work_wait(abea_ctx *ctx, Work &w) {
  if (w.done_pending) HIP_TRY(ctx, hipEventSynchronize(w.done));
  w.done_pending = false;
  return ABEA_OK;
}

int work_mark(abea_ctx *ctx, Work &w, hipStream_t st) {
  HIP_TRY(ctx, hipEventRecord(w.done, st));
  w.last_stream = st;
  w.done_pending = true;
  return ABEA_OK;
}

void work_free(Work &w, hipStream_t st) {
  if (w.done_pending && w.done) (void)hipEventSynchronize(w.done);
  w.done_pending = false;
  DevBuf *bufs[] = {&w.reads, &w.rstat, &w.queue, &w.xmean, &w.krank,
                    &w.trace, &w.scratch, &w.path_len, &w.path_src, &w.tend};
  for (DevBuf *b : bufs) free_buf(*b, st);
  if (w.staging_pending && w.staging_done) (void)hipEventSynchronize(w.staging_done);
  w.staging_pending = false;
  if (w.h_reads) (void)hipHostFree(w.h_reads);
  w.h_reads = nullptr;
  w.h_cap = 0;
  for (void *h : w.retired_host) (void)hipHostFree(h);
  w.retired_host.clear();
  if (w.staging_done) (void)hipEventDestroy(w.staging_done);
  w.staging_done = nullptr;
  if (w.done) (void)hipEventDestroy(w.done);
  w.done = nullptr;
  for (auto &ev : w.tev) {
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
  }
}

/* Alg. 5.2 transition constants, each computed in double and rounded once;
 * the printed epsilon "1^{-10}" reads as 1e-10. */
void transitions(int64_t n_events, int64_t n_kmers, float *skip, float *stay, float *step) {
  const double epk = (double)n_events / (double)n_kmers;
  const double lskip = std::log(1e-10);
  const double lstay = std::log(1.0 - 1.0 / (epk + 1.0));
  const double lstep = std::log(1.0 - std::exp(lskip) - std::exp(lstay));
  *skip = (float)lskip;
  *stay = (float)lstay;
  *step = (float)lstep;
}

bool split_kernels(const abea_ctx *ctx) { return ctx->launch.workers == ABEA_WORKERS_SPLIT; }

/* Wavefronts of the fused kernel that are resident at once on the device. */
int resident_workers(abea_ctx *ctx, bool edge) {
  const int gpc = align_groups_per_cu(ctx->cpl, refills_per_group(ctx->W, ctx->cpl), ctx->launch.waves_per_group,
                                      edge, (ctx->flags & ABEA_F_TRIM) != 0, ctx->W);
  return std::max(1, gpc * ctx->num_cus * ctx->launch.waves_per_group);
}

/* Slot clearing of interior bands for a launch of `waves` wavefronts.  Edge
 * clearing trades per-band VALU work (every slot's window test) for scalar
 * work (two wave masks that follow the band); the scalar instructions cost a
 * lone wavefront more issue time than the vector ones they replace, and cost
 * less than them when other wavefronts on the SIMD keep the VALU busy.  At
 * four slots per lane it saves twice the vector work and wins either way; at
 * two it wins once the launch alone holds two wavefronts per SIMD. */
bool edge_clearing(const abea_ctx *ctx, int waves) {
  if (ctx->cpl != 2 && ctx->cpl != 4) return false;
  switch (ctx->launch.band_clear) {
    case ABEA_CLEAR_WINDOW: return false;
    case ABEA_CLEAR_EDGES: return true;
    default: return ctx->cpl == 4 || waves >= 2 * 4 * ctx->num_cus;
  }
}

/* Plan a batch from host offsets.
 *  - Reads are sorted by computed bands (n_e + n_k - 1, 0 for an empty read),
 *    longest first, so the longest band chains start first and every read
 *    fits the trace region of any read planned before it.
 *  - Pair scratch: n_e + n_k - 1 slots per read (a path never has more).
 *  - Trace, fused kernel with P workers: read s < P gets its own region and
 *    worker s reuses it for every later read it takes; P is the requested
 *    worker count, capped by residency and by the trace budget (admission by
 *    traceback bytes).
 *  - Trace, split kernels: every read of a part has its own region; the reads
 *    are cut into consecutive parts whose traces fit the budget, run one
 *    part after the other.
 * Only a read whose own trace exceeds the budget is refused (ABEA_E_NOMEM). */
int plan_batch(abea_ctx *ctx, Work &w, int n, const uint64_t *eo, const uint64_t *ko,
               uint64_t pair_capacity, bool fused_only, uint64_t budget_in) {
  Plan &P = w.plan;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  P.n = n;
  /* no allocation when the vectors already have the capacity (the
   * no-allocation entry point reserves it at creation) */
  w.order.resize(n);
  w.comp.resize(n);
  std::vector<uint64_t> &comp = w.comp;
  uint64_t need = 0;
  for (int r = 0; r < n; ++r) {
    if (eo[r + 1] < eo[r] || ko[r + 1] < ko[r])
      return fail(ctx, ABEA_E_INVAL, "offsets decrease at read %d", r);
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    if (ne > 0x3fffffffull || nk > 0x3fffffffull)
      return fail(ctx, ABEA_E_INVAL, "read %d is too long", r);
    comp[r] = (ne > 0 && nk > 0) ? ne + nk - 1 : 0;
    need += comp[r];
  }
  P.pairs_needed = need;
  if (pair_capacity < need)
    return fail(ctx, ABEA_E_CAPACITY, "pair_capacity %llu < %llu", (unsigned long long)pair_capacity,
                (unsigned long long)need);
  /* longest first, ties in read order (an in-place sort: no buffer) */
  std::iota(w.order.begin(), w.order.end(), 0);
  std::sort(w.order.begin(), w.order.end(),
            [&](int a, int b) { return comp[a] != comp[b] ? comp[a] > comp[b] : a < b; });

  /* trace words of planned read s, and the worker count */
  const int G = bands_per_group(ctx->cpl);
  auto words = [&](int s) -> uint64_t { return ((comp[w.order[s]] + G - 1) / G) * 64u; };
  const uint64_t budget = budget_in == UINT64_MAX ? ctx->trace_budget : budget_in;
  const bool split = split_kernels(ctx) && !fused_only;
  if (n > 0 && budget > 0 && words(0) * sizeof(uint2) > budget)
    return fail(ctx, ABEA_E_NOMEM, "the trace of the longest read (%llu bytes) exceeds the trace budget %llu",
                (unsigned long long)(words(0) * sizeof(uint2)), (unsigned long long)budget);
  int workers = n;
  const bool pool = !split && ctx->launch.workers > 0;
  P.edge = edge_clearing(ctx, pool ? std::min(n, ctx->launch.workers) : n);
  if (pool) workers = std::min(n, std::min(ctx->launch.workers, resident_workers(ctx, P.edge)));
  if (!split && budget > 0) {
    uint64_t sum = 0;
    int fit = 0;
    while (fit < workers && (sum + words(fit)) * sizeof(uint2) <= budget) sum += words(fit++);
    workers = fit; /* at least the longest read, which fits (checked above) */
  }
  P.workers = split ? 0 : workers;
  P.cpl = ctx->cpl;
  P.wpg = ctx->launch.waves_per_group;

  if ((size_t)n > w.h_cap) {
    /* a larger pinned staging buffer; the old one may still feed a queued
     * upload and is freed with the Work (freeing pinned memory here would
     * wait for the whole device) */
    const size_t cap = std::max<size_t>({(size_t)n, 2 * w.h_cap, 1024});
    ReadDesc *h = nullptr;
    void *dv = nullptr;
    /* mapped: a kernel reads it (see stage_plan) */
    HIP_TRY(ctx, hipHostMalloc((void **)&h, cap * sizeof(ReadDesc), hipHostMallocMapped | hipHostMallocCoherent));
    if (hipHostGetDevicePointer(&dv, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      return fail(ctx, ABEA_E_HIP, "hipHostGetDevicePointer failed");
    }
    if (w.h_reads) w.retired_host.push_back(w.h_reads);
    w.h_reads = h;
    w.d_view = (ReadDesc *)dv;
    w.h_cap = cap;
    w.staging_pending = false;
  }
  /* the previous call's upload must have left the staging buffer */
  if (w.staging_pending) HIP_TRY(ctx, hipEventSynchronize(w.staging_done));
  w.staging_pending = false;

  P.parts.assign(1, 0);
  uint64_t tr = 0, tr_max = 0, pr = 0;
  for (int s = 0; s < n; ++s) {
    const int r = w.order[s];
    ReadDesc &d = w.h_reads[s];
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    if (split && budget > 0 && comp[r] > 0 && (tr + words(s)) * sizeof(uint2) > budget) {
      P.parts.push_back(s); /* the next part reuses the trace buffer from 0 */
      tr = 0;
    }
    d.ev_off = eo[r];
    d.km_off = ko[r];
    d.n_e = (int32_t)ne;
    d.n_k = (int32_t)nk;
    d.orig = r;
    d.tr_off = (s < workers) ? tr : 0;
    d.spare = 0;
    d.pr_off = pr;
    d.lp_skip = d.lp_stay = d.lp_step = 0.f;
    if (comp[r] == 0) continue;
    transitions((int64_t)ne, (int64_t)nk, &d.lp_skip, &d.lp_stay, &d.lp_step);
    if (s < workers) tr += words(s);
    tr_max = std::max(tr_max, tr);
    pr += comp[r];
  }
  P.parts.push_back(n);
  P.n_trace = tr_max;
  P.n_scratch = pr;
  /* the 256 longest reads (about one per CU) issue at raised priority */
  {
    const int u = std::min(n, 256) - 1;
    P.urgent_len = u >= 0 ? (int32_t)std::max<uint64_t>(comp[w.order[u]] + 1, 1) : 0x7fffffff;
  }
  P.n_events = eo[n];
  P.n_kmers = ko[n];
  return ABEA_OK;
}

int ensure_work(abea_ctx *ctx, Work &w, hipStream_t st, bool staged_events) {
  const Plan &P = w.plan;
  const size_t n = (size_t)std::max(P.n, 1);
  int rc;
  if ((rc = ensure(ctx, &w, w.reads, sizeof(ReadDesc) * n, st))) return rc;
  if ((rc = ensure(ctx, &w, w.rstat, sizeof(int32_t) * n, st))) return rc;
  if ((rc = ensure(ctx, &w, w.queue, sizeof(uint32_t), st))) return rc;
  if ((staged_events || (ctx->flags & ABEA_F_SCALE_EVENTS)) &&
      (rc = ensure(ctx, &w, w.xmean, sizeof(float) * (size_t)P.n_events, st)))
    return rc;
  if (staged_events && (rc = ensure(ctx, &w, w.krank, sizeof(uint32_t) * (size_t)P.n_kmers, st))) return rc;
  if ((rc = ensure(ctx, &w, w.trace, sizeof(uint2) * (size_t)P.n_trace, st))) return rc;
  if ((rc = ensure(ctx, &w, w.scratch, sizeof(int2) * (size_t)P.n_scratch, st))) return rc;
  if ((rc = ensure(ctx, &w, w.path_len, sizeof(uint64_t) * n, st))) return rc;
  if ((rc = ensure(ctx, &w, w.path_src, sizeof(uint64_t) * n, st))) return rc;
  if ((rc = ensure(ctx, &w, w.tend, sizeof(int32_t) * n, st))) return rc;
  return ABEA_OK;
}

/* Enqueue the kernels of a planned batch whose plan is on the device. */
int enqueue_kernels(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st, bool timed) {
  const Plan &P = w.plan;
  const int n = P.n;
  const ReadDesc *reads = (const ReadDesc *)w.reads.p;
  int32_t *rstat = (int32_t *)w.rstat.p;
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[0], st));
  /* inputs at per-read addresses (serving: mapped host memory) are staged
   * by k_prep, ranks and event means, and so are the means of events scaled
   * to the model; otherwise the band fill reads both in place from the
   * device batch */
  const bool scale_events = (ctx->flags & ABEA_F_SCALE_EVENTS) != 0;
  const bool staged_in = io.in_addr != nullptr;
  const bool staged = staged_in || scale_events;
  HIP_TRY(ctx, launch_prep(reads, n, io.events, io.ev_stride, io.ranks, io.in_addr, io.scale, io.shift,
                           scale_events, staged ? (float *)w.xmean.p : nullptr,
                           staged_in ? (uint32_t *)w.krank.p : nullptr, rstat, (uint32_t *)w.queue.p, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[1], st));

  AlignArgs a;
  a.reads = reads;
  a.xsrc = staged ? (const float *)w.xmean.p : io.events;
  a.xstride = staged ? 1 : io.ev_stride;
  a.ranks = staged_in ? (const uint32_t *)w.krank.p : io.ranks;
  a.model = (const ModelEntry *)ctx->model.p;
  a.n_model = ctx->n_model;
  a.scale_events = scale_events ? 1 : 0;
  a.scale = io.scale;
  a.shift = io.shift;
  a.rstat = rstat;
  a.trace = (uint2 *)w.trace.p;
  a.scratch = (int2 *)w.scratch.p;
  a.path_len = (uint64_t *)w.path_len.p;
  a.path_src = (uint64_t *)w.path_src.p;
  a.out_ll = io.ll;
  a.out_cells = io.cells;
  a.out_status = io.status;
  a.queue = (uint32_t *)w.queue.p;
  a.n_reads = n;
  a.n_workers = P.workers;
  a.W = ctx->W;
  a.urgent_len = P.urgent_len;
  a.tend = (int32_t *)w.tend.p;
  a.trim = (ctx->flags & ABEA_F_TRIM) != 0;
  /* one trimmed event, probability 1/100: in double, rounded once */
  a.lp_trim = (float)std::log(1.0 / 100.0);
  /* the band or fused kernel's own start and end: with other batches in
   * flight its dispatch may wait for free CUs, which these do not count */
  hipEvent_t k0 = timed ? w.tev[2] : nullptr, k1 = timed ? w.tev[3] : nullptr;
  const bool launched = n > 0 && (P.workers == 0 || (P.workers > 0 && P.workers <= n));
  if (P.workers == 0) {
    /* split kernels, part after part over the same trace buffer (with more
     * than one part the band interval runs from the first part's band fill
     * to the last part's) */
    const int np = (int)P.parts.size() - 1;
    for (int p = 0; p < np; ++p) {
      AlignArgs ap = a;
      ap.reads = reads + P.parts[p];
      ap.rstat = rstat + P.parts[p];
      ap.n_reads = P.parts[p + 1] - P.parts[p];
      HIP_TRY(ctx, launch_band(ap, P.cpl, refills_per_group(ctx->W, P.cpl), P.edge, st, p == 0 ? k0 : nullptr,
                               p == np - 1 ? k1 : nullptr));
      if (p < np - 1) HIP_TRY(ctx, launch_backtrack(ap, P.cpl, st));
    }
  } else {
    HIP_TRY(ctx, launch_align(a, P.cpl, refills_per_group(ctx->W, P.cpl), P.wpg, P.edge, st, k0, k1));
  }
  if (timed && !launched) { /* nothing dispatched: an empty interval */
    HIP_TRY(ctx, hipEventRecord(w.tev[2], st));
    HIP_TRY(ctx, hipEventRecord(w.tev[3], st));
  }
  if (P.workers == 0 && P.parts.size() >= 2) {
    AlignArgs ap = a;
    const int lp = (int)P.parts.size() - 2;
    ap.reads = reads + P.parts[lp];
    ap.rstat = rstat + P.parts[lp];
    ap.n_reads = P.parts[lp + 1] - P.parts[lp];
    HIP_TRY(ctx, launch_backtrack(ap, P.cpl, st));
  }
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[4], st));

  HIP_TRY(ctx, launch_scan((const uint64_t *)w.path_len.p, n, io.pair_offset, st));
  HIP_TRY(ctx, launch_compact((const int2 *)w.scratch.p, (const uint64_t *)w.path_src.p,
                              io.pair_offset, n, io.pairs, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[5], st));
  w.timed = timed;
  return ABEA_OK;
}

/* The plan into device memory on `st`: by a kernel reading the mapped pinned
 * staging, so that the call issues no copy-engine command (a copy queued
 * behind this stream's earlier work would hold back every other stream's
 * copies until that work ends); a copy when the staging is not mapped. */
int stage_plan(abea_ctx *ctx, Work &w, int n, hipStream_t st) {
  if (w.d_view)
    HIP_TRY(ctx, launch_stage_plan(w.d_view, (ReadDesc *)w.reads.p, n, st));
  else
    HIP_TRY(ctx, hipMemcpyAsync(w.reads.p, w.h_reads, sizeof(ReadDesc) * n, hipMemcpyHostToDevice, st));
  return ABEA_OK;
}

/* Upload the plan and enqueue the batch on `st`. */
int run_planned(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st) {
  int rc;
  if ((rc = ensure_work(ctx, w, st))) return rc;
  if ((rc = stage_plan(ctx, w, w.plan.n, st))) return rc;
  HIP_TRY(ctx, hipEventRecord(w.staging_done, st));
  w.staging_pending = true;
  if ((rc = enqueue_kernels(ctx, w, io, st, (ctx->flags & ABEA_F_TIMING) != 0))) return rc;
  return work_mark(ctx, w, st);
}

/* ---- host-API staging ---------------------------------------------------- */

/* fn(lo, hi) over [0, n) on up to eight host threads, about `grain` items or
 * more each; the calling thread takes the first range, and any range whose
 * thread cannot start runs on it too. */
template <typename F>
void parallel_for(size_t n, size_t grain, F fn) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t T = std::min<size_t>({8, hw, std::max<size_t>(1, n / std::max<size_t>(grain, 1))});
  if (T <= 1) {
    fn(0, n);
    return;
  }
  const size_t per = (n + T - 1) / T;
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (size_t t = 1; t < T; ++t) {
    const size_t lo = std::min(n, t * per), hi = std::min(n, lo + per);
    if (lo >= hi) break;
    try {
      th.emplace_back(fn, lo, hi);
    } catch (...) {
      fn(lo, hi);
    }
  }
  fn(0, std::min(n, per));
  for (auto &x : th) x.join();
}

/* The pinned staging ring of the host API (two chunks), at the first call. */
int stage_init(abea_ctx *ctx) {
  for (int i = 0; i < 2; ++i) {
    if (!ctx->h_stage[i]) HIP_TRY(ctx, hipHostMalloc(&ctx->h_stage[i], ABEA_HOST_STAGING_CHUNK, hipHostMallocDefault));
    if (!ctx->stage_ev[i]) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->stage_ev[i], hipEventDisableTiming));
  }
  return ABEA_OK;
}

/* The next ring chunk, once the copy that last used it is done. */
int stage_take(abea_ctx *ctx, int *slot) {
  const int sl = ctx->stage_next;
  ctx->stage_next ^= 1;
  if (ctx->stage_pending[sl]) HIP_TRY(ctx, hipEventSynchronize(ctx->stage_ev[sl]));
  ctx->stage_pending[sl] = false;
  *slot = sl;
  return ABEA_OK;
}

/* dst[0, bytes) on the device from fill(off, len, chunk), chunk by chunk on
 * the context's stream: the host fills one chunk while the other is in
 * flight. */
template <typename Fill>
int stage_up(abea_ctx *ctx, void *dst, size_t bytes, Fill fill) {
  const size_t C = ABEA_HOST_STAGING_CHUNK;
  for (size_t off = 0; off < bytes; off += C) {
    int sl, rc;
    if ((rc = stage_take(ctx, &sl))) return rc;
    const size_t len = std::min(C, bytes - off);
    fill(off, len, (char *)ctx->h_stage[sl]);
    HIP_TRY(ctx, hipMemcpyAsync((char *)dst + off, ctx->h_stage[sl], len, hipMemcpyHostToDevice, ctx->own_stream));
    HIP_TRY(ctx, hipEventRecord(ctx->stage_ev[sl], ctx->own_stream));
    ctx->stage_pending[sl] = true;
  }
  return ABEA_OK;
}

int stage_copy_up(abea_ctx *ctx, void *dst, const void *src, size_t bytes) {
  const char *s = (const char *)src;
  return stage_up(ctx, dst, bytes, [s](size_t off, size_t len, char *d) {
    parallel_for(len, 1u << 20, [d, s, off](size_t lo, size_t hi) { std::memcpy(d + lo, s + off + lo, hi - lo); });
  });
}

/* src[0, bytes) on the device to drain(off, len, chunk), chunk by chunk:
 * the next chunk's copy is in flight while the host drains the last one. */
template <typename Drain>
int stage_down(abea_ctx *ctx, const void *src, size_t bytes, Drain drain) {
  const size_t C = ABEA_HOST_STAGING_CHUNK;
  int prev = -1;
  size_t prev_off = 0, prev_len = 0;
  for (size_t off = 0;; off += C) {
    int sl = -1, rc;
    if (off < bytes) {
      if ((rc = stage_take(ctx, &sl))) return rc;
      const size_t len = std::min(C, bytes - off);
      HIP_TRY(ctx, hipMemcpyAsync(ctx->h_stage[sl], (const char *)src + off, len, hipMemcpyDeviceToHost,
                                  ctx->own_stream));
      HIP_TRY(ctx, hipEventRecord(ctx->stage_ev[sl], ctx->own_stream));
      ctx->stage_pending[sl] = true;
    }
    if (prev >= 0) {
      HIP_TRY(ctx, hipEventSynchronize(ctx->stage_ev[prev]));
      ctx->stage_pending[prev] = false;
      drain(prev_off, prev_len, (const char *)ctx->h_stage[prev]);
    }
    if (off >= bytes) break;
    prev = sl;
    prev_off = off;
    prev_len = std::min(C, bytes - off);
  }
  return ABEA_OK;
}

int model_entries(const abea_model_t *model, std::vector<ModelEntry> &me) {
  if (!model->level_mean || !model->level_stdv || model->k < 1 || model->k > ABEA_MAX_K) return ABEA_E_INVAL;
  const uint32_t n_model = 1u << (2 * model->k);
  me.resize(n_model);
  /* Alg. 5.3: ln(1/sqrt(2 pi)) - ln(sigma) - 0.5 z^2, split into a per-entry
   * constant c and the factor h = 0.5/sigma^2 of (x - mu')^2, each computed
   * in double and rounded once. */
  for (uint32_t r = 0; r < n_model; ++r) {
    const float sd = model->level_stdv[r];
    if (!(sd > 0.0f) || !std::isfinite(sd) || !std::isfinite(model->level_mean[r])) return ABEA_E_INVAL;
    const double sigma = (double)sd;
    me[r].mean = model->level_mean[r];
    me[r].c = (float)(std::log(1.0 / std::sqrt(2.0 * M_PI)) - std::log(sigma));
    me[r].h = (float)(0.5 / (sigma * sigma));
    me[r].pad = 0.0f;
  }
  return ABEA_OK;
}

int stage_copy_down(abea_ctx *ctx, void *dst, const void *src, size_t bytes) {
  char *d = (char *)dst;
  return stage_down(ctx, src, bytes, [d](size_t off, size_t len, const char *s) {
    parallel_for(len, 1u << 20, [d, off, s](size_t lo, size_t hi) { std::memcpy(d + off + lo, s + lo, hi - lo); });
  });
}

int check_batch(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *r) {
  if (!ctx) return ABEA_E_INVAL;
  if (!b || !r) return fail(ctx, ABEA_E_INVAL, "null batch or result");
  if (b->n_reads < 0) return fail(ctx, ABEA_E_INVAL, "n_reads < 0");
  if (!b->event_offset || !b->kmer_offset || !r->pair_offset)
    return fail(ctx, ABEA_E_INVAL, "null offsets");
  if (b->n_reads > 0) {
    if (!b->scale || !b->shift || !r->log_likelihood || !r->status)
      return fail(ctx, ABEA_E_INVAL, "null per-read array");
    if (b->event_offset[b->n_reads] > 0 && !b->events) return fail(ctx, ABEA_E_INVAL, "null events");
    if (b->kmer_offset[b->n_reads] > 0 && !b->kmer_rank) return fail(ctx, ABEA_E_INVAL, "null k-mer ranks");
  }
  return ABEA_OK;
}

}  // namespace abea_rt

using namespace abea_rt;

extern "C" {

const char *abea_strerror(int status) {
  switch (status) {
    case ABEA_OK: return "ok";
    case ABEA_E_INVAL: return "invalid argument";
    case ABEA_E_NOMEM: return "out of memory";
    case ABEA_E_HIP: return "HIP runtime error";
    case ABEA_E_CAPACITY: return "pair capacity too small";
    case ABEA_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *abea_last_error(const abea_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int abea_create(const abea_config_t *cfg, const abea_model_t *model, abea_ctx **out) {
  if (!cfg || !model || !out) return ABEA_E_INVAL;
  *out = nullptr;
  if (cfg->bandwidth < 2 || cfg->bandwidth > ABEA_MAX_BANDWIDTH) return ABEA_E_INVAL;
  if (model->k < 1 || model->k > ABEA_MAX_K) return ABEA_E_INVAL;
  if (cfg->flags & ~ABEA_F_ALL) return ABEA_E_INVAL;
  const uint32_t n_model = 1u << (2 * model->k);
  std::vector<ModelEntry> me;
  if (model_entries(model, me) != ABEA_OK) return ABEA_E_INVAL;
  abea_ctx *ctx = new (std::nothrow) abea_ctx();
  if (!ctx) return ABEA_E_NOMEM;
  ctx->device = cfg->device;
  ctx->W = cfg->bandwidth;
  ctx->cpl = cells_per_lane(ctx->W);
  ctx->flags = cfg->flags;
  ctx->k = model->k;
  ctx->n_model = n_model;
  ctx->trace_budget = cfg->arena_bytes == ABEA_ARENA_UNBOUNDED ? 0 : cfg->arena_bytes;
  int rc = ABEA_OK;
  do {
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "hipSetDevice: %s", hipGetErrorString(e)); break; }
    e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "device attribute: %s", hipGetErrorString(e)); break; }
    int pools = 0;
    e = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, cfg->device);
    ctx->pools = (e == hipSuccess && pools != 0);
    (void)hipGetLastError();
    if (cfg->arena_bytes == ABEA_ARENA_AUTO) {
      /* a fraction of the device memory free now (the thesis's GPU memory
       * fraction, 0.9 by default) */
      size_t fr = 0, tot = 0;
      e = hipMemGetInfo(&fr, &tot);
      if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "hipMemGetInfo: %s", hipGetErrorString(e)); break; }
      ctx->trace_budget = std::max<uint64_t>((uint64_t)((double)fr * ABEA_ARENA_AUTO_FRACTION), 1);
    }
    if ((rc = ensure(ctx, nullptr, ctx->model, sizeof(ModelEntry) * n_model))) break;
    e = hipMemcpy(ctx->model.p, me.data(), sizeof(ModelEntry) * n_model, hipMemcpyHostToDevice);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "model upload: %s", hipGetErrorString(e)); break; }
    e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "stream: %s", hipGetErrorString(e)); break; }
    if ((rc = work_init(ctx, ctx->main))) break;
    /* the no-allocation entry point: the device's fixed scratch (its
     * address taken once per device, with the device current), and host
     * buffers for a plan of up to ABEA_NOALLOC_MAX_READS reads */
    e = noalloc_scratch(cfg->device, &ctx->noalloc_scratch);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "scratch address: %s", hipGetErrorString(e)); break; }
    if ((rc = work_init(ctx, ctx->noalloc))) break;
    ctx->noalloc.order.reserve(ABEA_NOALLOC_MAX_READS);
    ctx->noalloc.comp.reserve(ABEA_NOALLOC_MAX_READS);
    ctx->noalloc.plan.parts.reserve(ABEA_NOALLOC_MAX_READS + 2);
    e = hipHostMalloc((void **)&ctx->noalloc.h_reads, sizeof(ReadDesc) * ABEA_NOALLOC_MAX_READS,
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_NOMEM, "pinned plan staging: %s", hipGetErrorString(e)); break; }
    {
      void *dv = nullptr;
      e = hipHostGetDevicePointer(&dv, ctx->noalloc.h_reads, 0);
      if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "plan staging address: %s", hipGetErrorString(e)); break; }
      ctx->noalloc.d_view = (ReadDesc *)dv;
    }
    ctx->noalloc.h_cap = ABEA_NOALLOC_MAX_READS;
    ctx->err.reserve(512); /* error messages never reallocate */
  } while (0);
  if (rc != ABEA_OK) {
    abea_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return ABEA_OK;
}

void abea_destroy(abea_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  /* wait for this context's own work only (its last batch, and the host
   * API's copies on its stream), then release in order on its stream */
  (void)work_wait(ctx, ctx->main);
  hipStream_t st = ctx->own_stream;
  (void)work_wait(ctx, ctx->noalloc);
  if (st) (void)hipStreamSynchronize(st);
  detect_free(ctx, st);
  meth_free(ctx, st);
  work_free(ctx->main, st);
  work_free(ctx->noalloc, st);
  DevBuf *bufs[] = {&ctx->model, &ctx->events, &ctx->ranks, &ctx->scale, &ctx->shift,
                    &ctx->pairs, &ctx->pair_offset, &ctx->ll, &ctx->status, &ctx->cells};
  for (DevBuf *b : bufs) free_buf(*b, st);
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (int i = 0; i < 2; ++i) {
    if (ctx->h_stage[i]) (void)hipHostFree(ctx->h_stage[i]);
    if (ctx->stage_ev[i]) (void)hipEventDestroy(ctx->stage_ev[i]);
  }
  delete ctx;
}

int abea_cells_per_lane(int32_t bandwidth) {
  if (bandwidth < 2 || bandwidth > ABEA_MAX_BANDWIDTH) return 0;
  return cells_per_lane(bandwidth);
}

int abea_set_launch(abea_ctx *ctx, const abea_launch_t *l) {
  if (!ctx) return ABEA_E_INVAL;
  int rc;
  if (!l) return fail(ctx, ABEA_E_INVAL, "null launch");
  if (l->workers < ABEA_WORKERS_SPLIT) return fail(ctx, ABEA_E_INVAL, "workers < -1");
  if (l->waves_per_group != 1 && l->waves_per_group != 2 && l->waves_per_group != 4)
    return fail(ctx, ABEA_E_INVAL, "waves_per_group must be 1, 2 or 4");
  const int minc = cells_per_lane(ctx->W);
  int c = l->cells_per_lane == 0 ? minc : l->cells_per_lane;
  if (c < minc || c > 16 || (c & (c - 1)) != 0)
    return fail(ctx, ABEA_E_INVAL, "cells_per_lane %d: need a power of two in [%d, 16]", l->cells_per_lane, minc);
  if (refills_per_group(ctx->W, c) == 0) return fail(ctx, ABEA_E_INVAL, "cells_per_lane %d too small", c);
  if (l->band_clear != ABEA_CLEAR_AUTO && l->band_clear != ABEA_CLEAR_WINDOW && l->band_clear != ABEA_CLEAR_EDGES)
    return fail(ctx, ABEA_E_INVAL, "band_clear %d: need 0, 1 or 2", l->band_clear);
  if (l->band_clear == ABEA_CLEAR_EDGES && c != 2 && c != 4)
    return fail(ctx, ABEA_E_INVAL, "band_clear ABEA_CLEAR_EDGES needs 2 or 4 cells_per_lane, not %d", c);
  /* the context's queued batch was planned with the old form */
  if ((rc = work_wait(ctx, ctx->main))) return rc;
  ctx->launch = *l;
  ctx->cpl = c;
  return ABEA_OK;
}

int abea_get_plan_info(const abea_ctx *ctx, abea_plan_info_t *info) {
  if (!ctx || !info) return ABEA_E_INVAL;
  const Plan &P = ctx->main.plan;
  info->n_reads = P.n;
  info->workers = P.workers;
  info->cells_per_lane = P.cpl;
  info->waves_per_group = P.wpg;
  info->band_clear = P.edge ? ABEA_CLEAR_EDGES : ABEA_CLEAR_WINDOW;
  info->parts = std::max(1, (int)P.parts.size() - 1);
  info->trace_bytes = P.n_trace * sizeof(uint2);
  info->scratch_bytes = P.n_scratch * sizeof(int2);
  info->trace_budget = ctx->trace_budget;
  return ABEA_OK;
}

int abea_align_batch_device(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *r, void *stream) {
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  if (b->n_reads > 0 && (!r->pairs && r->pair_capacity > 0)) return fail(ctx, ABEA_E_INVAL, "null pairs");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int n = b->n_reads;
  if ((rc = plan_batch(ctx, ctx->main, n, b->event_offset, b->kmer_offset, r->pair_capacity))) return rc;
  if (n == 0) {
    /* a one-block kernel writes pair_offset[0] = 0 (no memset node, so the
     * call stays safe to capture in a graph) */
    HIP_TRY(ctx, launch_scan(nullptr, 0, r->pair_offset, st));
    return ABEA_OK;
  }
  DevIO io;
  io.events = (const float *)b->events;
  io.ranks = b->kmer_rank;
  io.scale = b->scale;
  io.shift = b->shift;
  io.pairs = (int2 *)r->pairs;
  io.pair_offset = r->pair_offset;
  io.ll = r->log_likelihood;
  io.status = r->status;
  io.cells = r->cells;
  return run_planned(ctx, ctx->main, io, st);
}

int abea_align_batch_device_noalloc(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *r,
                                    void *stream) {
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  if (b->n_reads > 0 && (!r->pairs && r->pair_capacity > 0)) return fail(ctx, ABEA_E_INVAL, "null pairs");
  if (b->n_reads > ABEA_NOALLOC_MAX_READS)
    return fail(ctx, ABEA_E_NOMEM, "%d reads: the no-allocation call takes at most %d", b->n_reads,
                ABEA_NOALLOC_MAX_READS);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int n = b->n_reads;
  const uint64_t *eo = b->event_offset, *ko = b->kmer_offset;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  /* the buffers other than the trace, laid out in the scratch array */
  uint64_t slots = 0;
  for (int i = 0; i < n; ++i) {
    if (eo[i + 1] < eo[i] || ko[i + 1] < ko[i]) return fail(ctx, ABEA_E_INVAL, "offsets decrease at read %d", i);
    const uint64_t ne = eo[i + 1] - eo[i], nk = ko[i + 1] - ko[i];
    if (ne > 0 && nk > 0) slots += ne + nk - 1;
  }
  const uint64_t nr = (uint64_t)std::max(n, 1);
  auto up = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  Work &w = ctx->noalloc;
  /* the event means are staged only for events scaled to the model (the
   * band fill reads them in place otherwise) */
  const uint64_t xbytes = (ctx->flags & ABEA_F_SCALE_EVENTS) ? sizeof(float) * eo[n] : 0;
  DevBuf *bufs[] = {&w.reads, &w.rstat, &w.queue, &w.path_len, &w.path_src, &w.tend, &w.xmean, &w.scratch};
  const uint64_t bytes[] = {sizeof(ReadDesc) * nr, sizeof(int32_t) * nr, sizeof(uint32_t), sizeof(uint64_t) * nr,
                            sizeof(uint64_t) * nr, sizeof(int32_t) * nr, xbytes, sizeof(int2) * slots};
  static_assert(sizeof(bufs) / sizeof(bufs[0]) == sizeof(bytes) / sizeof(bytes[0]), "one size per buffer");
  uint64_t fixed = 0;
  for (uint64_t x : bytes) fixed += up(x);
  if (fixed >= ABEA_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, ABEA_E_NOMEM,
                "the batch needs %llu bytes of scratch before its trace; the fixed array holds %llu",
                (unsigned long long)fixed, (unsigned long long)ABEA_NOALLOC_SCRATCH_BYTES);
  /* the rest holds the trace: the fused kernel admits as many reads at once
   * as their traces fit in it */
  const uint64_t budget = ABEA_NOALLOC_SCRATCH_BYTES - fixed;
  if ((rc = plan_batch(ctx, w, n, eo, ko, r->pair_capacity, true, budget))) return rc;
  if (n == 0) {
    HIP_TRY(ctx, launch_scan(nullptr, 0, r->pair_offset, st));
    return ABEA_OK;
  }
  unsigned char *base = (unsigned char *)ctx->noalloc_scratch;
  uint64_t off = 0;
  for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) {
    bufs[i]->p = base + off;
    bufs[i]->cap = bytes[i];
    bufs[i]->borrowed = true;
    off += up(bytes[i]);
  }
  w.trace.p = base + off;
  w.trace.cap = budget;
  w.trace.borrowed = true;
  if ((rc = stage_plan(ctx, w, n, st))) return rc;
  HIP_TRY(ctx, hipEventRecord(w.staging_done, st));
  w.staging_pending = true;
  DevIO io;
  io.events = (const float *)b->events;
  io.ranks = b->kmer_rank;
  io.scale = b->scale;
  io.shift = b->shift;
  io.pairs = (int2 *)r->pairs;
  io.pair_offset = r->pair_offset;
  io.ll = r->log_likelihood;
  io.status = r->status;
  io.cells = r->cells;
  if ((rc = enqueue_kernels(ctx, w, io, st, false))) return rc;
  return work_mark(ctx, w, st);
}

int abea_align_batch(abea_ctx *ctx, const abea_batch_t *b, abea_result_t *r) {
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int n = b->n_reads;
  if ((rc = plan_batch(ctx, ctx->main, n, b->event_offset, b->kmer_offset, r->pair_capacity))) return rc;
  if (n == 0) {
    r->pair_offset[0] = 0;
    return ABEA_OK;
  }
  const Plan &P = ctx->main.plan;
  if (P.pairs_needed > 0 && !r->pairs) return fail(ctx, ABEA_E_INVAL, "null pairs");
  hipStream_t st = ctx->own_stream;
  Work *w = &ctx->main;
  if ((rc = stage_init(ctx))) return rc;
  if ((rc = ensure(ctx, w, ctx->events, sizeof(float) * (size_t)P.n_events, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->ranks, sizeof(uint32_t) * (size_t)P.n_kmers, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->scale, sizeof(float) * (size_t)n, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->shift, sizeof(float) * (size_t)n, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->pairs, sizeof(abea_pair_t) * (size_t)P.pairs_needed, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->pair_offset, sizeof(uint64_t) * (size_t)(n + 1), st))) return rc;
  if ((rc = ensure(ctx, w, ctx->ll, sizeof(float) * (size_t)n, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->status, sizeof(int32_t) * (size_t)n, st))) return rc;
  if ((rc = ensure(ctx, w, ctx->cells, sizeof(uint64_t) * (size_t)n, st))) return rc;
  /* inputs through the pinned ring: the event means gathered out of the
   * 12-byte records, then the ranks, scales and shifts */
  const abea_event_t *ev = b->events;
  rc = stage_up(ctx, ctx->events.p, sizeof(float) * (size_t)P.n_events, [ev](size_t off, size_t len, char *dst) {
    float *d = (float *)dst;
    const abea_event_t *src = ev + off / sizeof(float);
    parallel_for(len / sizeof(float), 1u << 16, [d, src](size_t lo, size_t hi) {
      for (size_t i = lo; i < hi; ++i) d[i] = src[i].mean;
    });
  });
  if (rc) return rc;
  if ((rc = stage_copy_up(ctx, ctx->ranks.p, b->kmer_rank, sizeof(uint32_t) * (size_t)P.n_kmers))) return rc;
  if ((rc = stage_copy_up(ctx, ctx->scale.p, b->scale, sizeof(float) * (size_t)n))) return rc;
  if ((rc = stage_copy_up(ctx, ctx->shift.p, b->shift, sizeof(float) * (size_t)n))) return rc;
  DevIO io;
  io.events = (const float *)ctx->events.p;
  io.ev_stride = 1;
  io.ranks = (const uint32_t *)ctx->ranks.p;
  io.scale = (const float *)ctx->scale.p;
  io.shift = (const float *)ctx->shift.p;
  io.pairs = (int2 *)ctx->pairs.p;
  io.pair_offset = (uint64_t *)ctx->pair_offset.p;
  io.ll = (float *)ctx->ll.p;
  io.status = (int32_t *)ctx->status.p;
  io.cells = (uint64_t *)ctx->cells.p;
  if ((rc = run_planned(ctx, ctx->main, io, st))) return rc;
  /* the per-read results (small), then the pairs through the ring */
  HIP_TRY(ctx, hipMemcpyAsync(r->pair_offset, io.pair_offset, sizeof(uint64_t) * (n + 1),
                              hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(r->log_likelihood, io.ll, sizeof(float) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(r->status, io.status, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  if (r->cells)
    HIP_TRY(ctx, hipMemcpyAsync(r->cells, io.cells, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const uint64_t total = r->pair_offset[n];
  if (total > r->pair_capacity) return fail(ctx, ABEA_E_HIP, "internal: %llu pairs exceed capacity",
                                            (unsigned long long)total);
  return stage_copy_down(ctx, r->pairs, io.pairs, sizeof(abea_pair_t) * total);
}

int abea_get_timings(abea_ctx *ctx, float *out, int n) {
  if (!ctx || !out || n < 0) return ABEA_E_INVAL;
  Work &w = ctx->main;
  if (!w.timed) return fail(ctx, ABEA_E_UNSUPPORTED, "context not created with ABEA_F_TIMING");
  HIP_TRY(ctx, hipEventSynchronize(w.tev[5]));
  /* prep, band or fused kernel, backtrack, scan + compaction */
  static const int from[4] = {0, 2, 3, 4}, to[4] = {1, 3, 4, 5};
  for (int q = 0; q < n && q < 4; ++q) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, w.tev[from[q]], w.tev[to[q]]));
    out[q] = ms;
  }
  return ABEA_OK;
}

/* ---- captured graphs --------------------------------------------------- */

int abea_graph_create(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *r, abea_graph **out) {
  if (!out) return fail(ctx, ABEA_E_INVAL, "null graph out");
  *out = nullptr;
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  if (b->n_reads > 0 && (!r->pairs && r->pair_capacity > 0)) return fail(ctx, ABEA_E_INVAL, "null pairs");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  abea_graph *g = new (std::nothrow) abea_graph();
  if (!g) return ABEA_E_NOMEM;
  g->ctx = ctx;
  Work &w = g->work;
  const int n = b->n_reads;
  hipError_t e;
  do {
    if ((rc = work_init(ctx, w))) break;
    e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "stream: %s", hipGetErrorString(e)); break; }
    if ((rc = plan_batch(ctx, w, n, b->event_offset, b->kmer_offset, r->pair_capacity))) break;
    if ((rc = ensure_work(ctx, w, g->cap_stream))) break;
    /* the plan goes to the device once; replays do not copy */
    if (n > 0) {
      e = hipMemcpyAsync(w.reads.p, w.h_reads, sizeof(ReadDesc) * n, hipMemcpyHostToDevice, g->cap_stream);
      if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "plan upload: %s", hipGetErrorString(e)); break; }
    }
    e = hipStreamSynchronize(g->cap_stream);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "plan upload: %s", hipGetErrorString(e)); break; }
    e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "begin capture: %s", hipGetErrorString(e)); break; }
    int erc = ABEA_OK;
    if (n == 0) {
      hipError_t le = launch_scan(nullptr, 0, r->pair_offset, g->cap_stream);
      if (le != hipSuccess) erc = fail(ctx, ABEA_E_HIP, "capture: %s", hipGetErrorString(le));
    } else {
      DevIO io;
      io.events = (const float *)b->events;
      io.ranks = b->kmer_rank;
      io.scale = b->scale;
      io.shift = b->shift;
      io.pairs = (int2 *)r->pairs;
      io.pair_offset = r->pair_offset;
      io.ll = r->log_likelihood;
      io.status = r->status;
      io.cells = r->cells;
      erc = enqueue_kernels(ctx, w, io, g->cap_stream, false);
    }
    e = hipStreamEndCapture(g->cap_stream, &g->graph);
    if (erc != ABEA_OK) { rc = erc; break; }
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "end capture: %s", hipGetErrorString(e)); break; }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "instantiate: %s", hipGetErrorString(e)); break; }
  } while (0);
  if (rc != ABEA_OK) {
    abea_graph_destroy(g);
    return rc;
  }
  *out = g;
  return ABEA_OK;
}

int abea_graph_launch(abea_graph *g, void *stream) {
  if (!g || !g->exec) return ABEA_E_INVAL;
  abea_ctx *ctx = g->ctx;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipGraphLaunch(g->exec, (hipStream_t)stream));
  return work_mark(ctx, g->work, (hipStream_t)stream);
}

int abea_graph_info(const abea_graph *g, abea_plan_info_t *info) {
  if (!g || !info) return ABEA_E_INVAL;
  const Plan &P = g->work.plan;
  info->n_reads = P.n;
  info->workers = P.workers;
  info->cells_per_lane = P.cpl;
  info->waves_per_group = P.wpg;
  info->band_clear = P.edge ? ABEA_CLEAR_EDGES : ABEA_CLEAR_WINDOW;
  info->parts = std::max(1, (int)P.parts.size() - 1);
  info->trace_bytes = P.n_trace * sizeof(uint2);
  info->scratch_bytes = P.n_scratch * sizeof(int2);
  info->trace_budget = g->ctx->trace_budget;
  return ABEA_OK;
}

void abea_graph_destroy(abea_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  /* wait for the graph's last replay only, then release its buffers in
   * order on its own stream */
  (void)work_wait(g->ctx, g->work);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  work_free(g->work, g->cap_stream);
  if (g->cap_stream) {
    (void)hipStreamSynchronize(g->cap_stream);
    (void)hipStreamDestroy(g->cap_stream);
  }
  delete g;
}

}  // extern "C"
