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
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"
#include "abea_runtime.h"

using namespace abea;

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



int ensure(abea_ctx *ctx, Work *w, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (bytes <= b.cap) return ABEA_OK;
  /* kernels queued by earlier calls may still use the old buffer */
  if (w && w->last_stream) HIP_TRY(ctx, hipStreamSynchronize(w->last_stream));
  HIP_TRY(ctx, hipDeviceSynchronize());
  if (b.p) HIP_TRY(ctx, hipFree(b.p));
  b.p = nullptr;
  b.cap = 0;
  const size_t rounded = (bytes + (2u << 20) - 1) & ~size_t((2u << 20) - 1);
  hipError_t e = hipMalloc(&b.p, rounded);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, ABEA_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", rounded, hipGetErrorString(e));
  }
  b.cap = rounded;
  return ABEA_OK;
}

void free_buf(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

int work_init(abea_ctx *ctx, Work &w) {
  HIP_TRY(ctx, hipEventCreateWithFlags(&w.staging_done, hipEventDisableTiming));
  for (auto &ev : w.tev) HIP_TRY(ctx, hipEventCreate(&ev));
  return ABEA_OK;
}

void work_free(Work &w) {
  DevBuf *bufs[] = {&w.reads, &w.rstat, &w.queue, &w.xmean, &w.kparam,
                    &w.trace, &w.scratch, &w.path_len, &w.path_src};
  for (DevBuf *b : bufs) free_buf(*b);
  if (w.h_reads) (void)hipHostFree(w.h_reads);
  w.h_reads = nullptr;
  w.h_cap = 0;
  if (w.staging_done) (void)hipEventDestroy(w.staging_done);
  w.staging_done = nullptr;
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
  const int gpc =
      align_groups_per_cu(ctx->cpl, refills_per_group(ctx->W, ctx->cpl), ctx->launch.waves_per_group, edge);
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
 *  - Trace: fused kernel with P workers: read s < P gets its own region and
 *    worker s reuses it for every later read it takes; P is the requested
 *    worker count, capped by residency and by the trace budget (admission by
 *    traceback bytes).  Split kernels: every read gets its own region. */
int plan_batch(abea_ctx *ctx, Work &w, int n, const uint64_t *eo, const uint64_t *ko,
               uint64_t pair_capacity) {
  Plan &P = w.plan;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  P.n = n;
  w.order.resize(n);
  std::vector<uint64_t> comp(n);
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
  std::iota(w.order.begin(), w.order.end(), 0);
  std::stable_sort(w.order.begin(), w.order.end(), [&](int a, int b) { return comp[a] > comp[b]; });

  /* trace words of planned read s, and the worker count */
  const int G = bands_per_group(ctx->cpl);
  auto words = [&](int s) -> uint64_t { return ((comp[w.order[s]] + G - 1) / G) * 64u; };
  int workers = n;
  const bool pool = !split_kernels(ctx) && ctx->launch.workers > 0;
  P.edge = edge_clearing(ctx, pool ? std::min(n, ctx->launch.workers) : n);
  if (pool) workers = std::min(n, std::min(ctx->launch.workers, resident_workers(ctx, P.edge)));
  if (ctx->arena_bytes > 0) {
    uint64_t sum = 0;
    int fit = 0;
    while (fit < workers && (sum + words(fit)) * sizeof(uint2) <= ctx->arena_bytes) sum += words(fit++);
    if (fit < workers) {
      if (split_kernels(ctx) || fit == 0)
        return fail(ctx, ABEA_E_NOMEM, "trace of %s needs more than arena_bytes = %llu",
                    fit == 0 ? "the longest read" : "the batch", (unsigned long long)ctx->arena_bytes);
      workers = fit;
    }
  }
  P.workers = split_kernels(ctx) ? 0 : workers;
  P.cpl = ctx->cpl;
  P.wpg = ctx->launch.waves_per_group;

  if ((size_t)n > w.h_cap) {
    if (w.staging_pending) HIP_TRY(ctx, hipEventSynchronize(w.staging_done));
    w.staging_pending = false;
    if (w.h_reads) (void)hipHostFree(w.h_reads);
    w.h_reads = nullptr;
    w.h_cap = 0;
    const size_t cap = std::max<size_t>(n, 1024);
    HIP_TRY(ctx, hipHostMalloc((void **)&w.h_reads, cap * sizeof(ReadDesc), hipHostMallocDefault));
    w.h_cap = cap;
  }
  /* the previous call's upload must have left the staging buffer */
  if (w.staging_pending) HIP_TRY(ctx, hipEventSynchronize(w.staging_done));
  w.staging_pending = false;

  uint64_t tr = 0, pr = 0;
  for (int s = 0; s < n; ++s) {
    const int r = w.order[s];
    ReadDesc &d = w.h_reads[s];
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
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
    pr += comp[r];
  }
  P.n_trace = tr;
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



int ensure_work(abea_ctx *ctx, Work &w) {
  const Plan &P = w.plan;
  const size_t n = (size_t)std::max(P.n, 1);
  int rc;
  if ((rc = ensure(ctx, &w, w.reads, sizeof(ReadDesc) * n))) return rc;
  if ((rc = ensure(ctx, &w, w.rstat, sizeof(int32_t) * n))) return rc;
  if ((rc = ensure(ctx, &w, w.queue, sizeof(uint32_t)))) return rc;
  if ((rc = ensure(ctx, &w, w.xmean, sizeof(float) * (size_t)P.n_events))) return rc;
  if ((rc = ensure(ctx, &w, w.kparam, sizeof(KParam) * (size_t)P.n_kmers))) return rc;
  if ((rc = ensure(ctx, &w, w.trace, sizeof(uint2) * (size_t)P.n_trace))) return rc;
  if ((rc = ensure(ctx, &w, w.scratch, sizeof(int2) * (size_t)P.n_scratch))) return rc;
  if ((rc = ensure(ctx, &w, w.path_len, sizeof(uint64_t) * n))) return rc;
  if ((rc = ensure(ctx, &w, w.path_src, sizeof(uint64_t) * n))) return rc;
  return ABEA_OK;
}

/* Enqueue the kernels of a planned batch whose plan is on the device. */
int enqueue_kernels(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st, bool timed) {
  const Plan &P = w.plan;
  const int n = P.n;
  const ReadDesc *reads = (const ReadDesc *)w.reads.p;
  int32_t *rstat = (int32_t *)w.rstat.p;
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[0], st));
  HIP_TRY(ctx, launch_prep(reads, n, io.events, io.ranks, io.in_addr, io.scale, io.shift,
                           (const ModelEntry *)ctx->model.p, ctx->n_model,
                           (ctx->flags & ABEA_F_SCALE_EVENTS) != 0, (float *)w.xmean.p,
                           (KParam *)w.kparam.p, rstat, (uint32_t *)w.queue.p, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[1], st));

  AlignArgs a;
  a.reads = reads;
  a.xmean = (const float *)w.xmean.p;
  a.kparam = (const KParam *)w.kparam.p;
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
  /* the band or fused kernel's own start and end: with other batches in
   * flight its dispatch may wait for free CUs, which these do not count */
  hipEvent_t k0 = timed ? w.tev[2] : nullptr, k1 = timed ? w.tev[3] : nullptr;
  const bool launched = n > 0 && (P.workers == 0 || (P.workers > 0 && P.workers <= n));
  if (P.workers == 0) {
    HIP_TRY(ctx, launch_band(a, P.cpl, refills_per_group(ctx->W, P.cpl), P.edge, st, k0, k1));
  } else {
    HIP_TRY(ctx, launch_align(a, P.cpl, refills_per_group(ctx->W, P.cpl), P.wpg, P.edge, st, k0, k1));
  }
  if (timed && !launched) { /* nothing dispatched: an empty interval */
    HIP_TRY(ctx, hipEventRecord(w.tev[2], st));
    HIP_TRY(ctx, hipEventRecord(w.tev[3], st));
  }
  if (P.workers == 0) HIP_TRY(ctx, launch_backtrack(a, P.cpl, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[4], st));

  HIP_TRY(ctx, launch_scan((const uint64_t *)w.path_len.p, n, io.pair_offset, st));
  HIP_TRY(ctx, launch_compact((const int2 *)w.scratch.p, (const uint64_t *)w.path_src.p,
                              io.pair_offset, n, io.pairs, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(w.tev[5], st));
  w.timed = timed;
  return ABEA_OK;
}

/* Upload the plan and enqueue the batch on `st`. */
int run_planned(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st) {
  int rc;
  if ((rc = ensure_work(ctx, w))) return rc;
  w.last_stream = st;
  HIP_TRY(ctx, hipMemcpyAsync(w.reads.p, w.h_reads, sizeof(ReadDesc) * w.plan.n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(w.staging_done, st));
  w.staging_pending = true;
  return enqueue_kernels(ctx, w, io, st, (ctx->flags & ABEA_F_TIMING) != 0);
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
  if (!model->level_mean || !model->level_stdv) return ABEA_E_INVAL;
  const uint32_t n_model = 1u << (2 * model->k);
  std::vector<ModelEntry> me(n_model);
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
  abea_ctx *ctx = new (std::nothrow) abea_ctx();
  if (!ctx) return ABEA_E_NOMEM;
  ctx->device = cfg->device;
  ctx->W = cfg->bandwidth;
  ctx->cpl = cells_per_lane(ctx->W);
  ctx->flags = cfg->flags;
  ctx->k = model->k;
  ctx->n_model = n_model;
  ctx->arena_bytes = cfg->arena_bytes;
  int rc = ABEA_OK;
  do {
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "hipSetDevice: %s", hipGetErrorString(e)); break; }
    e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, cfg->device);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "device attribute: %s", hipGetErrorString(e)); break; }
    if ((rc = ensure(ctx, nullptr, ctx->model, sizeof(ModelEntry) * n_model))) break;
    e = hipMemcpy(ctx->model.p, me.data(), sizeof(ModelEntry) * n_model, hipMemcpyHostToDevice);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "model upload: %s", hipGetErrorString(e)); break; }
    e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "stream: %s", hipGetErrorString(e)); break; }
    if ((rc = work_init(ctx, ctx->main))) break;
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
  (void)hipDeviceSynchronize();
  work_free(ctx->main);
  DevBuf *bufs[] = {&ctx->model, &ctx->events, &ctx->ranks, &ctx->scale, &ctx->shift,
                    &ctx->pairs, &ctx->pair_offset, &ctx->ll, &ctx->status, &ctx->cells};
  for (DevBuf *b : bufs) free_buf(*b);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  delete ctx;
}

int abea_cells_per_lane(int32_t bandwidth) {
  if (bandwidth < 2 || bandwidth > ABEA_MAX_BANDWIDTH) return 0;
  return cells_per_lane(bandwidth);
}

int abea_set_launch(abea_ctx *ctx, const abea_launch_t *l) {
  if (!ctx) return ABEA_E_INVAL;
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
  /* buffers of an earlier call may still be in use by queued kernels */
  if (ctx->main.last_stream) HIP_TRY(ctx, hipStreamSynchronize(ctx->main.last_stream));
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
  info->reserved = 0;
  info->trace_bytes = P.n_trace * sizeof(uint2);
  info->scratch_bytes = P.n_scratch * sizeof(int2);
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
  if ((rc = ensure(ctx, w, ctx->events, sizeof(abea_event_t) * (size_t)P.n_events))) return rc;
  if ((rc = ensure(ctx, w, ctx->ranks, sizeof(uint32_t) * (size_t)P.n_kmers))) return rc;
  if ((rc = ensure(ctx, w, ctx->scale, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, w, ctx->shift, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, w, ctx->pairs, sizeof(abea_pair_t) * (size_t)P.pairs_needed))) return rc;
  if ((rc = ensure(ctx, w, ctx->pair_offset, sizeof(uint64_t) * (size_t)(n + 1)))) return rc;
  if ((rc = ensure(ctx, w, ctx->ll, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, w, ctx->status, sizeof(int32_t) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, w, ctx->cells, sizeof(uint64_t) * (size_t)n))) return rc;
  if (P.n_events)
    HIP_TRY(ctx, hipMemcpyAsync(ctx->events.p, b->events, sizeof(abea_event_t) * P.n_events,
                                hipMemcpyHostToDevice, st));
  if (P.n_kmers)
    HIP_TRY(ctx, hipMemcpyAsync(ctx->ranks.p, b->kmer_rank, sizeof(uint32_t) * P.n_kmers,
                                hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->scale.p, b->scale, sizeof(float) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->shift.p, b->shift, sizeof(float) * n, hipMemcpyHostToDevice, st));
  DevIO io;
  io.events = (const float *)ctx->events.p;
  io.ranks = (const uint32_t *)ctx->ranks.p;
  io.scale = (const float *)ctx->scale.p;
  io.shift = (const float *)ctx->shift.p;
  io.pairs = (int2 *)ctx->pairs.p;
  io.pair_offset = (uint64_t *)ctx->pair_offset.p;
  io.ll = (float *)ctx->ll.p;
  io.status = (int32_t *)ctx->status.p;
  io.cells = (uint64_t *)ctx->cells.p;
  if ((rc = run_planned(ctx, ctx->main, io, st))) return rc;
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
  if (total)
    HIP_TRY(ctx, hipMemcpy(r->pairs, io.pairs, sizeof(abea_pair_t) * total, hipMemcpyDeviceToHost));
  return ABEA_OK;
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
    if ((rc = plan_batch(ctx, w, n, b->event_offset, b->kmer_offset, r->pair_capacity))) break;
    if ((rc = ensure_work(ctx, w))) break;
    /* the plan goes to the device once; replays do not copy */
    if (n > 0) {
      e = hipMemcpy(w.reads.p, w.h_reads, sizeof(ReadDesc) * n, hipMemcpyHostToDevice);
      if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "plan upload: %s", hipGetErrorString(e)); break; }
    }
    e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "stream: %s", hipGetErrorString(e)); break; }
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
  g->work.last_stream = (hipStream_t)stream;
  HIP_TRY(ctx, hipGraphLaunch(g->exec, (hipStream_t)stream));
  return ABEA_OK;
}

int abea_graph_info(const abea_graph *g, abea_plan_info_t *info) {
  if (!g || !info) return ABEA_E_INVAL;
  const Plan &P = g->work.plan;
  info->n_reads = P.n;
  info->workers = P.workers;
  info->cells_per_lane = P.cpl;
  info->waves_per_group = P.wpg;
  info->band_clear = P.edge ? ABEA_CLEAR_EDGES : ABEA_CLEAR_WINDOW;
  info->reserved = 0;
  info->trace_bytes = P.n_trace * sizeof(uint2);
  info->scratch_bytes = P.n_scratch * sizeof(int2);
  return ABEA_OK;
}

void abea_graph_destroy(abea_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  work_free(g->work);
  delete g;
}

}  // extern "C"
