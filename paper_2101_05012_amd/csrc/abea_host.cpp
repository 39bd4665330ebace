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

using namespace abea;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

struct Plan {
  int n = 0;
  std::vector<int> order;
  uint64_t n_trace = 0;   /* uint2 words */
  uint64_t n_scratch = 0; /* pair slots */
  uint64_t n_events = 0;
  uint64_t n_kmers = 0;
  uint64_t pairs_needed = 0;
};

}  // namespace

struct abea_ctx {
  int device = 0;
  int W = 100;
  int cpl = 2;
  uint32_t flags = 0;
  uint32_t k = 6;
  uint32_t n_model = 0;
  DevBuf model;
  hipStream_t own_stream = nullptr;
  hipStream_t last_stream = nullptr;
  /* planned-batch state */
  DevBuf reads, rstat, xmean, kparam, trace, scratch, path_len, path_src;
  /* host-API copies of inputs and outputs */
  DevBuf events, ranks, scale, shift, pairs, pair_offset, ll, status, cells;
  /* pinned staging of the plan */
  ReadDesc *h_reads = nullptr;
  int32_t *h_rstat = nullptr;
  size_t h_cap = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  hipEvent_t tev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  Plan plan;
  std::string err;
};

namespace {

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

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((ctx), e_ == hipErrorOutOfMemory ? ABEA_E_NOMEM : ABEA_E_HIP, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                            \
  } while (0)

int ensure(abea_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (bytes <= b.cap) return ABEA_OK;
  /* kernels queued by earlier calls may still use the old buffer */
  if (ctx->last_stream) HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
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

/* Plan a batch from host offsets: sort reads longest first (so the longest
 * band chains start first), give each read its trace, move-bit and pair
 * scratch regions, and compute its constants. */
int plan_batch(abea_ctx *ctx, int n, const uint64_t *eo, const uint64_t *ko, uint64_t pair_capacity) {
  Plan &P = ctx->plan;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  P.n = n;
  P.order.resize(n);
  std::vector<uint64_t> len(n);
  uint64_t need = 0;
  for (int r = 0; r < n; ++r) {
    if (eo[r + 1] < eo[r] || ko[r + 1] < ko[r])
      return fail(ctx, ABEA_E_INVAL, "offsets decrease at read %d", r);
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    if (ne > 0x3fffffffull || nk > 0x3fffffffull)
      return fail(ctx, ABEA_E_INVAL, "read %d is too long", r);
    len[r] = ne + nk;
    if (ne > 0 && nk > 0) need += ne + nk - 1;
  }
  P.pairs_needed = need;
  if (pair_capacity < need)
    return fail(ctx, ABEA_E_CAPACITY, "pair_capacity %llu < %llu", (unsigned long long)pair_capacity,
                (unsigned long long)need);
  std::iota(P.order.begin(), P.order.end(), 0);
  std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) { return len[a] > len[b]; });

  if ((size_t)n > ctx->h_cap) {
    if (ctx->staging_pending) HIP_TRY(ctx, hipEventSynchronize(ctx->staging_done));
    ctx->staging_pending = false;
    if (ctx->h_reads) (void)hipHostFree(ctx->h_reads);
    if (ctx->h_rstat) (void)hipHostFree(ctx->h_rstat);
    ctx->h_reads = nullptr;
    ctx->h_rstat = nullptr;
    ctx->h_cap = 0;
    const size_t cap = std::max<size_t>(n, 1024);
    HIP_TRY(ctx, hipHostMalloc((void **)&ctx->h_reads, cap * sizeof(ReadDesc), hipHostMallocDefault));
    HIP_TRY(ctx, hipHostMalloc((void **)&ctx->h_rstat, cap * sizeof(int32_t), hipHostMallocDefault));
    ctx->h_cap = cap;
  }
  /* the previous call's upload must have left the staging buffers */
  if (ctx->staging_pending) HIP_TRY(ctx, hipEventSynchronize(ctx->staging_done));
  ctx->staging_pending = false;

  const int G = bands_per_group(ctx->cpl);
  uint64_t tr = 0, pr = 0;
  for (int s = 0; s < n; ++s) {
    const int r = P.order[s];
    ReadDesc &d = ctx->h_reads[s];
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    d.ev_off = eo[r];
    d.km_off = ko[r];
    d.n_e = (int32_t)ne;
    d.n_k = (int32_t)nk;
    d.orig = r;
    d.tr_off = tr;
    d.spare = 0;
    d.pr_off = pr;
    d.lp_skip = d.lp_stay = d.lp_step = 0.f;
    if (ne == 0 || nk == 0) {
      ctx->h_rstat[s] = READ_EMPTY;
      continue;
    }
    ctx->h_rstat[s] = READ_OK;
    transitions((int64_t)ne, (int64_t)nk, &d.lp_skip, &d.lp_stay, &d.lp_step);
    const uint64_t computed = ne + nk - 1; /* bands 2 .. n_e+n_k */
    tr += ((computed + G - 1) / G) * 64u; /* 64 lanes x uint2 per group of G bands */
    pr += computed;
  }
  P.n_trace = tr;
  P.n_scratch = pr;
  P.n_events = eo[n];
  P.n_kmers = ko[n];
  return ABEA_OK;
}

struct DevIO {
  const float *events;
  const uint32_t *ranks;
  const float *scale;
  const float *shift;
  int2 *pairs;
  uint64_t *pair_offset;
  float *ll;
  int32_t *status;
  uint64_t *cells;
};

/* Enqueue the planned batch on `st`. */
int run_planned(abea_ctx *ctx, const DevIO &io, hipStream_t st) {
  const Plan &P = ctx->plan;
  const int n = P.n;
  int rc;
  if ((rc = ensure(ctx, ctx->reads, sizeof(ReadDesc) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->rstat, sizeof(int32_t) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->xmean, sizeof(float) * (size_t)P.n_events))) return rc;
  if ((rc = ensure(ctx, ctx->kparam, sizeof(KParam) * (size_t)P.n_kmers))) return rc;
  if ((rc = ensure(ctx, ctx->trace, sizeof(uint2) * (size_t)P.n_trace))) return rc;
  if ((rc = ensure(ctx, ctx->scratch, sizeof(int2) * (size_t)P.n_scratch))) return rc;
  if ((rc = ensure(ctx, ctx->path_len, sizeof(uint64_t) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->path_src, sizeof(uint64_t) * (size_t)n))) return rc;
  ctx->last_stream = st;

  HIP_TRY(ctx, hipMemcpyAsync(ctx->reads.p, ctx->h_reads, sizeof(ReadDesc) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->rstat.p, ctx->h_rstat, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(ctx->staging_done, st));
  ctx->staging_pending = true;

  const ReadDesc *reads = (const ReadDesc *)ctx->reads.p;
  int32_t *rstat = (int32_t *)ctx->rstat.p;
  const bool timed = (ctx->flags & ABEA_F_TIMING) != 0;
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[0], st));
  HIP_TRY(ctx, launch_prep(reads, n, io.events, io.ranks, io.scale, io.shift,
                           (const ModelEntry *)ctx->model.p, ctx->n_model, (float *)ctx->xmean.p,
                           (KParam *)ctx->kparam.p, rstat, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[1], st));

  BandArgs ba;
  ba.reads = reads;
  ba.xmean = (const float *)ctx->xmean.p;
  ba.kparam = (const KParam *)ctx->kparam.p;
  ba.rstat = rstat;
  ba.trace = (uint2 *)ctx->trace.p;
  ba.out_ll = io.ll;
  ba.out_cells = io.cells;
  ba.W = ctx->W;
  HIP_TRY(ctx, launch_band(ba, n, ctx->cpl, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[2], st));

  BacktrackArgs bt;
  bt.reads = reads;
  bt.rstat = rstat;
  bt.trace = (const uint2 *)ctx->trace.p;
  bt.scratch = (int2 *)ctx->scratch.p;
  bt.path_len = (uint64_t *)ctx->path_len.p;
  bt.path_src = (uint64_t *)ctx->path_src.p;
  bt.out_status = io.status;
  bt.out_ll = io.ll;
  HIP_TRY(ctx, launch_backtrack(bt, n, ctx->cpl, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[3], st));

  HIP_TRY(ctx, launch_scan((const uint64_t *)ctx->path_len.p, n, io.pair_offset, st));
  HIP_TRY(ctx, launch_compact((const int2 *)ctx->scratch.p, (const uint64_t *)ctx->path_src.p,
                              io.pair_offset, n, io.pairs, st));
  if (timed) HIP_TRY(ctx, hipEventRecord(ctx->tev[4], st));
  ctx->timed = timed;
  return ABEA_OK;
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

}  // namespace

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
  int rc = ABEA_OK;
  do {
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "hipSetDevice: %s", hipGetErrorString(e)); break; }
    if ((rc = ensure(ctx, ctx->model, sizeof(ModelEntry) * n_model))) break;
    e = hipMemcpy(ctx->model.p, me.data(), sizeof(ModelEntry) * n_model, hipMemcpyHostToDevice);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "model upload: %s", hipGetErrorString(e)); break; }
    e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "stream: %s", hipGetErrorString(e)); break; }
    e = hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming);
    if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "event: %s", hipGetErrorString(e)); break; }
    for (auto &ev : ctx->tev) {
      e = hipEventCreate(&ev);
      if (e != hipSuccess) { rc = fail(ctx, ABEA_E_HIP, "event: %s", hipGetErrorString(e)); break; }
    }
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
  DevBuf *bufs[] = {&ctx->model, &ctx->reads, &ctx->rstat, &ctx->xmean, &ctx->kparam,
                    &ctx->trace, &ctx->scratch, &ctx->path_len, &ctx->path_src,
                    &ctx->events, &ctx->ranks, &ctx->scale, &ctx->shift, &ctx->pairs,
                    &ctx->pair_offset, &ctx->ll, &ctx->status, &ctx->cells};
  for (DevBuf *b : bufs) free_buf(*b);
  if (ctx->h_reads) (void)hipHostFree(ctx->h_reads);
  if (ctx->h_rstat) (void)hipHostFree(ctx->h_rstat);
  if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
  for (auto &ev : ctx->tev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  delete ctx;
}

int abea_align_batch_device(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *r, void *stream) {
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  if (b->n_reads > 0 && (!r->pairs && r->pair_capacity > 0)) return fail(ctx, ABEA_E_INVAL, "null pairs");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int n = b->n_reads;
  if ((rc = plan_batch(ctx, n, b->event_offset, b->kmer_offset, r->pair_capacity))) return rc;
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
  return run_planned(ctx, io, st);
}

int abea_align_batch(abea_ctx *ctx, const abea_batch_t *b, abea_result_t *r) {
  int rc = check_batch(ctx, b, r);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int n = b->n_reads;
  if ((rc = plan_batch(ctx, n, b->event_offset, b->kmer_offset, r->pair_capacity))) return rc;
  if (n == 0) {
    r->pair_offset[0] = 0;
    return ABEA_OK;
  }
  if (ctx->plan.pairs_needed > 0 && !r->pairs) return fail(ctx, ABEA_E_INVAL, "null pairs");
  const Plan &P = ctx->plan;
  hipStream_t st = ctx->own_stream;
  if ((rc = ensure(ctx, ctx->events, sizeof(abea_event_t) * (size_t)P.n_events))) return rc;
  if ((rc = ensure(ctx, ctx->ranks, sizeof(uint32_t) * (size_t)P.n_kmers))) return rc;
  if ((rc = ensure(ctx, ctx->scale, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->shift, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->pairs, sizeof(abea_pair_t) * (size_t)P.pairs_needed))) return rc;
  if ((rc = ensure(ctx, ctx->pair_offset, sizeof(uint64_t) * (size_t)(n + 1)))) return rc;
  if ((rc = ensure(ctx, ctx->ll, sizeof(float) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->status, sizeof(int32_t) * (size_t)n))) return rc;
  if ((rc = ensure(ctx, ctx->cells, sizeof(uint64_t) * (size_t)n))) return rc;
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
  if ((rc = run_planned(ctx, io, st))) return rc;
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
  if (!ctx->timed) return fail(ctx, ABEA_E_UNSUPPORTED, "context not created with ABEA_F_TIMING");
  HIP_TRY(ctx, hipEventSynchronize(ctx->tev[4]));
  for (int q = 0; q < n && q < 4; ++q) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->tev[q], ctx->tev[q + 1]));
    out[q] = ms;
  }
  return ABEA_OK;
}

}  // extern "C"
