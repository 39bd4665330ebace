/*
 * abea_detect_host.cpp -- host side of event detection (include/abea.h,
 * abea_detect_events*): argument checks, the tile plan of a raw batch, the
 * context's detection buffers and the launches of abea_detect.hip.
 *
 * A read of n samples has ceil(n / ED_TILE) tiles of ED_TILE boundaries;
 * the plan is each read's first tile (a prefix sum over the host sample
 * offsets).  The plan and the offsets stay in mapped pinned host memory that
 * the two kernels needing them read directly: the call issues no copy-engine
 * command, which, queued behind this stream's earlier work, would hold back
 * every other stream's copies.  Buffers grow in stream order like the
 * alignment's (abea_rt::ensure).
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"
#include "abea_runtime.h"

using namespace abea;

namespace abea_rt {

struct DetectWork {
  Work w; /* its events order buffer growth and the plan's staging */
  DevBuf tiles, flags, count, first_cp, base, bsum;
  /* the host entry point's device copies */
  DevBuf raw, offset, pa_scale, events, event_offset;
  char *h_plan = nullptr; /* mapped pinned: sample offsets, then first tiles */
  char *d_plan = nullptr; /* h_plan as the device addresses it */
  size_t h_cap = 0;
  std::vector<void *> retired_host;
  /* ABEA_F_TIMING: k_ed_detect's dispatch, k_ed_events's, the whole batch */
  hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
};

void detect_free(abea_ctx *ctx, hipStream_t st) {
  DetectWork *d = ctx->detect;
  if (!d) return;
  (void)work_wait(ctx, d->w);
  DevBuf *bufs[] = {&d->tiles, &d->flags, &d->count,    &d->first_cp, &d->base,
                    &d->bsum,  &d->raw,   &d->offset,   &d->pa_scale, &d->events, &d->event_offset};
  for (DevBuf *b : bufs) free_buf(*b, st);
  if (d->w.staging_pending && d->w.staging_done) (void)hipEventSynchronize(d->w.staging_done);
  d->w.staging_pending = false;
  if (d->h_plan) (void)hipHostFree(d->h_plan);
  for (void *h : d->retired_host) (void)hipHostFree(h);
  for (hipEvent_t &e : d->tev)
    if (e) (void)hipEventDestroy(e);
  work_free(d->w, st);
  delete d;
  ctx->detect = nullptr;
}

}  // namespace abea_rt

namespace {

using namespace abea_rt;

const abea_detect_params_t kDefaultParams = ABEA_DETECT_DEFAULT_PARAMS;

int detect_check(abea_ctx *ctx, const abea_raw_batch_t *raw, const abea_detect_params_t *p,
                 const void *events, uint64_t cap, const uint64_t *event_offset) {
  if (!ctx) return ABEA_E_INVAL;
  if (!raw || !event_offset) return fail(ctx, ABEA_E_INVAL, "null raw batch or event_offset");
  const int n = raw->n_reads;
  if (n < 0) return fail(ctx, ABEA_E_INVAL, "n_reads < 0");
  if (!raw->sample_offset) return fail(ctx, ABEA_E_INVAL, "null sample_offset");
  const uint64_t *so = raw->sample_offset;
  if (so[0] != 0) return fail(ctx, ABEA_E_INVAL, "sample offsets must start at 0");
  for (int r = 0; r < n; ++r) {
    if (so[r + 1] < so[r]) return fail(ctx, ABEA_E_INVAL, "sample offsets decrease at read %d", r);
    if (so[r + 1] - so[r] >= (1ull << 31)) return fail(ctx, ABEA_E_INVAL, "read %d has 2^31 samples or more", r);
  }
  if (n > 0 && (!raw->offset || !raw->pa_scale)) return fail(ctx, ABEA_E_INVAL, "null per-read array");
  if (so[n] > 0 && !raw->samples) return fail(ctx, ABEA_E_INVAL, "null samples");
  if (cap > 0 && !events) return fail(ctx, ABEA_E_INVAL, "null events");
  if (p->window_short < 2 || p->window_long < p->window_short || p->window_long > ABEA_DETECT_MAX_WINDOW)
    return fail(ctx, ABEA_E_INVAL, "windows %d, %d out of range", p->window_short, p->window_long);
  if (!std::isfinite(p->threshold_short) || !std::isfinite(p->threshold_long) || p->threshold_short < 0.f ||
      p->threshold_long < 0.f)
    return fail(ctx, ABEA_E_INVAL, "thresholds must be finite and >= 0");
  return ABEA_OK;
}

int detect_work(abea_ctx *ctx, DetectWork **out) {
  if (!ctx->detect) {
    DetectWork *d = new (std::nothrow) DetectWork();
    if (!d) return fail(ctx, ABEA_E_NOMEM, "detection state");
    int rc = work_init(ctx, d->w);
    for (hipEvent_t &e : d->tev)
      if (rc == ABEA_OK && hipEventCreate(&e) != hipSuccess) rc = fail(ctx, ABEA_E_HIP, "hipEventCreate failed");
    if (rc) {
      for (hipEvent_t &e : d->tev)
        if (e) (void)hipEventDestroy(e);
      work_free(d->w);
      delete d;
      return rc;
    }
    ctx->detect = d;
  }
  *out = ctx->detect;
  return ABEA_OK;
}

/* Plan and enqueue a checked batch whose samples and per-read arrays are on
 * the device. */
int detect_enqueue(abea_ctx *ctx, DetectWork *D, const abea_raw_batch_t *raw, const abea_detect_params_t &p,
                   const int16_t *samples, const float *offset, const float *pa_scale, float *events, uint64_t cap,
                   uint64_t *event_offset, hipStream_t st) {
  const int n = raw->n_reads;
  const uint64_t *so = raw->sample_offset;
  const size_t need = (size_t)(n + 1) * (sizeof(uint64_t) + sizeof(uint32_t));
  if (need > D->h_cap) {
    /* a larger pinned plan buffer; the old one may still feed a queued
     * upload and is freed with the detection state */
    const size_t cap_b = std::max<size_t>({need, 2 * D->h_cap, 4096});
    char *h = nullptr;
    void *dv = nullptr;
    HIP_TRY(ctx, hipHostMalloc((void **)&h, cap_b, hipHostMallocMapped | hipHostMallocCoherent));
    if (hipHostGetDevicePointer(&dv, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      return fail(ctx, ABEA_E_HIP, "hipHostGetDevicePointer failed");
    }
    if (D->h_plan) D->retired_host.push_back(D->h_plan);
    D->h_plan = h;
    D->d_plan = (char *)dv;
    D->h_cap = cap_b;
    D->w.staging_pending = false;
  }
  if (D->w.staging_pending) HIP_TRY(ctx, hipEventSynchronize(D->w.staging_done));
  D->w.staging_pending = false;
  uint64_t *h_so = (uint64_t *)D->h_plan;
  uint32_t *h_tf = (uint32_t *)(h_so + n + 1);
  uint64_t tiles = 0;
  for (int r = 0; r <= n; ++r) {
    h_so[r] = so[r];
    h_tf[r] = (uint32_t)tiles;
    if (r < n) tiles += (so[r + 1] - so[r] + ED_TILE - 1) / ED_TILE;
    if (tiles > 0xffffffffull) return fail(ctx, ABEA_E_INVAL, "batch of %llu tiles is too large",
                                           (unsigned long long)tiles);
  }
  const uint32_t n_tiles = (uint32_t)tiles;
  const uint32_t nb = ed_scan_blocks(n_tiles);
  Work *w = &D->w;
  int rc;
  if ((rc = ensure(ctx, w, D->tiles, sizeof(EdTile) * (size_t)n_tiles, st))) return rc;
  if ((rc = ensure(ctx, w, D->flags, sizeof(uint64_t) * (size_t)n_tiles * (ED_TILE / 64), st))) return rc;
  if ((rc = ensure(ctx, w, D->count, sizeof(uint32_t) * (size_t)n_tiles, st))) return rc;
  if ((rc = ensure(ctx, w, D->first_cp, sizeof(int32_t) * (size_t)n_tiles, st))) return rc;
  if ((rc = ensure(ctx, w, D->base, sizeof(uint64_t) * (size_t)n_tiles, st))) return rc;
  if ((rc = ensure(ctx, w, D->bsum, sizeof(uint64_t) * (size_t)(nb + 1), st))) return rc;

  DetectArgs a;
  a.raw = samples;
  a.sample_offset = (const uint64_t *)D->d_plan;
  a.tile_first = (const uint32_t *)(D->d_plan + sizeof(uint64_t) * (size_t)(n + 1));
  a.tiles = (EdTile *)D->tiles.p;
  a.offset = offset;
  a.pa_scale = pa_scale;
  a.n_reads = n;
  a.n_tiles = n_tiles;
  a.w_short = p.window_short;
  a.w_long = p.window_long;
  a.thr_short = (float)((double)p.threshold_short * (double)p.threshold_short);
  a.thr_long = (float)((double)p.threshold_long * (double)p.threshold_long);
  a.flags = (uint64_t *)D->flags.p;
  a.count = (uint32_t *)D->count.p;
  a.first_cp = (int32_t *)D->first_cp.p;
  a.base = (uint64_t *)D->base.p;
  a.block_sum = (uint64_t *)D->bsum.p;
  a.events = events;
  a.capacity = cap;
  a.event_offset = event_offset;
  D->timed = (ctx->flags & ABEA_F_TIMING) != 0;
  HIP_TRY(ctx, launch_detect(a, st, D->timed ? D->tev : nullptr));
  /* the plan is read until the last kernel; the host may rewrite it after */
  HIP_TRY(ctx, hipEventRecord(D->w.staging_done, st));
  D->w.staging_pending = true;
  return work_mark(ctx, D->w, st);
}

}  // namespace

extern "C" {

int abea_detect_events_device(abea_ctx *ctx, const abea_raw_batch_t *raw, const abea_detect_params_t *params,
                              abea_event_t *events, uint64_t event_capacity, uint64_t *event_offset,
                              void *stream) {
  const abea_detect_params_t &p = params ? *params : kDefaultParams;
  int rc = detect_check(ctx, raw, &p, events, event_capacity, event_offset);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  DetectWork *D;
  if ((rc = detect_work(ctx, &D))) return rc;
  return detect_enqueue(ctx, D, raw, p, raw->samples, raw->offset, raw->pa_scale, (float *)events, event_capacity,
                        event_offset, (hipStream_t)stream);
}

int abea_detect_events(abea_ctx *ctx, const abea_raw_batch_t *raw, const abea_detect_params_t *params,
                       abea_event_t *events, uint64_t event_capacity, uint64_t *event_offset) {
  const abea_detect_params_t &p = params ? *params : kDefaultParams;
  int rc = detect_check(ctx, raw, &p, events, event_capacity, event_offset);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  DetectWork *D;
  if ((rc = detect_work(ctx, &D))) return rc;
  const int n = raw->n_reads;
  const uint64_t n_samples = raw->sample_offset[n];
  /* a read has at most as many events as samples */
  const uint64_t dcap = std::min<uint64_t>(event_capacity, n_samples);
  hipStream_t st = ctx->own_stream;
  Work *w = &D->w;
  if ((rc = stage_init(ctx))) return rc;
  if ((rc = ensure(ctx, w, D->raw, sizeof(int16_t) * (size_t)n_samples, st))) return rc;
  if ((rc = ensure(ctx, w, D->offset, sizeof(float) * (size_t)std::max(n, 1), st))) return rc;
  if ((rc = ensure(ctx, w, D->pa_scale, sizeof(float) * (size_t)std::max(n, 1), st))) return rc;
  if ((rc = ensure(ctx, w, D->events, sizeof(abea_event_t) * (size_t)dcap, st))) return rc;
  if ((rc = ensure(ctx, w, D->event_offset, sizeof(uint64_t) * (size_t)(n + 1), st))) return rc;
  if ((rc = stage_copy_up(ctx, D->raw.p, raw->samples, sizeof(int16_t) * (size_t)n_samples))) return rc;
  if ((rc = stage_copy_up(ctx, D->offset.p, raw->offset, sizeof(float) * (size_t)n))) return rc;
  if ((rc = stage_copy_up(ctx, D->pa_scale.p, raw->pa_scale, sizeof(float) * (size_t)n))) return rc;
  if ((rc = detect_enqueue(ctx, D, raw, p, (const int16_t *)D->raw.p, (const float *)D->offset.p,
                           (const float *)D->pa_scale.p, (float *)D->events.p, dcap, (uint64_t *)D->event_offset.p,
                           st)))
    return rc;
  HIP_TRY(ctx, hipMemcpyAsync(event_offset, D->event_offset.p, sizeof(uint64_t) * (size_t)(n + 1),
                              hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const uint64_t total = event_offset[n];
  if (total > event_capacity)
    return fail(ctx, ABEA_E_CAPACITY, "event_capacity %llu < %llu events", (unsigned long long)event_capacity,
                (unsigned long long)total);
  return stage_copy_down(ctx, events, D->events.p, sizeof(abea_event_t) * (size_t)total);
}

int abea_get_detect_timings(abea_ctx *ctx, float *out, int n) {
  if (!ctx || !out || n < 0) return ABEA_E_INVAL;
  DetectWork *D = ctx->detect;
  if (!(ctx->flags & ABEA_F_TIMING) || !D || !D->timed)
    return fail(ctx, ABEA_E_INVAL, "no timed detection call (ABEA_F_TIMING)");
  HIP_TRY(ctx, hipEventSynchronize(D->tev[5]));
  float t[3] = {0.f, 0.f, 0.f};
  HIP_TRY(ctx, hipEventElapsedTime(&t[0], D->tev[0], D->tev[1]));
  HIP_TRY(ctx, hipEventElapsedTime(&t[1], D->tev[2], D->tev[3]));
  HIP_TRY(ctx, hipEventElapsedTime(&t[2], D->tev[4], D->tev[5]));
  for (int i = 0; i < n && i < 3; ++i) out[i] = t[i];
  return ABEA_OK;
}

}  // extern "C"
