/*
 * abea_meth_host.cpp -- host side of methylation scoring (include/abea.h,
 * abea_set_methylated_model and abea_methylation_device): the methylated
 * model table, the per-read plan (offsets and the Alg. 5.2 transition
 * constants, which need the host offsets) and the launches of abea_meth.hip.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"
#include "abea_runtime.h"

using namespace abea;

namespace abea_rt {

struct MethWork {
  Work w; /* its events order buffer growth and the plan's staging */
  DevBuf model, reads, kfirst, klast, sites, n_sites;
  /* pinned plan staging, read by k_meth_stage: the reads (MethRead), then
   * the pair tiles and the k-mer tiles (MethTile), in 8-byte words */
  uint64_t *h_plan = nullptr;
  uint64_t *d_view = nullptr; /* h_plan as the device addresses it */
  size_t h_cap = 0;           /* words */
  std::vector<void *> retired_host;
  /* ABEA_F_TIMING: the two kernels' dispatches */
  hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
};

void meth_free(abea_ctx *ctx, hipStream_t st) {
  MethWork *m = ctx->meth;
  if (!m) return;
  (void)work_wait(ctx, m->w);
  DevBuf *bufs[] = {&m->model, &m->reads, &m->kfirst, &m->klast, &m->sites, &m->n_sites};
  for (DevBuf *b : bufs) free_buf(*b, st);
  if (m->w.staging_pending && m->w.staging_done) (void)hipEventSynchronize(m->w.staging_done);
  m->w.staging_pending = false;
  if (m->h_plan) (void)hipHostFree(m->h_plan);
  for (void *h : m->retired_host) (void)hipHostFree(h);
  for (hipEvent_t &e : m->tev)
    if (e) (void)hipEventDestroy(e);
  work_free(m->w, st);
  delete m;
  ctx->meth = nullptr;
}

}  // namespace abea_rt

using namespace abea_rt;

extern "C" {

int abea_set_methylated_model(abea_ctx *ctx, const abea_model_t *model) {
  if (!ctx) return ABEA_E_INVAL;
  if (!model) return fail(ctx, ABEA_E_INVAL, "null methylated model");
  if (model->k != ctx->k) return fail(ctx, ABEA_E_INVAL, "methylated model has k = %u, the context %u", model->k, ctx->k);
  std::vector<ModelEntry> me;
  if (model_entries(model, me) != ABEA_OK) return fail(ctx, ABEA_E_INVAL, "bad methylated model entries");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!ctx->meth) {
    MethWork *m = new (std::nothrow) MethWork();
    if (!m) return fail(ctx, ABEA_E_NOMEM, "methylation state");
    int rc = work_init(ctx, m->w);
    for (hipEvent_t &e : m->tev)
      if (rc == ABEA_OK && hipEventCreate(&e) != hipSuccess) rc = fail(ctx, ABEA_E_HIP, "hipEventCreate failed");
    if (rc) {
      for (hipEvent_t &e : m->tev)
        if (e) (void)hipEventDestroy(e);
      work_free(m->w);
      delete m;
      return rc;
    }
    ctx->meth = m;
  }
  MethWork *m = ctx->meth;
  /* the previous table may still be read by a queued call */
  int rc = work_wait(ctx, m->w);
  if (rc) return rc;
  if ((rc = ensure(ctx, nullptr, m->model, sizeof(ModelEntry) * me.size()))) return rc;
  HIP_TRY(ctx, hipMemcpy(m->model.p, me.data(), sizeof(ModelEntry) * me.size(), hipMemcpyHostToDevice));
  return ABEA_OK;
}

int abea_methylation_device(abea_ctx *ctx, const abea_batch_t *b, const abea_result_t *res, float *llr,
                            int32_t *n_events, void *stream) {
  if (!ctx) return ABEA_E_INVAL;
  if (!b || !res) return fail(ctx, ABEA_E_INVAL, "null batch or alignment result");
  if (!ctx->meth || !ctx->meth->model.p) return fail(ctx, ABEA_E_INVAL, "no methylated model (abea_set_methylated_model)");
  const int n = b->n_reads;
  if (n < 0) return fail(ctx, ABEA_E_INVAL, "n_reads < 0");
  if (!b->event_offset || !b->kmer_offset) return fail(ctx, ABEA_E_INVAL, "null offsets");
  const uint64_t *eo = b->event_offset, *ko = b->kmer_offset;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  for (int r = 0; r < n; ++r)
    if (eo[r + 1] < eo[r] || ko[r + 1] < ko[r]) return fail(ctx, ABEA_E_INVAL, "offsets decrease at read %d", r);
  const uint64_t K = ko[n];
  if (K >= (1ull << 32)) return fail(ctx, ABEA_E_INVAL, "batch of %llu k-mers is too large", (unsigned long long)K);
  if (n > 0) {
    if (!b->scale || !b->shift || !res->pair_offset || !res->status)
      return fail(ctx, ABEA_E_INVAL, "null per-read array");
    if (eo[n] > 0 && !b->events) return fail(ctx, ABEA_E_INVAL, "null events");
    if (K > 0 && (!b->kmer_rank || !llr)) return fail(ctx, ABEA_E_INVAL, "null k-mer ranks or llr");
  }
  if (n == 0 || K == 0) return ABEA_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  MethWork *M = ctx->meth;
  hipStream_t st = (hipStream_t)stream;
  /* the tiles: ceil((n_e + n_k - 1) / METH_CHUNK) runs of a bound of each
   * read's pairs, ceil(n_k / METH_CHUNK) runs of its k-mers */
  uint64_t n_pt = 0, n_kt = 0;
  for (int r = 0; r < n; ++r) {
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    if (ne > 0 && nk > 0) n_pt += (ne + nk - 1 + METH_CHUNK - 1) / METH_CHUNK;
    n_kt += (nk + METH_CHUNK - 1) / METH_CHUNK;
  }
  if (n_pt >= (1ull << 31) || n_kt >= (1ull << 31))
    return fail(ctx, ABEA_E_INVAL, "batch too large for methylation scoring");
  const size_t rw = sizeof(MethRead) / 8, tw = sizeof(MethTile) / 8;
  const size_t words = rw * (size_t)n + tw * (size_t)(n_pt + n_kt);
  if (words > M->h_cap) {
    const size_t cap = std::max<size_t>({words, 2 * M->h_cap, 8192});
    uint64_t *h = nullptr;
    HIP_TRY(ctx, hipHostMalloc((void **)&h, cap * 8, hipHostMallocMapped | hipHostMallocCoherent));
    void *dv = nullptr;
    if (hipHostGetDevicePointer(&dv, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      return fail(ctx, ABEA_E_HIP, "hipHostGetDevicePointer failed");
    }
    if (M->h_plan) M->retired_host.push_back(M->h_plan);
    M->h_plan = h;
    M->d_view = (uint64_t *)dv;
    M->h_cap = cap;
    M->w.staging_pending = false;
  }
  if (M->w.staging_pending) HIP_TRY(ctx, hipEventSynchronize(M->w.staging_done));
  M->w.staging_pending = false;
  MethRead *h_reads = reinterpret_cast<MethRead *>(M->h_plan);
  MethTile *h_pt = reinterpret_cast<MethTile *>(M->h_plan + rw * (size_t)n);
  MethTile *h_kt = h_pt + n_pt;
  uint64_t ip = 0, ik = 0;
  for (int r = 0; r < n; ++r) {
    MethRead &d = h_reads[r];
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    d.ev_off = eo[r];
    d.km_off = ko[r];
    d.n_k = (int32_t)std::min<uint64_t>(nk, 0x7fffffff);
    d.lp_skip = d.lp_stay = d.lp_step = 0.f;
    if (ne > 0 && nk > 0) {
      transitions((int64_t)ne, (int64_t)nk, &d.lp_skip, &d.lp_stay, &d.lp_step);
      for (uint64_t c = 0; c * METH_CHUNK < ne + nk - 1; ++c) h_pt[ip++] = MethTile{(uint32_t)r, (uint32_t)c};
    }
    for (uint64_t c = 0; c * METH_CHUNK < nk; ++c) h_kt[ik++] = MethTile{(uint32_t)r, (uint32_t)c};
  }
  Work *w = &M->w;
  int rc;
  if ((rc = ensure(ctx, w, M->reads, 8 * words, st))) return rc;
  if ((rc = ensure(ctx, w, M->kfirst, sizeof(int32_t) * (size_t)K, st))) return rc;
  if ((rc = ensure(ctx, w, M->klast, sizeof(int32_t) * (size_t)K, st))) return rc;
  if ((rc = ensure(ctx, w, M->sites, sizeof(uint2) * (size_t)K, st))) return rc;
  if ((rc = ensure(ctx, w, M->n_sites, sizeof(uint32_t), st))) return rc;
  /* the plan staged and the site counter zeroed by a kernel (no copy-engine
   * command: one queued behind this stream's work would hold back every other
   * stream's copies); the host buffer is free again once it has run */
  HIP_TRY(ctx, launch_meth_stage(M->d_view, (uint64_t *)M->reads.p, words, (uint32_t *)M->n_sites.p, st));
  HIP_TRY(ctx, hipEventRecord(M->w.staging_done, st));
  M->w.staging_pending = true;

  MethArgs a;
  a.reads = (const MethRead *)M->reads.p;
  a.n_reads = n;
  a.k = (int32_t)ctx->k;
  a.n_kmers = K;
  a.pair_tiles = (const MethTile *)((const uint64_t *)M->reads.p + rw * (size_t)n);
  a.kmer_tiles = a.pair_tiles + n_pt;
  a.n_pair_tiles = (uint32_t)n_pt;
  a.n_kmer_tiles = (uint32_t)n_kt;
  a.events = (const float *)b->events;
  a.ev_stride = 3;
  a.scale_events = (ctx->flags & ABEA_F_SCALE_EVENTS) != 0;
  a.ranks = b->kmer_rank;
  a.scale = b->scale;
  a.shift = b->shift;
  a.model = (const ModelEntry *)ctx->model.p;
  a.meth_model = (const ModelEntry *)M->model.p;
  a.pairs = (const int2 *)res->pairs;
  a.pair_offset = res->pair_offset;
  a.status = res->status;
  a.kfirst = (int32_t *)M->kfirst.p;
  a.klast = (int32_t *)M->klast.p;
  a.sites = (uint2 *)M->sites.p;
  a.n_sites = (uint32_t *)M->n_sites.p;
  a.llr = llr;
  a.n_ev = n_events;
  M->timed = (ctx->flags & ABEA_F_TIMING) != 0;
  HIP_TRY(ctx, launch_meth(a, st, M->timed ? M->tev : nullptr));
  return work_mark(ctx, M->w, st);
}

int abea_get_meth_timings(abea_ctx *ctx, float *out, int n) {
  if (!ctx || !out || n < 0) return ABEA_E_INVAL;
  MethWork *M = ctx->meth;
  if (!(ctx->flags & ABEA_F_TIMING) || !M || !M->timed)
    return fail(ctx, ABEA_E_INVAL, "no timed methylation call (ABEA_F_TIMING)");
  HIP_TRY(ctx, hipEventSynchronize(M->tev[3]));
  float t[2] = {0.f, 0.f};
  HIP_TRY(ctx, hipEventElapsedTime(&t[0], M->tev[0], M->tev[1]));
  HIP_TRY(ctx, hipEventElapsedTime(&t[1], M->tev[2], M->tev[3]));
  for (int i = 0; i < n && i < 2; ++i) out[i] = t[i];
  return ABEA_OK;
}

}  // extern "C"
