/*
 * abea_runtime.h -- host runtime structures of libabea.so shared by the
 * direct API, captured graphs and the serving loop.  Not installed; not part
 * of the C ABI.
 */
#ifndef ABEA_RUNTIME_H
#define ABEA_RUNTIME_H

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"

namespace abea_rt {

using namespace abea;

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  bool pooled = false;   /* from the stream-ordered allocator (hipMallocAsync) */
  bool borrowed = false; /* a range of memory the buffer does not own (never freed) */
};

struct Plan {
  int n = 0;
  int workers = 0;        /* fused kernel: wavefronts (0 for the split kernels) */
  int cpl = 2;            /* slots per lane the plan was made for */
  int wpg = 1;            /* wavefronts per workgroup of the fused kernel */
  bool edge = false;      /* interior bands clear only the two slots beside the band */
  uint64_t n_trace = 0;   /* uint2 words */
  uint64_t n_scratch = 0; /* pair slots */
  uint64_t n_events = 0;
  uint64_t n_kmers = 0;
  uint64_t pairs_needed = 0;
  int32_t urgent_len = 0x7fffffff;
  /* split kernels under a trace budget: planned reads [parts[p], parts[p+1])
   * form part p, whose traces fit the budget together; the parts run one
   * after the other over the same trace buffer */
  std::vector<int> parts;
};

/* Device buffers and staging of one planned batch.  The context owns one for
 * its direct calls; every captured graph owns its own, so graphs can run
 * concurrently on different streams. */
struct Work {
  Plan plan;
  std::vector<int> order;
  std::vector<uint64_t> comp; /* per caller read: computed bands (n_e + n_k - 1, 0 if empty) */
  DevBuf reads, rstat, queue, xmean, krank, trace, scratch, path_len, path_src, tend;
  ReadDesc *h_reads = nullptr; /* pinned staging of the plan */
  ReadDesc *d_view = nullptr;  /* h_reads as the device addresses it (mapped), or null */
  size_t h_cap = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  /* timing (ABEA_F_TIMING): before and after k_prep; start and end of the
   * band or fused kernel, taken from its dispatch (no wait for free CUs
   * counted); after the backtrack; after the compaction */
  hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  /* the stream of the last enqueued batch, and an event recorded after it:
   * later work that must wait for it (a buffer's release, a new launch
   * form) waits for the event, never for the device */
  hipStream_t last_stream = nullptr;
  hipEvent_t done = nullptr;
  bool done_pending = false;
  /* pinned plan staging outgrown by a larger batch: freed with the Work (a
   * pinned free on the call path would wait for the whole device) */
  std::vector<void *> retired_host;
};

struct DevIO {
  const float *events;
  int ev_stride = 3; /* floats from one event mean to the next: 3 (abea_event_t) or 1 (means only) */
  const uint32_t *ranks;
  const uint64_t *in_addr = nullptr; /* per-read input addresses (see launch_prep) */
  const float *scale;
  const float *shift;
  int2 *pairs;
  uint64_t *pair_offset;
  float *ll;
  int32_t *status;
  uint64_t *cells;
};

struct DetectWork; /* event detection's state (abea_detect_host.cpp), made at its first call */
struct MethWork;   /* methylation scoring's state (abea_meth_host.cpp), made with its model */

}  // namespace abea_rt

struct abea_ctx {
  int device = 0;
  int W = 100;
  uint32_t flags = 0;
  uint32_t k = 6;
  uint32_t n_model = 0;
  uint64_t trace_budget = 0; /* trace bytes of one batch (0 = unbounded) */
  int num_cus = 0;
  bool pools = false; /* the device supports the stream-ordered allocator */
  abea_launch_t launch = {0, 1, 0, 0};
  int cpl = 2; /* slots per lane in use */
  abea_rt::DevBuf model;
  hipStream_t own_stream = nullptr;
  abea_rt::Work main;
  /* the no-allocation entry point: its own plan (host buffers sized at
   * creation for ABEA_NOALLOC_MAX_READS) and the device's fixed scratch */
  abea_rt::Work noalloc;
  void *noalloc_scratch = nullptr;
  /* host-API copies of inputs (the event means only) and outputs */
  abea_rt::DevBuf events, ranks, scale, shift, pairs, pair_offset, ll, status, cells;
  /* host-API pinned staging ring: two chunks, each with the event of the
   * copy that last used it */
  void *h_stage[2] = {nullptr, nullptr};
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  bool stage_pending[2] = {false, false};
  int stage_next = 0;
  abea_rt::DetectWork *detect = nullptr;
  abea_rt::MethWork *meth = nullptr;
  std::string err;
};

namespace abea_rt {

int fail(abea_ctx *ctx, int code, const char *fmt, ...);
#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((ctx), e_ == hipErrorOutOfMemory ? ABEA_E_NOMEM : ABEA_E_HIP, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                            \
  } while (0)

/* Grow a device buffer to at least `bytes`.  w == nullptr: a set-up buffer
 * that no queued work uses yet (plain hipMalloc).  Otherwise a buffer of w's
 * batches, grown in stream order on `st`: the old buffer is released on `st`
 * after w's last batch, the new one allocated on `st`; no other stream, and
 * not the host, waits. */
int ensure(abea_ctx *ctx, Work *w, DevBuf &b, size_t bytes, hipStream_t st = nullptr);
/* Release a buffer; a pooled one in stream order on `st`, which must be
 * ordered after every use of the buffer. */
void free_buf(DevBuf &b, hipStream_t st = nullptr);
int work_init(abea_ctx *ctx, Work &w);
/* Wait (host) for w's last enqueued batch. */
int work_wait(abea_ctx *ctx, Work &w);
/* Release w's buffers on `st` (ordered after w's last batch). */
void work_free(Work &w, hipStream_t st = nullptr);
/* Record w.done on `st` after a batch was enqueued there. */
int work_mark(abea_ctx *ctx, Work &w, hipStream_t st);
/* Plan a batch from host offsets into w (see the definition).  fused_only:
 * run the fused kernel even if the context's form is the split kernels;
 * budget: the trace budget to plan with (UINT64_MAX: the context's). */
int plan_batch(abea_ctx *ctx, Work &w, int n, const uint64_t *eo, const uint64_t *ko, uint64_t pair_capacity,
               bool fused_only = false, uint64_t budget = UINT64_MAX);
/* Device buffers of a planned batch, grown in stream order on `st`.
 * staged_events: the batch's inputs sit at per-read addresses and k_prep
 * stages the ranks and the event means (the means also for events scaled to
 * the model); otherwise the band fill reads the device batch in place and no
 * staging buffer is needed. */
int ensure_work(abea_ctx *ctx, Work &w, hipStream_t st, bool staged_events = false);
/* Kernels of a planned batch whose plan is on the device. */
int enqueue_kernels(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st, bool timed);
/* The host API's pinned staging ring (two chunks, made at the first call)
 * and copies through it on the context's own stream; the copy down returns
 * once the data is in dst. */
int stage_init(abea_ctx *ctx);
int stage_copy_up(abea_ctx *ctx, void *dst, const void *src, size_t bytes);
int stage_copy_down(abea_ctx *ctx, void *dst, const void *src, size_t bytes);
/* Release the detection state on `st` after its last work. */
void detect_free(abea_ctx *ctx, hipStream_t st);
/* Release the methylation state on `st` after its last work. */
void meth_free(abea_ctx *ctx, hipStream_t st);
/* Device model table of a pore model (Alg. 5.3 terms per entry); ABEA_E_INVAL
 * for a bad model. */
int model_entries(const abea_model_t *model, std::vector<ModelEntry> &me);
/* Alg. 5.2 transition constants of a read (double, rounded once). */
void transitions(int64_t n_events, int64_t n_kmers, float *skip, float *stay, float *step);

}  // namespace abea_rt

#endif
