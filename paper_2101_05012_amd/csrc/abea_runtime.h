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
};

/* Device buffers and staging of one planned batch.  The context owns one for
 * its direct calls; every captured graph owns its own, so graphs can run
 * concurrently on different streams. */
struct Work {
  Plan plan;
  std::vector<int> order;
  DevBuf reads, rstat, queue, xmean, kparam, trace, scratch, path_len, path_src;
  ReadDesc *h_reads = nullptr; /* pinned staging of the plan */
  size_t h_cap = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  /* timing (ABEA_F_TIMING): before and after k_prep; start and end of the
   * band or fused kernel, taken from its dispatch (no wait for free CUs
   * counted); after the backtrack; after the compaction */
  hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  hipStream_t last_stream = nullptr;
};

struct DevIO {
  const float *events;
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

}  // namespace abea_rt

struct abea_ctx {
  int device = 0;
  int W = 100;
  uint32_t flags = 0;
  uint32_t k = 6;
  uint32_t n_model = 0;
  uint64_t arena_bytes = 0; /* trace budget of one batch (0 = unbounded) */
  int num_cus = 0;
  abea_launch_t launch = {0, 1, 0, 0};
  int cpl = 2; /* slots per lane in use */
  abea_rt::DevBuf model;
  hipStream_t own_stream = nullptr;
  abea_rt::Work main;
  /* host-API copies of inputs and outputs */
  abea_rt::DevBuf events, ranks, scale, shift, pairs, pair_offset, ll, status, cells;
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

/* Grow a device buffer to at least `bytes` (waits for queued work first). */
int ensure(abea_ctx *ctx, Work *w, DevBuf &b, size_t bytes);
void free_buf(DevBuf &b);
int work_init(abea_ctx *ctx, Work &w);
void work_free(Work &w);
/* Plan a batch from host offsets into w (see the definition). */
int plan_batch(abea_ctx *ctx, Work &w, int n, const uint64_t *eo, const uint64_t *ko, uint64_t pair_capacity);
/* Device buffers of a planned batch. */
int ensure_work(abea_ctx *ctx, Work &w);
/* Kernels of a planned batch whose plan is on the device. */
int enqueue_kernels(abea_ctx *ctx, Work &w, const DevIO &io, hipStream_t st, bool timed);

}  // namespace abea_rt

#endif
