/*
 * abea_server.cpp -- continuous-batching serving loop of libabea.so.
 *
 * Reads arrive one at a time (a simulated sequencer in the thesis's
 * on-the-fly setting, Ch. 5 §5.5 and Ch. 6); a background thread admits
 * them into micro-batches and keeps several micro-batches on the device at
 * once, each on its own stream with its own buffers ("slots").
 *   - Reads wait in length classes (factor-2 bins of n_e + n_k); a free slot
 *     takes reads of the class whose first read has waited longest, so a
 *     micro-batch is not held up by one long read and no read starves.
 *   - Admission is by traceback bytes: a read needs
 *     ceil((n_e + n_k - 1) / G) * 512 bytes of trace tiles; the reads on the
 *     device never need more than trace_budget_bytes together.
 *   - A read that arrives while others are on the device joins the next
 *     micro-batch as soon as a slot and trace memory are free; its work
 *     overlaps the running micro-batches on the device.
 *   - Band state lives in the kernel's registers and the trace stays in
 *     device memory; only inputs and results cross PCIe.
 *   - A read's result does not depend on the micro-batch it ran in (each
 *     read is aligned by its own wavefront).
 * Each result carries its arrival, admission and completion times (steady
 * clock), so the caller can report per-read latency.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/abea.h"
#include "abea_internal.h"
#include "abea_runtime.h"

using namespace abea;
using namespace abea_rt;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

/* Length classes of admission: class c holds reads with 2^c <= n_e + n_k <
 * 2^(c+1); a micro-batch takes reads of one class, so its kernel lasts about
 * as long as each of its reads. */
constexpr int N_CLASSES = 40;

int length_class(uint64_t len) {
  int c = 0;
  while (c < N_CLASSES - 1 && (len >> (c + 1)) != 0) ++c;
  return c;
}

/* Host buffers of queued reads, by size class (powers of two, at least
 * 4 KB).  Buffers are carved from one pinned arena allocated with the server
 * and recycled per class, so a queued read is copied once, into pinned
 * memory, and goes to the device by DMA from there; when the arena is used
 * up a read gets a pageable buffer, copied through the slot's pinned staging
 * at launch. */
class BufPool {
 public:
  static int cls(size_t n) {
    int c = 12;
    while (c < 47 && ((size_t)1 << c) < n) ++c;
    return c;
  }
  int init(size_t bytes) {
    size_ = bytes;
    if (bytes == 0) return ABEA_OK;
    void *p = nullptr, *d = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      size_ = 0;
      return ABEA_E_NOMEM;
    }
    arena_ = (uint8_t *)p;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipGetLastError();
      return ABEA_E_HIP;
    }
    dev_ = (uint64_t)(uintptr_t)d;
    return ABEA_OK;
  }
  /* device address of a pinned buffer from get() */
  uint64_t dev_addr(const uint8_t *p) const { return dev_ + (uint64_t)(p - arena_); }
  uint8_t *get(size_t n, int *c_out, bool *pinned) {
    const int c = cls(n);
    const size_t sz = (size_t)1 << c;
    *c_out = c;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!free_[c].empty()) {
        uint8_t *p = free_[c].back();
        free_[c].pop_back();
        *pinned = true;
        return p;
      }
      if (bump_ + sz <= size_) {
        uint8_t *p = arena_ + bump_;
        bump_ += sz;
        *pinned = true;
        return p;
      }
    }
    *pinned = false;
    return new (std::nothrow) uint8_t[sz];
  }
  void put(uint8_t *p, int c, bool pinned) {
    if (!p) return;
    if (!pinned) {
      delete[] p;
      return;
    }
    std::lock_guard<std::mutex> lk(mu_);
    free_[c].push_back(p);
  }
  ~BufPool() {
    if (arena_) (void)hipHostFree(arena_);
  }

 private:
  std::mutex mu_;
  std::vector<uint8_t *> free_[48];
  uint8_t *arena_ = nullptr;
  uint64_t dev_ = 0;
  size_t size_ = 0, bump_ = 0;
};

/* A pointer that moves (the source forgets it); returned to the pool by
 * hand. */
struct Owned {
  uint8_t *p = nullptr;
  Owned() = default;
  Owned(Owned &&o) noexcept : p(o.p) { o.p = nullptr; }
  Owned &operator=(Owned &&o) noexcept {
    p = o.p;
    o.p = nullptr;
    return *this;
  }
  Owned(const Owned &) = delete;
  Owned &operator=(const Owned &) = delete;
};

/* A queued read: its event means (the only event field the alignment
 * reads) then its k-mer ranks, in one pooled pinned buffer. */
struct SrvRead {
  uint64_t tag = 0;
  int64_t t_arrival = 0;
  int64_t t_admit = 0;
  Owned buf;
  int buf_cls = 0;
  bool pinned = false;
  uint64_t ne = 0, nk = 0;
  float scale = 1.f, shift = 0.f;
  uint64_t trace_bytes = 0;
  const float *means() const { return reinterpret_cast<const float *>(buf.p); }
  const uint32_t *ranks() const { return reinterpret_cast<const uint32_t *>(buf.p + ne * sizeof(float)); }
};

/* A finished read; its pairs wait in its slot's pinned result buffer, which
 * the slot keeps until every result of its micro-batch has been polled
 * (slot -1: a read that completed without running, with no pairs). */
struct Done {
  abea_completion_t c;
  int slot;
  uint64_t off;
};

enum SlotState { FREE = 0, RUNNING = 1, COPYING = 2, HARVESTED = 3 };

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev_meta = nullptr, ev_done = nullptr;
  Work work;
  /* mapped pinned staging of reads whose buffer is not pinned (the prep
   * kernel reads it in place), pinned staging of the small inputs and of the
   * results */
  float *h_ev = nullptr; /* event means */
  uint32_t *h_rk = nullptr;
  uint64_t dh_ev = 0, dh_rk = 0; /* their device addresses */
  uint64_t *h_addr = nullptr;    /* per read: device addresses of its events, ranks */
  float *h_sc = nullptr, *h_sh = nullptr;
  uint64_t *h_eo = nullptr, *h_ko = nullptr;
  abea_pair_t *h_pairs = nullptr;
  uint64_t *h_po = nullptr, *h_cells = nullptr;
  float *h_ll = nullptr;
  int32_t *h_st = nullptr;
  /* device inputs and results */
  DevBuf d_addr, d_sc, d_sh, d_pairs, d_po, d_ll, d_st, d_cells;
  std::vector<SrvRead> reads;
  uint64_t trace_bytes = 0;
  int state = FREE;         /* changed by the worker; HARVESTED -> FREE under the lock */
  int64_t t_launched = 0;   /* when the micro-batch was enqueued */
  uint64_t outstanding = 0; /* harvested results not yet polled (under the lock) */
};

}  // namespace

struct abea_server {
  abea_ctx *ctx = nullptr;
  abea_server_config_t cfg{};
  int G = 16;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work; /* new reads, polled results or stop */
  std::condition_variable cv_done; /* new completions */
  std::deque<SrvRead> pending[N_CLASSES]; /* arrival order within a class */
  uint64_t n_pending = 0;
  std::deque<Done> done;
  BufPool pool;
  std::thread worker;
  bool stop = false;
  int error = ABEA_OK;
  std::string err;
  /* under mu */
  uint64_t inflight_trace = 0;
  uint64_t inflight_reads = 0;
  abea_server_stats_t stats{};
};

namespace {

uint64_t trace_bytes_of(int G, uint64_t ne, uint64_t nk) {
  if (ne == 0 || nk == 0) return 0;
  const uint64_t comp = ne + nk - 1;
  return ((comp + G - 1) / G) * 64u * sizeof(uint2);
}

void release_read(abea_server *S, SrvRead &R) {
  S->pool.put(R.buf.p, R.buf_cls, R.pinned);
  R.buf.p = nullptr;
}

void release_reads(abea_server *S, std::vector<SrvRead> &reads) {
  for (SrvRead &R : reads) release_read(S, R);
}

/* Complete a queued read without running it (cancelled, timed out), under
 * the server lock: its buffer goes back to the pool, its completion has no
 * pairs. */
void complete_unrun(abea_server *S, SrvRead &R, int status, int64_t t) {
  Done d;
  d.c.tag = R.tag;
  d.c.status = status;
  d.c.log_likelihood = -__builtin_inff();
  d.c.cells = 0;
  d.c.n_pairs = 0;
  d.c.pair_offset = 0;
  d.c.t_arrival_ns = R.t_arrival;
  d.c.t_admit_ns = t;
  d.c.t_done_ns = t;
  d.slot = -1;
  d.off = 0;
  release_read(S, R);
  S->done.push_back(d);
  S->n_pending -= 1;
  S->stats.completed += 1;
  if (status == ABEA_READ_CANCELLED) S->stats.cancelled += 1;
  if (status == ABEA_READ_TIMED_OUT) S->stats.timed_out += 1;
}

/* Reads queued longer than max_queue_wait_ns complete as timed out; each
 * class's queue is checked from its front (its oldest reads). */
bool expire(abea_server *S) {
  const int64_t limit = S->cfg.max_queue_wait_ns;
  if (limit <= 0) return false;
  bool any = false;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    const int64_t t = now_ns();
    for (auto &P : S->pending)
      while (!P.empty() && t - P.front().t_arrival > limit) {
        complete_unrun(S, P.front(), ABEA_READ_TIMED_OUT, t);
        P.pop_front();
        any = true;
      }
  }
  if (any) S->cv_done.notify_all();
  return any;
}

void slot_free(abea_server *S, Slot &s) {
  if (s.st) (void)hipStreamSynchronize(s.st);
  release_reads(S, s.reads);
  work_free(s.work, s.st);
  DevBuf *bufs[] = {&s.d_addr, &s.d_sc, &s.d_sh, &s.d_pairs, &s.d_po, &s.d_ll, &s.d_st, &s.d_cells};
  for (DevBuf *b : bufs) free_buf(*b, s.st);
  if (s.st) (void)hipStreamSynchronize(s.st);
  void *hosts[] = {s.h_ev, s.h_rk, s.h_addr, s.h_sc, s.h_sh, s.h_eo, s.h_ko, s.h_pairs, s.h_po, s.h_cells,
                   s.h_ll, s.h_st};
  for (void *h : hosts)
    if (h) (void)hipHostFree(h);
  if (s.ev_meta) (void)hipEventDestroy(s.ev_meta);
  if (s.ev_done) (void)hipEventDestroy(s.ev_done);
  if (s.st) (void)hipStreamDestroy(s.st);
  s = Slot();
}

template <typename T>
int host_alloc(abea_ctx *ctx, T **p, uint64_t n, unsigned flags = hipHostMallocDefault) {
  HIP_TRY(ctx, hipHostMalloc((void **)p, sizeof(T) * std::max<uint64_t>(n, 1), flags));
  return ABEA_OK;
}

template <typename T>
int mapped_alloc(abea_ctx *ctx, T **p, uint64_t n, uint64_t *dev) {
  int rc = host_alloc(ctx, p, n, hipHostMallocMapped | hipHostMallocCoherent);
  if (rc) return rc;
  void *d = nullptr;
  HIP_TRY(ctx, hipHostGetDevicePointer(&d, (void *)*p, 0));
  *dev = (uint64_t)(uintptr_t)d;
  return ABEA_OK;
}

/* Buffers of one slot sized for the configured micro-batch capacity, so that
 * admission never allocates device memory. */
int slot_init(abea_server *S, Slot &s) {
  abea_ctx *ctx = S->ctx;
  const abea_server_config_t &c = S->cfg;
  const uint64_t nr = (uint64_t)c.max_batch_reads, ne = c.max_batch_events, nk = c.max_batch_kmers;
  const uint64_t np = ne + nk; /* pair capacity: sum of n_e + n_k - 1 */
  int rc;
  HIP_TRY(ctx, hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
  HIP_TRY(ctx, hipEventCreateWithFlags(&s.ev_meta, hipEventDisableTiming));
  HIP_TRY(ctx, hipEventCreateWithFlags(&s.ev_done, hipEventDisableTiming));
  if ((rc = work_init(ctx, s.work))) return rc;
  if ((rc = mapped_alloc(ctx, &s.h_ev, ne, &s.dh_ev))) return rc;
  if ((rc = mapped_alloc(ctx, &s.h_rk, nk, &s.dh_rk))) return rc;
  if ((rc = host_alloc(ctx, &s.h_addr, 2 * nr))) return rc;
  if ((rc = host_alloc(ctx, &s.h_sc, nr))) return rc;
  if ((rc = host_alloc(ctx, &s.h_sh, nr))) return rc;
  if ((rc = host_alloc(ctx, &s.h_eo, nr + 1))) return rc;
  if ((rc = host_alloc(ctx, &s.h_ko, nr + 1))) return rc;
  if ((rc = host_alloc(ctx, &s.h_pairs, np))) return rc;
  if ((rc = host_alloc(ctx, &s.h_po, nr + 1))) return rc;
  if ((rc = host_alloc(ctx, &s.h_cells, nr))) return rc;
  if ((rc = host_alloc(ctx, &s.h_ll, nr))) return rc;
  if ((rc = host_alloc(ctx, &s.h_st, nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_addr, sizeof(uint64_t) * 2 * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_sc, sizeof(float) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_sh, sizeof(float) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_pairs, sizeof(abea_pair_t) * np))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_po, sizeof(uint64_t) * (nr + 1)))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_ll, sizeof(float) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_st, sizeof(int32_t) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, s.d_cells, sizeof(uint64_t) * nr))) return rc;
  /* the planned batch's own buffers at their largest */
  Work &w = s.work;
  const uint64_t trace_max = ((np + S->G - 1) / S->G + nr) * 64u * sizeof(uint2);
  if ((rc = ensure(ctx, nullptr, w.reads, sizeof(ReadDesc) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, w.rstat, sizeof(int32_t) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, w.queue, sizeof(uint32_t)))) return rc;
  if ((rc = ensure(ctx, nullptr, w.xmean, sizeof(float) * ne))) return rc;
  if ((rc = ensure(ctx, nullptr, w.krank, sizeof(uint32_t) * nk))) return rc;
  if ((rc = ensure(ctx, nullptr, w.trace,
                   c.trace_budget_bytes ? std::min<uint64_t>(c.trace_budget_bytes, trace_max) : trace_max)))
    return rc;
  if ((rc = ensure(ctx, nullptr, w.scratch, sizeof(int2) * np))) return rc;
  if ((rc = ensure(ctx, nullptr, w.path_len, sizeof(uint64_t) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, w.path_src, sizeof(uint64_t) * nr))) return rc;
  if ((rc = ensure(ctx, nullptr, w.tend, sizeof(int32_t) * nr))) return rc;
  if ((rc = host_alloc(ctx, &w.h_reads, nr))) return rc;
  w.h_cap = nr;
  return ABEA_OK;
}

/* Enqueue a micro-batch on the slot's stream: the reads' pinned buffers go
 * to the device by DMA, then the kernels run, then the small per-read
 * results come back. */
int slot_launch(abea_server *S, Slot &s) {
  abea_ctx *ctx = S->ctx;
  hipStream_t st = s.st;
  const int64_t t_begin = now_ns();
  const int n = (int)s.reads.size();
  uint64_t eo = 0, ko = 0;
  s.h_eo[0] = s.h_ko[0] = 0;
  for (int r = 0; r < n; ++r) {
    const SrvRead &R = s.reads[r];
    eo += R.ne;
    ko += R.nk;
    s.h_eo[r + 1] = eo;
    s.h_ko[r + 1] = ko;
    s.h_sc[r] = R.scale;
    s.h_sh[r] = R.shift;
  }
  int rc;
  if ((rc = plan_batch(ctx, s.work, n, s.h_eo, s.h_ko, eo + ko))) return rc;
  if ((rc = ensure_work(ctx, s.work, st, true))) return rc;
  /* the prep kernel reads every read's events and ranks in place from
   * mapped pinned host memory: from the read's own buffer, or for a read
   * queued in pageable memory from the slot's mapped staging */
  for (int r = 0; r < n; ++r) {
    const SrvRead &R = s.reads[r];
    uint64_t a_ev, a_rk;
    if (R.pinned) {
      a_ev = S->pool.dev_addr(R.buf.p);
      a_rk = a_ev + R.ne * sizeof(float);
    } else {
      if (R.ne) std::memcpy(s.h_ev + s.h_eo[r], R.means(), sizeof(float) * R.ne);
      if (R.nk) std::memcpy(s.h_rk + s.h_ko[r], R.ranks(), sizeof(uint32_t) * R.nk);
      a_ev = s.dh_ev + s.h_eo[r] * sizeof(float);
      a_rk = s.dh_rk + s.h_ko[r] * sizeof(uint32_t);
    }
    s.h_addr[2 * r] = a_ev;
    s.h_addr[2 * r + 1] = a_rk;
  }
  HIP_TRY(ctx, hipMemcpyAsync(s.d_addr.p, s.h_addr, sizeof(uint64_t) * 2 * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.d_sc.p, s.h_sc, sizeof(float) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.d_sh.p, s.h_sh, sizeof(float) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.work.reads.p, s.work.h_reads, sizeof(ReadDesc) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(s.work.staging_done, st));
  s.work.staging_pending = true;
  DevIO io;
  io.events = nullptr;
  io.ranks = nullptr;
  io.in_addr = (const uint64_t *)s.d_addr.p;
  io.scale = (const float *)s.d_sc.p;
  io.shift = (const float *)s.d_sh.p;
  io.pairs = (int2 *)s.d_pairs.p;
  io.pair_offset = (uint64_t *)s.d_po.p;
  io.ll = (float *)s.d_ll.p;
  io.status = (int32_t *)s.d_st.p;
  io.cells = (uint64_t *)s.d_cells.p;
  if ((rc = enqueue_kernels(ctx, s.work, io, st, false))) return rc;
  if ((rc = work_mark(ctx, s.work, st))) return rc;
  HIP_TRY(ctx, hipMemcpyAsync(s.h_po, s.d_po.p, sizeof(uint64_t) * (n + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.h_ll, s.d_ll.p, sizeof(float) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.h_st, s.d_st.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(s.h_cells, s.d_cells.p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipEventRecord(s.ev_meta, st));
  s.state = RUNNING;
  s.t_launched = now_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.enqueue_ns += (uint64_t)(s.t_launched - t_begin);
  }
  return ABEA_OK;
}

/* Advance a slot whose work may have finished; true if anything changed. */
bool slot_poll(abea_server *S, int si, int *rc) {
  abea_ctx *ctx = S->ctx;
  Slot &s = S->slots[si];
  *rc = ABEA_OK;
  if (s.state == RUNNING) {
    hipError_t q = hipEventQuery(s.ev_meta);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) {
      *rc = fail(ctx, ABEA_E_HIP, "serving: %s", hipGetErrorString(q));
      return false;
    }
    /* the inputs are on the device: recycle their pinned buffers */
    release_reads(S, s.reads);
    const int n = (int)s.reads.size();
    const uint64_t total = s.h_po[n];
    if (total) {
      hipError_t e = hipMemcpyAsync(s.h_pairs, s.d_pairs.p, sizeof(abea_pair_t) * total, hipMemcpyDeviceToHost, s.st);
      if (e != hipSuccess) {
        *rc = fail(ctx, ABEA_E_HIP, "serving: %s", hipGetErrorString(e));
        return false;
      }
    }
    hipError_t e = hipEventRecord(s.ev_done, s.st);
    if (e != hipSuccess) {
      *rc = fail(ctx, ABEA_E_HIP, "serving: %s", hipGetErrorString(e));
      return false;
    }
    s.state = COPYING;
    return true;
  }
  if (s.state == COPYING) {
    hipError_t q = hipEventQuery(s.ev_done);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) {
      *rc = fail(ctx, ABEA_E_HIP, "serving: %s", hipGetErrorString(q));
      return false;
    }
    const int64_t t = now_ns();
    const int n = (int)s.reads.size();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stats.device_ns += (uint64_t)(t - s.t_launched);
      for (int r = 0; r < n; ++r) {
        Done d;
        const SrvRead &R = s.reads[r];
        d.c.tag = R.tag;
        d.c.status = s.h_st[r];
        d.c.log_likelihood = s.h_ll[r];
        d.c.cells = s.h_cells[r];
        d.c.n_pairs = s.h_po[r + 1] - s.h_po[r];
        d.c.pair_offset = 0;
        d.c.t_arrival_ns = R.t_arrival;
        d.c.t_admit_ns = R.t_admit;
        d.c.t_done_ns = t;
        d.slot = si;
        d.off = s.h_po[r];
        S->done.push_back(d);
      }
      s.outstanding = (uint64_t)n;
      S->inflight_trace -= s.trace_bytes;
      S->inflight_reads -= (uint64_t)n;
      S->stats.completed += (uint64_t)n;
      s.state = n ? HARVESTED : FREE;
      S->stats.harvest_ns += (uint64_t)(now_ns() - t);
    }
    S->cv_done.notify_all();
    s.reads.clear();
    s.trace_bytes = 0;
    return true;
  }
  if (s.state == HARVESTED) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (s.outstanding == 0) {
      s.state = FREE;
      return true;
    }
  }
  return false;
}

/* Take pending reads for a free slot: from the length class whose first
 * read has waited longest, in arrival order, within the slot's capacity and
 * the trace budget (a read that alone exceeds the budget was refused at
 * submission). */
bool admit(abea_server *S, Slot &s) {
  const abea_server_config_t &c = S->cfg;
  std::lock_guard<std::mutex> lk(S->mu);
  int cls = -1;
  for (int q = 0; q < N_CLASSES; ++q)
    if (!S->pending[q].empty() && (cls < 0 || S->pending[q].front().t_arrival < S->pending[cls].front().t_arrival))
      cls = q;
  if (cls < 0) return false;
  std::deque<SrvRead> &P = S->pending[cls];
  uint64_t ne = 0, nk = 0, tb = 0;
  const int64_t t = now_ns();
  while (!P.empty() && (int64_t)s.reads.size() < c.max_batch_reads) {
    SrvRead &R = P.front();
    if (ne + R.ne > c.max_batch_events || nk + R.nk > c.max_batch_kmers) break;
    if (c.trace_budget_bytes && S->inflight_trace + tb + R.trace_bytes > c.trace_budget_bytes) break;
    ne += R.ne;
    nk += R.nk;
    tb += R.trace_bytes;
    R.t_admit = t;
    s.reads.push_back(std::move(R));
    P.pop_front();
  }
  if (s.reads.empty()) return false;
  S->n_pending -= s.reads.size();
  s.trace_bytes = tb;
  S->inflight_trace += tb;
  S->inflight_reads += s.reads.size();
  S->stats.max_inflight_trace_bytes = std::max(S->stats.max_inflight_trace_bytes, S->inflight_trace);
  S->stats.max_inflight_reads = std::max(S->stats.max_inflight_reads, S->inflight_reads);
  S->stats.micro_batches += 1;
  S->stats.admitted += s.reads.size();
  return true;
}

void worker_main(abea_server *S) {
  (void)hipSetDevice(S->ctx->device);
  const int ns = (int)S->slots.size();
  for (;;) {
    bool progress = false;
    int rc = ABEA_OK;
    for (int si = 0; si < ns && !rc; ++si)
      if (slot_poll(S, si, &rc)) progress = true;
    if (!rc && expire(S)) progress = true;
    if (!rc) {
      bool stopping;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        stopping = S->stop;
      }
      for (int si = 0; si < ns && !stopping; ++si) {
        Slot &s = S->slots[si];
        if (s.state != FREE) continue;
        if (!admit(S, s)) break;
        if ((rc = slot_launch(S, s))) break;
        progress = true;
      }
    }
    std::unique_lock<std::mutex> lk(S->mu);
    if (rc) {
      S->error = rc;
      S->err = S->ctx->err;
      S->cv_done.notify_all();
      return;
    }
    /* idle: nothing on the device (results waiting to be polled may stay) */
    bool idle = true;
    for (Slot &s : S->slots) idle = idle && (s.state == FREE || s.state == HARVESTED);
    if (S->stop && idle) return;
    if (!progress) {
      if (idle && S->n_pending == 0)
        S->cv_work.wait_for(lk, std::chrono::milliseconds(10));
      else
        S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

}  // namespace

extern "C" {

int64_t abea_server_now_ns(void) { return now_ns(); }

int abea_server_create(abea_ctx *ctx, const abea_server_config_t *cfg, abea_server **out) {
  if (!ctx) return ABEA_E_INVAL;
  if (!cfg || !out) return fail(ctx, ABEA_E_INVAL, "null argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch_reads < 1 || cfg->max_batch_events < 1 ||
      cfg->max_batch_kmers < 1)
    return fail(ctx, ABEA_E_INVAL, "serving config out of range");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  abea_server *S = new (std::nothrow) abea_server();
  if (!S) return ABEA_E_NOMEM;
  S->ctx = ctx;
  S->cfg = *cfg;
  S->G = bands_per_group(ctx->cpl);
  S->slots.resize(cfg->slots);
  int rc = S->pool.init(cfg->host_staging_bytes ? cfg->host_staging_bytes : ((size_t)1 << 30));
  if (rc) rc = fail(ctx, rc, "pinned host arena of %llu bytes", (unsigned long long)cfg->host_staging_bytes);
  for (Slot &s : S->slots) {
    if (rc) break;
    rc = slot_init(S, s);
  }
  if (rc) {
    for (Slot &s : S->slots) slot_free(S, s);
    delete S;
    return rc;
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return ABEA_OK;
}

int abea_server_submit(abea_server *S, const abea_batch_t *b, const uint64_t *tags, const int64_t *arrival_ns) {
  if (!S) return ABEA_E_INVAL;
  abea_ctx *ctx = S->ctx;
  if (!b || !tags) return fail(ctx, ABEA_E_INVAL, "null batch or tags");
  if (b->n_reads < 0 || !b->event_offset || !b->kmer_offset) return fail(ctx, ABEA_E_INVAL, "bad batch");
  const int n = b->n_reads;
  if (n == 0) return ABEA_OK;
  const int64_t t_entry = now_ns();
  if (!b->scale || !b->shift) return fail(ctx, ABEA_E_INVAL, "null scale/shift");
  const uint64_t *eo = b->event_offset, *ko = b->kmer_offset;
  if (eo[0] != 0 || ko[0] != 0) return fail(ctx, ABEA_E_INVAL, "offsets must start at 0");
  if (eo[n] > 0 && !b->events) return fail(ctx, ABEA_E_INVAL, "null events");
  if (ko[n] > 0 && !b->kmer_rank) return fail(ctx, ABEA_E_INVAL, "null k-mer ranks");
  const abea_server_config_t &c = S->cfg;
  for (int r = 0; r < n; ++r) {
    if (eo[r + 1] < eo[r] || ko[r + 1] < ko[r]) return fail(ctx, ABEA_E_INVAL, "offsets decrease at read %d", r);
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    if (ne > c.max_batch_events || nk > c.max_batch_kmers || ne > 0x3fffffffull || nk > 0x3fffffffull)
      return fail(ctx, ABEA_E_CAPACITY, "read %d (%llu events, %llu k-mers) exceeds a micro-batch", r,
                  (unsigned long long)ne, (unsigned long long)nk);
    if (c.trace_budget_bytes && trace_bytes_of(S->G, ne, nk) > c.trace_budget_bytes)
      return fail(ctx, ABEA_E_CAPACITY, "read %d needs %llu trace bytes, over the budget", r,
                  (unsigned long long)trace_bytes_of(S->G, ne, nk));
  }
  const int64_t t = now_ns();
  uint64_t n_pageable = 0;
  std::vector<SrvRead> rs(n);
  for (int r = 0; r < n; ++r) {
    SrvRead &R = rs[r];
    const uint64_t ne = eo[r + 1] - eo[r], nk = ko[r + 1] - ko[r];
    R.tag = tags[r];
    R.t_arrival = arrival_ns ? arrival_ns[r] : t;
    R.ne = ne;
    R.nk = nk;
    R.buf.p = S->pool.get(ne * sizeof(float) + nk * sizeof(uint32_t), &R.buf_cls, &R.pinned);
    if (!R.buf.p) {
      release_reads(S, rs);
      return fail(ctx, ABEA_E_NOMEM, "pinned host buffer for read %d", r);
    }
    {
      /* only the event means are kept: 4 of the event's 12 bytes */
      float *dst = reinterpret_cast<float *>(R.buf.p);
      const abea_event_t *src = b->events + eo[r];
      for (uint64_t e = 0; e < ne; ++e) dst[e] = src[e].mean;
    }
    if (nk) std::memcpy(R.buf.p + ne * sizeof(float), b->kmer_rank + ko[r], sizeof(uint32_t) * nk);
    R.scale = b->scale[r];
    R.shift = b->shift[r];
    R.trace_bytes = trace_bytes_of(S->G, ne, nk);
    n_pageable += R.pinned ? 0 : 1;
  }
  const int64_t t_copied = now_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error || S->stop) {
      const int e = S->error ? S->error : ABEA_E_INVAL;
      const std::string m = S->error ? S->err : std::string("server is stopping");
      release_reads(S, rs);
      return fail(ctx, e, "%s", m.c_str());
    }
    for (SrvRead &R : rs) {
      const int q = length_class(R.ne + R.nk);
      S->pending[q].push_back(std::move(R));
    }
    S->n_pending += (uint64_t)n;
    S->stats.submitted += (uint64_t)n;
    S->stats.submit_ns += (uint64_t)(now_ns() - t_entry);
    S->stats.submit_copy_ns += (uint64_t)(t_copied - t);
    S->stats.pageable_reads += n_pageable;
  }
  S->cv_work.notify_one();
  return ABEA_OK;
}

int abea_server_cancel(abea_server *S, const uint64_t *tags, int n, int *n_cancelled) {
  if (!S) return ABEA_E_INVAL;
  if (n_cancelled) *n_cancelled = 0;
  if (n < 0 || (n > 0 && !tags)) return fail(S->ctx, ABEA_E_INVAL, "bad tags");
  if (n == 0) return ABEA_OK;
  int k = 0;
  {
    std::unordered_set<uint64_t> want;
    try {
      want.insert(tags, tags + n);
    } catch (...) {
      return fail(S->ctx, ABEA_E_NOMEM, "tag set");
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const int64_t t = now_ns();
    for (auto &P : S->pending) {
      if (P.empty()) continue;
      std::deque<SrvRead> keep;
      for (SrvRead &R : P) {
        if (want.count(R.tag)) {
          complete_unrun(S, R, ABEA_READ_CANCELLED, t);
          ++k;
        } else {
          keep.push_back(std::move(R));
        }
      }
      P.swap(keep);
    }
  }
  if (n_cancelled) *n_cancelled = k;
  if (k) S->cv_done.notify_all();
  return ABEA_OK;
}

int abea_server_poll(abea_server *S, abea_completion_t *out, int max_out, abea_pair_t *pairs, uint64_t pair_capacity,
                     int32_t timeout_us, int *n_out) {
  if (!S) return ABEA_E_INVAL;
  abea_ctx *ctx = S->ctx;
  if (!n_out || (max_out > 0 && !out)) return fail(ctx, ABEA_E_INVAL, "null output");
  *n_out = 0;
  /* take the results under the lock; copy their pairs after releasing it
   * (a slot is not reused while results of it are outstanding, so its
   * buffers stay valid), then count them off */
  std::vector<Done> taken;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_us > 0 && !S->error)
      S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                          [&] { return !S->done.empty() || S->error; });
    if (S->done.empty() && S->error) return fail(ctx, S->error, "%s", S->err.c_str());
    uint64_t used = 0;
    while ((int)taken.size() < max_out && !S->done.empty()) {
      Done &d = S->done.front();
      const uint64_t np = d.c.n_pairs;
      if (pairs && used + np > pair_capacity) {
        if (taken.empty())
          return fail(ctx, ABEA_E_CAPACITY, "next result has %llu pairs; pair capacity %llu",
                      (unsigned long long)np, (unsigned long long)pair_capacity);
        break;
      }
      d.c.pair_offset = pairs ? used : 0;
      used += pairs ? np : 0;
      taken.push_back(d);
      S->done.pop_front();
    }
  }
  const int k = (int)taken.size();
  for (int i = 0; i < k; ++i) {
    const Done &d = taken[i];
    if (pairs && d.c.n_pairs && d.slot >= 0)
      std::memcpy(pairs + d.c.pair_offset, S->slots[d.slot].h_pairs + d.off, sizeof(abea_pair_t) * d.c.n_pairs);
    out[i] = d.c;
  }
  bool freed = false; /* a slot's results are all taken: it can run again */
  if (k) {
    std::lock_guard<std::mutex> lk(S->mu);
    for (const Done &d : taken)
      if (d.slot >= 0 && --S->slots[d.slot].outstanding == 0) freed = true;
  }
  *n_out = k;
  if (freed) S->cv_work.notify_one();
  return ABEA_OK;
}

int abea_server_stats(abea_server *S, abea_server_stats_t *st) {
  if (!S || !st) return ABEA_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  *st = S->stats;
  st->pending = S->n_pending;
  st->inflight_reads = S->inflight_reads;
  st->inflight_trace_bytes = S->inflight_trace;
  st->error = S->error;
  return ABEA_OK;
}

void abea_server_destroy(abea_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto &P : S->pending) {
      for (SrvRead &R : P) release_read(S, R);
      P.clear();
    }
    S->n_pending = 0;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ctx->device);
  for (Slot &s : S->slots) slot_free(S, s);
  delete S;
}

}  // extern "C"
