/*
 * abea.h -- C ABI of the MI355X (gfx950) Adaptive Banded Event Alignment
 * library (libabea.so).
 *
 * The operation is the alignment of nanopore signal events against the
 * k-mers of a read under a pore model, by the adaptive banded dynamic
 * programme of the thesis "Computer Architecture-Aware Optimisation of DNA
 * Analysis Systems", Ch. 5 (GPU Accelerated Adaptive Banded Event Alignment):
 *   - inputs and outputs of Alg. 5.1 (§5.2.3): the read's k-mers, the pore
 *     model and the event table {mean, stdv, duration}; the output alignment
 *     is a list of {event index, k-mer index} pairs;
 *   - cell score and log-emission of Alg. 5.2 and 5.3 (only the event mean is
 *     read); per-read model scaling mu = level_mean*scale + shift (paragraph
 *     after Alg. 5.3);
 *   - batches are serialised as concatenated arrays with exclusive prefix-sum
 *     offsets (§5.4.2.1 "Data array serialisation", Alg. 5.9).
 *
 * All functions return an int status: ABEA_OK (0) or a negative ABEA_E_*
 * code.  None throws, aborts or exits.  Per-read outcomes are reported per read
 * and do not fail the call.
 */
#ifndef ABEA_H
#define ABEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define ABEA_OK 0
#define ABEA_E_INVAL (-1)       /* bad argument: null pointer, n_reads < 0, W out of range,
                                   k out of range, offsets not starting at 0 or decreasing */
#define ABEA_E_NOMEM (-2)       /* a device or pinned-host allocation failed */
#define ABEA_E_HIP (-3)         /* the HIP runtime reported an error (see abea_last_error) */
#define ABEA_E_CAPACITY (-4)    /* result.pair_capacity is too small; nothing was written */
#define ABEA_E_UNSUPPORTED (-5) /* valid request the build cannot serve */

/* ---- per-read outcome (result.status[r]) ------------------------------ */
#define ABEA_READ_OK 0
#define ABEA_READ_EMPTY 1     /* the read has no events or no k-mers */
#define ABEA_READ_BAND_LOST 2 /* terminal cell (n_e-1, n_k-1) outside the last band, or -inf */
#define ABEA_READ_BAD_RANK 3  /* a k-mer rank >= 4^k */
#define ABEA_READ_CANCELLED 4 /* serving: cancelled while queued (abea_server_cancel) */
#define ABEA_READ_TIMED_OUT 5 /* serving: queued longer than max_queue_wait_ns */

/* Failed reads (status != ABEA_READ_OK) get zero pairs and log_likelihood = -INFINITY. */

/* ---- limits ------------------------------------------------------------ */
#define ABEA_MAX_BANDWIDTH 512 /* band width W: 2 <= W <= 512 */
#define ABEA_MAX_K 12          /* k-mer length: 1 <= k <= 12 (model has 4^k entries) */

/* ---- config flags -------------------------------------------------------- */
#define ABEA_F_TIMING 1u /* record device time of every kernel of each call (abea_get_timings) */
/* Scale the events to the model instead of the model to the events (the
 * per-read scaling paragraph after Alg. 5.3 allows either side; the thesis's
 * CLI calls it --scale-events): every event mean becomes
 * x' = (x - shift[r]) / scale[r] (float32 subtract, then correctly rounded
 * float32 divide) and the model levels are used unscaled.  Without the flag
 * the model is scaled: mu' = fmaf(level_mean, scale[r], shift[r]).  sigma is
 * unscaled in both modes.  scale[r] must be finite and non-zero. */
#define ABEA_F_SCALE_EVENTS 2u
/* Trim states (the trim paragraph after Alg. 5.3; the trim comments of the
 * core-kernel, Alg. 5.6): events at either end of a read (open pore,
 * adaptor) may stay unaligned at ln(1/100) each.  Leading trims form a column
 * at k-mer -1 inside the bands, (e, -1) = (e-1, -1) + ln(1/100) from the
 * origin, from which the first k-mer is entered by a diagonal step only; the
 * path ends at the last k-mer's cell (u, n_k-1) that is best with the
 * n_e-1-u trailing events trimmed (float32 sums in event order; ties to
 * fewer trims).  The pairs then run from (t, 0) to (u, n_k-1), t and n_e-1-u
 * the trimmed events; log_likelihood includes the trims.  Without the flag
 * the alignment is global, from (0, 0) to (n_e-1, n_k-1). */
#define ABEA_F_TRIM 4u
#define ABEA_F_ALL (ABEA_F_TIMING | ABEA_F_SCALE_EVENTS | ABEA_F_TRIM)

/* One event of the event table (Alg. 5.1 input "events[]": mean, stdv, n).
 * 12 bytes; only .mean is read (Alg. 5.3). */
typedef struct {
  float mean;
  float stdv;
  float duration;
} abea_event_t;

/* One alignment pair (Alg. 5.1 output "alignment[]"). */
typedef struct {
  int32_t event_idx;
  int32_t kmer_idx;
} abea_pair_t;

/* Pore model (Ch. 5 §5.2.1, "pore-model"): 4^k entries indexed by k-mer rank
 * (base-4 number of the k-mer, first base most significant).  level_stdv > 0.
 * Host pointers; copied by abea_create. */
typedef struct {
  uint32_t k;
  const float *level_mean;
  const float *level_stdv;
} abea_model_t;

/* arena_bytes values: ABEA_ARENA_AUTO takes a fraction of the device memory
 * free when the context is created (the thesis's GPU memory fraction, its
 * CLI's --cuda-mem-frac, 0.9 by default; §5.4.2.2 sizes its pre-allocation
 * from free memory); ABEA_ARENA_UNBOUNDED sets no budget. */
#define ABEA_ARENA_AUTO 0ull
#define ABEA_ARENA_UNBOUNDED UINT64_MAX
#define ABEA_ARENA_AUTO_FRACTION 0.9

typedef struct {
  int32_t bandwidth;    /* W, the band width (thesis: typically 100) */
  int32_t device;       /* HIP device ordinal */
  uint64_t arena_bytes; /* traceback budget of one batch in bytes (admission by traceback
                           bytes): the fused kernel runs only as many reads at once as their
                           trace fits in it, and the split kernels run the batch in parts
                           whose traces fit it; a read whose own trace exceeds it fails the
                           call with ABEA_E_NOMEM.  ABEA_ARENA_AUTO or ABEA_ARENA_UNBOUNDED,
                           or a byte count; see abea_launch_t */
  uint32_t flags;       /* ABEA_F_* */
} abea_config_t;

/*
 * A batch of reads, serialised (Alg. 5.9): read r owns
 *   events    [event_offset[r], event_offset[r+1])
 *   kmer_rank [kmer_offset[r],  kmer_offset[r+1])
 * event_offset and kmer_offset hold n_reads+1 exclusive prefix sums starting
 * at 0.  scale[r] and shift[r] scale the model means for read r.
 */
typedef struct {
  int32_t n_reads;
  const abea_event_t *events;
  const uint64_t *event_offset;
  const uint32_t *kmer_rank;
  const uint64_t *kmer_offset;
  const float *scale;
  const float *shift;
} abea_batch_t;

/*
 * Results.  Read r's pairs are pairs[pair_offset[r] .. pair_offset[r+1]) in
 * path order, from (0, 0) to (n_e-1, n_k-1) (with ABEA_F_TRIM from the first
 * untrimmed event to the last); every cell of the path is a pair
 * (a k-mer entered by a skip too).  pair_capacity must be at least
 * sum_r max(0, n_e_r + n_k_r - 1) (a path never has more cells).
 */
typedef struct {
  abea_pair_t *pairs;
  uint64_t pair_capacity;
  uint64_t *pair_offset;  /* [n_reads+1] */
  float *log_likelihood;  /* [n_reads]: score of the terminal cell */
  int32_t *status;        /* [n_reads]: ABEA_READ_* */
  uint64_t *cells;        /* [n_reads] or NULL: DP cells filled inside the table */
} abea_result_t;

typedef struct abea_ctx abea_ctx;

/*
 * Create a context on cfg->device: copies the pore model to the device and
 * precomputes its per-entry emission terms (Alg. 5.3).  *out receives the
 * context; the caller owns it and frees it with abea_destroy.
 * Errors: ABEA_E_INVAL (null pointer, W or k out of range, non-positive or
 * non-finite level_stdv), ABEA_E_NOMEM, ABEA_E_HIP.
 */
int abea_create(const abea_config_t *cfg, const abea_model_t *model, abea_ctx **out);

/*
 * Align a batch held in host memory; synchronous.  Every pointer in *batch
 * and *res is a host pointer; the call copies the inputs to the device, runs
 * the alignment and copies the results back before returning, and keeps no
 * reference to the caller's buffers.  Copies go through a pinned staging ring
 * the context owns (two chunks of ABEA_HOST_STAGING_CHUNK bytes, allocated at
 * the first call): the event means (the only event field read, Alg. 5.3) are
 * gathered into it by host threads while the previous chunk is in flight,
 * and the pairs come back through it the same way.  A context is not
 * thread-safe.
 * Errors: ABEA_E_INVAL, ABEA_E_CAPACITY (nothing written), ABEA_E_NOMEM,
 * ABEA_E_HIP.
 */
#define ABEA_HOST_STAGING_CHUNK (32ull << 20)
int abea_align_batch(abea_ctx *ctx, const abea_batch_t *batch, abea_result_t *res);

/*
 * Align a batch whose arrays are already in device memory; asynchronous.
 *   batch->event_offset, batch->kmer_offset : HOST arrays (n_reads+1); the
 *       library plans the batch from them and uploads what the kernels need;
 *   batch->events, ->kmer_rank, ->scale, ->shift : DEVICE pointers;
 *   res->pairs, ->pair_offset, ->log_likelihood, ->status, ->cells : DEVICE
 *       pointers (cells may be NULL);
 *   stream : a hipStream_t (NULL = the default stream).
 * The work is enqueued on `stream` and the call returns; results are valid
 * once the stream is synchronised.  Device buffers of the context are reused
 * by the next call on the same context, so calls on one context must be
 * ordered on one stream.
 * Errors as abea_align_batch.
 */
int abea_align_batch_device(abea_ctx *ctx, const abea_batch_t *batch,
                            const abea_result_t *res, void *stream);

/*
 * No-allocation variant of abea_align_batch_device, for callers that cannot
 * allocate memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, semantics (device
 * inputs and outputs, host offsets, asynchronous on `stream`) and results,
 * bit for bit, but the call allocates nothing:
 *   - every device buffer beyond the caller's inputs and outputs (plan,
 *     trace tiles, pair scratch, per-read lengths, and with
 *     ABEA_F_SCALE_EVENTS the scaled event means; ranks and events are read
 *     in place) lies in one fixed array of ABEA_NOALLOC_SCRATCH_BYTES that the
 *     library holds on each device it runs on until the process ends;
 *   - the plan is staged through pinned host memory that abea_create set
 *     aside for ABEA_NOALLOC_MAX_READS reads.
 * It always runs the fused kernel (band fill and backtrack by one wavefront
 * per read) with the context's worker count (0: one per read), capped by how
 * many of the longest reads' traces fit in what the other buffers leave of
 * the array (admission by traceback bytes).
 * Limits: n_reads <= ABEA_NOALLOC_MAX_READS, and 8 B per path slot (sum
 * of n_e + n_k - 1), 100 B per read (and 4 B per event with
 * ABEA_F_SCALE_EVENTS) and the
 * trace of at least the longest read (ceil((n_e + n_k - 1) / (32 /
 * cells_per_lane)) * 512 B) must fit in ABEA_NOALLOC_SCRATCH_BYTES; a batch
 * beyond them fails with ABEA_E_NOMEM and nothing is enqueued.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the kernels write whatever they read of it first, so
 * nothing needs clearing): calls that overlap on one device race, whichever
 * contexts make them; order them on one stream.  abea_get_timings and
 * abea_get_plan_info do not report these calls.
 * Errors: as abea_align_batch_device, plus ABEA_E_NOMEM beyond the limits.
 */
#define ABEA_NOALLOC_SCRATCH_BYTES (256ull << 20)
#define ABEA_NOALLOC_MAX_READS 16384
int abea_align_batch_device_noalloc(abea_ctx *ctx, const abea_batch_t *batch, const abea_result_t *res,
                                    void *stream);

/* ---- event detection ------------------------------------------------------
 * The step before the alignment: each read's raw signal (digitised current
 * samples) is cut into events {mean, stdv, n} where the signal level changes
 * suddenly (the thesis, Ch. 5 §5.2.2 "Methylation calling", its
 * event-detection paragraph; the events are the event table of Alg. 5.1).
 * The thesis gives no algorithm for the step; the detector is a two-window
 * change-point test:
 *   - statistic: at a boundary i of a read of n samples (between samples i-1
 *     and i, w <= i <= n-w) the squared two-sample t statistic of the w
 *     samples before and the w after with population variances,
 *     w D^2 / V, D = S_r - S_l, V = w (Q_l + Q_r) - S_l^2 - S_r^2 over the
 *     integer sums S and sums of squares Q, evaluated in float32 as
 *     ((float)D * (float)D) * (float)w / (float)(double)V (+inf when V = 0
 *     and D != 0, 0 when both are 0);
 *   - peaks: boundary i is a change point of a detector (w, t) if its
 *     statistic exceeds (float)(t*t), is greater than at every defined
 *     boundary up to w-1 before it and not less than at every one up to w-1
 *     after it; a short and a long detector, every peak of either starts an
 *     event;
 *   - events: the runs of samples between consecutive change points (sample
 *     0 to the first, ..., the last to n), none for a read without samples;
 *     for an event of len samples with integer sum s,
 *     m = (double)s / len, M2 = the sum in sample order of ((double)x - m)^2,
 *     mean = (float)((m + offset) * pa_scale),
 *     stdv = (float)(sqrt(M2 / len) * pa_scale), duration = (float)len (samples).
 * Results are bit-identical to the CPU reference of the same definition. */
#define ABEA_DETECT_MAX_WINDOW 16

typedef struct {
  int32_t window_short;    /* 2 <= window_short <= window_long <= ABEA_DETECT_MAX_WINDOW */
  int32_t window_long;
  float threshold_short;   /* t thresholds (finite, >= 0) */
  float threshold_long;
} abea_detect_params_t;

/* Defaults, fitted to 4 kHz sampling at 450 bases/s: about 1.7 events per
 * k-mer, the over-segmentation the thesis reports (1.5-2 events per k-mer). */
#define ABEA_DETECT_DEFAULT_PARAMS {3, 8, 1.5f, 5.0f}

/*
 * A batch of raw reads, serialised as the alignment batches (Alg. 5.9):
 * read r owns samples[sample_offset[r] .. sample_offset[r+1]) (int16 digitiser
 * levels; at most 2^31 - 1 samples per read); its current in pA is
 * (sample + offset[r]) * pa_scale[r], pa_scale[r] > 0.
 */
typedef struct {
  int32_t n_reads;
  const int16_t *samples;
  const uint64_t *sample_offset; /* HOST array [n_reads+1], exclusive prefix sums from 0 */
  const float *offset;           /* [n_reads] */
  const float *pa_scale;         /* [n_reads] */
} abea_raw_batch_t;

/*
 * Detect the events of a raw batch held in device memory; asynchronous on
 * `stream` (a hipStream_t, NULL = the default stream).
 *   raw->samples, ->offset, ->pa_scale : DEVICE pointers; raw->sample_offset
 *       a HOST array the library plans from (and uploads);
 *   events : DEVICE array of event_capacity records: the batch's events, read
 *       by read; event_offset : DEVICE array [n_reads+1] receiving each read's
 *       first event and, in event_offset[n_reads], the batch's event count.
 * A read has at most as many events as samples, so event_capacity >= the
 * batch's sample count always suffices.  With less, the events at index
 * event_capacity and beyond are not written: once the stream is
 * synchronised, event_offset[n_reads] > event_capacity tells the caller.
 * Device buffers of the context are reused by the next call, so detection
 * calls on one context must be ordered on one stream.
 * Errors: ABEA_E_INVAL (null pointer, n_reads < 0, offsets not starting at 0
 * or decreasing, a read of 2^31 samples or more, windows or thresholds out of
 * range), ABEA_E_NOMEM, ABEA_E_HIP.
 */
int abea_detect_events_device(abea_ctx *ctx, const abea_raw_batch_t *raw, const abea_detect_params_t *params,
                              abea_event_t *events, uint64_t event_capacity, uint64_t *event_offset,
                              void *stream);

/*
 * The same for a raw batch in host memory; synchronous.  Every pointer is a
 * host pointer (events: event_capacity records; event_offset: n_reads+1).
 * Errors: as abea_detect_events_device, and ABEA_E_CAPACITY (nothing written
 * to events; event_offset holds the offsets that were needed).
 */
int abea_detect_events(abea_ctx *ctx, const abea_raw_batch_t *raw, const abea_detect_params_t *params,
                       abea_event_t *events, uint64_t event_capacity, uint64_t *event_offset);

/*
 * Device time in milliseconds of the last detection call on a context created
 * with ABEA_F_TIMING: out[0] the change-point kernel (statistics and peaks),
 * out[1] the event kernel (event statistics), each from the start to the end
 * of its own dispatch, out[2] the whole batch on its stream.  Synchronises
 * with that call.  n is the length of out.
 * Errors: ABEA_E_INVAL (no timed detection call), ABEA_E_HIP.
 */
int abea_get_detect_timings(abea_ctx *ctx, float *out, int n);

/* ---- methylation scoring ---------------------------------------------------
 * The step after the alignment: the events aligned to the k-mers go through
 * HMM profiling to decide whether a base is methylated (the thesis, Ch. 5
 * §5.2.2 "Methylation calling"; the thesis gives no algorithm for the
 * profile).  The profile here:
 *   - a site is a CpG whose C starts k-mer i of a read (the first two bases of
 *     k-mer i are C, G; k >= 2); its window is the k-mers holding that C,
 *     max(0, i-k+1) .. i;
 *   - the window's events run from the first event the alignment paired with
 *     the window's first k-mer to the last it paired with k-mer i;
 *   - under the context's pore model and under a methylated model, the
 *     best-path score of those events through the window's k-mers with the
 *     alignment's own cell score (Alg. 5.2 moves with the read's transition
 *     constants, Alg. 5.3 emission, the model scaled per read, or the events
 *     with ABEA_F_SCALE_EVENTS): a virtual origin before the first cell scores
 *     0, cells outside the window -inf, the score is the window's last cell's;
 *   - LLR = score(methylated) - score(unmethylated), float32: above 0 favours
 *     a methylated C.
 * Results are bit-identical to the CPU reference of the same definition. */

/*
 * The context's methylated pore model: 4^k entries indexed by k-mer rank
 * (k the context's), level_stdv > 0, host pointers copied by the call (the
 * emission terms are prepared as for abea_create's model).  Replaces an
 * earlier one after the context's queued methylation work.
 * Errors: ABEA_E_INVAL (null, another k, a bad entry), ABEA_E_NOMEM, ABEA_E_HIP.
 */
int abea_set_methylated_model(abea_ctx *ctx, const abea_model_t *model);

/*
 * Methylation scores of an aligned batch in device memory; asynchronous on
 * `stream` (NULL = the default stream).
 *   batch : the batch as aligned (abea_align_batch_device): events, kmer_rank,
 *       scale, shift DEVICE pointers, event_offset and kmer_offset HOST arrays;
 *   res : its alignment, DEVICE pointers: pairs, pair_offset [n_reads+1],
 *       status [n_reads] (reads whose status is not ABEA_READ_OK get no score);
 *   llr : DEVICE float [total k-mers]: at each k-mer that starts a CpG the
 *       site's LLR, NaN elsewhere;
 *   n_events : DEVICE int32 [total k-mers] or NULL: the events of each site's
 *       window, 0 elsewhere.
 * The alignment must be complete on `stream` (enqueue it there first).
 * Calls on one context must be ordered on one stream.
 * Errors: ABEA_E_INVAL (null pointer, no methylated model, offsets not
 * starting at 0 or decreasing, 2^32 k-mers or more), ABEA_E_NOMEM, ABEA_E_HIP.
 */
int abea_methylation_device(abea_ctx *ctx, const abea_batch_t *batch, const abea_result_t *res, float *llr,
                            int32_t *n_events, void *stream);

/*
 * Device time in milliseconds of the last methylation call on a context
 * created with ABEA_F_TIMING: out[0] the k-mer event ranges and the site list
 * (from the start of the first kernel's dispatch to the end of the second's),
 * out[1] the per-site profile kernel (its dispatch).  Synchronises with that
 * call.
 * Errors: ABEA_E_INVAL (no timed methylation call), ABEA_E_HIP.
 */
int abea_get_meth_timings(abea_ctx *ctx, float *out, int n);

/*
 * Device time in milliseconds of each stage of the last direct call
 * (abea_align_batch or abea_align_batch_device), when the context was
 * created with ABEA_F_TIMING: out[0] k-mer parameter preparation, out[1] band
 * fill (split kernels; in several parts, from the first part's band fill to
 * the last part's) or band fill + backtrack (fused kernel), from the start
 * to the end of that kernel's dispatch (time spent waiting for free compute
 * units behind other work on the device is not counted), out[2] backtrack
 * (split kernels; 0 for the fused kernel), out[3] path-length scan and
 * compaction.  Synchronises the stream of the last call.  n is the length of
 * out.
 */
int abea_get_timings(abea_ctx *ctx, float *out, int n);

/* ---- launch form ----------------------------------------------------------
 * How the band fill (Alg. 5.1-5.3) and the backtrack are scheduled; every
 * form gives bit-identical results.  The thesis runs a pre-kernel, a
 * core-kernel with one thread block per read and a post-kernel (Ch. 5
 * §5.4.1) and pre-allocates memory for a batch with a CPU fall-back for reads
 * that do not fit (§5.4.2.2, §5.4.3); here:
 *   workers == ABEA_WORKERS_SPLIT : one wavefront per read, band fill and
 *       backtrack as two kernels (every read's trace is in memory at once,
 *       or, under a trace budget, the reads of one part at a time);
 *   workers == 0 : one fused kernel, one wavefront per read that fills the
 *       bands and then backtracks (the default; one launch per batch);
 *   workers  > 0 : the fused kernel as a persistent pool of that many
 *       wavefronts (capped by residency and by arena_bytes) that take reads,
 *       longest first, from a device work queue; trace memory is that of the
 *       `workers` longest reads only.
 * waves_per_group: wavefronts (reads) per workgroup of the fused kernel, 1, 2
 * or 4.  cells_per_lane: band slots per lane, 0 = the smallest power of two
 * with 64*c >= W + 2, else a power of two at least that and at most 16.
 * band_clear: which band slots the band fill resets to -inf after each band
 * whose cells all lie inside the DP table (every form gives the same
 * results; only the speed differs):
 *   ABEA_CLEAR_WINDOW : every slot outside the band's cells;
 *   ABEA_CLEAR_EDGES  : only the two slots beside the band (k-mers K-1 and
 *       K+W), the only ones the next two bands read; fewer vector and more
 *       scalar instructions per band, faster when the SIMDs hold several
 *       wavefronts, slower for a lone one; needs 2 or 4 cells_per_lane;
 *   ABEA_CLEAR_AUTO (0): edges at 4 cells_per_lane, and at 2 when the launch
 *       has at least two wavefronts per SIMD of the device (reads, or pool
 *       workers), else window.
 * Bands with cells outside the table always clear every slot outside them.
 * Applies to later calls and graphs; waits for the context's queued work.
 * Errors: ABEA_E_INVAL.
 */
#define ABEA_WORKERS_SPLIT (-1)
#define ABEA_CLEAR_AUTO 0
#define ABEA_CLEAR_WINDOW 1
#define ABEA_CLEAR_EDGES 2
typedef struct {
  int32_t workers;
  int32_t waves_per_group;
  int32_t cells_per_lane;
  int32_t band_clear; /* ABEA_CLEAR_* */
} abea_launch_t;
int abea_set_launch(abea_ctx *ctx, const abea_launch_t *launch);

/* The smallest cells_per_lane the band fill uses for a band width (what
 * cells_per_lane = 0 selects), or 0 if the width is out of range.  Needs no
 * device. */
int abea_cells_per_lane(int32_t bandwidth);

/* How a batch was planned: the context's last direct call, or a graph. */
typedef struct {
  int32_t n_reads;
  int32_t workers;         /* fused-kernel wavefronts (0: split kernels) */
  int32_t cells_per_lane;
  int32_t waves_per_group;
  uint64_t trace_bytes;    /* device trace memory of the batch */
  uint64_t scratch_bytes;  /* device pair scratch of the batch */
  int32_t band_clear;      /* ABEA_CLEAR_WINDOW or ABEA_CLEAR_EDGES, as resolved */
  int32_t parts;           /* split kernels: parts the batch runs in under the trace budget;
                              fused kernel: 1 */
  uint64_t trace_budget;   /* the context's trace budget in bytes (0: none) */
} abea_plan_info_t;
int abea_get_plan_info(const abea_ctx *ctx, abea_plan_info_t *info);

/* ---- captured batches (HIP graphs) ------------------------------------------
 * abea_graph_create plans a device-resident batch (pointers as in
 * abea_align_batch_device) with the context's current launch form, gives it
 * device buffers of its own, uploads the plan and captures the batch's
 * kernels into a HIP graph.  abea_graph_launch replays the graph on `stream`
 * (asynchronous; results valid once the stream is synchronised); each replay
 * recomputes every output from the batch's inputs, so the caller may change
 * the input values (not their sizes) between replays.  The batch and result
 * buffers must stay valid until abea_graph_destroy.  Replays of one graph
 * must not overlap each other; different graphs may run concurrently on
 * different streams.  The graph holds no reference to the context's own
 * buffers; the context must outlive it.
 * Errors: as abea_align_batch_device.
 */
typedef struct abea_graph abea_graph;
int abea_graph_create(abea_ctx *ctx, const abea_batch_t *batch, const abea_result_t *res,
                      abea_graph **out);
int abea_graph_launch(abea_graph *graph, void *stream);
int abea_graph_info(const abea_graph *graph, abea_plan_info_t *info);
void abea_graph_destroy(abea_graph *graph);

/* ---- serving loop (continuous batching) ------------------------------------
 * A background thread of the library admits reads, as they arrive, into
 * micro-batches and keeps up to `slots` micro-batches on the device at once,
 * each on its own stream with its own buffers (all allocated by
 * abea_server_create; admission allocates nothing).
 *   - Reads wait in length classes (factor-2 bins of n_e + n_k); a free slot
 *     takes, in arrival order, reads of the class whose first read has
 *     waited longest, so a micro-batch lasts about as long as each of its
 *     reads.
 *   - Admission is by traceback bytes: a read needs
 *     ceil((n_e + n_k - 1) / (32 / cells_per_lane)) * 512 bytes of trace tiles
 *     and the reads on the device never need more than trace_budget_bytes
 *     together (0 = no budget).  A read that arrives while others run joins
 *     the next micro-batch as soon as a slot and trace memory are free.
 *   - Each result is bit-identical to abea_align_batch on the read alone
 *     (a read is aligned by its own wavefront whatever batch it is in).
 * The server uses the context's model, band width and launch form; do not
 * call abea_set_launch or destroy the context while a server exists.
 * submit and poll may be called from different threads.
 */
typedef struct {
  int32_t slots;              /* micro-batches on the device at once, 1..16 */
  int32_t max_batch_reads;    /* reads per micro-batch */
  uint64_t max_batch_events;  /* events per micro-batch (also the largest read) */
  uint64_t max_batch_kmers;   /* k-mers per micro-batch (also the largest read) */
  uint64_t trace_budget_bytes;/* traceback bytes of all reads on the device (0 = none) */
  uint64_t host_staging_bytes;/* pinned host arena for queued reads (0 = 1 GiB); reads beyond
                                 it are queued in pageable memory and staged at launch */
  int64_t max_queue_wait_ns;  /* a read still queued this long after its arrival completes as
                                 ABEA_READ_TIMED_OUT without running (0 = no limit); checked
                                 by the background thread in queue order */
} abea_server_config_t;

/* One finished read.  Times are abea_server_now_ns() values: arrival (given
 * at submission), admission into a micro-batch (for a cancelled or timed-out
 * read: when it left the queue), and the moment its results were in host
 * memory. */
typedef struct {
  uint64_t tag;
  int32_t status;         /* ABEA_READ_* */
  float log_likelihood;
  uint64_t cells;
  uint64_t pair_offset;   /* first pair in the caller's pairs buffer */
  uint64_t n_pairs;
  int64_t t_arrival_ns;
  int64_t t_admit_ns;
  int64_t t_done_ns;
} abea_completion_t;

typedef struct {
  uint64_t submitted, admitted, completed, pending;
  uint64_t micro_batches;
  uint64_t inflight_reads, max_inflight_reads;
  uint64_t inflight_trace_bytes, max_inflight_trace_bytes;
  int32_t error;          /* sticky ABEA_E_* of the background thread, 0 if none */
  int32_t reserved;
  /* where the background thread's time goes (nanoseconds, summed over
   * micro-batches): enqueueing copies and kernels, from enqueue to results on
   * the host, and turning finished micro-batches into results */
  uint64_t enqueue_ns, device_ns, harvest_ns;
  /* time spent inside abea_server_submit, summed over calls and threads,
   * and the part of it spent taking host buffers and copying reads in */
  uint64_t submit_ns, submit_copy_ns;
  /* reads that found the pinned arena full and took a pageable buffer */
  uint64_t pageable_reads;
  /* reads that completed without running: cancelled, timed out in the queue */
  uint64_t cancelled, timed_out;
} abea_server_stats_t;

typedef struct abea_server abea_server;

/* Steady-clock time in nanoseconds (the clock of the completion times). */
int64_t abea_server_now_ns(void);

/* Create a server on ctx's device; *out receives it (free with
 * abea_server_destroy).  Errors: ABEA_E_INVAL, ABEA_E_NOMEM, ABEA_E_HIP. */
int abea_server_create(abea_ctx *ctx, const abea_server_config_t *cfg, abea_server **out);

/* Queue reads (host pointers, layout of abea_batch_t; copied before the call
 * returns).  tags[r] identifies read r in its completion; arrival_ns[r] is
 * its arrival time (NULL = now).  Errors: ABEA_E_INVAL, ABEA_E_CAPACITY (a
 * read larger than a micro-batch or than the trace budget; nothing queued),
 * or the background thread's sticky error. */
int abea_server_submit(abea_server *server, const abea_batch_t *reads, const uint64_t *tags,
                       const int64_t *arrival_ns);

/* Cancel queued reads: every read with one of the n tags that has not been
 * admitted into a micro-batch yet leaves the queue and completes, through
 * abea_server_poll, with status ABEA_READ_CANCELLED, no pairs and
 * log_likelihood -INFINITY.  Reads already admitted run to the end.
 * *n_cancelled (may be NULL) receives how many reads were cancelled.  Every
 * submitted read still completes exactly once.  Errors: ABEA_E_INVAL. */
int abea_server_cancel(abea_server *server, const uint64_t *tags, int n, int *n_cancelled);

/* Collect up to max_out finished reads, waiting up to timeout_us for the
 * first; their pairs are copied into pairs[] (capacity pair_capacity), read
 * i's at out[i].pair_offset.  pairs = NULL takes the results without their
 * pairs (out[i].n_pairs still counts them; pair_capacity is ignored).
 * *n_out receives the count (0 on timeout).  Several threads may poll.
 * Errors: ABEA_E_CAPACITY if the next result's pairs do not fit (nothing
 * taken), or the background thread's sticky error. */
int abea_server_poll(abea_server *server, abea_completion_t *out, int max_out, abea_pair_t *pairs,
                     uint64_t pair_capacity, int32_t timeout_us, int *n_out);

int abea_server_stats(abea_server *server, abea_server_stats_t *stats);

/* Stop admitting, drop queued reads, wait for the device work in flight and
 * free the server.  NULL is allowed. */
void abea_server_destroy(abea_server *server);

/* Free the context and all its device memory.  NULL is allowed. */
void abea_destroy(abea_ctx *ctx);

/* Static description of a status code. */
const char *abea_strerror(int status);

/* Message of the last error on this context ("" if none). */
const char *abea_last_error(const abea_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ABEA_H */
