/*
 * abea_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously sequential CPU implementation of Adaptive Banded
 * Event Alignment (ABEA), written from the thesis (Ch. 5 "GPU Accelerated
 * Adaptive Banded Event Alignment", §5.2.3 and Algorithms 5.1-5.3).  It exists
 * to check the HIP library.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or constant with the HIP library.
 */
#ifndef ABEA_ORACLE_H
#define ABEA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-read outcome (numerically the same as the library's, compared by name). */
enum {
  ORACLE_READ_OK = 0,
  ORACLE_READ_EMPTY = 1,     /* n_events == 0 or n_kmers == 0 */
  ORACLE_READ_BAND_LOST = 2, /* terminal cell outside the last band, or -inf */
  ORACLE_READ_BAD_RANK = 3   /* a k-mer rank >= model size */
};

/* Call-level errors. */
enum { ORACLE_E_INVAL = -1, ORACLE_E_NOMEM = -2, ORACLE_E_CAPACITY = -4 };

/* Option bits. */
enum {
  /* Paper-literal emission: z = (x - mu)/sigma (IEEE divide), em = c - 0.5*z*z.
   * Default (0) is the canonical form em = c - ((x - mu)^2 * h), h = 0.5/sigma^2. */
  ORACLE_FORM_LITERAL = 1u,
  /* PLANTED MISTAKE for tests only: reverses the band-move comparison. */
  ORACLE_PLANT_SK_REVERSED = 2u,
  /* PLANTED MISTAKE for tests only: drops the emission term from the up move. */
  ORACLE_PLANT_DROP_UP_EMISSION = 4u,
  /* PLANTED MISTAKE for tests only: uses the event index of the diagonal
   * neighbour (e-1) in the emission. */
  ORACLE_PLANT_EVENT_OFF_BY_ONE = 8u,
  /* Events scaled to the model instead of the model to the events (the
   * per-read scaling paragraph after Alg. 5.3 allows either): every event
   * mean becomes x' = (x - shift) / scale (float32 subtract, then IEEE
   * float32 divide), and the model levels are used unscaled.  sigma is not
   * scaled in either mode. */
  ORACLE_SCALE_EVENTS = 16u,
  /* Trim states (the trim paragraph after Alg. 5.3; the trim comments of the
   * core-kernel, Alg. 5.6): open-pore or adaptor events at either end of a
   * read may be left unaligned at ln(1/100) each.  A column at k-mer -1
   * holds the leading trim, (e, -1) = (e-1, -1) + lp_trim from the origin;
   * the first k-mer is entered from it by a diagonal step only; the path
   * ends at the cell (u, n_k-1) that is best with the n_e-1-u trailing
   * events trimmed, End(e) = max(S(e, n_k-1), End(e-1) + lp_trim) with ties
   * to the smaller trim; the backtrack starts there and stops at k = -1. */
  ORACLE_TRIM = 32u,
  /* PLANTED MISTAKE for tests only (with ORACLE_TRIM): no trailing trim. */
  ORACLE_PLANT_TRIM_NO_TAIL = 64u,
  /* PLANTED MISTAKE for tests only (with ORACLE_TRIM): the first k-mer may
   * also be entered from the trim column by a skip. */
  ORACLE_PLANT_TRIM_SKIP_IN = 128u
};

typedef struct {
  int64_t cells;       /* in-table cells filled over bands 2..n_e+n_k */
  int64_t n_bands;     /* n_e + n_k + 1 (bands 0..n_e+n_k) */
  int64_t kmer_moves;  /* bands placed by a k-mer step */
  int64_t path_len;    /* number of (event, k-mer) pairs */
  double min_margin;   /* smallest decision margin (band moves and path cells) */
  double min_move_margin; /* smallest band-move margin alone */
  int64_t in_table_bands;    /* bands (2..n_e+n_k) whose W cells all lie in the table */
  int64_t in_table_inf_ends; /* of those, bands with an end cell (offset 0 or W-1) at -inf */
} oracle_stats_t;

/* Transition log-probabilities of Alg. 5.2: out = {lp_skip, lp_stay, lp_step},
 * each computed in double from events_per_kmer = n_events/n_kmers and rounded
 * once to float. */
void oracle_transitions(int64_t n_events, int64_t n_kmers, float out[3]);

/* Emission terms per model entry (Alg. 5.3), computed in double and rounded
 * once: c = ln(1/sqrt(2 pi)) - ln(sigma), h = 0.5 / sigma^2. */
void oracle_model_terms(int64_t n, const float *level_stdv, float *c, float *h);

/* Gaussian log-emission of one event mean against one (scaled) model level,
 * in the form selected by `flags`. */
float oracle_emission(float x, float mu, float sigma, float c, float h, uint32_t flags);

/*
 * Align one read (Alg. 5.1).
 *   event_mean   : n_e event means, `event_stride` floats apart
 *   rank         : n_k k-mer ranks; model arrays have n_model entries
 *   c, h         : from oracle_model_terms()
 *   pairs        : out, 2*(n_e+n_k) int32 (event_idx, kmer_idx) in path order
 *   trace_out    : optional, (n_e+n_k+1)*W bytes, 0 none / 1 D / 2 U / 3 L
 *   ll_out       : optional, 2*(n_e+n_k+1) int64 lower-left (event, k-mer)
 * Returns an ORACLE_READ_* status (>= 0) or an ORACLE_E_* error (< 0).
 */
int oracle_align(const float *event_mean, int64_t event_stride, int64_t n_e,
                 const uint32_t *rank, int64_t n_k,
                 const float *level_mean, const float *level_stdv,
                 const float *c, const float *h, int64_t n_model,
                 float scale, float shift, int32_t W, uint32_t flags,
                 int32_t *pairs, float *score, oracle_stats_t *stats,
                 uint8_t *trace_out, int64_t *ll_out);

/* Band limits of a band with lower-left (E, K): inclusive [*min_j, *max_j]
 * (empty when *min_j > *max_j).  Exposed for the footnote test of Alg. 5.1. */
void oracle_band_limits(int64_t E, int64_t K, int64_t n_e, int64_t n_k, int32_t W,
                        int64_t *min_j, int64_t *max_j);

/*
 * Align a whole batch with `n_threads` POSIX threads, one read per task,
 * longest first (the CPU baseline).  Pairs of read r go to
 * pairs[2*pair_slot[r] ...]; pair_slot must give each read room for
 * n_e+n_k pairs.  Per-read outputs are indexed by read; min_margin (may be
 * NULL) receives each read's oracle_stats_t.min_margin.
 */
int oracle_align_batch(int32_t n_reads, const float *events, int64_t event_stride,
                       const uint64_t *event_offset, const uint32_t *rank,
                       const uint64_t *kmer_offset, const float *scale, const float *shift,
                       const float *level_mean, const float *level_stdv,
                       const float *c, const float *h, int64_t n_model,
                       int32_t W, uint32_t flags, int32_t n_threads,
                       const uint64_t *pair_slot, int32_t *pairs,
                       int64_t *path_len, float *score, int32_t *status, int64_t *cells,
                       double *min_margin);

#ifdef __cplusplus
}
#endif
#endif
