/*
 * abea_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain CPU reference of Adaptive Banded Event Alignment (ABEA), written from
 * the thesis, Ch. 5 "GPU Accelerated Adaptive Banded Event Alignment":
 *   - Alg. 5.1 "Adaptive Banded Event Alignment" (band loop, initialisation of
 *     the first two bands, band moves, limits in a band, backtrack),
 *   - Alg. 5.2 "... cell score computation" (transition constants, the three
 *     moves and the arg-max),
 *   - Alg. 5.3 "... log probability computation" (Gaussian log-emission), with
 *     the per-read scaling paragraph that follows it: the model scaled to the
 *     events (mu*scale + shift), or, as an option, the events scaled to the
 *     model ((x - shift)/scale).
 * Where the text is silent or garbled the readings used are listed in the
 * design notes of the repository (band-move direction, initial lower-left,
 * tie-breaks, epsilon = 1e-10, inclusive band limits, global alignment).
 *
 * Everything is FP32 except the per-read and per-model constants, which are
 * computed in double and rounded once.  Build with -ffp-contract=off: the only
 * fused operation is the explicit fmaf() of the model scaling.
 *
 * No blocking, fusion or reordering: one band after the other, one cell after
 * the other, exactly as the algorithm states.
 */
#include "abea_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NEG_INF (-INFINITY)

enum { T_NONE = 0, T_D = 1, T_U = 2, T_L = 3 };

void oracle_transitions(int64_t n_events, int64_t n_kmers, float out[3]) {
  /* Alg. 5.2 constants.  The printed epsilon "1^{-10}" reads as 1e-10. */
  double events_per_kmer = (double)n_events / (double)n_kmers;
  double epsilon = 1e-10;
  double lp_skip = log(epsilon);
  double lp_stay = log(1.0 - 1.0 / (events_per_kmer + 1.0));
  double lp_step = log(1.0 - exp(lp_skip) - exp(lp_stay));
  out[0] = (float)lp_skip;
  out[1] = (float)lp_stay;
  out[2] = (float)lp_step;
}

void oracle_model_terms(int64_t n, const float *level_stdv, float *c, float *h) {
  /* Alg. 5.3: ln(1/sqrt(2 pi)) - ln(sigma) - 0.5 z^2.  The first two terms
   * depend only on the model entry; 0.5 z^2 = (x - mu)^2 * (0.5 / sigma^2). */
  const double pi = 3.14159265358979323846;
  for (int64_t r = 0; r < n; ++r) {
    double sigma = (double)level_stdv[r];
    c[r] = (float)(log(1.0 / sqrt(2.0 * pi)) - log(sigma));
    h[r] = (float)(0.5 / (sigma * sigma));
  }
}

float oracle_emission(float x, float mu, float sigma, float c, float h, uint32_t flags) {
  if (flags & ORACLE_FORM_LITERAL) {
    float z = (x - mu) / sigma;
    return c - 0.5f * (z * z);
  }
  float d = x - mu;
  float t = d * d;
  float u = t * h;
  return c - u;
}

void oracle_band_limits(int64_t E, int64_t K, int64_t n_e, int64_t n_k, int32_t W,
                        int64_t *min_j, int64_t *max_j) {
  /* Offset j of a band with lower-left (E, K) is the cell (E - j, K + j).
   * Keep 0 <= j < W, 0 <= E - j < n_e and 0 <= K + j < n_k. */
  int64_t lo = 0, hi = W - 1;
  if (E - (n_e - 1) > lo) lo = E - (n_e - 1);
  if (-K > lo) lo = -K;
  if (E < hi) hi = E;
  if ((n_k - 1) - K < hi) hi = (n_k - 1) - K;
  *min_j = lo;
  *max_j = hi;
}

/* Score of offset jj of a band, -inf outside [0, W). */
static float band_get(const float *S, int64_t band, int64_t jj, int32_t W) {
  if (jj < 0 || jj >= W) return NEG_INF;
  return S[band * W + jj];
}

/* The trim cell of band i: (i-1, -1), the event i-1 left unaligned after
 * the trim cell above it (band i-1; the origin for i = 1), if the band
 * holds k-mer -1 and the event exists. */
static void trim_cell(float *S, uint8_t *T, const int64_t *E, const int64_t *K, int64_t i, int64_t n_e,
                      int32_t W, float lp_trim) {
  const int64_t e = i - 1;
  const int64_t j = -1 - K[i];
  if (e < 0 || e > n_e - 1 || j < 0 || j >= W) return;
  S[i * W + j] = band_get(S, i - 1, -1 - K[i - 1], W) + lp_trim;
  T[i * W + j] = T_U;
}

int oracle_align(const float *event_mean, int64_t event_stride, int64_t n_e,
                 const uint32_t *rank, int64_t n_k,
                 const float *level_mean, const float *level_stdv,
                 const float *c, const float *h, int64_t n_model,
                 float scale, float shift, int32_t W, uint32_t flags,
                 int32_t *pairs, float *score, oracle_stats_t *stats,
                 uint8_t *trace_out, int64_t *ll_out) {
  oracle_stats_t st;
  memset(&st, 0, sizeof st);
  st.min_margin = INFINITY;
  st.min_move_margin = INFINITY;
  *score = NEG_INF;
  if (W < 2 || n_e < 0 || n_k < 0) return ORACLE_E_INVAL;
  if (n_e == 0 || n_k == 0) {
    if (stats) *stats = st;
    return ORACLE_READ_EMPTY;
  }
  for (int64_t k = 0; k < n_k; ++k)
    if ((int64_t)rank[k] >= n_model) {
      if (stats) *stats = st;
      return ORACLE_READ_BAD_RANK;
    }

  float lp[3];
  oracle_transitions(n_e, n_k, lp);
  const float lp_skip = lp[0], lp_stay = lp[1], lp_step = lp[2];
  /* trim: one event left unaligned, probability 1/100, in double then float */
  const int trim = (flags & ORACLE_TRIM) != 0;
  const float lp_trim = (float)log(1.0 / 100.0);

  /* Per-read scaling (paragraph after Alg. 5.3), sigma never scaled:
   * by default the model level of every k-mer of the read is scaled,
   * mu = level_mean*scale + shift with one rounding, and the events are used
   * as they are; with ORACLE_SCALE_EVENTS every event is scaled to the model,
   * x' = (x - shift)/scale, and the model levels are used as they are. */
  float *mu = (float *)malloc(sizeof(float) * (size_t)n_k);
  float *xs = (float *)malloc(sizeof(float) * (size_t)n_e);
  if (!mu || !xs) {
    free(mu); free(xs);
    return ORACLE_E_NOMEM;
  }
  const int scale_events = (flags & ORACLE_SCALE_EVENTS) != 0;
  for (int64_t k = 0; k < n_k; ++k)
    mu[k] = scale_events ? level_mean[rank[k]] : fmaf(level_mean[rank[k]], scale, shift);
  for (int64_t e = 0; e < n_e; ++e) {
    const float x = event_mean[e * event_stride];
    if (scale_events) {
      const float d = x - shift;
      xs[e] = d / scale;
    } else {
      xs[e] = x;
    }
  }

  const int64_t last = n_e + n_k; /* bands 0..last; the last holds (n_e-1, n_k-1) */
  const int64_t nb = last + 1;
  float *S = (float *)malloc(sizeof(float) * (size_t)(nb * W));
  uint8_t *T = (uint8_t *)malloc((size_t)(nb * W));
  int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
  if (!S || !T || !E || !K) {
    free(mu); free(xs); free(S); free(T); free(E); free(K);
    return ORACLE_E_NOMEM;
  }
  st.n_bands = nb;

  /* initialise_first_two_bands: both bands -inf with no trace; band 0 has its
   * lower-left at (W/2 - 1, -1 - W/2) so that the virtual origin (-1, -1) is
   * at its centre offset W/2 with score 0; band 1 is band 0 moved one k-mer. */
  const int32_t half = W / 2;
  for (int32_t j = 0; j < W; ++j) {
    S[0 * W + j] = NEG_INF; T[0 * W + j] = T_NONE;
    S[1 * W + j] = NEG_INF; T[1 * W + j] = T_NONE;
  }
  E[0] = half - 1;
  K[0] = -1 - half;
  E[1] = E[0];
  K[1] = K[0] + 1;
  S[0 * W + half] = 0.0f;
  /* with trim, band 1 holds the first trim cell (0, -1), up of the origin */
  if (trim) trim_cell(S, T, E, K, 1, n_e, W, lp_trim);

  for (int64_t i = 2; i <= last; ++i) {
    /* Suzuki-Kasahara rule on the previous band: move towards the better of
     * its two end cells (offset 0 = largest event / smallest k-mer, offset
     * W-1 = smallest event / largest k-mer); alternate when both are -inf. */
    float lo = S[(i - 1) * W + 0];
    float hi = S[(i - 1) * W + (W - 1)];
    int kmer_move;
    if (lo == NEG_INF && hi == NEG_INF) {
      kmer_move = (int)(i % 2 == 1);
    } else {
      kmer_move = (flags & ORACLE_PLANT_SK_REVERSED) ? (hi < lo) : (lo < hi);
      double mm = fabs((double)lo - (double)hi);
      if (mm < st.min_move_margin) st.min_move_margin = mm;
    }
    if (kmer_move) {
      E[i] = E[i - 1];
      K[i] = K[i - 1] + 1;
      st.kmer_moves++;
    } else {
      E[i] = E[i - 1] + 1;
      K[i] = K[i - 1];
    }

    int64_t min_j, max_j;
    oracle_band_limits(E[i], K[i], n_e, n_k, W, &min_j, &max_j);
    for (int32_t j = 0; j < W; ++j) {
      S[i * W + j] = NEG_INF;
      T[i * W + j] = T_NONE;
    }
    if (max_j >= min_j) st.cells += max_j - min_j + 1;

    for (int64_t j = min_j; j <= max_j; ++j) {
      const int64_t e = E[i] - j;
      const int64_t k = K[i] + j;
      /* neighbours: up (e-1, k), left (e, k-1) in band i-1; diag (e-1, k-1)
       * in band i-2.  The first k-mer has no left neighbour: (e, -1) is
       * outside the table, or with trim a trim cell, which is entered from
       * only by a diagonal step */
      const float up = band_get(S, i - 1, k - K[i - 1], W);
      const float left = (k == 0 && !(flags & ORACLE_PLANT_TRIM_SKIP_IN)) ? NEG_INF
                                                                         : band_get(S, i - 1, k - 1 - K[i - 1], W);
      const float diag = band_get(S, i - 2, k - 1 - K[i - 2], W);
      const int64_t e_em = (flags & ORACLE_PLANT_EVENT_OFF_BY_ONE) ? (e > 0 ? e - 1 : 0) : e;
      const uint32_t r = rank[k];
      const float em = oracle_emission(xs[e_em], mu[k], level_stdv[r], c[r], h[r], flags);
      const float score_d = (diag + lp_step) + em;
      const float score_u = (flags & ORACLE_PLANT_DROP_UP_EMISSION) ? (up + lp_stay)
                                                                    : (up + lp_stay) + em;
      const float score_l = left + lp_skip;
      /* max of the three, first maximum in the order D, U, L */
      float s = score_d;
      uint8_t d = T_D;
      if (score_u > s) { s = score_u; d = T_U; }
      if (score_l > s) { s = score_l; d = T_L; }
      S[i * W + j] = s;
      T[i * W + j] = d;
    }
    if (trim) trim_cell(S, T, E, K, i, n_e, W, lp_trim);
    /* a band wholly inside the table: are its end cells, which place the
     * next band, finite? (both -inf is the case the move rule alternates) */
    if (K[i] >= 0 && K[i] + W - 1 <= n_k - 1 && E[i] <= n_e - 1 && E[i] - (W - 1) >= 0) {
      st.in_table_bands++;
      if (S[i * W] == NEG_INF || S[i * W + W - 1] == NEG_INF) st.in_table_inf_ends++;
    }
  }

  int status = ORACLE_READ_OK;
  /* the end of the path: (n_e-1, n_k-1), or with trim the last k-mer's cell
   * that is best with the remaining events trimmed */
  int64_t e_end = n_e - 1;
  float end_score = NEG_INF;
  {
    const int64_t jt = E[last] - (n_e - 1);
    if (jt >= 0 && jt < W) end_score = S[last * W + jt];
  }
  if (trim) {
    float best = NEG_INF;
    int64_t u = -1;
    for (int64_t e = 0; e < n_e; ++e) {
      const int64_t i = e + n_k + 1; /* the band of (e, n_k-1) */
      const float s_end = band_get(S, i, E[i] - e, W);
      const float t = (flags & ORACLE_PLANT_TRIM_NO_TAIL) ? NEG_INF : best + lp_trim;
      if (t != NEG_INF && s_end != NEG_INF) {
        const double mm = fabs((double)t - (double)s_end);
        if (mm < st.min_margin) st.min_margin = mm;
      }
      if (t > s_end) {
        best = t;
      } else {
        best = s_end;
        u = e;
      }
    }
    end_score = best;
    e_end = u;
  }
  if (end_score == NEG_INF) {
    status = ORACLE_READ_BAND_LOST;
  } else {
    *score = end_score;
    /* backtrack from the end cell to the origin (with trim: to the trim
     * column), emitting every cell */
    int64_t e = e_end, k = n_k - 1, n = 0;
    while (e >= 0 && k >= 0) {
      pairs[2 * n + 0] = (int32_t)e;
      pairs[2 * n + 1] = (int32_t)k;
      n++;
      const int64_t i = e + k + 2;
      const int64_t j = E[i] - e;
      const uint8_t d = T[i * W + j];
      {
        /* decision margin of this path cell */
        const float up = band_get(S, i - 1, k - K[i - 1], W);
        const float left = (k == 0 && !(flags & ORACLE_PLANT_TRIM_SKIP_IN)) ? NEG_INF
                                                                           : band_get(S, i - 1, k - 1 - K[i - 1], W);
        const float diag = band_get(S, i - 2, k - 1 - K[i - 2], W);
        const uint32_t r = rank[k];
        const float em = oracle_emission(xs[e], mu[k], level_stdv[r], c[r], h[r],
                                         flags & ORACLE_FORM_LITERAL);
        double cand[3] = {(double)((diag + lp_step) + em), (double)((up + lp_stay) + em),
                          (double)(left + lp_skip)};
        double best = cand[d - 1], second = -INFINITY;
        for (int q = 0; q < 3; ++q)
          if (q != d - 1 && cand[q] > second) second = cand[q];
        double mg = (second == -INFINITY) ? INFINITY : best - second;
        if (mg < st.min_margin) st.min_margin = mg;
      }
      if (d == T_D) { e--; k--; }
      else if (d == T_U) { e--; }
      else if (d == T_L) { k--; }
      else { status = ORACLE_READ_BAND_LOST; n = 0; break; }
    }
    /* the walk ends at the origin; with trim at the trim column, having
     * left e+1 leading events unaligned */
    const int ended = trim ? (k == -1 && e >= -1) : (e == -1 && k == -1);
    if (status == ORACLE_READ_OK && !ended) {
      status = ORACLE_READ_BAND_LOST;
      n = 0;
    }
    if (status == ORACLE_READ_OK) {
      for (int64_t a = 0, b = n - 1; a < b; ++a, --b) {
        int32_t t0 = pairs[2 * a], t1 = pairs[2 * a + 1];
        pairs[2 * a] = pairs[2 * b];
        pairs[2 * a + 1] = pairs[2 * b + 1];
        pairs[2 * b] = t0;
        pairs[2 * b + 1] = t1;
      }
      st.path_len = n;
    } else {
      *score = NEG_INF;
    }
  }
  if (st.min_move_margin < st.min_margin) st.min_margin = st.min_move_margin;

  if (trace_out) memcpy(trace_out, T, (size_t)(nb * W));
  if (ll_out)
    for (int64_t i = 0; i < nb; ++i) {
      ll_out[2 * i] = E[i];
      ll_out[2 * i + 1] = K[i];
    }
  if (stats) *stats = st;
  free(mu); free(xs); free(S); free(T); free(E); free(K);
  return status;
}

/* ---- batch driver for the CPU baseline: a thread pool over reads ---- */

typedef struct {
  int32_t n_reads;
  const float *events;
  int64_t stride;
  const uint64_t *eo, *ko;
  const uint32_t *rank;
  const float *scale, *shift, *lm, *ls, *c, *h;
  int64_t n_model;
  int32_t W;
  uint32_t flags;
  const uint64_t *pair_slot;
  int32_t *pairs;
  int64_t *path_len;
  float *score;
  int32_t *status;
  int64_t *cells;
  double *min_margin;
  const int32_t *order;
  int32_t next;
  int32_t error;
} batch_job_t;

static void *batch_worker(void *arg) {
  batch_job_t *J = (batch_job_t *)arg;
  for (;;) {
    int32_t t = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (t >= J->n_reads) break;
    int32_t r = J->order[t];
    int64_t ne = (int64_t)(J->eo[r + 1] - J->eo[r]);
    int64_t nk = (int64_t)(J->ko[r + 1] - J->ko[r]);
    oracle_stats_t st;
    float sc;
    int s = oracle_align(J->events + J->eo[r] * J->stride, J->stride, ne,
                         J->rank + J->ko[r], nk, J->lm, J->ls, J->c, J->h, J->n_model,
                         J->scale[r], J->shift[r], J->W, J->flags,
                         J->pairs + 2 * J->pair_slot[r], &sc, &st, NULL, NULL);
    if (s < 0) {
      __atomic_store_n(&J->error, s, __ATOMIC_RELAXED);
      s = ORACLE_READ_BAND_LOST;
    }
    J->status[r] = s;
    J->score[r] = sc;
    J->path_len[r] = st.path_len;
    J->cells[r] = st.cells;
    if (J->min_margin) J->min_margin[r] = st.min_margin;
  }
  return NULL;
}

static const uint64_t *g_sort_len;
static int cmp_len_desc(const void *a, const void *b) {
  uint64_t la = g_sort_len[*(const int32_t *)a], lb = g_sort_len[*(const int32_t *)b];
  if (la != lb) return la > lb ? -1 : 1;
  return *(const int32_t *)a - *(const int32_t *)b;
}

int oracle_align_batch(int32_t n_reads, const float *events, int64_t event_stride,
                       const uint64_t *event_offset, const uint32_t *rank,
                       const uint64_t *kmer_offset, const float *scale, const float *shift,
                       const float *level_mean, const float *level_stdv,
                       const float *c, const float *h, int64_t n_model,
                       int32_t W, uint32_t flags, int32_t n_threads,
                       const uint64_t *pair_slot, int32_t *pairs,
                       int64_t *path_len, float *score, int32_t *status, int64_t *cells,
                       double *min_margin) {
  if (n_reads < 0 || n_threads < 1 || W < 2) return ORACLE_E_INVAL;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_reads + 1));
  uint64_t *len = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_reads + 1));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!order || !len || !th) {
    free(order); free(len); free(th);
    return ORACLE_E_NOMEM;
  }
  for (int32_t r = 0; r < n_reads; ++r) {
    order[r] = r;
    len[r] = (event_offset[r + 1] - event_offset[r]) + (kmer_offset[r + 1] - kmer_offset[r]);
  }
  g_sort_len = len;
  qsort(order, (size_t)n_reads, sizeof(int32_t), cmp_len_desc);
  batch_job_t J = {n_reads, events, event_stride, event_offset, kmer_offset, rank,
                   scale, shift, level_mean, level_stdv, c, h, n_model, W, flags,
                   pair_slot, pairs, path_len, score, status, cells, min_margin, order, 0, 0};
  int32_t started = 0;
  for (int32_t t = 0; t < n_threads; ++t) {
    if (pthread_create(&th[t], NULL, batch_worker, &J) != 0) break;
    started++;
  }
  if (started == 0) batch_worker(&J);
  for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(order); free(len); free(th);
  return J.error;
}
