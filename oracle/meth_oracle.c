/*
 * meth_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain CPU reference of methylation scoring, the step after the alignment:
 * the thesis (Ch. 5 §5.2.2, "Methylation calling") sends the events aligned
 * to the reference's k-mers through HMM profiling to decide whether a base is
 * methylated, without giving the profile's algorithm.  The reading recorded
 * in the design notes of the repository:
 *
 *   sites      a CpG whose C starts k-mer i of the read (the first two bases
 *              of k-mer i are C, G); its window is the k-mers that contain
 *              that C, j0 = max(0, i-k+1) .. j1 = i;
 *   events     from the read's alignment (path-ordered pairs): e0 = the
 *              first event paired with k-mer j0, e1 = the last event paired
 *              with k-mer j1;
 *   profile    for each of two models (the pore model and a methylated one),
 *              the best-path score of events e0..e1 through the window's
 *              k-mers with the alignment's own cell score (Alg. 5.2 moves
 *              with the read's transition constants, Alg. 5.3 emission, the
 *              model scaled per read as in the alignment): a virtual origin
 *              before (e0, j0) scores 0, cells outside the window are -inf,
 *              and the score is that of (e1, j1);
 *   score      LLR = score(methylated) - score(unmethylated), in float32.
 *
 * Build with -ffp-contract=off; the cell arithmetic is oracle_emission's and
 * the cell recurrence of oracle_align's, in the same order.
 */
#include "meth_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

int oracle_meth_is_site(uint32_t rank, int32_t k) {
  if (k < 2) return 0;
  const uint32_t b0 = (rank >> (2 * (k - 1))) & 3u;
  const uint32_t b1 = (rank >> (2 * (k - 2))) & 3u;
  return b0 == 1u && b1 == 2u;
}

/* Best-path score of events x[e0..e1] through k-mers j0..j1 (mu, sigma, c, h
 * per k-mer of the window). */
float oracle_meth_profile(const float *x, int64_t n_ev, const float *mu, const float *sigma, const float *c,
                          const float *h, int64_t n_km, const float lp[3], uint32_t flags) {
  const float NI = -INFINITY;
  const float lp_skip = lp[0], lp_stay = lp[1], lp_step = lp[2];
  float *S = (float *)malloc(sizeof(float) * (size_t)(n_ev * n_km));
  if (!S) return NAN;
  for (int64_t e = 0; e < n_ev; ++e) {
    for (int64_t j = 0; j < n_km; ++j) {
      const float diag = (e == 0 && j == 0) ? 0.0f : (e > 0 && j > 0) ? S[(e - 1) * n_km + (j - 1)] : NI;
      const float up = e > 0 ? S[(e - 1) * n_km + j] : NI;
      const float left = j > 0 ? S[e * n_km + (j - 1)] : NI;
      const float em = oracle_emission(x[e], mu[j], sigma[j], c[j], h[j], flags);
      const float score_d = (diag + lp_step) + em;
      const float score_u = (up + lp_stay) + em;
      const float score_l = left + lp_skip;
      float s = score_d;
      if (score_u > s) s = score_u;
      if (score_l > s) s = score_l;
      S[e * n_km + j] = s;
    }
  }
  const float v = S[n_ev * n_km - 1];
  free(S);
  return v;
}

int oracle_meth_read(const float *event_mean, int64_t event_stride, int64_t n_e, const uint32_t *rank,
                     int64_t n_k, int32_t k, const oracle_meth_model_t *mu_model,
                     const oracle_meth_model_t *mm_model, float scale, float shift, uint32_t flags,
                     const int32_t *pairs, int64_t n_pairs, float *llr, int32_t *n_ev) {
  for (int64_t i = 0; i < n_k; ++i) {
    llr[i] = NAN;
    n_ev[i] = 0;
  }
  if (n_e == 0 || n_k == 0 || n_pairs == 0) return 0;
  /* first and last event paired with each k-mer (the pairs run in path
   * order, so a k-mer's pairs are consecutive) */
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_k);
  int64_t *lastv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_k);
  if (!first || !lastv) {
    free(first);
    free(lastv);
    return -1;
  }
  for (int64_t i = 0; i < n_k; ++i) first[i] = lastv[i] = -1;
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int64_t e = pairs[2 * p], q = pairs[2 * p + 1];
    if (q < 0 || q >= n_k) continue;
    if (first[q] < 0) first[q] = e;
    lastv[q] = e;
  }
  float lp[3];
  oracle_transitions(n_e, n_k, lp);
  const int scale_events = (flags & ORACLE_SCALE_EVENTS) != 0;
  const int64_t W = k;
  float mu_u[64], mu_m[64], sg_u[64], sg_m[64], c_u[64], c_m[64], h_u[64], h_m[64];
  int rc = 0;
  for (int64_t i = 0; i < n_k && rc == 0; ++i) {
    if (!oracle_meth_is_site(rank[i], k)) continue;
    const int64_t j0 = i - (W - 1) > 0 ? i - (W - 1) : 0, j1 = i;
    const int64_t e0 = first[j0], e1 = lastv[j1];
    if (e0 < 0 || e1 < e0) continue;
    const int64_t nk = j1 - j0 + 1, ne = e1 - e0 + 1;
    float *x = (float *)malloc(sizeof(float) * (size_t)ne);
    if (!x) {
      rc = -1;
      break;
    }
    for (int64_t e = 0; e < ne; ++e) {
      const float v = event_mean[(e0 + e) * event_stride];
      if (scale_events) {
        const float d = v - shift;
        x[e] = d / scale;
      } else {
        x[e] = v;
      }
    }
    for (int64_t j = 0; j < nk; ++j) {
      const uint32_t r = rank[j0 + j];
      mu_u[j] = scale_events ? mu_model->level_mean[r] : fmaf(mu_model->level_mean[r], scale, shift);
      mu_m[j] = scale_events ? mm_model->level_mean[r] : fmaf(mm_model->level_mean[r], scale, shift);
      sg_u[j] = mu_model->level_stdv[r];
      sg_m[j] = mm_model->level_stdv[r];
      c_u[j] = mu_model->c[r];
      c_m[j] = mm_model->c[r];
      h_u[j] = mu_model->h[r];
      h_m[j] = mm_model->h[r];
    }
    const float vu = oracle_meth_profile(x, ne, mu_u, sg_u, c_u, h_u, nk, lp, flags);
    const float vm = oracle_meth_profile(x, ne, mu_m, sg_m, c_m, h_m, nk, lp, flags);
    free(x);
    llr[i] = vm - vu;
    n_ev[i] = (int32_t)ne;
  }
  free(first);
  free(lastv);
  return rc;
}

/* ---- batch over host threads ---- */

typedef struct {
  int32_t n;
  const float *events;
  int64_t stride;
  const uint64_t *eo, *ko, *po;
  const uint32_t *ranks;
  int32_t k;
  const oracle_meth_model_t *mu, *mm;
  const float *scale, *shift;
  uint32_t flags;
  const int32_t *pairs;
  const int32_t *status;
  float *llr;
  int32_t *n_ev;
  int next, err;
  pthread_mutex_t lock;
} meth_job_t;

static void *meth_worker(void *arg) {
  meth_job_t *J = (meth_job_t *)arg;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    const int r = J->next++;
    pthread_mutex_unlock(&J->lock);
    if (r >= J->n) break;
    const uint64_t e0 = J->eo[r], k0 = J->ko[r], p0 = J->po[r];
    const int64_t n_pairs = J->status[r] == 0 ? (int64_t)(J->po[r + 1] - p0) : 0;
    if (oracle_meth_read(J->events + e0 * J->stride, J->stride, (int64_t)(J->eo[r + 1] - e0), J->ranks + k0,
                         (int64_t)(J->ko[r + 1] - k0), J->k, J->mu, J->mm, J->scale[r], J->shift[r], J->flags,
                         J->pairs + 2 * p0, n_pairs, J->llr + k0, J->n_ev + k0) < 0)
      J->err = 1;
  }
  return NULL;
}

int oracle_meth_batch(int32_t n_reads, const float *events, int64_t event_stride, const uint64_t *event_offset,
                      const uint32_t *ranks, const uint64_t *kmer_offset, int32_t k,
                      const oracle_meth_model_t *mu_model, const oracle_meth_model_t *mm_model, const float *scale,
                      const float *shift, uint32_t flags, const int32_t *pairs, const uint64_t *pair_offset,
                      const int32_t *status, int32_t n_threads, float *llr, int32_t *n_ev) {
  if (n_reads < 0 || k < 2 || k > 64) return -1;
  if (n_threads < 1) n_threads = 1;
  meth_job_t J;
  memset(&J, 0, sizeof J);
  J.n = n_reads;
  J.events = events;
  J.stride = event_stride;
  J.eo = event_offset;
  J.ko = kmer_offset;
  J.po = pair_offset;
  J.ranks = ranks;
  J.k = k;
  J.mu = mu_model;
  J.mm = mm_model;
  J.scale = scale;
  J.shift = shift;
  J.flags = flags;
  J.pairs = pairs;
  J.status = status;
  J.llr = llr;
  J.n_ev = n_ev;
  pthread_mutex_init(&J.lock, NULL);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -1;
  int started = 0;
  for (int32_t t = 0; t < n_threads; ++t) {
    if (pthread_create(&th[t], NULL, meth_worker, &J) != 0) break;
    ++started;
  }
  if (started == 0) meth_worker(&J);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&J.lock);
  return J.err ? -1 : 0;
}
