/*
 * meth_oracle.h -- TEST INFRASTRUCTURE: CPU reference of methylation scoring
 * (the thesis, Ch. 5 §5.2.2, "Methylation calling": HMM profiling of the
 * aligned events; the profile is the reading described in meth_oracle.c).
 * Shares nothing with the HIP library.
 */
#ifndef METH_ORACLE_H
#define METH_ORACLE_H

#include <stdint.h>

#include "abea_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A pore model with its emission terms (oracle_model_terms). */
typedef struct {
  const float *level_mean;
  const float *level_stdv;
  const float *c;
  const float *h;
} oracle_meth_model_t;

/* 1 if k-mer `rank` starts with C, G (a CpG site at the k-mer's first base). */
int oracle_meth_is_site(uint32_t rank, int32_t k);

/* Best-path score of n_ev events through n_km k-mers (per k-mer mu, sigma,
 * c, h), from a virtual origin before the first cell to the last cell. */
float oracle_meth_profile(const float *x, int64_t n_ev, const float *mu, const float *sigma, const float *c,
                          const float *h, int64_t n_km, const float lp[3], uint32_t flags);

/* One read: llr[i] and n_ev[i] for every k-mer i (NaN and 0 where k-mer i is
 * not a site).  pairs: the read's alignment, (event, k-mer) in path order.
 * flags: ORACLE_SCALE_EVENTS as for oracle_align.  Returns 0, or -1. */
int oracle_meth_read(const float *event_mean, int64_t event_stride, int64_t n_e, const uint32_t *rank,
                     int64_t n_k, int32_t k, const oracle_meth_model_t *mu_model,
                     const oracle_meth_model_t *mm_model, float scale, float shift, uint32_t flags,
                     const int32_t *pairs, int64_t n_pairs, float *llr, int32_t *n_ev);

/* A batch over host threads: read r's pairs are pairs[pair_offset[r] ..
 * pair_offset[r+1]) (none are used unless status[r] == 0); outputs per
 * k-mer of the batch. */
int oracle_meth_batch(int32_t n_reads, const float *events, int64_t event_stride, const uint64_t *event_offset,
                      const uint32_t *ranks, const uint64_t *kmer_offset, int32_t k,
                      const oracle_meth_model_t *mu_model, const oracle_meth_model_t *mm_model, const float *scale,
                      const float *shift, uint32_t flags, const int32_t *pairs, const uint64_t *pair_offset,
                      const int32_t *status, int32_t n_threads, float *llr, int32_t *n_ev);

#ifdef __cplusplus
}
#endif

#endif
