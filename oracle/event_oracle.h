/*
 * event_oracle.h -- TEST INFRASTRUCTURE: CPU reference of event detection
 * (the thesis, Ch. 5 §5.2.2, event-detection paragraph; the detector is the
 * reading described in event_oracle.c).  Shares nothing with the HIP library.
 */
#ifndef EVENT_ORACLE_H
#define EVENT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t w_short; /* window of the short detector (samples) */
  int32_t w_long;  /* window of the long detector */
  float t_short;   /* t threshold of the short detector */
  float t_long;    /* t threshold of the long detector */
} oracle_ed_params_t;

/* T(i) of one detector at boundary i, or -1 where undefined (i < w or
 * i > n - w). */
float oracle_ed_stat(const int16_t *x, int64_t n, int32_t w, int64_t i);

/* Event statistics of len >= 1 samples: out = {mean, stdv, duration}. */
void oracle_ed_stats(const int16_t *x, int64_t len, float offset, float pa_scale, float out[3]);

/* Change points of one read: cp[i] = 1 where an event starts at sample i
 * (1 <= i <= n-1); cp has n+1 entries.  Returns their number, or -1. */
int64_t oracle_ed_change_points(const int16_t *x, int64_t n, const oracle_ed_params_t *p, uint8_t *cp);

/* Events of one read into events[3*m] (at most n of them).  Returns m, or -1. */
int64_t oracle_ed_read(const int16_t *x, int64_t n, float offset, float pa_scale, const oracle_ed_params_t *p,
                       float *events);

/* A batch: read r's events go to events[3*sample_offset[r] ...] (a read has
 * at most as many events as samples), their count to n_events[r]. */
int oracle_ed_batch(int32_t n_reads, const int16_t *raw, const uint64_t *sample_offset, const float *offset,
                    const float *pa_scale, const oracle_ed_params_t *p, int32_t n_threads, float *events,
                    int64_t *n_events);

#ifdef __cplusplus
}
#endif

#endif
