/*
 * event_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain CPU reference of event detection: the segmentation of a read's raw
 * signal into events {mean, stdv, n} at sudden changes of the signal level
 * (the thesis, Ch. 5 §5.2.2 "Methylation calling", its event-detection
 * paragraph).  The thesis names the step and its output but gives no
 * algorithm; the detector here is the reading recorded in the design notes of
 * the repository:
 *
 *   statistic  For a window length w and a boundary i (between samples i-1
 *              and i, defined for w <= i <= n-w), the squared two-sample t
 *              statistic of the w samples before and the w after, with
 *              population variances:  t^2 = (m_r - m_l)^2 / ((v_l + v_r) / w).
 *              From the integer window sums S and sums of squares Q this is
 *              w D^2 / V with D = S_r - S_l, V = w (Q_l + Q_r) - S_l^2 - S_r^2,
 *              exact integers; the quotient is taken in float32:
 *              T = ((float)D * (float)D) * (float)w / (float)(double)V
 *              (each operation rounded), T = +inf if V = 0 and D != 0, and
 *              T = 0 if V = 0 and D = 0.
 *   peaks      A boundary i is a peak of the detector (w, t_min) if
 *              T(i) > (float)(t_min^2), T(i) > T(j) for every defined j with
 *              i-w < j < i, and T(i) >= T(j) for every defined j with
 *              i < j < i+w (a plateau keeps its first boundary).
 *   events     Two detectors, a short window and a long one; every peak of
 *              either starts an event.  The events are the runs of samples
 *              between consecutive change points, from sample 0 to sample n
 *              (none if n = 0).
 *   stats      For an event of samples a..b-1 (len = b-a) with the exact
 *              integer sum S and sum of squares Q: m = (double)S / len and
 *              V = len*Q - S^2 (len^2 times the population variance, an exact
 *              integer, rounded once to double); then, in pA,
 *              mean = (float)((m + offset) * pa_scale),
 *              stdv = (float)(sqrt((double)V) / len * pa_scale),
 *              duration = (float)len.
 *
 * Build with -ffp-contract=off: no operation is fused.
 */
#include "event_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>

float oracle_ed_stat(const int16_t *x, int64_t n, int32_t w, int64_t i) {
  if (w < 1 || i < w || i > n - w) return -1.0f; /* undefined */
  int64_t sl = 0, sr = 0, ql = 0, qr = 0;
  for (int32_t j = 0; j < w; ++j) {
    const int64_t a = x[i - w + j];
    const int64_t b = x[i + j];
    sl += a;
    ql += a * a;
    sr += b;
    qr += b * b;
  }
  const int64_t d = sr - sl;
  const int64_t v = (int64_t)w * (ql + qr) - sl * sl - sr * sr;
  if (v == 0) return d != 0 ? INFINITY : 0.0f;
  const float df = (float)d;
  const float num = (df * df) * (float)w;
  const float den = (float)(double)v;
  return num / den;
}

void oracle_ed_stats(const int16_t *x, int64_t len, float offset, float pa_scale, float out[3]) {
  int64_t s = 0, q = 0;
  for (int64_t j = 0; j < len; ++j) {
    s += x[j];
    q += (int64_t)x[j] * x[j];
  }
  const double m = (double)s / (double)len;
  const __int128 v = (__int128)len * q - (__int128)s * s;
  out[0] = (float)((m + (double)offset) * (double)pa_scale);
  out[1] = (float)(sqrt((double)v) / (double)len * (double)pa_scale);
  out[2] = (float)len;
}

/* Mark the peaks of one detector in cp[0..n] (cp[i] |= 1); T is scratch of
 * n+1 floats. */
static void mark_peaks(const int16_t *x, int64_t n, int32_t w, float t_min, float *T, uint8_t *cp) {
  for (int64_t i = 0; i <= n; ++i) T[i] = oracle_ed_stat(x, n, w, i);
  const float thr = (float)((double)t_min * (double)t_min);
  for (int64_t i = w; i <= n - w; ++i) {
    if (!(T[i] > thr)) continue;
    int peak = 1;
    for (int64_t j = i - w + 1; j < i && peak; ++j)
      if (j >= w && !(T[i] > T[j])) peak = 0;
    for (int64_t j = i + 1; j < i + w && peak; ++j)
      if (j <= n - w && !(T[i] >= T[j])) peak = 0;
    if (peak) cp[i] = 1;
  }
}

int64_t oracle_ed_change_points(const int16_t *x, int64_t n, const oracle_ed_params_t *p, uint8_t *cp) {
  if (n < 0 || !p) return -1;
  for (int64_t i = 0; i <= n; ++i) cp[i] = 0;
  float *T = (float *)malloc(sizeof(float) * (size_t)(n + 1));
  if (!T) return -1;
  mark_peaks(x, n, p->w_short, p->t_short, T, cp);
  mark_peaks(x, n, p->w_long, p->t_long, T, cp);
  free(T);
  int64_t m = 0;
  for (int64_t i = 0; i <= n; ++i) m += cp[i];
  return m;
}

int64_t oracle_ed_read(const int16_t *x, int64_t n, float offset, float pa_scale, const oracle_ed_params_t *p,
                       float *events) {
  if (n == 0) return 0;
  uint8_t *cp = (uint8_t *)malloc((size_t)(n + 1));
  if (!cp) return -1;
  if (oracle_ed_change_points(x, n, p, cp) < 0) {
    free(cp);
    return -1;
  }
  int64_t m = 0, a = 0;
  for (int64_t i = 1; i <= n; ++i) {
    if (i == n || cp[i]) {
      oracle_ed_stats(x + a, i - a, offset, pa_scale, events + 3 * m);
      ++m;
      a = i;
    }
  }
  free(cp);
  return m;
}

/* ---- batch over host threads (one read per task, longest first) ---- */

typedef struct {
  const int16_t *raw;
  const uint64_t *so;
  const float *offset, *pa_scale;
  const oracle_ed_params_t *p;
  float *events;
  int64_t *n_events;
  const int32_t *order;
  int32_t n;
  int next;
  int err;
  pthread_mutex_t mu;
} ed_job_t;

static void *ed_worker(void *arg) {
  ed_job_t *J = (ed_job_t *)arg;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    const int t = J->next++;
    pthread_mutex_unlock(&J->mu);
    if (t >= J->n) break;
    const int32_t r = J->order[t];
    const uint64_t a = J->so[r], b = J->so[r + 1];
    const int64_t m = oracle_ed_read(J->raw + a, (int64_t)(b - a), J->offset[r], J->pa_scale[r], J->p,
                                     J->events + 3 * a);
    J->n_events[r] = m;
    if (m < 0) J->err = 1;
  }
  return NULL;
}

static const uint64_t *g_so;
static int cmp_len(const void *a, const void *b) {
  const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  const uint64_t lx = g_so[x + 1] - g_so[x], ly = g_so[y + 1] - g_so[y];
  return lx < ly ? 1 : lx > ly ? -1 : (x > y) - (x < y);
}

int oracle_ed_batch(int32_t n_reads, const int16_t *raw, const uint64_t *sample_offset, const float *offset,
                    const float *pa_scale, const oracle_ed_params_t *p, int32_t n_threads, float *events,
                    int64_t *n_events) {
  if (n_reads < 0 || !p) return -1;
  if (n_threads < 1) n_threads = 1;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_reads > 0 ? n_reads : 1));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!order || !th) {
    free(order);
    free(th);
    return -1;
  }
  for (int32_t r = 0; r < n_reads; ++r) order[r] = r;
  g_so = sample_offset;
  qsort(order, (size_t)n_reads, sizeof(int32_t), cmp_len);
  ed_job_t J = {raw, sample_offset, offset, pa_scale, p, events, n_events, order, n_reads, 0, 0,
                PTHREAD_MUTEX_INITIALIZER};
  int started = 0;
  for (int32_t t = 0; t < n_threads; ++t) {
    if (pthread_create(&th[t], NULL, ed_worker, &J) != 0) break;
    ++started;
  }
  if (started == 0) ed_worker(&J);
  for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(order);
  free(th);
  return J.err ? -1 : 0;
}
