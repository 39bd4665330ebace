/*
 * abea_detect.hip -- gfx950 kernels of event detection: the segmentation of
 * each read's raw signal into events {mean, stdv, n} at sudden changes of the
 * signal level (the thesis, Ch. 5 §5.2.2 "Methylation calling", its
 * event-detection paragraph; its output is the event table of Alg. 5.1).
 *
 * The thesis gives no algorithm for the step.  The detector is a two-window
 * change-point test:
 *   - at a boundary i (between samples i-1 and i; defined for
 *     w <= i <= n-w) the squared two-sample t statistic of the w samples
 *     before and the w after, with population variances, is w D^2 / V with
 *     D = S_r - S_l and V = w (Q_l + Q_r) - S_l^2 - S_r^2 (S sums, Q sums of
 *     squares: exact integers); the quotient is taken in float32 as
 *     ((float)D * (float)D) * (float)w / (float)(double)V, +inf for V = 0 and
 *     D != 0, 0 for V = 0 and D = 0;
 *   - i is a peak of the detector (w, t) if its statistic exceeds t^2 (as a
 *     float), is greater than the statistic at every defined boundary up to
 *     w-1 before it and not less than at every one up to w-1 after it;
 *   - a short and a long detector; every peak of either starts an event;
 *   - an event's mean and stdv come from its exact integer sum S and sum of
 *     squares Q: m = (double)S / len, V = len*Q - S^2 (exact, then rounded
 *     once to double), mean = (float)((m + offset) * pa_scale),
 *     stdv = (float)(sqrt(V) / len * pa_scale), pA = (raw + offset) * pa_scale.
 *
 * The work is a stream over the raw samples:
 *   k_ed_tiles     the tile table (one wavefront per read);
 *   k_ed_detect    one workgroup per tile of 1024 boundaries of one read:
 *                  samples to LDS as prefix sums, both statistics, peaks
 *                  (four consecutive boundaries per thread, their window
 *                  maxima shared), one bit per boundary, and the tile's
 *                  event count and first change point;
 *   k_ed_scan      exclusive scan of the tile counts, per 1024 tiles, then
 *                  over the blocks (k_ed_scan_top);
 *   k_ed_events    one workgroup per tile: the tile's event starts in order,
 *                  the end of its last event from the first change point of
 *                  the read's next tiles, and one thread per event for its
 *                  statistics;
 *   k_ed_offsets   each read's first event.
 * Both streaming kernels stage their samples as prefix sums with wavefront
 * scans by DPP (no LDS permutes), and the statistics share the prefix
 * sums' LDS once those are no longer read.
 */
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "abea_internal.h"

namespace abea {

namespace {

constexpr int TS = ED_TILE;   /* boundaries per tile */
constexpr int WMAX = ED_MAX_WINDOW;
constexpr int XH = 2 * WMAX;  /* samples kept before (and after) the tile */
constexpr int THL = WMAX;     /* statistics kept before (and after) the tile */
constexpr int NX = TS + 2 * XH;
constexpr int NT = TS + 2 * THL;
constexpr int WORDS = TS / 64; /* flag words per tile */
constexpr int THREADS = 256;
constexpr int SCAN_TILES = 1024; /* tiles per block of the first scan level */
constexpr int EXT = 256; /* samples staged after the tile for events that run past it */
constexpr int NE = TS + EXT; /* samples the event kernel stages per tile */

/* a / b rounded to nearest, for 0 <= a < 2^64 and 1 <= b < 2^64: a
 * reciprocal estimate refined by one Newton step, a first quotient, and two
 * corrections from exact residuals (FMA).  It is the refinement the general
 * FP32 division performs; the general one also scales operands whose
 * quotient or reciprocal would leave the normal range and patches zero,
 * infinite and NaN operands, none of which arises here (a = 0 gives +0). */
__device__ __forceinline__ float div_small(float a, float b) {
  const float y0 = __builtin_amdgcn_rcpf(b);
  const float e = __builtin_fmaf(-b, y0, 1.0f);
  const float y = __builtin_fmaf(e, y0, y0);
  const float q0 = a * y;
  const float r0 = __builtin_fmaf(-b, q0, a);
  const float q1 = __builtin_fmaf(r0, y, q0);
  const float r1 = __builtin_fmaf(-b, q1, a);
  return __builtin_fmaf(r1, y, q1);
}

/* statistic of the detector with window w at boundary j of a read of n
 * samples, from prefix sums: P[c] and PQ[c] sum the staged samples before
 * sample j (and their squares).  Q_l + Q_r and V are taken in double, where
 * every value is an integer below 2^41 (at most 2 * 16 * 2^30 for the sums of
 * squares, 2^40 for w (Q_l + Q_r) and S^2), so each operation is exact and V
 * is the exact integer.  Branch-free: the loads stay inside the staged range
 * for every boundary of the tile and its halo. */
__device__ __forceinline__ float ed_stat(const int *P, const double *PQ, int c, int w, int j, int n) {
  const int sl = P[c] - P[c - w];
  const int sr = P[c + w] - P[c];
  const double q = PQ[c + w] - PQ[c - w];
  const double dl = (double)sl, dr = (double)sr;
  const double v = __builtin_fma(-dl, dl, __builtin_fma(-dr, dr, (double)w * q));
  const int d = sr - sl;
  const float df = (float)d;
  const float num = (df * df) * (float)w;
  const float den = (float)v;
  const float qt = div_small(num, v == 0.0 ? 1.0f : den);
  const float t = v != 0.0 ? qt : (d != 0 ? INFINITY : 0.0f);
  return (j >= w && j <= n - w) ? t : -1.0f;
}

/* per lane: the larger of a and b, and the largest of a, b and c (one
 * v_max_f32 / v_max3_f32 without canonicalisation: the statistics are never
 * NaN) */
__device__ __forceinline__ float max2(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float max3(float a, float b, float c) {
  float r;
  asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

/* largest of v[i0 .. i0+cnt-1] and init (cnt >= 0, compile-time indices) */
template <int I0, int CNT, int NV>
__device__ __forceinline__ float run_max(const float (&v)[NV], float init) {
  float m = init;
  int i = I0;
#pragma unroll
  for (; i + 1 < I0 + CNT; i += 2) m = max3(m, v[i], v[i + 1]);
  if constexpr ((CNT & 1) != 0) m = max2(m, v[I0 + CNT - 1]);
  return m;
}

/* Peaks of the detector (window W, thr = t^2) at the four boundaries
 * ts[q0 .. q0+3]: boundary q is a peak if ts[q] is above thr and above every
 * statistic up to W-1 before it, and not below any up to W-1 after it.
 * Undefined boundaries hold -1, below every defined statistic, so they never
 * block a peak; thr >= 0 takes part in the maximum before (t > thr and
 * t > max(before) is t > max(thr, before)).  The four windows on each side
 * share all but three of their W-1 values, so their maxima are built from
 * one common maximum.  With W = 0 the window is w_rt (at run time). */
template <int W>
__device__ __forceinline__ uint32_t ed_peaks4(const float *ts, int q0, int w_rt, float thr) {
  uint32_t bits = 0;
  if constexpr (W > 0) {
    constexpr int H = W - 1;          /* neighbours on each side, >= 1 */
    constexpr int R = (H + 3) / 4;    /* float4s of neighbours on each side */
    constexpr int NV = 4 + 8 * R;
    constexpr int C = 4 * R;          /* v[C + j] is ts[q0 + j] */
    float v[NV];
    const float4 *p = reinterpret_cast<const float4 *>(ts + q0 - C);
#pragma unroll
    for (int f = 0; f < NV / 4; ++f) {
      const float4 x = p[f];
      v[4 * f] = x.x;
      v[4 * f + 1] = x.y;
      v[4 * f + 2] = x.z;
      v[4 * f + 3] = x.w;
    }
    float L[4], Rm[4];
    if constexpr (H >= 4) {
      /* before: window j is v[C+j-H .. C+j-1]; all four hold v[C+3-H .. C-1] */
      const float cl = run_max<C + 3 - H, H - 3>(v, thr);
      const float a12 = max2(v[C - H + 1], v[C - H + 2]);
      const float b01 = max2(v[C], v[C + 1]);
      L[0] = max3(v[C - H], a12, cl);
      L[1] = max3(a12, cl, v[C]);
      L[2] = max3(v[C - H + 2], cl, b01);
      L[3] = max3(cl, b01, v[C + 2]);
      /* after: window j is v[C+j+1 .. C+j+H]; all four hold v[C+4 .. C+H] */
      const float cr = run_max<C + 5, H - 4>(v, v[C + 4]);
      const float c23 = max2(v[C + 2], v[C + 3]);
      const float e12 = max2(v[C + H + 1], v[C + H + 2]);
      Rm[0] = max3(v[C + 1], c23, cr);
      Rm[1] = max3(c23, cr, v[C + H + 1]);
      Rm[2] = max3(v[C + 3], cr, e12);
      Rm[3] = max3(cr, e12, v[C + H + 3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        L[j] = thr;
        Rm[j] = v[C + j + 1];
#pragma unroll
        for (int m = 1; m <= H; ++m) L[j] = max2(L[j], v[C + j - m]);
#pragma unroll
        for (int m = 2; m <= H; ++m) Rm[j] = max2(Rm[j], v[C + j + m]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) bits |= ((v[C + j] > L[j]) & (v[C + j] >= Rm[j])) ? (1u << j) : 0u;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = q0 + j;
      const float t = ts[q];
      float lm = thr, rm = -1.0f;
      for (int m = 1; m < w_rt; ++m) {
        lm = fmaxf(lm, ts[q - m]);
        rm = fmaxf(rm, ts[q + m]);
      }
      bits |= ((t > lm) & (t >= rm)) ? (1u << j) : 0u;
    }
  }
  return bits;
}

/* v of lane l-n of the same row of 16 lanes, cyclically (DPP row_ror:n) */
template <int N>
__device__ __forceinline__ uint32_t row_ror(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x120 + N, 0xF, 0xF, true);
}

/* Stage samples base+k, k in [0, NS), of a read (zero outside [0, lim)) as
 * prefix sums: P[k] and PQ[k] sum the first k values and their squares
 * (QT: long long, or double, exact for NS * 2^30 < 2^53).
 * Thread t takes PER_ consecutive samples; the sums are scanned over the wave
 * and over the waves.  Ends with a barrier. */
/* inclusive scan over the 64 lanes of a wavefront by DPP: within each row
 * of 16 lanes by shifts of 1, 2, 4 and 8 (lanes without a source add 0),
 * then lane 15 of each row into the next row and lane 31 into the upper
 * half */
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
__device__ __forceinline__ int wave_scan(int v) {
  v += dpp_i<0x111, 0xF>(v); /* row_shr:1 */
  v += dpp_i<0x112, 0xF>(v); /* row_shr:2 */
  v += dpp_i<0x114, 0xF>(v); /* row_shr:4 */
  v += dpp_i<0x118, 0xF>(v); /* row_shr:8 */
  v += dpp_i<0x142, 0xA>(v); /* row_bcast:15 into rows 1 and 3 */
  v += dpp_i<0x143, 0xC>(v); /* row_bcast:31 into rows 2 and 3 */
  return v;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)dpp_i<CTRL, ROWS>((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)dpp_i<CTRL, ROWS>((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
/* the same over 64-bit integers, and over doubles that hold integers below
 * 2^53 (every sum exact) */
__device__ __forceinline__ double wave_scan(double v) {
  v += dpp_d<0x111, 0xF>(v);
  v += dpp_d<0x112, 0xF>(v);
  v += dpp_d<0x114, 0xF>(v);
  v += dpp_d<0x118, 0xF>(v);
  v += dpp_d<0x142, 0xA>(v);
  v += dpp_d<0x143, 0xC>(v);
  return v;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_l(long long v) {
  const uint64_t b = (uint64_t)v;
  const uint32_t lo = (uint32_t)dpp_i<CTRL, ROWS>((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)dpp_i<CTRL, ROWS>((int)(uint32_t)(b >> 32));
  return (long long)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ long long wave_scan(long long v) {
  v += dpp_l<0x111, 0xF>(v);
  v += dpp_l<0x112, 0xF>(v);
  v += dpp_l<0x114, 0xF>(v);
  v += dpp_l<0x118, 0xF>(v);
  v += dpp_l<0x142, 0xA>(v);
  v += dpp_l<0x143, 0xC>(v);
  return v;
}

template <int NS, typename QT>
__device__ __forceinline__ void stage_prefix(const int16_t *x, int64_t base, int64_t lim, int *P, QT *PQ, int *wsum,
                                             QT *wsq) {
  constexpr int PER_ = (NS + THREADS - 1) / THREADS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int v[PER_];
  int s = 0;
  QT q = 0;
#pragma unroll
  for (int e = 0; e < PER_; ++e) {
    const int k = PER_ * (int)threadIdx.x + e;
    const int64_t si = base + k;
    v[e] = (k < NS && si >= 0 && si < lim) ? (int)x[si] : 0;
    s += v[e];
    q += (QT)(v[e] * v[e]);
  }
  const int si = wave_scan(s);
  const QT qi = wave_scan(q);
  if (lane == 63) {
    wsum[wave] = si;
    wsq[wave] = qi;
  }
  __syncthreads();
  int ps = si - s;
  QT pq = qi - q;
  for (int w = 0; w < wave; ++w) {
    ps += wsum[w];
    pq += wsq[w];
  }
  if (threadIdx.x == 0) {
    P[0] = 0;
    PQ[0] = 0;
  }
#pragma unroll
  for (int e = 0; e < PER_; ++e) {
    const int k = PER_ * (int)threadIdx.x + e;
    ps += v[e];
    pq += (QT)(v[e] * v[e]);
    if (k < NS) {
      P[k + 1] = ps;
      PQ[k + 1] = pq;
    }
  }
  __syncthreads();
}

}  // namespace

/* the tile table: one wavefront per read writes its tiles' entries */
__global__ void k_ed_tiles(DetectArgs a) {
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= a.n_reads) return;
  const uint64_t s0 = a.sample_offset[r];
  const uint32_t n = (uint32_t)(a.sample_offset[r + 1] - s0);
  const uint32_t t0 = a.tile_first[r], t1 = a.tile_first[r + 1];
  for (uint32_t t = t0 + (threadIdx.x & 63); t < t1; t += 64) {
    EdTile e;
    e.s0 = s0;
    e.n = n;
    e.i0 = (t - t0) * (uint32_t)TS;
    e.read = (uint32_t)r;
    e.g_end = t1;
    a.tiles[t] = e;
  }
}

/* WS, WL: the detector windows fixed at compile time, or 0 to read them
 * from the arguments */
template <int WS, int WL>
__global__ __launch_bounds__(THREADS) void k_ed_detect(DetectArgs a) {
  /* the prefix sums, then (once every thread holds its statistics in
   * registers) the two rows of statistics in the same bytes: a smaller LDS
   * footprint, more workgroups per CU */
  __shared__ __align__(16) unsigned char lds[(NX + 1) * (sizeof(double) + sizeof(int))];
  double *PQ = reinterpret_cast<double *>(lds);
  int *P = reinterpret_cast<int *>(lds + (NX + 1) * sizeof(double));
  float *tsh = reinterpret_cast<float *>(lds);
  float *tlg = tsh + NT;
  static_assert(2 * NT * sizeof(float) <= sizeof(lds) && (NT * sizeof(float)) % 16 == 0, "statistics fit");
  __shared__ int wsum[THREADS / 64];
  __shared__ double wsq[THREADS / 64];
  __shared__ uint32_t wcnt[THREADS / 64];
  __shared__ int32_t wfirst[THREADS / 64];
  static_assert(TS == 4 * THREADS, "four boundaries per thread");
  static_assert(THL == WMAX && THL % 4 == 0, "the peak loads stay inside the statistics");
  const uint32_t g = blockIdx.x;
  const EdTile tl = a.tiles[g];
  const int64_t n = tl.n;
  const int64_t i0 = tl.i0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ws = WS > 0 ? WS : a.w_short;
  const int wl = WL > 0 ? WL : a.w_long;

  /* samples i0-XH .. i0+TS+XH-1 */
  stage_prefix<NX>(a.raw + tl.s0, i0 - XH, n, P, PQ, wsum, wsq);
  /* boundary j = i0 - THL + k: the sums before it are P[k + XH - THL] */
  /* j in 32 bits: reads hold fewer than 2^31 samples, so n - w fits, and a
   * j of 2^31 or more (past the read's end) wraps to a negative value, which
   * is outside [w, n - w] like j itself */
  constexpr int NIT = (NT + THREADS - 1) / THREADS;
  float rs[NIT], rl[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int k = (int)threadIdx.x + THREADS * it;
    if (k < NT) {
      const int j = (int)((uint32_t)i0 - (uint32_t)THL + (uint32_t)k);
      const int c = k + XH - THL;
      rs[it] = ed_stat(P, PQ, c, ws, j, (int)n);
      rl[it] = ed_stat(P, PQ, c, wl, j, (int)n);
    }
  }
  __syncthreads(); /* every thread is done with the prefix sums */
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int k = (int)threadIdx.x + THREADS * it;
    if (k < NT) {
      tsh[k] = rs[it];
      tlg[k] = rl[it];
    }
  }
  __syncthreads();
  /* thread t: boundaries 4t .. 4t+3 of the tile (statistics q0 .. q0+3);
   * the neighbours read lie in q0-16 .. q0+19, inside [0, NT) */
  const int q0 = 4 * (int)threadIdx.x + THL;
  const uint32_t nib = ed_peaks4<WS>(tsh, q0, ws, a.thr_short) | ed_peaks4<WL>(tlg, q0, wl, a.thr_long);
  /* flag word m of the wave (its boundaries 64m .. 64m+63) is lanes 16m ..
   * 16m+15, four bits each: its low half from the row's lanes 0-7, its high
   * half from lanes 8-15, gathered by three row rotations (lane 7 and lane
   * 15 of the row end with the halves) */
  uint32_t x = nib << (4 * (lane & 7));
  x |= row_ror<1>(x);
  x |= row_ror<2>(x);
  x |= row_ror<4>(x);
  if ((lane & 7) == 7) {
    uint32_t *f32 = reinterpret_cast<uint32_t *>(a.flags + (uint64_t)g * WORDS + 4 * wave);
    f32[lane >> 3] = x;
  }
  /* the wave's change points and its first one (wave-uniform masks) */
  const uint64_t b0 = __ballot(nib & 1u), b1 = __ballot(nib & 2u), b2 = __ballot(nib & 4u), b3 = __ballot(nib & 8u);
  if (lane == 0) {
    wcnt[wave] = (uint32_t)(__popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3));
    const uint64_t any = b0 | b1 | b2 | b3;
    int32_t f = INT32_MAX;
    if (any) {
      const int l = __builtin_ctzll(any);
      const int j = ((b0 >> l) & 1u) ? 0 : ((b1 >> l) & 1u) ? 1 : ((b2 >> l) & 1u) ? 2 : 3;
      f = 256 * wave + 4 * l + j;
    }
    wfirst[wave] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = (i0 == 0) ? 1u : 0u; /* the read's first event starts at sample 0 */
    int32_t f = INT32_MAX;
    for (int w = 0; w < THREADS / 64; ++w) {
      c += wcnt[w];
      f = min(f, wfirst[w]);
    }
    a.count[g] = c;
    /* the tile's first change point in the read, -1 if it has none */
    a.first_cp[g] = f == INT32_MAX ? -1 : (int32_t)(i0 + f);
  }
}

namespace {

/* exclusive scan of v over the workgroup (THREADS lanes); returns the prefix
 * and sets total */
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) before += sh[w];
    all += sh[w];
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

}  // namespace

/* first level: tiles [b*1024, (b+1)*1024), four consecutive per thread */
__global__ __launch_bounds__(THREADS) void k_ed_scan(DetectArgs a) {
  __shared__ uint64_t sh[THREADS / 64];
  const uint64_t t0 = (uint64_t)blockIdx.x * SCAN_TILES + 4u * threadIdx.x;
  uint32_t c[4];
  uint64_t s = 0;
  for (int q = 0; q < 4; ++q) {
    c[q] = (t0 + q < a.n_tiles) ? a.count[t0 + q] : 0u;
    s += c[q];
  }
  uint64_t total;
  uint64_t p = block_exclusive_scan(s, sh, total);
  for (int q = 0; q < 4; ++q) {
    if (t0 + q < a.n_tiles) a.base[t0 + q] = p;
    p += c[q];
  }
  if (threadIdx.x == 0) a.block_sum[blockIdx.x] = total;
}

/* second level, one workgroup: exclusive scan of the block sums in place;
 * block_sum[n_blocks] receives the batch's event count */
__global__ __launch_bounds__(THREADS) void k_ed_scan_top(DetectArgs a, uint32_t n_blocks) {
  __shared__ uint64_t sh[THREADS / 64];
  uint64_t carry = 0;
  for (uint32_t b0 = 0; b0 < n_blocks; b0 += THREADS) {
    const uint32_t b = b0 + threadIdx.x;
    const uint64_t v = b < n_blocks ? a.block_sum[b] : 0;
    uint64_t total;
    const uint64_t p = block_exclusive_scan(v, sh, total);
    if (b < n_blocks) a.block_sum[b] = carry + p;
    carry += total;
  }
  if (threadIdx.x == 0) a.block_sum[n_blocks] = carry;
}

__global__ __launch_bounds__(THREADS) void k_ed_events(DetectArgs a) {
  __shared__ uint64_t wf[WORDS];
  __shared__ uint32_t wpre[WORDS + 1];
  __shared__ int32_t starts[TS + 1];
  __shared__ long long tail_end;
  /* prefix sums of samples i0 .. i0+TS+EXT-1 of the read (zero past its end) */
  __shared__ int P[NE + 1];
  __shared__ long long PQ[NE + 1];
  __shared__ int wsum[THREADS / 64];
  __shared__ long long wsq[THREADS / 64];
  const uint32_t g = blockIdx.x;
  const EdTile tl = a.tiles[g];
  const int r = (int)tl.read;
  const int64_t n = tl.n;
  const int64_t i0 = tl.i0;
  const int first = (i0 == 0) ? 1 : 0;
  const uint64_t gbase = a.base[g] + a.block_sum[g / SCAN_TILES];
  const int16_t *x = a.raw + tl.s0;

  if (threadIdx.x < WORDS) wf[threadIdx.x] = a.flags[(uint64_t)g * WORDS + threadIdx.x];
  if (threadIdx.x == 0) tail_end = n;
  stage_prefix<NE>(x, i0, n, P, PQ, wsum, wsq);
  /* the event that runs past the tile ends at the read's next change point:
   * the first change point of the first later tile of the read that has one
   * (first_cp grows with the tile), or at the read's end; 256 tiles a step */
  for (uint32_t h0 = g + 1; h0 < tl.g_end; h0 += THREADS) {
    const uint32_t h = h0 + threadIdx.x;
    const int32_t f = h < tl.g_end ? a.first_cp[h] : -1;
    if (f >= 0) atomicMin(&tail_end, (long long)f);
    if (__syncthreads_or(f >= 0)) break;
  }
  /* the events before each flag word (wf is visible: stage_prefix ends with
   * a barrier): a scan of the 16 words' counts over 16 lanes of the first
   * wavefront */
  static_assert(WORDS == 16, "one lane per flag word");
  if (threadIdx.x < WORDS) {
    const uint32_t c = (uint32_t)__popcll(wf[threadIdx.x]);
    uint32_t inc = c;
#pragma unroll
    for (int d = 1; d < WORDS; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d, WORDS);
      if ((int)threadIdx.x >= d) inc += o;
    }
    wpre[threadIdx.x] = (uint32_t)first + inc - c;
    if (threadIdx.x == WORDS - 1) wpre[WORDS] = (uint32_t)first + inc;
    if (threadIdx.x == 0 && first) starts[0] = 0;
  }
  __syncthreads();
  /* a wavefront holds one flag word (k & 63 is the lane): a set bit's rank
   * in it is the count of set bits of the lanes below (mbcnt) */
  for (int k = threadIdx.x; k < TS; k += THREADS) {
    const uint64_t m = wf[k >> 6];
    if ((m >> (k & 63)) & 1u) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      starts[wpre[k >> 6] + below] = (int32_t)(i0 + k);
    }
  }
  __syncthreads();
  const int n_ev = (int)wpre[WORDS];
  const double off = (double)a.offset[r];
  const double sc = (double)a.pa_scale[r];
  const int64_t lim = i0 + NE; /* staged: [i0, lim) */
  for (int e = threadIdx.x; e < n_ev; e += THREADS) {
    const uint64_t idx = gbase + (uint64_t)e;
    if (idx >= a.capacity) continue;
    const int64_t b0 = starts[e];
    const int64_t b1 = (e + 1 < n_ev) ? (int64_t)starts[e + 1] : (int64_t)tail_end;
    /* the event's sums from the staged prefix sums; past the staged range
     * (an event that runs far beyond the tile) from memory */
    const int64_t bs = b1 < lim ? b1 : lim;
    int64_t s = (int64_t)P[bs - i0] - P[b0 - i0];
    int64_t q = PQ[bs - i0] - PQ[b0 - i0];
    for (int64_t j = bs; j < b1; ++j) {
      const int64_t v = x[j];
      s += v;
      q += v * v;
    }
    const int64_t len = b1 - b0;
    /* an event is no longer than its read (< 2^31 samples): its length
     * converts from 32 bits, to the same value */
    const int32_t len32 = (int32_t)len;
    const double dlen = (double)len32;
    /* len^2 times the population variance, exact, rounded once to double:
     * below 2^16 samples S fits 32 bits and len * Q and S^2 stay below 2^62
     * (samples are 16-bit), so 64 bits hold it; longer events take 128 */
    double m, vd;
    if (len < 65536) {
      const int32_t s32 = (int32_t)s;
      m = (double)s32 / dlen;
      vd = (double)(uint64_t)((int64_t)len32 * q - (int64_t)s32 * s32);
    } else {
      m = (double)s / dlen;
      const unsigned __int128 vv = (unsigned __int128)((__int128)len * q - (__int128)s * s);
      const uint64_t hi = (uint64_t)(vv >> 64);
      if (hi == 0) {
        vd = (double)(uint64_t)vv;
      } else {
        /* keep the top 64 bits and a sticky bit: one rounding to double */
        const int k = 64 - __builtin_clzll(hi);
        const unsigned __int128 low = vv & ((((unsigned __int128)1) << k) - 1);
        const uint64_t top = (uint64_t)(vv >> k) | (low != 0 ? 1u : 0u);
        vd = __builtin_ldexp((double)top, k);
      }
    }
    float *ev = a.events + 3 * idx;
    ev[0] = (float)((m + off) * sc);
    ev[1] = (float)(__builtin_sqrt(vd) / dlen * sc);
    ev[2] = (float)len32;
  }
}

__global__ void k_ed_offsets(DetectArgs a, uint32_t n_blocks) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > a.n_reads) return;
  const uint32_t t = a.tile_first[r];
  a.event_offset[r] = t < a.n_tiles ? a.base[t] + a.block_sum[t / SCAN_TILES] : a.block_sum[n_blocks];
}

uint32_t ed_scan_blocks(uint32_t n_tiles) { return (n_tiles + SCAN_TILES - 1) / SCAN_TILES; }

hipError_t launch_detect(const DetectArgs &a, hipStream_t st, hipEvent_t *tev) {
  const uint32_t nb = ed_scan_blocks(a.n_tiles);
  hipEvent_t e0 = tev ? tev[0] : nullptr, e1 = tev ? tev[1] : nullptr;
  hipEvent_t e2 = tev ? tev[2] : nullptr, e3 = tev ? tev[3] : nullptr;
  if (tev) {
    const hipError_t e = hipEventRecord(tev[4], st);
    if (e != hipSuccess) return e;
  }
  if (a.n_tiles > 0) {
    hipLaunchKernelGGL(k_ed_tiles, dim3((a.n_reads + 3) / 4), dim3(256), 0, st, a);
    /* the two streaming kernels take their start and end from their own
     * dispatch when timed */
    if (a.w_short == 3 && a.w_long == 8)
      hipExtLaunchKernelGGL((k_ed_detect<3, 8>), dim3(a.n_tiles), dim3(THREADS), 0, st, e0, e1, 0, a);
    else
      hipExtLaunchKernelGGL((k_ed_detect<0, 0>), dim3(a.n_tiles), dim3(THREADS), 0, st, e0, e1, 0, a);
    hipLaunchKernelGGL(k_ed_scan, dim3(nb), dim3(THREADS), 0, st, a);
  } else if (tev) {
    (void)hipEventRecord(e0, st);
    (void)hipEventRecord(e1, st);
  }
  hipLaunchKernelGGL(k_ed_scan_top, dim3(1), dim3(THREADS), 0, st, a, nb);
  if (a.n_tiles > 0) {
    hipExtLaunchKernelGGL(k_ed_events, dim3(a.n_tiles), dim3(THREADS), 0, st, e2, e3, 0, a);
  } else if (tev) {
    (void)hipEventRecord(e2, st);
    (void)hipEventRecord(e3, st);
  }
  const int nr = a.n_reads + 1;
  hipLaunchKernelGGL(k_ed_offsets, dim3((nr + 255) / 256), dim3(256), 0, st, a, nb);
  if (tev) {
    const hipError_t e = hipEventRecord(tev[5], st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace abea
