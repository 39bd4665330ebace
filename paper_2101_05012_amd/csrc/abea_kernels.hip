/*
 * abea_kernels.hip -- gfx950 kernels of Adaptive Banded Event Alignment.
 *
 * Thesis Ch. 5 ("GPU Accelerated Adaptive Banded Event Alignment") splits the
 * work into a pre-kernel (§5.4.1.1, Alg. 5.5: first bands and the per-read
 * "kcache" of model entries), a core-kernel (§5.4.1.2, Alg. 5.6-5.8: the band
 * loop) and a post-kernel (§5.4.1.3: backtrack).  The same three stages are
 * here, re-designed for CDNA4:
 *
 *  k_prep      one workgroup per read gathers the model entry of every k-mer
 *              position once and applies the read's scaling, mu' =
 *              fma(mean, scale, shift) (paragraph after Alg. 5.3), so the band
 *              loop streams its k-parameters sequentially.
 *  k_band      one 64-lane wavefront per read.  Band offset j lives in lane
 *              j / CPL, register j % CPL (CPL = cells per lane).  The two
 *              previous bands stay in VGPRs; the neighbour shift of one offset
 *              is a DPP wave_shl/wave_shr move whose edge lane receives -inf
 *              (or the entering event / k-mer parameter).  The band move
 *              (Suzuki-Kasahara rule) is a wave-uniform scalar decision from
 *              two readlanes -- no barrier, no LDS.  Only 2 trace bits per cell
 *              (two bit planes, packed across 32/CPL bands per 32-bit word) and
 *              one move bit per band reach HBM; scores never leave registers.
 *  k_backtrack one wavefront per read walks the path with wave-uniform scalar
 *              state, reading trace words with readlane from a register ring
 *              of prefetched tiles; pairs are gathered 64 at a time in lanes
 *              and stored coalesced.
 *  k_scan/k_compact turn per-read path lengths into the caller's compact
 *              pair layout.
 *
 * Arithmetic of a cell follows Alg. 5.2 and 5.3 exactly as the CPU reference
 * does: FP32, no contraction (-ffp-contract=off and the pragma below), the
 * emission as c - ((x - mu')^2 * h), the moves as (pred + lp) + em, and the
 * first maximum in the order diagonal, up, left.
 */
#include "abea_internal.h"

#pragma clang fp contract(off)

namespace abea {

#define ABEA_NINF (-__builtin_inff())

/* lane l receives v of lane l+1; lane 63 receives fill (DPP wave_shl:1) */
__device__ __forceinline__ float from_next_lane(float v, float fill) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                    0x130, 0xF, 0xF, false));
}
/* lane l receives v of lane l-1; lane 0 receives fill (DPP wave_shr:1) */
__device__ __forceinline__ float from_prev_lane(float v, float fill) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                    0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float rlane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ uint32_t rlane_u(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

/* Value at band offset (lane, reg) of a CPL-register band, as a scalar. */
template <int CPL>
__device__ __forceinline__ float read_offset(const float (&v)[CPL], int reg, int lane) {
  float r = rlane(v[0], lane);
#pragma unroll
  for (int c = 1; c < CPL; ++c) {
    float t = rlane(v[c], lane);
    r = (reg == c) ? t : r;
  }
  return r;
}

/* new[j] = old[j-1] for every offset j; offset 0 takes fill */
template <int CPL>
__device__ __forceinline__ void shift_to_higher(float (&x)[CPL], float fill) {
  float t = from_prev_lane(x[CPL - 1], fill);
#pragma unroll
  for (int c = CPL - 1; c >= 1; --c) x[c] = x[c - 1];
  x[0] = t;
}
/* new[j] = old[j+1] for every offset j; offset 64*CPL-1 takes fill */
template <int CPL>
__device__ __forceinline__ void shift_to_lower(float (&x)[CPL], float fill) {
  float t = from_next_lane(x[0], fill);
#pragma unroll
  for (int c = 0; c < CPL - 1; ++c) x[c] = x[c + 1];
  x[CPL - 1] = t;
}

/* ------------------------------------------------------------------ prep */

__global__ __launch_bounds__(256) void k_prep(const ReadDesc *__restrict__ reads,
                                              const uint32_t *__restrict__ ranks,
                                              const float *__restrict__ scale,
                                              const float *__restrict__ shift,
                                              const ModelEntry *__restrict__ model, uint32_t n_model,
                                              KParam *__restrict__ kparam,
                                              int32_t *__restrict__ rstat) {
  const ReadDesc rd = reads[blockIdx.x];
  if (rd.n_e <= 0 || rd.n_k <= 0) return;
  const float sc = scale[rd.orig];
  const float sh = shift[rd.orig];
  int bad = 0;
  for (int k = threadIdx.x; k < rd.n_k; k += blockDim.x) {
    const uint32_t r = ranks[rd.km_off + k];
    KParam p = {0.f, 0.f, 0.f, 0.f};
    if (r < n_model) {
      const ModelEntry me = model[r];
      p.mu = __builtin_fmaf(me.mean, sc, sh);
      p.c = me.c;
      p.h = me.h;
    } else {
      bad = 1;
    }
    kparam[rd.km_off + k] = p;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) rstat[blockIdx.x] = READ_BAD_RANK;
}

/* ------------------------------------------------------------------ band */

template <int CPL>
__global__ __launch_bounds__(64) void k_band(const BandArgs a) {
  constexpr int N = 64 * CPL;  /* offsets held by the wave */
  constexpr int G = 32 / CPL;  /* bands per trace word */
  const int lane = threadIdx.x;
  const int s = blockIdx.x;
  const ReadDesc rd = a.reads[s];
  const int n_e = rd.n_e, n_k = rd.n_k;
  const int W = a.W;

  if (a.rstat[s] != READ_OK) {
    if (lane == 0) {
      a.out_ll[rd.orig] = ABEA_NINF;
      if (a.out_cells) a.out_cells[rd.orig] = 0;
    }
    return;
  }
  const float lp_skip = rd.lp_skip, lp_stay = rd.lp_stay, lp_step = rd.lp_step;
  const float *__restrict__ ev = a.events + rd.ev_off * 3;
  const KParam *__restrict__ kp = a.kparam + rd.km_off;
  const int H = W / 2;

  int jv[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) jv[c] = lane * CPL + c;

  auto load_ev = [&](int e) -> float {
    float x = 0.0f;
    if (e >= 0 && e < n_e) x = ev[3 * (int64_t)e];
    return x;
  };
  auto load_kp = [&](int k) -> KParam {
    KParam p;
    p.mu = p.c = p.h = p.pad = 0.0f;
    if (k >= 0 && k < n_k) p = kp[k];
    return p;
  };

  /* bands 0 and 1 (initialise_first_two_bands): all -inf except the virtual
   * origin (-1,-1) at offset W/2 of band 0.  Band 0's lower-left is
   * (W/2-1, -1-W/2); band 1 is band 0 moved by one k-mer. */
  float A[CPL], B[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    A[c] = (jv[c] == H) ? 0.0f : ABEA_NINF;
    B[c] = ABEA_NINF;
  }
  int E = H - 1, K = -H; /* lower-left of band 1 */
  int m_prev = 1;

  /* event and k-parameter windows of band 1: offset j is event E-j, k-mer K+j */
  float X[CPL], PM[CPL], PC[CPL], PH[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    X[c] = load_ev(E - jv[c]);
    const KParam p = load_kp(K + jv[c]);
    PM[c] = p.mu;
    PC[c] = p.c;
    PH[c] = p.h;
  }
  /* chunks of the values that enter the windows next: lane l of NX holds
   * event xb+l; lane l of NP holds the k-parameters of k-mer kb+l. */
  int xb = E + 1;
  float NX = load_ev(xb + lane), NXn = load_ev(xb + 64 + lane);
  int kb = K + N;
  KParam NP = load_kp(kb + lane), NPn = load_kp(kb + 64 + lane);

  const int hi_lane = (W - 1) / CPL, hi_reg = (W - 1) % CPL;
  const int last = n_e + n_k;
  uint32_t TU = 0, TL = 0;
  int gb = 0;
  uint64_t g = 0;
  uint32_t mv = 0;
  uint64_t cells = 0;
  uint2 *__restrict__ trace = a.trace + rd.tr_off;
  uint32_t *__restrict__ moves = a.moves + rd.mv_off;
  const int lu = a.lanes_used;

  /* One band: Spp = band i-2 (overwritten by band i), Sp = band i-1. */
  auto step = [&](float(&Spp)[CPL], float(&Sp)[CPL], int i) {
    /* Suzuki-Kasahara placement: towards the better end of band i-1;
     * alternate while both ends are -inf. */
    const float lo = rlane(Sp[0], 0);
    const float hi = read_offset<CPL>(Sp, hi_reg, hi_lane);
    int m;
    if (lo == ABEA_NINF && hi == ABEA_NINF)
      m = i & 1;
    else
      m = (lo < hi) ? 1 : 0;

    float U[CPL], L[CPL], D[CPL];
    if (m) { /* k-mer move: offsets now see k-mer K+1+j */
      K += 1;
      const int kk = K + N - 1;
      if (kk - kb >= 64) {
        NP = NPn;
        kb += 64;
        NPn = load_kp(kb + 64 + lane);
      }
      const int ql = kk - kb;
      shift_to_lower<CPL>(PM, rlane(NP.mu, ql));
      shift_to_lower<CPL>(PC, rlane(NP.c, ql));
      shift_to_lower<CPL>(PH, rlane(NP.h, ql));
      /* up (e-1,k) is offset j+1 of band i-1, left (e,k-1) is offset j */
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        U[c] = Sp[c];
        L[c] = Sp[c];
      }
      shift_to_lower<CPL>(U, ABEA_NINF);
    } else { /* event move: offsets now see event E+1-j */
      E += 1;
      if (E - xb >= 64) {
        NX = NXn;
        xb += 64;
        NXn = load_ev(xb + 64 + lane);
      }
      shift_to_higher<CPL>(X, rlane(NX, E - xb));
      /* up is offset j of band i-1, left is offset j-1 */
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        U[c] = Sp[c];
        L[c] = Sp[c];
      }
      shift_to_higher<CPL>(L, ABEA_NINF);
    }
    /* diagonal (e-1,k-1) is offset j + m_i + m_{i-1} - 1 of band i-2 */
    const int dd = m + m_prev - 1;
#pragma unroll
    for (int c = 0; c < CPL; ++c) D[c] = Spp[c];
    if (dd > 0)
      shift_to_lower<CPL>(D, ABEA_NINF);
    else if (dd < 0)
      shift_to_higher<CPL>(D, ABEA_NINF);
    m_prev = m;

    /* limits in the band: cells inside the DP table */
    const int min_j = max(0, max(E - (n_e - 1), -K));
    const int max_j = min(W - 1, min(E, (n_k - 1) - K));
    if (max_j >= min_j) cells += (uint64_t)(max_j - min_j + 1);

#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      /* Alg. 5.3 log-emission and Alg. 5.2 cell score */
      const float d = X[c] - PM[c];
      const float t = d * d;
      const float u = t * PH[c];
      const float em = PC[c] - u;
      const float sd = (D[c] + lp_step) + em;
      const float su = (U[c] + lp_stay) + em;
      const float sl = L[c] + lp_skip;
      bool bu = su > sd;
      const float s1 = bu ? su : sd;
      bool bl = sl > s1;
      float sv = bl ? sl : s1;
      /* trace code in two bit planes: (0,0) diagonal, (1,0) up, (0,1) left,
       * (1,1) a cell outside the table */
      bu = bu && !bl;
      const bool valid = (jv[c] >= min_j) && (jv[c] <= max_j);
      sv = valid ? sv : ABEA_NINF;
      bu = bu || !valid;
      bl = bl || !valid;
      Spp[c] = sv;
      TU = TU + TU + (bu ? 1u : 0u);
      TL = TL + TL + (bl ? 1u : 0u);
    }

    if (++gb == G) {
      if (lane < lu) trace[g * (uint64_t)lu + lane] = make_uint2(TU, TL);
      ++g;
      gb = 0;
    }
    const int t = i - 2;
    mv |= (uint32_t)m << (t & 31);
    if ((t & 31) == 31) {
      if (lane == 0) moves[t >> 5] = mv;
      mv = 0;
    }
  };

  int i = 2;
  for (;;) {
    step(A, B, i);
    if (++i > last) break;
    step(B, A, i);
    if (++i > last) break;
  }
  /* flush the partial trace word and move word */
  if (gb > 0) {
    const int sh = (G - gb) * CPL;
    if (lane < lu) trace[g * (uint64_t)lu + lane] = make_uint2(TU << sh, TL << sh);
  }
  if (((last - 2) & 31) != 31) {
    if (lane == 0) moves[(last - 2) >> 5] = mv;
  }

  /* terminal cell (n_e-1, n_k-1) sits at offset E - (n_e-1) of the last band */
  float F[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) F[c] = (last & 1) ? B[c] : A[c];
  const int jt = E - (n_e - 1);
  float sc = ABEA_NINF;
  if (jt >= 0 && jt < W) sc = read_offset<CPL>(F, jt % CPL, jt / CPL);
  if (lane == 0) {
    a.rstat[s] = (sc == ABEA_NINF) ? READ_BAND_LOST : READ_OK;
    a.band_end[s] = E;
    a.out_ll[rd.orig] = sc;
    if (a.out_cells) a.out_cells[rd.orig] = cells;
  }
}

/* ------------------------------------------------------------- backtrack */

template <int CPL>
__global__ __launch_bounds__(64) void k_backtrack(const BacktrackArgs a) {
  constexpr int G = 32 / CPL;
  constexpr int P = 8; /* trace tiles in flight */
  const int lane = threadIdx.x;
  const int s = blockIdx.x;
  const ReadDesc rd = a.reads[s];
  const int orig = rd.orig;
  const int status = a.rstat[s];
  if (status != READ_OK) {
    if (lane == 0) {
      a.path_len[orig] = 0;
      a.path_src[orig] = 0;
      a.out_status[orig] = status;
    }
    return;
  }
  const int n_e = rd.n_e, n_k = rd.n_k, lu = a.lanes_used;
  const uint2 *__restrict__ tr = a.trace + rd.tr_off;
  const uint32_t *__restrict__ mvp = a.moves + rd.mv_off;
  const int n_words = (n_e + n_k - 1 + 31) >> 5;

  auto load_tile = [&](int grp) -> uint2 {
    uint2 v = make_uint2(0u, 0u);
    if (grp >= 0 && lane < lu) v = tr[(uint64_t)grp * lu + lane];
    return v;
  };
  auto load_mv = [&](int w) -> uint32_t {
    uint32_t v = 0u;
    if (w >= 0 && w < n_words) v = mvp[w];
    return v;
  };

  int e = n_e - 1, k = n_k - 1, i = n_e + n_k;
  int E = a.band_end[s];

  int gcur = (i - 2) / G;
  uint2 T[P];
#pragma unroll
  for (int p = 0; p < P; ++p) T[p] = load_tile(gcur - p);

  int wcur = (i - 2) >> 5;
  int mb = wcur - 63;
  uint32_t MV = load_mv(mb + lane), MVn = load_mv(mb - 64 + lane);
  uint32_t mword = rlane_u(MV, wcur - mb);

  int PE = 0, PK = 0;
  uint64_t q = 0;
  const uint64_t res_end = rd.pr_off + (uint64_t)(n_e + n_k - 1);
  int2 *__restrict__ out = a.scratch;
  bool ok = true;

  for (;;) {
    /* emit the cell; every 64 cells go out in one coalesced store */
    const int slot = (int)(q & 63);
    PE = (lane == slot) ? e : PE;
    PK = (lane == slot) ? k : PK;
    ++q;
    if ((q & 63) == 0) out[res_end - 1 - (q - 64 + lane)] = make_int2(PE, PK);

    const int t = i - 2;
    const int gi = t / G;
    while (gcur > gi) {
#pragma unroll
      for (int p = 0; p < P - 1; ++p) T[p] = T[p + 1];
      T[P - 1] = load_tile(gcur - P);
      --gcur;
    }
    const int j = E - e;
    const int ln = j / CPL;
    const int c = j - ln * CPL;
    const int bit = 31 - ((t - gi * G) * CPL + c);
    const uint32_t ub = (rlane_u(T[0].x, ln) >> bit) & 1u;
    const uint32_t lb = (rlane_u(T[0].y, ln) >> bit) & 1u;
    int steps;
    if (lb && ub) {
      ok = false;
      break;
    } else if (lb) {
      k -= 1;
      steps = 1;
    } else if (ub) {
      e -= 1;
      steps = 1;
    } else {
      e -= 1;
      k -= 1;
      steps = 2;
    }
    if (e < 0 || k < 0) break;
    /* lower-left event index of the new band from the move bits:
     * E(i-1) = E(i) - (1 - m_i) */
    for (int r = 0; r < steps; ++r) {
      const int tt = i - 2;
      const int wi = tt >> 5;
      while (wcur > wi) {
        --wcur;
        if (wcur < mb) {
          MV = MVn;
          mb -= 64;
          MVn = load_mv(mb - 64 + lane);
        }
        mword = rlane_u(MV, wcur - mb);
      }
      E -= 1 - (int)((mword >> (tt & 31)) & 1u);
      --i;
    }
  }
  if (ok && !(e == -1 && k == -1)) ok = false;
  const int rem = (int)(q & 63);
  if (rem > 0 && lane < rem) out[res_end - 1 - (q - rem + lane)] = make_int2(PE, PK);
  if (lane == 0) {
    a.path_len[orig] = ok ? q : 0;
    a.path_src[orig] = res_end - q;
    a.out_status[orig] = ok ? READ_OK : READ_BAND_LOST;
    if (!ok) a.out_ll[orig] = ABEA_NINF;
  }
}

/* ------------------------------------------------------- scan + compact */

__global__ __launch_bounds__(1024) void k_scan(const uint64_t *__restrict__ len, int n,
                                               uint64_t *__restrict__ off) {
  __shared__ uint64_t part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, tid * per);
  const int hi = min(n, lo + per);
  uint64_t sum = 0;
  for (int r = lo; r < hi; ++r) sum += len[r];
  part[tid] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = part[tid] - sum;
  for (int r = lo; r < hi; ++r) {
    off[r] = run;
    run += len[r];
  }
  if (tid == 1023) off[n] = part[1023];
}

__global__ __launch_bounds__(256) void k_compact(const int2 *__restrict__ scratch,
                                                 const uint64_t *__restrict__ src,
                                                 const uint64_t *__restrict__ off,
                                                 int2 *__restrict__ pairs) {
  const int r = blockIdx.x;
  const uint64_t o = off[r];
  const uint64_t n = off[r + 1] - o;
  const uint64_t s0 = src[r];
  for (uint64_t t = threadIdx.x; t < n; t += blockDim.x) pairs[o + t] = scratch[s0 + t];
}

/* ------------------------------------------------------------- launchers */

hipError_t launch_prep(const ReadDesc *reads, int n_planned, const uint32_t *ranks,
                       const float *scale, const float *shift, const ModelEntry *model,
                       uint32_t n_model, KParam *kparam, int32_t *rstat, hipStream_t st) {
  if (n_planned <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3(n_planned), dim3(256), 0, st, reads, ranks, scale, shift,
                     model, n_model, kparam, rstat);
  return hipGetLastError();
}

hipError_t launch_band(const BandArgs &a, int n_planned, int cpl, hipStream_t st) {
  if (n_planned <= 0) return hipSuccess;
  switch (cpl) {
    case 1: hipLaunchKernelGGL(k_band<1>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_band<2>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_band<4>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_band<8>, dim3(n_planned), dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_backtrack(const BacktrackArgs &a, int n_planned, int cpl, hipStream_t st) {
  if (n_planned <= 0) return hipSuccess;
  switch (cpl) {
    case 1: hipLaunchKernelGGL(k_backtrack<1>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_backtrack<2>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_backtrack<4>, dim3(n_planned), dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_backtrack<8>, dim3(n_planned), dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scan(const uint64_t *len, int n, uint64_t *offset, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, len, n, offset);
  return hipGetLastError();
}

hipError_t launch_compact(const int2 *scratch, const uint64_t *path_src, const uint64_t *offset,
                          int n, int2 *pairs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3(n), dim3(256), 0, st, scratch, path_src, offset, pairs);
  return hipGetLastError();
}

}  // namespace abea
