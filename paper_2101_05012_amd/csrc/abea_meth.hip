/*
 * abea_meth.hip -- gfx950 kernels of methylation scoring, the step after the
 * alignment: the events aligned to the reference's k-mers go through HMM
 * profiling to decide whether a base is methylated (the thesis, Ch. 5
 * §5.2.2 "Methylation calling"; it gives no algorithm for the profile).
 *
 * The profile:
 *   - a site is a CpG whose C starts k-mer i of a read (the first two bases
 *     of k-mer i are C, G); its window is the k-mers holding that C,
 *     j0 = max(0, i-k+1) .. i;
 *   - the window's events run from the first event the alignment paired with
 *     k-mer j0 to the last it paired with k-mer i;
 *   - under each of two models (the context's pore model and the methylated
 *     one) the best-path score of those events through the window's k-mers,
 *     with the alignment's own cell score (Alg. 5.2 moves with the read's
 *     transition constants, Alg. 5.3 emission, the model scaled per read): a
 *     virtual origin before the first cell scores 0, cells outside the window
 *     are -inf, and the score is the last cell's;
 *   - LLR = score(methylated) - score(unmethylated), float32.
 *
 * Kernels:
 *   k_meth_prep  one wavefront per read: the first and last event paired with
 *                each k-mer (the pairs run in path order, so a k-mer's pairs
 *                are consecutive), the sites appended to a list, and NaN / 0
 *                written for every k-mer that is not a scored site;
 *   k_meth_llr   one thread per listed site: both profiles in registers (a
 *                column of at most ABEA_MAX_K cells per model), then the LLR.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "abea_internal.h"

namespace abea {

namespace {

constexpr int KMAX = 12; /* the longest window: k <= ABEA_MAX_K */

__device__ __forceinline__ bool is_site(uint32_t rank, int k) {
  return k >= 2 && ((rank >> (2 * (k - 1))) & 3u) == 1u && ((rank >> (2 * (k - 2))) & 3u) == 2u;
}

}  // namespace

__global__ __launch_bounds__(256) void k_meth_prep(MethArgs a) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= a.n_reads) return;
  const MethRead rd = a.reads[r];
  const bool ok = a.status[r] == READ_OK;
  const uint64_t p0 = a.pair_offset[r], p1 = a.pair_offset[r + 1];
  const int32_t n = (int32_t)(p1 - p0);
  const int2 *pr = a.pairs + p0;
  int32_t *kf = a.kfirst + rd.km_off;
  int32_t *kl = a.klast + rd.km_off;
  if (ok) {
    for (int32_t t = lane; t < n; t += 64) {
      const int2 p = pr[t];
      if (p.y < 0 || p.y >= rd.n_k) continue;
      if (t == 0 || pr[t - 1].y != p.y) kf[p.y] = p.x;
      if (t == n - 1 || pr[t + 1].y != p.y) kl[p.y] = p.x;
    }
  }
  for (int32_t i0 = 0; i0 < rd.n_k; i0 += 64) {
    const int32_t i = i0 + lane;
    const bool site = ok && i < rd.n_k && is_site(a.ranks[rd.km_off + i], a.k);
    const uint64_t m = __ballot(site);
    uint32_t base = 0;
    if (lane == 0 && m) base = atomicAdd(a.n_sites, (uint32_t)__popcll(m));
    base = __shfl(base, 0, 64);
    if (site) {
      const uint32_t slot = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      a.sites[slot] = make_uint2((uint32_t)r, (uint32_t)i);
    } else if (i < rd.n_k) {
      a.llr[rd.km_off + i] = NAN;
      if (a.n_ev) a.n_ev[rd.km_off + i] = 0;
    }
  }
}

__global__ __launch_bounds__(256) void k_meth_llr(MethArgs a) {
  const uint32_t n_sites = *a.n_sites;
  const float NI = -INFINITY;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_sites; s += gridDim.x * blockDim.x) {
    const uint2 st = a.sites[s];
    const MethRead rd = a.reads[st.x];
    const int32_t i = (int32_t)st.y;
    const int32_t j0 = i - (a.k - 1) > 0 ? i - (a.k - 1) : 0;
    const int32_t nk = i - j0 + 1;
    const int32_t e0 = a.kfirst[rd.km_off + j0], e1 = a.klast[rd.km_off + i];
    const float scale = a.scale[st.x], shift = a.shift[st.x];
    /* the window's k-mer parameters under both models */
    float mu_u[KMAX], c_u[KMAX], h_u[KMAX], mu_m[KMAX], c_m[KMAX], h_m[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < nk) {
        const uint32_t rk = a.ranks[rd.km_off + j0 + j];
        const ModelEntry u = a.model[rk], m = a.meth_model[rk];
        mu_u[j] = a.scale_events ? u.mean : __builtin_fmaf(u.mean, scale, shift);
        mu_m[j] = a.scale_events ? m.mean : __builtin_fmaf(m.mean, scale, shift);
        c_u[j] = u.c;
        h_u[j] = u.h;
        c_m[j] = m.c;
        h_m[j] = m.h;
      } else {
        mu_u[j] = mu_m[j] = c_u[j] = c_m[j] = h_u[j] = h_m[j] = 0.0f;
      }
    }
    /* columns of the previous event (up and diagonal neighbours) */
    float su[KMAX], sm[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) su[j] = sm[j] = NI;
    const float *xm = a.events + (uint64_t)a.ev_stride * rd.ev_off;
    for (int32_t e = e0; e <= e1; ++e) {
      float x = xm[(uint64_t)a.ev_stride * e];
      if (a.scale_events) {
        const float d = x - shift;
        x = d / scale;
      }
      float du = (e == e0) ? 0.0f : NI; /* diagonal of k-mer 0: the origin before the first cell */
      float dm = du;
      float lu = NI, lm = NI; /* left neighbours in this event's row */
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        if (j < nk) {
          const float d_u = x - mu_u[j];
          const float em_u = c_u[j] - ((d_u * d_u) * h_u[j]);
          const float d_m = x - mu_m[j];
          const float em_m = c_m[j] - ((d_m * d_m) * h_m[j]);
          const float nu = fmaxf(fmaxf((du + rd.lp_step) + em_u, (su[j] + rd.lp_stay) + em_u), lu + rd.lp_skip);
          const float nm = fmaxf(fmaxf((dm + rd.lp_step) + em_m, (sm[j] + rd.lp_stay) + em_m), lm + rd.lp_skip);
          du = su[j];
          dm = sm[j];
          su[j] = nu;
          sm[j] = nm;
          lu = nu;
          lm = nm;
        }
      }
    }
    float vu = NI, vm = NI;
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j == nk - 1) {
        vu = su[j];
        vm = sm[j];
      }
    a.llr[rd.km_off + i] = vm - vu;
    if (a.n_ev) a.n_ev[rd.km_off + i] = e1 - e0 + 1;
  }
}

hipError_t launch_meth(const MethArgs &a, hipStream_t st) {
  if (a.n_reads > 0) {
    hipLaunchKernelGGL(k_meth_prep, dim3((a.n_reads + 3) / 4), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_meth_llr, dim3(2048), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace abea
