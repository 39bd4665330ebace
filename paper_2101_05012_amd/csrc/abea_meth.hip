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
 *   k_meth_bounds  one workgroup per 8192 pairs of one read (the tiles of a
 *                  bound of each read's path, from the host's offsets): the
 *                  first and last event paired with each k-mer (the pairs run
 *                  in path order, so a k-mer's pairs are consecutive);
 *   k_meth_sites   one workgroup per 8192 k-mers of one read: the sites
 *                  appended to a list (one atomic per workgroup), NaN / 0
 *                  written for every k-mer that is not a scored site;
 *   k_meth_llr     one thread per listed site: both profiles in registers (a
 *                  column of at most ABEA_MAX_K cells per model), then the LLR.
 */
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "abea_internal.h"

namespace abea {

namespace {

constexpr int KMAX = 12; /* the longest window: k <= ABEA_MAX_K */
constexpr int CHUNK = METH_CHUNK; /* pairs or k-mers per workgroup of the first two kernels */

__device__ __forceinline__ bool is_site(uint32_t rank, int k) {
  return k >= 2 && ((rank >> (2 * (k - 1))) & 3u) == 1u && ((rank >> (2 * (k - 2))) & 3u) == 2u;
}

}  // namespace

/* the plan (reads and tile tables) from pinned host memory into device
 * memory, and the site counter zeroed: a kernel, so that nothing of the call
 * waits in the copy engines' queues behind another stream's work */
__global__ __launch_bounds__(256) void k_meth_stage(const uint64_t *src, uint64_t *dst, size_t words,
                                                    uint32_t *n_sites) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *n_sites = 0u;
  if (i < words) dst[i] = src[i];
}

/* one workgroup per tile, a run of CHUNK pairs of one read (thread t takes
 * the run's pairs t, t+256, ...): the first and the last event paired with
 * each k-mer (a k-mer's pairs are consecutive in the path order).  The
 * read's fields are workgroup-uniform; the pairs are loaded eight
 * iterations ahead of the stores that use them. */
__global__ __launch_bounds__(256) void k_meth_bounds(MethArgs a) {
  const MethTile tl = a.pair_tiles[blockIdx.x];
  const int r = (int)tl.read;
  if (a.status[r] != READ_OK) return;
  const uint64_t p0 = a.pair_offset[r], p1 = a.pair_offset[r + 1];
  const uint64_t c0 = p0 + (uint64_t)tl.chunk * CHUNK;
  if (c0 >= p1) return;
  const uint64_t c1 = c0 + CHUNK < p1 ? c0 + CHUNK : p1;
  const MethRead rd = a.reads[r];
  constexpr int G = 8;
  for (int g = 0; g < CHUNK / 256; g += G) {
    int2 q[G];
    int yp[G], yn[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const uint64_t p = c0 + (uint64_t)(g + u) * 256 + threadIdx.x;
      q[u] = make_int2(0, -1);
      yp[u] = yn[u] = INT32_MIN; /* no neighbour: the run of the k-mer ends here */
      if (p < c1) {
        q[u] = a.pairs[p];
        if (p > p0) yp[u] = a.pairs[p - 1].y;
        if (p + 1 < p1) yn[u] = a.pairs[p + 1].y;
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (q[u].y < 0 || q[u].y >= rd.n_k) continue;
      if (yp[u] != q[u].y) a.kfirst[rd.km_off + q[u].y] = q[u].x;
      if (yn[u] != q[u].y) a.klast[rd.km_off + q[u].y] = q[u].x;
    }
  }
}

/* one workgroup per tile, a run of CHUNK k-mers of one read: the sites of an
 * aligned read go to the list (one atomic per workgroup: the sites are found
 * and counted first, one bit per iteration kept by each thread, then written
 * at the workgroup's base), every other k-mer gets NaN and 0 */
__global__ __launch_bounds__(256) void k_meth_sites(MethArgs a) {
  __shared__ uint32_t wcount[4], wbase[4];
  const MethTile tl = a.kmer_tiles[blockIdx.x];
  const int r = (int)tl.read;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const MethRead rd = a.reads[r];
  const bool ok = a.status[r] == READ_OK;
  const uint32_t j0 = tl.chunk * (uint32_t)CHUNK; /* the run's first k-mer in the read */
  const uint32_t j1 = (uint32_t)rd.n_k - j0 < (uint32_t)CHUNK ? (uint32_t)rd.n_k : j0 + CHUNK;
  uint32_t bits = 0, cnt = 0;
#pragma unroll 8
  for (int it = 0; it < CHUNK / 256; ++it) {
    const uint32_t j = j0 + (uint32_t)it * 256 + threadIdx.x;
    const bool site = ok && j < j1 && is_site(a.ranks[rd.km_off + j], a.k);
    bits |= (uint32_t)site << it;
    cnt += (uint32_t)__popcll(__ballot(site));
  }
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < 4; ++w) t += wcount[w];
    uint32_t b = t ? atomicAdd(a.n_sites, t) : 0u;
    for (int w = 0; w < 4; ++w) {
      wbase[w] = b;
      b += wcount[w];
    }
  }
  __syncthreads();
  uint32_t run = wbase[wave];
  for (int it = 0; it < CHUNK / 256; ++it) {
    const uint32_t j = j0 + (uint32_t)it * 256 + threadIdx.x;
    const bool site = (bits >> it) & 1u;
    const uint64_t m = __ballot(site);
    if (site) {
      const uint32_t slot = run + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      a.sites[slot] = make_uint2((uint32_t)r, j);
    } else if (j < j1) {
      a.llr[rd.km_off + j] = NAN;
      if (a.n_ev) a.n_ev[rd.km_off + j] = 0;
    }
    run += (uint32_t)__popcll(m);
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
    /* the next event's mean is loaded while this one's row is computed */
    float xnext = xm[(uint64_t)a.ev_stride * e0];
    for (int32_t e = e0; e <= e1; ++e) {
      float x = xnext;
      if (e < e1) xnext = xm[(uint64_t)a.ev_stride * (e + 1)];
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

hipError_t launch_meth_stage(const uint64_t *src, uint64_t *dst, size_t words, uint32_t *n_sites, hipStream_t st) {
  const size_t blocks = (words + 255) / 256;
  hipLaunchKernelGGL(k_meth_stage, dim3((uint32_t)(blocks > 0 ? blocks : 1)), dim3(256), 0, st, src, dst, words,
                     n_sites);
  return hipGetLastError();
}

hipError_t launch_meth(const MethArgs &a, hipStream_t st, hipEvent_t *tev) {
  if (a.n_reads > 0 && a.n_kmers > 0) {
    if (a.n_pair_tiles > 0)
      hipExtLaunchKernelGGL(k_meth_bounds, dim3(a.n_pair_tiles), dim3(256), 0, st, tev ? tev[0] : nullptr, nullptr, 0,
                            a);
    else if (tev)
      (void)hipEventRecord(tev[0], st);
    hipExtLaunchKernelGGL(k_meth_sites, dim3(a.n_kmer_tiles), dim3(256), 0, st, nullptr, tev ? tev[1] : nullptr, 0,
                          a);
    hipExtLaunchKernelGGL(k_meth_llr, dim3(2048), dim3(256), 0, st, tev ? tev[2] : nullptr,
                          tev ? tev[3] : nullptr, 0, a);
  }
  return hipGetLastError();
}

}  // namespace abea
