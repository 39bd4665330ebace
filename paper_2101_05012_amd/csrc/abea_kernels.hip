/*
 * abea_kernels.hip -- gfx950 kernels of Adaptive Banded Event Alignment.
 *
 * The thesis (Ch. 5 "GPU Accelerated Adaptive Banded Event Alignment")
 * splits the work into a pre-kernel (§5.4.1.1, Alg. 5.5: first bands and the
 * per-read "kcache" of model entries), a core-kernel (§5.4.1.2, Alg. 5.6-5.8:
 * the band loop, one thread block per read, four block barriers per band) and
 * a post-kernel (§5.4.1.3: one thread per read backtracks).  The same three
 * stages are here, re-designed for CDNA4:
 *
 *  k_prep      one workgroup per read: the read's status and, only where the
 *              band fill cannot read them in place (inputs at addresses of
 *              their own, e.g. mapped host memory, or events scaled to the
 *              model), a copy of the ranks and the event means.  The
 *              scaled model level of every k-mer position, mu' = fma(mean,
 *              scale, shift) (paragraph after Alg. 5.3), and its emission
 *              terms (the kcache) are made by the band fill itself, from
 *              the rank and the model entry it gathers.
 *  k_band      one 64-lane wavefront per read, no barrier and no score in
 *              memory.  K-mer k of a band lives in slot k mod N (N = 64*CPL >
 *              W; slot s is lane s / CPL, register s % CPL), so a cell's up
 *              neighbour is the same slot of the previous band and its left
 *              and diagonal neighbours are slot s-1 of the two previous bands:
 *              one DPP wave_ror:1 per band (the diagonal reuses the previous
 *              band's).  The slots keep their k-mers and are relabelled every
 *              few bands from a per-wave LDS k-mer ring; each band reads its
 *              events from an LDS event ring.  The band move (Suzuki-Kasahara
 *              rule) is a wave-uniform scalar decision.  Slots outside the band
 *              are cleared to -inf each band: every one of them, or (interior
 *              bands of launches that fill the SIMDs) only the two beside the
 *              band.  Only two trace bits per slot reach HBM (two bit planes,
 *              32/CPL bands per 32-bit word).
 *  k_backtrack one wavefront per read walks the path with wave-uniform scalar
 *              state: the trace bits of cell (e, k) are in group (e+k)/G, lane
 *              (k mod N)/CPL, so no band positions are needed.  Trace tiles
 *              stream through an LDS ring; pairs are gathered in lanes, up to
 *              64 at a time, and stored coalesced.
 *  k_align     the fused form: each wavefront fills a read's bands and then
 *              walks it, one read per wavefront or a persistent pool taking
 *              reads from a device work queue.
 *  k_scan/k_compact turn per-read path lengths into the caller's compact
 *              pair layout.
 *
 * Arithmetic of a cell follows Alg. 5.2 and 5.3 exactly as the CPU reference
 * does: FP32, no contraction (-ffp-contract=off and the pragma below), the
 * emission as c - ((x - mu')^2 * h), the moves as (pred + lp) + em, and the
 * first maximum in the order diagonal, up, left.
 */
#include "abea_internal.h"

#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>

#pragma clang fp contract(off)

namespace abea {

#define ABEA_NINF (-__builtin_inff())

template <int CPL>
struct Log2 {
  static constexpr int v = CPL == 1 ? 0 : CPL == 2 ? 1 : CPL == 4 ? 2 : CPL == 8 ? 3 : 4;
};

/* lane l receives v of lane l-1, lane 0 receives lane 63 (DPP wave_ror:1).
 * Every lane has a source, so bound_ctrl changes nothing; it is set because
 * it lets the compiler fold the rotation into the instruction that uses it. */
__device__ __forceinline__ float rot_up(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, true));
}
/* rot_up(l) + a and rot_up(d) + b, the rotations folded into the adds (two
 * v_add_f32_dpp, where a shared rotation would be a move and two adds).  The
 * s_nop gives the two wait states a DPP read needs after a VALU write of
 * its source, which the compiler does not track into inline assembly. */
__device__ __forceinline__ void add_rot2(float l, float a, float d, float b, float &lo, float &dout) {
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %2, %3 wave_ror:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %1, %4, %5 wave_ror:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(lo), "=&v"(dout)
      : "v"(l), "v"(a), "v"(d), "v"(b));
}
__device__ __forceinline__ float rlane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ uint32_t rlane_u(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
/* per lane: bit set in `mask` selects if_set, else if_clear (one v_cndmask) */
__device__ __forceinline__ float sel(float if_clear, float if_set, uint64_t mask) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(mask));
  return r;
}
/* a wave-uniform value held in a VGPR (one v_mov_b32) */
__device__ __forceinline__ float to_vgpr(float s) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(s));
  return r;
}
/* per lane: the largest of a, b and c (one v_max3_f32, no canonicalisation) */
__device__ __forceinline__ float vmax3(float a, float b, float c) {
  float r;
  asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
/* per lane: acc*2 + (bit of `mask`), one v_addc */
__device__ __forceinline__ uint32_t shift_in(uint32_t acc, uint64_t mask) {
  uint32_t r;
  uint64_t co;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(co) : "v"(acc), "s"(mask));
  return r;
}
/* per lane: the bit of `mask`, the first bit of a new accumulator (one
 * v_cndmask, where a shift-in would need a zeroed register) */
__device__ __forceinline__ uint32_t first_bit(uint64_t mask) {
  uint32_t r;
  asm("v_cndmask_b32_e64 %0, 0, 1, %1" : "=v"(r) : "s"(mask));
  return r;
}
__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }
/* lane `lane` of the result is `val` (uniform), the others keep `old`
 * (v_writelane; the compiler places the lane index in M0) */
__device__ int writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

#define ABEA_NINF_BITS ((int)0xff800000)

/* Value held by slot `slot` of a band, as a scalar. */
template <int CPL>
__device__ __forceinline__ float read_slot(const float (&v)[CPL], int slot) {
  const int ln = slot >> Log2<CPL>::v;
  const int r = slot & (CPL - 1);
  /* read every register, then pick the scalar: a per-lane select over the
   * registers would be turned into an indexed (memory) access */
  float t = rlane(v[0], ln);
#pragma unroll
  for (int c = 1; c < CPL; ++c) {
    const float u = rlane(v[c], ln);
    t = (r == c) ? u : t;
  }
  return t;
}

/* ------------------------------------------------------------------ prep */

__global__ __launch_bounds__(256) void k_prep(const ReadDesc *__restrict__ reads,
                                              const float *__restrict__ events, int events_stride,
                                              const uint32_t *__restrict__ ranks,
                                              const uint64_t *__restrict__ in_addr,
                                              const float *__restrict__ scale,
                                              const float *__restrict__ shift,
                                              int scale_events,
                                              float *__restrict__ xmean,
                                              uint32_t *__restrict__ krank,
                                              int32_t *__restrict__ rstat,
                                              uint32_t *__restrict__ queue) {
  /* the work-queue counter of the alignment kernel that follows */
  if (blockIdx.x == 0 && threadIdx.x == 0 && queue) *queue = 0u;
  const ReadDesc rd = reads[blockIdx.x];
  if (rd.n_e <= 0 || rd.n_k <= 0) {
    if (threadIdx.x == 0) rstat[blockIdx.x] = READ_EMPTY;
    return;
  }
  /* a rank outside the model is found by the band fill, which reads every
   * rank of the read */
  if (threadIdx.x == 0) rstat[blockIdx.x] = READ_OK;
  /* the read's events and ranks: in the batch arrays at its offsets (12-byte
   * events with the mean first, or the means alone), or (in_addr) at
   * addresses of its own, where only the event means are stored */
  const int ev_stride = in_addr ? 1 : events_stride;
  const float *ev =
      in_addr ? reinterpret_cast<const float *>(in_addr[2 * rd.orig]) : events + (uint64_t)ev_stride * rd.ev_off;
  const uint32_t *rk =
      in_addr ? reinterpret_cast<const uint32_t *>(in_addr[2 * rd.orig + 1]) : ranks + rd.km_off;
  if (krank)
    for (int k = threadIdx.x; k < rd.n_k; k += blockDim.x) krank[rd.km_off + k] = rk[k];
  if (!xmean) return;
  if (scale_events) {
    /* per-read scaling (paragraph after Alg. 5.3), the events to the model:
     * x' = (x - shift) / scale, float32 subtract, correctly rounded divide */
    const float sc = scale[rd.orig];
    const float sh = shift[rd.orig];
    for (int e = threadIdx.x; e < rd.n_e; e += blockDim.x) {
      const float d = ev[(int64_t)ev_stride * e] - sh;
      xmean[rd.ev_off + e] = d / sc;
    }
  } else {
    for (int e = threadIdx.x; e < rd.n_e; e += blockDim.x) xmean[rd.ev_off + e] = ev[(int64_t)ev_stride * e];
  }
}

/* ------------------------------------------------------------------ band */

/* Band move of the Suzuki-Kasahara rule from the bits of the two end cells
 * of the previous band, as a wave mask: all ones (k-mer move) if lo < hi,
 * else 0 (event move); when both are -inf the band parity decides, a k-mer
 * move for odd bands.  For odd bands hi is first raised to at least -FLT_MAX
 * (`nfm` holds -FLT_MAX in every lane): then lo < hi holds exactly when lo is
 * -inf too (no finite lo is below -FLT_MAX), and every other outcome is
 * unchanged.  The compare runs on the VALU with all lanes active, so its lane
 * mask is all ones or all zeros and its low half is the result. */
template <bool ODD>
__device__ __forceinline__ uint64_t sk_move_mask(int lo, int hi, float nfm) {
  float tv;
  uint64_t cm;
  if (ODD)
    asm volatile(
        "v_max_f32 %[tv], %[h], %[nfm]\n\t"
        "v_cmp_lt_f32_e64 %[cm], %[lo], %[tv]"
        : [tv] "=&v"(tv), [cm] "=s"(cm)
        : [lo] "s"(lo), [h] "s"(hi), [nfm] "v"(nfm));
  else
    asm volatile(
        "v_mov_b32 %[tv], %[h]\n\t"
        "v_cmp_lt_f32_e64 %[cm], %[lo], %[tv]"
        : [tv] "=&v"(tv), [cm] "=s"(cm)
        : [lo] "s"(lo), [h] "s"(hi));
  return cm;
}

/* The same decision with the last end cell left in its register: one compare
 * of lo against every lane's value of that register (raised to -FLT_MAX for
 * odd bands), whose bit for the end cell's lane is the answer.  No readlane
 * and no move of the last end cell into a VGPR. */
template <bool ODD>
__device__ __forceinline__ uint64_t sk_cmp_lane(int lo, float hv, float nfm) {
  float tv;
  uint64_t cm;
  if (ODD)
    asm volatile(
        "v_max_f32 %[tv], %[h], %[nfm]\n\t"
        "v_cmp_lt_f32_e64 %[cm], %[lo], %[tv]"
        : [tv] "=&v"(tv), [cm] "=s"(cm)
        : [lo] "s"(lo), [h] "v"(hv), [nfm] "v"(nfm));
  else
    asm volatile("v_cmp_lt_f32_e64 %[cm], %[lo], %[h]" : [cm] "=s"(cm) : [lo] "s"(lo), [h] "v"(hv));
  return cm;
}

/* The band move at two slots per lane with edge masks, from the lane
 * compare's mask cm: its bit hl (the last end cell's lane) goes straight into
 * SCC, and SCC moves the two edge masks one slot up, makes the move's wave
 * mask and adds the move to K (the shifted copy n0 of the top mask does not
 * depend on the move).  Returns the wave mask: all ones on a k-mer move. */
__device__ __forceinline__ uint64_t sk_move_edges2(uint64_t cm, int hl, uint64_t (&m)[2], int &K) {
  const uint64_t top = m[1];
  const uint64_t n0 = (top << 1) | (top >> 63); /* the top register, one slot higher */
  uint64_t mv;
  asm("s_bitcmp1_b64 %[cm], %[hl]\n\t"
      "s_cselect_b64 %[m1], %[m0], %[m1]\n\t"
      "s_cselect_b64 %[m0], %[n0], %[m0]\n\t"
      "s_cselect_b64 %[mv], -1, 0\n\t"
      "s_addc_u32 %[K], %[K], 0"
      : [m0] "+&s"(m[0]), [m1] "+&s"(m[1]), [mv] "=&s"(mv), [K] "+&s"(K)
      : [cm] "s"(cm), [hl] "s"(hl), [n0] "s"(n0)
      : "scc");
  return mv;
}

/* The register of slot (.. % CPL == r) of every lane, as one VGPR. */
template <int CPL>
__device__ __forceinline__ float pick(const float (&v)[CPL], int r) {
  float t = v[0];
#pragma unroll
  for (int c = 1; c < CPL; ++c) t = sel(t, v[c], ballot(r == c));
  return t;
}

/* The register holding slot `slot` of a band at four slots per lane, as one
 * VGPR: the register is chosen by the slot's two low bits in two levels of
 * selects, whose wave masks are made on the SALU. */
__device__ __forceinline__ float end_cell_reg4(const float (&v)[4], int slot) {
  uint64_t m0, m1;
  asm("s_bitcmp1_b32 %2, 0\n\t"
      "s_cselect_b64 %0, -1, 0\n\t"
      "s_bitcmp1_b32 %2, 1\n\t"
      "s_cselect_b64 %1, -1, 0"
      : "=&s"(m0), "=s"(m1)
      : "s"(slot)
      : "scc");
  const float a = sel(v[0], v[1], m0);
  const float b = sel(v[2], v[3], m0);
  return sel(a, b, m1);
}
/* Bits of the value held by slot `slot` at four slots per lane, as a scalar. */
__device__ __forceinline__ int end_cell_bits4(const float (&v)[4], int slot) {
  return __builtin_amdgcn_readlane(__float_as_int(end_cell_reg4(v, slot)), slot >> 2);
}

/* Wave masks, one per register, of the two slots beside a band of W cells
 * whose first k-mer is K: k-mers K - 1 and K + W. */
template <int CPL>
__device__ __forceinline__ void edge_init(uint64_t (&m)[CPL], int K, int W) {
  constexpr int N = 64 * CPL;
  constexpr int LC = Log2<CPL>::v;
  const int sa = (K - 1) & (N - 1), sb = (K + W) & (N - 1);
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    m[c] = (((sa & (CPL - 1)) == c) ? (1ull << (sa >> LC)) : 0ull) |
           (((sb & (CPL - 1)) == c) ? (1ull << (sb >> LC)) : 0ull);
}

/* The same masks after the band move `mneg` (-1: k-mer move, the band and
 * both slots one k-mer higher; 0: unchanged).  One slot higher is the next
 * register of the same lane, or register 0 of the next lane (lane 63 wraps to
 * lane 0); the shifted copy does not depend on the move, so only the selects
 * wait for it. */
template <int CPL>
__device__ __forceinline__ void edge_move(uint64_t (&m)[CPL], int mneg) {
  const uint64_t top = m[CPL - 1];
  const uint64_t n0 = (top << 1) | (top >> 63); /* the top register, one slot higher */
  /* 64-bit selects on one compare (the compiler would split each in two) */
  if constexpr (CPL == 2) {
    asm("s_cmp_lg_u32 %[mn], 0\n\t"
        "s_cselect_b64 %[m1], %[m0], %[m1]\n\t"
        "s_cselect_b64 %[m0], %[n0], %[m0]"
        : [m0] "+&s"(m[0]), [m1] "+&s"(m[1])
        : [n0] "s"(n0), [mn] "s"(mneg)
        : "scc");
  } else {
    static_assert(CPL == 4, "edge masks are kept for two or four slots per lane");
    asm("s_cmp_lg_u32 %[mn], 0\n\t"
        "s_cselect_b64 %[m3], %[m2], %[m3]\n\t"
        "s_cselect_b64 %[m2], %[m1], %[m2]\n\t"
        "s_cselect_b64 %[m1], %[m0], %[m1]\n\t"
        "s_cselect_b64 %[m0], %[n0], %[m0]"
        : [m0] "+&s"(m[0]), [m1] "+&s"(m[1]), [m2] "+&s"(m[2]), [m3] "+&s"(m[3])
        : [n0] "s"(n0), [mn] "s"(mneg)
        : "scc");
  }
}

/* Sizes of the band fill for CPL slots per lane.
 *   N   slots of the wave (64*CPL >= W + 2)
 *   G   bands per trace word (32/CPL, even)
 *   RX  entries of the event ring: holds every event of the band window
 *       plus the next G, in quarters of 64, one quarter spare (W + G <= RX - 128)
 *   RK  entries of the k-mer ring: holds k-mers K .. K+N+G, same rule
 *   S   sub-rings of the event ring: event e is in sub-ring e mod S.  At four
 *       slots per lane a register's slots hold k-mers of one residue mod 4,
 *       consecutive lanes k-mers 4 apart, so in a band the lanes of a
 *       register read events 4 apart: from one sub-ring, consecutive words
 *       (no LDS bank conflict), where a single ring would put them 4 words
 *       apart.  At two slots per lane the 2-way conflict of a single ring
 *       costs less than the sub-ring index arithmetic (measured on the
 *       W = 100 workloads); at one, lanes already read consecutive events.
 *   XS  floats of a sub-ring: RX/S entries and a mirror of its first G/S */
template <int CPL>
struct Geom {
  static constexpr int N = 64 * CPL;
  static constexpr int LC = Log2<CPL>::v;
  static constexpr int G = 32 / CPL;
  static constexpr int RX = CPL == 1 ? 256 : (128 * CPL > 1024 ? 1024 : 128 * CPL);
  static constexpr int RK = CPL == 1 ? 256 : 128 * CPL;
  static constexpr int S = CPL == 4 ? 4 : 1;
  static constexpr int LS = Log2<S>::v;
  static constexpr int XS = RX / S + G / S;
};

/* LDS of one wavefront: the band fill's event ring (S sub-rings, each with a
 * mirror of its first G/S entries behind its end, so that a run of G reads
 * never wraps) and k-mer ring, or the backtrack's trace-tile ring; the two
 * phases of a read never overlap. */
template <int CPL>
struct WaveLds {
  union {
    struct {
      float lx[Geom<CPL>::S * Geom<CPL>::XS];
      float4 lk[Geom<CPL>::RK];
    } band;
    uint2 ring[BT_RING_GROUPS * 64];
  };
};

/* Band fill of one read whose status is READ_OK (Alg. 5.1 loop, Alg. 5.2,
 * 5.3), by the calling wavefront: writes the read's trace tiles, its
 * log-likelihood and cell count, and returns READ_OK or READ_BAND_LOST.
 *
 * Slot s (lane s / CPL, register s % CPL) holds k-mer kv(s) = K_r + ((s -
 * K_r) mod N), fixed from one refill to the next (every RF bands, RF <= N - W
 * and RF <= G): a k-mer that leaves the band keeps its slot until
 * the next refill relabels the slot as the k-mer N higher, which cannot enter
 * the band before then.  At a refill the wavefront loads each slot's k-mer
 * parameters (mu', c, h) from the k-mer ring and the LDS address of its event
 * at the refill band; band b after it reads the event of the slot from that
 * address + b (the event of a cell (e, k) in band i is i - 2 - k).
 *
 * Every slot computes a score each band; the slots outside the band must read
 * as -inf wherever a later cell of the band takes them as a neighbour.  Edge
 * bands (some cell outside the DP table) clear every slot outside the cells
 * of the band in the table, and so do interior bands unless CLEAR_EDGES.
 * With CLEAR_EDGES (two or four slots per lane) interior bands clear only
 * k-mers K - 1 and K + W: the cells of the next band read band i at
 * k-mers K' - 1 .. K' + W - 1 and band i - 1 at K' - 1 .. K' + W - 2, with K'
 * = K or K + 1, so no other slot outside a band is ever read by a cell in one,
 * and what those slots hold (scores of k-mers outside the band, or NaN from
 * stale ring entries) never reaches the band, its end cells or the trace bits
 * of its cells. */
template <int CPL, int RPG, int CLEAR, bool TRIM>
__device__ __forceinline__ int band_read(const AlignArgs &a, const ReadDesc &rd, uint2 *trace,
                                         float *__restrict__ lx, float4 *__restrict__ lk, int &e_end) {
  /* CLEAR: slot clearing of interior bands, 0 the window, 1 the two edge
   * slots, 2 the two edge slots with W even at two slots per lane (then the
   * band's first and last slots always lie in different registers) */
  constexpr bool CLEAR_EDGES = CLEAR != 0;
  constexpr bool W_EVEN = CLEAR == 2;
  static_assert(!W_EVEN || CPL == 2, "the even-W form is for two slots per lane");
  constexpr int N = Geom<CPL>::N;
  constexpr int LC = Geom<CPL>::LC;
  constexpr int G = Geom<CPL>::G;
  constexpr int RX = Geom<CPL>::RX;
  constexpr int RK = Geom<CPL>::RK;
  constexpr int S = Geom<CPL>::S;
  constexpr int LS = Geom<CPL>::LS;
  constexpr int XS = Geom<CPL>::XS;
  constexpr int RXS = RX / S;
  static_assert(S == 1 || (G % S == 0 && (G / RPG) % S == 0),
                "refills at band offsets that are multiples of S keep each register's sub-ring fixed");
  constexpr int RF = G / RPG; /* bands between slot refills (RPG refills per group) */
  static_assert(RF >= 2 && RF % 2 == 0, "refill interval must be an even band count");

  const int lane = threadIdx.x & 63;
  const int n_e = rd.n_e, n_k = rd.n_k;
  const int W = a.W;

  const float lp_skip = rd.lp_skip, lp_stay = rd.lp_stay, lp_step = rd.lp_step;
  /* vector copies of the skip and step constants: the moves of a register's
   * first slot add them to a rotated neighbour, and only with a vector second
   * operand can the rotation fold into the add (v_add_f32_dpp) */
  const float lp_skip_v = to_vgpr(lp_skip), lp_step_v = to_vgpr(lp_step);
  /* the read's event means, in place (every xstride-th float) or staged */
  const int xs = a.xstride;
  const float *__restrict__ xm = a.xsrc + (uint64_t)xs * rd.ev_off;
  /* the read's ranks and the model they index; each k-mer's parameters are
   * made here (the kcache of the paragraph after Alg. 5.3): mu' =
   * fma(mean, scale, shift) with one rounding, or the unscaled mean when the
   * events are scaled to the model, and the entry's emission terms c, h */
  const uint32_t *__restrict__ rk = a.ranks + rd.km_off;
  const float4 *__restrict__ mdl = reinterpret_cast<const float4 *>(a.model);
  const uint32_t n_model = a.n_model;
  const bool scale_ev = a.scale_events != 0;
  const float ksc = a.scale[rd.orig];
  const float ksh = a.shift[rd.orig];
  uint32_t bad_rank = 0; /* this lane met a rank outside the model */
  const int H = W / 2;
  const float NI = ABEA_NINF;
  const float NFM = __int_as_float((int)0xff7fffff); /* -FLT_MAX */

  auto ldx = [&](int e) -> float {
    float v = 0.0f;
    if (e >= 0 && e < n_e) v = xm[(int64_t)xs * e];
    return v;
  };
  /* a k-mer's rank (positions outside the read take rank 0: their slots are
   * outside the table, whatever they hold never reaches a cell of it) */
  auto ldr = [&](int k) -> uint32_t {
    uint32_t r = 0;
    if (k >= 0 && k < n_k) r = rk[k];
    return r;
  };
  /* its model entry, gathered (a rank outside the model is noted, and
   * entry 0 read in its place) */
  auto gather = [&](uint32_t r) -> float4 {
    const bool ok = r < n_model;
    bad_rank |= ok ? 0u : 1u;
    return mdl[ok ? r : 0u];
  };
  /* the slot parameters (mu', c, h) of a gathered entry */
  auto kparam = [&](float4 m) -> float4 {
    return make_float4(scale_ev ? m.x : __builtin_fmaf(m.x, ksc, ksh), m.y, m.z, 0.0f);
  };
  /* event e = 64q + lane: sub-ring e mod S (the lane's low bits), entry
   * floor(e / S) mod RX/S */
  auto put_x = [&](int q, float v) {
    float *sub = lx + (lane & (S - 1)) * XS;
    const int idx = ((q * 64 + lane) >> LS) & (RXS - 1);
    sub[idx] = v;
    if (idx < G / S) sub[RXS + idx] = v;
  };
  auto put_k = [&](int q, float4 v) { lk[(q * 64 + lane) & (RK - 1)] = v; };

  /* Trim states (the trim paragraph after Alg. 5.3): a column at k-mer -1
   * whose cell (e, -1) is (e-1, -1) + lp_trim, every event before the read
   * left unaligned; it lies in a band only while the band's first k-mer is
   * -1 or less, i.e. in bands with cells outside the table.  The first
   * k-mer is entered from it diagonally only (its left neighbour is -inf).
   * The end: end_best over the bands of the last k-mer's cells, the best of
   * (e, n_k-1) and the previous best with event e trimmed (ties to fewer
   * trims); end_u the end cell's event. */
  constexpr bool trim = TRIM;
  const float lp_trim = a.lp_trim;
  float end_best = ABEA_NINF;
  int end_u = -1;

  /* Band 1 (initialise_first_two_bands): band 0 has lower-left (W/2-1,
   * -1-W/2) and holds only the virtual origin (-1,-1) with score 0; band 1 is
   * band 0 moved one k-mer and is all -inf (with trim: but for the trim cell
   * (0, -1) at offset W/2-1).  K is the first k-mer of the latest band, E the
   * event of its first cell. */
  int K = -H;
  int E = H - 1;
  /* bits of the end cells of the latest band, for the next band's move:
   * band 1's are -inf, unless the trim cell is its first (W = 2, 3) */
  int lo_c = (trim && H == 1) ? __float_as_int(lp_trim) : ABEA_NINF_BITS, hi_c = ABEA_NINF_BITS;
  /* edge kernels at two slots per lane keep the last end cell in its
   * register (hv, lane hl) and decide the move by one compare against every
   * lane; at four slots per lane (three or fewer wavefronts per SIMD) the
   * longer scalar chain of that form did not pay */
  constexpr bool LANE_MOVE = CLEAR_EDGES && CPL == 2;
  float hv = NI;
  int hl = 0;
  /* CLEAR_EDGES: interior bands clear only the two slots beside the band,
   * whose wave masks follow every band move on the SALU */
  static_assert(!CLEAR_EDGES || CPL == 2 || CPL == 4, "edge clearing needs two or four slots per lane");
  constexpr bool EDGE_MASKS = CLEAR_EDGES;
  uint64_t edge[CPL];
  if constexpr (EDGE_MASKS) edge_init<CPL>(edge, K, W);
  /* at two slots per lane: all ones when the first (last) slot of the latest
   * band is odd, i.e. in register 1 */
  uint64_t plo = (K & 1) ? ~0ull : 0ull;
  uint64_t phi = ((K + W - 1) & 1) ? ~0ull : 0ull; /* ~plo when W is even */
  float Spp[CPL], Sp[CPL], PM[CPL], PC[CPL], PH[CPL];
  int kvs[CPL]; /* kv(slot), the k-mer the slot holds */
  int xb[CPL]; /* ring index of the slot's event at band b = 0 of the group */
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int kv = K + ((lane * CPL + c - K) & (N - 1));
    Spp[c] = (kv == -1) ? 0.0f : NI;                   /* band 0: the origin, k-mer -1 */
    Sp[c] = (trim && kv == -1) ? 0.0f + lp_trim : NI; /* band 1: the trim cell (0, -1) */
    PM[c] = PC[c] = PH[c] = 0.0f;
    kvs[c] = kv;
    xb[c] = 0;
  }

  /* Rings: event e in sub-ring e mod S at entry (e / S) mod (RX / S), k-mer
   * k at lk[k mod RK], written a quarter (64 entries) at a time; the quarter
   * after the top one waits in registers. */
  int xtop = (E + G) >> 6;
  int ktop = (K + N + G - 1) >> 6;
  for (int q = (E - W + 1) >> 6; q <= xtop; ++q) put_x(q, ldx(q * 64 + lane));
  for (int q = K >> 6; q <= ktop; ++q) put_k(q, kparam(gather(ldr(q * 64 + lane))));
  float xpend = ldx((xtop + 1) * 64 + lane);
  /* the k-mer quarter after the top one: its model entries, gathered; the
   * one after that: its ranks (two loads in a chain, each a refill ahead) */
  float4 kpend = gather(ldr((ktop + 1) * 64 + lane));
  uint32_t rpend = ldr((ktop + 2) * 64 + lane);

  auto advance_rings = [&]() {
    if (((E + G) >> 6) > xtop) {
      ++xtop;
      put_x(xtop, xpend);
      xpend = ldx((xtop + 1) * 64 + lane);
    }
    if (((K + N + G - 1) >> 6) > ktop) {
      ++ktop;
      put_k(ktop, kparam(kpend));
      kpend = gather(rpend);
      rpend = ldr((ktop + 2) * 64 + lane);
    }
  };

  /* Relabel the slots for the current K (before band i's move) and load
   * their k-mer parameters and event addresses; b is the band's index in
   * its group, i = i0 + b. */
  auto refill = [&](int i, int b) {
    K = __builtin_amdgcn_readfirstlane(K);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int d = (lane * CPL + c - K) & (N - 1);
      const int kv = K + d;
      kvs[c] = kv;
      const float4 p = lk[kv & (RK - 1)];
      PM[c] = p.x;
      PC[c] = p.y;
      PH[c] = p.z;
      /* the slot's event at this refill band i: e = i - 2 - kv, with e
       * mod S = (S - c) mod S for every lane (kv = c mod S, i = 2 mod S);
       * its sub-ring entry less the band offset (b is a multiple of S) */
      xb[c] = (((i - 2 - kv) >> LS) & (RXS - 1)) - (b >> LS);
    }
  };

  const int last = n_e + n_k;
  uint32_t TD = 0, TU = 0;
  uint64_t cells = 0;

  /* One band i = i0 + b: Spp = band i-2 (overwritten by band i), Sp = band
   * i-1.  INTERIOR: all W cells of band i are inside the DP table. */
  /* the events of the slots for band b (of the current refill interval) */
  auto load_x = [&](float(&x)[CPL], int b) {
    /* event e_ref + (b - b_ref) of slot register c: sub-ring (r0 + b) mod S,
     * entry xb[c] + (r0 + b) / S, with r0 = e_ref mod S = (S - c) mod S */
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int r0 = (S - (c & (S - 1))) & (S - 1);
      x[c] = lx[((r0 + b) & (S - 1)) * XS + xb[c] + ((r0 + b) >> LS)];
    }
  };

  /* fresh: the band opens a trace word (its first register's bits start the
   * words TD and TU; a full group's G*CPL bits fill them, so nothing carries
   * from one group to the next) */
  auto band = [&](auto interior_tag, float(&Spp)[CPL], const float(&Sp)[CPL], int i, int b,
                  const float(&X)[CPL], bool fresh) {
    constexpr bool INTERIOR = decltype(interior_tag)::value;
    constexpr bool EDGE = INTERIOR && EDGE_MASKS;
    /* the band position is wave-uniform: keep it in SGPRs */
    K = __builtin_amdgcn_readfirstlane(K);
    /* Suzuki-Kasahara placement from the two end cells of band i-1 (taken
     * at the end of that band, into lo_c and hi_c); i0 is even, so i is odd
     * when b is.  The event of the first cell follows from K: e + k = i - 2
     * in band i. */
    const int lo = lo_c, hi = hi_c;
    uint64_t mv;
    if constexpr (LANE_MOVE) {
      static_assert(EDGE_MASKS && CPL == 2, "the lane-compare move keeps two-slot edge masks");
      /* the previous band of an interior band lies wholly inside the table,
       * so both its end cells are finite (each of its cells has its up or
       * left neighbour in the band before): the alternation for two -inf
       * end cells never applies, and odd bands compare as even ones */
      const uint64_t cm = ((b & 1) && !INTERIOR) ? sk_cmp_lane<true>(lo, hv, NFM) : sk_cmp_lane<false>(lo, hv, NFM);
      mv = sk_move_edges2(cm, __builtin_amdgcn_readfirstlane(hl), edge, K);
    } else {
      mv = (b & 1) ? sk_move_mask<true>(lo, hi, NFM) : sk_move_mask<false>(lo, hi, NFM);
      const int mneg = __builtin_amdgcn_readfirstlane((int)(uint32_t)mv);
      K -= mneg;
      if constexpr (EDGE_MASKS) edge_move<CPL>(edge, mneg);
    }
    if constexpr (CPL == 2) {
      /* a k-mer move changes the parity of both end slots */
      plo ^= mv;
      if constexpr (!W_EVEN) phi ^= mv;
    }

    /* cells of band i inside the band and the table: k-mers kv with
     * wlo <= kv < wlo + wlen (one unsigned compare against the SGPR wlo) */
    int wlo = K, wlen = W;
    if constexpr (!INTERIOR) {
      const int klo = max(K, max(0, i - 1 - n_e));
      const int khi = min(K + W - 1, min(n_k - 1, i - 2));
      wlen = max(0, khi - klo + 1);
      wlo = klo;
      cells += (uint64_t)wlen;
    }
    /* slot s-1 of a register's first slot is the last register of lane l-1:
     * left (e, k-1) in band i-1 and diag (e-1, k-1) in band i-2, each with
     * its move's constant added */
    float lf0, dg0;
    add_rot2(Sp[CPL - 1], lp_skip_v, Spp[CPL - 1], lp_step_v, lf0, dg0);
    float nv[CPL]; /* band i; band i-2 is still read below */
    float sv[CPL]; /* band i before the window mask */
    /* trim, in bands with cells outside the table: the first k-mer takes no
     * skip from the trim column (while the previous band may hold it), and
     * the trim cell (i-1, -1) of this band (while the band holds k-mer -1) */
    bool no_skip_in = false, trim_cell = false;
    if constexpr (!INTERIOR && TRIM) {
      no_skip_in = K <= 0;
      trim_cell = K <= -1 && i - 1 <= n_e - 1;
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const float x = X[c];
      const float up = Sp[c]; /* up (e-1, k): band i-1, slot s */
      /* left + lp_skip and diag + lp_step */
      const float lsk = (c == 0) ? lf0 : Sp[c - 1] + lp_skip;
      const float dst = (c == 0) ? dg0 : Spp[c - 1] + lp_step;
      /* Alg. 5.3 log-emission and Alg. 5.2 cell score */
      const float d = x - PM[c];
      const float t = d * d;
      const float u = t * PH[c];
      const float em = PC[c] - u;
      const float sd = dst + em;
      const float su = (up + lp_stay) + em;
      float sl = lsk;
      if constexpr (!INTERIOR && TRIM) {
        if (no_skip_in) sl = sel(sl, NI, ballot(kvs[c] == 0));
      }
      /* first maximum in the order D, U, L.  The value is the plain maximum
       * (scores are finite or -inf, never NaN or -0, so v_max3 gives the
       * bits of the first-maximum selects).  The trace bits say which
       * candidates equal it: D won iff sd is the maximum; otherwise U won iff
       * su is; otherwise L.  The compares stay off the chain from one band
       * to the next */
      sv[c] = vmax3(sd, su, sl);
      const uint64_t md = ballot(sv[c] == sd);
      const uint64_t mu = ballot(sv[c] == su);
      if constexpr (EDGE) {
        /* only the two slots beside the band are cleared: the next two bands
         * read no other slot outside this band (the others may hold any
         * value, the scores of k-mers outside the band) */
        nv[c] = sel(sv[c], NI, edge[c]);
      } else {
        const uint64_t valid = ballot((uint32_t)(kvs[c] - wlo) < (uint32_t)wlen);
        nv[c] = sel(NI, sv[c], valid);
        if constexpr (!INTERIOR && TRIM) {
          if (trim_cell) nv[c] = sel(nv[c], up + lp_trim, ballot(kvs[c] == -1));
        }
      }
      /* trace planes: the D bit, and the U bit (read only when D is clear) */
      if (fresh && c == 0) {
        TD = first_bit(md);
        TU = first_bit(mu);
      } else {
        TD = shift_in(TD, md);
        TU = shift_in(TU, mu);
      }
    }
    /* the end cells of this band for the next band's move.  Both lie in the
     * band; inside the table they are never masked, so they are read from
     * the unmasked scores, which keeps the window mask off the chain from
     * one band's move to the next */
    {
      const float(&src)[CPL] = INTERIOR ? sv : nv;
      const int sf = K & (N - 1);
      const int sh = (K + W - 1) & (N - 1);
      if constexpr (CPL == 2) {
        /* register of each end slot from its parity, as wave masks kept on
         * the SALU */
        lo_c = __builtin_amdgcn_readlane(__float_as_int(sel(src[0], src[1], plo)), sf >> LC);
        if constexpr (LANE_MOVE) {
          hv = W_EVEN ? sel(src[1], src[0], plo) : sel(src[0], src[1], phi);
          hl = sh >> LC;
        } else {
          hi_c = __builtin_amdgcn_readlane(__float_as_int(sel(src[0], src[1], phi)), sh >> LC);
        }
      } else if constexpr (CPL == 4) {
        lo_c = end_cell_bits4(src, sf);
        hi_c = end_cell_bits4(src, sh);
      } else {
        lo_c = __builtin_amdgcn_readlane(__float_as_int(pick<CPL>(src, sf & (CPL - 1))), sf >> LC);
        hi_c = __builtin_amdgcn_readlane(__float_as_int(pick<CPL>(src, sh & (CPL - 1))), sh >> LC);
      }
    }
    if constexpr (!INTERIOR && TRIM) {
      /* trim: band i holds (i-1-n_k, n_k-1) if it holds the last k-mer */
      if (i >= n_k + 1) {
        const float s_end =
            (n_k - 1 >= K && n_k - 1 <= K + W - 1) ? read_slot<CPL>(nv, (n_k - 1) & (N - 1)) : ABEA_NINF;
        const float t = end_best + lp_trim;
        if (t > s_end) {
          end_best = t;
        } else {
          end_best = s_end;
          end_u = i - 1 - n_k;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) Spp[c] = nv[c];
  };

  /* A full group of G bands from band i: slot refill every RF bands; the
   * events of the next band pair are read from LDS while the current pair
   * computes (the scheduling barrier keeps the reads ahead). */
  auto group = [&](auto interior_tag, int i) {
    float xa[2][CPL], xn[2][CPL];
    refill(i, 0);
    load_x(xa[0], 0);
    load_x(xa[1], 1);
#pragma unroll
    for (int b = 0; b < G; b += 2) {
      const bool ahead = (b + 2 < G) && ((b + 2) % RF != 0);
      if (ahead) {
        load_x(xn[0], b + 2);
        load_x(xn[1], b + 3);
      }
      __builtin_amdgcn_sched_barrier(0);
      band(interior_tag, Spp, Sp, i + b, b, xa[0], b == 0);
      band(interior_tag, Sp, Spp, i + b + 1, b + 1, xa[1], false);
      if (b + 2 < G) {
        if ((b + 2) % RF == 0) {
          refill(i + b + 2, b + 2);
          load_x(xa[0], b + 2);
          load_x(xa[1], b + 3);
        } else {
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            xa[0][c] = xn[0][c];
            xa[1][c] = xn[1][c];
          }
        }
      }
    }
  };

  /* Full groups of G bands (band i = 2 + t, group t / G): ring refill and
   * interior test once per group, one trace word per lane per group. */
  int i = 2;
  uint64_t g = 0;
  const bool gap_ok = N - W >= CPL; /* interior bands clear CPL slots outside the band */
  while (i + G - 1 <= last) {
    K = __builtin_amdgcn_readfirstlane(K);
    E = i - 3 - K; /* band i - 1 is the latest */
    advance_rings();
    /* with trim the last k-mer stays out of interior bands, whose cells the
     * end recurrence does not read */
    const bool interior = gap_ok & (K >= 0) & (E >= W - 1) & (E + G <= n_e - 1) &
                          (K + G + W - 1 <= n_k - 1 - (int)trim);
    if (interior) {
      group(std::true_type(), i);
      cells += (uint64_t)W * G;
    } else {
      group(std::false_type(), i);
    }
    trace[g * 64 + lane] = make_uint2(TD, TU);
    ++g;
    i += G;
  }
  /* the last, partial group */
  if (i <= last) {
    K = __builtin_amdgcn_readfirstlane(K);
    E = i - 3 - K;
    advance_rings();
    const int gb = last - i + 1;
    TD = 0;
    TU = 0;
    for (int b = 0;; b += 2) {
      if (b % RF == 0) refill(i + b, b);
      float x0[CPL], x1[CPL];
      load_x(x0, b);
      load_x(x1, b + 1);
      band(std::false_type(), Spp, Sp, i + b, b, x0, false);
      if (i + b + 1 > last) break;
      band(std::false_type(), Sp, Spp, i + b + 1, b + 1, x1, false);
      if (i + b + 2 > last) break;
    }
    i = last + 1;
    const int sh = (G - gb) * CPL;
    trace[g * 64 + lane] = make_uint2(TD << sh, TU << sh);
  }

  /* terminal cell (n_e-1, n_k-1) is in the last band if its k-mer is; with
   * trim the end cell the end recurrence chose */
  float sc = ABEA_NINF;
  e_end = n_e - 1;
  if constexpr (TRIM) {
    sc = end_best;
    e_end = end_u;
  } else {
    float F[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) F[c] = (last & 1) ? Sp[c] : Spp[c];
    if (n_k - 1 >= K && n_k - 1 <= K + W - 1) sc = read_slot<CPL>(F, (n_k - 1) & (N - 1));
  }
  /* every rank of the read has passed through the k-mer ring: one outside
   * the model makes the read's outcome a bad rank, with no alignment */
  if (ballot(bad_rank != 0u)) {
    if (lane == 0) {
      a.out_ll[rd.orig] = ABEA_NINF;
      if (a.out_cells) a.out_cells[rd.orig] = 0;
    }
    return READ_BAD_RANK;
  }
  if (lane == 0) {
    a.out_ll[rd.orig] = sc;
    if (a.out_cells) a.out_cells[rd.orig] = cells;
  }
  return (__float_as_int(sc) == ABEA_NINF_BITS) ? READ_BAND_LOST : READ_OK;
}

/* Outputs of a read whose band fill did not run (an empty read). */
__device__ __forceinline__ void band_skipped(const AlignArgs &a, const ReadDesc &rd) {
  if ((threadIdx.x & 63) == 0) {
    a.out_ll[rd.orig] = ABEA_NINF;
    if (a.out_cells) a.out_cells[rd.orig] = 0;
  }
}

/* Band fill alone, one wavefront per planned read. */
template <int CPL, int RPG, int EDGE, bool TRIM>
__global__ __launch_bounds__(64) void k_band(const AlignArgs a) {
  __shared__ WaveLds<CPL> lds;
  const int s = blockIdx.x;
  const ReadDesc rd = a.reads[s];
  if (a.rstat[s] != READ_OK) {
    band_skipped(a, rd);
    return;
  }
  /* the longest reads set the kernel's duration: let them issue first */
  const bool urgent = rd.n_e + rd.n_k >= a.urgent_len;
  if (urgent) __builtin_amdgcn_s_setprio(2);
  int e_end;
  const int st = band_read<CPL, RPG, EDGE, TRIM>(a, rd, a.trace + rd.tr_off, lds.band.lx, lds.band.lk, e_end);
  if (urgent) __builtin_amdgcn_s_setprio(0);
  if (threadIdx.x == 0) {
    a.rstat[s] = st;
    a.tend[s] = e_end;
  }
}

/* ------------------------------------------------------------- backtrack */

/* Bit of trace cell (band t, slot k) in its lane's 32-bit word: 31 - ((t mod
 * G) * CPL + k mod CPL), as (~((t << LC) + (k & (CPL - 1)))) & 31 in three
 * SALU instructions (the compiler would rebuild the five-instruction form). */
template <int CPL>
__device__ __forceinline__ int trace_bit(int t, int k) {
  int b;
  if constexpr (CPL == 1) {
    asm("s_andn2_b32 %0, 31, %1" : "=s"(b) : "s"(t));
  } else {
    int m;
    if constexpr (CPL == 2)
      asm("s_and_b32 %1, %3, 1\n\ts_lshl1_add_u32 %0, %2, %1\n\ts_andn2_b32 %0, 31, %0"
          : "=&s"(b), "=&s"(m) : "s"(t), "s"(k) : "scc");
    else if constexpr (CPL == 4)
      asm("s_and_b32 %1, %3, 3\n\ts_lshl2_add_u32 %0, %2, %1\n\ts_andn2_b32 %0, 31, %0"
          : "=&s"(b), "=&s"(m) : "s"(t), "s"(k) : "scc");
    else if constexpr (CPL == 8)
      asm("s_and_b32 %1, %3, 7\n\ts_lshl3_add_u32 %0, %2, %1\n\ts_andn2_b32 %0, 31, %0"
          : "=&s"(b), "=&s"(m) : "s"(t), "s"(k) : "scc");
    else
      asm("s_and_b32 %1, %3, 15\n\ts_lshl4_add_u32 %0, %2, %1\n\ts_andn2_b32 %0, 31, %0"
          : "=&s"(b), "=&s"(m) : "s"(t), "s"(k) : "scc");
  }
  return b;
}

/* The walk's move from its cell (t = e + k, k), whose trace bits sit at bit
 * `bit` of the lane's words: t falls by 1, and by 2 on a diagonal (D bit);
 * k falls unless the move is up (D bit, or no U bit: the word wk = D | ~U).
 * Each bit goes straight into SCC (s_bitcmp1) and one subtract with borrow
 * applies it: four SALU instructions. */
__device__ __forceinline__ void walk_move(int &t, int &k, uint32_t wd, uint32_t wk, int bit) {
  asm("s_bitcmp1_b32 %2, %4\n\t"
      "s_subb_u32 %0, %0, 1\n\t"
      "s_bitcmp1_b32 %3, %4\n\t"
      "s_subb_u32 %1, %1, 0"
      : "+s"(t), "+s"(k)
      : "s"(wd), "s"(wk), "s"(bit)
      : "scc");
}

/* Backtrack of one read (Alg. 5.1, after the band loop) by the calling
 * wavefront, from its trace tiles: writes the path's pairs backwards into
 * the read's scratch slots, its length and first slot, and its final status
 * (and -inf as log-likelihood if the walk fails).  The walk starts at
 * (e_start, n_k-1): (n_e-1, n_k-1), or with TRIM the end cell the band fill
 * chose; it ends at the origin, or with TRIM on reaching the trim column
 * k = -1 (whose cells are not pairs). */
template <int CPL, bool TRIM>
__device__ __forceinline__ void backtrack_read(const AlignArgs &a, const ReadDesc &rd, int status, int e_start,
                                               const uint2 *__restrict__ tr,
                                               uint2 *__restrict__ ring) {
  constexpr int N = 64 * CPL;
  constexpr int LC = Log2<CPL>::v;
  constexpr int LG = 5 - LC;           /* log2(G) */
  constexpr int G = 1 << LG;           /* bands per trace group */
  constexpr int RG = BT_RING_GROUPS;   /* tile groups in the LDS ring */
  constexpr int QG = RG / 4;           /* groups per refill quarter */

  const int lane = threadIdx.x & 63;
  const int orig = rd.orig;
  if (status != READ_OK) {
    if (lane == 0) {
      a.path_len[orig] = 0;
      a.path_src[orig] = 0;
      a.out_status[orig] = status;
    }
    return;
  }
  const int n_e = rd.n_e, n_k = rd.n_k;
  const int gmax = (n_e + n_k - 2) >> LG; /* last trace group of the read */
  auto ldt = [&](int grp) -> uint2 {
    uint2 v = make_uint2(0u, 0u);
    if (grp >= 0 && grp <= gmax) v = tr[(uint64_t)grp * 64 + lane];
    return v;
  };

  int e = __builtin_amdgcn_readfirstlane(e_start), k = n_k - 1;
  int gcur = (e + k) >> LG;
  /* quarters of QG groups, walked downwards: quarters qa, qa-1, qa-2 are in
   * the ring, qa-3 waits in registers */
  int qa = gcur / QG;
  for (int t = 0; t < 3; ++t)
    for (int p = 0; p < QG; ++p) {
      const int grp = (qa - t) * QG + p;
      ring[(grp & (RG - 1)) * 64 + lane] = ldt(grp);
    }
  uint2 pend[QG];
#pragma unroll
  for (int p = 0; p < QG; ++p) pend[p] = ldt((qa - 3) * QG + p);
  uint2 T = ring[(gcur & (RG - 1)) * 64 + lane];
  uint2 Tn = ring[((gcur - 1) & (RG - 1)) * 64 + lane];

  int PT = 0, PK = 0; /* gathered cells as t = e + k and k */
  uint64_t q = 0;      /* cells stored */
  uint32_t qn = 0;     /* cells gathered in lanes 0 .. qn-1, not stored yet */
  const uint64_t res_end = rd.pr_off + (uint64_t)(n_e + n_k - 1);
  int2 *__restrict__ out = a.scratch;
  bool ok = true;
  /* store the gathered cells in one coalesced store: lane l holds cell q + l
   * counted from the end of the read's slots */
  auto flush = [&]() {
    if (lane < (int)qn) out[res_end - 1 - (q + lane)] = make_int2(PT - PK, PK);
    q += qn;
    qn = 0;
  };

  for (;;) {
    /* the cells of the current group: one dependent step per cell, at most G
     * of them (t falls at every step), so the lanes are emptied before a
     * group that might not fit; the trace words of the lane the walk is in
     * stay in SGPRs until k leaves that lane's CPL k-mers */
    if (qn + G > 64) flush();
    const int lower = gcur << LG;
    int t = e + k;
    int klo = 0x7fffffff; /* first k-mer of the loaded lane (none yet) */
    uint32_t wd = 0, wk = 0; /* the lane's D-bit word, and its D | ~U word */
    for (;;) {
      t = __builtin_amdgcn_readfirstlane(t);
      k = __builtin_amdgcn_readfirstlane(k);
      PT = writelane(t, (int)qn, PT);
      PK = writelane(k, (int)qn, PK);
      ++qn;
      if (k < klo) {
        const int ln = (k & (N - 1)) >> LC;
        wd = rlane_u(T.x, ln);
        wk = wd | ~rlane_u(T.y, ln);
        klo = k & ~(CPL - 1);
      }
      /* diagonal (1,x): e-1, k-1; up (0,1): e-1; left (0,0): k-1 */
      walk_move(t, k, wd, wk, trace_bit<CPL>(t, k));
      /* stop when the walk left the group (t falls by 1 or 2 per step, so
       * this also ends a walk that leaves the table; the caller checks that
       * it ended at the origin), or with TRIM entered the trim column */
      if (t < lower) break;
      if constexpr (TRIM) {
        if (k < 0) break;
      }
    }
    e = t - k;
    if ((e | k) < 0) break;
    const int gi = t >> LG;
    if (gi != gcur) { /* the walk moved down by one group */
      gcur = gi;
      T = Tn;
      if (gcur - 1 < (qa - 1) * QG) {
        --qa;
#pragma unroll
        for (int p = 0; p < QG; ++p) ring[(((qa - 2) * QG + p) & (RG - 1)) * 64 + lane] = pend[p];
#pragma unroll
        for (int p = 0; p < QG; ++p) pend[p] = ldt((qa - 3) * QG + p);
      }
      Tn = ring[((gcur - 1) & (RG - 1)) * 64 + lane];
    }
  }
  flush();
  if (ok && !(TRIM ? (k == -1 && e >= -1) : (e == -1 && k == -1))) ok = false;
  if (lane == 0) {
    a.path_len[orig] = ok ? q : 0;
    a.path_src[orig] = res_end - q;
    a.out_status[orig] = ok ? READ_OK : READ_BAND_LOST;
    if (!ok) a.out_ll[orig] = ABEA_NINF;
  }
}

/* Backtrack alone, one wavefront per planned read. */
template <int CPL, bool TRIM>
__global__ __launch_bounds__(64) void k_backtrack(const AlignArgs a) {
  __shared__ WaveLds<CPL> lds;
  const int s = blockIdx.x;
  const ReadDesc rd = a.reads[s];
  backtrack_read<CPL, TRIM>(a, rd, a.rstat[s], TRIM ? a.tend[s] : rd.n_e - 1, a.trace + rd.tr_off, lds.ring);
}

/* ----------------------------------------------------------------- fused */

/* Band fill and backtrack of a read by one wavefront, with a device work
 * queue.  Worker w (wavefront w of the grid, w < n_workers) first aligns
 * planned read w, then takes reads n_workers + q for q = 0, 1, ... from the
 * queue counter until they run out.  Reads are planned longest first, so
 * every later read fits the trace slab of the worker's first read: worker w
 * keeps read w's trace region for all its reads.  n_workers = n_reads is the
 * plain one-launch form; fewer workers bound the trace memory (admission by
 * traceback bytes) and let the longest reads of the batch overlap the rest. */
template <int CPL, int RPG, int WPG, int EDGE, bool TRIM>
__global__ __launch_bounds__(64 * WPG) void k_align(const AlignArgs a) {
  __shared__ WaveLds<CPL> lds[WPG];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = blockIdx.x * WPG + wv;
  if (w >= a.n_workers) return;
  uint2 *slab = a.trace + a.reads[w].tr_off;
  int s = w;
  while (s < a.n_reads) {
    const ReadDesc rd = a.reads[s];
    int st = a.rstat[s];
    /* the longest reads set the kernel's duration: let them issue first */
    const bool urgent = rd.n_e + rd.n_k >= a.urgent_len;
    if (urgent) __builtin_amdgcn_s_setprio(2);
    int e_end = rd.n_e - 1;
    if (st == READ_OK)
      st = band_read<CPL, RPG, EDGE, TRIM>(a, rd, slab, lds[wv].band.lx, lds[wv].band.lk, e_end);
    else
      band_skipped(a, rd);
    /* the walk reads back what this wavefront's lanes just stored (each lane
     * its own words); keep the compiler from moving loads above the stores */
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    backtrack_read<CPL, TRIM>(a, rd, st, e_end, slab, lds[wv].ring);
    if (urgent) __builtin_amdgcn_s_setprio(0);
    asm volatile("" ::: "memory");
    uint32_t q = 0;
    if ((threadIdx.x & 63) == 0) q = atomicAdd(a.queue, 1u);
    s = a.n_workers + (int)__builtin_amdgcn_readfirstlane(q);
  }
}

/* ------------------------------------------------------- scan + compact */

/* Both kernels run as single-wavefront workgroups: while other batches'
 * alignment waves hold the chip, a one-wave group takes the first free wave
 * slot, where a multi-wave group would wait for a CU with that many free
 * slots at once. */
__global__ __launch_bounds__(64) void k_scan(const uint64_t *__restrict__ len, int n,
                                             uint64_t *__restrict__ off) {
  const int lane = threadIdx.x;
  const int per = (n + 63) >> 6;
  const int lo = min(n, lane * per);
  const int hi = min(n, lo + per);
  uint64_t sum = 0;
  for (int r = lo; r < hi; ++r) sum += len[r];
  uint64_t inc = sum; /* inclusive scan of the 64 lane sums */
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t v = __shfl_up(inc, d, 64);
    if (lane >= d) inc += v;
  }
  uint64_t run = inc - sum;
  for (int r = lo; r < hi; ++r) {
    off[r] = run;
    run += len[r];
  }
  if (lane == 63) off[n] = inc;
}

/* Read r's pairs (a contiguous run in the scratch, in path order) to its
 * place in the caller's array: COMPACT_SPLIT wavefronts per read, wavefront
 * y copying the y-th slice, so that the longest reads do not leave one
 * wavefront copying megabytes at the end of the kernel. */
constexpr int COMPACT_SPLIT = 8;
__global__ __launch_bounds__(64) void k_compact(const int2 *__restrict__ scratch,
                                                const uint64_t *__restrict__ src,
                                                const uint64_t *__restrict__ off,
                                                int2 *__restrict__ pairs) {
  const int r = blockIdx.x;
  const uint64_t o = off[r];
  const uint64_t n = off[r + 1] - o;
  /* slices in whole 64-pair steps */
  const uint64_t steps = (n + 63) >> 6;
  const uint64_t s0 = steps * blockIdx.y / COMPACT_SPLIT, s1 = steps * (blockIdx.y + 1) / COMPACT_SPLIT;
  const uint64_t end = min(n, s1 << 6);
  const int2 *__restrict__ in = scratch + src[r];
  int2 *__restrict__ out = pairs + o;
  uint64_t t = (s0 << 6) + threadIdx.x;
  /* eight loads in flight per lane */
  for (; t + 448 < end; t += 512) {
    int2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = in[t + 64 * j];
#pragma unroll
    for (int j = 0; j < 8; ++j) out[t + 64 * j] = v[j];
  }
  for (; t < end; t += 64) out[t] = in[t];
}

/* ------------------------------------------------------------- launchers */

hipError_t launch_prep(const ReadDesc *reads, int n_planned, const float *events, int ev_stride,
                       const uint32_t *ranks, const uint64_t *in_addr, const float *scale,
                       const float *shift, bool scale_events, float *xmean, uint32_t *krank,
                       int32_t *rstat, uint32_t *queue, hipStream_t st) {
  if (n_planned <= 0) return hipSuccess;
  /* one wavefront per read when there is nothing to stage */
  const int threads = (xmean || krank) ? 256 : 64;
  hipLaunchKernelGGL(k_prep, dim3(n_planned), dim3(threads), 0, st, reads, events, ev_stride, ranks, in_addr,
                     scale, shift, (int)scale_events, xmean, krank, rstat, queue);
  return hipGetLastError();
}

/* Kernel variant for (cells per lane, refills per group, edge clearing). */
/* the third argument is the clearing form (band_read's CLEAR); w_odd is the
 * parity of W */
#define ABEA_VARIANTS(CALL)                                          \
  if (cpl == 1 && rpg == 1 && !edge) CALL(1, 1, 0);                  \
  if (cpl == 1 && rpg == 2 && !edge) CALL(1, 2, 0);                  \
  if (cpl == 2 && rpg == 1 && !edge) CALL(2, 1, 0);                  \
  if (cpl == 2 && rpg == 2 && !edge) CALL(2, 2, 0);                  \
  if (cpl == 2 && rpg == 1 && edge && w_odd) CALL(2, 1, 1);          \
  if (cpl == 2 && rpg == 2 && edge && w_odd) CALL(2, 2, 1);          \
  if (cpl == 2 && rpg == 1 && edge && !w_odd) CALL(2, 1, 2);         \
  if (cpl == 2 && rpg == 2 && edge && !w_odd) CALL(2, 2, 2);         \
  if (cpl == 4 && rpg == 1 && !edge) CALL(4, 1, 0);                  \
  if (cpl == 4 && rpg == 2 && !edge) CALL(4, 2, 0);                  \
  if (cpl == 4 && rpg == 1 && edge) CALL(4, 1, 1);                   \
  if (cpl == 4 && rpg == 2 && edge) CALL(4, 2, 1);                   \
  if (cpl == 8 && rpg == 1 && !edge) CALL(8, 1, 0);                  \
  if (cpl == 8 && rpg == 2 && !edge) CALL(8, 2, 0);                  \
  if (cpl == 16 && rpg == 1 && !edge) CALL(16, 1, 0);

hipError_t launch_band(const AlignArgs &a, int cpl, int rpg, bool edge, hipStream_t st, hipEvent_t t0,
                       hipEvent_t t1) {
  if (a.n_reads <= 0) return hipSuccess;
  const bool w_odd = (a.W & 1) != 0;
#define ABEA_L(C, R, E)                                                                                 \
  {                                                                                                     \
    if (a.trim)                                                                                         \
      hipExtLaunchKernelGGL((k_band<C, R, E, true>), dim3(a.n_reads), dim3(64), 0, st, t0, t1, 0, a);  \
    else                                                                                                \
      hipExtLaunchKernelGGL((k_band<C, R, E, false>), dim3(a.n_reads), dim3(64), 0, st, t0, t1, 0, a); \
    return hipGetLastError();                                                                           \
  }
  ABEA_VARIANTS(ABEA_L)
#undef ABEA_L
  return hipErrorInvalidValue;
}

template <bool TRIM>
static hipError_t launch_backtrack_t(const AlignArgs &a, int cpl, hipStream_t st) {
  switch (cpl) {
    case 1: hipLaunchKernelGGL((k_backtrack<1, TRIM>), dim3(a.n_reads), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_backtrack<2, TRIM>), dim3(a.n_reads), dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_backtrack<4, TRIM>), dim3(a.n_reads), dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_backtrack<8, TRIM>), dim3(a.n_reads), dim3(64), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_backtrack<16, TRIM>), dim3(a.n_reads), dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_backtrack(const AlignArgs &a, int cpl, hipStream_t st) {
  if (a.n_reads <= 0) return hipSuccess;
  return a.trim ? launch_backtrack_t<true>(a, cpl, st) : launch_backtrack_t<false>(a, cpl, st);
}

template <int CPL, int RPG, int EDGE, bool TRIM>
static hipError_t launch_align_c(const AlignArgs &a, int wpg, hipStream_t st, hipEvent_t t0,
                                 hipEvent_t t1) {
  const dim3 grid((a.n_workers + wpg - 1) / wpg);
  switch (wpg) {
    case 1: hipExtLaunchKernelGGL((k_align<CPL, RPG, 1, EDGE, TRIM>), grid, dim3(64), 0, st, t0, t1, 0, a); break;
    case 2: hipExtLaunchKernelGGL((k_align<CPL, RPG, 2, EDGE, TRIM>), grid, dim3(128), 0, st, t0, t1, 0, a); break;
    case 4: hipExtLaunchKernelGGL((k_align<CPL, RPG, 4, EDGE, TRIM>), grid, dim3(256), 0, st, t0, t1, 0, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_align(const AlignArgs &a, int cpl, int rpg, int wpg, bool edge, hipStream_t st,
                        hipEvent_t t0, hipEvent_t t1) {
  if (a.n_reads <= 0 || a.n_workers <= 0) return hipSuccess;
  if (a.n_workers > a.n_reads) return hipErrorInvalidValue;
  const bool w_odd = (a.W & 1) != 0;
#define ABEA_L(C, R, E)                                                                                       \
  return a.trim ? launch_align_c<C, R, E, true>(a, wpg, st, t0, t1) : launch_align_c<C, R, E, false>(a, wpg, st, t0, t1)
  ABEA_VARIANTS(ABEA_L)
#undef ABEA_L
  return hipErrorInvalidValue;
}

template <int CPL, int RPG, int EDGE, bool TRIM>
static int groups_per_cu_c(int wpg) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (wpg) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_align<CPL, RPG, 1, EDGE, TRIM>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_align<CPL, RPG, 2, EDGE, TRIM>, 128, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_align<CPL, RPG, 4, EDGE, TRIM>, 256, 0); break;
  }
  return e == hipSuccess ? n : 0;
}

int align_groups_per_cu(int cpl, int rpg, int wpg, bool edge, bool trim, int W) {
  const bool w_odd = (W & 1) != 0;
#define ABEA_L(C, R, E) return trim ? groups_per_cu_c<C, R, E, true>(wpg) : groups_per_cu_c<C, R, E, false>(wpg)
  ABEA_VARIANTS(ABEA_L)
#undef ABEA_L
  return 0;
}

/* the plan from mapped pinned host memory into device memory, one thread per
 * read */
__global__ __launch_bounds__(256) void k_stage_plan(const ReadDesc *__restrict__ src, ReadDesc *__restrict__ dst,
                                                    int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_stage_plan(const ReadDesc *src, ReadDesc *dst, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_stage_plan, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_scan(const uint64_t *len, int n, uint64_t *offset, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, len, n, offset);
  return hipGetLastError();
}

hipError_t launch_compact(const int2 *scratch, const uint64_t *path_src, const uint64_t *offset,
                          int n, int2 *pairs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3(n, COMPACT_SPLIT), dim3(64), 0, st, scratch, path_src, offset, pairs);
  return hipGetLastError();
}

/* ------------------------------------------------ fixed device scratch */

/* Scratch of the no-allocation entry point: one array per device, held from
 * the library's load until the process ends.  Host code must not pass this
 * name to a kernel or a copy (in host code it is a host-side stand-in, not a
 * device address); it uses the address noalloc_scratch() returns. */
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void **ptr) {
  /* hipGetSymbolAddress once per device, with that device current (the
   * caller has made it current), kept for the life of the process */
  static std::mutex mu;
  static void *addr[NOALLOC_MAX_DEVICES] = {};
  *ptr = nullptr;
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

}  // namespace abea
