/*
 * abea_internal.h -- layout shared by the host runtime and the gfx950 kernels
 * of libabea.so.  Not installed; not part of the C ABI.
 */
#ifndef ABEA_INTERNAL_H
#define ABEA_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abea {

/* One read as planned by the host (reads are sorted longest first; the
 * kernels process planned position s = blockIdx.x). */
struct ReadDesc {
  uint64_t ev_off;  /* first event of the read in the batch event table */
  uint64_t km_off;  /* first k-mer of the read */
  uint64_t tr_off;  /* first trace tile word (uint2 units) */
  uint64_t spare;
  uint64_t pr_off;  /* first slot of the read's pair scratch (n_e+n_k-1 slots) */
  int32_t n_e;
  int32_t n_k;
  float lp_skip;
  float lp_stay;
  float lp_step;
  int32_t orig; /* index of the read in the caller's batch */
};
static_assert(sizeof(ReadDesc) == 64, "ReadDesc is one 64-byte line");

/* Pore-model entry on the device: scaled-free mean, emission constant
 * c = ln(1/sqrt(2 pi)) - ln(sigma) and h = 0.5/sigma^2. */
struct ModelEntry {
  float mean;
  float c;
  float h;
  float pad;
};


enum : int32_t { READ_OK = 0, READ_EMPTY = 1, READ_BAND_LOST = 2, READ_BAD_RANK = 3 };

/* Bands per trace tile word: every lane packs cpl slots x 1 bit per band into
 * a 32-bit word per bit plane. */
inline int bands_per_group(int cpl) { return 32 / cpl; }

/* The band fill relabels its slots rpg times per group of bands, every
 * 32/cpl/rpg bands; a k-mer that leaves the band keeps its slot until then,
 * so 64*cpl - W must be at least that interval (see band_read). */
inline bool band_shape_ok(int W, int cpl, int rpg) {
  const int rf = bands_per_group(cpl) / rpg;
  return rf >= 2 && 64 * cpl - W >= rf;
}
/* Refills per group for W and cpl: 1 if it fits, else 2, else 0 (no fit). */
inline int refills_per_group(int W, int cpl) {
  if (band_shape_ok(W, cpl, 1)) return 1;
  if (band_shape_ok(W, cpl, 2)) return 2;
  return 0;
}
/* Slots per lane for a band width: the smallest power of two that fits. */
inline int cells_per_lane(int W) {
  int c = 1;
  while (c < 16 && refills_per_group(W, c) == 0) c <<= 1;
  return c;
}

/* Trace-tile groups held in a wavefront's LDS ring during the backtrack. */
constexpr int BT_RING_GROUPS = 16;

/* Arguments of the band, backtrack and fused alignment kernels. */
struct AlignArgs {
  const ReadDesc *reads; /* [n_reads] planned reads, longest first */
  /* event means: read in place from the batch's event records (xstride
   * floats apart, the caller's device array), or the means k_prep staged
   * (xstride 1) when the reads' inputs sit at addresses of their own or the
   * events are scaled to the model */
  const float *xsrc;
  int32_t xstride;
  /* k-mer ranks: the batch's, read in place, or the copy k_prep staged; the
   * band fill gathers each one's model entry and scales it per read */
  const uint32_t *ranks;
  const ModelEntry *model;
  uint32_t n_model;
  int32_t scale_events;  /* events scaled to the model: the model levels stay unscaled */
  const float *scale;    /* [caller reads] */
  const float *shift;    /* [caller reads] */
  int32_t *rstat;        /* [n_reads] status from k_prep; k_band writes the band outcome */
  uint2 *trace;          /* bit-plane trace tiles: 64 lanes x uint2 per group of bands */
  int2 *scratch;         /* reversed-path pair scratch */
  uint64_t *path_len;    /* [caller reads] by original index */
  uint64_t *path_src;    /* [caller reads] by original index: first scratch slot of the path */
  float *out_ll;         /* [caller reads] by original index */
  uint64_t *out_cells;   /* [caller reads] by original index, or null */
  int32_t *out_status;   /* [caller reads] by original index */
  uint32_t *queue;       /* fused kernel: work-queue counter, zeroed by k_prep */
  int32_t n_reads;       /* planned reads */
  int32_t n_workers;     /* fused kernel: wavefronts; worker w starts with read w */
  int32_t W;
  int32_t urgent_len;    /* reads with n_e + n_k >= this run at raised wave priority */
  int32_t *tend;         /* [n_reads] split kernels: the event of each read's end cell (trim) */
  float lp_trim;         /* trim states: ln(1/100) per trimmed event */
  int32_t trim;          /* trim states on (leading and trailing events may stay unaligned) */
};

/* Kernel launchers (abea_kernels.hip). */
/* in_addr: null, or per original read index r the device addresses of its
 * event means (in_addr[2r], one float per event) and ranks (in_addr[2r+1]),
 * used instead of the batch arrays. */
/* k_prep sets each planned read's status (empty or not; the band fill finds
 * bad ranks), zeroes the work-queue counter and stages what the band fill
 * cannot read in place:
 * xmean: null, or where to stage the event means (scaled to the model as
 *   (x - shift)/scale when scale_events);
 * krank: null, or where to copy the ranks (for inputs at per-read addresses). */
/* ev_stride: floats from one event mean to the next in `events` (3 for the
 * 12-byte event records, 1 for a compact array of means) */
hipError_t launch_prep(const ReadDesc *reads, int n_planned, const float *events, int ev_stride,
                       const uint32_t *ranks, const uint64_t *in_addr, const float *scale,
                       const float *shift, bool scale_events, float *xmean, uint32_t *krank,
                       int32_t *rstat, uint32_t *queue, hipStream_t st);
/* t0, t1: null, or events that take the start and end time of the kernel's
 * own dispatch.  edge: interior bands clear only the two slots beside the
 * band (cpl 2 or 4), else every slot outside the band's cells */
hipError_t launch_band(const AlignArgs &a, int cpl, int rpg, bool edge, hipStream_t st,
                       hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_backtrack(const AlignArgs &a, int cpl, hipStream_t st);
/* fused band + backtrack with a.n_workers wavefronts, wpg per workgroup */
hipError_t launch_align(const AlignArgs &a, int cpl, int rpg, int wpg, bool edge, hipStream_t st,
                        hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
/* resident workgroups of the fused kernel per CU (occupancy) for band width W */
int align_groups_per_cu(int cpl, int rpg, int wpg, bool edge, bool trim, int W);
hipError_t launch_scan(const uint64_t *len, int n, uint64_t *offset, hipStream_t st);
/* dst[0, n) = src[0, n) by a kernel (src: the plan in mapped pinned host memory) */
hipError_t launch_stage_plan(const ReadDesc *src, ReadDesc *dst, int n, hipStream_t st);

/* Fixed scratch of the no-allocation entry point (abea_kernels.hip). */
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
/* The device address of `device`'s scratch array (hipGetSymbolAddress on
 * the first call for that device, which must be the current device). */
hipError_t noalloc_scratch(int device, void **ptr);
hipError_t launch_compact(const int2 *scratch, const uint64_t *path_src, const uint64_t *offset,
                          int n, int2 *pairs, hipStream_t st);

/* ---- event detection (abea_detect.hip) ---- */
constexpr int ED_TILE = 1024;       /* boundaries per tile of one read */
constexpr int ED_MAX_WINDOW = 16;   /* largest detector window */

/* One tile of event detection: its read, where the read's samples start,
 * the read's length, the tile's first boundary in the read and the end of
 * the read's tiles. */
struct EdTile {
  uint64_t s0;
  uint32_t n;
  uint32_t i0;
  uint32_t read;
  uint32_t g_end;
};
static_assert(sizeof(EdTile) == 24, "EdTile is 24 bytes");

struct DetectArgs {
  const int16_t *raw;            /* the batch's samples, concatenated */
  const uint64_t *sample_offset; /* [n_reads+1] */
  const uint32_t *tile_first;    /* [n_reads+1]: first tile of each read (ceil(n/ED_TILE) tiles) */
  EdTile *tiles;                 /* [n_tiles], made by the first launch from the two above */
  const float *offset;           /* [n_reads] pA = (raw + offset) * pa_scale */
  const float *pa_scale;         /* [n_reads] */
  int32_t n_reads;
  uint32_t n_tiles;
  int32_t w_short, w_long;       /* detector windows */
  float thr_short, thr_long;     /* squared t thresholds */
  uint64_t *flags;               /* [n_tiles * ED_TILE/64]: one bit per boundary, set at change points */
  uint32_t *count;               /* [n_tiles]: events starting in the tile */
  int32_t *first_cp;             /* [n_tiles]: the tile's first change point, -1 if none */
  uint64_t *base;                /* [n_tiles]: first event of the tile within its scan block */
  uint64_t *block_sum;           /* [blocks+1]: first event of each scan block, then the total */
  float *events;                 /* [capacity][3]: mean, stdv, duration */
  uint64_t capacity;
  uint64_t *event_offset;        /* [n_reads+1] */
};
/* Blocks of the tile-count scan for n_tiles tiles. */
uint32_t ed_scan_blocks(uint32_t n_tiles);
/* Detection of a planned batch: change points, the scan of the event counts,
 * the events (those beyond a.capacity are not written) and event_offset.
 * tev: null, or six events: start and end of k_ed_detect's dispatch, of
 * k_ed_events's, and before and after the whole batch. */
hipError_t launch_detect(const DetectArgs &a, hipStream_t st, hipEvent_t *tev = nullptr);

/* ---- methylation scoring (abea_meth.hip) ---- */
/* One read of a batch to score, in the caller's order. */
struct MethRead {
  uint64_t ev_off; /* first event of the read in the batch */
  uint64_t km_off; /* first k-mer of the read in the batch */
  int32_t n_k;
  float lp_skip, lp_stay, lp_step; /* the read's transition constants (Alg. 5.2) */
};
static_assert(sizeof(MethRead) == 32, "MethRead is 32 bytes");

constexpr int METH_CHUNK = 8192; /* pairs or k-mers of one read per workgroup */

/* One workgroup's share of a read: its chunk-th run of METH_CHUNK pairs (or
 * k-mers) */
struct MethTile {
  uint32_t read;
  uint32_t chunk;
};
static_assert(sizeof(MethTile) == 8, "MethTile is 8 bytes");

struct MethArgs {
  const MethRead *reads;       /* [n_reads] */
  int32_t n_reads;
  int32_t k;
  uint64_t n_kmers;            /* of the batch */
  const MethTile *pair_tiles;  /* [n_pair_tiles]: ceil((n_e + n_k - 1) / METH_CHUNK) per read, a bound of its pairs */
  const MethTile *kmer_tiles;  /* [n_kmer_tiles]: ceil(n_k / METH_CHUNK) per read */
  uint32_t n_pair_tiles, n_kmer_tiles;
  const float *events;         /* the batch's event records (ev_stride floats apart) */
  int32_t ev_stride;
  int32_t scale_events;        /* events scaled to the model instead of the model to the events */
  const uint32_t *ranks;
  const float *scale, *shift;  /* [n_reads] */
  const ModelEntry *model;      /* the pore model */
  const ModelEntry *meth_model; /* the methylated model */
  const int2 *pairs;           /* the batch's alignment: pairs, pair_offset [n_reads+1], status */
  const uint64_t *pair_offset;
  const int32_t *status;
  int32_t *kfirst, *klast;     /* [n_kmers]: first and last event paired with each k-mer */
  uint2 *sites;                /* [n_kmers]: (read, k-mer) of each site, in no particular order */
  uint32_t *n_sites;           /* zeroed before the launch */
  float *llr;                  /* [n_kmers] */
  int32_t *n_ev;               /* [n_kmers] or null */
};
/* tev: null, or four events: start of k_meth_bounds's dispatch and end of
 * k_meth_sites's, start and end of k_meth_llr's. */
hipError_t launch_meth(const MethArgs &a, hipStream_t st, hipEvent_t *tev = nullptr);
/* dst[0, words) = src[0, words) (src: device-readable pinned host memory)
 * and *n_sites = 0, by a kernel on `st` */
hipError_t launch_meth_stage(const uint64_t *src, uint64_t *dst, size_t words, uint32_t *n_sites, hipStream_t st);

}  // namespace abea

#endif
