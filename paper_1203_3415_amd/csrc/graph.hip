// Ingest, validation and typed-G* build on the device.
//
// Paper, Section "Notation and definitions" and Algorithm "Create A,B,C sets"
// (the O(m) partition of each vertex's neighbours into A^v bidirected, B^v
// outgoing-only and C^v incoming-only), realised as one typed, id-sorted
// neighbour list per vertex of the undirected version G*, plus the oriented
// lists N+(v) = { w in N(v) : (d*(v), v) < (d*(w), w) } that make every edge of
// G* appear in exactly one list (the degree ordering behind the triangle
// listing the paper cites for Algorithm "alternative").
//
// Pipeline (all kernels; one host wait at the end of validation, done by the
// caller):
//   offsets check -> arc check + in-degree count -> half-edge offsets (scan)
//   -> half-edge scatter (key = id<<1 | dir) -> per-row sort (small rows in
//   registers, mid rows by LDS bitonic sort, long rows by a bitmap over the
//   key space) -> merge of equal ids into typed entries -> G* offsets (scan)
//   -> G* write -> N+ flags, scan, write -> optional in-CSR transpose check.
// A single graph given with an in-CSR whose rows, like the out-CSR's, are
// strictly increasing skips the count, scatter and sort: each row's two
// halves are merged in place, and the in-CSR is checked on the way.  The
// scans are single-pass look-back scans whose values come from functors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "scan.h"

namespace motif {

namespace {

constexpr int kB = 256;           // threads per block for streaming kernels
constexpr int kSmallRow = 64;     // rows up to this length: sorted by one thread, in registers
constexpr int kMidRow = 4096;     // rows up to this length: LDS bitonic sort
constexpr int kWaveRow = 1024;    // ... by one wave when at most this long, else by the workgroup
constexpr int kLdsBitmapWords = 16384;  // big rows: the key bitmap sits in LDS when 2n bits fit in 64 KB
constexpr int kLdsBitmapRow = 256;  // ... and then takes every row longer than this
constexpr int kLdsBitmapBlock = 1024;  // threads of an LDS bitmap sort
constexpr int kLdsBitmapGrid = 512;    // LDS bitmap sorts in flight (two 64 KB workgroups per CU)
constexpr int kBigSlots = 32;     // concurrent bitmap sorts with the bitmaps in global memory
constexpr int kCheckGrid = 256;   // workgroups of an in-CSR check run beside a census

__device__ __forceinline__ void set_status(int32_t* st, int32_t code) { atomicMin(&st[kStatus], code); }

__device__ __forceinline__ int32_t row_of(const int32_t* off, int32_t n, int64_t i) {
  // last v in [0, n) with off[v] <= i (off valid, off[n] > i)
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Arcs are taken kArcsPerThread consecutive ones per thread: one binary
// search for the row of the first, then a forward walk over the offsets.
constexpr int kArcsPerThread = 8;
constexpr int kPlaceArcs = 2;  // elements per thread of the sorted-input placement

__device__ __forceinline__ bool rank_less(int32_t dv, int32_t v, int32_t dw, int32_t w) {
  return dv < dw || (dv == dw && v < w);
}

// ---------------------------------------------------------------- helpers --

__global__ void k_zero(uint32_t* p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_zero16(uint4* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The regions of a ZeroBatch: a 16-byte part and a tail of at most 3 words.
struct ZeroRanges {
  uint4* p16[ZeroBatch::kMax];
  size_t n16[ZeroBatch::kMax];
  uint32_t* tail[ZeroBatch::kMax];
  int32_t ntail[ZeroBatch::kMax];
  int32_t n;
};


__global__ void k_zero_many(ZeroRanges r) {
  const size_t stride = (size_t)gridDim.x * blockDim.x, t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (int k = 0; k < r.n; ++k) {
    for (size_t i = t; i < r.n16[k]; i += stride) r.p16[k][i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < (size_t)r.ntail[k]) r.tail[k][t] = 0u;
  }
}

}  // namespace

namespace {

unsigned grid_for(int64_t items, int block = kB) {
  int64_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

// ------------------------------------------------------------- validation --

__global__ void k_check_offsets(const int32_t* off, int32_t n, int64_t m, int32_t* st) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = off[v];
    if (v == 0 && a != 0) set_status(st, MOTIF_EINVAL_SHAPE);
    if (v == n && (int64_t)a != m) set_status(st, MOTIF_EINVAL_SHAPE);
    if (v < n && off[v + 1] < a) set_status(st, MOTIF_EINVAL_SHAPE);
  }
}

// Every arc: index range, self-loop, in-degree count.
// Per-block aggregation of arc targets: a block takes kArcsPerBlock
// consecutive arcs, counts them per target in an LDS hash (kAggSlots keys, at
// most half full), and touches each target's global counter once.  Hubs with
// thousands of in-arcs then see one atomic per block instead of one per arc.
constexpr int kArcsPerBlock = kB * kArcsPerThread;
constexpr int kAggSlots = 2 * kArcsPerBlock;
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ int32_t agg_insert(uint32_t* keys, uint32_t d) {
  uint32_t h = (d * 2654435761u) & (kAggSlots - 1);
  for (;;) {
    const uint32_t old = atomicCAS(&keys[h], kAggEmpty, d);
    if (old == kAggEmpty || old == d) return (int32_t)h;
    h = (h + 1) & (kAggSlots - 1);
  }
}

__global__ __launch_bounds__(kB) void k_count_in(const int32_t* off, const int32_t* idx, int32_t n, int64_t m,
                                                 int32_t* in_cnt, int32_t* st, const int32_t* skip) {
  __shared__ uint32_t akey[kAggSlots];
  __shared__ int32_t acnt[kAggSlots];
  if (st[kStatus] != 0) return;
  if (skip && *skip == 0) {
    // every row was in order: the in-CSR lookups of the placement stand
    if (blockIdx.x == 0 && threadIdx.x == 0 && st[kInMismatch]) set_status(st, MOTIF_ETRANSPOSE);
    return;
  }
  for (int i = threadIdx.x; i < kAggSlots; i += kB) {
    akey[i] = kAggEmpty;
    acnt[i] = 0;
  }
  __syncthreads();
  for (int64_t b0 = (int64_t)blockIdx.x * kArcsPerBlock; b0 < m; b0 += (int64_t)gridDim.x * kArcsPerBlock) {
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kArcsPerThread, i1 = min(m, i0 + kArcsPerThread);
    if (i0 < m) {
      int32_t u = row_of(off, n, i0);
      for (int64_t i = i0; i < i1; ++i) {
        while (u < n - 1 && off[u + 1] <= i) ++u;  // bounded even if the offsets were not valid
        const int32_t d = idx[i];
        if (d < 0 || d >= n) { set_status(st, MOTIF_EINDEX); continue; }
        if (d == u) { set_status(st, MOTIF_ESELFLOOP); continue; }
        atomicAdd(&acnt[agg_insert(akey, (uint32_t)d)], 1);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggSlots; i += kB) {
      if (akey[i] != kAggEmpty) {
        atomicAdd(&in_cnt[akey[i]], acnt[i]);
        akey[i] = kAggEmpty;
        acnt[i] = 0;
      }
    }
    __syncthreads();
  }
}

// Half-edges of row v (out-degree + in-degree), the values whose exclusive
// scan gives the half-edge offsets; 0 at v = n.
struct HalfCount {
  const int32_t* off;
  const int32_t* in_cnt;
  int32_t n;
  __device__ int32_t operator()(int64_t v) const { return v < n ? (off[v + 1] - off[v]) + in_cnt[v] : 0; }
};

// Half-edge keys: row u gets (d<<1|0) for arc u->d, row d gets (u<<1|1).
// Half-edge scatter with the same per-block aggregation: each arc takes a
// local rank among the block's arcs to its target, one global atomic per
// (block, target) reserves the range, and the arc's slot is base + rank (the
// order inside a row is arbitrary; rows are sorted next).
__global__ __launch_bounds__(kB) void k_scatter(const int32_t* off, const int32_t* idx, int32_t n, int64_t m,
                                                const int32_t* hoff, int32_t* fill, uint32_t* keys, int32_t* hrow,
                                                const int32_t* st, const int32_t* skip) {
  __shared__ uint32_t akey[kAggSlots];
  __shared__ int32_t acnt[kAggSlots];
  if (st[kStatus] != 0 || (skip && *skip == 0)) return;
  for (int i = threadIdx.x; i < kAggSlots; i += kB) {
    akey[i] = kAggEmpty;
    acnt[i] = 0;
  }
  __syncthreads();
  for (int64_t b0 = (int64_t)blockIdx.x * kArcsPerBlock; b0 < m; b0 += (int64_t)gridDim.x * kArcsPerBlock) {
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kArcsPerThread, i1 = min(m, i0 + kArcsPerThread);
    int32_t slot[kArcsPerThread], rank[kArcsPerThread];
    int32_t u0 = 0;
    if (i0 < m) {
      int32_t u = u0 = row_of(off, n, i0);
#pragma unroll
      for (int t = 0; t < kArcsPerThread; ++t) {
        const int64_t i = i0 + t;
        slot[t] = -1;
        if (i < i1) {
          while (u < n - 1 && off[u + 1] <= i) ++u;
          const int32_t d = idx[i];
          const int32_t a = hoff[u] + (int32_t)(i - off[u]);
          keys[a] = ((uint32_t)d << 1);
          hrow[a] = u;
          slot[t] = agg_insert(akey, (uint32_t)d);
          rank[t] = atomicAdd(&acnt[slot[t]], 1);
        }
      }
    }
    __syncthreads();
    // reserve each target's range once; acnt becomes the range base
    for (int i = threadIdx.x; i < kAggSlots; i += kB)
      if (akey[i] != kAggEmpty) acnt[i] = atomicAdd(&fill[akey[i]], acnt[i]);
    __syncthreads();
    if (i0 < m) {
      int32_t u = u0;
#pragma unroll
      for (int t = 0; t < kArcsPerThread; ++t) {
        const int64_t i = i0 + t;
        if (i < i1) {
          while (u < n - 1 && off[u + 1] <= i) ++u;
          const int32_t d = (int32_t)akey[slot[t]];
          const int32_t b = hoff[d] + (off[d + 1] - off[d]) + acnt[slot[t]] + rank[t];
          keys[b] = ((uint32_t)u << 1) | 1u;
          hrow[b] = d;
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggSlots; i += kB) {
      akey[i] = kAggEmpty;
      acnt[i] = 0;
    }
    __syncthreads();
  }
}

// Placement from a caller's in-CSR whose rows, like the out-CSR's, are
// strictly increasing: the half-edges of row v in key order are then the
// merge of its out row (keys x<<1) and its in row (keys s<<1|1), so an
// element's slot is its index in its own row plus the number of keys of the
// other row below its own (a binary search), and no sort is needed.  Each
// thread takes kPlaceArcs consecutive elements of the out rows or of the in
// rows (few, so that the chains of dependent searches stay short).  Indices are checked as the arc check does; a row found out of
// order sets st[kUnsorted], and then the general counting, scatter and sort
// run instead (they return at once otherwise).  Every slot stays inside its
// row whatever the input, since the rank is at most the other row's length.
//
// The in-CSR is checked here too, so that no census ever sees a G* whose
// in-entries do not mirror out-arcs: each in-arc s -> v is looked up in the
// out row of s.  With both CSRs strictly increasing (no repeats) and m arcs
// each, in-arcs that are all out-arcs make the in-CSR the transpose.  A miss
// is only recorded (st[kInMismatch]): a search in an out row that is itself
// out of order proves nothing, so the outcome waits until the order is known.
__global__ __launch_bounds__(kB) void k_place_sorted(const int32_t* off, const int32_t* idx, const int32_t* in_off,
                                                     const int32_t* in_idx, int32_t n, int64_t m, int32_t* hoff,
                                                     uint32_t* keys, int32_t* hrow, int32_t* st) {
  if (st[kStatus] != 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t v = t0; v <= n; v += stride) hoff[v] = off[v] + in_off[v];
  const int64_t chunks = (m + kPlaceArcs - 1) / kPlaceArcs;
  for (int64_t t = t0; t < 2 * chunks; t += stride) {
    const uint32_t side = t >= chunks ? 1u : 0u;  // 0: out rows, 1: in rows
    const int32_t* O = side ? in_off : off;
    const int32_t* I = side ? in_idx : idx;
    const int32_t* O2 = side ? off : in_off;
    const int32_t* I2 = side ? idx : in_idx;
    const int64_t i0 = (t - (side ? chunks : 0)) * kPlaceArcs, i1 = min(m, i0 + kPlaceArcs);
    int32_t u = row_of(O, n, i0);
    for (int64_t i = i0; i < i1; ++i) {
      while (u < n - 1 && O[u + 1] <= i) ++u;
      const int32_t x = I[i];
      if (x < 0 || x >= n) { set_status(st, MOTIF_EINDEX); continue; }
      if (x == u) { set_status(st, MOTIF_ESELFLOOP); continue; }
      if (i > O[u] && I[i - 1] >= x) { st[kUnsorted] = 1; continue; }
      // keys of the other row below this one: s < x for an out key x<<1,
      // x <= s for an in key s<<1|1
      int32_t lo = O2[u], hi = O2[u + 1];
      const int32_t base = lo;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t y = I2[mid];
        if (side ? y <= x : y < x) lo = mid + 1; else hi = mid;
      }
      const int64_t pos = (int64_t)off[u] + in_off[u] + (i - O[u]) + (lo - base);
      keys[pos] = ((uint32_t)x << 1) | side;
      hrow[pos] = u;
      if (side) {  // in-arc x -> u: u in the out row of x
        int32_t a = off[x], b = off[x + 1];
        while (a < b) {
          const int32_t mid = (a + b) >> 1;
          if (idx[mid] < u) a = mid + 1; else b = mid;
        }
        if (a >= off[x + 1] || idx[a] != u) st[kInMismatch] = 1;
      }
    }
  }
}

// Small rows sorted by their own thread; longer rows queued: up to mid_max
// keys for the bitonic sort, longer ones for the bitmap sort.
__global__ __launch_bounds__(kB) void k_sort_small(const int32_t* hoff, int32_t n, uint32_t* keys, int32_t* midq,
                                                   int32_t* bigq, int32_t mid_max, int32_t* st, const int32_t* skip) {
  if (st[kStatus] != 0 || (skip && *skip == 0)) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = hoff[v], len = hoff[v + 1] - a;
    if (len <= 1) continue;
    if (len <= kSmallRow) {
      // bitonic network over kSmallRow registers (padding keys sort last);
      // every index is a compile-time constant once the loops are unrolled
      uint32_t* r = keys + a;
      uint32_t x[kSmallRow];
#pragma unroll
      for (int i = 0; i < kSmallRow; ++i) x[i] = i < len ? r[i] : 0xFFFFFFFFu;
#pragma unroll
      for (int k = 2; k <= kSmallRow; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
          for (int i = 0; i < kSmallRow; ++i) {
            const int ij = i ^ j;
            if (ij > i) {
              const uint32_t lo = min(x[i], x[ij]), hi = max(x[i], x[ij]);
              const bool up = (i & k) == 0;
              x[i] = up ? lo : hi;
              x[ij] = up ? hi : lo;
            }
          }
#pragma unroll
      for (int i = 0; i < kSmallRow; ++i)
        if (i < len) r[i] = x[i];
    } else if (len <= mid_max) {
      midq[atomicAdd(&st[kMidCount], 1)] = (int32_t)v;
    } else {
      bigq[atomicAdd(&st[kBigCount], 1)] = (int32_t)v;
    }
  }
}

// Mid rows: bitonic sort in LDS, one workgroup per row (persistent grid).
__global__ __launch_bounds__(kB) void k_sort_mid(const int32_t* hoff, uint32_t* keys, const int32_t* midq,
                                                 const int32_t* st, const int32_t* skip) {
  __shared__ uint32_t s[kMidRow];
  static_assert(kB / 64 * kWaveRow <= kMidRow, "one LDS slice per wave");
  if (st[kStatus] != 0 || (skip && *skip == 0)) return;
  const int32_t count = st[kMidCount];
  // rows of at most kWaveRow keys: one wave each, in its own LDS slice, with
  // no workgroup barrier (most mid rows are a few hundred keys)
  {
    const int32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* ws = s + wv * kWaveRow;
    auto wave_sync = [] {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int32_t q = blockIdx.x * (kB / 64) + wv; q < count; q += gridDim.x * (kB / 64)) {
      const int32_t v = midq[q];
      const int32_t a = hoff[v], len = hoff[v + 1] - a;
      if (len > kWaveRow) continue;
      int P = 1;
      while (P < len) P <<= 1;
      for (int i = lane; i < P; i += 64) ws[i] = i < len ? keys[a + i] : 0xFFFFFFFFu;
      wave_sync();
      for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int i = lane; i < P; i += 64) {
            const int ij = i ^ j;
            if (ij > i) {
              const uint32_t x = ws[i], y = ws[ij];
              const bool up = (i & k) == 0;
              if ((x > y) == up) { ws[i] = y; ws[ij] = x; }
            }
          }
          wave_sync();
        }
      }
      for (int i = lane; i < len; i += 64) keys[a + i] = ws[i];
      wave_sync();
    }
  }
  __syncthreads();
  // longer rows: the whole workgroup
  for (int32_t q = blockIdx.x; q < count; q += gridDim.x) {
    const int32_t v = midq[q];
    const int32_t a = hoff[v], len = hoff[v + 1] - a;
    if (len <= kWaveRow) continue;
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kB) s[i] = i < len ? keys[a + i] : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < P; i += kB) {
          int ij = i ^ j;
          if (ij > i) {
            uint32_t x = s[i], y = s[ij];
            bool up = (i & k) == 0;
            if ((x > y) == up) { s[i] = y; s[ij] = x; }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < len; i += kB) keys[a + i] = s[i];
    __syncthreads();
  }
}

// Big rows: set one bit per key in a bitmap over [0, 2n), then compact in
// order.  A key seen twice is a repeated arc.  The bitmap is cleared once at
// the start and each word again as the compaction reads it.
template <bool LDS, int BS>
__global__ __launch_bounds__(BS) void k_sort_big(const int32_t* hoff, int32_t n, uint32_t* keys,
                                                 const int32_t* bigq, uint32_t* bitmaps, int32_t* st,
                                                 const int32_t* skip) {
  __shared__ int32_t sh[BS / 64];
  __shared__ uint32_t lbm[LDS ? kLdsBitmapWords : 1];
  if (st[kStatus] != 0 || (skip && *skip == 0)) return;
  const int32_t count = st[kBigCount];
  if ((int32_t)blockIdx.x >= count) return;
  const int64_t words = ((int64_t)2 * n + 31) / 32;
  uint32_t* bm = LDS ? lbm : bitmaps + (int64_t)blockIdx.x * words;
  const int64_t per = (words + BS - 1) / BS;
  for (int64_t w = threadIdx.x; w < words; w += BS) bm[w] = 0u;
  __syncthreads();
  for (int32_t q = blockIdx.x; q < count; q += gridDim.x) {
    const int32_t v = bigq[q];
    const int32_t a = hoff[v], len = hoff[v + 1] - a;
    for (int i = threadIdx.x; i < len; i += BS) {
      uint32_t key = keys[a + i];
      uint32_t bit = 1u << (key & 31u);
      uint32_t old = atomicOr(&bm[key >> 5], bit);
      if (old & bit) set_status(st, MOTIF_EDUP);
    }
    __syncthreads();
    const int64_t w0 = threadIdx.x * per, w1 = w0 + per < words ? w0 + per : words;
    int32_t cnt = 0;
    for (int64_t w = w0; w < w1; ++w) cnt += __popc(bm[w]);
    int32_t total;
    int32_t pos = block_excl_scan(cnt, sh, &total);
    for (int64_t w = w0; w < w1; ++w) {
      uint32_t b = bm[w];
      if (b) bm[w] = 0u;
      while (b) {
        int t = __ffs(b) - 1;
        b &= b - 1;
        if (pos < len) keys[a + pos] = (uint32_t)(w * 32 + t);
        ++pos;
      }
    }
    __syncthreads();
  }
}

// Element-parallel merge of the sorted half-edges of every row: a half-edge
// opens a new G* entry unless it carries the same neighbour as its
// predecessor in the row (the pair id<<1, id<<1|1 is one bidirected
// neighbour); equal keys are a repeated arc.  Position h closes the scan.
struct EntryFlag {
  const uint32_t* keys;
  const int32_t* hrow;
  const int32_t* hoff;
  int64_t h;
  int32_t* st;
  __device__ int32_t operator()(int64_t i) const {
    if (i == h) return 0;
    const uint32_t k = keys[i];
    const bool first = i == hoff[hrow[i]];
    if (!first && keys[i - 1] == k) set_status(st, MOTIF_EDUP);
    return (first || (keys[i - 1] >> 1) != (k >> 1)) ? 1 : 0;
  }
};

// gs_off[v] = position of row v's first half-edge in the scanned flags;
// with deg given, also the row's length.
__global__ void k_gather_off(const int32_t* pos, const int32_t* hoff, int32_t n, int32_t* gs_off, int32_t* deg,
                             const int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = pos[hoff[v]];
    gs_off[v] = a;
    if (deg && v < n) deg[v] = pos[hoff[v + 1]] - a;
  }
}

// Typed G* entries, plus the row of each entry and the degree of each row.
__global__ void k_write_gstar(const uint32_t* keys, const int32_t* hrow, const int32_t* hoff, int64_t h,
                              const int32_t* pos, uint32_t* gs_idx, int32_t* gs_row, const int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < h; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = hrow[i];
    const uint32_t k = keys[i];
    if (i != hoff[r] && (keys[i - 1] >> 1) == (k >> 1)) continue;  // second half of a pair
    const bool pair = i + 1 < hoff[r + 1] && (keys[i + 1] >> 1) == (k >> 1);
    const uint32_t t = pair ? 3u : ((k & 1u) ? 2u : 1u);
    gs_idx[pos[i]] = (k >> 1) | (t << kTypeShift);
    gs_row[pos[i]] = r;
  }
}

// 1 for entry j of row v when it points to a neighbour of higher rank (an
// entry of N+(v)); 0 past the last G* entry.
struct PlusFlag {
  const uint32_t* gs_idx;
  const int32_t* gs_row;
  const int32_t* deg;
  const int32_t* gs_off;
  int32_t n;
  __device__ int32_t operator()(int64_t j) const {
    if (j >= gs_off[n]) return 0;
    const int32_t v = gs_row[j];
    const int32_t w = (int32_t)(gs_idx[j] & kIdMask);
    return rank_less(deg[v], v, deg[w], w) ? 1 : 0;
  }
};

__global__ void k_write_plus(const uint32_t* gs_idx, const int32_t* flag_pos, const int32_t* gs_row,
                             const int32_t* deg, const int32_t* gs_off, int32_t n, uint32_t* np_idx,
                             const int32_t* st) {
  if (st[kStatus] != 0) return;
  const int64_t e = gs_off[n];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < e; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = gs_row[j];
    const uint32_t x = gs_idx[j];
    const int32_t w = (int32_t)(x & kIdMask);
    if (rank_less(deg[v], v, deg[w], w)) np_idx[flag_pos[j]] = x;
  }
}

// In-CSR given by the caller: every listed in-arc s -> v must be an arc of
// the out-CSR, listed once, and each row must have the in-degree counted from
// the out-CSR.  `has_in` (batch) marks the graphs that supplied an in-CSR.
__global__ void k_check_in_rows(const int32_t* in_off, const int32_t* in_cnt, int32_t n, const int32_t* gid,
                                const int32_t* has_in, int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (gid && !has_in[gid[v]]) continue;
    if (in_off[v + 1] - in_off[v] != in_cnt[v]) set_status(st, MOTIF_ETRANSPOSE);
  }
}

__global__ void k_check_in_arcs(const int32_t* in_off, const int32_t* in_idx, int32_t n, int64_t m,
                                const int32_t* gs_off, const uint32_t* gs_idx, const int32_t* gid,
                                const int32_t* has_in, uint32_t* marks, int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = row_of(in_off, n, i);
    if (gid && !has_in[gid[v]]) continue;
    int32_t s = in_idx[i];
    if (s < 0 || s >= n) { set_status(st, MOTIF_EINDEX); continue; }
    int32_t lo = gs_off[v], hi = gs_off[v + 1];
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if ((int32_t)(gs_idx[mid] & kIdMask) < s) lo = mid + 1; else hi = mid;
    }
    if (lo >= gs_off[v + 1] || (int32_t)(gs_idx[lo] & kIdMask) != s || !((gs_idx[lo] >> kTypeShift) & 2u)) {
      set_status(st, MOTIF_ETRANSPOSE);
      continue;
    }
    uint32_t bit = 1u << (lo & 31);
    if (atomicOr(&marks[lo >> 5], bit) & bit) set_status(st, MOTIF_ETRANSPOSE);
  }
}

// In-CSR check of a single graph against the built G*: every listed in-arc
// s -> v must be an arc of the out-CSR (entry v of G* row s carries the out
// bit, which only the out-CSR sets) and no entry may be claimed twice.  With
// the in-CSR's offsets checked (m arcs in all) and the out-CSR free of
// repeats, that makes the in-CSR the transpose, whichever CSR the G* in-bits
// were taken from.
__global__ void k_check_in_arcs_out(const int32_t* in_off, const int32_t* in_idx, int32_t n, int64_t m,
                                    const int32_t* gs_off, const uint32_t* gs_idx, uint32_t* marks, int32_t* st,
                                    const int32_t* skip) {
  if (st[kStatus] != 0 || (skip && *skip == 0)) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = row_of(in_off, n, i);
    const int32_t s = in_idx[i];
    if (s < 0 || s >= n) { set_status(st, MOTIF_EINDEX); continue; }
    int32_t lo = gs_off[s], hi = gs_off[s + 1];
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if ((int32_t)(gs_idx[mid] & kIdMask) < v) lo = mid + 1; else hi = mid;
    }
    if (lo >= gs_off[s + 1] || (int32_t)(gs_idx[lo] & kIdMask) != v || !((gs_idx[lo] >> kTypeShift) & 1u)) {
      set_status(st, MOTIF_ETRANSPOSE);
      continue;
    }
    const uint32_t bit = 1u << (lo & 31);
    if (atomicOr(&marks[lo >> 5], bit) & bit) set_status(st, MOTIF_ETRANSPOSE);
  }
}

// ------------------------------------------------------------------- pack --

__device__ __forceinline__ int32_t graph_of(const int64_t* pre, int32_t count, int64_t x) {
  int32_t lo = 0, hi = count - 1;  // last g with pre[g] <= x
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_pack_rows(const motif_graph_t* gs, int32_t count, const int64_t* voff, const int64_t* aoff,
                            int64_t N, int64_t M, int32_t* uoff, int32_t* uin_off, int32_t* gid, int32_t* has_in,
                            int32_t* st) {
  for (int64_t V = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; V <= N; V += (int64_t)gridDim.x * blockDim.x) {
    if (V == N) {
      uoff[N] = (int32_t)M;
      uin_off[N] = (int32_t)M;
      continue;
    }
    const int32_t g = graph_of(voff, count, V);
    const motif_graph_t G = gs[g];
    const int64_t v = V - voff[g];
    const int32_t a = G.out_off[v], b = G.out_off[v + 1];
    if (v == 0) has_in[g] = G.in_off != nullptr;
    if ((v == 0 && a != 0) || b < a || (v == G.n - 1 && (int64_t)b != G.m)) set_status(st, MOTIF_EINVAL_SHAPE);
    uoff[V] = (int32_t)(aoff[g] + a);
    gid[V] = g;
    if (G.in_off) {
      const int32_t ia = G.in_off[v], ib = G.in_off[v + 1];
      if ((v == 0 && ia != 0) || ib < ia || (v == G.n - 1 && (int64_t)ib != G.m)) set_status(st, MOTIF_EINVAL_SHAPE);
      uin_off[V] = (int32_t)(aoff[g] + ia);
    } else {
      uin_off[V] = (int32_t)aoff[g];  // empty in-rows; not checked
    }
  }
}

__global__ void k_pack_arcs(const motif_graph_t* gs, int32_t count, const int64_t* voff, const int64_t* aoff,
                            int64_t M, int32_t* uidx, int32_t* uin_idx, int32_t* st) {
  for (int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; A < M; A += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = graph_of(aoff, count, A);
    const motif_graph_t G = gs[g];
    const int64_t a = A - aoff[g];
    int32_t d = G.out_idx[a];
    if (d < 0 || d >= G.n) { set_status(st, MOTIF_EINDEX); d = 0; }
    uidx[A] = (int32_t)(voff[g] + d);
    if (G.in_idx) {
      int32_t s = G.in_idx[a];
      if (s < 0 || s >= G.n) { set_status(st, MOTIF_EINDEX); s = 0; }
      uin_idx[A] = (int32_t)(voff[g] + s);
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host ---

void enqueue_zero(void* ptr, size_t bytes, hipStream_t s) {
  size_t words = (bytes + 3) / 4;
  if (!words) return;
  if (((uintptr_t)ptr & 15u) == 0 && words >= 1024) {  // 16-byte stores for the bulk
    const size_t n16 = words / 4;
    hipLaunchKernelGGL(k_zero16, dim3(grid_for((int64_t)n16)), dim3(kB), 0, s, (uint4*)ptr, n16);
    words -= n16 * 4;
    if (!words) return;
    ptr = (uint32_t*)ptr + n16 * 4;
  }
  hipLaunchKernelGGL(k_zero, dim3(grid_for((int64_t)words)), dim3(kB), 0, s, (uint32_t*)ptr, words);
}

void enqueue_zero_batch(const ZeroBatch& z, hipStream_t s) {
  if (!z.n) return;
  ZeroRanges r{};
  size_t most = 1;
  for (int k = 0; k < z.n; ++k) {
    const size_t words = (z.bytes[k] + 3) / 4;
    r.p16[k] = (uint4*)z.ptr[k];
    r.n16[k] = words / 4;
    r.tail[k] = (uint32_t*)z.ptr[k] + (words / 4) * 4;
    r.ntail[k] = (int32_t)(words % 4);
    most = std::max(most, r.n16[k]);
  }
  r.n = z.n;
  hipLaunchKernelGGL(k_zero_many, dim3(grid_for((int64_t)most)), dim3(kB), 0, s, r);
}

namespace {
__global__ void k_status_out(int32_t* dst, const int32_t* st) {
  if (threadIdx.x == 0) dst[0] = st[kStatus];
}
}  // namespace

void enqueue_status_out(int32_t* dst, const int32_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, s, dst, st);
}

namespace {
// Undirected census: every G* entry and every N+ entry becomes type A
// (bidirected), so the directed census of the result is the census of the
// undirected version G* with each edge read as a pair of arcs.
__global__ void k_all_bidirected(const int32_t* gs_off, uint32_t* gs_idx, const int32_t* np_off, uint32_t* np_idx,
                                 int32_t n, const int32_t* st) {
  if (st[kStatus] != 0) return;
  const int64_t ng = gs_off[n], nn = np_off[n];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) {
    gs_idx[i] |= 3u << kTypeShift;
    if (i < nn) np_idx[i] |= 3u << kTypeShift;
  }
}

// out[u] = sum of dir[c] over the directed classes c of undirected class u;
// a count in a class with a one-way arc is impossible after the override
// and is reported as a self-check failure (nothing written then).
__global__ void k_project_undirected(const uint64_t* dir, const int16_t* und_of, int32_t C, int32_t U, uint64_t* out,
                                     int32_t* st) {
  __shared__ unsigned long long acc[32];
  __shared__ int32_t bad;
  if (st[kStatus] != 0) return;
  if (threadIdx.x < 32) acc[threadIdx.x] = 0;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int32_t c = threadIdx.x; c < C; c += blockDim.x) {
    const uint64_t v = dir[c];
    if (!v) continue;
    if (und_of[c] < 0) bad = 1;
    else atomicAdd(&acc[und_of[c]], (unsigned long long)v);
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) atomicMin(&st[kStatus], MOTIF_EINTERNAL);
    return;
  }
  if (threadIdx.x < U) out[threadIdx.x] = acc[threadIdx.x];
}
}  // namespace

void enqueue_all_bidirected(const DevGraph& g, hipStream_t s, const int32_t* st) {
  hipLaunchKernelGGL(k_all_bidirected, dim3(grid_for(g.gs_cap)), dim3(kB), 0, s, g.gs_off,
                     const_cast<uint32_t*>(g.gs_idx), g.np_off, const_cast<uint32_t*>(g.np_idx), g.n, st);
}

void enqueue_project_undirected(const uint64_t* dir, const int16_t* und_of, int32_t C, int32_t U, uint64_t* out,
                                int32_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_project_undirected, dim3(1), dim3(1024), 0, s, dir, und_of, C, U, out, st);
}

size_t build_bytes(int64_t N, int64_t M, int32_t G, bool batch) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t b = 0;
  b += 4 * al(sizeof(int32_t) * (N + 1));          // in_cnt, hoff, fill, deg
  b += al(sizeof(int32_t) * (N + 1));              // gs_off
  b += al(sizeof(int32_t) * (N + 1));              // np_off
  b += al(sizeof(uint32_t) * 2 * (M + 1));         // keys
  b += al(sizeof(uint32_t) * 2 * (M + 1));         // gs_idx
  b += al(sizeof(uint32_t) * (M + 1));             // np_idx
  b += 2 * al(sizeof(int32_t) * (N + 1));          // sort queues
  b += al(sizeof(uint32_t) * kBigSlots * ((2 * N + 31) / 32 + 1));
  b += al(sizeof(uint32_t) * ((2 * M + 31) / 32 + 1));  // transpose marks
  b += scan1_bytes(N + 1) + 2 * scan1_bytes(2 * M + 1);  // look-back words of the three scans
  b += 3 * al(sizeof(int32_t) * (2 * M + 1));      // half-edge rows, merge flags, G* entry rows
  if (batch) {
    b += 2 * al(sizeof(int32_t) * (N + 1)) + 2 * al(sizeof(int32_t) * (M + 1)) + al(sizeof(int32_t) * (N + 1));
    b += 2 * al(sizeof(int64_t) * (G + 1)) + al(sizeof(motif_graph_t) * G) + al(sizeof(int32_t) * G);
  }
  return b;
}

BuildInput enqueue_pack(Pipeline& p, const motif_graph_t* graphs, int32_t count, const int64_t* voff,
                        const int64_t* aoff, hipStream_t s) {
  const int64_t N = voff[count], M = aoff[count];
  Arena& A = p.arena;
  int32_t* uoff = A.take<int32_t>(N + 1);
  int32_t* uidx = A.take<int32_t>(M + 1);
  int32_t* uin_off = A.take<int32_t>(N + 1);
  int32_t* uin_idx = A.take<int32_t>(M + 1);
  int32_t* gid = A.take<int32_t>(N + 1);
  int64_t* dvoff = A.take<int64_t>(count + 1);
  int64_t* daoff = A.take<int64_t>(count + 1);
  motif_graph_t* dg = A.take<motif_graph_t>(count);
  int32_t* has_in = A.take<int32_t>(count);
  const bool copy_error =
      hipMemcpyAsync(dvoff, voff, sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(daoff, aoff, sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(dg, graphs, sizeof(motif_graph_t) * count, hipMemcpyHostToDevice, s) != hipSuccess;
  hipLaunchKernelGGL(k_pack_rows, dim3(grid_for(N + 1)), dim3(kB), 0, s, dg, count, dvoff, daoff, N, M, uoff,
                     uin_off, gid, has_in, p.status);
  bool any_in = false;
  for (int32_t g = 0; g < count; ++g) any_in |= graphs[g].in_off != nullptr;
  if (M > 0)
    hipLaunchKernelGGL(k_pack_arcs, dim3(grid_for(M)), dim3(kB), 0, s, dg, count, dvoff, daoff, M, uidx,
                       any_in ? uin_idx : nullptr, p.status);
  BuildInput in{};
  in.out_off = uoff;
  in.out_idx = uidx;
  in.in_off = any_in ? uin_off : nullptr;
  in.in_idx = any_in ? uin_idx : nullptr;
  in.n = (int32_t)N;
  in.m = M;
  in.gid = gid;
  in.ngraphs = count;
  in.has_in = has_in;
  in.voff = dvoff;
  int64_t mx = 0;
  for (int32_t g = 0; g < count; ++g) mx = std::max<int64_t>(mx, voff[g + 1] - voff[g]);
  in.max_graph_n = (int32_t)mx;
  in.copy_error = copy_error;
  return in;
}

DevGraph enqueue_build(Pipeline& p, const BuildInput& in, hipStream_t s, hipEvent_t graph_ready, bool* ready_ok,
                       InCheck* deferred) {
  Arena& A = p.arena;
  const int32_t n = in.n;
  const int64_t m = in.m;
  int32_t* st = p.status;
  int32_t* in_cnt = A.take<int32_t>(n + 1);
  int32_t* hoff = A.take<int32_t>(n + 1);
  int32_t* fill = A.take<int32_t>(n + 1);
  int32_t* deg = A.take<int32_t>(n + 1);
  int32_t* gs_off = A.take<int32_t>(n + 1);
  int32_t* np_off = A.take<int32_t>(n + 1);
  uint32_t* keys = A.take<uint32_t>(2 * m + 1);
  uint32_t* gs_idx = A.take<uint32_t>(2 * m + 1);
  uint32_t* np_idx = A.take<uint32_t>(m + 1);
  int32_t* hrow = A.take<int32_t>(2 * m + 1);
  int32_t* flags = A.take<int32_t>(2 * m + 1);
  int32_t* gs_row = A.take<int32_t>(2 * m + 1);
  int32_t* midq = A.take<int32_t>(n + 1);
  int32_t* bigq = A.take<int32_t>(n + 1);
  const int64_t bm_words = (2 * (int64_t)n + 31) / 32 + 1;
  uint32_t* bitmaps = A.take<uint32_t>(kBigSlots * bm_words);
  uint32_t* marks = A.take<uint32_t>((2 * m + 31) / 32 + 1);
  ZeroBatch z;
  z.add(in_cnt, sizeof(int32_t) * (n + 1));
  z.add(fill, sizeof(int32_t) * (n + 1));
  const Scan1 sc_half = scan1_take(A, n + 1, z);
  const Scan1 sc_entry = scan1_take(A, 2 * m + 1, z);
  const Scan1 sc_plus = scan1_take(A, 2 * m + 1, z);

  DevGraph g;
  g.n = n;
  g.gs_off = gs_off;
  g.gs_idx = gs_idx;
  g.np_off = np_off;
  g.np_idx = np_idx;
  g.gid = in.gid;
  g.voff = in.voff;
  g.ngraphs = in.ngraphs;
  g.max_graph_n = in.gid ? in.max_graph_n : n;
  g.gs_row = gs_row;
  g.gs_cap = 2 * m + 1;
  if (n == 0) {
    if (graph_ready) *ready_ok = hipEventRecord(graph_ready, s) == hipSuccess;
    return g;
  }

  enqueue_zero_batch(z, s);
  // A single graph with an in-CSR whose rows (and the out-CSR's) are
  // strictly increasing is placed by merging each row's two halves; the
  // counting, scatter and sort below then return at once.  Any other input
  // takes them.
  const bool from_in = !in.gid && in.in_off && m > 0;
  const int32_t* skip = from_in ? st + kUnsorted : nullptr;
  const unsigned arc_grid = grid_for((m + kArcsPerThread - 1) / kArcsPerThread);  // caps at 65536 blocks
  if (!in.gid) hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n + 1)), dim3(kB), 0, s, in.out_off, n, m, st);
  if (from_in) {
    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n + 1)), dim3(kB), 0, s, in.in_off, n, m, st);
    hipLaunchKernelGGL(k_place_sorted, dim3(grid_for(2 * ((m + kPlaceArcs - 1) / kPlaceArcs))), dim3(kB), 0, s,
                       in.out_off, in.out_idx, in.in_off, in.in_idx, n, m, hoff, keys, hrow, st);
  }
  if (m > 0)
    hipLaunchKernelGGL(k_count_in, dim3(arc_grid), dim3(kB), 0, s, in.out_off, in.out_idx, n, m, in_cnt, st, skip);
  enqueue_scan1(sc_half, hoff, HalfCount{in.out_off, in_cnt, n}, st, s, skip);
  if (m > 0)
    hipLaunchKernelGGL(k_scatter, dim3(arc_grid), dim3(kB), 0, s, in.out_off, in.out_idx, n, m, hoff, fill, keys,
                       hrow, st, skip);
  // With the bitmap in LDS a row costs about the same whatever its length
  // (a few words per thread to clear, count and compact), which beats the
  // bitonic sort's log^2 stages from a few hundred keys on.
  const bool lds_bitmap = (2 * (int64_t)n + 31) / 32 <= kLdsBitmapWords;
  hipLaunchKernelGGL(k_sort_small, dim3(grid_for(n)), dim3(kB), 0, s, hoff, n, keys, midq, bigq,
                     lds_bitmap ? kLdsBitmapRow : kMidRow, st, skip);
  hipLaunchKernelGGL(k_sort_mid, dim3(512), dim3(kB), 0, s, hoff, keys, midq, st, skip);
  if (lds_bitmap)
    hipLaunchKernelGGL((k_sort_big<true, kLdsBitmapBlock>), dim3(kLdsBitmapGrid), dim3(kLdsBitmapBlock), 0, s, hoff,
                       n, keys, bigq, bitmaps, st, skip);
  else
    hipLaunchKernelGGL((k_sort_big<false, kB>), dim3(kBigSlots), dim3(kB), 0, s, hoff, n, keys, bigq, bitmaps, st,
                       skip);
  // merge: entry flags over the 2m sorted half-edges, scanned into positions
  enqueue_scan1(sc_entry, flags, EntryFlag{keys, hrow, hoff, 2 * m, st}, st, s);
  hipLaunchKernelGGL(k_gather_off, dim3(grid_for(n + 1)), dim3(kB), 0, s, flags, hoff, n, gs_off, deg, st);
  hipLaunchKernelGGL(k_write_gstar, dim3(grid_for(2 * m)), dim3(kB), 0, s, keys, hrow, hoff, 2 * m, flags, gs_idx,
                     gs_row, st);
  // oriented rows N+: flags over the G* entries (at most 2m of them), scanned
  enqueue_scan1(sc_plus, flags, PlusFlag{gs_idx, gs_row, deg, gs_off, n}, st, s);
  hipLaunchKernelGGL(k_gather_off, dim3(grid_for(n + 1)), dim3(kB), 0, s, flags, gs_off, n, np_off, nullptr, st);
  hipLaunchKernelGGL(k_write_plus, dim3(grid_for(2 * m)), dim3(kB), 0, s, gs_idx, flags, gs_row, deg, gs_off, n,
                     np_idx, st);
  // G* and N+ are complete here; the in-CSR check below only compares
  if (graph_ready) *ready_ok = hipEventRecord(graph_ready, s) == hipSuccess;
  InCheck c{in_cnt, marks, from_in};
  if (deferred) *deferred = c;
  else enqueue_check_in(in, g, c, st, s, false);
  return g;
}

void enqueue_check_in(const BuildInput& in, const DevGraph& g, const InCheck& c, int32_t* st, hipStream_t s,
                      bool background) {
  if (!in.in_off || g.n == 0) return;
  const int32_t n = in.n;
  const int64_t m = in.m;
  // beside a census, a few waves per CU: the search chains are latency-bound
  // and a full grid would hold back the census's own launches
  unsigned grid = grid_for(m);
  if (background) grid = std::min(grid, (unsigned)kCheckGrid);
  if (!in.gid) {
    if (!c.offsets_checked)
      hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n + 1)), dim3(kB), 0, s, in.in_off, n, m, st);
    enqueue_zero(c.marks, sizeof(uint32_t) * ((2 * m + 31) / 32 + 1), s);
    // after a placement from sorted rows the in-CSR is already checked
    if (m > 0)
      hipLaunchKernelGGL(k_check_in_arcs_out, dim3(grid), dim3(kB), 0, s, in.in_off, in.in_idx, n, m, g.gs_off,
                         g.gs_idx, c.marks, st, c.offsets_checked ? st + kUnsorted : nullptr);
    return;
  }
  hipLaunchKernelGGL(k_check_in_rows, dim3(grid_for(n)), dim3(kB), 0, s, in.in_off, c.in_cnt, n, in.gid, in.has_in,
                     st);
  enqueue_zero(c.marks, sizeof(uint32_t) * ((2 * m + 31) / 32 + 1), s);
  if (m > 0)
    hipLaunchKernelGGL(k_check_in_arcs, dim3(grid), dim3(kB), 0, s, in.in_off, in.in_idx, n, m, g.gs_off, g.gs_idx,
                       in.gid, in.has_in, c.marks, st);
}

}  // namespace motif
