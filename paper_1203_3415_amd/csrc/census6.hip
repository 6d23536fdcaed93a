// Motifs of size 6: the paper's anchor method taken one size further (its
// stated extension to larger motifs, Section "Our approach").  As k = 4 uses
// an edge and k = 5 a connected triple, k = 6 uses a connected 4-set T as the
// anchor: every other vertex adjacent to T gets a label (its type towards each
// of the four anchor vertices, 2 bits each), the pairs of labelled vertices
// go to the classes of (T, label, label, no edge) by the closed form over
// label pairs, and every edge between two labelled vertices moves one
// occurrence from its no-edge class to the class with that edge.  A 6-set of
// class c is then counted once per connected 4-subset that dominates the
// other two vertices, and the totals are divided by that number (Fact
// "correction" carried over).
//
// Class table: the 2^30 codes of 6-vertex digraphs (arc i->j at bit
// 5i + (j < i ? j : j - 1)) are classified on the device.  A code is
// canonical when none of its 720 relabellings is smaller; the canonical codes
// of weakly connected digraphs, in increasing order, are the classes
// (1,530,843 of them); every relabelling of a class's code then gets the
// class id in a 4 GiB lookup table (disconnected codes: kNoClass).
//
// Anchors: every connected 4-set is found from its edges {a, b} whose ends
// dominate the other two vertices, and kept at the smallest such edge (ids
// compared as pairs), so each is listed once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace motif {

namespace {

constexpr uint32_t kCodes6 = 1u << 30;
constexpr uint32_t kNoClass = 0xFFFFFFFFu;
constexpr int kPerms6 = 720;
constexpr int kBits6 = 30;

__host__ __device__ constexpr int bit6(int i, int j) { return i * 5 + (j < i ? j : j - 1); }

// LDS writes of the wave done and visible to its other lanes.
__device__ __forceinline__ void wave_sync6() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The code relabelled by the permutation whose bit map is pos[0..29] (bit b
// of the code moves to bit pos[b]).
__device__ __forceinline__ uint32_t relabel6(const uint8_t* pos, uint32_t x) {
  uint32_t y = 0;
  for (uint32_t t = x; t; t &= t - 1u) y |= 1u << pos[__builtin_ctz(t)];
  return y;
}

// Weak connectivity of a 6-vertex code.
__device__ __forceinline__ bool connected6(uint32_t x) {
  uint32_t adj[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (i != j && ((x >> bit6(i, j)) & 1u)) {
        adj[i] |= 1u << j;
        adj[j] |= 1u << i;
      }
  uint32_t reach = 1u;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    uint32_t nx = reach;
#pragma unroll
    for (int v = 0; v < 6; ++v)
      if ((reach >> v) & 1u) nx |= adj[v];
    reach = nx;
  }
  return reach == 63u;
}

// Mark the canonical codes of connected digraphs (bit x of marks) and count
// all canonical codes (every digraph class, connected or not).  One wave per
// code: the lanes try 64 relabellings at a time and stop at the first round
// in which one of them is smaller (almost always the first round).
__global__ void k6_mark(const uint8_t* __restrict__ pos_g, uint32_t* __restrict__ marks,
                        unsigned long long* __restrict__ n_canon) {
  __shared__ uint8_t pos[kPerms6 * kBits6];
  for (int i = threadIdx.x; i < kPerms6 * kBits6; i += blockDim.x) pos[i] = pos_g[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long mine = 0;
  for (uint64_t x = wave; x < kCodes6; x += nwaves) {
    bool smaller = false;
    for (int p0 = 0; p0 < kPerms6 && !smaller; p0 += 64) {
      const int p = p0 + lane;
      const bool s = p > 0 && p < kPerms6 && relabel6(pos + p * kBits6, (uint32_t)x) < (uint32_t)x;
      smaller = __ballot(s) != 0ull;
    }
    if (smaller || lane != 0) continue;
    ++mine;
    if (connected6((uint32_t)x)) atomicOr(&marks[x >> 5], 1u << (x & 31u));
  }
  if (lane == 0 && mine) atomicAdd(n_canon, mine);
}

// Exclusive prefix sums of the popcounts of marks, in blocks of 1024 words:
// rank[w] = marked bits before word w within its block, bsum[b] = block total.
__global__ void k6_rank_local(const uint32_t* __restrict__ marks, uint32_t* __restrict__ rank,
                              uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s[1024];
  const uint64_t w = blockIdx.x * 1024ull + threadIdx.x;
  const uint32_t v = __popc(marks[w]);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  rank[w] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

// Exclusive scan of the block totals (one block; nb <= 32768) and the total.
__global__ void k6_rank_blocks(uint32_t* __restrict__ bsum, int32_t nb, uint32_t* __restrict__ total) {
  __shared__ uint32_t s[1024];
  constexpr int kPer = 32;  // block totals per thread
  uint32_t loc[kPer];
  uint32_t sum = 0;
  for (int i = 0; i < kPer; ++i) {
    const int idx = threadIdx.x * kPer + i;
    loc[i] = idx < nb ? bsum[idx] : 0u;
    sum += loc[i];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - sum;
  for (int i = 0; i < kPer; ++i) {
    const int idx = threadIdx.x * kPer + i;
    if (idx < nb) bsum[idx] = run;
    run += loc[i];
  }
  if (threadIdx.x == 1023) *total = s[1023];
}

// codes[id] = the id-th marked code in increasing order.
__global__ void k6_codes(const uint32_t* __restrict__ marks, const uint32_t* __restrict__ rank,
                         const uint32_t* __restrict__ bsum, uint32_t* __restrict__ codes, uint32_t ncls) {
  const uint64_t w = blockIdx.x * 1024ull + threadIdx.x;
  uint32_t m = marks[w];
  uint32_t id = bsum[blockIdx.x] + rank[w];
  for (; m; m &= m - 1u, ++id)
    if (id < ncls) codes[id] = (uint32_t)(w << 5) + (uint32_t)__builtin_ctz(m);
}

__global__ void k6_fill(uint4* __restrict__ p, uint64_t n16, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(v, v, v, v);
}

// lut[relabelling of codes[c]] = c for every class c and all 720 relabellings;
// thread t takes class t / 8 and every 8th relabelling from t % 8.
__global__ void k6_expand(const uint8_t* __restrict__ pos_g, const uint32_t* __restrict__ codes, uint32_t ncls,
                          uint32_t* __restrict__ lut) {
  __shared__ uint8_t pos[kPerms6 * kBits6];
  for (int i = threadIdx.x; i < kPerms6 * kBits6; i += blockDim.x) pos[i] = pos_g[i];
  __syncthreads();
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < (uint64_t)ncls * 8;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t c = (uint32_t)(t >> 3), x = codes[c];
    for (int p = (int)(t & 7u); p < kPerms6; p += 8) lut[relabel6(pos + p * kBits6, x)] = c;
  }
}

// Anchors of one class: connected 4-subsets dominating the other two vertices.
__global__ void k6_mult(const uint32_t* __restrict__ codes, uint32_t ncls, uint8_t* __restrict__ mult) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncls) return;
  const uint32_t x = codes[c];
  uint32_t adj[6] = {0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      if (i != j && ((x >> bit6(i, j)) & 1u)) {
        adj[i] |= 1u << j;
        adj[j] |= 1u << i;
      }
  int count = 0;
  for (uint32_t s = 0; s < 64u; ++s) {
    if (__popc(s) != 4) continue;
    uint32_t reach = 1u << __builtin_ctz(s);
    for (int it = 0; it < 3; ++it) {
      uint32_t nx = reach;
      for (int v = 0; v < 6; ++v)
        if ((reach >> v) & 1u) nx |= adj[v] & s;
      reach = nx;
    }
    if (reach != s) continue;
    bool dom = true;
    for (int w = 0; w < 6; ++w)
      if (!((s >> w) & 1u) && !(adj[w] & s)) dom = false;
    count += dom;
  }
  mult[c] = (uint8_t)count;
}

// ------------------------------------------------------------- census ----

// Type of v in u's G* row (1: arc u->v only, 2: v->u only, 3: both), 0 if
// not adjacent.  Rows are sorted by id.
__device__ __forceinline__ uint32_t gs_type(const DevGraph& G, int32_t u, int32_t v) {
  int32_t lo = G.gs_off[u], hi = G.gs_off[u + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int32_t)(G.gs_idx[mid] & kIdMask) < v) lo = mid + 1; else hi = mid;
  }
  if (lo < G.gs_off[u + 1] && (int32_t)(G.gs_idx[lo] & kIdMask) == v) return G.gs_idx[lo] >> kTypeShift;
  return 0u;
}

constexpr int kHash6 = 2048;        // wave hash slots: the anchor edge's neighbourhood
constexpr int kMembers6 = kHash6 / 2;  // at most d*(a) + d*(b) - 2 members per edge
constexpr uint32_t kEmpty6 = 0xFFFFFFFFu;
constexpr int kWaves6 = 4;          // waves per workgroup of k6_anchors

// Connected 4-sets, each once: wave per G* edge {a, b} (a < b, from a's row);
// members adj(e) = N(a) u N(b) \ {a, b} with their types towards a and b;
// every member pair {x, y} makes a connected 4-set; it is kept when {a, b} is
// its smallest dominating edge.  FILL: write (a, b, x, y) to out (a counter
// in ctr[0]); else count into ctr[1].
template <bool FILL>
__global__ __launch_bounds__(64 * kWaves6) void k6_anchors(DevGraph G, int4* __restrict__ out,
                                                            unsigned long long* __restrict__ ctr,
                                                            unsigned long long cap, int32_t* st) {
  __shared__ uint32_t hkey[kWaves6][kHash6];
  __shared__ uint32_t hlab[kWaves6][kHash6];
  __shared__ int32_t mem[kWaves6][kMembers6];
  __shared__ uint32_t mlab[kWaves6][kMembers6];
  __shared__ int32_t nmem[kWaves6];
  if (st[kStatus] != 0) return;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* key = hkey[wv];
  uint32_t* lab = hlab[wv];
  for (int i = lane; i < kHash6; i += 64) {
    key[i] = kEmpty6;
    lab[i] = 0u;
  }
  if (lane == 0) nmem[wv] = 0;
  wave_sync6();
  unsigned long long counted = 0;
  const int64_t total = G.gs_off[G.n];
  const int64_t nwaves = (int64_t)gridDim.x * kWaves6;
  for (int64_t e = blockIdx.x * (int64_t)kWaves6 + wv; e < total; e += nwaves) {
    const int32_t b = (int32_t)(G.gs_idx[e] & kIdMask);
    // the row of e: last a with gs_off[a] <= e
    int32_t lo = 0, hi = G.n - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (G.gs_off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int32_t a = lo;
    if (b <= a) continue;  // each edge once (uniform over the wave)
    const int32_t ra = G.gs_off[a], da = G.gs_off[a + 1] - ra, rb = G.gs_off[b], db = G.gs_off[b + 1] - rb;
    if (da + db > kMembers6) {
      if (lane == 0) atomicMin(&st[kStatus], MOTIF_ETOOBIG);
      return;
    }
    // labels: bits 0-1 type towards a, bits 2-3 type towards b
    for (int side = 0; side < 2; ++side) {
      const int32_t r0 = side ? rb : ra, d0 = side ? db : da, other = side ? a : b;
      for (int32_t i = lane; i < d0; i += 64) {
        const uint32_t f = G.gs_idx[r0 + i];
        const uint32_t x = f & kIdMask;
        if ((int32_t)x == other) continue;
        uint32_t h = (x * 2654435761u) >> (32 - 11);
        for (;;) {
          const uint32_t old = atomicCAS(&key[h], kEmpty6, x);
          if (old == kEmpty6) {
            const int32_t slot = atomicAdd(&nmem[wv], 1);
            mem[wv][slot] = (int32_t)x;
            mlab[wv][slot] = h;  // the member's hash slot, its label read below
          }
          if (old == kEmpty6 || old == x) {
            atomicOr(&lab[h], (f >> kTypeShift) << (2 * side));
            break;
          }
          h = (h + 1) & (kHash6 - 1);
        }
      }
      wave_sync6();
    }
    const int32_t M = nmem[wv];
    for (int32_t i = lane; i < M; i += 64) mlab[wv][i] = lab[mlab[wv][i]];
    wave_sync6();
    const int64_t npairs = (int64_t)M * (M - 1) / 2;
    const unsigned long long keep_ab = ((unsigned long long)a << 32) | (unsigned)b;
    for (int64_t t0 = 0; t0 < npairs; t0 += 64) {
      const int64_t t = t0 + lane;
      bool keep = false;
      int32_t x = 0, y = 0;
      if (t < npairs) {
        // pair (i, j), i < j, of index t in row-major order of the upper triangle
        int32_t i = (int32_t)((2 * M - 1 - sqrt((double)(2 * M - 1) * (2 * M - 1) - 8.0 * (double)t)) / 2);
        if (i < 0) i = 0;
        while (i > 0 && (int64_t)i * (2 * M - i - 1) / 2 > t) --i;
        while ((int64_t)(i + 1) * (2 * M - i - 2) / 2 <= t) ++i;
        const int32_t j = i + 1 + (int32_t)(t - (int64_t)i * (2 * M - i - 1) / 2);
        x = mem[wv][i];
        y = mem[wv][j];
        const uint32_t lx = mlab[wv][i], ly = mlab[wv][j];
        // undirected adjacency of {a, b, x, y} as 4-bit rows (0 = a, 1 = b, 2 = x, 3 = y)
        const bool xy = gs_type(G, x, y) != 0u;
        uint32_t adj[4];
        adj[0] = 2u | ((lx & 3u) ? 4u : 0u) | ((ly & 3u) ? 8u : 0u);
        adj[1] = 1u | ((lx >> 2) ? 4u : 0u) | ((ly >> 2) ? 8u : 0u);
        adj[2] = ((lx & 3u) ? 1u : 0u) | ((lx >> 2) ? 2u : 0u) | (xy ? 8u : 0u);
        adj[3] = ((ly & 3u) ? 1u : 0u) | ((ly >> 2) ? 2u : 0u) | (xy ? 4u : 0u);
        const int32_t id[4] = {a, b, x, y};
        unsigned long long best = ~0ull;
        for (int p = 0; p < 4; ++p)
          for (int q = p + 1; q < 4; ++q) {
            if (!((adj[p] >> q) & 1u)) continue;
            bool dom = true;
            for (int w = 0; w < 4; ++w)
              if (w != p && w != q && !(((adj[w] >> p) | (adj[w] >> q)) & 1u)) dom = false;
            if (!dom) continue;
            const int32_t u = min(id[p], id[q]), v = max(id[p], id[q]);
            const unsigned long long kk = ((unsigned long long)u << 32) | (unsigned)v;
            if (kk < best) best = kk;
          }
        keep = best == keep_ab;
      }
      if (FILL) {
        const uint64_t bm = __ballot(keep);
        if (bm) {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(&ctr[0], (unsigned long long)__popcll(bm));
          base = __shfl(base, 0);
          const unsigned long long at = base + __popcll(bm & ((1ull << lane) - 1ull));
          if (keep && at < cap) out[at] = make_int4(a, b, x, y);
        }
      } else {
        counted += keep;
      }
    }
    // clear the table for the next edge
    wave_sync6();
    for (int32_t i = lane; i < M; i += 64) {
      const int32_t x = mem[wv][i];
      uint32_t h = ((uint32_t)x * 2654435761u) >> (32 - 11);
      while (key[h] != (uint32_t)x) h = (h + 1) & (kHash6 - 1);
      lab[h] = 0u;
    }
    wave_sync6();
    for (int32_t i = lane; i < M; i += 64) {
      const int32_t x = mem[wv][i];
      uint32_t h = ((uint32_t)x * 2654435761u) >> (32 - 11);
      while (key[h] != (uint32_t)x) h = (h + 1) & (kHash6 - 1);
      key[h] = kEmpty6;
    }
    if (lane == 0) nmem[wv] = 0;
    wave_sync6();
  }
  if (!FILL) {
    for (int o = 32; o; o >>= 1) counted += __shfl_xor(counted, o);
    if (lane == 0 && counted) atomicAdd(&ctr[1], counted);
  }
}

// Code bits of a labelled vertex in slot S (4 or 5): L holds its types towards
// the anchor vertices 0..3, 2 bits each (1 = arc anchor -> vertex).
template <int S>
__device__ __forceinline__ uint32_t slot6(uint32_t L) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t t = (L >> (2 * i)) & 3u;
    c |= (t & 1u) ? (1u << bit6(i, S)) : 0u;
    c |= (t & 2u) ? (1u << bit6(S, i)) : 0u;
  }
  return c;
}

constexpr int kB6 = 256;           // threads per workgroup of k6_census
constexpr int kMemCap6 = 4096;     // labelled vertices per anchor
constexpr int kAggBits6 = 10;      // class sums kept in LDS: 1,024 slots
constexpr int kAgg6 = 1 << kAggBits6;
constexpr int kAggProbe6 = 16;     // probes before a class goes straight to the accumulator

// One workgroup per anchor 4-set of the list: labels in the workgroup's byte
// slice lab (n bytes, all zero between anchors), the 255 label counts in LDS.
// The anchors' contributions are summed per class in an LDS table and added
// to acc once per class when the table is half full and at the end: many
// anchors hit the same few classes (those of two vertices joined to the
// anchor and not to each other above all), and one global atomic per
// contribution queued on those few addresses.
__global__ __launch_bounds__(kB6) void k6_census(DevGraph G, const int4* __restrict__ anchors, int64_t nanchors,
                                                 const uint32_t* __restrict__ lut, uint64_t* __restrict__ acc,
                                                 uint32_t* __restrict__ labels, int64_t label_words, int32_t* st) {
  __shared__ int32_t cnt[256];
  __shared__ int32_t mem[kMemCap6];
  __shared__ int32_t nmem, nz, nagg;
  __shared__ uint32_t zl[256];
  __shared__ uint32_t base_sh;
  __shared__ uint32_t akey[kAgg6];
  __shared__ uint64_t aval[kAgg6];
  if (st[kStatus] != 0) return;
  uint32_t* lab = labels + (int64_t)blockIdx.x * label_words;
  auto lab_get = [&](int32_t v) {
    return (__hip_atomic_load(&lab[v >> 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (8 * (v & 3))) & 0xFFu;
  };
  auto emit = [&](uint32_t code, uint64_t w) {
    const uint32_t c = lut[code];
    if (c == kNoClass) {  // a connected 6-set always has a class
      atomicMin(&st[kStatus], MOTIF_EINTERNAL);
      return;
    }
    uint32_t h = (c * 2654435761u) >> (32 - kAggBits6);
    for (int i = 0; i < kAggProbe6; ++i) {
      const uint32_t old = atomicCAS(&akey[h], kEmpty6, c);
      if (old == kEmpty6) atomicAdd(&nagg, 1);
      if (old == kEmpty6 || old == c) {
        atomicAdd(&aval[h], w);
        return;
      }
      h = (h + 1) & (kAgg6 - 1);
    }
    atomicAdd(&acc[c], w);  // a crowded stretch of the table
  };
  auto flush = [&] {  // between barriers
    for (int i = threadIdx.x; i < kAgg6; i += kB6) {
      if (akey[i] != kEmpty6) {
        atomicAdd(&acc[akey[i]], aval[i]);
        akey[i] = kEmpty6;
        aval[i] = 0;
      }
    }
  };
  cnt[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < kAgg6; i += kB6) {
    akey[i] = kEmpty6;
    aval[i] = 0;
  }
  if (threadIdx.x == 0) {
    nmem = 0;
    nz = 0;
    nagg = 0;
    base_sh = 0;
  }
  __syncthreads();
  for (int64_t q = blockIdx.x; q < nanchors; q += gridDim.x) {
    const int4 A = anchors[q];
    const int32_t t[4] = {A.x, A.y, A.z, A.w};
    auto in_t = [&](int32_t v) { return v == t[0] || v == t[1] || v == t[2] || v == t[3]; };
    // the anchor's own arcs (slots 0..3)
    if (threadIdx.x < 6) {
      const int i = threadIdx.x < 3 ? 0 : threadIdx.x < 5 ? 1 : 2;
      const int j = threadIdx.x < 3 ? threadIdx.x + 1 : threadIdx.x < 5 ? threadIdx.x - 1 : 3;
      const uint32_t ty = gs_type(G, t[i], t[j]);
      const uint32_t bits = ((ty & 1u) ? 1u << bit6(i, j) : 0u) | ((ty & 2u) ? 1u << bit6(j, i) : 0u);
      if (bits) atomicOr(&base_sh, bits);
    }
    // labels of the neighbours of T (first writer of a vertex lists it)
    for (int i = 0; i < 4; ++i) {
      const int32_t r0 = G.gs_off[t[i]], d0 = G.gs_off[t[i] + 1] - r0;
      for (int32_t e = threadIdx.x; e < d0; e += kB6) {
        const uint32_t f = G.gs_idx[r0 + e];
        const int32_t w = (int32_t)(f & kIdMask);
        if (in_t(w)) continue;
        const int sh = 8 * (w & 3);
        const uint32_t old = __hip_atomic_fetch_or(&lab[w >> 2], ((f >> kTypeShift) << (2 * i)) << sh,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (((old >> sh) & 0xFFu) == 0u) {
          const int32_t s = atomicAdd(&nmem, 1);
          if (s < kMemCap6) mem[s] = w;
          else atomicMin(&st[kStatus], MOTIF_ETOOBIG);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int32_t M = min(nmem, kMemCap6);
    const uint32_t base = base_sh;
    for (int32_t i = threadIdx.x; i < M; i += kB6) atomicAdd(&cnt[lab_get(mem[i])], 1);
    // edges between two labelled vertices, each from the N+ row of its lower-rank end
    for (int32_t i = threadIdx.x; i < M; i += kB6) {
      const int32_t x = mem[i];
      const uint32_t Lx = lab_get(x);
      for (int32_t p = G.np_off[x], pe = G.np_off[x + 1]; p < pe; ++p) {
        const uint32_t f = G.np_idx[p];
        const int32_t y = (int32_t)(f & kIdMask);
        if (in_t(y)) continue;
        const uint32_t Ly = lab_get(y);
        if (!Ly) continue;
        const uint32_t c0 = base | slot6<4>(Lx) | slot6<5>(Ly);
        const uint32_t r = f >> kTypeShift;  // type of y relative to x
        const uint32_t rel = ((r & 1u) ? 1u << bit6(4, 5) : 0u) | ((r & 2u) ? 1u << bit6(5, 4) : 0u);
        emit(c0 | rel, 1ull);
        emit(c0, ~0ull);
      }
    }
    __syncthreads();
    // closed form over the pairs of non-empty label sets
    if (cnt[threadIdx.x] > 0) zl[atomicAdd(&nz, 1)] = threadIdx.x;
    __syncthreads();
    const int32_t Z = nz;
    for (int32_t u = threadIdx.x; u < Z * (Z + 1) / 2; u += kB6) {
      int32_t i = 0, rem = u;
      while (rem >= Z - i) {
        rem -= Z - i;
        ++i;
      }
      const int32_t j = i + rem;
      const uint32_t La = zl[i], Lb = zl[j];
      const uint64_t na = (uint64_t)cnt[La], nb = (uint64_t)cnt[Lb];
      const uint64_t w = i == j ? na * (na - 1) / 2 : na * nb;
      if (w) emit(base | slot6<4>(La) | slot6<5>(Lb), w);
    }
    __syncthreads();
    // clear the labels, the counts and the anchor code
    for (int32_t i = threadIdx.x; i < M; i += kB6) {
      const int32_t w = mem[i];
      __hip_atomic_fetch_and(&lab[w >> 2], ~(0xFFu << (8 * (w & 3))), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    cnt[threadIdx.x] = 0;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const bool full = nagg > kAgg6 / 2;  // read by every thread between the same barriers
    if (full) flush();
    __syncthreads();
    if (threadIdx.x == 0) {
      nmem = 0;
      nz = 0;
      base_sh = 0;
      if (full) nagg = 0;
    }
    __syncthreads();
  }
  flush();
}

// The bit map of every relabelling of 6 vertices (lexicographic order,
// identity first): pos[p * 30 + b] = where bit b goes.
std::vector<uint8_t> perm_bit_maps6() {
  std::vector<uint8_t> pos((size_t)kPerms6 * kBits6);
  int perm[6] = {0, 1, 2, 3, 4, 5};
  for (int p = 0; p < kPerms6; ++p) {
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j)
        if (i != j) pos[(size_t)p * kBits6 + bit6(i, j)] = (uint8_t)bit6(perm[i], perm[j]);
    std::next_permutation(perm, perm + 6);
  }
  return pos;
}

}  // namespace

int32_t build_tables6(Tables6* T) {
  const std::vector<uint8_t> pos = perm_bit_maps6();
  uint8_t* dpos = nullptr;
  uint32_t *marks = nullptr, *rank = nullptr, *bsum = nullptr, *total = nullptr;
  unsigned long long* ncanon = nullptr;
  constexpr uint64_t kWords = kCodes6 / 32;  // 2^25
  constexpr int32_t kBlocks = (int32_t)(kWords / 1024);
  int32_t rc = 0;
  auto fail = [&](int32_t code) {
    rc = code;
    return code;
  };
  do {
    if (hipMalloc(&dpos, pos.size()) != hipSuccess || hipMalloc(&marks, kWords * 4) != hipSuccess ||
        hipMalloc(&rank, kWords * 4) != hipSuccess || hipMalloc(&bsum, kBlocks * 4) != hipSuccess ||
        hipMalloc(&total, 4) != hipSuccess || hipMalloc(&ncanon, 8) != hipSuccess) {
      fail(MOTIF_ENOMEM);
      break;
    }
    if (hipMemcpy(dpos, pos.data(), pos.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(marks, 0, kWords * 4) != hipSuccess || hipMemset(ncanon, 0, 8) != hipSuccess) {
      fail(MOTIF_EDEVICE);
      break;
    }
    hipLaunchKernelGGL(k6_mark, dim3(65536), dim3(256), 0, 0, dpos, marks, ncanon);
    hipLaunchKernelGGL(k6_rank_local, dim3(kBlocks), dim3(1024), 0, 0, marks, rank, bsum);
    hipLaunchKernelGGL(k6_rank_blocks, dim3(1), dim3(1024), 0, 0, bsum, kBlocks, total);
    uint32_t ncls = 0;
    unsigned long long nall = 0;
    if (hipMemcpy(&ncls, total, 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&nall, ncanon, 8, hipMemcpyDeviceToHost) != hipSuccess) {
      fail(MOTIF_EDEVICE);
      break;
    }
    // the table must hold every weakly connected digraph on 6 vertices
    // (1,530,843) among all 1,540,944 digraphs on 6 vertices
    if (ncls != (uint32_t)kClasses6 || nall != 1540944ull) {
      fail(MOTIF_EINTERNAL);
      break;
    }
    if (hipMalloc(&T->codes, sizeof(uint32_t) * ncls) != hipSuccess ||
        hipMalloc(&T->mult, ncls) != hipSuccess || hipMalloc(&T->lut, sizeof(uint32_t) * (size_t)kCodes6) != hipSuccess) {
      fail(MOTIF_ENOMEM);
      break;
    }
    hipLaunchKernelGGL(k6_codes, dim3(kBlocks), dim3(1024), 0, 0, marks, rank, bsum, T->codes, ncls);
    hipLaunchKernelGGL(k6_fill, dim3(65536), dim3(256), 0, 0, reinterpret_cast<uint4*>(T->lut),
                       (uint64_t)kCodes6 / 4, kNoClass);
    hipLaunchKernelGGL(k6_expand, dim3(8192), dim3(256), 0, 0, dpos, T->codes, ncls, T->lut);
    hipLaunchKernelGGL(k6_mult, dim3((ncls + 255) / 256), dim3(256), 0, 0, T->codes, ncls, T->mult);
    T->host_codes.resize(ncls);
    T->host_mult.resize(ncls);
    if (hipMemcpy(T->host_codes.data(), T->codes, sizeof(uint32_t) * ncls, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(T->host_mult.data(), T->mult, ncls, hipMemcpyDeviceToHost) != hipSuccess) {
      fail(MOTIF_EDEVICE);
      break;
    }
    for (uint32_t c = 0; c < ncls; ++c)
      if (T->host_mult[c] == 0 || (c > 0 && T->host_codes[c] <= T->host_codes[c - 1])) {
        fail(MOTIF_EINTERNAL);
        break;
      }
  } while (false);
  (void)hipFree(dpos);  // tear-down of temporaries: nothing to report
  (void)hipFree(marks);
  (void)hipFree(rank);
  (void)hipFree(bsum);
  (void)hipFree(total);
  (void)hipFree(ncanon);
  if (rc) free_tables6(T);
  return rc;
}

void free_tables6(Tables6* T) {
  (void)hipFree(T->lut);  // tear-down: nothing to report
  (void)hipFree(T->codes);
  (void)hipFree(T->mult);
  T->lut = nullptr;
  T->codes = nullptr;
  T->mult = nullptr;
  T->host_codes.clear();
  T->host_mult.clear();
}

int32_t enqueue_anchors6(const DevGraph& g, int4* out, unsigned long long* ctr, unsigned long long cap, bool fill,
                         int num_cus, int32_t* status, hipStream_t s) {
  const dim3 grid((unsigned)std::max(1, num_cus * 4));
  if (fill)
    hipLaunchKernelGGL((k6_anchors<true>), grid, dim3(64 * kWaves6), 0, s, g, out, ctr, cap, status);
  else
    hipLaunchKernelGGL((k6_anchors<false>), grid, dim3(64 * kWaves6), 0, s, g, out, ctr, cap, status);
  return hipGetLastError() == hipSuccess ? 0 : MOTIF_EDEVICE;
}

void enqueue_census6(const DevGraph& g, const int4* anchors, int64_t nanchors, const Tables6& T, uint64_t* acc,
                     uint32_t* labels, int64_t label_words, int grid, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k6_census, dim3((unsigned)std::max(1, grid)), dim3(kB6), 0, s, g, anchors, nanchors, T.lut, acc,
                     labels, label_words, status);
}

}  // namespace motif
