// Census kernels for k = 3, 4, 5 (gfx950, wave64) and the exact final division.
//
// Every k-set S is charged to the anchors that see it -- a vertex (k = 3,
// v-Patterns), an undirected edge of G* (k = 4, e-Patterns), a connected
// triple (k = 5, Delta-Patterns) -- and each class total is divided at the end
// by the number of anchors that see one occurrence (Fact "correction").
// Per anchor, the neighbours of the anchor are labelled by their types to the
// anchor vertices (the sets A/B/C of Section "Counting isomorphic patterns of
// size 3", the 15 sets of Section "Counting isomorphic patterns of size 4 in
// directed graphs", the 63 sets of Algorithm "partfive").  Then:
//   * pairs of neighbours with no edge between them: closed forms C(n_T,2)
//     and n_Ti * n_Tj on the set sizes (Facts "base" and "basefive");
//   * every edge between two neighbours (an "m-variable" contribution): one
//     occurrence moves from the no-edge pattern to the pattern with that edge
//     (Theorem "lema4d", Corollary "coro:a", Lemma "lema5d").
// The pattern of (anchor, label of v1, label of v2, edge v1-v2) is read from
// one lookup table on the full k(k-1)-bit code, which replaces the paper's
// hard-coded pattern matrices (pattern, pattern->, pattern<-, pattern<->).
//
// Device layout: typed id-sorted G* rows and oriented rows N+(v) (graph.hip).
// Each edge between two neighbours is found exactly once, from its endpoint of
// lower rank (d*, id), by scanning that endpoint's N+ row and reading the
// other endpoint's label.  Labels live in a dense per-workgroup array indexed
// by vertex id (LDS when it fits, else a private slice of global memory):
// 4 bits per vertex for k = 4, 8 bits for k = 5.  Class counters are uint64
// in LDS (9364 x 8 B = 73 KB for k = 5) and are flushed once per workgroup and
// graph with 64-bit global atomics, so the result does not depend on the
// schedule.  Counters wrap modulo 2^64; the intermediate "negative" values of
// the edge moves cancel exactly.
//
// k4_kernel and k5_kernel follow this per anchor.  The default kernels for
// k = 4, 5 (kr_kernel) compute the same sums with the neighbourhood of the
// highest-ranked anchor vertex scanned once for all of its anchors; for
// k = 4 small anchors run on single waves with their labels in LDS hashes,
// for k = 5 the triples of one centre and one heavier side share that
// side's sums and are corrected per lighter side.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "scan.h"

namespace motif {

namespace {

// Bit of the arc i -> j (i != j) in the adjacency codes that index the
// device class tables.  Row-major with the diagonal left out, except for
// k = 5, where the two arcs between slots 3 and 4 (the members of a pair in
// the closed forms) are moved to bits 0 and 1 and the rest keep their order
// above them: a code without that edge and its three variants with it are
// then four consecutive entries of the 2 MB table, one aligned 8-byte read
// (lut_quad) instead of two.  (For k = 4 the table sits in LDS, and the same
// order measured slightly slower.)  The host table keeps row-major order;
// device_lut_order writes the device copy in this one.
template <int K>
__host__ __device__ constexpr int cbit(int i, int j) {
  const int n = i * (K - 1) + (j < i ? j : j - 1);
  if (K != 5) return n;
  const int a = (K - 2) * K, b = (K - 1) * (K - 1) + K - 2;  // row-major bits of (3, 4) and (4, 3)
  return n == a ? 0 : n == b ? 1 : n < a ? n + 2 : n < b ? n + 1 : n;
}
static_assert(cbit<5>(3, 4) == 0 && cbit<5>(4, 3) == 1 && cbit<5>(0, 1) == 2 && cbit<5>(4, 2) == 19 &&
                  cbit<5>(3, 2) == 16 && cbit<5>(4, 0) == 17,
              "k = 5 order");

// Code bits of a neighbour placed in slot S whose types towards the anchor
// vertices 0..K-3 are packed 2 bits each in L (1 = arc anchor->x, 2 = arc
// x->anchor, 3 = both).
template <int K, int S>
__device__ __forceinline__ uint32_t slot_code(uint32_t L) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < K - 2; ++i) {
    const uint32_t t = (L >> (2 * i)) & 3u;
    c |= (t & 1u) ? (1u << cbit<K>(i, S)) : 0u;
    c |= (t & 2u) ? (1u << cbit<K>(S, i)) : 0u;
  }
  return c;
}

// Code bits of the edge between slot K-2 (x) and slot K-1 (y); t = type of y
// relative to x.
template <int K>
__device__ __forceinline__ uint32_t rel_code(uint32_t t) {
  return ((t & 1u) ? (1u << cbit<K>(K - 2, K - 1)) : 0u) | ((t & 2u) ? (1u << cbit<K>(K - 1, K - 2)) : 0u);
}

// k = 5: the classes of code c0 (no edge between slots 3 and 4) and of c0
// with that edge of each type, in one read; entry r of the word is the class
// of c0 | rel_code<5>(r), r = 0..3 (rel_code<5>(r) == r in the order of
// cbit).  lut must be 8-byte aligned.
__device__ __forceinline__ uint64_t lut_quad(const uint16_t* lut, uint32_t c0) {
  return *reinterpret_cast<const uint64_t*>(lut + c0);
}
__device__ __forceinline__ uint32_t quad_at(uint64_t q, uint32_t r) { return (uint32_t)(q >> (16u * r)) & 0xFFFFu; }

__device__ __forceinline__ uint32_t flip(uint32_t t) { return ((t & 1u) << 1) | ((t & 2u) >> 1); }

// k = 4: slot of the label pair (a, b), 1 <= a <= b <= 15, among the 120 such
// pairs (row-major upper triangle).
constexpr int kPairs4 = 120;
__device__ __forceinline__ uint32_t pair_slot4(uint32_t a, uint32_t b) {
  const uint32_t a0 = a - 1u;
  return a0 * 15u - (a0 * (a0 - 1u)) / 2u + (b - a);
}

constexpr int num_classes(int k) { return k == 3 ? 13 : k == 4 ? 199 : 9364; }

constexpr int kMaxHubs = 512;  // rows of the per-core W table in LDS
constexpr int kMaxBig = 64;          // cores whose W / M tables are built once per call
constexpr int kBigMinDeg = 256;      // ... among vertices of at least this degree
constexpr int64_t kBigBytes = 512ll << 20;  // ... within this many bytes of tables
constexpr int kBigRow = 12;          // words per W row (9 used, 16-byte aligned), big-core tables and WG slices
constexpr int kUnroll = 4;
// Smallest cost of a work-queue tile of the core-reuse kernels: on small
// graphs `tile` tiles per workgroup would cut below one core's units, and
// every tile sets its cores up again (measured best tile costs: about 135
// for k = 4 and 370-850 for k = 5 on graphs of 10^3-10^5 arcs).
constexpr int32_t kMinTileCost4 = 128;
constexpr int32_t kMinTileCost5 = 512;
constexpr int kBucketShift = 6;     // the row-scan layout records the row at every 64th entry ...
constexpr int kBuckets = 1024;      // ... for layouts of up to 64 K entries (else plain binary search)         // N+ entries per lane and pass of the flattened scans
constexpr int kLightDegMax = 256;  // cap of the k = 4 light-side limit (wave hash load <= 1/2)
constexpr int kWaveHashBits = 9;
constexpr int kWaveHash = 1 << kWaveHashBits;  // slots of the wave-private hash of N(side): load <= 1/2
constexpr uint32_t kEmptySlot = ~0u;
constexpr int kLight5Max = 767;     // cap of the k = 5 light-partner limit (a partner must fit the table alone)
constexpr int kNP5 = 32;            // light partners c per sub-chunk of a k = 5 unit (2 type bits each in 64)
constexpr int kT5Bits = 10;
constexpr int kT5 = 1 << kT5Bits;   // slots of the merged table of the sub-chunk's N(c) ...
constexpr int kT5Load = 768;        // ... holding at most this many keys (sum of d*(c) + 1)
static_assert(kLight5Max + 1 <= kT5Load, "a light partner must fit the table alone");
constexpr uint32_t kInT5 = 64u;     // label bit 6: the vertex is a key of that table
constexpr int kU5 = 16 * 48;        // per-unit move counters: (x label, y label, r), labels of 4 bits
constexpr int kSoloDegMax = 64;     // cap of the k = 4 solo-core limit (one lane per core neighbour)
constexpr int kSoloHashBits = 8;
constexpr int kSoloHash = 1 << kSoloHashBits;  // keys of the solo hash of N(c) u N(s): load < 1/2

// Work-placement limits of the core-reuse kernels, from the tuning (each
// clamped to its cap above).
struct Limits {
  int32_t solo, light, light5;
};

__device__ __forceinline__ uint32_t hash_slot(int32_t y) {
  return ((uint32_t)y * 2654435761u) >> (32 - kWaveHashBits);  // Fibonacci hashing
}

// Ordering point for LDS traffic inside one wave: LDS operations of a wave
// complete in issue order, so only the compiler has to be kept from moving
// accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

using u64 = unsigned long long;
constexpr u64 kMinusOne = ~0ull;

template <int C, int BLOCK>
__device__ __forceinline__ void hist_flush(u64* hist, uint64_t* acc, int32_t g) {
  if (g >= 0) {
    for (int c = threadIdx.x; c < C; c += BLOCK) {
      const u64 v = hist[c];
      if (v) atomicAdd((u64*)&acc[(int64_t)g * C + c], v);
      hist[c] = 0;
    }
  }
}

// Dense label array: BITS (4 or 8) bits per vertex in 32-bit words.  In LDS
// (GLOBAL = false) plain loads see the LDS atomics of other waves after a
// barrier.  In a private global slice (GLOBAL = true) the updates are device
// atomics performed in L2, so reads also go to L2 (agent-scope atomic loads
// bypass the per-CU L1, which those atomics do not update).
//
// Vertices are indexed from `base`, the first vertex of the graph being
// worked on, so that a batch of small graphs needs label room for its
// largest graph only (and keeps the labels in LDS); a kernel moves `base`
// when it moves to another graph, with every label of the previous one
// cleared.
template <int BITS, bool GLOBAL = false>
struct Labels {
  uint32_t* w;
  uint32_t base = 0;
  static constexpr int kPer = 32 / BITS;
  static constexpr uint32_t kMask = (1u << BITS) - 1u;
  __device__ __forceinline__ uint32_t word(uint32_t i) const {
    if constexpr (GLOBAL) return __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return w[i];
  }
  __device__ __forceinline__ uint32_t get(uint32_t x) const {
    x -= base;
    return (word(x / kPer) >> ((x % kPer) * BITS)) & kMask;
  }
  __device__ __forceinline__ void set_bits(uint32_t x, uint32_t v) const {
    x -= base;
    atomicOr(&w[x / kPer], v << ((x % kPer) * BITS));
  }
  __device__ __forceinline__ void clear_bits(uint32_t x, uint32_t v) const {
    x -= base;
    atomicAnd(&w[x / kPer], ~(v << ((x % kPer) * BITS)));
  }
  __device__ __forceinline__ void clear_all(uint32_t x) const {
    x -= base;
    if constexpr (GLOBAL) __hip_atomic_store(&w[x / kPer], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else w[x / kPer] = 0u;
  }
};

// Workgroup barrier.  With GLOBAL, first wait until every memory operation of
// this wave has completed (global atomics included: the plain barrier only
// waits for LDS traffic), so state kept in a private global slice is
// consistent for all waves after it.
template <bool GLOBAL>
__device__ __forceinline__ void bar() {
  if constexpr (GLOBAL) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

__device__ __forceinline__ int32_t find_row(const int32_t* off, int32_t lo, int32_t hi, int64_t j) {
  // last v in [lo, hi) with off[v] <= j
  hi -= 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ================================================================== k = 3 ==
//
// Anchor = vertex v (Definition "v-Patterns").  Closed form per vertex: the
// six pair counts n_a n_b, n_a n_c, n_b n_c, C(n_a,2), C(n_b,2), C(n_c,2)
// (Figure "star").  Edges between two neighbours of v are exactly the
// triangles at v (Algorithm "alternative"), listed once each as
// u -> w -> x in rank order: x in N+(u) and in N+(w).  For each corner the
// pair of the other two corners leaves its open class, and the triangle class
// gains one occurrence per corner (the division by 3 removes the repetition).
//
// One wave per vertex u, vertices handed out in chunks from a device counter
// so that every wave of the chip stays busy and a heavy vertex delays only
// its own wave.  The wave counts the types of u's row with ballots (a hub's
// row is read 64 entries at a time), adds the six closed forms, puts N+(u)
// into a wave-private LDS hash (vertex -> type), lays the N+ rows of its
// members end to end over the lanes and looks every entry x up: a hit is a
// triangle.  A u with more than kTriHash / 2 higher-ranked neighbours
// binary-searches N+(u) instead of the hash.  Counts go to a per-wave LDS
// histogram, flushed when the wave's vertex moves to another graph of a batch.
constexpr int kTriHashBits = 10;
constexpr int kTriHash = 1 << kTriHashBits;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k3_kernel(DevGraph G, const uint16_t* __restrict__ lut_g,
                                                   uint64_t* __restrict__ acc, const int32_t* st,
                                                   int32_t* __restrict__ queue, int32_t chunk) {
  constexpr int K = 3, C = 13, NW = BLOCK / 64;
  __shared__ u64 whist[NW * 16];
  __shared__ uint16_t lut[64];
  __shared__ uint32_t th[NW * kTriHash];
  __shared__ uint16_t tslot[NW * (kTriHash / 2)];  // slot of each key of N+(u), to empty exactly those
  if (st[kStatus] != 0) return;
  for (int i = threadIdx.x; i < 64; i += BLOCK) lut[i] = lut_g[i];
  for (int i = threadIdx.x; i < NW * 16; i += BLOCK) whist[i] = 0;
  for (int i = threadIdx.x; i < NW * kTriHash; i += BLOCK) th[i] = kEmptySlot;
  __syncthreads();
  const int32_t lane = (int32_t)(threadIdx.x & 63u);
  uint32_t* H = th + (threadIdx.x >> 6) * kTriHash;
  uint16_t* HS = tslot + (threadIdx.x >> 6) * (kTriHash / 2);
  u64* hist = whist + (threadIdx.x >> 6) * 16;
  auto tri = [&](uint32_t tuw, uint32_t tux, uint32_t twx) {
    const uint32_t full = slot_code<K, 1>(tuw) | slot_code<K, 2>(tux) | rel_code<K>(twx);
    atomicAdd(&hist[lut[full]], 3ull);
    atomicAdd(&hist[lut[slot_code<K, 1>(tuw) | slot_code<K, 2>(tux)]], kMinusOne);
    atomicAdd(&hist[lut[slot_code<K, 1>(flip(tuw)) | slot_code<K, 2>(twx)]], kMinusOne);
    atomicAdd(&hist[lut[slot_code<K, 1>(flip(tux)) | slot_code<K, 2>(flip(twx))]], kMinusOne);
  };
  auto flush = [&](int32_t g) {  // this wave's counts to graph g's accumulator
    wave_sync();
    if (g >= 0 && lane < C) {
      const u64 v = hist[lane];
      if (v) atomicAdd((u64*)&acc[(int64_t)g * C + lane], v);
    }
    if (lane < C) hist[lane] = 0;
    wave_sync();
  };
  const int32_t n = G.n;
  int32_t cur_g = -1;
  for (;;) {
    int32_t v0 = 0;
    if (lane == 0) v0 = atomicAdd(queue, chunk);
    v0 = __shfl(v0, 0);
    if (v0 >= n) break;
    const int32_t v1 = min(n, v0 + chunk);
    for (int32_t u = v0; u < v1; ++u) {
      const int32_t g = G.gid ? G.gid[u] : 0;
      if (g != cur_g) {
        flush(cur_g);
        cur_g = g;
      }
      // type counts of u's row: 1 = B, 2 = C, 3 = A
      const int32_t ra = G.gs_off[u], rb = G.gs_off[u + 1];
      uint32_t nb = 0, nc = 0, na = 0;
      for (int32_t j0 = ra; j0 < rb; j0 += 64) {
        const int32_t j = j0 + lane;
        const uint32_t t = j < rb ? G.gs_idx[j] >> kTypeShift : 0u;
        nb += (uint32_t)__popcll(__ballot(t == 1u));
        nc += (uint32_t)__popcll(__ballot(t == 2u));
        na += (uint32_t)__popcll(__ballot(t == 3u));
      }
      if (lane < 6) {
        const uint32_t ta = lane < 2 ? 3u : lane == 2 ? 1u : lane == 3 ? 3u : lane == 4 ? 1u : 2u;
        const uint32_t tb = lane == 0 ? 1u : lane == 1 ? 2u : lane == 2 ? 2u : lane == 3 ? 3u : lane == 4 ? 1u : 2u;
        const u64 x = lane == 0 ? (u64)na * nb : lane == 1 ? (u64)na * nc : lane == 2 ? (u64)nb * nc
                    : lane == 3 ? (u64)na * (na - (na > 0)) / 2 : lane == 4 ? (u64)nb * (nb - (nb > 0)) / 2
                                                                : (u64)nc * (nc - (nc > 0)) / 2;
        if (x) atomicAdd(&hist[lut[slot_code<K, 1>(ta) | slot_code<K, 2>(tb)]], x);
      }
      // triangles u -> w -> x
      const int32_t ua = G.np_off[u], du = G.np_off[u + 1] - ua;
      if (du < 2) continue;
      const bool hashed = du <= kTriHash / 2;
      if (hashed) {
        for (int32_t i = lane; i < du; i += 64) {
          const uint32_t e = G.np_idx[ua + i];
          uint32_t h = ((e & kIdMask) * 2654435761u) >> (32 - kTriHashBits);
          const uint32_t ent = ((e & kIdMask) << 2) | (e >> kTypeShift);  // id < 2^30 - 1: never kEmptySlot
          while (atomicCAS(&H[h], kEmptySlot, ent) != kEmptySlot) h = (h + 1) & (kTriHash - 1);
          HS[i] = (uint16_t)h;  // du <= kTriHash / 2: i in range
        }
        wave_sync();
      }
      for (int32_t i0 = 0; i0 < du; i0 += 64) {
        // lanes take members w of N+(u); their rows are laid end to end
        const int32_t i = i0 + lane;
        int32_t len = 0, rb2 = 0;
        uint32_t tuw = 0;
        if (i < du) {
          const uint32_t e = G.np_idx[ua + i];
          const int32_t w = (int32_t)(e & kIdMask);
          tuw = e >> kTypeShift;
          rb2 = G.np_off[w];
          len = G.np_off[w + 1] - rb2;
        }
        int32_t inc = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int32_t tt = __shfl_up(inc, d);
          if (lane >= d) inc += tt;
        }
        const int32_t tot = __shfl(inc, 63);
        const int32_t rs = rb2 - (inc - len);
        for (int32_t jb = 0; jb < tot; jb += 64 * kUnroll) {
          uint32_t fs[kUnroll], ts[kUnroll];
#pragma unroll
          for (int uu = 0; uu < kUnroll; ++uu) {
            const int32_t j = jb + uu * 64 + lane;
            int32_t sl = 0;
#pragma unroll
            for (int st2 = 32; st2; st2 >>= 1)
              if (__shfl(inc, sl + st2 - 1) <= j) sl += st2;
            ts[uu] = (uint32_t)__shfl((int32_t)tuw, sl);
            const int32_t srs = __shfl(rs, sl);
            fs[uu] = j < tot ? G.np_idx[srs + j] : 0u;
          }
#pragma unroll
          for (int uu = 0; uu < kUnroll; ++uu) {
            if (jb + uu * 64 + lane >= tot) continue;
            const uint32_t f = fs[uu], x = f & kIdMask;
            uint32_t tux = 0;
            if (hashed) {
              uint32_t h = (x * 2654435761u) >> (32 - kTriHashBits);
              for (;;) {
                const uint32_t e = H[h];
                if (e == kEmptySlot) break;
                if ((e >> 2) == x) {
                  tux = e & 3u;
                  break;
                }
                h = (h + 1) & (kTriHash - 1);
              }
            } else {
              int32_t lo = ua, hi = ua + du;
              while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if ((G.np_idx[mid] & kIdMask) < x) lo = mid + 1; else hi = mid;
              }
              if (lo < ua + du && (G.np_idx[lo] & kIdMask) == x) tux = G.np_idx[lo] >> kTypeShift;
            }
            if (tux) tri(ts[uu], tux, f >> kTypeShift);
          }
        }
      }
      if (hashed) {
        wave_sync();
        for (int32_t i = lane; i < du; i += 64) H[HS[i]] = kEmptySlot;  // the slots this vertex filled
        wave_sync();
      }
    }
  }
  flush(cur_g);
}

// Closed form over the non-empty neighbour sets of one anchor: pairs within a
// set, C(n,2), and across two sets, n_i n_j (Facts "base" / "basefive").
template <int K, int NL, int BLOCK>
__device__ __forceinline__ void closed_form(u64* hist, const uint16_t* lut, const int32_t* cnt, int32_t* nzl,
                                            int32_t* nz_count, uint32_t base) {
  static_assert(NL <= 64, "one label per lane of the first wave");
  if (threadIdx.x < 64) {  // the non-empty sets, compacted by a ballot of the first wave
    const int32_t lane = (int32_t)threadIdx.x;
    const bool nz = lane > 0 && lane < NL && cnt[lane] != 0;
    const unsigned long long m = __ballot(nz);
    if (nz) nzl[__popcll(m & ((1ull << lane) - 1ull))] = lane;
    if (lane == 0) *nz_count = __popcll(m);
  }
  __syncthreads();
  const int32_t z = *nz_count;
  for (int32_t q = threadIdx.x; q < z * z; q += BLOCK) {
    const int32_t a = q / z, b = q - a * z;
    if (a > b) continue;
    const uint32_t La = (uint32_t)nzl[a], Lb = (uint32_t)nzl[b];
    const u64 na = (u64)cnt[La], nb = (u64)cnt[Lb];
    const u64 w = a == b ? na * (na - 1) / 2 : na * nb;
    if (w) atomicAdd(&hist[lut[base | slot_code<K, K - 2>(La) | slot_code<K, K - 1>(Lb)]], w);
  }
}

// ================================================================== k = 4 ==
//
// Anchor = undirected edge e = {u, v} of G*, visited once (from the row of
// its smaller id; Definition "e-Patterns", iterated over E* so that a
// bidirected pair is one anchor).  Slot 0 = u, slot 1 = v.  Neighbour label =
// (type to u) | (type to v) << 2: one of the 15 sets A1..C2, AA..CC.
template <int BLOCK, int LCAP>
__global__ __launch_bounds__(BLOCK) void k4_kernel(DevGraph G, const uint16_t* __restrict__ lut_g,
                                                   uint64_t* __restrict__ acc, const int32_t* st,
                                                   int32_t* __restrict__ queue, uint32_t* __restrict__ glabels,
                                                   int64_t label_words, int32_t tile) {
  constexpr int K = 4, C = 199, NL = 16;
  __shared__ u64 hist[C];
  __shared__ uint16_t lut[4096];
  __shared__ int32_t cnt[NL], nzl[NL], nz_count;
  __shared__ int32_t sh_j0;
  __shared__ uint32_t lds_labels[LCAP > 0 ? LCAP / 4 : 1];
  if (st[kStatus] != 0) return;
  Labels<4, LCAP == 0> lab{LCAP > 0 ? lds_labels : glabels + (int64_t)blockIdx.x * label_words};
  for (int i = threadIdx.x; i < 4096; i += BLOCK) lut[i] = lut_g[i];
  for (int i = threadIdx.x; i < C; i += BLOCK) hist[i] = 0;
  if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
  if (LCAP > 0)
    for (int i = threadIdx.x; i < LCAP / 4; i += BLOCK) lds_labels[i] = 0u;
  bar<LCAP == 0>();

  const int32_t n = G.n;
  const int32_t total = G.gs_off[n];
  int32_t cur_g = -1, u = 0;
  for (;;) {
    if (threadIdx.x == 0)  // 64-bit cursor: pulls past the end never wrap
      sh_j0 = (int32_t)min((u64)total, (u64)atomicAdd(reinterpret_cast<u64*>(queue), (u64)tile));
    bar<LCAP == 0>();
    const int32_t j0 = sh_j0;
    bar<LCAP == 0>();
    if (j0 >= total) break;
    const int32_t j1 = min(total, j0 + tile);
    u = find_row(G.gs_off, 0, n, j0);
    for (int32_t j = j0; j < j1; ++j) {
      while (G.gs_off[u + 1] <= j) ++u;
      const uint32_t ev = G.gs_idx[j];
      const int32_t v = (int32_t)(ev & kIdMask);
      if (v < u) continue;  // each undirected edge once
      const int32_t g = G.gid ? G.gid[u] : 0;
      if (g != cur_g) {
        hist_flush<C, BLOCK>(hist, acc, cur_g);
        cur_g = g;
        lab.base = G.voff ? (uint32_t)G.voff[g] : 0u;  // every label of the previous anchor is cleared
        bar<LCAP == 0>();
      }
      const uint32_t tuv = ev >> kTypeShift;
      const uint32_t base = ((tuv & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tuv & 2u) ? 1u << cbit<K>(1, 0) : 0u);
      const int32_t ua = G.gs_off[u], du = G.gs_off[u + 1] - ua;
      const int32_t va = G.gs_off[v], dv = G.gs_off[v + 1] - va;
      // 1. labels: type to u in bits 0-1, type to v in bits 2-3
      for (int32_t i = threadIdx.x; i < du + dv; i += BLOCK) {
        if (i < du) {
          const uint32_t e = G.gs_idx[ua + i];
          const uint32_t x = e & kIdMask;
          if ((int32_t)x != v) lab.set_bits(x, e >> kTypeShift);
        } else {
          const uint32_t e = G.gs_idx[va + i - du];
          const uint32_t x = e & kIdMask;
          if ((int32_t)x != u) lab.set_bits(x, (e >> kTypeShift) << 2);
        }
      }
      bar<LCAP == 0>();
      // 2. set sizes and edges inside adj(e)
      for (int32_t i = threadIdx.x; i < du + dv; i += BLOCK) {
        uint32_t x;
        if (i < du) {
          x = G.gs_idx[ua + i] & kIdMask;
          if ((int32_t)x == v) continue;
        } else {
          x = G.gs_idx[va + i - du] & kIdMask;
          if ((int32_t)x == u || (lab.get(x) & 3u)) continue;  // counted from u's row
        }
        const uint32_t L = lab.get(x);
        atomicAdd(&cnt[L], 1);
        const uint32_t cx = base | slot_code<K, 2>(L);
        for (int32_t p = G.np_off[x]; p < G.np_off[x + 1]; ++p) {
          const uint32_t f = G.np_idx[p];
          const uint32_t Ly = lab.get(f & kIdMask);
          if (Ly) {
            const uint32_t c0 = cx | slot_code<K, 3>(Ly);
            atomicAdd(&hist[lut[c0 | rel_code<K>(f >> kTypeShift)]], 1ull);
            atomicAdd(&hist[lut[c0]], kMinusOne);
          }
        }
      }
      bar<LCAP == 0>();
      // 3. closed form over the 15 sets
      closed_form<K, NL, BLOCK>(hist, lut, cnt, nzl, &nz_count, base);
      bar<LCAP == 0>();
      // 4. reset
      for (int32_t i = threadIdx.x; i < du + dv; i += BLOCK) {
        const uint32_t x = (i < du ? G.gs_idx[ua + i] : G.gs_idx[va + i - du]) & kIdMask;
        lab.clear_all(x);
      }
      if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
      bar<LCAP == 0>();
    }
  }
  hist_flush<C, BLOCK>(hist, acc, cur_g);
}

// ================================================================== k = 5 ==
//
// Anchor = connected triple T (Definition "Delta-Patterns"), enumerated once:
// for a centre b and two neighbours a, c of b (a before c in b's row) the
// triple {a, b, c} is an induced path centred at b when a and c are not
// adjacent; when they are, it is a triangle and is taken only at its
// smallest-id vertex (Algorithm "calckp": each triple once).  Slots: 0 = b,
// 1 = a, 2 = c.  Neighbour label = (type to b) | (type to a) << 2 |
// (type to c) << 4: one of the 63 sets of Algorithm "partfive".  A work unit
// is one entry (b, a) of b's row; N(b) labels stay set across consecutive
// units of the same centre, N(a) across the unit, N(c) per triple.
template <int BLOCK, int LCAP>
__global__ __launch_bounds__(BLOCK) void k5_kernel(DevGraph G, const uint16_t* __restrict__ lut,
                                                   uint64_t* __restrict__ acc, const int32_t* st,
                                                   int32_t* __restrict__ queue, uint32_t* __restrict__ glabels,
                                                   int64_t label_words, int32_t tile) {
  constexpr int K = 5, C = 9364, NL = 64;
  __shared__ u64 hist[C];
  __shared__ int32_t cnt[NL], nzl[NL], nz_count;
  __shared__ int32_t sh_j0;
  __shared__ uint32_t lds_labels[LCAP > 0 ? LCAP / 4 : 1];
  if (st[kStatus] != 0) return;
  Labels<8, LCAP == 0> lab{LCAP > 0 ? lds_labels : glabels + (int64_t)blockIdx.x * label_words};
  for (int i = threadIdx.x; i < C; i += BLOCK) hist[i] = 0;
  if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
  if (LCAP > 0)
    for (int i = threadIdx.x; i < LCAP / 4; i += BLOCK) lds_labels[i] = 0u;
  bar<LCAP == 0>();

  const int32_t n = G.n;
  const int32_t total = G.gs_off[n];
  int32_t cur_g = -1, b = 0, cur_b = -1;
  for (;;) {
    if (threadIdx.x == 0)  // 64-bit cursor: pulls past the end never wrap
      sh_j0 = (int32_t)min((u64)total, (u64)atomicAdd(reinterpret_cast<u64*>(queue), (u64)tile));
    bar<LCAP == 0>();
    const int32_t j0 = sh_j0;
    bar<LCAP == 0>();
    if (j0 >= total) break;
    const int32_t j1 = min(total, j0 + tile);
    b = find_row(G.gs_off, 0, n, j0);
    for (int32_t j = j0; j < j1; ++j) {
      while (G.gs_off[b + 1] <= j) ++b;
      const int32_t ba = G.gs_off[b], bend = G.gs_off[b + 1];
      if (j + 1 >= bend) continue;  // no partner c after a in b's row
      if (b != cur_b) {
        if (cur_b >= 0) {
          for (int32_t i = G.gs_off[cur_b] + threadIdx.x; i < G.gs_off[cur_b + 1]; i += BLOCK)
            lab.clear_bits(G.gs_idx[i] & kIdMask, 3u);
        }
        bar<LCAP == 0>();
        lab.base = G.voff ? (uint32_t)G.voff[G.gid[b]] : 0u;  // the previous centre's labels are cleared
        for (int32_t i = ba + threadIdx.x; i < bend; i += BLOCK) {
          const uint32_t e = G.gs_idx[i];
          lab.set_bits(e & kIdMask, e >> kTypeShift);
        }
        cur_b = b;
      }
      const int32_t g = G.gid ? G.gid[b] : 0;
      if (g != cur_g) {
        hist_flush<C, BLOCK>(hist, acc, cur_g);
        cur_g = g;
      }
      const uint32_t ea = G.gs_idx[j];
      const int32_t a = (int32_t)(ea & kIdMask);
      const uint32_t tba = ea >> kTypeShift;
      const int32_t aa = G.gs_off[a], da = G.gs_off[a + 1] - aa;
      for (int32_t i = threadIdx.x; i < da; i += BLOCK) {
        const uint32_t e = G.gs_idx[aa + i];
        lab.set_bits(e & kIdMask, (e >> kTypeShift) << 2);
      }
      bar<LCAP == 0>();
      for (int32_t jc = j + 1; jc < bend; ++jc) {
        const uint32_t ec = G.gs_idx[jc];
        const int32_t c = (int32_t)(ec & kIdMask);
        const uint32_t tbc = ec >> kTypeShift;
        const uint32_t tac = (lab.get((uint32_t)c) >> 2) & 3u;
        if (tac && (b > a || b > c)) continue;  // triangle: taken at its smallest id
        const uint32_t base = ((tba & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tba & 2u) ? 1u << cbit<K>(1, 0) : 0u) |
                              ((tbc & 1u) ? 1u << cbit<K>(0, 2) : 0u) | ((tbc & 2u) ? 1u << cbit<K>(2, 0) : 0u) |
                              ((tac & 1u) ? 1u << cbit<K>(1, 2) : 0u) | ((tac & 2u) ? 1u << cbit<K>(2, 1) : 0u);
        const int32_t ca = G.gs_off[c], dc = G.gs_off[c + 1] - ca;
        for (int32_t i = threadIdx.x; i < dc; i += BLOCK) {
          const uint32_t e = G.gs_idx[ca + i];
          lab.set_bits(e & kIdMask, (e >> kTypeShift) << 4);
        }
        bar<LCAP == 0>();
        const int32_t db = bend - ba;
        for (int32_t i = threadIdx.x; i < db + da + dc; i += BLOCK) {
          uint32_t x;
          if (i < db) {
            x = G.gs_idx[ba + i] & kIdMask;
            if ((int32_t)x == a || (int32_t)x == c) continue;
          } else if (i < db + da) {
            x = G.gs_idx[aa + i - db] & kIdMask;
            if ((int32_t)x == b || (int32_t)x == c || (lab.get(x) & 3u)) continue;
          } else {
            x = G.gs_idx[ca + i - db - da] & kIdMask;
            if ((int32_t)x == a || (int32_t)x == b || (lab.get(x) & 15u)) continue;
          }
          const uint32_t L = lab.get(x) & 63u;
          atomicAdd(&cnt[L], 1);
          const uint32_t cx = base | slot_code<K, 3>(L);
          for (int32_t p = G.np_off[x]; p < G.np_off[x + 1]; ++p) {
            const uint32_t f = G.np_idx[p];
            const int32_t y = (int32_t)(f & kIdMask);
            const uint32_t Ly = lab.get((uint32_t)y) & 63u;
            if (Ly && y != a && y != b && y != c) {
              const uint32_t c0 = cx | slot_code<K, 4>(Ly);
              atomicAdd(&hist[lut[c0 | rel_code<K>(f >> kTypeShift)]], 1ull);
              atomicAdd(&hist[lut[c0]], kMinusOne);
            }
          }
        }
        bar<LCAP == 0>();
        closed_form<K, NL, BLOCK>(hist, lut, cnt, nzl, &nz_count, base);
        bar<LCAP == 0>();
        for (int32_t i = threadIdx.x; i < dc; i += BLOCK) lab.clear_bits(G.gs_idx[ca + i] & kIdMask, 3u << 4);
        if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
        bar<LCAP == 0>();
      }
      // Skipped triples read a-labels without a barrier: every wave must have
      // left the triple loop before any wave clears them, or a late wave would
      // see "not adjacent" for a skipped triangle and fall out of barrier step.
      bar<LCAP == 0>();
      for (int32_t i = threadIdx.x; i < da; i += BLOCK) lab.clear_bits(G.gs_idx[aa + i] & kIdMask, 3u << 2);
      bar<LCAP == 0>();
    }
  }
  if (cur_b >= 0) {
    for (int32_t i = G.gs_off[cur_b] + threadIdx.x; i < G.gs_off[cur_b + 1]; i += BLOCK)
      lab.clear_bits(G.gs_idx[i] & kIdMask, 3u);
  }
  bar<LCAP == 0>();
  hist_flush<C, BLOCK>(hist, acc, cur_g);
}

// ======================================================= core reuse ==
//
// The same sums as k4_kernel / k5_kernel, reorganised so that the
// neighbourhood of the highest-ranked anchor vertex is scanned once per work
// unit instead of once per anchor.  Core kappa = the higher-rank endpoint of
// the anchor edge (k = 4) or the centre b of the connected triple (k = 5);
// the other anchor vertices are the "sides".  Per core, once:
//   M[tx][ty][r] = edges x -> y (N+ orientation) with both ends in N(kappa),
//                  by the types of x, y towards kappa and the edge type r;
//   W[q][tp][r]  = edges p -> q (N+ orientation, p in N(kappa)) for every q.
// Per anchor, with R' = (sides and their neighbours) \ {kappa}, the edges
// inside adj(anchor) are
//   sum over M with core-only labels
//   - the edges of M that touch R'   (scanned from R' or counted in W)
//   + the same edges with their true labels when both ends are in adj(anchor),
// where edges touching R' are found from the N+ row of their lower-rank end
// when that end is in R', and otherwise counted in W[q] for q in R' (minus
// the part already found from R').  The set sizes of the closed form for
// core-only neighbours are the type counts of N(kappa) minus those in R'.
//
// W is a private global slice per workgroup, 16 uint32 per vertex of the
// largest graph (indexed by the vertex's position in its graph), except for
// the hub vertices, whose rows sit in LDS.
//
// Every scan of a list of N+ rows (the rows of N(kappa) at set-up and
// tear-down, the rows of R' per anchor) is flattened: the rows of up to BLOCK
// listed vertices are laid end to end and dealt out one entry per thread, so
// the work of an anchor is spread over the whole workgroup whatever the row
// lengths.
template <int K, int BLOCK, int LCAP>
__global__ __launch_bounds__(BLOCK) void kr_kernel(DevGraph G, const uint16_t* __restrict__ lut_g,
                                                   uint64_t* __restrict__ acc, const int32_t* st,
                                                   int32_t* __restrict__ queue, uint32_t* __restrict__ glabels,
                                                   int64_t label_words, const int32_t* __restrict__ hub_id,
                                                   uint32_t* __restrict__ wg, int64_t w_stride, int32_t tile,
                                                   const int32_t* __restrict__ cpre,
                                                   const int32_t* __restrict__ big_id,
                                                   const uint32_t* __restrict__ wbig, int64_t wbig_stride,
                                                   const uint32_t* __restrict__ mbig, Limits lim) {
  constexpr int C = K == 4 ? 199 : 9364, NL = K == 4 ? 16 : 64, LB = K == 4 ? 4 : 8;
  constexpr int S1 = K - 2, S2 = K - 1;  // member slots
  // LDS rows of W: fewer where the k = 5 counters and labels leave no room
  constexpr int HUBS = (K == 5 && LCAP == 32768) ? 80 : (K == 4 && LCAP == 65536) ? 384 : kMaxHubs;
  constexpr bool GL = LCAP == 0;
  __shared__ u64 hist[C];
  __shared__ uint16_t lut_lds[K == 4 ? 4096 : 1];
  __shared__ int32_t cnt[NL], nzl[NL], nz_count;
  __shared__ uint32_t Mc[27];
  __shared__ uint32_t W[HUBS * 9];
  __shared__ int32_t ncore[4];
  __shared__ int32_t sh_j0, sh_j1;
  __shared__ u64 seg_ctr[2];  // (rows << 32) | entries of the chunk being laid out
  constexpr int NW = BLOCK / 64;
  // k = 4: per anchor, the inner-edge moves counted per label pair (a <= b)
  // and arc type, 32-bit wrapping (per anchor they stay far inside int32);
  // the classes and the no-edge halves are added once, in the closed form.
  // The wave paths' tables share the row-scan layout's words: the two are
  // never in use at the same time (workgroup phases are barrier-separated).
  constexpr int TW = K == 4 ? kPairs4 * 3 : 0;
  constexpr int SEGW = 4 * BLOCK + kBuckets;  // with one word of row information per row
  constexpr int POOLW = NW * TW > SEGW ? NW * TW : SEGW;
  __shared__ __align__(16) int32_t seg_pool[POOLW];
  int32_t* const seg_v = seg_pool;
  int32_t* const seg_start = seg_pool + BLOCK;
  int32_t* const seg_base = seg_pool + 2 * BLOCK;
  int32_t* const seg_at = seg_pool + 3 * BLOCK;
  int32_t* const seg_lab = seg_pool + 3 * BLOCK + kBuckets;  // rowinfo of each laid-out row
  uint32_t* const wT = reinterpret_cast<uint32_t*>(seg_pool);
  constexpr int WH = K == 4 ? kWaveHash : 0;  // per-wave hash words
  constexpr int NCN = K == 4 ? NW : kNP5;     // set-size rows: one per wave (k = 4), per light partner (k = 5)
  __shared__ uint32_t wh[K == 4 ? NW * WH : 1];  // light anchors: per-wave hashes of the sides' neighbourhoods
  __shared__ int32_t wcnt[NCN * NL];
  // k = 5 light partners of one unit: merged table of their neighbourhoods
  // (vertex -> 2 type bits per partner, partner index + 1 of the vertex
  // itself), per-unit move counters, the a-part set sizes, the partners
  constexpr int T5 = K == 5 ? kT5 : 1, P5 = K == 5 ? kNP5 : 1;
  __shared__ uint32_t tkey[T5];
  __shared__ u64 ttyp[T5];
  __shared__ uint8_t tpid[T5];
  __shared__ uint32_t U5[K == 5 ? kU5 : 1];
  // two buffers: the partner set of the next sub-chunk is chosen while the
  // current one finishes; sb is the buffer of the current sub-chunk
  __shared__ int32_t cnUb[2][16];
  __shared__ int32_t p5_vb[2][P5], p5_rowb[2][P5], p5_offb[2][P5], p5_ctlb[2][5], p5_dc[P5];
  __shared__ uint16_t tlist[K == 5 ? kT5Load : 1];  // slots of the table's keys
  __shared__ uint32_t p5_baseb[2][P5], p5_db[P5];
  // k = 4: the workgroup path's move table (kept zero between anchors), and
  // the label pair (a, b) of each table slot
  __shared__ __align__(16) uint32_t bT[K == 4 ? TW : 1];
  __shared__ uint8_t pair_a[K == 4 ? kPairs4 : 1], pair_b[K == 4 ? kPairs4 : 1];
  __shared__ int32_t unit_list[BLOCK], unit_ctr[3];
  __shared__ int32_t lbk[K == 4 ? 32 : 1];  // k = 4 light units: counts and fills per log2 degree bucket
  __shared__ uint32_t lds_labels[LCAP > 0 ? LCAP / 4 : 1];
  if (st[kStatus] != 0) return;
  Labels<LB, GL> lab{LCAP > 0 ? lds_labels : glabels + (int64_t)blockIdx.x * label_words};
  uint32_t* WG = wg + (int64_t)blockIdx.x * w_stride;
  const uint16_t* lut = K == 4 ? lut_lds : lut_g;
  if (K == 4)
    for (int i = threadIdx.x; i < 4096; i += BLOCK) lut_lds[i] = lut_g[i];
  for (int i = threadIdx.x; i < C; i += BLOCK) hist[i] = 0;
  if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
  if (threadIdx.x < 27) Mc[threadIdx.x] = 0;
  if (threadIdx.x < 4) ncore[threadIdx.x] = 0;
  if (threadIdx.x < 2) seg_ctr[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < HUBS * 9; i += BLOCK) W[i] = 0u;
  for (int i = threadIdx.x; i < NW * WH; i += BLOCK) wh[i] = kEmptySlot;
  for (int i = threadIdx.x; i < NCN * NL; i += BLOCK) wcnt[i] = 0;
  if (K == 5) {
    for (int i = threadIdx.x; i < T5; i += BLOCK) {
      tkey[i] = kEmptySlot;
      ttyp[i] = 0ull;
      tpid[i] = 0;
    }
    for (int i = threadIdx.x; i < kU5; i += BLOCK) U5[i] = 0u;
    if (threadIdx.x < 32) cnUb[threadIdx.x >> 4][threadIdx.x & 15] = 0;
  }
  if (K == 4) {
    for (int i = threadIdx.x; i < TW; i += BLOCK) bT[i] = 0u;
    if (threadIdx.x < 15)  // pairs (a, b), 1 <= a <= b <= 15, row a from slot pair_slot4(a, a)
      for (uint32_t b = threadIdx.x + 1u; b <= 15u; ++b) {
        const uint32_t t = pair_slot4(threadIdx.x + 1u, b);
        pair_a[t] = (uint8_t)(threadIdx.x + 1u);
        pair_b[t] = (uint8_t)b;
      }
  }
  if (LCAP > 0)
    for (int i = threadIdx.x; i < LCAP / 4; i += BLOCK) lds_labels[i] = 0u;
  __syncthreads();

  const int32_t n = G.n;
  const int32_t total = G.gs_off[n];
  // the per-unit move counters of the k = 5 light path are 32-bit and stay
  // within 3 |E*| in magnitude: exact while |E*| < 2^29
  const bool fact5 = total < (1 << 30);
  int32_t cur_g = -1, row = 0, core = -1, par = 0;
  int32_t sb = 0;  // k = 5: buffer of the current light sub-chunk
  int32_t cbig = -1;  // slot of the current core among the precomputed big cores, or -1
  int64_t wbase = 0;  // first vertex of the core's graph
  auto wrow = [&](int32_t q) { return WG + (int64_t)(q - wbase) * kBigRow; };
  auto hub = [&](int32_t q) {
    const int32_t h = hub_id[q];
    return h < HUBS ? h : -1;
  };
  // W row of q for the current core: precomputed table of a big core, LDS
  // row of a hub, or the workgroup's global row
  struct Row9 {
    uint32_t v[9];
  };
  auto load_w = [&](int32_t q) {
    Row9 w;
    const int32_t hq = cbig >= 0 ? -1 : hub(q);
    if (hq >= 0) {
#pragma unroll
      for (int tr = 0; tr < 9; ++tr) w.v[tr] = W[hq * 9 + tr];
    } else {
      const uint4* w4 = reinterpret_cast<const uint4*>(
          cbig >= 0 ? wbig + cbig * wbig_stride + (int64_t)(q - wbase) * kBigRow : wrow(q));
      const uint4 x0 = w4[0], x1 = w4[1], x2 = w4[2];
      w.v[0] = x0.x; w.v[1] = x0.y; w.v[2] = x0.z; w.v[3] = x0.w;
      w.v[4] = x1.x; w.v[5] = x1.y; w.v[6] = x1.z; w.v[7] = x1.w; w.v[8] = x2.x;
    }
    return w;
  };
  // contribution of one edge between slots S1 (x) and S2 (y) of weight w
  auto edge = [&](uint32_t base, uint32_t Lx, uint32_t Ly, uint32_t r, u64 w) {
    const uint32_t c0 = base | slot_code<K, S1>(Lx) | slot_code<K, S2>(Ly);
    if constexpr (K == 5) {
      const uint64_t q = lut_quad(lut, c0);
      atomicAdd(&hist[quad_at(q, r)], w);
      atomicAdd(&hist[quad_at(q, 0)], (u64)0 - w);
    } else {
      atomicAdd(&hist[lut[c0 | rel_code<K>(r)]], w);
      atomicAdd(&hist[lut[c0]], (u64)0 - w);
    }
  };
  // k = 4: the same move counted in the anchor's table T at (min label, max
  // label, arc type seen from the smaller label's member): swapping the two
  // members flips the arc type and keeps the class.  The no-edge half is the
  // negated sum of a pair's three counts (the class of a member pair without
  // an edge does not depend on which member is in which slot).
  auto edge4 = [&](uint32_t* T, uint32_t, uint32_t Lx, uint32_t Ly, uint32_t r, u64 w) {
    const bool sw = Lx > Ly;
    const uint32_t a = sw ? Ly : Lx, b = sw ? Lx : Ly, rr = sw ? flip(r) : r;
    atomicAdd(&T[pair_slot4(a, b) * 3u + rr - 1u], (uint32_t)w);
  };
  // Closed form of label pair slot t with the anchor's moves: the pair's
  // member pairs go to its no-edge class, then each counted move takes one
  // from there to the class with the edge.  zero: clear the pair's counts.
  auto t_close = [&](const int32_t* cntv, uint32_t* T, uint32_t base, int32_t t, bool zero) {
    const uint32_t La = pair_a[t], Lb = pair_b[t];
    const u64 na = (u64)cntv[La], nb = (u64)cntv[Lb];
    const int32_t s1 = (int32_t)T[3 * t], s2 = (int32_t)T[3 * t + 1], s3 = (int32_t)T[3 * t + 2];
    if (zero) {
      T[3 * t] = 0u;
      T[3 * t + 1] = 0u;
      T[3 * t + 2] = 0u;
    }
    const u64 w0 = (La == Lb ? na * (na - (na > 0)) / 2 : na * nb) - (u64)((int64_t)s1 + s2 + s3);
    const uint32_t c0 = base | slot_code<K, S1>(La) | slot_code<K, S2>(Lb);
    if (w0) atomicAdd(&hist[lut[c0]], w0);
    if (s1) atomicAdd(&hist[lut[c0 | rel_code<K>(1u)]], (u64)(int64_t)s1);
    if (s2) atomicAdd(&hist[lut[c0 | rel_code<K>(2u)]], (u64)(int64_t)s2);
    if (s3) atomicAdd(&hist[lut[c0 | rel_code<K>(3u)]], (u64)(int64_t)s3);
  };
  // Flattened scan of the N+ rows of the vertices pick(0 .. items-1): pick
  // returns a vertex (or -1) and does the per-vertex work, visit(v, f, info)
  // handles one entry f of N+(v), where info = rowinfo(v) is computed once
  // per row when the rows are laid out (by default v's label for k = 4, 0 for
  // k = 5).  Uniform across the workgroup; ends with a barrier.
  // seg_ctr alternates between two words so that one of them can be cleared
  // while the other is read.
  // pre() runs once on every thread before the first rows are laid out
  // (independent work that can share the first pass's latency).
  auto flat_rows_pre = [&](int32_t items, auto&& pre, auto&& pick, auto&& visit, auto&& rowinfo) {
    if (items <= 0) {
      pre();
      bar<GL>();
      return;
    }
    for (int32_t i0 = 0; i0 < items; i0 += BLOCK) {
      if (i0 == 0) pre();
      const int32_t i = i0 + (int32_t)threadIdx.x;
      if (i < items) {
        const int32_t v = pick(i);
        if (v >= 0) {
          const int32_t len = G.np_off[v + 1] - G.np_off[v];
          if (len > 0) {  // |N+(v)| <= sqrt(2 |E*|), so BLOCK rows fit in 32 bits
            const u64 old = atomicAdd(&seg_ctr[par], (1ull << 32) | (u64)len);
            const int32_t sl = (int32_t)(old >> 32);
            const int32_t start = (int32_t)(uint32_t)old;
            seg_v[sl] = v;
            seg_lab[sl] = (int32_t)rowinfo(v);
            seg_start[sl] = start;
            seg_base[sl] = G.np_off[v] - start;  // entry j of the layout is np_idx[seg_base + j]
            // this row holds the bucket boundaries b * 64 in [start, start + len)
            for (int32_t b = (start + (1 << kBucketShift) - 1) >> kBucketShift;
                 b <= (start + len - 1) >> kBucketShift && b < kBuckets; ++b)
              seg_at[b] = sl;
          }
        }
      }
      bar<GL>();
      const u64 ctr = seg_ctr[par];
      const int32_t nseg = (int32_t)(ctr >> 32), tot = (int32_t)(uint32_t)ctr;
      if (threadIdx.x == 0) seg_ctr[par ^ 1] = 0;
      const int32_t last_b = (tot - 1) >> kBucketShift;
      const bool bucketed = last_b < kBuckets;
      // kUnroll entries per thread and pass, their loads issued together
      for (int32_t jb = threadIdx.x; jb < tot; jb += kUnroll * BLOCK) {
        int32_t vv[kUnroll];
        uint32_t ff[kUnroll], ll[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t j = jb + u * BLOCK;
          vv[u] = -1;
          ll[u] = 0u;
          if (j < tot) {
            // the row of j lies between the rows of the bucket boundaries around j
            const int32_t b = j >> kBucketShift;
            int32_t lo = bucketed ? seg_at[b] : 0;
            int32_t hi = bucketed && b < last_b ? seg_at[b + 1] : nseg - 1;
            while (lo < hi) {
              const int32_t mid = (lo + hi + 1) >> 1;
              if (seg_start[mid] <= j) lo = mid; else hi = mid - 1;
            }
            vv[u] = seg_v[lo];
            ll[u] = (uint32_t)seg_lab[lo];
            ff[u] = G.np_idx[seg_base[lo] + j];
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (vv[u] >= 0) visit(vv[u], ff[u], ll[u]);
      }
      bar<GL>();
      par ^= 1;
    }
  };
  auto flat_rows = [&](int32_t items, auto&& pick, auto&& visit) {
    flat_rows_pre(items, [] {}, pick, visit, [&](int32_t v) { return K == 4 ? lab.get((uint32_t)v) : 0u; });
  };
  // per-core set-up (labels of N(core), type counts, M, W) and tear-down
  auto core_setup = [&](int32_t c) {
    const int32_t ca = G.gs_off[c], dcn = G.gs_off[c + 1] - ca;
    cbig = big_id ? big_id[c] : -1;
    for (int32_t i = threadIdx.x; i < dcn; i += BLOCK) {
      const uint32_t e = G.gs_idx[ca + i];
      lab.set_bits(e & kIdMask, e >> kTypeShift);
      atomicAdd(&ncore[e >> kTypeShift], 1);
    }
    if (cbig >= 0) {  // W and M were built once for this core (k_core_tables)
      if (threadIdx.x < 27) Mc[threadIdx.x] = mbig[cbig * 32 + threadIdx.x];
      bar<GL>();
      return;
    }
    bar<GL>();
    flat_rows(
        dcn, [&](int32_t i) { return (int32_t)(G.gs_idx[ca + i] & kIdMask); },
        [&](int32_t y, uint32_t f, uint32_t Ly) {
          const int32_t x = (int32_t)(f & kIdMask);
          if (x == c) return;
          const uint32_t r = f >> kTypeShift, ty = (K == 4 ? Ly : lab.get((uint32_t)y)) & 3u;
          const int32_t h = hub(x);
          if (h >= 0) atomicAdd(&W[h * 9 + (ty - 1) * 3 + (r - 1)], 1u);
          else atomicAdd(&wrow(x)[(ty - 1) * 3 + (r - 1)], 1u);
          const uint32_t tx = lab.get((uint32_t)x) & 3u;
          if (tx) atomicAdd(&Mc[(ty - 1) * 9 + (tx - 1) * 3 + (r - 1)], 1u);
        });
    // W rows were built by L2 atomics: wait for them, then drop stale L1 lines
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  };
  auto core_teardown = [&](int32_t c) {
    bar<GL>();
    const int32_t ca = G.gs_off[c], dcn = G.gs_off[c + 1] - ca;
    if (cbig >= 0) {
      for (int32_t i = threadIdx.x; i < dcn; i += BLOCK) lab.clear_bits(G.gs_idx[ca + i] & kIdMask, 3u);
      if (threadIdx.x < 27) Mc[threadIdx.x] = 0;
      if (threadIdx.x < 4) ncore[threadIdx.x] = 0;
      bar<GL>();
      cbig = -1;
      return;
    }
    flat_rows(
        dcn,
        [&](int32_t i) {
          const int32_t y = (int32_t)(G.gs_idx[ca + i] & kIdMask);
          lab.clear_bits((uint32_t)y, 3u);
          return y;
        },
        [&](int32_t, uint32_t f, uint32_t) {
          const int32_t x = (int32_t)(f & kIdMask);
          if (x == c || hub(x) >= 0) return;
          uint4* w4 = reinterpret_cast<uint4*>(wrow(x));
          w4[0] = make_uint4(0, 0, 0, 0);
          w4[1] = make_uint4(0, 0, 0, 0);
          w4[2] = make_uint4(0, 0, 0, 0);
        });
    for (int i = threadIdx.x; i < HUBS * 9; i += BLOCK) W[i] = 0u;
    __builtin_amdgcn_s_waitcnt(0);
    if (threadIdx.x < 27) Mc[threadIdx.x] = 0;
    if (threadIdx.x < 4) ncore[threadIdx.x] = 0;
    bar<GL>();
  };

  // One anchor: core c, sides s0 (and s1 for k = 5) whose labels are set.
  auto anchor = [&](int32_t c, int32_t s0, int32_t s1, uint32_t base) {
    auto EDGE = [&](uint32_t bs, uint32_t Lx, uint32_t Ly, uint32_t r, u64 w) {
      if constexpr (K == 4) edge4(bT, bs, Lx, Ly, r, w);
      else edge(bs, Lx, Ly, r, w);
    };
    const int32_t a0 = G.gs_off[s0], d0 = G.gs_off[s0 + 1] - a0;
    const int32_t a1 = K == 5 ? G.gs_off[s1] : 0, d1 = K == 5 ? G.gs_off[s1 + 1] - a1 : 0;
    const int32_t nsides = K == 5 ? 2 : 1;
    auto is_side = [&](int32_t y) { return y == s0 || (K == 5 && y == s1); };
    // list position -> vertex q of R' (each once); the O(1) part per q:
    // set sizes and the edges p -> q counted in W[q]
    auto pick = [&](int32_t i) -> int32_t {
      int32_t q;
      if (i < nsides) {
        q = i == 0 ? s0 : s1;
      } else if (i < nsides + d0) {
        q = (int32_t)(G.gs_idx[a0 + i - nsides] & kIdMask);
        if (q == c || is_side(q)) return -1;
      } else {
        q = (int32_t)(G.gs_idx[a1 + i - nsides - d0] & kIdMask);
        if (q == c || is_side(q) || ((lab.get((uint32_t)q) >> 2) & 3u)) return -1;  // listed from s0's row
      }
      const uint32_t Lq = lab.get((uint32_t)q);
      const bool mq = !is_side(q);  // R' vertices other than the sides are members
      const uint32_t cq = Lq & 3u;
      if (mq) atomicAdd(&cnt[Lq], 1);
      // edges p -> q (p in N(core), p of lower rank than q): row W[q]
      const Row9 wq = load_w(q);
#pragma unroll
      for (int tr = 0; tr < 9; ++tr) {
        const uint32_t w = wq.v[tr];
        if (!w) continue;
        const uint32_t tp = (uint32_t)(tr / 3) + 1u, r = (uint32_t)(tr % 3) + 1u;
        if (cq) EDGE(base, tp, cq, r, (u64)0 - (u64)w);
        if (mq) EDGE(base, tp, Lq, r, (u64)w);
      }
      return q;
    };
    // one edge q -> y of N+(q) with q in R'
    auto visit = [&](int32_t q, uint32_t f, uint32_t Lrow) {
      const int32_t y = (int32_t)(f & kIdMask);
      if (y == c) return;
      const uint32_t Ly = lab.get((uint32_t)y);
      const bool sy = is_side(y);
      if (!Ly && !sy) return;
      const uint32_t Lq = K == 4 ? Lrow : lab.get((uint32_t)q);
      const bool mq = !is_side(q), my = !sy;
      const uint32_t r = f >> kTypeShift, cq = Lq & 3u, cy = Ly & 3u;
      // (cq, cy) takes -1, and +1 back when p = q is also counted in W[y]
      // (y a side neighbour or a side): only the net is added
      const bool inw = sy || (Ly >> 2);
      if (cq && cy && !inw) EDGE(base, cq, cy, r, kMinusOne);
      if (mq && my) EDGE(base, Lq, Ly, r, 1ull);
      if (cq && my && inw) EDGE(base, cq, Ly, r, kMinusOne);
    };
    flat_rows(nsides + d0 + d1, pick, visit);
    // edges inside N(core) with core-only labels
    if (threadIdx.x < 27) {
      const uint32_t w = Mc[threadIdx.x];
      if (w) {
        const uint32_t tx = threadIdx.x / 9 + 1, ty = (threadIdx.x / 3) % 3 + 1, r = threadIdx.x % 3 + 1;
        EDGE(base, tx, ty, r, (u64)w);
      }
    }
    // sizes of the core-only sets: N(core) minus the sides minus R'
    if (threadIdx.x < 3) {
      const int32_t a = threadIdx.x + 1;
      int32_t v = ncore[a];
      for (int L = 4 + a; L < NL; L += 4) v -= cnt[L];
      // the type of each side towards the core sits in its own label
      const uint32_t t0 = lab.get((uint32_t)s0) & 3u;
      const uint32_t t1 = K == 5 ? lab.get((uint32_t)s1) & 3u : 0u;
      v -= (t0 == (uint32_t)a) + (K == 5 && t1 == (uint32_t)a);
      cnt[a] = v;
    }
    bar<GL>();
    if constexpr (K == 4) {  // every pair once: some moves sit on empty sets
      for (int32_t t = threadIdx.x; t < kPairs4; t += BLOCK) t_close(cnt, bT, base, t, true);
    } else {
      closed_form<K, NL, BLOCK>(hist, lut, cnt, nzl, &nz_count, base);
    }
    bar<GL>();
    if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
  };

  // Light k = 4 anchor {c, s} (d*(s) <= lim.light) on one wave.  The types
  // of N(s) towards s sit in a wave-private hash table instead of the dense
  // labels (which then hold only the core's types), so the waves of the
  // workgroup take different anchors of the same core at the same time with
  // no workgroup barrier.  Entry i of s's row stands for R' member i, the
  // entry of c standing for s itself, and R' is taken 64 members at a time:
  // one lane per member, their N+ rows laid end to end over the wave.  Same
  // sums as anchor().
  auto wave_anchor4 = [&](int32_t c, int32_t s, uint32_t base) {
    const int32_t lane = (int32_t)(threadIdx.x & 63u);
    uint32_t* H = wh + (threadIdx.x >> 6) * WH;
    int32_t* cn = wcnt + (threadIdx.x >> 6) * NL;
    uint32_t* E = wT + (threadIdx.x >> 6) * TW;
    for (int32_t i = lane; i < TW / 4; i += 64) reinterpret_cast<uint4*>(E)[i] = make_uint4(0u, 0u, 0u, 0u);
    const int32_t a0 = G.gs_off[s], d0 = G.gs_off[s + 1] - a0;
    const uint32_t Ls = lab.get((uint32_t)s) & 3u;
    for (int32_t i = lane; i < d0; i += 64) {
      const uint32_t e = G.gs_idx[a0 + i];
      const int32_t q = (int32_t)(e & kIdMask);
      if (q == c) continue;
      uint32_t h = hash_slot(q);
      const uint32_t ent = ((uint32_t)q << 2) | (e >> kTypeShift);  // q < 2^30 - 1: never kEmptySlot
      while (atomicCAS(&H[h], kEmptySlot, ent) != kEmptySlot) h = (h + 1) & (kWaveHash - 1);
    }
    wave_sync();  // hash table complete
    for (int32_t i0 = 0; i0 < d0; i0 += 64) {
      const int32_t i = i0 + lane;
      int32_t q = -1;
      uint32_t Lq = 0;
      int32_t len = 0, rb = 0;
      if (i < d0) {
        const uint32_t e = G.gs_idx[a0 + i];
        q = (int32_t)(e & kIdMask);
        bool mq = true;
        if (q == c) {
          q = s;
          Lq = Ls;
          mq = false;
        } else {
          Lq = (lab.get((uint32_t)q) & 3u) | ((e >> kTypeShift) << 2);
          atomicAdd(&cn[Lq], 1);
        }
        const uint32_t cq = Lq & 3u;
        const Row9 wq = load_w(q);
#pragma unroll
        for (int tr = 0; tr < 9; ++tr) {
          const uint32_t w = wq.v[tr];
          if (!w) continue;
          const uint32_t tp = (uint32_t)(tr / 3) + 1u, r = (uint32_t)(tr % 3) + 1u;
          if (cq) edge4(E, base, tp, cq, r, (u64)0 - (u64)w);
          if (mq) edge4(E, base, tp, Lq, r, (u64)w);
        }
        rb = G.np_off[q];
        len = G.np_off[q + 1] - rb;
      }
      int32_t inc = len;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(inc, d);
        if (lane >= d) inc += t;
      }
      const int32_t tot = __shfl(inc, 63);
      const int32_t rs = rb - (inc - len);  // flat entry j of this lane's row is np_idx[rs + j]
      for (int32_t jb = 0; jb < tot; jb += 64 * kUnroll) {
        int32_t sqs[kUnroll];
        uint32_t sLs[kUnroll], fs[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t j = jb + u * 64 + lane;
          int32_t sl = 0;  // number of lanes whose rows end at or before j
#pragma unroll
          for (int st2 = 32; st2; st2 >>= 1)
            if (__shfl(inc, sl + st2 - 1) <= j) sl += st2;
          sqs[u] = __shfl(q, sl);
          sLs[u] = (uint32_t)__shfl((int32_t)Lq, sl);
          const int32_t srs = __shfl(rs, sl);
          fs[u] = j < tot ? G.np_idx[srs + j] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t j = jb + u * 64 + lane;
          if (j >= tot) continue;
          const int32_t sq = sqs[u];
          const uint32_t sL = sLs[u], f = fs[u];
          const int32_t y = (int32_t)(f & kIdMask);
          if (y != c) {
            const bool sy = y == s;
            uint32_t Ly = lab.get((uint32_t)y) & 3u;
            if (!sy) {
              uint32_t h = hash_slot(y);
              for (;;) {
                const uint32_t e = H[h];
                if (e == kEmptySlot) break;
                if ((e >> 2) == (uint32_t)y) {
                  Ly |= (e & 3u) << 2;
                  break;
                }
                h = (h + 1) & (kWaveHash - 1);
              }
            }
            if (Ly || sy) {
              const bool mq = sq != s, my = !sy;
              const uint32_t r = f >> kTypeShift, cq = sL & 3u, cy = Ly & 3u;
              // (cq, cy) takes -1, and +1 back when p = sq is also counted in
              // W[y] (y a side neighbour or the side): only the net is added
              const bool inw = sy || (Ly >> 2);
              if (cq && cy && !inw) edge4(E, base, cq, cy, r, kMinusOne);
              if (mq && my) edge4(E, base, sL, Ly, r, 1ull);
              if (cq && my && inw) edge4(E, base, cq, Ly, r, kMinusOne);
            }
          }
        }
      }
    }
    // edges inside N(core) with core-only labels
    if (lane < 27) {
      const uint32_t w = Mc[lane];
      if (w) edge4(E, base, (uint32_t)lane / 9 + 1, ((uint32_t)lane / 3) % 3 + 1, (uint32_t)lane % 3 + 1, (u64)w);
    }
    wave_sync();
    // sizes of the core-only sets: N(core) minus s minus R'
    if (lane >= 1 && lane <= 3) {
      int32_t v = ncore[lane];
      for (int L = 4 + lane; L < NL; L += 4) v -= cn[L];
      v -= (int32_t)(Ls == (uint32_t)lane);
      cn[lane] = v;
    }
    wave_sync();
    for (int32_t t = lane; t < kPairs4; t += 64) t_close(cn, E, base, t, false);
    wave_sync();
    if (lane < NL) cn[lane] = 0;
    for (int32_t i = lane; i < WH; i += 64) H[i] = kEmptySlot;
    wave_sync();
  };
  // Solo k = 4 anchor {c, s} with d*(c) <= lim.solo on one wave: the plain
  // per-anchor method (as in k4_kernel) with the labels of N(c) u N(s) in a
  // wave-private hash (keys, then complemented label bits, in the wave's
  // table), so small cores need no workgroup set-up at all.  Members are the
  // hash entries; each member's N+ row is scanned and every labelled
  // neighbour is an inner edge; then the closed form over the 15 sets.
  auto wave_solo4 = [&](int32_t c, int32_t s, uint32_t base) {
    const int32_t lane = (int32_t)(threadIdx.x & 63u);
    uint32_t* key = wh + (threadIdx.x >> 6) * WH;
    uint32_t* nlab = key + kSoloHash;
    int32_t* cn = wcnt + (threadIdx.x >> 6) * NL;
    uint32_t* E = wT + (threadIdx.x >> 6) * TW;
    for (int32_t i = lane; i < TW / 4; i += 64) reinterpret_cast<uint4*>(E)[i] = make_uint4(0u, 0u, 0u, 0u);
    auto slot = [](uint32_t x) { return (x * 2654435761u) >> (32 - kSoloHashBits); };
    auto insert = [&](uint32_t x, uint32_t bits) {
      uint32_t h = slot(x);
      for (;;) {
        const uint32_t old = atomicCAS(&key[h], kEmptySlot, x);
        if (old == kEmptySlot || old == x) {
          atomicAnd(&nlab[h], ~bits);
          return;
        }
        h = (h + 1) & (kSoloHash - 1);
      }
    };
    const int32_t ca = G.gs_off[c], dc = G.gs_off[c + 1] - ca;  // dc <= lim.solo <= 64
    if (lane < dc) {
      const uint32_t e = G.gs_idx[ca + lane];
      if ((int32_t)(e & kIdMask) != s) insert(e & kIdMask, e >> kTypeShift);
    }
    wave_sync();
    const int32_t sa = G.gs_off[s], ds = G.gs_off[s + 1] - sa;  // ds <= dc
    if (lane < ds) {
      const uint32_t e = G.gs_idx[sa + lane];
      if ((int32_t)(e & kIdMask) != c) insert(e & kIdMask, (e >> kTypeShift) << 2);
    }
    wave_sync();
    for (int32_t i0 = 0; i0 < kSoloHash; i0 += 64) {
      const uint32_t xk = key[i0 + lane];
      uint32_t Lx = 0;
      int32_t len = 0, rb = 0;
      if (xk != kEmptySlot) {
        Lx = ~nlab[i0 + lane];
        atomicAdd(&cn[Lx], 1);
        rb = G.np_off[xk];
        len = G.np_off[xk + 1] - rb;
      }
      int32_t inc = len;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(inc, d);
        if (lane >= d) inc += t;
      }
      const int32_t tot = __shfl(inc, 63);
      const int32_t rs = rb - (inc - len);
      for (int32_t jb = 0; jb < tot; jb += 64 * kUnroll) {
        uint32_t sLs[kUnroll], fs[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t j = jb + u * 64 + lane;
          int32_t sl = 0;
#pragma unroll
          for (int st2 = 32; st2; st2 >>= 1)
            if (__shfl(inc, sl + st2 - 1) <= j) sl += st2;
          sLs[u] = (uint32_t)__shfl((int32_t)Lx, sl);
          const int32_t srs = __shfl(rs, sl);
          fs[u] = j < tot ? G.np_idx[srs + j] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (jb + u * 64 + lane >= tot) continue;
          const uint32_t f = fs[u], y = f & kIdMask;
          uint32_t h = slot(y);
          for (;;) {
            const uint32_t kk = key[h];
            if (kk == kEmptySlot) break;
            if (kk == y) {
              edge4(E, base, sLs[u], ~nlab[h], f >> kTypeShift, 1ull);
              break;
            }
            h = (h + 1) & (kSoloHash - 1);
          }
        }
      }
    }
    wave_sync();
    for (int32_t t = lane; t < kPairs4; t += 64) t_close(cn, E, base, t, false);
    wave_sync();
    if (lane < NL) cn[lane] = 0;
    for (int32_t i = lane; i < WH; i += 64) key[i] = kEmptySlot;
    wave_sync();
  };
  // ---- k = 5, light partners: the side-a part shared by a unit's triples --
  //
  // For a unit (b = core, a) the triples (b; a, c) with a light partner c
  // share most of their sums: the members of N(a), their W rows and their N+
  // rows carry the same labels in every triple except where they meet N[c].
  // A sub-chunk of up to kNP5 light partners is therefore done as
  //   U  = the sums of {a} u N(a) \ {b} with every partner absent (labels of
  //        b and a only), kept without the base code as counters per
  //        (label x, label y, r) and added once per distinct base;
  //   plus, per partner c, the difference to its own triple: items and edges
  //        that meet N[c] (a member of N(c), an edge into N(c) or into c)
  //        are moved to their labels in the triple, and c itself, when it is
  //        in N(a), leaves the a-part and becomes a side;
  //   plus the part of each triple outside N[a]: c and its neighbours
  //        outside N[a], each vertex taken once for all the partners it
  //        belongs to;
  //   plus the closed form of each triple (one wave per partner).
  // Both parts share one flattened scan.  The partners' neighbourhoods sit in
  // one LDS table (key -> 2 type bits per partner, partner index + 1 of the
  // vertex itself); label bit 6 marks its keys, so vertices outside every
  // N(c) cost no lookup.  The sums equal those of anchor() for each triple.
  auto u5i = [](uint32_t X, uint32_t Y, uint32_t r) { return X * 48u + Y * 3u + (r - 1u); };
  auto t5_slot = [](uint32_t v) { return (v * 2654435761u) >> (32 - kT5Bits); };
  auto t5_insert = [&](uint32_t v) -> uint32_t {  // at most kT5Load < kT5 keys: a slot is always found
    uint32_t h = t5_slot(v);
    for (int i = 0; i < kT5; ++i) {
      const uint32_t old = atomicCAS(&tkey[h], kEmptySlot, v);
      if (old == kEmptySlot) tlist[atomicAdd(&p5_ctlb[sb][4], 1)] = (uint16_t)h;
      if (old == kEmptySlot || old == v) return h;
      h = (h + 1) & (kT5 - 1);
    }
    return kT5;
  };
  auto t5_find = [&](uint32_t v) -> uint32_t {  // v carries label bit 6, so it is a key
    uint32_t h = t5_slot(v);
    for (int i = 0; i < kT5; ++i) {
      if (tkey[h] == v) return h;
      h = (h + 1) & (kT5 - 1);
    }
    return kT5;
  };
  // moves of one edge q -> y (r = type of y relative to q, sign s): the edge
  // terms of anchor() with the pair that cancels when y is in R' left out.
  // Of its three terms the first (y outside the sides and R', core-labelled)
  // and the third (y a side or in R') never apply together and carry the
  // same signs, so they share one table read and one pair of counters; the
  // table reads are issued before the counters.
  auto emove = [&](uint32_t base, uint32_t Lq, bool mq, uint32_t Ly, bool sy, uint32_t r, u64 s) {
    const bool it = sy || (Ly >> 2);
    const uint32_t cq = Lq & 3u, cy = Ly & 3u;
    const bool e13 = cq && (it ? !sy : cy != 0u), e2 = mq && !sy;
    const uint32_t b13 = base | slot_code<K, S1>(cq) | slot_code<K, S2>(it ? Ly : cy);
    const uint32_t b2 = base | slot_code<K, S1>(Lq) | slot_code<K, S2>(Ly);
    const uint64_t q13 = e13 ? lut_quad(lut, b13) : 0ull;
    const uint64_t q2 = e2 ? lut_quad(lut, b2) : 0ull;
    if (e13) {
      atomicAdd(&hist[quad_at(q13, r)], (u64)0 - s);
      atomicAdd(&hist[quad_at(q13, 0)], s);
    }
    if (e2) {
      atomicAdd(&hist[quad_at(q2, r)], s);
      atomicAdd(&hist[quad_at(q2, 0)], (u64)0 - s);
    }
  };
  auto umove = [&](uint32_t Lq, bool mq, uint32_t Ly, bool sy, uint32_t r) {
    const bool it = sy || (Ly >> 2);
    const uint32_t cq = Lq & 3u, cy = Ly & 3u;
    if (cq && (it ? !sy : cy != 0u)) atomicAdd(&U5[u5i(cq, it ? Ly : cy, r)], ~0u);
    if (mq && !sy) atomicAdd(&U5[u5i(Lq, Ly, r)], 1u);
  };
  auto pairs2 = [](u64 t) { return (t | (t >> 1)) & 0x5555555555555555ull; };  // bit 2p: partner p present
  auto t5_get = [&](uint32_t v, uint32_t lv, u64& t, int32_t& pv) {
    t = 0ull;
    pv = -1;
    if (lv & kInT5) {
      const uint32_t h = t5_find(v);
      if (h < kT5) {
        t = ttyp[h];
        pv = (int32_t)tpid[h] - 1;
      }
    }
  };
  // labels of an N+ entry y for partner p: side flag and label in the triple
  auto ylab = [&](int32_t y, int32_t a, uint32_t ly, u64 ty, int32_t py, int32_t p, bool& syT) -> uint32_t {
    syT = y == a || py == p;
    return syT ? (ly & 3u) : ((ly & 15u) | (((uint32_t)(ty >> (2 * p)) & 3u) << 4));
  };
  // a-part item i of {a} u N(a) \ {b}: set size and W row, into U and into
  // the per-partner differences
  auto u5_pick = [&](int32_t b, int32_t a, int32_t aa, int32_t i) -> int32_t {
    int32_t q = a;
    if (i > 0) {
      q = (int32_t)(G.gs_idx[aa + i - 1] & kIdMask);
      if (q == b) return -1;
    }
    const bool mq = i > 0;
    const uint32_t Lq = lab.get((uint32_t)q) & (mq ? 15u : 3u), cq = Lq & 3u;
    if (mq) atomicAdd(&cnUb[sb][Lq], 1);
    const Row9 wq = load_w(q);
#pragma unroll
    for (int tr = 0; tr < 9; ++tr) {
      const uint32_t w = wq.v[tr];
      if (!w) continue;
      const uint32_t tp = (uint32_t)(tr / 3) + 1u, r = (uint32_t)(tr % 3) + 1u;
      if (cq) atomicAdd(&U5[u5i(tp, cq, r)], (uint32_t)0 - w);
      if (mq) atomicAdd(&U5[u5i(tp, Lq, r)], w);
    }
    return q;
  };
  // per-partner part of a table entry, one thread per (vertex v, partner p)
  // pair: set sizes and W row of v in p's triple minus what U holds for it.
  // self: v is the partner itself (a side), else v in N(p) with type tv.
  auto pair5 = [&](int32_t a, int32_t p, int32_t v, bool self, uint32_t tv) {
    if (v == a) return;  // a side in every triple, as in U
    const uint32_t lv = lab.get((uint32_t)v);
    const bool ina = (lv >> 2) & 3u;  // in N(a): an item of U
    const uint32_t LU = lv & 15u, cv = lv & 3u;
    const uint32_t LT = cv | (tv << 4) | (ina ? (lv & 12u) : 0u);
    int32_t* cn = wcnt + p * NL;
    if (self) {
      if (ina) atomicAdd(&cn[LU], -1);
    } else {
      if (ina) atomicAdd(&cn[LU], -1);
      atomicAdd(&cn[LT], 1);
    }
    const uint32_t bp = p5_baseb[sb][p];
    const Row9 wv = load_w(v);
    // self: side of its own triple; when in N(a), its member terms in U
    // leave.  Else a member with label LT instead of LU (or of nothing).
    const bool plus = !self, minus = ina || cv;
    const uint32_t Lm = ina ? LU : cv;
    // table reads of one type tp (three r) first, then the counters
#pragma unroll
    for (int t3 = 0; t3 < 3; ++t3) {
      const uint32_t bt = bp | slot_code<K, S1>((uint32_t)t3 + 1u);
      const uint32_t cpl = bt | slot_code<K, S2>(LT), cmi = bt | slot_code<K, S2>(Lm);
      const bool on = (wv.v[t3 * 3] | wv.v[t3 * 3 + 1] | wv.v[t3 * 3 + 2]) != 0u;
      const uint64_t qp = on && plus ? lut_quad(lut, cpl) : 0ull;
      const uint64_t qm = on && minus ? lut_quad(lut, cmi) : 0ull;
#pragma unroll
      for (int r3 = 0; r3 < 3; ++r3) {
        const u64 w = wv.v[t3 * 3 + r3];
        if (!w) continue;
        if (plus) {
          atomicAdd(&hist[quad_at(qp, (uint32_t)r3 + 1u)], w);
          atomicAdd(&hist[quad_at(qp, 0)], (u64)0 - w);
        }
        if (minus) {
          atomicAdd(&hist[quad_at(qm, (uint32_t)r3 + 1u)], (u64)0 - w);
          atomicAdd(&hist[quad_at(qm, 0)], w);
        }
      }
    }
  };
  // c-part item k: a key of the partner table outside N[a]
  auto c5_pick = [&](int32_t a, int32_t k) -> int32_t {
    const int32_t q = (int32_t)tkey[tlist[k]];
    return q == a || ((lab.get((uint32_t)q) >> 2) & 3u) ? -1 : q;
  };
  // entry (y, r) of N+(q) for an item q of either part
  // row information of q for the merged scan: label << 16 | table slot + 1
  // (0 when q is no key), found once per row
  auto s5_rowinfo = [&](int32_t q) -> uint32_t {
    const uint32_t lq = lab.get((uint32_t)q);
    const uint32_t h = (lq & kInT5) ? t5_find((uint32_t)q) : (uint32_t)kT5;
    return (lq << 16) | (h < kT5 ? h + 1u : 0u);
  };
  auto s5_visit = [&](int32_t b, int32_t a, int32_t q, uint32_t f, uint32_t qinfo) {
    const int32_t y = (int32_t)(f & kIdMask);
    if (y == b) return;
    const uint32_t r = f >> kTypeShift;
    const uint32_t lq = qinfo >> 16, ly = lab.get((uint32_t)y);
    u64 tq = 0ull, ty;
    int32_t pq = -1, py;
    if (qinfo & 0xFFFFu) {
      const uint32_t hq = (qinfo & 0xFFFFu) - 1u;
      tq = ttyp[hq];
      pq = (int32_t)tpid[hq] - 1;
    }
    t5_get((uint32_t)y, ly, ty, py);
    if (q != a && !((lq >> 2) & 3u)) {  // c-part: q is outside N[a]
      const uint32_t cq = lq & 3u;
      if (pq >= 0) {
        bool syT;
        const uint32_t LyT = ylab(y, a, ly, ty, py, pq, syT);
        if (syT || LyT) emove(p5_baseb[sb][pq], cq, false, LyT, syT, r, 1ull);
      }
      for (u64 m = pairs2(tq); m; m &= m - 1ull) {
        const int32_t p = __builtin_ctzll(m) >> 1;
        bool syT;
        const uint32_t LyT = ylab(y, a, ly, ty, py, p, syT);
        if (syT || LyT) emove(p5_baseb[sb][p], cq | (((uint32_t)(tq >> (2 * p)) & 3u) << 4), true, LyT, syT, r, 1ull);
      }
      return;
    }
    const bool mq = q != a, syU = y == a;
    const uint32_t Lq = lq & (mq ? 15u : 3u), LyU = ly & (syU ? 3u : 15u);
    const bool inU = syU || LyU;
    if (inU) umove(Lq, mq, LyU, syU, r);
    if (!((lq | ly) & kInT5)) return;
    if (pq >= 0) {  // partner q: its member edge leaves, its side edge comes in
      if (inU) emove(p5_baseb[sb][pq], Lq, mq, LyU, syU, r, kMinusOne);
      bool syT;
      const uint32_t LyT = ylab(y, a, ly, ty, py, pq, syT);
      if (syT || LyT) emove(p5_baseb[sb][pq], Lq & 3u, false, LyT, syT, r, 1ull);
    }
    u64 cm = pairs2((mq ? tq : 0ull) | ty);
    if (py >= 0) cm |= 1ull << (2 * py);
    if (pq >= 0) cm &= ~(1ull << (2 * pq));
    for (u64 m = cm; m; m &= m - 1ull) {
      const int32_t p = __builtin_ctzll(m) >> 1;
      const uint32_t bp = p5_baseb[sb][p];
      const uint32_t LT = mq ? (Lq | (((uint32_t)(tq >> (2 * p)) & 3u) << 4)) : Lq;
      bool syT;
      const uint32_t LyT = ylab(y, a, ly, ty, py, p, syT);
      if (syT || LyT) emove(bp, LT, mq, LyT, syT, r, 1ull);
      if (inU) emove(bp, Lq, mq, LyU, syU, r, kMinusOne);
    }
  };
  // closed form of light partner p on one wave: its set sizes are the a-part
  // sizes plus its own differences; then the non-empty sets of the 63
  auto close5 = [&](int32_t p, int32_t a) {
    const int32_t lane = (int32_t)(threadIdx.x & 63u);
    const int32_t c2 = p5_vb[sb][p];
    const uint32_t base = p5_baseb[sb][p];
    int32_t* cn = wcnt + p * NL;
    if (lane < 16) cn[lane] += cnUb[sb][lane];
    wave_sync();
    // sizes of the core-only sets: N(core) minus the sides minus R'
    if (lane >= 1 && lane <= 3) {
      int32_t v = ncore[lane];
      for (int L = 4 + lane; L < NL; L += 4) v -= cn[L];
      v -= (int32_t)((lab.get((uint32_t)a) & 3u) == (uint32_t)lane) + (int32_t)((lab.get((uint32_t)c2) & 3u) == (uint32_t)lane);
      cn[lane] = v;
    }
    wave_sync();
    // the non-empty sets (NL = 64 labels, one per lane) compacted to the low
    // lanes by a lane permutation
    const int32_t myc = cn[lane];
    const bool nzb = lane > 0 && myc != 0;
    const unsigned long long nzm = __ballot(nzb);
    const int32_t nz = __popcll(nzm);
    const int32_t pos = __popcll(nzm & ((1ull << lane) - 1ull));
    const int32_t dst = nzb ? pos : nz + (lane - pos);
    const int32_t lbl = __builtin_amdgcn_ds_permute(dst * 4, lane);
    const int32_t cnt_c = __builtin_amdgcn_ds_permute(dst * 4, myc);
    for (int32_t pq0 = 0; pq0 < nz * nz; pq0 += 64) {
      const int32_t pq = pq0 + lane;
      const int32_t ia = pq / nz, ib = pq - ia * nz;
      const int32_t sa = min(ia, 63), sb = min(ib, 63);
      const uint32_t La = (uint32_t)__shfl(lbl, sa), Lb = (uint32_t)__shfl(lbl, sb);
      const u64 na = (u64)(int64_t)__shfl(cnt_c, sa), nb = (u64)(int64_t)__shfl(cnt_c, sb);
      if (pq < nz * nz && ia <= ib) {
        const u64 w = ia == ib ? na * (na - 1) / 2 : na * nb;
        if (w) atomicAdd(&hist[lut[base | slot_code<K, K - 2>(La) | slot_code<K, K - 1>(Lb)]], w);
      }
    }
    wave_sync();
    cn[lane] = 0;
    wave_sync();
  };
  // A unit of a new core: flush the histogram on a graph change and set up
  // the core's tables (the previous core's are torn down first).  The graph
  // is checked even for the current core: the small-core pass of a tile may
  // have moved the histogram to another graph in between.
  auto enter_core = [&](int32_t c) {
    const int32_t g = G.gid ? G.gid[c] : 0;
    if (g != cur_g) {
      hist_flush<C, BLOCK>(hist, acc, cur_g);
      cur_g = g;
      bar<GL>();
    }
    if (c == core) return;
    if (core >= 0) core_teardown(core);
    wbase = G.voff ? G.voff[g] : 0;
    lab.base = (uint32_t)wbase;  // the previous core's labels are cleared
    core = c;
    core_setup(c);
  };

  // One pull of the cost-cut work queue by wave 0: [sh_j0, sh_j1) are the
  // entries whose cost prefix lies in the pulled interval (sh_j0 = -1 once
  // the queue is empty).  Tiles of tc cost units, the last quarter of the
  // cost (from split) in tiles of tc_end from a second counter.  Each cut is
  // a 64-way search of cpre: about four dependent reads instead of ~20.
  // The two counters are 64-bit: every pull adds to the first, also after it
  // has passed split, so it may run past the 31-bit range of the costs.
  auto pull_tile = [&](int32_t tot_cost, int32_t tc, int32_t split, int32_t tc_end) {
    if (threadIdx.x < 64) {
      const int32_t lane = (int32_t)threadIdx.x;
      u64* q64 = reinterpret_cast<u64*>(queue);
      int64_t c0 = 0, c1 = 0;
      if (lane == 0) {
        c0 = (int64_t)atomicAdd(&q64[0], (u64)tc);
        c1 = min((int64_t)split, c0 + tc);
        if (c0 >= split) {
          c0 = split + (int64_t)atomicAdd(&q64[1], (u64)tc_end);
          c1 = min((int64_t)tot_cost, c0 + tc_end);
        }
      }
      c0 = __shfl(c0, 0);
      c1 = __shfl(c1, 0);
      auto first_at = [&](int64_t key) -> int32_t {  // first entry whose cost prefix is >= key
        int32_t lo = 0, hi = total;
        while (lo < hi) {
          const int32_t step = (hi - lo + 63) >> 6;
          const int32_t pr = lo + lane * step;
          const int32_t cnt = __popcll(__ballot(pr < hi && (int64_t)cpre[pr] < key));
          if (cnt == 0) {
            hi = lo;
          } else {
            const int32_t nlo = lo + (cnt - 1) * step + 1;
            hi = min(hi, lo + cnt * step);
            lo = nlo;
          }
        }
        return lo;
      };
      const bool done = c0 >= tot_cost;
      const int32_t a0 = done ? -1 : first_at(c0);
      const int32_t a1 = done ? -1 : first_at(c1);
      if (lane == 0) {
        sh_j0 = a0;
        sh_j1 = a1;
      }
    }
  };

  if constexpr (K == 4) {
    // Tiles of G* entries cut by estimated cost: cpre is the exclusive prefix
    // sum of a per-entry cost (UnitCost4), and a tile is the run of
    // entries whose prefix falls in one cost interval of the queue, about
    // `tile` tiles per workgroup.  Within a tile, the entries of one core
    // row are sorted into heavy units (whole workgroup, one after another)
    // and light units (one wave each).
    const int32_t tot_cost = cpre[total];
    const int64_t parts = (int64_t)gridDim.x * (tile > 0 ? tile : 1);
    const int32_t tc = (int32_t)max((int64_t)kMinTileCost4, ((int64_t)tot_cost + parts - 1) / parts);
    // The last quarter of the cost is cut four times finer (second counter),
    // so the tiles still running at the end are small.
    const int32_t split = tot_cost - tot_cost / 4, tc_end = max(1, tc / 4);
    for (;;) {
      pull_tile(tot_cost, tc, split, tc_end);
      bar<GL>();
      const int32_t j0 = sh_j0, j1 = sh_j1;
      bar<GL>();
      if (j0 < 0) break;
      if (j0 >= j1) continue;
      // units of small cores: one wave each, no core set-up, in chunks of
      // BLOCK entries of one graph
      for (int32_t jc = j0; jc < j1;) {
        int32_t jce = min(j1, jc + BLOCK);
        const int32_t g = G.gid ? G.gid[G.gs_row[jc]] : 0;
        if (G.gid) jce = min(jce, G.gs_off[(int32_t)G.voff[g + 1]]);
        if (g != cur_g) {
          hist_flush<C, BLOCK>(hist, acc, cur_g);
          cur_g = g;
        }
        if (threadIdx.x < 2) unit_ctr[threadIdx.x] = 0;
        bar<GL>();
        {
          const int32_t j = jc + (int32_t)threadIdx.x;
          if (j < jce) {
            const int32_t c = G.gs_row[j];
            const int32_t dc = G.gs_off[c + 1] - G.gs_off[c];
            if (dc <= lim.solo) {
              const int32_t x = (int32_t)(G.gs_idx[j] & kIdMask), dx = G.gs_off[x + 1] - G.gs_off[x];
              if (dx < dc || (dx == dc && x < c)) unit_list[atomicAdd(&unit_ctr[0], 1)] = j;
            }
          }
        }
        bar<GL>();
        const int32_t nsolo = unit_ctr[0];
        for (;;) {
          int32_t u = 0;
          if ((threadIdx.x & 63u) == 0) u = atomicAdd(&unit_ctr[1], 1);
          u = __shfl(u, 0);
          if (u >= nsolo) break;
          const int32_t j = unit_list[u];
          const uint32_t ej = G.gs_idx[j];
          const uint32_t tcx = ej >> kTypeShift;
          wave_solo4(G.gs_row[j], (int32_t)(ej & kIdMask),
                     ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u));
        }
        bar<GL>();
        jc = jce;
      }
      // units of the other cores, one core row at a time
      row = G.gs_row[j0];
      for (int32_t js = j0; js < j1;) {
        while (G.gs_off[row + 1] <= js) ++row;
        const int32_t c = row;
        const int32_t rowa = G.gs_off[c], rowb = G.gs_off[c + 1];
        if (rowb - rowa <= lim.solo) {  // taken above
          js = min(j1, rowb);
          continue;
        }
        const int32_t je = min(min(j1, rowb), js + BLOCK);
        if (threadIdx.x < 3) unit_ctr[threadIdx.x] = 0;
        if (threadIdx.x < 32) lbk[threadIdx.x] = 0;
        bar<GL>();
        {
          // heavy units to the front of the list; light units to the back,
          // counted per log2 of the side's degree and then placed largest
          // bucket first, so the waves take the long anchors first
          const int32_t j = js + (int32_t)threadIdx.x;
          int32_t bk = -1;
          if (j < je) {
            const int32_t x = (int32_t)(G.gs_idx[j] & kIdMask);
            const int32_t dc = rowb - rowa, dx = G.gs_off[x + 1] - G.gs_off[x];
            if (dx < dc || (dx == dc && x < c)) {  // anchor edge {c, x} owned by its higher-rank end
              if (dx > lim.light) {
                unit_list[atomicAdd(&unit_ctr[0], 1)] = j;
              } else {
                bk = 31 - __clz(max(dx, 1));  // 0 .. 8
                atomicAdd(&unit_ctr[1], 1);
                atomicAdd(&lbk[bk], 1);
              }
            }
          }
          bar<GL>();
          if (bk >= 0) {
            int32_t pos = 0;
            for (int32_t b2 = bk + 1; b2 < 16; ++b2) pos += lbk[b2];
            pos += atomicAdd(&lbk[16 + bk], 1);
            unit_list[BLOCK - 1 - pos] = j;
          }
        }
        bar<GL>();
        const int32_t nheavy = unit_ctr[0], nlight = unit_ctr[1];
        if (nheavy + nlight > 0) {
          enter_core(c);
          for (int32_t u = 0; u < nheavy; ++u) {
            const int32_t j = unit_list[u];
            const uint32_t ej = G.gs_idx[j];
            const int32_t x = (int32_t)(ej & kIdMask);
            const uint32_t tcx = ej >> kTypeShift;
            const int32_t xa = G.gs_off[x], xb = G.gs_off[x + 1];
            for (int32_t i = xa + threadIdx.x; i < xb; i += BLOCK) {
              const uint32_t e = G.gs_idx[i];
              if ((int32_t)(e & kIdMask) != c) lab.set_bits(e & kIdMask, (e >> kTypeShift) << 2);
            }
            bar<GL>();
            anchor(c, x, -1, ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u));
            for (int32_t i = xa + threadIdx.x; i < xb; i += BLOCK) {
              const uint32_t e = G.gs_idx[i];
              if ((int32_t)(e & kIdMask) != c) lab.clear_bits(e & kIdMask, 3u << 2);
            }
            bar<GL>();
          }
          for (;;) {  // light units are handed to the waves one at a time
            int32_t u = 0;
            if ((threadIdx.x & 63u) == 0) u = atomicAdd(&unit_ctr[2], 1);
            u = __shfl(u, 0);
            if (u >= nlight) break;
            const uint32_t ej = G.gs_idx[unit_list[BLOCK - 1 - u]];
            const uint32_t tcx = ej >> kTypeShift;
            wave_anchor4(c, (int32_t)(ej & kIdMask),
                         ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u));
          }
          bar<GL>();
        }
        js = je;
      }
    }
    if (core >= 0) core_teardown(core);
    hist_flush<C, BLOCK>(hist, acc, cur_g);
    return;
  }

  // Tiles of units cut by estimated cost (UnitCost5) as for k = 4, about
  // `tile` per workgroup, the last quarter four times finer: the units of a
  // light core stay together (one core set-up), a heavy core's are spread.
  const int32_t tot_cost = cpre[total];
  const int64_t parts = (int64_t)gridDim.x * (tile > 0 ? tile : 1);
  const int32_t tc = (int32_t)max((int64_t)kMinTileCost5, ((int64_t)tot_cost + parts - 1) / parts);
  const int32_t split = tot_cost - tot_cost / 4, tc_end = max(1, tc / 4);
  for (;;) {
    pull_tile(tot_cost, tc, split, tc_end);
    bar<GL>();
    const int32_t j0 = sh_j0, j1 = sh_j1;
    bar<GL>();
    if (j0 < 0) break;
    if (j0 >= j1) continue;
    row = G.gs_row[j0];
    for (int32_t j = j0; j < j1; ++j) {
      while (G.gs_off[row + 1] <= j) ++row;
      const int32_t c = row;
      const int32_t rowa = G.gs_off[c], rowb = G.gs_off[c + 1];
      const uint32_t ej = G.gs_idx[j];
      const int32_t x = (int32_t)(ej & kIdMask);
      bool unit;
      if (K == 4) {  // anchor edge {c, x} owned by its higher-rank end
        const int32_t dc = rowb - rowa, dx = G.gs_off[x + 1] - G.gs_off[x];
        unit = dx < dc || (dx == dc && x < c);
      } else {  // unit (b = c, a = x) with the neighbours of b of lower rank than x as partners
        unit = rowb - rowa >= 2;
      }
      if (!unit) continue;
      if (c != core) {
        if (core >= 0) core_teardown(core);
        const int32_t g = G.gid ? G.gid[c] : 0;
        if (g != cur_g) {
          hist_flush<C, BLOCK>(hist, acc, cur_g);
          cur_g = g;
          bar<GL>();
        }
        wbase = G.voff ? G.voff[g] : 0;
        lab.base = (uint32_t)wbase;  // the previous core's labels are cleared
        core = c;
        core_setup(c);
      }
      const uint32_t tcx = ej >> kTypeShift;
      // side labels of x (bits 2-3)
      const int32_t xa = G.gs_off[x], xb = G.gs_off[x + 1];
      for (int32_t i = xa + threadIdx.x; i < xb; i += BLOCK) {
        const uint32_t e = G.gs_idx[i];
        if ((int32_t)(e & kIdMask) != c) lab.set_bits(e & kIdMask, (e >> kTypeShift) << 2);
      }
      bar<GL>();
      if (K == 4) {
        const uint32_t base = ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u);
        anchor(c, x, -1, base);
      } else {
        // partners: the neighbours c2 of b of lower rank (d*, id) than x, so
        // that of the two sides of a triple the heavier one is shared by the
        // unit and the lighter one is done per triple.  Scanned BLOCK at a
        // time: light partners (d*(c2) <= kLight5C) in sub-chunks, the
        // others on the workgroup one by one; x's types stay in the dense
        // labels for both
        const int32_t dx = xb - xa;
        for (int32_t jc0 = rowa; jc0 < rowb; jc0 += BLOCK) {
          const int32_t jce = min(rowb, jc0 + BLOCK);
          if (threadIdx.x < 3) unit_ctr[threadIdx.x] = 0;
          bar<GL>();
          {
            const int32_t jc = jc0 + (int32_t)threadIdx.x;
            if (jc < jce) {
              const int32_t c2 = (int32_t)(G.gs_idx[jc] & kIdMask);
              const int32_t d2 = G.gs_off[c2 + 1] - G.gs_off[c2];
              if (d2 < dx || (d2 == dx && c2 < x)) {
                if (fact5 && d2 <= lim.light5)
                  unit_list[BLOCK - 1 - atomicAdd(&unit_ctr[1], 1)] = jc;
                else
                  unit_list[atomicAdd(&unit_ctr[0], 1)] = jc;
              }
            }
          }
          bar<GL>();
          const int32_t nheavy = unit_ctr[0], nlight = unit_ctr[1];
          for (int32_t u = 0; u < nheavy; ++u) {
            const uint32_t ec = G.gs_idx[unit_list[u]];
            const int32_t c2 = (int32_t)(ec & kIdMask);
            const uint32_t tbc = ec >> kTypeShift;
            const uint32_t tac = (lab.get((uint32_t)c2) >> 2) & 3u;
            if (tac && (c > x || c > c2)) continue;  // triangle: taken at its smallest id
            const uint32_t base = ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u) |
                                  ((tbc & 1u) ? 1u << cbit<K>(0, 2) : 0u) | ((tbc & 2u) ? 1u << cbit<K>(2, 0) : 0u) |
                                  ((tac & 1u) ? 1u << cbit<K>(1, 2) : 0u) | ((tac & 2u) ? 1u << cbit<K>(2, 1) : 0u);
            const int32_t ca2 = G.gs_off[c2], cb2 = G.gs_off[c2 + 1];
            for (int32_t i = ca2 + threadIdx.x; i < cb2; i += BLOCK) {
              const uint32_t e = G.gs_idx[i];
              if ((int32_t)(e & kIdMask) != c) lab.set_bits(e & kIdMask, (e >> kTypeShift) << 4);
            }
            bar<GL>();
            anchor(c, x, c2, base);
            for (int32_t i = ca2 + threadIdx.x; i < cb2; i += BLOCK) {
              const uint32_t e = G.gs_idx[i];
              if ((int32_t)(e & kIdMask) != c) lab.clear_bits(e & kIdMask, 3u << 4);
            }
            bar<GL>();
          }
          if (nlight > 0) {
            // light partners, up to kNP5 at a time with at most kT5Load keys
            // in the merged table; triangles not taken here are dropped.
            // The last wave chooses the next sub-chunk's partners (into the
            // other buffer) while the current sub-chunk finishes.
            constexpr int PW = NW - 1;
            auto pick5 = [&](int32_t u0, int32_t b) {
              if ((int32_t)(threadIdx.x >> 6) == PW) {
                const int32_t lane = (int32_t)(threadIdx.x & 63u), u = u0 + lane;
                const bool in = lane < kNP5 && u < nlight;
                int32_t c2 = -1, cost = 0, rs2 = 0;
                uint32_t base = 0;
                if (lane < 16) cnUb[b][lane] = 0;
                if (in) {
                  const uint32_t ec = G.gs_idx[unit_list[BLOCK - 1 - u]];
                  c2 = (int32_t)(ec & kIdMask);
                  const uint32_t tbc = ec >> kTypeShift;
                  const uint32_t tac = (lab.get((uint32_t)c2) >> 2) & 3u;
                  if (tac && (c > x || c > c2)) {
                    c2 = -1;  // triangle: taken at its smallest id
                  } else {
                    rs2 = G.gs_off[c2];
                    cost = G.gs_off[c2 + 1] - rs2 + 1;
                    base = ((tcx & 1u) ? 1u << cbit<K>(0, 1) : 0u) | ((tcx & 2u) ? 1u << cbit<K>(1, 0) : 0u) |
                           ((tbc & 1u) ? 1u << cbit<K>(0, 2) : 0u) | ((tbc & 2u) ? 1u << cbit<K>(2, 0) : 0u) |
                           ((tac & 1u) ? 1u << cbit<K>(1, 2) : 0u) | ((tac & 2u) ? 1u << cbit<K>(2, 1) : 0u);
                  }
                }
                int32_t inc = cost;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                  const int32_t t = __shfl_up(inc, d);
                  if (lane >= d) inc += t;
                }
                // a prefix of the lanes: lane 0 always fits (cost <= lim.light5 + 1 <= kT5Load)
                const bool take = in && inc <= kT5Load;
                const int32_t ntake = __popcll(__ballot(take));
                const bool act = take && c2 >= 0;
                const unsigned long long am = __ballot(act);
                if (act) {
                  const int32_t k = __popcll(am & ((1ull << lane) - 1ull));
                  p5_vb[b][k] = c2;
                  p5_rowb[b][k] = rs2;
                  p5_baseb[b][k] = base;
                  p5_offb[b][k] = inc - cost;
                }
                const int32_t tot = __shfl(inc, ntake - 1);
                if (lane == 0) {
                  p5_ctlb[b][0] = __popcll(am);
                  p5_ctlb[b][1] = u0 + ntake;
                  p5_ctlb[b][2] = tot;
                  p5_ctlb[b][3] = 0;
                  p5_ctlb[b][4] = 0;
                }
              }
            };
            sb = 0;
            pick5(0, 0);
            bar<GL>();
            for (;;) {
              const int32_t np = p5_ctlb[sb][0], tot = p5_ctlb[sb][2], u1 = p5_ctlb[sb][1];
              if (np > 0) {
                // merged table: partner k's row at [p5_offb[sb][k] + 1, ...), k itself at p5_offb[sb][k]
                for (int32_t t = threadIdx.x; t < tot; t += BLOCK) {
                  int32_t lo = 0, hi = np - 1;
                  while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (p5_offb[sb][mid] <= t) lo = mid; else hi = mid - 1;
                  }
                  const int32_t c2 = p5_vb[sb][lo], kk = t - p5_offb[sb][lo];
                  if (kk == 0) {
                    const uint32_t h = t5_insert((uint32_t)c2);
                    if (h < kT5) tpid[h] = (uint8_t)(lo + 1);
                    lab.set_bits((uint32_t)c2, kInT5);
                  } else {
                    const uint32_t e = G.gs_idx[p5_rowb[sb][lo] + kk - 1];
                    const uint32_t v = e & kIdMask;
                    if ((int32_t)v != c) {
                      const uint32_t h = t5_insert(v);
                      if (h < kT5) atomicOr(&ttyp[h], (u64)(e >> kTypeShift) << (2 * lo));
                      lab.set_bits(v, kInT5);
                    }
                  }
                }
                // distinct base codes of the sub-chunk with their multiplicities
                if ((int32_t)threadIdx.x < np) {
                  const uint32_t bs = p5_baseb[sb][threadIdx.x];
                  bool first = true;
                  int32_t nb = 0;
                  for (int32_t k = 0; k < np; ++k) {
                    const bool same = p5_baseb[sb][k] == bs;
                    nb += same;
                    first = first && !(same && k < (int32_t)threadIdx.x);
                  }
                  if (first) {
                    const int32_t d = atomicAdd(&p5_ctlb[sb][3], 1);
                    p5_db[d] = bs;
                    p5_dc[d] = nb;
                  }
                }
                // edges inside N(core): the same for every triple of the unit
                if (threadIdx.x < 27) {
                  const uint32_t w = Mc[threadIdx.x];
                  if (w) U5[u5i(threadIdx.x / 9 + 1, (threadIdx.x / 3) % 3 + 1, threadIdx.x % 3 + 1)] += w;
                }
                bar<GL>();
                {
                  const int32_t na = 1 + (xb - xa);
                  // the per-(vertex, partner) pairs of the table share the
                  // latency of the first layout pass: they go to the last
                  // threads, whose waves have no item when the items and the
                  // pairs fit in one pass together
                  auto pairs = [&] {
                    for (int32_t t = BLOCK - 1 - (int32_t)threadIdx.x; t < tot; t += BLOCK) {
                      int32_t lo = 0, hi = np - 1;
                      while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (p5_offb[sb][mid] <= t) lo = mid; else hi = mid - 1;
                      }
                      const int32_t c2 = p5_vb[sb][lo], kk = t - p5_offb[sb][lo];
                      if (kk == 0) {
                        pair5(x, lo, c2, true, 0u);
                      } else {
                        const uint32_t e = G.gs_idx[p5_rowb[sb][lo] + kk - 1];
                        if ((int32_t)(e & kIdMask) != c) pair5(x, lo, (int32_t)(e & kIdMask), false, e >> kTypeShift);
                      }
                    }
                  };
                  flat_rows_pre(
                      na + p5_ctlb[sb][4], pairs,
                      [&](int32_t i) { return i < na ? u5_pick(c, x, xa, i) : c5_pick(x, i - na); },
                      [&](int32_t q, uint32_t f, uint32_t qi) { s5_visit(c, x, q, f, qi); }, s5_rowinfo);
                }
                {
                  const int32_t nd = p5_ctlb[sb][3];
                  for (int32_t t = threadIdx.x; t < kU5; t += BLOCK) {
                    const uint32_t w = U5[t];
                    if (!w) continue;
                    U5[t] = 0u;
                    const uint32_t X = (uint32_t)t / 48u, Y = ((uint32_t)t / 3u) % 16u, r = (uint32_t)t % 3u + 1u;
                    const u64 w64 = (u64)(int64_t)(int32_t)w;
                    const uint32_t sx = slot_code<K, S1>(X) | slot_code<K, S2>(Y);
                    for (int32_t d0 = 0; d0 < nd; d0 += 4) {  // table reads of 4 bases, then the counters
                      uint64_t kq[4];
#pragma unroll
                      for (int u = 0; u < 4; ++u) kq[u] = lut_quad(lut, p5_db[min(d0 + u, nd - 1)] | sx);
#pragma unroll
                      for (int u = 0; u < 4; ++u) {
                        if (d0 + u >= nd) break;
                        const u64 wd = w64 * (u64)p5_dc[d0 + u];
                        atomicAdd(&hist[quad_at(kq[u], r)], wd);
                        atomicAdd(&hist[quad_at(kq[u], 0)], (u64)0 - wd);
                      }
                    }
                  }
                }
                // the table is not read any more: cleared alongside the closed forms
                for (int32_t k = threadIdx.x; k < p5_ctlb[sb][4]; k += BLOCK) {
                  const uint32_t h = tlist[k];
                  lab.clear_bits(tkey[h], kInT5);
                  tkey[h] = kEmptySlot;
                  ttyp[h] = 0ull;
                  tpid[h] = 0;
                }
              }
              if (u1 < nlight) pick5(u1, sb ^ 1);
              for (int32_t p = (int32_t)(threadIdx.x >> 6); p < np; p += NW) close5(p, x);
              bar<GL>();
              if (u1 >= nlight) break;
              sb ^= 1;
            }
          }
          // skipped triples read x's labels without a barrier (see k5_kernel)
          bar<GL>();
        }
      }
      for (int32_t i = xa + threadIdx.x; i < xb; i += BLOCK) {
        const uint32_t e = G.gs_idx[i];
        if ((int32_t)(e & kIdMask) != c) lab.clear_bits(e & kIdMask, 3u << 2);
      }
      bar<GL>();
    }
  }
  if (core >= 0) core_teardown(core);
  hist_flush<C, BLOCK>(hist, acc, cur_g);
}

// Per-entry cost estimate of the k = 4 core-reuse kernel, for cutting its
// work queue into tiles of similar cost: 1 for an entry that is not a unit,
// else a fixed part (larger for a heavy unit, which takes the whole
// workgroup) plus a quarter of the side's degree; 0 past the last entry.
// Clamped to cmax so that the prefix sum stays below 2^31; any positive costs
// give a correct tiling.  The values are scanned as they are computed.
struct UnitCost4 {
  DevGraph G;
  int32_t cmax, light_deg;
  __device__ int32_t operator()(int64_t j) const {
    if (j >= G.gs_off[G.n]) return 0;
    const int32_t r = G.gs_row[j], x = (int32_t)(G.gs_idx[j] & kIdMask);
    const int32_t dr = G.gs_off[r + 1] - G.gs_off[r], dx = G.gs_off[x + 1] - G.gs_off[x];
    if (dx < dr || (dx == dr && x < r)) return min(cmax, (dx > light_deg ? 40 : 4) + (dx >> 2));
    return 1;
  }
};

// The same for the k = 5 core-reuse kernel: every G* entry (b, a) is a unit
// whose partners are about half of b's row, taken in sub-chunks, so its cost
// grows with d*(b); the fixed part covers the unit's labels and barriers.
struct UnitCost5 {
  DevGraph G;
  int32_t cmax;
  __device__ int32_t operator()(int64_t j) const {
    if (j >= G.gs_off[G.n]) return 0;
    const int32_t r = G.gs_row[j];
    return min(cmax, 8 + (G.gs_off[r + 1] - G.gs_off[r]));
  }
};

// Hub slots for the core-reuse scheme: the vertices of largest degree get one
// of kMaxHubs rows of the per-core W table; the threshold is the smallest
// power of two whose degree bucket and all above hold at most kMaxHubs
// vertices (and at least 32).  The same buckets choose the big cores (at most
// nbig, degree >= kBigMinDeg).  hs[0..31] = counts per floor(log2 d),
// hs[33] = hub slot counter, hs[35] = big-core slot counter (all zero at the
// start).  Which vertices get slots never changes the result, only where the
// work goes.
__global__ void k_degree_buckets(const int32_t* gs_off, int32_t n, int32_t* hs, const int32_t* st) {
  __shared__ int32_t b[32];
  if (st[kStatus] != 0) return;
  if (threadIdx.x < 32) b[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = gs_off[v + 1] - gs_off[v];
    if (d > 0) atomicAdd(&b[31 - __clz(d)], 1);
  }
  __syncthreads();
  if (threadIdx.x < 32 && b[threadIdx.x]) atomicAdd(&hs[threadIdx.x], b[threadIdx.x]);
}

// Every workgroup derives both thresholds from the buckets, then hands out
// the slots.
__global__ void k_assign_hubs(const int32_t* gs_off, int32_t n, int32_t* hs, int32_t* hub_id, int32_t nbig,
                              int32_t* big_id, int32_t* big_list, const int32_t* st) {
  __shared__ int32_t thr[2];
  if (st[kStatus] != 0) return;
  if (threadIdx.x == 0) {
    int32_t cum = 0, b = 30;
    while (b > 5 && cum + hs[b] <= kMaxHubs) cum += hs[b--];
    thr[0] = 1 << (b + 1);
    cum = 0;
    b = 30;
    while ((1 << b) >= kBigMinDeg && cum + hs[b] <= nbig) cum += hs[b--];
    thr[1] = b == 30 ? 0x7fffffff : 1 << (b + 1);
  }
  __syncthreads();
  const int32_t t = thr[0], tb = thr[1];
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = gs_off[v + 1] - gs_off[v];
    int32_t h = -1;
    if (d >= t) {
      h = atomicAdd(&hs[33], 1);
      if (h >= kMaxHubs) h = -1;
    }
    hub_id[v] = h;
    if (big_id) {
      int32_t b = -1;
      if (d >= tb) {
        b = atomicAdd(&hs[35], 1);
        if (b >= nbig) b = -1;
        else big_list[b] = (int32_t)v;
      }
      big_id[v] = b;
    }
  }
}

// Types of the neighbours of each big core, 2 bits per vertex of its graph.
__global__ void k_big_labels(DevGraph G, const int32_t* hs, const int32_t* big_list, uint32_t* lbig, int64_t lstride,
                             const int32_t* st) {
  if (st[kStatus] != 0 || (int32_t)blockIdx.y >= min(hs[35], kMaxBig)) return;
  const int32_t c = big_list[blockIdx.y];
  const int64_t wbase = G.voff ? G.voff[G.gid[c]] : 0;
  uint32_t* L = lbig + blockIdx.y * lstride;
  for (int32_t i = G.gs_off[c] + blockIdx.x * blockDim.x + threadIdx.x; i < G.gs_off[c + 1];
       i += gridDim.x * blockDim.x) {
    const uint32_t e = G.gs_idx[i];
    const int64_t x = (int64_t)(e & kIdMask) - wbase;
    atomicOr(&L[x >> 4], (e >> kTypeShift) << (2 * (x & 15)));
  }
}

// W rows and M counts of each big core (the per-core set-up of the core-reuse
// kernel, done once): thread (entry y of the core's row, lane s of 4) takes
// every fourth entry of N+(y).  The rows of hub vertices, which many entries
// hit, are summed in LDS first and added once per workgroup (their global
// atomics otherwise queue up on a few addresses).
__global__ __launch_bounds__(256) void k_core_tables(DevGraph G, const int32_t* hs, const int32_t* big_list,
                                                     const uint32_t* lbig, int64_t lstride, uint32_t* wbig,
                                                     int64_t wstride, uint32_t* mbig, const int32_t* hub_id,
                                                     const int32_t* st) {
  __shared__ uint32_t M[27];
  __shared__ uint32_t Wh[kMaxHubs * 9];
  __shared__ int32_t hubx[kMaxHubs];
  if (st[kStatus] != 0 || (int32_t)blockIdx.y >= min(hs[35], kMaxBig)) return;
  if (threadIdx.x < 27) M[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < kMaxHubs * 9; i += 256) Wh[i] = 0u;
  __syncthreads();
  const int32_t b = blockIdx.y, c = big_list[b];
  const int64_t wbase = G.voff ? G.voff[G.gid[c]] : 0;
  const uint32_t* L = lbig + b * lstride;
  uint32_t* Wb = wbig + b * wstride;
  const int32_t ca = G.gs_off[c], dc = G.gs_off[c + 1] - ca;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 4 * (int64_t)dc;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ey = G.gs_idx[ca + (int32_t)(t >> 2)];
    const int32_t y = (int32_t)(ey & kIdMask);
    const uint32_t ty = ey >> kTypeShift;
    for (int32_t p = G.np_off[y] + (int32_t)(t & 3); p < G.np_off[y + 1]; p += 4) {
      const uint32_t f = G.np_idx[p];
      const int32_t x = (int32_t)(f & kIdMask);
      if (x == c) continue;
      const uint32_t r = f >> kTypeShift;
      const int64_t xl = (int64_t)x - wbase;
      const int32_t h = hub_id[x];
      if (h >= 0) {
        hubx[h] = x;
        atomicAdd(&Wh[h * 9 + (ty - 1) * 3 + (r - 1)], 1u);
      } else {
        atomicAdd(&Wb[xl * kBigRow + (ty - 1) * 3 + (r - 1)], 1u);
      }
      const uint32_t tx = (L[xl >> 4] >> (2 * (xl & 15))) & 3u;
      if (tx) atomicAdd(&M[(ty - 1) * 9 + (tx - 1) * 3 + (r - 1)], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < 27 && M[threadIdx.x]) atomicAdd(&mbig[b * 32 + threadIdx.x], M[threadIdx.x]);
  for (int i = threadIdx.x; i < kMaxHubs * 9; i += 256)
    if (Wh[i]) atomicAdd(&Wb[((int64_t)hubx[i / 9] - wbase) * kBigRow + i % 9], Wh[i]);
}

// =========================================================== finalise ==
// Exact division of every class total by its anchor multiplicity; a non-zero
// remainder is a self-check failure and blocks the write.
__global__ void k_div_check(const uint64_t* acc, const uint8_t* mult, int32_t C, int64_t total, int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    if (acc[i] % mult[i % C]) atomicMin(&st[kStatus], MOTIF_EINTERNAL);
}

__global__ void k_div_write(const uint64_t* acc, const uint8_t* mult, int32_t C, int64_t total, uint64_t* out,
                            const int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = acc[i] / mult[i % C];
}

unsigned blocks_for(int64_t items, int block) {
  int64_t g = (items + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
}

int label_cap_k4(int32_t n) {
  const int64_t bytes = ((int64_t)n + 7) / 8 * 4;
  return bytes <= 8192 ? 8192 : bytes <= 65536 ? 65536 : 0;
}
int label_cap_k5(int32_t n) {
  const int64_t bytes = ((int64_t)n + 3) / 4 * 4;
  return bytes <= 16384 ? 16384 : bytes <= 32768 ? 32768 : 0;
}
int64_t label_words(int k, int32_t n) { return k == 4 ? ((int64_t)n + 7) / 8 : ((int64_t)n + 3) / 4; }

// Number of big-core table slots for graphs of at most maxn vertices.
int big_slots(int64_t maxn) {
  const int64_t per = (int64_t)kBigRow * 4 * (maxn > 0 ? maxn : 1);
  return (int)std::min<int64_t>(kMaxBig, kBigBytes / per);
}
int64_t big_label_words(int64_t maxn) { return ((maxn > 0 ? maxn : 1) + 15) / 16; }

int grid_size(const Tuning& t, int num_cus) { return num_cus * t.grid_per_cu; }

// Largest per-entry cost that keeps the exclusive cost prefix of gs_cap
// entries (costs >= 1) within int32: tot <= cmax * gs_cap <= 2^31 - 1.
int32_t cost_cap(int64_t gs_cap) {
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(1 << 16, ((int64_t(1) << 31) - 1) / gs_cap));
}

}  // namespace

std::vector<uint16_t> device_lut_order(int k, const uint16_t* lut, size_t len) {
  if (k != 5) return std::vector<uint16_t>(lut, lut + len);
  // row-major bit n of the arc (i, j) goes to bit to[n]
  int to[20] = {};
  for (int i = 0, n = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      if (i != j) to[n++] = cbit<5>(i, j);
  const int bits = k * (k - 1);
  std::vector<uint16_t> out(len);
  for (size_t x = 0; x < len; ++x) {
    uint32_t y = 0;
    for (int n = 0; n < bits; ++n)
      if ((x >> n) & 1u) y |= 1u << to[n];
    out[y] = lut[x];
  }
  return out;
}

size_t pipeline_bytes(int64_t N, int64_t M, int32_t G, bool batch, int k, int num_cus, int64_t maxn,
                      const Tuning& t) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t b = build_bytes(N, M, G, batch);
  const bool reuse = (k == 4 || k == 5) && t.heavy == 1;
  if (reuse)
    b += al(sizeof(int32_t) * (N + 1)) + al(64 * sizeof(int32_t)) +
         al(sizeof(uint32_t) * kBigRow * (size_t)(maxn > 0 ? maxn : N) * grid_size(t, num_cus));
  if (reuse)  // cost prefix of the G* entries and its look-back words
    b += al(sizeof(int32_t) * (2 * M + 1)) + scan1_bytes(2 * M + 1);
  if (reuse) {
    const int64_t mn = maxn > 0 ? maxn : N;
    const int nb = big_slots(mn);
    if (nb > 0)  // big-core ids, list, labels, W rows, M counts
      b += al(sizeof(int32_t) * (N + 1)) + al(sizeof(int32_t) * kMaxBig) +
           al(sizeof(uint32_t) * (size_t)nb * big_label_words(mn)) + al(sizeof(uint32_t) * (size_t)nb * kBigRow * mn) +
           al(sizeof(uint32_t) * 32 * kMaxBig);
  }
  b += 2 * al(sizeof(uint64_t) * (size_t)G * num_classes(k));  // accumulators (+ output staging)
  b += al(64 * sizeof(int32_t));                               // queue counters
  // labels are indexed within one graph: room for the largest one
  const int32_t ln = (int32_t)(maxn > 0 ? maxn : N);
  const int cap = k == 4 ? label_cap_k4(ln) : k == 5 ? label_cap_k5(ln) : 1;
  if (cap == 0) b += al(sizeof(uint32_t) * (size_t)label_words(k, ln) * grid_size(t, num_cus));
  return b + 4096;
}

#define LAUNCH_K4(BLOCK, CAP)                                                                                   \
  hipLaunchKernelGGL((k4_kernel<BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[4], acc, p.status, queue, \
                     glabels, lw, t.tile)
#define LAUNCH_KR(K, BLOCK, CAP)                                                                        \
  hipLaunchKernelGGL((kr_kernel<K, BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[K], acc, p.status, queue, \
                     glabels, lw, hub_id, wg, ws, t.tile, cpre, big_id, wbig, wbig_stride, mbig, lim)
#define LAUNCH_K5(BLOCK, CAP)                                                                                   \
  hipLaunchKernelGGL((k5_kernel<BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[5], acc, p.status, queue, \
                     glabels, lw, t.tile)

size_t w_slice_bytes(int k, int64_t maxn, const Tuning& t, int num_cus) {
  if (!((k == 4 || k == 5) && t.heavy == 1)) return 0;
  return sizeof(uint32_t) * kBigRow * (size_t)(maxn > 0 ? maxn : 1) * (size_t)grid_size(t, num_cus);
}

BigTables take_big_tables(Pipeline& p, int k, int32_t n, int64_t maxn, const Tuning& t, ZeroBatch& z) {
  BigTables b;
  const bool reuse = (k == 4 || k == 5) && t.heavy == 1;
  b.nbig = reuse && n > 0 ? big_slots(maxn) : 0;
  if (b.nbig == 0) return b;
  const int64_t lstride = big_label_words(maxn), wstride = (int64_t)kBigRow * maxn;
  b.big_id = p.arena.take<int32_t>(n + 1);
  b.big_list = p.arena.take<int32_t>(kMaxBig);
  b.lbig = p.arena.take<uint32_t>((size_t)b.nbig * lstride);
  b.wbig = p.arena.take<uint32_t>((size_t)b.nbig * wstride);
  b.mbig = p.arena.take<uint32_t>(32 * kMaxBig);
  z.add(b.lbig, sizeof(uint32_t) * (size_t)b.nbig * lstride);
  z.add(b.wbig, sizeof(uint32_t) * (size_t)b.nbig * wstride);
  z.add(b.mbig, sizeof(uint32_t) * 32 * kMaxBig);
  return b;
}

void enqueue_census(Pipeline& p, const DevGraph& g, int k, uint64_t* acc, uint64_t* out, hipStream_t s,
                    bool use_wpool, hipEvent_t side_start, bool* side_ok, const BigTables* pre) {
  bool forked = side_start == nullptr;
  auto fork_side = [&] {
    if (forked) return;
    forked = true;
    *side_ok = hipEventRecord(side_start, s) == hipSuccess;
  };
  const DevTables& T = dev_tables();
  const int C = num_classes(k);
  const int64_t total = (int64_t)g.ngraphs * C;
  // every region the set-up needs cleared goes into one batch, launched
  // before the first kernel that reads any of them
  ZeroBatch z;
  z.add(acc, sizeof(uint64_t) * total);
  int32_t* queue = p.arena.take<int32_t>(64);
  z.add(queue, 64 * sizeof(int32_t));
  const Tuning& t = p.tune.k[k];
  const int grid = grid_size(t, p.num_cus);
  const Limits lim{std::min(t.solo_deg, kSoloDegMax), std::min(t.light_deg, kLightDegMax),
                   std::min(t.light5, kLight5Max)};
  bool marked = false;  // the profiling events bracket the main census kernel only
  if (g.n > 0) {
    if (k == 3) {
      enqueue_zero_batch(z, s);
      fork_side();
      profile_mark(k, 1, true, s);
      marked = true;
      hipLaunchKernelGGL((k3_kernel<256>), dim3(grid), dim3(256), 0, s, g, T.lut[3], acc, p.status, queue,
                         std::max(1, t.tile));
    } else {
      const bool reuse = t.heavy == 1;
      // labels are indexed within one graph (Labels::base): room for the largest
      const int32_t ln = g.max_graph_n > 0 ? g.max_graph_n : g.n;
      const int cap = k == 4 ? label_cap_k4(ln) : label_cap_k5(ln);
      const int64_t lw = label_words(k, ln);
      uint32_t* glabels = nullptr;
      if (cap == 0) {
        glabels = p.arena.take<uint32_t>((size_t)lw * grid);
        z.add(glabels, sizeof(uint32_t) * (size_t)lw * grid);
      }
      int32_t* hub_id = nullptr;
      uint32_t* wg = nullptr;
      int64_t ws = 0;
      const int64_t maxn = g.max_graph_n > 0 ? g.max_graph_n : g.n;
      const BigTables bt = pre ? *pre : take_big_tables(p, k, g.n, maxn, t, z);
      const int nbig = bt.nbig;
      int32_t *big_id = bt.big_id, *big_list = bt.big_list;
      uint32_t *lbig = bt.lbig, *wbig = bt.wbig, *mbig = bt.mbig;
      const int64_t lstride = big_label_words(maxn), wbig_stride = (int64_t)kBigRow * maxn;
      int32_t* hs = nullptr;
      int32_t* cost = nullptr;
      Scan1 sc_cost;
      if (reuse) {
        ws = kBigRow * (int64_t)(g.max_graph_n > 0 ? g.max_graph_n : g.n);
        if (use_wpool && p.wpool && p.wpool_bytes >= sizeof(uint32_t) * (size_t)ws * grid) {
          wg = p.wpool;  // all zero: every earlier census cleared the rows it used
        } else {
          wg = p.arena.take<uint32_t>((size_t)ws * grid);
          z.add(wg, sizeof(uint32_t) * (size_t)ws * grid);
        }
        hub_id = p.arena.take<int32_t>(g.n + 1);
        hs = p.arena.take<int32_t>(64);
        z.add(hs, 64 * sizeof(int32_t));
        cost = p.arena.take<int32_t>((size_t)g.gs_cap);
        sc_cost = scan1_take(p.arena, g.gs_cap, z);
      }
      enqueue_zero_batch(z, s);
      if (reuse) {
        hipLaunchKernelGGL(k_degree_buckets, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.gs_off, g.n, hs, p.status);
        hipLaunchKernelGGL(k_assign_hubs, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.gs_off, g.n, hs, hub_id,
                           nbig, big_id, big_list, p.status);
        const int32_t cmax = cost_cap(g.gs_cap);
        if (k == 4)
          enqueue_scan1(sc_cost, cost, UnitCost4{g, cmax, lim.light}, p.status, s);
        else
          enqueue_scan1(sc_cost, cost, UnitCost5{g, cmax}, p.status, s);
        if (nbig > 0)
          hipLaunchKernelGGL(k_big_labels, dim3(16, nbig), dim3(256), 0, s, g, hs, big_list, lbig, lstride, p.status);
        fork_side();
        if (nbig > 0) {
          hipLaunchKernelGGL(k_core_tables, dim3(64, nbig), dim3(256), 0, s, g, hs, big_list, lbig, lstride, wbig,
                             wbig_stride, mbig, hub_id, p.status);
        }
      }
      const int32_t* cpre = reuse ? cost : nullptr;
      fork_side();
      profile_mark(k, 1, true, s);
      marked = true;
      if (k == 4 && reuse) {
        if (t.block == 512) {
          if (cap == 8192) LAUNCH_KR(4, 512, 8192); else if (cap == 65536) LAUNCH_KR(4, 512, 65536); else LAUNCH_KR(4, 512, 0);
        } else if (t.block == 1024) {
          if (cap == 8192) LAUNCH_KR(4, 1024, 8192); else if (cap == 65536) LAUNCH_KR(4, 1024, 65536); else LAUNCH_KR(4, 1024, 0);
        } else {
          if (cap == 8192) LAUNCH_KR(4, 256, 8192); else if (cap == 65536) LAUNCH_KR(4, 256, 65536); else LAUNCH_KR(4, 256, 0);
        }
      } else if (k == 4) {
        if (t.block == 512) {
          if (cap == 8192) LAUNCH_K4(512, 8192); else if (cap == 65536) LAUNCH_K4(512, 65536); else LAUNCH_K4(512, 0);
        } else if (t.block == 1024) {
          if (cap == 8192) LAUNCH_K4(1024, 8192); else if (cap == 65536) LAUNCH_K4(1024, 65536); else LAUNCH_K4(1024, 0);
        } else {
          if (cap == 8192) LAUNCH_K4(256, 8192); else if (cap == 65536) LAUNCH_K4(256, 65536); else LAUNCH_K4(256, 0);
        }
      } else if (reuse) {
        if (t.block == 512) {
          if (cap == 16384) LAUNCH_KR(5, 512, 16384); else if (cap == 32768) LAUNCH_KR(5, 512, 32768); else LAUNCH_KR(5, 512, 0);
        } else {
          if (cap == 16384) LAUNCH_KR(5, 1024, 16384); else if (cap == 32768) LAUNCH_KR(5, 1024, 32768); else LAUNCH_KR(5, 1024, 0);
        }
      } else {
        if (t.block == 512) {
          if (cap == 16384) LAUNCH_K5(512, 16384); else if (cap == 32768) LAUNCH_K5(512, 32768); else LAUNCH_K5(512, 0);
        } else {
          if (cap == 16384) LAUNCH_K5(1024, 16384); else if (cap == 32768) LAUNCH_K5(1024, 32768); else LAUNCH_K5(1024, 0);
        }
      }
    }
  }
  if (g.n == 0) enqueue_zero_batch(z, s);
  fork_side();
  if (!marked) profile_mark(k, 1, true, s);
  profile_mark(k, 1, false, s);
  if (out) enqueue_finalise(p, k, g.ngraphs, acc, out, s);
}

void enqueue_finalise(Pipeline& p, int k, int32_t ngraphs, const uint64_t* acc, uint64_t* out, hipStream_t s) {
  const int C = num_classes(k);
  enqueue_divide(acc, dev_tables().mult[k], C, (int64_t)ngraphs * C, out, p.status, s);
}

void enqueue_divide(const uint64_t* acc, const uint8_t* mult, int32_t C, int64_t total, uint64_t* out,
                    int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_div_check, dim3(blocks_for(total, 256)), dim3(256), 0, s, acc, mult, C, total, status);
  hipLaunchKernelGGL(k_div_write, dim3(blocks_for(total, 256)), dim3(256), 0, s, acc, mult, C, total, out, status);
}

}  // namespace motif
