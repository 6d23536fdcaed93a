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
#include <hip/hip_runtime.h>

#include "internal.h"

namespace motif {

namespace {

template <int K>
__host__ __device__ constexpr int cbit(int i, int j) {
  return i * (K - 1) + (j < i ? j : j - 1);
}

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

__device__ __forceinline__ uint32_t flip(uint32_t t) { return ((t & 1u) << 1) | ((t & 2u) >> 1); }

constexpr int num_classes(int k) { return k == 3 ? 13 : k == 4 ? 199 : 9364; }

constexpr int kMaxHubs = 512;  // rows of the per-core W table in LDS

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
template <int BITS, bool GLOBAL = false>
struct Labels {
  uint32_t* w;
  static constexpr int kPer = 32 / BITS;
  static constexpr uint32_t kMask = (1u << BITS) - 1u;
  __device__ __forceinline__ uint32_t word(uint32_t i) const {
    if constexpr (GLOBAL) return __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return w[i];
  }
  __device__ __forceinline__ uint32_t get(uint32_t x) const {
    return (word(x / kPer) >> ((x % kPer) * BITS)) & kMask;
  }
  __device__ __forceinline__ void set_bits(uint32_t x, uint32_t v) const {
    atomicOr(&w[x / kPer], v << ((x % kPer) * BITS));
  }
  __device__ __forceinline__ void clear_bits(uint32_t x, uint32_t v) const {
    atomicAnd(&w[x / kPer], ~(v << ((x % kPer) * BITS)));
  }
  __device__ __forceinline__ void clear_all(uint32_t x) const {
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
// u -> w -> x in rank order: N+(u) ∩ N+(w).  For each corner the pair of the
// other two corners leaves its open class, and the triangle class gains one
// occurrence per corner (the division by 3 removes the repetition).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k3_kernel(DevGraph G, const uint16_t* __restrict__ lut_g,
                                                   uint64_t* __restrict__ acc, const int32_t* st, int32_t tv) {
  constexpr int K = 3, C = 13;
  __shared__ u64 hist[C];
  __shared__ uint16_t lut[64];
  if (st[kStatus] != 0) return;
  for (int i = threadIdx.x; i < 64; i += BLOCK) lut[i] = lut_g[i];
  for (int i = threadIdx.x; i < C; i += BLOCK) hist[i] = 0;
  __syncthreads();
  const int32_t n = G.n;
  const int32_t ntiles = (n + tv - 1) / tv;
  int32_t cur_g = -1;
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int32_t v0 = t * tv;
    const int32_t v1 = min(n, v0 + tv);
    while (v0 < v1) {
      const int32_t g = G.gid ? G.gid[v0] : 0;
      int32_t end = v1;
      if (G.gid) {  // first vertex of the tile in a later graph
        int32_t lo = v0, hi = v1;
        while (lo < hi) {
          int32_t mid = (lo + hi) >> 1;
          if (G.gid[mid] > g) hi = mid; else lo = mid + 1;
        }
        end = lo;
      }
      if (g != cur_g) {
        __syncthreads();
        hist_flush<C, BLOCK>(hist, acc, cur_g);
        cur_g = g;
        __syncthreads();
      }
      // closed form at every vertex of [v0, end)
      for (int32_t v = v0 + threadIdx.x; v < end; v += BLOCK) {
        u64 na = 0, nb = 0, nc = 0;
        for (int32_t j = G.gs_off[v]; j < G.gs_off[v + 1]; ++j) {
          const uint32_t ty = G.gs_idx[j] >> kTypeShift;
          na += ty == 3u;
          nb += ty == 1u;
          nc += ty == 2u;
        }
        const u64 w[6] = {na * nb, na * nc, nb * nc, na * (na - (na > 0)) / 2, nb * (nb - (nb > 0)) / 2,
                          nc * (nc - (nc > 0)) / 2};
        const uint32_t ta[6] = {3, 3, 1, 3, 1, 2};
        const uint32_t tb[6] = {1, 2, 2, 3, 1, 2};
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (w[q]) atomicAdd(&hist[lut[slot_code<K, 1>(ta[q]) | slot_code<K, 2>(tb[q])]], w[q]);
      }
      // triangles through the oriented edges leaving [v0, end)
      const int32_t j0 = G.np_off[v0], j1 = G.np_off[end];
      for (int32_t j = j0 + threadIdx.x; j < j1; j += BLOCK) {
        const int32_t u = find_row(G.np_off, v0, end, j);
        const uint32_t e = G.np_idx[j];
        const int32_t w = (int32_t)(e & kIdMask);
        const uint32_t tuw = e >> kTypeShift;
        const int32_t ua = G.np_off[u], ub = G.np_off[u + 1];
        for (int32_t p = G.np_off[w]; p < G.np_off[w + 1]; ++p) {
          const uint32_t f = G.np_idx[p];
          const int32_t x = (int32_t)(f & kIdMask);
          int32_t lo = ua, hi = ub;
          while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if ((int32_t)(G.np_idx[mid] & kIdMask) < x) lo = mid + 1; else hi = mid;
          }
          if (lo < ub && (int32_t)(G.np_idx[lo] & kIdMask) == x) {
            const uint32_t tux = G.np_idx[lo] >> kTypeShift, twx = f >> kTypeShift;
            const uint32_t full = slot_code<K, 1>(tuw) | slot_code<K, 2>(tux) | rel_code<K>(twx);
            atomicAdd(&hist[lut[full]], 3ull);
            atomicAdd(&hist[lut[slot_code<K, 1>(tuw) | slot_code<K, 2>(tux)]], kMinusOne);
            atomicAdd(&hist[lut[slot_code<K, 1>(flip(tuw)) | slot_code<K, 2>(twx)]], kMinusOne);
            atomicAdd(&hist[lut[slot_code<K, 1>(flip(tux)) | slot_code<K, 2>(flip(twx))]], kMinusOne);
          }
        }
      }
      v0 = end;
    }
  }
  __syncthreads();
  hist_flush<C, BLOCK>(hist, acc, cur_g);
}

// Closed form over the non-empty neighbour sets of one anchor: pairs within a
// set, C(n,2), and across two sets, n_i n_j (Facts "base" / "basefive").
template <int K, int NL, int BLOCK>
__device__ __forceinline__ void closed_form(u64* hist, const uint16_t* lut, const int32_t* cnt, int32_t* nzl,
                                            int32_t* nz_count, uint32_t base) {
  if (threadIdx.x == 0) {
    int32_t z = 0;
    for (int L = 1; L < NL; ++L)
      if (cnt[L]) nzl[z++] = L;
    *nz_count = z;
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
    if (threadIdx.x == 0) sh_j0 = atomicAdd(queue, tile);
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
    if (threadIdx.x == 0) sh_j0 = atomicAdd(queue, tile);
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
                                                   uint32_t* __restrict__ wg, int64_t w_stride, int32_t tile) {
  constexpr int C = K == 4 ? 199 : 9364, NL = K == 4 ? 16 : 64, LB = K == 4 ? 4 : 8;
  constexpr int S1 = K - 2, S2 = K - 1;  // member slots
  // LDS rows of W: fewer where the k = 5 counters and labels leave no room
  constexpr int HUBS = (K == 5 && LCAP == 65536) ? 256 : kMaxHubs;
  constexpr bool GL = LCAP == 0;
  __shared__ u64 hist[C];
  __shared__ uint16_t lut_lds[K == 4 ? 4096 : 1];
  __shared__ int32_t cnt[NL], nzl[NL], nz_count;
  __shared__ uint32_t Mc[27];
  __shared__ uint32_t W[HUBS * 9];
  __shared__ int32_t ncore[4];
  __shared__ int32_t sh_j0;
  __shared__ u64 seg_ctr[2];  // (rows << 32) | entries of the chunk being laid out
  __shared__ int32_t seg_v[BLOCK], seg_start[BLOCK];
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
  if (LCAP > 0)
    for (int i = threadIdx.x; i < LCAP / 4; i += BLOCK) lds_labels[i] = 0u;
  __syncthreads();

  const int32_t n = G.n;
  const int32_t total = G.gs_off[n];
  int32_t cur_g = -1, row = 0, core = -1, par = 0;
  int64_t wbase = 0;  // first vertex of the core's graph
  auto wrow = [&](int32_t q) { return WG + (int64_t)(q - wbase) * 16; };
  auto hub = [&](int32_t q) {
    const int32_t h = hub_id[q];
    return h < HUBS ? h : -1;
  };
  // contribution of one edge between slots S1 (x) and S2 (y) of weight w
  auto edge = [&](uint32_t base, uint32_t Lx, uint32_t Ly, uint32_t r, u64 w) {
    const uint32_t c0 = base | slot_code<K, S1>(Lx) | slot_code<K, S2>(Ly);
    atomicAdd(&hist[lut[c0 | rel_code<K>(r)]], w);
    atomicAdd(&hist[lut[c0]], (u64)0 - w);
  };
  // Flattened scan of the N+ rows of the vertices pick(0 .. items-1): pick
  // returns a vertex (or -1) and does the per-vertex work, visit(v, f) handles
  // one entry f of N+(v).  Uniform across the workgroup; ends with a barrier.
  // seg_ctr alternates between two words so that one of them can be cleared
  // while the other is read.
  auto flat_rows = [&](int32_t items, auto&& pick, auto&& visit) {
    for (int32_t i0 = 0; i0 < items; i0 += BLOCK) {
      const int32_t i = i0 + (int32_t)threadIdx.x;
      if (i < items) {
        const int32_t v = pick(i);
        if (v >= 0) {
          const int32_t len = G.np_off[v + 1] - G.np_off[v];
          if (len > 0) {  // |N+(v)| <= sqrt(2 |E*|), so BLOCK rows fit in 32 bits
            const u64 old = atomicAdd(&seg_ctr[par], (1ull << 32) | (u64)len);
            const int32_t sl = (int32_t)(old >> 32);
            seg_v[sl] = v;
            seg_start[sl] = (int32_t)(uint32_t)old;
          }
        }
      }
      bar<GL>();
      const u64 ctr = seg_ctr[par];
      const int32_t nseg = (int32_t)(ctr >> 32), tot = (int32_t)(uint32_t)ctr;
      if (threadIdx.x == 0) seg_ctr[par ^ 1] = 0;
      int32_t sl = 0;
      for (int32_t j = threadIdx.x; j < tot; j += BLOCK) {
        int32_t hi = nseg - 1;  // last row starting at or before j (starts increase with sl)
        while (sl < hi) {
          const int32_t mid = (sl + hi + 1) >> 1;
          if (seg_start[mid] <= j) sl = mid; else hi = mid - 1;
        }
        const int32_t v = seg_v[sl];
        visit(v, G.np_idx[G.np_off[v] + (j - seg_start[sl])]);
      }
      bar<GL>();
      par ^= 1;
    }
  };
  // per-core set-up (labels of N(core), type counts, M, W) and tear-down
  auto core_setup = [&](int32_t c) {
    const int32_t ca = G.gs_off[c], dcn = G.gs_off[c + 1] - ca;
    for (int32_t i = threadIdx.x; i < dcn; i += BLOCK) {
      const uint32_t e = G.gs_idx[ca + i];
      lab.set_bits(e & kIdMask, e >> kTypeShift);
      atomicAdd(&ncore[e >> kTypeShift], 1);
    }
    bar<GL>();
    flat_rows(
        dcn, [&](int32_t i) { return (int32_t)(G.gs_idx[ca + i] & kIdMask); },
        [&](int32_t y, uint32_t f) {
          const int32_t x = (int32_t)(f & kIdMask);
          if (x == c) return;
          const uint32_t r = f >> kTypeShift, ty = lab.get((uint32_t)y) & 3u;
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
    flat_rows(
        dcn,
        [&](int32_t i) {
          const int32_t y = (int32_t)(G.gs_idx[ca + i] & kIdMask);
          lab.clear_bits((uint32_t)y, 3u);
          return y;
        },
        [&](int32_t, uint32_t f) {
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
      uint32_t wq[9];
      const int32_t hq = hub(q);
      if (hq >= 0) {
#pragma unroll
        for (int tr = 0; tr < 9; ++tr) wq[tr] = W[hq * 9 + tr];
      } else {
        const uint4* w4 = reinterpret_cast<const uint4*>(wrow(q));
        const uint4 x0 = w4[0], x1 = w4[1], x2 = w4[2];
        wq[0] = x0.x; wq[1] = x0.y; wq[2] = x0.z; wq[3] = x0.w;
        wq[4] = x1.x; wq[5] = x1.y; wq[6] = x1.z; wq[7] = x1.w; wq[8] = x2.x;
      }
#pragma unroll
      for (int tr = 0; tr < 9; ++tr) {
        const uint32_t w = wq[tr];
        if (!w) continue;
        const uint32_t tp = (uint32_t)(tr / 3) + 1u, r = (uint32_t)(tr % 3) + 1u;
        if (cq) edge(base, tp, cq, r, (u64)0 - (u64)w);
        if (mq) edge(base, tp, Lq, r, (u64)w);
      }
      return q;
    };
    // one edge q -> y of N+(q) with q in R'
    auto visit = [&](int32_t q, uint32_t f) {
      const int32_t y = (int32_t)(f & kIdMask);
      if (y == c) return;
      const uint32_t Ly = lab.get((uint32_t)y);
      const bool sy = is_side(y);
      if (!Ly && !sy) return;
      const uint32_t Lq = lab.get((uint32_t)q);
      const bool mq = !is_side(q), my = !sy;
      const uint32_t r = f >> kTypeShift, cq = Lq & 3u, cy = Ly & 3u;
      if (cq && cy) edge(base, cq, cy, r, kMinusOne);
      if (mq && my) edge(base, Lq, Ly, r, 1ull);
      if (cq && (sy || (Ly >> 2))) {  // p = q is also counted in W[y]
        if (cy) edge(base, cq, cy, r, 1ull);
        if (my) edge(base, cq, Ly, r, kMinusOne);
      }
    };
    flat_rows(nsides + d0 + d1, pick, visit);
    // edges inside N(core) with core-only labels
    if (threadIdx.x < 27) {
      const uint32_t w = Mc[threadIdx.x];
      if (w) {
        const uint32_t tx = threadIdx.x / 9 + 1, ty = (threadIdx.x / 3) % 3 + 1, r = threadIdx.x % 3 + 1;
        edge(base, tx, ty, r, (u64)w);
      }
    }
    // sizes of the core-only sets: N(core) minus the sides minus R'
    if (threadIdx.x < 3) {
      const int32_t a = threadIdx.x + 1;
      int32_t v = ncore[a];
      for (int L = 4; L < NL; ++L)
        if ((L & 3) == a) v -= cnt[L];
      // the type of each side towards the core sits in its own label
      const uint32_t t0 = lab.get((uint32_t)s0) & 3u;
      const uint32_t t1 = K == 5 ? lab.get((uint32_t)s1) & 3u : 0u;
      v -= (t0 == (uint32_t)a) + (K == 5 && t1 == (uint32_t)a);
      cnt[a] = v;
    }
    bar<GL>();
    closed_form<K, NL, BLOCK>(hist, lut, cnt, nzl, &nz_count, base);
    bar<GL>();
    if (threadIdx.x < NL) cnt[threadIdx.x] = 0;
  };

  for (;;) {
    if (threadIdx.x == 0) sh_j0 = atomicAdd(queue, tile);
    bar<GL>();
    const int32_t j0 = sh_j0;
    bar<GL>();
    if (j0 >= total) break;
    const int32_t j1 = min(total, j0 + tile);
    row = find_row(G.gs_off, 0, n, j0);
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
      } else {  // unit (b = c, a = x) with partners after x in c's row
        unit = j + 1 < rowb;
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
        for (int32_t jc = j + 1; jc < rowb; ++jc) {
          const uint32_t ec = G.gs_idx[jc];
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
        // skipped triples read x's labels without a barrier (see k5_kernel)
        bar<GL>();
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

// Hub slots for the core-reuse scheme: the vertices of largest degree get one
// of kMaxHubs rows of the per-core W table; the threshold is the smallest
// power of two whose degree bucket and all above hold at most kMaxHubs
// vertices (and at least 32).  hs[0..31] = counts per floor(log2 d),
// hs[32] = threshold, hs[33] = slot counter.  Which vertices get slots never
// changes the result, only where the work goes.
__global__ void k_degree_buckets(const int32_t* gs_off, int32_t n, int32_t* hs, const int32_t* st) {
  if (st[kStatus] != 0) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = gs_off[v + 1] - gs_off[v];
    if (d > 0) atomicAdd(&hs[31 - __clz(d)], 1);
  }
}

__global__ void k_hub_threshold(int32_t* hs, const int32_t* st) {
  if (st[kStatus] != 0 || threadIdx.x != 0) return;
  int32_t cum = 0, b = 31;
  while (b > 5 && cum + hs[b] <= kMaxHubs) cum += hs[b--];
  hs[32] = 1 << (b + 1);
  hs[33] = 0;
}

__global__ void k_assign_hubs(const int32_t* gs_off, int32_t n, int32_t* hs, int32_t* hub_id, const int32_t* st) {
  if (st[kStatus] != 0) return;
  const int32_t t = hs[32];
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = gs_off[v + 1] - gs_off[v];
    int32_t h = -1;
    if (d >= t) {
      h = atomicAdd(&hs[33], 1);
      if (h >= kMaxHubs) h = -1;
    }
    hub_id[v] = h;
  }
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
  return bytes <= 16384 ? 16384 : bytes <= 65536 ? 65536 : 0;
}
int64_t label_words(int k, int32_t n) { return k == 4 ? ((int64_t)n + 7) / 8 : ((int64_t)n + 3) / 4; }

int grid_size(int k, int num_cus) {
  const Tuning& t = tuning_for(k);
  return num_cus * t.grid_per_cu;
}

}  // namespace

size_t pipeline_bytes(int64_t N, int64_t M, int32_t G, bool batch, int k, int num_cus, int64_t maxn) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t b = build_bytes(N, M, G, batch);
  if ((k == 4 || k == 5) && tuning_for(k).heavy == 1)
    b += al(sizeof(int32_t) * (N + 1)) + al(64 * sizeof(int32_t)) +
         al(sizeof(uint32_t) * 16 * (size_t)(maxn > 0 ? maxn : N) * grid_size(k, num_cus));
  b += 2 * al(sizeof(uint64_t) * (size_t)G * num_classes(k));  // accumulators (+ output staging)
  b += al(64 * sizeof(int32_t));                               // queue counters
  const int cap = k == 4 ? label_cap_k4((int32_t)N) : k == 5 ? label_cap_k5((int32_t)N) : 1;
  if (cap == 0) b += al(sizeof(uint32_t) * (size_t)label_words(k, (int32_t)N) * grid_size(k, num_cus));
  return b + 4096;
}

#define LAUNCH_K4(BLOCK, CAP)                                                                                   \
  hipLaunchKernelGGL((k4_kernel<BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[4], acc, p.status, queue, \
                     glabels, lw, t.tile)
#define LAUNCH_KR(K, BLOCK, CAP)                                                                        \
  hipLaunchKernelGGL((kr_kernel<K, BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[K], acc, p.status, queue, \
                     glabels, lw, hub_id, wg, ws, t.tile)
#define LAUNCH_K5(BLOCK, CAP)                                                                                   \
  hipLaunchKernelGGL((k5_kernel<BLOCK, CAP>), dim3(grid), dim3(BLOCK), 0, s, g, T.lut[5], acc, p.status, queue, \
                     glabels, lw, t.tile)

void enqueue_census(Pipeline& p, const DevGraph& g, int k, uint64_t* acc, uint64_t* out, hipStream_t s) {
  const DevTables& T = dev_tables();
  const int C = num_classes(k);
  const int64_t total = (int64_t)g.ngraphs * C;
  enqueue_zero(acc, sizeof(uint64_t) * total, s);
  int32_t* queue = p.arena.take<int32_t>(64);
  enqueue_zero(queue, 64 * sizeof(int32_t), s);
  const Tuning& t = tuning_for(k);
  const int grid = grid_size(k, p.num_cus);
  profile_mark(k, 1, true, s);
  if (g.n > 0) {
    if (k == 3) {
      const int tv = t.tile > 0 ? t.tile * 16 : 256;
      hipLaunchKernelGGL((k3_kernel<256>), dim3(grid), dim3(256), 0, s, g, T.lut[3], acc, p.status, tv);
    } else {
      const bool reuse = t.heavy == 1;
      const int cap = k == 4 ? label_cap_k4(g.n) : label_cap_k5(g.n);
      const int64_t lw = label_words(k, g.n);
      uint32_t* glabels = nullptr;
      if (cap == 0) {
        glabels = p.arena.take<uint32_t>((size_t)lw * grid);
        enqueue_zero(glabels, sizeof(uint32_t) * (size_t)lw * grid, s);
      }
      int32_t* hub_id = nullptr;
      uint32_t* wg = nullptr;
      int64_t ws = 0;
      if (reuse) {
        ws = 16 * (int64_t)(g.max_graph_n > 0 ? g.max_graph_n : g.n);
        wg = p.arena.take<uint32_t>((size_t)ws * grid);
        enqueue_zero(wg, sizeof(uint32_t) * (size_t)ws * grid, s);
        hub_id = p.arena.take<int32_t>(g.n + 1);
        int32_t* hs = p.arena.take<int32_t>(64);
        enqueue_zero(hs, 64 * sizeof(int32_t), s);
        hipLaunchKernelGGL(k_degree_buckets, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.gs_off, g.n, hs, p.status);
        hipLaunchKernelGGL(k_hub_threshold, dim3(1), dim3(64), 0, s, hs, p.status);
        hipLaunchKernelGGL(k_assign_hubs, dim3(blocks_for(g.n, 256)), dim3(256), 0, s, g.gs_off, g.n, hs, hub_id,
                           p.status);
      }
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
          if (cap == 16384) LAUNCH_KR(5, 512, 16384); else if (cap == 65536) LAUNCH_KR(5, 512, 65536); else LAUNCH_KR(5, 512, 0);
        } else {
          if (cap == 16384) LAUNCH_KR(5, 1024, 16384); else if (cap == 65536) LAUNCH_KR(5, 1024, 65536); else LAUNCH_KR(5, 1024, 0);
        }
      } else {
        if (t.block == 512) {
          if (cap == 16384) LAUNCH_K5(512, 16384); else if (cap == 65536) LAUNCH_K5(512, 65536); else LAUNCH_K5(512, 0);
        } else {
          if (cap == 16384) LAUNCH_K5(1024, 16384); else if (cap == 65536) LAUNCH_K5(1024, 65536); else LAUNCH_K5(1024, 0);
        }
      }
    }
  }
  profile_mark(k, 1, false, s);
  hipLaunchKernelGGL(k_div_check, dim3(blocks_for(total, 256)), dim3(256), 0, s, acc, T.mult[k], C, total, p.status);
  hipLaunchKernelGGL(k_div_write, dim3(blocks_for(total, 256)), dim3(256), 0, s, acc, T.mult[k], C, total, out,
                     p.status);
}

}  // namespace motif
