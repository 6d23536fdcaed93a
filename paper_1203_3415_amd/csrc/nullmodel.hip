// Null-model ensembles on the device: degree-preserving arc-switch
// randomisation, the fused "randomise + census + z-scores" job, and the
// z-score kernel (the paper's step (iii), Section "Implementation", and its
// random-graph ensembles, Section "Results and Discussion").
//
// Arc switch: pick two arcs a->b and c->d; rewire them to a->d and c->b
// unless that makes a self-loop or an arc already present.  Out-degrees stay
// because every arc keeps its source (its slot in the out-CSR row); only the
// targets of two slots are exchanged, so in-degrees stay too.  Rows need not
// stay sorted (the census sorts them).
//
// One workgroup randomises one graph at a time.  When the graph fits, its
// offsets, targets and one lock word per row live in LDS for the whole run.
// Each round, every thread draws one proposal (two arc slots, from a
// counter-based generator, so the result is a function of the seed alone).
// A proposal first reserves the two source rows: atomicMin of the thread's
// index into each row's lock, so the lowest-numbered proposal on a row wins,
// whatever the timing.  A proposal that holds both rows checks the two rows
// (only it reads or writes them in this round) and swaps.  Which proposals
// run depends only on the proposals, not on the graph, and each executed
// switch is its own inverse, so every round is a symmetric move between
// graphs of the same degrees: the chain keeps the uniform distribution over
// them, as the one-switch-at-a-time chain does.  Every proposal counts as an
// attempt, whether it loses its reservation, is rejected or is executed.
//
// Mutual-preserving switch (optional): one-way arcs are exchanged only with
// one-way arcs and reciprocated pairs only with reciprocated pairs, so each
// vertex also keeps its numbers of reciprocated, one-way-out and one-way-in
// neighbours.  A one-way pair a->b, c->d becomes a->d, c->b; a reciprocated
// pair a<->b, c<->d becomes a<->d, c<->b.  Either is rejected if a and d, or
// c and b, are already joined in either direction (or on a self-loop or a
// repeated target).  Each slot's kind (bit 31 of its target while the kernel
// runs) never changes.  These switches also read (one-way) or write
// (reciprocated) the target rows b and d, so a proposal that holds its two
// source rows marks them as held and claims b and d (atomicMin of its index,
// among such proposals); it runs only if it wins both claims and neither b
// nor d is a row held by another proposal.  A proposal draws its first slot
// uniformly and its second uniformly among the slots of the same kind (from a
// list of the slots ordered by kind, fixed for the run), so each kind gets
// switches_per_arc attempts per arc whatever the reciprocity, and the
// proposals still do not depend on the current graph.  Everything that decides whether a
// proposal runs is the same before and after the round's switches (the
// reservations and so the held rows, the slots' kinds, and the set {b, d} of
// every proposal that holds its source rows), and the running proposals touch
// disjoint rows, so
// the round stays a symmetric move and the chain keeps the uniform
// distribution over the graphs with the same three degree sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.h"

namespace motif {

namespace {

constexpr int kSwB = kSwitchProposals;  // threads per workgroup = proposals per round
constexpr int kSwLds = 38 * 1024;       // LDS words for one graph: n + 1 offsets, m targets, n locks
constexpr int kSwPerCu = 2;             // switch workgroups per CU when their graphs fit in half the LDS
constexpr uint32_t kFree = 0xFFFFFFFFu;
// lock word index | kHeld: the row's winning proposal holds both its rows
// (indices are below 1024; a free word has both top bits set)
constexpr uint32_t kHeld = 0x40000000u, kHeldMask = 0xC0000000u;

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) used as a counter-based generator: output i of
// stream `key` is the finaliser applied to key + (i + 1) * gamma.
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Row (source vertex) of arc slot i: the last v with off[v] <= i.
__device__ __forceinline__ int32_t row_of(const int32_t* off, int32_t n, int32_t i) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Does row [p, pe) of idx hold x?  Eight loads per step, issued together, so a
// long (hub) row is not a chain of dependent loads.
// Targets are compared without bit 31 (the slot kind of the mutual-preserving
// switch).
constexpr int32_t kTarget = 0x7FFFFFFF;
constexpr int32_t kMutualBit = (int32_t)0x80000000u;
__device__ __forceinline__ bool row_has(const int32_t* idx, int32_t p, int32_t pe, int32_t x) {
  bool hit = false;
  for (; p + 8 <= pe && !hit; p += 8) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = idx[p + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) hit |= (v[u] & kTarget) == x;
  }
  for (; p < pe && !hit; ++p) hit = (idx[p] & kTarget) == x;
  return hit;
}

// Position of target x in row [p, pe) (present by construction).
__device__ __forceinline__ int32_t row_find(const int32_t* idx, int32_t p, int32_t pe, int32_t x) {
  while (p < pe - 1 && (idx[p] & kTarget) != x) ++p;
  return p;
}

// Lock words: in LDS plain accesses; in global memory device-scope atomics,
// which are performed in L2 (the per-CU L1 does not see them).
template <bool LDS>
__device__ __forceinline__ void lock_min(uint32_t* w, uint32_t v) {
  if constexpr (LDS) atomicMin(w, v);
  else __hip_atomic_fetch_min(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ uint32_t lock_get(uint32_t* w) {
  if constexpr (LDS) return *w;
  else return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ void lock_set(uint32_t* w, uint32_t v) {
  if constexpr (LDS) *w = v;
  else __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__device__ __forceinline__ void sw_barrier() {
  if constexpr (!LDS) __builtin_amdgcn_s_waitcnt(0);  // global atomics and stores of this wave done
  __syncthreads();
}

// Randomise the graphs list[0..count) of gs, one workgroup per graph.  LDS:
// the graph is held in LDS ((n + 1) + m + n words, + n target claims when
// MUT), kSwLds / PER_CU words: with PER_CU = 2 two workgroups share a CU
// (a round is a short chain of LDS reads between barriers, and a second
// workgroup fills the gaps), for lists whose graphs all fit in half.  When
// the words left over hold a 16-bit source row per arc slot (n <= 65,536),
// the rows of a round's two slots are read from that table instead of a
// binary search of the offsets (a switch moves targets, never slots).
// Otherwise it is switched in place in global memory with this
// workgroup's lock slice glock + blockIdx.x * lock_stride (lock_stride >= n,
// or 2n when MUT, of every listed graph).  MUT: the slots ordered by kind go
// to gperm + blockIdx.x * perm_stride (perm_stride >= m of every listed graph).
// (the second launch bound is in waves per SIMD: PER_CU workgroups of
// kSwB / 64 waves over the CU's four SIMDs)
template <bool LDS, bool MUT, int PER_CU>
__global__ __launch_bounds__(kSwB, PER_CU * kSwB / 256) void k_switch(const SwitchGraph* __restrict__ gs,
                                                           const int32_t* __restrict__ list, int32_t count,
                                                           uint32_t* __restrict__ glock, int64_t lock_stride,
                                                           int32_t* __restrict__ gperm, int64_t perm_stride,
                                                           const int32_t* st) {
  __shared__ int32_t lds[LDS ? kSwLds / PER_CU : 1];
  __shared__ int32_t wsum[2][kSwB / 64];
  if (st[kStatus] != 0) return;
  const uint32_t tid = threadIdx.x;
  for (int32_t q = blockIdx.x; q < count; q += gridDim.x) {
    const SwitchGraph G = gs[list[q]];
    const int32_t n = G.n, m = G.m;
    if (m < 2 || n < 2) continue;  // nothing to switch (uniform over the workgroup)
    const int32_t* off;
    int32_t* idx;
    uint32_t* lock;
    uint32_t* claim = nullptr;  // MUT: target-row claims
    if constexpr (LDS) {
      int32_t* loff = lds;
      int32_t* lidx = lds + (n + 1);
      uint32_t* llock = reinterpret_cast<uint32_t*>(lidx + m);
      for (int32_t i = tid; i <= n; i += kSwB) loff[i] = G.off[i];
      for (int32_t i = tid; i < m; i += kSwB) lidx[i] = G.idx[i];
      for (int32_t i = tid; i < (MUT ? 2 * n : n); i += kSwB) llock[i] = kFree;
      off = loff;
      idx = lidx;
      lock = llock;
      if constexpr (MUT) claim = llock + n;
    } else {
      off = G.off;
      idx = G.idx;
      lock = glock + (int64_t)blockIdx.x * lock_stride;
      for (int32_t i = tid; i < (MUT ? 2 * n : n); i += kSwB) lock_set<LDS>(&lock[i], kFree);
      if constexpr (MUT) claim = lock + n;
    }
    sw_barrier<LDS>();
    const uint16_t* srow = nullptr;  // source row of each slot, when it fits (uniform per graph)
    if constexpr (LDS) {
      const int64_t used = (int64_t)(n + 1) + m + (MUT ? 2 : 1) * (int64_t)n;
      if (n <= 65536 && used + (m + 1) / 2 <= kSwLds / PER_CU) {
        uint16_t* s16 = reinterpret_cast<uint16_t*>(lds + used);
        for (int32_t i = tid; i < m; i += kSwB) s16[i] = (uint16_t)row_of(off, n, i);
        srow = s16;
        sw_barrier<LDS>();
      }
    }
    auto slot_row = [&](int32_t i) { return srow ? (int32_t)srow[i] : row_of(off, n, i); };
    int32_t* perm = nullptr;  // MUT: slot indices, reciprocated first, each kind in slot order
    int32_t nmut = 0;         // MUT: reciprocated slots
    if constexpr (MUT) {
      // slot kinds: bit 31 set on a->b when b->a exists (each slot is
      // written by one thread; readers compare without bit 31)
      const int32_t lane = (int32_t)(tid & 63u), wv = (int32_t)(tid >> 6);
      int32_t mine = 0;
      for (int32_t i = tid; i < m; i += kSwB) {
        const int32_t a = slot_row(i), b = idx[i] & kTarget;
        if (row_has(idx, off[b], off[b + 1], a)) {
          idx[i] |= kMutualBit;
          ++mine;
        }
      }
      for (int o = 32; o; o >>= 1) mine += __shfl_xor(mine, o);
      if (lane == 0) wsum[0][wv] = mine;
      sw_barrier<LDS>();
      for (int w = 0; w < kSwB / 64; ++w) nmut += wsum[0][w];
      // stable partition of the slots by kind, kSwB slots at a time
      perm = gperm + (int64_t)blockIdx.x * perm_stride;
      const uint64_t below = (1ull << lane) - 1ull;
      int32_t next_m = 0, next_s = nmut;
      for (int32_t c0 = 0; c0 < m; c0 += kSwB) {
        const int32_t i = c0 + (int32_t)tid;
        const bool live = i < m, f = live && (idx[i] & kMutualBit);
        const uint64_t bm = __ballot(f), bl = __ballot(live);
        sw_barrier<LDS>();  // the previous chunk's counts have been read
        if (lane == 0) {
          wsum[0][wv] = __popcll(bm);
          wsum[1][wv] = __popcll(bl);
        }
        sw_barrier<LDS>();
        int32_t om = 0, ol = 0, tm = 0, tl = 0;
        for (int w = 0; w < kSwB / 64; ++w) {
          if (w < wv) {
            om += wsum[0][w];
            ol += wsum[1][w];
          }
          tm += wsum[0][w];
          tl += wsum[1][w];
        }
        if (live) {
          const int32_t rm = om + __popcll(bm & below), rl = ol + __popcll(bl & below);
          perm[f ? next_m + rm : next_s + (rl - rm)] = i;
        }
        next_m += tm;
        next_s += tl - tm;
      }
      // the list was written to global memory by other threads of this
      // workgroup: wait for the stores, then drop stale L1 lines
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // Round-tagged reservations (one-way switches in LDS): a reservation
    // word holds (round + 1) << 11 | (2047 - index) and is raised with
    // atomicMax, so within a round the largest word is the lowest proposal
    // index, the winner atomicMin gives on cleared words, and words of
    // earlier rounds never win.  Two sets are used on alternate rounds: a
    // set is raised again only two rounds later, after a barrier that every
    // reader of its earlier round has passed, so nothing is cleared and a
    // round needs one barrier instead of three.  The switches are the same.
    // Taken when n more words fit beside the source rows and the tags stay
    // below 2^31.
    uint32_t* lock2 = nullptr;
    if constexpr (LDS && !MUT) {
      const int64_t used = (int64_t)(n + 1) + m + n + (m + 1) / 2;
      if (srow && used + n <= kSwLds / PER_CU && G.rounds < (int64_t(1) << 20)) {
        lock2 = reinterpret_cast<uint32_t*>(lds + used);
        for (int32_t i = tid; i < n; i += kSwB) {
          lock[i] = 0u;
          lock2[i] = 0u;
        }
        sw_barrier<LDS>();
      }
    }
    if (lock2) {
      for (int64_t r = 0; r < G.rounds; ++r) {
        const uint64_t x = sm64_mix(G.key + (uint64_t)(r * kSwB + tid + 1) * kGamma);
        const int32_t i = (int32_t)(((x & 0xFFFFFFFFull) * (uint64_t)m) >> 32);
        const int32_t j = (int32_t)(((x >> 32) * (uint64_t)m) >> 32);
        const int32_t a = slot_row(i), c = slot_row(j);
        const bool cand = a != c;
        uint32_t* L = (r & 1) ? lock2 : lock;
        const uint32_t v = ((uint32_t)(r + 1) << 11) | (2047u - tid);
        if (cand) {
          atomicMax(&L[a], v);
          atomicMax(&L[c], v);
        }
        sw_barrier<LDS>();
        if (cand && L[a] == v && L[c] == v) {
          const int32_t b = idx[i], d = idx[j];
          const bool ok = a != d && c != b && b != d && !row_has(idx, off[a], off[a + 1], d) &&
                          !row_has(idx, off[c], off[c + 1], b);
          if (ok) {
            idx[i] = d;
            idx[j] = b;
          }
        }
      }
      sw_barrier<LDS>();  // the last round's switches before the write-back
    } else {
      for (int64_t r = 0; r < G.rounds; ++r) {
        const uint64_t x = sm64_mix(G.key + (uint64_t)(r * kSwB + tid + 1) * kGamma);
        int32_t i = (int32_t)(((x & 0xFFFFFFFFull) * (uint64_t)m) >> 32);
        int32_t j = (int32_t)(((x >> 32) * (uint64_t)m) >> 32);
        if constexpr (MUT) {  // first slot uniform, second uniform among the slots of its kind
          const bool km = i < nmut;
          const int32_t lo = km ? 0 : nmut, nk = km ? nmut : m - nmut;
          j = perm[lo + (int32_t)(((x >> 32) * (uint64_t)nk) >> 32)];
          i = perm[i];
        }
        const int32_t a = slot_row(i), c = slot_row(j);
        const bool cand = a != c;  // two arcs of one row: the switch changes nothing
        if (cand) {
          lock_min<LDS>(&lock[a], tid);
          lock_min<LDS>(&lock[c], tid);
        }
        sw_barrier<LDS>();
        if constexpr (!MUT) {
          if (cand && lock_get<LDS>(&lock[a]) == tid && lock_get<LDS>(&lock[c]) == tid) {
            // rows a and c are this proposal's alone until the next barrier
            const int32_t b = idx[i], d = idx[j];
            const bool ok = a != d && c != b && b != d && !row_has(idx, off[a], off[a + 1], d) &&
                            !row_has(idx, off[c], off[c + 1], b);
            if (ok) {
              idx[i] = d;
              idx[j] = b;
            }
          }
          sw_barrier<LDS>();
          if (cand) {
            lock_set<LDS>(&lock[a], kFree);
            lock_set<LDS>(&lock[c], kFree);
          }
        } else {
          // holds both source rows (then marked as held) and the two slots are of one kind
          int32_t wi = 0, wj = 0;
          bool held = cand && lock_get<LDS>(&lock[a]) == tid && lock_get<LDS>(&lock[c]) == tid;
          if (held) {
            lock_set<LDS>(&lock[a], tid | kHeld);
            lock_set<LDS>(&lock[c], tid | kHeld);
            wi = idx[i];
            wj = idx[j];
            held = (wi & kMutualBit) == (wj & kMutualBit);
          }
          const int32_t b = wi & kTarget, d = wj & kTarget;
          if (held) {
            lock_min<LDS>(&claim[b], tid);
            lock_min<LDS>(&claim[d], tid);
          }
          sw_barrier<LDS>();
          auto held_by_other = [&](int32_t row) {
            return row != a && row != c && (lock_get<LDS>(&lock[row]) & kHeldMask) == kHeld;
          };
          if (held && lock_get<LDS>(&claim[b]) == tid && lock_get<LDS>(&claim[d]) == tid && !held_by_other(b) &&
              !held_by_other(d)) {
            // rows a, b, c and d are this proposal's alone until the next barrier
            const bool ok = a != d && c != b && b != d && !row_has(idx, off[a], off[a + 1], d) &&
                            !row_has(idx, off[d], off[d + 1], a) && !row_has(idx, off[c], off[c + 1], b) &&
                            !row_has(idx, off[b], off[b + 1], c);
            if (ok) {
              const int32_t kind = wi & kMutualBit;
              idx[i] = d | kind;
              idx[j] = b | kind;
              if (kind) {  // the reverse arcs: b->a becomes b->c, d->c becomes d->a
                idx[row_find(idx, off[b], off[b + 1], a)] = c | kind;
                idx[row_find(idx, off[d], off[d + 1], c)] = a | kind;
              }
            }
          }
          sw_barrier<LDS>();
          if (cand) {
            lock_set<LDS>(&lock[a], kFree);
            lock_set<LDS>(&lock[c], kFree);
          }
          if (held) {
            lock_set<LDS>(&claim[b], kFree);
            lock_set<LDS>(&claim[d], kFree);
          }
        }
        sw_barrier<LDS>();
      }
    }
    if constexpr (LDS) {
      for (int32_t i = tid; i < m; i += kSwB) G.idx[i] = idx[i] & kTarget;
    } else if constexpr (MUT) {
      for (int32_t i = tid; i < m; i += kSwB) idx[i] &= kTarget;
    }
    sw_barrier<LDS>();
  }
}

// Every listed graph before it is switched.  Pass 0: offsets monotone from
// 0 to m (the kernel reads the rows they delimit).  Pass 1, run only when
// every graph passed pass 0: targets in [0, n) (the mutual-preserving switch
// reads the rows they name) and no self-loops.  Graph q = blockIdx.y +
// t gridDim.y; rows spread over x.
__global__ void k_check_graphs(const SwitchGraph* __restrict__ gs, int32_t count, int32_t pass, int32_t* st) {
  if (pass == 1 && st[kStatus] != 0) return;
  for (int32_t q = blockIdx.y; q < count; q += gridDim.y) {
    const SwitchGraph G = gs[q];
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= G.n; v += (int64_t)gridDim.x * blockDim.x) {
      if (pass == 0) {
        const int32_t a = G.off[v];
        if ((v == 0 && a != 0) || (v == G.n && a != G.m) || (v < G.n && G.off[v + 1] < a))
          atomicMin(&st[kStatus], MOTIF_EINVAL_SHAPE);
      } else if (v < G.n) {
        for (int32_t i = G.off[v], e = G.off[v + 1]; i < e; ++i) {
          const int32_t t = G.idx[i];
          if (t < 0 || t >= G.n) atomicMin(&st[kStatus], MOTIF_EINDEX);
          else if (t == (int32_t)v) atomicMin(&st[kStatus], MOTIF_ESELFLOOP);
        }
      }
    }
  }
}

// Offsets of a graph whose rows will be switched: monotone, from 0 to m (the
// switch kernel reads the rows they delimit).
__global__ void k_check_rows(const int32_t* off, int32_t n, int64_t m, int32_t* st) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = off[v];
    const bool bad = (v == 0 && a != 0) || (v == n && (int64_t)a != m) || (v < n && off[v + 1] < a);
    if (bad) atomicMin(&st[kStatus], MOTIF_EINVAL_SHAPE);
  }
}

// dst[g * m + i] = src[i] for g < copies.
__global__ void k_replicate(const int32_t* __restrict__ src, int64_t m, int32_t copies, int32_t* __restrict__ dst,
                            const int32_t* st) {
  if (st[kStatus] != 0) return;
  const int64_t total = m * copies;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t % m];
}

// Unsigned 128-bit integers from 64-bit halves (exact sums of counts and of
// their squares).
struct U128 {
  uint64_t lo = 0, hi = 0;
};
__device__ __forceinline__ U128 add(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
  return r;
}
__device__ __forceinline__ U128 mul64(uint64_t a, uint64_t b) {
  U128 r;
  r.lo = a * b;
  r.hi = __umul64hi(a, b);
  return r;
}
// a * b for a < 2^64 and b < 2^128, assuming the product is below 2^128.
__device__ __forceinline__ U128 mul(uint64_t a, U128 b) {
  U128 r = mul64(a, b.lo);
  r.hi += a * b.hi;
  return r;
}
__device__ __forceinline__ bool less(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ U128 sub(U128 a, U128 b) {  // a >= b
  U128 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
  return r;
}
__device__ __forceinline__ double to_double(U128 a) { return (double)a.hi * 18446744073709551616.0 + (double)a.lo; }

// z_c = (h_real,c - mean_c) / sd_c over the `count` randomised graphs, sample
// standard deviation (ddof = 1), from exact integer sums:
//   S1 = sum h, S2 = sum h^2, var_num = N S2 - S1^2 = N (N - 1) var,
//   z = (N h_real - S1) / N / sqrt(var_num / (N (N - 1))).
// NaN where N < 2, var = 0, or a count of the class reaches 2^40 (its sums
// would then need more than 128 bits for N up to 2^16 graphs).
__global__ void k_zscores(const uint64_t* __restrict__ hists, int32_t C, int32_t count, double* __restrict__ z,
                          const int32_t* st) {
  if (st[kStatus] != 0) return;
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint64_t real = hists[c];
  const uint64_t N = (uint64_t)count;
  bool exact = N >= 2 && N <= 65536 && real < (1ull << 40);
  U128 s1, s2;
  for (int32_t g = 1; g <= count; ++g) {
    const uint64_t h = hists[(int64_t)g * C + c];
    exact = exact && h < (1ull << 40);
    s1 = add(s1, U128{h, 0});
    s2 = add(s2, mul64(h, h));
  }
  double out = __builtin_nan("");
  if (exact) {
    const U128 a = mul(N, s2);
    const U128 b = mul(s1.lo, s1);  // s1 < 2^56: one 64-bit half
    if (less(b, a)) {
      const double var = to_double(sub(a, b)) / ((double)N * (double)(N - 1));
      const U128 nr = mul64(N, real);
      const double num = less(nr, s1) ? -to_double(sub(s1, nr)) : to_double(sub(nr, s1));
      out = num / (double)N / sqrt(var);
    }
  }
  z[c] = out;
}

unsigned blocks(int64_t items, int b) {
  const int64_t g = (items + b - 1) / b;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, g));
}

}  // namespace

int32_t enqueue_switch(Pipeline& p, const SwitchGraph* host_graphs, int32_t count, bool mutual, hipStream_t s) {
  // three lists: graphs that fit in half the LDS array (two workgroups per
  // CU), graphs that need all of it (one per CU), graphs switched in global
  // memory; each list largest graph first, so that the graphs taken last by
  // the persistent workgroups are the short ones
  auto words = [&](const SwitchGraph& G) { return (int64_t)(G.n + 1) + G.m + (mutual ? 2 : 1) * (int64_t)G.n; };
  std::vector<int32_t> half_list, full_list, glob_list;
  int64_t max_glob_n = 0;
  for (int32_t g = 0; g < count; ++g) {
    const SwitchGraph& G = host_graphs[g];
    const int64_t w = words(G);
    if (w <= kSwLds / kSwPerCu) {
      half_list.push_back(g);
    } else if (w <= kSwLds) {
      full_list.push_back(g);
    } else {
      glob_list.push_back(g);
      max_glob_n = std::max<int64_t>(max_glob_n, G.n);
    }
  }
  auto larger_first = [&](int32_t a, int32_t b) { return host_graphs[a].m > host_graphs[b].m; };
  std::stable_sort(half_list.begin(), half_list.end(), larger_first);
  std::stable_sort(full_list.begin(), full_list.end(), larger_first);
  std::stable_sort(glob_list.begin(), glob_list.end(), larger_first);
  SwitchGraph* dg = p.arena.take<SwitchGraph>(std::max(count, 1));
  int32_t* dl = p.arena.take<int32_t>(std::max(count, 1));
  if (hipMemcpyAsync(dg, host_graphs, sizeof(SwitchGraph) * count, hipMemcpyHostToDevice, s) != hipSuccess)
    return MOTIF_EDEVICE;
  std::vector<int32_t> lists(full_list);
  lists.insert(lists.end(), half_list.begin(), half_list.end());
  lists.insert(lists.end(), glob_list.begin(), glob_list.end());
  if (!lists.empty() &&
      hipMemcpyAsync(dl, lists.data(), sizeof(int32_t) * lists.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return MOTIF_EDEVICE;
  // the copies above read pageable host memory: wait before it goes out of scope
  if (hipStreamSynchronize(s) != hipSuccess) return MOTIF_EDEVICE;
  int64_t max_n = 0;
  for (int32_t g = 0; g < count; ++g) max_n = std::max<int64_t>(max_n, host_graphs[g].n);
  if (count > 0) {
    const dim3 cg((unsigned)std::min<int64_t>(64, (max_n + 256) / 256), (unsigned)std::min(count, 4096));
    for (int32_t pass = 0; pass < 2; ++pass)
      hipLaunchKernelGGL(k_check_graphs, cg, dim3(256), 0, s, dg, count, pass, p.status);
  }
  const int grid = std::max(1, p.num_cus);
  const int grid_full = (int)std::min<int64_t>(grid, (int64_t)full_list.size());
  const int grid_half = (int)std::min<int64_t>((int64_t)grid * kSwPerCu, (int64_t)half_list.size());
  // MUT: one slot list per workgroup (the launches run one after the other)
  int64_t max_m = 1;
  for (int32_t g = 0; g < count; ++g) max_m = std::max<int64_t>(max_m, host_graphs[g].m);
  int32_t* perm =
      mutual ? p.arena.take<int32_t>((size_t)std::max(grid, grid_half) * (size_t)max_m) : nullptr;
  if (!full_list.empty()) {
    const int32_t nl = (int32_t)full_list.size();
    if (mutual)
      hipLaunchKernelGGL((k_switch<true, true, 1>), dim3(grid_full), dim3(kSwB), 0, s, dg, dl, nl, nullptr, 0, perm,
                         max_m, p.status);
    else
      hipLaunchKernelGGL((k_switch<true, false, 1>), dim3(grid_full), dim3(kSwB), 0, s, dg, dl, nl, nullptr, 0,
                         nullptr, 0, p.status);
  }
  if (!half_list.empty()) {
    const int32_t nl = (int32_t)half_list.size();
    const int32_t* hl = dl + full_list.size();
    if (mutual)
      hipLaunchKernelGGL((k_switch<true, true, kSwPerCu>), dim3(grid_half), dim3(kSwB), 0, s, dg, hl, nl, nullptr, 0,
                         perm, max_m, p.status);
    else
      hipLaunchKernelGGL((k_switch<true, false, kSwPerCu>), dim3(grid_half), dim3(kSwB), 0, s, dg, hl, nl, nullptr,
                         0, nullptr, 0, p.status);
  }
  if (!glob_list.empty()) {
    const int gw = (int)std::min<int64_t>(grid, (int64_t)glob_list.size());
    const int64_t stride = (mutual ? 2 : 1) * max_glob_n;
    uint32_t* locks = p.arena.take<uint32_t>((size_t)gw * (size_t)stride);
    const int32_t* gl = dl + full_list.size() + half_list.size();
    if (mutual)
      hipLaunchKernelGGL((k_switch<false, true, 1>), dim3(gw), dim3(kSwB), 0, s, dg, gl, (int32_t)glob_list.size(),
                         locks, stride, perm, max_m, p.status);
    else
      hipLaunchKernelGGL((k_switch<false, false, 1>), dim3(gw), dim3(kSwB), 0, s, dg, gl, (int32_t)glob_list.size(),
                         locks, stride, nullptr, 0, p.status);
  }
  return 0;
}

size_t switch_bytes(int32_t count, int64_t max_n, int64_t max_m, int num_cus) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  // lock slices and slot lists sized for the mutual-preserving switch (two
  // words per vertex, one per arc)
  const size_t wg = (size_t)std::max(1, num_cus);
  return al(sizeof(SwitchGraph) * std::max(count, 1)) + al(sizeof(int32_t) * std::max(count, 1)) +
         al(2 * sizeof(uint32_t) * wg * (size_t)std::max<int64_t>(max_n, 1)) +
         al(sizeof(int32_t) * wg * kSwPerCu * (size_t)std::max<int64_t>(max_m, 1));
}

uint64_t switch_key(uint64_t seed, int64_t graph) { return sm64_mix(seed + (uint64_t)(graph + 1) * kGamma); }

void enqueue_check_rows(const int32_t* off, int32_t n, int64_t m, int32_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_check_rows, dim3(blocks(n + 1, 256)), dim3(256), 0, s, off, n, m, st);
}

void enqueue_replicate(const int32_t* src, int64_t m, int32_t copies, int32_t* dst, const int32_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_replicate, dim3(blocks(m * copies, 256)), dim3(256), 0, s, src, m, copies, dst, st);
}

void enqueue_zscores(const uint64_t* hists, int32_t C, int32_t count, double* z, const int32_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_zscores, dim3(blocks(C, 256)), dim3(256), 0, s, hists, C, count, z, st);
}

}  // namespace motif
