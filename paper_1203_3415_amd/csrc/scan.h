// Device-side prefix sums shared by the build and the census set-up.
//
// k_scan1 is a single-pass exclusive scan with decoupled look-back (Merrill
// and Garland, "Single-pass Parallel Prefix Scan with Decoupled Look-back",
// NVIDIA technical report NVR-2016-002): every workgroup scans one tile,
// publishes the tile's sum at once, then its first wave reads the published
// words of the 64 preceding tiles at a time until it meets one that carries
// an inclusive prefix.  Tile numbers come from a ticket taken when the
// workgroup starts, so a tile only waits for tiles whose workgroups are
// already running, each of which publishes its sum before it waits itself.
// The values to scan come from a functor, so the kernel that used to write
// a flag array before a three-launch scan is folded into the scan.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace motif {

// Tiles of 4,096 values: 2 * 10^6 values are 489 tiles, so a tile reads at
// most eight windows of 64 published words.
constexpr int kScanBlock = 512;
constexpr int kScanItems1 = 8;
constexpr int kScanTile1 = kScanBlock * kScanItems1;

// Exclusive block scan of one value per thread (wave64 shuffles + LDS);
// sh holds blockDim.x / 64 ints.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (w == 0) {
    int32_t s = lane < nw ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int32_t y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < nw) sh[lane] = s;
  }
  __syncthreads();
  int32_t r = x - v + (w ? sh[w - 1] : 0);
  *total = sh[nw - 1];
  __syncthreads();
  return r;
}

// Look-back words: bits 32-33 = 1 (the tile's own sum) or 2 (the inclusive
// prefix through the tile), bits 0-31 = the value; 0 = not yet published.
constexpr uint64_t kScanAgg = uint64_t(1) << 32;
constexpr uint64_t kScanInc = uint64_t(2) << 32;

// Slot of element e of a tile in the LDS staging array: one pad word every
// 16 words, so that both the strided order (element i * kScanBlock + t read
// by thread t, coalesced in global memory) and the blocked order (elements
// t * kScanItems1 + i, what the running sums need) are free of bank
// conflicts.
__device__ __forceinline__ int scan1_slot(int e) { return e + (e >> 4); }
constexpr int kScanLds = kScanTile1 + kScanTile1 / 16;

// out[i] = f(0) + ... + f(i - 1) for i < len.  tiles (scan1_tiles(len)
// words) and *ticket must be zero at launch; grid = scan1_tiles(len).  The
// sums must fit in int32.  f is evaluated in the strided order, so that the
// loads it makes are coalesced, on indices clamped to len - 1 (the value
// there is discarded); f(len - 1) must be safe to call.  When st is given and
// its status word is set, the workgroups that see it scan zeros instead of
// calling f (f may read data that a failed earlier step left unwritten);
// every tile still publishes, so the look-back always ends.
//
// skip (optional): when *skip is 0 at launch the whole scan returns at once
// (the word is final before the launch, so every workgroup agrees).
template <class F>
__global__ __launch_bounds__(kScanBlock) void k_scan1(int32_t* out, int64_t len, F f, uint64_t* tiles,
                                                      uint32_t* ticket, const int32_t* st, const int32_t* skip) {
  __shared__ int32_t sh[kScanBlock / 64];
  __shared__ int32_t stage[kScanLds];
  __shared__ uint32_t tile_s;
  __shared__ int32_t excl_s;
  if (skip && *skip == 0) return;
  if (threadIdx.x == 0) tile_s = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint32_t tile = tile_s;
  const int64_t tbase = (int64_t)tile * kScanTile1;
  const int t = threadIdx.x;
  if (st == nullptr || st[kStatus] == 0) {
    int32_t w[kScanItems1];
#pragma unroll
    for (int i = 0; i < kScanItems1; ++i) {
      const int64_t e = tbase + (int64_t)i * kScanBlock + t;
      w[i] = f(e < len ? e : len - 1);
      if (e >= len) w[i] = 0;
    }
#pragma unroll
    for (int i = 0; i < kScanItems1; ++i) stage[scan1_slot(i * kScanBlock + t)] = w[i];
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems1; ++i) stage[scan1_slot(i * kScanBlock + t)] = 0;
  }
  __syncthreads();
  int32_t v[kScanItems1];
  int32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems1; ++i) {
    v[i] = stage[scan1_slot(t * kScanItems1 + i)];
    sum += v[i];
  }
  int32_t total;
  int32_t run = block_excl_scan(sum, sh, &total);
  if (t < 64) {
    const int lane = t;
    if (lane == 0)
      __hip_atomic_store(&tiles[tile], (tile == 0 ? kScanInc : kScanAgg) | (uint32_t)total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    int32_t excl = 0;
    if (tile > 0) {
      int64_t j = (int64_t)tile - 1;  // lane l reads tile j - l
      for (;;) {
        const int64_t idx = j - lane;
        const uint64_t w =
            idx >= 0 ? __hip_atomic_load(&tiles[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanInc;
        const uint32_t flag = (uint32_t)(w >> 32);
        const uint64_t inc = __ballot(flag == 2u);
        const uint64_t none = __ballot(flag == 0u);
        const int first = inc ? __ffsll((long long)inc) - 1 : 64;  // nearest tile with an inclusive prefix
        const uint64_t upto = first >= 63 ? ~uint64_t(0) : (uint64_t(2) << first) - 1;
        if (none & upto) continue;  // a nearer tile has not published yet
        int32_t x = lane <= first ? (int32_t)(uint32_t)w : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        excl += x;
        if (first < 64) break;
        j -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(&tiles[tile], kScanInc | (uint32_t)(excl + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) excl_s = excl;
  }
  __syncthreads();
  run += excl_s;
#pragma unroll
  for (int i = 0; i < kScanItems1; ++i) {
    stage[scan1_slot(t * kScanItems1 + i)] = run;
    run += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems1; ++i) {
    const int64_t e = tbase + (int64_t)i * kScanBlock + t;
    if (e < len) out[e] = stage[scan1_slot(i * kScanBlock + t)];
  }
}

inline int64_t scan1_tiles(int64_t len) { return len > 0 ? (len + kScanTile1 - 1) / kScanTile1 : 0; }

// Look-back words and ticket of one k_scan1 launch, taken from an arena and
// added to a zero batch that runs before the launch.
struct Scan1 {
  uint64_t* tiles = nullptr;  // scan1_tiles(len) words, then the ticket
  int64_t len = 0;
};

inline Scan1 scan1_take(Arena& A, int64_t len, ZeroBatch& z) {
  Scan1 sc;
  sc.len = len;
  const int64_t words = scan1_tiles(len) + 1;
  sc.tiles = A.take<uint64_t>((size_t)words);
  z.add(sc.tiles, sizeof(uint64_t) * (size_t)words);
  return sc;
}

inline size_t scan1_bytes(int64_t len) { return sizeof(uint64_t) * (size_t)(scan1_tiles(len) + 1) + 256; }

template <class F>
void enqueue_scan1(const Scan1& sc, int32_t* out, const F& f, const int32_t* st, hipStream_t s,
                   const int32_t* skip = nullptr) {
  if (sc.len <= 0) return;
  const int64_t nt = scan1_tiles(sc.len);
  hipLaunchKernelGGL((k_scan1<F>), dim3((unsigned)nt), dim3(kScanBlock), 0, s, out, sc.len, f, sc.tiles,
                     (uint32_t*)(sc.tiles + nt), st, skip);
}

}  // namespace motif
