// Internal declarations shared by the host orchestration (api.cpp, server.cpp)
// and the device code (graph.hip, census.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <vector>

#include "../../include/motif.h"

namespace motif {

// G* entry: neighbour id in bits 0..29, type in bits 30..31 relative to the
// row vertex r: 1 = B (arc r->x only), 2 = C (arc x->r only), 3 = A (both),
// the partition A^v / B^v / C^v of Section "Notation and definitions".
constexpr uint32_t kIdMask = 0x3FFFFFFFu;
constexpr int kTypeShift = 30;
constexpr int32_t kMaxN = 1 << 30;

// Device status word slots.
enum StatusSlot : int {
  kStatus = 0,       // 0 or a MOTIF_E* code (the most negative one wins)
  kMidCount = 1,     // number of mid-size segments queued for sorting
  kBigCount = 2,     // number of big segments queued for sorting
  kQueue = 3,        // anchor work-queue cursor
  kQueue2 = 4,       // second work-queue cursor
  kUnsorted = 5,     // build from an in-CSR: 1 when a row is not strictly increasing
  kInMismatch = 6,   // build from an in-CSR: 1 when an in-arc was not found among the out-arcs
  kStatusWords = 16,
};

// Built undirected typed graph (possibly the disjoint union of a batch).
struct DevGraph {
  int32_t n = 0;
  const int32_t* gs_off = nullptr;  // [n+1]
  const uint32_t* gs_idx = nullptr; // [2m*] sorted by id per row, typed
  const int32_t* np_off = nullptr;  // [n+1]
  const uint32_t* np_idx = nullptr; // [m*]  N+(v): neighbours of higher rank
  const int32_t* gid = nullptr;     // [n] graph of each vertex (batch) or null
  const int64_t* voff = nullptr;    // [ngraphs+1] first vertex of each graph (batch) or null
  int32_t ngraphs = 1;
  int32_t max_graph_n = 0;          // largest vertex count of one graph
  const int32_t* gs_row = nullptr;  // [2m*] row (vertex) of each G* entry
  int64_t gs_cap = 0;               // 2m + 1 >= entries of G* + 1
};

// Device class tables uploaded by motif_init.
struct DevTables {
  const uint16_t* lut[6] = {};   // index k
  const uint8_t* mult[6] = {};
  const int16_t* und_of[6] = {};  // undirected class of each directed class, -1 if an arc is one-way
};
const DevTables& dev_tables();

// Thrown by Arena::take when a workspace was sized too small; the entry
// points turn it into MOTIF_EINTERNAL after draining what was enqueued.
struct WorkspaceError : std::runtime_error {
  WorkspaceError() : std::runtime_error("motif: workspace sizing error") {}
};

// Grow-only device arena with a bump allocator.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  void reset() { used = 0; }
  // Regions taken after a mark can be given back once the kernels that use
  // them are enqueued: later work on the same stream runs after them.
  size_t mark() const { return used; }
  void rewind(size_t m) { used = m; }
  // Every region is carved before the kernels that use it are launched, so an
  // undersized arena is caught before any kernel could write past it: the
  // call throws WorkspaceError, and kernels already enqueued only touch
  // regions taken before it.
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used + bytes > cap) throw WorkspaceError();
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// Launch parameters used by the census kernels.
struct Tuning {
  int block = 256;
  int grid_per_cu = 4;
  int tile = 16;
  int heavy = 1;  // census scheme for k = 4, 5: 1 = core reuse, 0 = per-anchor scan
  // Work-placement limits of the core-reuse kernels (degrees in G*):
  int solo_deg = 64;    // k = 4: cores of at most this degree run whole anchors on one wave (<= 64)
  int light_deg = 192;  // k = 4: sides of at most this degree run on one wave (<= 256)
  int light5 = 512;     // k = 5: lighter sides of at most this degree take the factored path (<= 767)
};
// The tuning of every k, copied once per call so that a concurrent
// motif_set_tuning() or autotune never changes a call between the sizing of
// its workspace and its launches.
struct TuningSet {
  Tuning k[6];
};
TuningSet tuning_snapshot();
// The tuning a call uses on device `dev`: the defaults (for a batch whose
// graphs have at most max_n >= 0 vertices, the small-graph batch default of
// k = 4 where it applies), with the autotuner's cached entry for (k, batch,
// floor(log2 arcs)) in place of k's when there is one, for each of ks[0..nk).
TuningSet tuning_for_call(int dev, int32_t nk, const int32_t* ks, bool batch, int64_t arcs, int64_t max_n = -1);

// Buffers of one census pipeline (one stream).
struct Pipeline {
  Arena arena;
  int32_t* status = nullptr;       // device [kStatusWords]
  int32_t* host_status = nullptr;  // pinned host copy
  int num_cus = 0;
  // second stream for the smaller sizes of a multi-size census, forked after
  // the shared build and joined before the status is read (default priority)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_pre = nullptr;  // the largest census's big-core tables are clear (cleared on `side`)
  TuningSet tune;  // the tuning this call was sized with (set before any enqueue)
  // Per-workgroup W rows of the k = 4, 5 core-reuse kernels for the census
  // on this pipeline's own stream: zeroed once when allocated, and left zero
  // by every census (each core's tear-down clears the rows it touched), so
  // no call has to clear them.  Null where the W rows come from the arena.
  uint32_t* wpool = nullptr;
  size_t wpool_bytes = 0;
  // k = 6 census buffers (class sums, label slices, anchor list), grown on
  // demand and kept for the next call on this stream
  uint8_t* k6_buf = nullptr;
  size_t k6_bytes = 0;
};

// The class table of size k (len = 2^(k(k-1)) entries, indexed by row-major
// adjacency codes) rewritten in the code order the census kernels use.
std::vector<uint16_t> device_lut_order(int k, const uint16_t* lut, size_t len);

// Bytes the arena needs for a union graph of N vertices, M arcs, G graphs
// (G > 1 includes the packing buffers of a batch) under tuning t.
size_t pipeline_bytes(int64_t N, int64_t M, int32_t G, bool batch, int k, int num_cus, int64_t maxn,
                      const Tuning& t);
size_t build_bytes(int64_t N, int64_t M, int32_t G, bool batch);

// Inputs of the build: either one graph or a packed batch.
struct BuildInput {
  const int32_t* out_off;
  const int32_t* out_idx;
  const int32_t* in_off;  // may be null
  const int32_t* in_idx;  // may be null
  int32_t n;
  int64_t m;
  const int32_t* gid = nullptr;     // batch only
  int32_t ngraphs = 1;
  const int32_t* has_in = nullptr;  // batch only: graph supplied an in-CSR
  const int64_t* voff = nullptr;    // batch only: first vertex of each graph (device)
  int32_t max_graph_n = 0;          // largest vertex count of one graph
  bool copy_error = false;          // a host-to-device copy could not be enqueued
};

// Enqueue validation + G* + N+ build, then the in-CSR check when an in-CSR
// is given.  Returns the built view (device pointers into the arena).  Does
// not wait.  graph_ready (optional): recorded on s once G* and N+ are
// written, before the in-CSR check (*ready_ok: whether the record
// succeeded).  deferred (optional): the in-CSR check is not enqueued; what it
// needs is returned there for enqueue_check_in on another stream.
struct InCheck {
  const int32_t* in_cnt = nullptr;  // in-degrees counted from the out-CSR (batch builds)
  uint32_t* marks = nullptr;        // one bit per G* entry
  bool offsets_checked = false;     // the build already checked the in-CSR offsets
};
DevGraph enqueue_build(Pipeline& p, const BuildInput& in, hipStream_t s, hipEvent_t graph_ready = nullptr,
                       bool* ready_ok = nullptr, InCheck* deferred = nullptr);
// The in-CSR check of a build (nothing when no in-CSR was given); its outcome
// lands in the status word.  background: a bounded grid, for a stream that
// runs beside a census.
void enqueue_check_in(const BuildInput& in, const DevGraph& g, const InCheck& c, int32_t* status, hipStream_t s,
                      bool background);

// Enqueue the census of k into acc[ngraphs * C] (accumulators, zeroed here)
// and, unless out is null, the exact division into out[ngraphs * C] (written
// only if every remainder is zero).  use_wpool: the W rows may come from
// p.wpool (only for work on the pipeline's own stream, one census at a time).
struct ZeroBatch;

// Big-core tables of a k = 4, 5 core-reuse census (nbig = 0: none).
struct BigTables {
  int nbig = 0;
  int32_t* big_id = nullptr;    // [n + 1]
  int32_t* big_list = nullptr;  // [kMaxBig]
  uint32_t* lbig = nullptr;     // labels, zeroed
  uint32_t* wbig = nullptr;     // W rows, zeroed
  uint32_t* mbig = nullptr;     // M counts, zeroed
};
// Takes the tables of a census of k on graphs of n vertices (at most maxn
// each) from the arena and adds the regions to clear to z.
BigTables take_big_tables(Pipeline& p, int k, int32_t n, int64_t maxn, const Tuning& t, ZeroBatch& z);

// side_start (optional) is recorded on s once the set-up has done its
// bandwidth-heavy clears and the small kernels before the core tables: work
// on a second stream that waits for it then runs beside the rest of this
// census instead of crowding those steps.  pre (optional): big-core tables
// taken before the build and already cleared in stream order.
void enqueue_census(Pipeline& p, const DevGraph& g, int k, uint64_t* acc, uint64_t* out, hipStream_t s,
                    bool use_wpool, hipEvent_t side_start = nullptr, bool* side_ok = nullptr,
                    const BigTables* pre = nullptr);
// The exact division alone: out[i] = acc[i] / multiplicity, after a check
// that every remainder is zero (Fact "correction").
void enqueue_finalise(Pipeline& p, int k, int32_t ngraphs, const uint64_t* acc, uint64_t* out, hipStream_t s);
// The same for any table: out[i] = acc[i] / mult[i % C], i < total.
void enqueue_divide(const uint64_t* acc, const uint8_t* mult, int32_t C, int64_t total, uint64_t* out,
                    int32_t* status, hipStream_t s);

// ---- k = 6 (census6.hip) ----
constexpr int32_t kClasses6 = 1530843;  // weakly connected digraphs on 6 vertices
struct Tables6 {
  uint32_t* lut = nullptr;    // device [2^30]: class of each code, 0xFFFFFFFF when disconnected
  uint32_t* codes = nullptr;  // device [kClasses6]: canonical code of each class, increasing
  uint8_t* mult = nullptr;    // device [kClasses6]: anchors (connected dominating 4-subsets) per occurrence
  std::vector<uint32_t> host_codes;
  std::vector<uint8_t> host_mult;
};
// Classify all 2^30 codes on the current device (synchronous, a few seconds;
// 4 GiB for the table).  MOTIF_EINTERNAL if the class counts come out wrong.
int32_t build_tables6(Tables6* T);
void free_tables6(Tables6* T);
// Connected 4-sets of g, each once: count into ctr[1] (fill = false) or write
// them to out[0 .. cap) with ctr[0] as the cursor (fill = true).
int32_t enqueue_anchors6(const DevGraph& g, int4* out, unsigned long long* ctr, unsigned long long cap, bool fill,
                         int num_cus, int32_t* status, hipStream_t s);
// acc[class] += every 6-set of each anchor, counted once per anchor (labels:
// `grid` zeroed slices of label_words words).
void enqueue_census6(const DevGraph& g, const int4* anchors, int64_t nanchors, const Tables6& T, uint64_t* acc,
                     uint32_t* labels, int64_t label_words, int grid, int32_t* status, hipStream_t s);
// Bytes of the per-workgroup W rows of a k = 4, 5 core-reuse census (0 otherwise).
size_t w_slice_bytes(int k, int64_t maxn, const Tuning& t, int num_cus);

// Pack `count` device graphs into one union CSR inside the arena.
// Host arrays voff/aoff are the prefix sums of n and m.
BuildInput enqueue_pack(Pipeline& p, const motif_graph_t* graphs, int32_t count,
                        const int64_t* voff, const int64_t* aoff, hipStream_t s);

// Zero fill helper (a kernel, so it is safe inside captured graphs).
void enqueue_zero(void* ptr, size_t bytes, hipStream_t s);
// Several regions cleared by one kernel launch.
struct ZeroBatch {
  static constexpr int kMax = 16;
  void* ptr[kMax] = {};
  size_t bytes[kMax] = {};
  int n = 0;
  // Regions must be 16-byte aligned (arena regions are); a full batch is an
  // internal sizing error, reported like a workspace error.
  void add(void* p, size_t b) {
    if (!b) return;
    if (n == kMax || ((uintptr_t)p & 15u)) throw WorkspaceError();
    ptr[n] = p;
    bytes[n] = b;
    ++n;
  }
};
void enqueue_zero_batch(const ZeroBatch& z, hipStream_t s);
// dst[0] = st[kStatus], stream-ordered (a kernel).
void enqueue_status_out(int32_t* dst, const int32_t* st, hipStream_t s);
// Undirected census: every entry of the built G* and N+ becomes type A; then
// the directed class totals dir[C] are summed into the U undirected classes.
void enqueue_all_bidirected(const DevGraph& g, hipStream_t s, const int32_t* st);
void enqueue_project_undirected(const uint64_t* dir, const int16_t* und_of, int32_t C, int32_t U, uint64_t* out,
                                int32_t* st, hipStream_t s);


// Device setup (class tables) for the current device; returns the device id.
int32_t ensure_init(int* dev);
int device_cus(int dev);

// Validation + build + census on a pipeline whose arena is already sized
// (host waits for the status word twice).  Used by every entry point.
int32_t run_census_on(Pipeline& p, const BuildInput& in, int32_t k, uint64_t* hist, hipStream_t s);
// Same for several k over one build; hists[i] receives the census of ks[i].
int32_t run_census_multi_on(Pipeline& p, const BuildInput& in, int32_t nk, const int32_t* ks, uint64_t* const* hists,
                            hipStream_t s);
int32_t read_status(Pipeline& p, hipStream_t s);

// ---- null-model ensembles (nullmodel.hip) ----
// One graph to randomise in place by arc switches: its out-CSR (targets
// rewritten), the key of its random stream and the number of rounds of
// kSwitchProposals proposals each.
struct SwitchGraph {
  const int32_t* off;
  int32_t* idx;
  int32_t n;
  int32_t m;
  uint64_t key;
  int64_t rounds;
};
constexpr int kSwitchProposals = 1024;  // proposals (attempted switches) per round
// Enqueue the check and the randomisation of host_graphs[0..count)
// (descriptors copied to the arena; waits for that copy).  The check sets
// MOTIF_EINVAL_SHAPE (offsets), MOTIF_EINDEX or MOTIF_ESELFLOOP (targets) in
// the status word, and nothing is switched once it is set.  mutual: the
// mutual-preserving switch.
int32_t enqueue_switch(Pipeline& p, const SwitchGraph* host_graphs, int32_t count, bool mutual, hipStream_t s);
size_t switch_bytes(int32_t count, int64_t max_n, int64_t max_m, int num_cus);
// Key of graph `graph`'s random stream under `seed`.
uint64_t switch_key(uint64_t seed, int64_t graph);
// Sets MOTIF_EINVAL_SHAPE unless off[0..n] is monotone from 0 to m.
void enqueue_check_rows(const int32_t* off, int32_t n, int64_t m, int32_t* st, hipStream_t s);
// dst[g * m + i] = src[i] for g < copies.
void enqueue_replicate(const int32_t* src, int64_t m, int32_t copies, int32_t* dst, const int32_t* st, hipStream_t s);
// z-scores of row 0 of hists[(count + 1) * C] against rows 1..count.
void enqueue_zscores(const uint64_t* hists, int32_t C, int32_t count, double* z, const int32_t* st, hipStream_t s);
// The fused batch census under an explicit tuning (api.cpp).
int32_t census_batch_with(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists, hipStream_t s,
                          const TuningSet& tune);

// Optional event timing of the build and of the census kernel (motif_profile_*):
// no-ops unless profiling is enabled.  `what` is 0 = build, 1 = census kernel.
void profile_mark(int k, int what, bool begin, hipStream_t s);

}  // namespace motif
