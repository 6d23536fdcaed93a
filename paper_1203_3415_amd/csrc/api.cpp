// C ABI entry points: argument checks, device class tables, per-stream
// workspaces, the single-graph and batched census pipelines, tuning and the
// autotuner.  All arithmetic of the census runs in the kernels of graph.hip
// and census.hip; this file only orchestrates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "classes.h"
#include "internal.h"

namespace motif {

namespace {

std::mutex g_mu;

// Autotuner cache key: (k, batch of several graphs?, floor(log2 of the
// total arc count)).
using TuneKey = std::tuple<int32_t, int32_t, int32_t>;

// Workspace of motif_census_noalloc(): a fixed device array, so that call
// allocates nothing.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (kept per device in
// DeviceState::scratch); the array's name is not a device address on the host.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr size_t kScratchHead = 256;  // status words at the start, then the arena
static __device__ __align__(256) char scratch[kScratchBytes];

struct DeviceState {
  bool ready = false;
  int num_cus = 0;
  char* scratch = nullptr;           // device address of `scratch` on this device
  int32_t* scratch_host = nullptr;   // pinned host copy of its status words
  std::string arch;  // gcnArchName up to the first ':'
  DevTables tables;
  std::vector<void*> owned;  // table buffers
  std::map<hipStream_t, Pipeline*> pipes;
  std::map<TuneKey, Tuning> tuned;  // filled by motif_autotune / motif_tune_cache_load
  // per-stream buffer of the randomised copies made by motif_null_model
  std::map<hipStream_t, std::pair<int32_t*, size_t>> null_copies;
  // k = 6 class table, built on first use (t6_rc 0 once built)
  Tables6 t6;
  int32_t t6_rc = 1;
};

std::map<int, DeviceState> g_dev;
int32_t g_init_err = 0;

// Guarded by g_mu; every call works on a copy (tuning_snapshot).
TuningSet g_tuning = {{
    {256, 4, 16, 1}, {256, 4, 16, 1}, {256, 4, 16, 1},
    {256, 4, 16, 1},    // k = 3: tile*16 vertices per tile (at most 1024)
    // k = 4: core reuse (tile = cost tiles per workgroup); solo / light limits
    // from a sweep on the n = 1e5, m = 1e6 workload
    {1024, 1, 4, 1, 48, 224, 512},
    // k = 5: core reuse, light-partner limit from a sweep on the n = 2e4 workload
    {1024, 1, 128, 1, 64, 192, 384},
}};
// Batches of small graphs (one fused census of many graphs of at most
// kBatchSmallN vertices): for k = 4 the autotuner's choice on 1,001 graphs of
// n = 2,000 (null-model ensembles: many small cores, so smaller workgroups,
// two per CU, finer tiles; fused census 25.0 -> 23.0 ms).  Used while k's
// tuning has not been set explicitly.
const Tuning kBatchTuning4 = {512, 2, 16, 1, 32, 256, 512};
constexpr int64_t kBatchSmallN = 16384;
bool g_batch_default[6] = {false, false, false, false, true, false};

int32_t current_device(int* dev) {
  if (hipGetDevice(dev) != hipSuccess) return MOTIF_EDEVICE;
  return 0;
}

// Upload class tables to the current device (caller holds g_mu).
int32_t init_device_locked(int dev) {
  DeviceState& d = g_dev[dev];
  if (d.ready) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MOTIF_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MOTIF_EDEVICE;
  d.num_cus = prop.multiProcessorCount;
  d.arch = prop.gcnArchName;
  d.arch = d.arch.substr(0, d.arch.find(':'));
  for (int k = 3; k <= 5; ++k) {
    const ClassTable* t = class_table(k);
    void *lut = nullptr, *mult = nullptr, *und = nullptr;
    if (hipMalloc(&lut, t->lut.size() * sizeof(uint16_t)) != hipSuccess) return MOTIF_ENOMEM;
    d.owned.push_back(lut);
    if (hipMalloc(&mult, t->mult.size()) != hipSuccess) return MOTIF_ENOMEM;
    d.owned.push_back(mult);
    if (hipMalloc(&und, t->und_of.size() * sizeof(int16_t)) != hipSuccess) return MOTIF_ENOMEM;
    d.owned.push_back(und);
    const std::vector<uint16_t> dlut = device_lut_order(k, t->lut.data(), t->lut.size());
    if (hipMemcpy(lut, dlut.data(), dlut.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mult, t->mult.data(), t->mult.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(und, t->und_of.data(), t->und_of.size() * sizeof(int16_t), hipMemcpyHostToDevice) != hipSuccess)
      return MOTIF_EDEVICE;
    d.tables.lut[k] = (const uint16_t*)lut;
    d.tables.mult[k] = (const uint8_t*)mult;
    d.tables.und_of[k] = (const int16_t*)und;
  }
  // the allocation-free entry point's workspace: this device's copy of the
  // array, and a pinned word block its status is read back into
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return MOTIF_EDEVICE;
  d.scratch = static_cast<char*>(sp);
  if (hipHostMalloc(&d.scratch_host, kStatusWords * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    d.scratch_host = nullptr;
    return MOTIF_ENOMEM;
  }
  d.ready = true;
  return 0;
}

}  // namespace

int32_t ensure_init(int* dev_out) {
  int dev;
  if (current_device(&dev)) return MOTIF_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  int32_t rc = init_device_locked(dev);
  if (dev_out) *dev_out = dev;
  return rc;
}

int device_cus(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_dev[dev].num_cus;
}

namespace {

// Pipeline (workspace) of a stream on a device, with at least `bytes` of arena.
int32_t get_pipeline(int dev, hipStream_t s, size_t bytes, Pipeline** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& d = g_dev[dev];
  Pipeline*& p = d.pipes[s];
  if (!p) {
    p = new Pipeline();
    p->num_cus = d.num_cus;
    if (hipMalloc(&p->status, kStatusWords * sizeof(int32_t)) != hipSuccess) return MOTIF_ENOMEM;
    if (hipHostMalloc(&p->host_status, kStatusWords * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return MOTIF_ENOMEM;
  }
  if (p->arena.cap < bytes) {
    if (p->arena.base) {  // a failure here shows up as a failed allocation below
      (void)hipStreamSynchronize(s);
      if (p->side) (void)hipStreamSynchronize(p->side);
      (void)hipFree(p->arena.base);
      p->arena.base = nullptr;
      p->arena.cap = 0;
    }
    size_t want = std::max(bytes, p->arena.cap + p->arena.cap / 2);
    if (hipMalloc(&p->arena.base, want) != hipSuccess) {
      p->arena.base = nullptr;
      if (hipMalloc(&p->arena.base, bytes) != hipSuccess) {
        p->arena.base = nullptr;
        return MOTIF_ENOMEM;
      }
      want = bytes;
    }
    p->arena.cap = want;
  }
  p->arena.reset();
  *out = p;
  return 0;
}

// Grow the pipeline's zeroed W-row pool to at least `bytes` (see
// Pipeline::wpool); waits for the stream before replacing an old pool.
int32_t ensure_wpool(Pipeline* p, hipStream_t s, size_t bytes) {
  if (bytes == 0 || p->wpool_bytes >= bytes) return 0;
  if (p->wpool) {
    (void)hipStreamSynchronize(s);  // a failure here shows up as a failed allocation below
    (void)hipFree(p->wpool);
    p->wpool = nullptr;
    p->wpool_bytes = 0;
  }
  void* w = nullptr;
  if (hipMalloc(&w, bytes) != hipSuccess) return 0;  // the census then takes its W rows from the arena
  if (hipMemsetAsync(w, 0, bytes, s) != hipSuccess) {
    (void)hipFree(w);
    return 0;
  }
  p->wpool = static_cast<uint32_t*>(w);
  p->wpool_bytes = bytes;
  return 0;
}

}  // namespace

// Copy the device status word to the host and wait for the stream.
int32_t read_status(Pipeline& p, hipStream_t s) {
  if (hipMemcpyAsync(p.host_status, p.status, sizeof(int32_t) * kStatusWords, hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return MOTIF_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return MOTIF_EDEVICE;
  return p.host_status[kStatus];
}

namespace {

bool check_shape(int32_t n, int64_t m) { return n >= 0 && m >= 0 && n < kMaxN && m < kMaxN; }

// ---- profiling ----
struct ProfState {
  bool on = false;
  bool build = false;  // build events too
  hipEvent_t ev[6][4] = {};
  bool have[6] = {};
  bool have_build[6] = {};
};
ProfState g_prof;

}  // namespace

const DevTables& dev_tables() {
  int dev = 0;
  (void)hipGetDevice(&dev);  // device 0 if it fails; tables were set up by ensure_init
  return g_dev[dev].tables;
}

TuningSet tuning_snapshot() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tuning;
}

namespace {
int32_t size_bucket(int64_t arcs) { return arcs > 1 ? 63 - __builtin_clzll((unsigned long long)arcs) : 0; }
}  // namespace

TuningSet tuning_for_call(int dev, int32_t nk, const int32_t* ks, bool batch, int64_t arcs, int64_t max_n) {
  std::lock_guard<std::mutex> lk(g_mu);
  TuningSet t = g_tuning;
  if (batch && max_n >= 0 && max_n <= kBatchSmallN && g_batch_default[4]) t.k[4] = kBatchTuning4;
  const DeviceState& d = g_dev[dev];
  for (int32_t i = 0; i < nk; ++i) {
    auto it = d.tuned.find(TuneKey{ks[i], batch ? 1 : 0, size_bucket(arcs)});
    if (it != d.tuned.end()) t.k[ks[i]] = it->second;
  }
  return t;
}

namespace {

constexpr int kTuneReps = 3;  // timed runs per autotuner candidate (the median is kept)

motif_tuning_t to_public(const Tuning& t) {
  motif_tuning_t o{};
  o.block = t.block;
  o.grid_per_cu = t.grid_per_cu;
  o.tile = t.tile;
  o.heavy = t.heavy == 1 ? 1 : 2;
  o.solo_deg = t.solo_deg;
  o.light_deg = t.light_deg;
  o.light5 = t.light5;
  return o;
}

// Checks every non-zero field of `in` for k and writes it into *t.
int32_t apply_public(int32_t k, const motif_tuning_t& in, Tuning* t) {
  Tuning r = *t;
  if (in.block) {
    const bool ok = k == 3 ? in.block == 256 : k == 4 ? (in.block == 256 || in.block == 512 || in.block == 1024)
                                                     : (in.block == 512 || in.block == 1024);
    if (!ok) return MOTIF_EINVAL_ARG;
    r.block = in.block;
  }
  if (in.grid_per_cu) {
    if (in.grid_per_cu < 1 || in.grid_per_cu > 16) return MOTIF_EINVAL_ARG;
    r.grid_per_cu = in.grid_per_cu;
  }
  if (in.tile) {
    if (in.tile < 1 || in.tile > 4096) return MOTIF_EINVAL_ARG;
    r.tile = in.tile;
  }
  if (in.heavy) {
    // 1 = core-reuse scheme, 2 = per-anchor scan (k = 4, 5)
    if (in.heavy < 1 || in.heavy > 2) return MOTIF_EINVAL_ARG;
    r.heavy = in.heavy == 2 ? 0 : 1;
  }
  if (in.solo_deg) {
    if (in.solo_deg < 1 || in.solo_deg > 64) return MOTIF_EINVAL_ARG;
    r.solo_deg = in.solo_deg;
  }
  if (in.light_deg) {
    if (in.light_deg < 1 || in.light_deg > 256) return MOTIF_EINVAL_ARG;
    r.light_deg = in.light_deg;
  }
  if (in.light5) {
    if (in.light5 < 1 || in.light5 > 767) return MOTIF_EINVAL_ARG;
    r.light5 = in.light5;
  }
  *t = r;
  return 0;
}

// One tunable of k and the values the autotuner tries for it.
struct TuneAxis {
  int Tuning::*mem;
  std::vector<int> values;
  bool reuse_only;  // only meaningful for the core-reuse scheme
  int& field(Tuning& t) const { return t.*mem; }
};

std::vector<TuneAxis> tune_axes(int k) {
  if (k == 3) return {{&Tuning::tile, {4, 8, 16, 32, 64}, false}, {&Tuning::grid_per_cu, {2, 4, 8}, false}};
  if (k == 4)
    return {{&Tuning::heavy, {1, 0}, false},
            {&Tuning::block, {512, 1024}, false},
            {&Tuning::grid_per_cu, {1, 2}, false},
            {&Tuning::tile, {2, 3, 4, 8, 16}, false},
            {&Tuning::solo_deg, {16, 32, 48, 64}, true},
            {&Tuning::light_deg, {96, 128, 160, 192, 224, 256}, true}};
  return {{&Tuning::block, {512, 1024}, false},
          {&Tuning::tile, {16, 32, 64, 128, 256}, false},
          {&Tuning::light5, {128, 256, 384, 512, 640, 767}, true}};
}

}  // namespace

// Set while motif_census_noalloc() runs on this thread: no profiling events
// are created or recorded for it.
thread_local bool t_no_events = false;

void profile_mark(int k, int what, bool begin, hipStream_t s) {
  if (!g_prof.on || t_no_events || k < 3 || k > 5 || (what == 0 && !g_prof.build)) return;
  hipEvent_t& e = g_prof.ev[k][what * 2 + (begin ? 0 : 1)];
  if (!e && hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
    return;  // no timing for this mark; the census is unaffected
  }
  (void)hipEventRecord(e, s);
  if (what == 1 && !begin) g_prof.have[k] = true;
  if (what == 0 && !begin) g_prof.have_build[k] = true;
}

// A workspace sizing error stopped an enqueue half way: the kernels already
// enqueued only touch regions taken before it; wait for them (on both
// streams) so that the workspace can be reused, and report the error.
int32_t drain_after_error(Pipeline& p, hipStream_t s) {
  (void)hipStreamSynchronize(s);  // best effort: the error below is what the caller acts on
  if (p.side) (void)hipStreamSynchronize(p.side);
  return MOTIF_EINTERNAL;
}

int32_t run_census_multi_enqueue(Pipeline& p, const BuildInput& in, int32_t nk, const int32_t* ks,
                                 uint64_t* const* hists, hipStream_t s);

// One census on a sized pipeline: build + status wait + census + status wait.
// The census is enqueued right behind the build, with no host wait in
// between: every census kernel returns at once when the build has set the
// status word, and the exact division writes nothing then.
int32_t run_census_on(Pipeline& p, const BuildInput& in, int32_t k, uint64_t* hist, hipStream_t s) {
  const int C = motif_num_classes(k);
  try {
    p.arena.reset();
    enqueue_zero(p.status, sizeof(int32_t) * kStatusWords, s);
    profile_mark(k, 0, true, s);
    DevGraph g = enqueue_build(p, in, s);
    profile_mark(k, 0, false, s);
    uint64_t* acc = p.arena.take<uint64_t>((size_t)in.ngraphs * C);
    enqueue_census(p, g, k, acc, hist, s, true);
  } catch (const WorkspaceError&) {
    return drain_after_error(p, s);
  }
  return read_status(p, s);
}

// Several sizes over one build.  The largest size runs on the caller's
// stream; the others follow each other on the pipeline's second stream,
// forked after the build, so their workgroups fill the compute units that the
// largest census leaves idle at its end.  Each census has its own workspace.
int32_t run_census_multi_on(Pipeline& p, const BuildInput& in, int32_t nk, const int32_t* ks, uint64_t* const* hists,
                            hipStream_t s) {
  try {
    return run_census_multi_enqueue(p, in, nk, ks, hists, s);
  } catch (const WorkspaceError&) {
    return drain_after_error(p, s);
  }
}

int32_t run_census_multi_enqueue(Pipeline& p, const BuildInput& in, int32_t nk, const int32_t* ks,
                                 uint64_t* const* hists, hipStream_t s) {
  p.arena.reset();
  // A second stream takes the in-CSR check and every size but the largest,
  // so that neither delays the largest census on the caller's stream.
  const bool fork = nk > 1 || in.in_off != nullptr;
  if (fork) {
    if (!p.side && hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking) != hipSuccess) return MOTIF_EDEVICE;
    if (!p.ev_fork && hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming) != hipSuccess) return MOTIF_EDEVICE;
    if (!p.ev_join && hipEventCreateWithFlags(&p.ev_join, hipEventDisableTiming) != hipSuccess) return MOTIF_EDEVICE;
    if (!p.ev_pre && hipEventCreateWithFlags(&p.ev_pre, hipEventDisableTiming) != hipSuccess) return MOTIF_EDEVICE;
  }
  int32_t top = 0;
  for (int32_t i = 1; i < nk; ++i)
    if (ks[i] > ks[top]) top = i;
  // The largest census's big-core tables (307 MB on the n = 10^5 graph) are
  // cleared on the second stream while the build runs: the build is a chain
  // of latency-bound kernels that leaves the bandwidth free.  (The previous
  // call on this pipeline has ended on both streams, so the region is idle.)
  auto device_error = [&] {
    (void)hipStreamSynchronize(s);  // best effort: the error is what the caller acts on
    (void)hipStreamSynchronize(p.side);
    return MOTIF_EDEVICE;
  };
  BigTables pre;
  bool pre_on_side = false;
  if (fork) {
    ZeroBatch zb;
    pre = take_big_tables(p, ks[top], in.n, in.gid ? in.max_graph_n : in.n, p.tune.k[ks[top]], zb);
    if (pre.nbig > 0) {
      enqueue_zero_batch(zb, p.side);
      if (hipEventRecord(p.ev_pre, p.side) != hipSuccess) return device_error();
      pre_on_side = true;
    }
  }
  enqueue_zero(p.status, sizeof(int32_t) * kStatusWords, s);
  for (int32_t i = 0; i < nk; ++i) profile_mark(ks[i], 0, true, s);  // the shared build, seen by every k
  InCheck check;
  DevGraph g = enqueue_build(p, in, s, nullptr, nullptr, fork ? &check : nullptr);
  for (int32_t i = 0; i < nk; ++i) profile_mark(ks[i], 0, false, s);
  if (pre_on_side && hipStreamWaitEvent(s, p.ev_pre, 0) != hipSuccess) return device_error();
  uint64_t* acc[3] = {};  // nk <= 3 (checked by the entry point)
  acc[top] = p.arena.take<uint64_t>((size_t)in.ngraphs * motif_num_classes(ks[top]));
  // the second stream starts once the largest census has done the clears
  // and small kernels of its set-up (G* and N+ are complete by then)
  bool side_ok = true;
  enqueue_census(p, g, ks[top], acc[top], fork ? nullptr : hists[top], s, true, fork ? p.ev_fork : nullptr,
                 &side_ok, fork ? &pre : nullptr);
  if (fork && (!side_ok || hipStreamWaitEvent(p.side, p.ev_fork, 0) != hipSuccess)) return device_error();
  for (int32_t i = 0; i < nk; ++i) {
    if (i == top) continue;
    acc[i] = p.arena.take<uint64_t>((size_t)in.ngraphs * motif_num_classes(ks[i]));
    enqueue_census(p, g, ks[i], acc[i], nullptr, p.side, false);
  }
  if (!fork) return read_status(p, s);
  // after the smaller sizes: the check then runs beside the largest census
  // rather than beside its set-up
  enqueue_check_in(in, g, check, p.status, p.side, true);
  if (hipEventRecord(p.ev_join, p.side) != hipSuccess || hipStreamWaitEvent(s, p.ev_join, 0) != hipSuccess)
    return device_error();
  // Every division runs after the join, on the caller's stream: a failed
  // in-CSR check then leaves every output unwritten, and the side sizes'
  // divisions do not wait on the second stream for compute units that the
  // largest census holds until its end.
  for (int32_t i = 0; i < nk; ++i) enqueue_finalise(p, ks[i], in.ngraphs, acc[i], hists[i], s);
  return read_status(p, s);
}

int32_t run_census(const BuildInput& in, int32_t k, uint64_t* hist, hipStream_t s) {
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  const TuningSet tune = tuning_for_call(dev, 1, &k, false, in.m);
  Pipeline* p = nullptr;
  rc = get_pipeline(dev, s, pipeline_bytes(in.n, in.m, in.ngraphs, false, k, device_cus(dev), in.n, tune.k[k]), &p);
  if (rc) return rc;
  p->tune = tune;
  ensure_wpool(p, s, w_slice_bytes(k, in.n, tune.k[k], device_cus(dev)));
  return run_census_on(*p, in, k, hist, s);
}

// Fused census of a batch under an explicit tuning (motif_census_batch and
// the autotuner's candidates).
int32_t census_batch_with(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists, hipStream_t s,
                          const TuningSet& tune) {
  std::vector<int64_t> voff(count + 1, 0), aoff(count + 1, 0);
  for (int32_t g = 0; g < count; ++g) {
    const motif_graph_t& G = graphs[g];
    if (!check_shape(G.n, G.m)) return MOTIF_EINVAL_SHAPE;
    if (G.n == 0 && G.m != 0) return MOTIF_EINVAL_SHAPE;
    if ((G.n > 0 && !G.out_off) || (G.m > 0 && !G.out_idx)) return MOTIF_EINVAL_ARG;
    if (G.in_off && G.m > 0 && !G.in_idx) return MOTIF_EINVAL_ARG;
    voff[g + 1] = voff[g] + G.n;
    aoff[g + 1] = aoff[g] + G.m;
  }
  if (voff[count] >= kMaxN || aoff[count] >= kMaxN) return MOTIF_EINVAL_SHAPE;
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  const int C = motif_num_classes(k);
  if (voff[count] == 0) {
    enqueue_zero(hists, sizeof(uint64_t) * C * (size_t)count, s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  // Graphs with n = 0 contribute no vertices; the pack kernel never sees them.
  Pipeline* p = nullptr;
  int64_t maxn = 0;
  for (int32_t g = 0; g < count; ++g) maxn = std::max<int64_t>(maxn, graphs[g].n);
  rc = get_pipeline(dev, s,
                    pipeline_bytes(voff[count], aoff[count], count, true, k, device_cus(dev), maxn, tune.k[k]), &p);
  if (rc) return rc;
  p->tune = tune;
  ensure_wpool(p, s, w_slice_bytes(k, maxn, tune.k[k], device_cus(dev)));
  try {
    p->arena.reset();
    enqueue_zero(p->status, sizeof(int32_t) * kStatusWords, s);
    profile_mark(k, 0, true, s);
    BuildInput in = enqueue_pack(*p, graphs, count, voff.data(), aoff.data(), s);
    if (in.copy_error) {
      (void)hipStreamSynchronize(s);  // copies already enqueued end before the workspace is reused
      return MOTIF_EDEVICE;
    }
    DevGraph g = enqueue_build(*p, in, s);
    profile_mark(k, 0, false, s);
    uint64_t* acc = p->arena.take<uint64_t>((size_t)count * C);
    enqueue_census(*p, g, k, acc, hists, s, true);
  } catch (const WorkspaceError&) {
    return drain_after_error(*p, s);
  }
  return read_status(*p, s);
}

}  // namespace motif

using namespace motif;

extern "C" {

int32_t motif_init(void) {
  int dev;
  return ensure_init(&dev);
}

int32_t motif_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_dev) {  // tear-down: errors change nothing a caller could act on
    (void)hipSetDevice(kv.first);
    (void)hipDeviceSynchronize();
    for (void* ptr : kv.second.owned) (void)hipFree(ptr);
    if (kv.second.scratch_host) (void)hipHostFree(kv.second.scratch_host);
    for (auto& nc : kv.second.null_copies) (void)hipFree(nc.second.first);
    free_tables6(&kv.second.t6);
    for (auto& pp : kv.second.pipes) {
      if (pp.second->side) (void)hipStreamDestroy(pp.second->side);
      if (pp.second->ev_fork) (void)hipEventDestroy(pp.second->ev_fork);
      if (pp.second->ev_join) (void)hipEventDestroy(pp.second->ev_join);
      if (pp.second->ev_pre) (void)hipEventDestroy(pp.second->ev_pre);
      if (pp.second->k6_buf) (void)hipFree(pp.second->k6_buf);
      if (pp.second->arena.base) (void)hipFree(pp.second->arena.base);
      if (pp.second->wpool) (void)hipFree(pp.second->wpool);
      if (pp.second->status) (void)hipFree(pp.second->status);
      if (pp.second->host_status) (void)hipHostFree(pp.second->host_status);
      delete pp.second;
    }
  }
  g_dev.clear();
  return 0;
}

int32_t motif_num_classes(int32_t k) {
  switch (k) {
    case 3: return 13;
    case 4: return 199;
    case 5: return 9364;
    default: return MOTIF_EINVAL_K;
  }
}

int32_t motif_class_code(int32_t k, int32_t cls, uint32_t* canon_code) {
  const ClassTable* t = class_table(k);
  if (!t) return MOTIF_EINVAL_K;
  if (cls < 0 || cls >= (int32_t)t->canon.size() || !canon_code) return MOTIF_EINVAL_ARG;
  *canon_code = t->canon[cls];
  return 0;
}

int32_t motif_class_multiplicity(int32_t k, int32_t cls) {
  const ClassTable* t = class_table(k);
  if (!t) return MOTIF_EINVAL_K;
  if (cls < 0 || cls >= (int32_t)t->mult.size()) return MOTIF_EINVAL_ARG;
  return t->mult[cls];
}

int32_t motif_num_undirected_classes(int32_t k) {
  const ClassTable* t = class_table(k);
  return t ? (int32_t)t->und_canon.size() : MOTIF_EINVAL_K;
}

int32_t motif_undirected_class_code(int32_t k, int32_t cls, uint32_t* canon_code) {
  const ClassTable* t = class_table(k);
  if (!t) return MOTIF_EINVAL_K;
  if (cls < 0 || cls >= (int32_t)t->und_canon.size() || !canon_code) return MOTIF_EINVAL_ARG;
  *canon_code = t->und_canon[cls];
  return 0;
}

int32_t motif_class_undirected(int32_t k, int32_t cls) {
  const ClassTable* t = class_table(k);
  if (!t) return MOTIF_EINVAL_K;
  if (cls < 0 || cls >= (int32_t)t->und_of.size()) return MOTIF_EINVAL_ARG;
  return t->und_of[cls];
}

int32_t motif_class_of_code(int32_t k, uint32_t code) {
  const ClassTable* t = class_table(k);
  if (!t) return MOTIF_EINVAL_K;
  if (code >= t->lut.size()) return MOTIF_EINVAL_ARG;
  return t->lut[code] == 0xFFFF ? -1 : (int32_t)t->lut[code];
}

const char* motif_strerror(int32_t code) {
  switch (code) {
    case MOTIF_OK: return "ok";
    case MOTIF_EINVAL_K: return "k must be 3, 4 or 5";
    case MOTIF_EINVAL_SHAPE: return "invalid CSR shape (n, m or offsets)";
    case MOTIF_EINDEX: return "neighbour index out of range";
    case MOTIF_ESELFLOOP: return "self-loop";
    case MOTIF_EDUP: return "repeated arc";
    case MOTIF_ETRANSPOSE: return "in-CSR is not the transpose of the out-CSR";
    case MOTIF_ENOMEM: return "out of memory";
    case MOTIF_EDEVICE: return "HIP device error or no gfx950 device";
    case MOTIF_EAGAIN: return "not admitted now; retry";
    case MOTIF_ETOOBIG: return "request exceeds the server's memory budget";
    case MOTIF_ETIMEOUT: return "timed out";
    case MOTIF_ECANCELED: return "cancelled";
    case MOTIF_EINVAL_ARG: return "invalid argument";
    case MOTIF_EINTERNAL: return "internal self-check failed";
    case MOTIF_EPARSE: return "malformed network file";
    case MOTIF_EIO: return "network file cannot be read";
    default: return "unknown error";
  }
}

int32_t motif_census(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off, const int32_t* in_idx,
                     int32_t n, int64_t m, int32_t k, uint64_t* hist, void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!check_shape(n, m)) return MOTIF_EINVAL_SHAPE;
  if (!hist || !out_off || (m > 0 && !out_idx)) return MOTIF_EINVAL_ARG;
  if (in_off && m > 0 && !in_idx) return MOTIF_EINVAL_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    if (m != 0) return MOTIF_EINVAL_SHAPE;
    int dev;
    int32_t rc = ensure_init(&dev);
    if (rc) return rc;
    enqueue_zero(hist, sizeof(uint64_t) * motif_num_classes(k), s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  BuildInput in{};
  in.out_off = out_off;
  in.out_idx = out_idx;
  in.in_off = in_off;
  in.in_idx = in_off ? in_idx : nullptr;
  in.n = n;
  in.m = m;
  return run_census(in, k, hist, s);
}

// ---- k = 6 ----

// The k = 6 class table of device dev (current), built once; a failed build
// (say, out of device memory) is tried again by the next call.
static int32_t ensure_tables6(int dev, const Tables6** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& d = g_dev[dev];
  if (d.t6_rc != 0) {
    const int32_t rc = build_tables6(&d.t6);
    d.t6_rc = rc == 0 ? 0 : 1;
    if (rc) return rc;
  }
  *out = &d.t6;
  return 0;
}

int32_t motif_census6(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off, const int32_t* in_idx,
                      int32_t n, int64_t m, uint64_t* hist, void* stream) {
  if (!check_shape(n, m) || (n == 0 && m != 0)) return MOTIF_EINVAL_SHAPE;
  if (!hist || !out_off || (m > 0 && !out_idx)) return MOTIF_EINVAL_ARG;
  if (in_off && m > 0 && !in_idx) return MOTIF_EINVAL_ARG;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  const Tables6* T = nullptr;
  if (int32_t rc = ensure_tables6(dev, &T)) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    enqueue_zero(hist, sizeof(uint64_t) * kClasses6, s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  BuildInput in{};
  in.out_off = out_off;
  in.out_idx = out_idx;
  in.in_off = in_off;
  in.in_idx = in_off ? in_idx : nullptr;
  in.n = n;
  in.m = m;
  const int cus = device_cus(dev);
  Pipeline* p = nullptr;
  if (int32_t rc = get_pipeline(dev, s, build_bytes(n, m, 1, false) + 4096, &p)) return rc;
  DevGraph g;
  unsigned long long* ctr = nullptr;
  try {
    p->arena.reset();
    enqueue_zero(p->status, sizeof(int32_t) * kStatusWords, s);
    g = enqueue_build(*p, in, s);
    ctr = p->arena.take<unsigned long long>(2);
  } catch (const WorkspaceError&) {
    return drain_after_error(*p, s);
  }
  if (int32_t rc = read_status(*p, s)) return rc;
  // the anchors: counted, then listed (each connected 4-set once)
  int4* anchors = nullptr;
  uint64_t* acc = nullptr;
  uint32_t* labels = nullptr;
  int32_t rc = 0;
  // a census workgroup's anchor is a short chain of dependent reads, so the
  // chip wants all the workgroups it can hold (five per CU by LDS; the grid
  // must not exceed what is resident, since the workgroups stride over the
  // anchor list); each needs its own byte labels, n bytes, hence fewer for
  // large n
  const int grid = (n <= 65536 ? 4 : 2) * cus;
  const int64_t label_words = ((int64_t)n + 3) / 4;
  do {
    unsigned long long host_ctr[2] = {0, 0};
    enqueue_zero(ctr, sizeof(host_ctr), s);
    if ((rc = enqueue_anchors6(g, nullptr, ctr, 0, false, cus, p->status, s))) break;
    if (hipMemcpyAsync(host_ctr, ctr, sizeof(host_ctr), hipMemcpyDeviceToHost, s) != hipSuccess) {
      rc = MOTIF_EDEVICE;
      break;
    }
    if ((rc = read_status(*p, s))) break;  // also waits for the count
    const unsigned long long na = host_ctr[1];
    if (na >= (1ull << 31)) { rc = MOTIF_ETOOBIG; break; }
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t acc_b = al(sizeof(uint64_t) * kClasses6);
    const size_t lab_b = al(sizeof(uint32_t) * (size_t)grid * (size_t)label_words);
    const size_t need = acc_b + lab_b + al(sizeof(int4) * (size_t)std::max(na, 1ull));
    if (p->k6_bytes < need) {  // nothing of an earlier call is in flight: read_status waited above
      const size_t want = std::max(need, p->k6_bytes + p->k6_bytes / 2);
      (void)hipFree(p->k6_buf);
      p->k6_buf = nullptr;
      p->k6_bytes = 0;
      if (hipMalloc(&p->k6_buf, want) != hipSuccess) {
        p->k6_buf = nullptr;
        rc = MOTIF_ENOMEM;
        break;
      }
      p->k6_bytes = want;
    }
    acc = reinterpret_cast<uint64_t*>(p->k6_buf);
    labels = reinterpret_cast<uint32_t*>(p->k6_buf + acc_b);
    anchors = reinterpret_cast<int4*>(p->k6_buf + acc_b + lab_b);
    enqueue_zero(acc, sizeof(uint64_t) * kClasses6, s);
    enqueue_zero(labels, sizeof(uint32_t) * (size_t)grid * (size_t)label_words, s);
    if (na > 0) {
      enqueue_zero(ctr, sizeof(host_ctr), s);
      if ((rc = enqueue_anchors6(g, anchors, ctr, na, true, cus, p->status, s))) break;
      enqueue_census6(g, anchors, (int64_t)na, *T, acc, labels, label_words, grid, p->status, s);
    }
    enqueue_divide(acc, T->mult, kClasses6, kClasses6, hist, p->status, s);
    rc = read_status(*p, s);
  } while (false);
  if (rc) (void)hipStreamSynchronize(s);  // the buffers are reused by the next call only after this work
  return rc;
}

int32_t motif_class6_codes(uint32_t* codes) {
  if (!codes) return MOTIF_EINVAL_ARG;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  const Tables6* T = nullptr;
  if (int32_t rc = ensure_tables6(dev, &T)) return rc;
  std::copy(T->host_codes.begin(), T->host_codes.end(), codes);
  return 0;
}

int32_t motif_class6_multiplicities(uint8_t* mult) {
  if (!mult) return MOTIF_EINVAL_ARG;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  const Tables6* T = nullptr;
  if (int32_t rc = ensure_tables6(dev, &T)) return rc;
  std::copy(T->host_mult.begin(), T->host_mult.end(), mult);
  return 0;
}

int32_t motif_census_async(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off,
                           const int32_t* in_idx, int32_t n, int64_t m, int32_t k, uint64_t* hist, int32_t* status,
                           void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!check_shape(n, m) || (n == 0 && m != 0)) return MOTIF_EINVAL_SHAPE;
  if (!hist || !status || !out_off || (m > 0 && !out_idx)) return MOTIF_EINVAL_ARG;
  if (in_off && m > 0 && !in_idx) return MOTIF_EINVAL_ARG;
  hipStream_t s = (hipStream_t)stream;
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  const TuningSet tune = tuning_for_call(dev, 1, &k, false, m);
  Pipeline* p = nullptr;
  rc = get_pipeline(dev, s, pipeline_bytes(n, m, 1, false, k, device_cus(dev), n, tune.k[k]), &p);
  if (rc) return rc;
  p->tune = tune;
  ensure_wpool(p, s, w_slice_bytes(k, n, tune.k[k], device_cus(dev)));
  BuildInput in{};
  in.out_off = out_off;
  in.out_idx = out_idx;
  in.in_off = in_off;
  in.in_idx = in_off ? in_idx : nullptr;
  in.n = n;
  in.m = m;
  try {
    p->arena.reset();
    enqueue_zero(p->status, sizeof(int32_t) * kStatusWords, s);
    if (n == 0) {
      enqueue_zero(hist, sizeof(uint64_t) * motif_num_classes(k), s);
    } else {
      profile_mark(k, 0, true, s);
      DevGraph g = enqueue_build(*p, in, s);
      profile_mark(k, 0, false, s);
      uint64_t* acc = p->arena.take<uint64_t>((size_t)motif_num_classes(k));
      enqueue_census(*p, g, k, acc, hist, s, true);
    }
    enqueue_status_out(status, p->status, s);
  } catch (const WorkspaceError&) {
    return drain_after_error(*p, s);
  }
  return 0;
}

int32_t motif_census_noalloc(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off,
                             const int32_t* in_idx, int32_t n, int64_t m, int32_t k, uint64_t* hist, void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!check_shape(n, m) || (n == 0 && m != 0)) return MOTIF_EINVAL_SHAPE;
  if (!hist || !out_off || (m > 0 && !out_idx)) return MOTIF_EINVAL_ARG;
  if (in_off && m > 0 && !in_idx) return MOTIF_EINVAL_ARG;
  hipStream_t s = (hipStream_t)stream;
  int dev;
  if (current_device(&dev)) return MOTIF_EDEVICE;
  char* base = nullptr;
  int32_t* host_status = nullptr;
  int cus = 0;
  {
    // set up by motif_init(); nothing is initialised (allocated) here
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end() || !it->second.ready || !it->second.scratch) return MOTIF_EDEVICE;
    base = it->second.scratch;
    host_status = it->second.scratch_host;
    cus = it->second.num_cus;
  }
  // One workspace per device: calls are serialised here, and each returns
  // only after its work has finished, so two calls never overlap in it.
  static std::mutex scratch_mu;
  std::lock_guard<std::mutex> lk(scratch_mu);
  TuningSet tune = tuning_for_call(dev, 1, &k, false, m);
  const size_t room = kScratchBytes - kScratchHead;
  size_t need = pipeline_bytes(n, m, 1, false, k, cus, n, tune.k[k]);
  if (need > room && (k == 4 || k == 5) && tune.k[k].heavy == 1) {
    // the per-anchor scheme needs no per-workgroup W rows: same result, less room
    tune.k[k].heavy = 0;
    need = pipeline_bytes(n, m, 1, false, k, cus, n, tune.k[k]);
  }
  if (need > room) return MOTIF_ETOOBIG;
  Pipeline p;
  p.arena.base = base + kScratchHead;
  p.arena.cap = room;
  p.status = reinterpret_cast<int32_t*>(base);
  p.host_status = host_status;
  p.num_cus = cus;
  p.tune = tune;
  if (n == 0) {
    enqueue_zero(hist, sizeof(uint64_t) * motif_num_classes(k), s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  BuildInput in{};
  in.out_off = out_off;
  in.out_idx = out_idx;
  in.in_off = in_off;
  in.in_idx = in_off ? in_idx : nullptr;
  in.n = n;
  in.m = m;
  t_no_events = true;
  const int32_t rc = run_census_on(p, in, k, hist, s);
  t_no_events = false;
  return rc;
}

int32_t motif_census_undirected(const int32_t* out_off, const int32_t* out_idx, int32_t n, int64_t m, int32_t k,
                                uint64_t* hist, void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!check_shape(n, m) || (n == 0 && m != 0)) return MOTIF_EINVAL_SHAPE;
  if (!hist || !out_off || (m > 0 && !out_idx)) return MOTIF_EINVAL_ARG;
  hipStream_t s = (hipStream_t)stream;
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  const ClassTable* ct = class_table(k);
  const int32_t C = motif_num_classes(k), U = (int32_t)ct->und_canon.size();
  if (n == 0) {
    enqueue_zero(hist, sizeof(uint64_t) * U, s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  const TuningSet tune = tuning_for_call(dev, 1, &k, false, m);
  Pipeline* p = nullptr;
  rc = get_pipeline(dev, s, pipeline_bytes(n, m, 1, false, k, device_cus(dev), n, tune.k[k]), &p);
  if (rc) return rc;
  p->tune = tune;
  ensure_wpool(p, s, w_slice_bytes(k, n, tune.k[k], device_cus(dev)));
  BuildInput in{};
  in.out_off = out_off;
  in.out_idx = out_idx;
  in.n = n;
  in.m = m;
  try {
    p->arena.reset();
    enqueue_zero(p->status, sizeof(int32_t) * kStatusWords, s);
    profile_mark(k, 0, true, s);
    DevGraph g = enqueue_build(*p, in, s);
    enqueue_all_bidirected(g, s, p->status);
    profile_mark(k, 0, false, s);
    uint64_t* acc = p->arena.take<uint64_t>((size_t)C);
    uint64_t* dir = p->arena.take<uint64_t>((size_t)C);
    enqueue_census(*p, g, k, acc, dir, s, true);
    enqueue_project_undirected(dir, dev_tables().und_of[k], C, U, hist, p->status, s);
  } catch (const WorkspaceError&) {
    return drain_after_error(*p, s);
  }
  return read_status(*p, s);
}

int32_t motif_census_multi(const motif_graph_t* g, int32_t nk, const int32_t* ks, uint64_t* const* hists,
                           void* stream) {
  if (!g || !ks || !hists || nk < 1 || nk > 3) return MOTIF_EINVAL_ARG;
  bool seen[6] = {};
  for (int32_t i = 0; i < nk; ++i) {
    if (motif_num_classes(ks[i]) < 0) return MOTIF_EINVAL_K;
    if (seen[ks[i]] || !hists[i]) return MOTIF_EINVAL_ARG;
    seen[ks[i]] = true;
  }
  if (!check_shape(g->n, g->m)) return MOTIF_EINVAL_SHAPE;
  if (!g->out_off || (g->m > 0 && !g->out_idx)) return MOTIF_EINVAL_ARG;
  if (g->in_off && g->m > 0 && !g->in_idx) return MOTIF_EINVAL_ARG;
  hipStream_t s = (hipStream_t)stream;
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  if (g->n == 0) {
    if (g->m != 0) return MOTIF_EINVAL_SHAPE;
    for (int32_t i = 0; i < nk; ++i) enqueue_zero(hists[i], sizeof(uint64_t) * motif_num_classes(ks[i]), s);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
  }
  BuildInput in{};
  in.out_off = g->out_off;
  in.out_idx = g->out_idx;
  in.in_off = g->in_off;
  in.in_idx = g->in_off ? g->in_idx : nullptr;
  in.n = g->n;
  in.m = g->m;
  // one build plus the workspace of every size (the censuses may run at once)
  const TuningSet tune = tuning_for_call(dev, nk, ks, false, in.m);
  const size_t build = build_bytes(in.n, in.m, 1, false);
  size_t bytes = build;
  for (int32_t i = 0; i < nk; ++i)
    bytes += pipeline_bytes(in.n, in.m, 1, false, ks[i], device_cus(dev), in.n, tune.k[ks[i]]) - build;
  Pipeline* p = nullptr;
  rc = get_pipeline(dev, s, bytes, &p);
  if (rc) return rc;
  p->tune = tune;
  int32_t top = 0;  // the largest size runs on `stream` and may use the pool
  for (int32_t i = 1; i < nk; ++i)
    if (ks[i] > ks[top]) top = i;
  ensure_wpool(p, s, w_slice_bytes(ks[top], in.n, tune.k[ks[top]], device_cus(dev)));
  return run_census_multi_on(*p, in, nk, ks, hists, s);
}

int32_t motif_census_batch(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists, void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (count < 0 || (count > 0 && (!graphs || !hists))) return MOTIF_EINVAL_ARG;
  if (count == 0) return 0;
  int dev;
  int32_t rc = ensure_init(&dev);
  if (rc) return rc;
  int64_t arcs = 0, max_n = 0;
  for (int32_t g = 0; g < count; ++g) {
    arcs += std::max<int64_t>(0, graphs[g].m);
    max_n = std::max<int64_t>(max_n, graphs[g].n);
  }
  return census_batch_with(graphs, count, k, hists, (hipStream_t)stream,
                           tuning_for_call(dev, 1, &k, count > 1, arcs, max_n));
}

int32_t motif_census_batch_loop(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists,
                                void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (count < 0 || (count > 0 && (!graphs || !hists))) return MOTIF_EINVAL_ARG;
  const int C = motif_num_classes(k);
  for (int32_t g = 0; g < count; ++g) {
    const motif_graph_t& G = graphs[g];
    int32_t rc = motif_census(G.out_off, G.out_idx, G.in_off, G.in_idx, G.n, G.m, k, hists + (size_t)g * C, stream);
    if (rc) return rc;
  }
  return 0;
}

int32_t motif_get_tuning(int32_t k, motif_tuning_t* out) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!out) return MOTIF_EINVAL_ARG;
  *out = to_public(tuning_snapshot().k[k]);
  return 0;
}

int32_t motif_set_tuning(int32_t k, const motif_tuning_t* in) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!in) return MOTIF_EINVAL_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  Tuning t = g_tuning.k[k];
  if (int32_t rc = apply_public(k, *in, &t)) return rc;
  g_tuning.k[k] = t;
  g_batch_default[k] = false;  // an explicit choice holds for batches too
  // an explicit choice replaces what the autotuner cached for k
  for (auto& d : g_dev)
    for (auto it = d.second.tuned.begin(); it != d.second.tuned.end();)
      it = std::get<0>(it->first) == k ? d.second.tuned.erase(it) : std::next(it);
  return 0;
}

int32_t motif_autotune(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists, void* stream,
                       motif_tuning_t* best) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (count <= 0 || !graphs || !hists) return MOTIF_EINVAL_ARG;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  const int C = motif_num_classes(k);
  hipStream_t s = (hipStream_t)stream;
  int64_t arcs = 0;
  for (int32_t g = 0; g < count; ++g) arcs += std::max<int64_t>(0, graphs[g].m);
  const bool batch = count > 1;
  const TuneKey key{k, batch ? 1 : 0, size_bucket(arcs)};
  TuningSet base = tuning_snapshot();
  {
    std::lock_guard<std::mutex> lk(g_mu);  // start from the cached entry of this bucket, if any
    auto it = g_dev[dev].tuned.find(key);
    if (it != g_dev[dev].tuned.end()) base.k[k] = it->second;
  }
  std::vector<uint64_t> ref((size_t)count * C), cur((size_t)count * C);
  bool have_ref = false;
  // One candidate: warm-up, then the median wall time of kTuneReps runs; its
  // histograms must equal those of the first candidate.
  auto measure = [&](const Tuning& t, double* ms_out) -> int32_t {
    TuningSet ts = base;
    ts.k[k] = t;
    int32_t rc = census_batch_with(graphs, count, k, hists, s, ts);
    if (rc) return rc;
    std::vector<double> ms;
    for (int r = 0; r < kTuneReps; ++r) {
      auto t0 = std::chrono::steady_clock::now();
      rc = census_batch_with(graphs, count, k, hists, s, ts);
      auto t1 = std::chrono::steady_clock::now();
      if (rc) return rc;
      ms.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    std::sort(ms.begin(), ms.end());
    *ms_out = ms[ms.size() / 2];
    std::vector<uint64_t>& dst = have_ref ? cur : ref;
    if (hipMemcpyAsync(dst.data(), hists, sizeof(uint64_t) * ref.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MOTIF_EDEVICE;
    if (have_ref && cur != ref) return MOTIF_EINTERNAL;
    have_ref = true;
    return 0;
  };
  // Coordinate descent over the tunables of k, two passes: each field in
  // turn takes the best of its candidate values with the others held.
  Tuning bt = base.k[k];
  double best_ms = 0;
  if (int32_t rc = measure(bt, &best_ms)) return rc;
  const std::vector<TuneAxis> axes = tune_axes(k);
  for (int pass = 0; pass < 2; ++pass) {
    for (const TuneAxis& ax : axes) {
      if (ax.reuse_only && bt.heavy != 1) continue;
      for (int v : ax.values) {
        Tuning t = bt;
        if (ax.field(t) == v) continue;
        ax.field(t) = v;
        double ms = 0;
        if (int32_t rc = measure(t, &ms)) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          bt = t;
        }
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_dev[dev].tuned[key] = bt;
  }
  if (best) *best = to_public(bt);
  return 0;
}

int32_t motif_tune_cache_save(const char* path) {
  if (!path) return MOTIF_EINVAL_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return MOTIF_EINVAL_ARG;
  std::fprintf(f, "# arch cus k batch bucket block grid_per_cu tile heavy solo_deg light_deg light5\n");
  for (auto& d : g_dev)
    for (auto& e : d.second.tuned) {
      const Tuning& t = e.second;
      std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d\n", d.second.arch.c_str(), d.second.num_cus,
                   std::get<0>(e.first), std::get<1>(e.first), std::get<2>(e.first), t.block, t.grid_per_cu, t.tile,
                   t.heavy, t.solo_deg, t.light_deg, t.light5);
    }
  return std::fclose(f) == 0 ? 0 : MOTIF_EINVAL_ARG;
}

int32_t motif_tune_cache_load(const char* path) {
  if (!path) return MOTIF_EINVAL_ARG;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  FILE* f = std::fopen(path, "r");
  if (!f) return MOTIF_EINVAL_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& d = g_dev[dev];
  int32_t loaded = 0;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    char arch[64];
    int cus, k, batch, bucket;
    Tuning t;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d", arch, &cus, &k, &batch, &bucket, &t.block,
                    &t.grid_per_cu, &t.tile, &t.heavy, &t.solo_deg, &t.light_deg, &t.light5) != 12)
      continue;
    // entries of another kind of device, and values outside the accepted
    // ranges, are skipped
    if (d.arch != arch || d.num_cus != cus || motif_num_classes(k) < 0) continue;
    Tuning chk = g_tuning.k[k];
    if (apply_public(k, to_public(t), &chk)) continue;
    d.tuned[TuneKey{k, batch ? 1 : 0, bucket}] = chk;
    ++loaded;
  }
  std::fclose(f);
  return loaded;
}

}  // extern "C"

namespace {

// Validate the descriptors of graphs to randomise and fill the switch list.
int32_t switch_list(const motif_graph_t* graphs, int32_t count, int32_t switches_per_arc, uint64_t seed,
                    int64_t first_index, std::vector<SwitchGraph>* out, int64_t* max_n, int64_t* max_m) {
  if (switches_per_arc < 0) return MOTIF_EINVAL_ARG;
  out->clear();
  *max_n = 0;
  *max_m = 0;
  for (int32_t g = 0; g < count; ++g) {
    const motif_graph_t& G = graphs[g];
    if (!check_shape(G.n, G.m) || (G.n == 0 && G.m != 0)) return MOTIF_EINVAL_SHAPE;
    if ((G.n > 0 && !G.out_off) || (G.m > 0 && !G.out_idx)) return MOTIF_EINVAL_ARG;
    SwitchGraph sg;
    sg.off = G.out_off;
    sg.idx = const_cast<int32_t*>(G.out_idx);  // rewritten in place, as the call documents
    sg.n = G.n;
    sg.m = (int32_t)G.m;
    sg.key = switch_key(seed, first_index + g);
    sg.rounds = ((int64_t)switches_per_arc * G.m + kSwitchProposals - 1) / kSwitchProposals;
    out->push_back(sg);
    *max_n = std::max<int64_t>(*max_n, G.n);
    *max_m = std::max<int64_t>(*max_m, G.m);
  }
  return 0;
}

// Check every graph (one launch), then switch; one host wait at the end.
int32_t run_switch(Pipeline& p, const std::vector<SwitchGraph>& sg, bool mutual, hipStream_t s) {
  p.arena.reset();
  try {
    enqueue_zero(p.status, sizeof(int32_t) * kStatusWords, s);
    if (int32_t rc = enqueue_switch(p, sg.data(), (int32_t)sg.size(), mutual, s)) {
      (void)hipStreamSynchronize(s);  // best effort: the error is what the caller acts on
      return rc;
    }
  } catch (const WorkspaceError&) {
    return drain_after_error(p, s);
  }
  return read_status(p, s);
}

}  // namespace

extern "C" {

int32_t motif_null_randomize(const motif_graph_t* graphs, int32_t count, int32_t switches_per_arc, int32_t flags,
                             uint64_t seed, void* stream) {
  if (count < 0 || (count > 0 && !graphs) || (flags & ~MOTIF_SWITCH_MUTUAL)) return MOTIF_EINVAL_ARG;
  if (count == 0) return 0;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  std::vector<SwitchGraph> sg;
  int64_t max_n = 0, max_m = 0;
  if (int32_t rc = switch_list(graphs, count, switches_per_arc, seed, 0, &sg, &max_n, &max_m)) return rc;
  hipStream_t s = (hipStream_t)stream;
  Pipeline* p = nullptr;
  if (int32_t rc = get_pipeline(dev, s, switch_bytes(count, max_n, max_m, device_cus(dev)), &p)) return rc;
  return run_switch(*p, sg, (flags & MOTIF_SWITCH_MUTUAL) != 0, s);
}

int32_t motif_null_model(const motif_graph_t* real, int32_t count, int32_t k, int32_t switches_per_arc, int32_t flags,
                         uint64_t seed, uint64_t* hists, double* z, void* stream) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (!real || !hists || !z || count < 1 || switches_per_arc < 0) return MOTIF_EINVAL_ARG;
  if (flags & ~MOTIF_SWITCH_MUTUAL) return MOTIF_EINVAL_ARG;
  if (!check_shape(real->n, real->m) || (real->n == 0 && real->m != 0)) return MOTIF_EINVAL_SHAPE;
  if ((real->n > 0 && !real->out_off) || (real->m > 0 && !real->out_idx)) return MOTIF_EINVAL_ARG;
  if (real->in_off && real->m > 0 && !real->in_idx) return MOTIF_EINVAL_ARG;
  if ((int64_t)real->m * (count + 1) >= kMaxN || (int64_t)real->n * (count + 1) >= kMaxN) return MOTIF_EINVAL_SHAPE;
  int dev;
  if (int32_t rc = ensure_init(&dev)) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int C = motif_num_classes(k);
  // the randomised copies: one target array each, sharing the real graph's offsets
  int32_t* copies = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& buf = g_dev[dev].null_copies[s];
    const size_t need = sizeof(int32_t) * (size_t)std::max<int64_t>(1, real->m * count);
    if (buf.second < need) {
      if (buf.first) {
        (void)hipStreamSynchronize(s);  // a failure here shows up as a failed allocation below
        (void)hipFree(buf.first);
        buf = {nullptr, 0};
      }
      if (hipMalloc(&buf.first, need) != hipSuccess) {
        buf = {nullptr, 0};
        return MOTIF_ENOMEM;
      }
      buf.second = need;
    }
    copies = buf.first;
  }
  std::vector<motif_graph_t> all(count + 1);
  all[0] = *real;
  for (int32_t g = 1; g <= count; ++g) {
    all[g] = *real;
    all[g].out_idx = copies + (size_t)(g - 1) * (size_t)real->m;
    all[g].in_off = nullptr;  // the transpose of a randomised copy is built internally
    all[g].in_idx = nullptr;
  }
  std::vector<SwitchGraph> sg;
  int64_t max_n = 0, max_m = 0;
  if (int32_t rc = switch_list(all.data() + 1, count, switches_per_arc, seed, 0, &sg, &max_n, &max_m)) return rc;
  Pipeline* p = nullptr;
  if (int32_t rc = get_pipeline(dev, s, switch_bytes(count, max_n, max_m, device_cus(dev)), &p)) return rc;
  // 1. copy the real graph's targets into every slot, 2. randomise the slots
  enqueue_zero(p->status, sizeof(int32_t) * kStatusWords, s);
  if (real->n > 0) enqueue_check_rows(real->out_off, real->n, real->m, p->status, s);
  if (real->m > 0) enqueue_replicate(real->out_idx, real->m, count, copies, p->status, s);
  if (int32_t rc = run_switch(*p, sg, (flags & MOTIF_SWITCH_MUTUAL) != 0, s)) return rc;
  // 3. one fused census of the real graph and its copies
  int32_t rc = census_batch_with(all.data(), count + 1, k, hists, s,
                                 tuning_for_call(dev, 1, &k, true, real->m * (count + 1), real->n));
  if (rc) return rc;
  // 4. z-scores of the real graph against the copies
  enqueue_zscores(hists, C, count, z, p->status, s);
  return hipStreamSynchronize(s) == hipSuccess ? 0 : MOTIF_EDEVICE;
}

}  // extern "C"

struct motif_batch_plan {
  int dev = 0;
  hipStream_t caller = nullptr;   // the caller's stream (may be the null stream)
  hipStream_t stream = nullptr;   // private stream the graph is captured on
  hipEvent_t ready = nullptr;
  int32_t k = 0, count = 0;
  Pipeline p;
  motif_graph_t* graphs = nullptr;  // pinned copy of the descriptors
  int64_t* voff = nullptr;          // pinned
  int64_t* aoff = nullptr;          // pinned
  uint64_t* hists = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// The whole batched census (status reset, pack, build, census, division) as
// one stream-ordered sequence with no host interaction, so it can be captured.
// Returns false if a host-to-device copy could not be enqueued or the
// workspace was sized too small.
bool enqueue_plan(motif_batch_plan* b) {
  const int C = motif_num_classes(b->k);
  try {
    b->p.arena.reset();
    enqueue_zero(b->p.status, sizeof(int32_t) * kStatusWords, b->stream);
    BuildInput in = enqueue_pack(b->p, b->graphs, b->count, b->voff, b->aoff, b->stream);
    DevGraph g = enqueue_build(b->p, in, b->stream);
    uint64_t* acc = b->p.arena.take<uint64_t>((size_t)b->count * C);
    enqueue_census(b->p, g, b->k, acc, b->hists, b->stream, false);
    return !in.copy_error;
  } catch (const WorkspaceError&) {
    return false;
  }
}

void plan_free(motif_batch_plan* b) {
  if (!b) return;  // tear-down: errors change nothing a caller could act on
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->p.arena.base) (void)hipFree(b->p.arena.base);
  if (b->p.status) (void)hipFree(b->p.status);
  if (b->p.host_status) (void)hipHostFree(b->p.host_status);
  if (b->graphs) (void)hipHostFree(b->graphs);
  if (b->voff) (void)hipHostFree(b->voff);
  if (b->aoff) (void)hipHostFree(b->aoff);
  if (b->ready) (void)hipEventDestroy(b->ready);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Order the plan's private stream after everything already on the caller's.
int32_t plan_join_caller(motif_batch_plan* b) {
  if (hipEventRecord(b->ready, b->caller) != hipSuccess) return MOTIF_EDEVICE;
  if (hipStreamWaitEvent(b->stream, b->ready, 0) != hipSuccess) return MOTIF_EDEVICE;
  return 0;
}

}  // namespace

extern "C" {

motif_batch_plan_t* motif_batch_plan_create(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists,
                                            void* stream, int32_t* err) {
  int32_t dummy;
  if (!err) err = &dummy;
  *err = 0;
  if (motif_num_classes(k) < 0) { *err = MOTIF_EINVAL_K; return nullptr; }
  if (count <= 0 || !graphs || !hists) { *err = MOTIF_EINVAL_ARG; return nullptr; }
  int64_t N = 0, M = 0;
  for (int32_t g = 0; g < count; ++g) {
    const motif_graph_t& G = graphs[g];
    if (!check_shape(G.n, G.m) || (G.n == 0 && G.m != 0)) { *err = MOTIF_EINVAL_SHAPE; return nullptr; }
    if ((G.n > 0 && !G.out_off) || (G.m > 0 && !G.out_idx) || (G.in_off && G.m > 0 && !G.in_idx)) {
      *err = MOTIF_EINVAL_ARG;
      return nullptr;
    }
    N += G.n;
    M += G.m;
  }
  if (N == 0 || N >= kMaxN || M >= kMaxN) { *err = N == 0 ? MOTIF_EINVAL_ARG : MOTIF_EINVAL_SHAPE; return nullptr; }
  int dev;
  if ((*err = ensure_init(&dev))) return nullptr;
  motif_batch_plan* b = new motif_batch_plan();
  b->dev = dev;
  b->caller = (hipStream_t)stream;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess) {
    *err = MOTIF_EDEVICE;
    plan_free(b);
    return nullptr;
  }
  b->k = k;
  b->count = count;
  b->hists = hists;
  b->p.num_cus = device_cus(dev);
  int64_t maxn = 0;
  for (int32_t g = 0; g < count; ++g) maxn = std::max<int64_t>(maxn, graphs[g].n);
  b->p.tune = tuning_for_call(dev, 1, &k, count > 1, M, maxn);
  const size_t bytes = pipeline_bytes(N, M, count, true, k, b->p.num_cus, maxn, b->p.tune.k[k]);
  if (hipMalloc(&b->p.arena.base, bytes) != hipSuccess || hipMalloc(&b->p.status, kStatusWords * 4) != hipSuccess ||
      hipHostMalloc(&b->p.host_status, kStatusWords * 4, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&b->graphs, sizeof(motif_graph_t) * count, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&b->voff, sizeof(int64_t) * (count + 1), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&b->aoff, sizeof(int64_t) * (count + 1), hipHostMallocDefault) != hipSuccess) {
    *err = MOTIF_ENOMEM;
    plan_free(b);
    return nullptr;
  }
  b->p.arena.cap = bytes;
  std::memcpy(b->graphs, graphs, sizeof(motif_graph_t) * count);
  b->voff[0] = b->aoff[0] = 0;
  for (int32_t g = 0; g < count; ++g) {
    b->voff[g + 1] = b->voff[g] + graphs[g].n;
    b->aoff[g + 1] = b->aoff[g] + graphs[g].m;
  }
  // 1. eager run: validates the inputs and reports their error code
  if ((*err = plan_join_caller(b))) {
    plan_free(b);
    return nullptr;
  }
  const bool copied = enqueue_plan(b);
  *err = read_status(b->p, b->stream);
  if (!*err && !copied) *err = MOTIF_EDEVICE;
  if (*err) {
    plan_free(b);
    return nullptr;
  }
  // 2. capture the same sequence (profiling events stay out of the graph)
  const bool prof = g_prof.on;
  g_prof.on = false;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const bool ok = enqueue_plan(b);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (!ok && e == hipSuccess) e = hipErrorUnknown;
  }
  g_prof.on = prof;
  if (e != hipSuccess || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    *err = MOTIF_EDEVICE;
    plan_free(b);
    return nullptr;
  }
  return b;
}

int32_t motif_batch_plan_run(motif_batch_plan_t* b) {
  if (!b) return MOTIF_EINVAL_ARG;
  if (int32_t rc = plan_join_caller(b)) return rc;
  if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return MOTIF_EDEVICE;
  return read_status(b->p, b->stream);
}

int32_t motif_batch_plan_destroy(motif_batch_plan_t* b) {
  if (!b) return MOTIF_EINVAL_ARG;
  plan_free(b);
  return 0;
}

int32_t motif_profile_enable(int32_t on) {
  if (on < 0 || on > 2) return MOTIF_EINVAL_ARG;
  g_prof.on = on != 0;
  g_prof.build = on == 1;
  for (bool& h : g_prof.have) h = false;
  for (bool& h : g_prof.have_build) h = false;
  return 0;
}

int32_t motif_profile_read(int32_t k, float* kernel_ms, float* build_ms) {
  if (k < 3 || k > 5) return MOTIF_EINVAL_K;
  if (!g_prof.have[k]) return MOTIF_EINVAL_ARG;
  hipEvent_t* e = g_prof.ev[k];
  if (hipEventSynchronize(e[3]) != hipSuccess) return MOTIF_EDEVICE;
  if (kernel_ms && hipEventElapsedTime(kernel_ms, e[2], e[3]) != hipSuccess) return MOTIF_EDEVICE;
  if (build_ms) {
    if (!g_prof.have_build[k]) *build_ms = -1.0f;
    else if (hipEventElapsedTime(build_ms, e[0], e[1]) != hipSuccess) return MOTIF_EDEVICE;
  }
  return 0;
}

}  // extern "C"
