/*
 * motif.h -- C ABI of the MI355X (gfx950) exact directed motif census.
 *
 * What is computed (paper, Section "Problem statement", Problems Motifs-3,
 * Motifs-4 and Motifs-5): for a simple directed graph G and k in {3,4,5}, the
 * number of k-vertex subsets S whose induced subgraph is weakly connected
 * (connected in the undirected version G*, Section "Notation and
 * definitions"), grouped by the isomorphism class of the induced digraph G[S]
 * into 13, 199 or 9364 classes.  Counts are exact unsigned 64-bit integers.
 *
 * How (paper, "combinatorial acceleration"): every k-set is charged to the
 * anchors that see it -- a vertex (v-Patterns, Theorem "teo3"), an undirected
 * edge (e-Patterns, Theorem "lema4d" and its corollary) or a connected triple
 * (Delta-Patterns, Lemma "lema5d") -- using closed forms for neighbour pairs
 * with no edge between them (Facts "base"/"basefive") and edge counts between
 * the neighbour sets for the rest; each class total is finally divided by the
 * number of anchors that see one occurrence (Fact "correction").
 *
 * Class numbering.  The paper leaves positions arbitrary.  Here: for k
 * vertices the arc i->j (i != j) is bit  i*(k-1) + (j < i ? j : j-1)  of a
 * k(k-1)-bit code; the canonical code of a digraph is the minimum code over
 * all k! relabellings; class ids are the ranks of the canonical codes of the
 * weakly connected classes in ascending order.  motif_class_code() returns the
 * canonical code of a class so callers can map ids to other tools' numbering.
 *
 * Conventions for every entry point:
 *  - Return 0 on success, a negative MOTIF_E* code on error.  On error no
 *    output buffer is written.
 *  - Graphs are int32 out-CSR: the arcs of vertex u are u -> out_idx[j] for
 *    out_off[u] <= j < out_off[u+1].  n < 2^30 and m < 2^30 (a larger n or m
 *    returns MOTIF_EINVAL_SHAPE): a vertex id shares one 32-bit word with its
 *    two type bits in the typed undirected rows, and the 2m half-edges of
 *    those rows are addressed by int32 offsets.
 *  - Device pointers are hipMalloc'ed (or torch CUDA) memory owned by the
 *    caller; the library never frees them.  The library owns its internal
 *    workspaces and class tables (device memory), released by
 *    motif_shutdown().
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it.  motif_census(), motif_census_multi() and the batch calls then
 *    wait for that stream once, at the end, so that an invalid graph or a
 *    failed self-check is reported by the return code; the histogram is
 *    complete when they return.  motif_census_async() does not wait: it
 *    reports the outcome through a device status word instead.
 *  - Thread safety: calls on different streams may run concurrently (each
 *    stream gets its own workspace); calls on the same stream are ordered.
 */
#ifndef MOTIF_H_
#define MOTIF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define MOTIF_OK 0
#define MOTIF_EINVAL_K (-1)      /* k not in {3,4,5}                                  */
#define MOTIF_EINVAL_SHAPE (-2)  /* n/m out of range, offsets not monotone,
                                    out_off[0] != 0 or out_off[n] != m                */
#define MOTIF_EINDEX (-3)        /* a neighbour index outside [0, n)                   */
#define MOTIF_ESELFLOOP (-4)     /* an arc u -> u                                     */
#define MOTIF_EDUP (-5)          /* the same arc listed twice                          */
#define MOTIF_ETRANSPOSE (-6)    /* the in-CSR given is not the transpose of out-CSR  */
#define MOTIF_ENOMEM (-7)        /* device or host allocation failed                  */
#define MOTIF_EDEVICE (-8)       /* a HIP runtime call failed / no gfx950 device      */
#define MOTIF_EAGAIN (-9)        /* server: not admitted now (memory or slots busy)   */
#define MOTIF_ETOOBIG (-10)      /* server: request can never fit the HBM budget      */
#define MOTIF_ETIMEOUT (-11)     /* server: wait timed out                             */
#define MOTIF_ECANCELED (-12)    /* server: request was cancelled                      */
#define MOTIF_EINVAL_ARG (-13)   /* other bad argument (NULL pointer, bad count...)   */
#define MOTIF_EINTERNAL (-14)    /* self-check failed: a class total was not an exact
                                    multiple of its anchor multiplicity               */
#define MOTIF_EPARSE (-15)       /* network file: malformed line or id out of range    */
#define MOTIF_EIO (-16)          /* network file: cannot be opened or read             */

/* One graph in int32 CSR.  in_off/in_idx may be NULL (the transpose is built
 * internally); when given they must describe exactly the transpose of the
 * out-CSR (rows in any order).  For motif_census_batch() all pointers are
 * device pointers; for motif_server_submit() they are host pointers. */
typedef struct motif_graph {
  const int32_t* out_off; /* [n+1] */
  const int32_t* out_idx; /* [m]   */
  const int32_t* in_off;  /* [n+1] or NULL */
  const int32_t* in_idx;  /* [m]   or NULL */
  int32_t n;
  int64_t m;
} motif_graph_t;

/* ---- library state and class tables (host) ------------------------------- */

/* Builds the class tables for k = 3, 4, 5 on the host (code -> class, class
 * multiplicities) and uploads them to the current device.  Idempotent; called
 * implicitly by the census entry points.  Returns MOTIF_EDEVICE when no gfx950
 * device is present; the host-only helpers below still work then. */
int32_t motif_init(void);

/* Frees every device buffer the library owns (tables, workspaces). */
int32_t motif_shutdown(void);

/* 13, 199 or 9364 (paper, Problems Motifs-3/4/5); MOTIF_EINVAL_K otherwise. */
int32_t motif_num_classes(int32_t k);

/* Canonical k(k-1)-bit code of class `cls` (see "Class numbering" above).
 * Host-only; needs no device. */
int32_t motif_class_code(int32_t k, int32_t cls, uint32_t* canon_code);

/* Number of anchors that see one occurrence of class `cls`: vertices for k=3
 * (1 for an open wedge, 3 for a triangle: Algorithm "Count 3 Sized Patterns"),
 * undirected edges for k=4 (1/3/3/4/5/6 for P4/claw/tailed triangle/C4/
 * K4-minus-edge/K4, Fact "correction"), connected triples for k=5 (5 for the
 * 5-cycle, Figure "correction:five").  It is the number of connected
 * (k-2)-subsets that dominate the other two vertices.  Host-only.  Returns the
 * multiplicity (>= 1) or a negative error code. */
int32_t motif_class_multiplicity(int32_t k, int32_t cls);

/* Class id of an arbitrary k(k-1)-bit code, or -1 when the code's undirected
 * version is disconnected.  Host-only. */
int32_t motif_class_of_code(int32_t k, uint32_t code);

/* Undirected classes: the connected undirected graphs on k vertices, 2, 6 or
 * 21 for k = 3, 4, 5 (the undirected censuses of the paper, Sections
 * "Counting isomorphic patterns of size 4" (Table "ept") and "Counting
 * 5-sized patterns in undirected graphs").  Numbering: the edge {i, j},
 * i < j, is bit i(2k - i - 1)/2 + (j - i - 1) of a k(k-1)/2-bit code; the
 * canonical code is the minimum over all k! relabellings; class ids are the
 * ranks of the canonical codes of connected graphs, ascending.  Host-only. */
int32_t motif_num_undirected_classes(int32_t k);
int32_t motif_undirected_class_code(int32_t k, int32_t cls, uint32_t* canon_code);
/* Undirected class of directed class `cls` when every arc of its pattern is
 * reciprocated, else -1.  Host-only. */
int32_t motif_class_undirected(int32_t k, int32_t cls);

/* Static description of an error code. */
const char* motif_strerror(int32_t code);

/* ---- reading networks (host) ----------------------------------------------- */

#define MOTIF_FORMAT_AUTO 0       /* Pajek for a ".net" file name, else edge list      */
#define MOTIF_FORMAT_PAJEK 1
#define MOTIF_FORMAT_EDGE_LIST 2
#define MOTIF_READ_UNDIRECTED 1   /* edge list: each line is an undirected edge        */
#define MOTIF_READ_KEEP_ISOLATED 2 /* Pajek: keep the vertices of degree zero          */

typedef struct motif_read_stats {
  int64_t lines;              /* lines read                                          */
  int64_t arcs_read;          /* arcs listed (an undirected edge counts twice)       */
  int64_t self_loops_dropped; /* arcs u -> u                                          */
  int64_t duplicates_merged;  /* arcs listed more than once                          */
  int64_t isolated_dropped;   /* Pajek vertices with no neighbour, removed            */
} motif_read_stats_t;

/* Reads a network file into a HOST int32 out-CSR, as the paper prepares its
 * instances (Section "Results and Discussion": networks from public Pajek
 * and edge-list collections, vertices with no neighbours removed).
 *  Pajek: "*Vertices N" then "*Arcs" / "*Edges" ("u v [w]"), "*Arcslist" /
 *         "*Edgeslist" ("u v1 v2 ..."), or "*Matrix" sections; 1-based ids;
 *         an edge is both arcs; other sections are skipped; "%" comments.
 *  Edge list: "u v [anything]" per line, ids >= 0, each line the arc u -> v
 *         (both arcs with MOTIF_READ_UNDIRECTED); "#" or "%" comments.
 * Self-loops are dropped and repeated arcs merged (the census takes simple
 * digraphs); the vertices that keep a neighbour are renumbered 0..n-1 in the
 * order of their ids in the file; rows come out sorted.  *out_off ([n+1]),
 * *out_idx ([m], at least one entry) and, when orig_ids is not NULL,
 * *orig_ids ([n]: file id of each vertex, 0-based for Pajek) are malloc'ed
 * by the library; free them with motif_free().  stats may be NULL.  Errors:
 * MOTIF_EIO, MOTIF_EPARSE, MOTIF_EINVAL_ARG, MOTIF_EINVAL_SHAPE (n or m of
 * 2^30 or more), MOTIF_ENOMEM; nothing is returned through the pointers on
 * error.  Host-only; needs no device. */
int32_t motif_read_network(const char* path, int32_t format, int32_t flags, int32_t* n, int64_t* m,
                           int32_t** out_off, int32_t** out_idx, int64_t** orig_ids, motif_read_stats_t* stats);

/* Frees memory returned by motif_read_network(). */
void motif_free(void* p);

/* ---- census --------------------------------------------------------------- */

/* Exact census of one graph (paper, Algorithms "Count 3/4/5 Sized Patterns").
 *  out_off, out_idx : device, the graph (rows need not be sorted).
 *  in_off, in_idx   : device or both NULL; validated against the out-CSR.
 *  n, m             : vertex and arc counts.
 *  k                : 3, 4 or 5.
 *  hist             : device, motif_num_classes(k) uint64, overwritten.
 * Validation errors: MOTIF_EINVAL_SHAPE, MOTIF_EINDEX, MOTIF_ESELFLOOP,
 * MOTIF_EDUP, MOTIF_ETRANSPOSE.  n < k or m = 0 gives an all-zero histogram. */
int32_t motif_census(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off,
                     const int32_t* in_idx, int32_t n, int64_t m, int32_t k, uint64_t* hist,
                     void* stream);

/* Asynchronous form of motif_census() (same arguments and result), for callers
 * that synchronise the stream themselves.  Returns 0 once everything is
 * enqueued on `stream`, or an error found on the host before any work was
 * enqueued (MOTIF_EINVAL_K, MOTIF_EINVAL_SHAPE, MOTIF_EINVAL_ARG,
 * MOTIF_ENOMEM, MOTIF_EDEVICE).
 *  status : device, one int32 owned by the caller; written on `stream` after
 *           the census with 0 or the validation / self-check error code.
 *  hist   : written (on `stream`) only when the status is 0.
 * The stream's workspace is reused by the next call on the same stream, which
 * runs after this one in stream order; the caller keeps the input buffers
 * alive until it has synchronised. */
int32_t motif_census_async(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off,
                           const int32_t* in_idx, int32_t n, int64_t m, int32_t k, uint64_t* hist,
                           int32_t* status, void* stream);

/* Allocation-free form of motif_census(), for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, result and errors as
 * motif_census(); it calls no allocating routine.  Its workspace is a fixed
 * 128 MiB device array of the library (every device the library is set up on
 * holds it until the process ends); motif_init() must have run on the current
 * device first, else MOTIF_EDEVICE.  A graph whose workspace does not fit
 * returns MOTIF_ETOOBIG before any work is enqueued; for k = 4, 5 the
 * per-anchor scheme (no per-workgroup tables) is used when the default
 * scheme's workspace does not fit.  Calls on one device share the array:
 * they are serialised by a lock and each returns only after its work on
 * `stream` has finished, so they never overlap in it. */
int32_t motif_census_noalloc(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off,
                             const int32_t* in_idx, int32_t n, int64_t m, int32_t k, uint64_t* hist,
                             void* stream);

/* Undirected census: the connected k-vertex induced subgraphs of the
 * undirected version G* of the graph (u, v adjacent when u -> v or v -> u is
 * listed), grouped into the motif_num_undirected_classes(k) classes above.
 * An undirected graph may be given with each edge listed once or in both
 * directions.  Same pipeline as motif_census() with every edge of G* read as
 * a pair of arcs, then the all-reciprocated directed classes summed into
 * undirected ones.  hist: device, motif_num_undirected_classes(k) uint64.
 * Errors as for motif_census(). */
int32_t motif_census_undirected(const int32_t* out_off, const int32_t* out_idx, int32_t n, int64_t m, int32_t k,
                                uint64_t* hist, void* stream);

/* Census of one graph for several sizes: ks[0..nk) are distinct values of
 * {3, 4, 5} and hists[i] (device, motif_num_classes(ks[i]) uint64) receives
 * exactly what motif_census(..., ks[i], hists[i], ...) would write.  The
 * validation and the G* / N+ build run once and are shared (the paper's
 * motif profiles use several sizes of one network, Section "Results and
 * Discussion").  The largest size runs on `stream`, the others on a second
 * stream owned by the library, forked after the build; both are joined
 * before the call returns, so on return the work on `stream` includes all
 * of it.  `g` holds device pointers; errors as for motif_census(): on any
 * validation error no histogram is written; a self-check failure
 * (MOTIF_EINTERNAL) of one size may leave the other sizes written. */
int32_t motif_census_multi(const motif_graph_t* g, int32_t nk, const int32_t* ks, uint64_t* const* hists,
                           void* stream);

/* Census of `count` graphs in one fused pass: the graphs are packed into one
 * disjoint union on the device, built once, and censused by one persistent
 * kernel that pulls anchor tiles from a device work queue; each tile's counts
 * are routed to its own graph's histogram.  hists: device, count *
 * motif_num_classes(k) uint64 (graph g at offset g*C).  hists[g] equals
 * motif_census() on graph g alone, bit for bit.  `graphs` is a host array of
 * descriptors holding device pointers.  Used for null-model ensembles of
 * degree-preserving randomisations (paper, Section "Implementation", step
 * (iii); Section "Results and Discussion", random-graph ensembles). */
int32_t motif_census_batch(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists,
                           void* stream);

/* Same result as motif_census_batch() by the plain route: one motif_census()
 * pipeline per graph, enqueued back to back on `stream`.  Kept as the
 * baseline the fused launch is measured against. */
int32_t motif_census_batch_loop(const motif_graph_t* graphs, int32_t count, int32_t k,
                                uint64_t* hists, void* stream);

/* Reusable fused batch ("plan") for repeated censuses of the same batch
 * layout -- e.g. a null-model ensemble whose graphs are regenerated in place
 * on the device between rounds.  create(): validates and censuses the batch
 * once eagerly (on error returns NULL and sets *err), then captures the whole
 * device sequence (pack, build, census, exact division) into a hipGraph on a
 * private stream of the plan.  run(): orders itself after the work already
 * enqueued on `stream`, replays that graph -- one launch -- and waits for the
 * status word; it reads whatever the graph buffers hold at that moment, so
 * new graphs of identical n and m per slot may be written in place between
 * runs.  The descriptors are copied at create(); the device buffers they
 * point to and `hists` must outlive the plan.  Not thread-safe per plan. */
typedef struct motif_batch_plan motif_batch_plan_t;
motif_batch_plan_t* motif_batch_plan_create(const motif_graph_t* graphs, int32_t count, int32_t k,
                                            uint64_t* hists, void* stream, int32_t* err);
int32_t motif_batch_plan_run(motif_batch_plan_t* plan);
int32_t motif_batch_plan_destroy(motif_batch_plan_t* plan);

/* ---- motifs of size 6 ------------------------------------------------------ */

/* The paper's method taken to k = 6, its stated extension to larger motifs
 * (Section "Our approach"): anchors are the connected 4-sets (as edges anchor
 * k = 4 and connected triples k = 5), each other vertex adjacent to the
 * anchor is labelled by its types towards the four anchor vertices, label
 * pairs are counted in closed form and every edge between two labelled
 * vertices moves one occurrence to its class; a 6-set is seen once per
 * connected 4-subset that dominates its other two vertices, which the exact
 * division removes.
 * Classes: the 1,530,843 weakly connected digraphs on 6 vertices, numbered as
 * for k <= 5 (arc i->j at bit 5i + (j < i ? j : j - 1) of a 30-bit code,
 * canonical = minimum over the 720 relabellings, ids = ranks of the
 * canonical codes).  The class table is built on the device on first use
 * (a few seconds; it keeps 4 GiB of device memory until motif_shutdown). */
#define MOTIF_NUM_CLASSES6 1530843

/* Census of the connected 6-sets of a simple digraph (arguments as for
 * motif_census; hist: device, MOTIF_NUM_CLASSES6 uint64).  Research-grade:
 * the connected 4-sets are listed first (16 bytes each, device memory), so
 * the graph's connected 4-sets must number below 2^31; an anchor edge whose
 * ends have more than 1,024 neighbours in all, or an anchor with more than
 * 4,096 labelled vertices, returns MOTIF_ETOOBIG.  Waits for the stream.
 * Errors as for motif_census, plus MOTIF_ETOOBIG and MOTIF_ENOMEM. */
int32_t motif_census6(const int32_t* out_off, const int32_t* out_idx, const int32_t* in_off, const int32_t* in_idx,
                      int32_t n, int64_t m, uint64_t* hist, void* stream);

/* Host copies of the k = 6 class table: the canonical code of every class
 * (codes: host, MOTIF_NUM_CLASSES6 uint32, increasing) and its multiplicity
 * (mult: host, MOTIF_NUM_CLASSES6 bytes: connected 4-subsets dominating the
 * other two vertices).  Build the table on the current device if needed. */
int32_t motif_class6_codes(uint32_t* codes);
int32_t motif_class6_multiplicities(uint8_t* mult);

/* ---- null-model ensembles on the device ------------------------------------ */

/* flags of the null-model calls */
#define MOTIF_SWITCH_MUTUAL 1 /* also keep every vertex's numbers of reciprocated,
                                 one-way-out and one-way-in neighbours        */

/* Degree-preserving randomisation of `count` graphs in place (the random
 * graphs of the paper's significance step (iii), Section "Implementation";
 * its ensembles in Section "Results and Discussion").  `graphs` is a host
 * array of descriptors holding DEVICE pointers; each graph's out_idx is
 * REWRITTEN (the const in motif_graph_t notwithstanding): switches_per_arc * m
 * attempted arc switches, each taking two arcs a->b, c->d and rewiring them
 * to a->d, c->b unless that makes a self-loop or a repeated arc.  Every arc
 * keeps its slot in its source's row, so out_off and all out- and in-degrees
 * are unchanged; rows are left unsorted; in_off/in_idx are ignored (the
 * graph's transpose changes).
 * flags = MOTIF_SWITCH_MUTUAL: one-way arcs are switched only with one-way
 * arcs (and only if no arc joins a and d, or c and b, in either direction),
 * reciprocated pairs only with reciprocated pairs (a<->b, c<->d become
 * a<->d, c<->b), so the numbers of reciprocated and one-way neighbours of
 * every vertex are kept as well.  Either way the chain's stationary
 * distribution is uniform over the graphs it can reach.
 * The input must be a simple digraph (rows may be unsorted); repeated arcs
 * are not detected here and leave the result unspecified.
 * Random numbers: SplitMix64 on a counter, one stream per (seed, graph
 * index), so the result depends only on the input, switches_per_arc, flags
 * and seed.  Errors (nothing is rewritten): MOTIF_EINVAL_SHAPE (offsets not
 * monotone from 0 to m), MOTIF_EINDEX (a target outside [0, n)),
 * MOTIF_ESELFLOOP, MOTIF_EINVAL_ARG (unknown flags).  Waits for the stream. */
int32_t motif_null_randomize(const motif_graph_t* graphs, int32_t count, int32_t switches_per_arc, int32_t flags,
                             uint64_t seed, void* stream);

/* The whole null-model job on the device: `count` randomisations of the real
 * graph (device pointers; its in-CSR, if given, is validated for the real
 * graph), each made as by motif_null_randomize(real copy, switches_per_arc,
 * flags, seed; graph i uses stream i of seed), then one fused census of the real
 * graph and its copies (motif_census_batch), then the z-scores.
 *  hists : device, (count + 1) * motif_num_classes(k) uint64; row 0 is the
 *          real graph, row i the i-th randomisation.
 *  z     : device, motif_num_classes(k) doubles: (h_real - mean) / sd over the
 *          copies, sample sd (ddof = 1), from exact integer sums; NaN where the
 *          sd is 0, count < 2, or a count of the class reaches 2^40.
 * The library keeps a device buffer of count * m int32 per stream for the
 * copies.  Errors as for motif_census() and motif_null_randomize(). */
int32_t motif_null_model(const motif_graph_t* real, int32_t count, int32_t k, int32_t switches_per_arc,
                         int32_t flags, uint64_t seed, uint64_t* hists, double* z, void* stream);

/* ---- tuning ---------------------------------------------------------------- */

/* Tunable launch parameters of the census kernels. */
typedef struct motif_tuning {
  int32_t block;        /* threads per workgroup for the anchor kernels (64..1024)  */
  int32_t grid_per_cu;  /* persistent workgroups per compute unit (1..16)           */
  int32_t tile;         /* work-queue granularity (1..4096): G* entries per tile,
                           except for the k = 4 and k = 5 core-reuse schemes,
                           where the queue is cut by estimated cost into about
                           `tile` tiles per workgroup (fewer on small graphs:
                           a tile holds at least 128 (k = 4) or 512 (k = 5)
                           cost units)                                         */
  int32_t heavy;        /* census scheme for k = 4, 5: 1 = core reuse (neighbourhood
                           of the highest-ranked anchor vertex scanned once per
                           work unit), 2 = per-anchor scan; 0 = keep              */
  /* Work placement of the core-reuse schemes (degrees in the undirected
   * graph G*); they move work between waves and workgroups, never change
   * the result. */
  int32_t solo_deg;     /* k = 4: a core (higher-ranked anchor end) of at most this
                           degree runs whole anchors on one wave (1..64)        */
  int32_t light_deg;    /* k = 4: an anchor whose other end has at most this
                           degree runs on one wave, else on the workgroup
                           (1..256)                                             */
  int32_t light5;       /* k = 5: a triple whose lighter side has at most this
                           degree takes the factored wave path (1..767)         */
} motif_tuning_t;

/* Read / override the default parameters for k (0 in a field = keep).
 * Setting them also drops the autotuner's cached entries for k.  Fused
 * censuses of more than one graph at k = 4, each of at most 16,384 vertices,
 * start from their own default (block 512, grid 2 per CU, tile 16, solo 32,
 * light 256: many small cores) until k's parameters are set here;
 * motif_get_tuning reads the single-graph defaults. */
int32_t motif_get_tuning(int32_t k, motif_tuning_t* out);
int32_t motif_set_tuning(int32_t k, const motif_tuning_t* in);

/* Autotuner: times the fused batch census of `graphs` (device pointers, as for
 * motif_census_batch; count = 1 tunes the single-graph path) under candidate
 * tunings -- a coordinate descent, two passes, over block, grid, tile, the
 * census scheme and the work-placement limits -- each candidate timed as the
 * median of 3 runs after a warm-up.  The fastest is cached for (this device,
 * k, batch or single graph, floor(log2(total arcs))) and used by every later
 * call that falls in that bucket; it is also written to *best.  `hists` is
 * scratch output (count * C uint64, device).  Every candidate's histograms
 * are checked equal to the first candidate's; a mismatch returns
 * MOTIF_EINTERNAL. */
int32_t motif_autotune(const motif_graph_t* graphs, int32_t count, int32_t k, uint64_t* hists,
                       void* stream, motif_tuning_t* best);

/* Save the autotuner cache as text (one line per entry, keyed by the
 * device's architecture name and compute-unit count) / load such a file into
 * the cache of the current device: entries of another device kind or with
 * out-of-range values are skipped.  load returns the number of entries taken
 * (>= 0) or an error code; save returns 0 or MOTIF_EINVAL_ARG (file error). */
int32_t motif_tune_cache_save(const char* path);
int32_t motif_tune_cache_load(const char* path);

/* ---- measurement ------------------------------------------------------------ */

/* on = 1: every census call records HIP events on its stream around the G*
 * build and around the main census kernel of k.  on = 2: around the census
 * kernel only (two events per size, so that timing a step perturbs it as
 * little as possible).  on = 0: off (the default).  Other values:
 * MOTIF_EINVAL_ARG. */
int32_t motif_profile_enable(int32_t on);

/* Durations in ms of the census kernel and of the build in the most recent
 * profiled call for k (waits for those events); *build_ms = -1 when that call
 * recorded no build events.  MOTIF_EINVAL_ARG if none. */
int32_t motif_profile_read(int32_t k, float* kernel_ms, float* build_ms);

/* ---- serving ---------------------------------------------------------------- */

/* Continuous-batching census server on the current device.  Requests arrive
 * with host CSR buffers; the server copies each graph into device memory it
 * owns, admits a request only while the summed device footprint of admitted
 * requests stays within hbm_budget_bytes and fewer than max_inflight requests
 * are on the device, runs admitted requests concurrently on separate HIP
 * streams (new requests start while others are still running) and copies each
 * histogram back to the caller's host buffer. */
typedef struct motif_server motif_server_t;

/* Returns NULL on failure (no device, bad arguments). */
motif_server_t* motif_server_create(size_t hbm_budget_bytes, int32_t max_inflight);

/* Device bytes a request for this graph and k would hold while admitted. */
int64_t motif_request_footprint(int32_t n, int64_t m, int32_t k);

/* Queue one request.  `g` holds HOST pointers; they are copied before this
 * call returns, so the caller may reuse them.  hist_out_host must stay valid
 * until the request completes (motif_server_wait returns) or is cancelled.
 * Returns MOTIF_ETOOBIG if the footprint exceeds the budget, MOTIF_EAGAIN if
 * the pending queue is full.  *ticket identifies the request. */
int32_t motif_server_submit(motif_server_t* s, const motif_graph_t* g, int32_t k,
                            uint64_t* hist_out_host, uint64_t* ticket);

/* Wait for a request.  timeout_us < 0 waits forever.  Returns the request's
 * own status (0 or a census error code), MOTIF_ETIMEOUT, or MOTIF_ECANCELED.
 * After a non-timeout return the ticket is released. */
int32_t motif_server_wait(motif_server_t* s, uint64_t ticket, int64_t timeout_us);

/* Cancel a request that has not started on the device yet (returns 0), or
 * MOTIF_EAGAIN if it is already running (it will complete normally). */
int32_t motif_server_cancel(motif_server_t* s, uint64_t ticket);

/* Server counters: completed requests, currently admitted requests, bytes
 * admitted, peak bytes admitted. */
int32_t motif_server_stats(motif_server_t* s, int64_t* completed, int64_t* inflight,
                           int64_t* bytes_inflight, int64_t* peak_bytes);

/* Drains outstanding work and frees everything the server owns. */
int32_t motif_server_destroy(motif_server_t* s);

#ifdef __cplusplus
}
#endif

#endif /* MOTIF_H_ */
