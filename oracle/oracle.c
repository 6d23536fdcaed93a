/*
 * CPU oracle for the exact directed motif census -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code, header, table or constant with the GPU
 * library: it computes the census from its plain definition.
 *
 * Definition (paper, Section "Problem statement", Problems Motifs-3/4/5, with
 * the undirected version G* of Section "Notation and definitions"):
 *   hist[c] = #{ S subset V : |S| = k, G*[S] connected, class(G[S]) = c }
 * where "connected" is weak connectivity (connectivity of G*) and class(H) is
 * the isomorphism class of the induced digraph H.
 *
 * Class numbering (the paper fixes none; it says positions are arbitrary and
 * hard coded, Algorithms "Count 3/4/5 Sized Patterns"): for k vertices, the
 * arc i->j (i != j) is bit  i*(k-1) + (j < i ? j : j-1)  of a k(k-1)-bit code.
 * canon(x) = min over all k! vertex permutations of the permuted code.  Class
 * id = rank of canon(x) among the distinct canonical codes of weakly connected
 * codes, ascending.
 *
 * Enumeration: ESU (Wernicke's exact subgraph enumeration, the algorithm of
 * the FANMOD tool the paper compares against): every connected k-subset is
 * emitted exactly once; its code is built over its vertices sorted by id and
 * mapped through the class table.
 *
 * Multiplicity (used only to test the GPU's final division): for a k-vertex
 * pattern, the number of (k-2)-subsets T whose G*[T] is connected and which
 * dominate the rest (every vertex outside T is adjacent to a vertex of T).
 * This is the number of anchors -- a vertex for k=3 (v-Patterns), an edge for
 * k=4 (e-Patterns, Fact "correction"), a connected triple for k=5
 * (Delta-Patterns), a connected 4-set for k=6 -- whose pattern set contains
 * the k-set.
 *
 * k = 6 (the paper's stated extension to larger motifs, Section "Our
 * approach"): 2^30 codes are too many for a brute-force class table, so the
 * k = 6 census (oracle_census6) reports each class by its canonical code
 * (minimum over the 720 relabellings, computed for each distinct code met,
 * and remembered), with the number of connected 6-sets of that class.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

static int bitpos(int k, int i, int j) { return i * (k - 1) + (j < i ? j : j - 1); }

/* All k! permutations of 0..k-1 in lexicographic order. */
static int all_perms(int k, int* out /* [k! * k] */) {
    int p[8], cnt = 0;
    for (int i = 0; i < k; ++i) p[i] = i;
    for (;;) {
        memcpy(out + cnt * k, p, sizeof(int) * k);
        ++cnt;
        int i = k - 2;
        while (i >= 0 && p[i] > p[i + 1]) --i;
        if (i < 0) break;
        int j = k - 1;
        while (p[j] < p[i]) --j;
        int t = p[i]; p[i] = p[j]; p[j] = t;
        for (int a = i + 1, b = k - 1; a < b; ++a, --b) { t = p[a]; p[a] = p[b]; p[b] = t; }
    }
    return cnt;
}

/* Code of the relabelled digraph: arc i->j becomes arc perm[i]->perm[j]. */
static uint32_t permute_code(int k, uint32_t code, const int* perm) {
    uint32_t out = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (i != j && ((code >> bitpos(k, i, j)) & 1u))
                out |= 1u << bitpos(k, perm[i], perm[j]);
    return out;
}

/* Weak connectivity of the k-vertex digraph with this code (DFS on G*). */
static int code_connected(int k, uint32_t code) {
    int adj[8][8] = {{0}};
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (i != j && ((code >> bitpos(k, i, j)) & 1u)) adj[i][j] = adj[j][i] = 1;
    int seen[8] = {0}, stack[8], sp = 0, nseen = 1;
    seen[0] = 1; stack[sp++] = 0;
    while (sp) {
        int a = stack[--sp];
        for (int b = 0; b < k; ++b)
            if (adj[a][b] && !seen[b]) { seen[b] = 1; ++nseen; stack[sp++] = b; }
    }
    return nseen == k;
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}

/*
 * Brute-force class table: cls_of_code[x] for every x in [0, 2^(k(k-1))),
 * 0xFFFF for codes whose G* is disconnected.  canon_of_class[c] receives the
 * canonical code of class c (room for 16384 entries).  Also reports the number
 * of isomorphism classes of all digraphs and the number of connected codes.
 */
int oracle_class_table(int k, uint16_t* cls_of_code, uint32_t* canon_of_class,
                       int32_t* n_classes, int32_t* n_all_classes, int64_t* n_connected_codes) {
    if (k < 2 || k > 5) return OR_EINVAL;
    const int nb = k * (k - 1);
    const uint32_t N = 1u << nb;
    int perms[120 * 5];
    const int np = all_perms(k, perms);
    uint32_t* canon = (uint32_t*)malloc(sizeof(uint32_t) * N);
    uint8_t* conn = (uint8_t*)malloc(N);
    if (!canon || !conn) { free(canon); free(conn); return OR_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t x = 0; x < (int64_t)N; ++x) {
        uint32_t best = (uint32_t)x;
        for (int p = 0; p < np; ++p) {
            uint32_t y = permute_code(k, (uint32_t)x, perms + p * k);
            if (y < best) best = y;
        }
        canon[x] = best;
        conn[x] = (uint8_t)code_connected(k, (uint32_t)x);
    }
    /* distinct canonical codes: those x with canon[x] == x */
    int32_t all = 0, nc = 0;
    int64_t ncodes = 0;
    uint32_t* reps = (uint32_t*)malloc(sizeof(uint32_t) * 16384);
    if (!reps) { free(canon); free(conn); return OR_ENOMEM; }
    for (uint32_t x = 0; x < N; ++x) {
        if (conn[x]) ++ncodes;
        if (canon[x] == x) {
            ++all;
            if (conn[x]) { if (nc < 16384) reps[nc] = x; ++nc; }
        }
    }
    qsort(reps, (size_t)nc, sizeof(uint32_t), cmp_u32);
    for (uint32_t x = 0; x < N; ++x) {
        if (!conn[x]) { cls_of_code[x] = 0xFFFF; continue; }
        uint32_t c = canon[x];
        int lo = 0, hi = nc - 1;
        while (lo < hi) { int mid = (lo + hi) / 2; if (reps[mid] < c) lo = mid + 1; else hi = mid; }
        cls_of_code[x] = (uint16_t)lo;
    }
    if (canon_of_class) memcpy(canon_of_class, reps, sizeof(uint32_t) * (size_t)nc);
    *n_classes = nc;
    *n_all_classes = all;
    *n_connected_codes = ncodes;
    free(reps); free(canon); free(conn);
    return 0;
}

/* Number of (k-2)-subsets of the code's vertices that induce a connected G*
 * and dominate the remaining two vertices. */
int oracle_multiplicity(int k, uint32_t code) {
    if (k < 3 || k > 6) return OR_EINVAL;
    int adj[8][8] = {{0}};
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (i != j && ((code >> bitpos(k, i, j)) & 1u)) adj[i][j] = adj[j][i] = 1;
    int count = 0;
    for (int mask = 0; mask < (1 << k); ++mask) {
        if (__builtin_popcount((unsigned)mask) != k - 2) continue;
        /* connectivity of the subset */
        int first = __builtin_ctz((unsigned)mask), seen = 1 << first, grow = 1;
        while (grow) {
            grow = 0;
            for (int a = 0; a < k; ++a) if (seen >> a & 1)
                for (int b = 0; b < k; ++b)
                    if ((mask >> b & 1) && !(seen >> b & 1) && adj[a][b]) { seen |= 1 << b; grow = 1; }
        }
        if (seen != mask) continue;
        int dom = 1;
        for (int w = 0; w < k; ++w) {
            if (mask >> w & 1) continue;
            int hit = 0;
            for (int a = 0; a < k; ++a) if ((mask >> a & 1) && adj[a][w]) hit = 1;
            if (!hit) dom = 0;
        }
        count += dom;
    }
    return count;
}

/* ------------------------------------------------ k = 6 canonical codes -- */

/* Relabelling of 30-bit codes one byte at a time: the permuted code is the OR
 * of the images of its four bytes (each bit is one arc), so tab[p][b][v] =
 * permute_code(6, v << 8b, perm p) gives the image in four lookups. */
static uint32_t (*perm6_tab)[4][256] = NULL;

static void perm6_init(void) {
#pragma omp critical(perm6)
    if (!perm6_tab) {
        static int perms[720 * 6];
        all_perms(6, perms);
        uint32_t (*t)[4][256] = malloc(sizeof(uint32_t) * 720 * 4 * 256);
        for (int p = 0; p < 720; ++p)
            for (int b = 0; b < 4; ++b)
                for (int v = 0; v < 256; ++v)
                    t[p][b][v] = ((uint32_t)v << (8 * b)) >> 30 ? 0u
                                 : permute_code(6, (uint32_t)v << (8 * b), perms + p * 6);
        perm6_tab = t;
    }
}

/* Canonical code of a 6-vertex code: the minimum over all 720 relabellings. */
uint32_t oracle_canon6(uint32_t code) {
    if (!perm6_tab) perm6_init();
    uint32_t best = code;
    for (int p = 0; p < 720; ++p) {
        const uint32_t y = perm6_tab[p][0][code & 255u] | perm6_tab[p][1][(code >> 8) & 255u] |
                           perm6_tab[p][2][(code >> 16) & 255u] | perm6_tab[p][3][code >> 24];
        if (y < best) best = y;
    }
    return best;
}

/* Open-addressing maps of one thread: code -> canonical code (a cache), and
 * canonical code -> number of sets.  Keys are codes + 1 (0 = empty). */
struct map6 {
    uint32_t* ck; uint32_t* cv; size_t ccap;      /* cache */
    uint32_t* hk; uint64_t* hv; size_t hcap, hn;  /* counts */
};

static size_t h6(uint32_t x, size_t cap) { return (size_t)((x * 2654435761u) ^ (x >> 15)) & (cap - 1); }

static void map6_add(struct map6* m, uint32_t canon, uint64_t add) {
    if (2 * (m->hn + 1) > m->hcap) {  /* grow: rehash into twice the room */
        size_t cap = m->hcap ? 2 * m->hcap : 1024;
        uint32_t* k = calloc(cap, sizeof(uint32_t));
        uint64_t* v = calloc(cap, sizeof(uint64_t));
        for (size_t i = 0; i < m->hcap; ++i)
            if (m->hk[i]) {
                size_t h = h6(m->hk[i], cap);
                while (k[h]) h = (h + 1) & (cap - 1);
                k[h] = m->hk[i];
                v[h] = m->hv[i];
            }
        free(m->hk); free(m->hv);
        m->hk = k; m->hv = v; m->hcap = cap;
    }
    size_t h = h6(canon + 1u, m->hcap);
    while (m->hk[h] && m->hk[h] != canon + 1u) h = (h + 1) & (m->hcap - 1);
    if (!m->hk[h]) { m->hk[h] = canon + 1u; ++m->hn; }
    m->hv[h] += add;
}

static void canon6_count(struct map6* m, uint32_t code) {
    size_t h = h6(code + 1u, m->ccap);
    uint32_t canon;
    if (m->ck[h] == code + 1u) {
        canon = m->cv[h];
    } else {  /* a direct-mapped cache: a miss recomputes and replaces */
        canon = oracle_canon6(code);
        m->ck[h] = code + 1u;
        m->cv[h] = canon;
    }
    map6_add(m, canon, 1);
}

/* ---------------------------------------------------------------- ESU ---- */

typedef struct {
    int n;
    const int64_t* uoff;   /* undirected (G*) adjacency, sorted, unique */
    const int32_t* uidx;
    const int64_t* aoff;   /* out-arcs, sorted */
    const int32_t* aidx;
    int k;
    const uint16_t* cls;
    uint64_t* hist;        /* this thread's histogram */
    double deadline;       /* omp wall-clock deadline, <= 0: none */
    volatile int* stop;    /* set once the deadline has passed */
    uint64_t emitted;
    struct map6* map6;     /* k = 6: this thread's canonical-code counts */
} esu_ctx;

static int has_edge_u(const esu_ctx* c, int a, int b) {
    int64_t lo = c->uoff[a], hi = c->uoff[a + 1];
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (c->uidx[mid] < b) lo = mid + 1; else hi = mid; }
    return lo < c->uoff[a + 1] && c->uidx[lo] == b;
}

static int has_arc(const esu_ctx* c, int a, int b) {
    int64_t lo = c->aoff[a], hi = c->aoff[a + 1];
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (c->aidx[mid] < b) lo = mid + 1; else hi = mid; }
    return lo < c->aoff[a + 1] && c->aidx[lo] == b;
}

static void emit(esu_ctx* c, const int* sub) {
    int k = c->k, v[6];
    memcpy(v, sub, sizeof(int) * k);
    for (int i = 1; i < k; ++i) { int t = v[i], j = i - 1; while (j >= 0 && v[j] > t) { v[j + 1] = v[j]; --j; } v[j + 1] = t; }
    uint32_t code = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (i != j && has_arc(c, v[i], v[j])) code |= 1u << bitpos(k, i, j);
    if (c->k == 6) {
        canon6_count(c->map6, code);
    } else {
        uint16_t cl = c->cls[code];
        if (cl != 0xFFFF) c->hist[cl] += 1;   /* ESU only emits connected sets */
    }
#ifdef _OPENMP
    if (c->deadline > 0 && (++c->emitted & 0xFFFF) == 0 && omp_get_wtime() > c->deadline) *c->stop = 1;
#endif
}

/* sub[0..depth) is the current subgraph, ext the extension set. */
static void extend(esu_ctx* c, int* sub, int depth, const int* ext, int next, int root) {
    if (depth == c->k) { emit(c, sub); return; }
    if (*c->stop) return;
    int* work = (int*)malloc(sizeof(int) * (size_t)next);
    memcpy(work, ext, sizeof(int) * (size_t)next);
    int nwork = next;
    while (nwork > 0 && !*c->stop) {
        int w = work[--nwork];
        /* ext' = remaining ext  U  { u in N(w) : u > root, u not in sub,
         *                             u not adjacent to any vertex of sub } */
        int64_t dw = c->uoff[w + 1] - c->uoff[w];
        int* ext2 = (int*)malloc(sizeof(int) * (size_t)(nwork + dw + 1));
        memcpy(ext2, work, sizeof(int) * (size_t)nwork);
        int n2 = nwork;
        for (int64_t p = c->uoff[w]; p < c->uoff[w + 1]; ++p) {
            int u = c->uidx[p];
            if (u <= root) continue;
            int bad = 0;
            for (int s = 0; s < depth && !bad; ++s)
                if (sub[s] == u || has_edge_u(c, sub[s], u)) bad = 1;
            if (!bad) ext2[n2++] = u;
        }
        sub[depth] = w;
        extend(c, sub, depth + 1, ext2, n2, root);
        free(ext2);
    }
    free(work);
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return x < y ? -1 : x > y;
}

/*
 * Census of the simple digraph given as out-CSR (rows may be unsorted).
 * hist[n_classes] is overwritten.  threads <= 0 means the OpenMP default.
 */
static int census_impl(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                       const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads,
                       const int32_t* roots, int32_t n_roots, double seconds, struct map6* result6);

int oracle_census(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                  const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads) {
    return census_impl(n, out_off, out_idx, k, cls_of_code, n_classes, hist, threads, NULL, n, 0.0, NULL);
}

/*
 * ESU from the given roots only: counts the connected k-sets whose smallest
 * vertex is one of `roots` (ESU emits each set from its smallest vertex).
 * Summed over all vertices this is the full census; a seeded subset of roots
 * is a bounded sample of the same work.
 */
int oracle_census_roots(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                        const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads,
                        const int32_t* roots, int32_t n_roots) {
    for (int32_t i = 0; i < n_roots; ++i)
        if (roots[i] < 0 || roots[i] >= n) return OR_EINVAL;
    return census_impl(n, out_off, out_idx, k, cls_of_code, n_classes, hist, threads, roots, n_roots, 0.0, NULL);
}

/*
 * Time-bounded sample of the census work: ESU from `roots` in the given order
 * until `seconds` of wall time have passed (then every thread stops where it
 * is).  hist receives the sets emitted so far; the caller turns that into a
 * rate (sets per second).  Used only to time the oracle on workloads far too
 * large to enumerate completely.
 */
int oracle_census_timed(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                        const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads,
                        const int32_t* roots, int32_t n_roots, double seconds) {
    for (int32_t i = 0; i < n_roots; ++i)
        if (roots[i] < 0 || roots[i] >= n) return OR_EINVAL;
    return census_impl(n, out_off, out_idx, k, cls_of_code, n_classes, hist, threads, roots, n_roots,
                       seconds > 0 ? seconds : 1e-9, NULL);
}

static int census_impl(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                       const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads,
                       const int32_t* roots, int32_t n_roots, double seconds, struct map6* result6) {
    if (k < 3 || k > 6 || n < 0 || (k == 6) != (result6 != NULL)) return OR_EINVAL;
    if (hist) memset(hist, 0, sizeof(uint64_t) * (size_t)n_classes);
    if (n == 0) return 0;
    int64_t m = out_off[n];
    int64_t* aoff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* aidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* uoff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* uidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    if (!aoff || !aidx || !deg || !uoff || !uidx) return OR_ENOMEM;
    for (int v = 0; v <= n; ++v) aoff[v] = out_off[v];
    memcpy(aidx, out_idx, sizeof(int32_t) * (size_t)m);
    for (int v = 0; v < n; ++v) qsort(aidx + aoff[v], (size_t)(aoff[v + 1] - aoff[v]), sizeof(int32_t), cmp_i32);
    /* G*: both directions, then sort + unique per row */
    for (int v = 0; v < n; ++v)
        for (int64_t p = aoff[v]; p < aoff[v + 1]; ++p) { deg[v]++; deg[aidx[p]]++; }
    uoff[0] = 0;
    for (int v = 0; v < n; ++v) uoff[v + 1] = uoff[v] + deg[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int v = 0; v < n; ++v) fill[v] = uoff[v];
    for (int v = 0; v < n; ++v)
        for (int64_t p = aoff[v]; p < aoff[v + 1]; ++p) { uidx[fill[v]++] = aidx[p]; uidx[fill[aidx[p]]++] = v; }
    int64_t w = 0;
    int64_t* uoff2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    uoff2[0] = 0;
    for (int v = 0; v < n; ++v) {
        qsort(uidx + uoff[v], (size_t)(uoff[v + 1] - uoff[v]), sizeof(int32_t), cmp_i32);
        int64_t start = w;
        for (int64_t p = uoff[v]; p < uoff[v + 1]; ++p)
            if (w == start || uidx[w - 1] != uidx[p]) uidx[w++] = uidx[p];
        uoff2[v + 1] = w;
    }
    free(fill);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = threads > 0 ? threads : omp_get_max_threads();
#endif
    uint64_t* th = (uint64_t*)calloc((size_t)nthreads * (size_t)(n_classes > 0 ? n_classes : 1), sizeof(uint64_t));
    struct map6* maps = NULL;
    if (k == 6) {
        perm6_init();
        maps = (struct map6*)calloc((size_t)nthreads, sizeof(struct map6));
        for (int t = 0; t < nthreads; ++t) {
            maps[t].ccap = (size_t)1 << 18;
            maps[t].ck = (uint32_t*)calloc(maps[t].ccap, sizeof(uint32_t));
            maps[t].cv = (uint32_t*)calloc(maps[t].ccap, sizeof(uint32_t));
        }
    }
    volatile int stop = 0;
    double deadline = 0.0;
#ifdef _OPENMP
    if (seconds > 0) deadline = omp_get_wtime() + seconds;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int ri = 0; ri < n_roots; ++ri) {
        const int root = roots ? roots[ri] : ri;
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        if (stop) continue;
        esu_ctx c = { n, uoff2, uidx, aoff, aidx, k, cls_of_code, th + (size_t)tid * n_classes, deadline, &stop, 0,
                      maps ? maps + tid : NULL };
        int sub[6];
        sub[0] = root;
        int64_t d = uoff2[root + 1] - uoff2[root];
        int* ext = (int*)malloc(sizeof(int) * (size_t)(d + 1));
        int ne = 0;
        for (int64_t p = uoff2[root]; p < uoff2[root + 1]; ++p)
            if (uidx[p] > root) ext[ne++] = uidx[p];
        extend(&c, sub, 1, ext, ne, root);
        free(ext);
    }
    if (k == 6) {
        for (int t = 0; t < nthreads; ++t) {
            for (size_t i = 0; i < maps[t].hcap; ++i)
                if (maps[t].hk[i]) map6_add(result6, maps[t].hk[i] - 1u, maps[t].hv[i]);
            free(maps[t].ck); free(maps[t].cv); free(maps[t].hk); free(maps[t].hv);
        }
        free(maps);
    } else {
        for (int t = 0; t < nthreads; ++t)
            for (int cl = 0; cl < n_classes; ++cl) hist[cl] += th[(size_t)t * n_classes + cl];
    }
    free(th); free(aoff); free(aidx); free(deg); free(uoff); free(uoff2); free(uidx);
    return 0;
}

/*
 * k = 6 census by canonical code: the connected 6-sets of the digraph, each
 * found once by ESU, grouped by the canonical code of their induced digraph.
 * Writes up to max_out (canonical code, count) pairs in increasing code
 * order and their number to *n_out (OR_ENOMEM if more than max_out classes
 * occur).
 */
static int cmp_pair(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

int oracle_census6(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t threads,
                   uint32_t* codes, uint64_t* counts, int64_t max_out, int64_t* n_out) {
    struct map6 res = {0};
    int rc = census_impl(n, out_off, out_idx, 6, NULL, 0, NULL, threads, NULL, n, 0.0, &res);
    if (rc) { free(res.hk); free(res.hv); return rc; }
    if ((int64_t)res.hn > max_out) { free(res.hk); free(res.hv); return OR_ENOMEM; }
    uint64_t* kv = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (res.hn + 1));
    size_t w = 0;
    for (size_t i = 0; i < res.hcap; ++i)
        if (res.hk[i]) { kv[2 * w] = res.hk[i] - 1u; kv[2 * w + 1] = res.hv[i]; ++w; }
    qsort(kv, w, 2 * sizeof(uint64_t), cmp_pair);
    for (size_t i = 0; i < w; ++i) { codes[i] = (uint32_t)kv[2 * i]; counts[i] = kv[2 * i + 1]; }
    *n_out = (int64_t)w;
    free(kv); free(res.hk); free(res.hv);
    return 0;
}
