/*
 * CPU method reference for the exact motif census -- TEST INFRASTRUCTURE ONLY.
 *
 * Like oracle.c, only the test suite, the smoke check, the benchmark's
 * CPU-baseline leg and the golden-file script use this file, and it shares no
 * code, header, table or constant with the GPU library.
 *
 * oracle.c computes the census from its plain definition (ESU enumeration of
 * every connected k-set).  That is far too slow for the largest workloads, so
 * this file writes out the paper's own combinatorial method, step by step and
 * in the paper's order, as a second and much faster CPU route to the same
 * numbers.  It is pinned against the ESU oracle on many small graphs and on
 * scaled-down workloads (tests/test_method_ref.py) before it is trusted for
 * the full-size ones.
 *
 *   k = 3  Algorithm "Count 3 Sized Patterns": anchor = a vertex v, its
 *          neighbours split into the sets A^v, B^v, C^v (Section "Notation and
 *          definitions"), Figure "star" / Theorem "teo3" / Table "starb".
 *   k = 4  Algorithm "Count 4 Sized Patterns" for directed graphs: anchor = an
 *          edge e = {u, v}, the 15 sets of Section "Counting isomorphic
 *          patterns of size 4 in directed graphs", Fact "base", Theorem
 *          "lema4d" / Corollary "coro:a", Fact "correction".
 *   k = 5  Algorithm "Count 5 Sized Patterns" for directed graphs: anchor = a
 *          connected triple (p1, p2, p3) (Algorithm "calckp"), the 63 sets of
 *          Algorithm "partfive", Fact "basefive", Lemma "lema5d", and the
 *          division by the number of connected triples that see a 5-set
 *          (Figure "correction:five").
 *   und.   Algorithm "und4" with Table "ept" (Theorem "teo4u") and Fact
 *   k = 4  "correction" on the undirected version G*: the six counts
 *          (P4, tailed triangle, claw S3, C4, K4 minus an edge, K4).
 *
 * For every anchor the three directed theorems apply one rule: for each set T
 * the pair pattern P(T,T) gains C(n_T,2) minus the edges inside T, and each
 * edge moves its occurrence to the pattern with that edge (directed or
 * bidirected); for each pair of sets T_i < T_j the same with n_i * n_j.
 * Anchor_frequencies() below is that rule, once, for 3, 15 or 63 sets.
 *
 * Readings, shared with the oracle's class numbering:
 *  - The paper's hard-coded pattern matrices (P, P->, P<-, P<->, the missing
 *    Table P, the 13 x 63 x 63 k = 5 matrix) are replaced by the class of the
 *    full adjacency code of (anchor vertices, v1, v2), read from the
 *    brute-force class table of oracle.c, passed in by the caller.
 *  - The m-variables: the paper scans all of E per anchor (Algorithm "vars");
 *    only edges with both ends in adj(anchor) count, so each such edge is
 *    found instead from its endpoint of lower rank (d*, id), whose oriented
 *    row N+ lists it once.  Same values.
 *  - k = 4 iterates E*, each adjacent pair once (Fact "correction" counts
 *    undirected edges).  k = 5 takes each connected 3-set once: an induced
 *    path at its centre, a triangle at its smallest vertex.
 *  - Divisions are exact; a non-zero remainder is reported (MR_EDIV).
 *  - Counts are uint64, and a pattern total may pass through "negative"
 *    values (wrapping) before the edges of later anchors add back.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MR_EINVAL (-1)
#define MR_ENOMEM (-2)
#define MR_EDIV (-3) /* a class total was not a multiple of its anchor count */

#define FLAG 0x80u   /* label bit: the vertex is one of the anchor's own vertices */

static int mbit(int k, int i, int j) { return i * (k - 1) + (j < i ? j : j - 1); }

/* ------------------------------------------------------------- G* build -- */

/* Typed undirected graph G*: row v lists every neighbour x once, sorted by
 * id, with the type of x relative to v (Section "Notation and definitions"):
 * 1 = B^v (arc v->x only), 2 = C^v (arc x->v only), 3 = A^v (both arcs).
 * pnb/pty: the oriented rows N+(v), the neighbours of higher rank (d*, id). */
typedef struct {
    int n;
    int64_t *off, *poff;
    int32_t *nb, *pnb;
    uint8_t *ty, *pty;
} gstar;

static void gstar_free(gstar* g) {
    free(g->off); free(g->poff); free(g->nb); free(g->pnb); free(g->ty); free(g->pty);
    memset(g, 0, sizeof *g);
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : x > y;
}

static int higher(const int64_t* off, int a, int b) { /* rank(b) > rank(a) */
    int64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
    return db > da || (db == da && b > a);
}

static int gstar_build(int32_t n, const int32_t* out_off, const int32_t* out_idx, gstar* g) {
    memset(g, 0, sizeof *g);
    g->n = n;
    const int64_t m = out_off[n];
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* half = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * m + 1)); /* (id << 2) | type */
    g->off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->poff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!cnt || !half || !g->off || !g->poff) { free(cnt); free(half); gstar_free(g); return MR_ENOMEM; }
    for (int32_t u = 0; u < n; ++u)
        for (int64_t p = out_off[u]; p < out_off[u + 1]; ++p) {
            const int32_t v = out_idx[p];
            if (v < 0 || v >= n || v == u) { free(cnt); free(half); gstar_free(g); return MR_EINVAL; }
            cnt[u]++; cnt[v]++;
        }
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!fill) { free(cnt); free(half); gstar_free(g); return MR_ENOMEM; }
    fill[0] = 0;
    for (int32_t v = 0; v < n; ++v) fill[v + 1] = fill[v] + cnt[v];
    memcpy(cnt, fill, sizeof(int64_t) * (size_t)(n + 1)); /* cnt = row starts of the half-edges */
    for (int32_t u = 0; u < n; ++u)
        for (int64_t p = out_off[u]; p < out_off[u + 1]; ++p) {
            const int32_t v = out_idx[p];
            half[fill[u]++] = ((int64_t)v << 2) | 1; /* v is an out-neighbour of u */
            half[fill[v]++] = ((int64_t)u << 2) | 2; /* u is an in-neighbour of v */
        }
    /* sort each row, merge the two half-edges of a reciprocated pair */
    int64_t w = 0;
    g->off[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t a = cnt[v], b = cnt[v + 1];
        qsort(half + a, (size_t)(b - a), sizeof(int64_t), cmp_i64);
        const int64_t start = w;
        for (int64_t p = a; p < b; ++p) {
            if (w > start && (half[w - 1] >> 2) == (half[p] >> 2)) half[w - 1] |= half[p] & 3;
            else half[w++] = half[p];
        }
        g->off[v + 1] = w;
    }
    free(fill); free(cnt);
    g->nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(w + 1));
    g->ty = (uint8_t*)malloc((size_t)w + 1);
    if (!g->nb || !g->ty) { free(half); gstar_free(g); return MR_ENOMEM; }
    for (int64_t p = 0; p < w; ++p) { g->nb[p] = (int32_t)(half[p] >> 2); g->ty[p] = (uint8_t)(half[p] & 3); }
    free(half);
    /* N+ rows */
    int64_t wp = 0;
    g->poff[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) wp += higher(g->off, v, g->nb[p]);
        g->poff[v + 1] = wp;
    }
    g->pnb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(wp + 1));
    g->pty = (uint8_t*)malloc((size_t)wp + 1);
    if (!g->pnb || !g->pty) { gstar_free(g); return MR_ENOMEM; }
    wp = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p)
            if (higher(g->off, v, g->nb[p])) { g->pnb[wp] = g->nb[p]; g->pty[wp] = g->ty[p]; ++wp; }
    return 0;
}

/* ------------------------------------------------- per-anchor frequencies -- */

/* Per-thread state of one anchor: labels, members, set sizes, m-variables. */
typedef struct {
    int k, ns;           /* anchor vertices k-2; ns = 4^(k-2) set labels (0 = none) */
    uint8_t* lab;        /* [n]: 2 type bits per anchor vertex, FLAG for anchor vertices */
    int32_t* mem;        /* members of adj(anchor) */
    int64_t nmem;
    uint64_t size[64];   /* n_T */
    int ne, nonempty[64];
    uint32_t* mdir;      /* [ns*ns]: directed edges from T_i to T_j */
    uint32_t* mbi;       /* [ns*ns]: bidirected edges between T_i <= T_j */
    uint64_t* hist;
} anchor_ws;

/* Code bits of a member in slot s whose types towards the anchor vertices
 * 0..k-3 are packed two bits each in L. */
static uint32_t member_code(int k, int s, uint32_t L) {
    uint32_t c = 0;
    for (int i = 0; i < k - 2; ++i) {
        const uint32_t t = (L >> (2 * i)) & 3u;
        if (t & 1u) c |= 1u << mbit(k, i, s); /* arc anchor_i -> member */
        if (t & 2u) c |= 1u << mbit(k, s, i); /* arc member -> anchor_i */
    }
    return c;
}

/* Pattern of (anchor, v1 in set Ti, v2 in set Tj) with edge r between v1 and
 * v2: r = 0 none, 1 = v1 -> v2, 2 = v2 -> v1, 3 = both. */
static uint16_t pattern(int k, const uint16_t* cls, uint32_t anchor_code, int Ti, int Tj, int r) {
    uint32_t c = anchor_code | member_code(k, k - 2, (uint32_t)Ti) | member_code(k, k - 1, (uint32_t)Tj);
    if (r & 1) c |= 1u << mbit(k, k - 2, k - 1);
    if (r & 2) c |= 1u << mbit(k, k - 1, k - 2);
    return cls[c];
}

static void add_member(anchor_ws* w, int32_t x) {
    const int T = w->lab[x] & (w->ns - 1);
    if (w->size[T]++ == 0) w->nonempty[w->ne++] = T;
    w->mem[w->nmem++] = x;
}

/* m-variables (Algorithm "vars" and its k = 5 form): every edge (x, y) with
 * both ends in adj(anchor), found once from the N+ row of its lower-ranked
 * end x; y's type relative to x says which variable it adds to. */
static void count_m_variables(const gstar* g, anchor_ws* w) {
    const uint32_t mask = (uint32_t)w->ns - 1;
    for (int64_t i = 0; i < w->nmem; ++i) {
        const int32_t x = w->mem[i];
        const uint32_t Tx = w->lab[x] & mask;
        for (int64_t p = g->poff[x]; p < g->poff[x + 1]; ++p) {
            const uint32_t Ly = w->lab[g->pnb[p]];
            if ((Ly & FLAG) || !(Ly & mask)) continue;
            const uint32_t Ty = Ly & mask, r = g->pty[p];
            if (r == 3) w->mbi[(Tx < Ty ? Tx : Ty) * w->ns + (Tx < Ty ? Ty : Tx)]++;
            else if (r == 1) w->mdir[Tx * w->ns + Ty]++;   /* x -> y */
            else w->mdir[Ty * w->ns + Tx]++;               /* y -> x */
        }
    }
}

static void sort_small(int* a, int n) {
    for (int i = 1; i < n; ++i) { int t = a[i], j = i - 1; while (j >= 0 && a[j] > t) { a[j + 1] = a[j]; --j; } a[j + 1] = t; }
}

/* Theorem "teo3" (directed, Table "starb"), Theorem "lema4d" / Corollary
 * "coro:a", Lemma "lema5d": the pattern frequencies of one anchor from its
 * set sizes and m-variables, added to the histogram; then the anchor's state
 * is cleared. */
static void anchor_frequencies(const uint16_t* cls, uint32_t anchor_code, anchor_ws* w) {
    const int k = w->k, ns = w->ns;
    uint64_t* h = w->hist;
    sort_small(w->nonempty, w->ne);
    for (int a = 0; a < w->ne; ++a) {
        const int T = w->nonempty[a];
        const uint64_t nT = w->size[T], mTT = w->mdir[T * ns + T], mbTT = w->mbi[T * ns + T];
        h[pattern(k, cls, anchor_code, T, T, 0)] += nT * (nT - 1) / 2 - mTT - mbTT;
        if (mbTT) h[pattern(k, cls, anchor_code, T, T, 3)] += mbTT;
        if (mTT) h[pattern(k, cls, anchor_code, T, T, 1)] += mTT;
        for (int b = a + 1; b < w->ne; ++b) {
            const int U = w->nonempty[b];
            const uint64_t mb = w->mbi[T * ns + U], mTU = w->mdir[T * ns + U], mUT = w->mdir[U * ns + T];
            h[pattern(k, cls, anchor_code, T, U, 0)] += w->size[T] * w->size[U] - mb - mTU - mUT;
            if (mb) h[pattern(k, cls, anchor_code, T, U, 3)] += mb;
            if (mTU) h[pattern(k, cls, anchor_code, T, U, 1)] += mTU;
            if (mUT) h[pattern(k, cls, anchor_code, T, U, 2)] += mUT;
        }
    }
    for (int a = 0; a < w->ne; ++a) {
        const int T = w->nonempty[a];
        w->size[T] = 0;
        for (int b = 0; b < w->ne; ++b) {
            const int U = w->nonempty[b];
            w->mdir[T * ns + U] = 0;
            w->mbi[T * ns + U] = 0;
        }
    }
    w->ne = 0;
    w->nmem = 0;
}

/* Set (or clear, t = 0 via clear_slot) the type bits of slot i for the
 * neighbours of anchor vertex a. */
static void set_slot(const gstar* g, uint8_t* lab, int32_t a, int i) {
    for (int64_t p = g->off[a]; p < g->off[a + 1]; ++p) lab[g->nb[p]] |= (uint8_t)(g->ty[p] << (2 * i));
}
static void clear_slot(const gstar* g, uint8_t* lab, int32_t a, int i) {
    for (int64_t p = g->off[a]; p < g->off[a + 1]; ++p) lab[g->nb[p]] &= (uint8_t)~(3u << (2 * i));
}

/* Type of v relative to u (from u's row), 0 if not adjacent. */
static uint32_t type_of(const gstar* g, int32_t u, int32_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (g->nb[mid] < v) lo = mid + 1; else hi = mid; }
    return (lo < g->off[u + 1] && g->nb[lo] == v) ? g->ty[lo] : 0u;
}

/* Code bits of the arcs between anchor slots i and j (t = type of slot j's
 * vertex relative to slot i's). */
static uint32_t pair_code(int k, int i, int j, uint32_t t) {
    return ((t & 1u) ? 1u << mbit(k, i, j) : 0u) | ((t & 2u) ? 1u << mbit(k, j, i) : 0u);
}

/* ------------------------------------------------------------ the census -- */

/* Anchors of each k, processed by one thread with workspace w:
 *   k = 3: vertex `unit`;
 *   k = 4: the G* entry `unit` = (u, v) when u < v, the edge {u, v};
 *   k = 5: the G* entry `unit` = (b, a): every connected triple with centre b
 *          and end a whose other end c is above a (each connected 3-set
 *          once: a path at its centre, a triangle at its smallest vertex). */
static void census_unit(const gstar* g, const uint16_t* cls, const int32_t* row_of, int64_t unit, anchor_ws* w) {
    uint8_t* lab = w->lab;
    const int k = w->k;
    if (k == 3) {
        const int32_t v = (int32_t)unit;
        set_slot(g, lab, v, 0);
        lab[v] |= FLAG;
        for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) add_member(w, g->nb[p]);
        count_m_variables(g, w);
        anchor_frequencies(cls, 0u, w);
        clear_slot(g, lab, v, 0);
        lab[v] &= (uint8_t)~FLAG;
        return;
    }
    const int32_t r = row_of[unit], x = g->nb[unit];
    if (k == 4) {
        const int32_t u = r, v = x;
        if (v < u) return;
        set_slot(g, lab, u, 0);
        set_slot(g, lab, v, 1);
        lab[u] |= FLAG; lab[v] |= FLAG;
        /* the 15 sets partition adj(e) = N(u) u N(v) \ {u, v} */
        for (int64_t p = g->off[u]; p < g->off[u + 1]; ++p)
            if (!(lab[g->nb[p]] & FLAG)) add_member(w, g->nb[p]);
        for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p)
            if (!(lab[g->nb[p]] & (FLAG | 3u))) add_member(w, g->nb[p]);
        count_m_variables(g, w);
        anchor_frequencies(cls, pair_code(4, 0, 1, g->ty[unit]), w);
        clear_slot(g, lab, u, 0);
        clear_slot(g, lab, v, 1);
        lab[u] &= (uint8_t)~FLAG; lab[v] &= (uint8_t)~FLAG;
        return;
    }
    /* k = 5: centre b = p2 (slot 1), end a = p1 (slot 0), end c = p3 (slot 2) */
    const int32_t b = r, a = x;
    const uint32_t tba = g->ty[unit]; /* type of a relative to b */
    set_slot(g, lab, b, 1);
    set_slot(g, lab, a, 0);
    lab[a] |= FLAG; lab[b] |= FLAG;
    for (int64_t q = g->off[b]; q < g->off[b + 1]; ++q) {
        const int32_t c = g->nb[q];
        if (c <= a) continue;
        const uint32_t tac = lab[c] & 3u; /* type of c relative to a; 0 = a, c not adjacent */
        if (tac && b > a) continue;       /* a triangle is taken at its smallest vertex */
        set_slot(g, lab, c, 2);
        lab[c] |= FLAG;
        /* Algorithm "partfive": adj(p1, p2, p3) in 63 sets, each member once */
        for (int64_t p = g->off[a]; p < g->off[a + 1]; ++p)
            if (!(lab[g->nb[p]] & FLAG)) add_member(w, g->nb[p]);
        for (int64_t p = g->off[b]; p < g->off[b + 1]; ++p)
            if (!(lab[g->nb[p]] & (FLAG | 3u))) add_member(w, g->nb[p]);
        for (int64_t p = g->off[c]; p < g->off[c + 1]; ++p)
            if (!(lab[g->nb[p]] & (FLAG | 15u))) add_member(w, g->nb[p]);
        count_m_variables(g, w);
        /* the triple's own arcs: a-b (tba), b-c, and a-c for a triangle */
        const uint32_t code = pair_code(5, 1, 0, tba) | pair_code(5, 1, 2, g->ty[q]) | pair_code(5, 0, 2, tac);
        anchor_frequencies(cls, code, w);
        clear_slot(g, lab, c, 2);
        lab[c] &= (uint8_t)~FLAG;
    }
    clear_slot(g, lab, a, 0);
    clear_slot(g, lab, b, 1);
    lab[a] &= (uint8_t)~FLAG; lab[b] &= (uint8_t)~FLAG;
}

/*
 * The census of the simple digraph given as out-CSR (rows may be unsorted) by
 * the paper's method.  cls_of_code: the oracle's class table for k (2^(k(k-1))
 * entries, 0xFFFF for disconnected codes); mult[c]: the number of anchors
 * that see one occurrence of class c (the oracle's multiplicity).  hist[C] is
 * overwritten.  threads <= 0: the OpenMP default.
 */
/* Pseudo-random choice of sampled units (Fibonacci hashing of the index), so
 * that a sample is not biased towards the vertices of low id. */
static uint64_t sample_hash(int64_t u) { return ((uint64_t)u * 0x9E3779B97F4A7C15ull) >> 24; }

static int census_strided(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                          const uint16_t* cls_of_code, const int32_t* mult, int32_t n_classes, uint64_t* hist,
                          int32_t threads, int64_t stride);

int mref_census(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k, const uint16_t* cls_of_code,
                const int32_t* mult, int32_t n_classes, uint64_t* hist, int32_t threads) {
    return census_strided(n, out_off, out_idx, k, cls_of_code, mult, n_classes, hist, threads, 1);
}

/*
 * Timing sample only: the same per-anchor work on a pseudo-random 1/stride
 * of the anchor units (vertices for k = 3, G* entries for k = 4, 5), summed
 * without the final division (a partial sum is not divisible).  stride * (its
 * time) estimates the full census time.
 */
int mref_census_sample(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                       const uint16_t* cls_of_code, int32_t n_classes, uint64_t* hist, int32_t threads,
                       int64_t stride) {
    if (stride < 2) return MR_EINVAL;
    return census_strided(n, out_off, out_idx, k, cls_of_code, NULL, n_classes, hist, threads, stride);
}

static int census_strided(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t k,
                          const uint16_t* cls_of_code, const int32_t* mult, int32_t n_classes, uint64_t* hist,
                          int32_t threads, int64_t stride) {
    if (k < 3 || k > 5 || n < 0) return MR_EINVAL;
    memset(hist, 0, sizeof(uint64_t) * (size_t)n_classes);
    if (n == 0) return 0;
    gstar g;
    int rc = gstar_build(n, out_off, out_idx, &g);
    if (rc) return rc;
    const int64_t entries = g.off[n];
    int32_t* row_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(entries + 1));
    if (!row_of) { gstar_free(&g); return MR_ENOMEM; }
    int64_t dmax = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) row_of[p] = v;
        if (g.off[v + 1] - g.off[v] > dmax) dmax = g.off[v + 1] - g.off[v];
    }
    const int64_t units = k == 3 ? n : entries;
    const int ns = 1 << (2 * (k - 2));
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = threads > 0 ? threads : omp_get_max_threads();
#endif
    uint64_t* th = (uint64_t*)calloc((size_t)nthreads * (size_t)n_classes, sizeof(uint64_t));
    int fail = th == NULL;
#pragma omp parallel num_threads(nthreads) reduction(| : fail)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        anchor_ws w;
        memset(&w, 0, sizeof w);
        w.k = k;
        w.ns = ns;
        w.lab = (uint8_t*)calloc((size_t)n, 1);
        w.mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * dmax + 1));
        w.mdir = (uint32_t*)calloc((size_t)ns * ns, sizeof(uint32_t));
        w.mbi = (uint32_t*)calloc((size_t)ns * ns, sizeof(uint32_t));
        w.hist = th ? th + (size_t)tid * n_classes : NULL;
        const int ok = w.lab && w.mem && w.mdir && w.mbi && w.hist;
        if (!ok) fail = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < units; ++u)
            if (ok && (stride == 1 || sample_hash(u) % (uint64_t)stride == 0))
                census_unit(&g, cls_of_code, row_of, u, &w);
        free(w.lab); free(w.mem); free(w.mdir); free(w.mbi);
    }
    if (!fail) {
        for (int t = 0; t < nthreads; ++t)
            for (int c = 0; c < n_classes; ++c) hist[c] += th[(size_t)t * n_classes + c];
        /* Fact "correction" and its k = 3, 5 forms: exact division */
        for (int c = 0; mult && c < n_classes; ++c) {
            if (mult[c] <= 0 || hist[c] % (uint64_t)mult[c]) { rc = MR_EDIV; break; }
            hist[c] /= (uint64_t)mult[c];
        }
    } else {
        rc = MR_ENOMEM;
    }
    if (rc) memset(hist, 0, sizeof(uint64_t) * (size_t)n_classes);
    free(th); free(row_of); gstar_free(&g);
    return rc;
}

/*
 * Undirected census of size 4 of G* (the undirected version of the digraph),
 * Algorithm "und4": for every edge e = {u, v}, X = N(u) \ N[v], Y = N(v) \
 * N[u], Z = N(u) n N(v), their sizes and the edge counts m_xx .. m_zz between
 * them, then the frequencies of Table "ept", summed over all edges and
 * divided as Fact "correction" says.  out[6] = (P4, tailed triangle
 * "x <-> C3", claw S3, C4, K4 minus an edge, K4), the order the paper's text
 * suggests for h[0..5].
 */
int mref_undirected4(int32_t n, const int32_t* out_off, const int32_t* out_idx, uint64_t* out, int32_t threads) {
    memset(out, 0, sizeof(uint64_t) * 6);
    if (n < 0) return MR_EINVAL;
    if (n == 0) return 0;
    gstar g;
    int rc = gstar_build(n, out_off, out_idx, &g);
    if (rc) return rc;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = threads > 0 ? threads : omp_get_max_threads();
#endif
    const int64_t entries = g.off[n];
    int32_t* row_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(entries + 1));
    if (!row_of) { gstar_free(&g); return MR_ENOMEM; }
    for (int32_t v = 0; v < n; ++v)
        for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) row_of[p] = v;
    uint64_t tot[6] = {0, 0, 0, 0, 0, 0};
    int fail = 0;
#pragma omp parallel num_threads(nthreads) reduction(| : fail)
    {
        /* lab bit 0: in N(u), bit 1: in N(v), FLAG: u or v.  X = 1, Y = 2, Z = 3 */
        uint8_t* lab = (uint8_t*)calloc((size_t)n, 1);
        int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(entries + 1));
        uint64_t loc[6] = {0, 0, 0, 0, 0, 0};
        if (!lab || !mem) fail = 1;
        /* one unit per G* entry (u, v): the edge {u, v} when u < v */
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < entries; ++q) {
            if (!lab || !mem) continue;
            {
                const int32_t u = row_of[q], v = g.nb[q];
                if (v < u) continue; /* each edge of G* once */
                int64_t nm = 0;
                for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p) lab[g.nb[p]] |= 1u;
                for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) lab[g.nb[p]] |= 2u;
                lab[u] |= FLAG; lab[v] |= FLAG;
                uint64_t nx = 0, ny = 0, nz = 0;
                for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p) {
                    const uint8_t L = lab[g.nb[p]];
                    if (L & FLAG) continue;
                    mem[nm++] = g.nb[p];
                    if (L == 3) ++nz; else ++nx;
                }
                for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) {
                    const uint8_t L = lab[g.nb[p]];
                    if (L == 2) { mem[nm++] = g.nb[p]; ++ny; }
                }
                /* m[a][b]: edges between the sets a <= b of {X = 1, Y = 2, Z = 3} */
                uint64_t mv[4][4];
                memset(mv, 0, sizeof mv);
                for (int64_t i = 0; i < nm; ++i) {
                    const int32_t x = mem[i];
                    const int a = lab[x] & 3;
                    for (int64_t p = g.poff[x]; p < g.poff[x + 1]; ++p) {
                        const uint8_t L = lab[g.pnb[p]];
                        if ((L & FLAG) || !(L & 3)) continue;
                        const int b = L & 3;
                        mv[a < b ? a : b][a < b ? b : a]++;
                    }
                }
                const uint64_t mxx = mv[1][1], mxy = mv[1][2], mxz = mv[1][3], myy = mv[2][2], myz = mv[2][3],
                               mzz = mv[3][3];
                /* Table "ept" */
                loc[0] += nx * ny - mxy;                                   /* P4 */
                loc[1] += (nx + ny) * nz - mxz - myz + mxx + myy;          /* tailed triangle */
                loc[2] += nx * (nx - 1) / 2 + ny * (ny - 1) / 2 - mxx - myy; /* claw S3 */
                loc[3] += mxy;                                             /* C4 */
                loc[4] += nz * (nz - 1) / 2 + mxz + myz - mzz;              /* K4 minus an edge */
                loc[5] += mzz;                                             /* K4 */
                for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p) lab[g.nb[p]] = 0;
                for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) lab[g.nb[p]] = 0;
                lab[u] = 0; lab[v] = 0;
            }
        }
#pragma omp critical
        for (int i = 0; i < 6; ++i) tot[i] += loc[i];
        free(lab); free(mem);
    }
    free(row_of);
    gstar_free(&g);
    if (fail) return MR_ENOMEM;
    /* Fact "correction": P4 once, tailed triangle and S3 three times, C4 four,
     * K4 minus an edge five, K4 six */
    static const uint64_t div[6] = {1, 3, 3, 4, 5, 6};
    for (int i = 0; i < 6; ++i) {
        if (tot[i] % div[i]) return MR_EDIV;
        out[i] = tot[i] / div[i];
    }
    return 0;
}
