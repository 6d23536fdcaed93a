/*
 * Degree-preserving arc-switch randomisation (input generation only).
 *
 * Attempt: pick two arcs a->b and c->d uniformly; rewire to a->d and c->b
 * unless that creates a self-loop or an arc already present.  In- and
 * out-degrees are preserved exactly.  Random numbers: splitmix64 seeded per
 * graph, so a graph is a deterministic function of (input, attempts, seed).
 * Arc membership: a bitmap over n*n for small n, else an open-addressing
 * hash set with tombstones (rebuilt when they pile up).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t splitmix64(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    int use_bitmap;
    uint64_t* bits;      /* bitmap over n*n */
    uint64_t* keys;      /* hash slots: 0 empty, 1 tombstone, key+2 */
    uint64_t cap, used, tomb;
} arcset;

static uint64_t mix(uint64_t k) { k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; return k; }

static int set_has(arcset* s, uint64_t key) {
    if (s->use_bitmap) return (int)((s->bits[key >> 6] >> (key & 63)) & 1u);
    uint64_t i = mix(key) & (s->cap - 1);
    for (;;) {
        uint64_t v = s->keys[i];
        if (v == 0) return 0;
        if (v == key + 2) return 1;
        i = (i + 1) & (s->cap - 1);
    }
}

static void set_insert_raw(arcset* s, uint64_t key) {
    uint64_t i = mix(key) & (s->cap - 1);
    while (s->keys[i] >= 2) i = (i + 1) & (s->cap - 1);
    if (s->keys[i] == 1) s->tomb--;
    s->keys[i] = key + 2;
    s->used++;
}

static void set_rebuild(arcset* s) {
    uint64_t* old = s->keys;
    uint64_t cap = s->cap;
    s->keys = (uint64_t*)calloc(cap, sizeof(uint64_t));
    s->used = 0;
    s->tomb = 0;
    for (uint64_t i = 0; i < cap; ++i)
        if (old[i] >= 2) set_insert_raw(s, old[i] - 2);
    free(old);
}

static void set_insert(arcset* s, uint64_t key) {
    if (s->use_bitmap) { s->bits[key >> 6] |= 1ull << (key & 63); return; }
    set_insert_raw(s, key);
}

static void set_erase(arcset* s, uint64_t key) {
    if (s->use_bitmap) { s->bits[key >> 6] &= ~(1ull << (key & 63)); return; }
    uint64_t i = mix(key) & (s->cap - 1);
    for (;;) {
        uint64_t v = s->keys[i];
        if (v == 0) return;
        if (v == key + 2) { s->keys[i] = 1; s->used--; s->tomb++; break; }
        i = (i + 1) & (s->cap - 1);
    }
    if (s->tomb > s->cap / 4) set_rebuild(s);
}

/* src/dst: the m arcs (dst is rewritten in place). Returns accepted switches. */
static int64_t switch_one(int32_t n, int64_t m, const int32_t* src, int32_t* dst, int64_t attempts, uint64_t seed) {
    arcset s;
    memset(&s, 0, sizeof(s));
    uint64_t nn = (uint64_t)n * (uint64_t)n;
    s.use_bitmap = nn <= (1ull << 28);
    if (s.use_bitmap) {
        s.bits = (uint64_t*)calloc(nn / 64 + 1, sizeof(uint64_t));
    } else {
        s.cap = 1;
        while (s.cap < (uint64_t)m * 4) s.cap <<= 1;
        s.keys = (uint64_t*)calloc(s.cap, sizeof(uint64_t));
    }
    for (int64_t i = 0; i < m; ++i) set_insert(&s, (uint64_t)src[i] * n + (uint64_t)dst[i]);
    uint64_t rs = seed;
    int64_t accepted = 0;
    for (int64_t t = 0; t < attempts; ++t) {
        int64_t i = (int64_t)(splitmix64(&rs) % (uint64_t)m);
        int64_t j = (int64_t)(splitmix64(&rs) % (uint64_t)m);
        if (i == j) continue;
        int32_t a = src[i], b = dst[i], c = src[j], d = dst[j];
        if (a == d || c == b) continue;
        uint64_t k1 = (uint64_t)a * n + (uint64_t)d, k2 = (uint64_t)c * n + (uint64_t)b;
        if (set_has(&s, k1) || set_has(&s, k2)) continue;
        set_erase(&s, (uint64_t)a * n + (uint64_t)b);
        set_erase(&s, (uint64_t)c * n + (uint64_t)d);
        set_insert(&s, k1);
        set_insert(&s, k2);
        dst[i] = d;
        dst[j] = b;
        ++accepted;
    }
    free(s.bits);
    free(s.keys);
    return accepted;
}

/* count graphs: dst_out[g*m .. (g+1)*m) receives graph g's rewired heads. */
int gg_arc_switch_many(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t attempts,
                       const uint64_t* seeds, int32_t count, int32_t* dst_out, int64_t* accepted) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t g = 0; g < count; ++g) {
        int32_t* d = dst_out + (int64_t)g * m;
        memcpy(d, dst, sizeof(int32_t) * (size_t)m);
        int64_t acc = switch_one(n, m, src, d, attempts, seeds[g]);
        if (accepted) accepted[g] = acc;
    }
    return 0;
}
