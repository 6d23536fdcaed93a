// Class tables: the "hard coded" pattern -> histogram-position matrices of the
// paper (Algorithms "Count 3/4/5 Sized Patterns"; the 13x63x63 Delta-Pattern
// matrices of Section "Counting 5-sized patterns in directed graphs") folded
// into one lookup on the full k(k-1)-bit adjacency code of the k-set.
//
// Canonical code = minimum code over all k! relabellings.  The table is built
// by orbit enumeration: codes are visited in ascending order; the first code
// of an orbit not yet labelled is its minimum, so applying every permutation
// to it labels the whole orbit at once (9608 orbits x 120 permutations for
// k = 5).  Class ids are the ranks of the minima of weakly connected orbits.
//
// Multiplicity of a class = number of connected (k-2)-vertex subsets T of one
// occurrence such that both remaining vertices have a neighbour in T: these
// are exactly the anchors (a vertex, an undirected edge, a connected triple)
// whose v-/e-/Delta-Pattern set contains the occurrence (Fact "correction",
// Figure "correction:five").
#include "classes.h"

#include <algorithm>
#include <mutex>

namespace motif {
namespace {

struct Perm {
  uint8_t to[32];  // bit b of the source code moves to bit to[b]
};

std::vector<Perm> bit_permutations(int k) {
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i;
  std::vector<Perm> out;
  do {
    Perm q{};
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j)
        if (i != j) q.to[code_bit(k, i, j)] = (uint8_t)code_bit(k, p[i], p[j]);
    out.push_back(q);
  } while (std::next_permutation(p.begin(), p.end()));
  return out;
}

uint32_t apply(const Perm& q, uint32_t code) {
  uint32_t out = 0;
  while (code) {
    int b = __builtin_ctz(code);
    code &= code - 1;
    out |= 1u << q.to[b];
  }
  return out;
}

// Undirected adjacency bitmasks of the k vertices.
void skeleton(int k, uint32_t code, uint32_t* nb) {
  for (int i = 0; i < k; ++i) nb[i] = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      if (i != j && (code >> code_bit(k, i, j) & 1u)) {
        nb[i] |= 1u << j;
        nb[j] |= 1u << i;
      }
}

// Is the vertex subset `mask` connected in the skeleton?
bool subset_connected(const uint32_t* nb, uint32_t mask) {
  if (!mask) return false;
  uint32_t reach = mask & (~mask + 1u);
  for (;;) {
    uint32_t grow = reach;
    for (uint32_t r = reach; r; r &= r - 1) grow |= nb[__builtin_ctz(r)] & mask;
    if (grow == reach) break;
    reach = grow;
  }
  return reach == mask;
}

uint8_t anchors_seeing(int k, uint32_t code) {
  uint32_t nb[8];
  skeleton(k, code, nb);
  const uint32_t all = (1u << k) - 1u;
  int count = 0;
  for (uint32_t t = 0; t <= all; ++t) {
    if (__builtin_popcount(t) != k - 2 || !subset_connected(nb, t)) continue;
    bool dominated = true;
    for (uint32_t rest = all & ~t; rest; rest &= rest - 1)
      if (!(nb[__builtin_ctz(rest)] & t)) dominated = false;
    count += dominated;
  }
  return (uint8_t)count;
}

ClassTable build(int k) {
  ClassTable t;
  t.k = k;
  t.nbits = k * (k - 1);
  const uint32_t N = 1u << t.nbits;
  const std::vector<Perm> perms = bit_permutations(k);
  std::vector<uint32_t> orbit_min(N, UINT32_MAX);
  std::vector<uint32_t> mins;
  for (uint32_t x = 0; x < N; ++x) {
    if (orbit_min[x] != UINT32_MAX) continue;
    mins.push_back(x);  // ascending, so this is the minimum of its orbit
    for (const Perm& q : perms) orbit_min[apply(q, x)] = x;
  }
  // class ids: connected orbit minima in ascending order
  std::vector<int32_t> id_of_min_index(mins.size(), -1);
  for (size_t i = 0; i < mins.size(); ++i) {
    uint32_t nb[8];
    skeleton(k, mins[i], nb);
    if (subset_connected(nb, (1u << k) - 1u)) {
      id_of_min_index[i] = (int32_t)t.canon.size();
      t.canon.push_back(mins[i]);
      t.mult.push_back(anchors_seeing(k, mins[i]));
    }
  }
  t.lut.assign(N, 0xFFFF);
  for (uint32_t x = 0; x < N; ++x) {
    size_t i = std::lower_bound(mins.begin(), mins.end(), orbit_min[x]) - mins.begin();
    if (id_of_min_index[i] >= 0) t.lut[x] = (uint16_t)id_of_min_index[i];
  }
  // Undirected classes: the all-reciprocated directed classes.  Undirected
  // code of such a class: edge {i, j} at und_bit(k, i, j); its canonical code
  // is the minimum over all k! relabellings; ids are ranks of the canonical
  // codes, ascending.
  std::vector<int> p(k);
  std::vector<uint32_t> und_code(t.canon.size(), 0);
  std::vector<char> symmetric(t.canon.size(), 0);
  for (size_t c = 0; c < t.canon.size(); ++c) {
    const uint32_t x = t.canon[c];
    bool sym = true;
    for (int i = 0; i < k && sym; ++i)
      for (int j = 0; j < k; ++j)
        if (i != j && ((x >> code_bit(k, i, j)) & 1u) != ((x >> code_bit(k, j, i)) & 1u)) sym = false;
    if (!sym) continue;
    symmetric[c] = 1;
    uint32_t best = UINT32_MAX;
    for (int i = 0; i < k; ++i) p[i] = i;
    do {
      uint32_t u = 0;
      for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j)
          if ((x >> code_bit(k, i, j)) & 1u) {
            const int a = std::min(p[i], p[j]), b2 = std::max(p[i], p[j]);
            u |= 1u << und_bit(k, a, b2);
          }
      best = std::min(best, u);
    } while (std::next_permutation(p.begin(), p.end()));
    und_code[c] = best;
    t.und_canon.push_back(best);
  }
  std::sort(t.und_canon.begin(), t.und_canon.end());
  t.und_of.assign(t.canon.size(), -1);
  for (size_t c = 0; c < t.canon.size(); ++c)
    if (symmetric[c])
      t.und_of[c] = (int16_t)(std::lower_bound(t.und_canon.begin(), t.und_canon.end(), und_code[c]) -
                              t.und_canon.begin());
  return t;
}

std::once_flag g_once[3];
ClassTable g_tables[3];

}  // namespace

const ClassTable* class_table(int k) {
  if (k < 3 || k > 5) return nullptr;
  std::call_once(g_once[k - 3], [k] { g_tables[k - 3] = build(k); });
  return &g_tables[k - 3];
}

}  // namespace motif
