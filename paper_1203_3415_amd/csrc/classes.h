// Host-side class tables for the census: code -> class id and per-class
// anchor multiplicities.  See classes.cpp.
#pragma once
#include <cstdint>
#include <vector>

namespace motif {

struct ClassTable {
  int k = 0;
  int nbits = 0;                 // k(k-1)
  std::vector<uint16_t> lut;     // [2^nbits] class id, 0xFFFF = disconnected
  std::vector<uint32_t> canon;   // [C] canonical (minimum) code of each class
  std::vector<uint8_t> mult;     // [C] anchors that see one occurrence
  // Undirected classes (the connected graphs on k vertices): the directed
  // classes whose arcs are all reciprocated, one per undirected graph.
  std::vector<int16_t> und_of;    // [C] undirected class of a directed class, -1 if an arc is one-way
  std::vector<uint32_t> und_canon; // [U] canonical undirected code of each undirected class
};

// Built once per k and cached (thread-safe).  k in {3,4,5}; nullptr otherwise.
const ClassTable* class_table(int k);

// Bit of the arc i -> j in a k-vertex code.
inline int code_bit(int k, int i, int j) { return i * (k - 1) + (j < i ? j : j - 1); }

// Bit of the edge {i, j}, i < j, in a k-vertex undirected code (k(k-1)/2 bits).
inline int und_bit(int k, int i, int j) { return i * (2 * k - i - 1) / 2 + (j - i - 1); }

}  // namespace motif
