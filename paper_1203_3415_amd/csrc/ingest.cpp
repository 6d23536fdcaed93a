// Reading networks from files into the int32 CSR the census takes.
//
// The paper's instances come from public network collections in the Pajek
// format and as plain edge lists, preprocessed by removing the vertices with
// no neighbours (Section "Results and Discussion").  This reader does the
// same on the host: it parses the file, drops self-loops, merges repeated
// arcs, removes the vertices of degree zero, renumbers the rest in the order
// of their ids in the file, and returns sorted out-CSR rows.
//
// Pajek (.net): a "*Vertices N" line, optionally followed by vertex lines
// ("id label ..."), then sections "*Arcs" / "*Edges" (one "u v [weight]" per
// line), "*Arcslist" / "*Edgeslist" ("u v1 v2 ..."), or "*Matrix" (N rows of
// N entries, non-zero = arc).  Ids are 1-based; an edge is both arcs.
// Keywords are matched without regard to case; "%" starts a comment line.
// Edge list: "u v [anything]" per line, ids non-negative integers, "#" or "%"
// starts a comment; each line is one arc u -> v (or an undirected edge with
// MOTIF_READ_UNDIRECTED).
#include <algorithm>
#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct Arc {
  int64_t u, v;
};

bool starts_with_ci(const char* s, const char* kw) {
  for (; *kw; ++s, ++kw)
    if (std::tolower((unsigned char)*s) != *kw) return false;
  return true;
}

const char* skip_ws(const char* p) {
  while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
  return p;
}

// Parses one integer token; returns false at the end of the line or on a
// token that is not an integer (which is then a parse error for ids).
bool next_int(const char*& p, int64_t* out, bool* bad) {
  p = skip_ws(p);
  if (!*p) return false;
  char* end = nullptr;
  errno = 0;
  const long long x = std::strtoll(p, &end, 10);
  if (end == p || errno == ERANGE || (*end && *end != ' ' && *end != '\t' && *end != '\r' && *end != '\n')) {
    *bad = true;
    return false;
  }
  p = end;
  *out = x;
  return true;
}

// Reads a whole line of any length.
bool read_line(FILE* f, std::string* line) {
  line->clear();
  char buf[4096];
  while (std::fgets(buf, sizeof buf, f)) {
    line->append(buf);
    if (!line->empty() && line->back() == '\n') return true;
  }
  return !line->empty();
}

enum Section { kNone, kVertices, kArcs, kEdges, kArcsList, kEdgesList, kMatrix };

int32_t parse_pajek(FILE* f, std::vector<Arc>* arcs, int64_t* nverts, motif_read_stats_t* st) {
  std::string line;
  Section sec = kNone;
  int64_t matrix_row = 0;
  *nverts = -1;
  while (read_line(f, &line)) {
    ++st->lines;
    const char* p = skip_ws(line.c_str());
    if (!*p || *p == '%') continue;
    if (*p == '*') {
      const char* kw = p + 1;
      if (starts_with_ci(kw, "vertices")) {
        bool bad = false;
        const char* q = kw + 8;
        int64_t nv = 0;
        if (!next_int(q, &nv, &bad) || nv < 0) return MOTIF_EPARSE;
        *nverts = nv;
        sec = kVertices;
      } else if (starts_with_ci(kw, "arcslist")) {
        sec = kArcsList;
      } else if (starts_with_ci(kw, "edgeslist")) {
        sec = kEdgesList;
      } else if (starts_with_ci(kw, "arcs")) {
        sec = kArcs;
      } else if (starts_with_ci(kw, "edges")) {
        sec = kEdges;
      } else if (starts_with_ci(kw, "matrix")) {
        sec = kMatrix;
        matrix_row = 0;
      } else {
        sec = kNone;  // another section (partitions, vectors, ...): skipped
      }
      continue;
    }
    if (*nverts < 0 && sec != kNone) return MOTIF_EPARSE;  // data before *Vertices
    bool bad = false;
    int64_t a = 0, b = 0;
    switch (sec) {
      case kNone:
      case kVertices:
        break;  // vertex lines carry labels and coordinates only
      case kArcs:
      case kEdges:
        if (!next_int(p, &a, &bad) || !next_int(p, &b, &bad)) return MOTIF_EPARSE;
        if (a < 1 || b < 1 || a > *nverts || b > *nverts) return MOTIF_EPARSE;
        arcs->push_back({a - 1, b - 1});
        if (sec == kEdges) arcs->push_back({b - 1, a - 1});
        break;
      case kArcsList:
      case kEdgesList:
        if (!next_int(p, &a, &bad) || a < 1 || a > *nverts) return MOTIF_EPARSE;
        while (next_int(p, &b, &bad)) {
          if (b < 1 || b > *nverts) return MOTIF_EPARSE;
          arcs->push_back({a - 1, b - 1});
          if (sec == kEdgesList) arcs->push_back({b - 1, a - 1});
        }
        if (bad) return MOTIF_EPARSE;
        break;
      case kMatrix: {
        if (matrix_row >= *nverts) return MOTIF_EPARSE;
        int64_t col = 0;
        while (*(p = skip_ws(p))) {
          char* end = nullptr;
          const double x = std::strtod(p, &end);
          if (end == p) return MOTIF_EPARSE;
          p = end;
          if (col >= *nverts) return MOTIF_EPARSE;
          if (x != 0.0) arcs->push_back({matrix_row, col});
          ++col;
        }
        if (col != *nverts) return MOTIF_EPARSE;
        ++matrix_row;
        break;
      }
    }
  }
  if (*nverts < 0) return MOTIF_EPARSE;
  return 0;
}

int32_t parse_edge_list(FILE* f, bool undirected, std::vector<Arc>* arcs, motif_read_stats_t* st) {
  std::string line;
  while (read_line(f, &line)) {
    ++st->lines;
    const char* p = skip_ws(line.c_str());
    if (!*p || *p == '#' || *p == '%') continue;
    bool bad = false;
    int64_t a = 0, b = 0;
    if (!next_int(p, &a, &bad)) return MOTIF_EPARSE;
    // the second id may be followed by anything (weights, timestamps)
    p = skip_ws(p);
    char* end = nullptr;
    errno = 0;
    b = std::strtoll(p, &end, 10);
    if (end == p || errno == ERANGE) return MOTIF_EPARSE;
    if (a < 0 || b < 0) return MOTIF_EPARSE;
    arcs->push_back({a, b});
    if (undirected) arcs->push_back({b, a});
  }
  return 0;
}

bool ends_with_ci(const char* s, const char* suf) {
  const size_t n = std::strlen(s), k = std::strlen(suf);
  if (k > n) return false;
  for (size_t i = 0; i < k; ++i)
    if (std::tolower((unsigned char)s[n - k + i]) != suf[i]) return false;
  return true;
}

}  // namespace

extern "C" {

int32_t motif_read_network(const char* path, int32_t format, int32_t flags, int32_t* n_out, int64_t* m_out,
                           int32_t** out_off, int32_t** out_idx, int64_t** orig_ids, motif_read_stats_t* stats) {
  if (!path || !n_out || !m_out || !out_off || !out_idx) return MOTIF_EINVAL_ARG;
  if (format == MOTIF_FORMAT_AUTO) format = ends_with_ci(path, ".net") ? MOTIF_FORMAT_PAJEK : MOTIF_FORMAT_EDGE_LIST;
  if (format != MOTIF_FORMAT_PAJEK && format != MOTIF_FORMAT_EDGE_LIST) return MOTIF_EINVAL_ARG;
  if (flags & ~(MOTIF_READ_UNDIRECTED | MOTIF_READ_KEEP_ISOLATED)) return MOTIF_EINVAL_ARG;
  motif_read_stats_t st{};
  FILE* f = std::fopen(path, "rb");
  if (!f) return MOTIF_EIO;
  std::vector<Arc> arcs;
  int64_t nverts = -1;
  int32_t rc;
  try {
    rc = format == MOTIF_FORMAT_PAJEK ? parse_pajek(f, &arcs, &nverts, &st)
                                      : parse_edge_list(f, (flags & MOTIF_READ_UNDIRECTED) != 0, &arcs, &st);
  } catch (const std::bad_alloc&) {
    rc = MOTIF_ENOMEM;
  }
  const bool read_error = std::ferror(f) != 0;
  std::fclose(f);
  if (rc) return rc;
  if (read_error) return MOTIF_EIO;
  st.arcs_read = (int64_t)arcs.size();
  try {
    // self-loops out, repeated arcs merged
    std::vector<Arc> keep;
    keep.reserve(arcs.size());
    for (const Arc& a : arcs) {
      if (a.u == a.v) ++st.self_loops_dropped;
      else keep.push_back(a);
    }
    std::vector<Arc>().swap(arcs);
    std::sort(keep.begin(), keep.end(), [](const Arc& x, const Arc& y) { return x.u < y.u || (x.u == y.u && x.v < y.v); });
    const size_t before = keep.size();
    keep.erase(std::unique(keep.begin(), keep.end(), [](const Arc& x, const Arc& y) { return x.u == y.u && x.v == y.v; }),
               keep.end());
    st.duplicates_merged = (int64_t)(before - keep.size());
    // the vertices kept, in the order of their ids in the file
    std::vector<int64_t> ids;
    if (format == MOTIF_FORMAT_PAJEK && (flags & MOTIF_READ_KEEP_ISOLATED)) {
      ids.resize((size_t)nverts);
      for (int64_t i = 0; i < nverts; ++i) ids[(size_t)i] = i;
    } else {
      ids.reserve(2 * keep.size());
      for (const Arc& a : keep) {
        ids.push_back(a.u);
        ids.push_back(a.v);
      }
      std::sort(ids.begin(), ids.end());
      ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
      if (format == MOTIF_FORMAT_PAJEK) st.isolated_dropped = nverts - (int64_t)ids.size();
    }
    if ((int64_t)ids.size() >= motif::kMaxN || (int64_t)keep.size() >= motif::kMaxN) return MOTIF_EINVAL_SHAPE;
    const int32_t n = (int32_t)ids.size();
    const int64_t m = (int64_t)keep.size();
    int32_t* off = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (size_t)(n + 1)));
    int32_t* idx = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, m)));
    int64_t* idv = orig_ids ? static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (size_t)std::max(1, n))) : nullptr;
    if (!off || !idx || (orig_ids && !idv)) {
      std::free(off);
      std::free(idx);
      std::free(idv);
      return MOTIF_ENOMEM;
    }
    auto rank = [&](int64_t id) { return (int32_t)(std::lower_bound(ids.begin(), ids.end(), id) - ids.begin()); };
    std::fill(off, off + n + 1, 0);
    for (const Arc& a : keep) ++off[rank(a.u) + 1];
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    // arcs are sorted by (u, v) and ranks keep the order, so rows come out sorted
    int64_t w = 0;
    for (const Arc& a : keep) idx[w++] = rank(a.v);
    if (idv) std::copy(ids.begin(), ids.end(), idv);
    *n_out = n;
    *m_out = m;
    *out_off = off;
    *out_idx = idx;
    if (orig_ids) *orig_ids = idv;
  } catch (const std::bad_alloc&) {
    return MOTIF_ENOMEM;
  }
  if (stats) *stats = st;
  return 0;
}

void motif_free(void* p) { std::free(p); }

}  // extern "C"
