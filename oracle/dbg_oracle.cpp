// TEST INFRASTRUCTURE ONLY -- the oracle.
//
// A plain, slow, obviously-correct CPU construction of the bi-directed de Bruijn
// graph of Kundeti, Rajasekaran, Dinh, Vaughn and Thapar ("Efficient parallel and
// out of core algorithms for constructing large bi-directed de Bruijn graphs").
// Only tests/, the smoke entry point and the CPU-baseline leg of the benchmark may
// load it.  It shares no code, header, table or helper with the GPU library: it
// works on std::string k-mers, compares them with std::string's operator<, and
// counts in std::map.  Nothing here is tuned.
//
// What it computes (all over the forward reads only, see the multiplicity reading
// in the design notes):
//   * nodes: every canonical k-mer (Sec. 2: the lexicographically smaller of a
//     k-mer and its reverse complement) with the number of read positions whose
//     k-mer canonicalises to it;
//   * edges: for every (k+1)-mer z of a read, the bi-directed edge of Sec. 2
//     between the k-molecules of (x, y) = (z[1..k], z[2..k+1]), in the canonical
//     form STEP-1 of algorithm BiConstruct (Sec. 3) gives it (with one reading for
//     the case x^ = y^); duplicates are removed and counted (STEP-2).
//   * edges are reported in ascending order of their canonical (k+1)-mer, nodes
//     in ascending k-mer order (the paper fixes no output order).
//
// Alphabet order: A < C < G < T (ASCII), which is the order under which the
// worked example of Sec. 2 (Fig. 2) calls GGA the positive strand of (GGA, TCC).
// Orientation: '+' (the paper's right-pointing head, positive strand) = 0,
// '-' (left-pointing head, negative strand) = 1.
//
// C ABI for ctypes (host memory only).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <string_view>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

const int PLUS = 0;   // right-pointing arrow head: the k-mer is the positive strand
const int MINUS = 1;  // left-pointing arrow head: the k-mer is the negative strand

char complement(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
  }
  return '?';
}

// Sec. 2: the reverse complement of s.
std::string reverse_complement(const std::string &s) {
  std::string r(s.rbegin(), s.rend());
  for (char &c : r) c = complement(c);
  return r;
}

// Sec. 2: the canonical k-mer is the lexicographically smaller of s and its
// reverse complement.
std::string canonical(const std::string &s) { return std::min(s, reverse_complement(s)); }

struct Edge {
  std::string u, v;
  int o1, o2;
  bool operator<(const Edge &b) const {
    return std::tie(u, v, o1, o2) < std::tie(b.u, b.v, b.o1, b.o2);
  }
};

int flip(int o) { return o == PLUS ? MINUS : PLUS; }

// The canonical bi-directed edge of a (k+1)-mer z.  Sec. 2: the consecutive k-mers
// x = z[1..k] and y = z[2..k+1] join the k-molecules of x and y, and the arrow head
// at each end says which strand of its molecule the k-mer is ('+' when it is the
// canonical k-mer).  The same adjacency read along the other strand is rc(y)
// followed by rc(x): the molecules swapped and both heads flipped.  STEP-1
// (Sec. 3) names every edge by one of these two readings: the one whose first
// molecule is the smaller.  When both molecules are the same it does not decide;
// the reading taken here keeps the one with the smaller orientation pair
// ('+' < '-'), so that a (k+1)-mer and its reverse complement get one record.
Edge step1_edge(const std::string &z, int k) {
  const std::string x = z.substr(0, k);
  const std::string y = z.substr(1, k);
  const std::string cx = canonical(x);
  const std::string cy = canonical(y);
  const int sx = (x == cx) ? PLUS : MINUS;
  const int sy = (y == cy) ? PLUS : MINUS;
  const Edge along = {cx, cy, sx, sy};
  const Edge against = {cy, cx, flip(sy), flip(sx)};
  if (cx < cy) return along;
  if (cy < cx) return against;
  const bool along_first = std::make_pair(along.o1, along.o2) <= std::make_pair(against.o1, against.o2);
  return along_first ? along : against;
}

// The string an edge record spells: sigma(u, o1) followed by the last base of
// sigma(v, o2), where sigma(w, +) = w and sigma(w, -) = reverse complement of w.
std::string edge_spelling(const Edge &e) {
  const std::string a = (e.o1 == PLUS) ? e.u : reverse_complement(e.u);
  const std::string b = (e.o2 == PLUS) ? e.v : reverse_complement(e.v);
  return a + b.substr(b.size() - 1);
}

// The oracle's own packer: base-4 value of a string, first base most
// significant, A=0 C=1 G=2 T=3, as two 64-bit words (lo, hi).
void pack_string(const std::string &s, uint64_t *lo, uint64_t *hi) {
  uint64_t l = 0, h = 0;
  for (char c : s) {
    uint64_t code = 0;
    switch (c) {
      case 'A': code = 0; break;
      case 'C': code = 1; break;
      case 'G': code = 2; break;
      case 'T': code = 3; break;
    }
    h = (h << 2) | (l >> 62);
    l = (l << 2) | code;
  }
  *lo = l;
  *hi = h;
}

struct Counts {
  std::map<std::string, uint64_t> nodes;
  std::map<Edge, uint64_t> edges;
};

// Count the k-mers and (k+1)-mers of reads [r0, r1).
void count_reads(const char *bases, const uint64_t *offsets, uint64_t r0, uint64_t r1, int k,
                 Counts *out) {
  for (uint64_t i = r0; i < r1; ++i) {
    const std::string read(bases + offsets[i], bases + offsets[i + 1]);
    const uint64_t len = read.size();
    for (uint64_t j = 0; j + k <= len; ++j) out->nodes[canonical(read.substr(j, k))] += 1;
    for (uint64_t j = 0; j + k + 1 <= len; ++j) out->edges[step1_edge(read.substr(j, k + 1), k)] += 1;
  }
}

struct Result {
  int k = 0;
  std::vector<std::pair<std::string, uint64_t>> nodes;  // ascending k-mer
  struct Row {
    std::string z;  // canonical (k+1)-mer spelled by the edge
    Edge e;
    uint64_t mult;
  };
  std::vector<Row> edges;  // ascending canonical (k+1)-mer
  int status = 0;          // 0 ok; 1 two distinct edges spelled the same (k+1)-mer
};

int resolve_threads(int n_threads) {
  if (n_threads > 0) return n_threads;
  const unsigned hc = std::thread::hardware_concurrency();
  return hc ? static_cast<int>(hc) : 1;
}

}  // namespace

extern "C" {

// Reverse complement of n bases; out must hold n bytes.  Returns 0, or 1 when a
// byte is not one of A, C, G, T.
int oracle_revcomp(const char *s, uint64_t n, char *out) {
  const std::string r = reverse_complement(std::string(s, s + n));
  std::memcpy(out, r.data(), n);
  return r.find('?') == std::string::npos ? 0 : 1;
}

// Build the graph of reads bases[offsets[i] .. offsets[i+1]) for i < n_reads.
// Bases must be upper-case A, C, G, T.  n_threads <= 0 uses every host core; the
// result does not depend on it.  Returns an opaque handle (free with oracle_free).
void *oracle_build(const char *bases, const uint64_t *offsets, uint64_t n_reads, int k,
                   int n_threads) {
  const int T = std::max(1, std::min<int>(resolve_threads(n_threads),
                                          static_cast<int>(std::max<uint64_t>(n_reads, 1))));
  std::vector<Counts> part(T);
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) {
    const uint64_t r0 = n_reads * t / T, r1 = n_reads * (t + 1) / T;
    pool.emplace_back(count_reads, bases, offsets, r0, r1, k, &part[t]);
  }
  for (auto &th : pool) th.join();
  // Merge the per-thread ordered maps into the first one.
  Counts &all = part[0];
  for (int t = 1; t < T; ++t) {
    for (const auto &kv : part[t].nodes) all.nodes[kv.first] += kv.second;
    for (const auto &kv : part[t].edges) all.edges[kv.first] += kv.second;
    part[t] = Counts();
  }
  Result *res = new Result;
  res->k = k;
  res->nodes.assign(all.nodes.begin(), all.nodes.end());
  for (const auto &kv : all.edges)
    res->edges.push_back({canonical(edge_spelling(kv.first)), kv.first, kv.second});
  std::sort(res->edges.begin(), res->edges.end(),
            [](const Result::Row &a, const Result::Row &b) { return a.z < b.z; });
  for (size_t i = 1; i < res->edges.size(); ++i)
    if (res->edges[i].z == res->edges[i - 1].z) res->status = 1;
  return res;
}

int oracle_status(void *h) { return static_cast<Result *>(h)->status; }
uint64_t oracle_n_nodes(void *h) { return static_cast<Result *>(h)->nodes.size(); }
uint64_t oracle_n_edges(void *h) { return static_cast<Result *>(h)->edges.size(); }

// Node table as packed words: key2[2*i] = lo, key2[2*i+1] = hi.
void oracle_get_nodes(void *h, uint64_t *key2, uint64_t *count) {
  const Result *r = static_cast<Result *>(h);
  for (size_t i = 0; i < r->nodes.size(); ++i) {
    pack_string(r->nodes[i].first, &key2[2 * i], &key2[2 * i + 1]);
    count[i] = r->nodes[i].second;
  }
}

// Edge list as packed words; orient = (o1 << 1) | o2.
void oracle_get_edges(void *h, uint64_t *u2, uint64_t *v2, uint8_t *orient, uint64_t *mult,
                      uint64_t *z2) {
  const Result *r = static_cast<Result *>(h);
  for (size_t i = 0; i < r->edges.size(); ++i) {
    const auto &row = r->edges[i];
    pack_string(row.e.u, &u2[2 * i], &u2[2 * i + 1]);
    pack_string(row.e.v, &v2[2 * i], &v2[2 * i + 1]);
    orient[i] = static_cast<uint8_t>((row.e.o1 << 1) | row.e.o2);
    mult[i] = row.mult;
    pack_string(row.z, &z2[2 * i], &z2[2 * i + 1]);
  }
}

// String views for small cases.  buf receives k (node) bytes, or k, k and k+1
// bytes for u, v and z (edge); no terminator is written.
void oracle_node_str(void *h, uint64_t i, char *buf) {
  const Result *r = static_cast<Result *>(h);
  std::memcpy(buf, r->nodes[i].first.data(), r->k);
}
void oracle_edge_str(void *h, uint64_t i, char *ubuf, char *vbuf, char *zbuf) {
  const Result *r = static_cast<Result *>(h);
  std::memcpy(ubuf, r->edges[i].e.u.data(), r->k);
  std::memcpy(vbuf, r->edges[i].e.v.data(), r->k);
  std::memcpy(zbuf, r->edges[i].z.data(), r->k + 1);
}

void oracle_free(void *h) { delete static_cast<Result *>(h); }

// Probe counts over all reads without building the whole graph: for each of the
// n_np node probes (k bytes each, concatenated) the number of read positions
// whose k-mer canonicalises to it, and for each of the n_ep edge probes (u, v as
// k bytes each, orient byte) the number of (k+1)-mers whose STEP-1 edge is that
// record.  Used for sampled checks at sizes the full oracle cannot hold in memory.
//
// Only a few windows can count toward a probe, and they are found by exact
// string match before anything is canonicalised.  The canonical k-mer of a window
// w is w or rc(w) (Sec. 2), so it equals p only if w is p or rc(p).  The edge of a
// (k+1)-mer w, read back through its spelling (edge_spelling), spells w along one
// of its two strands: the record (x^, y^, s_x, s_y) spells x followed by the last
// base of y, which is w, and the swapped record (y^, x^, not s_y, not s_x)
// spells rc(y) followed by the last base of rc(x), which is rc(w).  So a window
// can have record e only if it is spell(e) or rc(spell(e)).  Every window equal to
// one of those two strings is then canonicalised, or given its STEP-1 edge, and
// compared with the probe exactly as the full build would count it.
void oracle_probe(const char *bases, const uint64_t *offsets, uint64_t n_reads, int k,
                  int n_threads, const char *node_probes, uint64_t n_np, uint64_t *node_counts,
                  const char *edge_u, const char *edge_v, const uint8_t *edge_orient,
                  uint64_t n_ep, uint64_t *edge_counts) {
  std::vector<std::string> node_key(n_np);
  std::vector<Edge> edge_key(n_ep);
  // both strands of every probe's spelling -> the probes that spelling can match
  std::vector<std::string> spellings;
  spellings.reserve(2 * (n_np + n_ep));
  for (uint64_t i = 0; i < n_np; ++i) {
    node_key[i] = std::string(node_probes + i * k, node_probes + (i + 1) * k);
    spellings.push_back(node_key[i]);
    spellings.push_back(reverse_complement(node_key[i]));
  }
  for (uint64_t i = 0; i < n_ep; ++i) {
    edge_key[i] = Edge{std::string(edge_u + i * k, edge_u + (i + 1) * k),
                       std::string(edge_v + i * k, edge_v + (i + 1) * k), edge_orient[i] >> 1,
                       edge_orient[i] & 1};
    const std::string s = edge_spelling(edge_key[i]);
    spellings.push_back(s);
    spellings.push_back(reverse_complement(s));
  }
  std::unordered_map<std::string_view, std::vector<uint64_t>> node_match, edge_match;
  for (uint64_t i = 0; i < n_np; ++i)
    for (int r = 0; r < 2; ++r) {
      auto &probes = node_match[spellings[2 * i + r]];
      if (probes.empty() || probes.back() != i) probes.push_back(i);
    }
  for (uint64_t i = 0; i < n_ep; ++i)
    for (int r = 0; r < 2; ++r) {
      auto &probes = edge_match[spellings[2 * (n_np + i) + r]];
      if (probes.empty() || probes.back() != i) probes.push_back(i);
    }
  const int T = std::max(1, std::min<int>(resolve_threads(n_threads),
                                          static_cast<int>(std::max<uint64_t>(n_reads, 1))));
  std::vector<std::vector<uint64_t>> nc(T, std::vector<uint64_t>(n_np, 0));
  std::vector<std::vector<uint64_t>> ec(T, std::vector<uint64_t>(n_ep, 0));
  auto work = [&](int t) {
    const uint64_t r0 = n_reads * t / T, r1 = n_reads * (t + 1) / T;
    for (uint64_t i = r0; i < r1; ++i) {
      const std::string_view read(bases + offsets[i], offsets[i + 1] - offsets[i]);
      const uint64_t len = read.size();
      for (uint64_t j = 0; j + k <= len; ++j) {
        auto it = node_match.find(read.substr(j, k));
        if (it == node_match.end()) continue;
        const std::string c = canonical(std::string(read.substr(j, k)));
        for (uint64_t p : it->second)
          if (c == node_key[p]) nc[t][p] += 1;
      }
      for (uint64_t j = 0; j + k + 1 <= len; ++j) {
        auto it = edge_match.find(read.substr(j, k + 1));
        if (it == edge_match.end()) continue;
        const Edge e = step1_edge(std::string(read.substr(j, k + 1)), k);
        for (uint64_t p : it->second) {
          const Edge &q = edge_key[p];
          if (e.u == q.u && e.v == q.v && e.o1 == q.o1 && e.o2 == q.o2) ec[t][p] += 1;
        }
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) pool.emplace_back(work, t);
  for (auto &th : pool) th.join();
  for (uint64_t i = 0; i < n_np; ++i) {
    node_counts[i] = 0;
    for (int t = 0; t < T; ++t) node_counts[i] += nc[t][i];
  }
  for (uint64_t i = 0; i < n_ep; ++i) {
    edge_counts[i] = 0;
    for (int t = 0; t < T; ++t) edge_counts[i] += ec[t][i];
  }
}

int oracle_threads(int n_threads) { return resolve_threads(n_threads); }

}  // extern "C"
