// STEP-4 of Sec. 3: adjacency lists of the bi-directed graph from its node table
// and edge list.
//
// A node has two sides: side 0, by which a walk reading its canonical k-mer
// forward leaves it, and side 1, by which such a walk enters it.  The record
// (u, v, o1, o2) of a (k+1)-mer leaves u by side 0 when o1 = '+' (side 1 when
// '-') and enters v by side 1 when o2 = '+' (side 0 when '-'): its u end lies on
// side o1 and its v end on side 1 - o2 ('+' = 0).  These sides do not change when
// a record is written with its endpoints swapped, (v, u, not o2, not o1), as the
// STEP-1 table does in its ELSE branches.  The lists group the ends by (node,
// side), nodes in table order and side 0 first, and order each group by edge
// row, u end first.  As a CSR: bucket b = 2 * node + side holds entries
// offsets[b] .. offsets[b + 1] of (edge row, end).  Optionally the bucket of
// both ends of every edge (2 * node + side) is returned as well.
//
//   1. k_adj_index: a prefix index over the sorted node keys (first row of every
//      B-bit key prefix), so an endpoint is found by one index read and a
//      binary search over a few rows;
//   2. k_adj_count: each edge finds the rows of its endpoints, records the two
//      buckets and counts them, keeping each end's arrival rank in its bucket
//      (a side of a k-mer is an end of at most four distinct (k+1)-mers, so at
//      most eight ends: a byte);
//   3. k_adj_scan_*: exclusive scan of the bucket counts into the offsets;
//   4. k_adj_scatter: each incidence goes to its bucket's offset plus its rank
//      (no atomics);
//   5. k_adj_order: each bucket (at most a few entries: a side of a k-mer has
//      at most four one-base extensions, counted for both ends of an edge) is
//      sorted by (edge row, end).
#include "dbg_device.h"
#include "../../include/dbg.h"

namespace dbg {

constexpr int ADJ_NT = 256;
constexpr uint64_t ADJ_SCAN_TILE = (uint64_t)ADJ_NT * 16;

__device__ __forceinline__ void adj_status(dbg_result_t *res, uint32_t code) {
  atomicCAS(&res->status, 0u, code);
}

template <typename K> __device__ __forceinline__ uint64_t key_prefix(K key, int shift) {
  return (uint64_t)shr<K>(key, shift);
}

// first[p] = first row whose key prefix is >= p, for p in [0, 2^B]; every row
// writes the index entries from the previous row's prefix (exclusive) to its
// own (inclusive), and the last row also the ones after its prefix.
template <typename K>
__global__ __launch_bounds__(ADJ_NT) void k_adj_index(const K *keys, uint64_t n, int shift,
                                                      uint32_t nbins, uint32_t *first) {
  for (uint64_t i = blockIdx.x * (uint64_t)ADJ_NT + threadIdx.x; i <= n;
       i += (uint64_t)gridDim.x * ADJ_NT) {
    const uint64_t p = i < n ? key_prefix(keys[i], shift) : (uint64_t)nbins;
    const uint64_t q = i == 0 ? 0 : key_prefix(keys[i - 1], shift) + 1;
    for (uint64_t b = q; b <= p && b <= nbins; ++b) first[b] = (uint32_t)i;
  }
}

// Row of `key` in the node table, or n if absent.  The bounds are clamped so
// that keys wider than 2k bits or an unsorted table cannot lead outside it.
template <typename K>
__device__ __forceinline__ uint64_t adj_find(const K *keys, uint64_t n, const uint32_t *first,
                                             uint32_t nbins, int shift, K key) {
  const uint64_t p = key_prefix(key, shift);
  if (p >= nbins) return n;
  uint64_t hi = first[p + 1], lo = first[p];
  hi = hi < n ? hi : n;
  lo = lo < hi ? lo : hi;
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && keys[lo] == key ? lo : n;
}

template <typename K>
__global__ __launch_bounds__(ADJ_NT) void k_adj_count(const K *keys, uint64_t n,
                                                      const uint32_t *first, uint32_t nbins,
                                                      int shift,
                                                      const K *eu, const K *ev,
                                                      const uint8_t *orient, uint64_t m,
                                                      uint32_t *bucket, uint32_t *counts,
                                                      uint8_t *rank, uint32_t *edge_bucket,
                                                      dbg_result_t *res) {
  for (uint64_t j = blockIdx.x * (uint64_t)ADJ_NT + threadIdx.x; j < m;
       j += (uint64_t)gridDim.x * ADJ_NT) {
    const uint32_t o = orient[j];
    const uint64_t iu = adj_find(keys, n, first, nbins, shift, eu[j]);
    const uint64_t iv = adj_find(keys, n, first, nbins, shift, ev[j]);
    if (iu >= n || iv >= n || o > 3u) {
      adj_status(res, DBG_E_ARG);  // an endpoint is not in the node table
      bucket[2 * j] = bucket[2 * j + 1] = 0xffffffffu;
      continue;
    }
    const uint32_t bu = (uint32_t)(2 * iu + (o >> 1)), bv = (uint32_t)(2 * iv + ((o & 1u) ^ 1u));
    bucket[2 * j] = bu;
    bucket[2 * j + 1] = bv;
    if (edge_bucket) {
      edge_bucket[2 * j] = bu;
      edge_bucket[2 * j + 1] = bv;
    }
    const uint32_t ru = atomicAdd(&counts[bu], 1u), rv = atomicAdd(&counts[bv], 1u);
    if (ru > 255u || rv > 255u) adj_status(res, DBG_E_ARG);  // not a read set's graph
    rank[2 * j] = (uint8_t)ru;
    rank[2 * j + 1] = (uint8_t)rv;
  }
}

// Exclusive scan of nb = 2n bucket counts into offsets[0 .. nb] (u64).
__global__ __launch_bounds__(ADJ_NT) void k_adj_scan_reduce(const uint32_t *counts,
                                                            uint64_t nb, uint64_t *sums) {
  __shared__ uint64_t wsum[ADJ_NT / 64 + 1];
  const uint64_t base = blockIdx.x * ADJ_SCAN_TILE + threadIdx.x * (uint64_t)16;
  uint64_t s = 0;
  for (int r = 0; r < 16; ++r)
    if (base + r < nb) s += counts[base + r];
  uint64_t tot;
  block_exclusive_scan<ADJ_NT>(s, wsum, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_adj_scan_sums(uint64_t *a, uint64_t n) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < n; c0 += 1024) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t v = i < n ? a[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<1024>(v, wsum, &tot) + carry;
    if (i < n) a[i] = ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(ADJ_NT) void k_adj_scan_apply(const uint32_t *counts, uint64_t nb,
                                                           const uint64_t *sums,
                                                           uint64_t *offsets) {
  __shared__ uint64_t wsum[ADJ_NT / 64 + 1];
  const uint64_t base = blockIdx.x * ADJ_SCAN_TILE + threadIdx.x * (uint64_t)16;
  uint32_t c[16];
  uint64_t s = 0;
  for (int r = 0; r < 16; ++r) {
    c[r] = base + r < nb ? counts[base + r] : 0u;
    s += c[r];
  }
  uint64_t tot;
  uint64_t ex = block_exclusive_scan<ADJ_NT>(s, wsum, &tot) + sums[blockIdx.x];
  for (int r = 0; r < 16; ++r) {
    if (base + r <= nb) offsets[base + r] = ex;  // offsets[nb] = total
    ex += c[r];
  }
}

// Each incidence goes to its bucket's offset plus its arrival rank; k_adj_order
// fixes the order inside the bucket.
__global__ __launch_bounds__(ADJ_NT) void k_adj_scatter(const uint32_t *bucket,
                                                        const uint8_t *rank, uint64_t m,
                                                        const uint64_t *offsets,
                                                        uint32_t *inc_edge, uint8_t *inc_end,
                                                        const dbg_result_t *res) {
  if (res->status) return;
  for (uint64_t t = blockIdx.x * (uint64_t)ADJ_NT + threadIdx.x; t < 2 * m;
       t += (uint64_t)gridDim.x * ADJ_NT) {
    const uint64_t pos = offsets[bucket[t]] + rank[t];
    inc_edge[pos] = (uint32_t)(t >> 1);
    inc_end[pos] = (uint8_t)(t & 1);
  }
}

__global__ __launch_bounds__(ADJ_NT) void k_adj_order(const uint64_t *offsets, uint64_t nb,
                                                      uint32_t *inc_edge, uint8_t *inc_end,
                                                      const dbg_result_t *res) {
  if (res->status) return;
  for (uint64_t b = blockIdx.x * (uint64_t)ADJ_NT + threadIdx.x; b < nb;
       b += (uint64_t)gridDim.x * ADJ_NT) {
    const uint64_t s = offsets[b], e = offsets[b + 1];
    // insertion sort by (edge row, end): buckets hold a few entries
    for (uint64_t i = s + 1; i < e; ++i) {
      const uint32_t ke = inc_edge[i];
      const uint8_t kd = inc_end[i];
      const uint64_t key = ((uint64_t)ke << 1) | kd;
      uint64_t j = i;
      while (j > s && ((((uint64_t)inc_edge[j - 1]) << 1) | inc_end[j - 1]) > key) {
        inc_edge[j] = inc_edge[j - 1];
        inc_end[j] = inc_end[j - 1];
        --j;
      }
      inc_edge[j] = ke;
      inc_end[j] = kd;
    }
  }
}

__global__ void k_adj_result(dbg_result_t *res, uint64_t n, uint64_t m) {
  if (threadIdx.x || blockIdx.x) return;
  res->n_nodes = n;
  res->n_edges = m;
  res->flags = 0;
}

__global__ void k_adj_init(dbg_result_t *res) {
  if (threadIdx.x || blockIdx.x) return;
  res->status = 0;
}

__global__ __launch_bounds__(ADJ_NT) void k_adj_zero(uint32_t *a, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)ADJ_NT + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * ADJ_NT)
    a[i] = 0;
}

static inline unsigned adj_grid(uint64_t n, uint64_t cap) {
  uint64_t g = (n + ADJ_NT - 1) / ADJ_NT;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

static inline size_t adj_align(size_t x) { return (x + 255) & ~size_t(255); }

struct AdjLayout {
  size_t first, bucket, counts, rank, sums, total;
  int bits, shift;
  uint32_t nbins;
};

static AdjLayout adj_layout(uint64_t n, uint64_t m, int k) {
  AdjLayout L{};
  int b = 1;
  while (b < 24 && (1ull << (b + 3)) < n) ++b;  // about eight rows per prefix
  if (b > 2 * k) b = 2 * k;
  L.bits = b;
  L.shift = 2 * k - b;
  L.nbins = 1u << b;
  const uint64_t nb = 2 * n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = adj_align(off + bytes);
    return o;
  };
  L.first = take(((size_t)L.nbins + 1) * sizeof(uint32_t));
  L.bucket = take((size_t)(2 * m) * sizeof(uint32_t));
  L.counts = take((size_t)nb * sizeof(uint32_t));
  L.rank = take((size_t)(2 * m));
  L.sums = take((size_t)(nb / ADJ_SCAN_TILE + 1) * sizeof(uint64_t));
  L.total = off;
  return L;
}

template <typename K>
static hipError_t run_adjacency(const void *node_kmer, uint64_t n, const void *eu, const void *ev,
                                const uint8_t *orient, uint64_t m, const AdjLayout &L,
                                uint64_t *offsets, uint32_t *inc_edge, uint8_t *inc_end,
                                uint32_t *edge_bucket, dbg_result_t *res, char *ws,
                                hipStream_t st) {
  const K *keys = static_cast<const K *>(node_kmer);
  uint32_t *first = reinterpret_cast<uint32_t *>(ws + L.first);
  uint32_t *bucket = reinterpret_cast<uint32_t *>(ws + L.bucket);
  uint32_t *counts = reinterpret_cast<uint32_t *>(ws + L.counts);
  uint8_t *rank = reinterpret_cast<uint8_t *>(ws + L.rank);
  uint64_t *sums = reinterpret_cast<uint64_t *>(ws + L.sums);
  const uint64_t nb = 2 * n;
  const uint64_t nsum = nb / ADJ_SCAN_TILE + 1;
  hipLaunchKernelGGL(k_adj_init, dim3(1), dim3(1), 0, st, res);
  hipLaunchKernelGGL(k_adj_zero, dim3(adj_grid(nb, 8192)), dim3(ADJ_NT), 0, st, counts, nb);
  hipLaunchKernelGGL(k_adj_index<K>, dim3(adj_grid(n + 1, 8192)), dim3(ADJ_NT), 0, st, keys, n,
                     L.shift, L.nbins, first);
  hipLaunchKernelGGL(k_adj_count<K>, dim3(adj_grid(m, 16384)), dim3(ADJ_NT), 0, st, keys, n,
                     first, L.nbins, L.shift, static_cast<const K *>(eu), static_cast<const K *>(ev),
                     orient, m, bucket, counts, rank, edge_bucket, res);
  hipLaunchKernelGGL(k_adj_scan_reduce, dim3((unsigned)nsum), dim3(ADJ_NT), 0, st, counts, nb,
                     sums);
  hipLaunchKernelGGL(k_adj_scan_sums, dim3(1), dim3(1024), 0, st, sums, nsum);
  hipLaunchKernelGGL(k_adj_scan_apply, dim3((unsigned)nsum), dim3(ADJ_NT), 0, st, counts, nb,
                     sums, offsets);
  hipLaunchKernelGGL(k_adj_scatter, dim3(adj_grid(2 * m, 16384)), dim3(ADJ_NT), 0, st, bucket,
                     rank, m, offsets, inc_edge, inc_end, res);
  hipLaunchKernelGGL(k_adj_order, dim3(adj_grid(nb, 16384)), dim3(ADJ_NT), 0, st, offsets, nb,
                     inc_edge, inc_end, res);
  hipLaunchKernelGGL(k_adj_result, dim3(1), dim3(1), 0, st, res, n, m);
  return hipGetLastError();
}

}  // namespace dbg

extern "C" {

size_t dbg_adjacency_workspace_bytes(uint64_t n_nodes, uint64_t n_edges, int k) {
  if (k < 1 || k > 63 || (k & 1) == 0) return 0;
  return dbg::adj_layout(n_nodes, n_edges, k).total;
}

int dbg_adjacency(const void *node_kmer, uint64_t n_nodes, const void *edge_u,
                  const void *edge_v, const uint8_t *edge_orient, uint64_t n_edges, int k,
                  uint64_t *offsets, uint32_t *inc_edge, uint8_t *inc_end, uint32_t *edge_bucket,
                  dbg_result_t *result, void *workspace, size_t workspace_bytes,
                  hipStream_t stream) {
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (!offsets || !result || !workspace) return DBG_E_NULL;
  if (n_nodes && !node_kmer) return DBG_E_NULL;
  if (n_edges && (!edge_u || !edge_v || !edge_orient || !inc_edge || !inc_end)) return DBG_E_NULL;
  if (n_edges && !n_nodes) return DBG_E_ARG;
  if (n_nodes >= (1ull << 31) || n_edges >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DBG_E_WORKSPACE;
  const dbg::AdjLayout L = dbg::adj_layout(n_nodes, n_edges, k);
  if (workspace_bytes < L.total) return DBG_E_WORKSPACE;
  char *ws = static_cast<char *>(workspace);
  const hipError_t e =
      k <= 31 ? dbg::run_adjacency<uint64_t>(node_kmer, n_nodes, edge_u, edge_v, edge_orient,
                                             n_edges, L, offsets, inc_edge, inc_end, edge_bucket,
                                             result, ws, stream)
              : dbg::run_adjacency<unsigned __int128>(node_kmer, n_nodes, edge_u, edge_v,
                                                      edge_orient, n_edges, L, offsets, inc_edge,
                                                      inc_end, edge_bucket, result, ws, stream);
  return e == hipSuccess ? DBG_OK : DBG_E_HIP;
}

}  // extern "C"
