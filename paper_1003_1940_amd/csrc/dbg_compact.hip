// Bi-directed chain compaction (Sec. 7): the simplified graph of a built graph,
// from its node keys and STEP-4 adjacency lists (with the bucket of every edge
// end).
//
// Sides are those of the adjacency lists: side 0 of a node is left, side 1
// entered, by a walk reading its canonical k-mer forward.  An edge is a candidate
// when it is not a self-loop and each of its ends is the only end on its side
// (the per-end reading of the paper's "one in- and one out-edge" criterion).
//
// ListRankingTransform: node v has two copies, state 2v (v read forward) and
// 2v + 1 (read reverse-complemented).  Leaving state 2v + t is leaving v by side
// t; entering 2v + t is entering by side 1 - t.  One array holds, for every
// (node, side) bucket b = 2v + s, the bucket at the other end of its candidate
// edge, or NIL.  With that array, link:
//   succ(2v + t) = link[2v + t] ^ 1     (leave by side t, enter the other copy)
//   pred(2v + t) = link[2v + (t ^ 1)]   (entered by side 1 - t)
// so every state has at most one successor and one predecessor: lists and
// cycles, each with a twin that runs the other way.
//
// List ranking: every state holds one 64-bit word (pointer, done, rank).  First
// every list head walks its list and ranks its first CMP_WALK states directly
// (one read and one write per state; most chains of a read set's graph are
// short).  The states left -- deeper in long lists, or on cycles -- are ranked
// by Wyllie's pointer jumping, which continues from the walked states: a round
// replaces a pending state's pointer by its target's pointer and adds the
// target's rank; a state whose target is a head, or has already found its head,
// is done.  States are updated in place: a
// target word read while it changes is still a valid (state, distance) pair, so
// a round only ever jumps further.  Pending states are kept on a worklist that
// shrinks every round.  After ceil(log2(2n)) + 1 rounds every list state is done
// (ranks are below n < 2^31); the states left are on cycles.  Each cycle is
// broken on the fly at its smallest node (a min-label pointer jump over the
// cycle states finds it): the cycle through v+ of the smallest node v starts at
// v+, its twin ends at v-; then the ranking runs again on those states.
//
// Canonical copy: per node, both of its states know their list's head and their
// rank; the chain is the copy whose first k-mer (the head state's k-mer in its
// orientation) is smaller, or for a broken cycle the copy that starts at v+.
// Chains shorter than min_nodes (other than single nodes) are dissolved into
// single nodes.  Two exclusive scans number the chains in the order of their
// first node (and place their labels), and the kept edges in row order.
#include "dbg_device.h"
#include "../../include/dbg.h"

namespace dbg {

constexpr int CMP_NT = 256;
constexpr uint32_t CMP_NIL = 0xffffffffu;
constexpr uint64_t CMP_TILE = (uint64_t)CMP_NT * 16;
constexpr unsigned CMP_ROUND_GRID = 2048;
constexpr int CMP_MAX_COUNTERS = 112;
constexpr uint32_t CMP_WALK = 256;  // list states a head's walk ranks before jumping takes over

__device__ __forceinline__ void cmp_status(dbg_compact_result_t *res, uint32_t code) {
  atomicCAS(&res->status, 0u, code);
}

// jump word: [63:32] pointer (a state, or NIL for a head), [31] done, [30:0] rank
__device__ __forceinline__ uint64_t jword(uint32_t p, uint32_t done, uint32_t r) {
  return ((uint64_t)p << 32) | ((uint64_t)done << 31) | (uint64_t)r;
}
__device__ __forceinline__ uint32_t jptr(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ uint32_t jdone(uint64_t w) { return (uint32_t)(w >> 31) & 1u; }
__device__ __forceinline__ uint32_t jrank(uint64_t w) { return (uint32_t)w & 0x7fffffffu; }

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends `x` for every thread with `keep` set: one atomic per workgroup.  Every
// thread of the workgroup must call it (it holds barriers).
__device__ __forceinline__ void block_append(bool keep, uint32_t x, uint32_t *list,
                                             uint32_t *count, uint32_t *lds) {
  constexpr int NW = CMP_NT / 64;
  const uint64_t bal = __ballot(keep);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) lds[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int i = 0; i < NW; ++i) {
      const uint32_t c = lds[i];
      lds[i] = tot;
      tot += c;
    }
    lds[NW] = tot ? atomicAdd(count, tot) : 0u;
  }
  __syncthreads();
  if (keep) list[lds[NW] + lds[w] + __popcll(bal & lanemask_lt())] = x;
  __syncthreads();
}

__global__ __launch_bounds__(CMP_NT) void k_cmp_init(uint32_t *counters, uint32_t *cycmin,
                                                     uint64_t n, dbg_compact_result_t *res) {
  const uint64_t t0 = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x;
  if (t0 < (uint64_t)CMP_MAX_COUNTERS) counters[t0] = 0;
  if (t0 == 0) {
    res->n_chains = res->n_kept = res->label_len = 0;
    res->status = 0;
    res->n_cyclic = 0;
  }
  for (uint64_t v = t0; v < n; v += (uint64_t)gridDim.x * CMP_NT) cycmin[v] = CMP_NIL;
}

template <typename K>
__device__ __forceinline__ K state_kmer(const K *keys, uint32_t s, int k) {
  const K key = keys[s >> 1];
  return (s & 1u) ? revcomp(key, k) : key;
}

// A node's place in its chain, as a walk finds it: the chain's first node, the
// node's rank and orientation along the canonical walk, the chain length.
// head = NIL: not placed by a walk (a single node, or a long list or cycle that
// pointer jumping ranks).
struct alignas(16) NRec {
  uint32_t head;
  uint32_t rank;
  uint32_t len;
  uint32_t orient;
};

// Bit b of `single` is set when bucket b holds exactly one end: one bucket per
// lane, a wave's 64 bits assembled by a ballot (read as 32-bit words, little
// endian).
__global__ __launch_bounds__(CMP_NT) void k_cmp_single(const uint64_t *off, uint64_t nb,
                                                       uint64_t *single) {
  for (uint64_t base = blockIdx.x * (uint64_t)CMP_NT; base < nb;
       base += (uint64_t)gridDim.x * CMP_NT) {
    const uint64_t b = base + threadIdx.x;
    const bool one = b < nb && off[b + 1] == off[b] + 1;
    const uint64_t bits = __ballot(one);
    if (lane_id() == 0) single[b >> 6] = bits;
  }
}

// Per node v: the links of both sides s -- the bucket at the other end of the
// edge whose end is alone on side s of v, when that end too is alone on its side
// and the edge is not a self-loop; NIL otherwise -- and an empty place record.
// A node linked on one side only ends a chain: its state with a successor but no
// predecessor heads a list and is recorded in the workgroup's own segment of
// `heads` (nodes [blockIdx.x * chunk, ...) give at most that many heads; no
// global atomics).
__global__ __launch_bounds__(CMP_NT) void k_cmp_links(const uint64_t *off, uint64_t n,
                                                      const uint32_t *inc_edge,
                                                      const uint8_t *inc_end,
                                                      const uint32_t *edge_bucket, uint64_t m,
                                                      const uint32_t *single, uint64_t chunk,
                                                      uint32_t *link, NRec *place,
                                                      uint32_t *heads, uint32_t *seg_count,
                                                      dbg_compact_result_t *res) {
  __shared__ uint32_t seg;
  if (threadIdx.x == 0) seg = 0;
  __syncthreads();
  const uint64_t v0 = blockIdx.x * chunk;
  const uint64_t v1 = v0 + chunk < n ? v0 + chunk : n;
  for (uint64_t v = v0 + threadIdx.x; v < v1; v += CMP_NT) {
    uint32_t l[2];
    for (int s = 0; s < 2; ++s) {
      const uint64_t b = 2 * v + s;
      const uint64_t s0 = off[b], s1 = off[b + 1];
      uint32_t out = CMP_NIL;
      if (s1 == s0 + 1 && s0 < 2 * m) {
        const uint32_t e = inc_edge[s0];
        const uint32_t t = inc_end[s0];
        if (e >= m || t > 1u) {
          cmp_status(res, DBG_E_ARG);
        } else {
          const uint32_t bw = edge_bucket[2 * (uint64_t)e + (t ^ 1u)];  // the other end
          if (bw >= 2 * n) cmp_status(res, DBG_E_ARG);
          else if ((uint64_t)(bw >> 1) != v && ((single[bw >> 5] >> (bw & 31u)) & 1u)) out = bw;
        }
      }
      l[s] = out;
    }
    reinterpret_cast<uint2 *>(link)[v] = make_uint2(l[0], l[1]);
    place[v] = NRec{CMP_NIL, 0u, 0u, 0u};
    if ((l[0] == CMP_NIL) != (l[1] == CMP_NIL)) {
      const uint32_t h = (uint32_t)(2 * v) + (l[0] != CMP_NIL ? 0u : 1u);
      heads[v0 + atomicAdd(&seg, 1u)] = h;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) seg_count[blockIdx.x] = seg;
}

// Both ends of every chain walk it, reading links only, up to CMP_WALK states.
// A walk that reaches the tail knows the chain's length and its other end (the
// twin copy starts at the tail's twin); of the two copies the one whose first
// k-mer is smaller is canonical, and only that copy's walker walks again,
// writing every node's place.  Longer lists are left to pointer jumping.  A lane
// takes a new head from its workgroup's segment as soon as its walk ends (one
// flat loop, so lanes do not wait for each other).
template <typename K>
__global__ __launch_bounds__(CMP_NT) void k_cmp_walk(const uint32_t *link, NRec *place,
                                                     const uint32_t *heads,
                                                     const uint32_t *seg_count, uint64_t chunk,
                                                     const K *keys, int k) {
  __shared__ uint32_t next;
  if (threadIdx.x == 0) next = 0;
  __syncthreads();
  const uint32_t c = seg_count[blockIdx.x];
  const uint32_t *seg = heads + blockIdx.x * chunk;
  uint32_t h = 0, x = 0, b = CMP_NIL, r = 0, len = 0;
  int phase = 0;  // 0: take a head, 1: find the tail, 2: place the nodes
  while (true) {
    if (phase == 0) {
      const uint32_t j = atomicAdd(&next, 1u);
      if (j >= c) break;
      h = seg[j];
      x = h;
      b = link[h];  // bucket entered by the successor (never NIL for a head here)
      r = 1;
      phase = 1;
    } else if (phase == 1) {
      if (b == CMP_NIL) {  // x is the tail; r states
        const K a = state_kmer(keys, h, k), z = state_kmer(keys, x ^ 1u, k);
        if (a < z) {
          len = r;
          x = h;
          r = 0;
          phase = 2;
        } else {
          phase = 0;
        }
      } else if (r >= CMP_WALK) {
        phase = 0;
      } else {
        x = b ^ 1u;  // the state that enters by that bucket's side
        b = link[x];
        ++r;
      }
    } else {
      place[x >> 1] = NRec{h >> 1, r, len, x & 1u};
      if (++r == len) phase = 0;
      else x = link[x] ^ 1u;
    }
  }
}

// Nodes that no walk placed and that are linked: their states get first jump
// words (pointer = predecessor, pred(2v + t) = link of side 1 - t; heads are done
// at once) and the pending ones go on the first worklist.
__global__ __launch_bounds__(CMP_NT) void k_cmp_pending(const uint32_t *link, const NRec *place,
                                                        uint64_t n, uint64_t *word,
                                                        uint32_t *list, uint32_t *count) {
  __shared__ uint32_t lds[CMP_NT / 64 + 1];
  const uint64_t ns = 2 * n;
  for (uint64_t base = blockIdx.x * (uint64_t)CMP_NT; base < ns;
       base += (uint64_t)gridDim.x * CMP_NT) {
    const uint64_t x = base + threadIdx.x;
    bool keep = false;
    if (x < ns) {
      const uint64_t v = x >> 1;
      const uint2 l = reinterpret_cast<const uint2 *>(link)[v];
      if (place[v].head == CMP_NIL && (l.x != CMP_NIL || l.y != CMP_NIL)) {
        const uint32_t p = (x & 1u) ? l.x : l.y;
        keep = p != CMP_NIL;
        word[x] = keep ? jword(p, 0u, 1u) : jword(CMP_NIL, 1u, 0u);
      }
    }
    block_append(keep, (uint32_t)x, list, count, lds);
  }
}

// One round of pointer jumping over the pending states of `in`; the states still
// pending afterwards go to `out`.
__global__ __launch_bounds__(CMP_NT) void k_cmp_rank_round(const uint32_t *in,
                                                           const uint32_t *in_count,
                                                           uint32_t *out, uint32_t *out_count,
                                                           uint64_t *word, uint64_t ns,
                                                           dbg_compact_result_t *res) {
  __shared__ uint32_t lds[CMP_NT / 64 + 1];
  const uint64_t c = *in_count;
  const uint64_t stride = (uint64_t)gridDim.x * CMP_NT;
  for (uint64_t base = blockIdx.x * (uint64_t)CMP_NT; base < c; base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool keep = false;
    uint32_t x = 0;
    if (i < c) {
      x = in[i];
      const uint64_t w = word[x];  // only this thread writes word[x]
      const uint32_t y = jptr(w);
      if (y >= ns) {  // a pending state always points at a state
        cmp_status(res, DBG_E_INTERNAL);
      } else {
        const uint64_t wy = load_relaxed(&word[y]);
        uint64_t r = (uint64_t)jrank(w) + jrank(wy);
        if (r > 0x7fffffffull) r = 0x7fffffffull;  // only on cycles, re-ranked later
        uint64_t nw;
        if (jptr(wy) == CMP_NIL) nw = jword(y, 1u, jrank(w));       // y is the head
        else if (jdone(wy)) nw = jword(jptr(wy), 1u, (uint32_t)r);  // y knows its head
        else {
          nw = jword(jptr(wy), 0u, (uint32_t)r);
          keep = true;
        }
        store_relaxed(&word[x], nw);
      }
    }
    block_append(keep, x, out, out_count, lds);
  }
}

// Cycle states: word = (predecessor, smallest node seen so far).
__global__ __launch_bounds__(CMP_NT) void k_cmp_cyc_init(const uint32_t *list,
                                                         const uint32_t *count,
                                                         const uint32_t *link, uint64_t *word) {
  const uint64_t c = *count;
  for (uint64_t i = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x; i < c;
       i += (uint64_t)gridDim.x * CMP_NT) {
    const uint32_t x = list[i];
    const uint32_t p = link[x ^ 1u];  // NIL only after a bug; k_cmp_cyc_round flags it
    const uint32_t lo = (x >> 1) < (p >> 1) ? (x >> 1) : (p >> 1);
    word[x] = ((uint64_t)p << 32) | lo;
  }
}

__global__ __launch_bounds__(CMP_NT) void k_cmp_cyc_round(const uint32_t *list,
                                                          const uint32_t *count, uint64_t *word,
                                                          uint64_t ns,
                                                          dbg_compact_result_t *res) {
  const uint64_t c = *count;
  for (uint64_t i = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x; i < c;
       i += (uint64_t)gridDim.x * CMP_NT) {
    const uint32_t x = list[i];
    const uint64_t w = word[x];
    const uint32_t y = (uint32_t)(w >> 32);
    if (y >= ns) {  // cycle states point at cycle states
      cmp_status(res, DBG_E_INTERNAL);
      continue;
    }
    const uint64_t wy = load_relaxed(&word[y]);
    const uint32_t a = (uint32_t)w, b = (uint32_t)wy;
    store_relaxed(&word[x], (wy & 0xffffffff00000000ull) | (a < b ? a : b));
  }
}

// Break every cycle at its smallest node v: v+ heads the cycle through it, and
// the state after v- heads the twin.  Node v's smallest cycle node is recorded.
__global__ __launch_bounds__(CMP_NT) void k_cmp_cyc_break(const uint32_t *list,
                                                          const uint32_t *count,
                                                          const uint32_t *link, uint64_t n,
                                                          uint64_t *word, uint32_t *cycmin,
                                                          uint32_t *out, uint32_t *out_count,
                                                          dbg_compact_result_t *res) {
  __shared__ uint32_t lds[CMP_NT / 64 + 1];
  const uint64_t c = *count;
  for (uint64_t base = blockIdx.x * (uint64_t)CMP_NT; base < c;
       base += (uint64_t)gridDim.x * CMP_NT) {
    const uint64_t i = base + threadIdx.x;
    bool keep = false;
    uint32_t x = 0;
    if (i < c) {
      x = list[i];
      const uint32_t lo = (uint32_t)word[x];
      const uint32_t l1 = lo < n ? link[2 * (uint64_t)lo + 1] : CMP_NIL;
      if (l1 == CMP_NIL) {  // the smallest node of a cycle is linked on both sides
        cmp_status(res, DBG_E_INTERNAL);
        word[x] = jword(CMP_NIL, 1u, 0u);
      } else {
        if ((x & 1u) == 0) cycmin[x >> 1] = lo;
        const uint32_t h1 = 2 * lo, h2 = l1 ^ 1u;
        if (x == h1 || x == h2) {
          word[x] = jword(CMP_NIL, 1u, 0u);
          if (x == h1) atomicAdd((unsigned long long *)&res->n_cyclic, 1ull);
        } else {
          word[x] = jword(link[x ^ 1u], 0u, 1u);
          keep = true;
        }
      }
    }
    block_append(keep, x, out, out_count, lds);
  }
}

// Per node: its chain's first node, its rank and orientation along the chain's
// canonical walk, and its chain's length with bit 31 = cyclic -- from its place
// record, or for a single node directly, or from the jump words of its two
// states.  The node also marks the edges merged into its chain (keep = 0): the
// candidate edge on each linked side, written by the edge's u end only, except
// the edge that closed a broken cycle (the one leaving the chain's last node and
// entering its first).
template <typename K>
__global__ __launch_bounds__(CMP_NT) void k_cmp_nodes(const K *keys, uint64_t n, int k,
                                                      uint32_t min_nodes, const uint32_t *link,
                                                      const NRec *place, const uint64_t *word,
                                                      const uint32_t *cycmin,
                                                      const uint64_t *off,
                                                      const uint32_t *inc_edge,
                                                      const uint8_t *inc_end, uint64_t m,
                                                      uint32_t *node_rank, uint8_t *node_orient,
                                                      uint32_t *head, uint32_t *lenc,
                                                      uint8_t *keep, const uint32_t *final_count,
                                                      dbg_compact_result_t *res) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && *final_count != 0u)
    cmp_status(res, DBG_E_INTERNAL);
  for (uint64_t v = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * CMP_NT) {
    const uint2 l = reinterpret_cast<const uint2 *>(link)[v];
    const NRec p = place[v];
    uint32_t len = 1, rank = 0, o = 0, hd = (uint32_t)v, cyc = 0;
    if (p.head != CMP_NIL) {
      hd = p.head;
      rank = p.rank;
      len = p.len;
      o = p.orient;
    } else if (l.x != CMP_NIL || l.y != CMP_NIL) {
      const uint64_t w0 = word[2 * v], w1 = word[2 * v + 1];
      uint32_t h0 = jptr(w0) == CMP_NIL ? (uint32_t)(2 * v) : jptr(w0);
      uint32_t h1 = jptr(w1) == CMP_NIL ? (uint32_t)(2 * v + 1) : jptr(w1);
      if (h0 >= 2 * n || h1 >= 2 * n) {  // only after a failed ranking
        cmp_status(res, DBG_E_INTERNAL);
        h0 = (uint32_t)(2 * v);
        h1 = (uint32_t)(2 * v + 1);
      }
      const uint32_t r0 = jrank(w0), r1 = jrank(w1);
      len = r0 + r1 + 1;
      const uint32_t lo = cycmin[v];
      bool first;
      if (lo != CMP_NIL) {
        first = h0 == 2 * lo;
        cyc = 1;
      } else {
        first = state_kmer(keys, h0, k) < state_kmer(keys, h1, k);
      }
      o = first ? 0u : 1u;
      rank = first ? r0 : r1;
      hd = (first ? h0 : h1) >> 1;
    }
    if (len > 1 && len < min_nodes) {
      len = 1;
      rank = o = cyc = 0;
      hd = (uint32_t)v;
    }
    node_rank[v] = rank;
    node_orient[v] = (uint8_t)o;
    head[v] = hd;
    lenc[v] = len | (cyc << 31);
    if (len > 1) {
      const uint32_t links[2] = {l.x, l.y};
      for (uint32_t s = 0; s < 2; ++s) {
        if (links[s] == CMP_NIL) continue;
        const uint64_t at = off[2 * v + s];
        if (at >= 2 * m) continue;
        const uint32_t e = inc_edge[at];
        if (inc_end[at] != 0 || e >= m) continue;  // the v end leaves it to the u end
        const uint32_t ws = s ^ o;  // 0: the side the walk leaves by, 1: enters by
        const bool closing = cyc && ((rank == 0 && ws == 1u) || (rank == len - 1 && ws == 0u));
        if (!closing) keep[e] = 0;
      }
    }
  }
}

// Exclusive scans of pairs (a, b) of u64 over n elements; Src gives the pair
// of element i.
struct NodeSrc {
  const uint32_t *head;
  const uint32_t *lenc;
  uint32_t km1;
  __device__ void operator()(uint64_t v, uint64_t *a, uint64_t *b) const {
    const bool first = head[v] == (uint32_t)v;
    *a = first ? 1u : 0u;
    *b = first ? (uint64_t)km1 + (lenc[v] & 0x7fffffffu) : 0u;
  }
};

struct EdgeSrc {
  const uint8_t *keep;
  __device__ void operator()(uint64_t e, uint64_t *a, uint64_t *b) const {
    *a = keep[e];
    *b = 0;
  }
};

template <class Src>
__global__ __launch_bounds__(CMP_NT) void k_cmp_scan_reduce(Src src, uint64_t n,
                                                            uint64_t *sums) {
  __shared__ uint64_t wsum[CMP_NT / 64 + 1];
  const uint64_t base = blockIdx.x * CMP_TILE + threadIdx.x * (uint64_t)16;
  uint64_t sa = 0, sb = 0;
  for (int r = 0; r < 16; ++r) {
    if (base + r < n) {
      uint64_t a, b;
      src(base + r, &a, &b);
      sa += a;
      sb += b;
    }
  }
  uint64_t ta, tb;
  block_exclusive_scan<CMP_NT>(sa, wsum, &ta);
  block_exclusive_scan<CMP_NT>(sb, wsum, &tb);
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = ta;
    sums[2 * blockIdx.x + 1] = tb;
  }
}

// Exclusive scan of the per-tile pairs in place; totals[0..1] receive the sums.
__global__ __launch_bounds__(1024) void k_cmp_scan_sums(uint64_t *sums, uint64_t nt,
                                                        uint64_t *totals) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  uint64_t ca = 0, cb = 0;
  for (uint64_t c0 = 0; c0 < nt; c0 += 1024) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t a = i < nt ? sums[2 * i] : 0, b = i < nt ? sums[2 * i + 1] : 0;
    uint64_t ta, tb;
    const uint64_t ea = block_exclusive_scan<1024>(a, wsum, &ta) + ca;
    const uint64_t eb = block_exclusive_scan<1024>(b, wsum, &tb) + cb;
    if (i < nt) {
      sums[2 * i] = ea;
      sums[2 * i + 1] = eb;
    }
    ca += ta;
    cb += tb;
  }
  if (threadIdx.x == 0) {
    totals[0] = ca;
    totals[1] = cb;
  }
}

// Apply pass: every element gets its exclusive prefix (a, b); Sink writes.
template <class Src, class Sink>
__global__ __launch_bounds__(CMP_NT) void k_cmp_scan_apply(Src src, uint64_t n,
                                                           const uint64_t *sums, Sink sink) {
  __shared__ uint64_t wsum[CMP_NT / 64 + 1];
  const uint64_t base = blockIdx.x * CMP_TILE + threadIdx.x * (uint64_t)16;
  uint64_t va[16], vb[16], sa = 0, sb = 0;
  for (int r = 0; r < 16; ++r) {
    va[r] = vb[r] = 0;
    if (base + r < n) src(base + r, &va[r], &vb[r]);
    sa += va[r];
    sb += vb[r];
  }
  uint64_t ta, tb;
  uint64_t ea = block_exclusive_scan<CMP_NT>(sa, wsum, &ta) + sums[2 * blockIdx.x];
  uint64_t eb = block_exclusive_scan<CMP_NT>(sb, wsum, &tb) + sums[2 * blockIdx.x + 1];
  for (int r = 0; r < 16; ++r) {
    if (base + r < n) sink(base + r, ea, eb, va[r]);
    ea += va[r];
    eb += vb[r];
  }
}

// First nodes: number their chains and fill the chain table.
struct ChainSink {
  const uint32_t *lenc;
  uint64_t *head_info;  // per first node: label offset, chain number
  uint32_t *chain_head;
  uint32_t *chain_len;
  uint8_t *chain_cyclic;
  uint64_t *label_off;
  __device__ void operator()(uint64_t v, uint64_t a, uint64_t b, uint64_t is_first) const {
    if (!is_first) return;
    const uint32_t lc = lenc[v];
    head_info[2 * v] = b;
    head_info[2 * v + 1] = a;
    chain_head[a] = (uint32_t)v;
    chain_len[a] = lc & 0x7fffffffu;
    chain_cyclic[a] = (uint8_t)(lc >> 31);
    label_off[a] = b;
  }
};

__global__ void k_cmp_empty(uint64_t *label_off) {
  if (threadIdx.x || blockIdx.x) return;
  label_off[0] = 0;
}

// Chain totals into the result record and the last label offset.
__global__ void k_cmp_chain_totals(const uint64_t *totals, uint64_t *label_off,
                                   uint64_t label_cap, dbg_compact_result_t *res) {
  if (threadIdx.x || blockIdx.x) return;
  res->n_chains = totals[0];
  res->label_len = totals[1];
  label_off[totals[0]] = totals[1];
  if (totals[1] > label_cap) cmp_status(res, DBG_E_CAPACITY);
}

// Per node: its chain number and its bases of the chain's label (the last base
// of its k-mer as the walk reads it; the first node also the k - 1 before).
template <typename K>
__global__ __launch_bounds__(CMP_NT) void k_cmp_labels(const K *keys, uint64_t n, int k,
                                                       const uint32_t *head,
                                                       const uint64_t *head_info,
                                                       const uint32_t *node_rank,
                                                       const uint8_t *node_orient,
                                                       uint64_t label_cap,
                                                       uint32_t *node_chain, uint8_t *labels,
                                                       dbg_compact_result_t *res) {
  const uint64_t n_chains = res->n_chains;
  const bool write = res->status == 0;
  for (uint64_t v = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * CMP_NT) {
    const uint32_t hd = head[v];
    ulonglong2 hi = make_ulonglong2(0, CMP_NIL);
    if (hd < n) hi = reinterpret_cast<const ulonglong2 *>(head_info)[hd];
    const uint64_t c = hi.y;
    if (c >= n_chains) {  // every chain's first node was numbered
      cmp_status(res, DBG_E_INTERNAL);
      node_chain[v] = CMP_NIL;
      continue;
    }
    node_chain[v] = (uint32_t)c;
    if (!write) continue;
    const uint32_t r = node_rank[v];
    const K s = state_kmer(keys, (uint32_t)(2 * v + node_orient[v]), k);
    const uint64_t at = hi.x;
    if (at + (uint64_t)(k - 1) + r >= label_cap) {
      cmp_status(res, DBG_E_INTERNAL);
      continue;
    }
    uint8_t *dst = labels + at;
    const char *abc = "ACGT";
    dst[(uint64_t)(k - 1) + r] = (uint8_t)abc[(uint32_t)s & 3u];
    if (r == 0) {
      for (int i = 0; i < k - 1; ++i)
        dst[i] = (uint8_t)abc[(uint32_t)shr<K>(s, 2 * (k - 1 - i)) & 3u];
    }
  }
}

__global__ __launch_bounds__(CMP_NT) void k_cmp_fill_u8(uint8_t *a, uint64_t n, uint8_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)CMP_NT + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * CMP_NT)
    a[i] = v;
}

struct KeptSink {
  const uint32_t *edge_bucket;
  const uint32_t *node_chain;
  const uint8_t *node_orient;
  uint64_t n;
  uint32_t *kept_row;
  uint32_t *kept_u;
  uint32_t *kept_v;
  uint8_t *kept_orient;
  __device__ void operator()(uint64_t e, uint64_t a, uint64_t, uint64_t is_kept) const {
    if (!is_kept) return;
    const uint32_t bu = edge_bucket[2 * e], bv = edge_bucket[2 * e + 1];
    if (bu >= 2 * n || bv >= 2 * n) return;
    const uint32_t u = bu >> 1, v = bv >> 1;
    // an end on side s of a node read with orientation t lies on side s xor t of
    // its chain; o1 = side at u, o2 = 1 - side at v
    const uint32_t cu = (bu & 1u) ^ node_orient[u];
    const uint32_t cv = (bv & 1u) ^ node_orient[v];
    kept_row[a] = (uint32_t)e;  // a < number of kept edges <= m
    kept_u[a] = node_chain[u];
    kept_v[a] = node_chain[v];
    kept_orient[a] = (uint8_t)((cu << 1) | (cv ^ 1u));
  }
};

// Kept edges in row order: every thread takes 16 consecutive keep flags (0 or
// 1) as one vector, the workgroup scans their counts, and only the kept edges
// are visited.
__global__ __launch_bounds__(CMP_NT) void k_cmp_kept_apply(const uint8_t *keep, uint64_t m,
                                                           const uint64_t *sums, KeptSink sink) {
  __shared__ uint64_t wsum[CMP_NT / 64 + 1];
  const uint64_t base = blockIdx.x * CMP_TILE + threadIdx.x * (uint64_t)16;
  uint32_t mask = 0;
  if (base + 16 <= m) {
    const uint4 q = *reinterpret_cast<const uint4 *>(keep + base);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) mask |= ((w[i] >> (8 * j)) & 1u) << (4 * i + j);
  } else {
    for (int r = 0; r < 16; ++r)
      if (base + r < m && keep[base + r]) mask |= 1u << r;
  }
  uint64_t tot;
  uint64_t pos = block_exclusive_scan<CMP_NT>((uint64_t)__popc(mask), wsum, &tot) +
                 sums[2 * blockIdx.x];
  while (mask) {
    const int r = __ffs(mask) - 1;
    mask &= mask - 1;
    sink(base + r, pos++, 0, 1);
  }
}

__global__ void k_cmp_kept_total(const uint64_t *totals, dbg_compact_result_t *res) {
  if (threadIdx.x || blockIdx.x) return;
  res->n_kept = totals[0];
}

static inline unsigned cmp_grid(uint64_t n, uint64_t cap) {
  uint64_t g = (n + CMP_NT - 1) / CMP_NT;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

static inline size_t cmp_align(size_t x) { return (x + 255) & ~size_t(255); }

struct CmpLayout {
  size_t link, word, place, single, list0, list1, counters, cycmin, head, lenc, head_info, keep, sums, totals,
      heads, seg_count, total;
  int rounds;
  uint64_t tiles, chunk, segments;
};

static CmpLayout cmp_layout(uint64_t n, uint64_t m) {
  CmpLayout L{};
  // ranks stay below n; ceil(log2(2n)) + 1 rounds finish every list
  int r = 1;
  while (r < 40 && (1ull << r) < 2 * n) ++r;
  L.rounds = r + 1;
  const uint64_t big = n > m ? n : m;
  L.tiles = big / CMP_TILE + 1;
  // about 4096 workgroups collect and walk the chain ends, each over its own
  // range of nodes
  L.chunk = ((n + 4095) / 4096 + CMP_NT - 1) / CMP_NT * CMP_NT;
  if (L.chunk < CMP_NT) L.chunk = CMP_NT;
  L.segments = (n + L.chunk - 1) / L.chunk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = cmp_align(off + (bytes ? bytes : 1));
    return o;
  };
  L.link = take(2 * n * sizeof(uint32_t));
  L.word = take(2 * n * sizeof(uint64_t));
  L.place = take(n * sizeof(NRec));
  L.single = take((2 * n + 63) / 64 * sizeof(uint64_t) + CMP_NT / 8);
  L.list0 = take(2 * n * sizeof(uint32_t));
  L.list1 = take(2 * n * sizeof(uint32_t));
  L.counters = take(CMP_MAX_COUNTERS * sizeof(uint32_t));
  L.cycmin = take(n * sizeof(uint32_t));
  L.head = take(n * sizeof(uint32_t));
  L.lenc = take(n * sizeof(uint32_t));
  L.head_info = take(2 * n * sizeof(uint64_t));
  L.heads = take(n * sizeof(uint32_t));
  L.seg_count = take((L.segments + 1) * sizeof(uint32_t));
  L.keep = take(m);
  L.sums = take(2 * L.tiles * sizeof(uint64_t));
  L.totals = take(4 * sizeof(uint64_t));
  L.total = off;
  return L;
}

template <typename K>
static hipError_t run_compact(const void *node_kmer, uint64_t n, uint64_t m, int k,
                              const uint64_t *off, const uint32_t *inc_edge,
                              const uint8_t *inc_end, const uint32_t *edge_bucket,
                              uint32_t min_nodes, const dbg_chains_t &o, const CmpLayout &L,
                              dbg_compact_result_t *res, char *ws, hipStream_t st) {
  const K *keys = static_cast<const K *>(node_kmer);
  uint32_t *link = reinterpret_cast<uint32_t *>(ws + L.link);
  uint64_t *word = reinterpret_cast<uint64_t *>(ws + L.word);
  NRec *place = reinterpret_cast<NRec *>(ws + L.place);
  uint32_t *single = reinterpret_cast<uint32_t *>(ws + L.single);
  uint32_t *list[2] = {reinterpret_cast<uint32_t *>(ws + L.list0),
                       reinterpret_cast<uint32_t *>(ws + L.list1)};
  uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.counters);
  uint32_t *cycmin = reinterpret_cast<uint32_t *>(ws + L.cycmin);
  uint32_t *head = reinterpret_cast<uint32_t *>(ws + L.head);
  uint32_t *lenc = reinterpret_cast<uint32_t *>(ws + L.lenc);
  uint64_t *head_info = reinterpret_cast<uint64_t *>(ws + L.head_info);
  uint32_t *heads = reinterpret_cast<uint32_t *>(ws + L.heads);
  uint32_t *seg_count = reinterpret_cast<uint32_t *>(ws + L.seg_count);
  uint8_t *keep = reinterpret_cast<uint8_t *>(ws + L.keep);
  uint64_t *sums = reinterpret_cast<uint64_t *>(ws + L.sums);
  uint64_t *totals = reinterpret_cast<uint64_t *>(ws + L.totals);
  const int R = L.rounds;

  hipLaunchKernelGGL(k_cmp_init, dim3(cmp_grid(n > 128 ? n : 128, 4096)), dim3(CMP_NT), 0, st,
                     cnt, cycmin, n, res);
  if (n == 0) {  // no chains: only the first label offset
    hipLaunchKernelGGL(k_cmp_empty, dim3(1), dim3(1), 0, st, o.label_offsets);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_cmp_single, dim3(cmp_grid(2 * n, 16384)), dim3(CMP_NT), 0, st, off,
                     2 * n, reinterpret_cast<uint64_t *>(single));
  hipLaunchKernelGGL(k_cmp_links, dim3((unsigned)L.segments), dim3(CMP_NT), 0, st, off, n,
                     inc_edge, inc_end, edge_bucket, m, single, L.chunk, link, place, heads,
                     seg_count, res);
  hipLaunchKernelGGL(k_cmp_walk<K>, dim3((unsigned)L.segments), dim3(CMP_NT), 0, st, link, place,
                     heads, seg_count, L.chunk, keys, k);
  hipLaunchKernelGGL(k_cmp_pending, dim3(cmp_grid(2 * n, 8192)), dim3(CMP_NT), 0, st, link, place,
                     n, word, list[0], &cnt[0]);
  // lists: rounds 0 .. R-1 move states from list[r & 1] (count cnt[r]) to
  // list[(r + 1) & 1] (count cnt[r + 1])
  for (int r = 0; r < R; ++r)
    hipLaunchKernelGGL(k_cmp_rank_round, dim3(CMP_ROUND_GRID), dim3(CMP_NT), 0, st, list[r & 1],
                       &cnt[r], list[(r + 1) & 1], &cnt[r + 1], word, 2 * n, res);
  // cycles: the states left in list[R & 1]
  uint32_t *cl = list[R & 1];
  hipLaunchKernelGGL(k_cmp_cyc_init, dim3(CMP_ROUND_GRID), dim3(CMP_NT), 0, st, cl, &cnt[R], link,
                     word);
  for (int r = 0; r < R; ++r)
    hipLaunchKernelGGL(k_cmp_cyc_round, dim3(CMP_ROUND_GRID), dim3(CMP_NT), 0, st, cl, &cnt[R],
                       word, 2 * n, res);
  hipLaunchKernelGGL(k_cmp_cyc_break, dim3(CMP_ROUND_GRID), dim3(CMP_NT), 0, st, cl, &cnt[R],
                     link, n, word, cycmin, list[(R + 1) & 1], &cnt[R + 1], res);
  for (int r = R + 1; r <= 2 * R; ++r)
    hipLaunchKernelGGL(k_cmp_rank_round, dim3(CMP_ROUND_GRID), dim3(CMP_NT), 0, st, list[r & 1],
                       &cnt[r], list[(r + 1) & 1], &cnt[r + 1], word, 2 * n, res);
  if (m)
    hipLaunchKernelGGL(k_cmp_fill_u8, dim3(cmp_grid(m, 8192)), dim3(CMP_NT), 0, st, keep, m,
                       (uint8_t)1);
  hipLaunchKernelGGL(k_cmp_nodes<K>, dim3(cmp_grid(n, 16384)), dim3(CMP_NT), 0, st, keys, n, k,
                     min_nodes, link, place, word, cycmin, off, inc_edge, inc_end, m, o.node_rank,
                     o.node_orient, head, lenc, keep, &cnt[2 * R + 1], res);
  // chains in the order of their first node; label offsets
  const uint64_t nt_nodes = n / CMP_TILE + 1;
  const NodeSrc ns{head, lenc, (uint32_t)(k - 1)};
  hipLaunchKernelGGL(k_cmp_scan_reduce<NodeSrc>, dim3((unsigned)nt_nodes), dim3(CMP_NT), 0, st,
                     ns, n, sums);
  hipLaunchKernelGGL(k_cmp_scan_sums, dim3(1), dim3(1024), 0, st, sums, nt_nodes, totals);
  const ChainSink cs{lenc, head_info, o.chain_head, o.chain_len, o.chain_cyclic,
                     o.label_offsets};
  hipLaunchKernelGGL((k_cmp_scan_apply<NodeSrc, ChainSink>), dim3((unsigned)nt_nodes),
                     dim3(CMP_NT), 0, st, ns, n, sums, cs);
  hipLaunchKernelGGL(k_cmp_chain_totals, dim3(1), dim3(1), 0, st, totals, o.label_offsets,
                     o.label_capacity, res);
  hipLaunchKernelGGL(k_cmp_labels<K>, dim3(cmp_grid(n, 16384)), dim3(CMP_NT), 0, st, keys, n, k,
                     head, head_info, o.node_rank, o.node_orient, o.label_capacity,
                     o.node_chain, o.labels, res);
  // kept edges in row order
  if (m) {
    const uint64_t nt_edges = m / CMP_TILE + 1;
    const EdgeSrc es{keep};
    hipLaunchKernelGGL(k_cmp_scan_reduce<EdgeSrc>, dim3((unsigned)nt_edges), dim3(CMP_NT), 0, st,
                       es, m, sums);
    hipLaunchKernelGGL(k_cmp_scan_sums, dim3(1), dim3(1024), 0, st, sums, nt_edges, totals + 2);
    const KeptSink ks{edge_bucket, o.node_chain, o.node_orient, n,
                      o.kept_row, o.kept_u, o.kept_v, o.kept_orient};
    hipLaunchKernelGGL(k_cmp_kept_apply, dim3((unsigned)nt_edges), dim3(CMP_NT), 0, st, keep, m,
                       sums, ks);
    hipLaunchKernelGGL(k_cmp_kept_total, dim3(1), dim3(1), 0, st, totals + 2, res);
  }
  return hipGetLastError();
}

}  // namespace dbg

extern "C" {

size_t dbg_compact_workspace_bytes(uint64_t n_nodes, uint64_t n_edges) {
  return dbg::cmp_layout(n_nodes, n_edges).total;
}

int dbg_compact(const void *node_kmer, uint64_t n_nodes, uint64_t n_edges, int k,
                const uint64_t *adj_offsets, const uint32_t *inc_edge, const uint8_t *inc_end,
                const uint32_t *edge_bucket, uint32_t min_nodes,
                const dbg_chains_t *out, dbg_compact_result_t *result, void *workspace,
                size_t workspace_bytes, hipStream_t stream) {
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (!out || !result || !workspace || !out->label_offsets) return DBG_E_NULL;
  if (n_nodes && (!node_kmer || !adj_offsets || !out->node_chain || !out->node_rank ||
                  !out->node_orient || !out->chain_head || !out->chain_len ||
                  !out->chain_cyclic || !out->labels))
    return DBG_E_NULL;
  if (n_edges && (!inc_edge || !inc_end || !edge_bucket || !out->kept_row ||
                  !out->kept_u || !out->kept_v || !out->kept_orient))
    return DBG_E_NULL;
  if (n_edges && !n_nodes) return DBG_E_ARG;
  if (n_nodes >= (1ull << 31) || n_edges >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DBG_E_WORKSPACE;
  const dbg::CmpLayout L = dbg::cmp_layout(n_nodes, n_edges);
  if (workspace_bytes < L.total) return DBG_E_WORKSPACE;
  if (3 * L.rounds + 4 > dbg::CMP_MAX_COUNTERS) return DBG_E_INTERNAL;
  char *ws = static_cast<char *>(workspace);
  const hipError_t e =
      k <= 31 ? dbg::run_compact<uint64_t>(node_kmer, n_nodes, n_edges, k, adj_offsets,
                                           inc_edge, inc_end, edge_bucket, min_nodes,
                                           *out, L, result, ws, stream)
              : dbg::run_compact<unsigned __int128>(node_kmer, n_nodes, n_edges, k, adj_offsets,
                                                    inc_edge, inc_end, edge_bucket,
                                                    min_nodes, *out, L, result, ws, stream);
  return e == hipSuccess ? DBG_OK : DBG_E_HIP;
}

}  // extern "C"
