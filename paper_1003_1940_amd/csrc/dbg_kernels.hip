// gfx950 kernels of the graph builder and the per-table launch sequence.
//
// One table (edges: the canonical (k+1)-mers; nodes: the canonical k-mers) is
// built by
//   1. a scan of per-read key counts (keys of read i occupy [rbase[i], rbase[i+1]));
//   2. enumeration (STEP-1 and the k-mer collection of STEP-3, Sec. 3): every key
//      position is rolled through forward / reverse-complement registers and
//      canonicalised; the first pass histograms the top 8-bit digit per read set,
//      the second pass scatters keys into those 256 buckets (LDS-staged);
//   3. further most-significant-digit partition levels, only for buckets larger
//      than one workgroup's LDS capacity;
//   4. an LDS-resident least-significant-digit radix sort of every remaining
//      bucket (consecutive small buckets are batched), ranked with wave64 ballots;
//   5. a run-length reduce over the sorted keys (STEP-2 dedup with multiplicity,
//      STEP-3 dedup with counts), which also decodes edge records.
// Keys carry no payload, so the partition passes need no stability: equal keys
// are indistinguishable and every bucket is fully sorted in step 4.
#include <type_traits>

#include "dbg_device.h"
#include "dbg_internal.h"

namespace dbg {

// ---------------------------------------------------------------------------
// Small helpers.

__device__ __forceinline__ void set_status(Ctl *ctl, uint32_t code) {
  atomicCAS(&ctl->status, 0u, code);
}

// The node table has two routes (k-mers, or edge endpoints) chosen on the device;
// a kernel of one route returns at once when the build took the other.  Gate -1:
// the kernel belongs to both routes (and to the edge table).
__device__ __forceinline__ bool gated_off(const Ctl *ctl, int gate) {
  return gate >= 0 && (int)ctl->node_path != gate;
}

// First index i in [lo, hi) with a[i] > x (a ascending), hi if none.
__device__ __forceinline__ uint64_t upper_bound(const uint64_t *a, uint64_t lo, uint64_t hi,
                                                uint64_t x) {
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
// First index i in [lo, hi) with a[i] >= x, hi if none.
__device__ __forceinline__ uint64_t lower_bound(const uint64_t *a, uint64_t lo, uint64_t hi,
                                                uint64_t x) {
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename T> __device__ __forceinline__ T *buf(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---------------------------------------------------------------------------
// Control block set-up.

__global__ void k_init(Ctl *ctl, uint64_t *set_read_off, uint64_t n_reads, int write_sets) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Ctl c = {};
    *ctl = c;
    if (write_sets) {
      set_read_off[0] = 0;
      set_read_off[1] = n_reads;
    }
  }
}

__global__ void k_table_reset(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->n_keys = 0;
    ctl->n_tiles = 0;
    ctl->items[0] = ctl->items[1] = 0;
    ctl->level_tiles[0] = ctl->level_tiles[1] = 0;
    ctl->level_scatter_tiles[0] = ctl->level_scatter_tiles[1] = 0;
    ctl->n_batches = 0;
    ctl->n_uniform = 0;
    ctl->n_unique = 0;
    ctl->n_seg = 0;
  }
}

__global__ void k_fill_u64(uint64_t *a, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Workgroups are dispatched to the 8 XCDs in turn.  The scatter kernels give
// each XCD one contiguous eighth of the tiles, so that neighbouring tiles, whose
// output runs share cache lines at their ends, are written through the same L2.
constexpr uint32_t N_XCD = 8;
// Workgroup b of a one-tile-per-workgroup grid (a multiple of 8 workgroups, at
// least n): its tile, or n if it has none.
__device__ __forceinline__ uint64_t xcd_tile(uint64_t b, uint64_t n) {
  const uint64_t per = (n + N_XCD - 1) / N_XCD;
  const uint64_t i = b / N_XCD;
  const uint64_t t = (b % N_XCD) * per + i;
  return i < per && t < n ? t : n;
}

// ---------------------------------------------------------------------------
// 1. Per-read key counts c_i = max(0, L_i - len + 1) and their prefix rbase.

constexpr int SCAN_NT = 256, SCAN_PT = 16;
constexpr uint64_t SCAN_TILE = (uint64_t)SCAN_NT * SCAN_PT;

// A workgroup's SCAN_TILE reads: their offsets (and the next one) are loaded with
// consecutive threads on consecutive words into LDS, where thread t takes reads
// SCAN_PT t .. SCAN_PT t + SCAN_PT - 1.  One padding word after every SCAN_PT
// keeps those per-thread runs in different banks.
__device__ __forceinline__ uint32_t scan_pad(uint32_t i) { return i + i / SCAN_PT; }
constexpr uint32_t SCAN_LDS = SCAN_TILE + SCAN_TILE / SCAN_PT + 2;

__device__ __forceinline__ void stage_offsets(const uint64_t *off, uint64_t n_reads, uint64_t b0,
                                              uint64_t *lo) {
  for (uint32_t i = threadIdx.x; i <= (uint32_t)SCAN_TILE; i += SCAN_NT)
    lo[scan_pad(i)] = b0 + i <= n_reads ? off[b0 + i] : 0;
  __syncthreads();
}

// Key counts of this thread's reads (0 past the last read); a decreasing offset
// is reported.
__device__ __forceinline__ void read_key_counts(const uint64_t *lo, uint64_t b0,
                                                uint64_t n_reads, int len,
                                                uint64_t (&c)[SCAN_PT], Ctl *ctl) {
  const uint32_t i0 = threadIdx.x * SCAN_PT;
  uint64_t a = lo[scan_pad(i0)];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) {
    const uint64_t b = lo[scan_pad(i0 + r + 1)];
    c[r] = 0;
    if (b0 + i0 + r < n_reads) {
      bad |= b < a;
      const uint64_t L = b - a;
      c[r] = b >= a && L + 1 > (uint64_t)len ? L + 1 - (uint64_t)len : 0;
    }
    a = b;
  }
  if (bad) set_status(ctl, DBG_E_OFFSETS);
}

__global__ __launch_bounds__(SCAN_NT) void k_read_reduce(const uint64_t *off, uint64_t n_reads,
                                                         uint64_t n_bases, int len,
                                                         uint64_t *block_sums, Ctl *ctl) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  __shared__ uint64_t lo[SCAN_LDS];
  const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_TILE;
  stage_offsets(off, n_reads, b0, lo);
  uint64_t c[SCAN_PT], s = 0;
  read_key_counts(lo, b0, n_reads, len, c, ctl);
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) s += c[r];
  uint64_t total;
  block_exclusive_scan<SCAN_NT>(s, wsum, &total);
  if (threadIdx.x == 0) {
    block_sums[blockIdx.x] = total;
    if (blockIdx.x == 0 && off[0] != 0) set_status(ctl, DBG_E_OFFSETS);
    if (blockIdx.x == gridDim.x - 1 && off[n_reads] != n_bases) set_status(ctl, DBG_E_OFFSETS);
  }
}

// Exclusive scan of a[0..n) in place by one workgroup of 1024 threads; the sum
// goes to *total (if not null).
__global__ __launch_bounds__(1024) void k_scan_small(uint64_t *a, uint64_t n, uint64_t *total) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < n; c0 += 1024 * 4) {
    uint64_t v[4], s = 0;
    const uint64_t i0 = c0 + threadIdx.x * 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] = i0 + r < n ? a[i0 + r] : 0;
      s += v[r];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_scan<1024>(s, wsum, &tot) + carry;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (i0 + r < n) a[i0 + r] = ex;
      ex += v[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Exclusive scan of a long u64 array in three launches: chunk sums
// (k_chunk_reduce), a scan of those (k_scan_small), each chunk scanned from its
// offset (k_chunk_apply).  A chunk is SCAN_TILE entries.
__global__ __launch_bounds__(SCAN_NT) void k_chunk_reduce(const uint64_t *a, uint64_t n,
                                                          uint64_t *csum) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  const uint64_t i0 = blockIdx.x * SCAN_TILE + threadIdx.x * (uint64_t)SCAN_PT;
  uint64_t s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) s += i0 + r < n ? a[i0 + r] : 0;
  uint64_t tot;
  block_exclusive_scan<SCAN_NT>(s, wsum, &tot);
  if (threadIdx.x == 0) csum[blockIdx.x] = tot;
}
__global__ __launch_bounds__(SCAN_NT) void k_chunk_apply(uint64_t *a, uint64_t n,
                                                         const uint64_t *csum) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  const uint64_t i0 = blockIdx.x * SCAN_TILE + threadIdx.x * (uint64_t)SCAN_PT;
  uint64_t v[SCAN_PT], s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) {
    v[r] = i0 + r < n ? a[i0 + r] : 0;
    s += v[r];
  }
  uint64_t tot;
  uint64_t ex = block_exclusive_scan<SCAN_NT>(s, wsum, &tot) + csum[blockIdx.x];
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) {
    if (i0 + r < n) a[i0 + r] = ex;
    ex += v[r];
  }
}

__global__ __launch_bounds__(SCAN_NT) void k_read_apply(const uint64_t *off, uint64_t n_reads,
                                                        int len, const uint64_t *block_sums,
                                                        uint64_t *rbase, Ctl *ctl) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  __shared__ uint64_t lo[SCAN_LDS];
  const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_TILE;
  stage_offsets(off, n_reads, b0, lo);
  uint64_t c[SCAN_PT], s = 0;
  read_key_counts(lo, b0, n_reads, len, c, ctl);
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) s += c[r];
  uint64_t total;
  uint64_t ex = block_exclusive_scan<SCAN_NT>(s, wsum, &total) + block_sums[blockIdx.x];
  __syncthreads();  // every thread has read its offsets: the prefixes go in their place
  const uint32_t i0 = threadIdx.x * SCAN_PT;
#pragma unroll
  for (int r = 0; r < SCAN_PT; ++r) {
    lo[scan_pad(i0 + (uint32_t)r)] = ex;
    ex += c[r];
  }
  __syncthreads();
  // the grid covers reads 0 .. n_reads, so rbase[n_reads] (= total keys) too
  for (uint32_t i = threadIdx.x; i < (uint32_t)SCAN_TILE; i += SCAN_NT)
    if (b0 + i <= n_reads) rbase[b0 + i] = lo[scan_pad(i)];
}

// Per-set key ranges and enumeration tiles.  One workgroup.
__global__ __launch_bounds__(1024) void k_set_setup(const uint64_t *rbase, uint64_t n_reads,
                                                    const uint64_t *set_read_off, uint64_t n_sets,
                                                    uint64_t max_positions, uint64_t *set_kbase,
                                                    uint64_t *set_tbase, Ctl *ctl) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  if (ctl->status) return;
  if (threadIdx.x == 0) {
    const uint64_t nk = rbase[n_reads];
    ctl->n_keys = nk;
    if (nk > max_positions) set_status(ctl, DBG_E_OVERFLOW);
    if (set_read_off[0] != 0 || set_read_off[n_sets] != n_reads) set_status(ctl, DBG_E_OFFSETS);
  }
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 <= n_sets; c0 += 1024) {
    const uint64_t s = c0 + threadIdx.x;
    uint64_t tiles = 0;
    if (s <= n_sets) {
      const uint64_t r = set_read_off[s];
      if (s < n_sets && set_read_off[s + 1] < r) set_status(ctl, DBG_E_OFFSETS);
      const uint64_t kb = rbase[r <= n_reads ? r : n_reads];
      set_kbase[s] = kb;
      if (s < n_sets) {
        const uint64_t r1 = set_read_off[s + 1];
        const uint64_t kb1 = rbase[r1 <= n_reads ? r1 : n_reads];
        tiles = kb1 >= kb ? (kb1 - kb + TILE - 1) / TILE : 0;
      }
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<1024>(tiles, wsum, &tot) + carry;
    if (s <= n_sets) set_tbase[s] = ex;
    carry += tot;
  }
  if (threadIdx.x == 0) ctl->n_tiles = carry;
}

// Tile -> its descriptor: the set, the keys, the reads holding them (the read
// whose key range contains the tile's first key, through the one holding its
// last) and the packed words holding those reads.
__global__ void k_tile_map(const uint64_t *rbase, const uint64_t *offsets,
                           const uint64_t *set_read_off, uint64_t n_sets,
                           const uint64_t *set_kbase, const uint64_t *set_tbase, TileDesc *tiles,
                           uint64_t max_tiles, Ctl *ctl) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (ctl->status || t >= ctl->n_tiles) return;
  if (t >= max_tiles) {
    set_status(ctl, DBG_E_INTERNAL);
    return;
  }
  const uint64_t s = upper_bound(set_tbase, 0, n_sets + 1, t) - 1;
  const uint64_t tb = set_tbase[s];
  const uint64_t g = set_kbase[s] + (t - tb) * TILE;
  const uint64_t se = set_kbase[s + 1];
  const uint64_t ge = g + TILE < se ? g + TILE : se;
  const uint64_t r0 = set_read_off[s], r1 = set_read_off[s + 1];
  const uint64_t lo = upper_bound(rbase, r0, r1 + 1, g) - 1;
  // one past the read holding the next tile's first key, or the set's end
  const uint64_t hi = t + 1 < set_tbase[s + 1] ? upper_bound(rbase, r0, r1 + 1, ge) : r1;
  TileDesc d;
  d.start = g;
  d.read_lo = lo;
  d.read_hi = hi;
  d.g_base = rbase[lo];
  d.wb = offsets[lo] >> 5;
  d.we = (offsets[hi] + 31) >> 5;
  d.t_first = tb;
  d.set = (uint32_t)s;
  d.n = (uint32_t)(ge - g);
  tiles[t] = d;
}

// ---------------------------------------------------------------------------
// 2. Enumeration.

struct EnumArgs {
  const uint64_t *packed;
  uint64_t n_words;
  const uint64_t *offsets;
  const uint64_t *rbase;
  const TileDesc *tiles;
  int len;   // bases per key
  int bits;  // 2 * len
  int gate;
  uint32_t pfx_lo, pfx_hi;  // keys kept: prefix in [pfx_lo, pfx_hi)
};

// The top PFX_BITS bits of a key of `bits` bits (zero-extended when shorter).
template <typename K> __device__ __forceinline__ uint32_t key_prefix_bits(K key, int bits) {
  return bits >= PFX_BITS ? (uint32_t)shr<K>(key, bits - PFX_BITS)
                          : (uint32_t)key << (PFX_BITS - bits);
}

template <typename K> __device__ __forceinline__ bool in_slice(const EnumArgs &a, K key) {
  const uint32_t p = key_prefix_bits(key, a.bits);
  return p >= a.pfx_lo && p < a.pfx_hi;
}

struct TileRange {
  uint64_t start, end, read_lo, read_hi;
  uint64_t g_base, wb, we, t_first;
  uint32_t set;
};

__device__ __forceinline__ TileRange enum_tile(const EnumArgs &a, uint64_t t) {
  const TileDesc d = a.tiles[t];
  TileRange r;
  r.start = d.start;
  r.end = d.start + d.n;
  r.read_lo = d.read_lo;
  r.read_hi = d.read_hi;
  r.g_base = d.g_base;
  r.wb = d.wb;
  r.we = d.we;
  r.t_first = d.t_first;
  r.set = d.set;
  return r;
}

// A tile's keys are enumerated from LDS when its span of the packed stream (plus
// two words, so that a key's last word read never needs a bounds check) and its
// reads fit: positions are then 32-bit offsets from the first staged word and
// key indices 32-bit offsets from the first read's first key.  Tiles that do not
// fit (very long reads, or very many reads shorter than a key) read global memory.
constexpr uint32_t ENUM_WCAP = 1024;  // packed words staged per tile
constexpr uint32_t ENUM_RCAP = 1024;  // read rows staged per tile

// The staged arrays are addressed through LDS-typed pointers, so that every access
// compiles to an LDS instruction.
typedef __attribute__((address_space(3))) const uint64_t lds_u64;
typedef __attribute__((address_space(3))) const uint32_t lds_u32;

struct EnumLds {
  uint64_t words[ENUM_WCAP + 2];
  uint32_t rb[ENUM_RCAP];   // first key of each read, from the tile's first read's
  uint32_t off[ENUM_RCAP];  // first base of each read, from the first staged word's
};

struct TileSrc {
  bool fast;  // staged in LDS (uniform over the workgroup)
  // staged tile
  lds_u64 *lw;
  lds_u32 *lrb, *loff;
  uint64_t g_base;  // key index of rb[0]
  uint32_t nr;      // read rows staged (read_lo .. read_hi)
  // global memory
  const uint64_t *gw, *gr, *go;
  uint64_t n_words;
  __device__ __forceinline__ uint64_t word(uint64_t i) const { return i < n_words ? gw[i] : 0ull; }
  __device__ __forceinline__ uint64_t rbase(uint64_t i) const { return gr[i]; }
  __device__ __forceinline__ uint64_t offset(uint64_t i) const { return go[i]; }
};

// Stage a tile's words and reads when they fit (whole workgroup; contains a
// barrier).
__device__ __forceinline__ TileSrc stage_tile(const EnumArgs &a, const TileRange &tr,
                                              EnumLds &L) {
  TileSrc ts;
  ts.gw = a.packed;
  ts.n_words = a.n_words;
  ts.gr = a.rbase;
  ts.go = a.offsets;
  ts.lw = (lds_u64 *)L.words;
  ts.lrb = (lds_u32 *)L.rb;
  ts.loff = (lds_u32 *)L.off;
  const uint64_t wb = tr.wb;
  const uint64_t nw = tr.we - wb + 2;
  const uint64_t nr = tr.read_hi - tr.read_lo + 1;
  ts.fast = nw <= ENUM_WCAP + 2 && nr <= ENUM_RCAP;
  ts.nr = (uint32_t)nr;
  ts.g_base = tr.g_base;
  if (ts.fast) {
    for (uint32_t i = threadIdx.x; i < (uint32_t)nw; i += blockDim.x)
      L.words[i] = wb + i < a.n_words ? a.packed[wb + i] : 0ull;
    const uint64_t p0 = wb << 5;
    for (uint32_t i = threadIdx.x; i < (uint32_t)nr; i += blockDim.x) {
      L.rb[i] = (uint32_t)(a.rbase[tr.read_lo + i] - ts.g_base);
      L.off[i] = (uint32_t)(a.offsets[tr.read_lo + i] - p0);
    }
  }
  __syncthreads();
  return ts;
}

__device__ __forceinline__ uint64_t extract_key(const TileSrc &ts, uint64_t p, int len, uint64_t) {
  const uint64_t wi = p >> 5;
  const int o = (int)(p & 31) * 2;
  const uint64_t w0 = ts.word(wi);
  const uint64_t w1 = ts.word(wi + 1);
  const uint64_t v = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  return len == 32 ? v : (v >> (64 - 2 * len));
}
__device__ __forceinline__ u128 extract_key(const TileSrc &ts, uint64_t p, int len, u128) {
  const uint64_t wi = p >> 5;
  const int o = (int)(p & 31) * 2;
  const uint64_t w0 = ts.word(wi), w1 = ts.word(wi + 1), w2 = ts.word(wi + 2);
  const uint64_t hi = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  const uint64_t lo = o ? ((w1 << o) | (w2 >> (64 - o))) : w1;
  return shr<u128>(((u128)hi << 64) | (u128)lo, 128 - 2 * len);
}
// The same from the staged words (P: bases from the first staged word).
__device__ __forceinline__ uint64_t extract_staged(lds_u64 *w, uint32_t P, int len, uint64_t) {
  const uint32_t wi = P >> 5;
  const int o = (int)(P & 31) * 2;
  const uint64_t w0 = w[wi], w1 = w[wi + 1];
  const uint64_t v = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  return len == 32 ? v : (v >> (64 - 2 * len));
}
__device__ __forceinline__ u128 extract_staged(lds_u64 *w, uint32_t P, int len, u128) {
  const uint32_t wi = P >> 5;
  const int o = (int)(P & 31) * 2;
  const uint64_t w0 = w[wi], w1 = w[wi + 1], w2 = w[wi + 2];
  const uint64_t hi = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  const uint64_t lo = o ? ((w1 << o) | (w2 >> (64 - o))) : w1;
  return shr<u128>(((u128)hi << 64) | (u128)lo, 128 - 2 * len);
}

// Keys g0, g0+1, ... (< g_end, at most KPT) into out[]: the canonical key at each
// position, rolling the forward and reverse-complement registers by one base
// within a read and re-seeding them at each read start.  Returns the count.
// Staged tile: 32-bit positions and LDS reads only.
template <typename K, int KPT>
__device__ __forceinline__ int enum_keys_staged(const EnumArgs &a, const TileSrc &ts, uint64_t g0,
                                                uint64_t g_end, K (&out)[KPT]) {
  if (g0 >= g_end) return 0;
  const uint32_t gl0 = (uint32_t)(g0 - ts.g_base), gle = (uint32_t)(g_end - ts.g_base);
  // local read i with rb[i] <= gl0 < rb[i+1] (rb[0] = 0 and rb[nr-1] >= the tile's end)
  uint32_t lo = 0, hi = ts.nr - 1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ts.lrb[mid] <= gl0) lo = mid;
    else hi = mid;
  }
  uint32_t i = lo;
  uint32_t next = ts.lrb[i + 1];
  uint32_t P = ts.loff[i] + (gl0 - ts.lrb[i]);
  const int len = a.len;
  const K mask = low_mask<K>(2 * len);
  const int top = 2 * len - 2;
  K fw = extract_staged(ts.lw, P, len, K());
  K rc = revcomp(fw, len);
  int n = 0;
  uint32_t g = gl0;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    if (g < gle) {
      if (r > 0) {
        if (g == next) {
          do {
            ++i;
            next = ts.lrb[i + 1];
          } while (next == g);
          P = ts.loff[i];
          fw = extract_staged(ts.lw, P, len, K());
          rc = revcomp(fw, len);
        } else {
          const uint32_t q = P + (uint32_t)len;
          const uint32_t c = (uint32_t)(ts.lw[q >> 5] >> (62 - 2 * (int)(q & 31))) & 3u;
          fw = ((fw << 2) | (K)c) & mask;
          rc = (rc >> 2) | ((K)(3u - c) << top);
          ++P;
        }
      }
      out[r] = rc < fw ? rc : fw;
      ++n;
      ++g;
    }
  }
  return n;
}

// Tiles that do not fit in LDS: the same from global memory.
template <typename K, int KPT>
__device__ __forceinline__ int enum_keys_global(const EnumArgs &a, const TileSrc &ts, uint64_t g0,
                                                uint64_t g_end, uint64_t read_lo,
                                                uint64_t read_hi, K (&out)[KPT]) {
  if (g0 >= g_end) return 0;
  // read i with rbase[i] <= g0 < rbase[i+1]
  uint64_t lo = read_lo, hi = read_hi;  // rbase[lo] <= g0 < rbase[hi]
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (ts.rbase(mid) <= g0) lo = mid;
    else hi = mid;
  }
  uint64_t i = lo;
  uint64_t next = ts.rbase(i + 1);
  uint64_t p = ts.offset(i) + (g0 - ts.rbase(i));
  const int len = a.len;
  const K mask = low_mask<K>(2 * len);
  const int top = 2 * len - 2;
  K fw = extract_key(ts, p, len, K());
  K rc = revcomp(fw, len);
  int n = 0;
  uint64_t g = g0;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    if (g < g_end) {
      if (r > 0) {
        if (g == next) {
          do {
            ++i;
            next = ts.rbase(i + 1);
          } while (next == g);
          p = ts.offset(i);
          fw = extract_key(ts, p, len, K());
          rc = revcomp(fw, len);
        } else {
          const uint64_t q = p + len;
          const uint32_t c = (uint32_t)(ts.word(q >> 5) >> (62 - 2 * (int)(q & 31))) & 3u;
          fw = ((fw << 2) | (K)c) & mask;
          rc = (rc >> 2) | ((K)(3u - c) << top);
          ++p;
        }
      }
      out[r] = rc < fw ? rc : fw;
      ++n;
      ++g;
    }
  }
  return n;
}

// Where a thread's KPT positions start in the staged stream: P for the first
// and, when a read starts inside them, that read's first base P2 and the step rs
// at which it starts (otherwise P2 = P and rs = KPT).  A thread's positions meet
// at most one read start when reads hold at least KPT keys; `two` is set when
// some position meets a second one.
struct Seeds {
  uint32_t gl0, glast;  // the thread's first position and its range end (tile-local)
  uint32_t P, P2, rs;
  bool two;
};

template <int KPT>
__device__ __forceinline__ Seeds find_seeds(const TileSrc &ts, uint64_t g0, uint64_t g_end) {
  Seeds s;
  const bool any = g0 < g_end;
  s.gl0 = any ? (uint32_t)(g0 - ts.g_base) : 0u;
  const uint32_t gle = any ? (uint32_t)(g_end - ts.g_base) : 0u;
  s.glast = s.gl0 + (uint32_t)KPT < gle ? s.gl0 + (uint32_t)KPT : gle;
  uint32_t lo = 0, hi = ts.nr - 1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ts.lrb[mid] <= s.gl0) lo = mid;
    else hi = mid;
  }
  const uint32_t next = ts.lrb[lo + 1];  // first key of the following read (> gl0)
  const bool sw = any && next < s.glast;
  uint32_t j = lo + 1;
  if (sw)
    while (ts.lrb[j + 1] == next) ++j;  // past reads with no key
  s.two = sw && ts.lrb[j + 1] < s.glast;
  s.P = ts.loff[lo] + (s.gl0 - ts.lrb[lo]);
  s.P2 = sw ? ts.loff[j] : s.P;
  s.rs = sw ? next - s.gl0 : (uint32_t)KPT;
  return s;
}

// The 32 bases of the staged stream from base S, first base in the top bits.
__device__ __forceinline__ uint64_t window32(lds_u64 *w, uint32_t S) {
  const uint32_t wi = S >> 5;
  const int o = (int)(S & 31) * 2;
  const uint64_t w0 = w[wi], w1 = w[wi + 1];
  return o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
}

// Heads of the canonical keys: the first H = min(6, len) bases of the canonical
// key at each of a thread's positions, as a 2H-bit integer, which fixes the key's
// first radix digit and its slice prefix.  Taking the first bases of an integer
// key is monotone, so the head of the smaller of the key and its reverse
// complement (Sec. 2) is the smaller of their heads: the forward k-mer's first H
// bases and the reverse complement of its last H bases.  Both come, for all 16
// positions of a seed, from one 32-base window each (16 positions + H - 1 <= 21
// bases), with 32-bit field extracts: no key-wide arithmetic.  A seed that starts
// at step rs is read from its virtual start P2 - rs (at or after the previous
// read's last k-mer base), so that step r of either seed sits at the same window
// offset.  Same read-start rules and return value as enum_keys_two_seeds.
struct HeadWin {
  uint32_t f0, f1;  // forward bases [S, S + 16) and [S + 8, S + 24)
  uint32_t r0, r1;  // reverse complement of the last-H windows, steps 0..7 and 8..15
};

__device__ __forceinline__ HeadWin head_windows(lds_u64 *w, uint32_t S, int len, int H) {
  HeadWin hw;
  const uint64_t f = window32(w, S);
  hw.f0 = (uint32_t)(f >> 32);
  hw.f1 = (uint32_t)(f >> 16);
  // complement base S + len - H + j lands in bits [2j, 2j + 2)
  const uint64_t rc = reverse_pairs64(~window32(w, S + (uint32_t)(len - H)));
  hw.r0 = (uint32_t)rc;
  hw.r1 = (uint32_t)(rc >> 16);
  return hw;
}

__device__ __forceinline__ uint32_t head_at(const HeadWin &hw, int r, int H) {
  const uint32_t width = 2u * (uint32_t)H;
  const uint32_t fw = r < 8 ? __builtin_amdgcn_ubfe(hw.f0, 32u - width - 2u * r, width)
                            : __builtin_amdgcn_ubfe(hw.f1, 32u - width - 2u * (r - 8), width);
  const uint32_t rc = r < 8 ? __builtin_amdgcn_ubfe(hw.r0, 2u * r, width)
                            : __builtin_amdgcn_ubfe(hw.r1, 2u * (r - 8), width);
  return rc < fw ? rc : fw;
}

template <int KPT>
__device__ __forceinline__ int enum_heads_two_seeds(const EnumArgs &a, const TileSrc &ts,
                                                    uint64_t g0, uint64_t g_end,
                                                    uint32_t (&out)[KPT]) {
  static_assert(KPT == 16, "the head windows cover 16 positions");
  const Seeds sd = find_seeds<KPT>(ts, g0, g_end);
  if (__any(sd.two)) return -1;
  const int len = a.len;
  const int H = len < 6 ? len : 6;
  const HeadWin w1 = head_windows(ts.lw, sd.P, len, H);
  const HeadWin w2 = head_windows(ts.lw, sd.rs < (uint32_t)KPT ? sd.P2 - sd.rs : sd.P, len, H);
  int n = 0;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const uint32_t h1 = head_at(w1, r, H), h2 = head_at(w2, r, H);
    if (sd.gl0 + (uint32_t)r < sd.glast) {
      out[r] = (uint32_t)r < sd.rs ? h1 : h2;
      ++n;
    }
  }
  return n;
}

// The first radix digit and the slice prefix of a key from its head (the first
// H = min(6, len) bases): the same values as msd_digit(key, 2 len, 0) and
// key_prefix_bits(key, 2 len).
__device__ __forceinline__ uint32_t head_digit(uint32_t head, int len) {
  return len >= 4 ? head >> (2 * (len < 6 ? len : 6) - 8) : head;
}
__device__ __forceinline__ uint32_t head_prefix(uint32_t head, int len) {
  return head << (PFX_BITS - 2 * (len < 6 ? len : 6));
}

template <typename K, int KPT>
__device__ __forceinline__ int enum_keys(const EnumArgs &a, const TileSrc &ts, uint64_t g0,
                                         uint64_t g_end, uint64_t read_lo, uint64_t read_hi,
                                         K (&out)[KPT]) {
  if (ts.fast) return enum_keys_staged<K, KPT>(a, ts, g0, g_end, out);
  return enum_keys_global<K, KPT>(a, ts, g0, g_end, read_lo, read_hi, out);
}

// SL: the build is a key-space slice (keys outside [pfx_lo, pfx_hi) are dropped);
// full builds compile the test out.
template <typename K, bool SL>
__global__ __launch_bounds__(STREAM_NT) void k_enum_hist(EnumArgs a, uint32_t *thist,
                                                         const Ctl *ctl) {
  __shared__ uint32_t h[256];
  __shared__ EnumLds L;
  const uint64_t t = blockIdx.x;
  if (ctl->status || gated_off(ctl, a.gate) || t >= ctl->n_tiles) return;
  h[threadIdx.x] = 0;
  const TileRange tr = enum_tile(a, t);
  const TileSrc ts = stage_tile(a, tr, L);
  const uint64_t g0 = tr.start + threadIdx.x * (uint64_t)STREAM_KPT;
  uint32_t heads[STREAM_KPT];
  const int nh = ts.fast ? enum_heads_two_seeds<STREAM_KPT>(a, ts, g0, tr.end, heads) : -1;
  if (nh >= 0) {
#pragma unroll
    for (int r = 0; r < STREAM_KPT; ++r) {
      const uint32_t p = head_prefix(heads[r], a.len);
      if (r < nh && (!SL || (p >= a.pfx_lo && p < a.pfx_hi)))
        atomicAdd(&h[head_digit(heads[r], a.len)], 1u);
    }
  } else {
    // one key at a time (waves with short reads, tiles beyond the LDS staging):
    // the heads path above sets the kernel's registers
    for (int r = 0; r < STREAM_KPT; ++r) {
      K key[1];
      if (enum_keys<K, 1>(a, ts, g0 + r, tr.end, tr.read_lo, tr.read_hi, key) &&
          (!SL || in_slice(a, key[0])))
        atomicAdd(&h[msd_digit(key[0], a.bits, 0)], 1u);
    }
  }
  __syncthreads();
  thist[t * 256 + threadIdx.x] = h[threadIdx.x];
}

// Keys kept by the table (the totals row of the column prefix): the table's key
// count, bounded by the key buffers.
__global__ void k_kept_keys(const uint32_t *thist, uint64_t max_keys, Ctl *ctl, int gate) {
  __shared__ uint64_t wsum[256 / 64 + 1];
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t nt = ctl->n_tiles;
  uint64_t tot;
  block_exclusive_scan<256>((uint64_t)thist[nt * 256 + threadIdx.x], wsum, &tot);
  if (threadIdx.x == 0) {
    ctl->n_keys = tot;
    if (tot > max_keys) set_status(ctl, DBG_E_OVERFLOW);
  }
}

// Prefix counts over whole read sets: each workgroup takes tiles t = blockIdx.x,
// blockIdx.x + gridDim.x, ..., counts their keys' prefixes in LDS and adds the
// counts to the global ones once.
template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_prefix_hist(EnumArgs a, uint64_t *counts,
                                                           const Ctl *ctl) {
  __shared__ uint32_t h[PFX_BINS];
  __shared__ EnumLds L;
  if (ctl->status) return;
  for (uint32_t i = threadIdx.x; i < PFX_BINS; i += STREAM_NT) h[i] = 0;
  const uint64_t nt = ctl->n_tiles;
  for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    __syncthreads();  // the previous tile's staged words are dead
    const TileRange tr = enum_tile(a, t);
    const TileSrc ts = stage_tile(a, tr, L);
    const uint64_t g0 = tr.start + threadIdx.x * (uint64_t)STREAM_KPT;
    uint32_t heads[STREAM_KPT];
    const int nh = ts.fast ? enum_heads_two_seeds<STREAM_KPT>(a, ts, g0, tr.end, heads) : -1;
    if (nh >= 0) {
#pragma unroll
      for (int r = 0; r < STREAM_KPT; ++r)
        if (r < nh) atomicAdd(&h[head_prefix(heads[r], a.len)], 1u);
    } else {  // one key at a time, as in k_enum_hist
      for (int r = 0; r < STREAM_KPT; ++r) {
        K key[1];
        if (enum_keys<K, 1>(a, ts, g0 + r, tr.end, tr.read_lo, tr.read_hi, key))
          atomicAdd(&h[key_prefix_bits(key[0], a.bits)], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < PFX_BINS; i += STREAM_NT)
    if (h[i]) atomicAdd((unsigned long long *)&counts[i], (unsigned long long)h[i]);
}

// Column-wise exclusive prefix of the per-tile histograms over all tiles:
// thist[t][d] becomes the number of keys with digit d in tiles before t, and row
// n_tiles receives the totals.  Three steps: chunk sums, a scan of the chunk
// sums (one workgroup, one thread per digit), and the in-chunk prefixes.
constexpr uint64_t COL_CHUNK = 128;
constexpr int COL_BATCH = 16;  // independent loads in flight per thread

__global__ __launch_bounds__(256) void k_col_reduce(const uint32_t *thist, uint32_t *csum,
                                                    const uint64_t *n_tiles_p, const Ctl *ctl,
                                                    int gate) {
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t nt = *n_tiles_p;
  const uint64_t t0 = blockIdx.x * COL_CHUNK;
  if (t0 >= nt) return;
  const uint64_t t1 = t0 + COL_CHUNK < nt ? t0 + COL_CHUNK : nt;
  uint32_t sum = 0;
  for (uint64_t t = t0; t < t1; t += COL_BATCH) {
    uint32_t v[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) v[i] = t + i < t1 ? thist[(t + i) * 256 + threadIdx.x] : 0u;
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) sum += v[i];
  }
  csum[blockIdx.x * 256 + threadIdx.x] = sum;
}

// One workgroup per digit d: its column of chunk sums, a contiguous run of chunks
// per thread (sums modulo 2^32, like the tile prefixes).
__global__ __launch_bounds__(256) void k_col_scan(uint32_t *csum, const uint64_t *n_tiles_p,
                                                  const Ctl *ctl, int gate) {
  __shared__ uint64_t wsum[256 / 64 + 1];
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t nc = (*n_tiles_p + COL_CHUNK - 1) / COL_CHUNK;
  const uint32_t d = blockIdx.x;
  const uint64_t q = (nc + 255) / 256;
  const uint64_t c0 = threadIdx.x * q, c1 = c0 + q < nc ? c0 + q : nc;
  uint32_t sum = 0;
  for (uint64_t c = c0; c < c1; c += COL_BATCH) {
    uint32_t v[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) v[i] = c + i < c1 ? csum[(c + i) * 256 + d] : 0u;
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) sum += v[i];
  }
  uint64_t tot;
  uint32_t run = (uint32_t)block_exclusive_scan<256>((uint64_t)sum, wsum, &tot);
  for (uint64_t c = c0; c < c1; c += COL_BATCH) {
    uint32_t v[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) v[i] = c + i < c1 ? csum[(c + i) * 256 + d] : 0u;
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i)
      if (c + i < c1) {
        csum[(c + i) * 256 + d] = run;
        run += v[i];
      }
  }
}

__global__ __launch_bounds__(256) void k_col_apply(uint32_t *thist, const uint32_t *csum,
                                                   const uint64_t *n_tiles_p, const Ctl *ctl,
                                                   int gate) {
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t nt = *n_tiles_p;
  const uint64_t t0 = blockIdx.x * COL_CHUNK;
  if (t0 >= nt && !(t0 == 0 && nt == 0)) return;
  const uint64_t t1 = t0 + COL_CHUNK < nt ? t0 + COL_CHUNK : nt;
  uint32_t run = nt ? csum[blockIdx.x * 256 + threadIdx.x] : 0u;
  for (uint64_t t = t0; t < t1; t += COL_BATCH) {
    uint32_t v[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i) v[i] = t + i < t1 ? thist[(t + i) * 256 + threadIdx.x] : 0u;
#pragma unroll
    for (int i = 0; i < COL_BATCH; ++i)
      if (t + i < t1) {
        thist[(t + i) * 256 + threadIdx.x] = run;
        run += v[i];
      }
  }
  if (t1 == nt) thist[nt * 256 + threadIdx.x] = run;
}

// LDS-staged partition of one tile of keys (held in registers) by the digit
// msd_digit(key, bits, level): count per digit, reserve a range per digit in the
// destination buckets with one global atomic per digit, place keys
// digit-contiguously in LDS, then write each digit run with consecutive threads
// on consecutive addresses.  `cursor` points at the 256 bucket cursors of the
// parent.  Every thread of the workgroup must call it.
template <typename K, bool W = false, int HV = 1, int NT = STREAM_NT>
struct PartLds {
  // HV = 2: the tile passes through LDS in two halves (half the LDS, so twice
  // the workgroups per CU; the runs of a digit are written in two pieces)
  static constexpr int HALVES = HV;
  union {
    K keys[TILE / HALVES];
    EnumLds stage;  // the enumeration's staged words, dead once its keys are in registers
  };
  uint32_t wts[W ? TILE / HALVES : 1];  // record weights (W), moved with their keys
  uint64_t gbase[256];
  uint32_t cnt[256];
  uint32_t cnt0[HALVES > 1 ? 256 : 1];  // keys of each digit in the first half
  uint64_t wsum[NT / 64 + 1];
};

template <typename K, bool W = false, int HV = 1, int NT = STREAM_NT>
__device__ __forceinline__ void partition_tile(const K (&keys)[TILE / NT],
                                               const uint32_t (&wts)[TILE / NT], int n, int bits,
                                               int level, uint64_t *cursor, uint64_t my_base,
                                               K *dst, uint32_t *dstw, PartLds<K, W, HV, NT> &s,
                                               uint32_t valid = 0xffffffffu,
                                               uint32_t *row = nullptr) {
  // cursor != null: reserve each digit's range with one atomic on cursor[d];
  // otherwise thread d already holds its digit's destination start in my_base.
  // row != null: the tile is written in digit order to my_base onwards (the
  // same for every thread) and each digit's offset inside the tile to row[d].
  // Threads 0..255 own the digits; NT >= 256.
  constexpr int H = HV, KPT = (int)(TILE / NT);
  static_assert(NT >= 256 && (uint64_t)NT * KPT == TILE, "a digit per thread, whole tile");
  const uint32_t tid = threadIdx.x;
  const bool owner = NT == 256 || tid < 256;
  uint32_t dig[KPT];
#pragma unroll
  for (int r = 0; r < KPT; ++r) dig[r] = r < n ? msd_digit(keys[r], bits, level) : 0u;
  if (owner) {
    s.cnt[tid] = 0;
    if (H > 1) s.cnt0[tid] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < KPT; ++r)
    if (r < n && ((valid >> r) & 1u)) {
      atomicAdd(&s.cnt[dig[r]], 1u);
      if (H > 1 && r < KPT / 2) atomicAdd(&s.cnt0[dig[r]], 1u);
    }
  __syncthreads();
  const uint64_t c = owner ? s.cnt[tid] : 0;
  // destination of the first key of digit tid, reserved before the scan and the
  // placement below and only read after them: at deep levels the cursors are
  // spread over many buckets and the atomic's round trip goes to memory
  const uint64_t base =
      cursor ? (c ? (uint64_t)atomicAdd((unsigned long long *)&cursor[tid], (unsigned long long)c)
                  : 0)
             : my_base;
  uint64_t m;
  const uint64_t ex = block_exclusive_scan<NT>(c, s.wsum, &m);
  if (H == 1) {
    if (owner) s.cnt[tid] = (uint32_t)ex;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r)
      if (r < n && ((valid >> r) & 1u)) {
        const uint32_t q = atomicAdd(&s.cnt[dig[r]], 1u);
        s.keys[q] = keys[r];
        if (W) s.wts[q] = wts[r];
      }
    if (owner) {
      s.gbase[tid] = row ? base : base - ex;
      if (row) row[tid] = (uint32_t)ex;
    }
    __syncthreads();
    for (uint32_t idx = tid; idx < (uint32_t)m; idx += NT) {
      const K key = s.keys[idx];
      const uint64_t o = s.gbase[msd_digit(key, bits, level)] + idx;
      dst[o] = key;
      if (W) dstw[o] = s.wts[idx];
    }
    __syncthreads();
    return;
  }
  // two halves: keys r < 8 of every thread, then r >= 8; a digit's keys of the
  // first half precede its keys of the second in the destination
  static_assert(H == 1 || NT == 256, "halves: 256 threads");
  const uint64_t c0 = H > 1 ? s.cnt0[tid] : c;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const uint64_t ch = h == 0 ? c0 : c - c0;
    uint64_t mh;
    const uint64_t exh = block_exclusive_scan<STREAM_NT>(ch, s.wsum, &mh);
    s.gbase[tid] = base + (h == 0 ? 0 : c0) - exh;
    s.cnt[tid] = (uint32_t)exh;
    __syncthreads();
#pragma unroll
    for (int r = h * (STREAM_KPT / 2); r < (h + 1) * (STREAM_KPT / 2); ++r)
      if (r < n && ((valid >> r) & 1u)) {
        const uint32_t q = atomicAdd(&s.cnt[dig[r]], 1u);
        s.keys[q] = keys[r];
        if (W) s.wts[q] = wts[r];
      }
    __syncthreads();
    for (uint32_t idx = tid; idx < (uint32_t)mh; idx += STREAM_NT) {
      const K key = s.keys[idx];
      const uint64_t o = s.gbase[msd_digit(key, bits, level)] + idx;
      dst[o] = key;
      if (W) dstw[o] = s.wts[idx];
    }
    __syncthreads();
  }
}

// Second enumeration pass: keys go to cursor0[set][d] plus the number of keys
// with digit d in the set's earlier tiles (from the tile prefix), so no atomics.
template <typename K, bool SL>
__global__ __launch_bounds__(STREAM_NT) void k_enum_scatter(EnumArgs a, const uint64_t *cursor0,
                                                            const uint32_t *tpre, K *dst,
                                                            const Ctl *ctl) {
  // the staged words share LDS with the partition's key buffer: partition_tile
  // passes a barrier before it writes keys, after every thread has enumerated
  // the tile passes through LDS in two halves: the enumeration is ALU-heavy and
  // gains from the extra workgroups (the level scatters keep whole tiles, whose
  // longer runs write faster)
  __shared__ PartLds<K, false, 2> s;
  if (ctl->status || gated_off(ctl, a.gate)) return;
  const uint64_t nt = ctl->n_tiles;
  const uint64_t t = xcd_tile(blockIdx.x, nt);
  if (t >= nt) return;
  const TileRange tr = enum_tile(a, t);
  // digit d's destination (loaded before the staging, whose barrier would hold
  // the loads back): tile prefixes are counted modulo 2^32; a difference is exact
  // because a table holds fewer than 2^32 keys
  const uint32_t d = threadIdx.x;
  const uint64_t base = cursor0[(uint64_t)tr.set * 256 + d] +
                        (uint32_t)(tpre[t * 256 + d] - tpre[tr.t_first * 256 + d]);
  const TileSrc ts = stage_tile(a, tr, s.stage);
  K keys[STREAM_KPT];
  const int n = enum_keys<K, STREAM_KPT>(a, ts, tr.start + threadIdx.x * (uint64_t)STREAM_KPT,
                                         tr.end, tr.read_lo, tr.read_hi, keys);
  const uint32_t nowt[STREAM_KPT] = {};
  uint32_t valid = 0xffffffffu;
  if (SL) {
    valid = 0;
#pragma unroll
    for (int r = 0; r < STREAM_KPT; ++r)
      if (r < n && in_slice(a, keys[r])) valid |= 1u << r;
  }
  partition_tile<K, false, 2>(keys, nowt, n, a.bits, 0, nullptr, base, dst,
                                                    nullptr, s, valid);
}

// ---------------------------------------------------------------------------
// Bucket planning: after a parent's 256 sub-buckets are counted, scan the counts
// into cursors and sort the sub-buckets into three kinds.  Oversized ones (more
// keys than the LDS sort holds) go to the next partition level, or, when no
// digit is left (all their keys are equal), to the uniform list.  The others are
// packed into batches in key order, greedily: a sub-bucket joins the open batch
// while the batch stays within the capacity, else it opens the next one; an
// oversized sub-bucket closes the open batch (its keys lie in between).  Any two
// consecutive batches of a run hold more than the capacity together, so the
// batches of a parent number at most 2 (keys / capacity) + 1 plus one per
// oversized sub-bucket.

struct PlanArgs {
  Item *next_items;       // list receiving oversized buckets
  uint64_t *next_count;   // its counter in Ctl
  uint64_t *next_hist;    // histogram rows of that list (zeroed here; null: none kept)
  uint64_t item_cap;
  Batch *batches;
  uint64_t batch_cap;
  Item *uniform;
  uint64_t uniform_cap;
  Ctl *ctl;
  uint64_t local_cap;
  int bits;
  int gate;
  int in_tile_ok;           // children of at most SEG_TILES tiles are split within tiles
  SegBatch *segb;           // digit ranges of in-tile parents
  uint32_t *segt;           // their segment tables (SEG_TILES words each)
  uint64_t seg_cap;
  uint64_t *kw0, *kw1;      // key buffers 0 and 1 as 64-bit words (gathers)
  int key_words;            // 64-bit words per key
  const uint32_t *rows;     // digit offsets of every tile of an in-tile parent
};

// An in-tile parent: its tiles' rows give each digit's segment in every tile.
struct SegParent {
  uint64_t tbase;  // row of the first tile
  uint32_t tiles;
  uint32_t size;
};

// Offset of digit d's segment inside tile i of an in-tile parent (d = 256: the
// tile's size).
__device__ __forceinline__ uint32_t seg_row(const PlanArgs &p, const SegParent &sp, uint32_t i,
                                            uint32_t d) {
  if (d < 256) return p.rows[(sp.tbase + i) * 256 + d];
  const uint64_t rest = (uint64_t)sp.size - (uint64_t)i * TILE;
  return (uint32_t)(rest < TILE ? rest : TILE);
}

constexpr uint32_t PLAN_LARGE = 0xffffffffu;

struct PlanLds {
  uint64_t wsum[STREAM_NT / 64 + 1];
  uint64_t ex[256];         // first key of each sub-bucket (relative to the parent)
  uint64_t base[3];
  alignas(16) uint32_t sz[256];  // keys of each sub-bucket, PLAN_LARGE if oversized
  uint32_t bchild[256];     // first sub-bucket of each batch
  uint32_t blast[256];      // last sub-bucket of each batch
  uint32_t bsize[256];      // keys of each batch
  uint32_t nb;
};

// Called by the whole workgroup (256 threads), thread d passing the count c of
// sub-bucket d of the parent whose keys start at `off`; children live in buffer
// `src`; `child_level` is the digit level that would split a child.  sp: the
// parent was split within its tiles (its children lie in one segment per tile of
// buffer 1): small children go into digit ranges (SegBatch), oversized ones are
// first gathered into buffer 0 at their place in sorted order.
__device__ void plan_children(const PlanArgs &p, uint64_t c, uint64_t off, uint32_t src,
                              int child_level, uint64_t *cursor, PlanLds &s,
                              const SegParent *sp = nullptr) {
  const uint32_t d = threadIdx.x;
  uint64_t total;
  const uint64_t ex = block_exclusive_scan<STREAM_NT>(c, s.wsum, &total);
  if (!sp) cursor[d] = off + ex;
  const bool large = c > p.local_cap;
  s.ex[d] = ex;
  s.sz[d] = large ? PLAN_LARGE : (uint32_t)c;
  __syncthreads();
  if (d == 0) {
    const uint32_t cap = (uint32_t)p.local_cap;
    uint32_t nb = 0, first = 0, last = 0, fill = 0;  // fill = 0: no batch open
    const uint4 *z4 = reinterpret_cast<const uint4 *>(s.sz);
    for (uint32_t q4 = 0; q4 < 64; ++q4) {
      const uint4 v = z4[q4];
      const uint32_t zz[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t z = zz[i];
        if (z == 0) continue;
        const bool close = fill && (z == PLAN_LARGE || fill + z > cap);
        if (close) {
          s.bchild[nb] = first;
          s.blast[nb] = last;
          s.bsize[nb] = fill;
          ++nb;
          fill = 0;
        }
        if (z == PLAN_LARGE) continue;
        if (fill == 0) first = 4 * q4 + (uint32_t)i;
        last = 4 * q4 + (uint32_t)i;
        fill += z;
      }
    }
    if (fill) {
      s.bchild[nb] = first;
      s.blast[nb] = last;
      s.bsize[nb] = fill;
      ++nb;
    }
    s.nb = nb;
  }
  const bool digits_left = p.bits - 8 * child_level > 0;
  uint64_t n_large;
  const uint64_t lid = block_exclusive_scan<STREAM_NT>((uint64_t)large, s.wsum, &n_large);
  // (the scan's barriers also publish nb)
  const uint32_t nb = s.nb;
  if (d == 0) {
    uint64_t *nbat = sp ? &p.ctl->n_seg : &p.ctl->n_batches;
    s.base[0] = nb ? atomicAdd((unsigned long long *)nbat, (unsigned long long)nb) : 0;
    s.base[1] = n_large && digits_left
                    ? atomicAdd((unsigned long long *)p.next_count, n_large) : 0;
    s.base[2] = n_large && !digits_left
                    ? atomicAdd((unsigned long long *)&p.ctl->n_uniform, n_large) : 0;
  }
  __syncthreads();
  if (d < nb) {
    const uint64_t bi = s.base[0] + d;
    if (!sp) {
      if (bi < p.batch_cap)
        p.batches[bi] = Batch{off + s.ex[s.bchild[d]], s.bsize[d],
                              batch_src(src, child_level - 1, s.bchild[d], s.blast[d] + 1)};
      else set_status(p.ctl, DBG_E_INTERNAL);
    } else {
      if (bi < p.seg_cap)
        p.segb[bi] = SegBatch{off + s.ex[s.bchild[d]], s.bsize[d], sp->tiles, off,
                              batch_src(0, child_level - 1, s.bchild[d], s.blast[d] + 1), 0};
      else set_status(p.ctl, DBG_E_INTERNAL);
    }
  }
  if (sp) {
    // each digit range's segment table: where it starts and ends in every tile
    const uint32_t T = sp->tiles;
    for (uint32_t x = d; x < nb * T; x += STREAM_NT) {
      const uint32_t b = x / T, i = x - b * T;
      const uint64_t bi = s.base[0] + b;
      if (bi < p.seg_cap)
        p.segt[bi * SEG_TILES + i] =
            seg_row(p, *sp, i, s.bchild[b]) | seg_row(p, *sp, i, s.blast[b] + 1) << 16;
    }
  }
  if (sp && n_large) {
    // gather each oversized child: its segment of every tile, in tile order,
    // from buffer 1 into buffer 0 at its place (the children in between are
    // never written there: digit ranges write their own places)
    const uint32_t kw = (uint32_t)p.key_words;
    for (uint32_t q = 0; q < 256; ++q) {
      if (s.sz[q] != PLAN_LARGE) continue;  // the same for the whole workgroup
      uint64_t to = (off + s.ex[q]) * kw;
      for (uint32_t i = 0; i < sp->tiles; ++i) {
        const uint32_t lo = seg_row(p, *sp, i, q), hi = seg_row(p, *sp, i, q + 1);
        const uint64_t from = (off + (uint64_t)i * TILE + lo) * kw;
        const uint32_t nw = (hi - lo) * kw;
        for (uint32_t x = d; x < nw; x += STREAM_NT) p.kw0[to + x] = p.kw1[from + x];
        to += nw;
      }
    }
    src = 0;
  }
  if (large) {
    if (digits_left) {
      const uint64_t ii = s.base[1] + lid;
      if (ii < p.item_cap) {
        const uint32_t in_tile = p.in_tile_ok && c <= (uint64_t)SEG_TILES * TILE ? 1u : 0u;
        p.next_items[ii] = Item{off + ex, c, 0, src, in_tile};
        if (p.next_hist)
          for (int j = 0; j < 256; ++j) p.next_hist[ii * 256 + j] = 0;
      } else {
        set_status(p.ctl, DBG_E_INTERNAL);
      }
    } else {
      const uint64_t ui = s.base[2] + lid;
      if (ui < p.uniform_cap) p.uniform[ui] = Item{off + ex, c, 0, src, 0};
      else set_status(p.ctl, DBG_E_INTERNAL);
    }
  }
  __syncthreads();
}

// One workgroup per read set: plan the children of the level-0 partition.
__global__ __launch_bounds__(STREAM_NT) void k_set_plan(PlanArgs p, const uint32_t *tpre,
                                                        const uint64_t *set_tbase,
                                                        uint64_t *cursor0,
                                                        const uint64_t *set_kbase,
                                                        uint64_t n_sets) {
  __shared__ PlanLds lds;
  if (p.ctl->status || gated_off(p.ctl, p.gate)) return;
  const uint32_t d = threadIdx.x;
  for (uint64_t s = blockIdx.x; s < n_sets; s += gridDim.x) {
    const uint64_t c = (uint32_t)(tpre[set_tbase[s + 1] * 256 + d] - tpre[set_tbase[s] * 256 + d]);
    plan_children(p, c, set_kbase[s], 0, 1, cursor0 + s * 256, lds);
  }
}

// ---------------------------------------------------------------------------
// 3. Partition levels >= 1 over oversized buckets.

// One workgroup: tile offsets of the items of a list.  The tiles of buckets that
// are scattered come first, in list order (the tile mode's column prefix needs
// them so); the tiles of in-tile buckets follow, so that each kernel of a level
// walks only its own tiles.
__global__ __launch_bounds__(1024) void k_level_prep(Item *items, const uint64_t *n_items_p,
                                                     uint64_t *n_tiles_out,
                                                     uint64_t *n_scatter_tiles_out,
                                                     uint64_t *other_count, const Ctl *ctl,
                                                     int gate) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t n = *n_items_p;
  uint64_t carry[2] = {0, 0};
  for (int pass = 0; pass < 2; ++pass) {  // 0: scattered buckets, 1: in-tile buckets
    for (uint64_t c0 = 0; c0 < n; c0 += 1024) {
      const uint64_t i = c0 + threadIdx.x;
      const bool mine = i < n && items[i].in_tile == (uint32_t)pass;
      const uint64_t tiles = mine ? (items[i].size + TILE - 1) / TILE : 0;
      uint64_t tot;
      const uint64_t ex = block_exclusive_scan<1024>(tiles, wsum, &tot) + carry[pass];
      if (mine) items[i].tbase = ex + (pass ? carry[0] : 0);
      carry[pass] += tot;
    }
  }
  if (threadIdx.x == 0) {
    *n_scatter_tiles_out = carry[0];
    *n_tiles_out = carry[0] + carry[1];
    *other_count = 0;  // the other list receives this level's oversized children
  }
}

// Every tile of a level's list to the item it belongs to (one workgroup per item
// at a time, its threads over the item's tiles), so that the level kernels find a
// tile's bucket with one load.
__global__ __launch_bounds__(256) void k_level_tilemap(const Item *items,
                                                       const uint64_t *n_items_p,
                                                       const uint64_t *n_tiles_p, uint32_t *titem,
                                                       uint64_t titem_cap, Ctl *ctl, int gate) {
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t n_items = *n_items_p, n_tiles = *n_tiles_p;
  if (n_tiles > titem_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_status(ctl, DBG_E_INTERNAL);
    return;
  }
  for (uint64_t ii = blockIdx.x; ii < n_items; ii += gridDim.x) {
    const uint64_t t0 = items[ii].tbase;
    const uint64_t t1 = t0 + (items[ii].size + TILE - 1) / TILE;
    if (t1 > n_tiles) {
      if (threadIdx.x == 0) set_status(ctl, DBG_E_INTERNAL);
      return;
    }
    for (uint64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) titem[t] = (uint32_t)ii;
  }
}

struct LevelArgs {
  const Item *items;
  const uint64_t *n_items_p;
  const uint64_t *n_tiles_p;
  const uint64_t *n_scatter_tiles_p;  // tiles [0, this) belong to scattered buckets
  uint64_t *hist;     // per-item digit counts (atomic mode)
  uint32_t *tpre;     // per-tile digit counts, then their column prefix (tile mode), or null
  uint64_t *cursor;
  uint32_t *w0, *w1;  // record weights beside buffers 0 and 1 (weighted scatter)
  const uint32_t *titem;  // the item of every tile (k_level_tilemap)
  uint32_t *rows;     // digit offsets inside every tile of in-tile items
  int bits;
  int level;
  int gate;
};

// Tile mode (a level with one large bucket, whose 256 counters every tile would
// otherwise hit with atomics): every tile writes its 256 digit counts to a row, a
// column prefix over the rows gives each tile the exact offset of each digit
// within its bucket, and the scatter needs no atomics.  Atomic mode (levels with
// many buckets): counts and cursors are reserved with global atomics.
__device__ __forceinline__ uint64_t item_end_tile(const Item *items, uint64_t ii, uint64_t n_items,
                                                  uint64_t n_tiles) {
  return ii + 1 < n_items ? items[ii + 1].tbase : n_tiles;
}

template <typename K, int NT = STREAM_NT>
__device__ __forceinline__ int load_tile(const K *src, uint64_t start, uint64_t end,
                                         K (&keys)[TILE / NT]) {
  int n = 0;
#pragma unroll
  for (int r = 0; r < (int)(TILE / NT); ++r) {
    const uint64_t i = start + threadIdx.x + (uint64_t)r * NT;
    if (i < end) {
      keys[r] = src[i];
      n = r + 1;
    }
  }
  return n;
}

template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_level_hist(LevelArgs a, K *b0, K *b1,
                                                          const Ctl *ctl) {
  __shared__ uint32_t h[256];
  if (ctl->status || gated_off(ctl, a.gate)) return;
  const uint64_t n_tiles = *a.n_scatter_tiles_p;
  // a contiguous run of tiles per workgroup: consecutive tiles mostly share their
  // bucket, whose counts then go out once per run instead of once per tile
  const uint64_t per = (n_tiles + gridDim.x - 1) / gridDim.x;
  const uint64_t t0 = blockIdx.x * per;
  const uint64_t t1 = t0 + per < n_tiles ? t0 + per : n_tiles;
  constexpr uint64_t NONE = ~0ull;
  uint64_t cur = NONE;
  Item it{};
  h[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t t = t0; t < t1; ++t) {
    const uint64_t ii = a.titem[t];
    if (ii != cur) {  // the same for the whole workgroup
      if (cur != NONE && !a.tpre) {
        const uint32_t c = h[threadIdx.x];
        if (c) atomicAdd((unsigned long long *)&a.hist[cur * 256 + threadIdx.x], (unsigned long long)c);
        h[threadIdx.x] = 0;
      }
      __syncthreads();
      cur = ii;
      it = a.items[ii];
    }
    if (it.in_tile) continue;  // split within its tiles by k_level_tiles
    const uint64_t start = it.off + (t - it.tbase) * TILE;
    const uint64_t end = it.off + it.size < start + TILE ? it.off + it.size : start + TILE;
    K keys[STREAM_KPT];
    // strided layout: key r of thread q is start + q + r * STREAM_NT
    const int n = load_tile<K>(it.src ? b1 : b0, start, end, keys);
#pragma unroll
    for (int r = 0; r < STREAM_KPT; ++r)
      if (r < n) atomicAdd(&h[msd_digit(keys[r], a.bits, a.level)], 1u);
    __syncthreads();
    if (a.tpre) {
      a.tpre[t * 256 + threadIdx.x] = h[threadIdx.x];
      h[threadIdx.x] = 0;
      __syncthreads();
    }
  }
  if (cur != NONE && !a.tpre) {
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd((unsigned long long *)&a.hist[cur * 256 + threadIdx.x], (unsigned long long)c);
  }
}

__global__ __launch_bounds__(STREAM_NT) void k_level_plan(PlanArgs p, LevelArgs a) {
  __shared__ PlanLds lds;
  if (p.ctl->status || gated_off(p.ctl, p.gate)) return;
  const uint64_t n_items = *a.n_items_p;
  for (uint64_t ii = blockIdx.x; ii < n_items; ii += gridDim.x) {
    const Item it = a.items[ii];
    uint64_t c = 0;
    if (it.in_tile) {  // the sum over the bucket's tiles of digit d's segment
      const SegParent sp{it.tbase, (uint32_t)((it.size + TILE - 1) / TILE), (uint32_t)it.size};
      const uint32_t d = threadIdx.x;
      // the rows of all the bucket's tiles are independent loads: unrolled, they
      // are in flight together instead of one tile's round trip at a time
#pragma unroll 8
      for (uint32_t i = 0; i < sp.tiles; ++i) c += seg_row(p, sp, i, d + 1) - seg_row(p, sp, i, d);
      plan_children(p, c, it.off, 1u, a.level + 1, nullptr, lds, &sp);
      continue;
    }
    if (a.tpre) {
      const uint64_t t1 = item_end_tile(a.items, ii, n_items, *a.n_tiles_p);
      c = (uint32_t)(a.tpre[t1 * 256 + threadIdx.x] - a.tpre[it.tbase * 256 + threadIdx.x]);
    } else {
      c = a.hist[ii * 256 + threadIdx.x];
    }
    plan_children(p, c, it.off, 1u - it.src, a.level + 1, a.cursor + ii * 256, lds);
  }
}

// Threads of the in-tile pass: its tile of 128-bit keys takes 64 KB of LDS, so
// two workgroups fit a CU, and 512 threads keep twice the loads in flight (it
// measured faster than 256; the level scatter measured faster with 256).
template <typename K> constexpr int tiles_nt() { return sizeof(K) == 16 ? TILES_NT_WIDE : STREAM_NT; }

template <typename K, bool W>
__global__ __launch_bounds__(STREAM_NT) void k_level_scatter(LevelArgs a, K *b0, K *b1,
                                                             const Ctl *ctl) {
  constexpr int NT = STREAM_NT;
  __shared__ PartLds<K, W, 1, NT> s;
  if (ctl->status || gated_off(ctl, a.gate)) return;
  const uint64_t n_tiles = *a.n_scatter_tiles_p;
  // this XCD's eighth of the tiles, strided over its workgroups (gridDim.x is a
  // multiple of 8)
  const uint64_t per = (n_tiles + N_XCD - 1) / N_XCD;
  const uint64_t x0 = (blockIdx.x % N_XCD) * per;
  const uint64_t x1 = x0 + per < n_tiles ? x0 + per : n_tiles;
  for (uint64_t t = x0 + blockIdx.x / N_XCD; t < x1; t += gridDim.x / N_XCD) {
    const uint64_t ii = a.titem[t];
    const Item it = a.items[ii];
    if (it.in_tile) continue;  // split within its tiles by k_level_tiles
    const uint64_t start = it.off + (t - it.tbase) * TILE;
    const uint64_t end = it.off + it.size < start + TILE ? it.off + it.size : start + TILE;
    K keys[TILE / NT];
    // keys are placed through LDS, so any assignment of keys to threads works:
    // use the coalesced strided one (valid keys form a prefix of each thread's)
    const int n = load_tile<K, NT>(it.src ? b1 : b0, start, end, keys);
    uint32_t wts[TILE / NT] = {};
    if (W) load_tile<uint32_t, NT>(it.src ? a.w1 : a.w0, start, end, wts);
    uint64_t *cur = a.cursor + ii * 256;
    uint64_t my_base = 0;
    if (a.tpre) {  // column prefixes are counted modulo 2^32 (a table has < 2^32 keys)
      const uint32_t d = threadIdx.x;
      if (d < 256)
        my_base = cur[d] + (uint32_t)(a.tpre[t * 256 + d] - a.tpre[it.tbase * 256 + d]);
      cur = nullptr;
    }
    partition_tile<K, W, 1, NT>(keys, wts, n, a.bits, a.level, cur, my_base, it.src ? b0 : b1,
                                it.src ? a.w0 : a.w1, s);
  }
}

// In-tile items: every tile partitioned by the level's digit in LDS and written
// back whole, digit-contiguous, to buffer 1 at its own positions (in place when
// the item is already there), with the offset of each digit inside the tile in
// the tile's row.
template <typename K>
__global__ __launch_bounds__(tiles_nt<K>()) void k_level_tiles(LevelArgs a, K *b0, K *b1,
                                                               const Ctl *ctl) {
  constexpr int NT = tiles_nt<K>();
  __shared__ PartLds<K, false, 1, NT> s;
  if (ctl->status || gated_off(ctl, a.gate)) return;
  const uint64_t n_tiles = *a.n_tiles_p;
  for (uint64_t t = *a.n_scatter_tiles_p + blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint64_t ii = a.titem[t];
    const Item it = a.items[ii];
    if (!it.in_tile) continue;
    const uint64_t start = it.off + (t - it.tbase) * TILE;
    const uint64_t end = it.off + it.size < start + TILE ? it.off + it.size : start + TILE;
    K keys[TILE / NT];
    const int n = load_tile<K, NT>(it.src ? b1 : b0, start, end, keys);
    const uint32_t nowt[TILE / NT] = {};
    // every thread has its keys before any key is written (the partition passes
    // barriers first), so the tile may be rewritten in place
    partition_tile<K, false, 1, NT>(keys, nowt, n, a.bits, a.level, nullptr, start, b1, nullptr,
                                    s, 0xffffffffu, a.rows + t * 256);
  }
}

// ---------------------------------------------------------------------------
// 4. LDS-resident sort of each batch by most-significant-digit refinement.
// Keys within a batch agree on every bit above the highest bit in which any two
// differ (hb), so the batch is first partitioned by the 8 bits below hb by the
// whole workgroup (LDS histogram, scan, atomic cursors; no stability is needed
// since equal keys are indistinguishable).  Each resulting segment holds keys
// that agree above its `shift` and is finished by the cheapest method for its
// size:
//   1 key, or no bits left (all keys equal)  -> already sorted;
//   <= SMALL keys                             -> one lane's sorting network;
//   <= 64 keys                                -> one wave, each lane ranking its
//                                                key against the others;
//   more                                      -> one wave partitions it by its
//                                                next 8 bits, and its pieces are
//                                                classified again.
// Segments are refined in ping-pong between two LDS buffers; every finished
// segment ends in buffer `a` at its final position, which is written out with
// coalesced stores.

__device__ __forceinline__ int bit_length(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
__device__ __forceinline__ int bit_length(u128 x) {
  const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  return hi ? 128 - __clzll(hi) : (lo ? 64 - __clzll(lo) : 0);
}
__device__ __forceinline__ uint64_t wave_or_key(uint64_t v) { return wave_or(v); }
__device__ __forceinline__ uint64_t wave_and_key(uint64_t v) { return wave_and(v); }
__device__ __forceinline__ u128 wave_and_key(u128 v) {
  const uint64_t lo = wave_and_key((uint64_t)v), hi = wave_and_key((uint64_t)(v >> 64));
  return ((u128)hi << 64) | lo;
}
__device__ __forceinline__ u128 wave_or_key(u128 v) {
  const uint64_t lo = wave_or((uint64_t)v), hi = wave_or((uint64_t)(v >> 64));
  return ((u128)hi << 64) | lo;
}
__device__ __forceinline__ uint64_t read_lane_key(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ u128 read_lane_key(u128 v, int l) {
  return ((u128)read_lane_key((uint64_t)(v >> 64), l) << 64) | read_lane_key((uint64_t)v, l);
}

// The 8-bit digit below `shift` (bits [shift-8, shift), fewer when shift < 8).
template <typename K> __device__ __forceinline__ uint32_t seg_digit(K key, int shift) {
  if (shift >= 8) return (uint32_t)(key >> (shift - 8)) & 0xffu;
  return (uint32_t)key & ((1u << shift) - 1u);
}

// Batcher's odd-even merge sorting network on N registers (N a power of two).
template <int N, typename K> __device__ __forceinline__ void sort_network(K (&v)[N]) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const K x = v[i + j], y = v[i + j + k];
            const bool sw = y < x;
            v[i + j] = sw ? y : x;
            v[i + j + k] = sw ? x : y;
          }
}

// Sorting network on (key, count) pairs, ordered by key.
template <int N, typename K>
__device__ __forceinline__ void sort_network_kv(K (&v)[N], uint32_t (&c)[N]) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const K x = v[i + j], y = v[i + j + k];
            const uint32_t cx = c[i + j], cy = c[i + j + k];
            const bool sw = y < x;
            v[i + j] = sw ? y : x;
            v[i + j + k] = sw ? x : y;
            c[i + j] = sw ? cy : cx;
            c[i + j + k] = sw ? cx : cy;
          }
}

// One lane sorts c <= N (key, count) pairs of a segment into buffer 0.
template <int N, typename K, typename CT>
__device__ __forceinline__ void network_segment(const K *kb, const CT *cb, K *k0, CT *c0,
                                                uint32_t start, uint32_t c) {
  K v[N];
  uint32_t w[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool in = (uint32_t)j < c;
    v[j] = in ? kb[start + j] : all_ones<K>();
    w[j] = in ? (uint32_t)cb[start + j] : 0u;
  }
  sort_network_kv<N, K>(v, w);
#pragma unroll
  for (int j = 0; j < N; ++j)
    if ((uint32_t)j < c) {
      k0[start + j] = v[j];
      c0[start + j] = (CT)w[j];
    }
}

// segment descriptor: start, size (16 bits each), shift + 128 (8 bits), buffer (1 bit)
__device__ __forceinline__ uint64_t seg_pack(uint32_t start, uint32_t size, int shift,
                                             uint32_t buf) {
  return (uint64_t)start | ((uint64_t)size << 16) | ((uint64_t)(uint32_t)(shift + 128) << 32) |
         ((uint64_t)buf << 40);
}
__device__ __forceinline__ uint32_t seg_start(uint64_t d) { return (uint32_t)d & 0xffffu; }
__device__ __forceinline__ uint32_t seg_size(uint64_t d) { return (uint32_t)(d >> 16) & 0xffffu; }
__device__ __forceinline__ int seg_shift(uint64_t d) { return (int)((d >> 32) & 0xffu) - 128; }
__device__ __forceinline__ uint32_t seg_buf(uint64_t d) { return (uint32_t)(d >> 40) & 1u; }

__device__ __forceinline__ uint64_t key_hash(uint64_t k) { return k * 0x9E3779B97F4A7C15ull; }
__device__ __forceinline__ uint64_t key_hash(u128 k) {
  return ((uint64_t)k ^ ((uint64_t)(k >> 64) * 0xC2B2AE3D27D4EB4Full)) * 0x9E3779B97F4A7C15ull;
}

// LDS of the bucket sort for keys of any width.  Buffer 0 (key0/cnt0) holds the
// staged keys while duplicates are merged, then receives every finished piece of
// the sorted distinct keys; the table region is reused for buffer 1.  Counts of
// distinct keys: 16 bits suffice for unweighted batches (at most CAP keys);
// summed record weights (W) take 32.
template <typename K, bool W, int V>
struct LocalLds {
  using Key = K;
  using Cfg = LocalCfg<K, W, V>;
  using CT = typename std::conditional<W, uint32_t, uint16_t>::type;
  static constexpr int NT = Cfg::NT, NW = NT / 64, CAP = Cfg::CAP;
  // the table (an owner index and a count per slot) takes all of the region it
  // shares with buffer 1: fewer collisions for the same LDS
  static constexpr size_t TBYTES_B = (size_t)CAP * (sizeof(K) + sizeof(CT));
  static constexpr int SLOTS =
      (int)((size_t)Cfg::SLOTS * 8 > TBYTES_B ? (size_t)Cfg::SLOTS : TBYTES_B / 8);
  static constexpr size_t TBYTES_A = (size_t)SLOTS * 8;
  static constexpr size_t TBYTES = TBYTES_A > TBYTES_B ? TBYTES_A : TBYTES_B;
  K key0[CAP];        // staged keys, then distinct keys (sorted in place)
  CT cnt0[CAP];
  uint16_t ulist[CAP];  // table slot of each distinct key, in discovery order
  alignas(16) unsigned char t[TBYTES];  // hash table | buffer 1
  uint32_t hist[NW][256];
  uint64_t large[2][CAP / 64 + 1];
  uint64_t mid[CAP / (Cfg::SMALL + 1) + 1];
  uint32_t nlarge[2], nmid, nuniq, dirty, hbits;
  K wor[NW];
  K wand[NW];
  uint32_t wsum[NW + 1];
  __device__ uint32_t *own() { return reinterpret_cast<uint32_t *>(t); }
  __device__ uint32_t *tcnt() { return reinterpret_cast<uint32_t *>(t) + SLOTS; }
  __device__ K *k0() { return key0; }
  __device__ CT *c0() { return cnt0; }
  __device__ K *key1() { return reinterpret_cast<K *>(t); }
  __device__ CT *cnt1() { return reinterpret_cast<CT *>(t + (size_t)CAP * sizeof(K)); }
  __device__ K *keys_of(uint32_t b) { return b ? key1() : key0; }
  __device__ CT *cnts_of(uint32_t b) { return b ? cnt1() : cnt0; }
};

// LDS of the 64-bit bucket sort: one region is the hash table (a key and a
// count per slot) while duplicates are merged, and the two piece buffers
// afterwards; it is cleared before every batch.  An all-ones key marks an empty
// slot: it is never a key (for k <= 31 the all-T (k+1)-mer is not canonical, and
// k-mer keys use at most 62 bits).
template <bool W, int V>
struct SlotLds {
  using Key = uint64_t;
  using Cfg = LocalCfg<uint64_t, W, V>;
  using CT = typename std::conditional<W, uint32_t, uint16_t>::type;
  static constexpr int NT = Cfg::NT, NW = NT / 64, CAP = Cfg::CAP;
  static constexpr size_t BUF = (size_t)CAP * (sizeof(Key) + sizeof(CT));
  static constexpr int SLOTS = (int)(2 * BUF / 12);
  alignas(16) unsigned char r[2 * BUF];
  uint16_t ulist[CAP];
  uint32_t hist[NW][256];
  uint64_t large[2][CAP / 64 + 1];
  uint64_t mid[CAP / (Cfg::SMALL + 1) + 1];
  uint32_t nlarge[2], nmid, nuniq, dirty, hbits;
  Key wor[NW];
  Key wand[NW];
  uint32_t wsum[NW + 1];
  __device__ unsigned long long *tkey() { return reinterpret_cast<unsigned long long *>(r); }
  __device__ uint32_t *tcnt() { return reinterpret_cast<uint32_t *>(r + (size_t)SLOTS * 8); }
  __device__ Key *k0() { return reinterpret_cast<Key *>(r); }
  __device__ CT *c0() { return reinterpret_cast<CT *>(r + (size_t)CAP * sizeof(Key)); }
  __device__ Key *key1() { return reinterpret_cast<Key *>(r + BUF); }
  __device__ CT *cnt1() { return reinterpret_cast<CT *>(r + BUF + (size_t)CAP * sizeof(Key)); }
  __device__ Key *keys_of(uint32_t b) { return b ? key1() : k0(); }
  __device__ CT *cnts_of(uint32_t b) { return b ? cnt1() : c0(); }
};

// Finish or enqueue one segment [start, start+c) of distinct keys in buffer `buf`
// whose keys agree above `shift`.  Called by one lane.
template <typename S>
__device__ __forceinline__ void classify_segment(S &s, uint32_t start, uint32_t c, int shift,
                                                 uint32_t buf, int nxt) {
  using K = typename S::Key;
  using CT = typename S::CT;
  constexpr int SMALL = S::Cfg::SMALL;
  if (c == 0) return;
  K *kb = s.keys_of(buf);
  CT *cb = s.cnts_of(buf);
  K *k0 = s.k0();
  CT *c0 = s.c0();
  if (c == 1) {
    if (buf) {
      k0[start] = kb[start];
      c0[start] = cb[start];
    }
    return;
  }
  // distinct keys: c >= 2 always leaves bits to split on (shift > 0)
  if (c == 2) {
    const K x = kb[start], y = kb[start + 1];
    const CT cx = cb[start], cy = cb[start + 1];
    const bool sw = y < x;
    k0[start] = sw ? y : x;
    k0[start + 1] = sw ? x : y;
    c0[start] = sw ? cy : cx;
    c0[start + 1] = sw ? cx : cy;
  } else if (c <= 4) {
    network_segment<4, K, CT>(kb, cb, k0, c0, start, c);
  } else if (c <= 8) {
    network_segment<8, K, CT>(kb, cb, k0, c0, start, c);
  } else if (c <= (uint32_t)SMALL) {
    network_segment<SMALL, K, CT>(kb, cb, k0, c0, start, c);
  } else if (c <= 64) {
    s.mid[atomicAdd(&s.nmid, 1u)] = seg_pack(start, c, shift, buf);
  } else {
    s.large[nxt][atomicAdd(&s.nlarge[nxt], 1u)] = seg_pack(start, c, shift, buf);
  }
}

// Bits [off, off + nu) of the bitmap set, the rest of [off, off + m) left
// clear (the bitmap starts zeroed).  Words wholly inside the range belong to
// this batch alone and are stored; the two boundary words are or-ed.
__device__ __forceinline__ void mark_positions(uint32_t *bits, uint64_t off, uint32_t m,
                                               uint32_t nu) {
  const uint64_t w0 = off >> 5, w1 = (off + m - 1) >> 5;
  for (uint64_t wi = w0 + threadIdx.x; wi <= w1; wi += blockDim.x) {
    const uint64_t p0 = wi << 5;
    const uint64_t lo = off > p0 ? off : p0;              // first position of the batch in the word
    const uint64_t hi_set = off + nu < p0 + 32 ? off + nu : p0 + 32;
    uint32_t mask = 0;
    if (hi_set > lo) {
      const uint32_t a = (uint32_t)(lo - p0), c = (uint32_t)(hi_set - lo);
      mask = (c == 32 ? 0xffffffffu : ((1u << c) - 1u)) << a;
    }
    const bool inside = off <= p0 && p0 + 32 <= off + m;
    if (inside) bits[wi] = mask;
    else if (mask) atomicOr(&bits[wi], mask);
  }
}

// The batch's distinct keys, sorted in buffer 0, replace its first positions in
// b0, their counts go to the same positions of the 32-bit count array, and the
// bitmap marks those positions.  Reads LDS only.
template <typename S, bool W>
__device__ __forceinline__ void write_batch(S &s, const Batch &bt, uint32_t nu,
                                            typename S::Key *b0, uint32_t *cnts,
                                            uint32_t *bits) {
  using K = typename S::Key;
  using CT = typename S::CT;
  const K *key0 = s.k0();
  const CT *cnt0 = s.c0();
  for (uint32_t u = threadIdx.x; u < nu; u += S::NT) {
    b0[bt.off + u] = key0[u];
    cnts[bt.off + u] = (uint32_t)cnt0[u] >> (W ? 1 : 0);
  }
  mark_positions(bits, bt.off, bt.size, nu);
}

// After duplicates are merged: the batch's nu distinct keys and counts are in
// registers (uk, uc: key u = tid + j NT), hb is the highest bit in which the
// batch's keys differ.  Partition them by a digit of about log2(nu) bits just
// below hb into buffer 0, sort every bucket of up to 64 keys by ranking each key
// against the others, refine the rare larger pieces, then write the sorted
// distinct keys over the batch's first positions of b0, their counts (halved for
// weighted records) to the same positions of the count array, and mark those
// positions in the bitmap (write_batch).  Ends with a barrier.  The caller must have passed a
// barrier after its last read of the LDS the buffers overwrite.  DEFER: the
// sorted keys are left in buffer 0 for the caller to write out later (every
// thread has passed a barrier since they were placed).
template <typename S, bool W, int UPT, bool DEFER = false>
__device__ __forceinline__ void finish_batch(S &s, const typename S::Key (&uk)[UPT],
                                             const uint32_t (&uc)[UPT], uint32_t nu, int hb,
                                             int dw_bias, const Batch &bt,
                                             typename S::Key *b0, uint32_t *cnts,
                                             uint32_t *bits, int key_bits) {
  using K = typename S::Key;
  using CT = typename S::CT;
  constexpr int NT = S::NT, NW = S::NW;
  constexpr int MAXDW = NW >= 8 ? 11 : 10;  // log2 of the first partition's bins
  // the first partition's bins, BPT per thread; their starts are kept in the
  // distinct-key list, so there are at most CAP of them
  constexpr int BINS = NW * 256 <= S::CAP ? NW * 256 : (1 << MAXDW);
  constexpr int BPT = BINS / NT;
  static_assert(BPT * NT == BINS && BINS <= S::CAP && (1 << MAXDW) <= BINS,
                "first-partition bins: a whole number per thread, at most CAP");
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  K *key0 = s.k0();
  CT *cnt0 = s.c0();
  // digit of the first partition: about one distinct key per bucket (shifted
  // by the tuning's bias), at most MAXDW bits, taken just below hb.  When the
  // keys differ inside the digit of the level that made the batch (they share
  // every bit above it, and it lies in [da, db)), the bins are (digit - da)
  // followed by the bits below it instead: that digit takes only db - da
  // values, so the bits just below hb would leave most bins empty and crowd
  // the rest.
  int dw, dshift;
  uint32_t dsub = 0;
  const int lvl = batch_level(bt.src);
  const int dhi = key_bits - 8 * lvl;  // the level's digit: bits [dpos, dhi)
  const int dpos = dhi - 8 > 0 ? dhi - 8 : 0;
  if (lvl >= 0 && hb > dpos && hb <= dhi) {
    const uint32_t da = batch_da(bt.src), range = batch_db(bt.src) - da;
    const int rbits = bit_length((uint64_t)(range - 1));
    int x = MAXDW - rbits + dw_bias;
    const int xmax = MAXDW - rbits < dpos ? MAXDW - rbits : dpos;
    x = x < 0 ? 0 : x > xmax ? xmax : x;
    dw = dhi - dpos + x;
    dshift = dpos - x;
    dsub = da << x;
  } else {
    dw = (nu <= 256 ? 8 : bit_length((uint64_t)(nu - 1))) + dw_bias;
    dw = dw < 1 ? 1 : dw > MAXDW ? MAXDW : dw;
    dw = dw > hb ? hb : dw;
    dshift = hb - dw;
  }
  uint32_t *H = &s.hist[0][0];  // NW * 256 bins, zeroed by the caller
  uint32_t ud[UPT];
#pragma unroll
  for (int j = 0; j < UPT; ++j) {
    ud[j] = 0;
    if (tid + (uint32_t)j * NT < nu) {
      ud[j] = dw > 0 ? ((uint32_t)shr<K>(uk[j], dshift) & ((1u << dw) - 1u)) - dsub : 0u;
      atomicAdd(&H[ud[j]], 1u);
    }
  }
  __syncthreads();
  if (tid == 0) s.nuniq = 0;  // every thread holds nu; ready for the next batch
  // thread t owns bins BPT t .. BPT t + BPT - 1
  uint32_t c4[BPT], st4[BPT], sum4 = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    c4[q] = H[BPT * tid + q];
    sum4 += c4[q];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan<NT>(sum4, s.wsum, &tot);
  uint16_t *bstart = s.ulist;  // the list is read out: it now keeps the bucket starts
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    st4[q] = run;
    H[BPT * tid + q] = run;
    bstart[BPT * tid + q] = (uint16_t)run;
    run += c4[q];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < UPT; ++j)
    if (tid + (uint32_t)j * NT < nu) {
      const uint32_t q = atomicAdd(&H[ud[j]], 1u);
      key0[q] = uk[j];
      cnt0[q] = (CT)uc[j];
    }
  __syncthreads();
  // buckets of up to 64 keys: every distinct key counts the smaller keys of
  // its bucket, then all of them move to their final places at once (the
  // reads finish before the barrier, so the moves can be in place)
  constexpr uint32_t NOPOS = 0xffffffffu;
  uint32_t fin[UPT];
#pragma unroll
  for (int j = 0; j < UPT; ++j) {
    fin[j] = NOPOS;
    if (tid + (uint32_t)j * NT < nu) {
      const uint32_t b = bstart[ud[j]], e = H[ud[j]];
      if (e - b <= 64u) {
        // four reads in flight per step
        const K x = uk[j];
        uint32_t r = 0, i = b;
        for (; i + 4 <= e; i += 4) {
          const K a0 = key0[i], a1 = key0[i + 1], a2 = key0[i + 2], a3 = key0[i + 3];
          r += (a0 < x ? 1u : 0u) + (a1 < x ? 1u : 0u) + (a2 < x ? 1u : 0u) + (a3 < x ? 1u : 0u);
        }
        for (; i < e; ++i) r += key0[i] < x ? 1u : 0u;
        fin[j] = b + r;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < UPT; ++j)
    if (fin[j] != NOPOS) {
      key0[fin[j]] = uk[j];
      cnt0[fin[j]] = (CT)uc[j];
    }
#pragma unroll
  for (int q = 0; q < BPT; ++q)
    if (c4[q] > 64u) classify_segment(s, st4[q], c4[q], dshift, 0u, 0);
  __syncthreads();
  // pieces left over (usually none): refined until every piece is finished
  int cur = 0;
  while (s.nmid != 0 || s.nlarge[cur] != 0) {
    // pieces of SMALL+1..64 keys (or with no bits left): lane ranks its keys
    for (uint32_t i = w; i < s.nmid; i += NW) {
      const uint64_t d = s.mid[i];
      const uint32_t st = seg_start(d), c = seg_size(d), buf = seg_buf(d);
      const K *kb = s.keys_of(buf);
      const CT *cb = s.cnts_of(buf);
      const uint32_t me = lane;
      const K x = me < c ? kb[st + me] : all_ones<K>();
      const uint32_t xc = me < c ? cb[st + me] : 0u;
      uint32_t rank = 0;
      for (uint32_t j = 0; j < c; ++j) rank += kb[st + j] < x ? 1u : 0u;
      // c <= 64, so this runs once per piece: when the piece is already in
      // buffer 0 the wave's reads above precede its writes below (LDS
      // operations of one wave complete in order)
      if (me < c) {
        key0[st + rank] = x;
        cnt0[st + rank] = (CT)xc;
      }
    }
    __syncthreads();
    if (tid == 0) s.nmid = 0;
    const uint32_t nl = s.nlarge[cur];
    __syncthreads();
    if (nl == 0) break;
    // larger pieces: one wave each, partitioned by the 8 bits below their
    // highest differing bit into the other buffer
    for (uint32_t i = w; i < nl; i += NW) {
      const uint64_t d = s.large[cur][i];
      const uint32_t st = seg_start(d), c = seg_size(d), buf = seg_buf(d);
      const K *ik = s.keys_of(buf);
      const CT *ic = s.cnts_of(buf);
      K *ok = s.keys_of(buf ^ 1u);
      CT *oc = s.cnts_of(buf ^ 1u);
      if (buf == 0 && lane == 0) s.dirty = 1;  // buffer 1 overwrites the hash table
      uint32_t *h = s.hist[w];
      K dd = 0;
      const K kk = ik[st];
      for (uint32_t e = lane; e < c; e += 64) dd |= ik[st + e] ^ kk;
      const int shift = bit_length(wave_or_key(dd));
#pragma unroll
      for (int q = 0; q < 4; ++q) h[lane + 64 * q] = 0;
      for (uint32_t e = lane; e < c; e += 64) atomicAdd(&h[seg_digit(ik[st + e], shift)], 1u);
      uint32_t cnt[4], pre[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cnt[q] = h[4 * lane + q];
        pre[q] = sum;
        sum += cnt[q];
      }
      const uint32_t base = st + wave_inclusive_scan(sum) - sum;
#pragma unroll
      for (int q = 0; q < 4; ++q) h[4 * lane + q] = base + pre[q];
      for (uint32_t e = lane; e < c; e += 64) {
        const K key = ik[st + e];
        const uint32_t q = atomicAdd(&h[seg_digit(key, shift)], 1u);
        ok[q] = key;
        oc[q] = ic[st + e];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        classify_segment(s, base + pre[q], cnt[q], shift - 8, buf ^ 1u, cur ^ 1);
    }
    __syncthreads();
    if (tid == 0) s.nlarge[cur] = 0;
    cur ^= 1;
    __syncthreads();
  }
  if (!DEFER) {
    write_batch<S, W>(s, bt, nu, b0, cnts, bits);
    __syncthreads();
  }
}

// A batch descriptor read ahead is held in one VGPR, dword l in lane l < 4, so
// that the compiler cannot move it into scalar registers (and wait for the load)
// before it is used a whole batch later.  The index is clamped to the last
// descriptor: a descriptor is only used while its index is below n.
__device__ __forceinline__ uint32_t desc_lane_load(const Batch *batches, uint64_t i, uint64_t n) {
  static_assert(sizeof(Batch) == 16, "four dwords: off (lo, hi), size, src");
  const uint32_t l = lane_id();
  uint32_t v = 0;
  if (n && l < 4) v = reinterpret_cast<const uint32_t *>(batches + (i < n ? i : n - 1))[l];
  return v;
}
__device__ __forceinline__ Batch desc_unpack(uint32_t v) {
  const uint32_t lo = __builtin_amdgcn_readlane(v, 0), hi = __builtin_amdgcn_readlane(v, 1);
  return Batch{((uint64_t)hi << 32) | lo, (uint32_t)__builtin_amdgcn_readlane(v, 2),
               (uint32_t)__builtin_amdgcn_readlane(v, 3)};
}

// Digit ranges of in-tile buckets: the descriptor and the segment table read
// ahead in one VGPR each (descriptor dword l in lane l < 8, table word l in lane
// l), as desc_lane_load.
struct SegDesc {
  uint64_t out, item_off;
  uint32_t size, tiles, range;
};
// The lane index made opaque where it is used, so that per-lane addresses are
// formed in the loop rather than kept live across it (they were spilled, and
// the reloads waited for every memory operation in flight).
__device__ __forceinline__ uint32_t opaque_lane() {
  uint32_t l = lane_id();
  asm volatile("" : "+v"(l));
  return l;
}
__device__ __forceinline__ uint32_t seg_lane_load(const SegBatch *segb, uint64_t i, uint64_t n) {
  static_assert(sizeof(SegBatch) == 32, "eight dwords");
  const uint32_t l = opaque_lane();
  uint32_t v = 0;
  if (n && l < 8) v = reinterpret_cast<const uint32_t *>(segb + (i < n ? i : n - 1))[l];
  return v;
}
__device__ __forceinline__ uint32_t tab_lane_load(const uint32_t *segt, uint64_t i, uint64_t n) {
  static_assert(SEG_TILES == 64, "a table word per lane");
  return n ? segt[(i < n ? i : n - 1) * SEG_TILES + opaque_lane()] : 0u;
}
__device__ __forceinline__ SegDesc seg_unpack(uint32_t v) {
  auto rl = [&](int l) { return (uint32_t)__builtin_amdgcn_readlane(v, l); };
  return SegDesc{((uint64_t)rl(1) << 32) | rl(0), ((uint64_t)rl(5) << 32) | rl(4), rl(2), rl(3),
                 rl(6)};
}
// Keys of a digit range into registers (key e = tid + j NT as load_batch): the
// range is the concatenation of its segments in tile order (lane l < tiles holds
// tile l's segment in `tab`); each wave finds the segment of its 64 keys from the
// segment starts its lanes hold (ballots, then the few segment boundaries inside
// the wave's span).  Every lane of the wave must be active.
template <typename K, int NT, int LPT>
__device__ __forceinline__ void load_seg(const SegDesc &d, uint32_t tab, const K *b1,
                                         K (&pre)[LPT]) {
  const uint32_t l = opaque_lane();
  const bool mine = l < d.tiles;
  const uint32_t ra = tab & 0xffffu, rb = tab >> 16;
  const uint32_t sz = mine ? rb - ra : 0u;
  const uint32_t S = wave_inclusive_scan(sz) - sz;  // first key of segment l in the range
  const uint64_t P = d.item_off + (uint64_t)l * TILE + ra;  // its first key in buffer 1
  // the wave's first key (uniform), then every position before any load is
  // issued, so that nothing waits between the loads
  const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u;
  uint64_t pos[LPT];
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
    const uint32_t e0 = w0 + (uint32_t)j * NT;
    pos[j] = ~0ull;
    if (e0 >= d.size) continue;  // the same for the whole wave
    const uint32_t e = e0 + l;
    const uint32_t elast = e0 + 63 < d.size ? e0 + 63 : d.size - 1;
    const int i0 = __popcll(__ballot(mine && S <= e0)) - 1;
    const int i1 = __popcll(__ballot(mine && S <= elast)) - 1;
    uint32_t si = (uint32_t)__builtin_amdgcn_readlane(S, i0);
    uint64_t pi = read_lane(P, i0);
    for (int q = i0 + 1; q <= i1; ++q) {
      const uint32_t sq = (uint32_t)__builtin_amdgcn_readlane(S, q);
      const uint64_t pq = read_lane(P, q);
      if (e >= sq) {
        si = sq;
        pi = pq;
      }
    }
    if (e < d.size) pos[j] = pi + (e - si);
  }
#pragma unroll
  for (int j = 0; j < LPT; ++j) pre[j] = pos[j] != ~0ull ? b1[pos[j]] : K(0);
}

// Keys (and weights) of a batch into registers: key e = tid + j NT.
template <typename K, bool W, int NT, int LPT>
__device__ __forceinline__ void load_batch(const Batch &b, const K *b0, const K *b1,
                                           const uint32_t *w0, const uint32_t *w1,
                                           K (&pre)[LPT], uint32_t (&prew)[W ? LPT : 1]) {
  const K *src = batch_buf(b.src) ? b1 : b0;
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
    const uint32_t e = threadIdx.x + (uint32_t)j * NT;
    pre[j] = e < b.size ? src[b.off + e] : K(0);
  }
  if (W) {
    const uint32_t *srcw = batch_buf(b.src) ? w1 : w0;
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      const uint32_t e = threadIdx.x + (uint32_t)j * NT;
      prew[j] = e < b.size ? srcw[b.off + e] : 0u;
    }
  }
}

// One wave (all lanes active): the highest bit in which the batch's keys differ,
// from the waves' OR and AND of their keys, into s.hbits.
template <typename S> __device__ __forceinline__ void publish_high_bit(S &s) {
  using K = typename S::Key;
  const uint32_t l = lane_id();
  K o = 0, a = all_ones<K>();
  if (l < (uint32_t)S::NW) {
    o = s.wor[l];
    a = s.wand[l];
  }
  o = wave_or_key(o);
  a = wave_and_key(a);
  if (l == 0) s.hbits = (uint32_t)bit_length(o ^ a);
}

// Claimed slots of a wave appended to the distinct-key list with one atomic.
template <typename S, int LPT>
__device__ __forceinline__ void record_claims(S &s, uint32_t claimed, uint32_t ncl,
                                              const uint32_t (&hs)[LPT]) {
  const uint32_t incl = wave_inclusive_scan(ncl);
  const uint32_t wtot = read_lane(incl, 63);
  uint32_t base = 0;
  if (lane_id() == 0 && wtot) base = atomicAdd(&s.nuniq, wtot);
  base = read_lane(base, 0) + incl - ncl;
#pragma unroll
  for (int j = 0; j < LPT; ++j)
    if (claimed & (1u << j)) s.ulist[base++] = (uint16_t)hs[j];
}

// Sort a batch of up to CAP keys (consecutive small buckets) in LDS:
//  1. the batch's keys (loaded into registers while the previous batch was
//     sorted) and the bits in which they differ (OR ^ AND over all keys);
//  2. each key inserted into an LDS hash table, counting duplicates (summing
//     weights for weighted records);
//  3. the distinct keys and counts read out of the table into registers and
//     sorted by finish_batch, which writes them out.
// k_local_sort keys its table by the index of each key's first occurrence in
// the staged batch (so 128-bit keys need no 128-bit CAS); k_local_sort64 keeps
// 64-bit keys in the table slots themselves (no staging, one 64-bit CAS per key).
// W: weighted records (node table from edge endpoints): the weights, stored
// beside the keys in w0 / w1, are summed per distinct key instead of counting
// occurrences, and the sum is halved on output (each k-mer occurrence is seen
// twice).
// SEG: the batches are the digit ranges of in-tile buckets (segb, one segment
// per tile in buffer 1, found through the tiles' rows); their sorted distinct
// keys go to their places in buffer 0 as for any batch.
template <typename K, bool W, int V, bool SEG = false>
__global__ __launch_bounds__((LocalCfg<K, W, V>::NT)) void k_local_sort(
    const Batch *batches, const uint64_t *n_batches_p, K *b0, K *b1, const uint32_t *w0,
    const uint32_t *w1, uint32_t *cnts, uint32_t *bits, const Ctl *ctl, int gate, int dw_bias,
    int key_bits, const SegBatch *segb, const uint32_t *segt) {
  static_assert(!(SEG && W), "digit ranges of unweighted tables only");
  using S = LocalLds<K, W, V>;
  constexpr int NT = S::NT, NW = S::NW, SLOTS = S::SLOTS;
  constexpr uint32_t EMPTY = 0xffffffffu;
  constexpr int LPT = (S::CAP + NT - 1) / NT;  // keys per thread
  __shared__ S s;
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const uint64_t n_batches = *n_batches_p;
  const uint64_t G = gridDim.x;
  uint32_t *own = s.own(), *tcnt = s.tcnt();
  K pre[LPT];
  uint32_t prew[W ? LPT : 1];
  if (tid == 0) {
    s.dirty = 1;  // the table starts uninitialised
    s.nuniq = s.nmid = 0;
    s.nlarge[0] = s.nlarge[1] = 0;
  }
  __syncthreads();
  const Batch none = {0, 0, 0};
  Batch prev = none;  // the previous batch: written out once this batch's keys are in
  uint32_t prev_nu = 0;
  Batch nxt;
  uint32_t nd2;
  uint32_t nt2 = 0;  // SEG: the segment table read with nd2
  if constexpr (SEG) {
    nxt = none;
    if (blockIdx.x < n_batches) {
      const SegDesc d0 = seg_unpack(seg_lane_load(segb, blockIdx.x, n_batches));
      nxt = Batch{d0.out, d0.size, d0.range};
      load_seg<K, NT, LPT>(d0, tab_lane_load(segt, blockIdx.x, n_batches), b1, pre);
    }
    nd2 = seg_lane_load(segb, blockIdx.x + G, n_batches);
    nt2 = tab_lane_load(segt, blockIdx.x + G, n_batches);
  } else {
    nxt = blockIdx.x < n_batches ? batches[blockIdx.x] : none;
    load_batch<K, W, NT, LPT>(nxt, b0, b1, w0, w1, pre, prew);
    nd2 = desc_lane_load(batches, blockIdx.x + G, n_batches);
  }
  for (uint64_t bi = blockIdx.x; bi < n_batches; bi += G) {
    const Batch bt = nxt;
    const uint32_t m = bt.size;
    // 1. the bits in which the batch's keys differ (OR ^ AND; the first use of
    //    the keys, so the wait for them comes here)
    K kor = 0, kand = all_ones<K>();
#pragma unroll
    for (int j = 0; j < LPT; ++j)
      if (tid + (uint32_t)j * NT < m) {
        kor |= pre[j];
        kand &= pre[j];
      }
    kor = wave_or_key(kor);
    kand = wave_and_key(kand);
    if (lane == 0) {
      s.wor[w] = kor;
      s.wand[w] = kand;
    }
    // the previous batch's output, issued only now (the wait for this batch's
    // keys would otherwise also wait for these stores) and read out of buffer 0
    // before the keys are staged over it
    if (bi != blockIdx.x) {
      write_batch<S, W>(s, prev, prev_nu, b0, cnts, bits);
      __syncthreads();
    }
    // stage the keys
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      const uint32_t e = tid + (uint32_t)j * NT;
      if (e < m) s.key0[e] = pre[j];
    }
    if (s.dirty) {  // uniform: read after the previous batch's final barrier
      for (uint32_t q = tid; q < (uint32_t)SLOTS; q += NT) {
        own[q] = EMPTY;
        tcnt[q] = 0;
      }
    }
    // the piece lists are empty and the distinct-key counter is zero here: both
    // are left so by the previous batch
    for (uint32_t q = tid; q < (uint32_t)(NW * 256); q += NT) s.hist[0][q] = 0;
    __syncthreads();
    if (tid == 0) s.dirty = 0;
    if (w == 0) publish_high_bit(s);  // read after the barrier that ends the merge
    // 2. count duplicates in an LDS hash table keyed by the first occurrence:
    //    first probe of every key of this thread at once (independent LDS
    //    atomics in flight), then the keys that own the probed slots (again all
    //    at once), then linear probing for the few that collided
    {
      uint32_t hs[LPT], os[LPT];
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
        const uint32_t e = tid + (uint32_t)j * NT;
        hs[j] = 0;
        os[j] = EMPTY;
        if (e < m) {
          hs[j] = (uint32_t)(((key_hash(pre[j]) >> 32) * (uint64_t)SLOTS) >> 32);
          os[j] = atomicCAS(&own[hs[j]], EMPTY, e);
        }
      }
      bool same[LPT];
#pragma unroll
      for (int j = 0; j < LPT; ++j) same[j] = os[j] == EMPTY || s.key0[os[j]] == pre[j];
      uint32_t claimed = 0, ncl = 0;  // bit j: this thread's key j claimed slot hs[j]
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
        const uint32_t e = tid + (uint32_t)j * NT;
        if (e < m) {
          uint32_t h = hs[j], o = os[j];
          if (!same[j]) {
            const K key = pre[j];
            do {
              h = h + 1 == (uint32_t)SLOTS ? 0u : h + 1;
              o = atomicCAS(&own[h], EMPTY, e);
            } while (o != EMPTY && s.key0[o] != key);
            hs[j] = h;
          }
          if (o == EMPTY) {
            claimed |= 1u << j;
            ++ncl;
          }
          atomicAdd(&tcnt[h], W ? prew[j] : 1u);
        }
      }
      record_claims(s, claimed, ncl, hs);
    }
    __syncthreads();
    // the next batch's keys load while this one is sorted (descriptors are read
    // two batches ahead)
    if constexpr (SEG) {
      const SegDesc nxs = seg_unpack(nd2);
      const uint32_t tab = nt2;
      nxt = Batch{nxs.out, nxs.size, nxs.range};
      nd2 = seg_lane_load(segb, bi + 2 * G, n_batches);
      nt2 = tab_lane_load(segt, bi + 2 * G, n_batches);
      if (bi + G < n_batches) load_seg<K, NT, LPT>(nxs, tab, b1, pre);
    } else {
      nxt = desc_unpack(nd2);
      nd2 = desc_lane_load(batches, bi + 2 * G, n_batches);
      if (bi + G < n_batches) load_batch<K, W, NT, LPT>(nxt, b0, b1, w0, w1, pre, prew);
    }
    const int hb = (int)s.hbits;
    // 3. distinct keys read from the table into registers through the list of
    //    claimed slots (which are reset for the next batch)
    const uint32_t nu = s.nuniq;
    K uk[LPT];
    uint32_t uc[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      const uint32_t u = tid + (uint32_t)j * NT;
      uc[j] = 0;
      uk[j] = K(0);
      if (u < nu) {
        const uint32_t q = s.ulist[u];
        uk[j] = s.key0[own[q]];
        uc[j] = tcnt[q];
        own[q] = EMPTY;
        tcnt[q] = 0;
      }
    }
    finish_batch<S, W, LPT, true>(s, uk, uc, nu, hb, dw_bias, bt, b0, cnts, bits, key_bits);
    prev = bt;
    prev_nu = nu;
  }
  if (blockIdx.x < n_batches) write_batch<S, W>(s, prev, prev_nu, b0, cnts, bits);
}

template <bool W, int V>
__global__ __launch_bounds__((LocalCfg<uint64_t, W, V>::NT)) __attribute__((amdgpu_waves_per_eu(LocalCfg<uint64_t, W, V>::WAVES_PER_EU))) void k_local_sort64(
    const Batch *batches, const uint64_t *n_batches_p, uint64_t *b0, uint64_t *b1,
    const uint32_t *w0, const uint32_t *w1, uint32_t *cnts, uint32_t *bits, const Ctl *ctl,
    int gate, int dw_bias, int key_bits) {
  using S = SlotLds<W, V>;
  using K = uint64_t;
  constexpr int NT = S::NT, NW = S::NW, SLOTS = S::SLOTS;
  constexpr unsigned long long EMPTY = ~0ull;
  constexpr int LPT = (S::CAP + NT - 1) / NT;  // keys per thread
  __shared__ S s;
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const uint64_t n_batches = *n_batches_p;
  const uint64_t G = gridDim.x;
  unsigned long long *tkey = s.tkey();
  uint32_t *tcnt = s.tcnt();
  K pre[LPT];
  uint32_t prew[W ? LPT : 1];
  if (tid == 0) {
    s.dirty = 1;  // the region starts uninitialised
    s.nuniq = s.nmid = 0;
    s.nlarge[0] = s.nlarge[1] = 0;
  }
  __syncthreads();
  uint32_t prev_nu = 0;  // distinct keys of the previous batch, left in buffer 0
  const Batch none = {0, 0, 0};
  Batch prev = none;  // the previous batch: written out once this batch's keys are in
  Batch nxt = blockIdx.x < n_batches ? batches[blockIdx.x] : none;
  load_batch<K, W, NT, LPT>(nxt, b0, b1, w0, w1, pre, prew);
  uint32_t nd2 = desc_lane_load(batches, blockIdx.x + G, n_batches);
  for (uint64_t bi = blockIdx.x; bi < n_batches; bi += G) {
    const Batch bt = nxt;
    const uint32_t m = bt.size;
    // 1. the bits in which the batch's keys differ (OR ^ AND); the region was
    //    last read before the previous batch's final barrier, so it is made an
    //    empty table again here: the readout reset the claimed slots, so only
    //    the slots that buffer 0 overwrote need resetting, unless buffer 1 was
    //    used too (then all of it)
    K kor = 0, kand = all_ones<K>();
#pragma unroll
    for (int j = 0; j < LPT; ++j)
      if (tid + (uint32_t)j * NT < m) {
        kor |= pre[j];
        kand &= pre[j];
      }
    kor = wave_or_key(kor);
    kand = wave_and_key(kand);
    if (lane == 0) {
      s.wor[w] = kor;
      s.wand[w] = kand;
    }
    // the previous batch's output, issued only now: the wait for this batch's
    // keys (above) would otherwise also wait for these stores
    if (bi != blockIdx.x) write_batch<S, W>(s, prev, prev_nu, b0, cnts, bits);
    __syncthreads();  // read out before the region is cleared
    if (w == 0) publish_high_bit(s);  // read after the barrier that ends the merge
    if (s.dirty) {  // uniform: set before the previous batch's last barrier
      uint4 *r4 = reinterpret_cast<uint4 *>(s.r);
      constexpr uint32_t nkey4 = (uint32_t)SLOTS * 8 / 16, ncnt4 = (uint32_t)SLOTS * 4 / 16;
      const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u), zeros = make_uint4(0u, 0u, 0u, 0u);
      for (uint32_t q = tid; q < nkey4; q += NT) r4[q] = ones;
      for (uint32_t q = tid; q < ncnt4; q += NT) r4[nkey4 + q] = zeros;
    } else {
      // key0 = slots [0, nu), cnt0 = slots from CAP on (both inside the key part)
      constexpr uint32_t cslot = (uint32_t)(S::CAP * sizeof(K) / 8);
      const uint32_t ncs = (uint32_t)((prev_nu * sizeof(typename S::CT) + 7) / 8);
      for (uint32_t q = tid; q < prev_nu; q += NT) tkey[q] = EMPTY;
      for (uint32_t q = tid; q < ncs; q += NT) tkey[cslot + q] = EMPTY;
    }
    for (uint32_t q = tid; q < (uint32_t)(NW * 256); q += NT) s.hist[0][q] = 0;
    __syncthreads();
    if (tid == 0) s.dirty = 0;
    // 2. count duplicates in an LDS hash table holding the keys: first probe of
    //    every key of this thread at once, then linear probing for the few
    //    that collided
    {
      uint32_t hs[LPT];
      unsigned long long os[LPT];
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
        const uint32_t e = tid + (uint32_t)j * NT;
        hs[j] = 0;
        os[j] = EMPTY;
        if (e < m) {
          hs[j] = (uint32_t)(((key_hash(pre[j]) >> 32) * (uint64_t)SLOTS) >> 32);
          os[j] = atomicCAS(&tkey[hs[j]], EMPTY, (unsigned long long)pre[j]);
        }
      }
      uint32_t claimed = 0, ncl = 0;  // bit j: this thread's key j claimed slot hs[j]
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
        const uint32_t e = tid + (uint32_t)j * NT;
        if (e < m) {
          const unsigned long long key = pre[j];
          uint32_t h = hs[j];
          unsigned long long o = os[j];
          while (o != EMPTY && o != key) {
            h = h + 1 == (uint32_t)SLOTS ? 0u : h + 1;
            o = atomicCAS(&tkey[h], EMPTY, key);
          }
          hs[j] = h;
          if (o == EMPTY) {
            claimed |= 1u << j;
            ++ncl;
          }
          atomicAdd(&tcnt[h], W ? prew[j] : 1u);
        }
      }
      record_claims(s, claimed, ncl, hs);
    }
    __syncthreads();
    nxt = desc_unpack(nd2);
    nd2 = desc_lane_load(batches, bi + 2 * G, n_batches);
    if (bi + G < n_batches) load_batch<K, W, NT, LPT>(nxt, b0, b1, w0, w1, pre, prew);
    const int hb = (int)s.hbits;
    // 3. distinct keys and counts read out through the list of claimed slots
    const uint32_t nu = s.nuniq;
    K uk[LPT];
    uint32_t uc[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      const uint32_t u = tid + (uint32_t)j * NT;
      uc[j] = 0;
      uk[j] = K(0);
      if (u < nu) {
        const uint32_t q = s.ulist[u];
        uk[j] = (K)tkey[q];
        uc[j] = tcnt[q];
        tkey[q] = EMPTY;  // leave the table empty for the next batch
        tcnt[q] = 0;
      }
    }
    finish_batch<S, W, LPT, true>(s, uk, uc, nu, hb, dw_bias, bt, b0, cnts, bits, key_bits);
    prev_nu = nu;
    prev = bt;
  }
  if (blockIdx.x < n_batches) write_batch<S, W>(s, prev, prev_nu, b0, cnts, bits);
}

// Oversized buckets whose digits are exhausted hold one key repeated: one
// distinct key whose count is the bucket size.
template <typename K>
__global__ void k_uniform_emit(const Item *uni, const uint64_t *n_uni_p, K *b0, K *b1,
                               uint32_t *cnts, uint32_t *bits, const Ctl *ctl, int gate) {
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t n = *n_uni_p;
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < n;
       u += (uint64_t)gridDim.x * blockDim.x) {
    const Item it = uni[u];
    const K key = (it.src ? b1 : b0)[it.off];
    b0[it.off] = key;
    cnts[it.off] = (uint32_t)it.size;
    atomicOr(&bits[it.off >> 5], 1u << (it.off & 31));
  }
}

// Weighted records: the bucket's count is half the sum of its weights; one
// workgroup per bucket.
template <typename K>
__global__ __launch_bounds__(256) void k_uniform_emit_w(const Item *uni, const uint64_t *n_uni_p,
                                                        K *b0, K *b1, const uint32_t *w0,
                                                        const uint32_t *w1, uint32_t *cnts,
                                                        uint32_t *bits, const Ctl *ctl,
                                                        int gate) {
  __shared__ uint64_t wsum[256 / 64 + 1];
  if (ctl->status || gated_off(ctl, gate)) return;
  const uint64_t n = *n_uni_p;
  for (uint64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const Item it = uni[u];
    const uint32_t *wt = it.src ? w1 : w0;
    uint64_t sum = 0;
    for (uint64_t i = threadIdx.x; i < it.size; i += 256) sum += wt[it.off + i];
    uint64_t tot;
    block_exclusive_scan<256>(sum, wsum, &tot);
    if (threadIdx.x == 0) {
      const K key = (it.src ? b1 : b0)[it.off];
      b0[it.off] = key;
      cnts[it.off] = (uint32_t)(tot >> 1);
      atomicOr(&bits[it.off >> 5], 1u << (it.off & 31));
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Node table from edge endpoints (STEP-3 of Sec. 3 with counts).  Each distinct
// edge (u, v, multiplicity m) gives the records (u, m) and (v, m); each read of
// at least k bases gives (canonical first k-mer, 1) and (canonical last k-mer,
// 1).  Every k-mer occurrence is counted twice over these records, so a node's
// count is half its summed weight.  Reads shorter than k give two records of
// weight 0 on the first edge's u (an existing node), which leave every count
// unchanged and keep the record index a plain function of the read index.

// Chooses the route of the node table (after the node table's key offsets are
// known and the edge table is complete).
__global__ void k_node_path(Ctl *ctl, uint64_t n_reads, uint64_t n_sets, int mode, float ratio,
                            uint64_t key_buf_bytes, uint64_t weight_off, int key_bytes) {
  if (threadIdx.x || blockIdx.x) return;
  ctl->node_path = 0;
  ctl->n_records = 0;
  if (ctl->status || mode == 0) return;
  const uint64_t ne = ctl->n_edges, nk = ctl->n_keys;
  const uint64_t r = 2 * ne + 2 * n_reads;
  const bool fits = r * (uint64_t)key_bytes <= weight_off && weight_off + 4 * r <= key_buf_bytes;
  const bool ok = n_sets == 1 && !ctl->capacity_short && ne > 0 && nk < (1ull << 31) && fits;
  const bool take = ok && (mode == 1 || (double)r <= (double)ratio * (double)nk);
  if (take) {
    ctl->node_path = 1;
    ctl->n_records = r;
  }
}

// The records, written tile by tile (4096 records, the tiles of the level-0
// partition that follows), with each tile's counts of the top digit: the row
// that partition's tile mode reads, so the records are not read back to count
// them.  Record 2j and 2j+1: the endpoints u and v of distinct edge j with its
// multiplicity; record 2 ne + 2i and 2 ne + 2i + 1: the first and last k-mer of
// read i with weight 1 (weight 0 on the first edge's u for reads shorter than k).
template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_records(const K *u, const K *v,
                                                       const uint32_t *mult,
                                                       const uint64_t *packed, uint64_t n_words,
                                                       const uint64_t *offsets, int k, int bits,
                                                       K *keys, uint32_t *wts, uint32_t *thist,
                                                       const Ctl *ctl) {
  __shared__ uint32_t h[256];
  if (ctl->status || ctl->node_path != 1) return;
  const uint64_t ne = ctl->n_edges, n_rec = ctl->n_records;
  const uint64_t n_tiles = (n_rec + TILE - 1) / TILE;
  const K filler = u[0];
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    h[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < STREAM_KPT; ++j) {
      const uint64_t r = t * TILE + threadIdx.x + (uint64_t)j * STREAM_NT;
      if (r < n_rec) {
        K key;
        uint32_t w;
        if (r < 2 * ne) {
          const uint64_t e = r >> 1;
          key = (r & 1) ? v[e] : u[e];
          w = mult[e];
        } else {
          const uint64_t i = (r - 2 * ne) >> 1;
          const uint64_t a = offsets[i], b = offsets[i + 1];
          key = filler;
          w = 0;
          if (b >= a && b - a >= (uint64_t)k) {
            const uint64_t p = ((r - 2 * ne) & 1) ? b - (uint64_t)k : a;
            key = canonical<K>(extract_bases(packed, n_words, p, k, K(0)), k);
            w = 1;
          }
        }
        keys[r] = key;
        wts[r] = w;
        atomicAdd(&h[msd_digit(key, bits, 0)], 1u);
      }
    }
    __syncthreads();
    thist[t * 256 + threadIdx.x] = h[threadIdx.x];
    __syncthreads();
  }
}

// The records as one level-0 bucket of list 0.
__global__ void k_rec_init(Ctl *ctl, Item *items0, uint64_t *hist0) {
  if (ctl->status || ctl->node_path != 1) return;
  hist0[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    items0[0] = Item{0, ctl->n_records, 0, 0u, 0u};
    ctl->items[0] = 1;
  }
}

// ---------------------------------------------------------------------------
// 5. Emit the tables.  Every position marked in the bitmap holds a distinct key
// (buffer 0) and its count (the count array), and marked positions are in key order
// within each read set, so the output row of a marked position is the number of
// marked positions before it.  Tiles of TILE positions (128 bitmap words, one
// per thread).

constexpr int EMIT_NT = (int)(TILE / 32);

// Marked positions per tile: a wave counts EMIT_TPW tiles, two bitmap words per
// lane each, with all their loads in flight at once.
constexpr int EMIT_TPW = 8;
constexpr int EMIT_CNT_NT = 256;
constexpr uint64_t EMIT_CNT_TILES = (uint64_t)EMIT_CNT_NT / 64 * EMIT_TPW;  // per workgroup

__global__ __launch_bounds__(EMIT_CNT_NT) void k_emit_count(const uint32_t *bits,
                                                            uint64_t *tile_cnt, uint64_t n_tiles,
                                                            const Ctl *ctl) {
  static_assert(EMIT_NT == 2 * 64, "two words per lane");
  if (ctl->status) return;
  const uint64_t t0 = (blockIdx.x * (uint64_t)EMIT_CNT_NT + threadIdx.x) / 64 * EMIT_TPW;
  const uint32_t lane = lane_id();
  uint32_t c[EMIT_TPW];
#pragma unroll
  for (int j = 0; j < EMIT_TPW; ++j) {
    c[j] = 0;
    if (t0 + j < n_tiles) {
      const uint2 w = reinterpret_cast<const uint2 *>(bits + (t0 + j) * EMIT_NT)[lane];
      c[j] = (uint32_t)(__popc(w.x) + __popc(w.y));
    }
  }
#pragma unroll
  for (int j = 0; j < EMIT_TPW; ++j) {
    const uint32_t tot = wave_sum(c[j]);
    if (lane == 0 && t0 + j < n_tiles) tile_cnt[t0 + j] = tot;
  }
}

struct OutArgs {
  void *kmer;        // nodes: key per row
  uint32_t *count;   // nodes: count; edges: multiplicity
  void *u, *v;       // edges
  uint8_t *orient;
  void *zkey;        // optional
  uint64_t capacity;
  int k;
};

// One thread per output row: row i of a tile is the i-th marked position.  The
// tile's marked positions are first listed in LDS in order (each thread lists the
// marked bits of one half bitmap word, at its half-word popcount prefix), so
// consecutive threads read consecutive distinct keys and write consecutive rows
// with no staging of the keys themselves.
constexpr int EMIT_WNT = 256;

template <typename K, bool EDGES>
__global__ __launch_bounds__(EMIT_WNT) void k_emit_write(const uint32_t *bits,
                                                         const uint64_t *tile_base, const K *b0,
                                                         const uint32_t *cnts, OutArgs o,
                                                         uint64_t n_tiles, const Ctl *ctl) {
  static_assert(EMIT_WNT == 2 * EMIT_NT, "one thread per half bitmap word");
  __shared__ uint16_t lpos[TILE];  // marked positions of the tile, in order
  __shared__ uint64_t wsum[EMIT_WNT / 64 + 1];
  if (ctl->status) return;
  // tiles holding key positions (the endpoint records of a node table, or the
  // table's keys), each XCD a contiguous eighth
  const uint64_t used = !EDGES && ctl->node_path == 1 ? ctl->n_records : ctl->n_keys;
  const uint64_t nt_used = (used + TILE - 1) / TILE < n_tiles ? (used + TILE - 1) / TILE : n_tiles;
  const uint64_t tile = xcd_tile(blockIdx.x, nt_used);
  if (tile >= nt_used) return;
  const uint64_t w0 = tile * (uint64_t)EMIT_NT;
  const uint32_t word = bits[w0 + (threadIdx.x >> 1)];
  // bit b of word w marks position 32 w + b: even threads take bits 0..15
  uint32_t half = (threadIdx.x & 1) ? word >> 16 : word & 0xffffu;
  uint64_t tot;
  uint32_t e = (uint32_t)block_exclusive_scan<EMIT_WNT>((uint64_t)__popc(half), wsum, &tot);
  const uint32_t p0 = threadIdx.x * 16u;
  while (half) {
    lpos[e++] = (uint16_t)(p0 + (uint32_t)(__ffs(half) - 1));
    half &= half - 1u;
  }
  __syncthreads();
  const uint64_t base = tile_base[tile];
  for (uint32_t i = threadIdx.x; i < (uint32_t)tot; i += EMIT_WNT) {
    const uint64_t pos = (w0 << 5) + lpos[i];
    const uint64_t j = base + i;
    if (j >= o.capacity) break;
    const K key = b0[pos];
    o.count[j] = cnts[pos];
    if (EDGES) {
      K u, v;
      uint32_t orient;
      decode_edge(key, o.k, &u, &v, &orient);
      static_cast<K *>(o.u)[j] = u;
      static_cast<K *>(o.v)[j] = v;
      o.orient[j] = (uint8_t)orient;
      if (o.zkey) static_cast<K *>(o.zkey)[j] = key;
    } else {
      static_cast<K *>(o.kmer)[j] = key;
    }
  }
}

// Row offset of each read set: marked positions before its first key.
__global__ void k_set_rows(const uint32_t *bits, const uint64_t *tile_base,
                           const uint64_t *set_kbase, uint64_t n_sets, uint64_t *set_rows,
                           const Ctl *ctl) {
  if (ctl->status || !set_rows) return;
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s > n_sets) return;
  const uint64_t p = set_kbase[s];
  if (p >= ctl->n_keys) {
    set_rows[s] = ctl->n_unique;
    return;
  }
  const uint64_t t = p / TILE;
  uint64_t r = tile_base[t];
  for (uint64_t wi = t * EMIT_NT; wi < (p >> 5); ++wi) r += (uint64_t)__popc(bits[wi]);
  if (p & 31) r += (uint64_t)__popc(bits[p >> 5] & ((1u << (p & 31)) - 1u));
  set_rows[s] = r;
}

__global__ void k_table_done(Ctl *ctl, int edges, uint64_t capacity) {
  if (threadIdx.x || blockIdx.x) return;
  if (ctl->status) return;
  const uint64_t u = ctl->n_unique;
  if (edges) ctl->n_edges = u;
  else ctl->n_nodes = u;
  if (u > capacity) ctl->capacity_short = 1;
}

__global__ void k_write_result(const Ctl *ctl, dbg_result_t *res) {
  if (threadIdx.x || blockIdx.x) return;
  res->n_nodes = ctl->n_nodes;
  res->n_edges = ctl->n_edges;
  res->status = ctl->status ? ctl->status : (ctl->capacity_short ? (uint32_t)DBG_E_CAPACITY : 0u);
  res->flags = ctl->node_path == 1 ? DBG_FLAG_NODES_FROM_ENDPOINTS : 0u;
}

// ---------------------------------------------------------------------------
// ASCII -> 2-bit packing: one thread per 64-bit word (32 bases).

__global__ void k_pack(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed,
                       dbg_result_t *res) {
  const uint64_t wi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t n_words = (n_bases + 31) / 32;
  if (wi >= n_words) return;
  const uint64_t b0 = wi * 32;
  uint64_t word = 0;
  bool bad = false;
  for (int j = 0; j < 32; ++j) {
    uint32_t code = 0;
    if (b0 + j < n_bases) {
      switch (ascii[b0 + j]) {
        case 'A': case 'a': code = 0; break;
        case 'C': case 'c': code = 1; break;
        case 'G': case 'g': code = 2; break;
        case 'T': case 't': code = 3; break;
        default: bad = true;
      }
    }
    word |= (uint64_t)code << (62 - 2 * j);
  }
  packed[wi] = word;
  if (bad) atomicCAS(&res->status, 0u, (uint32_t)DBG_E_BASE);
}

hipError_t launch_pack(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed,
                       dbg_result_t *result, hipStream_t stream) {
  const uint64_t n_words = (n_bases + 31) / 32;
  if (!n_words) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, stream, ascii,
                     n_bases, packed, result);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-side launch sequence.

static hipEvent_t *g_stage_events = nullptr;

void set_stage_events(hipEvent_t *events) { g_stage_events = events; }

static inline void stage(int idx, hipStream_t st) {
  if (g_stage_events) (void)hipEventRecord(g_stage_events[idx], st);
}

// The LDS bucket sort: 64-bit keys live in the hash table's slots, 128-bit keys
// are hashed by the index of their first occurrence.  One workgroup (512
// threads) or two (256 threads) per CU, persistent over the batch list.
template <typename K, bool W, int V>
static void launch_local_sort(unsigned grid, hipStream_t st, const Batch *batches,
                              const uint64_t *n_batches, K *x0, K *x1, const uint32_t *wt0,
                              const uint32_t *wt1, uint32_t *cnts, uint32_t *bits,
                              const Ctl *ctl, int gate, int bias, int key_bits) {
  if constexpr (sizeof(K) == 8)
    hipLaunchKernelGGL((k_local_sort64<W, V>), dim3(grid), dim3(LocalCfg<K, W, V>::NT), 0, st,
                       batches, n_batches, reinterpret_cast<uint64_t *>(x0),
                       reinterpret_cast<uint64_t *>(x1), wt0, wt1, cnts, bits, ctl, gate, bias,
                       key_bits);
  else
    hipLaunchKernelGGL((k_local_sort<K, W, V>), dim3(grid), dim3(LocalCfg<K, W, V>::NT), 0, st,
                       batches, n_batches, x0, x1, wt0, wt1, cnts, bits, ctl, gate, bias,
                       key_bits, (const SegBatch *)nullptr, (const uint32_t *)nullptr);
}

// The digit ranges of a level's in-tile buckets (128-bit keys).
template <typename K, int V>
static void launch_seg_sort(unsigned grid, hipStream_t st, const SegBatch *segb,
                            const uint64_t *n_seg, const uint32_t *segt, K *x0, K *x1,
                            uint32_t *cnts, uint32_t *bits, const Ctl *ctl, int gate, int bias,
                            int key_bits) {
  static_assert(sizeof(K) == 16, "in-tile buckets: 128-bit keys");
  hipLaunchKernelGGL((k_local_sort<K, false, V, true>), dim3(grid),
                     dim3(LocalCfg<K, false, V>::NT), 0, st, (const Batch *)nullptr, n_seg, x0,
                     x1, (const uint32_t *)nullptr, (const uint32_t *)nullptr, cnts, bits, ctl,
                     gate, bias, key_bits, segb, segt);
}

// A grid rounded up to a multiple of the XCD count.
static inline uint64_t xcd_grid(uint64_t n) {
  return (n + N_XCD - 1) / N_XCD * N_XCD;
}

static inline unsigned grid_for(uint64_t n, uint64_t per, uint64_t cap) {
  uint64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

template <typename K>
static hipError_t run_table(const BuildArgs &A, const Layout &L, bool edges) {
  char *ws = static_cast<char *>(A.workspace);
  Ctl *ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
  uint64_t *set_read_off = A.set_read_offsets
                               ? const_cast<uint64_t *>(A.set_read_offsets)
                               : reinterpret_cast<uint64_t *>(ws + L.set_read_off);
  uint64_t *rbase = reinterpret_cast<uint64_t *>(ws + L.rbase);
  uint64_t *block_sums = reinterpret_cast<uint64_t *>(ws + L.block_sums);
  uint64_t *set_kbase = reinterpret_cast<uint64_t *>(ws + L.set_kbase);
  uint64_t *set_tbase = reinterpret_cast<uint64_t *>(ws + L.set_tbase);
  TileDesc *tiles = reinterpret_cast<TileDesc *>(ws + L.tiles);
  uint32_t *thist = reinterpret_cast<uint32_t *>(ws + L.thist);
  uint32_t *csum = reinterpret_cast<uint32_t *>(ws + L.csum);
  uint64_t *cursor0 = reinterpret_cast<uint64_t *>(ws + L.cursor0);
  Item *items[2] = {reinterpret_cast<Item *>(ws + L.items[0]),
                    reinterpret_cast<Item *>(ws + L.items[1])};
  uint64_t *hist[2] = {reinterpret_cast<uint64_t *>(ws + L.hist[0]),
                       reinterpret_cast<uint64_t *>(ws + L.hist[1])};
  uint64_t *cursor = reinterpret_cast<uint64_t *>(ws + L.cursor);
  Batch *batches = reinterpret_cast<Batch *>(ws + L.batches);
  Item *uniform = reinterpret_cast<Item *>(ws + L.uniform);
  uint64_t *rle_heads = reinterpret_cast<uint64_t *>(ws + L.rle_heads);
  K *x0 = reinterpret_cast<K *>(ws + L.keys[0]);
  K *x1 = reinterpret_cast<K *>(ws + L.keys[1]);
  uint32_t *runbits = reinterpret_cast<uint32_t *>(ws + L.bits);
  uint32_t *cnts = reinterpret_cast<uint32_t *>(ws + L.counts);
  uint32_t *titem = reinterpret_cast<uint32_t *>(ws + L.titem);
  const uint64_t titem_cap = L.max_tiles + L.item_cap;
  uint32_t *wt0 = reinterpret_cast<uint32_t *>(ws + L.keys[0] + L.weights);
  uint32_t *wt1 = reinterpret_cast<uint32_t *>(ws + L.keys[1] + L.weights);
  hipStream_t st = A.stream;
  const uint64_t S = A.n_sets;
  const int len = edges ? A.k + 1 : A.k;
  const int bits = 2 * len;
  const int ev = edges ? 0 : DBG_STAGE_EVENTS / 2;
  // The node table of a single-set build may be built from the edge endpoints
  // instead of the k-mers; the device picks the route (k_node_path) and the
  // kernels of the other route return at once.  g0 gates the k-mer route.
  const bool sliced = A.pfx_lo != 0 || A.pfx_hi != PFX_BINS;
  const bool two_routes = !edges && S == 1 && A.tuning.node_path != DBG_NODES_KMERS && !sliced;
  const int g0 = two_routes ? 0 : -1;
  const uint64_t n_words = (A.n_bases + 31) / 32;
  // workgroup shape of the LDS bucket sort, and the batch capacity it plans for
  const int lv = A.tuning.local_variant;
  const uint64_t cap_u = lv == 1 ? local_cap<K, false, 1>() : local_cap<K, false, 0>();
  const uint64_t cap_w = lv == 1 ? local_cap<K, true, 1>() : local_cap<K, true, 0>();

  stage(ev + 0, st);
  hipLaunchKernelGGL(k_table_reset, dim3(1), dim3(1), 0, st, ctl);
  hipLaunchKernelGGL(k_read_reduce, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, A.n_bases, len, block_sums, ctl);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, block_sums, L.read_blocks,
                     (uint64_t *)nullptr);
  hipLaunchKernelGGL(k_read_apply, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, len, block_sums, rbase, ctl);
  hipLaunchKernelGGL(k_set_setup, dim3(1), dim3(1024), 0, st, rbase, A.n_reads, set_read_off, S,
                     A.max_positions, set_kbase, set_tbase, ctl);
  hipLaunchKernelGGL(k_tile_map, dim3(grid_for(L.max_tiles, 256, 1u << 30)), dim3(256), 0, st,
                     rbase, A.read_offsets, set_read_off, S, set_kbase, set_tbase, tiles,
                     L.max_tiles, ctl);
  if (two_routes)
    hipLaunchKernelGGL(k_node_path, dim3(1), dim3(1), 0, st, ctl, A.n_reads, S,
                       A.tuning.node_path, A.tuning.endpoint_ratio,
                       (uint64_t)(A.max_keys + 2) * (uint64_t)L.key_bytes, (uint64_t)L.weights,
                       L.key_bytes);
  stage(ev + 1, st);
  EnumArgs ea{A.packed, n_words, A.read_offsets, rbase, tiles, len, bits, g0, A.pfx_lo,
              A.pfx_hi};
  if (sliced)
    hipLaunchKernelGGL((k_enum_hist<K, true>), dim3((unsigned)L.max_tiles), dim3(STREAM_NT), 0, st,
                       ea, thist, ctl);
  else
    hipLaunchKernelGGL((k_enum_hist<K, false>), dim3((unsigned)L.max_tiles), dim3(STREAM_NT), 0,
                       st, ea, thist, ctl);
  stage(ev + 2, st);
  if (two_routes) {
    const K *eu = static_cast<const K *>(A.edges.u);
    const uint64_t rec_tiles = (2 * A.edges.capacity + 2 * A.n_reads + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_records<K>, dim3(grid_for(rec_tiles, 1, 8192)), dim3(STREAM_NT), 0, st,
                       eu, static_cast<const K *>(A.edges.v), A.edges.mult, A.packed, n_words,
                       A.read_offsets, A.k, bits, x0, wt0, thist, ctl);
  }
  const unsigned col_chunks = (unsigned)((L.max_tiles + COL_CHUNK - 1) / COL_CHUNK);
  hipLaunchKernelGGL(k_col_reduce, dim3(col_chunks), dim3(256), 0, st, thist, csum,
                     &ctl->n_tiles, ctl, g0);
  hipLaunchKernelGGL(k_col_scan, dim3(256), dim3(256), 0, st, csum, &ctl->n_tiles, ctl, g0);
  hipLaunchKernelGGL(k_col_apply, dim3(col_chunks), dim3(256), 0, st, thist, csum,
                     &ctl->n_tiles, ctl, g0);
  hipLaunchKernelGGL(k_kept_keys, dim3(1), dim3(256), 0, st, thist, A.max_keys, ctl, g0);
  // column prefix of the per-tile digit counts of a level in tile mode
  const unsigned lcol_chunks =
      (unsigned)((L.max_tiles + L.item_cap + COL_CHUNK - 1) / COL_CHUNK);
  auto level_prefix = [&](const uint64_t *n_tiles_p, int gate) {
    hipLaunchKernelGGL(k_col_reduce, dim3(lcol_chunks), dim3(256), 0, st, thist, csum, n_tiles_p,
                       ctl, gate);
    hipLaunchKernelGGL(k_col_scan, dim3(256), dim3(256), 0, st, csum, n_tiles_p, ctl, gate);
    hipLaunchKernelGGL(k_col_apply, dim3(lcol_chunks), dim3(256), 0, st, thist, csum, n_tiles_p,
                       ctl, gate);
  };
  // The in-tile level (128-bit keys): the first level whose buckets average at
  // most a quarter of SEG_TILES tiles per read set; its buckets of at most
  // SEG_TILES tiles are split within their tiles, and their digit ranges are
  // sorted right after it (before a later level can write buffer 1).
  int seg_level = -1;
  if (sizeof(K) == 16 && A.tuning.in_tile) {
    const uint64_t per_set = (A.max_keys + S - 1) / S;
    seg_level = 1;
    for (uint64_t b = per_set >> 8; b > (uint64_t)SEG_TILES * TILE / 4; b >>= 8) ++seg_level;
  }
  SegBatch *segb = reinterpret_cast<SegBatch *>(ws + L.segb);
  uint32_t *segt = reinterpret_cast<uint32_t *>(ws + L.segt);
  uint64_t *kw0 = reinterpret_cast<uint64_t *>(x0), *kw1 = reinterpret_cast<uint64_t *>(x1);
  const int key_words = (int)(sizeof(K) / 8);
  PlanArgs pa{items[1], &ctl->items[1], hist[1], L.item_cap, batches, L.batch_cap,
              uniform, L.item_cap, ctl, cap_u, bits, g0, seg_level == 1 ? 1 : 0, segb, segt, L.seg_cap,
              kw0, kw1, key_words, thist};
  hipLaunchKernelGGL(k_set_plan, dim3(grid_for(S, 1, 4096)), dim3(STREAM_NT), 0, st, pa, thist,
                     set_tbase, cursor0, set_kbase, S);
  // persistent level grids.  With 128-bit keys the scatter holds two workgroups
  // per CU, and a grid of just that many (512) measured fastest: each XCD's
  // workgroups then work on one window of neighbouring tiles, whose runs of a
  // digit meet in its L2 (40M-read k = 63 build at quarter size: levels 16.05
  // ms per table at 8,192 workgroups, 15.68 at 2,048, 15.33 at 512, 16.8 at 256,
  // which leaves half the CU's slots empty); the in-tile pass is indifferent.
  // With 64-bit keys 8,192 measured faster than 2,048 and 1,024.
  const unsigned level_grid =
      (unsigned)xcd_grid(grid_for(L.max_tiles + L.item_cap, 1, sizeof(K) == 16 ? 512 : 8192));
  const unsigned tiles_grid = (unsigned)xcd_grid(grid_for(L.max_tiles + L.item_cap, 1, 8192));
  // endpoint route: the records are one bucket at level 0 (list 0 -> list 1)
  LevelArgs la0{items[0], &ctl->items[0], &ctl->level_tiles[0], &ctl->level_scatter_tiles[0],
                hist[0], thist, cursor, wt0, wt1, titem, thist, bits, 0, 1};
  const unsigned plan_grid = grid_for(L.item_cap, 1, 8192);
  if (two_routes) {
    hipLaunchKernelGGL(k_rec_init, dim3(1), dim3(256), 0, st, ctl, items[0], hist[0]);
    hipLaunchKernelGGL(k_level_prep, dim3(1), dim3(1024), 0, st, items[0], &ctl->items[0],
                       &ctl->level_tiles[0], &ctl->level_scatter_tiles[0], &ctl->items[1], ctl, 1);
    hipLaunchKernelGGL(k_level_tilemap, dim3(plan_grid), dim3(256), 0, st, items[0],
                       &ctl->items[0], &ctl->level_tiles[0], titem, titem_cap, ctl, 1);
    // (the records' tile rows were written by k_records)
    level_prefix(&ctl->level_tiles[0], 1);
    PlanArgs pw{items[1], &ctl->items[1], hist[1], L.item_cap, batches, L.batch_cap,
                uniform, L.item_cap, ctl, cap_w, bits, 1, 0, segb, segt, L.seg_cap,
                kw0, kw1, key_words, thist};
    hipLaunchKernelGGL(k_level_plan, dim3(plan_grid), dim3(STREAM_NT), 0, st, pw, la0);
  }
  stage(ev + 3, st);
  if (sliced)
    hipLaunchKernelGGL((k_enum_scatter<K, true>), dim3((unsigned)xcd_grid(L.max_tiles)), dim3(STREAM_NT), 0,
                       st, ea, cursor0, thist, x0, ctl);
  else
    hipLaunchKernelGGL((k_enum_scatter<K, false>), dim3((unsigned)xcd_grid(L.max_tiles)), dim3(STREAM_NT), 0,
                       st, ea, cursor0, thist, x0, ctl);
  if (two_routes)
    hipLaunchKernelGGL((k_level_scatter<K, true>), dim3(level_grid), dim3(STREAM_NT), 0, st, la0,
                       x0, x1, ctl);
  stage(ev + 4, st);
  // the run bitmap starts clear (the digit ranges of the in-tile level mark it
  // inside the level loop)
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(L.rle_tiles * (TILE / 64), 256, 8192)), dim3(256), 0,
                     st, reinterpret_cast<uint64_t *>(runbits), L.rle_tiles * (TILE / 64), 0ull);
  const int bias = A.tuning.lds_digit_bias;
  bool seg_done = false;
  for (int lev = 1; bits - 8 * lev > 0; ++lev) {
    const int li = lev & 1;
    hipLaunchKernelGGL(k_level_prep, dim3(1), dim3(1024), 0, st, items[li], &ctl->items[li],
                       &ctl->level_tiles[li], &ctl->level_scatter_tiles[li], &ctl->items[li ^ 1],
                       ctl, -1);
    hipLaunchKernelGGL(k_level_tilemap, dim3(plan_grid), dim3(256), 0, st, items[li],
                       &ctl->items[li], &ctl->level_tiles[li], titem, titem_cap, ctl, -1);
    // levels >= 1 split many buckets at once (at least one per set and top
    // digit), so their atomics spread over many counters: atomic mode
    LevelArgs la{items[li], &ctl->items[li], &ctl->level_tiles[li],
                 &ctl->level_scatter_tiles[li], hist[li], nullptr, cursor, wt0, wt1, titem, thist,
                 bits, lev, -1};
    hipLaunchKernelGGL(k_level_hist<K>, dim3(level_grid), dim3(STREAM_NT), 0, st, la, x0, x1, ctl);
    if (lev == seg_level)
      hipLaunchKernelGGL(k_level_tiles<K>, dim3(tiles_grid), dim3(tiles_nt<K>()), 0, st, la, x0,
                         x1, ctl);
    PlanArgs pl{items[li ^ 1], &ctl->items[li ^ 1], hist[li ^ 1], L.item_cap, batches,
                L.batch_cap, uniform, L.item_cap, ctl, cap_u, bits, g0,
                lev + 1 == seg_level ? 1 : 0, segb, segt, L.seg_cap, kw0, kw1, key_words, thist};
    hipLaunchKernelGGL(k_level_plan, dim3(plan_grid), dim3(STREAM_NT), 0, st, pl, la);
    if (two_routes) {
      PlanArgs pw = pl;
      pw.local_cap = cap_w;
      pw.gate = 1;
      pw.in_tile_ok = 0;
      hipLaunchKernelGGL(k_level_plan, dim3(plan_grid), dim3(STREAM_NT), 0, st, pw, la);
    }
    la.gate = g0;
    hipLaunchKernelGGL((k_level_scatter<K, false>), dim3(level_grid), dim3(STREAM_NT), 0, st, la,
                       x0, x1, ctl);
    if (two_routes) {
      la.gate = 1;
      hipLaunchKernelGGL((k_level_scatter<K, true>), dim3(level_grid), dim3(STREAM_NT), 0, st, la,
                         x0, x1, ctl);
    }
    if (lev == seg_level) {
      stage(ev + 5, st);
      if constexpr (sizeof(K) == 16) {
        if (lv == 0)
          launch_seg_sort<K, 0>(256, st, segb, &ctl->n_seg, segt, x0, x1, cnts, runbits, ctl,
                                g0, bias, bits);
        else if (lv == 1)
          launch_seg_sort<K, 1>(512, st, segb, &ctl->n_seg, segt, x0, x1, cnts, runbits, ctl,
                                g0, bias, bits);
        else
          launch_seg_sort<K, 2>(256, st, segb, &ctl->n_seg, segt, x0, x1, cnts, runbits, ctl,
                                g0, bias, bits);
      }
      stage(ev + 6, st);
      seg_done = true;
    }
  }
  if (!seg_done) {
    stage(ev + 5, st);
    stage(ev + 6, st);
  }
  stage(ev + 7, st);
  if (lv == 0) {
    launch_local_sort<K, false, 0>(256, st, batches, &ctl->n_batches, x0, x1, wt0, wt1, cnts,
                                   runbits, ctl, g0, bias, bits);
    if (two_routes)
      launch_local_sort<K, true, 0>(256, st, batches, &ctl->n_batches, x0, x1, wt0, wt1,
                                    cnts, runbits, ctl, 1, bias, bits);
  } else if (lv == 1) {
    launch_local_sort<K, false, 1>(512, st, batches, &ctl->n_batches, x0, x1, wt0, wt1, cnts,
                                   runbits, ctl, g0, bias, bits);
    if (two_routes)
      launch_local_sort<K, true, 1>(512, st, batches, &ctl->n_batches, x0, x1, wt0, wt1,
                                    cnts, runbits, ctl, 1, bias, bits);
  } else {
    launch_local_sort<K, false, 2>(256, st, batches, &ctl->n_batches, x0, x1, wt0, wt1, cnts,
                                   runbits, ctl, g0, bias, bits);
    if (two_routes)
      launch_local_sort<K, true, 2>(256, st, batches, &ctl->n_batches, x0, x1, wt0, wt1,
                                    cnts, runbits, ctl, 1, bias, bits);
  }
  stage(ev + 8, st);
  hipLaunchKernelGGL(k_uniform_emit<K>, dim3(64), dim3(256), 0, st, uniform, &ctl->n_uniform, x0,
                     x1, cnts, runbits, ctl, g0);
  if (two_routes)
    hipLaunchKernelGGL(k_uniform_emit_w<K>, dim3(64), dim3(256), 0, st, uniform, &ctl->n_uniform,
                       x0, x1, wt0, wt1, cnts, runbits, ctl, 1);
  hipLaunchKernelGGL(k_emit_count,
                     dim3((unsigned)((L.rle_tiles + EMIT_CNT_TILES - 1) / EMIT_CNT_TILES)),
                     dim3(EMIT_CNT_NT), 0, st, runbits, rle_heads, L.rle_tiles, ctl);
  {
    const uint64_t nch = (L.rle_tiles + SCAN_TILE - 1) / SCAN_TILE;
    uint64_t *rle_sums = reinterpret_cast<uint64_t *>(ws + L.rle_sums);
    hipLaunchKernelGGL(k_chunk_reduce, dim3((unsigned)nch), dim3(SCAN_NT), 0, st, rle_heads,
                       L.rle_tiles, rle_sums);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, rle_sums, nch, &ctl->n_unique);
    hipLaunchKernelGGL(k_chunk_apply, dim3((unsigned)nch), dim3(SCAN_NT), 0, st, rle_heads,
                       L.rle_tiles, rle_sums);
  }
  stage(ev + 9, st);
  OutArgs oa{};
  oa.k = A.k;
  uint64_t capacity;
  uint64_t *set_rows;
  if (edges) {
    oa.u = A.edges.u;
    oa.v = A.edges.v;
    oa.orient = A.edges.orient;
    oa.zkey = A.edges.zkey;
    oa.count = A.edges.mult;
    oa.capacity = capacity = A.edges.capacity;
    set_rows = A.edge_set_offsets;
    hipLaunchKernelGGL((k_emit_write<K, true>), dim3((unsigned)xcd_grid(L.rle_tiles)),
                       dim3(EMIT_WNT), 0, st, runbits, rle_heads, x0, cnts, oa, L.rle_tiles, ctl);
  } else {
    oa.kmer = A.nodes.kmer;
    oa.count = A.nodes.count;
    oa.capacity = capacity = A.nodes.capacity;
    set_rows = A.node_set_offsets;
    hipLaunchKernelGGL((k_emit_write<K, false>), dim3((unsigned)xcd_grid(L.rle_tiles)),
                       dim3(EMIT_WNT), 0, st, runbits, rle_heads, x0, cnts, oa, L.rle_tiles, ctl);
  }
  stage(ev + 10, st);
  hipLaunchKernelGGL(k_set_rows, dim3(grid_for(S + 1, 256, 1u << 30)), dim3(256), 0, st, runbits,
                     rle_heads, set_kbase, S, set_rows, ctl);
  hipLaunchKernelGGL(k_table_done, dim3(1), dim3(1), 0, st, ctl, edges ? 1 : 0, capacity);
  stage(ev + 11, st);
  return hipGetLastError();
}

template <typename K>
static hipError_t run_build(const BuildArgs &A, const Layout &L) {
  char *ws = static_cast<char *>(A.workspace);
  Ctl *ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
  hipLaunchKernelGGL(k_init, dim3(1), dim3(1), 0, A.stream, ctl,
                     reinterpret_cast<uint64_t *>(ws + L.set_read_off), A.n_reads,
                     A.set_read_offsets ? 0 : 1);
  hipError_t e = run_table<K>(A, L, true);
  if (e == hipSuccess) e = run_table<K>(A, L, false);
  hipLaunchKernelGGL(k_write_result, dim3(1), dim3(1), 0, A.stream, ctl, A.result);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

// Key offsets and tiles of one key length, then the prefix counts of its keys.
template <typename K>
static hipError_t run_prefix(const BuildArgs &A, const Layout &L, int len, uint64_t *counts) {
  char *ws = static_cast<char *>(A.workspace);
  Ctl *ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
  uint64_t *set_read_off = reinterpret_cast<uint64_t *>(ws + L.set_read_off);
  uint64_t *rbase = reinterpret_cast<uint64_t *>(ws + L.rbase);
  uint64_t *block_sums = reinterpret_cast<uint64_t *>(ws + L.block_sums);
  uint64_t *set_kbase = reinterpret_cast<uint64_t *>(ws + L.set_kbase);
  uint64_t *set_tbase = reinterpret_cast<uint64_t *>(ws + L.set_tbase);
  TileDesc *tiles = reinterpret_cast<TileDesc *>(ws + L.tiles);
  hipStream_t st = A.stream;
  hipLaunchKernelGGL(k_table_reset, dim3(1), dim3(1), 0, st, ctl);
  hipLaunchKernelGGL(k_read_reduce, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, A.n_bases, len, block_sums, ctl);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, block_sums, L.read_blocks,
                     (uint64_t *)nullptr);
  hipLaunchKernelGGL(k_read_apply, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, len, block_sums, rbase, ctl);
  hipLaunchKernelGGL(k_set_setup, dim3(1), dim3(1024), 0, st, rbase, A.n_reads, set_read_off,
                     (uint64_t)1, A.max_positions, set_kbase, set_tbase, ctl);
  hipLaunchKernelGGL(k_tile_map, dim3(grid_for(L.max_tiles, 256, 1u << 30)), dim3(256), 0, st,
                     rbase, A.read_offsets, set_read_off, (uint64_t)1, set_kbase, set_tbase,
                     tiles, L.max_tiles, ctl);
  hipLaunchKernelGGL(k_fill_u64, dim3(16), dim3(256), 0, st, counts, (uint64_t)PFX_BINS, 0ull);
  EnumArgs ea{A.packed, (A.n_bases + 31) / 32, A.read_offsets, rbase, tiles, len, 2 * len, -1,
              0u, PFX_BINS};
  hipLaunchKernelGGL(k_prefix_hist<K>, dim3(grid_for(L.max_tiles, 1, 2048)), dim3(STREAM_NT), 0,
                     st, ea, counts, ctl);
  return hipGetLastError();
}

hipError_t run_prefix_counts(const BuildArgs &A, const Layout &L, uint64_t *edge_counts,
                             uint64_t *node_counts) {
  char *ws = static_cast<char *>(A.workspace);
  Ctl *ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
  hipLaunchKernelGGL(k_init, dim3(1), dim3(1), 0, A.stream, ctl,
                     reinterpret_cast<uint64_t *>(ws + L.set_read_off), A.n_reads, 1);
  hipError_t e = A.k <= 31 ? run_prefix<uint64_t>(A, L, A.k + 1, edge_counts)
                           : run_prefix<u128>(A, L, A.k + 1, edge_counts);
  if (e == hipSuccess)
    e = A.k <= 31 ? run_prefix<uint64_t>(A, L, A.k, node_counts)
                  : run_prefix<u128>(A, L, A.k, node_counts);
  hipLaunchKernelGGL(k_write_result, dim3(1), dim3(1), 0, A.stream, ctl, A.result);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

hipError_t run_build_u64(const BuildArgs &a, const Layout &L) { return run_build<uint64_t>(a, L); }
hipError_t run_build_u128(const BuildArgs &a, const Layout &L) { return run_build<u128>(a, L); }

}  // namespace dbg
