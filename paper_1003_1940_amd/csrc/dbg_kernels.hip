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
#include "dbg_device.h"
#include "dbg_internal.h"

namespace dbg {

// ---------------------------------------------------------------------------
// Small helpers.

__device__ __forceinline__ void set_status(Ctl *ctl, uint32_t code) {
  atomicCAS(&ctl->status, 0u, code);
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
    ctl->n_batches = 0;
    ctl->n_uniform = 0;
    ctl->n_unique = 0;
  }
}

__global__ void k_fill_u64(uint64_t *a, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------
// 1. Per-read key counts c_i = max(0, L_i - len + 1) and their prefix rbase.

constexpr int SCAN_NT = 256, SCAN_PT = 16;
constexpr uint64_t SCAN_TILE = (uint64_t)SCAN_NT * SCAN_PT;

__device__ __forceinline__ uint64_t read_key_count(const uint64_t *off, uint64_t i, int len,
                                                   Ctl *ctl) {
  const uint64_t a = off[i], b = off[i + 1];
  if (b < a) {
    set_status(ctl, DBG_E_OFFSETS);
    return 0;
  }
  const uint64_t L = b - a;
  return L + 1 > (uint64_t)len ? L + 1 - (uint64_t)len : 0;
}

__global__ __launch_bounds__(SCAN_NT) void k_read_reduce(const uint64_t *off, uint64_t n_reads,
                                                         uint64_t n_bases, int len,
                                                         uint64_t *block_sums, Ctl *ctl) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * (uint64_t)SCAN_PT;
  uint64_t s = 0;
  for (int r = 0; r < SCAN_PT; ++r)
    if (base + r < n_reads) s += read_key_count(off, base + r, len, ctl);
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

__global__ __launch_bounds__(SCAN_NT) void k_read_apply(const uint64_t *off, uint64_t n_reads,
                                                        int len, const uint64_t *block_sums,
                                                        uint64_t *rbase, Ctl *ctl) {
  __shared__ uint64_t wsum[SCAN_NT / 64 + 1];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * (uint64_t)SCAN_PT;
  uint64_t c[SCAN_PT], s = 0;
  for (int r = 0; r < SCAN_PT; ++r) {
    c[r] = base + r < n_reads ? read_key_count(off, base + r, len, ctl) : 0;
    s += c[r];
  }
  uint64_t total;
  uint64_t ex = block_exclusive_scan<SCAN_NT>(s, wsum, &total) + block_sums[blockIdx.x];
  for (int r = 0; r < SCAN_PT; ++r) {
    if (base + r <= n_reads) rbase[base + r] = ex;  // rbase[n_reads] = total keys
    ex += c[r];
  }
}

// Per-set key ranges and enumeration tiles.  One workgroup.
__global__ __launch_bounds__(1024) void k_set_setup(const uint64_t *rbase, uint64_t n_reads,
                                                    const uint64_t *set_read_off, uint64_t n_sets,
                                                    uint64_t max_keys, uint64_t *set_kbase,
                                                    uint64_t *set_tbase, Ctl *ctl) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  if (ctl->status) return;
  if (threadIdx.x == 0) {
    const uint64_t nk = rbase[n_reads];
    ctl->n_keys = nk;
    if (nk > max_keys) set_status(ctl, DBG_E_OVERFLOW);
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

// Tile -> (set, read whose key range contains the tile's first key).
__global__ void k_tile_map(const uint64_t *rbase, const uint64_t *set_read_off, uint64_t n_sets,
                           const uint64_t *set_kbase, const uint64_t *set_tbase,
                           uint64_t *tile_read, uint32_t *tile_set, uint64_t max_tiles, Ctl *ctl) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (ctl->status || t >= ctl->n_tiles) return;
  if (t >= max_tiles) {
    set_status(ctl, DBG_E_INTERNAL);
    return;
  }
  const uint64_t s = upper_bound(set_tbase, 0, n_sets + 1, t) - 1;
  const uint64_t g = set_kbase[s] + (t - set_tbase[s]) * TILE;
  const uint64_t r0 = set_read_off[s], r1 = set_read_off[s + 1];
  tile_read[t] = upper_bound(rbase, r0, r1 + 1, g) - 1;
  tile_set[t] = (uint32_t)s;
}

// ---------------------------------------------------------------------------
// 2. Enumeration.

struct EnumArgs {
  const uint64_t *packed;
  uint64_t n_words;
  const uint64_t *offsets;
  const uint64_t *rbase;
  const uint64_t *set_read_off;
  const uint64_t *set_kbase;
  const uint64_t *set_tbase;
  const uint64_t *tile_read;
  const uint32_t *tile_set;
  int len;   // bases per key
  int bits;  // 2 * len
};

struct TileRange {
  uint64_t start, end, read_lo, read_hi;
  uint32_t set;
};

__device__ __forceinline__ TileRange enum_tile(const EnumArgs &a, uint64_t t) {
  TileRange r;
  const uint32_t s = a.tile_set[t];
  r.set = s;
  r.start = a.set_kbase[s] + (t - a.set_tbase[s]) * TILE;
  const uint64_t se = a.set_kbase[s + 1];
  r.end = r.start + TILE < se ? r.start + TILE : se;
  r.read_lo = a.tile_read[t];
  r.read_hi = (t + 1 < a.set_tbase[s + 1]) ? a.tile_read[t + 1] + 1 : a.set_read_off[s + 1];
  return r;
}

// Keys g0, g0+1, ... (< g_end, at most KPT) into out[]: the canonical key at each
// position, rolling the forward and reverse-complement registers by one base
// within a read and re-seeding them at each read start.  Returns the count.
template <typename K, int KPT>
__device__ __forceinline__ int enum_keys(const EnumArgs &a, uint64_t g0, uint64_t g_end,
                                         uint64_t read_lo, uint64_t read_hi, K (&out)[KPT]) {
  if (g0 >= g_end) return 0;
  uint64_t i = upper_bound(a.rbase, read_lo, read_hi + 1, g0) - 1;  // rbase[i] <= g0 < rbase[i+1]
  uint64_t next = a.rbase[i + 1];
  uint64_t p = a.offsets[i] + (g0 - a.rbase[i]);
  const int len = a.len;
  const K mask = low_mask<K>(2 * len);
  const int top = 2 * len - 2;
  K fw = extract_bases(a.packed, a.n_words, p, len, K());
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
            next = a.rbase[i + 1];
          } while (next == g);
          p = a.offsets[i];
          fw = extract_bases(a.packed, a.n_words, p, len, K());
          rc = revcomp(fw, len);
        } else {
          const uint32_t c = base_at(a.packed, p + len);
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

template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_enum_hist(EnumArgs a, uint64_t *hist0,
                                                         const Ctl *ctl) {
  __shared__ uint32_t h[256];
  const uint64_t t = blockIdx.x;
  if (ctl->status || t >= ctl->n_tiles) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const TileRange tr = enum_tile(a, t);
  K keys[STREAM_KPT];
  const int n = enum_keys<K, STREAM_KPT>(a, tr.start + threadIdx.x * (uint64_t)STREAM_KPT, tr.end,
                                         tr.read_lo, tr.read_hi, keys);
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r)
    if (r < n) atomicAdd(&h[msd_digit(keys[r], a.bits, 0)], 1u);
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  if (c)
    atomicAdd((unsigned long long *)&hist0[(uint64_t)tr.set * 256 + threadIdx.x],
              (unsigned long long)c);
}

// LDS-staged partition of one tile of keys (held in registers) by the digit
// msd_digit(key, bits, level): count per digit, reserve a range per digit in the
// destination buckets with one global atomic per digit, place keys
// digit-contiguously in LDS, then write each digit run with consecutive threads
// on consecutive addresses.  `cursor` points at the 256 bucket cursors of the
// parent.  Every thread of the workgroup must call it.
template <typename K>
struct PartLds {
  K keys[TILE];
  uint64_t gbase[256];
  uint32_t cnt[256];
  uint64_t wsum[STREAM_NT / 64 + 1];
};

template <typename K>
__device__ __forceinline__ void partition_tile(const K (&keys)[STREAM_KPT], int n, int bits,
                                               int level, uint64_t *cursor, K *dst,
                                               PartLds<K> &s) {
  const uint32_t tid = threadIdx.x;
  uint32_t dig[STREAM_KPT];
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r) dig[r] = r < n ? msd_digit(keys[r], bits, level) : 0u;
  s.cnt[tid] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r)
    if (r < n) atomicAdd(&s.cnt[dig[r]], 1u);
  __syncthreads();
  const uint64_t c = s.cnt[tid];
  uint64_t m;
  const uint64_t ex = block_exclusive_scan<STREAM_NT>(c, s.wsum, &m);
  s.gbase[tid] =
      c ? (uint64_t)atomicAdd((unsigned long long *)&cursor[tid], (unsigned long long)c) - ex : 0;
  s.cnt[tid] = (uint32_t)ex;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r)
    if (r < n) s.keys[atomicAdd(&s.cnt[dig[r]], 1u)] = keys[r];
  __syncthreads();
  for (uint32_t idx = tid; idx < (uint32_t)m; idx += STREAM_NT) {
    const K key = s.keys[idx];
    dst[s.gbase[msd_digit(key, bits, level)] + idx] = key;
  }
  __syncthreads();
}

template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_enum_scatter(EnumArgs a, uint64_t *cursor0, K *dst,
                                                            const Ctl *ctl) {
  __shared__ PartLds<K> s;
  const uint64_t t = blockIdx.x;
  if (ctl->status || t >= ctl->n_tiles) return;
  const TileRange tr = enum_tile(a, t);
  K keys[STREAM_KPT];
  const int n = enum_keys<K, STREAM_KPT>(a, tr.start + threadIdx.x * (uint64_t)STREAM_KPT, tr.end,
                                         tr.read_lo, tr.read_hi, keys);
  partition_tile<K>(keys, n, a.bits, 0, cursor0 + (uint64_t)tr.set * 256, dst, s);
}

// ---------------------------------------------------------------------------
// Bucket planning: after a parent's 256 sub-buckets are counted, scan the counts
// into cursors and sort each sub-bucket into one of three lists: small ones are
// grouped (consecutive, up to the LDS capacity) into batches for the LDS sort;
// oversized ones go to the next partition level, or, when no digit is left (all
// their keys are equal), to the uniform list.

struct PlanArgs {
  Item *next_items;       // list receiving oversized buckets
  uint64_t *next_count;   // its counter in Ctl
  uint64_t *next_hist;    // histogram rows of that list (zeroed here)
  uint64_t item_cap;
  Batch *batches;
  uint64_t batch_cap;
  Item *uniform;
  uint64_t uniform_cap;
  Ctl *ctl;
  uint64_t local_cap;
  int bits;
};

// Called by the whole workgroup (256 threads): counts[d] of the parent whose keys
// start at `off`; children live in buffer `src`; `child_level` is the digit level
// that would split a child.
__device__ void plan_children(const PlanArgs &p, const uint64_t *counts, uint64_t off,
                              uint32_t src, int child_level, uint64_t *cursor,
                              uint64_t *s_start, uint64_t *wsum) {
  const uint32_t tid = threadIdx.x;
  const uint64_t c = counts[tid];
  uint64_t total;
  const uint64_t ex = block_exclusive_scan<STREAM_NT>(c, wsum, &total);
  cursor[tid] = off + ex;
  s_start[tid] = ex;
  __syncthreads();
  if (tid == 0) {
    const bool digits_left = p.bits - 8 * child_level > 0;
    uint64_t b_off = 0, b_size = 0;
    for (int d = 0; d < 256; ++d) {
      const uint64_t sz = counts[d];
      if (sz == 0) continue;
      const uint64_t o = off + s_start[d];
      if (sz > p.local_cap) {
        if (b_size) {
          const uint64_t bi = atomicAdd((unsigned long long *)&p.ctl->n_batches, 1ull);
          if (bi < p.batch_cap) p.batches[bi] = Batch{b_off, (uint32_t)b_size, src};
          else set_status(p.ctl, DBG_E_INTERNAL);
          b_size = 0;
        }
        if (digits_left) {
          const uint64_t ii = atomicAdd((unsigned long long *)p.next_count, 1ull);
          if (ii < p.item_cap) {
            p.next_items[ii] = Item{o, sz, 0, src, 0};
            for (int j = 0; j < 256; ++j) p.next_hist[ii * 256 + j] = 0;
          } else {
            set_status(p.ctl, DBG_E_INTERNAL);
          }
        } else {
          const uint64_t ui = atomicAdd((unsigned long long *)&p.ctl->n_uniform, 1ull);
          if (ui < p.uniform_cap) p.uniform[ui] = Item{o, sz, 0, src, 0};
          else set_status(p.ctl, DBG_E_INTERNAL);
        }
      } else {
        if (b_size + sz > p.local_cap) {
          const uint64_t bi = atomicAdd((unsigned long long *)&p.ctl->n_batches, 1ull);
          if (bi < p.batch_cap) p.batches[bi] = Batch{b_off, (uint32_t)b_size, src};
          else set_status(p.ctl, DBG_E_INTERNAL);
          b_size = 0;
        }
        if (b_size == 0) b_off = o;
        b_size += sz;
      }
    }
    if (b_size) {
      const uint64_t bi = atomicAdd((unsigned long long *)&p.ctl->n_batches, 1ull);
      if (bi < p.batch_cap) p.batches[bi] = Batch{b_off, (uint32_t)b_size, src};
      else set_status(p.ctl, DBG_E_INTERNAL);
    }
  }
  __syncthreads();
}

// One workgroup per read set: plan the children of the level-0 partition.
__global__ __launch_bounds__(STREAM_NT) void k_set_plan(PlanArgs p, const uint64_t *hist0,
                                                        uint64_t *cursor0,
                                                        const uint64_t *set_kbase,
                                                        uint64_t n_sets) {
  __shared__ uint64_t s_start[256];
  __shared__ uint64_t wsum[STREAM_NT / 64 + 1];
  if (p.ctl->status) return;
  for (uint64_t s = blockIdx.x; s < n_sets; s += gridDim.x)
    plan_children(p, hist0 + s * 256, set_kbase[s], 0, 1, cursor0 + s * 256, s_start, wsum);
}

// ---------------------------------------------------------------------------
// 3. Partition levels >= 1 over oversized buckets.

// One workgroup: tile offsets of the items of a list.
__global__ __launch_bounds__(1024) void k_level_prep(Item *items, const uint64_t *n_items_p,
                                                     uint64_t *n_tiles_out, uint64_t *other_count,
                                                     const Ctl *ctl) {
  __shared__ uint64_t wsum[1024 / 64 + 1];
  if (ctl->status) return;
  const uint64_t n = *n_items_p;
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < n; c0 += 1024) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t tiles = i < n ? (items[i].size + TILE - 1) / TILE : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<1024>(tiles, wsum, &tot) + carry;
    if (i < n) items[i].tbase = ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *n_tiles_out = carry;
    *other_count = 0;  // the other list receives this level's oversized children
  }
}

struct LevelArgs {
  const Item *items;
  const uint64_t *n_items_p;
  const uint64_t *n_tiles_p;
  uint64_t *hist;
  uint64_t *cursor;
  int bits;
  int level;
};

__device__ __forceinline__ uint64_t find_item(const Item *items, uint64_t n, uint64_t t) {
  uint64_t lo = 0, hi = n;  // last item with tbase <= t
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (items[mid].tbase <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename K>
__device__ __forceinline__ int load_tile(const K *src, uint64_t start, uint64_t end,
                                         K (&keys)[STREAM_KPT]) {
  int n = 0;
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r) {
    const uint64_t i = start + threadIdx.x + (uint64_t)r * STREAM_NT;
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
  if (ctl->status) return;
  const uint64_t n_tiles = *a.n_tiles_p, n_items = *a.n_items_p;
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint64_t ii = find_item(a.items, n_items, t);
    const Item it = a.items[ii];
    const uint64_t start = it.off + (t - it.tbase) * TILE;
    const uint64_t end = it.off + it.size < start + TILE ? it.off + it.size : start + TILE;
    h[threadIdx.x] = 0;
    __syncthreads();
    K keys[STREAM_KPT];
    // strided layout: key r of thread q is start + q + r * STREAM_NT
    const int n = load_tile<K>(it.src ? b1 : b0, start, end, keys);
#pragma unroll
    for (int r = 0; r < STREAM_KPT; ++r)
      if (r < n) atomicAdd(&h[msd_digit(keys[r], a.bits, a.level)], 1u);
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd((unsigned long long *)&a.hist[ii * 256 + threadIdx.x], (unsigned long long)c);
    __syncthreads();
  }
}

__global__ __launch_bounds__(STREAM_NT) void k_level_plan(PlanArgs p, LevelArgs a) {
  __shared__ uint64_t s_start[256];
  __shared__ uint64_t wsum[STREAM_NT / 64 + 1];
  if (p.ctl->status) return;
  const uint64_t n_items = *a.n_items_p;
  for (uint64_t ii = blockIdx.x; ii < n_items; ii += gridDim.x) {
    const Item it = a.items[ii];
    plan_children(p, a.hist + ii * 256, it.off, 1u - it.src, a.level + 1, a.cursor + ii * 256,
                  s_start, wsum);
  }
}

template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_level_scatter(LevelArgs a, K *b0, K *b1,
                                                             const Ctl *ctl) {
  __shared__ PartLds<K> s;
  if (ctl->status) return;
  const uint64_t n_tiles = *a.n_tiles_p, n_items = *a.n_items_p;
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint64_t ii = find_item(a.items, n_items, t);
    const Item it = a.items[ii];
    const uint64_t start = it.off + (t - it.tbase) * TILE;
    const uint64_t end = it.off + it.size < start + TILE ? it.off + it.size : start + TILE;
    K keys[STREAM_KPT];
    // keys are placed through LDS, so any assignment of keys to threads works:
    // use the coalesced strided one (valid keys form a prefix of each thread's)
    const int n = load_tile<K>(it.src ? b1 : b0, start, end, keys);
    partition_tile<K>(keys, n, a.bits, a.level, a.cursor + ii * 256, it.src ? b0 : b1, s);
  }
}

// ---------------------------------------------------------------------------
// 4. LDS-resident sort of each batch: least-significant-digit radix passes over
// the bits in which the batch's keys differ.  Wave w owns the contiguous chunk
// [w * 64 * KPT, (w+1) * 64 * KPT) of the batch; within it, element
// (w * KPT + j) * 64 + lane is held in register j of that lane, so "register j
// before register j+1, lane order within a register" is the current order.
// Ranking is stable: a key's rank counts the equal digits before it in that
// order (earlier registers through a running per-wave count, the same register
// through the ballot peers in lower lanes), and the waves are laid out in order
// by an exclusive scan over (digit, wave).  Slots past the batch hold the
// all-ones key, which is never canonical and, having the largest digit in every
// pass, stays behind every real key.

__device__ __forceinline__ int bit_length(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
__device__ __forceinline__ int bit_length(u128 x) {
  const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  return hi ? 128 - __clzll(hi) : (lo ? 64 - __clzll(lo) : 0);
}
__device__ __forceinline__ uint64_t wave_or_key(uint64_t v) { return wave_or(v); }
__device__ __forceinline__ u128 wave_or_key(u128 v) {
  const uint64_t lo = wave_or((uint64_t)v), hi = wave_or((uint64_t)(v >> 64));
  return ((u128)hi << 64) | lo;
}

template <typename K>
struct LocalLds {
  K keys[LOCAL_NT * LocalCfg<K>::KPT];
  uint32_t wcnt[LOCAL_NW][256];
  K wor[LOCAL_NW];
  uint32_t wsum[LOCAL_NW + 1];
};

template <typename K>
__global__ __launch_bounds__(LOCAL_NT) void k_local_sort(const Batch *batches,
                                                         const uint64_t *n_batches_p, K *b0,
                                                         K *b1, const Ctl *ctl) {
  constexpr int KPT = LocalCfg<K>::KPT;
  __shared__ LocalLds<K> s;
  if (ctl->status) return;
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint64_t n_batches = *n_batches_p;
  for (uint64_t bi = blockIdx.x; bi < n_batches; bi += gridDim.x) {
    const Batch b = batches[bi];
    const K *src = b.src ? b1 : b0;
    const uint32_t m = b.size;
    const uint32_t nwa = (m + 64u * KPT - 1) / (64u * KPT);  // waves holding elements
    const bool active = w < nwa;
    K kv[KPT];
    K diff = 0;
    const K k0 = src[b.off];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t e = (w * KPT + j) * 64 + lane;
      kv[j] = e < m ? src[b.off + e] : all_ones<K>();
      if (e < m) diff |= kv[j] ^ k0;
    }
    diff = wave_or_key(diff);
    if (lane == 0) s.wor[w] = diff;
    __syncthreads();
    K all = 0;
#pragma unroll
    for (int i = 0; i < LOCAL_NW; ++i) all |= s.wor[i];
    const int passes = (bit_length(all) + 7) >> 3;
    for (int p = 0; p < passes; ++p) {
      const int shift = 8 * p;
      uint32_t dg[KPT], rank[KPT];
      if (active) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s.wcnt[w][lane + 64 * q] = 0;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
          const uint32_t d = (uint32_t)(kv[j] >> shift) & 0xffu;
          const uint64_t peers = match_digit8(d);
          const uint32_t before = (uint32_t)__popcll(peers & lt);
          const uint32_t base = s.wcnt[w][d];
          if (before == 0) s.wcnt[w][d] = base + (uint32_t)__popcll(peers);
          dg[j] = d;
          rank[j] = base + before;
        }
      }
      __syncthreads();
      uint32_t run = 0;
      if (tid < 256)
        for (uint32_t v = 0; v < nwa; ++v) {
          const uint32_t c = s.wcnt[v][tid];
          s.wcnt[v][tid] = run;
          run += c;
        }
      uint32_t tot;
      const uint32_t dbase = block_exclusive_scan<LOCAL_NT>(tid < 256 ? run : 0u, s.wsum, &tot);
      if (tid < 256)
        for (uint32_t v = 0; v < nwa; ++v) s.wcnt[v][tid] += dbase;
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < KPT; ++j) s.keys[s.wcnt[w][dg[j]] + rank[j]] = kv[j];
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < KPT; ++j) kv[j] = s.keys[(w * KPT + j) * 64 + lane];
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const uint32_t e = (w * KPT + j) * 64 + lane;
        if (e < m) b0[b.off + e] = kv[j];
      }
    }
    __syncthreads();
  }
}

// Oversized buckets whose digits are exhausted hold one key repeated: they are
// already sorted and only need to be in buffer 0.
template <typename K>
__global__ void k_uniform_copy(const Item *uni, const uint64_t *n_uni_p, K *b0, const K *b1,
                               const Ctl *ctl) {
  if (ctl->status) return;
  const uint64_t n = *n_uni_p;
  for (uint64_t u = 0; u < n; ++u) {
    const Item it = uni[u];
    if (it.src == 0) continue;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < it.size;
         i += (uint64_t)gridDim.x * blockDim.x)
      b0[it.off + i] = b1[it.off + i];
  }
}

// ---------------------------------------------------------------------------
// 5. Run-length reduce of the sorted keys.  Position i starts a run when it is
// the first key of a read set or differs from key i-1.  Thread q of tile t owns
// positions [t*TILE + q*KPT, +KPT).

struct RleArgs {
  const uint64_t *set_kbase;
  uint64_t n_sets;
  uint64_t *tile_heads;
  uint64_t *hpos;  // position of the first key of each run, plus hpos[U] = n
};

template <typename K>
__device__ __forceinline__ uint32_t run_heads(const K *keys, uint64_t n, const RleArgs &a,
                                              uint64_t i0, K (&kv)[STREAM_KPT]) {
  uint32_t flags = 0;
  if (i0 >= n) return 0;
  uint64_t ns = lower_bound(a.set_kbase, 0, a.n_sets + 1, i0);
  uint64_t bnd = ns <= a.n_sets ? a.set_kbase[ns] : ~0ull;
  K prev = i0 ? keys[i0 - 1] : K(0);
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r) {
    const uint64_t i = i0 + r;
    if (i < n) {
      kv[r] = keys[i];
      bool h = (i == 0) || kv[r] != prev;
      if (i == bnd) {
        h = true;
        while (ns <= a.n_sets && a.set_kbase[ns] == i) ++ns;
        bnd = ns <= a.n_sets ? a.set_kbase[ns] : ~0ull;
      }
      if (h) flags |= 1u << r;
      prev = kv[r];
    }
  }
  return flags;
}

template <typename K>
__global__ __launch_bounds__(STREAM_NT) void k_rle_count(const K *keys, RleArgs a,
                                                         const Ctl *ctl) {
  __shared__ uint64_t wsum[STREAM_NT / 64 + 1];
  if (ctl->status) return;
  const uint64_t n = ctl->n_keys;
  const uint64_t i0 = blockIdx.x * TILE + threadIdx.x * (uint64_t)STREAM_KPT;
  K kv[STREAM_KPT];
  const uint32_t f = run_heads<K>(keys, n, a, i0, kv);
  uint64_t tot;
  block_exclusive_scan<STREAM_NT>((uint64_t)__popc(f), wsum, &tot);
  if (threadIdx.x == 0) a.tile_heads[blockIdx.x] = tot;
}

struct OutArgs {
  void *kmer;        // nodes: key per row
  void *u, *v;       // edges
  uint8_t *orient;
  void *zkey;        // optional
  uint64_t capacity;
  int k;
};

template <typename K, bool EDGES>
__global__ __launch_bounds__(STREAM_NT) void k_rle_write(const K *keys, RleArgs a, OutArgs o,
                                                         const Ctl *ctl) {
  __shared__ uint64_t wsum[STREAM_NT / 64 + 1];
  if (ctl->status) return;
  const uint64_t n = ctl->n_keys;
  const uint64_t i0 = blockIdx.x * TILE + threadIdx.x * (uint64_t)STREAM_KPT;
  K kv[STREAM_KPT];
  const uint32_t f = run_heads<K>(keys, n, a, i0, kv);
  uint64_t tot;
  uint64_t j = block_exclusive_scan<STREAM_NT>((uint64_t)__popc(f), wsum, &tot) +
               a.tile_heads[blockIdx.x];
#pragma unroll
  for (int r = 0; r < STREAM_KPT; ++r) {
    if (f & (1u << r)) {
      a.hpos[j] = i0 + r;
      if (j < o.capacity) {
        if (EDGES) {
          K u, v;
          uint32_t orient;
          decode_edge(kv[r], o.k, &u, &v, &orient);
          static_cast<K *>(o.u)[j] = u;
          static_cast<K *>(o.v)[j] = v;
          o.orient[j] = (uint8_t)orient;
          if (o.zkey) static_cast<K *>(o.zkey)[j] = kv[r];
        } else {
          static_cast<K *>(o.kmer)[j] = kv[r];
        }
      }
      ++j;
    }
  }
  if (n && i0 <= n - 1 && n - 1 < i0 + STREAM_KPT) a.hpos[ctl->n_unique] = n;
}

// counts / multiplicities from run starts; per-set row offsets; result counters.
__global__ void k_finalize(const uint64_t *hpos, uint32_t *count, uint64_t capacity,
                           const Ctl *ctl) {
  if (ctl->status) return;
  const uint64_t u = ctl->n_unique;
  const uint64_t lim = u < capacity ? u : capacity;
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < lim;
       j += (uint64_t)gridDim.x * blockDim.x)
    count[j] = (uint32_t)(hpos[j + 1] - hpos[j]);
}

__global__ void k_set_uoff(const uint64_t *hpos, const uint64_t *set_kbase, uint64_t n_sets,
                           uint64_t *set_uoff, const Ctl *ctl) {
  if (ctl->status || !set_uoff) return;
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s > n_sets) return;
  set_uoff[s] = lower_bound(hpos, 0, ctl->n_unique, set_kbase[s]);
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
  res->reserved = 0;
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
  uint64_t *tile_read = reinterpret_cast<uint64_t *>(ws + L.tile_read);
  uint32_t *tile_set = reinterpret_cast<uint32_t *>(ws + L.tile_set);
  uint64_t *hist0 = reinterpret_cast<uint64_t *>(ws + L.hist0);
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
  uint64_t *hpos = reinterpret_cast<uint64_t *>(ws + L.keys[1]);
  hipStream_t st = A.stream;
  const uint64_t S = A.n_sets;
  const int len = edges ? A.k + 1 : A.k;
  const int bits = 2 * len;
  const int ev = edges ? 0 : 10;

  stage(ev + 0, st);
  hipLaunchKernelGGL(k_table_reset, dim3(1), dim3(1), 0, st, ctl);
  hipLaunchKernelGGL(k_read_reduce, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, A.n_bases, len, block_sums, ctl);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, block_sums, L.read_blocks,
                     (uint64_t *)nullptr);
  hipLaunchKernelGGL(k_read_apply, dim3((unsigned)L.read_blocks), dim3(SCAN_NT), 0, st,
                     A.read_offsets, A.n_reads, len, block_sums, rbase, ctl);
  hipLaunchKernelGGL(k_set_setup, dim3(1), dim3(1024), 0, st, rbase, A.n_reads, set_read_off, S,
                     A.max_keys, set_kbase, set_tbase, ctl);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(S * 256, 256, 4096)), dim3(256), 0, st, hist0,
                     S * 256, 0ull);
  hipLaunchKernelGGL(k_tile_map, dim3(grid_for(L.max_tiles, 256, 1u << 30)), dim3(256), 0, st,
                     rbase, set_read_off, S, set_kbase, set_tbase, tile_read, tile_set,
                     L.max_tiles, ctl);
  stage(ev + 1, st);
  EnumArgs ea{A.packed, (A.n_bases + 31) / 32, A.read_offsets, rbase, set_read_off, set_kbase,
              set_tbase, tile_read, tile_set, len, bits};
  hipLaunchKernelGGL(k_enum_hist<K>, dim3((unsigned)L.max_tiles), dim3(STREAM_NT), 0, st, ea,
                     hist0, ctl);
  stage(ev + 2, st);
  PlanArgs pa{items[1], &ctl->items[1], hist[1], L.item_cap, batches, L.batch_cap,
              uniform, L.item_cap, ctl, local_cap<K>(), bits};
  hipLaunchKernelGGL(k_set_plan, dim3(grid_for(S, 1, 4096)), dim3(STREAM_NT), 0, st, pa, hist0,
                     cursor0, set_kbase, S);
  stage(ev + 3, st);
  hipLaunchKernelGGL(k_enum_scatter<K>, dim3((unsigned)L.max_tiles), dim3(STREAM_NT), 0, st, ea,
                     cursor0, x0, ctl);
  stage(ev + 4, st);
  const unsigned level_grid = grid_for(L.max_tiles + L.item_cap, 1, 8192);
  for (int lev = 1; bits - 8 * lev > 0; ++lev) {
    const int li = lev & 1;
    hipLaunchKernelGGL(k_level_prep, dim3(1), dim3(1024), 0, st, items[li], &ctl->items[li],
                       &ctl->level_tiles[li], &ctl->items[li ^ 1], ctl);
    LevelArgs la{items[li], &ctl->items[li], &ctl->level_tiles[li], hist[li], cursor, bits, lev};
    hipLaunchKernelGGL(k_level_hist<K>, dim3(level_grid), dim3(STREAM_NT), 0, st, la, x0, x1, ctl);
    PlanArgs pl{items[li ^ 1], &ctl->items[li ^ 1], hist[li ^ 1], L.item_cap, batches,
                L.batch_cap, uniform, L.item_cap, ctl, local_cap<K>(), bits};
    hipLaunchKernelGGL(k_level_plan, dim3(grid_for(L.item_cap, 1, 4096)), dim3(STREAM_NT), 0, st,
                       pl, la);
    hipLaunchKernelGGL(k_level_scatter<K>, dim3(level_grid), dim3(STREAM_NT), 0, st, la, x0, x1,
                       ctl);
  }
  stage(ev + 5, st);
  hipLaunchKernelGGL(k_local_sort<K>, dim3(grid_for(L.batch_cap, 1, 2048)), dim3(LOCAL_NT), 0, st,
                     batches, &ctl->n_batches, x0, x1, ctl);
  stage(ev + 6, st);
  hipLaunchKernelGGL(k_uniform_copy<K>, dim3(1024), dim3(256), 0, st, uniform, &ctl->n_uniform, x0,
                     x1, ctl);
  RleArgs ra{set_kbase, S, rle_heads, hpos};
  hipLaunchKernelGGL(k_rle_count<K>, dim3((unsigned)L.rle_tiles), dim3(STREAM_NT), 0, st, x0, ra,
                     ctl);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, rle_heads, L.rle_tiles,
                     &ctl->n_unique);
  stage(ev + 7, st);
  OutArgs oa{};
  oa.k = A.k;
  uint32_t *count;
  uint64_t capacity;
  uint64_t *set_uoff;
  if (edges) {
    oa.u = A.edges.u;
    oa.v = A.edges.v;
    oa.orient = A.edges.orient;
    oa.zkey = A.edges.zkey;
    oa.capacity = capacity = A.edges.capacity;
    count = A.edges.mult;
    set_uoff = A.edge_set_offsets;
    hipLaunchKernelGGL((k_rle_write<K, true>), dim3((unsigned)L.rle_tiles), dim3(STREAM_NT), 0,
                       st, x0, ra, oa, ctl);
  } else {
    oa.kmer = A.nodes.kmer;
    oa.capacity = capacity = A.nodes.capacity;
    count = A.nodes.count;
    set_uoff = A.node_set_offsets;
    hipLaunchKernelGGL((k_rle_write<K, false>), dim3((unsigned)L.rle_tiles), dim3(STREAM_NT), 0,
                       st, x0, ra, oa, ctl);
  }
  stage(ev + 8, st);
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(A.max_keys, 256, 65536)), dim3(256), 0, st, hpos,
                     count, capacity, ctl);
  hipLaunchKernelGGL(k_set_uoff, dim3(grid_for(S + 1, 256, 1u << 30)), dim3(256), 0, st, hpos,
                     set_kbase, S, set_uoff, ctl);
  hipLaunchKernelGGL(k_table_done, dim3(1), dim3(1), 0, st, ctl, edges ? 1 : 0, capacity);
  stage(ev + 9, st);
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

hipError_t run_build_u64(const BuildArgs &a, const Layout &L) { return run_build<uint64_t>(a, L); }
hipError_t run_build_u128(const BuildArgs &a, const Layout &L) { return run_build<u128>(a, L); }

}  // namespace dbg
