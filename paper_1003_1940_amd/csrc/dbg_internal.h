// Internal layout shared by the kernels and the host-side launch sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dbg.h"

namespace dbg {

// Streaming kernels (enumeration, partition, run-length reduce): 256 threads x
// 16 keys = one 4096-key tile per workgroup.
constexpr int STREAM_NT = 256;
constexpr int STREAM_KPT = 16;
constexpr uint64_t TILE = (uint64_t)STREAM_NT * STREAM_KPT;
constexpr int TILES_NT_WIDE = 512;  // threads of the in-tile pass for 128-bit keys

// LDS-resident bucket sort: a workgroup of NT threads sorts a batch of
// consecutive small buckets of up to CAP keys entirely in LDS (see
// k_local_sort): duplicates are merged in an LDS hash table of SLOTS slots, the
// distinct keys are sorted, and the runs are expanded again.
// W = true: weighted records (the node table built from edge endpoints), whose
// 32-bit weights are summed instead of counted; their wider counts take LDS, so
// the 64-bit variant holds fewer keys.  V selects the workgroup shape: 0 = 512
// threads and the largest batch that fits the 160 KB of LDS (one workgroup per
// CU), 1 = 256 threads and half the batch (two workgroups per CU: more batches
// in flight for small inputs, more keys left for deeper partition levels),
// 2 = the batch of 0 with more threads (768 for 64-bit keys, 1024 for 128-bit
// keys): the same LDS, more waves to hide its latency.
template <typename K, bool W = false, int V = 0> struct LocalCfg {
  static_assert(V >= 0 && V <= 2, "three workgroup shapes");
  static constexpr int NT = V == 1 ? 256 : V == 2 ? (sizeof(K) == 8 ? 768 : 1024) : 512;
  static constexpr int CAP = (sizeof(K) == 8 ? (W ? 5120 : 6144) : 3072) >> (V == 1 ? 1 : 0);
  static constexpr int SLOTS = CAP * 3 / 2;
  static constexpr int SMALL = sizeof(K) == 8 ? 16 : 8;  // segments sorted by one lane's network
  static constexpr int WAVES_PER_EU = (NT / 64 + 3) / 4;
};
template <typename K, bool W = false, int V = 0> constexpr uint64_t local_cap() {
  return (uint64_t)LocalCfg<K, W, V>::CAP;
}
constexpr int LOCAL_VARIANTS = 3;

// Key-space slices: a build can keep only the keys whose top PFX_BITS bits (the
// prefix) lie in [pfx_lo, pfx_hi); slices of disjoint prefix ranges give disjoint
// parts of both sorted tables.
constexpr int PFX_BITS = 12;
constexpr uint32_t PFX_BINS = 1u << PFX_BITS;

// Most-significant-digit levels: level 0 is the enumeration scatter; a key of b
// bits has ceil(b / 8) digits.
constexpr int MAX_LEVELS = 16;

struct Ctl {
  uint32_t status;  // first error found on the device (dbg_status), 0 if none
  uint32_t pad0;
  uint64_t n_keys;          // keys of the table being built
  uint64_t n_tiles;         // enumeration tiles of that table
  uint64_t items[2];        // oversized buckets waiting for the next level (two lists)
  uint64_t level_tiles[2];  // 4096-key tiles over each list's buckets
  uint64_t level_scatter_tiles[2];  // the first ones: tiles of buckets that are scattered
  uint64_t n_batches;       // batches of small buckets for the LDS sort
  uint64_t n_uniform;       // oversized buckets whose digits are exhausted (all keys equal)
  uint64_t n_unique;        // distinct keys of the table
  uint64_t n_edges, n_nodes;
  uint32_t capacity_short;  // an output table had more rows than its capacity
  uint32_t node_path;       // 0: node table from k-mers, 1: from edge endpoints
  uint64_t n_records;       // weighted endpoint records (node_path 1)
  uint64_t n_seg;           // digit ranges of in-tile buckets planned at the current level
};

struct Item {  // an oversized bucket: keys [off, off + size) of buffer `src`
  uint64_t off, size, tbase;
  uint32_t src;
  uint32_t in_tile;  // 1: split within each of its tiles (at most SEG_TILES of them)
};

// Buckets of at most SEG_TILES tiles are split tile by tile: every tile is
// partitioned by the level's digit in place (its keys move to buffer 1 at the
// tile's own positions, digit-contiguous, and its 256 digit offsets go to a row),
// so the keys of a range of digits lie in one segment per tile.
constexpr int SEG_TILES = 64;

struct SegBatch {  // digits [da, db) of an in-tile bucket: one segment per tile
  uint64_t out;       // where the range's keys start in sorted order (buffer 0)
  uint32_t size;      // keys in the range
  uint32_t tiles;     // tiles of the bucket
  uint64_t item_off;  // first key of the bucket (its first tile)
  uint32_t range;     // batch_src(0, level, da, db)
  uint32_t pad;
};
// Beside every SegBatch, a table of SEG_TILES words: word i = the range's
// first and end offsets inside tile i (each at most TILE, 16 bits apiece).

// One enumeration tile: everything its workgroup needs before loading the packed
// words, in one 64-byte record (so a tile's set-up is one dependent load).
struct TileDesc {
  uint64_t start;             // its first key (key index over all positions)
  uint64_t read_lo, read_hi;  // reads [read_lo, read_hi) hold its keys
  uint64_t g_base;            // first key of read read_lo
  uint64_t wb, we;            // packed words [wb, we) hold those reads' bases
  uint64_t t_first;           // first tile of its read set
  uint32_t set;               // its read set
  uint32_t n;                 // its keys (at most TILE)
};

struct Batch {  // consecutive small buckets [off, off + size) of buffer `src`
  uint64_t off;
  uint32_t size;
  uint32_t src;  // batch_src: the buffer, and the digit range the buckets span
};

// A batch's buckets are the children [da, db) of one parent split by the digit
// of partition level `level`: its keys share every bit above that digit and the
// digit lies in [da, db).  Packed with the buffer into Batch::src (and into
// SegBatch::range): bit 0 buffer, bits 1..5 level + 1 (0: no range known),
// bits 6..13 da, bits 14..22 db.
__host__ __device__ inline uint32_t batch_src(uint32_t buf, int level, uint32_t da, uint32_t db) {
  return buf | (uint32_t)(level + 1) << 1 | da << 6 | db << 14;
}
__host__ __device__ inline uint32_t batch_buf(uint32_t src) { return src & 1u; }
__host__ __device__ inline int batch_level(uint32_t src) { return (int)((src >> 1) & 31u) - 1; }
__host__ __device__ inline uint32_t batch_da(uint32_t src) { return (src >> 6) & 0xffu; }
__host__ __device__ inline uint32_t batch_db(uint32_t src) { return (src >> 14) & 0x1ffu; }

// Byte layout of a caller-provided workspace.
struct Layout {
  size_t ctl, set_read_off, rbase, block_sums, set_kbase, set_tbase, tiles;
  size_t thist, csum, cursor0, items[2], hist[2], cursor, batches, uniform, rle_heads, bits, set_uoff;
  size_t counts;  // uint32 count of each distinct key, beside buffer 0
  size_t segb;    // SegBatch list of the in-tile level
  size_t segt;    // their segment tables, SEG_TILES words each
  size_t rle_sums;  // chunk sums of the per-tile distinct counts
  size_t titem;   // uint32 item of every tile of a partition level
  size_t keys[2];
  size_t weights;  // byte offset of the record weights inside each key buffer
  size_t total;
  uint64_t max_tiles, item_cap, batch_cap, seg_cap, rle_tiles, read_blocks;
  int key_bytes;
};

// max_positions bounds the k-mer positions the enumeration visits, max_keys the
// keys a table keeps (the same unless the build is a key-space slice).
Layout make_layout(uint64_t n_reads, uint64_t n_sets, uint64_t max_keys, int k,
                   uint64_t max_positions);

struct BuildArgs {
  const uint64_t *packed;
  uint64_t n_bases;
  const uint64_t *read_offsets;
  uint64_t n_reads;
  const uint64_t *set_read_offsets;  // null: one set
  uint64_t n_sets;
  uint64_t max_keys;
  uint64_t max_positions;  // >= max_keys; > max_keys only for a slice
  uint32_t pfx_lo, pfx_hi;  // key prefixes kept: [pfx_lo, pfx_hi) of [0, PFX_BINS)
  int k;
  dbg_nodes_t nodes;
  dbg_edges_t edges;
  uint64_t *node_set_offsets;  // optional, n_sets + 1
  uint64_t *edge_set_offsets;  // optional
  dbg_result_t *result;
  void *workspace;
  hipStream_t stream;
  dbg_tuning_t tuning;
};

hipError_t run_build_u64(const BuildArgs &a, const Layout &L);
hipError_t run_build_u128(const BuildArgs &a, const Layout &L);
// Counts of the canonical (k+1)-mer and k-mer prefixes (PFX_BINS each, uint64).
hipError_t run_prefix_counts(const BuildArgs &a, const Layout &L, uint64_t *edge_counts,
                             uint64_t *node_counts);
void set_stage_events(hipEvent_t *events);
hipError_t launch_pack(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed,
                       dbg_result_t *result, hipStream_t stream);

}  // namespace dbg
