// C ABI of the graph builder: argument checks, workspace layout and dispatch on
// the key width (64-bit keys for k <= 31, 128-bit keys for 33 <= k <= 63).
#include <mutex>

#include "dbg_internal.h"

// Workspace of dbg_build_noalloc: one array on every device the library runs on,
// held until the process ends.  In host code the name only stands for the
// symbol; the array's device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[DBG_NOALLOC_SCRATCH_BYTES];

namespace dbg {

// Device address of the scratch array on each device, looked up once per
// device with that device current.
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

static int scratch_address(hipStream_t stream, void **out) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return DBG_E_HIP;
  int dev = cur;
  if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess) return DBG_E_HIP;
  if (dev < 0 || dev >= MAX_DEVICES) return DBG_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return DBG_E_HIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return DBG_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DBG_OK;
}

// Process-wide tuning: copied under the lock at the start of each build call.
static std::mutex g_tuning_mu;
static dbg_tuning_t g_tuning = {DBG_NODES_AUTO, 0.6f, 2, 0, 1, {0, 0, 0}};

static dbg_tuning_t current_tuning() {
  std::lock_guard<std::mutex> lock(g_tuning_mu);
  return g_tuning;
}

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(uint64_t n_reads, uint64_t n_sets, uint64_t max_keys, int k,
                   uint64_t max_positions) {
  Layout L{};
  L.key_bytes = k <= 31 ? 8 : 16;
  // list capacities follow from the smallest batch any workgroup shape takes
  const uint64_t cap =
      k <= 31 ? local_cap<uint64_t, true, 1>() : local_cap<unsigned __int128, true, 1>();
  const int edge_bits = 2 * (k + 1);
  const uint64_t levels = (uint64_t)((edge_bits + 7) / 8);  // digit levels incl. level 0
  L.max_tiles = (max_positions + TILE - 1) / TILE + n_sets;
  L.item_cap = max_keys / cap + 2;
  // batches per level <= 2 * keys / cap + parents + oversized children
  L.batch_cap = levels * (2 * (max_keys / cap) + 1) + n_sets + 3 * levels * L.item_cap + 64;
  // digit ranges of in-tile buckets (one level has them): at most two per
  // capacity's worth of keys plus one per bucket
  L.seg_cap = 2 * (max_keys / cap) + L.item_cap + 64;
  L.rle_tiles = (max_keys + TILE - 1) / TILE;
  if (L.rle_tiles == 0) L.rle_tiles = 1;
  L.read_blocks = n_reads / ((uint64_t)256 * 16) + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.ctl = take(sizeof(Ctl));
  L.set_read_off = take(2 * sizeof(uint64_t));
  L.rbase = take((n_reads + 1) * sizeof(uint64_t));
  L.block_sums = take(L.read_blocks * sizeof(uint64_t));
  L.set_kbase = take((n_sets + 1) * sizeof(uint64_t));
  L.set_tbase = take((n_sets + 1) * sizeof(uint64_t));
  L.tiles = take(L.max_tiles * sizeof(TileDesc));
  // per-tile digit counts: enumeration tiles, or the tiles of a partition level
  // (at most one partial tile per bucket more)
  const uint64_t rows = L.max_tiles + L.item_cap;
  L.thist = take((rows + 1) * 256 * sizeof(uint32_t));
  L.titem = take(rows * sizeof(uint32_t));
  L.csum = take(((rows + 63) / 64 + 1) * 256 * sizeof(uint32_t));
  L.cursor0 = take(n_sets * 256 * sizeof(uint64_t));
  for (int i = 0; i < 2; ++i) L.items[i] = take(L.item_cap * sizeof(Item));
  for (int i = 0; i < 2; ++i) L.hist[i] = take(L.item_cap * 256 * sizeof(uint64_t));
  L.cursor = take(L.item_cap * 256 * sizeof(uint64_t));
  L.batches = take(L.batch_cap * sizeof(Batch));
  L.segb = take(L.seg_cap * sizeof(SegBatch));
  L.segt = take(L.seg_cap * SEG_TILES * sizeof(uint32_t));
  L.uniform = take(L.item_cap * sizeof(Item));
  L.rle_heads = take(L.rle_tiles * sizeof(uint64_t));
  L.rle_sums = take((L.rle_tiles / 4096 + 2) * sizeof(uint64_t));
  L.bits = take(L.rle_tiles * (TILE / 8));
  // the count of each distinct key, at the key's position in buffer 0
  L.counts = take((max_keys + 2) * sizeof(uint32_t));
  L.set_uoff = 0;
  // key buffers: ping-pong for the partition levels; after the bucket sort
  // buffer 0 holds the distinct keys
  const size_t kb = (max_keys + 2) * (size_t)L.key_bytes;
  for (int i = 0; i < 2; ++i) L.keys[i] = take(kb);
  // weighted records: keys in [0, R w), weights from here on (R <= this / w)
  L.weights = (kb / (size_t)(L.key_bytes + 4) * (size_t)L.key_bytes) & ~size_t(15);
  L.total = off;
  return L;
}

static int check_common(uint64_t n_bases, const uint64_t *packed, const uint64_t *read_offsets,
                        int k, uint64_t max_keys, const dbg_nodes_t *nodes,
                        const dbg_edges_t *edges, dbg_result_t *result, void *workspace) {
  if (!read_offsets || !nodes || !edges || !result || !workspace) return DBG_E_NULL;
  if (n_bases && !packed) return DBG_E_NULL;
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (max_keys >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (nodes->capacity && (!nodes->kmer || !nodes->count)) return DBG_E_NULL;
  if (edges->capacity && (!edges->u || !edges->v || !edges->orient || !edges->mult))
    return DBG_E_NULL;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DBG_E_WORKSPACE;
  return DBG_OK;
}

static int run(const BuildArgs &a, size_t workspace_bytes) {
  const Layout L = make_layout(a.n_reads, a.n_sets, a.max_keys, a.k, a.max_positions);
  if (workspace_bytes < L.total) return DBG_E_WORKSPACE;
  const hipError_t e = a.k <= 31 ? run_build_u64(a, L) : run_build_u128(a, L);
  return e == hipSuccess ? DBG_OK : DBG_E_HIP;
}

}  // namespace dbg

extern "C" {

size_t dbg_workspace_bytes(uint64_t n_reads, uint64_t n_sets, uint64_t max_keys, int k) {
  if (k < 1 || k > 63 || (k & 1) == 0 || n_sets == 0) return 0;
  return dbg::make_layout(n_reads, n_sets, max_keys, k, max_keys).total;
}

size_t dbg_slice_workspace_bytes(uint64_t n_reads, uint64_t max_positions, uint64_t max_keys,
                                 int k) {
  if (k < 1 || k > 63 || (k & 1) == 0 || max_keys > max_positions) return 0;
  return dbg::make_layout(n_reads, 1, max_keys, k, max_positions).total;
}

int dbg_build(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
              uint64_t n_reads, int k, uint64_t max_keys, const dbg_nodes_t *nodes,
              const dbg_edges_t *edges, dbg_result_t *result, void *workspace,
              size_t workspace_bytes, hipStream_t stream) {
  const int c = dbg::check_common(n_bases, packed, read_offsets, k, max_keys, nodes, edges, result,
                                  workspace);
  if (c != DBG_OK) return c;
  dbg::BuildArgs a{};
  a.packed = packed;
  a.n_bases = n_bases;
  a.read_offsets = read_offsets;
  a.n_reads = n_reads;
  a.set_read_offsets = nullptr;
  a.n_sets = 1;
  a.max_keys = max_keys;
  a.max_positions = max_keys;
  a.pfx_lo = 0;
  a.pfx_hi = dbg::PFX_BINS;
  a.k = k;
  a.nodes = *nodes;
  a.edges = *edges;
  a.result = result;
  a.workspace = workspace;
  a.stream = stream;
  a.tuning = dbg::current_tuning();
  return dbg::run(a, workspace_bytes);
}

int dbg_build_noalloc(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, int k, uint64_t max_keys, const dbg_nodes_t *nodes,
                      const dbg_edges_t *edges, dbg_result_t *result, hipStream_t stream) {
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (max_keys >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (n_reads >= DBG_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)) return DBG_E_SCRATCH;
  const size_t need = dbg::make_layout(n_reads, 1, max_keys, k, max_keys).total;
  if (need > DBG_NOALLOC_SCRATCH_BYTES) return DBG_E_SCRATCH;
  void *ws = nullptr;
  const int rc = dbg::scratch_address(stream, &ws);
  if (rc != DBG_OK) return rc;
  return dbg_build(packed, n_bases, read_offsets, n_reads, k, max_keys, nodes, edges, result, ws,
                   DBG_NOALLOC_SCRATCH_BYTES, stream);
}

int dbg_build_batched(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, const uint64_t *set_read_offsets, uint64_t n_sets,
                      int k, uint64_t max_keys, const dbg_nodes_t *nodes,
                      const dbg_edges_t *edges, uint64_t *node_set_offsets,
                      uint64_t *edge_set_offsets, dbg_result_t *result, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  const int c = dbg::check_common(n_bases, packed, read_offsets, k, max_keys, nodes, edges, result,
                                  workspace);
  if (c != DBG_OK) return c;
  if (!set_read_offsets) return DBG_E_NULL;
  if (n_sets == 0 || n_sets >= (1ull << 31)) return DBG_E_ARG;
  dbg::BuildArgs a{};
  a.packed = packed;
  a.n_bases = n_bases;
  a.read_offsets = read_offsets;
  a.n_reads = n_reads;
  a.set_read_offsets = set_read_offsets;
  a.n_sets = n_sets;
  a.max_keys = max_keys;
  a.max_positions = max_keys;
  a.pfx_lo = 0;
  a.pfx_hi = dbg::PFX_BINS;
  a.k = k;
  a.nodes = *nodes;
  a.edges = *edges;
  a.node_set_offsets = node_set_offsets;
  a.edge_set_offsets = edge_set_offsets;
  a.result = result;
  a.workspace = workspace;
  a.stream = stream;
  a.tuning = dbg::current_tuning();
  return dbg::run(a, workspace_bytes);
}

int dbg_build_slice(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                    uint64_t n_reads, int k, uint64_t max_positions, uint64_t max_keys,
                    uint32_t prefix_lo, uint32_t prefix_hi, const dbg_nodes_t *nodes,
                    const dbg_edges_t *edges, dbg_result_t *result, void *workspace,
                    size_t workspace_bytes, hipStream_t stream) {
  const int c = dbg::check_common(n_bases, packed, read_offsets, k, max_keys, nodes, edges, result,
                                  workspace);
  if (c != DBG_OK) return c;
  if (max_positions >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (max_keys > max_positions || prefix_lo > prefix_hi || prefix_hi > DBG_PREFIX_BINS)
    return DBG_E_ARG;
  dbg::BuildArgs a{};
  a.packed = packed;
  a.n_bases = n_bases;
  a.read_offsets = read_offsets;
  a.n_reads = n_reads;
  a.set_read_offsets = nullptr;
  a.n_sets = 1;
  a.max_keys = max_keys;
  a.max_positions = max_positions;
  a.pfx_lo = prefix_lo;
  a.pfx_hi = prefix_hi;
  a.k = k;
  a.nodes = *nodes;
  a.edges = *edges;
  a.result = result;
  a.workspace = workspace;
  a.stream = stream;
  a.tuning = dbg::current_tuning();
  return dbg::run(a, workspace_bytes);
}

size_t dbg_prefix_workspace_bytes(uint64_t n_reads, uint64_t max_positions, int k) {
  if (k < 1 || k > 63 || (k & 1) == 0) return 0;
  return dbg::make_layout(n_reads, 1, 0, k, max_positions).total;
}

int dbg_prefix_counts(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, int k, uint64_t max_positions, uint64_t *edge_counts,
                      uint64_t *node_counts, dbg_result_t *result, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  if (!read_offsets || !edge_counts || !node_counts || !result || !workspace) return DBG_E_NULL;
  if (n_bases && !packed) return DBG_E_NULL;
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (max_positions >= (1ull << 32)) return DBG_E_OVERFLOW;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DBG_E_WORKSPACE;
  const dbg::Layout L = dbg::make_layout(n_reads, 1, 0, k, max_positions);
  if (workspace_bytes < L.total) return DBG_E_WORKSPACE;
  dbg::BuildArgs a{};
  a.packed = packed;
  a.n_bases = n_bases;
  a.read_offsets = read_offsets;
  a.n_reads = n_reads;
  a.n_sets = 1;
  a.max_keys = 0;
  a.max_positions = max_positions;
  a.pfx_lo = 0;
  a.pfx_hi = dbg::PFX_BINS;
  a.k = k;
  a.result = result;
  a.workspace = workspace;
  a.stream = stream;
  return dbg::run_prefix_counts(a, L, edge_counts, node_counts) == hipSuccess ? DBG_OK
                                                                              : DBG_E_HIP;
}

int dbg_bounds(const uint64_t *read_offsets, uint64_t n_reads, int k, uint64_t *max_nodes,
               uint64_t *max_edges) {
  if (!read_offsets || !max_nodes || !max_edges) return DBG_E_NULL;
  if (k < 1 || k > 63 || (k & 1) == 0) return DBG_E_K;
  if (read_offsets[0] != 0) return DBG_E_OFFSETS;
  uint64_t nk = 0, ne = 0;
  for (uint64_t i = 0; i < n_reads; ++i) {
    if (read_offsets[i + 1] < read_offsets[i]) return DBG_E_OFFSETS;
    const uint64_t len = read_offsets[i + 1] - read_offsets[i];
    if (len >= (uint64_t)k) nk += len - (uint64_t)k + 1;
    if (len > (uint64_t)k) ne += len - (uint64_t)k;
  }
  *max_nodes = nk;
  *max_edges = ne;
  return DBG_OK;
}

int dbg_pack_ascii(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed,
                   dbg_result_t *result, hipStream_t stream) {
  if (n_bases && (!ascii || !packed)) return DBG_E_NULL;
  if (!result) return DBG_E_NULL;
  return dbg::launch_pack(ascii, n_bases, packed, result, stream) == hipSuccess ? DBG_OK
                                                                                : DBG_E_HIP;
}

int dbg_set_stage_events(hipEvent_t *events, int n_events) {
  if (events && n_events < DBG_STAGE_EVENTS) return DBG_E_ARG;
  dbg::set_stage_events(events);
  return DBG_OK;
}

int dbg_set_tuning(const dbg_tuning_t *tuning) {
  dbg_tuning_t t = {DBG_NODES_AUTO, 0.6f, 2, 0, 1, {0, 0, 0}};
  if (tuning) {
    if (tuning->node_path < DBG_NODES_AUTO || tuning->node_path > DBG_NODES_ENDPOINTS)
      return DBG_E_ARG;
    if (!(tuning->endpoint_ratio >= 0.0f && tuning->endpoint_ratio <= 2.0f)) return DBG_E_ARG;
    if (tuning->local_variant < 0 || tuning->local_variant >= dbg::LOCAL_VARIANTS)
      return DBG_E_ARG;
    if (tuning->lds_digit_bias < -3 || tuning->lds_digit_bias > 3) return DBG_E_ARG;
    if (tuning->in_tile != 0 && tuning->in_tile != 1) return DBG_E_ARG;
    t = *tuning;
  }
  std::lock_guard<std::mutex> lock(dbg::g_tuning_mu);
  dbg::g_tuning = t;
  return DBG_OK;
}

int dbg_get_tuning(dbg_tuning_t *tuning) {
  if (!tuning) return DBG_E_NULL;
  *tuning = dbg::current_tuning();
  return DBG_OK;
}

const char *dbg_strerror(int status) {
  switch (status) {
    case DBG_OK: return "ok";
    case DBG_E_NULL: return "a required pointer is null";
    case DBG_E_K: return "k must be odd and in [1, 63]";
    case DBG_E_OFFSETS: return "read or set offsets are not monotone or do not match n_bases";
    case DBG_E_OVERFLOW: return "more keys than max_keys, or max_keys >= 2^32";
    case DBG_E_CAPACITY: return "output capacity below the number of distinct rows";
    case DBG_E_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case DBG_E_HIP: return "HIP launch failure";
    case DBG_E_BASE: return "input byte is not one of A, C, G, T";
    case DBG_E_ARG: return "invalid argument";
    case DBG_E_INTERNAL: return "internal list capacity exceeded";
    case DBG_E_SCRATCH: return "the build needs more workspace than the no-allocation scratch holds";
  }
  return "unknown status";
}

}  // extern "C"
