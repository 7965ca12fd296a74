/*
 * dbg.h -- C ABI of the MI355X (gfx950) bi-directed de Bruijn graph builder.
 *
 * Computes, for a set of DNA reads over {A, C, G, T} and an odd k, the graph of
 * Kundeti, Rajasekaran, Dinh, Vaughn and Thapar, "Efficient Parallel and Out of
 * Core Algorithms for Constructing Large Bi-directed de Bruijn Graphs":
 *   - the node table: every canonical k-mer (Sec. 2: the lexicographically
 *     smaller of a k-mer and its reverse complement) with the number of read
 *     positions whose k-mer canonicalises to it (STEP-3 of BiConstruct, Sec. 3,
 *     with counts);
 *   - the edge list: for every (k+1)-mer of the reads, the canonical bi-directed
 *     edge (u, v, o1, o2) of STEP-1 (Sec. 3), deduplicated with multiplicities
 *     (STEP-2).
 * Counts are taken over the reads as given (each (k+1)-mer position contributes
 * 1), not over reads plus reverse complements, which would double every count.
 *
 * Encodings
 *   bases:   A=0 C=1 G=2 T=3; complement = 3 - code.  Lexicographic order A<C<G<T.
 *   packed:  base j of the concatenated read stream sits in bits
 *            [63 - 2(j mod 32), 62 - 2(j mod 32)] of 64-bit word j / 32
 *            (first base most significant).  Read i is bases
 *            [read_offsets[i], read_offsets[i+1]); reads may start anywhere.
 *   keys:    a string of L bases is the integer sum c_j 4^(L-1-j), so integer
 *            order is string order.  k <= 31: node keys and edge keys ((k+1)-mers,
 *            up to 64 bits at k = 31) are one uint64_t.  33 <= k <= 63: two
 *            uint64_t per key, low word first (a little-endian 128-bit integer).
 *   orient:  (o1 << 1) | o2 with '+' (right-pointing head; the k-mer is the
 *            canonical strand) = 0 and '-' (left-pointing head) = 1.
 *   an edge (u, v, o1, o2) stands for the (k+1)-mer: strand o1 of u followed by
 *   the last base of strand o2 of v; read along the other strand the same edge
 *   is (v, u, not o2, not o1).  u <= v always; when u = v the smaller
 *   orientation pair of the two readings is reported (this only decides
 *   homopolymer (k+1)-mers, which the printed table would otherwise give two
 *   records).
 *
 * Output order (deterministic, exactly one correct output exists)
 *   nodes ascending by k-mer key; edges ascending by the canonical (k+1)-mer they
 *   stand for (zkey).  Edge records and canonical (k+1)-mers are in one-to-one
 *   correspondence.
 *
 * Ownership and execution
 *   Every pointer marked "device" is device memory owned by the caller (for
 *   example allocated through PyTorch).  The library never allocates or frees
 *   memory and never synchronises: all work is enqueued on `stream`, and results
 *   (including dbg_result_t) are valid once the caller has synchronised with the
 *   stream.  Concurrent calls are safe on different streams with distinct
 *   workspaces and outputs.
 *
 * Errors
 *   Arguments checked on the host return a non-zero dbg_status and enqueue
 *   nothing.  Conditions only visible to the device (malformed offsets, more
 *   keys than max_keys, output capacity too small) are written to
 *   dbg_result_t.status (first error wins); after a device-side error the
 *   remaining kernels return early and the outputs are undefined, except for
 *   DBG_E_CAPACITY, where the first `capacity` rows are valid and n_nodes /
 *   n_edges hold the true counts.
 */
#ifndef DBG_H
#define DBG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DBG_OK = 0,
  DBG_E_NULL = 1,       /* a required pointer is null */
  DBG_E_K = 2,          /* k is even, < 1 or > 63 (Sec. 2 requires odd k) */
  DBG_E_OFFSETS = 3,    /* offsets not monotone, offsets[0] != 0 or offsets[n] != n_bases */
  DBG_E_OVERFLOW = 4,   /* more keys than max_keys, or max_keys >= 2^32 */
  DBG_E_CAPACITY = 5,   /* more distinct nodes or edges than the output capacity */
  DBG_E_WORKSPACE = 6,  /* workspace smaller than dbg_workspace_bytes() */
  DBG_E_HIP = 7,        /* a HIP launch failed */
  DBG_E_BASE = 8,       /* a byte other than A, C, G, T (either case) */
  DBG_E_ARG = 9,        /* other invalid argument (e.g. n_sets == 0) */
  DBG_E_INTERNAL = 10,  /* internal list capacity exceeded (a bug) */
  DBG_E_SCRATCH = 11    /* dbg_build_noalloc: the build needs more than its static scratch */
} dbg_status;

/* Node table outputs (device).  kmer: capacity rows of one uint64_t (k <= 31) or
 * two (k >= 33).  count: capacity uint32_t. */
typedef struct {
  void *kmer;
  uint32_t *count;
  uint64_t capacity;
} dbg_nodes_t;

/* Edge list outputs (device).  u, v: capacity rows, same width as node keys.
 * orient: capacity bytes.  mult: capacity uint32_t.  zkey: optional (NULL to
 * skip), capacity rows of the canonical (k+1)-mer, one uint64_t (k <= 31) or two
 * (k >= 33). */
typedef struct {
  void *u;
  void *v;
  uint8_t *orient;
  uint32_t *mult;
  void *zkey;
  uint64_t capacity;
} dbg_edges_t;

/* Device-resident result record, written at the end of a build. */
typedef struct {
  uint64_t n_nodes; /* distinct canonical k-mers (true count, even beyond capacity) */
  uint64_t n_edges; /* distinct canonical edges */
  uint32_t status;  /* DBG_OK or the first device-side error */
  uint32_t flags;   /* DBG_FLAG_* bits describing how the build ran */
} dbg_result_t;

/* dbg_result_t.flags: the node table was built from the edge endpoints (see
 * dbg_tuning_t) rather than from the enumerated k-mers. */
#define DBG_FLAG_NODES_FROM_ENDPOINTS 1u

/* Bytes of device workspace a build needs.  n_reads, n_sets as passed to the
 * build; max_keys is an upper bound on the number of k-mer positions
 * (sum over reads of max(0, L - k + 1)); n_bases is always a valid bound.
 * Returns 0 for invalid k. */
size_t dbg_workspace_bytes(uint64_t n_reads, uint64_t n_sets, uint64_t max_keys, int k);

/* Exact worst case of a build's table sizes, on the host: the k-mer positions
 * (sum over reads of max(0, L - k + 1), Sec. 4's n) and the (k+1)-mer positions
 * (sum of max(0, L - k)) of reads given by host offsets[n_reads + 1].  Every
 * node is one position's canonical k-mer and every edge one position's record,
 * so capacities of these sizes always hold the tables; max_nodes is also the
 * max_keys bound of dbg_workspace_bytes / dbg_build.  Errors: DBG_E_NULL,
 * DBG_E_K, DBG_E_OFFSETS (offsets[0] != 0 or decreasing). */
int dbg_bounds(const uint64_t *read_offsets, uint64_t n_reads, int k, uint64_t *max_nodes,
               uint64_t *max_edges);

/* Build the graph of one read set (Sec. 3, BiConstruct STEP-1 to STEP-3).
 *   packed        device, ceil(n_bases / 32) words (layout above)
 *   n_bases       bases in the stream (= read_offsets[n_reads])
 *   read_offsets  device, n_reads + 1 base offsets, read_offsets[0] = 0
 *   max_keys      bound used for the workspace (see dbg_workspace_bytes), < 2^32
 *   nodes, edges  host structs holding device output pointers and capacities;
 *                 full output needs capacity >= the distinct count (always
 *                 enough: capacity >= max_keys)
 *   result        device dbg_result_t
 *   workspace     device, >= dbg_workspace_bytes(n_reads, 1, max_keys, k) bytes,
 *                 256-byte aligned; its contents are clobbered. */
int dbg_build(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
              uint64_t n_reads, int k, uint64_t max_keys, const dbg_nodes_t *nodes,
              const dbg_edges_t *edges, dbg_result_t *result, void *workspace,
              size_t workspace_bytes, hipStream_t stream);

/* No-allocation build, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it).  The
 * same build as dbg_build, launch for launch, with the workspace taken from a
 * static device array of DBG_NOALLOC_SCRATCH_BYTES bytes that the library holds
 * on every device it runs on until the process ends; the caller still passes
 * the inputs, the output tables and the result record.  A build that needs more
 * workspace than that (dbg_workspace_bytes(n_reads, 1, max_keys, k) above
 * DBG_NOALLOC_SCRATCH_BYTES: about 2.8 M k-mer positions for k <= 31 and 1.6 M
 * for k >= 33, with reads of 100-150 bases) returns DBG_E_SCRATCH and enqueues
 * nothing.  Every call on a device shares that device's array and leaves its
 * contents behind (each build initialises what it reads): calls in stream
 * order on one stream are safe,
 * calls that overlap on one device (other streams, other threads) race and
 * must not be issued.  The first call on a device looks up the array's address
 * there (DBG_E_HIP if that fails); nothing is allocated or freed.  Other errors
 * as dbg_build. */
#define DBG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int dbg_build_noalloc(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, int k, uint64_t max_keys, const dbg_nodes_t *nodes,
                      const dbg_edges_t *edges, dbg_result_t *result, hipStream_t stream);

/* Build the graphs of n_sets independent read sets in one launch sequence.  Set s
 * is reads [set_read_offsets[s], set_read_offsets[s+1]) of the same stream
 * (device array, n_sets + 1 entries, first 0, last n_reads).  Outputs are the
 * per-set tables concatenated in set order; node_set_offsets / edge_set_offsets
 * (device, n_sets + 1 entries each) receive where each set's rows begin.  Each
 * set's rows are exactly what dbg_build gives for that set alone. */
int dbg_build_batched(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, const uint64_t *set_read_offsets, uint64_t n_sets,
                      int k, uint64_t max_keys, const dbg_nodes_t *nodes,
                      const dbg_edges_t *edges, uint64_t *node_set_offsets,
                      uint64_t *edge_set_offsets, dbg_result_t *result, void *workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* Pack ASCII bases (device, n_bases bytes of A/C/G/T, either case) into the
 * 2-bit stream (device, ceil(n_bases / 32) words; bits past the last base are 0):
 * the reads are strings over the four-letter DNA alphabet of Sec. 1 and Sec. 2,
 * coded A=0, C=1, G=2, T=3 so that numeric order is the lexicographic order of
 * Fig. 2 (the canonical k-mer is the smaller of the pair in that order).
 * A byte outside {A,C,G,T,a,c,g,t} sets result->status = DBG_E_BASE (result is
 * device memory; its other fields are untouched). */
int dbg_pack_ascii(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed,
                   dbg_result_t *result, hipStream_t stream);

/* Profiling aid.  When `events` is non-null, every later build records
 * events[i] (hipEvent_t handles created by the caller) on its stream at fixed
 * stage boundaries, DBG_STAGE_EVENTS per build: for the edge table (base 0)
 * and then the node table (base DBG_STAGE_EVENTS / 2),
 *   base+0 table start             base+6  after the digit-range bucket sort
 *   base+1 after key offsets               of the in-tile level (one kernel)
 *   base+2 after the enumeration   base+7  after the remaining partition levels
 *          histogram (one kernel)  base+8  after the LDS bucket sort of the
 *   base+3 after bucket planning           other batches (one kernel)
 *          (and the node table's   base+9  after run counting
 *          records from edge       base+10 after the run-length write (one
 *          endpoints, when taken)          kernel)
 *   base+4 after the enumeration   base+11 table end
 *          scatter (one kernel)
 *   base+5 after the partition levels up to the in-tile level (equal to
 *          base+6 when the build has no in-tile level)
 * n_events must be >= DBG_STAGE_EVENTS.  Process-wide setting, meant for
 * single-stream benchmarking; pass NULL to stop recording. */
#define DBG_STAGE_EVENTS 24
int dbg_set_stage_events(hipEvent_t *events, int n_events);

/* How the node table is built.  STEP-3 of Sec. 3 gives the node set as the
 * endpoints of the distinct edges; with counts this is: every k-mer occurrence
 * is the first k-mer or the last k-mer of a (k+1)-mer occurrence, or both ends
 * of a read, so twice a node's count equals the sum, over the distinct edges,
 * of the edge multiplicity for each endpoint equal to the node, plus the number
 * of reads that begin with the node and the number that end with it.
 *   DBG_NODES_KMERS      enumerate every k-mer of every read and sort them;
 *   DBG_NODES_ENDPOINTS  sort 2 records per distinct edge (endpoint, weight =
 *                        multiplicity) and 2 per read (its end k-mers, weight
 *                        1), sum the weights and halve them;
 *   DBG_NODES_AUTO       endpoints when their records number at most
 *                        `endpoint_ratio` times the k-mers.
 * Both give identical tables.  The endpoint route is taken only by single-set
 * builds whose edge table fitted its capacity, that had at least one edge, and
 * whose records fit the workspace's key buffers (records <= 8/12 of max_keys
 * for k <= 31, 16/20 for k >= 33); otherwise the k-mers are enumerated. */
typedef enum {
  DBG_NODES_AUTO = -1,
  DBG_NODES_KMERS = 0,
  DBG_NODES_ENDPOINTS = 1
} dbg_node_path;

typedef struct {
  int node_path;        /* dbg_node_path; default DBG_NODES_AUTO */
  float endpoint_ratio; /* for DBG_NODES_AUTO; default 0.6 */
  /* Shape of the LDS bucket sort: 0 = 512-thread workgroups holding up to 6,144
   * keys (64-bit; 3,072 for 128-bit keys), one per CU; 1 = 256-thread
   * workgroups holding half as many, two per CU; 2 = the batch of 0 with more
   * threads: 768 for 64-bit keys (three waves per SIMD instead of two), 1,024
   * for 128-bit keys (four instead of two).  Default 2. */
  int local_variant;
  /* Added to the width of the first partition of each batch's distinct keys
   * (normally log2 of their number, 8 to 11 bits), in [-3, 3].  Default 0. */
  int lds_digit_bias;
  /* 128-bit keys: 1 = at the first partition level whose buckets average at
   * most 65,536 keys per read set, buckets of at most 64 tiles of 4,096 keys are
   * split within each tile (one read and one write of their keys, no histogram
   * pass and no global cursors) and the bucket sort reads each digit range as
   * one segment per tile; 0 = every level scatters through global cursors.
   * Default 1. */
  int in_tile;
  int reserved[3];      /* zero */
} dbg_tuning_t;

/* Process-wide tuning read by every later build call (calls in flight keep the
 * values they started with).  NULL restores the defaults.  Every setting gives
 * the same tables; only the time changes.  Returns DBG_E_ARG for an unknown
 * node_path or local_variant, a ratio outside [0, 2], a bias outside [-3, 3] or
 * an in_tile other than 0 or 1. */
int dbg_set_tuning(const dbg_tuning_t *tuning);
/* Copies the current tuning into *tuning (DBG_E_NULL if null). */
int dbg_get_tuning(dbg_tuning_t *tuning);

/* Key-space slices (the out-of-memory build, Sec. 6).  The paper sorts more
 * keys than fit in memory as sorted runs merged R ways.  Here a build keeps only
 * the keys whose top DBG_PREFIX_BITS bits (the prefix of the canonical
 * (k+1)-mer for the edge table, of the canonical k-mer for the node table) lie
 * in [prefix_lo, prefix_hi).  Slices of disjoint, increasing prefix ranges give
 * disjoint, increasing parts of both sorted tables, so the tables of a sequence
 * of slices covering [0, DBG_PREFIX_BINS) concatenate to the full tables: no
 * merge.  Each slice re-reads the packed reads (2 bits per base) and needs key
 * buffers only for its own keys.
 *
 * dbg_prefix_counts: edge_counts / node_counts (device, DBG_PREFIX_BINS uint64_t
 * each) receive the number of (k+1)-mer / k-mer positions of each prefix, from
 * which a caller plans slices that fit a key budget.  max_positions bounds the
 * k-mer positions (n_bases always does); result->status reports DBG_E_OFFSETS
 * or DBG_E_OVERFLOW.  Workspace: dbg_prefix_workspace_bytes.
 *
 * dbg_build_slice: dbg_build restricted to the prefixes [prefix_lo, prefix_hi);
 * max_positions bounds the positions (as max_keys does for dbg_build), max_keys
 * the keys each table keeps (result->status = DBG_E_OVERFLOW when a table has
 * more; the slice must then be split).  The node table always enumerates
 * k-mers (the edge-endpoint route needs the whole edge table).  Host errors as
 * dbg_build, and DBG_E_ARG for max_keys > max_positions or a bad range.
 * Workspace: dbg_slice_workspace_bytes.  Both enqueue on `stream` and never
 * synchronise or allocate. */
#define DBG_PREFIX_BITS 12
#define DBG_PREFIX_BINS (1u << DBG_PREFIX_BITS)
size_t dbg_prefix_workspace_bytes(uint64_t n_reads, uint64_t max_positions, int k);
int dbg_prefix_counts(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                      uint64_t n_reads, int k, uint64_t max_positions, uint64_t *edge_counts,
                      uint64_t *node_counts, dbg_result_t *result, void *workspace,
                      size_t workspace_bytes, hipStream_t stream);
size_t dbg_slice_workspace_bytes(uint64_t n_reads, uint64_t max_positions, uint64_t max_keys,
                                 int k);
int dbg_build_slice(const uint64_t *packed, uint64_t n_bases, const uint64_t *read_offsets,
                    uint64_t n_reads, int k, uint64_t max_positions, uint64_t max_keys,
                    uint32_t prefix_lo, uint32_t prefix_hi, const dbg_nodes_t *nodes,
                    const dbg_edges_t *edges, dbg_result_t *result, void *workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* STEP-4 of Sec. 3: adjacency lists of a built graph.  A node has two sides:
 * side 0, by which a walk reading its canonical k-mer forward leaves it, and
 * side 1, by which such a walk enters it.  A distinct edge (u, v, o1, o2) leaves
 * u by side o1 and enters v by side 1 - o2 ('+' = 0, '-' = 1), so its u end lies
 * on side o1 of u and its v end on side 1 - o2 of v; a self-loop gives its node
 * two ends.  (The sides are the same when the record is written with its
 * endpoints swapped, as the STEP-1 table's ELSE branches do, and a walk through
 * a node uses one end on each side: the walk rule of Sec. 2.)  The lists group
 * the ends by (node, side) -- nodes in node-table order, side 0 first -- and
 * order each group by edge row, u end first.  Output as a CSR over the 2 n_nodes
 * buckets b = 2 * node + side:
 *   offsets   device, 2 n_nodes + 1 uint64_t: bucket b holds entries
 *             offsets[b] .. offsets[b + 1] - 1;
 *   inc_edge  device, 2 n_edges uint32_t: edge row of each entry;
 *   inc_end   device, 2 n_edges bytes: 0 for the u end, 1 for the v end;
 *   edge_bucket device, 2 n_edges uint32_t, or NULL: the buckets of the u end
 *             and the v end of every edge (edge_bucket[2 j], edge_bucket[2 j + 1];
 *             node row = bucket >> 1, side = bucket & 1).
 * Inputs are a build's tables (device): node_kmer (n_nodes keys, ascending),
 * edge_u / edge_v / edge_orient (n_edges rows), key width as in dbg_build; the
 * counts are the build's n_nodes / n_edges (read from its result record).
 * result (device) receives status DBG_OK, or DBG_E_ARG when an edge endpoint is
 * not in the node table or a (node, side) holds more than 256 ends (a side of a
 * read set's k-mer holds at most 8: four one-base extensions, two ends each);
 * then the entries are not written.  Host errors:
 * DBG_E_K, DBG_E_NULL, DBG_E_ARG (edges without nodes), DBG_E_OVERFLOW
 * (n_nodes >= 2^31 or n_edges >= 2^32), DBG_E_WORKSPACE.  Enqueues on `stream`,
 * never synchronises or allocates. */
size_t dbg_adjacency_workspace_bytes(uint64_t n_nodes, uint64_t n_edges, int k);
int dbg_adjacency(const void *node_kmer, uint64_t n_nodes, const void *edge_u,
                  const void *edge_v, const uint8_t *edge_orient, uint64_t n_edges, int k,
                  uint64_t *offsets, uint32_t *inc_edge, uint8_t *inc_end, uint32_t *edge_bucket,
                  dbg_result_t *result, void *workspace, size_t workspace_bytes,
                  hipStream_t stream);

/* Bi-directed chain compaction (Sec. 7): the simplified graph of a built graph.
 * Sides are those of dbg_adjacency.  An edge is a candidate when it is not a
 * self-loop and each of its ends is the only end on its side (the paper's "one
 * in- and one out-edge" criterion, read per edge end).  ListRankingTransform
 * gives every node v a forward copy v+ and a reverse-complement copy v-; the
 * candidates link the copies into lists and cycles, which are ranked by pointer
 * jumping; a cycle is broken at its smallest node, starting at v+.  Of a chain's
 * two copies the one whose first k-mer is smaller is kept (for a broken cycle,
 * the one starting at v+).  Chains shorter than min_nodes are not merged (the
 * paper keeps chains of three or more nodes; 0 and 1 keep all).
 *
 * Output (device buffers owned by the caller):
 *   node_chain, node_rank  n_nodes uint32_t: chain of every node and its
 *                          position along the chain's walk;
 *   node_orient            n_nodes bytes: 0 when the walk reads the node's
 *                          canonical k-mer forward, 1 when reverse-complemented;
 *   chain_head, chain_len  capacity n_nodes uint32_t: first node (row) and node
 *                          count of every chain; chains are numbered in the order
 *                          of their first node, a node alone is a chain of one;
 *   chain_cyclic           capacity n_nodes bytes: 1 for a broken cycle;
 *   label_offsets          n_nodes + 1 uint64_t: chain c spells
 *                          labels[label_offsets[c] .. label_offsets[c + 1]),
 *                          k + chain_len - 1 ASCII bases (A, C, G, T);
 *   labels, label_capacity at most label_capacity bytes (n_chains * (k - 1) +
 *                          n_nodes are written; n_nodes * k always suffices);
 *   kept_row, kept_u,      capacity n_edges: every edge that is not merged into
 *   kept_v, kept_orient    a chain, in row order: its row, the chains of its u
 *                          and v ends, and (o1 << 1) | o2 on chain sides (an end
 *                          on side s of a node with orientation t lies on side
 *                          s xor t of its chain; o1 = side at u, o2 = 1 - side
 *                          at v, as in the input edges).
 * Inputs (device): the build's node_kmer (ascending) with the true node and edge
 * counts, and dbg_adjacency's offsets, inc_edge, inc_end and edge_bucket of the
 * same graph (the edge sides come from the buckets).  result (device) receives n_chains, n_kept, label_len,
 * n_cyclic (cycles broken, before min_nodes) and status: DBG_OK, DBG_E_ARG (an
 * input row out of range), DBG_E_CAPACITY (labels longer than label_capacity:
 * no label byte written) or DBG_E_INTERNAL (ranking did not finish: a bug).
 * Host errors: DBG_E_K, DBG_E_NULL, DBG_E_ARG (edges without nodes),
 * DBG_E_OVERFLOW (n_nodes >= 2^31 or n_edges >= 2^32), DBG_E_WORKSPACE.
 * Enqueues on `stream`, never synchronises or allocates. */
typedef struct {
  uint32_t *node_chain;
  uint32_t *node_rank;
  uint8_t *node_orient;
  uint32_t *chain_head;
  uint32_t *chain_len;
  uint8_t *chain_cyclic;
  uint64_t *label_offsets;
  uint8_t *labels;
  uint64_t label_capacity;
  uint32_t *kept_row;
  uint32_t *kept_u;
  uint32_t *kept_v;
  uint8_t *kept_orient;
} dbg_chains_t;

typedef struct {
  uint64_t n_chains;  /* chains, single nodes included */
  uint64_t n_kept;    /* edges not merged into a chain */
  uint64_t label_len; /* bases of all labels */
  uint64_t n_cyclic;  /* cycles broken open (before min_nodes) */
  uint32_t status;
  uint32_t pad;
} dbg_compact_result_t;

size_t dbg_compact_workspace_bytes(uint64_t n_nodes, uint64_t n_edges);
int dbg_compact(const void *node_kmer, uint64_t n_nodes, uint64_t n_edges, int k,
                const uint64_t *adj_offsets, const uint32_t *inc_edge, const uint8_t *inc_end,
                const uint32_t *edge_bucket, uint32_t min_nodes,
                const dbg_chains_t *out, dbg_compact_result_t *result, void *workspace,
                size_t workspace_bytes, hipStream_t stream);

/* Static description of a status code. */
const char *dbg_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* DBG_H */
