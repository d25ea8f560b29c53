/*
 * bvs.h - C ABI of the MI355X (gfx950) vector-set search library.
 *
 * The library implements the data-parallel hot path of the cascade search
 * for vector sets under the Hausdorff distance:
 *
 *   FlyHash encoding      h = WTA(W v), W a sparse 0/1 random projection into
 *                         L = code_bits outputs, WTA keeping the wta_k largest
 *                         (Def. 7; Alg. 1)
 *   set sketches          count Bloom filter C = sum of member codes (Def. 8,
 *                         Alg. 3) and binary Bloom filter B = OR of member
 *                         codes, used as the set sketch (Def. 10, Alg. 5)
 *   filtering             first layer: sets with C[p] >= M at one of the A
 *                         largest positions p of the query's count filter;
 *                         second layer: the T sets of the first layer closest
 *                         to the query sketch in Hamming distance (Alg. 6)
 *   re-ranking            exact Hausdorff distance (Def. 4) to the T
 *                         survivors and the k smallest (Alg. 6, Def. 5)
 *   brute force           exact Hausdorff distance to every set, k smallest
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are device pointers, h_* are host pointers.  The
 *   library never allocates device memory: the caller passes the index
 *   memory, workspaces and outputs, sized with the *_bytes queries, and
 *   owns them (bvs_search_noalloc alone uses a fixed array that the
 *   library's code object holds on each GPU).  The library keeps no host
 *   pointer after a call returns.
 * - Every call returns a bvs_status; bvs_last_error() gives a thread-local
 *   message for the last non-OK status.  Argument errors are detected on
 *   the host before anything is launched.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is enqueued on it.  Calls that validate device data
 *   (bvs_build_index, bvs_encode, bvs_search, bvs_search_candidates,
 *   bvs_query_sketch, bvs_bruteforce, bvs_hausdorff_all) synchronise the
 *   stream before returning so that they can report BVS_ERANGE.
 * - Vectors are float32 rows [n][dim], row-major.  Every value must lie on
 *   the 2^-12 grid (4096 * x is an integer) with |x| <= 1, and every row
 *   must have Euclidean norm <= 2; otherwise BVS_ERANGE.  On this grid the
 *   projection sums, squared distances and rankings are exact integers.
 * - Sets are given by offsets [n_sets + 1] (host, uint64): set j holds rows
 *   offsets[j] .. offsets[j+1]-1; offsets[0] = 0 and offsets must strictly
 *   increase (a set has at least one vector, Def. 2).  A set id is its
 *   position j.  Database sets hold at most 255 vectors, query sets at most
 *   65535 (BVS_ERANGE otherwise); calls that compute Hausdorff distances
 *   take query sets of at most 256 vectors (BVS_ENOTSUP otherwise).
 * - Results are sorted ascending by (distance, id); distances are Euclidean
 *   (not squared), float32.  With fewer than k results, count[q] says how
 *   many are valid and the rest are id = 0xFFFFFFFF, distance = +inf.
 * - The index is immutable after build; concurrent searches on one index
 *   with distinct workspaces are allowed.  Outputs depend only on the data,
 *   the parameters and the query, never on batch composition or stream.
 */
#ifndef BVS_H
#define BVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BVS_OK = 0,
  BVS_EINVAL = -1,   /* invalid argument (null pointer, bad size, bad offsets) */
  BVS_ERANGE = -2,   /* data outside the supported range (grid, norm, set size) */
  BVS_ENOSPC = -3,   /* index memory or workspace smaller than required */
  BVS_EDEVICE = -4,  /* a HIP call failed */
  BVS_ESTATE = -5,   /* object in the wrong state */
  BVS_ENOTSUP = -6   /* parameter combination not supported by the kernels */
} bvs_status;

/* Parameters Theta of Alg. 6 plus the hashing parameters of Def. 7.
 *   dim           d, 1..1024
 *   code_bits     L (the Bloom filter length b equals L): a power of two,
 *                 256..4096
 *   fan_in        s, input dimensions summed per projection output, 1..d;
 *                 L * s <= 65536 and the WTA key must fit 32 bits
 *                 (s * 8192 < 2^(32 - log2 L))
 *   wta_k         L_wta, ones per code, 1..L
 *   access_lists  A, inverted lists (positions) visited, 1..8
 *   min_count     M, minimum count in the first layer, 0..255
 *   top_t         T, survivors of the second layer, 1..4096
 *   flags         must be 0
 *   seed          seed of the projection (see bvs_projection) */
typedef struct bvs_params {
  uint32_t dim;
  uint32_t code_bits;
  uint32_t fan_in;
  uint32_t wta_k;
  uint32_t access_lists;
  uint32_t min_count;
  uint32_t top_t;
  uint32_t flags;
  uint64_t seed;
} bvs_params;

typedef struct bvs_index bvs_index;  /* opaque host handle */

typedef struct bvs_index_info {
  uint64_t n_sets;       /* n */
  uint64_t n_vectors;    /* N */
  uint64_t ld_sets;      /* leading dimension of the sketch views (n rounded up to 256) */
  uint32_t dim_padded;   /* d rounded up to 64 (row stride of the internal planes) */
  uint32_t max_set_size;
} bvs_index_info;

/* Fills *p with defaults: L = 1024, wta_k = 64, A = 3 and M = 1 are the
 * paper's defaults (Sec. 6.1.5); s = 8 and T = 1000 are this library's
 * (the paper's default of 50k candidates exceeds the T limit above);
 * dim is left 0 and must be set. */
void bvs_params_default(bvs_params* p);

/* Checks a parameter block; BVS_EINVAL / BVS_ENOTSUP with a message. */
bvs_status bvs_params_check(const bvs_params* p);

/* The random projection W of Def. 7 as index rows, host only.
 * h_idx[L][s] (uint16): the s distinct input dimensions of output j, sorted
 * ascending.  Construction: one splitmix64 stream seeded with p->seed; each
 * draw u gives i = ((u >> 32) * d) >> 32; a dimension already in the row is
 * redrawn; rows are filled in order 0..L-1. */
bvs_status bvs_projection(const bvs_params* p, uint16_t* h_idx);

/* Device bytes of the index for n_sets sets holding n_vectors vectors. */
bvs_status bvs_index_bytes(const bvs_params* p, uint64_t n_sets, uint64_t n_vectors,
                           uint64_t* out_bytes);
/* Device workspace bytes needed by bvs_build_index (released after it). */
bvs_status bvs_build_workspace_bytes(const bvs_params* p, uint64_t n_sets,
                                     uint64_t n_vectors, uint64_t* out_bytes);

/* Builds the index (Algs. 1, 3, 5): validates and converts the vectors,
 * encodes every vector and writes the per-set count Bloom filters
 * (uint8 [L][ld_sets], position-major) and binary Bloom filters
 * (chunk-major: 128-bit chunk c of set j at word offset 2*(c*ld_sets + j)).
 * d_vectors: float32 [n_vectors][dim]; h_offsets: [n_sets + 1].
 * The index keeps its own exact copy of the vectors; d_vectors may be freed
 * after the call.  d_index_mem must stay valid while the index is used.
 * On success *out receives a handle to release with bvs_index_destroy. */
bvs_status bvs_build_index(const bvs_params* p, const float* d_vectors,
                           const uint64_t* h_offsets, uint64_t n_sets,
                           void* d_index_mem, uint64_t index_bytes,
                           void* d_workspace, uint64_t workspace_bytes,
                           void* stream, bvs_index** out);

/* Releases the host handle (the caller frees the device memory). */
void bvs_index_destroy(bvs_index* ix);

/* Changes the search-time parameters of Alg. 6 of a built index: A
 * (access_lists), M (min_count) and T (top_t).  The sketches and bitmaps of
 * the index do not depend on them, so no rebuild is needed; they are
 * validated as by bvs_params_check (BVS_EINVAL / BVS_ENOTSUP, index
 * unchanged).  The index is otherwise immutable: this call must not overlap
 * any other call on the index, workspaces must be sized again afterwards,
 * and batched plans created before it must be created again. */
bvs_status bvs_index_set_search_params(bvs_index* ix, uint32_t access_lists, uint32_t min_count,
                                       uint32_t top_t);

bvs_status bvs_index_get_info(const bvs_index* ix, bvs_index_info* info);
bvs_status bvs_index_get_params(const bvs_index* ix, bvs_params* p);

/* Device views of the sketches (Defs. 8 and 10) for inspection:
 *   *d_count: uint8 [L][ld_sets]; entry (i, j) = C^(j)[i]
 *   *d_bits:  uint64 [L/128][ld_sets][2]; bit i of set j is bit (i % 64) of
 *             word (i % 128) / 64 of chunk i / 128.
 * Columns j >= n_sets are zero. */
bvs_status bvs_sketch_views(const bvs_index* ix, const uint8_t** d_count,
                            const uint64_t** d_bits);

/* Workspace bytes for bvs_encode on n vectors. */
bvs_status bvs_encode_workspace_bytes(const bvs_index* ix, uint64_t n, uint64_t* out_bytes);
/* FlyHash codes (Def. 7, Alg. 1) of arbitrary vectors with the index's
 * projection: d_codes uint64 [n][L/64], output j is bit j % 64 of word j / 64. */
bvs_status bvs_encode(const bvs_index* ix, const float* d_x, uint64_t n,
                      void* d_workspace, uint64_t workspace_bytes,
                      uint64_t* d_codes, void* stream);

/* Workspace bytes for bvs_search, bvs_search_candidates and bvs_query_sketch
 * on n_q query sets holding n_q_vectors vectors in total. */
bvs_status bvs_search_workspace_bytes(const bvs_index* ix, uint32_t n_q,
                                      uint64_t n_q_vectors, uint64_t* out_bytes);

/* Query-side preparation of Alg. 6: the query count filter C_Q
 * (d_cq uint16 [n_q][L]), the query sketch S_Q (d_sq uint64 [n_q][L/64])
 * and the A positions of largest count, ties to the lower position
 * (d_pos uint32 [n_q][A]).  Any output pointer may be NULL. */
bvs_status bvs_query_sketch(const bvs_index* ix, const float* d_q,
                            const uint64_t* h_q_offsets, uint32_t n_q,
                            void* d_workspace, uint64_t workspace_bytes,
                            uint16_t* d_cq, uint64_t* d_sq, uint32_t* d_pos,
                            void* stream);

/* Both filter layers of Alg. 6: F2 of every query, sorted by (score, id).
 * d_ids uint32 [n_q][T], d_scores uint16 [n_q][T], d_count uint32 [n_q]
 * (= min(T, |F1|)); unused slots are id 0xFFFFFFFF, score 0xFFFF. */
bvs_status bvs_search_candidates(const bvs_index* ix, const float* d_q,
                                 const uint64_t* h_q_offsets, uint32_t n_q,
                                 void* d_workspace, uint64_t workspace_bytes,
                                 uint32_t* d_ids, uint16_t* d_scores,
                                 uint32_t* d_count, void* stream);

/* The whole cascade search (Alg. 6): top-k (k <= T, k <= 64) of every
 * query.  d_ids uint32 [n_q][k], d_dist float32 [n_q][k], d_count uint32 [n_q]. */
bvs_status bvs_search(const bvs_index* ix, const float* d_q,
                      const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                      void* d_workspace, uint64_t workspace_bytes,
                      uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                      void* stream);

/* bvs_search for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same search, identical outputs, with its workspace taken from a fixed
 * array of bvs_search_noalloc_max_bytes() = 64 MiB that the library holds in
 * device memory on every GPU it runs on until the process ends.  No device
 * or host-pinned memory is allocated, no stage events are recorded and no
 * work counters are collected.  The call runs on the current device, which
 * must be the index's (BVS_ESTATE otherwise); a batch whose bvs_search
 * workspace (bvs_search_workspace_bytes) exceeds 64 MiB is rejected with
 * BVS_ENOSPC before anything is launched.  Every call on one GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller; each call
 * clears what it needs before use, so successive calls are independent.
 * Synchronises `stream` like bvs_search. */
uint64_t bvs_search_noalloc_max_bytes(void);
bvs_status bvs_search_noalloc(const bvs_index* ix, const float* d_q,
                              const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                              uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                              void* stream);

/* Workspace bytes for bvs_bruteforce / bvs_hausdorff_all. */
bvs_status bvs_bruteforce_workspace_bytes(const bvs_index* ix, uint32_t n_q,
                                          uint64_t n_q_vectors, uint64_t* out_bytes);

/* Exact top-k (k <= 64) by Hausdorff distance over every set (Def. 5 with
 * failure probability 0); outputs as for bvs_search. */
bvs_status bvs_bruteforce(const bvs_index* ix, const float* d_q,
                          const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                          void* d_workspace, uint64_t workspace_bytes,
                          uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                          void* stream);

/* Exact squared Hausdorff distance (Def. 4) of every query to every set,
 * scaled by 2^24 (an integer on the grid): d_h2 uint32 [n_q][n_sets]. */
bvs_status bvs_hausdorff_all(const bvs_index* ix, const float* d_q,
                             const uint64_t* h_q_offsets, uint32_t n_q,
                             void* d_workspace, uint64_t workspace_bytes,
                             uint32_t* d_h2, void* stream);

/* ------------------------------------------------------------------------
 * Other set measures in the re-rank (Sec. 3.2, where the paper compares
 * them with the Hausdorff distance; Sec. 6 reports search with MeanMin).
 * Only the aggregation of the exact pairwise distances changes:
 *   BVS_METRIC_HAUSDORFF  Def. 4 (what bvs_search and bvs_bruteforce use)
 *   BVS_METRIC_MEANMIN    (1 / |Q|) sum over q in Q of min over v in V of
 *                         |q - v|: the MeanMin distance from the query set
 *                         to the database set (not symmetric)
 *   BVS_METRIC_MIN        min over q in Q, v in V of |q - v|
 * The filter layers are unchanged (F2 as for bvs_search); every candidate of
 * F2 is measured in full (no bound or screen applies to these measures).
 * Min distances are exact (the square root of an exact integer, as for
 * Hausdorff).  MeanMin is a mean of square roots: each sqrt of the exact
 * 2^24-scaled squared distance is taken in float64, summed in float64 and
 * divided by |Q|, then rounded once to float32; results are ranked by that
 * float32 value, ties to the lower id.  Outputs, workspaces and errors as
 * for bvs_search / bvs_bruteforce; BVS_EINVAL for an unknown metric. */
#define BVS_METRIC_HAUSDORFF 0
#define BVS_METRIC_MEANMIN 1
#define BVS_METRIC_MIN 2
bvs_status bvs_search_metric(const bvs_index* ix, int metric, const float* d_q,
                             const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                             void* d_workspace, uint64_t workspace_bytes,
                             uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                             void* stream);
bvs_status bvs_bruteforce_metric(const bvs_index* ix, int metric, const float* d_q,
                                 const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                                 void* d_workspace, uint64_t workspace_bytes,
                                 uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                                 void* stream);

/* ------------------------------------------------------------------------
 * Full-scan search (Alg. 2, the paper's first method): every set is scored
 * by Haus^H, Def. 4 with the Hamming distance between FlyHash codes (Def. 7)
 * in place of the Euclidean distance, the first c = top_t sets by
 * (Haus^H, id) are kept (Alg. 2 keeps every set at most the c-th smallest;
 * ties beyond c go to the lower ids), and those are re-ranked by the exact
 * Hausdorff distance as in bvs_search.  It needs the codes of every database
 * vector, kept in sparse form (the wta_k positions of each code, uint16,
 * rows padded to a multiple of 8) in caller memory attached to the index:
 *   bvs_codes_bytes      device bytes of that memory: N rows of the padded
 *                        positions, and the set ids ordered by size
 *   bvs_codes_attach     encodes every vector of the index (random or
 *                        learned projection) into d_mem, using a workspace of
 *                        bvs_codes_attach_workspace_bytes; synchronises; the
 *                        memory must outlive the index's use of the full
 *                        scan; attaching again replaces it.  wta_k must be at
 *                        most 255 (BVS_ENOTSUP).
 * The search calls return BVS_ESTATE when nothing is attached and take a
 * workspace of bvs_search_full_workspace_bytes.
 *   bvs_full_scores            Haus^H of every query to every set:
 *                              d_scores uint16 [n_q][n_sets]
 *   bvs_search_full_candidates F of every query: ids, scores and count as
 *                              for bvs_search_candidates (top_t slots)
 *   bvs_search_full            the whole of Alg. 2; outputs as bvs_search */
bvs_status bvs_codes_bytes(const bvs_index* ix, uint64_t* out_bytes);
bvs_status bvs_codes_attach_workspace_bytes(const bvs_index* ix, uint64_t* out_bytes);
bvs_status bvs_codes_attach(bvs_index* ix, void* d_mem, uint64_t bytes,
                            void* d_workspace, uint64_t workspace_bytes, void* stream);
bvs_status bvs_search_full_workspace_bytes(const bvs_index* ix, uint32_t n_q,
                                           uint64_t n_q_vectors, uint64_t* out_bytes);
bvs_status bvs_full_scores(const bvs_index* ix, const float* d_q,
                           const uint64_t* h_q_offsets, uint32_t n_q,
                           void* d_workspace, uint64_t workspace_bytes,
                           uint16_t* d_scores, void* stream);
bvs_status bvs_search_full_candidates(const bvs_index* ix, const float* d_q,
                                      const uint64_t* h_q_offsets, uint32_t n_q,
                                      void* d_workspace, uint64_t workspace_bytes,
                                      uint32_t* d_ids, uint16_t* d_scores,
                                      uint32_t* d_count, void* stream);
bvs_status bvs_search_full(const bvs_index* ix, const float* d_q,
                           const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                           void* d_workspace, uint64_t workspace_bytes,
                           uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                           void* stream);

/* ------------------------------------------------------------------------
 * Inverted lists (Def. 9, Alg. 4) as the first filter layer.  By default the
 * first layer is read from position-major bitmaps (M = 1) or count columns
 * (M >= 2) of every set; with lists attached and BVS_FIRST_LAYER_LISTS
 * chosen, it is the union over the query's A positions of the prefixes of
 * count >= M of the inverted lists, which reads only those entries (the
 * difference matters when A times the list length is far below n).  Both
 * give the same F1 and therefore the same results.  List p holds the sets
 * with C^(j)[p] >= 1 ordered by decreasing count (equal counts in no
 * particular order, as in Alg. 4):
 *   cum   uint32 [L][257]   cum[p][c] = entries of list p with count >= c
 *   start uint64 [L + 1]    list p is ids[start[p] .. start[p + 1])
 *   ids   uint32 [nnz]      set ids; nnz = sum over sets of |B|
 * bvs_lists_bytes runs the counting pass (workspace of
 * bvs_lists_workspace_bytes; synchronises) and returns the device bytes of
 * the lists; bvs_lists_attach builds them into caller memory (which must
 * outlive their use) and synchronises.  bvs_index_set_first_layer selects
 * the source (BVS_ESTATE for lists when none are attached; with M = 0 every
 * set is a member and the lists are not read); like
 * bvs_index_set_search_params it must not overlap other calls on the index,
 * and workspaces must be sized again (lists mode adds n_q * ld / 8 bytes). */
#define BVS_FIRST_LAYER_BITMAPS 0
#define BVS_FIRST_LAYER_LISTS 1
bvs_status bvs_lists_workspace_bytes(const bvs_index* ix, uint64_t* out_bytes);
bvs_status bvs_lists_bytes(const bvs_index* ix, void* d_workspace, uint64_t workspace_bytes,
                           void* stream, uint64_t* out_bytes);
bvs_status bvs_lists_attach(bvs_index* ix, void* d_mem, uint64_t bytes,
                            void* d_workspace, uint64_t workspace_bytes, void* stream);
bvs_status bvs_lists_views(const bvs_index* ix, const uint32_t** d_cum,
                           const uint64_t** d_start, const uint32_t** d_ids, uint64_t* nnz);
bvs_status bvs_index_set_first_layer(bvs_index* ix, int mode);

/* ------------------------------------------------------------------------
 * Batched search: many query sets of uneven size through the whole cascade
 * (Alg. 6) with no host round trip.  The exact re-rank of every query runs
 * either in ONE persistent launch (resident workgroups take (query,
 * 64-candidate chunk) items from a device counter, largest queries first)
 * or as the phase sequence of bvs_search run once per size class of the
 * queries (up to 2, 4, 8 and 16 tiles of 16 vectors, each class with
 * kernels sized for it).  Results are identical to bvs_search on the same
 * queries (the cascade is exact given F2, and F2 is a function of the query
 * alone).
 *
 * Life cycle: bvs_batch_create (host only: validates the offsets, orders the
 * queries by size, sizes the workspace) -> bvs_batch_bind (uploads the
 * offsets, runs the autotuner when asked, and with config.graph captures
 * the whole launch sequence into a hipGraph; synchronises the stream) ->
 * bvs_batch_launch any number of times (enqueues the graph, or the launch
 * sequence; never synchronises) -> bvs_batch_status (synchronises and
 * reports BVS_ERANGE for off-grid query data of the last launch) ->
 * bvs_batch_destroy.  Between launches the caller may rewrite the query
 * vectors in place (same offsets); the bound buffers must stay valid until
 * the last launch has completed.  Graph capture needs a stream other than
 * the null stream.
 *
 * Autotuner: with lds_rows or waves = 0, bind times every valid shape of the
 * persistent re-rank, query rows staged in LDS in {32, 64, 128} x waves per
 * workgroup (sets in flight against one staged query, one wave per set) in
 * {2, 4, 8}, and (with both 0) the phase sequence by size class, reported
 * as shape 0 x 0, on the bound batch itself, after running the cascade up to
 * F2 once; shapes whose kernel spills registers or does not fit a CU are
 * skipped.  The fastest shape is cached per process for the shape class
 * (dim, T, k, largest query tile count, log2 n_q) and reused by later binds
 * of the same class without timing.
 */
typedef struct bvs_batch bvs_batch;

typedef struct bvs_batch_config {
  uint32_t lds_rows;   /* 16..256, multiple of 16; 0 = autotune */
  uint32_t waves;      /* 2, 4 or 8; 0 = autotune */
  uint32_t graph;      /* nonzero: capture the launch sequence at bind */
  uint32_t flags;      /* 0 or BVS_BATCH_PHASES */
} bvs_batch_config;

/* config.flags: re-rank with the phase sequence by size class, no tuning
 * (lds_rows and waves must then be 0). */
#define BVS_BATCH_PHASES 1u

#define BVS_TUNE_MAX 16
typedef struct bvs_batch_info {
  uint32_t n_q, max_rows;          /* queries, vectors in the largest */
  uint64_t n_q_vectors;            /* vectors over all queries */
  uint64_t workspace_bytes;        /* needed by bvs_batch_bind */
  uint32_t lds_rows, waves;        /* re-rank shape in use (0 before bind; 0 and 0:
                                      the phase sequence by size class) */
  uint32_t blocks;                 /* persistent workgroups launched (0: phases) */
  uint32_t from_cache;             /* shape taken from the tuner cache */
  uint32_t graph;                  /* launches replay a captured graph */
  uint32_t n_tried;                /* shapes timed by the tuner */
  uint32_t tried_lds_rows[BVS_TUNE_MAX];
  uint32_t tried_waves[BVS_TUNE_MAX];
  float tried_ms[BVS_TUNE_MAX];    /* re-rank time of each shape */
} bvs_batch_info;

/* Host only.  h_q_offsets [n_q + 1] is copied.  k as for bvs_search. */
bvs_status bvs_batch_create(const bvs_index* ix, const uint64_t* h_q_offsets,
                            uint32_t n_q, uint32_t k,
                            const bvs_batch_config* config, bvs_batch** out);

/* Binds device buffers: d_q float32 [n_q_vectors][dim], the workspace of
 * bvs_batch_info.workspace_bytes, and outputs as for bvs_search.  May be
 * called again to rebind (the previous graph is released). */
bvs_status bvs_batch_bind(bvs_batch* b, const float* d_q, void* d_workspace,
                          uint64_t workspace_bytes, uint32_t* d_ids,
                          float* d_dist, uint32_t* d_count, void* stream);

/* Enqueues one batched search on `stream`; BVS_ESTATE before bind. */
bvs_status bvs_batch_launch(bvs_batch* b, void* stream);

/* Synchronises `stream` and checks the last launch's query data. */
bvs_status bvs_batch_status(bvs_batch* b, void* stream);

bvs_status bvs_batch_get_info(const bvs_batch* b, bvs_batch_info* out);

/* Frees the plan and its graph (not the caller's buffers). */
void bvs_batch_destroy(bvs_batch* b);

/* ------------------------------------------------------------------------
 * Precision form of the re-rank.  The exact re-rank reads two int8 planes
 * per element and does four int8 matrix-core products per tile.  This form
 * first ranks F2 by approximate Hausdorff values computed from a BF16 or an
 * OCP FP8 E4M3 copy of the vectors (one matrix-core product per tile, FP32
 * accumulation), then re-checks exactly (the exact re-rank, which equals a
 * float64 evaluation) every candidate whose approximate distance is within
 * a relative margin of the k-th approximate distance, and returns the
 * first k of the re-checked candidates by exact distance.  Reported
 * distances are therefore exact; a true neighbour is missed only if its
 * approximate distance exceeds the k-th one by more than the margin.
 *
 * Encodings: BF16 = float32 rounded to nearest even to 16 bits; E4M3 = OCP
 * 8-bit float (bias 7, 3 mantissa bits, largest 448), rounded to nearest
 * even, with a float32 scale per set s = max|x| / 448 and components
 * e4m3(clamp(x / s, +-448)).  Approximate squared distances use the exact
 * norms: |x|^2 + |y|^2 - 2 s_x s_y (x~ . y~), clamped at 0.
 */
#define BVS_LOWP_BF16 1
#define BVS_LOWP_FP8 2

/* Device bytes of the fmt copy of the database: N rows of 2 dp (BF16) or dp
 * rounded up to 128 (FP8) bytes, plus FP8 scales. */
bvs_status bvs_lowp_bytes(const bvs_index* ix, int fmt, uint64_t* out_bytes);

/* Builds the fmt copy from the index's exact planes into d_mem (caller
 * owned, at least bvs_lowp_bytes) and attaches it to the index; the memory
 * must outlive the index's use of that format.  Synchronises `stream`.
 * Attaching again replaces the previous copy of that format. */
bvs_status bvs_lowp_attach(bvs_index* ix, int fmt, void* d_mem, uint64_t bytes, void* stream);

/* Workspace bytes for bvs_search_lowp and bvs_hausdorff_lowp. */
bvs_status bvs_lowp_workspace_bytes(const bvs_index* ix, uint32_t n_q, uint64_t n_q_vectors,
                                    uint64_t* out_bytes);

/* Cascade search with the precision form of the re-rank: F2 as in
 * bvs_search, approximate values in fmt, exact re-check of the candidates
 * with approximate squared value <= v_k * f, f = float32(1 + margin)^2 in
 * float32 arithmetic, v_k the k-th smallest approximate value (all of F2
 * when |F2| < k), then the first k by (exact distance, id).  Outputs as
 * for bvs_search; d_rechecked (uint32 [n_q], may be NULL) receives the
 * number of re-checked candidates.  BVS_ESTATE if fmt is not attached;
 * margin must be finite and >= 0. */
bvs_status bvs_search_lowp(const bvs_index* ix, int fmt, float margin, const float* d_q,
                           const uint64_t* h_q_offsets, uint32_t n_q, uint32_t k,
                           void* d_workspace, uint64_t workspace_bytes,
                           uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                           uint32_t* d_rechecked, void* stream);

/* Approximate squared Hausdorff values in fmt of query q against the sets
 * d_ids [n_q][m] (uint32), into d_h2 float32 [n_q][m]. */
bvs_status bvs_hausdorff_lowp(const bvs_index* ix, int fmt, const float* d_q,
                              const uint64_t* h_q_offsets, uint32_t n_q,
                              const uint32_t* d_ids, uint32_t m,
                              void* d_workspace, uint64_t workspace_bytes,
                              float* d_h2, void* stream);

/* ------------------------------------------------------------------------
 * Learned projection.  The paper hashes with a learned projection before
 * the winner-take-all (Sec. 4.1; it does not specify the network or its
 * training).  Here the projection W of Def. 7 is replaced by a two-layer
 * network y = W2 relu(W1 x + b1) + b2 (dim -> hidden -> code_bits), and the
 * code of x keeps the wta_k largest bfloat16(y), ties to the lower index.
 * Inference runs on the matrix cores with bfloat16 operands (x, W1,
 * relu(...), W2) and float32 accumulation.  Everything after the codes
 * (sketches, filters, re-rank, the batched and precision forms) is
 * unchanged.
 *
 * Weights are float32, packed: W1 [hidden][dim], b1 [hidden],
 * W2 [code_bits][hidden], b2 [code_bits] (bvs_mlp_weight_count floats).
 * Requirements: dim % 8 == 0, hidden % 8 == 0 (<= 8192), code_bits a power
 * of two in 256..4096 (BVS_ENOTSUP otherwise).
 *
 * Training (bvs_train_projection): triplets (q, p, n) of set ids into the
 * training collection (sets given like database sets, up to 65535 vectors
 * each): a query set q, a set p among the exact nearest of q by Hausdorff
 * distance, and another set n.  Objective: soft codes c = sigmoid((y - t) /
 * tau), t the midpoint of the wta_k-th and (wta_k+1)-th largest y of the row
 * (held constant); soft sketches S = 1 - prod over the set's rows of (1 - c)
 * (the OR of Def. 10); soft Hamming h(A, B) = sum S_A + S_B - 2 S_A S_B; loss
 * = mean over triplets of max(0, margin + h(q, p) - h(q, n)).  Adam (beta1
 * 0.9, beta2 0.999, eps 1e-8) on the float32 weights, batches of
 * batch_triplets triplets; epoch e visits them in a Fisher-Yates shuffle of
 * the identity driven by splitmix64 seeded with seed ^ (e + 1) *
 * 0xD1B54A32D192ED03.
 */
typedef struct bvs_train_config {
  uint32_t dim, hidden, code_bits, wta_k;
  uint32_t batch_triplets, epochs;
  float lr, tau, margin;
  uint32_t reserved;       /* 0 */
  uint64_t seed;
} bvs_train_config;

bvs_status bvs_mlp_weight_count(uint32_t dim, uint32_t hidden, uint32_t code_bits, uint64_t* out_floats);

/* Uniform initialisation in +-sqrt(6 / fan_in), biases 0, from splitmix64 of
 * (seed, parameter index).  Synchronises `stream`. */
bvs_status bvs_mlp_init(uint32_t dim, uint32_t hidden, uint32_t code_bits, uint64_t seed, float* d_weights,
                        void* stream);

/* Index and build-workspace bytes of an index with a learned projection. */
bvs_status bvs_learned_index_bytes(const bvs_params* p, uint32_t hidden, uint64_t n_sets, uint64_t n_vectors,
                                   uint64_t* out_bytes);
bvs_status bvs_learned_build_workspace_bytes(const bvs_params* p, uint32_t hidden, uint64_t n_sets,
                                             uint64_t n_vectors, uint64_t* out_bytes);

/* As bvs_build_index, with the codes of the network d_weights (copied into
 * the index as bfloat16; p->fan_in and p->seed are not used).  Queries of
 * every search call are then encoded with the same network. */
bvs_status bvs_build_index_learned(const bvs_params* p, uint32_t hidden, const float* d_weights,
                                   const float* d_vectors, const uint64_t* h_offsets, uint64_t n_sets,
                                   void* d_index_mem, uint64_t index_bytes, void* d_workspace,
                                   uint64_t workspace_bytes, void* stream, bvs_index** out);

/* Training workspace for batches of up to max_batch_rows vectors (the rows
 * of the distinct sets of a batch). */
bvs_status bvs_train_workspace_bytes(const bvs_train_config* c, uint64_t max_batch_rows, uint64_t* out_bytes);

/* Loss and gradients (packed like the weights, into d_grads) of one batch
 * of n_triplets <= batch_triplets triplets (h_triplets uint32 [n][3]). */
bvs_status bvs_train_gradients(const bvs_train_config* c, const float* d_vectors, const uint64_t* h_offsets,
                               uint64_t n_sets, const uint32_t* h_triplets, uint32_t n_triplets,
                               const float* d_weights, float* d_grads, float* h_loss,
                               void* d_workspace, uint64_t workspace_bytes, void* stream);

/* Trains d_weights in place for c->epochs epochs; h_epoch_loss (may be
 * NULL) receives the mean batch loss of each epoch.  BVS_ENOSPC when a
 * batch has more rows than the workspace holds. */
bvs_status bvs_train_projection(const bvs_train_config* c, const float* d_vectors, const uint64_t* h_offsets,
                                uint64_t n_sets, const uint32_t* h_triplets, uint64_t n_triplets,
                                float* d_weights, void* d_workspace, uint64_t workspace_bytes,
                                float* h_epoch_loss, void* stream);

/* Checkpoint and resume of training.  A training state (device memory of
 * bvs_train_state_bytes, caller owned) holds Adam's first and second moments
 * (float32, packed like the weights) and the counts of Adam steps and of
 * epochs done; bvs_train_state_init zeroes it (synchronises).
 * bvs_train_projection_resume trains c->epochs more epochs continuing from the
 * state, which it updates in place: saving the weights and the state after a
 * call and resuming from copies of them later gives the training of one
 * longer call (the same batches in the same order and the same Adam steps;
 * the gradients' floating-point sums are accumulated in no fixed order, so
 * equal up to rounding). */
bvs_status bvs_train_state_bytes(const bvs_train_config* c, uint64_t* out_bytes);
bvs_status bvs_train_state_init(const bvs_train_config* c, void* d_state, void* stream);
bvs_status bvs_train_projection_resume(const bvs_train_config* c, const float* d_vectors,
                                       const uint64_t* h_offsets, uint64_t n_sets,
                                       const uint32_t* h_triplets, uint64_t n_triplets,
                                       float* d_weights, void* d_state, void* d_workspace,
                                       uint64_t workspace_bytes, float* h_epoch_loss, void* stream);

/* Stage timing.  When enabled, the library records a pair of HIP events on
 * the call's stream around every stage it launches and, after the call's
 * final synchronisation, adds the elapsed time to a process-wide table.
 * Every stage also runs inside a roctx range named after it (visible to a
 * profiler's marker trace).  Test hook: when the environment variable
 * BVS_TEST_FAIL names a stage (e.g. "rerank"), every call reaching that
 * stage returns BVS_EDEVICE without launching it; the index stays valid and
 * the next call without the variable succeeds.
 * Stages: 0 convert, 1 encode (query vectors), 2 query sketch, 3 cutoff
 * (first-layer bitmaps, sampled scores and the per-query score cutoff),
 * 4 filter (member-only scoring with bounded append), 5 select (top-T of the
 * appended candidates), 6 re-rank (exact Hausdorff of the candidates), 7
 * top-k, 8 brute force (Hausdorff to every set), 9 fallback (dense scores
 * and histogram selection, used when the sampled cutoff did not hold T
 * candidates or overflowed its buffer), 10 approximate re-rank of the
 * precision form (encoding of the queries, approximate values, selection
 * of the candidates to re-check), 11 exact re-check of the precision form,
 * 12 full scan (query tables and the Hamming-Hausdorff score of every set),
 * 13 lists (first-layer membership gathered from the inverted lists).
 * Work counters (summed over calls): 0 first-layer member pairs scored by
 * the filter stage, 1 database vectors read in full (both planes) by the
 * re-rank stage, 2 re-rank candidates abandoned early (screened ones
 * included), 3 re-rank candidates, 4 database vectors whose high plane the
 * re-rank's screen read, 5 candidates the screen rejected, 6 database
 * vectors read by the approximate re-rank of bvs_search_lowp.  bvs_search
 * and batches screen the candidates after the first 64 on their high planes
 * unless the environment sets BVS_SCREEN=0 (the results are the same).
 * bvs_profile_enable(flags) resets the table; flags: BVS_PROFILE_TIMING
 * records the stage events, BVS_PROFILE_COUNTERS collects the work counters
 * (their atomics slow the counted kernels somewhat), 0 turns both off. */
#define BVS_PROFILE_TIMING 1
#define BVS_PROFILE_COUNTERS 2
#define BVS_N_STAGES 14
#define BVS_N_COUNTERS 7
typedef struct bvs_stage_times {
  double ms[BVS_N_STAGES];
  uint64_t calls[BVS_N_STAGES];
  uint64_t counters[BVS_N_COUNTERS];
} bvs_stage_times;
bvs_status bvs_profile_enable(int flags);
bvs_status bvs_profile_read(bvs_stage_times* out);
const char* bvs_stage_name(int stage);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* bvs_last_error(void);

/* Library version string. */
const char* bvs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BVS_H */
