// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "bvs.h"
#include <stdint.h>

namespace bvs {

// Geometry of the hashing step shared by the encode kernels.
struct HashGeom {
  uint32_t dim, dim_padded;    // d and d rounded up to 64
  uint32_t L, lgL, R;          // code bits, log2 L (L is a power of two) or 0, L / 64
  uint32_t s, SP;              // fan-in and fan-in rounded up to 8 (row stride of idx)
  uint32_t wta_k;
  const uint16_t* idx;         // device [L][SP] byte offsets 2 i into the staged vector; padding reads the zero slot dim_padded
};

// float32 rows -> exact int8 planes a = 64 * hi + lo (a = 4096 x), squared
// norms of a, status bits, and (when scr is not null) per row the screening
// pair {|hi|^2, float bits of an upper bound of |lo - 31.5| / 64} with the
// 31.5 taken on the d real coordinates only.
hipError_t launch_convert(const float* x, uint64_t n_rows, uint32_t d, uint32_t dp,
                          int8_t* hi, uint8_t* lo, uint32_t* norms, uint2* scr, uint32_t* status,
                          int n_cu, hipStream_t st);

// Codes of single vectors: codes [n][R] uint64.
hipError_t launch_encode_vectors(const HashGeom& g, const int8_t* hi, const uint8_t* lo,
                                 uint64_t n, uint64_t* codes, int n_cu, hipStream_t st);

// Per-set sketches in row-major scratch: counts [n][L] u8, bits [n][R] u64.
hipError_t launch_encode_sets(const HashGeom& g, const int8_t* hi, const uint8_t* lo,
                              const uint64_t* offsets, uint64_t n_sets,
                              uint8_t* cnt_rm, uint64_t* bits_rm, int n_cu, hipStream_t st);

// Row-major scratch -> index layouts: counts [L][ld], bits chunk-major [R/2][ld][2].
hipError_t launch_transpose_sketches(const uint8_t* cnt_rm, const uint64_t* bits_rm,
                                     uint64_t n_sets, uint64_t ld, uint32_t L,
                                     uint8_t* cnt, uint64_t* bits, hipStream_t st);

// Bitmaps of C >= 1 from the count columns, tile-major: planes [ld/256][L][4] u64.
hipError_t launch_bitmap_planes(const uint8_t* cnt, uint64_t ld, uint32_t L, uint64_t* planes, hipStream_t st);

// Query sketches from query codes: C_Q [n_q][L] u16, S_Q [n_q][R] u64,
// top-A positions [n_q][A] u32, gate masks [n_q][R] u64 (bits of the A
// positions) and the chunk mask of the gates [n_q] u64.
hipError_t launch_query_sketch(const uint64_t* codes, const uint64_t* q_off, uint32_t n_q,
                               uint32_t L, uint32_t R, uint32_t A,
                               uint16_t* cq, uint64_t* sq, uint32_t* pos,
                               uint64_t* gate, uint64_t* gate_chunks, hipStream_t st);

// Second-layer scoring (Alg. 6, sketch filter).
struct FilterArgs {
  const uint4* bits;           // chunk-major binary Bloom filters [L/128][ld]
  const uint8_t* cnt;          // count Bloom filters [L][ld]
  uint64_t ld, n_sets;
  uint32_t RC;                 // L / 128
  const uint4* sq;             // query sketches [n_q][RC]
  const uint4* gate;           // gate masks [n_q][RC]
  const uint64_t* gate_chunks; // [n_q]
  const uint32_t* pos;         // [n_q][A]
  uint32_t A, M, n_q;
  uint32_t block_stride;       // set block of grid block b is b * block_stride
  uint16_t* scores;            // dense / sample output [n_q][ld_out]
  uint64_t ld_out;
  const uint32_t* cutoff;      // append mode: [n_q]
  uint64_t* cand;              // append mode: [n_q][cap] keys (score << 32 | id)
  uint32_t cap;
  uint32_t* cand_count;        // append mode: [n_q]
  const uint64_t* planes;      // tile-major bitmaps [ld/256][L][4] (bit j % 256 of row p of tile j / 256: set j has p)
  uint32_t L;                  // sketch length
  // bit-sliced scoring (see launch_filter_sliced)
  const uint16_t* spop;        // |B| of every set [ld]
  uint32_t parts;              // parts of a row list (4: 8 bytes of a tile row each)
  uint32_t LP;                 // list stride, L + 48
  uint32_t* lists;             // [n_q rounded up to 32][4][LP] row offsets by rank (bank-scheduled)
  uint32_t* qbits;             // [n_q] |S_Q|
  uint32_t* order;             // [n_q] queries by decreasing |S_Q| (blocks of 16)
  uint32_t* sbits;             // [n_q] |S_Q| by rank
  uint32_t* gsteps;            // [2 ceil(n_q / 32)] steps of 16 rows (per half of a rank pair)
  uint32_t* rpos;              // [n_q rounded up to 32][A] tile-row byte offsets of the top-A positions, by rank
  uint32_t* rcut;              // [n_q rounded up to 32] cutoff by rank
  uint32_t* fail;              // set to 1 when the result must come from the dense path
  uint32_t* any_long;          // 1 when some rank pair needs the long-sketch instance
  unsigned long long* stats;   // work counters (see bvs_stage_times), may be null
  const uint32_t* run_if;      // dense mode: skip all work unless *run_if != 0 (may be null)
  const uint64_t* member;      // first layer from the inverted lists: [n_q][ld / 64] bitmaps (may be null)
};
hipError_t launch_filter_dense(FilterArgs a, hipStream_t st);
hipError_t launch_filter_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st);
hipError_t launch_filter_append(FilterArgs a, hipStream_t st);
// Member-only scoring: tiles of 256 sets in LDS, first-layer members
// compacted into lanes.  Sample mode writes member scores (the caller
// pre-fills the sample buffer with 0xFFFF); append mode as above.
hipError_t launch_filter_sparse_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st);
hipError_t launch_filter_sparse_append(FilterArgs a, hipStream_t st);
// Bit-sliced scoring (first layer M <= 1), append mode only: the same
// appended keys as launch_filter_sparse_append.  launch_query_rows fills
// lists, qbits, order and rpos from the query sketches sq [n_q][R] and the
// top-A positions first.
hipError_t launch_set_weight(const uint64_t* bits, uint32_t RC, uint64_t ld, uint16_t* w, hipStream_t st);
hipError_t launch_query_rows(const FilterArgs& a, const uint64_t* sq, uint32_t R, hipStream_t st);
hipError_t launch_filter_sliced(const FilterArgs& a, hipStream_t st);
// Sample mode: the member scores of n_sample_blocks spread tiles, written to
// scores[q][block * 256 + set] (the caller pre-fills 0xFFFF), as the
// member-only sample; lists as for launch_filter_sliced.
hipError_t launch_filter_sliced_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st);
uint32_t sliced_parts();
size_t sliced_lds_bytes(uint32_t L);
// Per-query cutoffs from the sample; with order (ranks -> queries) also
// written by rank into rcut.
hipError_t launch_cutoff(const uint16_t* sample, uint32_t S, uint32_t L, uint32_t r, uint32_t n_q,
                         uint32_t* cutoff, const uint32_t* order, uint32_t* rcut, hipStream_t st);
hipError_t launch_sort_append(const uint64_t* cand, const uint32_t* cand_count, const uint32_t* cutoff, uint32_t cap,
                              uint32_t T, uint32_t L, uint32_t n_q, uint32_t* f2_ids, uint16_t* f2_scores,
                              uint32_t* f2_count, uint32_t* fail, hipStream_t st);

// Dense top-T selection of the scores; writes F2 sorted by (score, id).
struct SelectBufs {
  uint32_t* hist;     // [n_q][L + 2]
  uint32_t* sel;      // [n_q][4]: tau, count_below, need_eq, Tq
  uint32_t* ctr;      // [n_q]
  uint32_t* eqcnt;    // [n_q][nblk]
  uint64_t* cand;     // [n_q][T]
};
uint32_t select_blocks(uint64_t ld);
// With run_if != null every kernel does nothing unless *run_if != 0 (a
// decision taken on the device, so the launches can sit in a graph).
hipError_t launch_select(const uint16_t* scores, uint64_t ld, uint32_t L, uint32_t T, uint32_t n_q,
                         const SelectBufs& b, uint32_t* f2_ids, uint16_t* f2_scores,
                         uint32_t* f2_count, const uint32_t* run_if, hipStream_t st);

// Exact squared Hausdorff distances (scaled by 2^24).
// scr: per-row screening pairs written by launch_convert; bounded re-ranks
// screen with the high planes first when both sides have them (null: no
// screening).
// Set measure of the re-rank (Sec. 3.2): the Hausdorff distance of Def. 4,
// the mean over the query's vectors of their distance to the set (MeanMin,
// query to set), or the smallest distance between the two sets (Min).
enum : uint32_t { kMetricHausdorff = 0, kMetricMeanMin = 1, kMetricMin = 2 };
struct HausDb {
  const int8_t* hi; const uint8_t* lo; const uint32_t* norms; const uint64_t* offsets;
  uint64_t n_sets; uint32_t dp;
  const uint2* scr;
  // Result key of a set: Hausdorff and Min give 2^24 times the squared
  // distance (an integer); MeanMin gives the float32 bits of the distance
  // (a mean of square roots, accumulated in float64), which order like
  // the values.  Metrics other than Hausdorff are never bounded or screened.
  uint32_t metric = kMetricHausdorff;
};
struct HausQ {
  const int8_t* hi; const uint8_t* lo; const uint32_t* norms; const uint64_t* offsets;
  uint32_t n_q; uint32_t max_rows;
  const uint2* scr;
  // candidate mode: the n_q queries served are qids[0 .. n_q) (null: 0 .. n_q);
  // ids, counts, results and bounds stay indexed by query
  const uint32_t* qids;
};
// Candidate mode: items are ids[q][0 .. count[q]) with stride T.  Items that
// provably cannot be among the k nearest may be abandoned (h2 = all ones);
// thr [n_q] is scratch for the shared bound.
// sel [n_q][T] and sel_count [n_q] (both may be null: no screening) are
// scratch for the candidates that pass the high-plane screen; with q.qids
// the caller zeroes sel_count of the listed queries beforehand.
hipError_t launch_haus_cand(const HausDb& db, const HausQ& q, const uint32_t* ids,
                            const uint32_t* count, uint32_t T, uint32_t k, uint32_t* thr,
                            uint32_t* h2, unsigned long long* stats, uint32_t* sel, uint32_t* sel_count,
                            hipStream_t st);
// All sets: h2 [n_q][n_sets].
// Exact value of every (query, set) pair into h2 [n_q][n_sets]; h_q_off are
// the query offsets on the host, d_qids a device list of
// haus_all_list_words(n_q) words (the queries grouped by size; the call
// synchronises the stream after uploading it).
uint32_t haus_all_list_words(uint32_t n_q);
hipError_t launch_haus_all(const HausDb& db, const HausQ& q, uint32_t* h2, const uint64_t* h_q_off, uint32_t* d_qids,
                           hipStream_t st);
size_t haus_lds_bytes(uint32_t max_rows, uint32_t dp);
uint32_t haus_lds_rows(uint32_t max_rows, uint32_t dp);
uint32_t haus_max_rows_supported(uint32_t dp);

// Candidates per re-rank work item (and the size of the first, unbounded
// phase of the candidate re-rank).
static constexpr uint32_t kCandPerItem = 64;

// Persistent re-rank of a whole batch (one launch): candidates as for
// launch_haus_cand; queries are taken in `order` (largest first).
struct QueueArgs {
  const uint32_t* ids;       // [n_q][T] candidate ids
  const uint32_t* count;     // [n_q] candidates per query
  uint32_t T, k;
  const uint32_t* order;     // [n_q] queries, largest first
  uint32_t nch;              // items per query: ceil(T / 64)
  uint32_t lds_rows;         // query rows staged in LDS (multiple of 16)
  uint32_t* ctl;             // [1 + n_q]: item counter, then per-query bounds
  uint32_t* h2;              // [n_q][T] out
  unsigned long long* stats; // work counters, may be null
};
size_t haus_queue_lds_bytes(uint32_t lds_rows, uint32_t dp);
// Resident workgroups per CU and scratch bytes per lane of a queue kernel.
hipError_t haus_queue_occupancy(uint32_t dp, uint32_t lds_rows, uint32_t waves, uint32_t* blocks_per_cu,
                                uint32_t* spill_bytes);
// Clears ctl, then launches `blocks` workgroups of `waves` waves.
hipError_t launch_haus_queue(const HausDb& db, const HausQ& q, const QueueArgs& a, uint32_t waves,
                             uint32_t blocks, hipStream_t st);

// Full-scan search (Alg. 2).  pos [n][KP] uint16: the K code positions of
// every vector (from codes [n][R] uint64).  Queries go in packs: runs of
// consecutive queries of the batch, at most kPackQ, whose vectors fill
// consecutive slots of at most kPackGroups groups of 64; packs [n_packs] =
// {first query, queries, groups, 0}.  table [n_packs][GP][L] uint64: bit i of
// entry (k, g, p) says whether the vector in slot 64 g + i of pack k has
// position p (GP >= the groups of every pack).  Scan: scores[q][j] = Haus^H
// (Hamming form of Def. 4) of query q to set j for the n_sets sets listed in
// order [n_sets] (any order; by size keeps the lanes of a wave together).
static constexpr int kPackQ = 8;
static constexpr uint32_t kPackGroups = 4;
hipError_t launch_code_positions(const uint64_t* codes, uint64_t n, uint32_t R, uint32_t K, uint32_t KP,
                                 uint16_t* pos, int n_cu, hipStream_t st);
hipError_t launch_query_table(const uint64_t* codes, const uint64_t* q_off, const uint4* packs, uint32_t n_packs,
                              uint32_t L, uint32_t R, uint32_t GP, uint64_t* table, hipStream_t st);
hipError_t launch_full_scan(const uint16_t* pos, const uint64_t* offsets, const uint32_t* order, uint64_t n_sets,
                            uint32_t K, uint32_t KP, uint32_t L, const uint64_t* table, const uint64_t* q_off,
                            const uint4* packs, uint32_t n_packs, uint32_t GP, uint16_t* scores, uint64_t ld,
                            hipStream_t st);

// Inverted lists (Def. 9, Alg. 4) from the position-major counts: pass
// fill = false writes hist [L][256] (scratch), cum [L][257], len [L] and
// start [L + 1]; fill = true writes ids [start[L]] (cursor [L][256] scratch).
hipError_t launch_list_build(const uint8_t* cnt, uint64_t ld, uint64_t n_sets, uint32_t L, uint32_t* hist,
                             uint32_t* cursor, uint64_t* len, uint32_t* cum, uint64_t* start, uint32_t* ids,
                             hipStream_t st, bool fill);
// First layer from the lists: member [n_q][ld / 64] = OR over the A positions
// of the query of the bits of the sets with count >= M.
hipError_t launch_list_gather(const uint32_t* ids, const uint64_t* start, const uint32_t* cum, const uint32_t* pos,
                              uint32_t A, uint32_t M, uint32_t n_q, uint64_t ld, uint64_t* member, int n_cu,
                              hipStream_t st);

// First k by (h2, id) of each query.  ids_in may be NULL (item index = id).
// tmp must hold 2 * n_q * ceil(n_items / 4096) * k uint64.  Reported
// distances are sqrt(h2) / 4096, or the float32 whose bits are h2 when
// key_is_dist (MeanMin keys).
hipError_t launch_topk(const uint32_t* h2, const uint32_t* ids_in, const uint32_t* count_in,
                       uint64_t n_items, uint64_t stride, uint32_t n_q, uint32_t k,
                       uint64_t* tmp, uint32_t* ids, float* dist, uint32_t* count,
                       hipStream_t st, bool key_is_dist = false);
uint64_t topk_tmp_words(uint64_t n_items, uint32_t n_q, uint32_t k);

// Precision form (BVS_LOWP_BF16 / BVS_LOWP_FP8 copies of the vectors).
struct LowpDb {
  const uint8_t* rows; const float* scale; const uint32_t* norms; const uint64_t* offsets;
  uint64_t n_sets; uint32_t row_bytes;
};
struct LowpQ {
  const uint8_t* rows; const float* scale; const uint32_t* norms; const uint64_t* offsets;
  uint32_t n_q, max_rows, row_bytes;
};
uint32_t lowp_row_bytes(int fmt, uint32_t dp);
// Encode the sets [offsets] of the int8 planes into fmt rows (and FP8 scales).
hipError_t launch_lowp_encode(const int8_t* hi, const uint8_t* lo, uint32_t dp, const uint64_t* offsets,
                              uint64_t n_sets, int fmt, uint32_t row_bytes, uint8_t* out, float* scale,
                              hipStream_t st);
// Approximate squared Hausdorff values (float bits) of ids[q][i0 .. min(count[q], lim)).
// With bounds (float bits per query, all ones: none), values that provably
// exceed bounds[q] * factor (float32) come out all ones.  stats (nullable):
// rows read, added to work counter 6.
hipError_t launch_haus_lowp(int fmt, const LowpDb& db, const LowpQ& q, const uint32_t* ids, const uint32_t* count,
                            uint32_t stride, uint32_t i0, uint32_t lim, const uint32_t* bounds, float factor,
                            uint32_t* out, unsigned long long* stats, hipStream_t st);
// bounds[q] = k-th smallest of vals[q][0 .. min(count[q], n)) (stride T,
// n <= 64) for q < n_q, all ones when fewer than k.
hipError_t launch_kth_bound(const uint32_t* vals, const uint32_t* count, uint32_t T, uint32_t n, uint32_t k,
                            uint32_t n_q, uint32_t* bounds, hipStream_t st);
// Candidates to re-check: the prefix of (value, id) order within factor of the k-th value.
hipError_t launch_lowp_select(const uint32_t* approx, const uint32_t* ids, const uint32_t* count, uint32_t T,
                              uint32_t n_q, uint32_t k, float factor, uint32_t* r_ids, uint32_t* r_count,
                              hipStream_t st);

// Learned projection (bfloat16 weights; biases float32).
struct Mlp {
  uint32_t d, H, L, wta_k;
  const uint16_t* W1;   // [H][d]
  const float* b1;      // [H]
  const uint16_t* W2;   // [L][H]
  const float* b2;      // [L]
};
// C = A B (see k_gemm for the layouts), bfloat16 operands, float32 accumulation.
hipError_t launch_gemm(bool at, bool bt, const uint16_t* A, uint64_t lda, const uint16_t* B, uint64_t ldb,
                       uint32_t M, uint32_t N, uint32_t K, const float* bias, bool relu, float* C32, uint16_t* C16,
                       uint64_t ldc, hipStream_t st);
hipError_t launch_rows_to_bf16(const float* X, uint32_t d, const uint64_t* rows, uint64_t n, uint16_t* out,
                               hipStream_t st);
hipError_t launch_planes_to_bf16(const int8_t* hi, const uint8_t* lo, uint32_t dp, uint32_t d, uint64_t n,
                                 uint16_t* out, hipStream_t st);
hipError_t launch_f32_to_bf16(const float* x, uint64_t n, uint16_t* out, hipStream_t st);
hipError_t launch_wta_rows(const float* Y, uint64_t ldy, uint64_t n, uint32_t L, uint32_t k, uint64_t* codes,
                           hipStream_t st);
hipError_t launch_sets_from_codes(const uint64_t* codes, const uint64_t* offsets, uint64_t base, uint64_t s0,
                                  uint64_t n_sets, uint32_t R, uint8_t* cnt_rm, uint64_t* bits_rm, hipStream_t st);
// Codes of n bfloat16 rows X16 [n][d] through the network (scratch H16 [n][H], Y [n][L]).
hipError_t encode_learned(const Mlp& m, const uint16_t* X16, uint64_t n, uint16_t* H16, float* Y, uint64_t* codes,
                          hipStream_t st);
// Training kernels.
hipError_t launch_row_thresholds(const float* Y, uint64_t n, uint32_t L, uint32_t k, float* thr, hipStream_t st);
hipError_t launch_set_soft(const float* Y, const float* thr, const uint32_t* row_off, uint32_t n_sets, uint32_t L,
                           float tau, float* LS, float* S, hipStream_t st);
hipError_t launch_triplet(const float* S, const uint32_t* trip, uint32_t n_trip, uint32_t L, float margin,
                          float* dS, float* loss, hipStream_t st);
hipError_t launch_soft_backward(const float* Y, const float* thr, const uint32_t* row_off, uint32_t n_sets, uint32_t L,
                                float tau, const float* LS, const float* dS, float* dY, uint16_t* dY16,
                                hipStream_t st);
hipError_t launch_relu_backward(const float* dH, const uint16_t* H16, uint64_t n, float* dP, uint16_t* dP16,
                                hipStream_t st);
hipError_t launch_colsum(const float* X, uint64_t n, uint32_t C, float* out, hipStream_t st);
hipError_t launch_add_loss(const float* loss, double* acc, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, uint32_t step, uint16_t* w16, hipStream_t st);
hipError_t launch_mlp_init(float* w, uint32_t d, uint32_t H, uint32_t L, uint64_t seed, hipStream_t st);

// Fill a u32 buffer (used instead of hipMemsetAsync so work stays graph-safe).
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st,
                           const uint32_t* run_if = nullptr);

}  // namespace bvs
