// Exact Hausdorff re-rank (Def. 4) of candidate sets and of every database
// set, one launch per stage, the high-plane screen of the bounded
// candidates, and the top-k of the results.  The distance arithmetic and
// the screen's bound live in haus_core.h.
//
// Mapping.  One workgroup (8 waves) takes one query and a range of items
// (candidate sets or database sets).  It stages as many of the query's rows
// as fit in LDS; each wave walks its items one at a time.
#include "haus_core.h"

namespace bvs {

static constexpr uint32_t kHausWaves = 8;

// LDS budget for the staged query of the per-launch kernels.
static constexpr size_t kStageBudget = 120 * 1024;

// Rows of a query of max_rows vectors that the per-launch kernels stage.
uint32_t haus_lds_rows(uint32_t max_rows, uint32_t dp) {
  uint32_t rows = std::min<uint32_t>((max_rows + 15) / 16 * 16, kMaxQueryTiles * 16);
  while (rows > 16 && haus_stage_bytes(rows, dp) > kStageBudget) rows -= 16;
  return rows;
}

size_t haus_lds_bytes(uint32_t max_rows, uint32_t dp) { return haus_stage_bytes(haus_lds_rows(max_rows, dp), dp); }

// Candidate mode: grid (G, n_q).  Block b of query q takes the candidates
// i0 + b * kCandPerBlock ... of ids[q][i0 .. i1), i1 = min(count[q], lim);
// waves take them round-robin.  With bounds != nullptr, candidates whose
// lower bound exceeds bounds[q] are abandoned (h2 = kAbandoned).

//
// With sel != nullptr the positions i index sel[q][i], the candidates that
// passed the screen (count[q] of them), instead of the candidates directly.

template <int KS, int MAXQT, bool HASG>
__global__ void __launch_bounds__(64 * kHausWaves)
k_haus_cand(HausDb db, HausQ qs, uint32_t lds_rows, const uint32_t* __restrict__ ids,
            const uint32_t* __restrict__ count, uint32_t T, uint32_t i0, uint32_t lim,
            const uint32_t* __restrict__ bounds, uint32_t* __restrict__ h2, unsigned long long* __restrict__ stats,
            const uint32_t* __restrict__ sel) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t q = qs.qids ? qs.qids[blockIdx.y] : blockIdx.y;
  const uint32_t i1 = min(count[q], lim);
  const uint32_t b0 = i0 + blockIdx.x * kCandPerBlock;
  if (b0 >= i1) return;
  const uint32_t b1 = min(i1, b0 + kCandPerBlock);
  const uint32_t bound = bounds ? bounds[q] : 0xFFFFFFFFu;
  const QView qv = stage_query(qs, q, KS * 64, lds_rows, smem);
  const uint32_t w = wave_id();
  uint32_t rows = 0, abandoned = 0, items = 0;
  // the id of the candidate after next and the offsets of the next one load
  // while this one is computed (out-of-range ids read set 0, unused)
  const cptr<uint32_t> idq = as_const(ids) + (uint64_t)q * T;
  const uint32_t* selq = sel ? sel + (uint64_t)q * T : nullptr;
  const cptr<uint64_t> offs = as_const(db.offsets);
  auto cand_at = [&](uint32_t i) { return selq ? selq[i] : i; };
  auto id_at = [&](uint32_t i) { return i < b1 ? idq[cand_at(i)] : 0u; };
  uint32_t jn = id_at(b0 + w);
  uint64_t o0 = offs[jn], o1 = offs[jn + 1];
  jn = id_at(b0 + w + kHausWaves);
  for (uint32_t it = b0 + w; it < b1; it += kHausWaves) {
    const uint64_t n0 = offs[jn], n1 = offs[jn + 1];
    jn = id_at(it + 2 * kHausWaves);
    const uint32_t hsq = haus_item<KS, MAXQT, HASG>(db, o0, (uint32_t)(o1 - o0), qv, bound, stats ? &rows : nullptr);
    if (lane_id() == 0) h2[(uint64_t)q * T + cand_at(it)] = hsq;
    abandoned += hsq == kAbandoned ? 1u : 0u;
    ++items;
    o0 = n0;
    o1 = n1;
  }
  if (stats) stats_add(stats, 1, rows, abandoned, items);
}

// High-plane screen of candidates [i0, count[q]) against bounds[q] (see
// haus_core.h): rejected candidates get h2 = kAbandoned, the others are
// appended to sel[q][0 .. sel_count[q]) in no particular order (the exact
// pass writes each result at its candidate's index, so the order does not
// change any result).  Grid (G, n_q) as k_haus_cand; the whole query is
// staged (its high plane and screening pairs).  At head dimensions up to 384
// and queries of up to 128 vectors it fits 64 VGPRs, eight waves per SIMD.
template <int KS, int MAXQT>
__global__ void __launch_bounds__(64 * kHausWaves, KS <= 6 && MAXQT <= 8 ? 8 : 1)
k_haus_screen(HausDb db, HausQ qs, const uint32_t* __restrict__ ids, const uint32_t* __restrict__ count, uint32_t T,
              uint32_t i0, const uint32_t* __restrict__ bounds, uint32_t* __restrict__ h2, uint32_t* __restrict__ sel,
              uint32_t* __restrict__ sel_count, unsigned long long* __restrict__ stats) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t q = qs.qids ? qs.qids[blockIdx.y] : blockIdx.y;
  const uint32_t i1 = count[q];
  const uint32_t b0 = i0 + blockIdx.x * kCandPerBlock;
  if (b0 >= i1) return;
  const uint32_t b1 = min(i1, b0 + kCandPerBlock);
  const uint32_t bound = bounds[q];
  const QView qv = stage_query_screen(qs, q, KS * 64, smem);
  const uint32_t w = wave_id(), lane = lane_id();
  uint32_t rows = 0, rejected = 0;
  const cptr<uint32_t> idq = as_const(ids) + (uint64_t)q * T;
  const cptr<uint64_t> offs = as_const(db.offsets);
  auto id_at = [&](uint32_t i) { return i < b1 ? idq[i] : 0u; };
  uint32_t jn = id_at(b0 + w);
  uint64_t o0 = offs[jn], o1 = offs[jn + 1];
  jn = id_at(b0 + w + kHausWaves);
  for (uint32_t it = b0 + w; it < b1; it += kHausWaves) {
    const uint64_t n0 = offs[jn], n1 = offs[jn + 1];
    jn = id_at(it + 2 * kHausWaves);
    const uint32_t m = (uint32_t)(o1 - o0);
    rows += min(16u, m);
    const bool far = bound != 0xFFFFFFFFu && screen_set<KS, MAXQT, false>(db, o0, m, qv, bound);
    if (lane == 0) {
      if (far) {
        h2[(uint64_t)q * T + it] = kAbandoned;
      } else {
        const uint32_t pos = atomicAdd(sel_count + q, 1u);
        sel[(uint64_t)q * T + pos] = it;
      }
    }
    rejected += far ? 1u : 0u;
    o0 = n0;
    o1 = n1;
  }
  if (stats) {
    stats_add(stats, 2, rejected, rejected);   // abandoned and candidates
    __syncthreads();   // stats_add reuses its LDS words
    stats_add(stats, 4, rows, rejected);
  }
}

// One wave per query: bounds[q] = k-th smallest of h2[q][0 .. min(count, n)),
// n <= 64, or all ones when fewer than k are there.  With qids, wave b
// serves query qids[b].
__global__ void __launch_bounds__(64)
k_kth_bound(const uint32_t* __restrict__ h2, const uint32_t* __restrict__ count, uint32_t T, uint32_t n, uint32_t k,
            uint32_t* __restrict__ bounds, const uint32_t* __restrict__ qids) {
  const uint32_t q = qids ? qids[blockIdx.x] : blockIdx.x, lane = lane_id();
  const uint32_t nv = min(count[q], n);
  const uint32_t v = lane < nv ? h2[(uint64_t)q * T + lane] : 0xFFFFFFFFu;
  const uint32_t kth = wave_kth_smallest(v, nv, k);
  if (lane == 0) bounds[q] = kth;
}

hipError_t launch_kth_bound(const uint32_t* vals, const uint32_t* count, uint32_t T, uint32_t n, uint32_t k,
                            uint32_t n_q, uint32_t* bounds, hipStream_t st) {
  if (n > 64 || k == 0) return hipErrorInvalidValue;
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kth_bound, dim3(n_q), dim3(64), 0, st, vals, count, T, n, k, bounds,
                     (const uint32_t*)nullptr);
  return hipGetLastError();
}

// All-sets mode.  Work units (query, chunk of kAllChunk sets) are numbered so
// that units sharing a chunk of the database run at the same time on the same
// XCD: consecutive workgroup ids are dealt round-robin over the 8 XCDs, so the
// unit index is rebuilt from (id % 8, id / 8).  The queries are qids[0 ..
// nql) (a class of the size grouping below).
static constexpr uint32_t kAllChunk = 128;
static constexpr uint32_t kNoQuery = 0xFFFFFFFFu;   // padding of a query tile

template <int KS, int MAXQT, bool HASG>
__global__ void __launch_bounds__(64 * kHausWaves)
k_haus_all(HausDb db, HausQ qs, uint32_t lds_rows, uint64_t n_units, const uint32_t* __restrict__ qids, uint32_t nql,
           uint32_t* __restrict__ h2) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t b = blockIdx.x, nb = gridDim.x;   // nb is a multiple of 8
  const uint64_t unit = (b % 8) * (nb / 8) + b / 8;
  if (unit >= n_units) return;
  const uint32_t q = qids[unit % nql];
  const uint32_t chunk = (uint32_t)(unit / nql);
  const uint64_t s0 = (uint64_t)chunk * kAllChunk;
  const uint64_t s1 = min(db.n_sets, s0 + kAllChunk);
  const QView qv = stage_query(qs, q, KS * 64, lds_rows, smem);
  const uint32_t w = wave_id();
  for (uint64_t j = s0 + w; j < s1; j += kHausWaves) {
    const uint64_t o0 = db.offsets[j];
    const uint32_t m = (uint32_t)(db.offsets[j + 1] - o0);
    const uint32_t hsq = haus_item<KS, MAXQT, HASG>(db, o0, m, qv);
    if (lane_id() == 0) h2[(uint64_t)q * db.n_sets + j] = hsq;
  }
}

// Query-tiled all-sets mode: a unit is (tile of QT queries, chunk of
// kAllChunk sets); the tile's queries are qids[QT tile .. + QT) (kNoQuery
// pads the last tile of a class; its first entry is always a query).  The
// workgroup stages the QT queries (lds_rows rows each, the rest read from
// global memory) and each wave computes its sets against all of them
// (haus_multi), so every set is read once per QT queries.  Units are numbered
// over the XCDs as in k_haus_all.  WV waves per workgroup: the staged
// queries take most of the LDS, so one workgroup runs per CU and WV sets its
// waves per SIMD (12 where the registers allow three per SIMD, else 8).
template <int KS, int MAXQT, bool HASG, int QT, int WV>
__global__ void __launch_bounds__(64 * WV)
k_haus_all_qt(HausDb db, HausQ qs, uint32_t lds_rows, uint64_t n_units, const uint32_t* __restrict__ qids,
              uint32_t n_tiles, uint32_t* __restrict__ h2) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t b = blockIdx.x, nb = gridDim.x;   // nb is a multiple of 8
  const uint64_t unit = (b % 8) * (nb / 8) + b / 8;
  if (unit >= n_units) return;
  const uint32_t* tq = qids + (uint64_t)(unit % n_tiles) * QT;
  const uint32_t chunk = (uint32_t)(unit / n_tiles);
  const uint64_t s0 = (uint64_t)chunk * kAllChunk;
  const uint64_t s1 = min(db.n_sets, s0 + kAllChunk);
  const size_t per_q = haus_stage_bytes(lds_rows, KS * 64);
  uint32_t qid[QT];
  QView qv[QT];
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    qid[i] = tq[i];
    qv[i] = stage_query(qs, qid[i] == kNoQuery ? tq[0] : qid[i], KS * 64, lds_rows, smem + i * per_q);
  }
  const uint32_t w = wave_id();
  for (uint64_t j = s0 + w; j < s1; j += WV) {
    const uint64_t o0 = db.offsets[j];
    const uint32_t m = (uint32_t)(db.offsets[j + 1] - o0);
    uint32_t out[QT];
    haus_multi<KS, MAXQT, HASG, QT>(db, o0, m, qv, out);
    if (lane_id() == 0) {
#pragma unroll
      for (int i = 0; i < QT; ++i)
        if (qid[i] != kNoQuery) h2[(uint64_t)qid[i] * db.n_sets + j] = out[i];
    }
  }
}

// Instantiation for head dimension dp, queries of up to max_rows vectors
// and lds_rows staged rows: f(KS, MAXQT, HASG).
template <typename F>
static hipError_t dispatch_haus(uint32_t dp, uint32_t max_rows, uint32_t lds_rows, F&& f) {
  const uint32_t nqt = (max_rows + 15) / 16;
  const bool hasg = lds_rows < nqt * 16;
  auto by_g = [&](auto ks, auto mqt) -> hipError_t {
    if (hasg) return f(ks, mqt, std::true_type());
    return f(ks, mqt, std::false_type());
  };
  auto by_q = [&](auto ks) -> hipError_t {
    if (nqt <= 2) return by_g(ks, std::integral_constant<int, 2>());
    if (nqt <= 4) return by_g(ks, std::integral_constant<int, 4>());
    if (nqt <= 8) return by_g(ks, std::integral_constant<int, 8>());
    if (nqt <= 16) return by_g(ks, std::integral_constant<int, 16>());
    return hipErrorInvalidValue;
  };
  switch (dp / 64) {
    case 1: return by_q(std::integral_constant<int, 1>());
    case 2: return by_q(std::integral_constant<int, 2>());
    case 4: return by_q(std::integral_constant<int, 4>());
    case 6: return by_q(std::integral_constant<int, 6>());
    case 8: return by_q(std::integral_constant<int, 8>());
    case 12: return by_q(std::integral_constant<int, 12>());
    case 16: return by_q(std::integral_constant<int, 16>());
    default: return hipErrorInvalidValue;
  }
}

uint32_t haus_max_rows_supported(uint32_t dp) {
  (void)dp;
  return kMaxQueryTiles * 16;
}

// Whether dispatch_haus can select the (KS, MQ, HG) variant: query tiles
// from global memory only where MQ tiles can exceed the staging budget.
template <int KS, int MQ, bool HG>
constexpr bool haus_variant_used() {
  return !HG || haus_stage_bytes(MQ * 16, KS * 64) > kStageBudget;
}

// Exact phases: full distances for the first max(k, 32) candidates, the
// best by sketch distance (max(k, 16) without the screening buffers: the
// re-check of a few near candidates); their k-th smallest bounds those up to
// kCandPerBlock, whose k-th smallest (abandoned ones exceed it) bounds the
// remaining candidates; each bound is at least the query's k-th distance.
// Given the screening buffers (and screening pairs on both sides, and a
// query that fits the screen's LDS), the remaining candidates are screened
// on their high planes first and only the survivors take the exact pass.
hipError_t launch_haus_cand(const HausDb& db, const HausQ& q, const uint32_t* ids, const uint32_t* count,
                            uint32_t T, uint32_t k, uint32_t* thr, uint32_t* h2, unsigned long long* stats,
                            uint32_t* sel, uint32_t* sel_count, hipStream_t st) {
  if (q.n_q == 0) return hipSuccess;
  const uint32_t lds_rows = haus_lds_rows(q.max_rows, db.dp);
  const size_t lds = haus_stage_bytes(lds_rows, db.dp);
  const uint32_t n0 = std::min(T, kCandPerBlock);
  return dispatch_haus(db.dp, q.max_rows, lds_rows, [&](auto ks, auto mqt, auto hg) -> hipError_t {
    constexpr int KS = decltype(ks)::value, MQ = decltype(mqt)::value;
    constexpr bool HG = decltype(hg)::value;
    if constexpr (!haus_variant_used<KS, MQ, HG>()) {
      return hipErrorInvalidValue;
    } else {
      auto kern = k_haus_cand<KS, MQ, HG>;
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      if (db.metric != kMetricHausdorff) {
        // no bound applies to the other measures: every candidate in full
        const uint32_t G = (T + kCandPerBlock - 1) / kCandPerBlock;
        hipLaunchKernelGGL(kern, dim3(G, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, lds_rows, ids, count, T, 0u,
                           T, (const uint32_t*)nullptr, h2, stats, (const uint32_t*)nullptr);
        return hipGetLastError();
      }
      // the first na candidates bound the next ones up to n0, whose k-th
      // distance then bounds the rest
      const uint32_t na = std::min(n0, std::max(k, sel ? 32u : 16u));
      hipLaunchKernelGGL(kern, dim3(1, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, lds_rows, ids, count, T, 0u,
                         na, (const uint32_t*)nullptr, h2, stats, (const uint32_t*)nullptr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (T <= na) return hipSuccess;
      if (na < n0) {
        hipLaunchKernelGGL(k_kth_bound, dim3(q.n_q), dim3(64), 0, st, h2, count, T, na, k, thr, q.qids);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(1, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, lds_rows, ids, count, T, na,
                           n0, (const uint32_t*)thr, h2, stats, (const uint32_t*)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (T <= n0) return hipSuccess;
      }
      hipLaunchKernelGGL(k_kth_bound, dim3(q.n_q), dim3(64), 0, st, h2, count, T, n0, k, thr, q.qids);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const uint32_t G = (T - n0 + kCandPerBlock - 1) / kCandPerBlock;
      const size_t slds = screen_stage_bytes((q.max_rows + 15) / 16 * 16, db.dp);
      if (sel && sel_count && db.scr && q.scr && slds <= kStageBudget) {
        // the rest: high-plane screen, then the exact pass over the survivors
        if (!q.qids && (e = launch_fill_u32(sel_count, q.n_q, 0, st)) != hipSuccess) return e;
        auto skern = k_haus_screen<KS, MQ>;
        if ((e = hipFuncSetAttribute((const void*)skern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)slds)) !=
            hipSuccess)
          return e;
        hipLaunchKernelGGL(skern, dim3(G, q.n_q), dim3(64 * kHausWaves), slds, st, db, q, ids, count, T, n0,
                           (const uint32_t*)thr, h2, sel, sel_count, stats);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(G, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, lds_rows, ids,
                           (const uint32_t*)sel_count, T, 0u, T, (const uint32_t*)thr, h2, stats,
                           (const uint32_t*)sel);
        return hipGetLastError();
      }
      hipLaunchKernelGGL(kern, dim3(G, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, lds_rows, ids, count, T, n0,
                         T, (const uint32_t*)thr, h2, stats, (const uint32_t*)nullptr);
      return hipGetLastError();
    }
  });
}

// The brute force groups the queries by their tiles of 16 vectors: those of
// one or two tiles share a pass over the database QT = 8 or 4 at a time,
// those of three to eight tiles two at a time (up to 64 rows staged, the
// rest from global memory), larger ones one at a time; QT is the largest of
// {8, 4, 2} whose staged rows fit the LDS budget at dp (else one at a time).
// Each class is one launch over its tiles of query ids.
struct AllClass {
  uint32_t qt, rows, mqt;   // queries per tile, staged rows per query, tiles kept per query
  bool hg;                  // query tiles past the staged rows come from global memory
};

static AllClass all_class(uint32_t nqt, uint32_t dp) {
  AllClass c{1, 0, 16, false};
  if (nqt > 8) {
    c.rows = haus_lds_rows(nqt * 16, dp);
    c.hg = c.rows < nqt * 16;
    return c;
  }
  const uint32_t need = nqt * 16;
  c.mqt = nqt <= 2 ? 2 : nqt <= 4 ? 4 : 8;
  c.rows = std::min<uint32_t>(need, 64);
  for (uint32_t t : {8u, 4u, 2u}) {
    if (t == 8 && c.mqt != 2) continue;   // eight queries per tile only for the smallest class
    if (t * haus_stage_bytes(c.rows, dp) <= kStageBudget) {
      c.qt = t;
      c.hg = c.rows < need;
      return c;
    }
  }
  c.qt = 1;
  c.mqt = 16;
  c.rows = haus_lds_rows(need, dp);
  c.hg = c.rows < need;
  return c;
}

template <typename F>
static hipError_t dispatch_ks(uint32_t dp, F&& f) {
  switch (dp / 64) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 4: return f(std::integral_constant<int, 4>());
    case 6: return f(std::integral_constant<int, 6>());
    case 8: return f(std::integral_constant<int, 8>());
    case 12: return f(std::integral_constant<int, 12>());
    case 16: return f(std::integral_constant<int, 16>());
    default: return hipErrorInvalidValue;
  }
}

uint32_t haus_all_list_words(uint32_t n_q) { return n_q + 7 * 5; }   // padding: < 8 per class

hipError_t launch_haus_all(const HausDb& db, const HausQ& q, uint32_t* h2, const uint64_t* h_q_off, uint32_t* d_qids,
                           hipStream_t st) {
  if (q.n_q == 0 || db.n_sets == 0) return hipSuccess;
  // classes: 1, 2, 3-4, 5-8 and more than 8 query tiles
  std::vector<uint32_t> cls[5];
  for (uint32_t i = 0; i < q.n_q; ++i) {
    const uint32_t nqt = (uint32_t)((h_q_off[i + 1] - h_q_off[i] + 15) / 16);
    cls[nqt <= 1 ? 0 : nqt <= 2 ? 1 : nqt <= 4 ? 2 : nqt <= 8 ? 3 : 4].push_back(i);
  }
  static constexpr uint32_t kClassTiles[5] = {1, 2, 4, 8, 16};
  std::vector<uint32_t> list;
  AllClass cc[5];
  size_t at[5];
  for (int c = 0; c < 5; ++c) {
    cc[c] = all_class(kClassTiles[c], db.dp);
    at[c] = list.size();
    list.insert(list.end(), cls[c].begin(), cls[c].end());
    while ((list.size() - at[c]) % cc[c].qt) list.push_back(kNoQuery);
  }
  if (list.size() > haus_all_list_words(q.n_q)) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyAsync(d_qids, list.data(), list.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the list is a local
  if (e != hipSuccess) return e;
  const uint32_t n_chunks = (uint32_t)((db.n_sets + kAllChunk - 1) / kAllChunk);
  for (int c = 0; c < 5; ++c) {
    if (cls[c].empty()) continue;
    const AllClass k = cc[c];
    const uint32_t* qids = d_qids + at[c];
    const uint32_t n_list = (uint32_t)((c + 1 < 5 ? at[c + 1] : list.size()) - at[c]);
    const uint32_t n_tiles = n_list / k.qt;
    const uint64_t n_units = (uint64_t)n_chunks * n_tiles;
    const uint64_t grid = align_up(n_units, 8);
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const size_t lds = k.qt * haus_stage_bytes(k.rows, db.dp);
    e = dispatch_ks(db.dp, [&](auto ks) -> hipError_t {
      constexpr int KS = decltype(ks)::value;
      auto go_w = [&](uint32_t waves, auto kern, auto... args) -> hipError_t {
        hipError_t r = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(64 * waves), lds, st, db, q, k.rows, n_units, args..., h2);
        return hipGetLastError();
      };
      auto go = [&](auto kern, auto... args) { return go_w(kHausWaves, kern, args...); };
      if (k.qt == 1) {
        if (k.hg) {
          if constexpr (haus_variant_used<KS, 16, true>()) return go(k_haus_all<KS, 16, true>, qids, n_list);
          return hipErrorInvalidValue;
        }
        return go(k_haus_all<KS, 16, false>, qids, n_list);
      }
      // 12 waves where that instance fits 168 VGPRs without spilling
      auto qt_kernel = [&](auto mq, auto hg, auto qt) -> hipError_t {
        constexpr int MQ = decltype(mq)::value, QT = decltype(qt)::value;
        constexpr bool HG = decltype(hg)::value;
        constexpr int WV = !HG && KS <= 6 && (QT == 2 || (QT == 4 && MQ == 2)) ? 12 : (int)kHausWaves;
        return go_w(WV, k_haus_all_qt<KS, MQ, HG, QT, WV>, qids, n_tiles);
      };
      using std::integral_constant;
      if (k.qt == 8)
        return qt_kernel(integral_constant<int, 2>(), std::false_type(), integral_constant<int, 8>());
      auto by_mq = [&](auto mq) -> hipError_t {
        if (k.qt == 4) return k.hg ? qt_kernel(mq, std::true_type(), integral_constant<int, 4>())
                                   : qt_kernel(mq, std::false_type(), integral_constant<int, 4>());
        return k.hg ? qt_kernel(mq, std::true_type(), integral_constant<int, 2>())
                    : qt_kernel(mq, std::false_type(), integral_constant<int, 2>());
      };
      if (k.mqt == 2) return by_mq(std::integral_constant<int, 2>());
      if (k.mqt == 4) return by_mq(std::integral_constant<int, 4>());
      return by_mq(std::integral_constant<int, 8>());
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- top-k
static constexpr uint32_t kTopkChunk = 4096;

// Bitonic sort of the first NP (a power of two, at most 4096) keys.
__device__ void bitonic_sort_4096(uint64_t* k, uint32_t NP) {
  for (uint32_t size = 2; size <= NP; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < NP / 2; i += blockDim.x) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == asc) { k[lo] = b; k[hi] = a; }
      }
      __syncthreads();
    }
  }
}

// Keys are (h2 << 32 | id): ascending order is (distance, id).  Grid
// (chunks, n_q); each block sorts one chunk of up to 4096 keys and keeps k.
__global__ void __launch_bounds__(1024)
k_topk(const uint32_t* __restrict__ h2, const uint32_t* __restrict__ ids_in, const uint32_t* __restrict__ count_in,
       const uint64_t* __restrict__ keys_in, uint64_t n_items, uint64_t stride, uint32_t k,
       uint64_t* __restrict__ keys_out, uint32_t* __restrict__ ids, float* __restrict__ dist,
       uint32_t* __restrict__ count, uint32_t n_valid_total, uint32_t key_is_dist) {
  __shared__ uint64_t s[kTopkChunk];
  const uint32_t q = blockIdx.y, chunk = blockIdx.x;
  const uint64_t n_valid = count_in ? (uint64_t)count_in[q] : n_items;
  const uint64_t base = (uint64_t)chunk * kTopkChunk;
  for (uint32_t i = threadIdx.x; i < kTopkChunk; i += blockDim.x) {
    const uint64_t it = base + i;
    uint64_t key = ~0ull;
    if (it < n_valid) {
      if (keys_in) {
        key = keys_in[(uint64_t)q * stride + it];
      } else {
        const uint32_t id = ids_in ? ids_in[(uint64_t)q * stride + it] : (uint32_t)it;
        key = ((uint64_t)h2[(uint64_t)q * stride + it] << 32) | id;
      }
    }
    s[i] = key;
  }
  __syncthreads();
  // only the valid keys of the chunk need sorting; the padding after them
  // already holds the largest key
  const uint64_t nv_chunk = n_valid > base ? std::min<uint64_t>(n_valid - base, kTopkChunk) : 0;
  uint32_t NP = 2;
  while (NP < nv_chunk) NP <<= 1;
  bitonic_sort_4096(s, NP);
  if (ids) {
    const uint32_t nv = count_in ? count_in[q] : n_valid_total;
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
      const uint64_t key = s[i];
      const bool ok = key != ~0ull;
      ids[(uint64_t)q * k + i] = ok ? (uint32_t)key : 0xFFFFFFFFu;
      const uint32_t hk = (uint32_t)(key >> 32);
      dist[(uint64_t)q * k + i] =
          !ok ? __builtin_inff() : key_is_dist ? __uint_as_float(hk) : sqrtf((float)hk) * (1.0f / 4096.0f);
    }
    if (threadIdx.x == 0) count[q] = min(k, nv);
  } else {
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x)
      keys_out[((uint64_t)q * gridDim.x + chunk) * k + i] = s[i];
  }
}

// Small lists: one wave per query over at most 64 kTopkLaneKeys keys (the
// same keys as k_topk), k rounds of a wave minimum, each taking the winner
// out of its lane (keys are unique: ids or positions differ; padding keys
// are all ones and end the rounds).
static constexpr uint32_t kTopkLaneKeys = 16;
static constexpr uint32_t kTopkWaveMaxK = 64;

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
    v = min(v, (uint64_t)hi << 32 | lo);
  }
  return v;
}

__global__ void __launch_bounds__(256)
k_topk_wave(const uint32_t* __restrict__ h2, const uint32_t* __restrict__ ids_in, const uint32_t* __restrict__ count_in,
            const uint64_t* __restrict__ keys_in, uint64_t n_items, uint64_t stride, uint32_t k, uint32_t n_q,
            uint32_t* __restrict__ ids, float* __restrict__ dist, uint32_t* __restrict__ count,
            uint32_t n_valid_total, uint32_t key_is_dist) {
  const uint32_t q = blockIdx.x * 4 + wave_id(), lane = lane_id();
  if (q >= n_q) return;
  const uint64_t n_valid = count_in ? (uint64_t)count_in[q] : n_items;
  uint64_t key[kTopkLaneKeys];
#pragma unroll
  for (uint32_t u = 0; u < kTopkLaneKeys; ++u) {
    const uint64_t it = lane + (uint64_t)BVS_WAVE * u;
    key[u] = ~0ull;
    if (it < n_valid) {
      if (keys_in) {
        key[u] = keys_in[(uint64_t)q * stride + it];
      } else {
        const uint32_t id = ids_in ? ids_in[(uint64_t)q * stride + it] : (uint32_t)it;
        key[u] = ((uint64_t)h2[(uint64_t)q * stride + it] << 32) | id;
      }
    }
  }
  for (uint32_t i = 0; i < k; ++i) {
    uint64_t m = key[0];
#pragma unroll
    for (uint32_t u = 1; u < kTopkLaneKeys; ++u) m = min(m, key[u]);
    const uint64_t w = wave_min_u64(m);
    if (lane == 0) {
      const bool ok = w != ~0ull;
      ids[(uint64_t)q * k + i] = ok ? (uint32_t)w : 0xFFFFFFFFu;
      const uint32_t hk = (uint32_t)(w >> 32);
      dist[(uint64_t)q * k + i] =
          !ok ? __builtin_inff() : key_is_dist ? __uint_as_float(hk) : sqrtf((float)hk) * (1.0f / 4096.0f);
    }
#pragma unroll
    for (uint32_t u = 0; u < kTopkLaneKeys; ++u) key[u] = key[u] == w ? ~0ull : key[u];
  }
  if (lane == 0) count[q] = min(k, count_in ? count_in[q] : n_valid_total);
}

uint64_t topk_tmp_words(uint64_t n_items, uint32_t n_q, uint32_t k) {
  const uint64_t chunks = (n_items + kTopkChunk - 1) / kTopkChunk;
  return 2 * (uint64_t)n_q * chunks * k + 16;
}

hipError_t launch_topk(const uint32_t* h2, const uint32_t* ids_in, const uint32_t* count_in, uint64_t n_items,
                       uint64_t stride, uint32_t n_q, uint32_t k, uint64_t* tmp, uint32_t* ids, float* dist,
                       uint32_t* count, hipStream_t st, bool key_is_dist) {
  if (n_q == 0) return hipSuccess;
  const uint32_t kd = key_is_dist ? 1u : 0u;
  const uint32_t n_valid_total = (uint32_t)std::min<uint64_t>(n_items, 0xFFFFFFFFull);
  uint64_t chunks = (n_items + kTopkChunk - 1) / kTopkChunk;
  if (chunks == 0) chunks = 1;
  if (count_in && chunks != 1) return hipErrorInvalidValue;   // candidate lists hold at most 4096 items
  const bool wave = k <= kTopkWaveMaxK;   // lists of up to 64 kTopkLaneKeys keys
  if (chunks == 1) {
    if (wave && n_items <= BVS_WAVE * kTopkLaneKeys)
      hipLaunchKernelGGL(k_topk_wave, dim3((n_q + 3) / 4), dim3(256), 0, st, h2, ids_in, count_in,
                         (const uint64_t*)nullptr, n_items, stride, k, n_q, ids, dist, count, n_valid_total, kd);
    else
      hipLaunchKernelGGL(k_topk, dim3(1, n_q), dim3(1024), 0, st, h2, ids_in, count_in, (const uint64_t*)nullptr,
                         n_items, stride, k, (uint64_t*)nullptr, ids, dist, count, n_valid_total, kd);
    return hipGetLastError();
  }
  // First pass: per chunk top-k keys into tmp[0 ..], then merge passes.
  const uint64_t half = (uint64_t)n_q * chunks * k;
  uint64_t* a = tmp;
  uint64_t* b = tmp + half;
  hipLaunchKernelGGL(k_topk, dim3((uint32_t)chunks, n_q), dim3(1024), 0, st, h2, ids_in, count_in,
                     (const uint64_t*)nullptr, n_items, stride, k, a, (uint32_t*)nullptr, (float*)nullptr,
                     (uint32_t*)nullptr, n_valid_total, kd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t n_in = chunks * k;
  while (true) {
    const uint64_t c2 = (n_in + kTopkChunk - 1) / kTopkChunk;
    if (c2 == 1) {
      // Padding keys (all ones) sort last; count = min(k, n_items).
      if (wave && n_in <= BVS_WAVE * kTopkLaneKeys)
        hipLaunchKernelGGL(k_topk_wave, dim3((n_q + 3) / 4), dim3(256), 0, st, (const uint32_t*)nullptr,
                           (const uint32_t*)nullptr, (const uint32_t*)nullptr, a, n_in, n_in, k, n_q, ids, dist,
                           count, n_valid_total, kd);
      else
        hipLaunchKernelGGL(k_topk, dim3(1, n_q), dim3(1024), 0, st, (const uint32_t*)nullptr,
                           (const uint32_t*)nullptr, (const uint32_t*)nullptr, a, n_in, n_in, k, (uint64_t*)nullptr,
                           ids, dist, count, n_valid_total, kd);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      return hipSuccess;
    }
    hipLaunchKernelGGL(k_topk, dim3((uint32_t)c2, n_q), dim3(1024), 0, st, (const uint32_t*)nullptr,
                       (const uint32_t*)nullptr, (const uint32_t*)nullptr, a, n_in, n_in, k, b, (uint32_t*)nullptr,
                       (float*)nullptr, (uint32_t*)nullptr, n_valid_total, kd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(a, b);
    n_in = c2 * k;
  }
}

}  // namespace bvs
