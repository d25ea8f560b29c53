// Exact Hausdorff distance (Def. 4) between a query set and database sets on
// the gfx950 matrix cores, and the top-k of the results.
//
// Exactness.  On the 2^-12 grid a = 4096 x is an integer with |a| <= 4096; it
// is stored split as a = 64 hi + lo with hi in [-64, 64] and lo in [0, 63],
// both int8.  Then
//   a . b = 4096 (hi_a . hi_b) + 64 (hi_a . lo_b + lo_a . hi_b) + lo_a . lo_b
// is four int8 x int8 -> int32 matrix-core products, and
//   D2 = |a|^2 + |b|^2 - 2 a . b = 2^24 |x - y|^2
// is an exact integer below 2^28 when both norms are at most 2 (checked when
// the data are converted), so every comparison below is exact and the ranking
// matches a float64 evaluation bit for bit.
//
// Mapping.  One workgroup (8 waves) takes one query and a range of items
// (candidate sets or database sets).  The query's planes sit in LDS with a
// 16-byte row pad; each wave walks its items one at a time, and for each
// 16-vector tile of the item keeps the tile's planes for all of d in
// registers (the A operand: 16 rows x 64 k per lane group) while it loops
// over the query's 16-row tiles read from LDS (the B operand).  The 16x16
// int32 output has database vectors on rows and query vectors on columns:
//   column minimum over q (per database vector) -> DPP row-16 reduction;
//   row minimum over v (per query vector) -> carried per lane across tiles,
//   reduced over the four lane groups at the end of the item.
// Hausdorff^2 = max(max_v min_q D2, max_q min_v D2).
#include "device.h"
#include "launch.h"

namespace bvs {

static constexpr uint32_t kHausWaves = 8;

__host__ __device__ constexpr uint32_t q_row_stride(uint32_t dp) { return dp + 16; }

size_t haus_lds_bytes(uint32_t max_rows, uint32_t dp) {
  const uint32_t rows = (max_rows + 15) / 16 * 16;
  return (size_t)rows * q_row_stride(dp) * 2 + (size_t)rows * 4;
}

// Squared Hausdorff distance (2^24-scaled) of one database set against the
// staged query.  The item is abandoned, returning kAbandoned, as soon as the
// largest completed column minimum (a lower bound of the result) exceeds
// `bound`: such a set cannot be among the k nearest when `bound` is at least
// the k-th smallest distance.
static constexpr uint32_t kAbandoned = 0xFFFFFFFFu;

template <int KS, int MAXQT>
__device__ __forceinline__ uint32_t haus_item(const HausDb& db, uint64_t o0, uint32_t m, const uint8_t* qh_s,
                                              const uint8_t* ql_s, const uint32_t* qn_s, uint32_t mq,
                                              uint32_t nqt, uint32_t bound = 0xFFFFFFFFu,
                                              uint32_t* rows_read = nullptr) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t dp = KS * 64;
  const uint32_t QS = q_row_stride(dp);
  uint32_t qmin[MAXQT];
#pragma unroll
  for (int i = 0; i < MAXQT; ++i) qmin[i] = 0xFFFFFFFFu;
  uint32_t colmax = 0;
  for (uint32_t vt = 0; vt < m; vt += 16) {
    if (rows_read) *rows_read += min(16u, m - vt);
    const uint32_t vrow = vt + c16;
    const bool vrow_ok = vrow < m;
    v4i ah[KS], al[KS];
    {
      const v4i* ph = (const v4i*)(db.hi + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
      const v4i* pl = (const v4i*)(db.lo + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const v4i z = {0, 0, 0, 0};
        ah[k] = vrow_ok ? __builtin_nontemporal_load(ph + 4 * k) : z;
        al[k] = vrow_ok ? __builtin_nontemporal_load(pl + 4 * k) : z;
      }
    }
    uint32_t nv[4], vmin[4];
    bool vok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t v = vt + 4 * g + r;
      vok[r] = v < m;
      nv[r] = vok[r] ? db.norms[o0 + v] : 0u;
      vmin[r] = 0xFFFFFFFFu;
    }
#pragma unroll
    for (int qt = 0; qt < MAXQT; ++qt) {
      if ((uint32_t)qt < nqt) {
        v4i hh = {0, 0, 0, 0}, hl = {0, 0, 0, 0}, lh = {0, 0, 0, 0}, ll = {0, 0, 0, 0};
        const uint8_t* bh = qh_s + (qt * 16 + c16) * QS + 16 * g;
        const uint8_t* bl = ql_s + (qt * 16 + c16) * QS + 16 * g;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const v4i b_h = *(const v4i*)(bh + 64 * k);
          const v4i b_l = *(const v4i*)(bl + 64 * k);
          hh = mfma_i8(ah[k], b_h, hh);
          hl = mfma_i8(ah[k], b_l, hl);
          lh = mfma_i8(al[k], b_h, lh);
          ll = mfma_i8(al[k], b_l, ll);
        }
        const uint32_t qi = qt * 16 + c16;
        const bool qok = qi < mq;
        const uint32_t qn = qn_s[qi];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t dot = (uint32_t)hh[r] * 4096u + ((uint32_t)hl[r] + (uint32_t)lh[r]) * 64u + (uint32_t)ll[r];
          uint32_t d2 = nv[r] + qn - 2u * dot;
          d2 = (qok && vok[r]) ? d2 : 0xFFFFFFFFu;
          vmin[r] = min(vmin[r], d2);
          qmin[qt] = min(qmin[qt], d2);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t cm = row16_min_u32(vmin[r]);
      if (vok[r]) colmax = max(colmax, cm);
    }
    if (bound != 0xFFFFFFFFu && vt + 16 < m && wave_max_u32(colmax) > bound) return kAbandoned;
  }
  uint32_t rowmax = 0;
#pragma unroll
  for (int qt = 0; qt < MAXQT; ++qt) {
    if ((uint32_t)qt < nqt) {
      uint32_t rm = qmin[qt];
      rm = min(rm, shfl_xor_u32(rm, 16));
      rm = min(rm, shfl_xor_u32(rm, 32));
      if ((uint32_t)qt * 16 + c16 < mq) rowmax = max(rowmax, rm);
    }
  }
  return wave_max_u32(max(colmax, rowmax));
}

// Stage query q's planes and norms into LDS (rows padded to 16 with zeros).
__device__ __forceinline__ void stage_query(const HausQ& qs, uint32_t q, uint32_t dp, uint8_t* qh_s, uint8_t* ql_s,
                                            uint32_t* qn_s, uint32_t& mq, uint32_t& nqt) {
  const uint64_t o0 = qs.offsets[q];
  mq = (uint32_t)(qs.offsets[q + 1] - o0);
  nqt = (mq + 15) / 16;
  const uint32_t rows = nqt * 16;
  const uint32_t QS = q_row_stride(dp);
  const uint32_t c16n = dp / 16;
  for (uint32_t i = threadIdx.x; i < rows * c16n; i += blockDim.x) {
    const uint32_t r = i / c16n, c = i % c16n;
    uint4 h = make_uint4(0, 0, 0, 0), l = make_uint4(0, 0, 0, 0);
    if (r < mq) {
      h = *(const uint4*)(qs.hi + (o0 + r) * dp + 16 * c);
      l = *(const uint4*)(qs.lo + (o0 + r) * dp + 16 * c);
    }
    *(uint4*)(qh_s + r * QS + 16 * c) = h;
    *(uint4*)(ql_s + r * QS + 16 * c) = l;
  }
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x) qn_s[r] = r < mq ? qs.norms[o0 + r] : 0u;
  __syncthreads();
}

// Candidate mode: grid (G, n_q).  Block b of query q takes the candidates
// i0 + b * kCandPerBlock ... of ids[q][i0 .. i1), i1 = min(count[q], lim);
// waves take them round-robin.  With bounds != nullptr, candidates whose
// lower bound exceeds bounds[q] are abandoned (h2 = kAbandoned).
static constexpr uint32_t kCandPerBlock = 64;

template <int KS, int MAXQT>
__global__ void __launch_bounds__(64 * kHausWaves)
k_haus_cand(HausDb db, HausQ qs, const uint32_t* __restrict__ ids, const uint32_t* __restrict__ count, uint32_t T,
            uint32_t i0, uint32_t lim, const uint32_t* __restrict__ bounds, uint32_t* __restrict__ h2,
            unsigned long long* __restrict__ stats) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t q = blockIdx.y;
  const uint32_t i1 = min(count[q], lim);
  const uint32_t b0 = i0 + blockIdx.x * kCandPerBlock;
  if (b0 >= i1) return;
  const uint32_t b1 = min(i1, b0 + kCandPerBlock);
  const uint32_t bound = bounds ? bounds[q] : 0xFFFFFFFFu;
  const uint32_t dp = KS * 64;
  const uint32_t rows_max = (qs.max_rows + 15) / 16 * 16;
  uint8_t* qh_s = smem;
  uint8_t* ql_s = smem + rows_max * q_row_stride(dp);
  uint32_t* qn_s = (uint32_t*)(smem + 2 * rows_max * q_row_stride(dp));
  uint32_t mq, nqt;
  stage_query(qs, q, dp, qh_s, ql_s, qn_s, mq, nqt);
  const uint32_t w = wave_id();
  uint32_t rows = 0, abandoned = 0, items = 0;
  for (uint32_t it = b0 + w; it < b1; it += kHausWaves) {
    const uint32_t j = ids[(uint64_t)q * T + it];
    const uint64_t o0 = db.offsets[j];
    const uint32_t m = (uint32_t)(db.offsets[j + 1] - o0);
    const uint32_t hsq = haus_item<KS, MAXQT>(db, o0, m, qh_s, ql_s, qn_s, mq, nqt, bound,
                                              stats ? &rows : nullptr);
    if (lane_id() == 0) h2[(uint64_t)q * T + it] = hsq;
    abandoned += hsq == kAbandoned ? 1u : 0u;
    ++items;
  }
  if (stats) stats_add(stats, 1, rows, abandoned, items);
}

// One wave per query: bounds[q] = k-th smallest of h2[q][0 .. min(count, n)),
// n <= 64, or all ones when fewer than k are there.
__global__ void __launch_bounds__(64)
k_kth_bound(const uint32_t* __restrict__ h2, const uint32_t* __restrict__ count, uint32_t T, uint32_t n, uint32_t k,
            uint32_t* __restrict__ bounds) {
  const uint32_t q = blockIdx.x, lane = lane_id();
  const uint32_t nv = min(count[q], n);
  const uint32_t v = lane < nv ? h2[(uint64_t)q * T + lane] : 0xFFFFFFFFu;
  uint32_t rank = 0;
  for (uint32_t i = 0; i < nv; ++i) {
    const uint32_t o = (uint32_t)__shfl((int)v, (int)i, BVS_WAVE);
    rank += (o < v || (o == v && i < lane)) ? 1u : 0u;
  }
  const uint64_t hit = ballot(lane < nv && rank == k - 1);
  const uint32_t kth = (uint32_t)__shfl((int)v, hit ? (int)__builtin_ctzll(hit) : 0, BVS_WAVE);
  if (lane == 0) bounds[q] = (nv >= k && hit) ? kth : 0xFFFFFFFFu;
}

// All-sets mode.  Work units (query, chunk of kAllChunk sets) are numbered so
// that units sharing a chunk of the database run at the same time on the same
// XCD: consecutive workgroup ids are dealt round-robin over the 8 XCDs, so the
// unit index is rebuilt from (id % 8, id / 8).
static constexpr uint32_t kAllChunk = 128;

template <int KS, int MAXQT>
__global__ void __launch_bounds__(64 * kHausWaves)
k_haus_all(HausDb db, HausQ qs, uint32_t n_chunks, uint64_t n_units, uint32_t* __restrict__ h2) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t b = blockIdx.x, nb = gridDim.x;   // nb is a multiple of 8
  const uint64_t unit = (b % 8) * (nb / 8) + b / 8;
  if (unit >= n_units) return;
  const uint32_t q = (uint32_t)(unit % qs.n_q);
  const uint32_t chunk = (uint32_t)(unit / qs.n_q);
  const uint64_t s0 = (uint64_t)chunk * kAllChunk;
  const uint64_t s1 = min(db.n_sets, s0 + kAllChunk);
  const uint32_t dp = KS * 64;
  const uint32_t rows_max = (qs.max_rows + 15) / 16 * 16;
  uint8_t* qh_s = smem;
  uint8_t* ql_s = smem + rows_max * q_row_stride(dp);
  uint32_t* qn_s = (uint32_t*)(smem + 2 * rows_max * q_row_stride(dp));
  uint32_t mq, nqt;
  stage_query(qs, q, dp, qh_s, ql_s, qn_s, mq, nqt);
  const uint32_t w = wave_id();
  for (uint64_t j = s0 + w; j < s1; j += kHausWaves) {
    const uint64_t o0 = db.offsets[j];
    const uint32_t m = (uint32_t)(db.offsets[j + 1] - o0);
    const uint32_t hsq = haus_item<KS, MAXQT>(db, o0, m, qh_s, ql_s, qn_s, mq, nqt);
    if (lane_id() == 0) h2[(uint64_t)q * db.n_sets + j] = hsq;
  }
  (void)n_chunks;
}

template <typename F>
static hipError_t dispatch_haus(uint32_t dp, uint32_t max_rows, F&& f) {
  const uint32_t nqt = (max_rows + 15) / 16;
  auto by_q = [&](auto ks) -> hipError_t {
    if (nqt <= 2) return f(ks, std::integral_constant<int, 2>());
    if (nqt <= 4) return f(ks, std::integral_constant<int, 4>());
    if (nqt <= 8) return f(ks, std::integral_constant<int, 8>());
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
  // 8 query tiles in registers, and the staged query within 120 KB of LDS.
  uint32_t rows = 128;
  while (rows > 16 && haus_lds_bytes(rows, dp) > 120 * 1024) rows -= 16;
  return rows;
}

// Three exact phases: full distances for the first kCandPerBlock candidates
// (the best by sketch distance), their k-th smallest as a bound per query,
// then the remaining candidates with abandoning against that bound.
hipError_t launch_haus_cand(const HausDb& db, const HausQ& q, const uint32_t* ids, const uint32_t* count,
                            uint32_t T, uint32_t k, uint32_t* thr, uint32_t* h2, unsigned long long* stats,
                            hipStream_t st) {
  if (q.n_q == 0) return hipSuccess;
  const size_t lds = haus_lds_bytes(q.max_rows, db.dp);
  const uint32_t n0 = std::min(T, kCandPerBlock);
  return dispatch_haus(db.dp, q.max_rows, [&](auto ks, auto mqt) -> hipError_t {
    constexpr int KS = decltype(ks)::value, MQ = decltype(mqt)::value;
    hipError_t e = hipFuncSetAttribute((const void*)k_haus_cand<KS, MQ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_haus_cand<KS, MQ>), dim3(1, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, ids, count, T,
                       0u, n0, (const uint32_t*)nullptr, h2, stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (T <= n0) return hipSuccess;
    hipLaunchKernelGGL(k_kth_bound, dim3(q.n_q), dim3(64), 0, st, h2, count, T, n0, k, thr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint32_t G = (T - n0 + kCandPerBlock - 1) / kCandPerBlock;
    hipLaunchKernelGGL((k_haus_cand<KS, MQ>), dim3(G, q.n_q), dim3(64 * kHausWaves), lds, st, db, q, ids, count, T,
                       n0, T, (const uint32_t*)thr, h2, stats);
    return hipGetLastError();
  });
}

hipError_t launch_haus_all(const HausDb& db, const HausQ& q, uint32_t* h2, hipStream_t st) {
  if (q.n_q == 0 || db.n_sets == 0) return hipSuccess;
  const uint32_t n_chunks = (uint32_t)((db.n_sets + kAllChunk - 1) / kAllChunk);
  const uint64_t n_units = (uint64_t)n_chunks * q.n_q;
  const uint64_t grid = align_up(n_units, 8);
  if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const size_t lds = haus_lds_bytes(q.max_rows, db.dp);
  return dispatch_haus(db.dp, q.max_rows, [&](auto ks, auto mqt) -> hipError_t {
    constexpr int KS = decltype(ks)::value, MQ = decltype(mqt)::value;
    hipError_t e = hipFuncSetAttribute((const void*)k_haus_all<KS, MQ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_haus_all<KS, MQ>), dim3((uint32_t)grid), dim3(64 * kHausWaves), lds, st, db, q,
                       n_chunks, n_units, h2);
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------- top-k
static constexpr uint32_t kTopkChunk = 4096;

__device__ void bitonic_sort_4096(uint64_t* k) {
  for (uint32_t size = 2; size <= kTopkChunk; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < kTopkChunk / 2; i += blockDim.x) {
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
       uint32_t* __restrict__ count, uint32_t n_valid_total) {
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
  bitonic_sort_4096(s);
  if (ids) {
    const uint32_t nv = count_in ? count_in[q] : n_valid_total;
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
      const uint64_t key = s[i];
      const bool ok = key != ~0ull;
      ids[(uint64_t)q * k + i] = ok ? (uint32_t)key : 0xFFFFFFFFu;
      dist[(uint64_t)q * k + i] = ok ? sqrtf((float)(uint32_t)(key >> 32)) * (1.0f / 4096.0f) : __builtin_inff();
    }
    if (threadIdx.x == 0) count[q] = min(k, nv);
  } else {
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x)
      keys_out[((uint64_t)q * gridDim.x + chunk) * k + i] = s[i];
  }
}

uint64_t topk_tmp_words(uint64_t n_items, uint32_t n_q, uint32_t k) {
  const uint64_t chunks = (n_items + kTopkChunk - 1) / kTopkChunk;
  return 2 * (uint64_t)n_q * chunks * k + 16;
}

hipError_t launch_topk(const uint32_t* h2, const uint32_t* ids_in, const uint32_t* count_in, uint64_t n_items,
                       uint64_t stride, uint32_t n_q, uint32_t k, uint64_t* tmp, uint32_t* ids, float* dist,
                       uint32_t* count, hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  const uint32_t n_valid_total = (uint32_t)std::min<uint64_t>(n_items, 0xFFFFFFFFull);
  uint64_t chunks = (n_items + kTopkChunk - 1) / kTopkChunk;
  if (chunks == 0) chunks = 1;
  if (count_in && chunks != 1) return hipErrorInvalidValue;   // candidate lists hold at most 4096 items
  if (chunks == 1) {
    hipLaunchKernelGGL(k_topk, dim3(1, n_q), dim3(1024), 0, st, h2, ids_in, count_in, (const uint64_t*)nullptr,
                       n_items, stride, k, (uint64_t*)nullptr, ids, dist, count, n_valid_total);
    return hipGetLastError();
  }
  // First pass: per chunk top-k keys into tmp[0 ..], then merge passes.
  const uint64_t half = (uint64_t)n_q * chunks * k;
  uint64_t* a = tmp;
  uint64_t* b = tmp + half;
  hipLaunchKernelGGL(k_topk, dim3((uint32_t)chunks, n_q), dim3(1024), 0, st, h2, ids_in, count_in,
                     (const uint64_t*)nullptr, n_items, stride, k, a, (uint32_t*)nullptr, (float*)nullptr,
                     (uint32_t*)nullptr, n_valid_total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t n_in = chunks * k;
  while (true) {
    const uint64_t c2 = (n_in + kTopkChunk - 1) / kTopkChunk;
    if (c2 == 1) {
      // Padding keys (all ones) sort last; count = min(k, n_items).
      hipLaunchKernelGGL(k_topk, dim3(1, n_q), dim3(1024), 0, st, (const uint32_t*)nullptr, (const uint32_t*)nullptr,
                         (const uint32_t*)nullptr, a, n_in, n_in, k, (uint64_t*)nullptr, ids, dist, count,
                         n_valid_total);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      return hipSuccess;
    }
    hipLaunchKernelGGL(k_topk, dim3((uint32_t)c2, n_q), dim3(1024), 0, st, (const uint32_t*)nullptr,
                       (const uint32_t*)nullptr, (const uint32_t*)nullptr, a, n_in, n_in, k, b, (uint32_t*)nullptr,
                       (float*)nullptr, (uint32_t*)nullptr, n_valid_total);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(a, b);
    n_in = c2 * k;
  }
}

}  // namespace bvs
