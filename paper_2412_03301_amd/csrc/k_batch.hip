// Persistent exact re-rank for a batch of queries of uneven size.
//
// One launch covers every query.  Work items are (query, chunk of
// kCandPerBlock candidates); item order is all first chunks, then the other
// chunks query by query, with queries taken largest first (the order array,
// built on the host from the query sizes) so that the big items start early
// and the small ones fill the tail.  Resident workgroups take items from a
// global counter until none are left, so every workgroup ends after at most
// n_items + 1 atomic increments and nothing ever waits on another workgroup.
//
// The first chunk of a query is computed in full; its workgroup then
// publishes the k-th smallest of those distances as the query's bound (an
// atomic word: 0 = not yet, else bound + 1).  A later chunk reads the word
// once when it starts: with a bound it first screens each set on its first
// tile's high planes (haus_core.h) and abandons sets that provably cannot be
// among the k nearest, without one it computes every distance.  Either way
// the k nearest are computed exactly, so the result does not depend on
// timing.
#include "haus_core.h"

namespace bvs {

template <int KS, int NW>
__global__ void __launch_bounds__(64 * NW)
k_haus_queue(HausDb db, HausQ qs, QueueArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_h2[kCandPerBlock];
  const uint32_t n_q = qs.n_q, nch = a.nch;
  const uint32_t n_items = n_q * nch;
  const uint32_t w = wave_id();
  uint32_t rows = 0, abandoned = 0, items = 0, srows = 0, screened = 0;
  uint32_t staged = 0xFFFFFFFFu;
  QView qv;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.ctl, 1u);
    __syncthreads();
    const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
    if (item >= n_items) break;
    uint32_t q, chunk;
    if (item < n_q) {
      q = a.order[item];
      chunk = 0;
    } else {
      const uint32_t j = item - n_q;
      q = a.order[j / (nch - 1)];
      chunk = 1 + j % (nch - 1);
    }
    q = (uint32_t)__builtin_amdgcn_readfirstlane((int)q);
    const uint32_t cnt = a.count[q];
    const uint32_t b0 = chunk * kCandPerBlock;
    if (b0 < cnt) {
      const uint32_t b1 = min(cnt, b0 + kCandPerBlock);
      if (q != staged) {
        qv = stage_query(qs, q, KS * 64, a.lds_rows, smem);
        staged = q;
      }
      uint32_t bound = 0xFFFFFFFFu;
      if (chunk > 0) {
        const uint32_t v = __hip_atomic_load(a.ctl + 1 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) bound = v - 1;
      }
      for (uint32_t it = b0 + w; it < b1; it += NW) {
        const uint32_t j = a.ids[(uint64_t)q * a.T + it];
        const uint64_t o0 = db.offsets[j];
        const uint32_t m = (uint32_t)(db.offsets[j + 1] - o0);
        // candidates after the first chunk: the high-plane screen first
        uint32_t hsq;
        if (bound != 0xFFFFFFFFu && db.scr && qv.sg && screen_set<KS, kMaxQueryTiles, true>(db, o0, m, qv, bound)) {
          hsq = kAbandoned;
          srows += min(16u, m);
          ++screened;
        } else {
          hsq = haus_item<KS, kMaxQueryTiles, true>(db, o0, m, qv, bound, a.stats ? &rows : nullptr);
        }
        if (lane_id() == 0) {
          a.h2[(uint64_t)q * a.T + it] = hsq;
          if (chunk == 0) s_h2[it] = hsq;
        }
        abandoned += hsq == kAbandoned ? 1u : 0u;
        ++items;
      }
      if (chunk == 0 && nch > 1) {
        __syncthreads();
        if (w == 0) {
          const uint32_t lane = lane_id();
          const uint32_t kth = wave_kth_smallest(lane < b1 ? s_h2[lane] : 0xFFFFFFFFu, b1, a.k);
          if (lane == 0 && kth != 0xFFFFFFFFu)
            __hip_atomic_store(a.ctl + 1 + q, kth + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    // the item counter and the staged query are rewritten by the next item
    __syncthreads();
  }
  if (a.stats) {
    stats_add(a.stats, 1, rows, abandoned, items);
    __syncthreads();   // stats_add reuses its LDS words
    stats_add(a.stats, 4, srows, screened);
  }
}

template <typename F>
static hipError_t dispatch_queue(uint32_t dp, uint32_t waves, F&& f) {
  auto by_w = [&](auto ks) -> hipError_t {
    switch (waves) {
      case 2: return f(ks, std::integral_constant<int, 2>());
      case 4: return f(ks, std::integral_constant<int, 4>());
      case 8: return f(ks, std::integral_constant<int, 8>());
      default: return hipErrorInvalidValue;
    }
  };
  switch (dp / 64) {
    case 1: return by_w(std::integral_constant<int, 1>());
    case 2: return by_w(std::integral_constant<int, 2>());
    case 4: return by_w(std::integral_constant<int, 4>());
    case 6: return by_w(std::integral_constant<int, 6>());
    case 8: return by_w(std::integral_constant<int, 8>());
    case 12: return by_w(std::integral_constant<int, 12>());
    case 16: return by_w(std::integral_constant<int, 16>());
    default: return hipErrorInvalidValue;
  }
}

size_t haus_queue_lds_bytes(uint32_t lds_rows, uint32_t dp) { return haus_stage_bytes(lds_rows, dp); }

hipError_t haus_queue_occupancy(uint32_t dp, uint32_t lds_rows, uint32_t waves, uint32_t* blocks_per_cu,
                                uint32_t* spill_bytes) {
  const size_t lds = haus_queue_lds_bytes(lds_rows, dp);
  return dispatch_queue(dp, waves, [&](auto ks, auto nw) -> hipError_t {
    constexpr int KS = decltype(ks)::value, NW = decltype(nw)::value;
    const void* kern = (const void*)k_haus_queue<KS, NW>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipFuncAttributes attr;
    if ((e = hipFuncGetAttributes(&attr, kern)) != hipSuccess) return e;
    int nb = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 64 * NW, lds)) != hipSuccess) return e;
    *blocks_per_cu = (uint32_t)std::max(nb, 0);
    *spill_bytes = (uint32_t)attr.localSizeBytes;
    return hipSuccess;
  });
}

hipError_t launch_haus_queue(const HausDb& db, const HausQ& q, const QueueArgs& a, uint32_t waves, uint32_t blocks,
                             hipStream_t st) {
  if (q.n_q == 0) return hipSuccess;
  if (a.lds_rows == 0 || a.lds_rows % 16 != 0 || blocks == 0) return hipErrorInvalidValue;
  const size_t lds = haus_queue_lds_bytes(a.lds_rows, db.dp);
  hipError_t e = launch_fill_u32(a.ctl, 1ull + q.n_q, 0, st);   // item counter and bounds
  if (e != hipSuccess) return e;
  return dispatch_queue(db.dp, waves, [&](auto ks, auto nw) -> hipError_t {
    constexpr int KS = decltype(ks)::value, NW = decltype(nw)::value;
    auto kern = k_haus_queue<KS, NW>;
    hipError_t e2 = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * NW), lds, st, db, q, a);
    return hipGetLastError();
  });
}

}  // namespace bvs
