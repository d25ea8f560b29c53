// Winner-take-all threshold of a wave: the k-th largest of the 64 R keys the
// wave's lanes hold (Def. 7: the k largest outputs of a vector's projection
// become its code).  Shared by the FlyHash encoders and the learned
// projection's rows.
#pragma once

#include "device.h"

namespace bvs {

// The k-th largest of the values v[0 .. N) of all lanes (unique across the
// wave), bit by bit below the high bits already fixed in theta: a prefix
// above the largest value kmax admits none, so those bits are skipped.
template <int N>
__device__ __forceinline__ uint32_t kth_search(const uint32_t (&v)[N], uint32_t k, int b0, uint32_t theta,
                                               uint32_t kmax) {
  for (int b = b0; b >= 0; --b) {
    const uint32_t cand = theta | (1u << b);
    if (cand > kmax) continue;
    // per-lane count, then one wave sum (no per-key ballots held in scalars)
    uint32_t local = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) local += v[t] >= cand ? 1u : 0u;
    const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_sum_dpp_u32(local));
    if (cnt == k) {
      // Exactly k values reach the prefix: the k-th largest is their minimum.
      uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
      for (int t = 0; t < N; ++t) mn = v[t] >= cand ? min(mn, v[t]) : mn;
      return wave_min_dpp_u32(mn);
    }
    if (cnt > k) theta = cand;
  }
  return theta;
}

// Middle value of three.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// The k-th largest of the wave's 64 R unique keys.  For k <= 64 the smallest
// of the 64 lanes' largest keys is a lower bound (64 distinct keys reach it):
// the answer lies between it and the largest key, so it shares their common
// high bits, which are set without counting.  With R >= 16 the search first
// runs over each lane's KT = 6 largest keys (kept sorted as the keys stream
// by: a maximum and KT - 1 medians of three per key); its result th is the
// k-th largest of all keys whenever no lane's last kept key reaches th (then
// every key at or above th is kept), else the search runs again over all
// keys.  (For FlyHash codes at L = 4096 and k = 64 a lane holds more than 6
// of the 64 largest keys for about one vector in a hundred.)
template <int R>
__device__ __forceinline__ uint32_t kth_largest(uint32_t (&key)[R], uint32_t k, int topbit) {
  uint32_t lm = 0;
#pragma unroll
  for (int t = 0; t < R; ++t) lm = max(lm, key[t]);
  const uint32_t kmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_dpp_u32(lm));
  uint32_t theta = 0;
  int b0 = topbit;
  if (k <= 64) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min_dpp_u32(lm));
    const uint32_t diff = lo ^ kmax;
    if (diff != 0) {
      const int hb = 31 - __builtin_clz(diff);
      theta = hb >= 31 ? 0u : (kmax & ~((2u << hb) - 1u));
      b0 = min(b0, hb);
    }
    if constexpr (R >= 16) {
      // The keys are all computed before the first is kept: left free to
      // interleave the keeping with the code that computes the keys, the
      // compiler can hold more values live than the register budget and
      // spill.
#pragma unroll
      for (int t = 0; t < R; ++t) asm volatile("" : "+v"(key[t]));
      constexpr int KT = 6;
      uint32_t c[KT];
#pragma unroll
      for (int i = 0; i < KT; ++i) c[i] = 0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const uint32_t x = key[t];
#pragma unroll
        for (int i = KT - 1; i >= 1; --i) c[i] = med3_u32(c[i - 1], c[i], x);
        c[0] = max(c[0], x);
      }
      const uint32_t th = kth_search<KT>(c, k, b0, theta, kmax);
      if (ballot(c[KT - 1] >= th) == 0) return th;
    }
  }
  return kth_search<R>(key, k, b0, theta, kmax);
}

}  // namespace bvs
