// Full-scan search of Alg. 2 on gfx950: the Hausdorff distance over Hamming
// distances of FlyHash codes (Haus^H) from one query set to every database
// set.
//
// Every code has exactly wta_k = K ones, so Hamming(a, b) = 2K - 2 |a AND b|
// and Haus^H = 2K - 2 min(min_q max_v ov(q, v), min_v max_q ov(q, v)) with
// ov the overlap |q AND v|.  The overlaps are counted bit-sliced:
//
//   query table   T[g][p] (LDS, uint64 per code position p): bit i is set
//                 when vector 64 g + i of the query has position p in its
//                 code (groups g of 64 query vectors)
//   database      each vector stored as its K code positions (uint16, rows
//                 padded to KP = K rounded up to 8), the index's codes in
//                 sparse form
//   one lane      one database set; for each of its vectors, the K table
//                 words of the vector's positions are summed in vertical
//                 counters (Harley-Seal carry-save adders over 64 slots at
//                 once: slot i of plane b is bit b of ov(q_i, v)), which
//                 give ov(q, v) for the 64 query vectors of a group at once
//
// Per vector the counters update the running per-query maxima over the set
// (a bit-sliced maximum) and give the vector's largest overlap over the
// query (a bit-sliced search from the top plane); at the end of the set the
// smallest per-query maximum closes the other direction.  A wave's lanes
// take sets of similar size (the index keeps the sets ordered by size), so
// lanes finish together.
#include "device.h"
#include "launch.h"

namespace bvs {

// ---------------------------------------------------------------- positions
// One wave per vector: word l of the code (lane l < R) holds popcount ones;
// an exclusive prefix over the lanes gives where they go.
__global__ void __launch_bounds__(256)
k_code_positions(const uint64_t* __restrict__ codes, uint64_t n, uint32_t R, uint32_t K, uint32_t KP,
                 uint16_t* __restrict__ pos) {
  const uint32_t lane = lane_id();
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / BVS_WAVE;
  const uint64_t nwaves = (gridDim.x * (uint64_t)blockDim.x) / BVS_WAVE;
  for (uint64_t v = wave; v < n; v += nwaves) {
    uint64_t w = lane < R ? codes[v * R + lane] : 0ull;
    const uint32_t c = popc64(w);
    // inclusive prefix over the wave by shuffles, then exclusive
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, d, BVS_WAVE);
      if ((int)lane >= d) incl += o;
    }
    uint32_t at = incl - c;
    while (w) {
      const uint32_t b = (uint32_t)__builtin_ctzll(w);
      w &= w - 1;
      if (at < K) pos[v * KP + at] = (uint16_t)(64 * lane + b);
      ++at;
    }
  }
}

hipError_t launch_code_positions(const uint64_t* codes, uint64_t n, uint32_t R, uint32_t K, uint32_t KP,
                                 uint16_t* pos, int n_cu, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (R > 64 || KP < K || KP % 8 != 0) return hipErrorInvalidValue;
  const uint64_t want = (n + 3) / 4;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(want, (uint64_t)n_cu * 32);
  hipLaunchKernelGGL(k_code_positions, dim3(grid), dim3(256), 0, st, codes, n, R, K, KP, pos);
  return hipGetLastError();
}

// ---------------------------------------------------------------- query tables
// Queries are packed: a pack is a run of consecutive queries of the batch
// whose vectors fill consecutive slots of up to GP groups of 64 (slot of a
// vector = its index in the batch minus that of the pack's first vector).
// packs[k] = {first query, queries, groups, 0}.
// table[k][g][p] for g < groups: bit i says whether the vector in slot
// 64 g + i has position p in its code.  Grid (L / 256, n_packs).
__global__ void __launch_bounds__(256)
k_query_table(const uint64_t* __restrict__ codes, const uint64_t* __restrict__ q_off, const uint4* __restrict__ packs,
              uint32_t L, uint32_t R, uint32_t GP, uint64_t* __restrict__ table) {
  const uint32_t k = blockIdx.y;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= L) return;
  const uint4 pk = packs[k];
  const uint64_t v0 = q_off[pk.x];
  const uint32_t total = (uint32_t)(q_off[pk.x + pk.y] - v0);
  const uint32_t wd = p / 64, bt = p % 64;
  for (uint32_t g = 0; g < pk.z; ++g) {
    uint64_t m = 0;
    const uint32_t i1 = min(total, 64 * g + 64);
    for (uint32_t i = 64 * g; i < i1; ++i) m |= ((codes[(v0 + i) * R + wd] >> bt) & 1ull) << (i - 64 * g);
    table[((uint64_t)k * GP + g) * L + p] = m;
  }
}

hipError_t launch_query_table(const uint64_t* codes, const uint64_t* q_off, const uint4* packs, uint32_t n_packs,
                              uint32_t L, uint32_t R, uint32_t GP, uint64_t* table, hipStream_t st) {
  if (n_packs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_query_table, dim3((L + 255) / 256, n_packs), dim3(256), 0, st, codes, q_off, packs, L, R, GP,
                     table);
  return hipGetLastError();
}

// ---------------------------------------------------------------- bit-sliced counters
// Carry-save adder on 64 slots: l = a ^ b ^ c (sum), h = majority (carry).
__device__ __forceinline__ void csa(uint64_t& h, uint64_t& l, uint64_t a, uint64_t b, uint64_t c) {
  const uint64_t u = a ^ b;
  h = (a & b) | (u & c);
  l = u ^ c;
}

// Adds a one-bit-per-slot value into planes c[first .. NB).
template <int NB>
__device__ __forceinline__ void ripple_add(uint64_t (&c)[NB], int first, uint64_t x) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b >= first) {
      const uint64_t t = c[b] & x;
      c[b] ^= x;
      x = t;
    }
  }
}

// Slot-wise a = max(a, b) of two NB-bit bit-sliced numbers.
template <int NB>
__device__ __forceinline__ void bs_max(uint64_t (&a)[NB], const uint64_t (&b)[NB]) {
  uint64_t gt = 0, eq = ~0ull;
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    gt |= eq & b[i] & ~a[i];
    eq &= ~(a[i] ^ b[i]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) a[i] = (b[i] & gt) | (a[i] & ~gt);
}

// Largest value among the slots of `valid` (0 when none).
template <int NB>
__device__ __forceinline__ uint32_t bs_max_value(const uint64_t (&a)[NB], uint64_t valid) {
  uint64_t cand = valid;
  uint32_t v = 0;
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    const uint64_t t = cand & a[i];
    if (t) {
      cand = t;
      v |= 1u << i;
    }
  }
  return v;
}

// Smallest value among the slots of `valid` (all ones in NB bits when none).
template <int NB>
__device__ __forceinline__ uint32_t bs_min_value(const uint64_t (&a)[NB], uint64_t valid) {
  if (!valid) return (1u << NB) - 1;
  uint64_t cand = valid;
  uint32_t v = 0;
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    const uint64_t t = cand & ~a[i];
    if (t) {
      cand = t;
    } else {
      v |= 1u << i;
    }
  }
  return v;
}

// ---------------------------------------------------------------- scan
// Sets per workgroup of the scan (one per lane): eight waves share one copy
// of the pack's tables in LDS.
static constexpr uint32_t kScanThreads = 512;

// Slots [64 g, 64 g + 64) of query i of a pack whose queries start at slots
// s[0 .. nq] (s[nq] = the pack's vector count), as a mask of the group.
__device__ __forceinline__ uint64_t pack_mask(uint32_t s0, uint32_t s1, uint32_t g) {
  const uint32_t lo = max(s0, 64 * g), hi = min(s1, 64 * g + 64);
  if (lo >= hi) return 0ull;
  const uint32_t w = hi - lo;
  return (w == 64 ? ~0ull : ((1ull << w) - 1)) << (lo - 64 * g);
}

// Haus^H of the queries of pack blockIdx.y to the sets order[blockIdx.x *
// kScanThreads + t]; scores[q][set] = 2K - 2 ov (uint16).  K code positions
// per vector (row stride KP): the first 16 KB16 are held in registers and
// summed by carry-save blocks of 16, the rest added one at a time; NB >= 5
// planes hold counts up to K.
// LDS: the pack's tables, groups * L uint64.  Per vector, each group's
// counts give ov for its 64 slots: the slot-wise maxima over the set update
// (rowmax), and each query of the group takes the largest count among its
// slots (vmax); at the end each query takes the smallest per-slot maximum
// among its slots.
template <int NB, int GP, int KB16>
__global__ void __launch_bounds__(kScanThreads)
k_full_scan(const uint16_t* __restrict__ pos, const uint64_t* __restrict__ offsets, const uint32_t* __restrict__ order,
            uint64_t n_sets, uint32_t K, uint32_t KP, uint32_t L, const uint64_t* __restrict__ table,
            const uint64_t* __restrict__ q_off, const uint4* __restrict__ packs, uint16_t* __restrict__ scores,
            uint64_t ld) {
  extern __shared__ __align__(16) uint64_t tab[];
  const uint4 pk = packs[blockIdx.y];
  const uint32_t q0 = pk.x, nq = pk.y, ng = pk.z;
  {
    const uint4* src = (const uint4*)(table + (uint64_t)blockIdx.y * GP * L);
    copy_to_lds(src, tab, ng * L / 2);
  }
  uint32_t sl[kPackQ + 1];
  {
    const uint64_t v0 = q_off[q0];
#pragma unroll
    for (int i = 0; i <= kPackQ; ++i) sl[i] = (uint32_t)(q_off[q0 + min((uint32_t)i, nq)] - v0);
  }
  __builtin_amdgcn_s_waitcnt(0);   // the query table has landed in LDS
  __syncthreads();
  const uint64_t it = (uint64_t)blockIdx.x * kScanThreads + threadIdx.x;
  if (it >= n_sets) return;
  const uint32_t j = order[it];
  const uint64_t o0 = offsets[j];
  const uint32_t m = (uint32_t)(offsets[j + 1] - o0);
  uint64_t rowmax[GP][NB];
#pragma unroll
  for (int g = 0; g < GP; ++g)
#pragma unroll
    for (int b = 0; b < NB; ++b) rowmax[g][b] = 0;
  uint32_t colmin[kPackQ];
#pragma unroll
  for (int i = 0; i < kPackQ; ++i) colmin[i] = 0xFFFFu;
  // each vector's first 16 KB16 positions are loaded once for every group,
  // the whole row at once (each of its cache lines fetched once), one
  // vector ahead of its use; one spare word: no zero-length array at KB16 = 0
  uint4 pn[2 * KB16 + 1];
#pragma unroll
  for (int e = 0; e < 2 * KB16; ++e) pn[e] = *(const uint4*)(pos + o0 * KP + 8 * e);
  for (uint32_t v = 0; v < m; ++v) {
    const uint16_t* pv = pos + (o0 + v) * KP;
    uint4 pr[2 * KB16 + 1];
#pragma unroll
    for (int e = 0; e < 2 * KB16; ++e) pr[e] = pn[e];
    if (v + 1 < m) {
#pragma unroll
      for (int e = 0; e < 2 * KB16; ++e) pn[e] = *(const uint4*)(pv + KP + 8 * e);
    }
    uint32_t vmax[kPackQ];
#pragma unroll
    for (int i = 0; i < kPackQ; ++i) vmax[i] = 0;
#pragma unroll
    for (int g = 0; g < GP; ++g) {
      if ((uint32_t)g >= ng) continue;
      const uint64_t* tg = tab + (uint64_t)g * L;
      uint64_t c[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) c[b] = 0;
#pragma unroll
      for (int blk = 0; blk < KB16; ++blk) {
        // 16 positions from two 16-byte words of the row
        const uint4 w0 = pr[2 * blk], w1 = pr[2 * blk + 1];
        const uint32_t pw[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        uint64_t x[16];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          x[2 * e] = tg[pw[e] & 0xFFFFu];
          x[2 * e + 1] = tg[pw[e] >> 16];
        }
        uint64_t twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
        csa(twosA, c[0], c[0], x[0], x[1]);
        csa(twosB, c[0], c[0], x[2], x[3]);
        csa(foursA, c[1], c[1], twosA, twosB);
        csa(twosA, c[0], c[0], x[4], x[5]);
        csa(twosB, c[0], c[0], x[6], x[7]);
        csa(foursB, c[1], c[1], twosA, twosB);
        csa(eightsA, c[2], c[2], foursA, foursB);
        csa(twosA, c[0], c[0], x[8], x[9]);
        csa(twosB, c[0], c[0], x[10], x[11]);
        csa(foursA, c[1], c[1], twosA, twosB);
        csa(twosA, c[0], c[0], x[12], x[13]);
        csa(twosB, c[0], c[0], x[14], x[15]);
        csa(foursB, c[1], c[1], twosA, twosB);
        csa(eightsB, c[2], c[2], foursA, foursB);
        csa(sixteens, c[3], c[3], eightsA, eightsB);
        ripple_add<NB>(c, 4, sixteens);
      }
      for (uint32_t e = 16 * KB16; e < K; ++e) ripple_add<NB>(c, 0, tg[pv[e]]);
      bs_max<NB>(rowmax[g], c);
#pragma unroll
      for (int i = 0; i < kPackQ; ++i) {
        if ((uint32_t)i < nq) {
          const uint64_t mk = pack_mask(sl[i], sl[i + 1], g);
          if (mk) vmax[i] = max(vmax[i], bs_max_value<NB>(c, mk));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kPackQ; ++i) colmin[i] = min(colmin[i], vmax[i]);
  }
#pragma unroll
  for (int i = 0; i < kPackQ; ++i) {
    if ((uint32_t)i < nq) {
      uint32_t rowmin = 0xFFFFu;
#pragma unroll
      for (int g = 0; g < GP; ++g) {
        if ((uint32_t)g < ng) {
          const uint64_t mk = pack_mask(sl[i], sl[i + 1], g);
          if (mk) rowmin = min(rowmin, bs_min_value<NB>(rowmax[g], mk));
        }
      }
      const uint32_t ov = min(colmin[i], rowmin);
      scores[(uint64_t)(q0 + i) * ld + j] = (uint16_t)(2 * K - 2 * ov);
    }
  }
}

// Planes of the counters: enough for K, and at least the five a block of
// 16 inputs reaches.
uint32_t full_planes(uint32_t K) {
  uint32_t b = 5;
  while ((1u << b) <= K) ++b;
  return b;
}

hipError_t launch_full_scan(const uint16_t* pos, const uint64_t* offsets, const uint32_t* order, uint64_t n_sets,
                            uint32_t K, uint32_t KP, uint32_t L, const uint64_t* table, const uint64_t* q_off,
                            const uint4* packs, uint32_t n_packs, uint32_t GP, uint16_t* scores, uint64_t ld,
                            hipStream_t st) {
  if (n_packs == 0 || n_sets == 0) return hipSuccess;
  const uint32_t NB = full_planes(K);
  if (NB > 8 || GP < 1 || GP > kPackGroups || KP < K || KP % 8 != 0 || L % 2 != 0) return hipErrorInvalidValue;
  const uint32_t gp = GP == 1 ? 1u : GP == 2 ? 2u : 4u;
  const size_t lds = (size_t)gp * L * 8;
  const uint64_t blocks = (n_sets + kScanThreads - 1) / kScanThreads;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((uint32_t)blocks, n_packs), dim3(kScanThreads), lds, st, pos, offsets, order, n_sets, K,
                       KP, L, table, q_off, packs, scores, ld);
    return hipGetLastError();
  };
  // blocks of 16 positions held in registers: 4 from K = 64 (7 or 8 planes),
  // 2 from K = 32 (6 planes), none below (5 planes)
  auto by_g = [&](auto nb) -> hipError_t {
    constexpr int B = decltype(nb)::value;
    constexpr int KB = B >= 7 ? 4 : B == 6 ? 2 : 0;
    if (gp == 1) return go(k_full_scan<B, 1, KB>);
    if (gp == 2) return go(k_full_scan<B, 2, KB>);
    return go(k_full_scan<B, 4, KB>);
  };
  switch (NB) {
    case 5: return by_g(std::integral_constant<int, 5>());
    case 6: return by_g(std::integral_constant<int, 6>());
    case 7: return by_g(std::integral_constant<int, 7>());
    default: return by_g(std::integral_constant<int, 8>());
  }
}

}  // namespace bvs
