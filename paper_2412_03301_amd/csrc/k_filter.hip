// Both filter layers of the cascade search (Alg. 6) on gfx950.
//
// filter     one thread per database set, a tile of QT queries per workgroup:
//            streams the set's binary Bloom filter in 128-bit chunks from the
//            chunk-major layout (64 consecutive sets per wave instruction,
//            1 KB contiguous), XOR + popcount against each query sketch (the
//            query words are wave-uniform and come through scalar loads), and
//            applies the first layer: with M = 1, C[p] >= 1 is the sketch bit p,
//            tested in the chunk that holds p; with M >= 2 the count columns
//            C[p][set] are read; M = 0 admits every set.
// select     the first min(T, |F1|) sets by (score, id).  Main path: score a
//            spread sample of 64 blocks of 256 sets, take per query the score
//            whose sample rank corresponds to about 3 T sets of the whole
//            database as a cutoff, then score every set once more, appending
//            only members with score <= cutoff (bounded buffer), and sort the
//            appended (score, id) keys.  The result is exact whenever the
//            buffer did not overflow and it holds at least T sets (or the
//            cutoff admitted every member); otherwise the caller runs the
//            dense path: every score is written, a histogram gives the
//            threshold tau, scores < tau are appended unordered, ties at tau
//            are filled lowest ids first, and a bitonic sort orders F2.
//            Both paths are deterministic and give identical F2.
#include "device.h"
#include "launch.h"

namespace bvs {

// Grid rows of a launch gated on a device flag (see FilterArgs::run_if).
static constexpr uint32_t kGatedRows = 8;

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Scores of one block of 256 sets against QT queries.  Set block b of the
// grid is blockIdx.x * block_stride.  Dense mode writes every score
// (0xFFFF = not in F1) to scores[q][blockIdx.x * 256 + t]; append mode keeps
// only F1 members with score <= cutoff[q], appending (score << 32 | id) to
// cand[q][0 .. cap) and counting them in cand_count[q] (the count may exceed
// cap; the entries beyond cap are dropped and the caller detects it).
template <int QT, bool APPEND>
__device__ __forceinline__ void filter_tile(const FilterArgs& a, uint32_t q0) {
  const uint64_t j = (uint64_t)blockIdx.x * a.block_stride * 256ull + threadIdx.x;
  const uint32_t nq = min((uint32_t)QT, a.n_q - q0);
  const uint32_t lane = lane_id();
  const uint32_t M = a.M;
  uint32_t acc[QT], hit[QT];
  uint64_t gcm[QT];
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    acc[i] = 0;
    hit[i] = 0;
    gcm[i] = (M == 1 && (uint32_t)i < nq) ? a.gate_chunks[q0 + i] : 0;
  }
  const uint4* col = a.bits + j;
  const uint32_t RC = a.RC;
  const uint64_t ld = a.ld;
#pragma unroll 4
  for (uint32_t c = 0; c < RC; ++c) {
    const uint4 x = col[(uint64_t)c * ld];
#pragma unroll
    for (int i = 0; i < QT; ++i) {
      if ((uint32_t)i < nq) {
        const uint4 s = a.sq[(uint64_t)(q0 + i) * RC + c];
        acc[i] += popc32(x.x ^ s.x) + popc32(x.y ^ s.y) + popc32(x.z ^ s.z) + popc32(x.w ^ s.w);
        if ((gcm[i] >> c) & 1) {
          const uint4 g = a.gate[(uint64_t)(q0 + i) * RC + c];
          hit[i] |= (x.x & g.x) | (x.y & g.y) | (x.z & g.z) | (x.w & g.w);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    if ((uint32_t)i < nq) {
      const uint32_t q = q0 + i;
      bool member;
      if (a.member) {
        member = (a.member[(uint64_t)q * (ld / 64) + j / 64] >> (j % 64)) & 1ull;
      } else if (M == 0) {
        member = true;
      } else if (M == 1) {
        member = hit[i] != 0;
      } else {
        member = false;
        for (uint32_t t = 0; t < a.A; ++t) {
          const uint32_t p = a.pos[(uint64_t)q * a.A + t];
          member |= a.cnt[(uint64_t)p * ld + j] >= M;
        }
      }
      member = member && j < a.n_sets;
      if (!APPEND) {
        a.scores[(uint64_t)q * a.ld_out + (uint64_t)blockIdx.x * 256 + threadIdx.x] =
            member ? (uint16_t)acc[i] : (uint16_t)0xFFFF;
      } else {
        const bool take = member && acc[i] <= a.cutoff[q];
        const uint64_t tb = ballot(take);
        if (tb) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&a.cand_count[q], popc64(tb));
          base = (uint32_t)__shfl((int)base, 0, BVS_WAVE);
          const uint32_t slot = base + mbcnt64(tb);
          if (take && slot < a.cap) a.cand[(uint64_t)q * a.cap + slot] = ((uint64_t)acc[i] << 32) | (uint32_t)j;
        }
      }
    }
  }
}

// Grid (set blocks, y): block y takes query tiles y, y + gridDim.y, ...
template <int QT, bool APPEND>
__global__ void __launch_bounds__(256)
k_filter(FilterArgs a) {
  if (!APPEND && a.run_if && *a.run_if == 0) return;
  for (uint32_t q0 = blockIdx.y * QT; q0 < a.n_q; q0 += gridDim.y * QT) filter_tile<QT, APPEND>(a, q0);
}

template <bool APPEND>
static hipError_t go_filter(const FilterArgs& a, uint32_t n_blocks, hipStream_t st) {
  auto go = [&](auto qt) -> hipError_t {
    constexpr int QT = decltype(qt)::value;
    // a gated launch usually does nothing: few blocks, each looping over tiles
    const uint32_t tiles = (a.n_q + QT - 1) / QT;
    dim3 grid(n_blocks, a.run_if ? std::min(tiles, kGatedRows) : tiles);
    hipLaunchKernelGGL((k_filter<QT, APPEND>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
  };
  if (a.n_q >= 16) return go(std::integral_constant<int, 16>());
  if (a.n_q >= 8) return go(std::integral_constant<int, 8>());
  if (a.n_q >= 4) return go(std::integral_constant<int, 4>());
  return go(std::integral_constant<int, 1>());
}

hipError_t launch_filter_dense(FilterArgs a, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  a.block_stride = 1;
  a.ld_out = a.ld;
  return go_filter<false>(a, (uint32_t)(a.ld / 256), st);
}

hipError_t launch_filter_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)(a.ld / 256);
  a.block_stride = std::max(1u, nb / n_sample_blocks);
  a.ld_out = (uint64_t)n_sample_blocks * 256;
  return go_filter<false>(a, n_sample_blocks, st);
}

hipError_t launch_filter_append(FilterArgs a, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  a.block_stride = 1;
  return go_filter<true>(a, (uint32_t)(a.ld / 256), st);
}

// ---------------------------------------------------------------- member-only scoring
// First-layer membership of the 256 sets of a tile for query q, as four
// 64-bit masks (uniform across the wave).
__device__ __forceinline__ void tile_members(const FilterArgs& a, uint32_t q, uint64_t tile0, uint32_t lane,
                                             const uint64_t (&vmask)[4], uint64_t (&m)[4]) {
  if (a.member) {
    // first layer read from the inverted lists
    const cptr<uint64_t> mb = as_const(a.member) + (uint64_t)q * (a.ld / 64) + tile0 / 64;
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = mb[i] & vmask[i];
  } else if (a.M == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = vmask[i];
  } else if (a.M == 1) {
    // C[p] >= 1 for one of the query's A positions: OR of their bitmap rows
    const cptr<uint64_t> pl = as_const(a.planes) + (tile0 / 256) * a.L * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = 0;
    for (uint32_t t = 0; t < a.A; ++t) {
      const uint64_t r = (uint64_t)as_const(a.pos)[(uint64_t)q * a.A + t] * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) m[i] |= pl[r + i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] &= vmask[i];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bool mem = false;
      for (uint32_t t = 0; t < a.A; ++t) {
        const uint32_t p = a.pos[(uint64_t)q * a.A + t];
        mem |= a.cnt[(uint64_t)p * a.ld + tile0 + 64u * i + lane] >= a.M;
      }
      m[i] = ballot(mem) & vmask[i];
    }
  }
}

// One workgroup (16 waves) per tile of 256 sets; the tile's binary Bloom
// filters are staged in LDS chunk-major ([chunk][set], 16 B per entry).
// Each wave takes whole queries: it reads the query's first-layer masks for
// the tile (prefetched one query ahead), compacts the members into lanes
// (ascending set order) and computes the Hamming distance only for them.
// Chunks are processed in groups of 8: the group's query words come through
// scalar loads and its tile entries through LDS reads, then one wait covers
// both (scalar and LDS loads share a completion counter), then 8 VALU
// operations per chunk and member.
template <int RC, bool APPEND>
__global__ void __launch_bounds__(1024)
k_filter_sparse(FilterArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  constexpr uint32_t NW = 16;
  constexpr int G = RC < 8 ? RC : 8;
  uint4* tile = (uint4*)smem;                         // [RC][256]
  uint8_t* lists = smem + (size_t)RC * 256 * 16;      // [NW][256]
  const uint64_t tile0 = (uint64_t)blockIdx.x * a.block_stride * 256ull;
  for (uint32_t i = threadIdx.x; i < RC * 256; i += blockDim.x) {
    const uint32_t c = i / 256, s = i % 256;
    tile[i] = a.bits[(uint64_t)c * a.ld + tile0 + s];
  }
  __syncthreads();
  const uint32_t w = wave_id(), lane = lane_id();
  uint8_t* list = lists + w * 256;
  uint64_t vmask[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t b = tile0 + 64u * i;
    vmask[i] = b >= a.n_sets ? 0ull : (a.n_sets - b >= 64 ? ~0ull : (1ull << (a.n_sets - b)) - 1);
  }
  uint64_t mn[4];
  uint64_t pairs = 0;
  if (w < a.n_q) tile_members(a, w, tile0, lane, vmask, mn);
  for (uint32_t q = w; q < a.n_q; q += NW) {
    uint64_t m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = mn[i];
    if (q + NW < a.n_q) tile_members(a, q + NW, tile0, lane, vmask, mn);
    const uint32_t nm = popc64(m[0]) + popc64(m[1]) + popc64(m[2]) + popc64(m[3]);
    pairs += nm;
    if (nm == 0) continue;
    uint32_t base = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if ((m[i] >> lane) & 1) list[base + mbcnt64(m[i])] = (uint8_t)(64 * i + lane);
      base += popc64(m[i]);
    }
    wave_lds_sync();
    const cptr<uint4> sqq = as_const(a.sq) + (uint64_t)q * RC;
    const uint32_t cut = APPEND ? as_const(a.cutoff)[q] : 0u;
    for (uint32_t g = 0; g < nm; g += 64) {
      const uint32_t idx = g + lane;
      const bool act = idx < nm;
      const uint32_t sl = act ? list[idx] : 0u;
      uint32_t acc = 0;
      for (int c0 = 0; c0 < RC; c0 += G) {
        // keep the query words per group in scalar registers (not hoisted)
        asm volatile("" ::: "memory");
        uint4 sv[G], xv[G];
#pragma unroll
        for (int j = 0; j < G; ++j) sv[j] = sqq[c0 + j];
#pragma unroll
        for (int j = 0; j < G; ++j) xv[j] = tile[(c0 + j) * 256 + sl];
#pragma unroll
        for (int j = 0; j < G; ++j)
          acc += popc32(xv[j].x ^ sv[j].x) + popc32(xv[j].y ^ sv[j].y) + popc32(xv[j].z ^ sv[j].z) +
                 popc32(xv[j].w ^ sv[j].w);
      }
      if (!APPEND) {
        if (act) a.scores[(uint64_t)q * a.ld_out + (uint64_t)blockIdx.x * 256 + sl] = (uint16_t)acc;
      } else {
        const bool take = act && acc <= cut;
        const uint64_t tb = ballot(take);
        if (tb) {
          uint32_t b0 = 0;
          if (lane == 0) b0 = atomicAdd(&a.cand_count[q], popc64(tb));
          b0 = (uint32_t)__shfl((int)b0, 0, BVS_WAVE);
          const uint32_t slot = b0 + mbcnt64(tb);
          if (take && slot < a.cap) a.cand[(uint64_t)q * a.cap + slot] = ((uint64_t)acc << 32) | (uint32_t)(tile0 + sl);
        }
      }
    }
    wave_lds_sync();
  }
  if (APPEND && a.stats) stats_add(a.stats, 0, (uint32_t)pairs);
}

template <bool APPEND>
static hipError_t go_sparse(const FilterArgs& a, uint32_t n_blocks, hipStream_t st) {
  auto go = [&](auto rc) -> hipError_t {
    constexpr int RC = decltype(rc)::value;
    const size_t lds = (size_t)RC * 256 * 16 + 16 * 256;
    hipError_t e = hipFuncSetAttribute((const void*)k_filter_sparse<RC, APPEND>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_filter_sparse<RC, APPEND>), dim3(n_blocks), dim3(1024), lds, st, a);
    return hipGetLastError();
  };
  switch (a.RC) {
    case 2: return go(std::integral_constant<int, 2>());
    case 4: return go(std::integral_constant<int, 4>());
    case 8: return go(std::integral_constant<int, 8>());
    case 16: return go(std::integral_constant<int, 16>());
    case 32: return go(std::integral_constant<int, 32>());
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_filter_sparse_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)(a.ld / 256);
  a.block_stride = std::max(1u, nb / n_sample_blocks);
  a.ld_out = (uint64_t)n_sample_blocks * 256;
  return go_sparse<false>(a, n_sample_blocks, st);
}

hipError_t launch_filter_sparse_append(FilterArgs a, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  a.block_stride = 1;
  return go_sparse<true>(a, (uint32_t)(a.ld / 256), st);
}

// ---------------------------------------------------------------- select
static constexpr uint32_t SEL_CH = 4096;   // sets per block in the dense select passes

uint32_t select_blocks(uint64_t ld) { return (uint32_t)((ld + SEL_CH - 1) / SEL_CH); }

// Exclusive scan of one flag per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan_flag(bool f, uint32_t* wsum, uint32_t& total) {
  const uint32_t lane = lane_id(), w = threadIdx.x / BVS_WAVE;
  const uint64_t m = ballot(f);
  const uint32_t r = mbcnt64(m);
  if (lane == 0) wsum[w] = popc64(m);
  __syncthreads();
  uint32_t base = 0;
  total = 0;
  for (uint32_t i = 0; i < 4; ++i) {
    const uint32_t s = wsum[i];
    if (i < w) base += s;
    total += s;
  }
  __syncthreads();
  return base + r;
}

__device__ __forceinline__ void hist_query(const uint16_t* __restrict__ scores, uint64_t ld, uint32_t L,
                                           uint32_t* __restrict__ hist, uint32_t q, uint32_t* h) {
  const uint32_t nb = L + 2;
  for (uint32_t i = threadIdx.x; i < nb; i += 256) h[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * SEL_CH;
  const uint16_t* sc = scores + (uint64_t)q * ld;
  for (uint32_t i = threadIdx.x * 8; i < SEL_CH; i += 256 * 8) {
    if (base + i < ld) {
      const uint4 v = *(const uint4*)(sc + base + i);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t s = (w[e / 2] >> (16 * (e % 2))) & 0xFFFF;
        atomicAdd(&h[s == 0xFFFF ? L + 1 : s], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t* gh = hist + (uint64_t)q * nb;
  for (uint32_t i = threadIdx.x; i < nb; i += 256)
    if (h[i]) atomicAdd(&gh[i], h[i]);
  __syncthreads();   // h is cleared again for the next query
}

// Grid (blocks of SEL_CH sets, y): block y takes queries y, y + gridDim.y, ...
__global__ void __launch_bounds__(256)
k_hist(const uint16_t* __restrict__ scores, uint64_t ld, uint32_t L, uint32_t n_q, uint32_t* __restrict__ hist,
       const uint32_t* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  extern __shared__ uint32_t h[];
  for (uint32_t q = blockIdx.y; q < n_q; q += gridDim.y) hist_query(scores, ld, L, hist, q, h);
}

// One block per query: tau = smallest score s with #{score <= s} >= Tq,
// Tq = min(T, |F1|).
__global__ void __launch_bounds__(256)
k_threshold(const uint32_t* __restrict__ hist, uint32_t L, uint32_t T, uint32_t* __restrict__ sel,
            uint32_t* __restrict__ ctr, const uint32_t* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  __shared__ uint32_t part[256];
  __shared__ uint32_t total_s;
  const uint32_t q = blockIdx.x, t = threadIdx.x;
  const uint32_t* h = hist + (uint64_t)q * (L + 2);
  const uint32_t nb = L + 1;   // scores 0..L
  const uint32_t per = (nb + 255) / 256;
  const uint32_t b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += h[b];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (uint32_t i = 0; i < 256; ++i) { const uint32_t v = part[i]; part[i] = run; run += v; }
    total_s = run;
  }
  __syncthreads();
  const uint32_t total = total_s;
  const uint32_t Tq = min(T, total);
  uint32_t* sq = sel + (uint64_t)q * 4;
  if (t == 0) {
    ctr[q] = 0;
    if (Tq == 0) { sq[0] = 0xFFFFFFFFu; sq[1] = 0; sq[2] = 0; sq[3] = 0; }
  }
  if (Tq == 0) return;
  const uint32_t pre = part[t];
  if (pre < Tq && pre + s >= Tq) {
    uint32_t cum = pre;
    for (uint32_t b = b0; b < b1; ++b) {
      if (cum + h[b] >= Tq) {
        sq[0] = b; sq[1] = cum; sq[2] = Tq - cum; sq[3] = Tq;
        break;
      }
      cum += h[b];
    }
  }
}

__device__ __forceinline__ void compact_query(const uint16_t* __restrict__ scores, uint64_t ld,
                                              const uint32_t* __restrict__ sel, uint32_t* __restrict__ ctr,
                                              uint32_t* __restrict__ eqcnt, uint32_t nblk,
                                              uint64_t* __restrict__ cand, uint32_t T, uint32_t q, uint32_t* wsum) {
  const uint32_t blk = blockIdx.x, lane = lane_id();
  const uint32_t tau = sel[(uint64_t)q * 4], Tq = sel[(uint64_t)q * 4 + 3];
  uint32_t eq = 0;
  if (Tq != 0) {
    const uint64_t base = (uint64_t)blk * SEL_CH;
    const uint16_t* sc = scores + (uint64_t)q * ld;
    for (uint32_t i = threadIdx.x; i < SEL_CH; i += 256) {
      const uint64_t jj = base + i;
      const uint32_t s = jj < ld ? sc[jj] : 0xFFFFu;
      const bool below = s < tau;
      eq += (s == tau) ? 1u : 0u;
      const uint64_t m = ballot(below);
      if (m) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(&ctr[q], popc64(m));
        b = (uint32_t)__shfl((int)b, 0, BVS_WAVE);
        if (below) cand[(uint64_t)q * T + b + mbcnt64(m)] = ((uint64_t)s << 32) | (uint32_t)jj;
      }
    }
  }
  eq = wave_sum_u32(eq);
  if (lane == 0) wsum[threadIdx.x / BVS_WAVE] = eq;
  __syncthreads();
  if (threadIdx.x == 0) eqcnt[(uint64_t)q * nblk + blk] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();   // wsum is rewritten for the next query
}

__global__ void __launch_bounds__(256)
k_compact(const uint16_t* __restrict__ scores, uint64_t ld, uint32_t n_q, const uint32_t* __restrict__ sel,
          uint32_t* __restrict__ ctr, uint32_t* __restrict__ eqcnt, uint32_t nblk, uint64_t* __restrict__ cand,
          uint32_t T, const uint32_t* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  __shared__ uint32_t wsum[4];
  for (uint32_t q = blockIdx.y; q < n_q; q += gridDim.y) compact_query(scores, ld, sel, ctr, eqcnt, nblk, cand, T, q, wsum);
}

// Every early return is uniform over the block.
__device__ __forceinline__ void ties_query(const uint16_t* __restrict__ scores, uint64_t ld,
                                           const uint32_t* __restrict__ sel, const uint32_t* __restrict__ eqcnt,
                                           uint32_t nblk, uint64_t* __restrict__ cand, uint32_t T, uint32_t q,
                                           uint32_t* wsum, uint32_t* red) {
  const uint32_t blk = blockIdx.x;
  const uint32_t tau = sel[(uint64_t)q * 4], cb = sel[(uint64_t)q * 4 + 1], ne = sel[(uint64_t)q * 4 + 2];
  if (ne == 0) return;
  const uint32_t* ec = eqcnt + (uint64_t)q * nblk;
  if (ec[blk] == 0) return;
  uint32_t p = 0;
  for (uint32_t b = threadIdx.x; b < blk; b += 256) p += ec[b];
  p = wave_sum_u32(p);
  if (lane_id() == 0) red[threadIdx.x / BVS_WAVE] = p;
  __syncthreads();
  uint32_t prefix = red[0] + red[1] + red[2] + red[3];
  if (prefix >= ne) return;   // uniform across the block
  const uint64_t base = (uint64_t)blk * SEL_CH;
  const uint16_t* sc = scores + (uint64_t)q * ld;
  for (uint32_t i0 = 0; i0 < SEL_CH && prefix < ne; i0 += 256) {
    const uint64_t jj = base + i0 + threadIdx.x;
    const bool f = jj < ld && sc[jj] == tau;
    uint32_t tot;
    const uint32_t r = block_excl_scan_flag(f, wsum, tot);
    if (f && prefix + r < ne) cand[(uint64_t)q * T + cb + prefix + r] = ((uint64_t)tau << 32) | (uint32_t)jj;
    prefix += tot;
  }
}

__global__ void __launch_bounds__(256)
k_ties(const uint16_t* __restrict__ scores, uint64_t ld, uint32_t n_q, const uint32_t* __restrict__ sel,
       const uint32_t* __restrict__ eqcnt, uint32_t nblk, uint64_t* __restrict__ cand, uint32_t T,
       const uint32_t* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t red[4];
  for (uint32_t q = blockIdx.y; q < n_q; q += gridDim.y) {
    ties_query(scores, ld, sel, eqcnt, nblk, cand, T, q, wsum, red);
    __syncthreads();   // red and wsum are rewritten for the next query
  }
}

// Bitonic sort of NP (power of two) u64 keys in LDS by a block of 512 threads.
__device__ void bitonic_sort_lds(uint64_t* k, uint32_t NP) {
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

__global__ void __launch_bounds__(512)
k_sort_f2(const uint64_t* __restrict__ cand, const uint32_t* __restrict__ sel, uint32_t T, uint32_t NP,
          uint32_t* __restrict__ f2_ids, uint16_t* __restrict__ f2_scores, uint32_t* __restrict__ f2_count,
          const uint32_t* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  extern __shared__ uint64_t keys[];
  const uint32_t q = blockIdx.x;
  const uint32_t Tq = sel[(uint64_t)q * 4 + 3];
  for (uint32_t i = threadIdx.x; i < NP; i += blockDim.x)
    keys[i] = i < Tq ? cand[(uint64_t)q * T + i] : ~0ull;
  __syncthreads();
  bitonic_sort_lds(keys, NP);
  for (uint32_t i = threadIdx.x; i < T; i += blockDim.x) {
    const bool ok = i < Tq;
    const uint64_t key = keys[i];
    f2_ids[(uint64_t)q * T + i] = ok ? (uint32_t)key : 0xFFFFFFFFu;
    if (f2_scores) f2_scores[(uint64_t)q * T + i] = ok ? (uint16_t)(key >> 32) : (uint16_t)0xFFFF;
  }
  if (threadIdx.x == 0) f2_count[q] = Tq;
}

hipError_t launch_select(const uint16_t* scores, uint64_t ld, uint32_t L, uint32_t T, uint32_t n_q,
                         const SelectBufs& b, uint32_t* f2_ids, uint16_t* f2_scores, uint32_t* f2_count,
                         const uint32_t* run_if, hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  const uint32_t nblk = select_blocks(ld);
  // a gated launch usually does nothing: few blocks, each looping over queries
  const uint32_t gy = run_if ? std::min(n_q, kGatedRows) : n_q;
  hipError_t e = launch_fill_u32(b.hist, (uint64_t)n_q * (L + 2), 0, st, run_if);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hist, dim3(nblk, gy), dim3(256), (L + 2) * sizeof(uint32_t), st, scores, ld, L, n_q, b.hist,
                     run_if);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_threshold, dim3(n_q), dim3(256), 0, st, b.hist, L, T, b.sel, b.ctr, run_if);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact, dim3(nblk, gy), dim3(256), 0, st, scores, ld, n_q, b.sel, b.ctr, b.eqcnt, nblk,
                     b.cand, T, run_if);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ties, dim3(nblk, gy), dim3(256), 0, st, scores, ld, n_q, b.sel, b.eqcnt, nblk, b.cand, T,
                     run_if);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint32_t NP = 1;
  while (NP < T) NP <<= 1;
  if (NP < 2) NP = 2;
  hipLaunchKernelGGL(k_sort_f2, dim3(n_q), dim3(512), NP * sizeof(uint64_t), st, b.cand, b.sel, T, NP, f2_ids,
                     f2_scores, f2_count, run_if);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sampled cutoff
// One block per query: histogram of the sampled scores; the cutoff is the
// smallest score s with #{sample members with score <= s} >= r, or all ones
// (admit every member) when the sample holds fewer than r members.  With
// order, block b serves query order[b] (rank b) and also writes rcut[b].
__global__ void __launch_bounds__(256)
k_cutoff(const uint16_t* __restrict__ sample, uint32_t S, uint32_t L, uint32_t r, uint32_t* __restrict__ cutoff,
         const uint32_t* __restrict__ order, uint32_t* __restrict__ rcut) {
  extern __shared__ uint32_t h[];
  __shared__ uint32_t wsum[4];
  const uint32_t t = threadIdx.x;
  const uint32_t q = order ? order[blockIdx.x] : blockIdx.x;
  const uint32_t nb = L + 1;
  for (uint32_t i = t; i < nb; i += 256) h[i] = 0;
  __syncthreads();
  // S is a multiple of 256 (whole sampled blocks): eight scores per 16-byte
  // load, a thread's loads all in flight before its histogram updates
  const uint4* sq = (const uint4*)(sample + (uint64_t)q * S);
  for (uint32_t i0 = t; i0 < S / 8; i0 += 256 * 8) {
    uint4 x[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) x[u] = i0 + 256 * u < S / 8 ? sq[i0 + 256 * u] : make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      const uint32_t w4[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
      for (uint32_t e = 0; e < 8; ++e) {
        const uint32_t v = (w4[e / 2] >> (16 * (e & 1))) & 0xFFFFu;
        if (v != 0xFFFFu) atomicAdd(&h[v], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t per = (nb + 255) / 256;
  const uint32_t b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += h[b];
  // block exclusive scan of the threads' sums: a wave scan, then the four
  // waves' totals
  const uint32_t lane = lane_id(), wv = t / BVS_WAVE;
  uint32_t inc = s;
#pragma unroll
  for (int d = 1; d < BVS_WAVE; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)inc, d, BVS_WAVE);
    if (lane >= (uint32_t)d) inc += o;
  }
  if (lane == BVS_WAVE - 1) wsum[wv] = inc;
  __syncthreads();
  uint32_t pre = inc - s, total = 0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    if (i < wv) pre += wsum[i];
    total += wsum[i];
  }
  if (total < r) {
    if (t == 0) {
      cutoff[q] = 0xFFFFFFFFu;
      if (rcut) rcut[blockIdx.x] = 0xFFFFFFFFu;
    }
    return;
  }
  if (pre < r && pre + s >= r) {
    uint32_t cum = pre;
    for (uint32_t b = b0; b < b1; ++b) {
      cum += h[b];
      if (cum >= r) {
        cutoff[q] = b;
        if (rcut) rcut[blockIdx.x] = b;
        break;
      }
    }
  }
}

hipError_t launch_cutoff(const uint16_t* sample, uint32_t S, uint32_t L, uint32_t r, uint32_t n_q,
                         uint32_t* cutoff, const uint32_t* order, uint32_t* rcut, hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  if (S % 256 != 0 || ((uintptr_t)sample & 15) != 0) return hipErrorInvalidValue;   // read 8 scores at a time
  hipLaunchKernelGGL(k_cutoff, dim3(n_q), dim3(256), (L + 1) * sizeof(uint32_t), st, sample, S, L, r, cutoff, order,
                     rcut);
  return hipGetLastError();
}

// One block per query: the first T appended keys by (score, id) as F2.  A
// histogram of the scores (16-bit counters, two per word) gives the T-th
// smallest score; only keys at or under it are sorted.  A query whose
// buffer overflowed, or that holds fewer than T sets although its cutoff
// excluded some members, is counted in *fail and left untouched.
__global__ void __launch_bounds__(1024)
k_sort_append(const uint64_t* __restrict__ cand, const uint32_t* __restrict__ cand_count,
              const uint32_t* __restrict__ cutoff, uint32_t cap, uint32_t np, uint32_t T, uint32_t L,
              uint32_t* __restrict__ f2_ids, uint16_t* __restrict__ f2_scores, uint32_t* __restrict__ f2_count,
              uint32_t* __restrict__ fail) {
  extern __shared__ uint64_t keys[];                 // [np >= cap], then the histogram and the scan
  uint32_t* hist = (uint32_t*)(keys + np);           // [(L + 2) / 2] packed counters
  uint32_t* part = hist + (L + 2) / 2;               // [16] per-wave sums
  __shared__ uint32_t thr_s, m_s;
  const uint32_t q = blockIdx.x, tid = threadIdx.x, bd = blockDim.x;
  const uint32_t n = cand_count[q];
  const bool ok = n <= cap && (n >= T || cutoff[q] == 0xFFFFFFFFu);
  if (!ok) {
    if (tid == 0) atomicAdd(fail, 1u);
    return;
  }
  const uint64_t* cq = cand + (uint64_t)q * cap;
  const uint32_t nbw = (L + 2) / 2;
  if (tid == 0) {
    thr_s = 0xFFFFFFFFu;
    m_s = 0;
  }
  if (n > T) {
    for (uint32_t i = tid; i < nbw; i += bd) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += bd) {
      const uint32_t sc = (uint32_t)(cq[i] >> 32);
      atomicAdd(&hist[sc >> 1], 1u << (16 * (sc & 1)));
    }
    __syncthreads();
    // thread t sums bins [t per, (t + 1) per); block exclusive scan; the
    // thread whose range reaches T finds the score
    const uint32_t nb = L + 1, per = (nb + bd - 1) / bd;
    const uint32_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    auto bin = [&](uint32_t b) { return (hist[b >> 1] >> (16 * (b & 1))) & 0xFFFFu; };
    uint32_t own = 0;
    for (uint32_t b = b0; b < b1; ++b) own += bin(b);
    uint32_t inc = own;
    const uint32_t lane = lane_id(), w = tid / BVS_WAVE;
#pragma unroll
    for (int d = 1; d < BVS_WAVE; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)inc, d, BVS_WAVE);
      if (lane >= (uint32_t)d) inc += o;
    }
    if (lane == BVS_WAVE - 1) part[w] = inc;
    __syncthreads();
    uint32_t pre = inc - own;
    for (uint32_t i = 0; i < w; ++i) pre += part[i];
    if (pre < T && pre + own >= T) {
      uint32_t cum = pre;
      for (uint32_t b = b0; b < b1; ++b) {
        cum += bin(b);
        if (cum >= T) {
          thr_s = b;
          break;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t thr = thr_s;
  for (uint32_t i = tid; i < n; i += bd) {
    const uint64_t key = cq[i];
    if ((uint32_t)(key >> 32) <= thr) keys[atomicAdd(&m_s, 1u)] = key;
  }
  __syncthreads();
  const uint32_t m = m_s;
  uint32_t NP = 2;
  while (NP < m) NP <<= 1;
  for (uint32_t i = m + tid; i < NP; i += bd) keys[i] = ~0ull;
  __syncthreads();
  bitonic_sort_lds(keys, NP);
  const uint32_t Tq = min(T, n);
  for (uint32_t i = tid; i < T; i += bd) {
    const bool v = i < Tq;
    const uint64_t key = v ? keys[i] : ~0ull;
    f2_ids[(uint64_t)q * T + i] = v ? (uint32_t)key : 0xFFFFFFFFu;
    if (f2_scores) f2_scores[(uint64_t)q * T + i] = v ? (uint16_t)(key >> 32) : (uint16_t)0xFFFF;
  }
  if (tid == 0) f2_count[q] = Tq;
}

hipError_t launch_sort_append(const uint64_t* cand, const uint32_t* cand_count, const uint32_t* cutoff, uint32_t cap,
                              uint32_t T, uint32_t L, uint32_t n_q, uint32_t* f2_ids, uint16_t* f2_scores,
                              uint32_t* f2_count, uint32_t* fail, hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  uint32_t np = 2;
  while (np < cap) np <<= 1;   // the sort pads at most cap keys to a power of two
  const size_t lds = (size_t)np * sizeof(uint64_t) + ((L + 2) / 2 + 16) * sizeof(uint32_t);
  hipError_t e = hipFuncSetAttribute((const void*)k_sort_append, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_append, dim3(n_q), dim3(1024), lds, st, cand, cand_count, cutoff, cap, np, T, L, f2_ids,
                     f2_scores, f2_count, fail);
  return hipGetLastError();
}

}  // namespace bvs
