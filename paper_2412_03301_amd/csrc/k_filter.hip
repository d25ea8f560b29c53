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
// select     the first min(T, |F1|) sets by (score, id), in four passes:
//            histogram of scores, threshold tau per query, unordered append of
//            every score < tau plus a count of score == tau per block, then an
//            ordered fill of the ties (lowest ids first); a final bitonic sort
//            orders F2 by (score, id).  Every step is deterministic.
#include "device.h"
#include "launch.h"

namespace bvs {

template <int QT>
__global__ void __launch_bounds__(256)
k_filter(const uint4* __restrict__ bits, const uint8_t* __restrict__ cnt, uint64_t ld, uint64_t n_sets,
         uint32_t RC, const uint4* __restrict__ sq, const uint4* __restrict__ gate,
         const uint64_t* __restrict__ gate_chunks, const uint32_t* __restrict__ pos, uint32_t A, uint32_t M,
         uint32_t n_q, uint16_t* __restrict__ scores) {
  const uint64_t j = blockIdx.x * 256ull + threadIdx.x;
  const uint32_t q0 = blockIdx.y * QT;
  const uint32_t nq = min((uint32_t)QT, n_q - q0);
  uint32_t acc[QT], hit[QT];
  uint64_t gcm[QT];
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    acc[i] = 0;
    hit[i] = 0;
    gcm[i] = (M == 1 && (uint32_t)i < nq) ? gate_chunks[q0 + i] : 0;
  }
  const uint4* col = bits + j;
#pragma unroll 4
  for (uint32_t c = 0; c < RC; ++c) {
    const uint4 x = col[(uint64_t)c * ld];
#pragma unroll
    for (int i = 0; i < QT; ++i) {
      if ((uint32_t)i < nq) {
        const uint4 s = sq[(uint64_t)(q0 + i) * RC + c];
        acc[i] += popc32(x.x ^ s.x) + popc32(x.y ^ s.y) + popc32(x.z ^ s.z) + popc32(x.w ^ s.w);
        if ((gcm[i] >> c) & 1) {
          const uint4 g = gate[(uint64_t)(q0 + i) * RC + c];
          hit[i] |= (x.x & g.x) | (x.y & g.y) | (x.z & g.z) | (x.w & g.w);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    if ((uint32_t)i < nq) {
      bool member;
      if (M == 0) {
        member = true;
      } else if (M == 1) {
        member = hit[i] != 0;
      } else {
        member = false;
        for (uint32_t a = 0; a < A; ++a) {
          const uint32_t p = pos[(uint64_t)(q0 + i) * A + a];
          member |= cnt[(uint64_t)p * ld + j] >= M;
        }
      }
      scores[(uint64_t)(q0 + i) * ld + j] = (j < n_sets && member) ? (uint16_t)acc[i] : (uint16_t)0xFFFF;
    }
  }
}

hipError_t launch_filter(const uint64_t* bits, const uint8_t* cnt, uint64_t ld, uint64_t n_sets, uint32_t L,
                         const uint64_t* sq, const uint64_t* gate, const uint64_t* gate_chunks,
                         const uint32_t* pos, uint32_t A, uint32_t M, uint32_t n_q, uint16_t* scores,
                         hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  const uint32_t RC = L / 128;
  const uint32_t gx = (uint32_t)(ld / 256);
  auto go = [&](auto qt) -> hipError_t {
    constexpr int QT = decltype(qt)::value;
    dim3 grid(gx, (n_q + QT - 1) / QT);
    hipLaunchKernelGGL(k_filter<QT>, grid, dim3(256), 0, st, (const uint4*)bits, cnt, ld, n_sets, RC,
                       (const uint4*)sq, (const uint4*)gate, gate_chunks, pos, A, M, n_q, scores);
    return hipGetLastError();
  };
  if (n_q >= 16) return go(std::integral_constant<int, 16>());
  if (n_q >= 8) return go(std::integral_constant<int, 8>());
  if (n_q >= 4) return go(std::integral_constant<int, 4>());
  return go(std::integral_constant<int, 1>());
}

// ---------------------------------------------------------------- select
static constexpr uint32_t SEL_CH = 4096;   // sets per block in the select passes

uint32_t select_blocks(uint64_t ld) { return (uint32_t)((ld + SEL_CH - 1) / SEL_CH); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

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

__global__ void __launch_bounds__(256)
k_hist(const uint16_t* __restrict__ scores, uint64_t ld, uint32_t L, uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t h[];
  const uint32_t q = blockIdx.y;
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
}

// One block per query: tau = smallest score s with #{score <= s} >= Tq,
// Tq = min(T, |F1|).
__global__ void __launch_bounds__(256)
k_threshold(const uint32_t* __restrict__ hist, uint32_t L, uint32_t T, uint32_t* __restrict__ sel,
            uint32_t* __restrict__ ctr) {
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

__global__ void __launch_bounds__(256)
k_compact(const uint16_t* __restrict__ scores, uint64_t ld, const uint32_t* __restrict__ sel,
          uint32_t* __restrict__ ctr, uint32_t* __restrict__ eqcnt, uint32_t nblk, uint64_t* __restrict__ cand,
          uint32_t T) {
  __shared__ uint32_t wsum[4];
  const uint32_t q = blockIdx.y, blk = blockIdx.x, lane = lane_id();
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
}

__global__ void __launch_bounds__(256)
k_ties(const uint16_t* __restrict__ scores, uint64_t ld, const uint32_t* __restrict__ sel,
       const uint32_t* __restrict__ eqcnt, uint32_t nblk, uint64_t* __restrict__ cand, uint32_t T) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t red[4];
  const uint32_t q = blockIdx.y, blk = blockIdx.x;
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
          uint32_t* __restrict__ f2_ids, uint16_t* __restrict__ f2_scores, uint32_t* __restrict__ f2_count) {
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
                         hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  const uint32_t nblk = select_blocks(ld);
  hipError_t e = launch_fill_u32(b.hist, (uint64_t)n_q * (L + 2), 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hist, dim3(nblk, n_q), dim3(256), (L + 2) * sizeof(uint32_t), st, scores, ld, L, b.hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_threshold, dim3(n_q), dim3(256), 0, st, b.hist, L, T, b.sel, b.ctr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact, dim3(nblk, n_q), dim3(256), 0, st, scores, ld, b.sel, b.ctr, b.eqcnt, nblk,
                     b.cand, T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ties, dim3(nblk, n_q), dim3(256), 0, st, scores, ld, b.sel, b.eqcnt, nblk, b.cand, T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint32_t NP = 1;
  while (NP < T) NP <<= 1;
  if (NP < 2) NP = 2;
  hipLaunchKernelGGL(k_sort_f2, dim3(n_q), dim3(512), NP * sizeof(uint64_t), st, b.cand, b.sel, T, NP, f2_ids,
                     f2_scores, f2_count);
  return hipGetLastError();
}

}  // namespace bvs
