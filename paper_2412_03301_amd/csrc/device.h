// Device helpers shared by the gfx950 kernels: wave-level ballots and
// reductions, DPP row reductions and the int8 matrix-core step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BVS_WAVE 64

namespace bvs {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Index of the calling wave in its workgroup, marked wave-uniform so that
// values derived from it live in scalar registers and drive scalar loads
// and branches.
__device__ __forceinline__ uint32_t wave_id() {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / BVS_WAVE));
}

// A pointer every lane holds the same value of, moved to scalar registers.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (T*)((uint64_t)hi << 32 | lo);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

#if defined(__HIP_DEVICE_COMPILE__)
#define BVS_LDS_AS __attribute__((address_space(3)))
#else
#define BVS_LDS_AS
#endif

// Copy rows 0 .. rows - 1 of NP row planes into LDS: row r of plane k is
// c16n 16-byte chunks at src[k] + r * sstride and goes to dst[k] + r *
// dstride; rows at or past mq become zero.  Each thread has four chunks of
// every plane in flight at once (their loads read row min(r, mq - 1), always
// inside the source).  rows must be 0 when mq is 0.  No barrier.
template <int NP>
__device__ __forceinline__ void stage_rows(const uint8_t* const (&src)[NP], uint8_t* const (&dst)[NP], uint64_t sstride,
                                           uint32_t dstride, uint32_t c16n, uint32_t rows, uint32_t mq) {
  const uint32_t n = rows * c16n, bd = blockDim.x;
  for (uint32_t i0 = threadIdx.x; i0 < n; i0 += 4 * bd) {
    uint4 x[NP][4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t i = min(i0 + u * bd, n - 1);
      const uint32_t r = min(i / c16n, mq - 1), c = i % c16n;
#pragma unroll
      for (int k = 0; k < NP; ++k) x[k][u] = *(const uint4*)(src[k] + r * sstride + 16 * c);
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t i = i0 + u * bd;
      if (i < n) {
        const uint32_t r = i / c16n, c = i % c16n;
#pragma unroll
        for (int k = 0; k < NP; ++k)
          *(uint4*)(dst[k] + r * dstride + 16 * c) = r < mq ? x[k][u] : make_uint4(0, 0, 0, 0);
      }
    }
  }
}

// Copy n16 16-byte words from global memory (src) into LDS (dst), both
// 16-byte aligned, with every word in flight at once: each wave moves whole
// chunks of 64 words by direct loads into LDS (16 bytes per lane, lane-
// contiguous from a wave-uniform LDS base), and a ragged tail of fewer than
// 64 words goes through registers.  The direct loads count as memory loads:
// wait for them (s_waitcnt) before the workgroup barrier that precedes the
// first read.
__device__ __forceinline__ void copy_to_lds(const uint4* __restrict__ src, void* dst, uint32_t n16) {
  const uint32_t nw = blockDim.x / BVS_WAVE;
  const uint32_t w = wave_id(), ln = lane_id();
  const uint32_t full = n16 / BVS_WAVE;
  for (uint32_t c = w; c < full; c += nw)
    __builtin_amdgcn_global_load_lds((const void*)(src + (uint64_t)c * BVS_WAVE + ln),
                                     (BVS_LDS_AS void*)((uint8_t*)dst + (size_t)c * BVS_WAVE * 16), 16, 0, 0);
  const uint32_t t = full * BVS_WAVE + threadIdx.x;
  if (t < n16) ((uint4*)dst)[t] = src[t];
}

// Read-only view of global data in the constant address space: uniform
// loads through it become scalar loads.  Only for data that no kernel writes
// while it is being read.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
#else
template <typename T>
using cptr = const T*;   // host pass of kernel bodies: plain pointer
#endif
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

__device__ __forceinline__ uint32_t popc32(uint32_t x) { return __builtin_popcount(x); }
__device__ __forceinline__ uint32_t popc64(uint64_t x) { return __builtin_popcountll(x); }

// Order LDS traffic of one wave: the write of one lane is visible to a later
// read of another lane of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) {
  return (uint32_t)__shfl_xor((int)v, m, BVS_WAVE);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, shfl_xor_u32(v, m));
  return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, shfl_xor_u32(v, m));
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_u32(v, m);
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint32_t olo = shfl_xor_u32(lo, m), ohi = shfl_xor_u32(hi, m);
    uint64_t s = ((uint64_t)hi << 32 | lo) + ((uint64_t)ohi << 32 | olo);
    lo = (uint32_t)s; hi = (uint32_t)(s >> 32);
  }
  return (uint64_t)hi << 32 | lo;
}

// Minimum over the 16 lanes of a DPP row (lanes 16r .. 16r+15); every lane
// of the row receives the result.  row_ror:n has DPP control 0x120 + n.
__device__ __forceinline__ uint32_t row16_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));
  return v;
}

__device__ __forceinline__ uint32_t row16_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));
  return v;
}

// Minimum / maximum over lanes l, l ^ 16, l ^ 32, l ^ 48 (the four DPP rows)
// with the gfx950 row-swap instructions: v_permlane32_swap exchanges the
// upper half of one operand with the lower half of the other, and
// v_permlane16_swap the odd rows of one with the even rows of the other, so
// swapping a value with itself pairs lane l with l ^ 32, then with l ^ 16.
__device__ __forceinline__ uint32_t rows4_min_u32(uint32_t v) {
  const auto a = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = min((uint32_t)a[0], (uint32_t)a[1]);
  const auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return min((uint32_t)b[0], (uint32_t)b[1]);
}
__device__ __forceinline__ uint32_t rows4_max_u32(uint32_t v) {
  const auto a = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = max((uint32_t)a[0], (uint32_t)a[1]);
  const auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return max((uint32_t)b[0], (uint32_t)b[1]);
}

__device__ __forceinline__ uint32_t row16_sum_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false);
  return v;
}
__device__ __forceinline__ uint32_t rows4_sum_u32(uint32_t v) {
  const auto a = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = (uint32_t)a[0] + (uint32_t)a[1];
  const auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (uint32_t)b[0] + (uint32_t)b[1];
}

// Maximum / minimum / sum over the wave without LDS traffic (every lane
// gets it).
// Float minima over the 16 lanes of a DPP row and over the four rows.
__device__ __forceinline__ float row16_min_f32(float v) {
  v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false)));
  v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false)));
  v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xF, 0xF, false)));
  v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xF, 0xF, false)));
  return v;
}
__device__ __forceinline__ float rows4_min_f32(float v) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fminf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  const auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fminf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

__device__ __forceinline__ uint32_t wave_max_dpp_u32(uint32_t v) { return rows4_max_u32(row16_max_u32(v)); }
__device__ __forceinline__ uint32_t wave_min_dpp_u32(uint32_t v) { return rows4_min_u32(row16_min_u32(v)); }
__device__ __forceinline__ uint32_t wave_sum_dpp_u32(uint32_t v) { return rows4_sum_u32(row16_sum_u32(v)); }

// One 16x16x64 int8 matrix-core step with int32 accumulation:
//   C[i][j] += sum_k A[i][k] * B[k][j]
// A row i and B column j both come from lane (i or j) + 16 * g, which holds
// 16 consecutive k of k-group g.  C[4 * (l / 16) + r][l % 16] is element r of
// lane l.  Integer accumulation wraps modulo 2^32, so sums whose true value
// fits int32 are exact whatever the partial sums are.
__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

__host__ __device__ constexpr uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Work counters: kStatSlots slots of kStatCounters counters; workgroups add their totals
// to slot (linear block id % kStatSlots) so that no single address takes
// every atomic.  The host sums the slots.
constexpr uint32_t kStatSlots = 64;
constexpr uint32_t kStatCounters = 7;

// Block-wide sum of up to three per-wave counters (lane 0 of each wave holds
// the wave's value; every wave must call), added to counters first, first+1,
// first+2 of the block's slot.  Uses one LDS word per wave and counter.
__device__ __forceinline__ void stats_add(unsigned long long* stats, uint32_t first, uint32_t a, uint32_t b = 0,
                                          uint32_t c = 0) {
  __shared__ uint32_t part[3][16];
  const uint32_t w = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  if ((threadIdx.x & 63) == 0) { part[0][w] = a; part[1][w] = b; part[2][w] = c; }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long t = 0;
    for (uint32_t i = 0; i < nw; ++i) t += part[threadIdx.x][i];
    const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (t && first + threadIdx.x < kStatCounters)
      atomicAdd(&stats[(blk % kStatSlots) * kStatCounters + first + threadIdx.x], t);
  }
}

// Status bits raised by kernels that validate data.
enum : uint32_t {
  ST_OFF_GRID = 1u,     // a value is not a multiple of 2^-12 or |x| > 1 (or not finite)
  ST_NORM = 2u,         // a row has Euclidean norm > 2
};

}  // namespace bvs
