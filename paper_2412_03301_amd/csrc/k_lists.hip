// Inverted lists of the count Bloom filters (Def. 9, Alg. 4) and the first
// filter layer read from them (Alg. 6, inverted-index filtering).
//
// For every position p the list holds the sets with C^(j)[p] >= 1, ordered by
// decreasing count (sets with equal counts in no particular order: Alg. 4
// sorts by count only).  Layout:
//   cum   [L][257] uint32   cum[p][c] = entries of list p with count >= c
//                           (cum[p][0] = cum[p][1] = the list's length,
//                           cum[p][256] = 0), so count class c occupies
//                           [cum[p][c + 1], cum[p][c]) of the list
//   start [L + 1]   uint64   list p is ids[start[p] .. start[p + 1])
//   ids   [nnz]     uint32   set ids
// The lists are built from the position-major count rows of the index: a
// histogram of each row's counts, a descending scan per row and one over the
// rows, then every nonzero entry takes a slot of its count class with an
// atomic cursor.  A query's first layer is then the union, over its A
// positions, of the prefixes of count >= M: their ids set bits of a
// per-query membership bitmap that the scoring kernels read.
#include "device.h"
#include "launch.h"

namespace bvs {

static constexpr uint32_t kListChunk = 4096;   // sets per block of the build passes

// Grid (ceil(ld / kListChunk), L).  hist [L][256] (zeroed by the caller).
__global__ void __launch_bounds__(256)
k_list_hist(const uint8_t* __restrict__ cnt, uint64_t ld, uint64_t n_sets, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const uint32_t p = blockIdx.y;
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t j0 = (uint64_t)blockIdx.x * kListChunk;
  const uint64_t j1 = min(n_sets, j0 + kListChunk);
  const uint8_t* row = cnt + (uint64_t)p * ld;
  for (uint64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const uint32_t c = row[j];
    if (c) atomicAdd(&h[c], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[(uint64_t)p * 256 + threadIdx.x], h[threadIdx.x]);
}

// One block of 256 threads per position: cum[p][c] = sum of hist[p][c'] for
// c' >= c (c = 1..255), cum[p][0] = cum[p][1], cum[p][256] = 0; len[p] =
// cum[p][1].
__global__ void __launch_bounds__(256)
k_list_cum(const uint32_t* __restrict__ hist, uint32_t* __restrict__ cum, uint64_t* __restrict__ len) {
  __shared__ uint32_t s[256];
  const uint32_t p = blockIdx.x, t = threadIdx.x;
  // reversed inclusive scan: position t holds the count of class 255 - t
  s[t] = t < 255 ? hist[(uint64_t)p * 256 + (255 - t)] : 0u;
  __syncthreads();
  for (uint32_t d = 1; d < 256; d <<= 1) {
    const uint32_t v = t >= d ? s[t - d] : 0u;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  // s[t] = entries with count >= 255 - t, for t < 255
  uint32_t* cp = cum + (uint64_t)p * 257;
  if (t < 255) cp[255 - t] = s[t];
  if (t == 0) {
    cp[256] = 0;
    cp[0] = s[254];
    len[p] = s[254];
  }
}

// start[0] = 0, start[p + 1] = start[p] + len[p]: one block of 1024 threads.
__global__ void __launch_bounds__(1024)
k_list_starts(const uint64_t* __restrict__ len, uint32_t L, uint64_t* __restrict__ start) {
  __shared__ uint64_t s[1024];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b = 0; b < L; b += 1024) {
    const uint32_t i = b + threadIdx.x;
    s[threadIdx.x] = i < L ? len[i] : 0ull;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      const uint64_t v = threadIdx.x >= d ? s[threadIdx.x - d] : 0ull;
      __syncthreads();
      s[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < L) start[i + 1] = carry + s[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) start[0] = 0;
}

// Grid (ceil(ld / kListChunk), L).  cursor [L][256] zeroed by the caller.
__global__ void __launch_bounds__(256)
k_list_fill(const uint8_t* __restrict__ cnt, uint64_t ld, uint64_t n_sets, const uint32_t* __restrict__ cum,
            const uint64_t* __restrict__ start, uint32_t* __restrict__ cursor, uint32_t* __restrict__ ids) {
  const uint32_t p = blockIdx.y;
  const uint64_t j0 = (uint64_t)blockIdx.x * kListChunk;
  const uint64_t j1 = min(n_sets, j0 + kListChunk);
  const uint8_t* row = cnt + (uint64_t)p * ld;
  const uint32_t* cp = cum + (uint64_t)p * 257;
  const uint64_t base = start[p];
  for (uint64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const uint32_t c = row[j];
    if (c) {
      const uint32_t slot = atomicAdd(&cursor[(uint64_t)p * 256 + c], 1u);
      ids[base + cp[c + 1] + slot] = (uint32_t)j;
    }
  }
}

hipError_t launch_list_build(const uint8_t* cnt, uint64_t ld, uint64_t n_sets, uint32_t L, uint32_t* hist,
                             uint32_t* cursor, uint64_t* len, uint32_t* cum, uint64_t* start, uint32_t* ids,
                             hipStream_t st, bool fill) {
  const dim3 grid((uint32_t)((n_sets + kListChunk - 1) / kListChunk), L);
  hipError_t e;
  if (!fill) {
    if ((e = launch_fill_u32(hist, (uint64_t)L * 256, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_list_hist, grid, dim3(256), 0, st, cnt, ld, n_sets, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_list_cum, dim3(L), dim3(256), 0, st, hist, cum, len);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_list_starts, dim3(1), dim3(1024), 0, st, len, L, start);
    return hipGetLastError();
  }
  if ((e = launch_fill_u32(cursor, (uint64_t)L * 256, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_list_fill, grid, dim3(256), 0, st, cnt, ld, n_sets, cum, start, cursor, ids);
  return hipGetLastError();
}

// Grid (chunks, A, n_q): the entries of count >= M of list pos[q][t] set the
// bits of their sets in member[q][ld / 64] (zeroed by the caller).
__global__ void __launch_bounds__(256)
k_list_gather(const uint32_t* __restrict__ ids, const uint64_t* __restrict__ start, const uint32_t* __restrict__ cum,
              const uint32_t* __restrict__ pos, uint32_t A, uint32_t M, uint64_t ld,
              unsigned long long* __restrict__ member) {
  const uint32_t t = blockIdx.y, q = blockIdx.z;
  const uint32_t p = pos[(uint64_t)q * A + t];
  const uint32_t n = cum[(uint64_t)p * 257 + M];
  const uint32_t* lst = ids + start[p];
  unsigned long long* mq = member + (uint64_t)q * (ld / 64);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t j = lst[i];
    atomicOr(&mq[j / 64], 1ull << (j % 64));
  }
}

hipError_t launch_list_gather(const uint32_t* ids, const uint64_t* start, const uint32_t* cum, const uint32_t* pos,
                              uint32_t A, uint32_t M, uint32_t n_q, uint64_t ld, uint64_t* member, int n_cu,
                              hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  if (M < 1 || M > 255) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32((uint32_t*)member, (uint64_t)n_q * (ld / 64) * 2, 0, st);
  if (e != hipSuccess) return e;
  // enough blocks per (query, position) to fill the chip for one query
  const uint32_t chunks = std::max(1u, std::min(64u, (uint32_t)n_cu / 4));
  hipLaunchKernelGGL(k_list_gather, dim3(chunks, A, n_q), dim3(256), 0, st, ids, start, cum, pos, A, M, ld,
                     (unsigned long long*)member);
  return hipGetLastError();
}

}  // namespace bvs
