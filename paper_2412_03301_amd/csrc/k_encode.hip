// FlyHash encoding and per-set Bloom sketches on gfx950.
//
//   convert         float32 rows -> exact int8 planes (a = 4096 x = 64 hi + lo),
//                   squared norms, and the pair the re-rank screens with
//                   (|hi|^2 and an upper bound of |lo - 31.5| / 64); validates
//                   the 2^-12 grid
//   encode_vectors  one wave per vector: projection y = W a (Def. 7) with the
//                   sparse rows of W read from an LDS copy of the index table,
//                   then winner-take-all (Alg. 1): the wta_k largest outputs
//   encode_sets     one wave per set: the same per member, accumulating the
//                   count Bloom filter (Def. 8, Alg. 3) in packed byte
//                   counters and the binary Bloom filter (Def. 10, Alg. 5)
//                   as OR bits; writes row-major scratch
//   transpose       scratch -> position-major counts and chunk-major bits
//   query_sketch    query count filter C_Q, sketch S_Q and the A positions of
//                   largest count (first steps of Alg. 6)
//
// Winner-take-all with ties to the lower output index: output j of a vector
// gets the unique key ((y_j + s*4096) << log2 L) | (L - 1 - j); y_j is an
// integer in [-s*4096, s*4096] on the grid, so a larger key means a larger
// y_j or, for equal y_j, a lower j.  The wta_k-th largest key is found by
// setting bits from the top while at least wta_k keys stay >= the prefix;
// counts are sums of wave ballots.  Lane l owns outputs j = l + 64 t, so the
// ballot of "key_t >= threshold" is directly code word t.
#include "device.h"
#include "launch.h"
#include "wta.h"

namespace bvs {

// ---------------------------------------------------------------- convert
__global__ void __launch_bounds__(256)
k_convert(const float* __restrict__ x, uint64_t n_rows, uint32_t d, uint32_t dp,
          int8_t* __restrict__ hi, uint8_t* __restrict__ lo, uint32_t* __restrict__ norms,
          uint2* __restrict__ scr, uint32_t* __restrict__ status) {
  const uint32_t lane = lane_id();
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / BVS_WAVE;
  const uint64_t nwaves = (gridDim.x * (uint64_t)blockDim.x) / BVS_WAVE;
  uint32_t bad = 0;
  // four consecutive elements per lane (one 16-byte load when rows of d
  // floats keep that alignment), their plane bytes stored as one word each
  const bool vec = d % 4 == 0 && ((uintptr_t)x & 15) == 0;
  for (uint64_t r = wave; r < n_rows; r += nwaves) {
    const float* xr = x + r * d;
    uint64_t ss = 0;
    uint32_t hs = 0, es = 0;
    for (uint32_t e0 = 4 * lane; e0 < dp; e0 += 4 * BVS_WAVE) {
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (vec && e0 + 3 < d) {
        const float4 f = *(const float4*)(xr + e0);
        v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
      } else {
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
          if (e0 + j < d) v[j] = xr[e0 + j];
      }
      uint32_t hw = 0, lw = 0;
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        int a = 0;
        if (e0 + j < d) {
          const float s = v[j] * 4096.0f;
          float ri = rintf(s);
          if (!(ri == s) || !(fabsf(v[j]) <= 1.0f)) { bad |= ST_OFF_GRID; ri = 0.0f; }
          a = (int)ri;
          const int e2 = 2 * (a & 63) - 63;   // 2 (lo - 31.5), zero on padding
          es += (uint32_t)(e2 * e2);
        }
        hw |= (uint32_t)(uint8_t)(int8_t)(a >> 6) << (8 * j);   // floor(a / 64) in [-64, 64]
        lw |= (uint32_t)(a & 63) << (8 * j);                     // a - 64 floor(a / 64) in [0, 63]
        ss += (uint64_t)(a * a);
        hs += (uint32_t)((a >> 6) * (a >> 6));
      }
      *(uint32_t*)(hi + r * dp + e0) = hw;   // dp is a multiple of 64
      *(uint32_t*)(lo + r * dp + e0) = lw;
    }
    ss = wave_sum_u64(ss);
    if (ss > (1ull << 26)) bad |= ST_NORM;  // ||x|| > 2
    if (scr) {
      // |hi|^2 <= 1024 * 64^2 and |2 lo - 63|^2 <= 1024 * 63^2 are exact
      // in float; the bound sqrt(es) / 128 is rounded up by the factor.
      hs = wave_sum_dpp_u32(hs);
      es = wave_sum_dpp_u32(es);
      const float rb = sqrtf((float)es) * (1.0f / 128.0f) * (1.0f + 0x1p-20f);
      if (lane == 0) scr[r] = make_uint2(hs, __float_as_uint(rb));
    }
    if (lane == 0) norms[r] = (uint32_t)(ss > 0xFFFFFFFFull ? 0xFFFFFFFFull : ss);
  }
  const uint64_t b1 = ballot(bad & ST_OFF_GRID), b2 = ballot(bad & ST_NORM);
  if (lane == 0 && (b1 | b2)) atomicOr(status, (b1 ? ST_OFF_GRID : 0u) | (b2 ? ST_NORM : 0u));
}

hipError_t launch_convert(const float* x, uint64_t n_rows, uint32_t d, uint32_t dp, int8_t* hi,
                          uint8_t* lo, uint32_t* norms, uint2* scr, uint32_t* status, int n_cu, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  if (dp % 4 != 0 || (((uintptr_t)hi | (uintptr_t)lo) & 3) != 0) return hipErrorInvalidValue;   // word stores
  const uint64_t want = (n_rows + 3) / 4;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(want, (uint64_t)n_cu * 32);
  hipLaunchKernelGGL(k_convert, dim3(grid), dim3(256), 0, st, x, n_rows, d, dp, hi, lo, norms, scr, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- hashing
// Stage one vector (a = 64 hi + lo) into the wave's LDS slot as int16.
__device__ __forceinline__ void stage_vector(int16_t* __restrict__ av, const int8_t* __restrict__ hi,
                                             const uint8_t* __restrict__ lo, uint64_t row, uint32_t dp,
                                             uint32_t lane) {
  const uint32_t* h4 = (const uint32_t*)(hi + row * dp);
  const uint32_t* l4 = (const uint32_t*)(lo + row * dp);
  for (uint32_t e4 = lane; e4 < dp / 4; e4 += BVS_WAVE) {
    const uint32_t h = h4[e4], l = l4[e4];
    int16_t v[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
      v[b] = (int16_t)(64 * (int)(int8_t)(h >> (8 * b)) + (int)((l >> (8 * b)) & 0xFF));
    uint2 packed;
    packed.x = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
    packed.y = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
    *(uint2*)(av + 4 * e4) = packed;
  }
}

// Keys of the R outputs owned by this lane (j = lane + 64 t).
template <int R>
__device__ __forceinline__ void hash_keys(const int16_t* __restrict__ av, const uint16_t* __restrict__ idx,
                                          uint32_t SP, uint32_t koff, uint32_t lgL, uint32_t L,
                                          uint32_t lane, uint32_t (&key)[R]) {
  // The row addresses depend only on the lane; rebuilding them per vector
  // from an opaque copy of the lane keeps the compiler from holding all R of
  // them live across the vector loop (which spills at R = 64).
  uint32_t ln = lane;
  asm volatile("" : "+v"(ln));
  const uint8_t* avb = (const uint8_t*)av;
  auto at = [avb](uint32_t off) { return (int)*(const int16_t*)(avb + off); };
#pragma unroll
  for (int t = 0; t < R; ++t) {
    // bound the gathers in flight
    if (t % 8 == 0) asm volatile("" ::: "memory");
    const uint32_t j = ln + 64u * t;
    const uint16_t* row = idx + j * SP;
    int y = 0;
    for (uint32_t i0 = 0; i0 < SP; i0 += 8) {
      const uint4 w = *(const uint4*)(row + i0);
      // entries are byte offsets: the address is one add with a half-word operand
      y += at(w.x & 0xFFFF) + at(w.x >> 16) + at(w.y & 0xFFFF) + at(w.y >> 16) +
           at(w.z & 0xFFFF) + at(w.z >> 16) + at(w.w & 0xFFFF) + at(w.w >> 16);
    }
    key[t] = ((uint32_t)(y + (int)koff) << lgL) | (L - 1u - j);
  }
}

struct EncodeShared {
  uint16_t* idx;   // [L][SP] byte offsets into av
  int16_t* av;     // this wave's staged vector, dim_padded + 8 entries (tail zero)
};

__device__ __forceinline__ EncodeShared encode_setup(const HashGeom& g, uint8_t* smem) {
  EncodeShared sh;
  sh.idx = (uint16_t*)smem;
  const uint32_t tab_bytes = (uint32_t)align_up((uint64_t)g.L * g.SP * 2, 16);
  const uint32_t w = wave_id();
  sh.av = (int16_t*)(smem + tab_bytes) + w * (g.dim_padded + 8);
  const uint32_t n16 = g.L * g.SP / 8;
  copy_to_lds((const uint4*)g.idx, sh.idx, n16);
  if (lane_id() < 8) sh.av[g.dim_padded + lane_id()] = 0;
  __builtin_amdgcn_s_waitcnt(0);   // the table has landed in LDS
  __syncthreads();
  return sh;
}

__host__ __device__ inline int key_topbit(const HashGeom& g) {
  const uint64_t maxkey = ((uint64_t)(2u * g.s * 4096u) << g.lgL) | (g.L - 1u);
  int b = 63;
  while (b > 0 && !((maxkey >> b) & 1)) --b;
  return b;
}

size_t encode_lds_bytes(const HashGeom& g, uint32_t waves) {
  return align_up((uint64_t)g.L * g.SP * 2, 16) + (size_t)waves * (g.dim_padded + 8) * 2;
}

template <int R>
__global__ void __launch_bounds__(1024)
k_encode_vectors(HashGeom g, const int8_t* __restrict__ hi, const uint8_t* __restrict__ lo, uint64_t n,
                 uint64_t* __restrict__ codes, int topbit) {
  extern __shared__ __align__(16) uint8_t smem[];
  const EncodeShared sh = encode_setup(g, smem);
  const uint32_t lane = lane_id();
  const uint32_t nw = blockDim.x / BVS_WAVE;
  const uint32_t koff = g.s * 4096u;
  for (uint64_t v = blockIdx.x * (uint64_t)nw + wave_id(); v < n; v += (uint64_t)gridDim.x * nw) {
    stage_vector(sh.av, hi, lo, v, g.dim_padded, lane);
    wave_lds_sync();
    uint32_t key[R];
    hash_keys<R>(sh.av, sh.idx, g.SP, koff, g.lgL, g.L, lane, key);
    const uint32_t th = kth_largest<R>(key, g.wta_k, topbit);
    uint64_t w0 = 0, w1 = 0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const uint64_t wv = ballot(key[t] >= th);
      if (t < 64) { if (lane == (uint32_t)t) w0 = wv; }
      else if (lane == (uint32_t)(t - 64)) w1 = wv;
    }
    if (lane < (uint32_t)R) codes[v * R + lane] = w0;
    if (R > 64 && lane + 64 < (uint32_t)R) codes[v * R + lane + 64] = w1;
    wave_lds_sync();
  }
}

template <int R>
__global__ void __launch_bounds__(512)
k_encode_sets(HashGeom g, const int8_t* __restrict__ hi, const uint8_t* __restrict__ lo,
              const uint64_t* __restrict__ offsets, uint64_t n_sets, uint8_t* __restrict__ cnt_rm,
              uint64_t* __restrict__ bits_rm, int topbit) {
  extern __shared__ __align__(16) uint8_t smem[];
  const EncodeShared sh = encode_setup(g, smem);
  const uint32_t lane = lane_id();
  const uint32_t nw = blockDim.x / BVS_WAVE;
  const uint32_t koff = g.s * 4096u;
  constexpr int NC = (R + 3) / 4;
  constexpr int NO = (R + 63) / 64;
  for (uint64_t set = blockIdx.x * (uint64_t)nw + wave_id(); set < n_sets;
       set += (uint64_t)gridDim.x * nw) {
    uint32_t cnt[NC];
    uint64_t orb[NO];
#pragma unroll
    for (int i = 0; i < NC; ++i) cnt[i] = 0;
#pragma unroll
    for (int i = 0; i < NO; ++i) orb[i] = 0;
    const uint64_t o0 = offsets[set], o1 = offsets[set + 1];
    for (uint64_t v = o0; v < o1; ++v) {
      stage_vector(sh.av, hi, lo, v, g.dim_padded, lane);
      wave_lds_sync();
      uint32_t key[R];
      hash_keys<R>(sh.av, sh.idx, g.SP, koff, g.lgL, g.L, lane, key);
      const uint32_t th = kth_largest<R>(key, g.wta_k, topbit);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const uint32_t b = key[t] >= th ? 1u : 0u;
        cnt[t / 4] += b << (8 * (t % 4));   // a set has at most 255 members
        orb[t / 64] |= (uint64_t)b << (t % 64);
      }
      wave_lds_sync();
    }
    uint8_t* cr = cnt_rm + set * g.L;
#pragma unroll
    for (int t = 0; t < R; ++t) cr[64u * t + lane] = (uint8_t)(cnt[t / 4] >> (8 * (t % 4)));
    uint64_t w0 = 0, w1 = 0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const uint64_t wv = ballot((orb[t / 64] >> (t % 64)) & 1);
      if (t < 64) { if (lane == (uint32_t)t) w0 = wv; }
      else if (lane == (uint32_t)(t - 64)) w1 = wv;
    }
    if (lane < (uint32_t)R) bits_rm[set * R + lane] = w0;
    if (R > 64 && lane + 64 < (uint32_t)R) bits_rm[set * R + lane + 64] = w1;
  }
}

template <typename F>
static hipError_t dispatch_R(uint32_t R, F&& f) {
  switch (R) {
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    default: return hipErrorInvalidValue;
  }
}

// Waves per workgroup: the projection table fills most of the LDS, so one
// workgroup runs per CU; queries use 16 waves (4 per SIMD), the set kernel,
// whose per-set counters need more registers, 8.
static constexpr uint32_t kEncodeVecWaves = 16;
static constexpr uint32_t kEncodeWaves = 8;

hipError_t launch_encode_vectors(const HashGeom& g, const int8_t* hi, const uint8_t* lo, uint64_t n,
                                 uint64_t* codes, int n_cu, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // 8 waves when 16 staging slots would not fit beside the table
  const uint32_t nw = encode_lds_bytes(g, kEncodeVecWaves) <= 160 * 1024 ? kEncodeVecWaves : kEncodeWaves;
  const size_t lds = encode_lds_bytes(g, nw);
  const int topbit = key_topbit(g);
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + nw - 1) / nw, (uint64_t)n_cu);
  return dispatch_R(g.R, [&](auto rc) -> hipError_t {
    constexpr int R = decltype(rc)::value;
    hipError_t e = hipFuncSetAttribute((const void*)k_encode_vectors<R>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_encode_vectors<R>, dim3(grid), dim3(64 * nw), lds, st, g, hi, lo, n,
                       codes, topbit);
    return hipGetLastError();
  });
}

hipError_t launch_encode_sets(const HashGeom& g, const int8_t* hi, const uint8_t* lo,
                              const uint64_t* offsets, uint64_t n_sets, uint8_t* cnt_rm,
                              uint64_t* bits_rm, int n_cu, hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  const size_t lds = encode_lds_bytes(g, kEncodeWaves);
  const int topbit = key_topbit(g);
  const uint32_t grid =
      (uint32_t)std::min<uint64_t>((n_sets + kEncodeWaves - 1) / kEncodeWaves, (uint64_t)n_cu);
  return dispatch_R(g.R, [&](auto rc) -> hipError_t {
    constexpr int R = decltype(rc)::value;
    hipError_t e = hipFuncSetAttribute((const void*)k_encode_sets<R>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_encode_sets<R>, dim3(grid), dim3(64 * kEncodeWaves), lds, st, g, hi, lo,
                       offsets, n_sets, cnt_rm, bits_rm, topbit);
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------- transposes
// counts [n][L] -> [L][ld]; tile = 128 sets x 256 positions.
__global__ void __launch_bounds__(256)
k_transpose_counts(const uint8_t* __restrict__ src, uint64_t n_sets, uint64_t ld, uint32_t L,
                   uint8_t* __restrict__ dst) {
  __shared__ uint8_t tile[128][256 + 4];
  const uint32_t p0 = blockIdx.x * 256u;
  const uint64_t s0 = (uint64_t)blockIdx.y * 128u;
  const uint32_t t = threadIdx.x;
  // read: 16 threads per set row (16 B each), 16 rows per pass
  for (uint32_t r = t / 16; r < 128; r += 16) {
    const uint64_t set = s0 + r;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (set < n_sets) v = *(const uint4*)(src + set * L + p0 + 16u * (t % 16));
    uint32_t* dw = (uint32_t*)&tile[r][16u * (t % 16)];
    dw[0] = v.x; dw[1] = v.y; dw[2] = v.z; dw[3] = v.w;
  }
  __syncthreads();
  // write: 8 threads per position row (16 sets each), 32 rows per pass
  for (uint32_t pr = t / 8; pr < 256; pr += 32) {
    const uint32_t c0 = 16u * (t % 8);
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w[q] = (uint32_t)tile[c0 + 4 * q + 0][pr] | ((uint32_t)tile[c0 + 4 * q + 1][pr] << 8) |
             ((uint32_t)tile[c0 + 4 * q + 2][pr] << 16) | ((uint32_t)tile[c0 + 4 * q + 3][pr] << 24);
    }
    if (s0 + c0 < ld) *(uint4*)(dst + (uint64_t)(p0 + pr) * ld + s0 + c0) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// bits [n][R] u64 -> chunk-major [R/2][ld] of 16-byte chunks; tile = 64 sets.
__global__ void __launch_bounds__(256)
k_transpose_bits(const uint64_t* __restrict__ src, uint64_t n_sets, uint64_t ld, uint32_t R,
                 uint64_t* __restrict__ dst) {
  extern __shared__ __align__(16) uint4 tb[];   // [64][RC + 1]
  const uint32_t RC = R / 2;
  const uint64_t s0 = (uint64_t)blockIdx.x * 64u;
  for (uint32_t i = threadIdx.x; i < 64u * RC; i += blockDim.x) {
    const uint32_t r = i / RC, c = i % RC;
    const uint64_t set = s0 + r;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (set < n_sets) v = ((const uint4*)(src + set * R))[c];
    tb[r * (RC + 1) + c] = v;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < 64u * RC; i += blockDim.x) {
    const uint32_t c = i / 64, r = i % 64;
    if (s0 + r < ld) ((uint4*)dst)[(uint64_t)c * ld + s0 + r] = tb[r * (RC + 1) + c];
  }
}

hipError_t launch_transpose_sketches(const uint8_t* cnt_rm, const uint64_t* bits_rm, uint64_t n_sets,
                                     uint64_t ld, uint32_t L, uint8_t* cnt, uint64_t* bits,
                                     hipStream_t st) {
  const uint32_t R = L / 64;
  dim3 g1(L / 256 ? L / 256 : 1, (uint32_t)((ld + 127) / 128));
  if (L % 256 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose_counts, g1, dim3(256), 0, st, cnt_rm, n_sets, ld, L, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)64 * (R / 2 + 1) * 16;
  e = hipFuncSetAttribute((const void*)k_transpose_bits, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose_bits, dim3((uint32_t)((ld + 63) / 64)), dim3(256), lds, st, bits_rm,
                     n_sets, ld, R, bits);
  return hipGetLastError();
}

// ---------------------------------------------------------------- bitmap planes
// Membership bitmaps of the first layer with M = 1, tile-major: for the tile
// of 256 sets t = j / 256, row p of the tile is the four words
// [(t L + p) 4 .. + 3], and bit (j % 64) of word (j % 256) / 64 of it is set
// when C^(j)[p] >= 1, i.e. set j is on the inverted list of position p
// (Def. 9).  A tile's L rows are one contiguous run of 32 L bytes.  One thread
// per word.
__global__ void __launch_bounds__(256)
k_bitmap_planes(const uint8_t* __restrict__ cnt, uint64_t ld, uint32_t L, uint64_t* __restrict__ planes) {
  const uint64_t wpp = ld / 64;
  const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
  if (i >= (uint64_t)L * wpp) return;
  const uint64_t p = i / wpp, w = i % wpp;
  const uint4* src = (const uint4*)(cnt + p * ld + w * 64);
  uint64_t bits = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint4 v = src[k];
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 16; ++e)
      if ((d[e / 4] >> (8 * (e % 4))) & 0xFF) bits |= 1ull << (16 * k + e);
  }
  planes[((w / 4) * L + p) * 4 + w % 4] = bits;
}

hipError_t launch_bitmap_planes(const uint8_t* cnt, uint64_t ld, uint32_t L, uint64_t* planes, hipStream_t st) {
  const uint64_t n = (uint64_t)L * (ld / 64);
  hipLaunchKernelGGL(k_bitmap_planes, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, cnt, ld, L, planes);
  return hipGetLastError();
}

// ---------------------------------------------------------------- query sketch
// One wave per query.  Lane l owns code word l (L <= 4096, so R <= 64): the
// counts of positions 64 l .. 64 l + 63 stay in its registers for the
// selection of the A largest.
__global__ void __launch_bounds__(64)
k_query_sketch(const uint64_t* __restrict__ codes, const uint64_t* __restrict__ q_off, uint32_t L,
               uint32_t R, uint32_t A, uint32_t lgL, uint16_t* __restrict__ cq, uint64_t* __restrict__ sq,
               uint32_t* __restrict__ pos, uint64_t* __restrict__ gate, uint64_t* __restrict__ gate_chunks) {
  const uint32_t q = blockIdx.x, lane = lane_id();
  const uint64_t o0 = q_off[q], o1 = q_off[q + 1];
  uint16_t* cqq = cq + (uint64_t)q * L;
  const bool own = lane < R;
  uint32_t c[64];
#pragma unroll
  for (int b = 0; b < 64; ++b) c[b] = 0;
  if (own) {
    // Eight vectors' words in flight at once (read at a clamped vector,
    // masked); their bits are summed in 4-bit fields (bit 4 i + j of the word
    // in field i of nib[j], at most 8 per batch) and then added to the counts.
    uint64_t orw = 0;
    for (uint64_t v0 = o0; v0 < o1; v0 += 8) {
      uint64_t w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = codes[min(v0 + u, o1 - 1) * R + lane];
      uint64_t nib[4] = {0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint64_t x = v0 + u < o1 ? w[u] : 0ull;
        orw |= x;
#pragma unroll
        for (int j = 0; j < 4; ++j) nib[j] += (x >> j) & 0x1111111111111111ull;
      }
#pragma unroll
      for (int b = 0; b < 64; ++b) c[b] += (uint32_t)(nib[b & 3] >> (4 * (b >> 2))) & 15u;
    }
    sq[(uint64_t)q * R + lane] = orw;
#pragma unroll
    for (int b = 0; b < 64; b += 2)
      *(uint32_t*)(cqq + 64u * lane + b) = (c[b] & 0xFFFF) | ((c[b + 1] & 0xFFFF) << 16);
  }
  // The A largest (count, -position) keys, one per round.
  uint32_t last = 0xFFFFFFFFu;
  uint32_t p[8];
  for (uint32_t a = 0; a < A; ++a) {
    uint32_t best = 0;
    if (own) {
#pragma unroll
      for (int b = 0; b < 64; ++b) {
        const uint32_t key = (c[b] << lgL) | (L - 1u - (64u * lane + (uint32_t)b));
        best = key < last ? max(best, key) : best;
      }
    }
    // keys are unique and >= 0; a lane with no candidate contributes 0, which
    // can only win when fewer than A positions exist (A <= L is checked).
    last = wave_max_u32(best);
    p[a] = L - 1u - (last & (L - 1u));
    if (lane == 0) pos[(uint64_t)q * A + a] = p[a];
  }
  uint64_t chunks = 0;
  for (uint32_t a = 0; a < A; ++a) chunks |= 1ull << (p[a] >> 7);
  if (own) {
    uint64_t gw = 0;
    for (uint32_t a = 0; a < A; ++a)
      if ((p[a] >> 6) == lane) gw |= 1ull << (p[a] & 63);
    gate[(uint64_t)q * R + lane] = gw;
  }
  if (lane == 0) gate_chunks[q] = chunks;
}

hipError_t launch_query_sketch(const uint64_t* codes, const uint64_t* q_off, uint32_t n_q, uint32_t L,
                               uint32_t R, uint32_t A, uint16_t* cq, uint64_t* sq, uint32_t* pos,
                               uint64_t* gate, uint64_t* gate_chunks, hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  if (R > 64 || A > 8) return hipErrorInvalidValue;
  uint32_t lgL = 0;
  while ((1u << lgL) < L) ++lgL;
  hipLaunchKernelGGL(k_query_sketch, dim3(n_q), dim3(64), 0, st, codes, q_off, L, R, A, lgL, cq, sq, pos,
                     gate, gate_chunks);
  return hipGetLastError();
}

// ---------------------------------------------------------------- fill
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v, const uint32_t* run_if) {
  if (run_if && *run_if == 0) return;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st, const uint32_t* run_if) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, p, n, v, run_if);
  return hipGetLastError();
}

}  // namespace bvs
