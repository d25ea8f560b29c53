// Learned projection ahead of the winner-take-all (Def. 7 applied to learned
// outputs): y = W2 relu(W1 x + b1) + b2, its inference on the matrix cores
// (bfloat16 operands, float32 accumulation), the codes and set sketches it
// gives, and the kernels of its triplet training (soft codes, soft sketches,
// soft Hamming triplet loss, backward pass, Adam).
#include "device.h"
#include "launch.h"
#include "wta.h"

namespace bvs {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_k A(m, k) B(k, n), bfloat16 operands, float32 accumulation.
//   A(m, k) = A[m * lda + k] (AT = false) or A[k * lda + m] (AT = true)
//   B(k, n) = B[n * ldb + k] (BT = false) or B[k * ldb + n] (BT = true)
// Epilogue: v = acc + bias[n] (bias may be null), relu if asked, then v to
// C32[m * ldc + n] and / or bfloat16(v) to C16 (either may be null).
// Workgroup tile 128 x 128 x 32 staged in LDS with k contiguous (two
// buffers); four waves, each a 64 x 64 block of 16 x 16 x 32 bf16
// matrix-core products.
// Leading dimensions are multiples of 8 elements (16-byte rows).
static constexpr int GM = 128, GN = 128, GK = 32, GPAD = 8;

// One 128 x 32 operand step in registers: two 16-byte chunks per thread,
// zero past the matrix, loaded ahead of the products of the step before.
struct GemmRegs {
  uint4 v[2];
};

// Load the chunks of the step at k0.  TR false: rows r0.., 32 contiguous k
// (128 rows x 4 chunks of 8); TR true: 32 k rows of 128 contiguous r (32 x
// 16 chunks of 8), transposed when stored.
template <bool TR>
__device__ __forceinline__ void gemm_load(const uint16_t* __restrict__ X, uint64_t ld, uint32_t r0, uint32_t R,
                                          uint32_t k0, uint32_t K, GemmRegs& g) {
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const uint32_t c = t + 256 * it;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (!TR) {
      const uint32_t gr = r0 + (c >> 2), gk = k0 + (c & 3) * 8;
      if (gr < R) {
        const uint16_t* p = X + (uint64_t)gr * ld + gk;
        if (gk + 8 <= K) {
          v = *(const uint4*)p;
        } else {
          uint16_t e[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) e[i] = gk + i < K ? p[i] : (uint16_t)0;
          v = make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                         e[6] | (uint32_t)e[7] << 16);
        }
      }
    } else {
      const uint32_t gk = k0 + (c >> 4), gr = r0 + (c & 15) * 8;
      if (gk < K) {
        const uint16_t* p = X + (uint64_t)gk * ld + gr;
        if (gr + 8 <= R) {
          v = *(const uint4*)p;
        } else {
          uint16_t e[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) e[i] = gr + i < R ? p[i] : (uint16_t)0;
          v = make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                         e[6] | (uint32_t)e[7] << 16);
        }
      }
    }
    g.v[it] = v;
  }
}

// Store loaded chunks into the LDS step, k contiguous per row.
template <bool TR>
__device__ __forceinline__ void gemm_store(const GemmRegs& g, uint16_t (*s)[GK + GPAD]) {
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const uint32_t c = t + 256 * it;
    if (!TR) {
      *(uint4*)&s[c >> 2][(c & 3) * 8] = g.v[it];
    } else {
      const uint32_t kk = c >> 4, rc = (c & 15) * 8;
      const uint32_t w[4] = {g.v[it].x, g.v[it].y, g.v[it].z, g.v[it].w};
#pragma unroll
      for (int i = 0; i < 8; ++i) s[rc + i][kk] = (uint16_t)(w[i / 2] >> (16 * (i % 2)));
    }
  }
}

// Two LDS steps: step i is stored into buffer i mod 2 behind one barrier,
// and the loads of step i + 1 are in flight while step i's products run
// (buffer (i + 1) mod 2 was last read in step i - 1, before that barrier).
template <bool AT, bool BT>
__global__ void __launch_bounds__(256)
k_gemm(const uint16_t* __restrict__ A, uint64_t lda, const uint16_t* __restrict__ B, uint64_t ldb, uint32_t M,
       uint32_t N, uint32_t K, const float* __restrict__ bias, int relu, float* __restrict__ C32,
       uint16_t* __restrict__ C16, uint64_t ldc) {
  __shared__ __align__(16) uint16_t sA[2][GM][GK + GPAD];
  __shared__ __align__(16) uint16_t sB[2][GN][GK + GPAD];
  const uint32_t m0 = blockIdx.y * GM, n0 = blockIdx.x * GN;
  const uint32_t w = wave_id(), lane = lane_id();
  const uint32_t wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const uint32_t r = lane & 15, g = lane >> 4;
  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  GemmRegs ra, rb;
  gemm_load<AT>(A, lda, m0, M, 0, K, ra);
  gemm_load<BT>(B, ldb, n0, N, 0, K, rb);
  uint32_t buf = 0;
  for (uint32_t k0 = 0; k0 < K; k0 += GK, buf ^= 1) {
    gemm_store<AT>(ra, sA[buf]);
    gemm_store<BT>(rb, sB[buf]);
    __syncthreads();
    if (k0 + GK < K) {
      gemm_load<AT>(A, lda, m0, M, k0 + GK, K, ra);
      gemm_load<BT>(B, ldb, n0, N, k0 + GK, K, rb);
    }
    v8bf af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *(const v8bf*)&sA[buf][wm + 16 * i + r][8 * g];
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = *(const v8bf*)&sB[buf][wn + 16 * j + r][8 * g];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t n = n0 + wn + 16 * j + r;
      if (n >= N) continue;
      const float bv = bias ? bias[n] : 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t m = m0 + wm + 16 * i + 4 * g + e;
        if (m >= M) continue;
        float v = acc[i][j][e] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (C32) C32[(uint64_t)m * ldc + n] = v;
        if (C16) C16[(uint64_t)m * ldc + n] = f2bf(v);
      }
    }
  }
}

hipError_t launch_gemm(bool at, bool bt, const uint16_t* A, uint64_t lda, const uint16_t* B, uint64_t ldb,
                       uint32_t M, uint32_t N, uint32_t K, const float* bias, bool relu, float* C32, uint16_t* C16,
                       uint64_t ldc, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  if ((lda | ldb) % 8 != 0) return hipErrorInvalidValue;
  const dim3 grid((N + GN - 1) / GN, (M + GM - 1) / GM);
  if (grid.y > 65535u) return hipErrorInvalidValue;
  if (!at && !bt)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, bias, relu ? 1 : 0,
                       C32, C16, ldc);
  else if (!at && bt)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, bias, relu ? 1 : 0,
                       C32, C16, ldc);
  else if (at && bt)
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, bias, relu ? 1 : 0,
                       C32, C16, ldc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------ conversions
// rows[i] of X (float32 [.][d]) -> bfloat16 out[i][d]; rows may be null (i).
__global__ void __launch_bounds__(256)
k_rows_to_bf16(const float* __restrict__ X, uint32_t d, const uint64_t* __restrict__ rows, uint64_t n,
               uint16_t* __restrict__ out) {
  const uint64_t total = n * d;
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < total; e += (uint64_t)gridDim.x * 256) {
    const uint64_t i = e / d, c = e % d;
    const uint64_t src = rows ? rows[i] : i;
    out[e] = f2bf(X[src * d + c]);
  }
}

hipError_t launch_rows_to_bf16(const float* X, uint32_t d, const uint64_t* rows, uint64_t n, uint16_t* out,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n * d + 255) / 256, 65536);
  hipLaunchKernelGGL(k_rows_to_bf16, dim3((uint32_t)blocks), dim3(256), 0, st, X, d, rows, n, out);
  return hipGetLastError();
}

// exact int8 planes (a = 64 hi + lo = 4096 x) -> bfloat16(x) [n][d]
__global__ void __launch_bounds__(256)
k_planes_to_bf16(const int8_t* __restrict__ hi, const uint8_t* __restrict__ lo, uint32_t dp, uint32_t d, uint64_t n,
                 uint16_t* __restrict__ out) {
  const uint64_t total = n * d;
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < total; e += (uint64_t)gridDim.x * 256) {
    const uint64_t i = e / d, c = e % d;
    const int a = 64 * (int)hi[i * dp + c] + (int)lo[i * dp + c];
    out[e] = f2bf((float)a / 4096.0f);
  }
}

hipError_t launch_planes_to_bf16(const int8_t* hi, const uint8_t* lo, uint32_t dp, uint32_t d, uint64_t n,
                                 uint16_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n * d + 255) / 256, 65536);
  hipLaunchKernelGGL(k_planes_to_bf16, dim3((uint32_t)blocks), dim3(256), 0, st, hi, lo, dp, d, n, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_f32_to_bf16(const float* __restrict__ x, uint64_t n, uint16_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) out[i] = f2bf(x[i]);
}

hipError_t launch_f32_to_bf16(const float* x, uint64_t n, uint16_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_f32_to_bf16, dim3((uint32_t)blocks), dim3(256), 0, st, x, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ winner-take-all
// Order-preserving 16-bit key of a bfloat16 value.
__device__ __forceinline__ uint32_t bf16_order(uint16_t b) { return (b & 0x8000u) ? (~b & 0xFFFFu) : (b | 0x8000u); }

// One wave per row of Y (float32 [n][L], row stride ldy): codes [n][L/64]
// of the k largest bfloat16(y), ties to the lower index.
template <int R>
__global__ void __launch_bounds__(256)
k_wta_rows(const float* __restrict__ Y, uint64_t ldy, uint64_t n, uint32_t lgL, uint32_t k,
           uint64_t* __restrict__ codes) {
  const uint64_t row = (uint64_t)blockIdx.x * 4 + wave_id();
  if (row >= n) return;
  const uint32_t lane = lane_id();
  const uint32_t L = R * 64;
  uint32_t key[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const uint32_t j = 64 * t + lane;
    key[t] = (bf16_order(f2bf(Y[row * ldy + j])) << lgL) | (L - 1 - j);
  }
  const uint32_t th = kth_largest<R>(key, k, 15 + (int)lgL);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const uint64_t wv = ballot(key[t] >= th);
    if (lane == (uint32_t)t) codes[row * R + t] = wv;
  }
}

hipError_t launch_wta_rows(const float* Y, uint64_t ldy, uint64_t n, uint32_t L, uint32_t k, uint64_t* codes,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t lgL = 0;
  while ((1u << lgL) < L) ++lgL;
  const uint64_t blocks = (n + 3) / 4;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  switch (L / 64) {
#define BVS_WTA_CASE(RR)                                                                                      \
  case RR:                                                                                                    \
    hipLaunchKernelGGL(k_wta_rows<RR>, dim3((uint32_t)blocks), dim3(256), 0, st, Y, ldy, n, lgL, k, codes); \
    break;
    BVS_WTA_CASE(4)
    BVS_WTA_CASE(8)
    BVS_WTA_CASE(16)
    BVS_WTA_CASE(32)
    BVS_WTA_CASE(64)
#undef BVS_WTA_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One wave per set: row-major counts [n][L] and OR words [n][R] of the codes
// of its members (rows offsets[s] - base .. of codes).
__global__ void __launch_bounds__(256)
k_sets_from_codes(const uint64_t* __restrict__ codes, const uint64_t* __restrict__ offsets, uint64_t base,
                  uint64_t s0, uint64_t n_sets, uint32_t R, uint8_t* __restrict__ cnt_rm,
                  uint64_t* __restrict__ bits_rm) {
  const uint64_t s = s0 + (uint64_t)blockIdx.x * 4 + wave_id();
  if (s >= s0 + n_sets) return;
  const uint32_t lane = lane_id();
  const uint64_t r0 = offsets[s] - base, r1 = offsets[s + 1] - base;
  for (uint32_t t = 0; t < R; ++t) {
    uint32_t c = 0;
    uint64_t orw = 0;
    for (uint64_t r = r0; r < r1; ++r) {
      const uint64_t wv = codes[r * R + t];
      c += (uint32_t)((wv >> lane) & 1u);
      orw |= wv;
    }
    cnt_rm[s * (uint64_t)R * 64 + 64 * t + lane] = (uint8_t)c;
    if (lane == 0) bits_rm[s * R + t] = orw;
  }
}

hipError_t launch_sets_from_codes(const uint64_t* codes, const uint64_t* offsets, uint64_t base, uint64_t s0,
                                  uint64_t n_sets, uint32_t R, uint8_t* cnt_rm, uint64_t* bits_rm, hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  const uint64_t blocks = (n_sets + 3) / 4;
  hipLaunchKernelGGL(k_sets_from_codes, dim3((uint32_t)blocks), dim3(256), 0, st, codes, offsets, base, s0, n_sets,
                     R, cnt_rm, bits_rm);
  return hipGetLastError();
}

// ------------------------------------------------------------------ training
// Order-preserving 32-bit key of a float.
__device__ __forceinline__ uint32_t f32_order(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float f32_unorder(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// k-th largest value (duplicates counted) of the per-lane keys.
template <int R>
__device__ __forceinline__ uint32_t wave_kth_value_key(const uint32_t (&key)[R], uint32_t k) {
  uint32_t th = 0;
  for (int b = 31; b >= 0; --b) {
    const uint32_t cand = th | (1u << b);
    uint32_t cnt = 0;
#pragma unroll
    for (int t = 0; t < R; ++t) cnt += popc64(ballot(key[t] >= cand));
    if (cnt >= k) th = cand;
  }
  return th;
}

// One wave per row: t = midpoint of the k-th and (k+1)-th largest y.
template <int R>
__global__ void __launch_bounds__(256)
k_row_thresholds(const float* __restrict__ Y, uint64_t n, uint32_t k, float* __restrict__ thr) {
  const uint64_t row = (uint64_t)blockIdx.x * 4 + wave_id();
  if (row >= n) return;
  const uint32_t lane = lane_id();
  uint32_t key[R];
#pragma unroll
  for (int t = 0; t < R; ++t) key[t] = f32_order(Y[row * (R * 64) + 64 * t + lane]);
  const float a = f32_unorder(wave_kth_value_key<R>(key, k));
  const float b = f32_unorder(wave_kth_value_key<R>(key, k + 1));
  if (lane == 0) thr[row] = 0.5f * (a + b);
}

__device__ __forceinline__ float softplus(float z) { return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z)); }

// One block per batch set: LS[s][j] = sum over its rows of log(1 - c_j)
// = -sum softplus(z), z = (y - t) / tau; S = 1 - exp(LS).
__global__ void __launch_bounds__(256)
k_set_soft(const float* __restrict__ Y, const float* __restrict__ thr, const uint32_t* __restrict__ row_off,
           uint32_t L, float inv_tau, float* __restrict__ LS, float* __restrict__ S) {
  const uint32_t s = blockIdx.x;
  const uint32_t r0 = row_off[s], r1 = row_off[s + 1];
  for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
    float acc = 0.f;
    for (uint32_t r = r0; r < r1; ++r) acc -= softplus((Y[(uint64_t)r * L + j] - thr[r]) * inv_tau);
    LS[(uint64_t)s * L + j] = acc;
    S[(uint64_t)s * L + j] = -expm1f(acc);
  }
}

// One block per triplet (batch-local set indices): the hinge, its mean in
// *loss, and the sketch gradients added to dS.
__global__ void __launch_bounds__(256)
k_triplet(const float* __restrict__ S, const uint32_t* __restrict__ trip, uint32_t L, float margin, float inv_nt,
          float* __restrict__ dS, float* __restrict__ loss) {
  __shared__ float part[4];
  __shared__ float s_l;
  const uint32_t q = trip[3 * blockIdx.x], p = trip[3 * blockIdx.x + 1], n = trip[3 * blockIdx.x + 2];
  const float* Sq = S + (uint64_t)q * L;
  const float* Sp = S + (uint64_t)p * L;
  const float* Sn = S + (uint64_t)n * L;
  float acc = 0.f;
  for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
    const float a = Sq[j], b = Sp[j], c = Sn[j];
    acc += (b - 2.f * a * b) - (c - 2.f * a * c);   // h(Q,P) - h(Q,N); the S_Q terms cancel
  }
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, BVS_WAVE);
  if (lane_id() == 0) part[threadIdx.x / BVS_WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_l = margin + part[0] + part[1] + part[2] + part[3];
    if (s_l > 0.f) atomicAdd(loss, s_l * inv_nt);
  }
  __syncthreads();
  if (s_l <= 0.f) return;
  for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
    const float a = Sq[j], b = Sp[j], c = Sn[j];
    atomicAdd(&dS[(uint64_t)q * L + j], 2.f * (c - b) * inv_nt);
    atomicAdd(&dS[(uint64_t)p * L + j], (1.f - 2.f * a) * inv_nt);
    atomicAdd(&dS[(uint64_t)n * L + j], -(1.f - 2.f * a) * inv_nt);
  }
}

// One block per batch set: dy = dS * prod_{others}(1 - c) * c (1 - c) / tau,
// prod_{others}(1 - c) = exp(LS + softplus(z)).  Writes float32 and bfloat16.
__global__ void __launch_bounds__(256)
k_soft_backward(const float* __restrict__ Y, const float* __restrict__ thr, const uint32_t* __restrict__ row_off,
                uint32_t L, float inv_tau, const float* __restrict__ LS, const float* __restrict__ dS,
                float* __restrict__ dY, uint16_t* __restrict__ dY16) {
  const uint32_t s = blockIdx.x;
  const uint32_t r0 = row_off[s], r1 = row_off[s + 1];
  for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
    const float g = dS[(uint64_t)s * L + j];
    const float ls = LS[(uint64_t)s * L + j];
    for (uint32_t r = r0; r < r1; ++r) {
      const float z = (Y[(uint64_t)r * L + j] - thr[r]) * inv_tau;
      const float c = 1.f / (1.f + expf(-z));
      const float v = g == 0.f ? 0.f : g * expf(ls + softplus(z)) * c * (1.f - c) * inv_tau;
      dY[(uint64_t)r * L + j] = v;
      dY16[(uint64_t)r * L + j] = f2bf(v);
    }
  }
}

// dpre = dh where the hidden unit was active, float32 and bfloat16.
__global__ void __launch_bounds__(256)
k_relu_backward(const float* __restrict__ dH, const uint16_t* __restrict__ H16, uint64_t n, float* __restrict__ dP,
                uint16_t* __restrict__ dP16) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const float v = (H16[i] & 0x7FFFu) != 0 ? dH[i] : 0.f;
    dP[i] = v;
    dP16[i] = f2bf(v);
  }
}

// Column sums of X [n][C] into out[C] (out cleared by the caller).
__global__ void __launch_bounds__(256)
k_colsum(const float* __restrict__ X, uint64_t n, uint32_t C, float* __restrict__ out) {
  const uint32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  const uint64_t r0 = (uint64_t)blockIdx.y * 256, r1 = min(n, r0 + 256);
  float acc = 0.f;
  for (uint64_t r = r0; r < r1; ++r) acc += X[r * C + c];
  atomicAdd(&out[c], acc);
}

// Adam on float32 parameters; refreshes the bfloat16 copy when given.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v, uint64_t n,
       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t* __restrict__ w16) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (w16) w16[i] = f2bf(wi);
  }
}

hipError_t launch_row_thresholds(const float* Y, uint64_t n, uint32_t L, uint32_t k, float* thr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 3) / 4;
  switch (L / 64) {
#define BVS_THR_CASE(RR)                                                                                      \
  case RR:                                                                                                    \
    hipLaunchKernelGGL(k_row_thresholds<RR>, dim3((uint32_t)blocks), dim3(256), 0, st, Y, n, k, thr);         \
    break;
    BVS_THR_CASE(4)
    BVS_THR_CASE(8)
    BVS_THR_CASE(16)
    BVS_THR_CASE(32)
    BVS_THR_CASE(64)
#undef BVS_THR_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_soft(const float* Y, const float* thr, const uint32_t* row_off, uint32_t n_sets, uint32_t L,
                           float tau, float* LS, float* S, hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_soft, dim3(n_sets), dim3(256), 0, st, Y, thr, row_off, L, 1.f / tau, LS, S);
  return hipGetLastError();
}

hipError_t launch_triplet(const float* S, const uint32_t* trip, uint32_t n_trip, uint32_t L, float margin,
                          float* dS, float* loss, hipStream_t st) {
  if (n_trip == 0) return hipSuccess;
  hipLaunchKernelGGL(k_triplet, dim3(n_trip), dim3(256), 0, st, S, trip, L, margin, 1.f / (float)n_trip, dS, loss);
  return hipGetLastError();
}

hipError_t launch_soft_backward(const float* Y, const float* thr, const uint32_t* row_off, uint32_t n_sets, uint32_t L,
                                float tau, const float* LS, const float* dS, float* dY, uint16_t* dY16,
                                hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  hipLaunchKernelGGL(k_soft_backward, dim3(n_sets), dim3(256), 0, st, Y, thr, row_off, L, 1.f / tau, LS, dS, dY,
                     dY16);
  return hipGetLastError();
}

hipError_t launch_relu_backward(const float* dH, const uint16_t* H16, uint64_t n, float* dP, uint16_t* dP16,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_relu_backward, dim3((uint32_t)blocks), dim3(256), 0, st, dH, H16, n, dP, dP16);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, uint64_t n, uint32_t C, float* out, hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)out, C, 0u, st);
  if (e != hipSuccess || n == 0) return e;
  const uint64_t gy = (n + 255) / 256;
  if (gy > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colsum, dim3((C + 255) / 256, (uint32_t)gy), dim3(256), 0, st, X, n, C, out);
  return hipGetLastError();
}

// acc += (double)loss: the sum of an epoch's batch losses, in batch order.
__global__ void k_add_loss(const float* __restrict__ loss, double* __restrict__ acc) { *acc += (double)*loss; }

hipError_t launch_add_loss(const float* loss, double* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_add_loss, dim3(1), dim3(1), 0, st, loss, acc);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, uint32_t step, uint16_t* w16, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const float c1 = 1.f / (1.f - powf(b1, (float)step));
  const float c2 = 1.f / (1.f - powf(b2, (float)step));
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_adam, dim3((uint32_t)blocks), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2, w16);
  return hipGetLastError();
}

hipError_t encode_learned(const Mlp& m, const uint16_t* X16, uint64_t n, uint16_t* H16, float* Y, uint64_t* codes,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n > 0xFFFFFFFFull) return hipErrorInvalidValue;
  hipError_t e = launch_gemm(false, false, X16, m.d, m.W1, m.d, (uint32_t)n, m.H, m.d, m.b1, true, nullptr, H16, m.H,
                             st);
  if (e != hipSuccess) return e;
  e = launch_gemm(false, false, H16, m.H, m.W2, m.H, (uint32_t)n, m.L, m.H, m.b2, false, Y, nullptr, m.L, st);
  if (e != hipSuccess) return e;
  return launch_wta_rows(Y, m.L, n, m.L, m.wta_k, codes, st);
}

// Uniform initialisation in +-sqrt(6 / fan_in) (biases 0) from splitmix64 of
// (seed, parameter index): W1 [H][d], b1 [H], W2 [L][H], b2 [L] packed.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void __launch_bounds__(256)
k_mlp_init(float* __restrict__ w, uint32_t d, uint32_t H, uint32_t L, uint64_t seed) {
  const uint64_t n1 = (uint64_t)H * d, n2 = (uint64_t)L * H;
  const uint64_t total = n1 + H + n2 + L;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < total; i += (uint64_t)gridDim.x * 256) {
    float v = 0.f;
    float a = 0.f;
    if (i < n1) a = sqrtf(6.0f / (float)d);
    else if (i >= n1 + H && i < n1 + H + n2) a = sqrtf(6.0f / (float)H);
    if (a != 0.f) {
      const uint64_t r = splitmix64_at(seed * 0x2545F4914F6CDD1Dull + i);
      const float u = (float)(r >> 40) * (1.0f / 16777216.0f);   // [0, 1)
      v = (2.f * u - 1.f) * a;
    }
    w[i] = v;
  }
}

hipError_t launch_mlp_init(float* w, uint32_t d, uint32_t H, uint32_t L, uint64_t seed, hipStream_t st) {
  const uint64_t total = (uint64_t)H * d + H + (uint64_t)L * H + L;
  const uint64_t blocks = std::min<uint64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_mlp_init, dim3((uint32_t)blocks), dim3(256), 0, st, w, d, H, L, seed);
  return hipGetLastError();
}

}  // namespace bvs
