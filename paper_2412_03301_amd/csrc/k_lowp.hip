// Precision form of the re-rank: approximate Hausdorff values (Def. 4) from
// BF16 or OCP FP8 E4M3 (per-set scale) copies of the vectors, with pairwise
// dot products on the gfx950 matrix cores in FP32 accumulation, then the
// selection of the candidates to re-check exactly.
//
// Encodings (bit-exact definitions):
//   bf16   upper 16 bits of the float32 value, rounded to nearest even
//   e4m3   OCP E4M3 ("FN"): bias 7, 3 mantissa bits, largest value 448,
//          subnormals m * 2^-9, rounded to nearest even
// A set's FP8 scale is s = float32(max |x|) / 448 (1 for an all-zero set);
// its components are stored as e4m3(clamp(x / s, +-448)).  BF16 rows are
// 2 dp bytes, FP8 rows dp bytes rounded up to 128 (zero padded).
//
// Approximate squared distance of database row v (scale s_v) and query row
// q (scale s_q): D~2 = |v|^2 + |q|^2 - 2 s_v s_q (v~ . q~), clamped at 0,
// with the exact norms of the unquantised rows.
//
// Matrix-core mapping as in the exact re-rank (haus_core.h): one wave per
// candidate set, the set's 16-row tile in registers as the A operand, the
// query's 16-row tiles as the B operand (first rows from LDS, the rest from
// global memory).  bf16: v_mfma_f32_16x16x32_bf16, 16 bytes per lane per
// step; fp8: v_mfma_f32_16x16x128_f8f6f4 (E4M3 on both sides), 32 bytes per
// lane per step.  A and B lanes hold the same k indices, so the dot
// products do not depend on the order of k inside a step.
#include "haus_core.h"

namespace bvs {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// |t| <= 448 and t finite.
__device__ __forceinline__ uint32_t e4m3_rne_bits(float t) {
  const uint32_t sign = (__float_as_uint(t) >> 24) & 0x80u;
  const float a = fabsf(t);
  uint32_t code;
  if (a < 0x1p-6f) {
    code = (uint32_t)rintf(a * 512.0f);   // multiples of 2^-9; 8 is the smallest normal
  } else {
    int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;
    uint32_t m = (uint32_t)rintf((ldexpf(a, -e) - 1.0f) * 8.0f);
    if (m == 8) {
      ++e;
      m = 0;
    }
    code = ((uint32_t)(e + 7) << 3) | m;
  }
  return code | sign;
}

// One wave per set: scale (fp8) and the encoded rows of the set.
__global__ void __launch_bounds__(256)
k_lowp_encode(const int8_t* __restrict__ hi, const uint8_t* __restrict__ lo, uint32_t dp,
              const uint64_t* __restrict__ offsets, uint64_t n_sets, int fmt, uint32_t row_bytes,
              uint8_t* __restrict__ out, float* __restrict__ scale) {
  const uint64_t set = (uint64_t)blockIdx.x * 4 + wave_id();
  if (set >= n_sets) return;
  const uint32_t lane = lane_id();
  const uint64_t r0 = offsets[set], r1 = offsets[set + 1];
  float s = 1.0f;
  if (fmt == BVS_LOWP_FP8) {
    int mx = 0;
    for (uint64_t r = r0; r < r1; ++r)
      for (uint32_t c = lane; c < dp; c += BVS_WAVE) mx = max(mx, abs(64 * (int)hi[r * dp + c] + (int)lo[r * dp + c]));
    mx = (int)wave_max_u32((uint32_t)mx);
    if (mx > 0) s = ((float)mx / 4096.0f) / 448.0f;
    if (lane == 0) scale[set] = s;
  }
  for (uint64_t r = r0; r < r1; ++r) {
    for (uint32_t c = lane; c < row_bytes / (fmt == BVS_LOWP_FP8 ? 1u : 2u); c += BVS_WAVE) {
      const float x = c < dp ? (float)(64 * (int)hi[r * dp + c] + (int)lo[r * dp + c]) / 4096.0f : 0.0f;
      if (fmt == BVS_LOWP_FP8) {
        const float t = fminf(fmaxf(x / s, -448.0f), 448.0f);
        out[r * row_bytes + c] = (uint8_t)e4m3_rne_bits(t);
      } else {
        ((uint16_t*)(out + r * row_bytes))[c] = (uint16_t)bf16_rne_bits(x);
      }
    }
  }
}

hipError_t launch_lowp_encode(const int8_t* hi, const uint8_t* lo, uint32_t dp, const uint64_t* offsets,
                              uint64_t n_sets, int fmt, uint32_t row_bytes, uint8_t* out, float* scale,
                              hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  const uint64_t blocks = (n_sets + 3) / 4;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lowp_encode, dim3((uint32_t)blocks), dim3(256), 0, st, hi, lo, dp, offsets, n_sets, fmt,
                     row_bytes, out, scale);
  return hipGetLastError();
}

uint32_t lowp_row_bytes(int fmt, uint32_t dp) {
  return fmt == BVS_LOWP_FP8 ? (uint32_t)align_up(dp, 128) : 2 * dp;
}

// --------------------------------------------------------------------------
template <int FMT>
struct LpOp;
template <>
struct LpOp<BVS_LOWP_BF16> {
  static constexpr int LB = 16;   // bytes per lane per step
  typedef v8bf T;
  static __device__ __forceinline__ T load(const uint8_t* p) { return __builtin_bit_cast(T, *(const v4i*)p); }
  static __device__ __forceinline__ T load_nt(const uint8_t* p) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load((const v4i*)p));
  }
  static __device__ __forceinline__ T zero() { return __builtin_bit_cast(T, v4i{0, 0, 0, 0}); }
  static __device__ __forceinline__ v4f mfma(T a, T b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct LpOp<BVS_LOWP_FP8> {
  static constexpr int LB = 32;
  typedef v8i T;
  static __device__ __forceinline__ T load(const uint8_t* p) {
    const v4i a = *(const v4i*)p, b = *(const v4i*)(p + 16);
    return T{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  }
  static __device__ __forceinline__ T load_nt(const uint8_t* p) {
    const v4i a = __builtin_nontemporal_load((const v4i*)p);
    const v4i b = __builtin_nontemporal_load((const v4i*)(p + 16));
    return T{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  }
  static __device__ __forceinline__ T zero() { return T{0, 0, 0, 0, 0, 0, 0, 0}; }
  // E4M3 on both operands (format codes 0), no block scaling
  static __device__ __forceinline__ v4f mfma(T a, T b, v4f c) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
  }
};

struct LpView {
  const uint8_t* s_rows;   // LDS, stride row_bytes + 16
  const uint32_t* s_norm;
  const uint8_t* g_rows;   // global, stride row_bytes (the query's first row)
  const uint32_t* g_norm;
  float q_scale;
  uint32_t mq, nqt, nqt_s;
};

constexpr float kInv2p24 = 1.0f / 16777216.0f;

// Approximate squared Hausdorff values of NS sets at once (float bits;
// non-negative, so they order like the values).  Set s is [o0[s], o0[s] +
// m[s]) with scale sv[s]; m[s] = 0 marks an absent set.  With NS = 2 every
// query tile read from LDS feeds both sets' matrix products, which halves
// the LDS traffic per product.  With one set and a threshold thr (float
// bits), the set is abandoned (all ones, which no threshold admits) as soon
// as a completed part of its value exceeds thr: the largest column minimum
// after each database tile, the largest row minimum of each query tile on
// the last one.
template <int FMT, int KC, int MAXQT, bool HASG, int NS>
__device__ __forceinline__ void lp_items(const LowpDb& db, const uint64_t (&o0)[NS], const uint32_t (&m)[NS],
                                         const float (&sv)[NS], const LpView& q, uint32_t (&res)[NS],
                                         uint32_t thr, uint32_t& rows_read) {
  const bool bounded = NS == 1 && thr != 0xFFFFFFFFu;
  using Op = LpOp<FMT>;
  constexpr uint32_t LB = Op::LB;
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t RB = db.row_bytes;
  const uint32_t SS = RB + 16;
  uint32_t mmax = 0;
  float svq[NS];
  uint32_t qmin[NS][MAXQT], colmax[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    mmax = max(mmax, m[s]);
    svq[s] = sv[s] * q.q_scale;
    colmax[s] = 0;
#pragma unroll
    for (int i = 0; i < MAXQT; ++i) qmin[s][i] = 0xFFFFFFFFu;
  }
  for (uint32_t vt = 0; vt < mmax; vt += 16) {
    const bool last = vt + 16 >= mmax;
#pragma unroll
    for (int s = 0; s < NS; ++s) rows_read += vt < m[s] ? min(16u, m[s] - vt) : 0u;
    typename Op::T a[NS][KC];
    float nv[NS][4];
    uint32_t vmin[NS][4];
    bool vok[NS][4];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const uint32_t vrow = vt + c16;
      const bool vrow_ok = vrow < m[s];
      const uint8_t* pa = db.rows + (o0[s] + (vrow_ok ? vrow : 0)) * RB + LB * g;
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) a[s][kc] = vrow_ok ? Op::load_nt(pa + 4 * LB * kc) : Op::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t v = vt + 4 * g + r;
        vok[s][r] = v < m[s];
        nv[s][r] = vok[s][r] ? (float)db.norms[o0[s] + v] * kInv2p24 : 0.0f;
        vmin[s][r] = 0xFFFFFFFFu;
      }
    }
#pragma unroll
    for (int qt = 0; qt < MAXQT; ++qt) {
      if ((uint32_t)qt < q.nqt) {
        // two accumulation chains per set keep the matrix pipe busy
        v4f acc[NS][2];
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s][0] = acc[s][1] = v4f{0.f, 0.f, 0.f, 0.f};
        const uint32_t qi = qt * 16 + c16;
        const uint8_t* pb;
        float nq;
        if (!HASG || (uint32_t)qt < q.nqt_s) {
          pb = q.s_rows + qi * SS + LB * g;
          nq = (float)q.s_norm[qi] * kInv2p24;
        } else {
          asm volatile("" ::: "memory");
          const uint8_t* gb = uniform_ptr(q.g_rows);
          uint32_t cl = c16;
          asm volatile("" : "+s"(gb), "+v"(cl));
          const uint32_t r = min(qt * 16 + cl, q.mq - 1);
          pb = gb + r * RB + LB * g;
          nq = (float)q.g_norm[r] * kInv2p24;
        }
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          const typename Op::T b = Op::load(pb + 4 * LB * kc);
#pragma unroll
          for (int s = 0; s < NS; ++s) acc[s][kc & 1] = Op::mfma(a[s][kc], b, acc[s][kc & 1]);
        }
        const bool qok = qi < q.mq;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const v4f d = acc[s][0] + acc[s][1];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float d2 = fmaxf(nv[s][r] + nq - 2.0f * svq[s] * d[r], 0.0f);
            const uint32_t bits = (qok && vok[s][r]) ? __float_as_uint(d2) : 0xFFFFFFFFu;
            vmin[s][r] = min(vmin[s][r], bits);
            qmin[s][qt] = min(qmin[s][qt], bits);
          }
        }
        if (bounded && last) {
          const uint32_t rm = qok ? rows4_min_u32(qmin[0][qt]) : 0u;
          if ((uint32_t)__builtin_amdgcn_readfirstlane((int)row16_max_u32(rm)) > thr) {
            res[0] = 0xFFFFFFFFu;
            return;
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t cm = row16_min_u32(vmin[s][r]);
        if (vok[s][r]) colmax[s] = max(colmax[s], cm);
      }
    }
    if (bounded && !last && (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_dpp_u32(colmax[0])) > thr) {
      res[0] = 0xFFFFFFFFu;
      return;
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    uint32_t rowmax = 0;
#pragma unroll
    for (int qt = 0; qt < MAXQT; ++qt) {
      if ((uint32_t)qt < q.nqt) {
        uint32_t rm = qmin[s][qt];
        rm = min(rm, shfl_xor_u32(rm, 16));
        rm = min(rm, shfl_xor_u32(rm, 32));
        if ((uint32_t)qt * 16 + c16 < q.mq) rowmax = max(rowmax, rm);
      }
    }
    res[s] = wave_max_u32(max(colmax[s], rowmax));
  }
}

__device__ __forceinline__ LpView lp_stage(const LowpQ& qs, uint32_t q, uint32_t lds_rows, uint8_t* smem) {
  LpView v;
  const uint64_t o0 = qs.offsets[q];
  v.mq = (uint32_t)(qs.offsets[q + 1] - o0);
  v.nqt = (v.mq + 15) / 16;
  v.nqt_s = min(v.nqt, lds_rows / 16);
  const uint32_t RB = qs.row_bytes, SS = RB + 16;
  const uint32_t rows = v.nqt_s * 16;
  uint32_t* s_norm = (uint32_t*)(smem + (size_t)lds_rows * SS);
  {
    const uint8_t* const src[1] = {qs.rows + o0 * RB};
    uint8_t* const dst[1] = {smem};
    stage_rows<1>(src, dst, RB, SS, RB / 16, rows, v.mq);
  }
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x) s_norm[r] = r < v.mq ? qs.norms[o0 + r] : 0u;
  v.s_rows = smem;
  v.s_norm = s_norm;
  v.g_rows = qs.rows + o0 * RB;
  v.g_norm = qs.norms + o0;
  v.q_scale = qs.scale ? qs.scale[q] : 1.0f;
  __syncthreads();
  return v;
}

static constexpr uint32_t kLpWaves = 8;
static constexpr uint32_t kLpPerBlock = 64;

// Grid (ceil((lim - i0) / 64), n_q): candidates ids[q][i0 .. min(count[q],
// lim)) (count may be null: lim for every query), results as float bits in
// out[q][i] (stride `stride`).  With bounds, candidates whose value provably
// exceeds float32(bounds[q] as float) * factor get all ones (bounds[q] all
// ones: no bound).
// Sets per wave: two where both sets' register tiles fit comfortably.
template <int FMT, int KC>
constexpr int lp_sets_per_wave() {
  return 1;   // two sets per wave measured slower (occupancy falls to 2 waves per SIMD)
}

template <int FMT, int KC, int MAXQT, bool HASG>
__global__ void __launch_bounds__(64 * kLpWaves)
k_haus_lp(LowpDb db, LowpQ qs, uint32_t lds_rows, const uint32_t* __restrict__ ids,
          const uint32_t* __restrict__ count, uint32_t stride, uint32_t i0, uint32_t lim,
          const uint32_t* __restrict__ bounds, float factor, uint32_t* __restrict__ out,
          unsigned long long* __restrict__ stats) {
  constexpr int NS = lp_sets_per_wave<FMT, KC>();
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t q = blockIdx.y;
  const uint32_t i1 = count ? min(count[q], lim) : lim;
  const uint32_t b0 = i0 + blockIdx.x * kLpPerBlock;
  if (b0 >= i1) return;
  const uint32_t b1 = min(i1, b0 + kLpPerBlock);
  uint32_t thr = 0xFFFFFFFFu;
  if (bounds && bounds[q] != 0xFFFFFFFFu) thr = __float_as_uint(__uint_as_float(bounds[q]) * factor);
  const LpView qv = lp_stage(qs, q, lds_rows, smem);
  uint32_t rows = 0;
  static_assert(NS == 1, "one set per wave");
  // the id of the candidate after next and the offsets and scale of the next
  // one load while this one is computed (out-of-range ids read set 0, unused)
  const uint32_t w = wave_id();
  const cptr<uint32_t> idq = as_const(ids) + (uint64_t)q * stride;
  const cptr<uint64_t> offs = as_const(db.offsets);
  auto id_at = [&](uint32_t i) { return i < b1 ? idq[i] : 0u; };
  auto scale_of = [&](uint32_t j) { return db.scale ? db.scale[j] : 1.0f; };
  uint32_t jn = id_at(b0 + w);
  uint64_t c0 = offs[jn], c1 = offs[jn + 1];
  float cs = scale_of(jn);
  jn = id_at(b0 + w + kLpWaves);
  for (uint32_t it = b0 + w; it < b1; it += kLpWaves) {
    const uint64_t n0 = offs[jn], n1 = offs[jn + 1];
    const float ns = scale_of(jn);
    jn = id_at(it + 2 * kLpWaves);
    uint64_t o0[1] = {c0};
    uint32_t m[1] = {(uint32_t)(c1 - c0)}, res[1];
    float sv[1] = {cs};
    lp_items<FMT, KC, MAXQT, HASG, 1>(db, o0, m, sv, qv, res, thr, rows);
    if (lane_id() == 0) out[(uint64_t)q * stride + it] = res[0];
    c0 = n0;
    c1 = n1;
    cs = ns;
  }
  if (stats) stats_add(stats, 6, rows);
}

static constexpr size_t kLpStageBudget = 128 * 1024;

uint32_t lowp_lds_rows(uint32_t max_rows, uint32_t row_bytes) {
  uint32_t rows = std::min<uint32_t>((max_rows + 15) / 16 * 16, kMaxQueryTiles * 16);
  while (rows > 16 && (size_t)rows * (row_bytes + 16) + (size_t)rows * 4 > kLpStageBudget) rows -= 16;
  return rows;
}

template <int FMT, int KC, int MQ, bool HG>
constexpr bool lp_variant_used() {
  constexpr uint32_t rb = FMT == BVS_LOWP_FP8 ? KC * 128 : KC * 64;
  return !HG || (size_t)MQ * 16 * (rb + 16) + (size_t)MQ * 16 * 4 > kLpStageBudget;
}

template <int FMT, typename F>
static hipError_t dispatch_lp_kc(uint32_t kc, F&& f) {
  if constexpr (FMT == BVS_LOWP_BF16) {
    switch (kc) {
      case 2: return f(std::integral_constant<int, 2>());
      case 4: return f(std::integral_constant<int, 4>());
      case 8: return f(std::integral_constant<int, 8>());
      case 12: return f(std::integral_constant<int, 12>());
      case 16: return f(std::integral_constant<int, 16>());
      case 24: return f(std::integral_constant<int, 24>());
      case 32: return f(std::integral_constant<int, 32>());
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (kc) {
      case 1: return f(std::integral_constant<int, 1>());
      case 2: return f(std::integral_constant<int, 2>());
      case 3: return f(std::integral_constant<int, 3>());
      case 4: return f(std::integral_constant<int, 4>());
      case 6: return f(std::integral_constant<int, 6>());
      case 8: return f(std::integral_constant<int, 8>());
      default: return hipErrorInvalidValue;
    }
  }
}

template <int FMT>
static hipError_t launch_lp_fmt(const LowpDb& db, const LowpQ& q, const uint32_t* ids, const uint32_t* count,
                                uint32_t stride, uint32_t i0, uint32_t lim, const uint32_t* bounds, float factor,
                                uint32_t* out, unsigned long long* stats, hipStream_t st) {
  const uint32_t RB = db.row_bytes;
  const uint32_t kc = RB / (4 * LpOp<FMT>::LB);
  const uint32_t lds_rows = lowp_lds_rows(q.max_rows, RB);
  const size_t lds = (size_t)lds_rows * (RB + 16) + (size_t)lds_rows * 4;
  const uint32_t nqt = (q.max_rows + 15) / 16;
  const bool hasg = lds_rows < nqt * 16;
  const uint32_t G = (lim - i0 + kLpPerBlock - 1) / kLpPerBlock;
  return dispatch_lp_kc<FMT>(kc, [&](auto kct) -> hipError_t {
    constexpr int KC = decltype(kct)::value;
    auto go = [&](auto mqt, auto hgt) -> hipError_t {
      constexpr int MQ = decltype(mqt)::value;
      constexpr bool HG = decltype(hgt)::value;
      if constexpr (!lp_variant_used<FMT, KC, MQ, HG>()) {
        return hipErrorInvalidValue;
      } else {
        auto kern = k_haus_lp<FMT, KC, MQ, HG>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(G, q.n_q), dim3(64 * kLpWaves), lds, st, db, q, lds_rows, ids, count,
                           stride, i0, lim, bounds, factor, out, stats);
        return hipGetLastError();
      }
    };
    if (nqt <= 4) {
      if (hasg) return go(std::integral_constant<int, 4>(), std::true_type());
      return go(std::integral_constant<int, 4>(), std::false_type());
    }
    if (nqt <= 8) {
      if (hasg) return go(std::integral_constant<int, 8>(), std::true_type());
      return go(std::integral_constant<int, 8>(), std::false_type());
    }
    if (nqt > 16) return hipErrorInvalidValue;
    if (hasg) return go(std::integral_constant<int, 16>(), std::true_type());
    return go(std::integral_constant<int, 16>(), std::false_type());
  });
}

hipError_t launch_haus_lowp(int fmt, const LowpDb& db, const LowpQ& q, const uint32_t* ids, const uint32_t* count,
                            uint32_t stride, uint32_t i0, uint32_t lim, const uint32_t* bounds, float factor,
                            uint32_t* out, unsigned long long* stats, hipStream_t st) {
  if (q.n_q == 0 || lim <= i0) return hipSuccess;
  if (fmt == BVS_LOWP_BF16)
    return launch_lp_fmt<BVS_LOWP_BF16>(db, q, ids, count, stride, i0, lim, bounds, factor, out, stats, st);
  if (fmt == BVS_LOWP_FP8)
    return launch_lp_fmt<BVS_LOWP_FP8>(db, q, ids, count, stride, i0, lim, bounds, factor, out, stats, st);
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------------------
// One block per query: sort the candidates by (approximate value, id), take
// the k-th value, and keep the sorted prefix within the margin:
//   value <= kth * factor  (float32 multiply; factor = (1 + margin)^2).
// With fewer than k candidates every candidate is kept.
__device__ void lp_bitonic(uint64_t* k, uint32_t NP) {
  for (uint32_t size = 2; size <= NP; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < NP / 2; i += blockDim.x) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == asc) {
          k[lo] = b;
          k[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(1024)
k_lowp_select(const uint32_t* __restrict__ approx, const uint32_t* __restrict__ ids,
              const uint32_t* __restrict__ count, uint32_t T, uint32_t k, float factor,
              uint32_t* __restrict__ r_ids, uint32_t* __restrict__ r_count) {
  extern __shared__ uint64_t keys[];
  __shared__ uint32_t s_r;
  const uint32_t q = blockIdx.x;
  const uint32_t n = count[q];
  uint32_t NP = 2;
  while (NP < n) NP <<= 1;
  for (uint32_t i = threadIdx.x; i < NP; i += blockDim.x)
    keys[i] = i < n ? ((uint64_t)approx[(uint64_t)q * T + i] << 32) | ids[(uint64_t)q * T + i] : ~0ull;
  if (threadIdx.x == 0) s_r = n;
  __syncthreads();
  lp_bitonic(keys, NP);
  if (n >= k) {
    const float thr = __uint_as_float((uint32_t)(keys[k - 1] >> 32)) * factor;
    // the kept candidates are a prefix: find where the values pass thr
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const bool in = __uint_as_float((uint32_t)(keys[i] >> 32)) <= thr;
      const bool next_in = i + 1 < n && __uint_as_float((uint32_t)(keys[i + 1] >> 32)) <= thr;
      if (in && !next_in) s_r = i + 1;
    }
  }
  __syncthreads();
  const uint32_t r = s_r;
  for (uint32_t i = threadIdx.x; i < r; i += blockDim.x) r_ids[(uint64_t)q * T + i] = (uint32_t)keys[i];
  if (threadIdx.x == 0) r_count[q] = r;
}

hipError_t launch_lowp_select(const uint32_t* approx, const uint32_t* ids, const uint32_t* count, uint32_t T,
                              uint32_t n_q, uint32_t k, float factor, uint32_t* r_ids, uint32_t* r_count,
                              hipStream_t st) {
  if (n_q == 0) return hipSuccess;
  uint32_t NP = 2;
  while (NP < T) NP <<= 1;
  const size_t lds = (size_t)NP * sizeof(uint64_t);
  hipError_t e = hipFuncSetAttribute((const void*)k_lowp_select, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lowp_select, dim3(n_q), dim3(1024), lds, st, approx, ids, count, T, k, factor, r_ids, r_count);
  return hipGetLastError();
}

}  // namespace bvs
