// Second filter layer of the cascade search (Alg. 6) by bit-sliced counting.
//
// For a query Q with binary sketch S_Q and a set with binary sketch B, the
// Hamming distance is |S_Q| + |B| - 2 <S_Q, B>, and <S_Q, B> is the number
// of positions p set in S_Q whose bit is set in B.  With the position-major
// bitmaps (row p = bit p of every set), the inner products of one query
// with a tile of 256 sets are the column sums of the rows p in S_Q: a
// workgroup stages the tile's L rows in LDS (32 B each, one contiguous run of
// the tile-major bitmaps) and every lane adds
// its query's rows into vertical counters held as bit slices (Harley-Seal
// carry-save tree: three logic operations per input row and 32-bit word,
// for 32 sets at once).  The cutoff test |S_Q| + |B| - 2 <S_Q, B> <= cut is
// a bit-sliced add and compare against per-set constants staged with the
// tile; first-layer membership (M = 1) is the OR of the rows of the query's
// top-A count positions, read from the same tile.  Only the members that
// pass are unpacked and appended, as (score << 32 | id) keys, like the
// member-only kernel.
#include "device.h"
#include "launch.h"

namespace bvs {

static constexpr uint32_t kRowBytes = 32;     // one tile row: 256 sets, one bit each
static constexpr uint32_t kPairRanks = 32;    // ranks whose row lists are scheduled together
static constexpr uint32_t kSmallSteps = 31;   // passes of at most 31 x 16 rows use 9 counter slices
static constexpr int kVSlices = 12;           // 2048 - u with 0 <= u <= 2048

// ---------------------------------------------------------------- set weights
// |B| of every set (popcount of its binary Bloom filter, chunk-major layout);
// padding sets get 0.
__global__ void __launch_bounds__(256)
k_set_weight(const uint4* __restrict__ bits, uint32_t RC, uint64_t ld, uint16_t* __restrict__ w) {
  const uint64_t j = blockIdx.x * 256ull + threadIdx.x;
  if (j >= ld) return;
  uint32_t s = 0;
  for (uint32_t c = 0; c < RC; ++c) {
    const uint4 x = bits[(uint64_t)c * ld + j];
    s += popc32(x.x) + popc32(x.y) + popc32(x.z) + popc32(x.w);
  }
  w[j] = (uint16_t)s;
}

hipError_t launch_set_weight(const uint64_t* bits, uint32_t RC, uint64_t ld, uint16_t* w, hipStream_t st) {
  hipLaunchKernelGGL(k_set_weight, dim3((uint32_t)((ld + 255) / 256)), dim3(256), 0, st, (const uint4*)bits, RC, ld,
                     w);
  return hipGetLastError();
}

// ---------------------------------------------------------------- query rows
// |S_Q| of every query: one wave per query.
__global__ void __launch_bounds__(64)
k_query_bits(const uint64_t* __restrict__ sq, uint32_t R, uint32_t* __restrict__ qbits) {
  const uint32_t q = blockIdx.x, lane = lane_id();
  uint32_t c = 0;
  for (uint32_t t = lane; t < R; t += BVS_WAVE) c += popc64(sq[(uint64_t)q * R + t]);
  c = wave_sum_u32(c);
  if (lane == 0) qbits[q] = c;
}

// One workgroup: queries ordered by list length (in blocks of 16 rows),
// longest first, so that the queries sharing a wave do similar work.  The
// order within a length is unspecified (results do not depend on it).
// Also writes |S_Q| by rank, and clears the flag of long-sketch pairs.
__global__ void __launch_bounds__(1024)
k_order_queries(const uint32_t* __restrict__ qbits, uint32_t n_q, uint32_t nbins, uint32_t* __restrict__ order,
                uint32_t* __restrict__ sbits, uint32_t* __restrict__ any_long) {
  extern __shared__ uint32_t hist[];
  if (threadIdx.x == 0) *any_long = 0;
  for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < n_q; q += blockDim.x) {
    const uint32_t b = min((qbits[q] + 15) / 16, nbins - 1);
    atomicAdd(&hist[nbins - 1 - b], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t i = 0; i < nbins; ++i) {
      const uint32_t v = hist[i];
      hist[i] = run;
      run += v;
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < n_q; q += blockDim.x) {
    const uint32_t b = min((qbits[q] + 15) / 16, nbins - 1);
    const uint32_t r = atomicAdd(&hist[nbins - 1 - b], 1u);
    order[r] = q;
    sbits[r] = qbits[q];
  }
}

// Row lists of kPairRanks = 32 consecutive ranks (eight groups of four),
// one wave per group.  A 64- or 128-bit LDS read of the scoring kernels is
// served 128 bytes at a time (32 banks of 4 bytes), i.e. for the lanes of 4
// queries; their 32-byte rows p fall on banks that depend on p mod 4 only,
// so the read has no bank conflict when, at every step, the four queries
// read rows of four different classes p mod 4.  The steps of a group are an
// edge colouring of its (query, class) multigraph: the 4 x 4 count matrix is
// padded to equal row and column sums D (padding = zero rows L + c of class
// c) and decomposed into permutations (Birkhoff-von Neumann: each
// permutation is a run of steps in which query r reads class sigma(r)).  D
// is the largest |S_Q| or class total of the group, so the padding is small.
// Steps from D to 16 n + 48 (n: the pair's steps of 16 rows, the same for
// both halves) read zero rows of class (step + r) mod 4.  Lists are indexed
// by rank; part k (of 4) adds 8 k bytes to every row offset.  The tile-row
// offsets of each rank's top-A positions (its first layer) are written by
// rank to rpos.
__global__ void __launch_bounds__(512)
k_pass_lists(const uint64_t* __restrict__ sq, uint32_t R, uint32_t L, uint32_t n_q, const uint32_t* __restrict__ order,
             uint32_t LP, uint32_t* __restrict__ lists, uint32_t* __restrict__ gsteps, uint32_t* __restrict__ any_long,
             const uint32_t* __restrict__ pos, uint32_t A, uint32_t* __restrict__ rpos) {
  __shared__ uint64_t sk[kPairRanks][64];   // sketches of the 32 queries (R <= 64)
  __shared__ uint32_t cnt[8][4][4];         // [group][query][class]
  __shared__ uint32_t seg_len[8][16];
  __shared__ uint32_t seg_perm[8][16];      // sigma(r) in bits 2r .. 2r+1
  __shared__ uint32_t nseg[8], depth[8];
  const uint32_t pair = blockIdx.x, g = wave_id(), lane = lane_id();
  const uint32_t r0 = pair * kPairRanks;
  for (uint32_t i = threadIdx.x; i < kPairRanks * R; i += blockDim.x) {
    const uint32_t rr = i / R, t = i % R;
    sk[rr][t] = r0 + rr < n_q ? sq[(uint64_t)order[r0 + rr] * R + t] : 0ull;
  }
  for (uint32_t i = threadIdx.x; i < kPairRanks * A; i += blockDim.x) {
    const uint32_t rr = i / A, t = i % A;
    if (r0 + rr < n_q) rpos[(uint64_t)(r0 + rr) * A + t] = pos[(uint64_t)order[r0 + rr] * A + t] * kRowBytes;
  }
  __syncthreads();
  for (uint32_t r = 0; r < 4; ++r) {
    uint32_t cc[4] = {0, 0, 0, 0};
    for (uint32_t t = lane; t < R; t += BVS_WAVE) {
      const uint64_t w = sk[4 * g + r][t];
#pragma unroll
      for (int c = 0; c < 4; ++c) cc[c] += popc64(w & (0x1111111111111111ull << c));
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t v = wave_sum_u32(cc[c]);
      if (lane == 0) cnt[g][r][c] = v;
    }
  }
  uint32_t D = 0;
  {
    wave_lds_sync();   // the counts written above by lane 0
    uint32_t (&N)[4][4] = cnt[g];
    uint32_t rs[4] = {0, 0, 0, 0}, cs[4] = {0, 0, 0, 0};
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) { rs[r] += N[r][c]; cs[c] += N[r][c]; }
    for (int i = 0; i < 4; ++i) D = max(D, max(rs[i], cs[i]));
    wave_lds_sync();
    if (lane == 0) {
      // pad to row and column sums D (north-west corner)
      for (int r = 0, c = 0; r < 4 && c < 4;) {
        const uint32_t x = min(D - rs[r], D - cs[c]);
        N[r][c] += x; rs[r] += x; cs[c] += x;
        if (rs[r] == D) ++r; else ++c;
      }
    }
    wave_lds_sync();
  }
  {
    // peel permutations with all entries positive, largest minimum first
    // (the first in the order a, b, c ascending on ties); each peel empties
    // an entry, so 16 always suffice.  Lane i < 24 evaluates permutation i.
    uint32_t mine = 0;
    for (uint32_t a = 0, i = 0; a < 4; ++a)
      for (uint32_t b = 0; b < 4; ++b)
        for (uint32_t c = 0; c < 4; ++c) {
          if (a == b || a == c || b == c) continue;
          if (i++ == lane) mine = a | b << 2 | c << 4 | (6 - a - b - c) << 6;
        }
    uint32_t left = D, k = 0;
    while (left > 0 && k < 16) {
      uint32_t m = 0;
      if (lane < 24) {
        m = cnt[g][0][mine & 3];
#pragma unroll
        for (uint32_t r = 1; r < 4; ++r) m = min(m, cnt[g][r][(mine >> (2 * r)) & 3]);
      }
      const uint32_t top = wave_max_dpp_u32(lane < 24 ? m << 5 | (31u - lane) : 0u);   // D < 2^27
      const uint32_t best = top >> 5;
      if (best == 0) break;   // cannot happen for equal row and column sums
      const uint32_t bperm = (uint32_t)__shfl((int)mine, (int)(31u - (top & 31u)), BVS_WAVE);
      wave_lds_sync();
      if (lane < 4) cnt[g][lane][(bperm >> (2 * lane)) & 3] -= best;
      if (lane == 0) {
        seg_len[g][k] = best;
        seg_perm[g][k] = bperm;
      }
      wave_lds_sync();
      left -= best;
      ++k;
    }
    if (lane == 0) {
      nseg[g] = k;
      depth[g] = D - left;
    }
  }
  __syncthreads();
  uint32_t dmax = 0;
  for (int i = 0; i < 8; ++i) dmax = max(dmax, depth[i]);
  const uint32_t nblk = (dmax + 15) / 16;
  if (threadIdx.x < 2) gsteps[2 * pair + threadIdx.x] = nblk;
  if (threadIdx.x == 0 && nblk > kSmallSteps) atomicOr(any_long, 1u);
  // Each (rank, class) of the group is written by the whole wave: lane t
  // takes sketch word t, whose members of class c are the j0-th and on of
  // the class in row order (j0: the members in the words before t), and the
  // class's j-th member goes to the j-th step whose permutation gives rank r
  // class c.  The class's steps past its members read its zero row; steps
  // from the depth to the end read zero rows by step.  The segments are held
  // in registers (16 at most; lengths past nseg read as 0).
  const uint32_t ns = nseg[g], dep = depth[g];
  const uint32_t end = 16 * nblk + 48;   // the scoring kernels read below this
  uint32_t sl[16], sp[16];
#pragma unroll
  for (uint32_t i = 0; i < 16; ++i) {
    sl[i] = i < ns ? seg_len[g][i] : 0u;
    sp[i] = seg_perm[g][i];
  }
#pragma unroll 1
  for (uint32_t r = 0; r < 4; ++r) {
    const uint32_t rank = r0 + 4 * g + r;
    uint32_t* out = lists + (uint64_t)rank * 4 * LP;   // part k's list at out + k LP
    const uint64_t word = lane < R ? sk[4 * g + r][lane] : 0ull;
#pragma unroll 1
    for (uint32_t c = 0; c < 4; ++c) {
      uint64_t w = word & (0x1111111111111111ull << c);
      const uint32_t nc = popc64(w);   // the word's members of class c
      uint32_t inc = nc;
#pragma unroll
      for (int d = 1; d < BVS_WAVE; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)inc, d, BVS_WAVE);
        if (lane >= (uint32_t)d) inc += o;
      }
      const uint32_t total = (uint32_t)__shfl((int)inc, BVS_WAVE - 1, BVS_WAVE);
      const uint32_t zero_row = (L + c) * kRowBytes;
      uint32_t j = inc - nc;
      // segment i holds the class's steps cum .. cum + len - 1 at list steps
      // start .. start + len - 1
      uint32_t start = 0, cum = 0;
#pragma unroll
      for (uint32_t i = 0; i < 16; ++i) {
        const uint32_t len = sl[i];
        if (((sp[i] >> (2 * r)) & 3) == c) {
          const uint32_t shift = start - cum;   // list step - class step (start >= cum)
          for (; w && j < cum + len; ++j) {
            const uint32_t v = (lane * 64 + (uint32_t)__builtin_ctzll(w)) * kRowBytes;
            w &= w - 1;
#pragma unroll
            for (uint32_t p = 0; p < 4; ++p) out[p * LP + j + shift] = v + p * 8;
          }
          for (uint32_t jz = max(cum, total) + lane; jz < cum + len; jz += BVS_WAVE) {
#pragma unroll
            for (uint32_t p = 0; p < 4; ++p) out[p * LP + jz + shift] = zero_row + p * 8;
          }
          cum += len;
        }
        start += len;
      }
    }
    for (uint32_t s2 = dep + lane; s2 < end; s2 += BVS_WAVE) {
      const uint32_t zero_row = (L + ((s2 + r) & 3)) * kRowBytes;
#pragma unroll
      for (uint32_t p = 0; p < 4; ++p) out[p * LP + s2] = zero_row + p * 8;
    }
  }
}

hipError_t launch_query_rows(const FilterArgs& a, const uint64_t* sq, uint32_t R, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  if (R > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_query_bits, dim3(a.n_q), dim3(BVS_WAVE), 0, st, sq, R, a.qbits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t nbins = a.L / 16 + 1;
  hipLaunchKernelGGL(k_order_queries, dim3(1), dim3(1024), nbins * 4, st, (const uint32_t*)a.qbits, a.n_q, nbins,
                     a.order, a.sbits, a.any_long);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t pairs = (a.n_q + kPairRanks - 1) / kPairRanks;
  hipLaunchKernelGGL(k_pass_lists, dim3(pairs), dim3(512), 0, st, sq, R, a.L, a.n_q, (const uint32_t*)a.order, a.LP,
                     a.lists, a.gsteps, a.any_long, a.pos, a.A, a.rpos);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scoring
template <int W>
struct Words {
  uint32_t v[W];
};

#if defined(__HIP_DEVICE_COMPILE__)
#define BVS_LDS __attribute__((address_space(3)))
#else
#define BVS_LDS
#endif

// LDS address of a pointer into the workgroup's shared memory.
__device__ __forceinline__ uint32_t lds_address(const void* p) {
  return (uint32_t)(uintptr_t)(const BVS_LDS uint8_t*)p;
}

// W words at an absolute LDS byte address (the row offsets of the lists are
// addresses: the kernel's only shared memory is the dynamic tile, which
// starts at 0 -- checked at launch of every workgroup).
template <int W>
__device__ __forceinline__ Words<W> lds_words(uint32_t addr) {
  Words<W> r;
  if constexpr (W == 4) {
    const uint4 x = *(const BVS_LDS uint4*)(uintptr_t)addr;
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  } else {
    const uint2 x = *(const BVS_LDS uint2*)(uintptr_t)addr;
    r.v[0] = x.x; r.v[1] = x.y;
  }
  return r;
}

// Three-input bitwise functions (one v_bitop3_b32 each; the truth tables
// are symmetric in the inputs).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t xnor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x69);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Carry-save step: (h, l) <- (carry, sum) of l + a + b, per bit.
template <int W>
__device__ __forceinline__ void csa(Words<W>& h, Words<W>& l, const Words<W>& a, const Words<W>& b) {
#pragma unroll
  for (int i = 0; i < W; ++i) {
    h.v[i] = maj3(l.v[i], a.v[i], b.v[i]);
    l.v[i] = xor3(l.v[i], a.v[i], b.v[i]);
  }
}

// Counter state of one lane: dot = s[0] + 2 s[1] + 4 s[2] + 8 s[3] + 16 H,
// H = sum_i 2^i s[4 + i], all per bit (set); S slices hold dot < 2^S.
template <int W, int S>
struct Slices {
  Words<W> s[S];
};

// Words of 8 rows (LDS byte offsets in o0, o1).
template <int W>
__device__ __forceinline__ void load8(uint4 o0, uint4 o1, Words<W> (&x)[8]) {
  x[0] = lds_words<W>(o0.x); x[1] = lds_words<W>(o0.y); x[2] = lds_words<W>(o0.z); x[3] = lds_words<W>(o0.w);
  x[4] = lds_words<W>(o1.x); x[5] = lds_words<W>(o1.y); x[6] = lds_words<W>(o1.z); x[7] = lds_words<W>(o1.w);
}

// Add 8 rows to the ones, twos and fours counters; returns the eights
// carry word.
template <int W, int S>
__device__ __forceinline__ Words<W> tree8(const Words<W> (&x)[8], Slices<W, S>& c) {
  Words<W> twosA, twosB, foursA, foursB, eights;
  csa(twosA, c.s[0], x[0], x[1]);
  csa(twosB, c.s[0], x[2], x[3]);
  csa(foursA, c.s[1], twosA, twosB);
  csa(twosA, c.s[0], x[4], x[5]);
  csa(twosB, c.s[0], x[6], x[7]);
  csa(foursB, c.s[1], twosA, twosB);
  csa(eights, c.s[2], foursA, foursB);
  return eights;
}

// Ripple one word of weight 2^K0 into the slices K0 and up.  With 9
// slices every slice takes it.  With 13, the slices below 8 (weights up to
// 128) always do; the carry out of them is nonzero at most once per 256
// rows, and only then (a wave-uniform test) does it ripple on.
template <int K0, int W, int S>
__device__ __forceinline__ void add_carry(Words<W> x, Slices<W, S>& c) {
  constexpr int K1 = S <= 9 ? S : 8;
#pragma unroll
  for (int k = K0; k < K1; ++k)
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const uint32_t cy = c.s[k].v[i] & x.v[i];
      c.s[k].v[i] ^= x.v[i];
      x.v[i] = cy;
    }
  if constexpr (S > 9) {
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) any |= x.v[i];
    if (ballot(any != 0)) {
#pragma unroll
      for (int k = 8; k < S; ++k)
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const uint32_t cy = c.s[k].v[i] & x.v[i];
          c.s[k].v[i] ^= x.v[i];
          x.v[i] = cy;
        }
    }
  }
}

// Word 3 of a raw buffer resource for dword loads (32-bit data format).
static constexpr int kRawBufferWord3 = 0x00020000;

// Row offsets of one step of 16 rows: entries 16 step .. 16 step + 15 of the
// list part at byte offset voff of the resource.  (Loads through the buffer
// intrinsic stay where they are issued: the offsets of a later step arrive
// while this one counts.)
__device__ __forceinline__ void list_offsets(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t step,
                                             uint4 (&o)[4]) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16 * j, step * 64, 0);
    o[j] = make_uint4(x.x, x.y, x.z, x.w);
  }
}

// Add the 16 rows at LDS offsets o to the counters below weight 16;
// returns the word of weight 16.
template <int W, int S>
__device__ __forceinline__ Words<W> sixteen_rows(const uint4 (&o)[4], Slices<W, S>& c) {
  Words<W> x[8];
  load8<W>(o[0], o[1], x);
  const Words<W> eA = tree8<W, S>(x, c);
  load8<W>(o[2], o[3], x);
  const Words<W> eB = tree8<W, S>(x, c);
  Words<W> sixteens;
  csa(sixteens, c.s[3], eA, eB);
  return sixteens;
}

// One tile of 256 sets for the queries of part q_part (of q_parts) of the
// wave passes: stage the tile's rows, count, then append the members that
// pass the cutoff (SAMPLE false) or write every member's score to block
// out_block of the sample rows (SAMPLE true).  16 waves; lane = (query
// slot, part): the lane counts W words (32 W sets) of its query's tile row,
// in S counter slices.  Two instances share the work by rank pairs
// (kPairRanks ranks):
//   W = 4, S = 9    pairs of at most kSmallSteps steps (|S_Q| < 512): one
//                   wave pass takes a whole pair
//   W = 2, S = 13   the other pairs (long sketches), half a pair per pass
template <int W, int S, bool SAMPLE>
__device__ __forceinline__ void sliced_tile(const FilterArgs& a, uint32_t tile, uint32_t out_block, uint32_t q_part,
                                            uint32_t q_parts, uint8_t* smem) {
  constexpr bool kSmall = S == 9;
  constexpr uint32_t PARTS = 8 / W;           // lanes per query
  constexpr uint32_t QPW = BVS_WAVE / PARTS;  // queries per wave pass
  constexpr uint32_t NW = 16;
  constexpr int CB = kSmall ? 12 : 13;        // bits of dot + (2048 - u)
  const uint32_t L = a.L;
  auto big = [&](uint32_t pr) { return as_const(a.gsteps)[2 * pr] > kSmallSteps; };
  uint8_t* rows = smem;                                           // [L + 4][32 B]
  uint32_t* vsl = (uint32_t*)(smem + (size_t)(L + 4) * kRowBytes);  // [2][kVSlices][8]
  uint16_t* nset = (uint16_t*)(vsl + 2 * kVSlices * 8);           // [256]
  const uint64_t tile0 = (uint64_t)tile * 256;
  // the tile's rows go straight from memory into LDS, all in flight at once
  // (the wait for them comes before the barrier below)
  copy_to_lds((const uint4*)(a.planes + (uint64_t)tile * L * 4), rows, 2 * L);
  if (threadIdx.x < 8) ((uint4*)rows)[2 * L + threadIdx.x] = make_uint4(0, 0, 0, 0);   // zero rows L .. L+3
  const uint32_t w = wave_id(), lane = lane_id();
  if (threadIdx.x < 256) {
    // per-set constants: 2048 - ceil(|B| / 2) and 2048 - floor(|B| / 2)
    const uint64_t j = tile0 + threadIdx.x;
    const uint32_t nb = j < a.n_sets ? a.spop[j] : 0u;
    nset[threadIdx.x] = (uint16_t)nb;
    const uint32_t v0 = 2048u - (nb + 1) / 2, v1 = 2048u - nb / 2;
#pragma unroll
    for (int i = 0; i < kVSlices; ++i) {
      const uint64_t b0 = ballot((v0 >> i) & 1), b1 = ballot((v1 >> i) & 1);
      if (lane == 0) {
        vsl[(0 * kVSlices + i) * 8 + 2 * w] = (uint32_t)b0;
        vsl[(0 * kVSlices + i) * 8 + 2 * w + 1] = (uint32_t)(b0 >> 32);
        vsl[(1 * kVSlices + i) * 8 + 2 * w] = (uint32_t)b1;
        vsl[(1 * kVSlices + i) * 8 + 2 * w + 1] = (uint32_t)(b1 >> 32);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);   // the tile's rows have landed in LDS
  __syncthreads();

  const uint32_t part = lane % PARTS, slot = lane / PARTS;
  const uint32_t pbytes = part * W * 4;
  Words<W> valid;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const uint64_t b = tile0 + 32u * (part * W + i);
    valid.v[i] = b >= a.n_sets ? 0u : (a.n_sets - b >= 32 ? ~0u : (1u << (a.n_sets - b)) - 1u);
  }
  uint32_t pairs = 0;
  // Round r of this workgroup covers passes NW (q_part + q_parts r) .. + NW - 1
  // (ranks are by decreasing |S_Q|, so a round's passes shorten with r and
  // within it); wave w takes its w-th pass in even rounds and its
  // (NW - 1 - w)-th in odd ones, so that the waves' totals even out before
  // the tile's closing barrier.
  for (uint32_t r = 0;; ++r) {
    const uint32_t qb0 = (NW * (q_part + q_parts * r) + ((r & 1) ? NW - 1 - w : w)) * QPW;
    if (NW * (q_part + q_parts * r) * QPW >= a.n_q) break;
    if (qb0 >= a.n_q) continue;
    if (big(qb0 / kPairRanks) == kSmall) continue;   // the other instance's pass
    // the pass's per-rank values: unconditional loads at a clamped rank (no
    // branches around them), all in flight at once
    const uint32_t qi = qb0 + slot;
    const bool active = qi < a.n_q;
    const uint32_t qc = active ? qi : a.n_q - 1;
    const uint32_t q = a.order[qc];
    const uint32_t sbq = a.sbits[qc];
    const uint32_t ctq = SAMPLE ? 0u : a.rcut[qc];
    const uint32_t qbq = active ? sbq : 0u;
    const uint32_t cutq = active ? ctq : 0u;
    const uint32_t nblk = as_const(a.gsteps)[2 * (qb0 / kPairRanks)];
    // The pass's row lists (QPW ranks of 4 parts) are read through a buffer
    // resource based at the list of its first rank: a scalar base, the
    // lane's list part (of 4, 8 bytes each: the one that starts its words)
    // as a vector offset, the step as a scalar offset.
    const uint32_t* lbase = a.lists + (uint64_t)qb0 * 4 * a.LP;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)lbase, (short)0, (int)(QPW * 4 * a.LP * 4), kRawBufferWord3);
    const uint32_t voff = (slot * 4 + part * (4 / PARTS)) * a.LP * 4;
    Slices<W, S> c;
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
      for (int i = 0; i < W; ++i) c.s[k].v[i] = 0;
    // 16 rows per step, in two halves of 8; two steps per iteration, whose
    // words of weight 16 meet in one more carry-save step (weight 32 out).
    // The steps' row offsets are held in register sets X and Y; the offsets
    // of step b + 2 load into X when step b is done and arrive while step
    // b + 1 counts (the lists are written up to entry 16 nblk + 48 of every
    // part, past every read here).
    uint4 X[4], Y[4];
    list_offsets(rs, voff, 0, X);
    list_offsets(rs, voff, 1, Y);
    // first layer (C[p] >= 1 at one of the top-A positions): the OR of those
    // rows of the tile, their offsets loaded four at a time (a repeated last
    // offset ORs the same row again)
    Words<W> m;
    if (a.M == 0) {
      m = valid;
    } else {
#pragma unroll
      for (int i = 0; i < W; ++i) m.v[i] = 0;
      for (uint32_t t0 = 0; t0 < a.A; t0 += 4) {
        uint32_t o[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) o[j] = a.rpos[(uint64_t)qc * a.A + min(t0 + j, a.A - 1)];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
          const Words<W> r = lds_words<W>(o[j] + pbytes);
#pragma unroll
          for (int i = 0; i < W; ++i) m.v[i] |= r.v[i];
        }
      }
#pragma unroll
      for (int i = 0; i < W; ++i) m.v[i] &= valid.v[i];
    }
    if (!active) {
#pragma unroll
      for (int i = 0; i < W; ++i) m.v[i] = 0;
    }

    uint32_t b = 0;
    for (; b + 1 < nblk; b += 2) {
      const Words<W> sA = sixteen_rows<W, S>(X, c);
      list_offsets(rs, voff, b + 2, X);
      __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of step b + 1
      const Words<W> sB = sixteen_rows<W, S>(Y, c);
      list_offsets(rs, voff, b + 3, Y);
      __builtin_amdgcn_sched_barrier(0);
      Words<W> thirtytwos;
      csa(thirtytwos, c.s[4], sA, sB);
      add_carry<5, W, S>(thirtytwos, c);
    }
    if (b < nblk) add_carry<4, W, S>(sixteen_rows<W, S>(X, c), c);

#pragma unroll
    for (int i = 0; i < W; ++i) pairs += popc32(m.v[i]);
    if constexpr (SAMPLE) {
      // every member's score: |S_Q| + |B| - 2 dot
#pragma unroll
      for (int i = 0; i < W; ++i) {
        uint32_t pw = m.v[i];
        while (pw) {
          const uint32_t sb = (uint32_t)__builtin_ctz(pw);
          pw &= pw - 1;
          uint32_t dot = 0;
#pragma unroll
          for (int k = 0; k < S; ++k) dot |= ((c.s[k].v[i] >> sb) & 1u) << k;
          const uint32_t jt = 32u * (part * W + i) + sb;
          a.scores[(uint64_t)q * a.ld_out + (uint64_t)out_block * 256 + jt] = (uint16_t)(qbq + nset[jt] - 2 * dot);
        }
      }
      continue;
    }

    // score <= cut  <=>  dot + (2048 - u) >= 2048 + g, with g = ceil((|S_Q| - cut) / 2)
    // and u = ceil(|B| / 2) (|S_Q| - cut even) or floor(|B| / 2) (odd);
    // dot + (2048 - u) < 2^CB and 2048 + g <= 2048 + |S_Q| / 2 < 2^CB
    const int64_t cd = (int64_t)qbq - (int64_t)cutq;
    const uint32_t par = (uint32_t)(cd & 1);
    const int64_t K0 = 2048 + ((cd + 1) >> 1);
    const uint32_t K = K0 < 0 ? 0u : (uint32_t)K0;
    Words<W> cy, br;
#pragma unroll
    for (int i = 0; i < W; ++i) { cy.v[i] = 0; br.v[i] = 0; }
#pragma unroll
    for (int k = 0; k < CB; ++k) {
      Words<W> v;
      if (k < kVSlices) {
        v = lds_words<W>(lds_address(vsl) + ((par * kVSlices + k) * 8) * 4 + pbytes);
      } else {
#pragma unroll
        for (int i = 0; i < W; ++i) v.v[i] = 0;
      }
      const uint32_t kw = ((K >> k) & 1) ? ~0u : 0u;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        // bit k of dot + V (complemented), its carry, and the borrow of (dot + V) - K
        const uint32_t d = k < S ? c.s[k < S ? k : 0].v[i] : 0u;
        const uint32_t nwb = xnor3(d, v.v[i], cy.v[i]);
        cy.v[i] = maj3(d, v.v[i], cy.v[i]);
        br.v[i] = maj3(nwb, kw, br.v[i]);
      }
    }
    uint32_t np = 0;
    Words<W> pass;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      pass.v[i] = m.v[i] & ~br.v[i];
      np += popc32(pass.v[i]);
    }
    if (np) {
      uint32_t slotc = atomicAdd(&a.cand_count[q], np);
#pragma unroll
      for (int i = 0; i < W; ++i) {
        uint32_t pw = pass.v[i];
        while (pw) {
          const uint32_t sb = (uint32_t)__builtin_ctz(pw);
          pw &= pw - 1;
          uint32_t dot = 0;
#pragma unroll
          for (int k = 0; k < S; ++k) dot |= ((c.s[k].v[i] >> sb) & 1u) << k;
          const uint32_t jt = 32u * (part * W + i) + sb;
          const uint32_t score = qbq + nset[jt] - 2 * dot;
          if (slotc < a.cap) a.cand[(uint64_t)q * a.cap + slotc] = ((uint64_t)score << 32) | (uint32_t)(tile0 + jt);
          ++slotc;
        }
      }
    }
  }
  if (!SAMPLE && a.stats) {
    const uint32_t wp = wave_sum_u32(pairs);
    if (lane == 0 && wp) atomicAdd(&a.stats[(blockIdx.x % kStatSlots) * kStatCounters], (unsigned long long)wp);
  }
}

// Virtual blocks vb = blockIdx.x, blockIdx.x + gridDim.x, ... below n_vb.
// Append mode: vb is a tile, XCD-aware (workgroup b runs on XCD b % 8, and
// vb takes tile (vb % 8) * per_xcd + vb / 8, so that the workgroups of one
// XCD share the cache lines of neighbouring tiles).  Sample mode: vb =
// (sample block, query part).  The long-sketch instance runs one workgroup
// per compute unit and returns at once unless some pair needs it.
template <int W, int S, bool SAMPLE>
__global__ void __launch_bounds__(1024)
k_filter_sliced(FilterArgs a, uint32_t per_xcd, uint32_t n_tiles, uint32_t n_vb, uint32_t q_parts) {
  extern __shared__ __align__(16) uint8_t smem[];
  if (S != 9 && *(const volatile uint32_t*)a.any_long == 0) return;
  if (lds_address(smem) != 0) {
    // (no static LDS in this kernel: the tile starts at LDS address 0, so
    // the row offsets are addresses; otherwise let the dense path answer)
    if (threadIdx.x == 0) atomicOr(a.fail, 1u);
    return;
  }
  for (uint32_t vb = blockIdx.x; vb < n_vb; vb += gridDim.x) {
    uint32_t tile, out_block = 0, q_part = 0;
    if (SAMPLE) {
      out_block = vb / q_parts;
      q_part = vb % q_parts;
      tile = out_block * a.block_stride;
    } else {
      tile = (vb % 8) * per_xcd + vb / 8;
    }
    if (tile < n_tiles) sliced_tile<W, S, SAMPLE>(a, tile, out_block, q_part, SAMPLE ? q_parts : 1, smem);
    __syncthreads();
  }
}


// Lists hold four parts (8 bytes of a tile row each); the 4-word instance
// uses parts 0 and 2.
uint32_t sliced_parts() { return 4u; }

size_t sliced_lds_bytes(uint32_t L) { return (size_t)(L + 4) * kRowBytes + 2 * kVSlices * 32 + 512; }

template <bool SAMPLE>
static hipError_t go_sliced(const FilterArgs& a, uint32_t n_vb, uint32_t q_parts, hipStream_t st) {
  if (a.L > 4096 || a.L % 256 != 0 || a.ld % 256 != 0 || a.parts != 4) return hipErrorInvalidValue;
  const uint32_t n_tiles = (uint32_t)(a.ld / 256);
  const uint32_t per_xcd = (n_tiles + 7) / 8;
  const size_t lds = sliced_lds_bytes(a.L);
  auto go = [&](auto kern, uint32_t grid) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, a, per_xcd, n_tiles, n_vb, q_parts);
    return hipGetLastError();
  };
  hipError_t e = go(k_filter_sliced<4, 9, SAMPLE>, n_vb);
  if (e != hipSuccess) return e;
  return go(k_filter_sliced<2, 13, SAMPLE>, std::min(n_vb, 256u));
}

hipError_t launch_filter_sliced(const FilterArgs& a, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  const uint32_t n_tiles = (uint32_t)(a.ld / 256);
  return go_sliced<false>(a, (n_tiles + 7) / 8 * 8, 1, st);
}

hipError_t launch_filter_sliced_sample(FilterArgs a, uint32_t n_sample_blocks, hipStream_t st) {
  if (a.n_q == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)(a.ld / 256);
  a.block_stride = std::max(1u, nb / n_sample_blocks);
  a.ld_out = (uint64_t)n_sample_blocks * 256;
  // several workgroups per sample block, each a share of the wave passes
  const uint32_t passes = (a.n_q + 16 * kPairRanks - 1) / (16 * kPairRanks);
  const uint32_t q_parts = std::max(1u, std::min(passes, 4u));
  return go_sliced<true>(a, n_sample_blocks * q_parts, q_parts, st);
}

}  // namespace bvs
