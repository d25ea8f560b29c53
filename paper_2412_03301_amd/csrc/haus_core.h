// Exact Hausdorff distance (Def. 4) of one database set against a query, on
// the gfx950 int8 matrix cores; shared by the per-launch and the persistent
// re-rank kernels.
//
// Exactness.  On the 2^-12 grid a = 4096 x is an integer with |a| <= 4096; it
// is stored split as a = 64 hi + lo with hi in [-64, 64] and lo in [0, 63],
// both int8.  Then
//   a . b = 4096 (hi_a . hi_b) + 64 (hi_a . lo_b + lo_a . hi_b) + lo_a . lo_b
// is four int8 x int8 -> int32 matrix-core products, and
//   D2 = |a|^2 + |b|^2 - 2 a . b = 2^24 |x - y|^2
// is an exact integer below 2^28 when both norms are at most 2 (checked when
// the data are converted), so every comparison is exact and the ranking
// matches a float64 evaluation bit for bit.
//
// One wave computes one set.  For each 16-vector tile of the set it keeps the
// tile's planes for all of d in registers (the A operand: 16 rows x 64 k per
// lane group) and loops over the query's 16-row tiles (the B operand).  The
// first query tiles come from LDS, where the workgroup staged them; tiles
// beyond the staged rows are read from global memory, where a query read by
// every wave of the chip stays in L2.  The 16x16 int32 output has database
// vectors on rows and query vectors on columns:
//   column minimum over q (per database vector) -> DPP row-16 reduction;
//   row minimum over v (per query vector) -> carried per lane across tiles,
//   reduced over the four lane groups at the end of the set.
// Hausdorff^2 = max(max_v min_q D2, max_q min_v D2).
//
// Screening.  With a bound, candidates can first be compared on the high
// planes alone, half the bytes.  Write lo = 31.5 + e (e = 0 on the padding
// coordinates); the triangle inequality gives
//   |a - b| >= 64 |hi_a - hi_b| - |e_a| - |e_b|,
// and |hi_a - hi_b|^2 = |hi_a|^2 + |hi_b|^2 - 2 hi_a . hi_b is one int8
// product.  Each row carries |hi|^2 and r = |e| / 64 rounded up (written at
// conversion); a pair is provably farther than sqrt(bound) when
//   |hi_a - hi_b|^2 > (sqrt(bound) / 64 + r_a + r_b)^2,
// evaluated in float with the right-hand side rounded up (every rounding of
// sqrt(bound) / 64 + r_a + r_b is covered by a relative bump, so the float
// threshold is at least the real one whatever the bound).  If some vector
// of the set's first tile is that far from every query row, or (for sets of
// one tile) some query row from every vector of the set, the Hausdorff
// distance exceeds the bound and the set is rejected without its low planes
// ever being read; the survivors go through the exact pass.
#pragma once
#include "device.h"
#include "launch.h"

namespace bvs {

// Query tiles a wave keeps row minima for: queries of up to 256 vectors.
static constexpr int kMaxQueryTiles = 16;

// Result of a set abandoned against its bound.
static constexpr uint32_t kAbandoned = 0xFFFFFFFFu;

static constexpr uint32_t kCandPerBlock = kCandPerItem;

__host__ __device__ constexpr uint32_t q_row_stride(uint32_t dp) { return dp + 16; }

// Bytes of LDS that staging `rows` query rows takes (planes with a 16-byte
// row pad against bank conflicts, the norms and the screening pairs).
__host__ __device__ constexpr size_t haus_stage_bytes(uint32_t rows, uint32_t dp) {
  return (size_t)rows * q_row_stride(dp) * 2 + (size_t)rows * 12;
}

// LDS of the screening pass: the high plane (same row stride) and the
// screening pair of `rows` query rows.
__host__ __device__ constexpr size_t screen_stage_bytes(uint32_t rows, uint32_t dp) {
  return (size_t)rows * q_row_stride(dp) + (size_t)rows * 8;
}

// |hi|^2 given to rows past the end of a set or a query: far from
// everything, and the sums below stay within int32.
static constexpr uint32_t kScreenPad = 1u << 28;

// Where a wave reads the query: rows [0, 16 nqt_s) staged in LDS (row stride
// dp + 16, zero padded), the rest from global memory (row stride dp).
struct QView {
  const uint8_t* hs;
  const uint8_t* ls;
  const uint32_t* ns;
  const uint2* ss;     // screening pairs of the staged rows (pad rows: kScreenPad)
  const uint8_t* hg;
  const uint8_t* lg;
  const uint32_t* ng;
  const uint2* sg;     // null when the query has no screening pairs
  uint32_t mq, nqt, nqt_s;
};

template <int KS>
__device__ __forceinline__ void tile_products(const v4i (&ah)[KS], const v4i (&al)[KS], const uint8_t* bh,
                                              const uint8_t* bl, v4i& hh, v4i& hl, v4i& lh, v4i& ll) {
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const v4i b_h = *(const v4i*)(bh + 64 * k);
    const v4i b_l = *(const v4i*)(bl + 64 * k);
    hh = mfma_i8(ah[k], b_h, hh);
    hl = mfma_i8(ah[k], b_l, hl);
    lh = mfma_i8(al[k], b_h, lh);
    ll = mfma_i8(al[k], b_l, ll);
  }
}

// sqrt(bound) / 64 rounded up: the factor covers the int -> float
// conversion (2^-24 relative), a square root within one ulp (2^-23) and the
// two multiplications' roundings.
__device__ __forceinline__ float screen_scale(uint32_t bound) {
  return sqrtf((float)bound) * (1.0f / 64.0f) * (1.0f + 0x1p-19f);
}

// Factor applied to the rounded sum tb + r_q + r_v: each of the two
// round-to-nearest additions of non-negative terms loses at most 2^-24 of
// the sum, and so does the multiplication by the factor itself, so
// fl(fl(fl(tb + r_q) + r_v) * (1 + 2^-21)) >= (tb + r_q + r_v) (1 - 2^-24)^3
// (1 + 2^-21) > tb + r_q + r_v whatever the sizes of the three terms.
static constexpr float kScreenSumUp = 1.0f + 0x1p-21f;

// Screen of the first database tile (rows [0, min(16, m)) of a set, whose
// high planes are in ah and whose screening pairs are sv[r] for the tile's
// row 4 (lane / 16) + r, pad for rows past the set): whether the set
// provably has Hausdorff^2 > bound, with tb >= sqrt(bound) / 64.  The query
// view needs the high planes and screening pairs of its staged rows (query
// tiles past them are read from global memory when HASG).  Per pair,
// |hi_a - hi_b|^2 - X^2 with X >= tb + r_a + r_b, by one fused multiply-add
// whose sign is exact; pad rows and columns come out far.  A database
// vector far from every query vector decides (column minima); when the tile
// is the whole set, so does a query vector far from every vector of the
// tile (row minima), checked after each query tile.
template <int KS, int MAXQT, bool HASG>
__device__ __forceinline__ bool screen_first_tile(uint32_t m, const QView& q, const v4i (&ah)[KS],
                                                  const uint2 (&sv)[4], float tb) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t dp = KS * 64;
  const uint32_t QS = q_row_stride(dp);
  const bool whole = m <= 16;
  float colm[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) colm[r] = __builtin_inff();
#pragma unroll
  for (int qt = 0; qt < MAXQT; ++qt) {
    if ((uint32_t)qt < q.nqt) {
      v4i hh = {0, 0, 0, 0};
      const uint32_t qi = qt * 16 + c16;
      uint2 sq;
      if (!HASG || (uint32_t)qt < q.nqt_s) {
        const uint8_t* bh = q.hs + qi * QS + 16 * g;
#pragma unroll
        for (int k = 0; k < KS; ++k) hh = mfma_i8(ah[k], *(const v4i*)(bh + 64 * k), hh);
        sq = q.ss[qi];
      } else {
        asm volatile("" ::: "memory");
        const uint8_t* hg = uniform_ptr(q.hg);
        uint32_t cl = c16;
        asm volatile("" : "+s"(hg), "+v"(cl));
        const uint32_t r = min(qt * 16 + cl, q.mq - 1);
        const uint8_t* bh = hg + r * dp + 16 * g;
#pragma unroll
        for (int k = 0; k < KS; ++k) hh = mfma_i8(ah[k], *(const v4i*)(bh + 64 * k), hh);
        sq = qi < q.mq ? q.sg[r] : make_uint2(kScreenPad, 0u);
      }
      const float tq = tb + __uint_as_float(sq.y);
      float rowm = __builtin_inff();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h2 = (int)(sv[r].x + sq.x) - 2 * hh[r];
        const float x = (tq + __uint_as_float(sv[r].y)) * kScreenSumUp;
        const float mf = fmaf(-x, x, (float)h2);
        rowm = fminf(rowm, mf);
        colm[r] = fminf(colm[r], mf);
      }
      if (whole) {
        const float rm = rows4_min_f32(rowm);
        if (ballot(qi < q.mq && rm > 0.0f)) return true;
      }
    }
  }
  bool far = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float cm = row16_min_f32(colm[r]);
    far = far || (4 * g + r < m && cm > 0.0f);
  }
  return ballot(far) != 0;
}

// Load the first tile's high planes and screening pairs of set [o0, o0 + m)
// and screen it against bound (true: the set is provably farther).
template <int KS, int MAXQT, bool HASG>
__device__ __forceinline__ bool screen_set(const HausDb& db, uint64_t o0, uint32_t m, const QView& q,
                                           uint32_t bound) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t dp = KS * 64;
  const bool vrow_ok = c16 < m;
  v4i ah[KS];
  uint2 sv[4];
  {
    const v4i* ph = (const v4i*)(db.hi + (o0 + (vrow_ok ? c16 : 0)) * dp + 16 * g);
    const v4i z = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KS; ++k) ah[k] = vrow_ok ? __builtin_nontemporal_load(ph + 4 * k) : z;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t v = 4 * g + r;
      sv[r] = v < m ? db.scr[o0 + v] : make_uint2(kScreenPad, 0u);
    }
  }
  return screen_first_tile<KS, MAXQT, HASG>(m, q, ah, sv, screen_scale(bound));
}

// MeanMin key (Sec. 3.2, query to set) from the per-lane query-row minima
// of haus_item: lane (g, c) holds, for query row 16 qt + c, the minimum over
// the set rows that lane group g saw; the four groups' minima make the row's
// distance to the set, D2_q = 2^24 min_v |q - v|^2 (exact).  The mean of
// sqrt(D2_q) / 4096 over the m_q rows is accumulated in float64 (square roots
// correctly rounded, one sum per lane of group 0 in row order, then a fixed
// butterfly over the wave), divided by m_q and rounded once to float32; its
// bits are the key.
template <int MAXQT>
__device__ __forceinline__ uint32_t mean_min_key(const uint32_t (&qmin)[MAXQT], const QView& q) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  double sum = 0.0;
#pragma unroll
  for (int qt = 0; qt < MAXQT; ++qt) {
    if ((uint32_t)qt < q.nqt) {
      const uint32_t rm = rows4_min_u32(qmin[qt]);
      if (g == 0 && (uint32_t)qt * 16 + c16 < q.mq) sum += sqrt((double)rm);
    }
  }
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) sum += __shfl_xor(sum, m, BVS_WAVE);
  const double mean = sum * (1.0 / 4096.0) / (double)q.mq;
  return __float_as_uint((float)mean);
}

// Result key of a set from its per-lane query-row minima and the largest of
// its vectors' distances to the query (colmax, per lane): Hausdorff (max of
// the two directed terms), Min (smallest pair) or MeanMin, by db.metric.
template <int MAXQT>
__device__ __forceinline__ uint32_t set_key(const HausDb& db, const uint32_t (&qmin)[MAXQT], uint32_t colmax,
                                            const QView& q) {
  const uint32_t c16 = lane_id() & 15;
  if (db.metric == kMetricMin) {
    // every pair's value went into some lane's query-row minima (pad pairs
    // hold all ones)
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int qt = 0; qt < MAXQT; ++qt)
      if ((uint32_t)qt < q.nqt) mn = min(mn, qmin[qt]);
    return wave_min_dpp_u32(mn);
  }
  if (db.metric == kMetricMeanMin) return mean_min_key<MAXQT>(qmin, q);
  uint32_t rowmax = 0;
#pragma unroll
  for (int qt = 0; qt < MAXQT; ++qt) {
    if ((uint32_t)qt < q.nqt) {
      const uint32_t rm = rows4_min_u32(qmin[qt]);
      if ((uint32_t)qt * 16 + c16 < q.mq) rowmax = max(rowmax, rm);
    }
  }
  return wave_max_dpp_u32(max(colmax, rowmax));
}

// Squared Hausdorff distance (2^24-scaled) of database set [o0, o0 + m)
// against the query (HASG: some query tiles may come from global memory).
// The set is abandoned, returning kAbandoned, as soon as a lower bound of
// the result exceeds `bound` (such a set cannot be among the k nearest when
// `bound` is at least the k-th smallest distance): the largest completed
// column minimum (a database vector's distance to the query) after each
// database tile, and, on the last database tile, the largest row minimum of
// each query tile (those query vectors' distances to the whole set) as soon
// as the tile is done.
template <int KS, int MAXQT, bool HASG>
__device__ __forceinline__ uint32_t haus_item(const HausDb& db, uint64_t o0, uint32_t m, const QView& q,
                                              uint32_t bound = 0xFFFFFFFFu, uint32_t* rows_read = nullptr) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t dp = KS * 64;
  const uint32_t QS = q_row_stride(dp);
  const bool bounded = bound != 0xFFFFFFFFu;
  uint32_t qmin[MAXQT];
#pragma unroll
  for (int i = 0; i < MAXQT; ++i) qmin[i] = 0xFFFFFFFFu;
  uint32_t colmax = 0;
  for (uint32_t vt = 0; vt < m; vt += 16) {
    const bool last = vt + 16 >= m;
    if (rows_read) *rows_read += min(16u, m - vt);
    const uint32_t vrow = vt + c16;
    const bool vrow_ok = vrow < m;
    v4i ah[KS], al[KS];
    {
      const v4i* ph = (const v4i*)(db.hi + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
      const v4i* pl = (const v4i*)(db.lo + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const v4i z = {0, 0, 0, 0};
        ah[k] = vrow_ok ? __builtin_nontemporal_load(ph + 4 * k) : z;
        al[k] = vrow_ok ? __builtin_nontemporal_load(pl + 4 * k) : z;
      }
    }
    uint32_t nv[4], vmin[4];
    bool vok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t v = vt + 4 * g + r;
      vok[r] = v < m;
      nv[r] = vok[r] ? db.norms[o0 + v] : 0u;
      vmin[r] = 0xFFFFFFFFu;
    }
#pragma unroll
    for (int qt = 0; qt < MAXQT; ++qt) {
      if ((uint32_t)qt < q.nqt) {
        v4i hh = {0, 0, 0, 0}, hl = {0, 0, 0, 0}, lh = {0, 0, 0, 0}, ll = {0, 0, 0, 0};
        const uint32_t qi = qt * 16 + c16;
        uint32_t qn;
        if (!HASG || (uint32_t)qt < q.nqt_s) {
          tile_products<KS>(ah, al, q.hs + qi * QS + 16 * g, q.ls + qi * QS + 16 * g, hh, hl, lh, ll);
          qn = q.ns[qi];
        } else {
          // Global tiles one at a time, with addresses rebuilt per database
          // tile from a uniform base and a 32-bit lane offset: otherwise the
          // compiler hoists 16 tiles' addresses and loads into registers.
          // Rows past the query's end repeat its last row; they are masked
          // below.
          asm volatile("" ::: "memory");
          const uint8_t* hg = uniform_ptr(q.hg);
          const uint8_t* lg = uniform_ptr(q.lg);
          uint32_t cl = c16;
          asm volatile("" : "+s"(hg), "+s"(lg), "+v"(cl));
          const uint32_t r = min(qt * 16 + cl, q.mq - 1);
          const uint32_t off = r * dp + 16 * g;
          tile_products<KS>(ah, al, hg + off, lg + off, hh, hl, lh, ll);
          qn = q.ng[r];
        }
        const bool qok = qi < q.mq;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t dot = (uint32_t)hh[r] * 4096u + ((uint32_t)hl[r] + (uint32_t)lh[r]) * 64u + (uint32_t)ll[r];
          uint32_t d2 = nv[r] + qn - 2u * dot;
          d2 = (qok && vok[r]) ? d2 : 0xFFFFFFFFu;
          vmin[r] = min(vmin[r], d2);
          qmin[qt] = min(qmin[qt], d2);
        }
        if (bounded && last) {
          const uint32_t rm = qok ? rows4_min_u32(qmin[qt]) : 0u;
          if ((uint32_t)__builtin_amdgcn_readfirstlane((int)row16_max_u32(rm)) > bound) return kAbandoned;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t cm = row16_min_u32(vmin[r]);
      if (vok[r]) colmax = max(colmax, cm);
    }
    if (bounded && !last && (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_dpp_u32(colmax)) > bound)
      return kAbandoned;
  }
  return set_key<MAXQT>(db, qmin, colmax, q);
}

// The distances of database set [o0, o0 + m) to QT queries at once (no
// bound): each 16-vector tile of the set is loaded into registers once and
// multiplied against every staged query's tiles, so the set is read from
// memory once for the QT queries.  out[i] is the result key of query i under
// db.metric, as haus_item returns it.  Queries past the end repeat a staged
// view; the caller ignores their keys.
template <int KS, int MAXQT, bool HASG, int QT>
__device__ __forceinline__ void haus_multi(const HausDb& db, uint64_t o0, uint32_t m, const QView (&q)[QT],
                                           uint32_t (&out)[QT]) {
  const uint32_t lane = lane_id();
  const uint32_t g = lane >> 4, c16 = lane & 15;
  const uint32_t dp = KS * 64;
  const uint32_t QS = q_row_stride(dp);
  uint32_t qmin[QT][MAXQT];
  uint32_t colmax[QT];
#pragma unroll
  for (int i = 0; i < QT; ++i) {
    colmax[i] = 0;
#pragma unroll
    for (int t = 0; t < MAXQT; ++t) qmin[i][t] = 0xFFFFFFFFu;
  }
  for (uint32_t vt = 0; vt < m; vt += 16) {
    const uint32_t vrow = vt + c16;
    const bool vrow_ok = vrow < m;
    v4i ah[KS], al[KS];
    {
      const v4i* ph = (const v4i*)(db.hi + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
      const v4i* pl = (const v4i*)(db.lo + (o0 + (vrow_ok ? vrow : 0)) * dp + 16 * g);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const v4i z = {0, 0, 0, 0};
        ah[k] = vrow_ok ? __builtin_nontemporal_load(ph + 4 * k) : z;
        al[k] = vrow_ok ? __builtin_nontemporal_load(pl + 4 * k) : z;
      }
    }
    uint32_t nv[4];
    bool vok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t v = vt + 4 * g + r;
      vok[r] = v < m;
      nv[r] = vok[r] ? db.norms[o0 + v] : 0u;
    }
#pragma unroll
    for (int i = 0; i < QT; ++i) {
      uint32_t vmin[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll
      for (int qt = 0; qt < MAXQT; ++qt) {
        if ((uint32_t)qt < q[i].nqt) {
          v4i hh = {0, 0, 0, 0}, hl = {0, 0, 0, 0}, lh = {0, 0, 0, 0}, ll = {0, 0, 0, 0};
          const uint32_t qi = qt * 16 + c16;
          uint32_t qn;
          if (!HASG || (uint32_t)qt < q[i].nqt_s) {
            tile_products<KS>(ah, al, q[i].hs + qi * QS + 16 * g, q[i].ls + qi * QS + 16 * g, hh, hl, lh, ll);
            qn = q[i].ns[qi];
          } else {
            asm volatile("" ::: "memory");
            const uint8_t* hg = uniform_ptr(q[i].hg);
            const uint8_t* lg = uniform_ptr(q[i].lg);
            uint32_t cl = c16;
            asm volatile("" : "+s"(hg), "+s"(lg), "+v"(cl));
            const uint32_t r = min(qt * 16 + cl, q[i].mq - 1);
            const uint32_t off = r * dp + 16 * g;
            tile_products<KS>(ah, al, hg + off, lg + off, hh, hl, lh, ll);
            qn = q[i].ng[r];
          }
          const bool qok = qi < q[i].mq;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t dot =
                (uint32_t)hh[r] * 4096u + ((uint32_t)hl[r] + (uint32_t)lh[r]) * 64u + (uint32_t)ll[r];
            uint32_t d2 = nv[r] + qn - 2u * dot;
            d2 = (qok && vok[r]) ? d2 : 0xFFFFFFFFu;
            vmin[r] = min(vmin[r], d2);
            qmin[i][qt] = min(qmin[i][qt], d2);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t cm = row16_min_u32(vmin[r]);
        if (vok[r]) colmax[i] = max(colmax[i], cm);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QT; ++i) out[i] = set_key<MAXQT>(db, qmin[i], colmax[i], q[i]);
}

// Stage the first min(16 ceil(m_q / 16), lds_rows) rows of query q into LDS
// (rows past the query zero filled) and describe where the rest is read.
// lds_rows is a multiple of 16.  Ends with a workgroup barrier.
__device__ __forceinline__ QView stage_query(const HausQ& qs, uint32_t q, uint32_t dp, uint32_t lds_rows,
                                             uint8_t* smem) {
  QView v;
  const uint64_t o0 = qs.offsets[q];
  v.mq = (uint32_t)(qs.offsets[q + 1] - o0);
  v.nqt = (v.mq + 15) / 16;
  v.nqt_s = min(v.nqt, lds_rows / 16);
  const uint32_t rows = v.nqt_s * 16;
  const uint32_t QS = q_row_stride(dp);
  uint8_t* qh_s = smem;
  uint8_t* ql_s = smem + (size_t)lds_rows * QS;
  uint32_t* qn_s = (uint32_t*)(smem + (size_t)2 * lds_rows * QS);
  uint2* qs_s = (uint2*)(qn_s + lds_rows);
  {
    const uint8_t* const src[2] = {(const uint8_t*)qs.hi + o0 * dp, qs.lo + o0 * dp};
    uint8_t* const dst[2] = {qh_s, ql_s};
    stage_rows<2>(src, dst, dp, QS, dp / 16, rows, v.mq);
  }
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x) {
    qn_s[r] = r < v.mq ? qs.norms[o0 + r] : 0u;
    if (qs.scr) qs_s[r] = r < v.mq ? qs.scr[o0 + r] : make_uint2(kScreenPad, 0u);
  }
  v.hs = qh_s;
  v.ls = ql_s;
  v.ns = qn_s;
  v.ss = qs_s;
  v.hg = (const uint8_t*)qs.hi + o0 * dp;
  v.lg = qs.lo + o0 * dp;
  v.ng = qs.norms + o0;
  v.sg = qs.scr ? qs.scr + o0 : nullptr;
  __syncthreads();
  return v;
}

// Stage the high plane and the screening pairs of all 16 ceil(m_q / 16) rows
// of query q (rows past the query: zero plane, pad pair) for the screen, and
// describe them as a query view (no low planes or norms).  Ends with a
// workgroup barrier.
__device__ __forceinline__ QView stage_query_screen(const HausQ& qs, uint32_t q, uint32_t dp, uint8_t* smem) {
  QView v = {};
  const uint64_t o0 = qs.offsets[q];
  v.mq = (uint32_t)(qs.offsets[q + 1] - o0);
  v.nqt = (v.mq + 15) / 16;
  v.nqt_s = v.nqt;
  const uint32_t rows = v.nqt * 16;
  const uint32_t QS = q_row_stride(dp);
  uint8_t* qh = smem;
  uint2* qp = (uint2*)(smem + (size_t)rows * QS);
  {
    const uint8_t* const src[1] = {(const uint8_t*)qs.hi + o0 * dp};
    uint8_t* const dst[1] = {qh};
    stage_rows<1>(src, dst, dp, QS, dp / 16, rows, v.mq);
  }
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x)
    qp[r] = r < v.mq ? qs.scr[o0 + r] : make_uint2(kScreenPad, 0u);
  v.hs = qh;
  v.ss = qp;
  __syncthreads();
  return v;
}

// k-th smallest of vals[0 .. nv), nv <= 64, computed by one whole wave (every
// lane gets it), or all ones when nv < k.
__device__ __forceinline__ uint32_t wave_kth_smallest(uint32_t v_lane, uint32_t nv, uint32_t k) {
  const uint32_t lane = lane_id();
  const uint32_t v = lane < nv ? v_lane : 0xFFFFFFFFu;
  uint32_t rank = 0;
  for (uint32_t i = 0; i < nv; ++i) {
    const uint32_t o = (uint32_t)__shfl((int)v, (int)i, BVS_WAVE);
    rank += (o < v || (o == v && i < lane)) ? 1u : 0u;
  }
  const uint64_t hit = ballot(lane < nv && rank == k - 1);
  const uint32_t kth = (uint32_t)__shfl((int)v, hit ? (int)__builtin_ctzll(hit) : 0, BVS_WAVE);
  return (nv >= k && hit) ? kth : 0xFFFFFFFFu;
}

}  // namespace bvs
