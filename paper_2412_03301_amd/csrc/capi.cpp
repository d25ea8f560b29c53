// Host runtime of the library: parameter and data validation, the device
// memory plan of the index and of each call's workspace, and the launch
// sequences behind the C ABI declared in include/bvs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bvs.h"
#include "device.h"
#include "launch.h"

using namespace bvs;

namespace {

thread_local std::string g_err;

bvs_status fail(bvs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(BVS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define BVS_TRY(expr)            \
  do {                           \
    bvs_status s_ = (expr);      \
    if (s_ != BVS_OK) return s_; \
  } while (0)

// ------------------------------------------------------------------ geometry
struct Geometry {
  uint32_t d, dp, L, lgL, R, s, SP, wta_k, A, M, T;
};

const uint32_t kSupportedKs[] = {1, 2, 4, 6, 8, 12, 16};

uint32_t padded_dim(uint32_t d) {
  const uint32_t ks = (d + 63) / 64;
  for (uint32_t k : kSupportedKs)
    if (k >= ks) return 64 * k;
  return 0;
}

bvs_status derive(const bvs_params* p, Geometry* g) {
  if (!p) return fail(BVS_EINVAL, "params is NULL");
  if (p->flags != 0) return fail(BVS_EINVAL, "flags must be 0");
  if (p->dim < 1 || p->dim > 1024) return fail(BVS_ENOTSUP, "dim %u outside 1..1024", p->dim);
  const uint32_t L = p->code_bits;
  if (L < 256 || L > 4096 || (L & (L - 1)) != 0)
    return fail(BVS_ENOTSUP, "code_bits %u must be a power of two in 256..4096", L);
  if (p->fan_in < 1 || p->fan_in > p->dim) return fail(BVS_EINVAL, "fan_in %u outside 1..dim", p->fan_in);
  const uint32_t SP = (p->fan_in + 7) / 8 * 8;
  if ((uint64_t)L * SP > 65536) return fail(BVS_ENOTSUP, "code_bits * fan_in (rounded to 8) exceeds 65536");
  uint32_t lgL = 0;
  while ((1u << lgL) < L) ++lgL;
  // key = ((y + s*4096) << lgL) | (L-1-j) with y + s*4096 <= s*8192 must fit 32 bits
  if (((uint64_t)p->fan_in * 8192ull) >= (1ull << (32 - lgL)))
    return fail(BVS_ENOTSUP, "fan_in %u too large for code_bits %u (winner-take-all key exceeds 32 bits)",
                p->fan_in, L);
  if (p->wta_k < 1 || p->wta_k > L) return fail(BVS_EINVAL, "wta_k %u outside 1..code_bits", p->wta_k);
  if (p->access_lists < 1 || p->access_lists > 8) return fail(BVS_EINVAL, "access_lists %u outside 1..8", p->access_lists);
  if (p->min_count > 255) return fail(BVS_EINVAL, "min_count %u outside 0..255", p->min_count);
  if (p->top_t < 1 || p->top_t > 4096) return fail(BVS_ENOTSUP, "top_t %u outside 1..4096", p->top_t);
  g->d = p->dim;
  g->dp = padded_dim(p->dim);
  g->L = L;
  g->lgL = lgL;
  g->R = L / 64;
  g->s = p->fan_in;
  g->SP = SP;
  g->wta_k = p->wta_k;
  g->A = p->access_lists;
  g->M = p->min_count;
  g->T = p->top_t;
  return BVS_OK;
}

// Bump allocator over a caller-provided block (base = nullptr only measures).
struct Carver {
  uint8_t* base;
  uint64_t off = 0;
  explicit Carver(void* b) : base((uint8_t*)b) {}
  template <typename T>
  T* take(uint64_t count) {
    off = align_up(off, 256);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int device_cus(int dev) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  return n;
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014).
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

void make_projection(const Geometry& g, uint64_t seed, uint16_t* out /* [L][s] */) {
  SplitMix64 rng{seed};
  std::vector<uint32_t> row;
  for (uint32_t j = 0; j < g.L; ++j) {
    row.clear();
    while (row.size() < g.s) {
      const uint32_t i = (uint32_t)(((rng.next() >> 32) * (uint64_t)g.d) >> 32);
      if (std::find(row.begin(), row.end(), i) == row.end()) row.push_back(i);
    }
    std::sort(row.begin(), row.end());
    for (uint32_t i = 0; i < g.s; ++i) out[(uint64_t)j * g.s + i] = (uint16_t)row[i];
  }
}

// Order of the gathers in the device projection table.  The encode kernel's
// lane l sums output j = 64 t + l from its row, entry i at step i, all 64
// lanes at once; an output's sum does not depend on the order of its
// entries, so each group of 64 rows is reordered to spread every step's 64
// reads over the LDS banks: step by step, each row (rows with the fewest
// distinct banks left first) takes the entry whose 4-byte word is already
// read in this step or else whose bank is least loaded so far.  Entries are
// byte offsets into the staged vector (2 bytes per element, a wave-aligned
// slot), so entry e lies in word e / 4; banks are words mod 64.
void order_projection_gathers(const Geometry& g, uint16_t* tab /* [L][SP] */) {
  constexpr uint32_t kBanks = 64;
  const uint32_t SP = g.SP;
  std::vector<std::vector<uint16_t>> left(64);
  std::vector<uint32_t> lanes(64), load(kBanks);
  std::vector<uint16_t> step_words;
  for (uint32_t j0 = 0; j0 + 64 <= g.L; j0 += 64) {
    for (uint32_t l = 0; l < 64; ++l) left[l].assign(tab + (size_t)(j0 + l) * SP, tab + (size_t)(j0 + l + 1) * SP);
    for (uint32_t i = 0; i < SP; ++i) {
      std::fill(load.begin(), load.end(), 0u);
      step_words.clear();
      auto distinct_banks = [&](uint32_t l) {
        uint64_t m = 0;
        for (uint16_t e : left[l]) m |= 1ull << ((e / 4u) % kBanks);
        return __builtin_popcountll(m);
      };
      for (uint32_t l = 0; l < 64; ++l) lanes[l] = l;
      std::stable_sort(lanes.begin(), lanes.end(),
                       [&](uint32_t a, uint32_t b) { return distinct_banks(a) < distinct_banks(b); });
      for (uint32_t l : lanes) {
        size_t best = 0;
        uint32_t best_cost = ~0u;
        for (size_t k = 0; k < left[l].size(); ++k) {
          const uint16_t w = left[l][k] / 4u;
          const bool shared = std::find(step_words.begin(), step_words.end(), w) != step_words.end();
          const uint32_t cost = shared ? 0u : load[w % kBanks] + 1u;
          if (cost < best_cost) {
            best_cost = cost;
            best = k;
          }
        }
        const uint16_t e = left[l][best];
        left[l].erase(left[l].begin() + (ptrdiff_t)best);
        tab[(size_t)(j0 + l) * SP + i] = e;
        const uint16_t w = e / 4u;
        if (std::find(step_words.begin(), step_words.end(), w) == step_words.end()) {
          step_words.push_back(w);
          ++load[w % kBanks];
        }
      }
    }
  }
}

bvs_status check_offsets(const uint64_t* off, uint64_t n, uint32_t max_size, const char* what, uint32_t* max_m) {
  if (!off) return fail(BVS_EINVAL, "%s offsets are NULL", what);
  if (off[0] != 0) return fail(BVS_EINVAL, "%s offsets[0] must be 0", what);
  uint64_t mm = 0;
  for (uint64_t j = 0; j < n; ++j) {
    if (off[j + 1] <= off[j]) return fail(BVS_EINVAL, "%s set %llu is empty or offsets decrease", what, (unsigned long long)j);
    mm = std::max<uint64_t>(mm, off[j + 1] - off[j]);
  }
  if (mm > max_size)
    return fail(BVS_ERANGE, "%s set of %llu vectors exceeds the limit %u", what, (unsigned long long)mm, max_size);
  *max_m = (uint32_t)mm;
  return BVS_OK;
}

bvs_status read_status(uint32_t* d_status, hipStream_t st, const char* what) {
  uint32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, d_status, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h & ST_OFF_GRID)
    return fail(BVS_ERANGE, "%s: a value is not on the 2^-12 grid, |x| > 1 or not finite", what);
  if (h & ST_NORM) return fail(BVS_ERANGE, "%s: a vector has Euclidean norm above 2", what);
  return BVS_OK;
}

// ------------------------------------------------------------------ stage timing
const char* const kStageNames[BVS_N_STAGES] = {"convert",  "encode",   "query_sketch", "cutoff",
                                               "filter",   "select",   "rerank",       "topk",
                                               "bruteforce", "fallback", "approx",     "recheck",
                                               "fullscan", "lists"};

struct ProfTable {
  std::mutex mu;
  bool on = false;        // stage events
  bool counters_on = false;
  double ms[BVS_N_STAGES] = {};
  uint64_t calls[BVS_N_STAGES] = {};
  uint64_t counters[BVS_N_COUNTERS] = {};
  std::vector<hipEvent_t> pool;
};
ProfTable g_prof;

// Events recorded around the stages of one call, on the call's stream.
struct CallProf {
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipStream_t st;
  bool on;          // record stage events
  bool count;       // collect work counters
  explicit CallProf(hipStream_t s, bool allowed = true) : st(s) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    on = allowed && g_prof.on;
    count = allowed && g_prof.counters_on;
  }
  hipEvent_t take() {
    {
      std::lock_guard<std::mutex> g(g_prof.mu);
      if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(int stage) {
    if (!on) return;
    Rec r{stage, take(), take()};
    if (r.a) (void)hipEventRecord(r.a, st);
    recs.push_back(r);
  }
  void end() {
    if (on && !recs.empty() && recs.back().b) (void)hipEventRecord(recs.back().b, st);
  }
  void release() {
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (auto& r : recs) {
      if (r.a) g_prof.pool.push_back(r.a);
      if (r.b) g_prof.pool.push_back(r.b);
    }
    recs.clear();
  }
  // Call after the stream has been synchronised.  stats: device work
  // counters of this call (may be null).
  void finish(const unsigned long long* d_stats = nullptr) {
    static_assert(BVS_N_COUNTERS == kStatCounters, "counter layout");
    std::vector<unsigned long long> c((size_t)kStatSlots * kStatCounters);
    if (count && d_stats &&
        hipMemcpy(c.data(), d_stats, c.size() * sizeof(c[0]), hipMemcpyDeviceToHost) == hipSuccess) {
      std::lock_guard<std::mutex> g(g_prof.mu);
      for (uint32_t s = 0; s < kStatSlots; ++s)
        for (int i = 0; i < BVS_N_COUNTERS; ++i) g_prof.counters[i] += c[(size_t)s * kStatCounters + i];
    }
    if (!on) return;
    std::vector<std::pair<int, float>> t;
    for (auto& r : recs) {
      float ms = 0.f;
      if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) t.emplace_back(r.stage, ms);
    }
    {
      std::lock_guard<std::mutex> g(g_prof.mu);
      for (auto& x : t) {
        g_prof.ms[x.first] += x.second;
        g_prof.calls[x.first] += 1;
      }
    }
    release();
  }
  ~CallProf() { release(); }
};

// Test hook: with BVS_TEST_FAIL set to a stage name, launching that stage
// reports a launch failure without launching anything, so that the error
// path (BVS_EDEVICE, the index left valid for the next call) can be tested
// without a faulting kernel.
bool test_fail_at(int stage) {
  const char* e = std::getenv("BVS_TEST_FAIL");
  return e && *e && std::strcmp(e, kStageNames[stage]) == 0;
}

// One stage of a call: the stage's launches between its HIP events (when
// timing) and inside a roctx range named after the stage (seen by a
// profiler's marker trace).
template <class F>
hipError_t staged(CallProf& p, int stage, F&& f) {
  if (test_fail_at(stage)) return hipErrorLaunchFailure;
  p.begin(stage);
  roctxRangePushA(kStageNames[stage]);
  const hipError_t e = f();
  roctxRangePop();
  p.end();
  return e;
}

enum { S_CONVERT = 0, S_ENCODE, S_QSKETCH, S_CUTOFF, S_FILTER, S_SELECT, S_RERANK, S_TOPK, S_BRUTE, S_FALLBACK,
       S_APPROX, S_RECHECK, S_FULLSCAN, S_LISTS };

}  // namespace

struct bvs_index {
  bvs_params p;
  Geometry g;
  uint64_t n, N, ld;
  uint32_t max_m;
  int device, n_cu;
  uint16_t* idx;
  uint64_t* offsets;
  int8_t* hi;
  uint8_t* lo;
  uint32_t* norms;
  uint2* scr;         // [N] {|hi|^2, |lo - 31.5| / 64 rounded up} for re-rank screening
  uint8_t* cnt;
  uint64_t* bits;
  uint64_t* planes;   // [ld/256][L][4]: bit j % 256 of row p of tile j / 256 set when C^(j)[p] >= 1
  uint16_t* spop;     // [ld]: |B| of every set (0 for padding)
  // attached precision copies, by format (BVS_LOWP_BF16, BVS_LOWP_FP8)
  uint8_t* lowp[3] = {nullptr, nullptr, nullptr};
  float* lowp_scale[3] = {nullptr, nullptr, nullptr};
  // learned projection (codes from the network instead of W)
  bool learned = false;
  uint32_t hidden = 0;
  uint16_t* w16 = nullptr;   // packed bfloat16 [W1 | b1 | W2 | b2]
  float* b1 = nullptr;       // [hidden]
  float* b2 = nullptr;       // [L]
  // attached sparse codes for the full scan (Alg. 2)
  uint16_t* fpos = nullptr;  // [N][KP] code positions of every vector
  uint32_t* forder = nullptr;  // [n] set ids by decreasing size (ties: lower id first)
  uint32_t fKP = 0;
  // attached inverted lists (Def. 9, Alg. 4) and the first layer's source
  uint32_t* lcum = nullptr;    // [L][257]
  uint64_t* lstart = nullptr;  // [L + 1]
  uint32_t* lids = nullptr;    // [nnz]
  uint64_t lnnz = 0;
  int first_layer = BVS_FIRST_LAYER_BITMAPS;
};

namespace {

void layout_index(Carver& c, const Geometry& g, uint64_t n, uint64_t N, bvs_index* ix) {
  const uint64_t ld = align_up(std::max<uint64_t>(n, 1), 256);
  ix->idx = c.take<uint16_t>((uint64_t)g.L * g.SP);
  ix->offsets = c.take<uint64_t>(n + 1);
  ix->hi = c.take<int8_t>(N * g.dp);
  ix->lo = c.take<uint8_t>(N * g.dp);
  ix->norms = c.take<uint32_t>(N);
  ix->scr = c.take<uint2>(N);
  ix->cnt = c.take<uint8_t>((uint64_t)g.L * ld);
  ix->bits = c.take<uint64_t>((uint64_t)g.R * ld);
  ix->planes = c.take<uint64_t>((uint64_t)g.L * (ld / 64));
  ix->spop = c.take<uint16_t>(ld);
  ix->ld = ld;
}

HashGeom hash_geom(const bvs_index* ix) {
  HashGeom h;
  h.dim = ix->g.d;
  h.dim_padded = ix->g.dp;
  h.L = ix->g.L;
  h.lgL = ix->g.lgL;
  h.R = ix->g.R;
  h.s = ix->g.s;
  h.SP = ix->g.SP;
  h.wta_k = ix->g.wta_k;
  h.idx = ix->idx;
  return h;
}

// Per-call query state carved from a workspace.
struct QueryWs {
  uint32_t* status;
  uint64_t* qoff;
  int8_t* qhi;
  uint8_t* qlo;
  uint32_t* qnorm;
  uint2* qscr;
  // search only
  uint64_t* codes;
  uint16_t* cq;
  uint64_t* sq;
  uint32_t* pos;
  uint64_t* gate;
  uint64_t* gate_chunks;
  uint16_t* scores;
  SelectBufs sel;
  uint16_t* sample;       // [n_q][kSampleBlocks * 256]
  uint32_t* cutoff;       // [n_q]
  uint32_t* cand_count;   // [n_q]
  uint64_t* cand_app;     // [n_q][cap]
  uint32_t cap;
  uint32_t* lists;        // [n_q rounded up to 32][4][L + 48] row lists by rank
  uint32_t* qbits;        // [n_q]
  uint32_t* order;        // [n_q]
  uint32_t* sbits;        // [n_q]
  uint32_t* gsteps;       // [n_q rounded up to 32, / 16]
  uint32_t* rpos;         // [n_q rounded up to 32][A] first-layer tile-row offsets by rank
  uint32_t* rcut;         // [n_q rounded up to 32] cutoff by rank
  uint32_t* any_long;     // [1]
  uint64_t* member;       // [n_q][ld / 64] first layer from the inverted lists (lists mode only)
  uint32_t* f2_ids;
  uint16_t* f2_scores;
  uint32_t* f2_count;
  uint32_t* h2;
  uint32_t* thr;          // [n_q] re-rank bound
  uint32_t* surv;         // [n_q][T] candidates that passed the re-rank screen
  uint32_t* surv_count;   // [n_q]
  uint32_t* qids;         // brute force: the queries grouped by size (haus_all_list_words)
  unsigned long long* stats;   // [kStatSlots][kStatCounters] work counters
  uint64_t* topk_tmp;
  // learned projection: query rows in bfloat16, hidden layer, outputs
  uint16_t* lx16;
  uint16_t* lh16;
  float* ly;
};

constexpr uint32_t kMaxK = 64;
constexpr uint32_t kSampleBlocks = 64;   // blocks of 256 sets scored to pick the cutoff
constexpr uint32_t kCutoffAlpha = 3;     // the cutoff aims at about 3 T appended sets
constexpr uint32_t kMinSampleRank = 24;  // ... from at least this many sampled members

// Capacity of the append buffer per query: 8 T rounded up to a power of two,
// within 4096..16384 (it is sorted in LDS).  BVS_APPEND_CAP overrides it
// (tests use a tiny value to exercise the dense fallback).
uint32_t append_capacity(uint32_t T) {
  uint32_t c = 4096;
  while (c < 8 * T && c < 16384) c <<= 1;
  if (const char* e = std::getenv("BVS_APPEND_CAP")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= 16384) c = (uint32_t)v;
  }
  return c;
}

// Member-only scoring unless BVS_FILTER=dense, or M = 0 (every set is a
// member, so the dense kernel does the same work with fewer steps).
bool use_sparse_filter(uint32_t M) {
  const char* e = std::getenv("BVS_FILTER");
  if (e && std::strcmp(e, "dense") == 0) return false;
  if (e && std::strcmp(e, "sparse") == 0) return true;
  return M >= 1;
}

// Bit-sliced scoring for the first layer M = 1 (the usual setting) when the
// sketch fits a tile (L a multiple of 256, at most 4096), unless
// BVS_FILTER=sparse or dense asks for another kernel.
bool use_sliced_filter(const Geometry& g) {
  const char* e = std::getenv("BVS_FILTER");
  if (e && (std::strcmp(e, "dense") == 0 || std::strcmp(e, "sparse") == 0)) return false;
  return g.M == 1 && g.L % 256 == 0 && g.L <= 4096;
}

// High-plane screening of bounded re-ranks unless BVS_SCREEN=0 (the
// results are the same either way; the switch serves comparisons).
bool screen_enabled() {
  const char* e = std::getenv("BVS_SCREEN");
  return !(e && std::strcmp(e, "0") == 0);
}

bool force_dense_select() {
  const char* e = std::getenv("BVS_SELECT");
  return e && std::strcmp(e, "dense") == 0;
}

// The first layer comes from the attached inverted lists (M >= 1 only: with
// M = 0 every set is a member).
bool lists_first_layer(const bvs_index* ix) {
  return ix->first_layer == BVS_FIRST_LAYER_LISTS && ix->lids && ix->g.M >= 1;
}

void layout_search(Carver& c, const bvs_index* ix, uint32_t n_q, uint64_t NQ, QueryWs* w) {
  const Geometry& g = ix->g;
  w->status = c.take<uint32_t>(4);
  w->qoff = c.take<uint64_t>(n_q + 1);
  w->qhi = c.take<int8_t>(NQ * g.dp);
  w->qlo = c.take<uint8_t>(NQ * g.dp);
  w->qnorm = c.take<uint32_t>(NQ);
  w->qscr = c.take<uint2>(NQ);
  w->codes = c.take<uint64_t>(NQ * g.R);
  w->cq = c.take<uint16_t>((uint64_t)n_q * g.L);
  w->sq = c.take<uint64_t>((uint64_t)n_q * g.R);
  w->pos = c.take<uint32_t>((uint64_t)n_q * g.A);
  w->gate = c.take<uint64_t>((uint64_t)n_q * g.R);
  w->gate_chunks = c.take<uint64_t>(n_q);
  w->scores = c.take<uint16_t>((uint64_t)n_q * ix->ld);
  w->sel.hist = c.take<uint32_t>((uint64_t)n_q * (g.L + 2));
  w->sel.sel = c.take<uint32_t>((uint64_t)n_q * 4);
  w->sel.ctr = c.take<uint32_t>(n_q);
  w->sel.eqcnt = c.take<uint32_t>((uint64_t)n_q * select_blocks(ix->ld));
  w->sel.cand = c.take<uint64_t>((uint64_t)n_q * g.T);
  w->cap = append_capacity(g.T);
  w->sample = c.take<uint16_t>((uint64_t)n_q * kSampleBlocks * 256);
  w->cutoff = c.take<uint32_t>(n_q);
  w->cand_count = c.take<uint32_t>(n_q);
  w->cand_app = c.take<uint64_t>((uint64_t)n_q * w->cap);
  w->lists = c.take<uint32_t>(align_up(n_q, 32) * sliced_parts() * (g.L + 48));
  w->qbits = c.take<uint32_t>(n_q);
  w->order = c.take<uint32_t>(n_q);
  w->sbits = c.take<uint32_t>(n_q);
  w->gsteps = c.take<uint32_t>(align_up(n_q, 32) / 16);
  w->rpos = c.take<uint32_t>(align_up(n_q, 32) * g.A);
  w->rcut = c.take<uint32_t>(align_up(n_q, 32));
  w->any_long = c.take<uint32_t>(1);
  w->member = lists_first_layer(ix) ? c.take<uint64_t>((uint64_t)n_q * (ix->ld / 64)) : nullptr;
  w->f2_ids = c.take<uint32_t>((uint64_t)n_q * g.T);
  w->f2_scores = c.take<uint16_t>((uint64_t)n_q * g.T);
  w->f2_count = c.take<uint32_t>(n_q);
  w->h2 = c.take<uint32_t>((uint64_t)n_q * g.T);
  w->thr = c.take<uint32_t>(n_q);
  w->surv = c.take<uint32_t>((uint64_t)n_q * g.T);
  w->surv_count = c.take<uint32_t>(n_q);
  w->stats = c.take<unsigned long long>((uint64_t)kStatSlots * kStatCounters);
  w->topk_tmp = c.take<uint64_t>(topk_tmp_words(g.T, n_q, kMaxK));
  w->lx16 = nullptr;
  w->lh16 = nullptr;
  w->ly = nullptr;
  if (ix->learned) {
    w->lx16 = c.take<uint16_t>(NQ * g.d);
    w->lh16 = c.take<uint16_t>(NQ * ix->hidden);
    w->ly = c.take<float>(NQ * g.L);
  }
}

Mlp index_mlp(const bvs_index* ix) {
  Mlp m;
  m.d = ix->g.d;
  m.H = ix->hidden;
  m.L = ix->g.L;
  m.wta_k = ix->g.wta_k;
  m.W1 = ix->w16;
  m.b1 = ix->b1;
  m.W2 = ix->w16 + (uint64_t)ix->hidden * ix->g.d + ix->hidden;
  m.b2 = ix->b2;
  return m;
}

// Codes of n converted rows (exact planes) through the index's projection.
hipError_t encode_planes(const bvs_index* ix, const int8_t* hi, const uint8_t* lo, uint64_t n, uint64_t* codes,
                         uint16_t* x16, uint16_t* h16, float* y, hipStream_t st) {
  if (!ix->learned) return launch_encode_vectors(hash_geom(ix), hi, lo, n, codes, ix->n_cu, st);
  hipError_t e = launch_planes_to_bf16(hi, lo, ix->g.dp, ix->g.d, n, x16, st);
  if (e != hipSuccess) return e;
  return encode_learned(index_mlp(ix), x16, n, h16, y, codes, st);
}

void layout_brute(Carver& c, const bvs_index* ix, uint32_t n_q, uint64_t NQ, QueryWs* w) {
  const Geometry& g = ix->g;
  std::memset(w, 0, sizeof *w);
  w->status = c.take<uint32_t>(4);
  w->qoff = c.take<uint64_t>(n_q + 1);
  w->qhi = c.take<int8_t>(NQ * g.dp);
  w->qlo = c.take<uint8_t>(NQ * g.dp);
  w->qnorm = c.take<uint32_t>(NQ);
  w->h2 = c.take<uint32_t>((uint64_t)n_q * ix->n);
  w->topk_tmp = c.take<uint64_t>(topk_tmp_words(ix->n, n_q, kMaxK));
  w->qids = c.take<uint32_t>(haus_all_list_words(n_q));
}

bvs_status check_queries(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                         uint32_t* max_rows) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (n_q == 0) return fail(BVS_EINVAL, "n_q must be positive");
  if (!d_q) return fail(BVS_EINVAL, "query vectors are NULL");
  BVS_TRY(check_offsets(h_q_off, n_q, 65535, "query", max_rows));
  const uint32_t lim = haus_max_rows_supported(ix->g.dp);
  if (*max_rows > lim)
    return fail(BVS_ENOTSUP, "query set of %u vectors exceeds the %u supported at dim %u", *max_rows, lim, ix->g.d);
  return BVS_OK;
}

// Upload offsets and convert the query vectors (status cleared first).
bvs_status prepare_queries(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                           const QueryWs& w, hipStream_t st, CallProf& prof) {
  const uint64_t NQ = h_q_off[n_q];
  HIP_TRY(launch_fill_u32(w.status, 4, 0, st));
  HIP_TRY(hipMemcpyAsync(w.qoff, h_q_off, (n_q + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(staged(prof, S_CONVERT, [&] {
    return launch_convert(d_q, NQ, ix->g.d, ix->g.dp, w.qhi, w.qlo, w.qnorm, w.qscr, w.status, ix->n_cu, st);
  }));
  return BVS_OK;
}

bvs_status query_side(const bvs_index* ix, uint32_t n_q, uint64_t NQ, const QueryWs& w, hipStream_t st,
                      CallProf& prof) {
  const Geometry& g = ix->g;
  const HashGeom hg = hash_geom(ix);
  (void)hg;
  HIP_TRY(staged(prof, S_ENCODE, [&] { return encode_planes(ix, w.qhi, w.qlo, NQ, w.codes, w.lx16, w.lh16, w.ly, st); }));
  HIP_TRY(staged(prof, S_QSKETCH, [&] {
    return launch_query_sketch(w.codes, w.qoff, n_q, g.L, g.R, g.A, w.cq, w.sq, w.pos, w.gate, w.gate_chunks, st);
  }));
  return BVS_OK;
}

FilterArgs filter_args(const bvs_index* ix, uint32_t n_q, const QueryWs& w) {
  const Geometry& g = ix->g;
  FilterArgs a;
  std::memset(&a, 0, sizeof a);
  a.bits = (const uint4*)ix->bits;
  a.cnt = ix->cnt;
  a.ld = ix->ld;
  a.n_sets = ix->n;
  a.RC = g.L / 128;
  a.sq = (const uint4*)w.sq;
  a.gate = (const uint4*)w.gate;
  a.gate_chunks = w.gate_chunks;
  a.pos = w.pos;
  a.A = g.A;
  a.M = g.M;
  a.n_q = n_q;
  a.scores = w.scores;
  a.cutoff = w.cutoff;
  a.cand = w.cand_app;
  a.cap = w.cap;
  a.cand_count = w.cand_count;
  a.planes = ix->planes;
  a.L = g.L;
  a.spop = ix->spop;
  a.parts = sliced_parts();
  a.LP = g.L + 48;
  a.lists = w.lists;
  a.qbits = w.qbits;
  a.order = w.order;
  a.sbits = w.sbits;
  a.gsteps = w.gsteps;
  a.rpos = w.rpos;
  a.rcut = w.rcut;
  a.any_long = w.any_long;
  a.fail = w.status + 1;   // raised when the dense path must answer
  a.stats = nullptr;   // set by the caller when profiling
  a.member = w.member;
  return a;
}

// Both filter layers: F2 of every query into f2_ids / f2_scores / f2_count.
// host_sync: the dense fallback is chosen on the host after reading the
// failure count; otherwise it is always enqueued and does nothing unless the
// count on the device is nonzero (no host round trip, graph-safe).
bvs_status run_filters(const bvs_index* ix, uint32_t n_q, uint64_t NQ, const QueryWs& w, uint32_t* f2_ids,
                       uint16_t* f2_scores, uint32_t* f2_count, hipStream_t st, CallProf& prof,
                       bool host_sync = true) {
  const Geometry& g = ix->g;
  BVS_TRY(query_side(ix, n_q, NQ, w, st, prof));
  FilterArgs a = filter_args(ix, n_q, w);
  if (prof.count) {
    HIP_TRY(launch_fill_u32((uint32_t*)w.stats, 2ull * kStatSlots * kStatCounters, 0, st));
    a.stats = w.stats;
  }
  if (w.member) {
    // first layer from the inverted lists: membership bitmaps before scoring
    HIP_TRY(staged(prof, S_LISTS, [&] {
      return launch_list_gather(ix->lids, ix->lstart, ix->lcum, w.pos, g.A, g.M, n_q, ix->ld, w.member, ix->n_cu, st);
    }));
  }
  if (!force_dense_select()) {
    const uint32_t n_blocks = (uint32_t)(ix->ld / 256);
    const bool sparse = w.member || use_sparse_filter(g.M);
    const bool sliced = !w.member && use_sliced_filter(g);
    uint32_t* d_fail = w.status + 1;
    HIP_TRY(launch_fill_u32(w.cand_count, n_q, 0, st));
    HIP_TRY(launch_fill_u32(d_fail, 1, 0, st));
    HIP_TRY(staged(prof, S_CUTOFF, [&]() -> hipError_t {
      hipError_t e;
      if (sliced) {
        e = launch_query_rows(a, w.sq, g.R, st);
        if (e != hipSuccess) return e;
      }
      if (ix->n <= w.cap) {
        // every member fits the buffer: admit them all
        e = launch_fill_u32(w.rcut, n_q, 0xFFFFFFFFu, st);
        if (e != hipSuccess) return e;
        return launch_fill_u32(w.cutoff, n_q, 0xFFFFFFFFu, st);
      }
      const uint32_t nsb = std::min(kSampleBlocks, n_blocks);
      FilterArgs as = a;
      as.scores = w.sample;
      if (sparse) {
        e = launch_fill_u32((uint32_t*)w.sample, (uint64_t)n_q * nsb * 128, 0xFFFFFFFFu, st);
        if (e != hipSuccess) return e;
        as.stats = nullptr;
        e = sliced ? launch_filter_sliced_sample(as, nsb, st) : launch_filter_sparse_sample(as, nsb, st);
      } else {
        e = launch_filter_sample(as, nsb, st);
      }
      if (e != hipSuccess) return e;
      const uint64_t S = (uint64_t)nsb * 256;
      const uint64_t sampled = std::min<uint64_t>(S, ix->n);
      // the cutoff is the r-th smallest sampled score: r aims at about 3T
      // appended sets, but at least kMinSampleRank sampled members (a rank of a
      // few samples is too noisy to hold T sets reliably, and a miss costs the
      // dense path), as long as the sets it admits fit half the buffer
      const uint64_t r_aim = (kCutoffAlpha * (uint64_t)g.T * sampled + ix->n - 1) / ix->n;
      const uint64_t r_fit = std::max<uint64_t>(1, (uint64_t)w.cap * sampled / (2 * ix->n));
      const uint32_t r = (uint32_t)std::max<uint64_t>(1, std::max(r_aim, std::min<uint64_t>(kMinSampleRank, r_fit)));
      return launch_cutoff(w.sample, (uint32_t)S, g.L, r, n_q, w.cutoff, sliced ? w.order : nullptr,
                           sliced ? w.rcut : nullptr, st);
    }));
    HIP_TRY(staged(prof, S_FILTER, [&]() -> hipError_t {
      if (sliced) return launch_filter_sliced(a, st);
      return sparse ? launch_filter_sparse_append(a, st) : launch_filter_append(a, st);
    }));
    HIP_TRY(staged(prof, S_SELECT, [&] {
      return launch_sort_append(w.cand_app, w.cand_count, w.cutoff, w.cap, g.T, g.L, n_q, f2_ids, f2_scores, f2_count,
                                d_fail, st);
    }));
    if (!host_sync) {
      FilterArgs ag = a;
      ag.run_if = d_fail;
      HIP_TRY(staged(prof, S_FALLBACK, [&]() -> hipError_t {
        hipError_t e = launch_filter_dense(ag, st);
        if (e != hipSuccess) return e;
        return launch_select(w.scores, ix->ld, g.L, g.T, n_q, w.sel, f2_ids, f2_scores, f2_count, d_fail, st);
      }));
      return BVS_OK;
    }
    uint32_t h_fail = 0;
    HIP_TRY(hipMemcpyAsync(&h_fail, d_fail, sizeof h_fail, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h_fail == 0) return BVS_OK;
  }
  HIP_TRY(staged(prof, S_FALLBACK, [&]() -> hipError_t {
    hipError_t e = launch_filter_dense(a, st);
    if (e != hipSuccess) return e;
    return launch_select(w.scores, ix->ld, g.L, g.T, n_q, w.sel, f2_ids, f2_scores, f2_count, nullptr, st);
  }));
  return BVS_OK;
}

HausDb haus_db(const bvs_index* ix, uint32_t metric = kMetricHausdorff) {
  HausDb d;
  d.metric = metric;
  d.hi = ix->hi;
  d.lo = ix->lo;
  d.norms = ix->norms;
  d.offsets = ix->offsets;
  d.n_sets = ix->n;
  d.dp = ix->g.dp;
  d.scr = screen_enabled() ? ix->scr : nullptr;
  return d;
}

HausQ haus_q(const QueryWs& w, uint32_t n_q, uint32_t max_rows) {
  HausQ q;
  q.hi = w.qhi;
  q.lo = w.qlo;
  q.norms = w.qnorm;
  q.scr = w.qscr;
  q.offsets = w.qoff;
  q.n_q = n_q;
  q.max_rows = max_rows;
  q.qids = nullptr;
  return q;
}

bvs_status need_ws(uint64_t have, uint64_t need, void* ws) {
  if (!ws) return fail(BVS_EINVAL, "workspace is NULL");
  if (have < need)
    return fail(BVS_ENOSPC, "workspace of %llu bytes, %llu needed", (unsigned long long)have, (unsigned long long)need);
  return BVS_OK;
}

// The whole cascade search of bvs_search on a workspace of ws_bytes at d_ws;
// prof_allowed = false records no stage events and collects no counters.
bool metric_ok(int metric) { return metric >= 0 && metric <= (int)kMetricMin; }

bvs_status search_impl(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, uint32_t k,
                       void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                       hipStream_t st, bool prof_allowed, uint32_t metric = kMetricHausdorff) {
  if (!metric_ok((int)metric)) return fail(BVS_EINVAL, "unknown metric %u", metric);
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!d_ids || !d_dist || !d_count) return fail(BVS_EINVAL, "NULL output");
  if (k < 1 || k > kMaxK || k > ix->g.T) return fail(BVS_EINVAL, "k %u outside 1..min(64, top_t)", k);
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_search_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  Carver c(d_ws);
  QueryWs w;
  layout_search(c, ix, n_q, NQ, &w);
  CallProf prof(st, prof_allowed);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  BVS_TRY(run_filters(ix, n_q, NQ, w, w.f2_ids, w.f2_scores, w.f2_count, st, prof));
  HIP_TRY(staged(prof, S_RERANK, [&] {
    return launch_haus_cand(haus_db(ix, metric), haus_q(w, n_q, max_rows), w.f2_ids, w.f2_count, ix->g.T, k, w.thr,
                            w.h2, prof.count ? w.stats : nullptr, w.surv, w.surv_count, st);
  }));
  HIP_TRY(staged(prof, S_TOPK, [&] {
    return launch_topk(w.h2, w.f2_ids, w.f2_count, ix->g.T, ix->g.T, n_q, k, w.topk_tmp, d_ids, d_dist, d_count, st,
                       metric == kMetricMeanMin);
  }));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish(prof.count ? w.stats : nullptr);
  return s;
}

// Exact top-k over every set by `metric` (bvs_bruteforce and its metric form).
bvs_status brute_impl(const bvs_index* ix, uint32_t metric, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                      uint32_t k, void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                      hipStream_t st) {
  if (!metric_ok((int)metric)) return fail(BVS_EINVAL, "unknown metric %u", metric);
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!d_ids || !d_dist || !d_count) return fail(BVS_EINVAL, "NULL output");
  if (k < 1 || k > kMaxK) return fail(BVS_EINVAL, "k %u outside 1..64", k);
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_bruteforce_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  Carver c(d_ws);
  QueryWs w;
  layout_brute(c, ix, n_q, NQ, &w);
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  HIP_TRY(staged(prof, S_BRUTE, [&] {
    return launch_haus_all(haus_db(ix, metric), haus_q(w, n_q, max_rows), w.h2, h_q_off, w.qids, st);
  }));
  HIP_TRY(staged(prof, S_TOPK, [&] {
    return launch_topk(w.h2, nullptr, nullptr, ix->n, ix->n, n_q, k, w.topk_tmp, d_ids, d_dist, d_count, st,
                       metric == kMetricMeanMin);
  }));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish();
  return s;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* bvs_last_error(void) { return g_err.c_str(); }
const char* bvs_version(void) { return "bvs 0.1 (gfx950)"; }

bvs_status bvs_profile_enable(int flags) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.on = (flags & BVS_PROFILE_TIMING) != 0;
  g_prof.counters_on = (flags & BVS_PROFILE_COUNTERS) != 0;
  for (int i = 0; i < BVS_N_STAGES; ++i) {
    g_prof.ms[i] = 0;
    g_prof.calls[i] = 0;
  }
  for (int i = 0; i < BVS_N_COUNTERS; ++i) g_prof.counters[i] = 0;
  return BVS_OK;
}

bvs_status bvs_profile_read(bvs_stage_times* out) {
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> g(g_prof.mu);
  for (int i = 0; i < BVS_N_STAGES; ++i) {
    out->ms[i] = g_prof.ms[i];
    out->calls[i] = g_prof.calls[i];
  }
  for (int i = 0; i < BVS_N_COUNTERS; ++i) out->counters[i] = g_prof.counters[i];
  return BVS_OK;
}

const char* bvs_stage_name(int stage) {
  return (stage >= 0 && stage < BVS_N_STAGES) ? kStageNames[stage] : "";
}

void bvs_params_default(bvs_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->code_bits = 1024;
  p->fan_in = 8;
  p->wta_k = 64;
  p->access_lists = 3;
  p->min_count = 1;
  p->top_t = 1000;
}

bvs_status bvs_params_check(const bvs_params* p) {
  Geometry g;
  return derive(p, &g);
}

bvs_status bvs_projection(const bvs_params* p, uint16_t* h_idx) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!h_idx) return fail(BVS_EINVAL, "h_idx is NULL");
  make_projection(g, p->seed, h_idx);
  return BVS_OK;
}

bvs_status bvs_index_bytes(const bvs_params* p, uint64_t n_sets, uint64_t n_vectors, uint64_t* out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  Carver c(nullptr);
  bvs_index tmp;
  layout_index(c, g, n_sets, n_vectors, &tmp);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_build_workspace_bytes(const bvs_params* p, uint64_t n_sets, uint64_t n_vectors, uint64_t* out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  (void)n_vectors;
  Carver c(nullptr);
  c.take<uint32_t>(4);
  c.take<uint8_t>(n_sets * g.L);
  c.take<uint64_t>(n_sets * g.R);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_build_index(const bvs_params* p, const float* d_vectors, const uint64_t* h_offsets, uint64_t n_sets,
                           void* d_index_mem, uint64_t index_bytes, void* d_ws, uint64_t ws_bytes, void* stream,
                           bvs_index** out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_sets == 0) return fail(BVS_EINVAL, "n_sets must be positive");
  if (n_sets >= 0xFFFFFFFFull) return fail(BVS_ENOTSUP, "n_sets must be below 2^32 - 1");
  if (!d_vectors) return fail(BVS_EINVAL, "vectors are NULL");
  uint32_t max_m = 0;
  BVS_TRY(check_offsets(h_offsets, n_sets, 255, "database", &max_m));
  const uint64_t N = h_offsets[n_sets];
  uint64_t need = 0, wneed = 0;
  BVS_TRY(bvs_index_bytes(p, n_sets, N, &need));
  BVS_TRY(bvs_build_workspace_bytes(p, n_sets, N, &wneed));
  if (!d_index_mem) return fail(BVS_EINVAL, "index memory is NULL");
  if (index_bytes < need)
    return fail(BVS_ENOSPC, "index memory of %llu bytes, %llu needed", (unsigned long long)index_bytes,
                (unsigned long long)need);
  BVS_TRY(need_ws(ws_bytes, wneed, d_ws));
  hipStream_t st = (hipStream_t)stream;

  bvs_index* ix = new bvs_index();
  ix->p = *p;
  ix->g = g;
  ix->n = n_sets;
  ix->N = N;
  ix->max_m = max_m;
  if (hipGetDevice(&ix->device) != hipSuccess) ix->device = 0;
  ix->n_cu = device_cus(ix->device);
  Carver c(d_index_mem);
  layout_index(c, g, n_sets, N, ix);
  Carver wc(d_ws);
  uint32_t* status = wc.take<uint32_t>(4);
  uint8_t* cnt_rm = wc.take<uint8_t>(n_sets * g.L);
  uint64_t* bits_rm = wc.take<uint64_t>(n_sets * g.R);

  // Projection rows as byte offsets into the staged vector (2 per element),
  // padded to SP entries; padding reads the zero slot dp.
  std::vector<uint16_t> proj((size_t)g.L * g.s), padded((size_t)g.L * g.SP, (uint16_t)(2 * g.dp));
  make_projection(g, p->seed, proj.data());
  for (uint32_t j = 0; j < g.L; ++j)
    for (uint32_t i = 0; i < g.s; ++i) padded[(size_t)j * g.SP + i] = (uint16_t)(2 * proj[(size_t)j * g.s + i]);
  order_projection_gathers(g, padded.data());

  auto run = [&]() -> bvs_status {
    HIP_TRY(hipMemcpyAsync(ix->idx, padded.data(), padded.size() * 2, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ix->offsets, h_offsets, (n_sets + 1) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_fill_u32(status, 4, 0, st));
    HIP_TRY(launch_convert(d_vectors, N, g.d, g.dp, ix->hi, ix->lo, ix->norms, ix->scr, status, ix->n_cu, st));
    HIP_TRY(launch_encode_sets(hash_geom(ix), ix->hi, ix->lo, ix->offsets, n_sets, cnt_rm, bits_rm, ix->n_cu, st));
    HIP_TRY(launch_transpose_sketches(cnt_rm, bits_rm, n_sets, ix->ld, g.L, ix->cnt, ix->bits, st));
    HIP_TRY(launch_bitmap_planes(ix->cnt, ix->ld, g.L, ix->planes, st));
    HIP_TRY(launch_set_weight(ix->bits, g.L / 128, ix->ld, ix->spop, st));
    return read_status(status, st, "database");
  };
  const bvs_status s = run();
  if (s != BVS_OK) {
    hipStreamSynchronize(st);
    delete ix;
    return s;
  }
  *out = ix;
  return BVS_OK;
}

void bvs_index_destroy(bvs_index* ix) { delete ix; }

bvs_status bvs_index_get_info(const bvs_index* ix, bvs_index_info* info) {
  if (!ix || !info) return fail(BVS_EINVAL, "NULL argument");
  info->n_sets = ix->n;
  info->n_vectors = ix->N;
  info->ld_sets = ix->ld;
  info->dim_padded = ix->g.dp;
  info->max_set_size = ix->max_m;
  return BVS_OK;
}

bvs_status bvs_index_get_params(const bvs_index* ix, bvs_params* p) {
  if (!ix || !p) return fail(BVS_EINVAL, "NULL argument");
  *p = ix->p;
  return BVS_OK;
}

bvs_status bvs_index_set_search_params(bvs_index* ix, uint32_t access_lists, uint32_t min_count, uint32_t top_t) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  bvs_params p = ix->p;
  p.access_lists = access_lists;
  p.min_count = min_count;
  p.top_t = top_t;
  Geometry g;
  BVS_TRY(derive(&p, &g));
  ix->p.access_lists = access_lists;
  ix->p.min_count = min_count;
  ix->p.top_t = top_t;
  ix->g.A = g.A;
  ix->g.M = g.M;
  ix->g.T = g.T;
  return BVS_OK;
}

bvs_status bvs_sketch_views(const bvs_index* ix, const uint8_t** d_count, const uint64_t** d_bits) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (d_count) *d_count = ix->cnt;
  if (d_bits) *d_bits = ix->bits;
  return BVS_OK;
}

bvs_status bvs_encode_workspace_bytes(const bvs_index* ix, uint64_t n, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  c.take<uint32_t>(4);
  c.take<int8_t>(n * ix->g.dp);
  c.take<uint8_t>(n * ix->g.dp);
  c.take<uint32_t>(n);
  if (ix->learned) {
    c.take<uint16_t>(n * ix->g.d);
    c.take<uint16_t>(n * ix->hidden);
    c.take<float>(n * ix->g.L);
  }
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_encode(const bvs_index* ix, const float* d_x, uint64_t n, void* d_ws, uint64_t ws_bytes,
                      uint64_t* d_codes, void* stream) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (n == 0) return BVS_OK;
  if (!d_x || !d_codes) return fail(BVS_EINVAL, "NULL argument");
  uint64_t need = 0;
  BVS_TRY(bvs_encode_workspace_bytes(ix, n, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  uint32_t* status = c.take<uint32_t>(4);
  int8_t* hi = c.take<int8_t>(n * ix->g.dp);
  uint8_t* lo = c.take<uint8_t>(n * ix->g.dp);
  uint32_t* norms = c.take<uint32_t>(n);
  uint16_t* x16 = ix->learned ? c.take<uint16_t>(n * ix->g.d) : nullptr;
  uint16_t* h16 = ix->learned ? c.take<uint16_t>(n * ix->hidden) : nullptr;
  float* y = ix->learned ? c.take<float>(n * ix->g.L) : nullptr;
  HIP_TRY(launch_fill_u32(status, 4, 0, st));
  HIP_TRY(launch_convert(d_x, n, ix->g.d, ix->g.dp, hi, lo, norms, nullptr, status, ix->n_cu, st));
  HIP_TRY(encode_planes(ix, hi, lo, n, d_codes, x16, h16, y, st));
  return read_status(status, st, "vectors");
}

bvs_status bvs_search_workspace_bytes(const bvs_index* ix, uint32_t n_q, uint64_t n_q_vectors, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  QueryWs w;
  layout_search(c, ix, n_q, n_q_vectors, &w);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_bruteforce_workspace_bytes(const bvs_index* ix, uint32_t n_q, uint64_t n_q_vectors, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  QueryWs w;
  layout_brute(c, ix, n_q, n_q_vectors, &w);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_query_sketch(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, void* d_ws,
                            uint64_t ws_bytes, uint16_t* d_cq, uint64_t* d_sq, uint32_t* d_pos, void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_search_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  QueryWs w;
  layout_search(c, ix, n_q, NQ, &w);
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  const Geometry& g = ix->g;
  BVS_TRY(query_side(ix, n_q, NQ, w, st, prof));
  if (d_cq) HIP_TRY(hipMemcpyAsync(d_cq, w.cq, (uint64_t)n_q * g.L * 2, hipMemcpyDeviceToDevice, st));
  if (d_sq) HIP_TRY(hipMemcpyAsync(d_sq, w.sq, (uint64_t)n_q * g.R * 8, hipMemcpyDeviceToDevice, st));
  if (d_pos) HIP_TRY(hipMemcpyAsync(d_pos, w.pos, (uint64_t)n_q * g.A * 4, hipMemcpyDeviceToDevice, st));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish();
  return s;
}

bvs_status bvs_search_candidates(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                                 void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, uint16_t* d_scores,
                                 uint32_t* d_count, void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!d_ids || !d_scores || !d_count) return fail(BVS_EINVAL, "NULL output");
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_search_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  QueryWs w;
  layout_search(c, ix, n_q, NQ, &w);
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  BVS_TRY(run_filters(ix, n_q, NQ, w, d_ids, d_scores, d_count, st, prof));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish(prof.count ? w.stats : nullptr);
  return s;
}

bvs_status bvs_search(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, uint32_t k,
                      void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                      void* stream) {
  return search_impl(ix, d_q, h_q_off, n_q, k, d_ws, ws_bytes, d_ids, d_dist, d_count, (hipStream_t)stream, true);
}

bvs_status bvs_bruteforce(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, uint32_t k,
                          void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                          void* stream) {
  return brute_impl(ix, kMetricHausdorff, d_q, h_q_off, n_q, k, d_ws, ws_bytes, d_ids, d_dist, d_count,
                    (hipStream_t)stream);
}

bvs_status bvs_search_metric(const bvs_index* ix, int metric, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                             uint32_t k, void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist,
                             uint32_t* d_count, void* stream) {
  if (!metric_ok(metric)) return fail(BVS_EINVAL, "unknown metric %d", metric);
  return search_impl(ix, d_q, h_q_off, n_q, k, d_ws, ws_bytes, d_ids, d_dist, d_count, (hipStream_t)stream, true,
                     (uint32_t)metric);
}

bvs_status bvs_bruteforce_metric(const bvs_index* ix, int metric, const float* d_q, const uint64_t* h_q_off,
                                 uint32_t n_q, uint32_t k, void* d_ws, uint64_t ws_bytes, uint32_t* d_ids,
                                 float* d_dist, uint32_t* d_count, void* stream) {
  if (!metric_ok(metric)) return fail(BVS_EINVAL, "unknown metric %d", metric);
  return brute_impl(ix, (uint32_t)metric, d_q, h_q_off, n_q, k, d_ws, ws_bytes, d_ids, d_dist, d_count,
                    (hipStream_t)stream);
}

bvs_status bvs_hausdorff_all(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                             void* d_ws, uint64_t ws_bytes, uint32_t* d_h2, void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!d_h2) return fail(BVS_EINVAL, "NULL output");
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_bruteforce_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  QueryWs w;
  layout_brute(c, ix, n_q, NQ, &w);
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  HIP_TRY(staged(prof, S_BRUTE,
                 [&] { return launch_haus_all(haus_db(ix), haus_q(w, n_q, max_rows), d_h2, h_q_off, w.qids, st); }));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish();
  return s;
}

}  // extern "C"

// ====================================================================== batch
struct bvs_batch {
  const bvs_index* ix = nullptr;
  uint32_t n_q = 0, k = 0, max_rows = 0;
  uint64_t NQ = 0;
  std::vector<uint64_t> off;      // query offsets (host copy)
  std::vector<uint32_t> order;    // queries by size, largest first
  bvs_batch_config cfg{};
  bvs_batch_info info{};
  bool bound = false;
  const float* d_q = nullptr;
  uint32_t* d_ids = nullptr;
  float* d_dist = nullptr;
  uint32_t* d_count = nullptr;
  QueryWs w{};
  uint32_t* d_order = nullptr;
  uint32_t* d_ctl = nullptr;
  // phase sequence of the re-rank: the queries by size class (up to 2, 4, 8
  // and 16 tiles of 16 vectors), each class with its own kernels
  std::vector<uint32_t> bucket;   // query ids, class after class
  uint32_t bucket_off[5] = {0, 0, 0, 0, 0};
  uint32_t bucket_rows[4] = {0, 0, 0, 0};
  uint32_t* d_bucket = nullptr;
  hipGraphExec_t exec = nullptr;
  std::unique_ptr<CallProf> pending;   // stage events of an eager launch
};

namespace {

// Largest LDS a persistent re-rank workgroup may stage (the kernel's own
// static LDS is below 1 KB).
constexpr size_t kQueueLdsLimit = 159 * 1024;

const uint32_t kTuneRows[] = {32, 64, 128};
const uint32_t kTuneWaves[] = {2, 4, 8};

// Tuner cache: shape class -> (lds_rows, waves).
struct TuneKey {
  uint32_t dp, T, k, nqt, lgq;
  bool operator<(const TuneKey& o) const {
    return std::tie(dp, T, k, nqt, lgq) < std::tie(o.dp, o.T, o.k, o.nqt, o.lgq);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<uint32_t, uint32_t>> g_tune;

TuneKey tune_key(const bvs_batch* b) {
  uint32_t lg = 0;
  while ((1u << lg) < b->n_q) ++lg;
  return TuneKey{b->ix->g.dp, b->ix->g.T, b->k, (b->max_rows + 15) / 16, lg};
}

void layout_batch(Carver& c, const bvs_index* ix, uint32_t n_q, uint64_t NQ, bvs_batch* b) {
  layout_search(c, ix, n_q, NQ, &b->w);
  b->d_order = c.take<uint32_t>(n_q);
  b->d_ctl = c.take<uint32_t>(1ull + n_q);
  b->d_bucket = c.take<uint32_t>(n_q);
}

QueueArgs queue_args(const bvs_batch* b) {
  QueueArgs a;
  a.ids = b->w.f2_ids;
  a.count = b->w.f2_count;
  a.T = b->ix->g.T;
  a.k = b->k;
  a.order = b->d_order;
  a.nch = (a.T + kCandPerItem - 1) / kCandPerItem;
  a.lds_rows = b->info.lds_rows;
  a.ctl = b->d_ctl;
  a.h2 = b->w.h2;
  a.stats = nullptr;
  return a;
}

// Query conversion and the cascade up to F2, with the fallback decided on
// the device.
bvs_status batch_filters(bvs_batch* b, hipStream_t st, CallProf& prof) {
  const bvs_index* ix = b->ix;
  QueryWs& w = b->w;
  HIP_TRY(launch_fill_u32(w.status, 4, 0, st));
  HIP_TRY(staged(prof, S_CONVERT, [&] {
    return launch_convert(b->d_q, b->NQ, ix->g.d, ix->g.dp, w.qhi, w.qlo, w.qnorm, w.qscr, w.status, ix->n_cu, st);
  }));
  return run_filters(ix, b->n_q, b->NQ, w, w.f2_ids, w.f2_scores, w.f2_count, st, prof, false);
}

bvs_status batch_rerank(bvs_batch* b, hipStream_t st, CallProf& prof) {
  if (b->info.waves == 0) {
    // the phase sequence of bvs_search, one size class at a time
    const QueryWs& w = b->w;
    HIP_TRY(staged(prof, S_RERANK, [&]() -> hipError_t {
      hipError_t e = launch_fill_u32(w.surv_count, b->n_q, 0, st);
      for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        const uint32_t n = b->bucket_off[c + 1] - b->bucket_off[c];
        if (n == 0) continue;
        HausQ hq = haus_q(w, n, b->bucket_rows[c]);
        hq.qids = b->d_bucket + b->bucket_off[c];
        e = launch_haus_cand(haus_db(b->ix), hq, w.f2_ids, w.f2_count, b->ix->g.T, b->k, w.thr, w.h2,
                             prof.count ? w.stats : nullptr, w.surv, w.surv_count, st);
      }
      return e;
    }));
    return BVS_OK;
  }
  QueueArgs a = queue_args(b);
  if (prof.count) a.stats = b->w.stats;
  HIP_TRY(staged(prof, S_RERANK, [&] {
    return launch_haus_queue(haus_db(b->ix), haus_q(b->w, b->n_q, b->max_rows), a, b->info.waves, b->info.blocks, st);
  }));
  return BVS_OK;
}

bvs_status batch_enqueue(bvs_batch* b, hipStream_t st, CallProf& prof) {
  BVS_TRY(batch_filters(b, st, prof));
  BVS_TRY(batch_rerank(b, st, prof));
  const uint32_t T = b->ix->g.T;
  HIP_TRY(staged(prof, S_TOPK, [&] {
    return launch_topk(b->w.h2, b->w.f2_ids, b->w.f2_count, T, T, b->n_q, b->k, b->w.topk_tmp, b->d_ids, b->d_dist,
                       b->d_count, st);
  }));
  return BVS_OK;
}

// Persistent grid of a shape, or 0 when the shape spills or does not fit.
uint32_t shape_blocks(const bvs_batch* b, uint32_t rows, uint32_t waves) {
  if (haus_queue_lds_bytes(rows, b->ix->g.dp) > kQueueLdsLimit) return 0;
  uint32_t bpc = 0, spill = 0;
  if (haus_queue_occupancy(b->ix->g.dp, rows, waves, &bpc, &spill) != hipSuccess) return 0;
  if (bpc == 0 || spill > 8) return 0;   // 8 bytes: the work-counter slot
  return bpc * (uint32_t)b->ix->n_cu;
}

// Times every candidate shape on the bound batch (F2 computed once first)
// and keeps the fastest.
bvs_status batch_tune(bvs_batch* b, hipStream_t st) {
  CallProf off(st, false);
  BVS_TRY(batch_filters(b, st, off));
  HIP_TRY(hipStreamSynchronize(st));
  const uint32_t rows_needed = (b->max_rows + 15) / 16 * 16;
  std::vector<uint32_t> rows_c, waves_c;
  if (b->cfg.lds_rows) {
    rows_c.push_back(b->cfg.lds_rows);
  } else {
    for (uint32_t r : kTuneRows) {
      const uint32_t rr = std::min(r, rows_needed);
      if (std::find(rows_c.begin(), rows_c.end(), rr) == rows_c.end()) rows_c.push_back(rr);
    }
  }
  if (b->cfg.waves) waves_c.push_back(b->cfg.waves);
  else waves_c.assign(std::begin(kTuneWaves), std::end(kTuneWaves));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BVS_EDEVICE, "hipEventCreate failed");
  }
  bvs_status status = BVS_OK;
  float best = 0.f;
  b->info.n_tried = 0;
  for (uint32_t r : rows_c) {
    for (uint32_t wv : waves_c) {
      const uint32_t blocks = shape_blocks(b, r, wv);
      if (!blocks || b->info.n_tried >= BVS_TUNE_MAX) continue;
      b->info.lds_rows = r;
      b->info.waves = wv;
      b->info.blocks = blocks;
      float ms = 0.f;
      status = [&]() -> bvs_status {
        BVS_TRY(batch_rerank(b, st, off));   // warm-up
        HIP_TRY(hipEventRecord(e0, st));
        BVS_TRY(batch_rerank(b, st, off));
        BVS_TRY(batch_rerank(b, st, off));
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        return BVS_OK;
      }();
      if (status != BVS_OK) break;
      ms *= 0.5f;
      const uint32_t i = b->info.n_tried++;
      b->info.tried_lds_rows[i] = r;
      b->info.tried_waves[i] = wv;
      b->info.tried_ms[i] = ms;
      if (i == 0 || ms < best) best = ms;
    }
    if (status != BVS_OK) break;
  }
  if (status == BVS_OK && !b->cfg.lds_rows && !b->cfg.waves && b->info.n_tried < BVS_TUNE_MAX) {
    // the phase sequence of bvs_search by size class (shape 0 x 0)
    b->info.lds_rows = 0;
    b->info.waves = 0;
    b->info.blocks = 0;
    float ms = 0.f;
    status = [&]() -> bvs_status {
      BVS_TRY(batch_rerank(b, st, off));
      HIP_TRY(hipEventRecord(e0, st));
      BVS_TRY(batch_rerank(b, st, off));
      BVS_TRY(batch_rerank(b, st, off));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      return BVS_OK;
    }();
    if (status == BVS_OK) {
      ms *= 0.5f;
      const uint32_t i = b->info.n_tried++;
      b->info.tried_lds_rows[i] = 0;
      b->info.tried_waves[i] = 0;
      b->info.tried_ms[i] = ms;
      if (i == 0 || ms < best) best = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != BVS_OK) return status;
  if (b->info.n_tried == 0) return fail(BVS_ENOTSUP, "no re-rank shape fits dim %u", b->ix->g.d);
  for (uint32_t i = 0; i < b->info.n_tried; ++i) {
    if (b->info.tried_ms[i] == best) {
      b->info.lds_rows = b->info.tried_lds_rows[i];
      b->info.waves = b->info.tried_waves[i];
      break;
    }
  }
  b->info.blocks = b->info.waves ? shape_blocks(b, b->info.lds_rows, b->info.waves) : 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[tune_key(b)] = {b->info.lds_rows, b->info.waves};
  return BVS_OK;
}

bvs_status batch_capture(bvs_batch* b, hipStream_t st) {
  if (!st) return fail(BVS_EINVAL, "graph capture needs a stream other than the null stream");
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  CallProf off(st, false);
  const bvs_status s = batch_enqueue(b, st, off);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &graph);
  if (s != BVS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  HIP_TRY(e);
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_TRY(ei);
  b->exec = exec;
  return BVS_OK;
}

void batch_release(bvs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  if (b->pending) b->pending->release();
  b->pending.reset();
  b->bound = false;
}

}  // namespace

extern "C" {

bvs_status bvs_batch_create(const bvs_index* ix, const uint64_t* h_q_off, uint32_t n_q, uint32_t k,
                            const bvs_batch_config* cfg, bvs_batch** out) {
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (n_q == 0) return fail(BVS_EINVAL, "n_q must be positive");
  uint32_t max_rows = 0;
  BVS_TRY(check_offsets(h_q_off, n_q, 65535, "query", &max_rows));
  if (max_rows > haus_max_rows_supported(ix->g.dp))
    return fail(BVS_ENOTSUP, "query set of %u vectors exceeds the %u supported", max_rows,
                haus_max_rows_supported(ix->g.dp));
  if (k < 1 || k > kMaxK || k > ix->g.T) return fail(BVS_EINVAL, "k %u outside 1..min(64, top_t)", k);
  bvs_batch_config c{};
  if (cfg) c = *cfg;
  if (c.flags & ~BVS_BATCH_PHASES) return fail(BVS_EINVAL, "config.flags %u: unknown flag", c.flags);
  if ((c.flags & BVS_BATCH_PHASES) && (c.lds_rows || c.waves))
    return fail(BVS_EINVAL, "config.flags BVS_BATCH_PHASES excludes a persistent shape (lds_rows, waves)");
  if (c.lds_rows && (c.lds_rows % 16 != 0 || c.lds_rows > 256))
    return fail(BVS_EINVAL, "config.lds_rows %u is not a multiple of 16 in 16..256", c.lds_rows);
  if (c.lds_rows && haus_queue_lds_bytes(c.lds_rows, ix->g.dp) > kQueueLdsLimit)
    return fail(BVS_ENOTSUP, "config.lds_rows %u does not fit in LDS at dim %u", c.lds_rows, ix->g.d);
  if (c.waves && c.waves != 2 && c.waves != 4 && c.waves != 8)
    return fail(BVS_EINVAL, "config.waves %u is not 2, 4 or 8", c.waves);
  std::unique_ptr<bvs_batch> b(new (std::nothrow) bvs_batch());
  if (!b) return fail(BVS_ENOSPC, "out of host memory");
  b->ix = ix;
  b->n_q = n_q;
  b->k = k;
  b->max_rows = max_rows;
  b->NQ = h_q_off[n_q];
  b->off.assign(h_q_off, h_q_off + n_q + 1);
  b->order.resize(n_q);
  for (uint32_t i = 0; i < n_q; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](uint32_t x, uint32_t y) {
    return h_q_off[x + 1] - h_q_off[x] > h_q_off[y + 1] - h_q_off[y];
  });
  b->cfg = c;
  {
    std::vector<uint32_t> cls[4];
    for (uint32_t i = 0; i < n_q; ++i) {
      const uint64_t m = h_q_off[i + 1] - h_q_off[i];
      const uint32_t nqt = (uint32_t)((m + 15) / 16);
      const int k = nqt <= 2 ? 0 : nqt <= 4 ? 1 : nqt <= 8 ? 2 : 3;
      cls[k].push_back(i);
      b->bucket_rows[k] = std::max<uint32_t>(b->bucket_rows[k], (uint32_t)m);
    }
    for (int k = 0; k < 4; ++k) {
      b->bucket_off[k] = (uint32_t)b->bucket.size();
      b->bucket.insert(b->bucket.end(), cls[k].begin(), cls[k].end());
    }
    b->bucket_off[4] = (uint32_t)b->bucket.size();
  }
  Carver cv(nullptr);
  bvs_batch tmp;
  layout_batch(cv, ix, n_q, b->NQ, &tmp);
  b->info.n_q = n_q;
  b->info.max_rows = max_rows;
  b->info.n_q_vectors = b->NQ;
  b->info.workspace_bytes = align_up(cv.off, 256);
  *out = b.release();
  return BVS_OK;
}

bvs_status bvs_batch_bind(bvs_batch* b, const float* d_q, void* d_ws, uint64_t ws_bytes, uint32_t* d_ids,
                          float* d_dist, uint32_t* d_count, void* stream) {
  if (!b) return fail(BVS_EINVAL, "batch is NULL");
  if (!d_q) return fail(BVS_EINVAL, "query vectors are NULL");
  if (!d_ids || !d_dist || !d_count) return fail(BVS_EINVAL, "NULL output");
  BVS_TRY(need_ws(ws_bytes, b->info.workspace_bytes, d_ws));
  hipStream_t st = (hipStream_t)stream;
  batch_release(b);
  b->d_q = d_q;
  b->d_ids = d_ids;
  b->d_dist = d_dist;
  b->d_count = d_count;
  Carver c(d_ws);
  layout_batch(c, b->ix, b->n_q, b->NQ, b);
  HIP_TRY(hipMemcpyAsync(b->w.qoff, b->off.data(), b->off.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b->d_order, b->order.data(), b->order.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b->d_bucket, b->bucket.data(), b->bucket.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  // re-rank shape: given, cached, or tuned now
  b->info.from_cache = 0;
  b->info.n_tried = 0;
  if (b->cfg.flags & BVS_BATCH_PHASES) {
    b->info.lds_rows = 0;
    b->info.waves = 0;
  } else if (b->cfg.lds_rows && b->cfg.waves) {
    b->info.lds_rows = b->cfg.lds_rows;
    b->info.waves = b->cfg.waves;
  } else {
    bool hit = false;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(tune_key(b));
      if (it != g_tune.end() && (!b->cfg.lds_rows || it->second.first == b->cfg.lds_rows) &&
          (!b->cfg.waves || it->second.second == b->cfg.waves)) {
        b->info.lds_rows = it->second.first;
        b->info.waves = it->second.second;
        hit = true;
      }
    }
    if (hit) b->info.from_cache = 1;
    else BVS_TRY(batch_tune(b, st));
  }
  b->info.blocks = b->info.waves ? shape_blocks(b, b->info.lds_rows, b->info.waves) : 0;
  if (b->info.waves && !b->info.blocks)
    return fail(BVS_ENOTSUP, "re-rank shape lds_rows %u, waves %u does not fit a CU", b->info.lds_rows,
                b->info.waves);
  b->info.graph = 0;
  if (b->cfg.graph) {
    BVS_TRY(batch_capture(b, st));
    b->info.graph = 1;
  }
  b->bound = true;
  return BVS_OK;
}

bvs_status bvs_batch_launch(bvs_batch* b, void* stream) {
  if (!b) return fail(BVS_EINVAL, "batch is NULL");
  if (!b->bound) return fail(BVS_ESTATE, "batch is not bound");
  hipStream_t st = (hipStream_t)stream;
  if (b->exec) {
    HIP_TRY(hipGraphLaunch(b->exec, st));
    return BVS_OK;
  }
  if (b->pending) {
    // stage events of the previous launch: finish them first
    HIP_TRY(hipStreamSynchronize(st));
    b->pending->finish(b->pending->count ? b->w.stats : nullptr);
    b->pending->release();
    b->pending.reset();
  }
  std::unique_ptr<CallProf> prof(new CallProf(st));
  BVS_TRY(batch_enqueue(b, st, *prof));
  if (prof->on || prof->count) b->pending = std::move(prof);
  return BVS_OK;
}

bvs_status bvs_batch_status(bvs_batch* b, void* stream) {
  if (!b) return fail(BVS_EINVAL, "batch is NULL");
  if (!b->bound) return fail(BVS_ESTATE, "batch is not bound");
  const bvs_status s = read_status(b->w.status, (hipStream_t)stream, "queries");
  if (b->pending) {
    b->pending->finish(b->pending->count ? b->w.stats : nullptr);
    b->pending->release();
    b->pending.reset();
  }
  return s;
}

bvs_status bvs_batch_get_info(const bvs_batch* b, bvs_batch_info* out) {
  if (!b || !out) return fail(BVS_EINVAL, "NULL argument");
  *out = b->info;
  return BVS_OK;
}

void bvs_batch_destroy(bvs_batch* b) {
  if (!b) return;
  batch_release(b);
  delete b;
}

}  // extern "C"

// ====================================================================== precision form
namespace {

struct LowpWs {
  QueryWs w;
  uint8_t* q_rows;      // [NQ][2 dp]
  float* q_scale;       // [n_q]
  uint32_t* approx;     // [n_q][T] float bits
  uint32_t* r_ids;      // [n_q][T]
  uint32_t* r_count;    // [n_q]
};

void layout_lowp(Carver& c, const bvs_index* ix, uint32_t n_q, uint64_t NQ, LowpWs* l) {
  layout_search(c, ix, n_q, NQ, &l->w);
  l->q_rows = c.take<uint8_t>(NQ * 2 * ix->g.dp);
  l->q_scale = c.take<float>(n_q);
  l->approx = c.take<uint32_t>((uint64_t)n_q * ix->g.T);
  l->r_ids = c.take<uint32_t>((uint64_t)n_q * ix->g.T);
  l->r_count = c.take<uint32_t>(n_q);
}

bool lowp_fmt_ok(int fmt) { return fmt == BVS_LOWP_BF16 || fmt == BVS_LOWP_FP8; }

LowpDb lowp_db(const bvs_index* ix, int fmt) {
  LowpDb d;
  d.rows = ix->lowp[fmt];
  d.scale = fmt == BVS_LOWP_FP8 ? ix->lowp_scale[fmt] : nullptr;
  d.norms = ix->norms;
  d.offsets = ix->offsets;
  d.n_sets = ix->n;
  d.row_bytes = lowp_row_bytes(fmt, ix->g.dp);
  return d;
}

// Encode the converted query planes of the workspace in fmt.
bvs_status lowp_queries(const bvs_index* ix, int fmt, uint32_t n_q, uint32_t max_rows, LowpWs& l, hipStream_t st,
                        LowpQ* q) {
  const uint32_t rb = lowp_row_bytes(fmt, ix->g.dp);
  HIP_TRY(launch_lowp_encode(l.w.qhi, l.w.qlo, ix->g.dp, l.w.qoff, n_q, fmt, rb, l.q_rows, l.q_scale, st));
  q->rows = l.q_rows;
  q->scale = fmt == BVS_LOWP_FP8 ? l.q_scale : nullptr;
  q->norms = l.w.qnorm;
  q->offsets = l.w.qoff;
  q->n_q = n_q;
  q->max_rows = max_rows;
  q->row_bytes = rb;
  return BVS_OK;
}

}  // namespace

extern "C" {

bvs_status bvs_lowp_bytes(const bvs_index* ix, int fmt, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  if (!lowp_fmt_ok(fmt)) return fail(BVS_EINVAL, "unknown precision format %d", fmt);
  Carver c(nullptr);
  c.take<uint8_t>(ix->N * lowp_row_bytes(fmt, ix->g.dp));
  if (fmt == BVS_LOWP_FP8) c.take<float>(ix->n);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_lowp_attach(bvs_index* ix, int fmt, void* d_mem, uint64_t bytes, void* stream) {
  uint64_t need = 0;
  BVS_TRY(bvs_lowp_bytes(ix, fmt, &need));
  if (!d_mem) return fail(BVS_EINVAL, "memory is NULL");
  if (bytes < need) return fail(BVS_ENOSPC, "%llu bytes given, %llu needed", (unsigned long long)bytes,
                                (unsigned long long)need);
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_mem);
  const uint32_t rb = lowp_row_bytes(fmt, ix->g.dp);
  uint8_t* rows = c.take<uint8_t>(ix->N * rb);
  float* scale = fmt == BVS_LOWP_FP8 ? c.take<float>(ix->n) : nullptr;
  HIP_TRY(launch_lowp_encode(ix->hi, ix->lo, ix->g.dp, ix->offsets, ix->n, fmt, rb, rows, scale, st));
  HIP_TRY(hipStreamSynchronize(st));
  ix->lowp[fmt] = rows;
  ix->lowp_scale[fmt] = scale;
  return BVS_OK;
}

bvs_status bvs_lowp_workspace_bytes(const bvs_index* ix, uint32_t n_q, uint64_t n_q_vectors, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  LowpWs l;
  layout_lowp(c, ix, n_q, n_q_vectors, &l);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_search_lowp(const bvs_index* ix, int fmt, float margin, const float* d_q, const uint64_t* h_q_off,
                           uint32_t n_q, uint32_t k, void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist,
                           uint32_t* d_count, uint32_t* d_rechecked, void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!lowp_fmt_ok(fmt)) return fail(BVS_EINVAL, "unknown precision format %d", fmt);
  if (!ix->lowp[fmt]) return fail(BVS_ESTATE, "precision format %d is not attached", fmt);
  if (!(margin >= 0.0f) || !std::isfinite(margin)) return fail(BVS_EINVAL, "margin must be finite and >= 0");
  if (!d_ids || !d_dist || !d_count) return fail(BVS_EINVAL, "NULL output");
  if (k < 1 || k > kMaxK || k > ix->g.T) return fail(BVS_EINVAL, "k %u outside 1..min(64, top_t)", k);
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_lowp_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  LowpWs l;
  layout_lowp(c, ix, n_q, NQ, &l);
  QueryWs& w = l.w;
  const uint32_t T = ix->g.T;
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  BVS_TRY(run_filters(ix, n_q, NQ, w, w.f2_ids, w.f2_scores, w.f2_count, st, prof));
  const float f1 = 1.0f + margin;
  const float factor = f1 * f1;
  LowpQ lq;
  bvs_status ls = BVS_OK;
  HIP_TRY(staged(prof, S_APPROX, [&]() -> hipError_t {
    ls = lowp_queries(ix, fmt, n_q, max_rows, l, st, &lq);
    if (ls != BVS_OK) return hipSuccess;
    // The first 64 candidates in full; their k-th value times the factor
    // bounds the rest: a candidate above it could not be selected anyway.
    const uint32_t n0 = std::min<uint32_t>(T, 64);
    unsigned long long* stats = prof.count ? w.stats : nullptr;
    hipError_t e = launch_haus_lowp(fmt, lowp_db(ix, fmt), lq, w.f2_ids, w.f2_count, T, 0, n0, nullptr, factor,
                                    l.approx, stats, st);
    if (e != hipSuccess) return e;
    if (T > n0) {
      if ((e = launch_kth_bound(l.approx, w.f2_count, T, n0, k, n_q, w.thr, st)) != hipSuccess) return e;
      e = launch_haus_lowp(fmt, lowp_db(ix, fmt), lq, w.f2_ids, w.f2_count, T, n0, T, w.thr, factor, l.approx,
                           stats, st);
      if (e != hipSuccess) return e;
    }
    return launch_lowp_select(l.approx, w.f2_ids, w.f2_count, T, n_q, k, factor, l.r_ids, l.r_count, st);
  }));
  BVS_TRY(ls);
  HIP_TRY(staged(prof, S_RECHECK, [&]() -> hipError_t {
    hipError_t e = launch_haus_cand(haus_db(ix), haus_q(w, n_q, max_rows), l.r_ids, l.r_count, T, k, w.thr, w.h2,
                                    prof.count ? w.stats : nullptr, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    return launch_topk(w.h2, l.r_ids, l.r_count, T, T, n_q, k, w.topk_tmp, d_ids, d_dist, d_count, st);
  }));
  if (d_rechecked)
    HIP_TRY(hipMemcpyAsync(d_rechecked, l.r_count, (uint64_t)n_q * 4, hipMemcpyDeviceToDevice, st));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish(prof.count ? w.stats : nullptr);
  return s;
}

bvs_status bvs_hausdorff_lowp(const bvs_index* ix, int fmt, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                              const uint32_t* d_ids, uint32_t m, void* d_ws, uint64_t ws_bytes, float* d_h2,
                              void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  if (!lowp_fmt_ok(fmt)) return fail(BVS_EINVAL, "unknown precision format %d", fmt);
  if (!ix->lowp[fmt]) return fail(BVS_ESTATE, "precision format %d is not attached", fmt);
  if (!d_ids || !d_h2) return fail(BVS_EINVAL, "NULL argument");
  if (m == 0) return BVS_OK;
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_lowp_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  LowpWs l;
  layout_lowp(c, ix, n_q, NQ, &l);
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, l.w, st, prof));
  LowpQ lq;
  BVS_TRY(lowp_queries(ix, fmt, n_q, max_rows, l, st, &lq));
  HIP_TRY(launch_haus_lowp(fmt, lowp_db(ix, fmt), lq, d_ids, nullptr, m, 0, m, nullptr, 1.0f, (uint32_t*)d_h2,
                           nullptr, st));
  const bvs_status s = read_status(l.w.status, st, "queries");
  prof.finish();
  return s;
}

}  // extern "C"

// ====================================================================== learned projection
namespace {

uint64_t mlp_floats(uint32_t d, uint32_t H, uint32_t L) { return (uint64_t)H * d + H + (uint64_t)L * H + L; }

bvs_status check_mlp_shape(uint32_t d, uint32_t H, uint32_t L) {
  if (d == 0 || d > 1024 || d % 8 != 0) return fail(BVS_ENOTSUP, "learned projection needs dim %% 8 == 0, <= 1024");
  if (H == 0 || H > 8192 || H % 8 != 0) return fail(BVS_ENOTSUP, "hidden size must be a multiple of 8 in 8..8192");
  if (L < 256 || L > 4096 || (L & (L - 1))) return fail(BVS_ENOTSUP, "code_bits must be a power of two in 256..4096");
  return BVS_OK;
}

// Rows encoded per pass of the learned build.
constexpr uint64_t kLearnChunkRows = 1u << 18;

void layout_learned_weights(Carver& c, const Geometry& g, uint32_t H, bvs_index* ix) {
  ix->w16 = c.take<uint16_t>(mlp_floats(g.d, H, g.L));
  ix->b1 = c.take<float>(H);
  ix->b2 = c.take<float>(g.L);
}

struct TrainWs {
  uint64_t* rows;        // [cap] source rows of the batch
  uint32_t* row_off;     // [max_sets + 1]
  uint32_t* trip;        // [B][3]
  uint16_t* x16;         // [cap][d]
  uint16_t* h16;         // [cap][H]
  float* y;              // [cap][L]
  float* thr;            // [cap]
  float* ls;             // [max_sets][L]
  float* s;              // [max_sets][L]
  float* ds;             // [max_sets][L]
  float* dy;             // [cap][L]
  uint16_t* dy16;        // [cap][L]
  float* dh;             // [cap][H]
  uint16_t* dp16;        // [cap][H]
  float* loss;           // [4]: the batch loss (float), then the epoch sum (double at word 2)
  float* grad;           // packed like the weights
  uint16_t* w16;         // packed bfloat16 weights
  float* adam_m;
  float* adam_v;
};

void layout_train(Carver& c, const bvs_train_config& t, uint64_t cap, TrainWs* w) {
  const uint64_t ms = 3ull * t.batch_triplets;
  const uint64_t nw = mlp_floats(t.dim, t.hidden, t.code_bits);
  w->rows = c.take<uint64_t>(cap);
  w->row_off = c.take<uint32_t>(ms + 1);
  w->trip = c.take<uint32_t>(3ull * t.batch_triplets);
  w->x16 = c.take<uint16_t>(cap * t.dim);
  w->h16 = c.take<uint16_t>(cap * t.hidden);
  w->y = c.take<float>(cap * t.code_bits);
  w->thr = c.take<float>(cap);
  w->ls = c.take<float>(ms * t.code_bits);
  w->s = c.take<float>(ms * t.code_bits);
  w->ds = c.take<float>(ms * t.code_bits);
  w->dy = c.take<float>(cap * t.code_bits);
  w->dy16 = c.take<uint16_t>(cap * t.code_bits);
  w->dh = c.take<float>(cap * t.hidden);
  w->dp16 = c.take<uint16_t>(cap * t.hidden);
  w->loss = c.take<float>(4);
  w->grad = c.take<float>(nw);
  w->w16 = c.take<uint16_t>(nw);
  w->adam_m = c.take<float>(nw);
  w->adam_v = c.take<float>(nw);
}

bvs_status check_train_config(const bvs_train_config* t) {
  if (!t) return fail(BVS_EINVAL, "config is NULL");
  BVS_TRY(check_mlp_shape(t->dim, t->hidden, t->code_bits));
  if (t->wta_k < 1 || t->wta_k >= t->code_bits) return fail(BVS_EINVAL, "wta_k outside 1..code_bits-1");
  if (t->batch_triplets < 1 || t->batch_triplets > 65536) return fail(BVS_EINVAL, "batch_triplets outside 1..65536");
  if (!(t->tau > 0.f) || !(t->lr >= 0.f) || !(t->margin >= 0.f) || !std::isfinite(t->tau) || !std::isfinite(t->lr) ||
      !std::isfinite(t->margin))
    return fail(BVS_EINVAL, "tau must be > 0, lr and margin >= 0, all finite");
  return BVS_OK;
}

// One batch of triplets: forward, loss, gradients into w.grad (packed).
// Sets are rows h_off[s] .. h_off[s+1] of d_vectors.
// Pinned host buffers that a batch's row and triplet lists are built in and
// copied from; `copied` is recorded once the copies have been enqueued, and
// the buffers are refilled only after it has completed, so the host builds
// the next batch while the device trains on this one.
struct TrainStage {
  uint64_t* rows = nullptr;   // [cap]
  uint32_t* roff = nullptr;   // [3 batch_triplets + 1]
  uint32_t* tl = nullptr;     // [3 batch_triplets]
  hipEvent_t copied = nullptr;
  bool pending = false;
  TrainStage() = default;
  TrainStage(const TrainStage&) = delete;
  TrainStage& operator=(const TrainStage&) = delete;
  ~TrainStage() {
    if (copied) {
      (void)hipEventSynchronize(copied);
      (void)hipEventDestroy(copied);
    }
    if (rows) (void)hipHostFree(rows);
    if (roff) (void)hipHostFree(roff);
    if (tl) (void)hipHostFree(tl);
  }
  hipError_t alloc(uint64_t cap, uint32_t batch_triplets) {
    hipError_t e = hipHostMalloc((void**)&rows, std::max<uint64_t>(cap, 1) * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&roff, (3ull * batch_triplets + 1) * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&tl, 3ull * batch_triplets * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&copied, hipEventDisableTiming);
    return e;
  }
};

bvs_status train_batch(const bvs_train_config& t, const float* d_vectors, const uint64_t* h_off, uint64_t n_sets,
                       const uint32_t* trips, uint32_t nt, uint64_t cap, const uint16_t* w16, const float* w32,
                       TrainWs& w, hipStream_t st, TrainStage& hs) {
  if (hs.pending) {
    HIP_TRY(hipEventSynchronize(hs.copied));
    hs.pending = false;
  }
  // distinct sets of the batch, in first-seen order
  std::map<uint32_t, uint32_t> local;
  std::vector<uint32_t> sets;
  uint32_t* tl = hs.tl;
  for (uint32_t i = 0; i < nt; ++i) {
    for (int k = 0; k < 3; ++k) {
      const uint32_t sid = trips[3ull * i + k];
      if (sid >= n_sets) return fail(BVS_EINVAL, "triplet %u names set %u of %llu", i, sid, (unsigned long long)n_sets);
      auto it = local.find(sid);
      if (it == local.end()) {
        it = local.emplace(sid, (uint32_t)sets.size()).first;
        sets.push_back(sid);
      }
      tl[3ull * i + k] = it->second;
    }
  }
  uint64_t nb = 0;
  for (uint32_t sid : sets) nb += h_off[sid + 1] - h_off[sid];
  if (nb > cap)
    return fail(BVS_ENOSPC, "a batch holds %llu rows; the workspace fits %llu", (unsigned long long)nb,
                (unsigned long long)cap);
  uint64_t* rows = hs.rows;
  uint32_t* roff = hs.roff;
  uint64_t at = 0;
  roff[0] = 0;
  for (size_t i = 0; i < sets.size(); ++i) {
    for (uint64_t r = h_off[sets[i]]; r < h_off[sets[i] + 1]; ++r) rows[at++] = r;
    roff[i + 1] = (uint32_t)at;
  }
  const uint32_t d = t.dim, H = t.hidden, L = t.code_bits;
  const uint32_t ns = (uint32_t)sets.size();
  HIP_TRY(hipMemcpyAsync(w.rows, rows, nb * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w.row_off, roff, (sets.size() + 1) * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w.trip, tl, 3ull * nt * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(hs.copied, st));
  hs.pending = true;
  const uint16_t* W1 = w16;
  const uint16_t* W2 = w16 + (uint64_t)H * d + H;
  const float* b1 = w32 + (uint64_t)H * d;
  const float* b2 = w32 + (uint64_t)H * d + H + (uint64_t)L * H;
  float* gW1 = w.grad;
  float* gb1 = w.grad + (uint64_t)H * d;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (uint64_t)L * H;
  // forward
  HIP_TRY(launch_rows_to_bf16(d_vectors, d, w.rows, nb, w.x16, st));
  HIP_TRY(launch_gemm(false, false, w.x16, d, W1, d, (uint32_t)nb, H, d, b1, true, nullptr, w.h16, H, st));
  HIP_TRY(launch_gemm(false, false, w.h16, H, W2, H, (uint32_t)nb, L, H, b2, false, w.y, nullptr, L, st));
  HIP_TRY(launch_row_thresholds(w.y, nb, L, t.wta_k, w.thr, st));
  HIP_TRY(launch_set_soft(w.y, w.thr, w.row_off, ns, L, t.tau, w.ls, w.s, st));
  // loss and sketch gradients
  HIP_TRY(launch_fill_u32((uint32_t*)w.ds, (uint64_t)ns * L, 0u, st));
  HIP_TRY(launch_fill_u32((uint32_t*)w.loss, 1, 0u, st));
  HIP_TRY(launch_triplet(w.s, w.trip, nt, L, t.margin, w.ds, w.loss, st));
  // backward
  HIP_TRY(launch_soft_backward(w.y, w.thr, w.row_off, ns, L, t.tau, w.ls, w.ds, w.dy, w.dy16, st));
  HIP_TRY(launch_gemm(false, true, w.dy16, L, W2, H, (uint32_t)nb, H, L, nullptr, false, w.dh, nullptr, H, st));
  HIP_TRY(launch_relu_backward(w.dh, w.h16, nb * H, w.dh, w.dp16, st));
  HIP_TRY(launch_gemm(true, true, w.dy16, L, w.h16, H, L, H, (uint32_t)nb, nullptr, false, gW2, nullptr, H, st));
  HIP_TRY(launch_gemm(true, true, w.dp16, H, w.x16, d, H, d, (uint32_t)nb, nullptr, false, gW1, nullptr, d, st));
  HIP_TRY(launch_colsum(w.dy, nb, L, gb2, st));
  HIP_TRY(launch_colsum(w.dh, nb, H, gb1, st));
  return BVS_OK;
}

// Offset of the header (step and epoch counts, uint64 each) in a training
// state: after Adam's two moment arrays.
uint64_t train_state_header(const bvs_train_config& t) {
  return align_up(2 * mlp_floats(t.dim, t.hidden, t.code_bits) * 4, 256);
}

uint64_t train_capacity(const bvs_train_config& t, uint64_t ws_bytes) {
  // largest row capacity whose layout fits ws_bytes
  uint64_t lo = 0, hi = 1ull << 26;
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) / 2;
    Carver c(nullptr);
    TrainWs w;
    layout_train(c, t, mid, &w);
    if (align_up(c.off, 256) <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

namespace {

// Epochs of triplet training from the Adam state in d_state (moments, then the
// step and epoch counts; updated in place), or from a fresh state in the
// workspace when d_state is null.  Epoch e (counted over all calls on one
// state) visits the triplets in the order of a Fisher-Yates shuffle of the
// identity driven by splitmix64 from seed ^ (e + 1) * 0xD1B54A32D192ED03, so a
// run split over several calls visits the same batches as one call.
bvs_status train_impl(const bvs_train_config* t, const float* d_vectors, const uint64_t* h_offsets, uint64_t n_sets,
                      const uint32_t* h_triplets, uint64_t n_triplets, float* d_weights, void* d_state, void* d_ws,
                      uint64_t ws_bytes, float* h_epoch_loss, hipStream_t st) {
  BVS_TRY(check_train_config(t));
  if (!d_vectors || !d_weights || !h_triplets) return fail(BVS_EINVAL, "NULL argument");
  if (n_triplets == 0) return fail(BVS_EINVAL, "no triplets");
  uint32_t max_m = 0;
  BVS_TRY(check_offsets(h_offsets, n_sets, 65535, "training", &max_m));
  const uint64_t cap = train_capacity(*t, ws_bytes);
  if (!d_ws || cap == 0) return fail(BVS_ENOSPC, "workspace too small");
  Carver c(d_ws);
  TrainWs w;
  layout_train(c, *t, cap, &w);
  const uint64_t nw = mlp_floats(t->dim, t->hidden, t->code_bits);
  uint64_t hdr[2] = {0, 0};   // step, epoch
  float* adam_m = w.adam_m;
  float* adam_v = w.adam_v;
  uint64_t* d_hdr = nullptr;
  if (d_state) {
    adam_m = (float*)d_state;
    adam_v = adam_m + nw;
    d_hdr = (uint64_t*)((uint8_t*)d_state + train_state_header(*t));
    HIP_TRY(hipMemcpyAsync(hdr, d_hdr, sizeof hdr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hdr[0] > 0xFFFFFFFFull) return fail(BVS_EINVAL, "training state holds step %llu", (unsigned long long)hdr[0]);
  } else {
    HIP_TRY(launch_fill_u32((uint32_t*)adam_m, nw, 0u, st));
    HIP_TRY(launch_fill_u32((uint32_t*)adam_v, nw, 0u, st));
  }
  HIP_TRY(launch_f32_to_bf16(d_weights, nw, w.w16, st));
  std::vector<uint64_t> order(n_triplets);
  std::vector<uint32_t> batch;
  TrainStage hs[2];
  HIP_TRY(hs[0].alloc(cap, t->batch_triplets));
  HIP_TRY(hs[1].alloc(cap, t->batch_triplets));
  double* d_ep_loss = (double*)(w.loss + 2);
  uint32_t step = (uint32_t)hdr[0];
  for (uint32_t ep = 0; ep < t->epochs; ++ep) {
    const uint64_t e_abs = hdr[1] + ep;
    uint64_t rng = t->seed ^ ((e_abs + 1) * 0xD1B54A32D192ED03ull);
    auto next = [&rng]() {
      rng += 0x9E3779B97F4A7C15ull;
      uint64_t z = rng;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      return z ^ (z >> 31);
    };
    for (uint64_t i = 0; i < n_triplets; ++i) order[i] = i;
    for (uint64_t i = n_triplets - 1; i > 0; --i) std::swap(order[i], order[next() % (i + 1)]);
    HIP_TRY(launch_fill_u32((uint32_t*)d_ep_loss, 2, 0u, st));
    uint64_t n_batches = 0;
    for (uint64_t b0 = 0; b0 < n_triplets; b0 += t->batch_triplets) {
      const uint32_t nt = (uint32_t)std::min<uint64_t>(t->batch_triplets, n_triplets - b0);
      batch.resize(3ull * nt);
      for (uint32_t i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k) batch[3ull * i + k] = h_triplets[3 * order[b0 + i] + k];
      BVS_TRY(train_batch(*t, d_vectors, h_offsets, n_sets, batch.data(), nt, cap, w.w16, d_weights, w, st,
                          hs[n_batches & 1]));
      HIP_TRY(launch_adam(d_weights, w.grad, adam_m, adam_v, nw, t->lr, 0.9f, 0.999f, 1e-8f, ++step, w.w16, st));
      HIP_TRY(launch_add_loss(w.loss, d_ep_loss, st));
      ++n_batches;
    }
    if (h_epoch_loss) {
      // the one host round trip of an epoch
      double ep_loss = 0.0;
      HIP_TRY(hipMemcpyAsync(&ep_loss, d_ep_loss, sizeof ep_loss, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      h_epoch_loss[ep] = (float)(ep_loss / std::max<uint64_t>(1, n_batches));
    }
  }
  if (d_hdr) {
    hdr[0] = step;
    hdr[1] += t->epochs;
    HIP_TRY(hipMemcpyAsync(d_hdr, hdr, sizeof hdr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return BVS_OK;
}

}  // namespace

extern "C" {

bvs_status bvs_mlp_weight_count(uint32_t dim, uint32_t hidden, uint32_t code_bits, uint64_t* out) {
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  BVS_TRY(check_mlp_shape(dim, hidden, code_bits));
  *out = mlp_floats(dim, hidden, code_bits);
  return BVS_OK;
}

bvs_status bvs_mlp_init(uint32_t dim, uint32_t hidden, uint32_t code_bits, uint64_t seed, float* d_weights,
                        void* stream) {
  BVS_TRY(check_mlp_shape(dim, hidden, code_bits));
  if (!d_weights) return fail(BVS_EINVAL, "weights are NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_mlp_init(d_weights, dim, hidden, code_bits, seed, st));
  HIP_TRY(hipStreamSynchronize(st));
  return BVS_OK;
}

bvs_status bvs_learned_index_bytes(const bvs_params* p, uint32_t hidden, uint64_t n_sets, uint64_t n_vectors,
                                   uint64_t* out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  BVS_TRY(check_mlp_shape(g.d, hidden, g.L));
  Carver c(nullptr);
  bvs_index tmp;
  layout_index(c, g, n_sets, n_vectors, &tmp);
  layout_learned_weights(c, g, hidden, &tmp);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_learned_build_workspace_bytes(const bvs_params* p, uint32_t hidden, uint64_t n_sets,
                                             uint64_t n_vectors, uint64_t* out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  BVS_TRY(check_mlp_shape(g.d, hidden, g.L));
  const uint64_t rows = std::min<uint64_t>(std::max<uint64_t>(n_vectors, 1), kLearnChunkRows + 256);
  Carver c(nullptr);
  c.take<uint32_t>(4);
  c.take<uint8_t>(n_sets * g.L);
  c.take<uint64_t>(n_sets * g.R);
  c.take<uint16_t>(rows * g.d);
  c.take<uint16_t>(rows * hidden);
  c.take<float>(rows * g.L);
  c.take<uint64_t>(rows * g.R);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_build_index_learned(const bvs_params* p, uint32_t hidden, const float* d_weights,
                                   const float* d_vectors, const uint64_t* h_offsets, uint64_t n_sets,
                                   void* d_index_mem, uint64_t index_bytes, void* d_ws, uint64_t ws_bytes,
                                   void* stream, bvs_index** out) {
  Geometry g;
  BVS_TRY(derive(p, &g));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  *out = nullptr;
  BVS_TRY(check_mlp_shape(g.d, hidden, g.L));
  if (!d_weights) return fail(BVS_EINVAL, "weights are NULL");
  if (n_sets == 0) return fail(BVS_EINVAL, "n_sets must be positive");
  if (n_sets >= 0xFFFFFFFFull) return fail(BVS_ENOTSUP, "n_sets must be below 2^32 - 1");
  if (!d_vectors) return fail(BVS_EINVAL, "vectors are NULL");
  uint32_t max_m = 0;
  BVS_TRY(check_offsets(h_offsets, n_sets, 255, "database", &max_m));
  const uint64_t N = h_offsets[n_sets];
  uint64_t need = 0, wneed = 0;
  BVS_TRY(bvs_learned_index_bytes(p, hidden, n_sets, N, &need));
  BVS_TRY(bvs_learned_build_workspace_bytes(p, hidden, n_sets, N, &wneed));
  if (!d_index_mem) return fail(BVS_EINVAL, "index memory is NULL");
  if (index_bytes < need)
    return fail(BVS_ENOSPC, "index memory of %llu bytes, %llu needed", (unsigned long long)index_bytes,
                (unsigned long long)need);
  BVS_TRY(need_ws(ws_bytes, wneed, d_ws));
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<bvs_index> ix(new bvs_index());
  ix->p = *p;
  ix->g = g;
  ix->n = n_sets;
  ix->N = N;
  ix->max_m = max_m;
  if (hipGetDevice(&ix->device) != hipSuccess) ix->device = 0;
  ix->n_cu = device_cus(ix->device);
  Carver c(d_index_mem);
  layout_index(c, g, n_sets, N, ix.get());
  layout_learned_weights(c, g, hidden, ix.get());
  ix->learned = true;
  ix->hidden = hidden;
  const uint64_t rows_cap = std::min<uint64_t>(std::max<uint64_t>(N, 1), kLearnChunkRows + 256);
  Carver wc(d_ws);
  uint32_t* status = wc.take<uint32_t>(4);
  uint8_t* cnt_rm = wc.take<uint8_t>(n_sets * g.L);
  uint64_t* bits_rm = wc.take<uint64_t>(n_sets * g.R);
  uint16_t* x16 = wc.take<uint16_t>(rows_cap * g.d);
  uint16_t* h16 = wc.take<uint16_t>(rows_cap * hidden);
  float* y = wc.take<float>(rows_cap * g.L);
  uint64_t* codes = wc.take<uint64_t>(rows_cap * g.R);
  const uint64_t nw = mlp_floats(g.d, hidden, g.L);
  auto run = [&]() -> bvs_status {
    HIP_TRY(hipMemcpyAsync(ix->offsets, h_offsets, (n_sets + 1) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_f32_to_bf16(d_weights, nw, ix->w16, st));
    HIP_TRY(hipMemcpyAsync(ix->b1, d_weights + (uint64_t)hidden * g.d, (uint64_t)hidden * 4,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(ix->b2, d_weights + (uint64_t)hidden * g.d + hidden + (uint64_t)g.L * hidden,
                           (uint64_t)g.L * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_fill_u32(status, 4, 0, st));
    HIP_TRY(launch_convert(d_vectors, N, g.d, g.dp, ix->hi, ix->lo, ix->norms, ix->scr, status, ix->n_cu, st));
    // codes and set sketches, a chunk of whole sets at a time
    uint64_t s0 = 0;
    while (s0 < n_sets) {
      uint64_t s1 = s0;
      while (s1 < n_sets && h_offsets[s1 + 1] - h_offsets[s0] <= rows_cap) ++s1;
      const uint64_t r0 = h_offsets[s0], nr = h_offsets[s1] - r0;
      HIP_TRY(encode_planes(ix.get(), ix->hi + r0 * g.dp, ix->lo + r0 * g.dp, nr, codes, x16, h16, y, st));
      HIP_TRY(launch_sets_from_codes(codes, ix->offsets, r0, s0, s1 - s0, g.R, cnt_rm, bits_rm, st));
      s0 = s1;
    }
    HIP_TRY(launch_transpose_sketches(cnt_rm, bits_rm, n_sets, ix->ld, g.L, ix->cnt, ix->bits, st));
    HIP_TRY(launch_bitmap_planes(ix->cnt, ix->ld, g.L, ix->planes, st));
    HIP_TRY(launch_set_weight(ix->bits, g.L / 128, ix->ld, ix->spop, st));
    return read_status(status, st, "database");
  };
  const bvs_status s = run();
  if (s != BVS_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  *out = ix.release();
  return BVS_OK;
}

bvs_status bvs_train_workspace_bytes(const bvs_train_config* t, uint64_t max_batch_rows, uint64_t* out) {
  BVS_TRY(check_train_config(t));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  Carver c(nullptr);
  TrainWs w;
  layout_train(c, *t, std::max<uint64_t>(max_batch_rows, 1), &w);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_train_gradients(const bvs_train_config* t, const float* d_vectors, const uint64_t* h_offsets,
                               uint64_t n_sets, const uint32_t* h_triplets, uint32_t n_triplets,
                               const float* d_weights, float* d_grads, float* h_loss, void* d_ws, uint64_t ws_bytes,
                               void* stream) {
  BVS_TRY(check_train_config(t));
  if (!d_vectors || !d_weights || !d_grads || !h_triplets) return fail(BVS_EINVAL, "NULL argument");
  if (n_triplets == 0 || n_triplets > t->batch_triplets)
    return fail(BVS_EINVAL, "n_triplets must be in 1..batch_triplets");
  uint32_t max_m = 0;
  BVS_TRY(check_offsets(h_offsets, n_sets, 65535, "training", &max_m));
  const uint64_t cap = train_capacity(*t, ws_bytes);
  if (!d_ws || cap == 0) return fail(BVS_ENOSPC, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  TrainWs w;
  layout_train(c, *t, cap, &w);
  const uint64_t nw = mlp_floats(t->dim, t->hidden, t->code_bits);
  TrainStage hs;
  HIP_TRY(hs.alloc(cap, t->batch_triplets));
  HIP_TRY(launch_f32_to_bf16(d_weights, nw, w.w16, st));
  BVS_TRY(train_batch(*t, d_vectors, h_offsets, n_sets, h_triplets, n_triplets, cap, w.w16, d_weights, w, st, hs));
  HIP_TRY(hipMemcpyAsync(d_grads, w.grad, nw * 4, hipMemcpyDeviceToDevice, st));
  float l = 0.f;
  HIP_TRY(hipMemcpyAsync(&l, w.loss, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h_loss) *h_loss = l;
  return BVS_OK;
}

bvs_status bvs_train_projection(const bvs_train_config* t, const float* d_vectors, const uint64_t* h_offsets,
                                uint64_t n_sets, const uint32_t* h_triplets, uint64_t n_triplets, float* d_weights,
                                void* d_ws, uint64_t ws_bytes, float* h_epoch_loss, void* stream) {
  return train_impl(t, d_vectors, h_offsets, n_sets, h_triplets, n_triplets, d_weights, nullptr, d_ws, ws_bytes,
                    h_epoch_loss, (hipStream_t)stream);
}

bvs_status bvs_train_state_bytes(const bvs_train_config* t, uint64_t* out) {
  BVS_TRY(check_train_config(t));
  if (!out) return fail(BVS_EINVAL, "out is NULL");
  *out = train_state_header(*t) + 256;
  return BVS_OK;
}

bvs_status bvs_train_state_init(const bvs_train_config* t, void* d_state, void* stream) {
  BVS_TRY(check_train_config(t));
  if (!d_state) return fail(BVS_EINVAL, "state is NULL");
  uint64_t bytes = 0;
  BVS_TRY(bvs_train_state_bytes(t, &bytes));
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_fill_u32((uint32_t*)d_state, bytes / 4, 0u, st));
  HIP_TRY(hipStreamSynchronize(st));
  return BVS_OK;
}

bvs_status bvs_train_projection_resume(const bvs_train_config* t, const float* d_vectors, const uint64_t* h_offsets,
                                       uint64_t n_sets, const uint32_t* h_triplets, uint64_t n_triplets,
                                       float* d_weights, void* d_state, void* d_ws, uint64_t ws_bytes,
                                       float* h_epoch_loss, void* stream) {
  if (!d_state) return fail(BVS_EINVAL, "state is NULL");
  return train_impl(t, d_vectors, h_offsets, n_sets, h_triplets, n_triplets, d_weights, d_state, d_ws, ws_bytes,
                    h_epoch_loss, (hipStream_t)stream);
}

}  // extern "C"

// ====================================================================== no-allocation search
// bvs_search for callers that cannot allocate: its workspace is a fixed
// array in device memory that the library's code object holds on every GPU
// it runs on, for the life of the process.  Host code never passes the
// array's name to a kernel: the name is a host-side stand-in, so the device
// address of each GPU's copy is looked up once per device and kept.
static constexpr uint64_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device).
bvs_status scratch_for_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(BVS_ENOTSUP, "device %d outside 0..%d", dev,
                                                         kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BVS_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BVS_OK;
}

}  // namespace

extern "C" {

uint64_t bvs_search_noalloc_max_bytes(void) { return kScratchBytes; }

bvs_status bvs_search_noalloc(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                              uint32_t k, uint32_t* d_ids, float* d_dist, uint32_t* d_count, void* stream) {
  uint32_t max_rows = 0;
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, &max_rows));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BVS_EDEVICE, "hipGetDevice failed");
  if (dev != ix->device)
    return fail(BVS_ESTATE, "current device %d is not the index's device %d", dev, ix->device);
  uint64_t need = 0;
  BVS_TRY(bvs_search_workspace_bytes(ix, n_q, h_q_off[n_q], &need));
  if (need > kScratchBytes)
    return fail(BVS_ENOSPC, "search needs %llu bytes of workspace, above the %llu of the no-allocation scratch",
                (unsigned long long)need, (unsigned long long)kScratchBytes);
  void* ws = nullptr;
  BVS_TRY(scratch_for_device(dev, &ws));
  return search_impl(ix, d_q, h_q_off, n_q, k, ws, kScratchBytes, d_ids, d_dist, d_count, (hipStream_t)stream,
                     false);
}

}  // extern "C"

// ====================================================================== full scan (Alg. 2)
namespace {

constexpr uint64_t kFullChunk = 1ull << 20;   // vectors encoded per attach step
constexpr uint32_t kPackCap = 2;              // groups of 64 slots a pack of several queries may fill

uint32_t full_kp(const Geometry& g) { return (uint32_t)align_up(g.wta_k, 8); }

void layout_codes(Carver& c, const bvs_index* ix, uint16_t** pos, uint32_t** order) {
  *pos = c.take<uint16_t>(ix->N * full_kp(ix->g));
  *order = c.take<uint32_t>(ix->n);
}

struct FullWs {
  QueryWs w;
  uint4* packs;      // [n_q] {first query, queries, groups, 0}
  uint64_t* table;   // [n_q][kPackGroups][L] (the first n_packs * GP * L used)
  uint32_t n_packs, GP;
  std::vector<uint32_t> h_packs;
};

void layout_full(Carver& c, const bvs_index* ix, uint32_t n_q, uint64_t NQ, FullWs* f) {
  layout_search(c, ix, n_q, NQ, &f->w);
  f->packs = c.take<uint4>(n_q);
  f->table = c.take<uint64_t>((uint64_t)n_q * kPackGroups * ix->g.L);
}

// Runs of consecutive queries whose vectors fit kPackCap groups of 64 (at most
// kPackQ queries); a query of more than 64 kPackCap vectors takes a pack of
// its own with as many groups as it needs (at most kPackGroups: queries hold
// at most 256 vectors).  GP = the launch's groups per pack (1, 2 or 4).
void make_packs(const uint64_t* h_q_off, uint32_t n_q, FullWs* f) {
  f->h_packs.clear();
  uint32_t q0 = 0, nq = 0;
  uint64_t total = 0;
  uint32_t gmax = 1;
  auto close = [&]() {
    if (!nq) return;
    const uint32_t groups = (uint32_t)((total + 63) / 64);
    gmax = std::max(gmax, groups);
    f->h_packs.insert(f->h_packs.end(), {q0, nq, groups, 0u});
    nq = 0;
    total = 0;
  };
  for (uint32_t q = 0; q < n_q; ++q) {
    const uint64_t m = h_q_off[q + 1] - h_q_off[q];
    if (nq && (nq == (uint32_t)kPackQ || total + m > 64ull * kPackCap)) close();
    if (!nq) q0 = q;
    ++nq;
    total += m;
    if (m > 64ull * kPackCap) close();
  }
  close();
  f->n_packs = (uint32_t)(f->h_packs.size() / 4);
  f->GP = gmax <= 1 ? 1 : gmax <= 2 ? 2 : 4;
}

bvs_status full_ready(const bvs_index* ix) {
  if (!ix->fpos) return fail(BVS_ESTATE, "no codes attached for the full scan (bvs_codes_attach)");
  return BVS_OK;
}

// Upload the pack list (after prepare_queries, on the call's stream; the host
// copy lives in FullWs until the call synchronises).
bvs_status upload_packs(const FullWs& f, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(f.packs, f.h_packs.data(), f.h_packs.size() * 4, hipMemcpyHostToDevice, st));
  return BVS_OK;
}

// Haus^H scores of every set into w.scores, then F = the first T by (score, id).
bvs_status full_filter(const bvs_index* ix, uint32_t n_q, uint64_t NQ, const FullWs& f, uint32_t* ids,
                       uint16_t* scores, uint32_t* count, hipStream_t st, CallProf& prof) {
  const Geometry& g = ix->g;
  const QueryWs& w = f.w;
  if (prof.count) HIP_TRY(launch_fill_u32((uint32_t*)w.stats, 2ull * kStatSlots * kStatCounters, 0, st));
  BVS_TRY(upload_packs(f, st));
  HIP_TRY(staged(prof, S_ENCODE, [&] { return encode_planes(ix, w.qhi, w.qlo, NQ, w.codes, w.lx16, w.lh16, w.ly, st); }));
  HIP_TRY(staged(prof, S_FULLSCAN, [&]() -> hipError_t {
    hipError_t e = launch_query_table(w.codes, w.qoff, f.packs, f.n_packs, g.L, g.R, f.GP, f.table, st);
    if (e != hipSuccess) return e;
    // sets past n (the padding of ld) stay excluded
    e = launch_fill_u32((uint32_t*)w.scores, (uint64_t)n_q * ix->ld / 2, 0xFFFFFFFFu, st);
    if (e != hipSuccess) return e;
    return launch_full_scan(ix->fpos, ix->offsets, ix->forder, ix->n, g.wta_k, ix->fKP, g.L, f.table, w.qoff,
                            f.packs, f.n_packs, f.GP, w.scores, ix->ld, st);
  }));
  HIP_TRY(staged(prof, S_SELECT, [&] {
    return launch_select(w.scores, ix->ld, g.L, g.T, n_q, w.sel, ids, scores, count, nullptr, st);
  }));
  return BVS_OK;
}

// Common prologue of the full-scan calls.
bvs_status full_begin(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, void* d_ws,
                      uint64_t ws_bytes, uint32_t* max_rows, FullWs* f) {
  BVS_TRY(check_queries(ix, d_q, h_q_off, n_q, max_rows));
  BVS_TRY(full_ready(ix));
  const uint64_t NQ = h_q_off[n_q];
  uint64_t need = 0;
  BVS_TRY(bvs_search_full_workspace_bytes(ix, n_q, NQ, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  Carver c(d_ws);
  layout_full(c, ix, n_q, NQ, f);
  make_packs(h_q_off, n_q, f);
  return BVS_OK;
}


}  // namespace

extern "C" {

bvs_status bvs_codes_bytes(const bvs_index* ix, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  uint16_t* p;
  uint32_t* o;
  layout_codes(c, ix, &p, &o);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_codes_attach_workspace_bytes(const bvs_index* ix, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  const uint64_t rows = std::max<uint64_t>(1, std::min<uint64_t>(ix->N, kFullChunk));
  Carver c(nullptr);
  c.take<uint64_t>(rows * ix->g.R);
  if (ix->learned) {
    c.take<uint16_t>(rows * ix->g.d);
    c.take<uint16_t>(rows * ix->hidden);
    c.take<float>(rows * ix->g.L);
  }
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_codes_attach(bvs_index* ix, void* d_mem, uint64_t bytes, void* d_ws, uint64_t ws_bytes, void* stream) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (ix->g.wta_k > 255) return fail(BVS_ENOTSUP, "the full scan counts overlaps of up to 255 positions (wta_k %u)",
                                     ix->g.wta_k);
  uint64_t need = 0, wneed = 0;
  BVS_TRY(bvs_codes_bytes(ix, &need));
  BVS_TRY(bvs_codes_attach_workspace_bytes(ix, &wneed));
  if (!d_mem) return fail(BVS_EINVAL, "code memory is NULL");
  if (bytes < need)
    return fail(BVS_ENOSPC, "code memory of %llu bytes, %llu needed", (unsigned long long)bytes,
                (unsigned long long)need);
  BVS_TRY(need_ws(ws_bytes, wneed, d_ws));
  hipStream_t st = (hipStream_t)stream;
  const Geometry& g = ix->g;
  const uint32_t KP = full_kp(g);
  Carver c(d_mem);
  uint16_t* pos;
  uint32_t* order;
  layout_codes(c, ix, &pos, &order);
  // sets by decreasing size, ties to the lower id (counting sort on the host)
  std::vector<uint64_t> off(ix->n + 1);
  HIP_TRY(hipMemcpyAsync(off.data(), ix->offsets, off.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<uint64_t> start(257, 0);
  for (uint64_t j = 0; j < ix->n; ++j) ++start[255 - (off[j + 1] - off[j]) + 1];
  for (int b = 1; b <= 256; ++b) start[b] += start[b - 1];
  std::vector<uint32_t> ord(ix->n);
  for (uint64_t j = 0; j < ix->n; ++j) ord[start[255 - (off[j + 1] - off[j])]++] = (uint32_t)j;
  HIP_TRY(hipMemcpyAsync(order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice, st));
  Carver wc(d_ws);
  const uint64_t rows = std::max<uint64_t>(1, std::min<uint64_t>(ix->N, kFullChunk));
  uint64_t* codes = wc.take<uint64_t>(rows * g.R);
  uint16_t* x16 = ix->learned ? wc.take<uint16_t>(rows * g.d) : nullptr;
  uint16_t* h16 = ix->learned ? wc.take<uint16_t>(rows * ix->hidden) : nullptr;
  float* y = ix->learned ? wc.take<float>(rows * g.L) : nullptr;
  for (uint64_t r0 = 0; r0 < ix->N; r0 += rows) {
    const uint64_t nr = std::min<uint64_t>(rows, ix->N - r0);
    HIP_TRY(encode_planes(ix, ix->hi + r0 * g.dp, ix->lo + r0 * g.dp, nr, codes, x16, h16, y, st));
    HIP_TRY(launch_code_positions(codes, nr, g.R, g.wta_k, KP, pos + r0 * KP, ix->n_cu, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  ix->fpos = pos;
  ix->forder = order;
  ix->fKP = KP;
  return BVS_OK;
}

bvs_status bvs_search_full_workspace_bytes(const bvs_index* ix, uint32_t n_q, uint64_t n_q_vectors, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  FullWs f;
  layout_full(c, ix, n_q, n_q_vectors, &f);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_full_scores(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, void* d_ws,
                           uint64_t ws_bytes, uint16_t* d_scores, void* stream) {
  if (!d_scores) return fail(BVS_EINVAL, "NULL output");
  uint32_t max_rows = 0;
  FullWs f;
  BVS_TRY(full_begin(ix, d_q, h_q_off, n_q, d_ws, ws_bytes, &max_rows, &f));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t NQ = h_q_off[n_q];
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, f.w, st, prof));
  HIP_TRY(staged(prof, S_ENCODE,
                 [&] { return encode_planes(ix, f.w.qhi, f.w.qlo, NQ, f.w.codes, f.w.lx16, f.w.lh16, f.w.ly, st); }));
  BVS_TRY(upload_packs(f, st));
  HIP_TRY(staged(prof, S_FULLSCAN, [&]() -> hipError_t {
    hipError_t e = launch_query_table(f.w.codes, f.w.qoff, f.packs, f.n_packs, ix->g.L, ix->g.R, f.GP, f.table, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32((uint32_t*)f.w.scores, (uint64_t)n_q * ix->ld / 2, 0xFFFFFFFFu, st);
    if (e != hipSuccess) return e;
    return launch_full_scan(ix->fpos, ix->offsets, ix->forder, ix->n, ix->g.wta_k, ix->fKP, ix->g.L, f.table,
                            f.w.qoff, f.packs, f.n_packs, f.GP, f.w.scores, ix->ld, st);
  }));
  for (uint32_t q = 0; q < n_q; ++q)
    HIP_TRY(hipMemcpyAsync(d_scores + (uint64_t)q * ix->n, f.w.scores + (uint64_t)q * ix->ld, ix->n * 2,
                           hipMemcpyDeviceToDevice, st));
  const bvs_status s = read_status(f.w.status, st, "queries");
  prof.finish();
  return s;
}

bvs_status bvs_search_full_candidates(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q,
                                      void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, uint16_t* d_scores,
                                      uint32_t* d_count, void* stream) {
  if (!d_ids || !d_scores || !d_count) return fail(BVS_EINVAL, "NULL output");
  uint32_t max_rows = 0;
  FullWs f;
  BVS_TRY(full_begin(ix, d_q, h_q_off, n_q, d_ws, ws_bytes, &max_rows, &f));
  hipStream_t st = (hipStream_t)stream;
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, f.w, st, prof));
  BVS_TRY(full_filter(ix, n_q, h_q_off[n_q], f, d_ids, d_scores, d_count, st, prof));
  const bvs_status s = read_status(f.w.status, st, "queries");
  prof.finish();
  return s;
}

bvs_status bvs_search_full(const bvs_index* ix, const float* d_q, const uint64_t* h_q_off, uint32_t n_q, uint32_t k,
                           void* d_ws, uint64_t ws_bytes, uint32_t* d_ids, float* d_dist, uint32_t* d_count,
                           void* stream) {
  if (!d_ids || !d_dist || !d_count) return fail(BVS_EINVAL, "NULL output");
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (k < 1 || k > kMaxK || k > ix->g.T) return fail(BVS_EINVAL, "k %u outside 1..min(64, top_t)", k);
  uint32_t max_rows = 0;
  FullWs f;
  BVS_TRY(full_begin(ix, d_q, h_q_off, n_q, d_ws, ws_bytes, &max_rows, &f));
  hipStream_t st = (hipStream_t)stream;
  const QueryWs& w = f.w;
  CallProf prof(st);
  BVS_TRY(prepare_queries(ix, d_q, h_q_off, n_q, w, st, prof));
  BVS_TRY(full_filter(ix, n_q, h_q_off[n_q], f, w.f2_ids, w.f2_scores, w.f2_count, st, prof));
  HIP_TRY(staged(prof, S_RERANK, [&] {
    return launch_haus_cand(haus_db(ix), haus_q(w, n_q, max_rows), w.f2_ids, w.f2_count, ix->g.T, k, w.thr, w.h2,
                            prof.count ? w.stats : nullptr, w.surv, w.surv_count, st);
  }));
  HIP_TRY(staged(prof, S_TOPK, [&] {
    return launch_topk(w.h2, w.f2_ids, w.f2_count, ix->g.T, ix->g.T, n_q, k, w.topk_tmp, d_ids, d_dist, d_count, st);
  }));
  const bvs_status s = read_status(w.status, st, "queries");
  prof.finish(prof.count ? w.stats : nullptr);
  return s;
}

}  // extern "C"

// ====================================================================== inverted lists (Def. 9, Alg. 4)
namespace {

struct ListWs {
  uint32_t* hist;
  uint32_t* cursor;
  uint64_t* len;
  uint32_t* cum;     // counting pass only
  uint64_t* start;   // counting pass only
};

void layout_list_ws(Carver& c, const bvs_index* ix, ListWs* w) {
  const uint32_t L = ix->g.L;
  w->hist = c.take<uint32_t>((uint64_t)L * 256);
  w->cursor = c.take<uint32_t>((uint64_t)L * 256);
  w->len = c.take<uint64_t>(L);
  w->cum = c.take<uint32_t>((uint64_t)L * 257);
  w->start = c.take<uint64_t>(L + 1ull);
}

void layout_lists(Carver& c, const bvs_index* ix, uint64_t nnz, uint32_t** cum, uint64_t** start, uint32_t** ids) {
  *cum = c.take<uint32_t>((uint64_t)ix->g.L * 257);
  *start = c.take<uint64_t>(ix->g.L + 1ull);
  *ids = c.take<uint32_t>(nnz);
}

}  // namespace

extern "C" {

bvs_status bvs_lists_workspace_bytes(const bvs_index* ix, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  Carver c(nullptr);
  ListWs w;
  layout_list_ws(c, ix, &w);
  *out = align_up(c.off, 256);
  return BVS_OK;
}

bvs_status bvs_lists_bytes(const bvs_index* ix, void* d_ws, uint64_t ws_bytes, void* stream, uint64_t* out) {
  if (!ix || !out) return fail(BVS_EINVAL, "NULL argument");
  uint64_t need = 0;
  BVS_TRY(bvs_lists_workspace_bytes(ix, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  ListWs w;
  layout_list_ws(c, ix, &w);
  HIP_TRY(launch_list_build(ix->cnt, ix->ld, ix->n, ix->g.L, w.hist, w.cursor, w.len, w.cum, w.start, nullptr, st,
                            false));
  uint64_t nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, w.start + ix->g.L, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  Carver m(nullptr);
  uint32_t* a;
  uint64_t* b;
  uint32_t* d;
  layout_lists(m, ix, nnz, &a, &b, &d);
  *out = align_up(m.off, 256);
  return BVS_OK;
}

bvs_status bvs_lists_attach(bvs_index* ix, void* d_mem, uint64_t bytes, void* d_ws, uint64_t ws_bytes, void* stream) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (!d_mem) return fail(BVS_EINVAL, "list memory is NULL");
  uint64_t need = 0;
  BVS_TRY(bvs_lists_workspace_bytes(ix, &need));
  BVS_TRY(need_ws(ws_bytes, need, d_ws));
  hipStream_t st = (hipStream_t)stream;
  Carver c(d_ws);
  ListWs w;
  layout_list_ws(c, ix, &w);
  // counting pass straight into the list memory's head (its layout does not
  // depend on nnz), then the fill
  Carver m(d_mem);
  uint32_t* cum;
  uint64_t* start;
  uint32_t* ids;
  layout_lists(m, ix, 0, &cum, &start, &ids);
  const uint64_t head = align_up(m.off, 256);
  if (bytes < head) return fail(BVS_ENOSPC, "list memory of %llu bytes, more needed", (unsigned long long)bytes);
  HIP_TRY(launch_list_build(ix->cnt, ix->ld, ix->n, ix->g.L, w.hist, w.cursor, w.len, cum, start, nullptr, st,
                            false));
  uint64_t nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, start + ix->g.L, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  Carver m2(d_mem);
  layout_lists(m2, ix, nnz, &cum, &start, &ids);
  if (bytes < align_up(m2.off, 256))
    return fail(BVS_ENOSPC, "list memory of %llu bytes, %llu needed", (unsigned long long)bytes,
                (unsigned long long)align_up(m2.off, 256));
  HIP_TRY(launch_list_build(ix->cnt, ix->ld, ix->n, ix->g.L, w.hist, w.cursor, w.len, cum, start, ids, st, true));
  HIP_TRY(hipStreamSynchronize(st));
  ix->lcum = cum;
  ix->lstart = start;
  ix->lids = ids;
  ix->lnnz = nnz;
  return BVS_OK;
}

bvs_status bvs_lists_views(const bvs_index* ix, const uint32_t** d_cum, const uint64_t** d_start,
                           const uint32_t** d_ids, uint64_t* nnz) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (!ix->lids) return fail(BVS_ESTATE, "no inverted lists attached (bvs_lists_attach)");
  if (d_cum) *d_cum = ix->lcum;
  if (d_start) *d_start = ix->lstart;
  if (d_ids) *d_ids = ix->lids;
  if (nnz) *nnz = ix->lnnz;
  return BVS_OK;
}

bvs_status bvs_index_set_first_layer(bvs_index* ix, int mode) {
  if (!ix) return fail(BVS_EINVAL, "index is NULL");
  if (mode != BVS_FIRST_LAYER_BITMAPS && mode != BVS_FIRST_LAYER_LISTS)
    return fail(BVS_EINVAL, "unknown first-layer mode %d", mode);
  if (mode == BVS_FIRST_LAYER_LISTS && !ix->lids)
    return fail(BVS_ESTATE, "no inverted lists attached (bvs_lists_attach)");
  ix->first_layer = mode;
  return BVS_OK;
}

}  // extern "C"
