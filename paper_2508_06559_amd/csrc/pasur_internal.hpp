// pasur_internal.hpp -- internals shared by the HIP translation units of
// libpasur (gfx950).  Not part of the public ABI (include/pasur.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cmath>
#include <cstdio>

#include "../../include/pasur.h"

namespace pasur {

void set_error(const char *fmt, ...);

#define PASUR_TRY_HIP(expr)                                                   \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::pasur::set_error("%s failed: %s", #expr, hipGetErrorString(e_));      \
      return PASUR_E_HIP;                                                     \
    }                                                                         \
  } while (0)

#define PASUR_TRY(expr)                                                       \
  do {                                                                        \
    int s_ = (expr);                                                          \
    if (s_ != PASUR_OK) return s_;                                            \
  } while (0)

template <class T>
int dev_alloc(T **p, int64_t n) {
  *p = nullptr;
  size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(T);
  hipError_t e = hipMalloc((void **)p, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    *p = nullptr;
    return PASUR_E_NOMEM;
  }
  return PASUR_OK;
}

template <class T>
void dev_free(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Exclusive scan of n int32 counts into out[0..n] (out[n] = total); the
// total is returned through *total (synchronises `stream`).  Fails with
// PASUR_E_OVERFLOW when the total exceeds INT32_MAX.
int scan_counts(const int32_t *d_counts, int64_t n, int32_t *d_out,
                int64_t *total, hipStream_t stream);

// Stable LSD radix sort of (key, value) pairs by key; every key bit at or
// above end_bit must be zero.  The result is in keys_out/vals_out, and
// keys/vals are overwritten.  Synchronises `stream`.
template <class K>
int radix_sort_pairs(K *keys, K *keys_out, int32_t *vals, int32_t *vals_out, int64_t n,
                     int end_bit, hipStream_t stream);

// Bit masks over the 52 card indices.
constexpr uint64_t kNumericMask = (1ull << 40) - 1;       // A..10, 40 cards
constexpr uint64_t kJackMask = 0xFull << 40;
constexpr uint64_t kClubMask = 0x0001111111111111ull;      // every 4th card
constexpr uint64_t kAllCards = (1ull << 52) - 1;

// 16-bit score key ordered by (bonus, ca, cb, d): bonus 2 bits, ca and cb
// 3 bits each (0..6 while the bonus is undecided, else 0), d + 128 8 bits.
__host__ __device__ inline uint32_t score_key(int ca, int cb, int d, int bonus) {
  return ((uint32_t)bonus << 14) | ((uint32_t)ca << 11) | ((uint32_t)cb << 8) |
         (uint32_t)(d + 128);
}
__host__ __device__ inline void score_unkey(uint32_t k, int *ca, int *cb,
                                            int *d, int *bonus) {
  *bonus = (int)((k >> 14) & 3);
  *ca = (int)((k >> 11) & 7);
  *cb = (int)((k >> 8) & 7);
  *d = (int)(k & 0xFF) - 128;
}

// Sampling shared by self-play and external-sampling CFR.
// The i-th output of SplitMix64 started at `seed` (its state after i + 1
// steps, through the generator's finaliser), as a double in [0, 1).
__device__ inline double splitmix_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Index of the sampled child among k (k >= 2) whose strategy is prob(0..k-1)
// (any accessor returning a child's probability): the first whose running
// sum (FP64, in child order) exceeds u * total; uniform choice when the
// policy is uniform or the total is 0.
template <class Prob>
__device__ __forceinline__ int choose_by(double u, int k, int policy, const Prob &prob) {
  const int uni = min((int)(u * (double)k), k - 1);
  if (policy == PASUR_PLAY_UNIFORM) return uni;
  double total = 0.0;
  for (int c = 0; c < k; ++c) total += prob(c);
  if (!(total > 0.0)) return uni;
  const double x = u * total;
  double acc = 0.0;
  int last = 0;
  for (int c = 0; c < k; ++c) {
    const double pc = prob(c);
    acc += pc;
    if (pc > 0.0) last = c;
    if (acc > x) return c;
  }
  return last;
}

// choose_by over a contiguous array p[0..k-1].
template <class T>
__device__ inline int choose(double u, const T *__restrict__ p, int k, int policy) {
  return choose_by(u, k, policy, [p](int c) { return (double)p[c]; });
}


// ---- DCFR iteration constants (computed on the host so that FP64 results
// stay bit-exact) --------------------------------------------------------------
struct IterConsts {
  double dpos, dneg;  // DCFR discounts for R > 0 and R <= 0
  double avg_w;       // weight of the previous average-strategy sum
  double avg_t;       // multiplier of the new term (t for CFR+, else 1)
  double eps;
  int variant, rm_mode;
  int flags;  // pasur_cfr_flags (DCFR only)
};

struct IterK {
  double dpos, dneg, avg_w, avg_t;
};

inline IterConsts consts_for(const pasur_cfr_params *p, int64_t t) {
  IterConsts ic;
  const double tm1 = (double)(t - 1);
  double pa = std::pow(tm1, p->alpha);
  double pb = std::pow(tm1, p->beta);
  ic.dpos = pa / (pa + 1.0);
  ic.dneg = pb / (pb + 1.0);
  if (p->variant != PASUR_DCFR)
    ic.avg_w = 1.0;
  else if (p->flags & PASUR_CFR_SNIPPET_AVG)
    ic.avg_w = 1.0 - 1.0 / std::pow((double)t, p->gamma);
  else
    ic.avg_w = std::pow(tm1 / (double)t, p->gamma);
  ic.avg_t = (double)t;
  ic.eps = p->eps;
  ic.variant = p->variant;
  ic.rm_mode = p->rm_mode;
  ic.flags = p->flags;
  return ic;
}

inline IterK iter_k(const pasur_cfr_params *p, int64_t t) {
  const IterConsts ic = consts_for(p, t);
  return IterK{ic.dpos, ic.dneg, ic.avg_w, ic.avg_t};
}

// ---- wave-level helpers of the chunked up sweeps ----------------------------
// The value of lane i-1 (lane_from_below) or lane i+1 (lane_from_above) of
// the wave, by a DPP whole-wave shift; lane 0 (resp. 63) receives 0.
__device__ __forceinline__ double lane_from_below(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_above(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0x130, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of v over each sibling group of the wave (the group's lanes are
// consecutive; pos = index within the group, k = group size), added in
// sibling order from 0.0 exactly as the sequential loop does, and returned
// on every lane of the group.  Each step moves values one lane; the steps
// stop once no lane of the wave needs another (kw = largest group of the
// wave).  Must run with all lanes of the wave active.
__device__ __forceinline__ double group_sum(double v, int pos, int k, int kw) {
  double acc = 0.0 + v;
  for (int s = 1; s < kw; ++s) {
    const double prev = lane_from_below(acc);
    acc = pos == s ? prev + v : acc;
  }
  for (int s = 1; s < kw; ++s) {
    const double next = lane_from_above(acc);
    acc = k - 1 - pos == s ? next : acc;
  }
  return acc;
}

// Largest value of x over the wave (x >= 0), as a wave-uniform scalar.
__device__ __forceinline__ int wave_max(int x) {
  int m = x;
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x111, 0xF, 0xF, false));  // row_shr:1
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x112, 0xF, 0xF, false));  // row_shr:2
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x114, 0xF, 0xF, false));  // row_shr:4
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x118, 0xF, 0xF, false));  // row_shr:8
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x142, 0xF, 0xF, false));  // row_bcast:15
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x143, 0xF, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(m, 63);
}

// ---- optional per-launch timing (pasur_profile_enable) ------------------------
struct ProfRec {
  int kernel, level;
  int64_t work[5];  // kernel-specific work counts (edges, parents, roots, ..., iterations)
  hipEvent_t a, b;
};
bool prof_on(int kernel);
void prof_push(const ProfRec &r);
void prof_events(hipEvent_t *a, hipEvent_t *b);  // two events from the pool

// Records HIP events around the launches made in its scope when profiling is on.
struct ProfScope {
  ProfRec rec;
  hipStream_t s;
  bool on;
  ProfScope(int kernel, int level, hipStream_t stream, int64_t w0 = 0, int64_t w1 = 0,
            int64_t w2 = 0, int64_t w3 = 0, int64_t w4 = 1)
      : s(stream), on(prof_on(kernel)) {
    if (!on) return;
    rec.kernel = kernel;
    rec.level = level;
    rec.work[0] = w0;
    rec.work[1] = w1;
    rec.work[2] = w2;
    rec.work[3] = w3;
    rec.work[4] = w4;
    prof_events(&rec.a, &rec.b);
    (void)hipEventRecord(rec.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.b, s);
    prof_push(rec);
  }
};

// ---- HBM-streaming schedule (pasur_sweep.hip) --------------------------------
struct SweepIndex;
void sweep_index_free(SweepIndex *x);
// Iterations t0 .. t0+n_iters-1 of one round with level-wide streaming
// launches (PASUR_SCHED_STREAM); same arguments as pasur_cfr_iterate.
int sweep_iterate(pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p,
                  int64_t t0, int n_iters, hipStream_t s);
// Whether the streaming schedule is expected to beat the persistent segment
// schedule on this round (PASUR_SCHED_AUTO).
bool sweep_pays(const pasur_fgt *f);


}  // namespace pasur

// Round game tree, device arrays per level.
struct pasur_gt {
  int round;
  int64_t n[9];
  uint64_t *pool[9];
  uint8_t *hands[9];
  uint64_t *rs[9];  // 8 signed bytes per node, see PASUR_GT_RS
  int32_t *parent[9];
  int32_t *child_begin[8];
  uint8_t *act_card[9];
  uint64_t *act_cap[9];
  uint8_t deck[52];
};

// Unfolded tree of one round.
struct pasur_fgt {
  int round;
  int64_t n[9];
  int32_t *gt[9];
  int32_t *sid[9];
  int32_t *parent[9];
  int32_t *child_begin[8];
  int64_t n_scores;
  int8_t *score_tab;  // 4 per score: ca, cb, d, bonus
  int64_t n_next;
  pasur_root *next_roots;
  int32_t *link;
  int16_t *leaf_base;
  int8_t *leaf_bonus;  // round 5: the final 7-club bonus state of each leaf
  // root_off[l][j] .. root_off[l][j+1]: level-l nodes of root j's subtree
  // (levels are root-major), on the device and copied to the host
  int64_t n_roots;
  int32_t *root_off[9];
  int32_t *h_root_off;  // 9 * (n_roots + 1), level-major
  // structure index of the streaming schedule, built on first use
  pasur::SweepIndex *sweep;
};
