// pasur_internal.hpp -- internals shared by the HIP translation units of
// libpasur (gfx950).  Not part of the public ABI (include/pasur.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
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
  // root_off[l][j] .. root_off[l][j+1]: level-l nodes of root j's subtree
  // (levels are root-major), on the device and copied to the host
  int64_t n_roots;
  int32_t *root_off[9];
  int32_t *h_root_off;  // 9 * (n_roots + 1), level-major
};
