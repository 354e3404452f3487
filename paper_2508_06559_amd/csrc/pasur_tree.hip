// pasur_tree.hip -- round game tree (move generation), the Unfolding
// Process and the Between-Hand linkage, as level-synchronous HIP kernels.
//
// Every level is laid out count -> exclusive scan -> fill, one thread per
// parent, so children land parent-major in canonical order without atomics.
#include "pasur_internal.hpp"


#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace pasur;

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) {
  return (unsigned)((n + kThreads - 1) / kThreads);
}

__device__ inline int card_value(int c) { return (c >> 2) + 1; }

// Scoring table of section "Pasur": each Ace 1, each Jack 1, the 2 of clubs
// 2, the 10 of diamonds 3.
__device__ inline int points_of(uint64_t m) {
  return __popcll(m & 0xFull) + 2 * (int)((m >> 4) & 1) + 3 * (int)((m >> 37) & 1) +
         __popcll(m & kJackMask);
}

// Mover's hand, ascending by card index.
struct Hand {
  uint8_t card[4];
  uint8_t bit[4];  // hand bit (0..7) of that card
  int k;
};

// Cards dealt to the two players in this round, per hand bit, and for each
// player the order of his 4 hand bits by ascending card index.
struct DealInfo {
  uint8_t card[8];
  uint8_t order[2][4];
};

__device__ inline Hand held_cards(const DealInfo &di, uint8_t hands, int mover) {
  Hand h;
  h.k = 0;
  for (int j = 0; j < 4; ++j) {
    int b = 4 * mover + di.order[mover][j];
    if ((hands >> b) & 1) {
      h.card[h.k] = di.card[b];
      h.bit[h.k] = (uint8_t)b;
      ++h.k;
    }
  }
  return h;
}

// Legal moves of a hand on a pool, in canonical order (card ascending, then
// capture mask ascending), passed to emit(hand slot, card, capture mask).
//  - numeric card: every set of pool numerics whose values complete 11,
//    enumerated in colex order (= ascending mask) by an explicit-stack
//    depth-first search over the pool numerics sorted by index (values are
//    non-decreasing in index, which bounds every frame); no capture -> lay;
//  - Jack: all pool numerics and Jacks, or a lay if there are none;
//  - Queen/King: one capture per same-rank pool card, else a lay.
template <class Emit>
__device__ inline void for_each_move(const Hand &h, uint64_t pool, Emit &&emit) {
  uint8_t num[40];
  int m = 0;
  for (uint64_t pn = pool & kNumericMask; pn; pn &= pn - 1) num[m++] = (uint8_t)(__ffsll((long long)pn) - 1);
  for (int s = 0; s < h.k; ++s) {
    const int c = h.card[s];
    bool found = false;
    if (c < 40) {
      int hh[11], tt[11], lim[11];
      uint64_t acc = 0;
      int d = 0;
      hh[0] = 0;
      tt[0] = 11 - card_value(c);
      lim[0] = m;
      while (true) {
        if (hh[d] >= lim[d]) {
          if (d == 0) break;
          --d;
          acc &= ~(1ull << num[hh[d]]);
          ++hh[d];
          continue;
        }
        const int v = card_value(num[hh[d]]);
        if (v > tt[d]) {  // every later card is at least as large
          hh[d] = lim[d];
          continue;
        }
        if (v == tt[d]) {
          emit(s, c, acc | (1ull << num[hh[d]]));
          found = true;
          ++hh[d];
          continue;
        }
        acc |= 1ull << num[hh[d]];
        lim[d + 1] = hh[d];
        tt[d + 1] = tt[d] - v;
        hh[d + 1] = 0;
        ++d;
      }
    } else if (c < 44) {
      uint64_t cap = pool & (kNumericMask | kJackMask);
      if (cap) {
        emit(s, c, cap);
        found = true;
      }
    } else {
      for (uint64_t cap = pool & (0xFull << (c & ~3)); cap; cap &= cap - 1) {
        emit(s, c, cap & (~cap + 1));
        found = true;
      }
    }
    if (!found) emit(s, c, 0ull);
  }
}

__global__ void k_gt_count(int64_t n, const uint64_t *__restrict__ pool,
                           const uint8_t *__restrict__ hands, DealInfo di, int mover,
                           int32_t *__restrict__ counts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Hand h = held_cards(di, hands[i], mover);
  int cnt = 0;
  for_each_move(h, pool[i], [&](int, int, uint64_t) { ++cnt; });
  counts[i] = cnt;
}

// ApplyActions (and the capture/Sur/clean-up scoring): children of node i
// written at child_begin[i] + j.
__global__ void k_gt_fill(int64_t n, int round, int ply, const uint64_t *__restrict__ pool,
                          const uint8_t *__restrict__ hands, const uint64_t *__restrict__ rs,
                          const int32_t *__restrict__ cb, DealInfo di,
                          uint64_t *__restrict__ c_pool, uint8_t *__restrict__ c_hands,
                          uint64_t *__restrict__ c_rs, int32_t *__restrict__ c_parent,
                          uint8_t *__restrict__ c_card, uint64_t *__restrict__ c_cap) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int mover = ply & 1;
  const uint64_t p0 = pool[i];
  const uint8_t h0 = hands[i];
  const uint64_t r0 = rs[i];
  Hand h = held_cards(di, h0, mover);
  int64_t q = cb[i];
  for_each_move(h, p0, [&](int s, int c, uint64_t cap) {
    uint64_t p = p0;
    int8_t r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (int8_t)((r0 >> (8 * k)) & 0xFF);
    const uint64_t cbit = 1ull << c;
    if (cap == 0) {
      p |= cbit;
    } else {
      const uint64_t taken = cap | cbit;
      r[mover] += (int8_t)__popcll(taken & kClubMask);
      r[3 + 2 * mover] += (int8_t)points_of(taken);
      r[2] = (int8_t)(mover + 1);
      if (cap == p0 && !(c >= 40 && c < 44) && round != 5) r[4 + 2 * mover] += 1;
      p &= ~cap;
    }
    if (round == 5 && ply == 7 && r[2] != 0) {
      const int w = r[2] - 1;
      r[w] += (int8_t)__popcll(p & kClubMask);
      r[3 + 2 * w] += (int8_t)points_of(p);
    }
    uint64_t packed = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) packed |= (uint64_t)(uint8_t)r[k] << (8 * k);
    c_pool[q] = p;
    c_hands[q] = (uint8_t)(h0 & ~(1u << h.bit[s]));
    c_rs[q] = packed;
    c_parent[q] = (int32_t)i;
    c_card[q] = (uint8_t)c;
    c_cap[q] = cap;
    ++q;
  });
}

// Root checks: canonical order (strictly ascending by pool, bonus, ca, cb,
// d), valid scores, pools made of cards dealt before the round, zero pad.
__global__ void k_check_roots(int64_t n, const pasur_root *__restrict__ roots,
                              uint64_t dealt_before, int *__restrict__ bad) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const pasur_root r = roots[j];
  bool ok = (r.pool & ~dealt_before) == 0 && r.pad == 0 && r.bonus >= 0 && r.bonus <= 2;
  ok = ok && (r.bonus == 0 ? (r.ca >= 0 && r.ca <= 6 && r.cb >= 0 && r.cb <= 6)
                           : (r.ca == 0 && r.cb == 0));
  if (ok && j > 0) {
    const pasur_root p = roots[j - 1];
    const uint32_t kp = score_key(p.ca, p.cb, p.d, p.bonus);
    const uint32_t kr = score_key(r.ca, r.cb, r.d, r.bonus);
    ok = r.pool > p.pool || (r.pool == p.pool && kr > kp);
  }
  if (!ok) atomicOr(bad, 1);
}

__global__ void k_pool_flags(int64_t n, const pasur_root *__restrict__ roots,
                             int32_t *__restrict__ flags) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  flags[j] = (j == 0 || roots[j].pool != roots[j - 1].pool) ? 1 : 0;
}

__global__ void k_pool_compact(int64_t n, const pasur_root *__restrict__ roots,
                               const int32_t *__restrict__ flags, const int32_t *__restrict__ pos,
                               uint64_t *__restrict__ pools) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (flags[j]) pools[pos[j]] = roots[j].pool;
}

__global__ void k_gt_root_init(int64_t n, uint8_t *__restrict__ hands, uint64_t *__restrict__ rs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  hands[i] = 0xFF;
  rs[i] = 0;
}

int validate_deck(const uint8_t *deck) {
  if (!deck) {
    set_error("deck is NULL");
    return PASUR_E_INVAL;
  }
  uint64_t seen = 0;
  for (int i = 0; i < 52; ++i) {
    if (deck[i] >= 52 || ((seen >> deck[i]) & 1)) {
      set_error("deck is not a permutation of 0..51 (slot %d)", i);
      return PASUR_E_INVAL;
    }
    seen |= 1ull << deck[i];
  }
  return PASUR_OK;
}

int check_roots(const uint8_t *deck, int round, const pasur_root *d_roots, int64_t n_roots,
                hipStream_t stream) {
  if (!d_roots || n_roots < 1) {
    set_error("need at least one root");
    return PASUR_E_INVAL;
  }
  if (n_roots > INT32_MAX) {
    set_error("too many roots");
    return PASUR_E_OVERFLOW;
  }
  uint64_t dealt = 0;
  for (int i = 0; i < 4 + 8 * round; ++i) dealt |= 1ull << deck[i];
  int *bad = nullptr;
  PASUR_TRY(dev_alloc(&bad, 1));
  int hbad = 0;
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), stream);
  if (e == hipSuccess) {
    k_check_roots<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, d_roots, dealt, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  dev_free(bad);
  if (e != hipSuccess) {
    set_error("root check: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  if (hbad) {
    set_error("roots must be strictly ascending by (pool, bonus, ca, cb, d), hold valid "
              "scores and pools of cards dealt before round %d", round);
    return PASUR_E_INVAL;
  }
  return PASUR_OK;
}

// Distinct pools of the (sorted) roots: flags, positions, count.
int distinct_pools(const pasur_root *d_roots, int64_t n_roots, int32_t **d_pos,
                   int64_t *n_pools, uint64_t *d_pools /* nullable */, hipStream_t stream) {
  int32_t *flags = nullptr;
  PASUR_TRY(dev_alloc(&flags, n_roots));
  int st = dev_alloc(d_pos, n_roots + 1);
  if (st) { dev_free(flags); return st; }
  k_pool_flags<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, d_roots, flags);
  st = scan_counts(flags, n_roots, *d_pos, n_pools, stream);
  if (!st && d_pools) {
    k_pool_compact<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, d_roots, flags, *d_pos,
                                                                d_pools);
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { set_error("pool compaction: %s", hipGetErrorString(e)); st = PASUR_E_HIP; }
  }
  dev_free(flags);
  if (st) dev_free(*d_pos);
  return st;
}

DealInfo deal_info(const uint8_t *deck, int round) {
  DealInfo di;
  for (int b = 0; b < 8; ++b) di.card[b] = deck[4 + 8 * round + b];
  for (int w = 0; w < 2; ++w) {
    int idx[4] = {0, 1, 2, 3};
    std::sort(idx, idx + 4, [&](int a, int b) { return di.card[4 * w + a] < di.card[4 * w + b]; });
    for (int j = 0; j < 4; ++j) di.order[w][j] = (uint8_t)idx[j];
  }
  return di;
}

}  // namespace

extern "C" void pasur_gt_free(pasur_gt *g) {
  if (!g) return;
  for (int l = 0; l < 9; ++l) {
    dev_free(g->pool[l]);
    dev_free(g->hands[l]);
    dev_free(g->rs[l]);
    dev_free(g->parent[l]);
    dev_free(g->act_card[l]);
    dev_free(g->act_cap[l]);
    if (l < 8) dev_free(g->child_begin[l]);
  }
  delete g;
}

extern "C" int pasur_build_round_tree(const uint8_t deck[52], int round,
                                      const pasur_root *d_roots, int64_t n_roots,
                                      pasur_gt **out_gt, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_gt) {
    set_error("out_gt is NULL");
    return PASUR_E_INVAL;
  }
  *out_gt = nullptr;
  if (round < 0 || round > 5) {
    set_error("round %d outside 0..5", round);
    return PASUR_E_RANGE;
  }
  PASUR_TRY(validate_deck(deck));
  PASUR_TRY(check_roots(deck, round, d_roots, n_roots, stream));

  pasur_gt *g = new pasur_gt();
  std::memset(g, 0, sizeof(*g));
  g->round = round;
  std::memcpy(g->deck, deck, 52);
  const DealInfo di = deal_info(deck, round);
  int st = PASUR_OK;
  int32_t *pos = nullptr, *counts = nullptr;
  int64_t n0 = 0;
  // level 0: distinct root pools (ascending because the roots are sorted)
  st = distinct_pools(d_roots, n_roots, &pos, &n0, nullptr, stream);
  if (!st) st = dev_alloc(&g->pool[0], n0);
  if (!st) {
    dev_free(pos);
    st = distinct_pools(d_roots, n_roots, &pos, &n0, g->pool[0], stream);
  }
  dev_free(pos);
  g->n[0] = n0;
  if (!st) st = dev_alloc(&g->hands[0], n0);
  if (!st) st = dev_alloc(&g->rs[0], n0);
  if (!st) {
    k_gt_root_init<<<grid_for(n0), kThreads, 0, stream>>>(n0, g->hands[0], g->rs[0]);
  }
  for (int l = 0; l < 8 && !st; ++l) {
    const int64_t n = g->n[l];
    st = dev_alloc(&counts, n);
    if (!st) st = dev_alloc(&g->child_begin[l], n + 1);
    if (st) break;
    k_gt_count<<<grid_for(n), kThreads, 0, stream>>>(n, g->pool[l], g->hands[l], di, l & 1,
                                                      counts);
    int64_t total = 0;
    st = scan_counts(counts, n, g->child_begin[l], &total, stream);
    dev_free(counts);
    if (st) break;
    const int L = l + 1;
    g->n[L] = total;
    st = dev_alloc(&g->pool[L], total);
    if (!st) st = dev_alloc(&g->hands[L], total);
    if (!st) st = dev_alloc(&g->rs[L], total);
    if (!st) st = dev_alloc(&g->parent[L], total);
    if (!st) st = dev_alloc(&g->act_card[L], total);
    if (!st) st = dev_alloc(&g->act_cap[L], total);
    if (st) break;
    k_gt_fill<<<grid_for(n), kThreads, 0, stream>>>(
        n, round, l, g->pool[l], g->hands[l], g->rs[l], g->child_begin[l], di, g->pool[L],
        g->hands[L], g->rs[L], g->parent[L], g->act_card[L], g->act_cap[L]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("gt fill level %d: %s", l, hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  if (!st) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      set_error("gt build: %s", hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  dev_free(counts);
  if (st) {
    pasur_gt_free(g);
    return st;
  }
  *out_gt = g;
  return PASUR_OK;
}

extern "C" int pasur_gt_sizes(const pasur_gt *gt, int64_t n[9]) {
  if (!gt || !n) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  for (int l = 0; l < 9; ++l) n[l] = gt->n[l];
  return PASUR_OK;
}

extern "C" int pasur_gt_read(const pasur_gt *gt, int field, int level, void *host_dst) {
  if (!gt || !host_dst) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (level < 0 || level > 8) {
    set_error("level %d outside 0..8", level);
    return PASUR_E_RANGE;
  }
  const int64_t n = gt->n[level];
  const void *src = nullptr;
  size_t bytes = 0;
  switch (field) {
    case PASUR_GT_POOL: src = gt->pool[level]; bytes = n * 8; break;
    case PASUR_GT_HANDS: src = gt->hands[level]; bytes = n; break;
    case PASUR_GT_RS: src = gt->rs[level]; bytes = n * 8; break;
    case PASUR_GT_PARENT: src = gt->parent[level]; bytes = n * 4; break;
    case PASUR_GT_CHILD_BEGIN:
      src = level < 8 ? gt->child_begin[level] : nullptr;
      bytes = (n + 1) * 4;
      break;
    case PASUR_GT_ACT_CARD: src = gt->act_card[level]; bytes = n; break;
    case PASUR_GT_ACT_CAP: src = gt->act_cap[level]; bytes = n * 8; break;
    default:
      set_error("unknown GT field %d", field);
      return PASUR_E_RANGE;
  }
  if (!src) {
    set_error("GT field %d does not exist at level %d", field, level);
    return PASUR_E_INVAL;
  }
  PASUR_TRY_HIP(hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
  return PASUR_OK;
}

// --------------------------------------------------------------------------
// Unfolding (section "In-Hand Updates") and Between-Hand linkage
// --------------------------------------------------------------------------
namespace {

__global__ void k_root_keys(int64_t n, const pasur_root *__restrict__ roots,
                            uint32_t *__restrict__ keys) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const pasur_root r = roots[j];
  keys[j] = score_key(r.ca, r.cb, r.d, r.bonus);
}

__global__ void k_key_flags(int64_t n, const uint32_t *__restrict__ keys, int32_t *__restrict__ flags) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  flags[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}

__global__ void k_score_table(int64_t n, const uint32_t *__restrict__ keys,
                              const int32_t *__restrict__ flags, const int32_t *__restrict__ pos,
                              uint32_t *__restrict__ ukeys, int8_t *__restrict__ tab) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || !flags[j]) return;
  int ca, cb, d, bonus;
  score_unkey(keys[j], &ca, &cb, &d, &bonus);
  const int32_t s = pos[j];
  ukeys[s] = keys[j];
  tab[4 * s + 0] = (int8_t)ca;
  tab[4 * s + 1] = (int8_t)cb;
  tab[4 * s + 2] = (int8_t)d;
  tab[4 * s + 3] = (int8_t)bonus;
}

// Per FGT root: its GT root (index of its pool among the distinct pools),
// its score id, and the descendant range [lo, hi) of that GT root on every
// level (a GT subtree is contiguous on each level because levels are
// parent-major).
__global__ void k_root_ranges(int64_t n_roots, const pasur_root *__restrict__ roots,
                              const int32_t *__restrict__ pool_pos, const uint64_t *__restrict__ gt_pool0,
                              const uint32_t *__restrict__ ukeys, int64_t n_scores,
                              const int32_t *const *__restrict__ gt_cb, int32_t *__restrict__ lo,
                              int32_t *__restrict__ hi, int32_t *__restrict__ root_sid,
                              int *__restrict__ bad) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_roots) return;
  const pasur_root r = roots[j];
  const int32_t g = pool_pos[j + 1] - 1;  // inclusive scan of pool-change flags
  if (gt_pool0[g] != r.pool) atomicOr(bad, 1);
  const uint32_t k = score_key(r.ca, r.cb, r.d, r.bonus);
  int64_t a = 0, b = n_scores;
  while (a < b) {
    int64_t m = (a + b) >> 1;
    if (ukeys[m] < k) a = m + 1; else b = m;
  }
  root_sid[j] = (int32_t)a;
  int32_t l0 = g, h0 = g + 1;
  lo[j] = l0;
  hi[j] = h0;
  for (int l = 0; l < 8; ++l) {
    l0 = gt_cb[l][l0];
    h0 = gt_cb[l][h0];
    lo[(int64_t)(l + 1) * n_roots + j] = l0;
    hi[(int64_t)(l + 1) * n_roots + j] = h0;
  }
}

__global__ void k_range_sizes(int64_t n_roots, const int32_t *__restrict__ lo,
                              const int32_t *__restrict__ hi, int32_t *__restrict__ sz) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_roots) return;
  sz[j] = hi[j] - lo[j];
}

// FGT node i of level l: root j (binary search in the level's root offsets),
// GT node, score id, parent and child range.
__global__ void k_fgt_fill(int64_t n, int level, int64_t n_roots, const int32_t *__restrict__ off,
                           const int32_t *__restrict__ off_up, const int32_t *__restrict__ off_dn,
                           const int32_t *__restrict__ lo, const int32_t *__restrict__ lo_up,
                           const int32_t *__restrict__ lo_dn, const int32_t *__restrict__ root_sid,
                           const int32_t *__restrict__ gt_parent, const int32_t *__restrict__ gt_cb,
                           int64_t n_dn, int32_t *__restrict__ f_gt, int32_t *__restrict__ f_sid,
                           int32_t *__restrict__ f_parent, int32_t *__restrict__ f_cb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t a = 0, b = n_roots;  // largest j with off[j] <= i
  while (b - a > 1) {
    int64_t m = (a + b) >> 1;
    if (off[m] <= i) a = m; else b = m;
  }
  // skip empty ranges (cannot happen for a round tree, kept for safety)
  while (a + 1 < n_roots && off[a + 1] <= i) ++a;
  const int64_t j = a;
  const int32_t g = lo[j] + (int32_t)(i - off[j]);
  f_gt[i] = g;
  f_sid[i] = root_sid[j];
  if (level > 0) f_parent[i] = off_up[j] + (gt_parent[g] - lo_up[j]);
  if (level < 8) {
    f_cb[i] = off_dn[j] + (gt_cb[g] - lo_dn[j]);
    if (i == n - 1) f_cb[n] = (int32_t)n_dn;
  }
}

__device__ inline void combine_score(const int8_t *s, uint64_t rs, int *ca, int *cb, int *d,
                                     int *bonus, int *pts) {
  const int acl = (int8_t)(rs & 0xFF), bcl = (int8_t)((rs >> 8) & 0xFF);
  const int apt = (int8_t)((rs >> 24) & 0xFF), asr = (int8_t)((rs >> 32) & 0xFF);
  const int bpt = (int8_t)((rs >> 40) & 0xFF), bsr = (int8_t)((rs >> 48) & 0xFF);
  int a = s[0], b = s[1], dd = s[2], bo = s[3];
  const int p = (apt + 5 * asr) - (bpt + 5 * bsr);
  if (bo == 0) {
    a += acl;
    b += bcl;
  }
  dd += p;
  if (bo == 0 && a >= 7) {
    bo = 1; a = 0; b = 0;
  } else if (bo == 0 && b >= 7) {
    bo = 2; a = 0; b = 0;
  }
  *ca = a; *cb = b; *d = dd; *bonus = bo; *pts = p;
}

// Leaf base utility (equations final_util, passuputil) and, for rounds 0..4,
// the sort key of the leaf's next-round root: the pool compressed to the
// cards dealt so far (order preserving), then the 16-bit score key.
__global__ void k_leaf_pass(int64_t n, int round, const int32_t *__restrict__ f_gt,
                            const int32_t *__restrict__ f_sid, const int8_t *__restrict__ tab,
                            const uint64_t *__restrict__ gt_rs, const uint64_t *__restrict__ gt_pool,
                            uint64_t dealt, int16_t *__restrict__ base,
                            int8_t *__restrict__ bonus_out, uint64_t *__restrict__ keys,
                            int32_t *__restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t t = f_gt[i];
  int ca, cb, d, bonus, pts;
  combine_score(tab + 4 * f_sid[i], gt_rs[t], &ca, &cb, &d, &bonus, &pts);
  if (round == 5) {
    base[i] = (int16_t)((bonus == 1 ? 7 : (bonus == 2 ? -7 : 0)) + pts);
    bonus_out[i] = (int8_t)bonus;
    return;
  }
  base[i] = (int16_t)pts;
  const uint64_t p = gt_pool[t];
  uint64_t cp = 0;
  for (uint64_t m = p; m; m &= m - 1) {
    const int c = __ffsll((long long)m) - 1;
    cp |= 1ull << __popcll(dealt & ((1ull << c) - 1));
  }
  keys[i] = (cp << 16) | score_key(ca, cb, d, bonus);
  idx[i] = (int32_t)i;
}

__global__ void k_u64_flags(int64_t n, const uint64_t *__restrict__ keys, int32_t *__restrict__ flags) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  flags[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}

struct DealtCards {
  uint8_t card[52];  // cards dealt up to the end of the round, ascending
};

__global__ void k_next_roots(int64_t n, const uint64_t *__restrict__ keys,
                             const int32_t *__restrict__ idx, const int32_t *__restrict__ flags,
                             const int32_t *__restrict__ pos, DealtCards dc,
                             pasur_root *__restrict__ next, int32_t *__restrict__ link) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t u = pos[k + 1] - 1;
  link[idx[k]] = u;
  if (!flags[k]) return;
  const uint64_t key = keys[k];
  uint64_t pool = 0;
  for (uint64_t m = key >> 16; m; m &= m - 1) pool |= 1ull << dc.card[__ffsll((long long)m) - 1];
  int ca, cb, d, bonus;
  score_unkey((uint32_t)(key & 0xFFFF), &ca, &cb, &d, &bonus);
  pasur_root r;
  r.pool = pool;
  r.ca = (int8_t)ca;
  r.cb = (int8_t)cb;
  r.d = (int8_t)d;
  r.bonus = (int8_t)bonus;
  r.pad = 0;
  next[u] = r;
}

__global__ void k_iota(int64_t n, int32_t *v) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) v[j] = (int32_t)j;
}

}  // namespace

extern "C" void pasur_fgt_free(pasur_fgt *f) {
  if (!f) return;
  for (int l = 0; l < 9; ++l) {
    dev_free(f->gt[l]);
    dev_free(f->sid[l]);
    dev_free(f->parent[l]);
    if (l < 8) dev_free(f->child_begin[l]);
  }
  dev_free(f->score_tab);
  dev_free(f->next_roots);
  dev_free(f->link);
  dev_free(f->leaf_base);
  dev_free(f->leaf_bonus);
  for (int l = 0; l < 9; ++l) dev_free(f->root_off[l]);
  std::free(f->h_root_off);
  sweep_index_free(f->sweep);
  delete f;
}

namespace {

struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
  template <class T>
  int alloc(T **p, int64_t n) {
    int st = dev_alloc(p, n);
    if (!st) ptrs.push_back((void *)*p);
    return st;
  }
};

int unfold_impl(const pasur_gt *gt, const pasur_root *d_roots, int64_t n_roots, pasur_fgt *f,
                hipStream_t stream) {
  Scratch s;
  // --- score table: distinct root scores, ascending by (bonus, ca, cb, d)
  uint32_t *keys = nullptr, *keys_sorted = nullptr, *ukeys = nullptr;
  int32_t *iv = nullptr, *iv2 = nullptr, *flags = nullptr, *pos = nullptr;
  PASUR_TRY(s.alloc(&keys, n_roots));
  PASUR_TRY(s.alloc(&keys_sorted, n_roots));
  PASUR_TRY(s.alloc(&iv, n_roots));
  PASUR_TRY(s.alloc(&iv2, n_roots));
  PASUR_TRY(s.alloc(&flags, n_roots));
  PASUR_TRY(s.alloc(&pos, n_roots + 1));
  k_root_keys<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, d_roots, keys);
  k_iota<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, iv);
  PASUR_TRY(radix_sort_pairs<uint32_t>(keys, keys_sorted, iv, iv2, n_roots, 16, stream));
  k_key_flags<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, keys_sorted, flags);
  int64_t ns = 0;
  PASUR_TRY(scan_counts(flags, n_roots, pos, &ns, stream));
  f->n_scores = ns;
  PASUR_TRY(dev_alloc(&f->score_tab, 4 * ns));
  PASUR_TRY(s.alloc(&ukeys, ns));
  // pos is exclusive: id of a flagged position k is pos[k]
  k_score_table<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, keys_sorted, flags, pos, ukeys,
                                                            f->score_tab);
  // --- GT root of every FGT root
  int32_t *pool_pos = nullptr;
  int64_t n_pools = 0;
  PASUR_TRY(distinct_pools(d_roots, n_roots, &pool_pos, &n_pools, nullptr, stream));
  s.ptrs.push_back(pool_pos);
  if (n_pools != gt->n[0]) {
    set_error("roots have %lld distinct pools, the game tree %lld roots", (long long)n_pools,
              (long long)gt->n[0]);
    return PASUR_E_INVAL;
  }
  // pool_pos is an exclusive scan of change flags, so pool_pos[j+1]-1 is
  // the distinct-pool index of root j
  int32_t *lo = nullptr, *hi = nullptr, *root_sid = nullptr;
  int *bad = nullptr;
  const int32_t **d_cb = nullptr;
  PASUR_TRY(s.alloc(&lo, 9 * n_roots));
  PASUR_TRY(s.alloc(&hi, 9 * n_roots));
  PASUR_TRY(s.alloc(&root_sid, n_roots));
  PASUR_TRY(s.alloc(&bad, 1));
  PASUR_TRY(s.alloc(&d_cb, 8));
  PASUR_TRY_HIP(hipMemcpyAsync((void *)d_cb, gt->child_begin, 8 * sizeof(int32_t *),
                               hipMemcpyHostToDevice, stream));
  PASUR_TRY_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
  k_root_ranges<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, d_roots, pool_pos,
                                                             gt->pool[0], ukeys, ns, d_cb, lo, hi,
                                                             root_sid, bad);
  int hbad = 0;
  PASUR_TRY_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  PASUR_TRY_HIP(hipStreamSynchronize(stream));
  if (hbad) {
    set_error("root pools do not match the game tree's level 0");
    return PASUR_E_INVAL;
  }
  // --- per level: root offsets
  int32_t **off = f->root_off;
  int32_t *sz = nullptr;
  PASUR_TRY(s.alloc(&sz, n_roots));
  f->n_roots = n_roots;
  for (int l = 0; l <= 8; ++l) {
    PASUR_TRY(dev_alloc(&off[l], n_roots + 1));
    k_range_sizes<<<grid_for(n_roots), kThreads, 0, stream>>>(n_roots, lo + (int64_t)l * n_roots,
                                                              hi + (int64_t)l * n_roots, sz);
    int64_t total = 0;
    PASUR_TRY(scan_counts(sz, n_roots, off[l], &total, stream));
    f->n[l] = total;
  }
  f->h_root_off = (int32_t *)std::malloc(sizeof(int32_t) * 9 * (size_t)(n_roots + 1));
  if (!f->h_root_off) {
    set_error("host allocation failed");
    return PASUR_E_NOMEM;
  }
  for (int l = 0; l <= 8; ++l)
    PASUR_TRY_HIP(hipMemcpy(f->h_root_off + (size_t)l * (n_roots + 1), off[l],
                            sizeof(int32_t) * (n_roots + 1), hipMemcpyDeviceToHost));
  // --- per level: FGT arrays
  for (int l = 0; l <= 8; ++l) {
    const int64_t n = f->n[l];
    PASUR_TRY(dev_alloc(&f->gt[l], n));
    PASUR_TRY(dev_alloc(&f->sid[l], n));
    if (l > 0) PASUR_TRY(dev_alloc(&f->parent[l], n));
    if (l < 8) PASUR_TRY(dev_alloc(&f->child_begin[l], n + 1));
    k_fgt_fill<<<grid_for(n), kThreads, 0, stream>>>(
        n, l, n_roots, off[l], l > 0 ? off[l - 1] : nullptr, l < 8 ? off[l + 1] : nullptr,
        lo + (int64_t)l * n_roots, l > 0 ? lo + (int64_t)(l - 1) * n_roots : nullptr,
        l < 8 ? lo + (int64_t)(l + 1) * n_roots : nullptr, root_sid,
        l > 0 ? gt->parent[l] : nullptr, l < 8 ? gt->child_begin[l] : nullptr,
        l < 8 ? f->n[l + 1] : 0, f->gt[l], f->sid[l], l > 0 ? f->parent[l] : nullptr,
        l < 8 ? f->child_begin[l] : nullptr);
    PASUR_TRY_HIP(hipGetLastError());
  }
  // --- leaves: base utilities and next-round linkage
  const int64_t nl = f->n[8];
  PASUR_TRY(dev_alloc(&f->leaf_base, nl));
  if (gt->round == 5) PASUR_TRY(dev_alloc(&f->leaf_bonus, nl));
  uint64_t *lkeys = nullptr, *lkeys2 = nullptr;
  int32_t *lidx = nullptr, *lidx2 = nullptr;
  const int r = gt->round;
  uint64_t dealt = 0;
  DealtCards dc;
  std::memset(&dc, 0, sizeof(dc));
  if (r < 5) {
    for (int i = 0; i < 4 + 8 * (r + 1); ++i) dealt |= 1ull << gt->deck[i];
    int k = 0;
    for (int c = 0; c < 52; ++c)
      if ((dealt >> c) & 1) dc.card[k++] = (uint8_t)c;
    PASUR_TRY(s.alloc(&lkeys, nl));
    PASUR_TRY(s.alloc(&lkeys2, nl));
    PASUR_TRY(s.alloc(&lidx, nl));
    PASUR_TRY(s.alloc(&lidx2, nl));
  }
  k_leaf_pass<<<grid_for(nl), kThreads, 0, stream>>>(nl, r, f->gt[8], f->sid[8], f->score_tab,
                                                     gt->rs[8], gt->pool[8], dealt, f->leaf_base,
                                                     f->leaf_bonus, lkeys, lidx);
  PASUR_TRY_HIP(hipGetLastError());
  if (r < 5) {
    const int nbits = __builtin_popcountll(dealt) + 16;
    PASUR_TRY(radix_sort_pairs<uint64_t>(lkeys, lkeys2, lidx, lidx2, nl, nbits, stream));
    int32_t *lflags = nullptr, *lpos = nullptr;
    PASUR_TRY(s.alloc(&lflags, nl));
    PASUR_TRY(s.alloc(&lpos, nl + 1));
    k_u64_flags<<<grid_for(nl), kThreads, 0, stream>>>(nl, lkeys2, lflags);
    int64_t nn = 0;
    PASUR_TRY(scan_counts(lflags, nl, lpos, &nn, stream));
    f->n_next = nn;
    PASUR_TRY(dev_alloc(&f->next_roots, nn));
    PASUR_TRY(dev_alloc(&f->link, nl));
    k_next_roots<<<grid_for(nl), kThreads, 0, stream>>>(nl, lkeys2, lidx2, lflags, lpos, dc,
                                                        f->next_roots, f->link);
    PASUR_TRY_HIP(hipGetLastError());
  }
  PASUR_TRY_HIP(hipStreamSynchronize(stream));
  return PASUR_OK;
}

}  // namespace

extern "C" int pasur_unfold_scores(const pasur_gt *gt, const pasur_root *d_roots, int64_t n_roots,
                                   pasur_fgt **out_fgt, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_fgt || !gt) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  *out_fgt = nullptr;
  PASUR_TRY(check_roots(gt->deck, gt->round, d_roots, n_roots, stream));
  pasur_fgt *f = new pasur_fgt();
  std::memset(f, 0, sizeof(*f));
  f->round = gt->round;
  int st = unfold_impl(gt, d_roots, n_roots, f, stream);
  if (st) {
    (void)hipStreamSynchronize(stream);
    pasur_fgt_free(f);
    return st;
  }
  *out_fgt = f;
  return PASUR_OK;
}

extern "C" int pasur_fgt_sizes(const pasur_fgt *f, int64_t n[9], int64_t *n_scores,
                               int64_t *n_next) {
  if (!f) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (n)
    for (int l = 0; l < 9; ++l) n[l] = f->n[l];
  if (n_scores) *n_scores = f->n_scores;
  if (n_next) *n_next = f->n_next;
  return PASUR_OK;
}

extern "C" const pasur_root *pasur_fgt_next_roots(const pasur_fgt *f) {
  return f ? f->next_roots : nullptr;
}

extern "C" int pasur_fgt_read(const pasur_fgt *f, int field, int level, void *host_dst) {
  if (!f || !host_dst) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (level < 0 || level > 8) {
    set_error("level %d outside 0..8", level);
    return PASUR_E_RANGE;
  }
  const int64_t n = f->n[level];
  const void *src = nullptr;
  size_t bytes = 0;
  switch (field) {
    case PASUR_FGT_GT: src = f->gt[level]; bytes = n * 4; break;
    case PASUR_FGT_SID: src = f->sid[level]; bytes = n * 4; break;
    case PASUR_FGT_PARENT: src = f->parent[level]; bytes = n * 4; break;
    case PASUR_FGT_CHILD_BEGIN:
      src = level < 8 ? f->child_begin[level] : nullptr;
      bytes = (n + 1) * 4;
      break;
    case PASUR_FGT_SCORE_TAB: src = f->score_tab; bytes = f->n_scores * 4; break;
    case PASUR_FGT_NEXT_ROOTS: src = f->next_roots; bytes = f->n_next * sizeof(pasur_root); break;
    case PASUR_FGT_LINK: src = f->link; bytes = f->n[8] * 4; break;
    case PASUR_FGT_LEAF_BASE: src = f->leaf_base; bytes = f->n[8] * 2; break;
    default:
      set_error("unknown FGT field %d", field);
      return PASUR_E_RANGE;
  }
  if (!src) {
    set_error("FGT field %d does not exist here", field);
    return PASUR_E_INVAL;
  }
  PASUR_TRY_HIP(hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
  return PASUR_OK;
}

extern "C" int pasur_gt_get_view(const pasur_gt *g, pasur_gt_view *out) {
  if (!g || !out) {
    pasur::set_error("null argument");
    return PASUR_E_INVAL;
  }
  std::memset(out, 0, sizeof(*out));
  out->round = g->round;
  for (int l = 0; l < 9; ++l) {
    out->n[l] = g->n[l];
    out->pool[l] = g->pool[l];
    out->hands[l] = g->hands[l];
    out->rs[l] = g->rs[l];
    out->parent[l] = g->parent[l];
    out->act_card[l] = g->act_card[l];
    out->act_cap[l] = g->act_cap[l];
    if (l < 8) out->child_begin[l] = g->child_begin[l];
  }
  return PASUR_OK;
}

extern "C" int pasur_fgt_get_view(const pasur_fgt *f, pasur_fgt_view *out) {
  if (!f || !out) {
    pasur::set_error("null argument");
    return PASUR_E_INVAL;
  }
  std::memset(out, 0, sizeof(*out));
  out->round = f->round;
  for (int l = 0; l < 9; ++l) {
    out->n[l] = f->n[l];
    out->gt[l] = f->gt[l];
    out->sid[l] = f->sid[l];
    out->parent[l] = f->parent[l];
    if (l < 8) out->child_begin[l] = f->child_begin[l];
  }
  out->score_tab = f->score_tab;
  out->n_scores = f->n_scores;
  out->next_roots = f->round < 5 ? f->next_roots : nullptr;
  out->n_next = f->round < 5 ? f->n_next : 0;
  out->link = f->round < 5 ? f->link : nullptr;
  out->leaf_base = f->leaf_base;
  return PASUR_OK;
}
