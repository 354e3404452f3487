// pasur_sweep.hip -- the HBM-streaming schedule of full-width DCFR
// (section "CFR Algorithm": CodeSnippets FindReachProbability and
// FindUtility, equations DFCR_REG, RM and DFCR_AVG) for rounds whose trees
// are far larger than what the persistent segment kernel keeps busy.
//
// One launch per level and sweep direction streams the level through HBM.
// A workgroup takes a tile of consecutive parents (at most kTile children),
// loads the children's state into LDS with coalesced accesses, runs one
// thread per parent over its children in child order -- the oracle's
// per-parent loops, in FP64 with no contraction -- and writes the results
// back through LDS, coalesced.  Three choices of representation keep the
// bytes per iteration low; none changes a result:
//
//  * No strategy array inside a call.  sigma^t of an edge is recomputed
//    from its stored regret and the sum of max(R, eps) (or R+) over its
//    siblings, in child order: x / sum, or 1/k when the sum is not
//    positive -- exactly the division the other schedules store.  The
//    first iteration of a call reads the sigma array (uniform, warm-started
//    or left by an earlier call); sigma^{T+1} is written back at the end.
//
//  * Chains are not iterated.  A node whose whole subtree is a chain of
//    single-child nodes ("passive"; in Pasur most nodes of levels 6 and 7,
//    where each player holds one card) has a constant utility -- its leaf's
//    -- and its descendants' edges are forced: sigma = 1 and zero regret
//    whatever the iteration.  Their utility is copied up once per call.
//    The last iteration's down sweep covers every node, so the reach arrays
//    end exactly as in the other schedules.  The one array that differs:
//    the average-strategy sums of edges below a passive parent are not
//    accumulated (they stay at their initial value); the average strategy
//    of such an edge is 1 either way.
//
//  * A compact tail.  Let S be the first level with passive nodes.  The
//    subtrees below the active nodes of level S (about 3% of a full game's
//    last round) are copied into contiguous arrays after a call's first
//    iteration, iterated there, and copied back before its last, so the
//    sweeps of levels S+1..8 touch only those copies.  The level arrays of
//    levels S-1 and S exchange the tail's boundary values (the reaches of
//    the heads' parents, the heads' utilities and strategies) through
//    per-tile ranges of the sorted head lists.
#pragma clang fp contract(off)

#include "pasur_internal.hpp"

#include <algorithm>
#include <vector>

namespace pasur {

// Structure index of one unfolded tree (built once, on first use).
struct SweepIndex {
  int64_t n[9];
  uint8_t *passive[9];  // levels 1..7: 1 where the node heads a chain (else 0)
  int64_t n_act[9];     // active (non-passive) nodes per level 0..7
  int32_t *act[9];      // their indices where n_act[l] < n[l] (all of levels S..7)
  int kmax[9];          // largest fan-out among the parents of level L (L = 1..8)
  int32_t *tile[9];     // level L: parent starts of its tiles (n_tile[L] + 1)
  int32_t *tile_c[9];   // level L: child starts of its tiles (n_tile[L] + 1)
  int64_t n_tile[9];
  // Compact tail (S = 0: none).  Active node i of level l (S..7) is act[l][i].
  int S;
  int64_t m[9];         // level L = S+1..8: children of level L-1's active nodes
  int32_t *cbc[9];      // level l = S..7: their compact CSR (n_act[l] + 1)
  int32_t *cmap[9];     // level L: compact child -> node of level L
  int32_t *jpos[9];     // level L = S+1..7: active node -> its compact child position
  int32_t *ppar[9];     // level L = S+1..7: active node -> its parent's active index;
                        // level S: -> its parent's index in bp
  int32_t *ttile[9];    // level L = S+1..8: tiles of the compact children (parent starts,
  int32_t *ttile_c[9];  // child starts; n_ttile[L] + 1 each), where the largest group fits
  int64_t n_ttile[9];
  int64_t n_bp;         // boundary parents: level S-1 nodes with an active child
  int32_t *bp;          // their indices (sorted)
  int32_t *bp_tile;     // first bp entry of each tile of level S-1 (n_tile[S-1] + 1)
  int32_t *act_tile;    // first act[S] entry of each tile of level S (n_tile[S] + 1)
};

void sweep_index_free(SweepIndex *x) {
  if (!x) return;
  for (int l = 0; l < 9; ++l) {
    dev_free(x->passive[l]);
    dev_free(x->act[l]);
    dev_free(x->tile[l]);
    dev_free(x->tile_c[l]);
    dev_free(x->cbc[l]);
    dev_free(x->cmap[l]);
    dev_free(x->jpos[l]);
    dev_free(x->ppar[l]);
    dev_free(x->ttile[l]);
    dev_free(x->ttile_c[l]);
  }
  dev_free(x->bp);
  dev_free(x->bp_tile);
  dev_free(x->act_tile);
  delete x;
}

namespace {

constexpr int kBlk = 256;
// Children per tile (a parent's children never straddle two tiles).
constexpr int kTile = 1024;
// Largest fan-out from which a level's up sweep takes the per-child form
// (round 6 of deal 40: level 5 489 -> 473 us; 8 leaves that level out).
constexpr int kWideKids = 5;

inline unsigned grid_of(int64_t n, int64_t cap = 256 * 32) {
  int64_t g = (n + kBlk - 1) / kBlk;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

#define SW_FOR(i, n)                                                           \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

// ---- index construction ----------------------------------------------------

// passive(h) = one child, and that child is a leaf (level 7) or passive.
__global__ void k_sw_passive(int64_t n, int last, const int32_t *__restrict__ cb,
                             const uint8_t *__restrict__ passive_next,
                             uint8_t *__restrict__ passive, int32_t *__restrict__ active) {
  SW_FOR(h, n) {
    const int32_t b = cb[h];
    const bool p = cb[h + 1] - b == 1 && (last || passive_next[b]);
    passive[h] = p ? 1 : 0;
    active[h] = p ? 0 : 1;
  }
}

__global__ void k_sw_compact(int64_t n, const int32_t *__restrict__ active,
                             const int32_t *__restrict__ pos, int32_t *__restrict__ list) {
  SW_FOR(h, n) if (active[h]) list[pos[h]] = (int32_t)h;
}

__global__ void k_sw_kmax(int64_t n, const int32_t *__restrict__ cb, int *__restrict__ out) {
  int m = 0;
  SW_FOR(h, n) m = max(m, cb[h + 1] - cb[h]);
  if (m > 0) atomicMax(out, m);
}

// Tile i of a level covers the parents from the parent of child
// i * stride (stride = kTile - (kmax - 1)) up to the next tile's, so its
// children never exceed kTile; the last entry is the parent count.
__global__ void k_sw_tiles(int64_t n_tile, int64_t n, int64_t n_par, int stride,
                           const int32_t *__restrict__ par, int32_t *__restrict__ ts) {
  SW_FOR(c, n_tile + 1) {
    const int64_t x = c * (int64_t)stride;
    ts[c] = c < n_tile && x < n ? par[x] : (int32_t)n_par;
  }
}

__global__ void k_sw_tile_c(int64_t n_tile, const int32_t *__restrict__ ts,
                            const int32_t *__restrict__ cb, int32_t *__restrict__ tc) {
  SW_FOR(w, n_tile + 1) tc[w] = cb[ts[w]];
}

__global__ void k_sw_kmin(int64_t n, const int32_t *__restrict__ cb, int *__restrict__ out) {
  int m = INT32_MAX;
  SW_FOR(h, n) m = min(m, cb[h + 1] - cb[h]);
  atomicMin(out, m);
}

__global__ void k_sw_iota(int64_t n, int32_t *__restrict__ v) { SW_FOR(i, n) v[i] = (int32_t)i; }

__global__ void k_sw_fill(int64_t n, int32_t v, int32_t *__restrict__ out) { SW_FOR(i, n) out[i] = v; }

// inv[act[i]] = i (inv pre-filled with -1)
__global__ void k_sw_invert(int64_t n, const int32_t *__restrict__ act, int32_t *__restrict__ inv) {
  SW_FOR(i, n) inv[act[i]] = (int32_t)i;
}

// children counts of the active parents
__global__ void k_sw_kids(int64_t n, const int32_t *__restrict__ act, const int32_t *__restrict__ cb,
                          int32_t *__restrict__ cnt) {
  SW_FOR(i, n) cnt[i] = cb[act[i] + 1] - cb[act[i]];
}

// compact child position -> node, per active parent
__global__ void k_sw_cmap(int64_t n, const int32_t *__restrict__ act, const int32_t *__restrict__ cb,
                          const int32_t *__restrict__ cbc, int32_t *__restrict__ cmap) {
  SW_FOR(i, n) {
    const int32_t b = cb[act[i]], e = cb[act[i] + 1], o = cbc[i];
    for (int32_t c = b; c < e; ++c) cmap[o + (c - b)] = c;
  }
}

// compact child position -> its parent's active index
__global__ void k_sw_cpar(int64_t n, const int32_t *__restrict__ cbc, int32_t *__restrict__ pc) {
  SW_FOR(i, n) for (int32_t j = cbc[i]; j < cbc[i + 1]; ++j) pc[j] = (int32_t)i;
}

// active node i of level L: its parent's active index and its compact child
// position among that parent's children
__global__ void k_sw_tailpos(int64_t n, const int32_t *__restrict__ act,
                             const int32_t *__restrict__ par, const int32_t *__restrict__ inv_up,
                             const int32_t *__restrict__ cb_up, const int32_t *__restrict__ cbc_up,
                             int32_t *__restrict__ ppar, int32_t *__restrict__ jpos) {
  SW_FOR(i, n) {
    const int32_t q = act[i], p = par[q], ip = inv_up[p];
    ppar[i] = ip;
    jpos[i] = cbc_up[ip] + (q - cb_up[p]);
  }
}

// 1 where active node i of level S has a different parent than node i-1
__global__ void k_sw_bpflag(int64_t n, const int32_t *__restrict__ act,
                            const int32_t *__restrict__ par, int32_t *__restrict__ flag) {
  SW_FOR(i, n) flag[i] = i == 0 || par[act[i]] != par[act[i - 1]] ? 1 : 0;
}

// the boundary parents and each active node's index among them
__global__ void k_sw_bpset(int64_t n, const int32_t *__restrict__ act,
                           const int32_t *__restrict__ par, const int32_t *__restrict__ flag,
                           const int32_t *__restrict__ excl, int32_t *__restrict__ ppar,
                           int32_t *__restrict__ bp) {
  SW_FOR(i, n) {
    ppar[i] = excl[i] + flag[i] - 1;
    if (flag[i]) bp[excl[i]] = par[act[i]];
  }
}

// For each tile of a level: the first entry of a sorted node list at or
// after the tile's first child.
__global__ void k_sw_tile_ranks(int64_t n_tile, const int32_t *__restrict__ ts,
                                const int32_t *__restrict__ cb, const int32_t *__restrict__ list,
                                int64_t n_list, int32_t *__restrict__ out) {
  SW_FOR(w, n_tile + 1) {
    const int32_t c0 = cb[ts[w]];
    int64_t lo = 0, hi = n_list;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (list[mid] < c0) lo = mid + 1;
      else hi = mid;
    }
    out[w] = (int32_t)lo;
  }
}

// The compact-tail part of the index (levels S..8), S >= 2, for levels
// S-1 and S with tiles.
int build_tail(pasur_fgt *f, SweepIndex *x, int S, hipStream_t s) {
  int st = PASUR_OK;
  int32_t *inv[9] = {nullptr};
  int32_t *tmp = nullptr, *tmp2 = nullptr;
  for (int l = S; l <= 7 && !st; ++l) {
    if (!x->act[l]) {  // every node of the level is active
      st = dev_alloc(&x->act[l], f->n[l]);
      if (!st) k_sw_iota<<<grid_of(f->n[l]), kBlk, 0, s>>>(f->n[l], x->act[l]);
    }
    if (!st) st = dev_alloc(&inv[l], f->n[l]);
    if (!st) {
      k_sw_fill<<<grid_of(f->n[l]), kBlk, 0, s>>>(f->n[l], -1, inv[l]);
      k_sw_invert<<<grid_of(x->n_act[l]), kBlk, 0, s>>>(x->n_act[l], x->act[l], inv[l]);
    }
  }
  // compact children of levels S+1..8
  for (int L = S + 1; L <= 8 && !st; ++L) {
    const int64_t na = x->n_act[L - 1];
    st = dev_alloc(&tmp, na);
    if (!st) st = dev_alloc(&x->cbc[L - 1], na + 1);
    if (st) break;
    k_sw_kids<<<grid_of(na), kBlk, 0, s>>>(na, x->act[L - 1], f->child_begin[L - 1], tmp);
    int64_t m = 0;
    st = scan_counts(tmp, na, x->cbc[L - 1], &m, s);
    dev_free(tmp);
    if (st) break;
    x->m[L] = m;
    st = dev_alloc(&x->cmap[L], m);
    if (st) break;
    k_sw_cmap<<<grid_of(na), kBlk, 0, s>>>(na, x->act[L - 1], f->child_begin[L - 1], x->cbc[L - 1],
                                           x->cmap[L]);
  }
  // tiles of the compact levels (every active parent has a child)
  for (int L = S + 1; L <= 8 && !st; ++L) {
    const int km = x->kmax[L];
    const int64_t m = x->m[L], na = x->n_act[L - 1];
    if (m == 0 || km > kTile / 2) continue;
    int32_t *pc = nullptr;
    st = dev_alloc(&pc, m);
    const int stride = kTile - (km - 1);
    const int64_t nt = (m + stride - 1) / stride;
    if (!st) st = dev_alloc(&x->ttile[L], nt + 1);
    if (!st) st = dev_alloc(&x->ttile_c[L], nt + 1);
    if (!st) {
      x->n_ttile[L] = nt;
      k_sw_cpar<<<grid_of(na), kBlk, 0, s>>>(na, x->cbc[L - 1], pc);
      k_sw_tiles<<<grid_of(nt + 1), kBlk, 0, s>>>(nt, m, na, stride, pc, x->ttile[L]);
      k_sw_tile_c<<<grid_of(nt + 1), kBlk, 0, s>>>(nt, x->ttile[L], x->cbc[L - 1], x->ttile_c[L]);
      const hipError_t e = hipStreamSynchronize(s);  // pc is read by k_sw_tiles
      if (e != hipSuccess) {
        set_error("sweep tail tiles: %s", hipGetErrorString(e));
        st = PASUR_E_HIP;
      }
    }
    dev_free(pc);
  }
  for (int L = S + 1; L <= 7 && !st; ++L) {
    const int64_t na = x->n_act[L];
    st = dev_alloc(&x->ppar[L], na);
    if (!st) st = dev_alloc(&x->jpos[L], na);
    if (!st)
      k_sw_tailpos<<<grid_of(na), kBlk, 0, s>>>(na, x->act[L], f->parent[L], inv[L - 1],
                                                f->child_begin[L - 1], x->cbc[L - 1], x->ppar[L],
                                                x->jpos[L]);
  }
  // the boundary between the level arrays and the tail
  if (!st) {
    const int64_t na = x->n_act[S];
    st = dev_alloc(&tmp, na);
    if (!st) st = dev_alloc(&tmp2, na + 1);
    if (!st) st = dev_alloc(&x->ppar[S], na);
    if (!st) {
      k_sw_bpflag<<<grid_of(na), kBlk, 0, s>>>(na, x->act[S], f->parent[S], tmp);
      st = scan_counts(tmp, na, tmp2, &x->n_bp, s);
    }
    if (!st) st = dev_alloc(&x->bp, x->n_bp);
    if (!st)
      k_sw_bpset<<<grid_of(na), kBlk, 0, s>>>(na, x->act[S], f->parent[S], tmp, tmp2, x->ppar[S],
                                              x->bp);
    if (!st) st = dev_alloc(&x->bp_tile, x->n_tile[S - 1] + 1);
    if (!st) st = dev_alloc(&x->act_tile, x->n_tile[S] + 1);
    if (!st) {
      k_sw_tile_ranks<<<grid_of(x->n_tile[S - 1] + 1), kBlk, 0, s>>>(
          x->n_tile[S - 1], x->tile[S - 1], f->child_begin[S - 2], x->bp, x->n_bp, x->bp_tile);
      k_sw_tile_ranks<<<grid_of(x->n_tile[S] + 1), kBlk, 0, s>>>(
          x->n_tile[S], x->tile[S], f->child_begin[S - 1], x->act[S], na, x->act_tile);
    }
  }
  dev_free(tmp);
  dev_free(tmp2);
  for (int l = 0; l < 9; ++l) dev_free(inv[l]);
  if (!st) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error("sweep tail index: %s", hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  if (!st) x->S = S;
  return st;
}

int build_index(pasur_fgt *f, hipStream_t s) {
  SweepIndex *x = new SweepIndex();
  for (int l = 0; l < 9; ++l) {
    x->n[l] = f->n[l];
    x->passive[l] = nullptr;
    x->act[l] = nullptr;
    x->tile[l] = nullptr;
    x->tile_c[l] = nullptr;
    x->n_tile[l] = 0;
    x->n_act[l] = f->n[l];
    x->kmax[l] = 0;
    x->m[l] = 0;
    x->cbc[l] = x->cmap[l] = x->jpos[l] = x->ppar[l] = nullptr;
    x->ttile[l] = x->ttile_c[l] = nullptr;
    x->n_ttile[l] = 0;
  }
  x->S = 0;
  x->n_bp = 0;
  x->bp = x->bp_tile = x->act_tile = nullptr;
  auto fail = [&](int st) {
    sweep_index_free(x);
    return st;
  };
  int32_t *active = nullptr, *pos = nullptr;
  int64_t mx = 1;
  for (int l = 1; l <= 7; ++l) mx = std::max<int64_t>(mx, f->n[l]);
  int st = dev_alloc(&active, mx);
  if (!st) st = dev_alloc(&pos, mx + 1);
  if (st) {
    dev_free(active);
    return fail(st);
  }
  // passive flags bottom-up, then the active lists of the levels that have
  // passive nodes
  for (int l = 7; l >= 1 && !st; --l) {
    const int64_t n = f->n[l];
    st = dev_alloc(&x->passive[l], n);
    if (st) break;
    k_sw_passive<<<grid_of(n), kBlk, 0, s>>>(n, l == 7, f->child_begin[l],
                                             l == 7 ? nullptr : x->passive[l + 1],
                                             x->passive[l], active);
    int64_t n_act = 0;
    st = n > 0 ? scan_counts(active, n, pos, &n_act, s) : PASUR_OK;
    if (st) break;
    x->n_act[l] = n_act;
    if (n_act < n) {
      st = dev_alloc(&x->act[l], n_act);
      if (st) break;
      k_sw_compact<<<grid_of(n), kBlk, 0, s>>>(n, active, pos, x->act[l]);
    }
  }
  dev_free(active);
  dev_free(pos);
  if (st) return fail(st);
  // largest fan-out per level, and the tiles of the levels whose parents'
  // children fit a tile
  int *d_km = nullptr;
  st = dev_alloc(&d_km, 18);
  if (st) return fail(st);
  k_sw_fill<<<1, kBlk, 0, s>>>(9, 0, d_km);
  k_sw_fill<<<1, kBlk, 0, s>>>(9, INT32_MAX, d_km + 9);
  for (int L = 1; L <= 8; ++L) {
    k_sw_kmax<<<grid_of(f->n[L - 1]), kBlk, 0, s>>>(f->n[L - 1], f->child_begin[L - 1], d_km + L);
    k_sw_kmin<<<grid_of(f->n[L - 1]), kBlk, 0, s>>>(f->n[L - 1], f->child_begin[L - 1], d_km + 9 + L);
  }
  int kmin[9];
  hipError_t e = hipMemcpyAsync(x->kmax, d_km, 9 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(kmin, d_km + 9, 9 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(d_km);
  if (e != hipSuccess) {
    set_error("sweep index: %s", hipGetErrorString(e));
    return fail(PASUR_E_HIP);
  }
  // tiles where every parent has a child (so a tile never holds more
  // parents than children) and the largest group fits a tile
  for (int L = 1; L <= 8; ++L) {
    const int km = x->kmax[L];
    if (kmin[L] < 1 || km > kTile / 2 || f->n[L] == 0) continue;
    const int stride = kTile - (km - 1);
    const int64_t nt = (f->n[L] + stride - 1) / stride;
    st = dev_alloc(&x->tile[L], nt + 1);
    if (!st) st = dev_alloc(&x->tile_c[L], nt + 1);
    if (st) return fail(st);
    x->n_tile[L] = nt;
    k_sw_tiles<<<grid_of(nt + 1), kBlk, 0, s>>>(nt, f->n[L], f->n[L - 1], stride, f->parent[L],
                                                x->tile[L]);
    k_sw_tile_c<<<grid_of(nt + 1), kBlk, 0, s>>>(nt, x->tile[L], f->child_begin[L - 1], x->tile_c[L]);
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("sweep index: %s", hipGetErrorString(e));
    return fail(PASUR_E_HIP);
  }
  // compact tail: levels 0..S-1 without passive nodes, S >= 2, levels S-1
  // and S tiled, and something to iterate below S
  int S = 0;
  for (int l = 1; l <= 7 && !S; ++l)
    if (x->n_act[l] < f->n[l]) S = l;
  if (S >= 2 && x->n_act[S] > 0 && x->tile[S - 1] && x->tile[S]) {
    st = build_tail(f, x, S, s);
    if (st) return fail(st);
  }
  f->sweep = x;
  return PASUR_OK;
}

// ---- sigma from regrets --------------------------------------------------------

__device__ __forceinline__ double rm_x(double R, int rm_mode, double eps) {
  return rm_mode == PASUR_RM_FLOOR ? fmax(R, eps) : fmax(R, 0.0);
}

// Regret matching of one edge from the sum of x over its siblings (in child
// order), rounded to the state type as the other schedules store it:
// x / sum, or 1/k when the sum is not positive.
template <class T>
__device__ __forceinline__ double sig_from(double x, double sum, int k) {
  return (double)(T)(sum > 0.0 ? x / sum : 1.0 / (double)k);
}
// The same from a stored sum Z (Z <= 0 stands for "not positive": Z = -k).
template <class T>
__device__ __forceinline__ double sig_of(T Rq, double Z, int rm_mode, double eps) {
  const double x = rm_x((double)Rq, rm_mode, eps);
  return (double)(T)(Z > 0.0 ? x / Z : 1.0 / -Z);
}
__device__ __forceinline__ double z_enc(double sum, int k) { return sum > 0.0 ? sum : -(double)k; }

// Sum of x over the children b..e-1, in order (the regret-matching sum).
template <class T>
__device__ __forceinline__ double x_sum(const T *__restrict__ R, int32_t b, int32_t e, int rm_mode,
                                        double eps) {
  double sum = 0.0;
  for (int32_t q = b; q < e; ++q) sum += rm_x((double)R[q], rm_mode, eps);
  return sum;
}

template <bool PAPER>
__device__ __forceinline__ double regret_update(double Rq, double r, const IterK &ik, int variant) {
  if (PAPER || variant == PASUR_DCFR) {
    const double d = Rq > 0.0 ? ik.dpos : ik.dneg;
    return d * Rq + r;
  }
  if (variant == PASUR_CFR_PLUS) {
    const double x = Rq + r;
    return x < 0.0 ? 0.0 : x;
  }
  return Rq + r;
}

// ---- per-call set-up and tear-down -----------------------------------------

// u of a passive node = its only child's utility (sigma = 1), once per call.
template <class T>
__global__ void k_sw_chain_u(int64_t n, const uint8_t *__restrict__ passive,
                             const int32_t *__restrict__ cb, T *__restrict__ u,
                             const T *__restrict__ u_next) {
  SW_FOR(h, n) if (passive[h]) u[h] = (T)(0.0 + (double)u_next[cb[h]]);
}

// sigma^{T+1} of every child of a level's parents, written back at the end
// of a call.
template <class T>
__global__ void k_sw_sigma_out(int64_t n, const int32_t *__restrict__ cb,
                               const T *__restrict__ R, T *__restrict__ sg, int rm_mode, double eps) {
  SW_FOR(h, n) {
    const int32_t b = cb[h], e = cb[h + 1];
    const double sum = x_sum(R, b, e, rm_mode, eps);
    for (int32_t q = b; q < e; ++q)
      sg[q] = (T)sig_from<T>(rm_x((double)R[q], rm_mode, eps), sum, e - b);
  }
}

// ---- the sweeps --------------------------------------------------------------

template <class T>
struct Reach {
  const T *ra_up, *rb_up;  // parents
  T *ra, *rb;              // nodes
  // tile sweeps of the level above the tail: the boundary parents' reaches
  // also go to bra/brb (entries bp_tile[w] .. bp_tile[w+1]-1 of bp per tile)
  const int32_t *bp, *bp_tile;
  T *bra, *brb;
  int mover;
};

// Tile geometry shared by the tile sweeps: tile w holds parents
// ts[w]..ts[w+1]-1 and their children tc[w]..tc[w+1]-1; thread t handles
// children t, t + kBlk, ... and parents t, t + kBlk, ... of the tile.
constexpr int kPer = kTile / kBlk;

struct TileMeta {
  int32_t h0, np, c0, nc;
};

__device__ __forceinline__ TileMeta tile_meta(const int32_t *__restrict__ ts,
                                              const int32_t *__restrict__ tc, int64_t w) {
  TileMeta m;
  m.h0 = ts[w];
  m.np = ts[w + 1] - m.h0;
  m.c0 = tc[w];
  m.nc = tc[w + 1] - m.c0;
  return m;
}

// FindReachProbability over LDS-staged tiles: the workgroup loads its
// tile's regrets (coalesced), one thread per parent computes the parent's
// regret-matching sum and its children's reaches in child order, and the
// reaches leave through LDS (coalesced).  The next tile's loads are issued
// into registers before the current tile is computed.  POS: the sum is
// always positive (regret floor eps > 0), so sigma is x / sum without the
// 1/k branch.
template <class T, bool POS, bool BND>
__global__ void __launch_bounds__(kBlk)
    k_sw_down_tile(int64_t n_tile, const int32_t *__restrict__ ts, const int32_t *__restrict__ tc,
                   const int32_t *__restrict__ cb, const T *__restrict__ R,
                   const T *__restrict__ sg_first, Reach<T> rc, int rm_mode, double eps) {
  __shared__ T sx[kTile], sa[kTile], sb[kTile];
  __shared__ int32_t scb[kTile + 1];
  if (POS) rm_mode = PASUR_RM_FLOOR;
  const int tid = threadIdx.x;
  const T *src = sg_first ? sg_first : R;
  // registers of the next tile
  TileMeta nm;
  T px[kPer], pa[kPer], pb[kPer];
  int32_t pcb[kPer + 1];
  int32_t pbr0 = 0, pbn = 0, pbj[kPer];
  auto fetch = [&](int64_t w) {
    nm = tile_meta(ts, tc, w);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < nm.nc) px[k] = src[nm.c0 + j];
      if (j < nm.np) {
        pa[k] = rc.ra_up[nm.h0 + j];
        pb[k] = rc.rb_up[nm.h0 + j];
      }
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= nm.np) pcb[k] = cb[nm.h0 + i];
    }
    if (BND) {
      pbr0 = rc.bp_tile[w];
      pbn = rc.bp_tile[w + 1] - pbr0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int r = tid + k * kBlk;
        if (r < pbn) pbj[k] = rc.bp[pbr0 + r] - nm.c0;
      }
    }
  };
  int64_t w = blockIdx.x;
  if (w < n_tile) fetch(w);
  for (; w < n_tile; w += gridDim.x) {
    const TileMeta m = nm;
    T ca[kPer], cbb[kPer];
    int32_t br0 = pbr0, bn = pbn, bj[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) sx[j] = px[k];
      ca[k] = pa[k];
      cbb[k] = pb[k];
      if (BND) bj[k] = pbj[k];
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= m.np) scb[i] = pcb[k] - m.c0;
    }
    __syncthreads();
    if (w + gridDim.x < n_tile) fetch(w + gridDim.x);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i >= m.np) break;
      const int32_t b = scb[i], e = scb[i + 1];
      double sum = 0.0;
      if (!sg_first) {

        for (int j = b; j < e; ++j) sum += rm_x((double)sx[j], rm_mode, eps);
      }
      const double xa = (double)ca[k], xb = (double)cbb[k];

      for (int j = b; j < e; ++j) {
        double s;
        if (sg_first) {
          s = (double)sx[j];
        } else {
          const double x = rm_x((double)sx[j], rm_mode, eps);
          s = POS ? (double)(T)(x / sum) : sig_from<T>(x, sum, e - b);
        }
        sa[j] = (T)(rc.mover == 0 ? xa * s : xa);
        sb[j] = (T)(rc.mover == 0 ? xb : xb * s);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        rc.ra[m.c0 + j] = sa[j];
        rc.rb[m.c0 + j] = sb[j];
      }
      if (BND && tid + k * kBlk < bn) {
        rc.bra[br0 + tid + k * kBlk] = sa[bj[k]];
        rc.brb[br0 + tid + k * kBlk] = sb[bj[k]];
      }
    }
    __syncthreads();  // before the next tile reuses LDS
  }
}

// FindReachProbability, one thread per parent (every parent of the level):
// its sum, then its children in order.
template <class T>
__global__ void __launch_bounds__(kBlk)
    k_sw_down_parent(int64_t n, const int32_t *__restrict__ cb, const T *__restrict__ R,
                     const T *__restrict__ sg_first, Reach<T> rc, int rm_mode, double eps) {
  SW_FOR(h, n) {
    const int32_t b = cb[h], e = cb[h + 1];
    const double sum = sg_first ? 0.0 : x_sum(R, b, e, rm_mode, eps);
    const double pa = (double)rc.ra_up[h], pb = (double)rc.rb_up[h];
    for (int32_t q = b; q < e; ++q) {
      const double s = sg_first ? (double)sg_first[q]
                                : sig_from<T>(rm_x((double)R[q], rm_mode, eps), sum, e - b);
      rc.ra[q] = (T)(rc.mover == 0 ? pa * s : pa);
      rc.rb[q] = (T)(rc.mover == 0 ? pb : pb * s);
    }
  }
}

// FindReachProbability over a node list: node q = list[i] (or i), parent
// par[q]; sigma from sg (indexed by q), else from R at rpos[q] (or q) and
// the parent's stored sum Zp, else from a loop over the siblings (cb).
template <class T>
__global__ void __launch_bounds__(kBlk)
    k_sw_down_list(int64_t n, const int32_t *__restrict__ list, const int32_t *__restrict__ par,
                   const int32_t *__restrict__ rpos, const T *__restrict__ R,
                   const T *__restrict__ sg, const double *__restrict__ Zp,
                   const int32_t *__restrict__ cb, Reach<T> rc, int rm_mode, double eps) {
  SW_FOR(i, n) {
    const int64_t q = list ? list[i] : i;
    const int32_t h = par[q];
    double s;
    if (sg) {
      s = (double)sg[q];
    } else if (Zp) {
      s = sig_of<T>(R[rpos ? rpos[q] : q], Zp[h], rm_mode, eps);
    } else {
      const int32_t b = cb[h], e = cb[h + 1];
      s = sig_from<T>(rm_x((double)R[q], rm_mode, eps), x_sum(R, b, e, rm_mode, eps), e - b);
    }
    const double pa = (double)rc.ra_up[h], pb = (double)rc.rb_up[h];
    rc.ra[q] = (T)(rc.mover == 0 ? pa * s : pa);
    rc.rb[q] = (T)(rc.mover == 0 ? pb : pb * s);
  }
}

// Arguments of one level's up sweep (children on level L, parents on L-1).
template <class T>
struct UpArgs {
  const int32_t *cb;    // level L-1
  T *R, *Sb;            // level L
  const T *sg_first;    // level L (first iteration of a call), else null
  const T *u;           // level L
  T *u_par;             // level L-1
  const int32_t *upos;  // position of parent h's utility in u_par (else h)
  double *Z;            // stored regret-matching sums of the parents (compact tail), else null
  const T *ra, *rb;     // level L-1
  double *vacc;         // roots (L == 1) or null
  // tile sweeps of the tail's first level: the heads (act[S][r], entries
  // act_tile[w] .. act_tile[w+1]-1 per tile) take their utility from u_act
  // and give their next strategy to sg_act, at index r
  const int32_t *act, *act_tile;
  const T *u_act;
  T *sg_act;
  int mover;
};

// FindUtility over LDS-staged tiles: the workgroup loads its tile's
// regrets, average sums and utilities (coalesced), one thread per parent
// runs the parent's update over its children in child order (the oracle's
// loops), and the regrets and average sums leave through LDS (coalesced).
// With BND, the tail's heads in the tile (a short list, about one in 37
// children) then take their next strategy, a thread per head; a per-child
// test inside the parents' loops would hold nearly every wave for a few
// heads.  The next tile's loads (children, CSR, the parents' reaches) are
// issued into registers before the current tile is computed.
template <class T, bool PAPER, bool BND>
__global__ void __launch_bounds__(kBlk)
    k_sw_up_tile(int64_t n_tile, const int32_t *__restrict__ ts, const int32_t *__restrict__ tc,
                 UpArgs<T> a, IterK ik, int variant, int rm_mode, double eps) {
  __shared__ T sR[kTile], sS[kTile], su[kTile], ss[kTile];
  __shared__ int32_t scb[kTile + 1];
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const double sgn = a.mover == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x;
  const bool first = a.sg_first != nullptr;
  // registers of the next tile
  TileMeta nm;
  T pR[kPer], pS[kPer], pu[kPer], pg[kPer], pa[kPer], pb[kPer];
  int32_t pcb[kPer + 1];
  int32_t phr0 = 0, phn = 0, phj[kPer];
  T phu[kPer];
  auto fetch = [&](int64_t w) {
    nm = tile_meta(ts, tc, w);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < nm.nc) {
        const int64_t q = nm.c0 + j;
        pR[k] = a.R[q];
        pS[k] = a.Sb[q];
        pu[k] = a.u[q];
        if (first) pg[k] = a.sg_first[q];
      }
      if (j < nm.np) {
        pa[k] = a.ra[nm.h0 + j];
        pb[k] = a.rb[nm.h0 + j];
      }
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= nm.np) pcb[k] = a.cb[nm.h0 + i];
    }
    if (BND) {
      phr0 = a.act_tile[w];
      phn = a.act_tile[w + 1] - phr0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int r = tid + k * kBlk;
        if (r < phn) {
          phj[k] = a.act[phr0 + r] - nm.c0;
          phu[k] = a.u_act[phr0 + r];
        }
      }
    }
  };
  int64_t w = blockIdx.x;
  if (w < n_tile) fetch(w);
  for (; w < n_tile; w += gridDim.x) {
    const TileMeta m = nm;
    const int32_t hr0 = phr0, hn = phn;  // the tile's heads: act[hr0 + r], r < hn
    int32_t hj[kPer];                    // their children within the tile
    T ca[kPer], cbb[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        sR[j] = pR[k];
        sS[j] = pS[k];
        su[j] = pu[k];
        if (first) ss[j] = pg[k];
      }
      ca[k] = pa[k];
      cbb[k] = pb[k];
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= m.np) scb[i] = pcb[k] - m.c0;
    }
    if (BND) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (tid + k * kBlk < phn) {
          su[phj[k]] = phu[k];
          hj[k] = phj[k];
        }
    }
    __syncthreads();
    if (w + gridDim.x < n_tile) fetch(w + gridDim.x);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i >= m.np) break;
      const int32_t h = m.h0 + i, b = scb[i], e = scb[i + 1], kk = e - b;
      // sigma^t from the regrets (unless given) and u(h) = sum sigma^t u,
      // both sums in child order
      double uh = 0.0;
      if (!first) {
        double sum = 0.0;

        for (int j = b; j < e; ++j) sum += rm_x((double)sR[j], rm_mode, eps);

        for (int j = b; j < e; ++j) {
          const double x = rm_x((double)sR[j], rm_mode, eps);
          const T sj = PAPER ? (T)(x / sum) : (T)sig_from<T>(x, sum, kk);
          ss[j] = sj;
          uh += (double)sj * (double)su[j];
        }
      } else {

        for (int j = b; j < e; ++j) uh += (double)ss[j] * (double)su[j];
      }
      const double opp = a.mover == 0 ? (double)cbb[k] : (double)ca[k];
      const double own = a.mover == 0 ? (double)ca[k] : (double)cbb[k];

      for (int j = b; j < e; ++j) {
        const double r = sgn * opp * ((double)su[j] - uh);
        sR[j] = (T)regret_update<PAPER>((double)sR[j], r, ik, variant);
        double add = own * (double)ss[j];
        if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
        sS[j] = (T)(ik.avg_w * (double)sS[j] + add);
      }
      a.u_par[h] = (T)uh;
      if (a.vacc) a.vacc[h] += uh;
    }
    __syncthreads();
    if (BND) {
      // the heads' next strategy from their updated regrets: a thread per
      // head finds the head's parent in the tile's CSR (binary search) and
      // takes the regret-matching sum over the siblings in child order
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int r = tid + k * kBlk;
        if (r >= hn) break;
        const int j = hj[k];
        int lo = 0, hi = m.np - 1;  // the parent i with scb[i] <= j < scb[i + 1]
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (scb[mid] <= j) lo = mid;
          else hi = mid - 1;
        }
        const int b = scb[lo], e = scb[lo + 1];
        double sum = 0.0;
        for (int q = b; q < e; ++q) sum += rm_x((double)sR[q], rm_mode, eps);
        a.sg_act[hr0 + r] = (T)sig_from<T>(rm_x((double)sR[j], rm_mode, eps), sum, e - b);
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        a.R[m.c0 + j] = sR[j];
        a.Sb[m.c0 + j] = sS[j];
      }
    }
    __syncthreads();  // before the next tile reuses LDS
  }
}

// The same update for levels whose sibling groups vary widely in size
// (levels that are not the tail's boundary): only the two sibling sums run
// one thread per parent, in child order -- the regret-matching sum, then
// u(h) = sum sigma^t u; sigma^t = x / sum and each child's regret and
// average-sum updates run one thread per child, so a wave does not wait on
// the largest group among its 64 parents.  Each child's arithmetic is that
// of k_sw_up_tile, so the results are the same bits.  The regrets and
// average sums leave straight from the child threads (coalesced).
template <class T, bool PAPER>
__global__ void __launch_bounds__(kBlk)
    k_sw_up_tile_wide(int64_t n_tile, const int32_t *__restrict__ ts,
                      const int32_t *__restrict__ tc, UpArgs<T> a, IterK ik, int variant,
                      int rm_mode, double eps) {
  __shared__ T sR[kTile], su[kTile], ss[kTile];
  __shared__ int32_t scb[kTile + 1];
  __shared__ int16_t sp[kTile];           // a child's parent within the tile
  __shared__ double sZ[kTile];            // parent: regret-matching sum, then u(h)
  __shared__ T sopp[kTile], sown[kTile];  // parent: the opponent's and own reach
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const double sgn = a.mover == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x;
  const bool first = a.sg_first != nullptr;
  // registers of the next tile
  TileMeta nm;
  T pR[kPer], pS[kPer], pu[kPer], pg[kPer], pa[kPer], pb[kPer];
  int32_t pcb[kPer + 1];
  auto fetch = [&](int64_t w) {
    nm = tile_meta(ts, tc, w);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < nm.nc) {
        const int64_t q = nm.c0 + j;
        pR[k] = a.R[q];
        pS[k] = a.Sb[q];
        pu[k] = a.u[q];
        if (first) pg[k] = a.sg_first[q];
      }
      if (j < nm.np) {
        pa[k] = a.ra[nm.h0 + j];
        pb[k] = a.rb[nm.h0 + j];
      }
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= nm.np) pcb[k] = a.cb[nm.h0 + i];
    }
  };
  int64_t w = blockIdx.x;
  if (w < n_tile) fetch(w);
  for (; w < n_tile; w += gridDim.x) {
    const TileMeta m = nm;
    T ca[kPer], cbb[kPer], cS[kPer];  // cS: child j's average sum, j = tid + k * kBlk
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        sR[j] = pR[k];
        cS[k] = pS[k];
        su[j] = pu[k];
        if (first) ss[j] = pg[k];
      }
      ca[k] = pa[k];
      cbb[k] = pb[k];
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= m.np) scb[i] = pcb[k] - m.c0;
    }
    __syncthreads();
    if (w + gridDim.x < n_tile) fetch(w + gridDim.x);
    // one thread per parent: the child -> parent map, the parent's reaches
    // and (unless sigma is given) the regret-matching sum in child order
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i >= m.np) break;
      const int32_t b = scb[i], e = scb[i + 1];
      double sum = 0.0;
      for (int j = b; j < e; ++j) {
        sp[j] = (int16_t)i;
        if (!first) sum += rm_x((double)sR[j], rm_mode, eps);
      }
      sZ[i] = sum;
      sopp[i] = a.mover == 0 ? cbb[k] : ca[k];
      sown[i] = a.mover == 0 ? ca[k] : cbb[k];
    }
    __syncthreads();
    // one thread per child: sigma^t from the regret and the sum
    if (!first) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * kBlk;
        if (j >= m.nc) break;
        const int i = sp[j];
        const double x = rm_x((double)sR[j], rm_mode, eps);
        ss[j] = PAPER ? (T)(x / sZ[i]) : (T)sig_from<T>(x, sZ[i], scb[i + 1] - scb[i]);
      }
      __syncthreads();
    }
    // one thread per parent: u(h) = sum sigma^t u in child order
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i >= m.np) break;
      const int32_t b = scb[i], e = scb[i + 1];
      double uh = 0.0;
      for (int j = b; j < e; ++j) uh += (double)ss[j] * (double)su[j];
      sZ[i] = uh;
      a.u_par[m.h0 + i] = (T)uh;
      if (a.vacc) a.vacc[m.h0 + i] += uh;
    }
    __syncthreads();
    // one thread per child: the regret and average-sum updates
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j >= m.nc) break;
      const int i = sp[j];
      const double uh = sZ[i], opp = (double)sopp[i], own = (double)sown[i];
      const double r = sgn * opp * ((double)su[j] - uh);
      double add = own * (double)ss[j];
      if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
      a.R[m.c0 + j] = (T)regret_update<PAPER>((double)sR[j], r, ik, variant);
      a.Sb[m.c0 + j] = (T)(ik.avg_w * (double)cS[k] + add);
    }
    __syncthreads();  // before the next tile reuses LDS
  }
}

// FindUtility on a level of the compact tail, over LDS-staged tiles of its
// compact children (the tail's parents are its active nodes, a.cb its
// compact CSR): as k_sw_up_tile, except that sigma^t comes from the
// parent's stored regret-matching sum (a.Z, as the tail's down sweep uses
// it) instead of a loop over the siblings, the parent's new sum is stored
// for the next iteration, and the parent's utility goes to its compact
// position (a.upos).  The operations are those of k_sw_up_parent on the
// tail, in the same order.  Not for a call's first iteration.
template <class T, bool PAPER>
__global__ void __launch_bounds__(kBlk)
    k_sw_up_tail_tile(int64_t n_tile, const int32_t *__restrict__ ts,
                      const int32_t *__restrict__ tc, UpArgs<T> a, IterK ik, int variant,
                      int rm_mode, double eps) {
  __shared__ T sR[kTile], sS[kTile], su[kTile], ss[kTile];
  __shared__ int32_t scb[kTile + 1];
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const double sgn = a.mover == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x;
  // registers of the next tile
  TileMeta nm;
  T pR[kPer], pS[kPer], pu[kPer], pa[kPer], pb[kPer];
  double pz[kPer];
  int32_t pcb[kPer + 1];
  auto fetch = [&](int64_t w) {
    nm = tile_meta(ts, tc, w);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < nm.nc) {
        const int64_t q = nm.c0 + j;
        pR[k] = a.R[q];
        pS[k] = a.Sb[q];
        pu[k] = a.u[q];
      }
      if (j < nm.np) {
        pa[k] = a.ra[nm.h0 + j];
        pb[k] = a.rb[nm.h0 + j];
        pz[k] = a.Z[nm.h0 + j];
      }
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= nm.np) pcb[k] = a.cb[nm.h0 + i];
    }
  };
  int64_t w = blockIdx.x;
  if (w < n_tile) fetch(w);
  for (; w < n_tile; w += gridDim.x) {
    const TileMeta m = nm;
    T ca[kPer], cbb[kPer];
    double cz[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        sR[j] = pR[k];
        sS[j] = pS[k];
        su[j] = pu[k];
      }
      ca[k] = pa[k];
      cbb[k] = pb[k];
      cz[k] = pz[k];
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i <= m.np) scb[i] = pcb[k] - m.c0;
    }
    __syncthreads();
    if (w + gridDim.x < n_tile) fetch(w + gridDim.x);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kBlk;
      if (i >= m.np) break;
      const int32_t h = m.h0 + i, b = scb[i], e = scb[i + 1], kk = e - b;
      // sigma^t from the stored sum and u(h) = sum sigma^t u, in child order
      const double Zh = cz[k];
      double uh = 0.0;
      for (int j = b; j < e; ++j) {
        const T sj = (T)sig_of<T>(sR[j], Zh, rm_mode, eps);
        ss[j] = sj;
        uh += (double)sj * (double)su[j];
      }
      const double opp = a.mover == 0 ? (double)cbb[k] : (double)ca[k];
      const double own = a.mover == 0 ? (double)ca[k] : (double)cbb[k];
      double sum = 0.0;
      for (int j = b; j < e; ++j) {
        const double r = sgn * opp * ((double)su[j] - uh);
        const T Rs = (T)regret_update<PAPER>((double)sR[j], r, ik, variant);
        sR[j] = Rs;
        sum += rm_x((double)Rs, rm_mode, eps);
        double add = own * (double)ss[j];
        if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
        sS[j] = (T)(ik.avg_w * (double)sS[j] + add);
      }
      a.u_par[a.upos ? a.upos[h] : h] = (T)uh;
      a.Z[h] = z_enc(sum, kk);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = tid + k * kBlk;
      if (j < m.nc) {
        a.R[m.c0 + j] = sR[j];
        a.Sb[m.c0 + j] = sS[j];
      }
    }
    __syncthreads();  // before the next tile reuses LDS
  }
}

// FindUtility, one thread per parent (all parents of the level, or those in
// `list`): the children in order, as the oracle's loops.
template <class T, bool PAPER>
__global__ void __launch_bounds__(kBlk)
    k_sw_up_parent(int64_t n, const int32_t *__restrict__ list, UpArgs<T> a, IterK ik,
                   int variant, int rm_mode, double eps) {
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const double sgn = a.mover == 0 ? 1.0 : -1.0;
  SW_FOR(i, n) {
    const int32_t h = list ? list[i] : (int32_t)i;
    const int32_t b = a.cb[h], e = a.cb[h + 1], k = e - b;
    // this iteration's regret-matching sum (sigma^t), unless sigma is given
    double Zh = 0.0;
    if (!a.sg_first) Zh = a.Z ? a.Z[h] : z_enc(x_sum(a.R, b, e, rm_mode, eps), k);
    auto sig = [&](int32_t q, T rq) -> double {
      return a.sg_first ? (double)a.sg_first[q] : sig_of<T>(rq, Zh, rm_mode, eps);
    };
    double uh = 0.0;
    for (int32_t q = b; q < e; ++q) uh += sig(q, a.R[q]) * (double)a.u[q];
    const double opp = a.mover == 0 ? (double)a.rb[h] : (double)a.ra[h];
    const double own = a.mover == 0 ? (double)a.ra[h] : (double)a.rb[h];
    double sum = 0.0;
    for (int32_t q = b; q < e; ++q) {
      const T rq = a.R[q];
      const double s = sig(q, rq);
      const double r = sgn * opp * ((double)a.u[q] - uh);
      const T Rs = (T)regret_update<PAPER>((double)rq, r, ik, variant);
      a.R[q] = Rs;
      sum += rm_x((double)Rs, rm_mode, eps);
      double add = own * s;
      if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
      a.Sb[q] = (T)(ik.avg_w * (double)a.Sb[q] + add);
    }
    a.u_par[a.upos ? a.upos[h] : h] = (T)uh;
    if (a.Z) a.Z[h] = z_enc(sum, k);
    if (a.vacc) a.vacc[h] += uh;
  }
}

// ---- compact tail: copies in and out -------------------------------------------

template <class T>
__global__ void k_sw_gather3(int64_t m, const int32_t *__restrict__ map, const T *__restrict__ a,
                             const T *__restrict__ b, const T *__restrict__ c, T *__restrict__ ao,
                             T *__restrict__ bo, T *__restrict__ co) {
  SW_FOR(j, m) {
    const int32_t q = map[j];
    ao[j] = a[q];
    bo[j] = b[q];
    co[j] = c[q];
  }
}

template <class T>
__global__ void k_sw_scatter3(int64_t m, const int32_t *__restrict__ map, const T *__restrict__ a,
                              const T *__restrict__ b, const T *__restrict__ c, T *__restrict__ ao,
                              T *__restrict__ bo, T *__restrict__ co) {
  SW_FOR(j, m) {
    const int32_t q = map[j];
    ao[q] = a[j];
    bo[q] = b[j];
    co[q] = c[j];
  }
}

template <class T>
__global__ void k_sw_scatter1(int64_t m, const int32_t *__restrict__ map, const T *__restrict__ a,
                              T *__restrict__ ao) {
  SW_FOR(j, m) ao[map[j]] = a[j];
}

// stored regret-matching sums of the tail's active parents
template <class T>
__global__ void k_sw_zgather(int64_t m, const int32_t *__restrict__ act,
                             const int32_t *__restrict__ cb, const T *__restrict__ R,
                             double *__restrict__ Zc, int rm_mode, double eps) {
  SW_FOR(i, m) {
    const int32_t b = cb[act[i]], e = cb[act[i] + 1];
    Zc[i] = z_enc(x_sum(R, b, e, rm_mode, eps), e - b);
  }
}

// sigma of the edges into the tail's heads, from the level arrays
template <class T>
__global__ void k_sw_sig_gather(int64_t m, const int32_t *__restrict__ act,
                                const int32_t *__restrict__ par, const int32_t *__restrict__ cb,
                                const T *__restrict__ R, T *__restrict__ out, int rm_mode,
                                double eps) {
  SW_FOR(i, m) {
    const int32_t q = act[i], h = par[q], b = cb[h], e = cb[h + 1];
    out[i] = (T)sig_from<T>(rm_x((double)R[q], rm_mode, eps), x_sum(R, b, e, rm_mode, eps), e - b);
  }
}

// kernel ids of the profile records (pasur_profile_read); work[0] = nodes
// (or children) of the launch, work[1] = parents, work[2] = entries of the
// tail's boundary lists
enum { PK_DOWN = 4, PK_UP = 5, PK_UP_PARENT = 6, PK_UP_LIST = 7, PK_SETUP = 8,
       PK_TAIL_DOWN = 9, PK_TAIL_UP = 10, PK_UP_BND = 11, PK_DOWN_BND = 12, PK_DOWN_LIST = 13,
       PK_DOWN_PARENT = 14 };

// Per-call buffers of the compact tail.
template <class T>
struct Tail {
  T *Rc[9], *Sc[9], *uc[9];  // levels S+1..8, m[L] each
  double *Zc[9];             // levels S..7, n_act[l] each
  T *rac[9], *rbc[9];        // levels S..7
  T *sgS, *uS;               // level S, n_act[S]
  T *bra, *brb;              // boundary parents, n_bp
};

template <class T>
size_t tail_bytes(const SweepIndex &x) {
  size_t b = 0;
  const int S = x.S;
  for (int L = S + 1; L <= 8; ++L) b += 3 * (size_t)x.m[L] * sizeof(T);
  for (int l = S; l <= 7; ++l) b += (size_t)x.n_act[l] * (8 + 2 * sizeof(T));
  b += 2 * (size_t)x.n_act[S] * sizeof(T) + 2 * (size_t)x.n_bp * sizeof(T);
  return b + 64 * 256;
}

template <class T>
void tail_carve(const SweepIndex &x, unsigned char *p, Tail<T> &tl) {
  auto take = [&](size_t bytes) {
    unsigned char *r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  const int S = x.S;
  for (int l = 0; l <= 8; ++l) {
    tl.Rc[l] = tl.Sc[l] = tl.uc[l] = tl.rac[l] = tl.rbc[l] = nullptr;
    tl.Zc[l] = nullptr;
  }
  for (int L = S + 1; L <= 8; ++L) {
    tl.Rc[L] = (T *)take(x.m[L] * sizeof(T));
    tl.Sc[L] = (T *)take(x.m[L] * sizeof(T));
    tl.uc[L] = (T *)take(x.m[L] * sizeof(T));
  }
  for (int l = S; l <= 7; ++l) {
    tl.Zc[l] = (double *)take(x.n_act[l] * 8);
    tl.rac[l] = (T *)take(x.n_act[l] * sizeof(T));
    tl.rbc[l] = (T *)take(x.n_act[l] * sizeof(T));
  }
  tl.sgS = (T *)take(x.n_act[S] * sizeof(T));
  tl.uS = (T *)take(x.n_act[S] * sizeof(T));
  tl.bra = (T *)take(x.n_bp * sizeof(T));
  tl.brb = (T *)take(x.n_bp * sizeof(T));
}

template <class T, bool PAPER>
int sweep_t(pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p, int64_t t0,
            int n_iters, hipStream_t s) {
  const SweepIndex &x = *f->sweep;
  const int rm = p->rm_mode, var = p->variant;
  const double eps = p->eps;
  const bool pos = PAPER && eps > 0.0;
  T *sg[9], *R[9], *Sb[9], *ra[9], *rb[9], *u[9];
  for (int l = 0; l <= 8; ++l) {
    sg[l] = (T *)st->sigma[l];
    R[l] = (T *)st->R[l];
    Sb[l] = (T *)st->Sbar[l];
    ra[l] = (T *)st->reachA[l];
    rb[l] = (T *)st->reachB[l];
    u[l] = (T *)st->u[l];
  }
  // The compact tail pays for its copies over a few iterations; the first
  // and last iteration of a call always run on the level arrays.
  const int S = n_iters >= 3 ? x.S : 0;
  unsigned char *buf = nullptr;
  Tail<T> tl;
  if (S) {
    PASUR_TRY_HIP(hipMallocAsync((void **)&buf, tail_bytes<T>(x), s));
    tail_carve<T>(x, buf, tl);
  }
  {
    ProfScope ps(PK_SETUP, 0, s);
    for (int l = 7; l >= 1; --l)
      if (x.n_act[l] < f->n[l])
        k_sw_chain_u<T><<<grid_of(f->n[l]), kBlk, 0, s>>>(f->n[l], x.passive[l],
                                                           f->child_begin[l], u[l], u[l + 1]);
  }
  auto reach = [&](int L) {
    Reach<T> rc;
    rc.ra_up = ra[L - 1];
    rc.rb_up = rb[L - 1];
    rc.ra = ra[L];
    rc.rb = rb[L];
    rc.bp = rc.bp_tile = nullptr;
    rc.bra = rc.brb = nullptr;
    rc.mover = (L - 1) & 1;
    return rc;
  };
  auto up_args = [&](int L) {
    UpArgs<T> a;
    a.cb = f->child_begin[L - 1];
    a.R = R[L];
    a.Sb = Sb[L];
    a.sg_first = nullptr;
    a.u = u[L];
    a.u_par = u[L - 1];
    a.upos = nullptr;
    a.Z = nullptr;
    a.ra = ra[L - 1];
    a.rb = rb[L - 1];
    a.vacc = L == 1 ? st->vacc : nullptr;
    a.act = a.act_tile = nullptr;
    a.u_act = nullptr;
    a.sg_act = nullptr;
    a.mover = (L - 1) & 1;
    return a;
  };
  // every node of level L (tiles, or one thread per parent)
  auto down_dense = [&](int L, const Reach<T> &rc, const T *sg_first) {
    if (x.tile[L]) {
      const int64_t nt = x.n_tile[L];
      ProfScope ps(rc.bp ? PK_DOWN_BND : PK_DOWN, L, s, f->n[L], f->n[L - 1], rc.bp ? x.n_bp : 0, 0,
                   1);
      auto kern = rc.bp ? (pos ? k_sw_down_tile<T, true, true> : k_sw_down_tile<T, false, true>)
                        : (pos ? k_sw_down_tile<T, true, false> : k_sw_down_tile<T, false, false>);
      kern<<<grid_of(nt * kBlk), kBlk, 0, s>>>(nt, x.tile[L], x.tile_c[L], f->child_begin[L - 1],
                                               R[L], sg_first, rc, rm, eps);
    } else if (f->n[L - 1] > 0) {
      ProfScope ps(PK_DOWN_PARENT, L, s, f->n[L], f->n[L - 1], 0, 0, 1);
      k_sw_down_parent<T><<<grid_of(f->n[L - 1]), kBlk, 0, s>>>(f->n[L - 1], f->child_begin[L - 1],
                                                                 R[L], sg_first, rc, rm, eps);
    }
  };
  // every parent of level L-1 (tiles, or one thread per parent)
  auto up_dense = [&](int L, const UpArgs<T> &a, const IterK &ik) {
    if (x.tile[L]) {
      const int64_t nt = x.n_tile[L];
      ProfScope ps(a.act ? PK_UP_BND : PK_UP, L, s, f->n[L], f->n[L - 1],
                   a.act ? x.n_act[x.S] : 0, 0, 1);
      // wide sibling groups: the per-child form (measured faster where the
      // largest group reaches kWideKids; slower on the tail boundary, whose
      // groups are nearly all of two)
      const bool wide = !a.act && x.kmax[L] >= kWideKids;
      auto kern = a.act ? (pos ? k_sw_up_tile<T, true, true> : k_sw_up_tile<T, false, true>)
                  : wide ? (pos ? k_sw_up_tile_wide<T, true> : k_sw_up_tile_wide<T, false>)
                         : (pos ? k_sw_up_tile<T, true, false> : k_sw_up_tile<T, false, false>);
      kern<<<grid_of(nt * kBlk), kBlk, 0, s>>>(nt, x.tile[L], x.tile_c[L], a, ik, var, rm, eps);
    } else if (f->n[L - 1] > 0) {
      const int64_t n = f->n[L - 1];
      ProfScope ps(PK_UP_PARENT, L, s, f->n[L], n, 0, 0, 1);
      k_sw_up_parent<T, PAPER><<<grid_of(n), kBlk, 0, s>>>(n, nullptr, a, ik, var, rm, eps);
    }
  };
  // one iteration on the level arrays (active parents of the chain levels
  // through their lists; every node on the last iteration's down sweep)
  auto iter_levels = [&](int64_t t, bool first, bool last) {
    const IterK ik = iter_k(p, t);
    for (int L = 1; L <= 7; ++L) {
      const Reach<T> rc = reach(L);
      if (last || x.n_act[L] == f->n[L]) {
        down_dense(L, rc, first ? sg[L] : nullptr);
      } else if (x.n_act[L] > 0) {
        const int64_t n = x.n_act[L];
        ProfScope ps(PK_DOWN_LIST, L, s, n, 0, 0, 0, 1);
        k_sw_down_list<T><<<grid_of(n), kBlk, 0, s>>>(n, x.act[L], f->parent[L], nullptr, R[L],
                                                       first ? sg[L] : nullptr, nullptr,
                                                       f->child_begin[L - 1], rc, rm, eps);
      }
    }
    for (int L = 8; L >= 1; --L) {
      UpArgs<T> a = up_args(L);
      a.sg_first = first ? sg[L] : nullptr;
      if (x.n_act[L - 1] < f->n[L - 1]) {
        const int64_t n = x.n_act[L - 1];
        if (n == 0) continue;
        ProfScope ps(PK_UP_LIST, L, s, x.m[L], n, 0, 0, 1);
        k_sw_up_parent<T, PAPER><<<grid_of(n), kBlk, 0, s>>>(n, x.act[L - 1], a, ik, var, rm, eps);
      } else {
        up_dense(L, a, ik);
      }
    }
  };
  // one iteration with the tail in its compact copies
  auto iter_compact = [&](int64_t t) {
    const IterK ik = iter_k(p, t);
    for (int L = 1; L <= S - 1; ++L) {
      Reach<T> rc = reach(L);
      if (L == S - 1) {
        rc.bp = x.bp;
        rc.bp_tile = x.bp_tile;
        rc.bra = tl.bra;
        rc.brb = tl.brb;
      }
      down_dense(L, rc, nullptr);
    }
    for (int L = S; L <= 7; ++L) {
      const int64_t n = x.n_act[L];
      if (n == 0) continue;
      Reach<T> rc;
      rc.ra_up = L > S ? tl.rac[L - 1] : tl.bra;
      rc.rb_up = L > S ? tl.rbc[L - 1] : tl.brb;
      rc.ra = tl.rac[L];
      rc.rb = tl.rbc[L];
      rc.bp = rc.bp_tile = nullptr;
      rc.bra = rc.brb = nullptr;
      rc.mover = (L - 1) & 1;
      ProfScope ps(PK_TAIL_DOWN, L, s, n, 0, 0, 0, 1);
      k_sw_down_list<T><<<grid_of(n), kBlk, 0, s>>>(
          n, nullptr, x.ppar[L], L > S ? x.jpos[L] : nullptr, L > S ? tl.Rc[L] : nullptr,
          L > S ? nullptr : tl.sgS, L > S ? tl.Zc[L - 1] : nullptr, nullptr, rc, rm, eps);
    }
    for (int L = 8; L >= S + 1; --L) {
      const int64_t n = x.n_act[L - 1];
      if (n == 0) continue;
      UpArgs<T> a = up_args(L);
      a.cb = x.cbc[L - 1];
      a.R = tl.Rc[L];
      a.Sb = tl.Sc[L];
      a.u = tl.uc[L];
      a.u_par = L - 1 > S ? tl.uc[L - 1] : tl.uS;
      a.upos = L - 1 > S ? x.jpos[L - 1] : nullptr;
      a.Z = tl.Zc[L - 1];
      a.ra = tl.rac[L - 1];
      a.rb = tl.rbc[L - 1];
      a.vacc = nullptr;
      ProfScope ps(PK_TAIL_UP, L, s, x.m[L], n, 0, 0, 1);
      if (x.ttile[L]) {
        const int64_t nt = x.n_ttile[L];
        auto kern = pos ? k_sw_up_tail_tile<T, true> : k_sw_up_tail_tile<T, false>;
        kern<<<grid_of(nt * kBlk), kBlk, 0, s>>>(nt, x.ttile[L], x.ttile_c[L], a, ik, var, rm, eps);
      } else {
        k_sw_up_parent<T, PAPER><<<grid_of(n), kBlk, 0, s>>>(n, nullptr, a, ik, var, rm, eps);
      }
    }
    for (int L = S; L >= 1; --L) {
      UpArgs<T> a = up_args(L);
      if (L == S) {
        a.act = x.act[S];
        a.act_tile = x.act_tile;
        a.u_act = tl.uS;
        a.sg_act = tl.sgS;
      }
      up_dense(L, a, ik);
    }
  };
  for (int it = 0; it < n_iters; ++it) {
    const int64_t t = t0 + it;
    const bool first = it == 0, last = it == n_iters - 1;
    if (!S || first || last) {
      if (S && last) {  // the tail's state back into the level arrays
        ProfScope ps(PK_SETUP, 3, s);
        for (int L = S + 1; L <= 8; ++L)
          k_sw_scatter3<T><<<grid_of(x.m[L]), kBlk, 0, s>>>(x.m[L], x.cmap[L], tl.Rc[L], tl.Sc[L],
                                                             tl.uc[L], R[L], Sb[L], u[L]);
        k_sw_scatter1<T><<<grid_of(x.n_act[S]), kBlk, 0, s>>>(x.n_act[S], x.act[S], tl.uS, u[S]);
      }
      iter_levels(t, first, last);
      if (S && first) {  // the tail's state into its compact copies
        ProfScope ps(PK_SETUP, 2, s);
        for (int L = S + 1; L <= 8; ++L)
          k_sw_gather3<T><<<grid_of(x.m[L]), kBlk, 0, s>>>(x.m[L], x.cmap[L], R[L], Sb[L], u[L],
                                                            tl.Rc[L], tl.Sc[L], tl.uc[L]);
        for (int l = S; l <= 7; ++l)
          k_sw_zgather<T><<<grid_of(x.n_act[l]), kBlk, 0, s>>>(x.n_act[l], x.act[l],
                                                                f->child_begin[l], R[l + 1],
                                                                tl.Zc[l], rm, eps);
        k_sw_sig_gather<T><<<grid_of(x.n_act[S]), kBlk, 0, s>>>(
            x.n_act[S], x.act[S], f->parent[S], f->child_begin[S - 1], R[S], tl.sgS, rm, eps);
      }
    } else {
      iter_compact(t);
    }
  }
  {
    ProfScope ps(PK_SETUP, 1, s);
    for (int L = 1; L <= 8; ++L)
      if (f->n[L - 1] > 0)
        k_sw_sigma_out<T><<<grid_of(f->n[L - 1]), kBlk, 0, s>>>(f->n[L - 1], f->child_begin[L - 1],
                                                                 R[L], sg[L], rm, eps);
  }
  hipError_t e = hipGetLastError();
  if (buf) (void)hipFreeAsync(buf, s);
  if (e != hipSuccess) {
    set_error("streaming sweeps: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  return PASUR_OK;
}

}  // namespace

bool sweep_pays(const pasur_fgt *f) {
  // Measured on whole games (1000 iterations per round, streaming vs
  // persistent segments): the streaming sweeps pay about 30 launches per
  // iteration and overtake the segment kernel between 7.7e6 nodes (137 vs
  // 112 ms, deal 1 round 5) and 9.7e6 (136 vs 146 ms, deal 1 round 6);
  // 1.1e7: 133 vs 181 ms; 3.5e7: 231 vs 454 ms; 1.1e8: 442 vs 1372 ms.
  int64_t nodes = 0;
  for (int l = 0; l <= 8; ++l) nodes += f->n[l];
  return nodes >= (int64_t)9 * 1000 * 1000;
}

int sweep_iterate(pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p,
                  int64_t t0, int n_iters, hipStream_t s) {
  if (n_iters == 0) return PASUR_OK;
  if (!f->sweep) PASUR_TRY(build_index(f, s));
  const bool paper = p->variant == PASUR_DCFR && p->rm_mode == PASUR_RM_FLOOR;
  if (st->dtype == PASUR_F32)
    return paper ? sweep_t<float, true>(f, st, p, t0, n_iters, s)
                 : sweep_t<float, false>(f, st, p, t0, n_iters, s);
  return paper ? sweep_t<double, true>(f, st, p, t0, n_iters, s)
               : sweep_t<double, false>(f, st, p, t0, n_iters, s);
}

}  // namespace pasur
