// pasur_cfr.hip -- full-width DCFR on one round's unfolded tree, leaf
// utilities, average strategy, round values and exact tree values (best
// response / minimax) as level-synchronous HIP kernels.
//
// State is stored as T (float or double); every arithmetic step runs in
// double registers, with the operations of each parent's update done in the
// order of the paper's FindUtility (sum, regret, discount, matching,
// average).  Contraction of a*b+c into fma is switched off so that the
// double-state path rounds exactly like a plain sequential implementation.
#pragma clang fp contract(off)

#include "pasur_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

using namespace pasur;

namespace {

// Optional per-launch timing of the sweep kernels (HIP events on the launch
// stream), off unless pasur_profile_enable(1) was called.
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;  // events of cleared records, reused
bool g_prof_on = false;
uint64_t g_prof_mask = ~0ull;  // kernel ids recorded (bit k)

void prof_clear() {
  for (auto &r : g_prof) {
    g_event_pool.push_back(r.a);
    g_event_pool.push_back(r.b);
  }
  g_prof.clear();
}

constexpr int kThreads = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

template <class T>
__global__ void k_init_level(int64_t n, const int32_t *__restrict__ parent,
                             const int32_t *__restrict__ cb_up, T *__restrict__ sigma,
                             T *__restrict__ R, T *__restrict__ Sbar) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t h = parent[q];
  const int32_t k = cb_up[h + 1] - cb_up[h];
  sigma[q] = (T)(1.0 / (double)k);
  R[q] = (T)0;
  Sbar[q] = (T)0;
}

template <class T>
__global__ void k_init_roots(int64_t n, T *__restrict__ ra, T *__restrict__ rb,
                             double *__restrict__ vacc) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  ra[j] = (T)1;
  rb[j] = (T)1;
  vacc[j] = 0.0;
}

// FindReachProbability, one level: the mover's reach picks up sigma of the
// edge taken, the other player's reach is inherited.
template <class T>
__global__ void k_down(int64_t n, int mover, const int32_t *__restrict__ parent,
                       const T *__restrict__ sigma, const T *__restrict__ ra_up,
                       const T *__restrict__ rb_up, T *__restrict__ ra, T *__restrict__ rb) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t h = parent[q];
  double a = (double)ra_up[h];
  double b = (double)rb_up[h];
  if (mover == 0) a *= (double)sigma[q];
  else b *= (double)sigma[q];
  ra[q] = (T)a;
  rb[q] = (T)b;
}

// FindUtility, one level, one thread per parent h (children cb[h]..cb[h+1]):
//   u(h) = sum sigma^t u;  r = s_p pi_{-p}(h) (u(q) - u(h));
//   R <- d R + r;  sigma^{t+1} = max(R, eps) / sum;  Sbar <- w Sbar + pi_p(h) sigma^t
// (with PASUR_CFR_SNIPPET_AVG the term also carries sigma^{t+1}, as stored).
constexpr double kSnippetTol = 1e-5;
template <class T>
__global__ void k_up(int64_t np, int mover, const int32_t *__restrict__ cb,
                     T *__restrict__ sigma, T *__restrict__ R, T *__restrict__ Sbar,
                     const T *__restrict__ u_child, T *__restrict__ u_par,
                     const T *__restrict__ ra, const T *__restrict__ rb, IterConsts ic,
                     double *__restrict__ vacc) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np) return;
  const int32_t b = cb[h], e = cb[h + 1];
  double uh = 0.0;
  for (int32_t q = b; q < e; ++q) uh += (double)sigma[q] * (double)u_child[q];
  u_par[h] = (T)uh;
  const double opp = mover == 0 ? (double)rb[h] : (double)ra[h];
  const double own = mover == 0 ? (double)ra[h] : (double)rb[h];
  const double sgn = mover == 0 ? 1.0 : -1.0;
  for (int32_t q = b; q < e; ++q) {
    const double r = sgn * opp * ((double)u_child[q] - uh);
    double Rq = (double)R[q];
    if (ic.variant == PASUR_DCFR) {
      const bool pos = (ic.flags & PASUR_CFR_SNIPPET_TOL) ? Rq >= kSnippetTol : Rq > 0.0;
      const double d = pos ? ic.dpos : ic.dneg;
      Rq = d * Rq + r;
    } else if (ic.variant == PASUR_CFR_PLUS) {
      Rq = Rq + r;
      if (Rq < 0.0) Rq = 0.0;
    } else {
      Rq = Rq + r;
    }
    R[q] = (T)Rq;
  }
  double sum = 0.0;
  for (int32_t q = b; q < e; ++q) {
    const double x = ic.rm_mode == PASUR_RM_FLOOR ? fmax((double)R[q], ic.eps)
                                                  : fmax((double)R[q], 0.0);
    sum += x;
  }
  const double inv_k = 1.0 / (double)(e - b);
  for (int32_t q = b; q < e; ++q) {
    const double x = ic.rm_mode == PASUR_RM_FLOOR ? fmax((double)R[q], ic.eps)
                                                  : fmax((double)R[q], 0.0);
    const double s_new = sum > 0.0 ? x / sum : inv_k;
    double add = own * (double)sigma[q];
    if (ic.variant == PASUR_CFR_PLUS) add *= ic.avg_t;
    if (ic.flags & PASUR_CFR_SNIPPET_AVG) add *= (double)(T)s_new;
    Sbar[q] = (T)(ic.avg_w * (double)Sbar[q] + add);
    sigma[q] = (T)s_new;
  }
  if (vacc) vacc[h] += uh;
}


// ---------------------------------------------------------------------------
// Persistent segment schedule.  The subgames below different roots never
// interact inside a round (every root has reach 1), so one workgroup owns a
// segment -- a run of consecutive roots of one tree, whose nodes are
// contiguous on every level -- and runs all iterations on it with workgroup
// barriers between levels.  When the segment's state fits in LDS (160 KB per
// workgroup on gfx950) it is loaded once, iterated in LDS and written back
// once; otherwise the same loop runs in place in global memory (L2/MALL
// resident).  Each parent is still updated by one thread in child order, so
// results are bit-identical to the level-synchronous kernels.  A launch can
// cover the trees of many deals (batched solve).
// ---------------------------------------------------------------------------

// One (tree, state) pair of a launch.
template <class T>
struct ItemDesc {
  const int32_t *off[9];     // per-root level offsets
  const int32_t *parent[9];  // levels 1..8
  const int32_t *cb[9];      // levels 0..7
  T *sigma[9], *R[9], *Sbar[9], *ra[9], *rb[9], *u[9];
  double *vacc;
};

struct Seg {
  int32_t item, j0, j1, pad;  // roots j0 .. j1-1 of item
};

extern __shared__ __align__(16) unsigned char g_lds[];
// per level of the segment in LDS (set at load): largest sibling group, and
// whether the up sweep runs one lane per child in chunks (1) or one lane per
// parent (0)
__shared__ int g_kmax[9];
__shared__ int g_chunked[9];
// g_fold[p] = 1: every node of level p has exactly one child, and the up
// phase of level p+1 is folded into that of level p (no barrier of its own)
__shared__ int g_fold[9];

// Byte layout of one segment's state in LDS (shared by host sizing and
// device carving).  Level l occupies one block starting at base[l]: its T
// arrays in fixed slots of stride[l] = align16(n_l * sizeof(T)) bytes --
// u (slot 0), sigma, R, Sbar (slots 1-3, levels 1..8), reachA, reachB
// (slots 4-5, levels 0..7; level 8 has only slots 0-3) -- then the 16-bit
// segment-local parent (levels 1..8) and child_begin (levels 0..7) indices.
// Levels 1..8 end with their chunk starts (16-bit, chunk_cap(n_l) entries):
// the up sweep hands children to lanes in chunks of at most 64 that never
// split a sibling group.  The roots' utility sums (double) follow the last
// level.
// Every address is base + slot * stride, so a kernel keeps two scalars per
// level instead of one offset per array.
enum { F_U = 0, F_SG = 1, F_R = 2, F_SB = 3, F_RA = 4, F_RB = 5 };

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }
__host__ __device__ inline uint32_t lds_tslots(int l) { return l == 8 ? 4u : 6u; }
// capacity of a level's chunk-start array: chunks hold at least 32 children
__host__ __device__ inline uint32_t chunk_cap(int n) { return (uint32_t)(n + 31) / 32u + 2u; }

struct LdsLayout {
  uint32_t base[9], stride[9];
  uint32_t vacc;  // double per root: running sum of root utilities
  uint32_t bytes;
};

__host__ __device__ inline LdsLayout lds_layout(const int cnt[9], uint32_t tsize) {
  LdsLayout L;
  uint32_t p = 0;
  for (int l = 0; l <= 8; ++l) {
    L.base[l] = p;
    L.stride[l] = align16((uint32_t)cnt[l] * tsize);
    p += lds_tslots(l) * L.stride[l];
    if (l >= 1) p += align16((uint32_t)cnt[l] * 2u);
    if (l <= 7) p += align16((uint32_t)(cnt[l] + 1) * 2u);
    if (l >= 1) p += align16(chunk_cap(cnt[l]) * 2u);
  }
  L.vacc = p;
  p += align16((uint32_t)cnt[0] * 8u);
  L.bytes = p;
  return L;
}

// A uniform value the optimiser must treat as unknown at each use.  Without
// it, loop-invariant code motion lifts every level's per-lane LDS addresses
// (9 levels x 8 arrays) out of the iteration loop; they do not fit in
// registers and spill to scratch, and each level phase then starts with
// scratch reloads.  Recomputing an address costs a few scalar operations.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  x = __builtin_amdgcn_readfirstlane(x);
  asm volatile("" : "+s"(x));
  return x;
}

template <class T>
struct LdsArr {
  uint32_t off;
  __device__ __forceinline__ T &operator[](int i) const { return reinterpret_cast<T *>(g_lds + off)[i]; }
};

// A segment's state in LDS, addressed through lds_layout.
template <class T>
struct SubLds {
  uint32_t base[9], stride[9], vacc;
  int cnt[9];
  __device__ __forceinline__ void vacc_add(int h, double v, double &) const {
    LdsArr<double>{opaque(vacc)}[h] += v;
  }
  __device__ __forceinline__ LdsArr<T> f(int l, int slot) const {
    return {opaque(base[l]) + slot * opaque(stride[l])};
  }
  __device__ __forceinline__ LdsArr<T> sg(int l) const { return f(l, F_SG); }
  __device__ __forceinline__ LdsArr<T> Rr(int l) const { return f(l, F_R); }
  __device__ __forceinline__ LdsArr<T> Sb(int l) const { return f(l, F_SB); }
  __device__ __forceinline__ LdsArr<T> uu(int l) const { return f(l, F_U); }
  __device__ __forceinline__ LdsArr<T> ra(int l) const { return f(l, F_RA); }
  __device__ __forceinline__ LdsArr<T> rb(int l) const { return f(l, F_RB); }
  __device__ __forceinline__ LdsArr<uint16_t> par(int l) const {
    return {opaque(base[l]) + lds_tslots(l) * opaque(stride[l])};
  }
  __device__ __forceinline__ LdsArr<uint16_t> cbl(int l) const {
    return {opaque(base[l]) + lds_tslots(l) * opaque(stride[l]) +
            (l >= 1 ? align16((uint32_t)cnt[l] * 2u) : 0u)};
  }
  __device__ __forceinline__ LdsArr<uint16_t> chk(int l) const {
    return {opaque(base[l]) + lds_tslots(l) * opaque(stride[l]) +
            align16((uint32_t)cnt[l] * 2u) + (l <= 7 ? align16((uint32_t)(cnt[l] + 1) * 2u) : 0u)};
  }
  static constexpr bool chunked() { return true; }
  __device__ __forceinline__ int par_sub(int) const { return 0; }
  __device__ __forceinline__ int cb_sub(int) const { return 0; }
};

// FindUtility for one parent whose children sit at b..e-1 of the level
// arrays: returns u(h) and updates R, sigma and Sbar of the children, in the
// same operation order as k_up.
template <class T, class AS, class AR, class AB, class AU>
__device__ __forceinline__ double update_parent(const AS &sg, const AR &Rr, const AB &Sb,
                                                const AU &uu, int b, int e, int mover,
                                                double opp, double own, const IterK &ik,
                                                int variant, int rm_mode, double eps) {
  const double sgn = mover == 0 ? 1.0 : -1.0;
  double uh = 0.0;
  for (int q = b; q < e; ++q) uh += (double)sg[q] * (double)uu[q];
  double sum = 0.0;
  for (int q = b; q < e; ++q) {
    const double r = sgn * opp * ((double)uu[q] - uh);
    double Rq = (double)Rr[q];
    if (variant == PASUR_DCFR) {
      const double d = Rq > 0.0 ? ik.dpos : ik.dneg;
      Rq = d * Rq + r;
    } else if (variant == PASUR_CFR_PLUS) {
      Rq = Rq + r;
      if (Rq < 0.0) Rq = 0.0;
    } else {
      Rq = Rq + r;
    }
    const T Rs = (T)Rq;
    Rr[q] = Rs;
    sum += rm_mode == PASUR_RM_FLOOR ? fmax((double)Rs, eps) : fmax((double)Rs, 0.0);
  }
  // sum is positive unless no regret is (RM+ or a zero floor); 1/k is then
  // computed on that branch only
  const double inv_k = sum > 0.0 ? 0.0 : 1.0 / (double)(e - b);
  for (int q = b; q < e; ++q) {
    const double x = rm_mode == PASUR_RM_FLOOR ? fmax((double)Rr[q], eps) : fmax((double)Rr[q], 0.0);
    const double s_new = sum > 0.0 ? x / sum : inv_k;
    double add = own * (double)sg[q];
    if (variant == PASUR_CFR_PLUS) add *= ik.avg_t;
    Sb[q] = (T)(ik.avg_w * (double)Sb[q] + add);
    sg[q] = (T)s_new;
  }
  return uh;
}

// FindUtility of node q of level F-1 whose only child c is on level F, as
// update_parent does it for one child: u(q) = 0 + sigma(c) u(c), the regret
// and average-sum updates of c; sigma(c) stays 1 (max(R, eps) / itself, or
// 1/k when that sum is 0).  Stores u(q) and returns it as the parent
// update will read it back (rounded to T).
template <class T, int F, class SubT>
__device__ __forceinline__ double fold_single(const SubT &S, int q, const IterK &ik, int variant) {
  const int mover = (F - 1) & 1;
  const double sgn = mover == 0 ? 1.0 : -1.0;
  const int c = (int)S.cbl(F - 1)[q] - S.cb_sub(F - 1);
  const double opp = mover == 0 ? (double)S.rb(F - 1)[q] : (double)S.ra(F - 1)[q];
  const double own = mover == 0 ? (double)S.ra(F - 1)[q] : (double)S.rb(F - 1)[q];
  const T sc = S.sg(F)[c], ucT = S.uu(F)[c], rc = S.Rr(F)[c], bc = S.Sb(F)[c];
  const double uq = 0.0 + (double)sc * (double)ucT;
  const double r = sgn * opp * ((double)ucT - uq);
  double Rq = (double)rc;
  if (variant == PASUR_DCFR) {
    const double d = Rq > 0.0 ? ik.dpos : ik.dneg;
    Rq = d * Rq + r;
  } else if (variant == PASUR_CFR_PLUS) {
    Rq = Rq + r;
    if (Rq < 0.0) Rq = 0.0;
  } else {
    Rq = Rq + r;
  }
  double add = own * (double)sc;
  if (variant == PASUR_CFR_PLUS) add *= ik.avg_t;
  S.Rr(F)[c] = (T)Rq;
  S.Sb(F)[c] = (T)(ik.avg_w * (double)bc + add);
  S.sg(F)[c] = (T)1.0;
  const T uqT = (T)uq;
  S.uu(F - 1)[q] = uqT;
  return (double)uqT;
}

// FindUtility for the parents h0, h0+nt, ... of level l-1 (children on level l).
template <class T, int L, class SubT>
__device__ __forceinline__ void up_one(const SubT &S, const IterK &k, int variant, int rm_mode,
                                       double eps, double &vacc_reg, bool fold = false) {
  const int mover = (L - 1) & 1;
  int t0 = threadIdx.x;
  asm volatile("" : "+v"(t0));  // per-lane start stays inside the phase (see opaque)
  for (int h = t0; h < S.cnt[L - 1]; h += blockDim.x) {
    const int b = (int)S.cbl(L - 1)[h] - S.cb_sub(L - 1);
    const int e = (int)S.cbl(L - 1)[h + 1] - S.cb_sub(L - 1);
    if constexpr (L <= 7) {
      if (fold)
        for (int q = b; q < e; ++q) (void)fold_single<T, L + 1>(S, q, k, variant);
    }
    const double opp = mover == 0 ? (double)S.rb(L - 1)[h] : (double)S.ra(L - 1)[h];
    const double own = mover == 0 ? (double)S.ra(L - 1)[h] : (double)S.rb(L - 1)[h];
    const double uh = update_parent<T>(S.sg(L), S.Rr(L), S.Sb(L), S.uu(L), b, e, mover, opp,
                                       own, k, variant, rm_mode, eps);
    S.uu(L - 1)[h] = (T)uh;
    if (L == 1) S.vacc_add(h, uh, vacc_reg);
  }
}

// Largest sibling group the chunked up sweep handles (chunks of at most 64
// children then start at least every 32 children).
constexpr int kMaxChunkGroup = 33;

// FindUtility on level L, one lane per child: wave w takes chunks w, w+nw,
// ... of the level's children (a chunk never splits a sibling group); the
// two per-parent sums (sigma*u, and the regret-matching denominator) are
// group_sum scans, every other operation is per child and in k_up's order.
// The last child of each group writes the parent's utility.
template <class T, int L, class SubT>
__device__ __forceinline__ void up_chunked(const SubT &S, const IterK &ik, int variant,
                                           int rm_mode, double eps, double &vacc_reg,
                                           bool fold = false) {
  const int mover = (L - 1) & 1;
  const double sgn = mover == 0 ? 1.0 : -1.0;
  const int lane = (int)(threadIdx.x & 63), nw = (int)(blockDim.x >> 6);
  int w = (int)(threadIdx.x >> 6);
  asm volatile("" : "+v"(w));  // (see opaque)
  const int n = S.cnt[L], cap = (int)chunk_cap(n);
  for (int c = w; c + 1 < cap; c += nw) {
    const int c0 = S.chk(L)[c], c1 = S.chk(L)[c + 1];
    if (c0 >= n) break;
    if (c1 <= c0) continue;
    const bool valid = c0 + lane < c1;
    const int q = valid ? c0 + lane : c1 - 1;
    const int h = (int)S.par(L)[q] - S.par_sub(L);
    const T sq = S.sg(L)[q], rq = S.Rr(L)[q], bq = S.Sb(L)[q];
    T uq = (T)0;
    if constexpr (L <= 7) {
      if (fold) {
        if (valid) uq = (T)fold_single<T, L + 1>(S, q, ik, variant);
      } else {
        uq = S.uu(L)[q];
      }
    } else {
      uq = S.uu(L)[q];
    }
    const int b = (int)S.cbl(L - 1)[h] - S.cb_sub(L - 1);
    const int e = (int)S.cbl(L - 1)[h + 1] - S.cb_sub(L - 1);
    const double opp = mover == 0 ? (double)S.rb(L - 1)[h] : (double)S.ra(L - 1)[h];
    const double own = mover == 0 ? (double)S.ra(L - 1)[h] : (double)S.rb(L - 1)[h];
    const int pos = q - b, k = e - b;
    const int kw = wave_max(k);
    const double uh = group_sum((double)sq * (double)uq, pos, k, kw);
    const double r = sgn * opp * ((double)uq - uh);
    double Rq = (double)rq;
    if (variant == PASUR_DCFR) {
      const double d = Rq > 0.0 ? ik.dpos : ik.dneg;
      Rq = d * Rq + r;
    } else if (variant == PASUR_CFR_PLUS) {
      Rq = Rq + r;
      if (Rq < 0.0) Rq = 0.0;
    } else {
      Rq = Rq + r;
    }
    const T Rs = (T)Rq;
    const double x = rm_mode == PASUR_RM_FLOOR ? fmax((double)Rs, eps) : fmax((double)Rs, 0.0);
    const double sum = group_sum(x, pos, k, kw);
    double add = own * (double)sq;
    if (variant == PASUR_CFR_PLUS) add *= ik.avg_t;
    if (valid) {
      const double s_new = sum > 0.0 ? x / sum : 1.0 / (double)k;
      S.Rr(L)[q] = Rs;
      S.Sb(L)[q] = (T)(ik.avg_w * (double)bq + add);
      S.sg(L)[q] = (T)s_new;
      if (pos == k - 1) {
        S.uu(L - 1)[h] = (T)uh;
        if (L == 1) S.vacc_add(h, uh, vacc_reg);
      }
    }
  }
}

// One level of the up sweep, then the workgroup barrier.
template <class T, int L, class SubT>
__device__ __forceinline__ void up_phase(const SubT &S, const IterK &k, int variant, int rm_mode,
                                         double eps, double &vacc_reg) {
  if constexpr (SubT::chunked()) {
    if (L >= 2 && g_fold[L - 1]) return;  // done by the phase of level L-1
    const bool fold = L <= 7 && g_fold[L];
    if (g_chunked[L])
      up_chunked<T, L>(S, k, variant, rm_mode, eps, vacc_reg, fold);
    else
      up_one<T, L>(S, k, variant, rm_mode, eps, vacc_reg, fold);
  } else {
    up_one<T, L>(S, k, variant, rm_mode, eps, vacc_reg);
  }
  __syncthreads();
}

// All iterations of one segment (FindReachProbability then FindUtility per
// iteration, as in k_down / k_up): every level is one phase of the whole
// workgroup, one thread per node (down) or per parent (up), with a barrier
// between levels.
//
// PAPER fixes the paper's variant (DCFR with the regret floor) at compile time,
// which removes the per-child variant tests from the loop.
template <class T, bool PAPER, class SubT>
__device__ __forceinline__ void subtree_iterations(const SubT &S, const IterK *__restrict__ ks,
                                                   int n_iters, int variant, int rm_mode,
                                                   double eps, double &vacc_reg) {
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int it = 0; it < n_iters; ++it) {
    const IterK k = ks[it];
    // FindReachProbability, two levels per phase: a node of the second level
    // l+1 starts from its grandparent's reaches and applies its parent's and
    // its own action probability, rounding to T after each level exactly as
    // the level-by-level form does (the movers alternate, so each level
    // scales one of the two reaches).
#pragma unroll
    for (int l = 1; l <= 7; l += 2) {
      const int l2 = l < 7 ? l + 1 : 0;  // second level of the phase (0: none)
      const int n1 = S.cnt[l], n2 = l2 ? S.cnt[l2] : 0;
      int t0 = tid;
      asm volatile("" : "+v"(t0));  // per-lane start stays inside the phase (see opaque)
      for (int i = t0; i < n1 + n2; i += nt) {
        if (i < n1) {
          const int h = (int)S.par(l)[i] - S.par_sub(l);
          double a = (double)S.ra(l - 1)[h];
          double b = (double)S.rb(l - 1)[h];
          if (((l - 1) & 1) == 0) a *= (double)S.sg(l)[i];
          else b *= (double)S.sg(l)[i];
          S.ra(l)[i] = (T)a;
          S.rb(l)[i] = (T)b;
        } else if (l2) {
          const int q = i - n1;
          const int h = (int)S.par(l2)[q] - S.par_sub(l2);
          const int g = (int)S.par(l)[h] - S.par_sub(l);
          double a = (double)S.ra(l - 1)[g];
          double b = (double)S.rb(l - 1)[g];
          if (((l - 1) & 1) == 0) a *= (double)S.sg(l)[h];
          else b *= (double)S.sg(l)[h];
          a = (double)(T)a;
          b = (double)(T)b;
          if (((l2 - 1) & 1) == 0) a *= (double)S.sg(l2)[q];
          else b *= (double)S.sg(l2)[q];
          S.ra(l2)[q] = (T)a;
          S.rb(l2)[q] = (T)b;
        }
      }
      __syncthreads();
    }
    up_phase<T, 8>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 7>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 6>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 5>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 4>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 3>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 2>(S, k, variant, rm_mode, eps, vacc_reg);
    up_phase<T, 1>(S, k, variant, rm_mode, eps, vacc_reg);
  }
}

template <class T, int BLOCK, bool PAPER>
__device__ __forceinline__ void seg_in_lds(const ItemDesc<T> &D, int j0, int nroots, const int lo[9],
                                  const int cnt[9], const LdsLayout &L,
                                  const IterK *__restrict__ ks, int n_iters, int variant,
                                  int rm_mode, double eps) {
  const int tid = threadIdx.x;
  SubLds<T> S;
#pragma unroll
  for (int l = 0; l <= 8; ++l) {
    S.base[l] = L.base[l];
    S.stride[l] = L.stride[l];
    S.cnt[l] = cnt[l];
  }
  S.vacc = L.vacc;
  const LdsArr<double> vacc{L.vacc};
  // load the segment's state
#pragma unroll
  for (int l = 0; l <= 8; ++l) {
    for (int i = tid; i < cnt[l]; i += BLOCK) {
      if (l >= 1) {
        S.sg(l)[i] = D.sigma[l][lo[l] + i];
        S.Rr(l)[i] = D.R[l][lo[l] + i];
        S.Sb(l)[i] = D.Sbar[l][lo[l] + i];
        S.par(l)[i] = (uint16_t)(D.parent[l][lo[l] + i] - lo[l - 1]);
      }
      if (l == 8) S.uu(l)[i] = D.u[l][lo[l] + i];
      if (l == 0) {
        S.ra(0)[i] = D.ra[0][lo[0] + i];
        S.rb(0)[i] = D.rb[0][lo[0] + i];
      }
    }
    if (l <= 7)
      for (int i = tid; i <= cnt[l]; i += BLOCK)
        S.cbl(l)[i] = (uint16_t)(D.cb[l][lo[l] + i] - lo[l + 1]);
  }
  for (int i = tid; i < nroots; i += BLOCK) vacc[i] = D.vacc[j0 + i];
  if (tid <= 8) g_kmax[tid] = 0;
  __syncthreads();
  // largest sibling group per level, then the chunk starts of the up sweep:
  // chunk c begins at the first sibling of child c*stride, stride = 64 - (kmax - 1),
  // so a chunk holds at most 64 children; unused entries hold n
#pragma unroll
  for (int l = 1; l <= 8; ++l) {
    int km = 0;
    for (int h = tid; h < cnt[l - 1]; h += BLOCK) {
      const int k = (int)S.cbl(l - 1)[h + 1] - (int)S.cbl(l - 1)[h];
      km = k > km ? k : km;
    }
    if (km > 0) atomicMax(&g_kmax[l], km);
  }
  __syncthreads();
  // Lanes per child pay off where siblings groups of 3 or more make the
  // per-parent loops diverge, unless chunking needs more passes than one lane
  // per parent (measured on the two-round and full-game trees).
#pragma unroll
  for (int l = 1; l <= 8; ++l) {
    const int km = g_kmax[l];
    const int stride = 64 - ((km > 1 ? km : 1) - 1);
    const int passes_child = ((cnt[l] + stride - 1) / stride + BLOCK / 64 - 1) / (BLOCK / 64);
    const int passes_parent = (cnt[l - 1] + BLOCK - 1) / BLOCK;
    const bool chunked = km >= 3 && km <= kMaxChunkGroup && passes_child <= passes_parent;
    if (tid == 0) g_chunked[l] = chunked ? 1 : 0;
    if (!chunked) continue;
    const int cap = (int)chunk_cap(cnt[l]);
    for (int c = tid; c < cap; c += BLOCK) {
      const int x = c * stride;
      S.chk(l)[c] = (uint16_t)(x < cnt[l] ? (int)S.cbl(l - 1)[S.par(l)[x]] : cnt[l]);
    }
  }
  // A level whose nodes all have one child folds into the phase above it when
  // that phase keeps the extra work parallel (one lane per child, or one
  // child per parent), one level at a time: the absorbing phase is not
  // itself folded.  Measured: folding into a one-lane-per-parent phase with
  // larger fan-out serialises the folded updates and costs more than the
  // barrier it saves.
  if (tid == 0) {
    for (int l = 0; l <= 8; ++l) g_fold[l] = 0;
    for (int f = 8; f >= 2; --f)
      if (g_kmax[f] == 1 && cnt[f] > 0 && !g_fold[f] &&
          (g_chunked[f - 1] || g_kmax[f - 1] == 1))
        g_fold[f - 1] = 1;
  }
  __syncthreads();
  double unused = 0.0;
  subtree_iterations<T, PAPER>(S, ks, n_iters, variant, rm_mode, eps, unused);
  // write the state back
#pragma unroll
  for (int l = 0; l <= 8; ++l) {
    for (int i = tid; i < cnt[l]; i += BLOCK) {
      if (l >= 1) {
        D.sigma[l][lo[l] + i] = S.sg(l)[i];
        D.R[l][lo[l] + i] = S.Rr(l)[i];
        D.Sbar[l][lo[l] + i] = S.Sb(l)[i];
      }
      if (l <= 7) {
        D.u[l][lo[l] + i] = S.uu(l)[i];
        D.ra[l][lo[l] + i] = S.ra(l)[i];
        D.rb[l][lo[l] + i] = S.rb(l)[i];
      }
    }
  }
  for (int i = tid; i < nroots; i += BLOCK) D.vacc[j0 + i] = vacc[i];
}

// Global-memory arrays addressed through a per-workgroup pointer table kept
// in LDS, so that the 72 per-level pointers are not all live in registers.
__shared__ void *g_ptab[8][9];
__shared__ int g_sub[2][9];

template <class T, int SLOT>
struct TabArr {
  int l;
  __device__ __forceinline__ T &operator[](int i) const { return reinterpret_cast<T *>(g_ptab[SLOT][l])[i]; }
};

template <class T, int BLOCK, bool PAPER>
__device__ __forceinline__ void seg_in_global(const ItemDesc<T> &D, int j0, int nroots, const int lo[9],
                                     const int cnt[9], const IterK *__restrict__ ks,
                                     int n_iters, int variant, int rm_mode, double eps) {
  if (threadIdx.x < 9) {
    const int l = threadIdx.x;
    g_ptab[0][l] = l >= 1 ? (void *)(D.sigma[l] + lo[l]) : nullptr;
    g_ptab[1][l] = l >= 1 ? (void *)(D.R[l] + lo[l]) : nullptr;
    g_ptab[2][l] = l >= 1 ? (void *)(D.Sbar[l] + lo[l]) : nullptr;
    g_ptab[3][l] = (void *)(D.u[l] + lo[l]);
    g_ptab[4][l] = l <= 7 ? (void *)(D.ra[l] + lo[l]) : nullptr;
    g_ptab[5][l] = l <= 7 ? (void *)(D.rb[l] + lo[l]) : nullptr;
    g_ptab[6][l] = l >= 1 ? (void *)(D.parent[l] + lo[l]) : nullptr;
    g_ptab[7][l] = l <= 7 ? (void *)(D.cb[l] + lo[l]) : nullptr;
    g_sub[0][l] = l >= 1 ? lo[l - 1] : 0;
    g_sub[1][l] = l <= 7 ? lo[l + 1] : 0;
  }
  __syncthreads();
  struct SubT {
    int cnt[9];
    __device__ __forceinline__ TabArr<T, 0> sg(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<T, 1> Rr(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<T, 2> Sb(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<T, 3> uu(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<T, 4> ra(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<T, 5> rb(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<const int32_t, 6> par(int l) const { return {l}; }
    __device__ __forceinline__ TabArr<const int32_t, 7> cbl(int l) const { return {l}; }
    __device__ __forceinline__ int par_sub(int l) const { return g_sub[0][l]; }
    __device__ __forceinline__ int cb_sub(int l) const { return g_sub[1][l]; }
    static constexpr bool chunked() { return false; }
    // Segments that run in global memory hold one root (the plan packs
    // several roots only into segments that fit in LDS); that root's sum is
    // kept in a register of thread 0, which updates it.
    double *vacc_g;
    __device__ __forceinline__ void vacc_add(int h, double v, double &reg) const {
      if (h == 0) reg += v;
      else vacc_g[h] += v;
    }
  } X;
#pragma unroll
  for (int l = 0; l <= 8; ++l) X.cnt[l] = cnt[l];
  X.vacc_g = D.vacc + j0;
  double vacc_reg = threadIdx.x == 0 ? D.vacc[j0] : 0.0;
  subtree_iterations<T, PAPER>(X, ks, n_iters, variant, rm_mode, eps, vacc_reg);
  if (threadIdx.x == 0) D.vacc[j0] = vacc_reg;
}

// One workgroup per segment; the segment runs in LDS when its state fits in
// the launch's dynamic LDS (lds_bytes), otherwise in global memory.
template <class T, int BLOCK, bool PAPER>
__global__ void __launch_bounds__(BLOCK)
    k_cfr_seg(const ItemDesc<T> *__restrict__ items, const Seg *__restrict__ segs,
              const IterK *__restrict__ ks, int n_iters, int variant, int rm_mode, double eps,
              uint32_t lds_bytes) {
  const Seg sg = segs[blockIdx.x];
  const ItemDesc<T> &D = items[sg.item];
  int lo[9], cnt[9];
  int mx = 0;
#pragma unroll
  for (int l = 0; l <= 8; ++l) {
    lo[l] = D.off[l][sg.j0];
    cnt[l] = D.off[l][sg.j1] - lo[l];
    mx = cnt[l] > mx ? cnt[l] : mx;
  }
  const LdsLayout L = lds_layout(cnt, sizeof(T));
  if (L.bytes <= lds_bytes && mx < 65535)
    seg_in_lds<T, BLOCK, PAPER>(D, sg.j0, sg.j1 - sg.j0, lo, cnt, L, ks, n_iters, variant, rm_mode, eps);
  else
    seg_in_global<T, BLOCK, PAPER>(D, sg.j0, sg.j1 - sg.j0, lo, cnt, ks, n_iters, variant, rm_mode,
                            eps);
}

template <class T>
__global__ void k_avg_strategy(int64_t np, const int32_t *__restrict__ cb,
                               const T *__restrict__ Sbar, T *__restrict__ out) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np) return;
  const int32_t b = cb[h], e = cb[h + 1];
  double s = 0.0;
  for (int32_t q = b; q < e; ++q) s += (double)Sbar[q];
  for (int32_t q = b; q < e; ++q)
    out[q] = (T)(s > 0.0 ? (double)Sbar[q] / s : 1.0 / (double)(e - b));
}

template <class T>
__global__ void k_leaf_util(int64_t n, const int16_t *__restrict__ base,
                            const int32_t *__restrict__ link, const double *__restrict__ V,
                            const int8_t *__restrict__ bonus0_literal, T *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pts = (double)base[i];
  if (bonus0_literal && bonus0_literal[i] == 0) pts -= 7.0;
  out[i] = (T)(V ? V[link[i]] + pts : pts);
}

// Exact values of one level from the level below: expectation under sigma,
// or max/min at the best-responding player's nodes.
template <class T, class L>
__global__ void k_values_up(int64_t np, int mover, int mode, const int32_t *__restrict__ cb,
                            const T *__restrict__ sigma, const L *__restrict__ child,
                            double *__restrict__ out) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np) return;
  const int32_t b = cb[h], e = cb[h + 1];
  const bool use_max = (mode == PASUR_TV_MINIMAX || mode == PASUR_TV_BR_A) && mover == 0;
  const bool use_min = (mode == PASUR_TV_MINIMAX || mode == PASUR_TV_BR_B) && mover == 1;
  double v;
  if (use_max) {
    v = -INFINITY;
    for (int32_t q = b; q < e; ++q) v = fmax(v, (double)child[q]);
  } else if (use_min) {
    v = INFINITY;
    for (int32_t q = b; q < e; ++q) v = fmin(v, (double)child[q]);
  } else {
    v = 0.0;
    for (int32_t q = b; q < e; ++q) v += (double)sigma[q] * (double)child[q];
  }
  out[h] = v;
}

__global__ void k_div(int64_t n, const double *__restrict__ a, double T, double *__restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = a[j] / T;
}

int check_state(const pasur_fgt *f, const pasur_cfr_state *st) {
  if (!f || !st) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (st->dtype != PASUR_F32 && st->dtype != PASUR_F64) {
    set_error("unknown dtype %d", st->dtype);
    return PASUR_E_RANGE;
  }
  for (int l = 0; l <= 8; ++l) {
    if (!st->u[l]) { set_error("u[%d] is NULL", l); return PASUR_E_INVAL; }
    if (l >= 1 && (!st->sigma[l] || !st->R[l] || !st->Sbar[l])) {
      set_error("sigma/R/Sbar[%d] is NULL", l);
      return PASUR_E_INVAL;
    }
    if (l <= 7 && (!st->reachA[l] || !st->reachB[l])) {
      set_error("reach[%d] is NULL", l);
      return PASUR_E_INVAL;
    }
  }
  if (!st->vacc) { set_error("vacc is NULL"); return PASUR_E_INVAL; }
  return PASUR_OK;
}

template <class T>
int init_t(const pasur_fgt *f, const pasur_cfr_state *st, hipStream_t s) {
  for (int l = 1; l <= 8; ++l)
    k_init_level<T><<<grid_for(f->n[l]), kThreads, 0, s>>>(
        f->n[l], f->parent[l], f->child_begin[l - 1], (T *)st->sigma[l], (T *)st->R[l],
        (T *)st->Sbar[l]);
  k_init_roots<T><<<grid_for(f->n[0]), kThreads, 0, s>>>(f->n[0], (T *)st->reachA[0],
                                                         (T *)st->reachB[0], st->vacc);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

template <class T>
int iterate_t(const pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p,
              int64_t t0, int n_iters, hipStream_t s) {
  for (int64_t t = t0; t < t0 + n_iters; ++t) {
    const IterConsts ic = consts_for(p, t);
    for (int l = 1; l <= 7; ++l) {
      ProfScope ps(0, l, s, f->n[l], f->n[l - 1]);
      k_down<T><<<grid_for(f->n[l]), kThreads, 0, s>>>(
          f->n[l], (l - 1) & 1, f->parent[l], (const T *)st->sigma[l],
          (const T *)st->reachA[l - 1], (const T *)st->reachB[l - 1], (T *)st->reachA[l],
          (T *)st->reachB[l]);
    }
    for (int l = 8; l >= 1; --l) {
      ProfScope ps(1, l, s, f->n[l], f->n[l - 1]);
      k_up<T><<<grid_for(f->n[l - 1]), kThreads, 0, s>>>(
          f->n[l - 1], (l - 1) & 1, f->child_begin[l - 1], (T *)st->sigma[l], (T *)st->R[l],
          (T *)st->Sbar[l], (const T *)st->u[l], (T *)st->u[l - 1],
          (const T *)st->reachA[l - 1], (const T *)st->reachB[l - 1], ic,
          l == 1 ? st->vacc : nullptr);
    }
  }
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}


constexpr uint32_t kLdsPerWorkgroup = 160 * 1024;
// static LDS: the global-memory path's pointer table and index offsets, the
// per-level sibling-group statistics
constexpr uint32_t kStaticLds = 8 * 9 * sizeof(void *) + 5 * 9 * sizeof(int) + 64;

inline bool paper_variant(int variant, int rm_mode) {
  return variant == PASUR_DCFR && rm_mode == PASUR_RM_FLOOR;
}

template <class T, int BLOCK>
void *seg_kernel(bool paper) {
  return paper ? (void *)k_cfr_seg<T, BLOCK, true> : (void *)k_cfr_seg<T, BLOCK, false>;
}

}  // namespace

namespace pasur {
bool prof_on(int kernel) { return g_prof_on && ((g_prof_mask >> (kernel & 63)) & 1ull); }
void prof_push(const ProfRec &r) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.push_back(r);
}
void prof_events(hipEvent_t *a, hipEvent_t *b) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (hipEvent_t *e : {a, b}) {
    if (!g_event_pool.empty()) {
      *e = g_event_pool.back();
      g_event_pool.pop_back();
    } else {
      (void)hipEventCreate(e);
    }
  }
}
}  // namespace pasur

struct pasur_plan {
  int dtype, block, variant, rm_mode;
  double eps;
  int64_t t_first, t_last;
  int n_items, n_segs;
  void *d_items;
  Seg *d_segs;
  IterK *d_ks;
  uint32_t lds_bytes;
  int64_t work[4];  // edges, internal nodes, roots, level-7 nodes
  int64_t n_lds_segs;
};

namespace {

template <class T>
int plan_build(pasur_plan *pl, const pasur_fgt *const *fgts, const pasur_cfr_state *const *states,
               const pasur_cfr_params *p, int force_global, hipStream_t s) {
  const int n_items = pl->n_items;
  std::vector<ItemDesc<T>> items((size_t)n_items);
  std::vector<Seg> segs;
  std::vector<int64_t> seg_size;
  const uint32_t budget = force_global ? 0u : kLdsPerWorkgroup - kStaticLds;
  uint32_t max_bytes = 0;
  for (int64_t k = 0; k < 4; ++k) pl->work[k] = 0;
  pl->n_lds_segs = 0;
  for (int it = 0; it < n_items; ++it) {
    const pasur_fgt *f = fgts[it];
    const pasur_cfr_state *st = states[it];
    ItemDesc<T> &D = items[(size_t)it];
    for (int l = 0; l <= 8; ++l) {
      D.off[l] = f->root_off[l];
      D.parent[l] = f->parent[l];
      D.cb[l] = l <= 7 ? f->child_begin[l] : nullptr;
      D.sigma[l] = l >= 1 ? (T *)st->sigma[l] : nullptr;
      D.R[l] = l >= 1 ? (T *)st->R[l] : nullptr;
      D.Sbar[l] = l >= 1 ? (T *)st->Sbar[l] : nullptr;
      D.ra[l] = l <= 7 ? (T *)st->reachA[l] : nullptr;
      D.rb[l] = l <= 7 ? (T *)st->reachB[l] : nullptr;
      D.u[l] = (T *)st->u[l];
    }
    D.vacc = st->vacc;
    // Segments: runs of consecutive roots, closed when the next root would
    // exceed seg_nodes nodes, the workgroup's thread count, or LDS.
    const int64_t nr = f->n_roots;
    auto cnt_of = [&](int64_t a, int64_t b, int cnt[9]) {
      int64_t tot = 0;
      for (int l = 0; l <= 8; ++l) {
        const int32_t *o = f->h_root_off + (size_t)l * (nr + 1);
        cnt[l] = o[b] - o[a];
        tot += cnt[l];
      }
      return tot;
    };
    int64_t j0 = 0;
    while (j0 < nr) {
      int64_t j1 = j0 + 1;
      int cnt[9];
      int64_t tot = cnt_of(j0, j1, cnt);
      while (p->seg_nodes > 0 && j1 < nr && j1 - j0 < pl->block) {
        int c2[9];
        const int64_t t2 = cnt_of(j0, j1 + 1, c2);
        int mx = 0;
        for (int l = 0; l <= 8; ++l) mx = c2[l] > mx ? c2[l] : mx;
        if (t2 > p->seg_nodes || lds_layout(c2, sizeof(T)).bytes > budget || mx >= 65535) break;
        ++j1;
        tot = t2;
        for (int l = 0; l <= 8; ++l) cnt[l] = c2[l];
      }
      int mx = 0;
      for (int l = 0; l <= 8; ++l) mx = cnt[l] > mx ? cnt[l] : mx;
      const uint32_t bytes = lds_layout(cnt, sizeof(T)).bytes;
      if (bytes <= budget && mx < 65535) {
        max_bytes = bytes > max_bytes ? bytes : max_bytes;
        pl->n_lds_segs += 1;
      }
      for (int l = 1; l <= 8; ++l) pl->work[0] += cnt[l];
      for (int l = 0; l <= 7; ++l) pl->work[1] += cnt[l];
      pl->work[2] += j1 - j0;
      pl->work[3] += cnt[7];
      Seg sg;
      sg.item = it;
      sg.j0 = (int32_t)j0;
      sg.j1 = (int32_t)j1;
      sg.pad = 0;
      segs.push_back(sg);
      seg_size.push_back(tot);
      j0 = j1;
    }
  }
  // longest segments first
  std::vector<size_t> idx(segs.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](size_t a, size_t b) { return seg_size[a] > seg_size[b]; });
  std::vector<Seg> sorted(segs.size());
  for (size_t i = 0; i < idx.size(); ++i) sorted[i] = segs[idx[i]];
  pl->n_segs = (int)sorted.size();
  pl->lds_bytes = force_global ? 0u : max_bytes;
  // iteration constants for t_first .. t_last, computed on the host
  const int64_t nt = pl->t_last - pl->t_first + 1;
  std::vector<IterK> ks((size_t)nt);
  for (int64_t i = 0; i < nt; ++i) {
    const IterConsts ic = consts_for(p, pl->t_first + i);
    ks[(size_t)i].dpos = ic.dpos;
    ks[(size_t)i].dneg = ic.dneg;
    ks[(size_t)i].avg_w = ic.avg_w;
    ks[(size_t)i].avg_t = ic.avg_t;
  }
  PASUR_TRY_HIP(hipMalloc(&pl->d_items, sizeof(ItemDesc<T>) * items.size()));
  PASUR_TRY_HIP(hipMalloc((void **)&pl->d_segs, sizeof(Seg) * (sorted.size() + 1)));
  PASUR_TRY_HIP(hipMalloc((void **)&pl->d_ks, sizeof(IterK) * ks.size()));
  PASUR_TRY_HIP(hipMemcpyAsync(pl->d_items, items.data(), sizeof(ItemDesc<T>) * items.size(),
                               hipMemcpyHostToDevice, s));
  PASUR_TRY_HIP(hipMemcpyAsync(pl->d_segs, sorted.data(), sizeof(Seg) * sorted.size(),
                               hipMemcpyHostToDevice, s));
  PASUR_TRY_HIP(hipMemcpyAsync(pl->d_ks, ks.data(), sizeof(IterK) * ks.size(),
                               hipMemcpyHostToDevice, s));
  PASUR_TRY_HIP(hipStreamSynchronize(s));  // host staging vectors go out of scope
  const bool paper = paper_variant(p->variant, p->rm_mode);
  void *kern = pl->block == 256   ? seg_kernel<T, 256>(paper)
               : pl->block == 512 ? seg_kernel<T, 512>(paper)
                                  : seg_kernel<T, 1024>(paper);
  // The attribute is a ceiling shared by every plan of this instance, so it
  // is raised to the whole budget (plans may be launched in any order); each
  // launch still asks for its own lds_bytes.
  PASUR_TRY_HIP(hipFuncSetAttribute((const void *)kern,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kLdsPerWorkgroup - kStaticLds)));
  return PASUR_OK;
}

template <class T, int BLOCK>
void plan_launch(const pasur_plan *pl, int64_t t0, int n_iters, hipStream_t s) {
  auto kern = paper_variant(pl->variant, pl->rm_mode) ? k_cfr_seg<T, BLOCK, true>
                                                      : k_cfr_seg<T, BLOCK, false>;
  kern<<<(unsigned)pl->n_segs, BLOCK, pl->lds_bytes, s>>>(
      (const ItemDesc<T> *)pl->d_items, pl->d_segs, pl->d_ks + (t0 - pl->t_first), n_iters,
      pl->variant, pl->rm_mode, pl->eps, pl->lds_bytes);
}

}  // namespace

extern "C" void pasur_plan_free(pasur_plan *pl) {
  if (!pl) return;
  if (pl->d_items) (void)hipFree(pl->d_items);
  if (pl->d_segs) (void)hipFree(pl->d_segs);
  if (pl->d_ks) (void)hipFree(pl->d_ks);
  delete pl;
}

extern "C" int pasur_plan_create(const pasur_fgt *const *fgts,
                                 const pasur_cfr_state *const *states, int n_items,
                                 const pasur_cfr_params *p, int64_t t_first, int64_t t_last,
                                 pasur_plan **out, void *stream) {
  if (!out || !fgts || !states || !p || n_items < 1) {
    set_error("null argument or empty batch");
    return PASUR_E_INVAL;
  }
  *out = nullptr;
  if (t_first < 1 || t_last < t_first) {
    set_error("need 1 <= t_first <= t_last");
    return PASUR_E_RANGE;
  }
  if (p->variant < 0 || p->variant > 2 || p->rm_mode < 0 || p->rm_mode > 1 ||
      p->schedule < 0 || p->schedule > PASUR_SCHED_AUTO || p->seg_nodes < 0 ||
      (p->block != 0 && p->block != 256 && p->block != 512 && p->block != 1024)) {
    set_error("unknown variant, regret-matching mode, schedule, block or segment size");
    return PASUR_E_RANGE;
  }
  if (p->schedule == PASUR_SCHED_LEVEL_SYNC || p->schedule == PASUR_SCHED_STREAM) {
    set_error("plans use the persistent segment schedule");
    return PASUR_E_RANGE;
  }
  if (p->flags) {
    set_error("the snippet flags run on PASUR_SCHED_LEVEL_SYNC only, not in plans");
    return PASUR_E_RANGE;
  }
  const int dtype = states[0]->dtype;
  for (int i = 0; i < n_items; ++i) {
    if (!fgts[i] || !states[i]) {
      set_error("item %d is NULL", i);
      return PASUR_E_INVAL;
    }
    PASUR_TRY(check_state(fgts[i], states[i]));
    if (states[i]->dtype != dtype) {
      set_error("all items of a plan need the same dtype");
      return PASUR_E_INVAL;
    }
  }
  pasur_plan *pl = new pasur_plan();
  std::memset(pl, 0, sizeof(*pl));
  pl->dtype = dtype;
  pl->block = p->block ? p->block : 1024;
  pl->variant = p->variant;
  pl->rm_mode = p->rm_mode;
  pl->eps = p->eps;
  pl->t_first = t_first;
  pl->t_last = t_last;
  pl->n_items = n_items;
  hipStream_t s = (hipStream_t)stream;
  const int fg = p->schedule == PASUR_SCHED_ROOT_GLOBAL;
  int st = dtype == PASUR_F32 ? plan_build<float>(pl, fgts, states, p, fg, s)
                              : plan_build<double>(pl, fgts, states, p, fg, s);
  if (st) {
    pasur_plan_free(pl);
    return st;
  }
  *out = pl;
  return PASUR_OK;
}

extern "C" int pasur_plan_iterate(const pasur_plan *pl, int64_t t0, int n_iters, void *stream) {
  if (!pl) {
    set_error("plan is NULL");
    return PASUR_E_INVAL;
  }
  if (n_iters < 0 || t0 < pl->t_first || t0 + n_iters - 1 > pl->t_last) {
    set_error("iterations %lld..%lld outside the plan's %lld..%lld", (long long)t0,
              (long long)(t0 + n_iters - 1), (long long)pl->t_first, (long long)pl->t_last);
    return PASUR_E_RANGE;
  }
  if (n_iters == 0) return PASUR_OK;
  hipStream_t s = (hipStream_t)stream;
  {
    ProfScope ps(pl->n_lds_segs == pl->n_segs ? 2 : 3, -1, s, pl->work[0], pl->work[1],
                 pl->work[2], pl->work[3], n_iters);
    const bool f32 = pl->dtype == PASUR_F32;
    switch (pl->block) {
      case 256: f32 ? plan_launch<float, 256>(pl, t0, n_iters, s) : plan_launch<double, 256>(pl, t0, n_iters, s); break;
      case 512: f32 ? plan_launch<float, 512>(pl, t0, n_iters, s) : plan_launch<double, 512>(pl, t0, n_iters, s); break;
      default: f32 ? plan_launch<float, 1024>(pl, t0, n_iters, s) : plan_launch<double, 1024>(pl, t0, n_iters, s); break;
    }
  }
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_plan_info(const pasur_plan *pl, int64_t info[8]) {
  if (!pl || !info) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  info[0] = pl->n_segs;
  info[1] = pl->n_lds_segs;
  info[2] = pl->lds_bytes;
  info[3] = pl->block;
  info[4] = pl->work[0];
  info[5] = pl->work[1];
  info[6] = pl->work[2];
  info[7] = pl->work[3];
  return PASUR_OK;
}

namespace {

int64_t widest_level(const pasur_fgt *f) {
  int64_t mx = 1;
  for (int l = 0; l <= 7; ++l) mx = f->n[l] > mx ? f->n[l] : mx;
  return mx;
}

// The up-sweep of tree values through two level buffers of at least
// widest_level(f) doubles each (every level is written in full before it
// is read, so the buffers need no clearing).
template <class T, class L>
void values_run(const pasur_fgt *f, const L *leaf, void *const sigma[9], int mode, double *out,
                double *buf0, double *buf1, hipStream_t s) {
  double *buf[2] = {buf0, buf1};
  int cur = 0;
  for (int l = 8; l >= 1; --l) {
    double *dst = l == 1 ? out : buf[cur];
    const T *sg = sigma ? (const T *)sigma[l] : nullptr;
    if (l == 8)
      k_values_up<T, L><<<grid_for(f->n[7]), kThreads, 0, s>>>(f->n[7], 1, mode,
                                                               f->child_begin[7], sg, leaf, dst);
    else
      k_values_up<T, double><<<grid_for(f->n[l - 1]), kThreads, 0, s>>>(
          f->n[l - 1], (l - 1) & 1, mode, f->child_begin[l - 1], sg, buf[cur ^ 1], dst);
    cur ^= 1;
  }
}

template <class T, class L>
int values_t(const pasur_fgt *f, const L *leaf, void *const sigma[9], int mode, double *out,
             hipStream_t s) {
  const int64_t mx = widest_level(f);
  double *buf[2] = {nullptr, nullptr};
  PASUR_TRY_HIP(hipMallocAsync((void **)&buf[0], mx * sizeof(double), s));
  hipError_t e = hipMallocAsync((void **)&buf[1], mx * sizeof(double), s);
  if (e != hipSuccess) {
    (void)hipFreeAsync(buf[0], s);
    set_error("hipMallocAsync: %s", hipGetErrorString(e));
    return PASUR_E_NOMEM;
  }
  values_run<T, L>(f, leaf, sigma, mode, out, buf[0], buf[1], s);
  e = hipGetLastError();
  (void)hipFreeAsync(buf[0], s);
  (void)hipFreeAsync(buf[1], s);
  if (e != hipSuccess) {
    set_error("tree values: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  return PASUR_OK;
}

int check_tree_values(const pasur_fgt *f, const double *d_leaf, int dtype, void *const sigma[9],
                      int mode, double *d_out) {
  if (!f || !d_leaf || !d_out) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (mode < 0 || mode > 3 || (dtype != PASUR_F32 && dtype != PASUR_F64)) {
    set_error("unknown mode or dtype");
    return PASUR_E_RANGE;
  }
  if (mode != PASUR_TV_MINIMAX) {
    if (!sigma) {
      set_error("sigma is NULL");
      return PASUR_E_INVAL;
    }
    for (int l = 1; l <= 8; ++l)
      if (!sigma[l]) {
        set_error("sigma[%d] is NULL", l);
        return PASUR_E_INVAL;
      }
  }
  return PASUR_OK;
}

// ---- pasur_tree_values_noalloc: the level buffers in a fixed device array.
// Each GPU the library runs on holds its own copy of `scratch` (two level
// buffers of kNoAllocLevel doubles, 32 MiB) until the process ends.  Host
// code never uses the array's name as an address: its per-device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, on the entry point's first call there.
constexpr int64_t kNoAllocLevel = (int64_t)1 << 21;
static __device__ __align__(256) double scratch[2 * kNoAllocLevel];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {nullptr};

int scratch_for_current_device(double **out) {
  int dev = 0;
  PASUR_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the scratch table covers", dev, kMaxDevices);
    return PASUR_E_RANGE;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return PASUR_E_HIP;
    }
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return PASUR_OK;
}

}  // namespace

extern "C" int pasur_cfr_init(const pasur_fgt *f, const pasur_cfr_state *st, void *stream) {
  PASUR_TRY(check_state(f, st));
  hipStream_t s = (hipStream_t)stream;
  return st->dtype == PASUR_F32 ? init_t<float>(f, st, s) : init_t<double>(f, st, s);
}

extern "C" int pasur_cfr_iterate(const pasur_fgt *f, const pasur_cfr_state *st,
                                 const pasur_cfr_params *p, int64_t t0, int n_iters,
                                 void *stream) {
  PASUR_TRY(check_state(f, st));
  if (!p) {
    set_error("params is NULL");
    return PASUR_E_INVAL;
  }
  if (t0 < 1 || n_iters < 0) {
    set_error("need t0 >= 1 and n_iters >= 0");
    return PASUR_E_RANGE;
  }
  if (p->variant < 0 || p->variant > 2 || p->rm_mode < 0 || p->rm_mode > 1) {
    set_error("unknown variant or regret-matching mode");
    return PASUR_E_RANGE;
  }
  if (p->schedule < 0 || p->schedule > PASUR_SCHED_AUTO ||
      (p->block != 0 && p->block != 256 && p->block != 512 && p->block != 1024)) {
    set_error("unknown schedule or block size");
    return PASUR_E_RANGE;
  }
  if (p->flags & ~(PASUR_CFR_SNIPPET_TOL | PASUR_CFR_SNIPPET_AVG)) {
    set_error("unknown CFR flags %d", p->flags);
    return PASUR_E_RANGE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (p->flags) {
    if (p->variant != PASUR_DCFR) {
      set_error("the snippet flags apply to DCFR only");
      return PASUR_E_RANGE;
    }
    if (p->schedule != PASUR_SCHED_LEVEL_SYNC && p->schedule != PASUR_SCHED_AUTO) {
      set_error("the snippet flags run on PASUR_SCHED_LEVEL_SYNC (or AUTO) only");
      return PASUR_E_RANGE;
    }
    return st->dtype == PASUR_F32 ? iterate_t<float>(f, st, p, t0, n_iters, s)
                                  : iterate_t<double>(f, st, p, t0, n_iters, s);
  }
  if (p->schedule == PASUR_SCHED_STREAM ||
      (p->schedule == PASUR_SCHED_AUTO && sweep_pays(f)))
    return sweep_iterate(const_cast<pasur_fgt *>(f), st, p, t0, n_iters, s);
  if (p->schedule == PASUR_SCHED_LEVEL_SYNC)
    return st->dtype == PASUR_F32 ? iterate_t<float>(f, st, p, t0, n_iters, s)
                                  : iterate_t<double>(f, st, p, t0, n_iters, s);
  if (n_iters == 0) return PASUR_OK;
  pasur_plan *pl = nullptr;
  PASUR_TRY(pasur_plan_create(&f, &st, 1, p, t0, t0 + n_iters - 1, &pl, stream));
  int rc = pasur_plan_iterate(pl, t0, n_iters, stream);
  hipError_t e = hipStreamSynchronize(s);  // the plan's buffers are freed below
  pasur_plan_free(pl);
  if (rc) return rc;
  if (e != hipSuccess) {
    set_error("iterate: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  return PASUR_OK;
}

extern "C" int pasur_average_strategy(const pasur_fgt *f, const pasur_cfr_state *st,
                                      void *const sigma_bar[9], void *stream) {
  PASUR_TRY(check_state(f, st));
  if (!sigma_bar) {
    set_error("sigma_bar is NULL");
    return PASUR_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  for (int l = 1; l <= 8; ++l) {
    if (!sigma_bar[l]) {
      set_error("sigma_bar[%d] is NULL", l);
      return PASUR_E_INVAL;
    }
    if (st->dtype == PASUR_F32)
      k_avg_strategy<float><<<grid_for(f->n[l - 1]), kThreads, 0, s>>>(
          f->n[l - 1], f->child_begin[l - 1], (const float *)st->Sbar[l], (float *)sigma_bar[l]);
    else
      k_avg_strategy<double><<<grid_for(f->n[l - 1]), kThreads, 0, s>>>(
          f->n[l - 1], f->child_begin[l - 1], (const double *)st->Sbar[l],
          (double *)sigma_bar[l]);
  }
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_leaf_utilities(const pasur_fgt *f, const double *d_V_next, int dtype,
                                    int flags, void *d_leaf, void *stream) {
  if (!f || !d_leaf) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (dtype != PASUR_F32 && dtype != PASUR_F64) {
    set_error("unknown dtype %d", dtype);
    return PASUR_E_RANGE;
  }
  if (flags & ~PASUR_LEAF_LITERAL_BONUS0) {
    set_error("unknown leaf-utility flags %d", flags);
    return PASUR_E_RANGE;
  }
  if (f->round < 5 && !d_V_next) {
    set_error("rounds 0..4 need the next round's root values");
    return PASUR_E_INVAL;
  }
  const double *V = f->round < 5 ? d_V_next : nullptr;
  const int8_t *b0 = f->round == 5 && (flags & PASUR_LEAF_LITERAL_BONUS0) ? f->leaf_bonus : nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (dtype == PASUR_F32)
    k_leaf_util<float><<<grid_for(f->n[8]), kThreads, 0, s>>>(f->n[8], f->leaf_base, f->link, V,
                                                              b0, (float *)d_leaf);
  else
    k_leaf_util<double><<<grid_for(f->n[8]), kThreads, 0, s>>>(f->n[8], f->leaf_base, f->link, V,
                                                               b0, (double *)d_leaf);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_round_values(const pasur_fgt *f, const pasur_cfr_state *st, int value_mode,
                                  int64_t T, void *const sigma_bar[9], double *d_V, void *stream) {
  PASUR_TRY(check_state(f, st));
  if (!d_V) {
    set_error("d_V is NULL");
    return PASUR_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (value_mode == PASUR_V_ITERATE_MEAN) {
    if (T < 1) {
      set_error("T must be >= 1");
      return PASUR_E_RANGE;
    }
    k_div<<<grid_for(f->n[0]), kThreads, 0, s>>>(f->n[0], st->vacc, (double)T, d_V);
    PASUR_TRY_HIP(hipGetLastError());
    return PASUR_OK;
  }
  if (value_mode != PASUR_V_SIGMA_BAR) {
    set_error("unknown value mode %d", value_mode);
    return PASUR_E_RANGE;
  }
  if (!sigma_bar) {
    set_error("sigma_bar is NULL");
    return PASUR_E_INVAL;
  }
  return st->dtype == PASUR_F32
             ? values_t<float, float>(f, (const float *)st->u[8], sigma_bar, PASUR_TV_EXPECT, d_V, s)
             : values_t<double, double>(f, (const double *)st->u[8], sigma_bar, PASUR_TV_EXPECT,
                                        d_V, s);
}

extern "C" int pasur_tree_values(const pasur_fgt *f, const double *d_leaf, int dtype,
                                 void *const sigma[9], int mode, double *d_out, void *stream) {
  PASUR_TRY(check_tree_values(f, d_leaf, dtype, sigma, mode, d_out));
  hipStream_t s = (hipStream_t)stream;
  return dtype == PASUR_F32 ? values_t<float, double>(f, d_leaf, sigma, mode, d_out, s)
                            : values_t<double, double>(f, d_leaf, sigma, mode, d_out, s);
}

namespace {

int check_exploitability(const pasur_fgt *const *fgts, int n_rounds, void *const *sigma_bar,
                         int dtype, int leaf_flags, const double *d_br_a, const double *d_br_b,
                         const double *d_v) {
  if (!fgts || !sigma_bar) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (!d_br_a && !d_br_b && !d_v) {
    set_error("no output requested");
    return PASUR_E_INVAL;
  }
  if (n_rounds < 1 || n_rounds > 6) {
    set_error("n_rounds %d outside 1..6", n_rounds);
    return PASUR_E_RANGE;
  }
  if (dtype != PASUR_F32 && dtype != PASUR_F64) {
    set_error("unknown dtype %d", dtype);
    return PASUR_E_RANGE;
  }
  if (leaf_flags & ~PASUR_LEAF_LITERAL_BONUS0) {
    set_error("unknown leaf-utility flags %d", leaf_flags);
    return PASUR_E_RANGE;
  }
  for (int r = 0; r < n_rounds; ++r) {
    const pasur_fgt *f = fgts[r];
    if (!f) {
      set_error("fgts[%d] is NULL", r);
      return PASUR_E_INVAL;
    }
    if (f->n[0] < 1) {
      set_error("fgts[%d] has no roots", r);
      return PASUR_E_INVAL;
    }
    if (r > 0 && (f->round != fgts[r - 1]->round + 1 || f->n[0] != fgts[r - 1]->n_next)) {
      set_error("fgts[%d] is not the unfolding of fgts[%d]'s next-round roots", r, r - 1);
      return PASUR_E_INVAL;
    }
    for (int l = 1; l <= 8; ++l)
      if (!sigma_bar[r * 9 + l]) {
        set_error("sigma_bar[%d*9+%d] is NULL", r, l);
        return PASUR_E_INVAL;
      }
  }
  if (fgts[n_rounds - 1]->round != 5) {
    set_error("the last tree must be round 5 (the hand's last round)");
    return PASUR_E_INVAL;
  }
  return PASUR_OK;
}

// One mode over all rounds, last first: each round's leaves are its round
// points plus the next round's value of the same mode at the linked root.
int composed_values(const pasur_fgt *const *fgts, int n_rounds, void *const *sigma_bar,
                    int dtype, int leaf_flags, int mode, double *out, hipStream_t s) {
  double *V = nullptr;  // the later round's root values
  for (int r = n_rounds - 1; r >= 0; --r) {
    const pasur_fgt *f = fgts[r];
    double *leaf = nullptr, *res = out;
    hipError_t e = hipMallocAsync((void **)&leaf, f->n[8] * sizeof(double), s);
    if (e == hipSuccess && r > 0) e = hipMallocAsync((void **)&res, f->n[0] * sizeof(double), s);
    int st = PASUR_OK;
    if (e != hipSuccess) {
      set_error("hipMallocAsync: %s", hipGetErrorString(e));
      st = PASUR_E_NOMEM;
    } else {
      const int8_t *b0 =
          f->round == 5 && (leaf_flags & PASUR_LEAF_LITERAL_BONUS0) ? f->leaf_bonus : nullptr;
      k_leaf_util<double><<<grid_for(f->n[8]), kThreads, 0, s>>>(f->n[8], f->leaf_base, f->link,
                                                                 V, b0, leaf);
      st = dtype == PASUR_F32
               ? values_t<float, double>(f, leaf, sigma_bar + r * 9, mode, res, s)
               : values_t<double, double>(f, leaf, sigma_bar + r * 9, mode, res, s);
    }
    if (leaf) (void)hipFreeAsync(leaf, s);
    if (V) (void)hipFreeAsync(V, s);
    V = r > 0 ? res : nullptr;
    if (st != PASUR_OK) {
      if (V && V != out) (void)hipFreeAsync(V, s);
      return st;
    }
  }
  return PASUR_OK;
}

}  // namespace

extern "C" int pasur_exploitability(const pasur_fgt *const *fgts, int n_rounds,
                                    void *const *sigma_bar, int dtype, int leaf_flags,
                                    double *d_br_a, double *d_br_b, double *d_v, void *stream) {
  PASUR_TRY(check_exploitability(fgts, n_rounds, sigma_bar, dtype, leaf_flags, d_br_a, d_br_b,
                                 d_v));
  hipStream_t s = (hipStream_t)stream;
  double *outs[3] = {d_br_a, d_br_b, d_v};
  const int modes[3] = {PASUR_TV_BR_A, PASUR_TV_BR_B, PASUR_TV_EXPECT};
  for (int m = 0; m < 3; ++m)
    if (outs[m])
      PASUR_TRY(composed_values(fgts, n_rounds, sigma_bar, dtype, leaf_flags, modes[m], outs[m], s));
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_tree_values_noalloc(const pasur_fgt *f, const double *d_leaf, int dtype,
                                         void *const sigma[9], int mode, double *d_out,
                                         void *stream) {
  PASUR_TRY(check_tree_values(f, d_leaf, dtype, sigma, mode, d_out));
  const int64_t mx = widest_level(f);
  if (mx > kNoAllocLevel) {
    set_error("a tree level of %lld nodes exceeds the %lld-node scratch of "
              "pasur_tree_values_noalloc (use pasur_tree_values)",
              (long long)mx, (long long)kNoAllocLevel);
    return PASUR_E_CAPACITY;
  }
  double *p = nullptr;
  PASUR_TRY(scratch_for_current_device(&p));
  hipStream_t s = (hipStream_t)stream;
  if (dtype == PASUR_F32)
    values_run<float, double>(f, d_leaf, sigma, mode, d_out, p, p + kNoAllocLevel, s);
  else
    values_run<double, double>(f, d_leaf, sigma, mode, d_out, p, p + kNoAllocLevel, s);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_clear();
  g_prof_on = on != 0;
  g_prof_mask = ~0ull;
  return PASUR_OK;
}

extern "C" int pasur_profile_select(uint64_t kernel_mask) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_mask = kernel_mask;
  return PASUR_OK;
}

extern "C" int pasur_profile_read(int64_t cap, int32_t *kernel, int32_t *level, float *ms,
                                  int64_t *work, int64_t *n_out) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!n_out) {
    set_error("n_out is NULL");
    return PASUR_E_INVAL;
  }
  *n_out = (int64_t)g_prof.size();
  const int64_t n = cap < *n_out ? cap : *n_out;
  for (int64_t i = 0; i < n; ++i) {
    PASUR_TRY_HIP(hipEventSynchronize(g_prof[i].b));
    float t = 0.f;
    PASUR_TRY_HIP(hipEventElapsedTime(&t, g_prof[i].a, g_prof[i].b));
    if (kernel) kernel[i] = g_prof[i].kernel;
    if (level) level[i] = g_prof[i].level;
    if (ms) ms[i] = t;
    if (work)
      for (int k = 0; k < 5; ++k) work[5 * i + k] = g_prof[i].work[k];
  }
  return PASUR_OK;
}
