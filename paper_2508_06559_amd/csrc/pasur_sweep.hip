// pasur_sweep.hip -- the HBM-streaming schedule of full-width DCFR
// (section "CFR Algorithm": CodeSnippets FindReachProbability and
// FindUtility, equations DFCR_REG, RM and DFCR_AVG) for rounds whose trees
// are far larger than what the persistent segment kernel keeps busy.
//
// One launch per level and sweep direction streams the level's state
// through HBM with coalesced accesses.  Two changes of representation keep
// the bytes per iteration low; neither changes a result:
//
//  * No per-edge strategy array inside a call.  sigma^t of an edge is
//    recomputed from its regret and the parent's regret-matching sum Z(h)
//    (one double per parent, written by the up sweep): sigma = x / Z with
//    x = max(R, eps) (or R+), exactly the division the other schedules store,
//    so the value is bit-identical.  Z(h) <= 0 encodes "no positive sum":
//    Z = -k and sigma = 1/k.  The first iteration of a call reads the sigma
//    array (uniform, warm-started or left by an earlier call); the last
//    writes sigma^{T+1} back.
//
//  * Chains are not iterated.  A node whose whole subtree is a chain of
//    single-child nodes ("passive"; in Pasur most nodes of levels 6 and 7,
//    where each player holds one card) has a constant utility -- its leaf's
//    -- and its descendants' edges are forced: sigma = 1 and zero regret
//    whatever the iteration.  Their utility is copied up once per call, and
//    the sweeps visit only the other ("active") parents of those levels
//    through index lists.  The last iteration's down sweep covers every node,
//    so the reach arrays end exactly as in the other schedules.  The one
//    array that differs: the average-strategy sums of edges below a passive
//    parent are not accumulated (they stay at their initial value); the
//    average strategy of such an edge is 1 either way.
//
// Per parent, the children's updates follow the oracle's order (the two
// per-parent sums are sequential in child order), with FP64 arithmetic and
// no contraction, so results are bit-identical to the persistent and the
// level-synchronous schedules on every array but those sums.
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
  int32_t *act[9];      // their indices where n_act[l] < n[l] (else null)
  int kmax[9];          // largest fan-out among the parents of level L (L = 1..8)
  int32_t *chunk[9];    // chunk starts over level L's children (chunked levels)
  int64_t n_chunk[9];
};

void sweep_index_free(SweepIndex *x) {
  if (!x) return;
  for (int l = 0; l < 9; ++l) {
    dev_free(x->passive[l]);
    dev_free(x->act[l]);
    dev_free(x->chunk[l]);
  }
  delete x;
}

namespace {

constexpr int kBlk = 256;
// Largest sibling group a chunked level handles: chunks of at most 64
// children that never split a group start at least every 32 children.
constexpr int kMaxChunkGroup = 33;

inline unsigned grid_of(int64_t n, int64_t cap = 256 * 32) {
  int64_t g = (n + kBlk - 1) / kBlk;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

// ---- index construction ----------------------------------------------------

// passive(h) = one child, and that child is a leaf (level 7) or passive.
__global__ void k_sw_passive(int64_t n, int last, const int32_t *__restrict__ cb,
                             const uint8_t *__restrict__ passive_next,
                             uint8_t *__restrict__ passive, int32_t *__restrict__ active) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
       h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = cb[h];
    const bool p = cb[h + 1] - b == 1 && (last || passive_next[b]);
    passive[h] = p ? 1 : 0;
    active[h] = p ? 0 : 1;
  }
}

__global__ void k_sw_compact(int64_t n, const int32_t *__restrict__ active,
                             const int32_t *__restrict__ pos, int32_t *__restrict__ list) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
       h += (int64_t)gridDim.x * blockDim.x)
    if (active[h]) list[pos[h]] = (int32_t)h;
}

__global__ void k_sw_kmax(int64_t n, const int32_t *__restrict__ cb, int *__restrict__ out) {
  int m = 0;
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
       h += (int64_t)gridDim.x * blockDim.x)
    m = max(m, cb[h + 1] - cb[h]);
  if (m > 0) atomicMax(out, m);
}

// Chunk c of a level's children starts at the first sibling of child
// c * stride (stride = 64 - (kmax - 1)), so no chunk exceeds 64 children or
// splits a sibling group; the last entry is n.
__global__ void k_sw_chunks(int64_t n_chunk, int64_t n, int stride,
                            const int32_t *__restrict__ par, const int32_t *__restrict__ cb,
                            int32_t *__restrict__ cs) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_chunk;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c * (int64_t)stride;
    cs[c] = c < n_chunk && x < n ? cb[par[x]] : (int32_t)n;
  }
}

int build_index(pasur_fgt *f, hipStream_t s) {
  SweepIndex *x = new SweepIndex();
  for (int l = 0; l < 9; ++l) {
    x->n[l] = f->n[l];
    x->passive[l] = nullptr;
    x->act[l] = nullptr;
    x->chunk[l] = nullptr;
    x->n_act[l] = f->n[l];
    x->n_chunk[l] = 0;
    x->kmax[l] = 0;
  }
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
  // largest fan-out per level and the chunk starts of the dense levels
  int *d_km = nullptr;
  st = dev_alloc(&d_km, 9);
  if (st) return fail(st);
  (void)hipMemsetAsync(d_km, 0, 9 * sizeof(int), s);
  for (int L = 1; L <= 8; ++L)
    k_sw_kmax<<<grid_of(f->n[L - 1]), kBlk, 0, s>>>(f->n[L - 1], f->child_begin[L - 1], d_km + L);
  hipError_t e = hipMemcpyAsync(x->kmax, d_km, 9 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(d_km);
  if (e != hipSuccess) {
    set_error("sweep index: %s", hipGetErrorString(e));
    return fail(PASUR_E_HIP);
  }
  for (int L = 1; L <= 8; ++L) {
    const int km = x->kmax[L];
    if (x->n_act[L - 1] < f->n[L - 1] || km < 1 || km > kMaxChunkGroup || f->n[L] == 0) continue;
    const int stride = 64 - (km - 1);
    const int64_t nc = (f->n[L] + stride - 1) / stride;
    st = dev_alloc(&x->chunk[L], nc + 1);
    if (st) return fail(st);
    x->n_chunk[L] = nc;
    k_sw_chunks<<<grid_of(nc + 1), kBlk, 0, s>>>(nc, f->n[L], stride, f->parent[L],
                                                 f->child_begin[L - 1], x->chunk[L]);
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("sweep index: %s", hipGetErrorString(e));
    return fail(PASUR_E_HIP);
  }
  f->sweep = x;
  return PASUR_OK;
}

// ---- per-call set-up and tear-down -----------------------------------------

__device__ __forceinline__ double rm_x(double R, int rm_mode, double eps) {
  return rm_mode == PASUR_RM_FLOOR ? fmax(R, eps) : fmax(R, 0.0);
}

// sigma of an edge from its (stored) regret and its parent's sum, rounded to
// the state type as the other schedules store it.
template <class T>
__device__ __forceinline__ double sig_of(T Rq, double Zh, int rm_mode, double eps) {
  const double x = rm_x((double)Rq, rm_mode, eps);
  const double s = Zh > 0.0 ? x / Zh : 1.0 / -Zh;
  return (double)(T)s;
}

// u of a passive node = its only child's utility (sigma = 1), once per call.
template <class T>
__global__ void k_sw_chain_u(int64_t n, const uint8_t *__restrict__ passive,
                             const int32_t *__restrict__ cb, T *__restrict__ u,
                             const T *__restrict__ u_next) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
       h += (int64_t)gridDim.x * blockDim.x)
    if (passive[h]) u[h] = (T)(0.0 + (double)u_next[cb[h]]);
}

// Regret-matching sum of a passive node's single edge (its regret stays 0,
// so this is the sum every later iteration would compute).
template <class T>
__global__ void k_sw_zinit(int64_t n, const uint8_t *__restrict__ passive,
                           const int32_t *__restrict__ cb, const T *__restrict__ R_next,
                           double *__restrict__ Z, int rm_mode, double eps) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
       h += (int64_t)gridDim.x * blockDim.x)
    if (passive[h]) {
      const double sum = 0.0 + rm_x((double)R_next[cb[h]], rm_mode, eps);
      Z[h] = sum > 0.0 ? sum : -1.0;
    }
}

// sigma^{T+1} of every edge of a level, written back at the end of a call.
template <class T>
__global__ void k_sw_sigma_out(int64_t n, const int32_t *__restrict__ par,
                               const T *__restrict__ R, const double *__restrict__ Zp,
                               T *__restrict__ sg, int rm_mode, double eps) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    sg[q] = (T)sig_of<T>(R[q], Zp[par[q]], rm_mode, eps);
}

// ---- the sweeps --------------------------------------------------------------

// FindReachProbability for level L: the mover's reach picks up sigma of the
// edge taken, the other reach is inherited.  `list` (optional) selects the
// nodes; sg_first (first iteration of a call) supplies sigma directly.
template <class T>
__global__ void __launch_bounds__(kBlk)
    k_sw_down(int64_t n, const int32_t *__restrict__ list, int mover,
              const int32_t *__restrict__ par, const T *__restrict__ R,
              const T *__restrict__ sg_first, const double *__restrict__ Zp,
              const T *__restrict__ ra_up, const T *__restrict__ rb_up, T *__restrict__ ra,
              T *__restrict__ rb, int rm_mode, double eps) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = list ? list[i] : i;
    const int32_t h = par[q];
    const double s = sg_first ? (double)sg_first[q] : sig_of<T>(R[q], Zp[h], rm_mode, eps);
    double a = (double)ra_up[h];
    double b = (double)rb_up[h];
    if (mover == 0) a *= s;
    else b *= s;
    ra[q] = (T)a;
    rb[q] = (T)b;
  }
}

// Arguments of one level's up sweep (children on level L, parents on L-1).
template <class T>
struct UpArgs {
  const int32_t *par;  // level L
  const int32_t *cb;   // level L-1
  T *R, *Sb;           // level L
  const T *sg_first;   // level L (first iteration of a call), else null
  const T *u;          // level L
  T *u_par;            // level L-1
  double *Z;           // level L-1
  const T *ra, *rb;    // level L-1
  double *vacc;        // roots (L == 1) or null
  int mover;
};

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

// FindUtility, one lane per child: wave w takes chunks w, w + nw, ... (at
// most 64 children each, sibling groups never split); the two per-parent
// sums (sigma*u, then the regret-matching sum) are in-order scans across
// the group's lanes (group_sum), every other step is per child in the
// order of the per-parent loop.
template <class T, bool PAPER>
__global__ void __launch_bounds__(kBlk)
    k_sw_up_chunk(int64_t n_chunk, const int32_t *__restrict__ cs, UpArgs<T> a, IterK ik,
                  int variant, int rm_mode, double eps) {
  if (PAPER) {
    variant = PASUR_DCFR;
    rm_mode = PASUR_RM_FLOOR;
  }
  const int lane = (int)(threadIdx.x & 63);
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const double sgn = a.mover == 0 ? 1.0 : -1.0;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < n_chunk; w += nw) {
    const int c0 = cs[w], c1 = cs[w + 1];
    if (c1 <= c0) continue;  // wave-uniform
    const bool valid = c0 + lane < c1;
    const int q = valid ? c0 + lane : c1 - 1;
    const int h = a.par[q];
    const int b = a.cb[h], e = a.cb[h + 1];
    const T rq = a.R[q], bq = a.Sb[q], uq = a.u[q];
    const double sq = a.sg_first ? (double)a.sg_first[q] : sig_of<T>(rq, a.Z[h], rm_mode, eps);
    const double opp = a.mover == 0 ? (double)a.rb[h] : (double)a.ra[h];
    const double own = a.mover == 0 ? (double)a.ra[h] : (double)a.rb[h];
    const int pos = q - b, k = e - b;
    const int kw = wave_max(k);
    const double uh = group_sum(sq * (double)uq, pos, k, kw);
    const double r = sgn * opp * ((double)uq - uh);
    const T Rs = (T)regret_update<PAPER>((double)rq, r, ik, variant);
    const double x = rm_x((double)Rs, rm_mode, eps);
    const double sum = group_sum(x, pos, k, kw);
    double add = own * sq;
    if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
    if (valid) {
      a.R[q] = Rs;
      a.Sb[q] = (T)(ik.avg_w * (double)bq + add);
      if (pos == k - 1) {
        a.u_par[h] = (T)uh;
        a.Z[h] = sum > 0.0 ? sum : -(double)k;
        if (a.vacc) a.vacc[h] += uh;
      }
    }
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
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t h = list ? list[i] : (int32_t)i;
    const int32_t b = a.cb[h], e = a.cb[h + 1];
    const double Zh = a.Z[h];
    double uh = 0.0;
    for (int32_t q = b; q < e; ++q) {
      const double s = a.sg_first ? (double)a.sg_first[q] : sig_of<T>(a.R[q], Zh, rm_mode, eps);
      uh += s * (double)a.u[q];
    }
    const double opp = a.mover == 0 ? (double)a.rb[h] : (double)a.ra[h];
    const double own = a.mover == 0 ? (double)a.ra[h] : (double)a.rb[h];
    double sum = 0.0;
    for (int32_t q = b; q < e; ++q) {
      const T rq = a.R[q];
      const double s = a.sg_first ? (double)a.sg_first[q] : sig_of<T>(rq, Zh, rm_mode, eps);
      const double r = sgn * opp * ((double)a.u[q] - uh);
      const T Rs = (T)regret_update<PAPER>((double)rq, r, ik, variant);
      a.R[q] = Rs;
      sum += rm_x((double)Rs, rm_mode, eps);
      double add = own * s;
      if (!PAPER && variant == PASUR_CFR_PLUS) add *= ik.avg_t;
      a.Sb[q] = (T)(ik.avg_w * (double)a.Sb[q] + add);
    }
    a.u_par[h] = (T)uh;
    a.Z[h] = sum > 0.0 ? sum : -(double)(e - b);
    if (a.vacc) a.vacc[h] += uh;
  }
}

// kernel ids of the profile records (pasur_profile_read)
enum { PK_DOWN = 4, PK_UP_CHUNK = 5, PK_UP_PARENT = 6, PK_UP_LIST = 7, PK_SETUP = 8 };

template <class T, bool PAPER>
int sweep_t(pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p, int64_t t0,
            int n_iters, hipStream_t s) {
  const SweepIndex &x = *f->sweep;
  const int rm = p->rm_mode, var = p->variant;
  const double eps = p->eps;
  T *sg[9], *R[9], *Sb[9], *ra[9], *rb[9], *u[9];
  for (int l = 0; l <= 8; ++l) {
    sg[l] = (T *)st->sigma[l];
    R[l] = (T *)st->R[l];
    Sb[l] = (T *)st->Sbar[l];
    ra[l] = (T *)st->reachA[l];
    rb[l] = (T *)st->reachB[l];
    u[l] = (T *)st->u[l];
  }
  // regret-matching sums per parent (levels 0..7), stream-ordered scratch
  int64_t zoff[9];
  zoff[0] = 0;
  for (int l = 0; l <= 7; ++l) zoff[l + 1] = zoff[l] + f->n[l];
  double *Zbuf = nullptr;
  PASUR_TRY_HIP(hipMallocAsync((void **)&Zbuf, (size_t)std::max<int64_t>(zoff[8], 1) * sizeof(double), s));
  double *Z[8];
  for (int l = 0; l <= 7; ++l) Z[l] = Zbuf + zoff[l];
  {
    ProfScope ps(PK_SETUP, 0, s);
    for (int l = 7; l >= 1; --l) {
      if (x.n_act[l] == f->n[l]) continue;
      k_sw_chain_u<T><<<grid_of(f->n[l]), kBlk, 0, s>>>(f->n[l], x.passive[l], f->child_begin[l],
                                                         u[l], u[l + 1]);
      k_sw_zinit<T><<<grid_of(f->n[l]), kBlk, 0, s>>>(f->n[l], x.passive[l], f->child_begin[l],
                                                       R[l + 1], Z[l], rm, eps);
    }
  }
  for (int it = 0; it < n_iters; ++it) {
    const int64_t t = t0 + it;
    const IterK ik = iter_k(p, t);
    const bool first = it == 0, last = it == n_iters - 1;
    // FindReachProbability, levels 1..7 (every node on the last iteration)
    for (int L = 1; L <= 7; ++L) {
      const bool dense = last || x.n_act[L] == f->n[L];
      const int64_t n = dense ? f->n[L] : x.n_act[L];
      if (n == 0) continue;
      ProfScope ps(PK_DOWN, L, s, n, 0, 0, 0, 1);
      k_sw_down<T><<<grid_of(n), kBlk, 0, s>>>(n, dense ? nullptr : x.act[L], (L - 1) & 1,
                                                f->parent[L], R[L], first ? sg[L] : nullptr,
                                                Z[L - 1], ra[L - 1], rb[L - 1], ra[L], rb[L],
                                                rm, eps);
    }
    // FindUtility, levels 8..1
    for (int L = 8; L >= 1; --L) {
      UpArgs<T> a;
      a.par = f->parent[L];
      a.cb = f->child_begin[L - 1];
      a.R = R[L];
      a.Sb = Sb[L];
      a.sg_first = first ? sg[L] : nullptr;
      a.u = u[L];
      a.u_par = u[L - 1];
      a.Z = Z[L - 1];
      a.ra = ra[L - 1];
      a.rb = rb[L - 1];
      a.vacc = L == 1 ? st->vacc : nullptr;
      a.mover = (L - 1) & 1;
      if (x.n_act[L - 1] < f->n[L - 1]) {
        const int64_t n = x.n_act[L - 1];
        if (n == 0) continue;
        ProfScope ps(PK_UP_LIST, L, s, 0, n, 0, 0, 1);
        k_sw_up_parent<T, PAPER><<<grid_of(n), kBlk, 0, s>>>(n, x.act[L - 1], a, ik, var, rm, eps);
      } else if (x.chunk[L]) {
        const int64_t nc = x.n_chunk[L];
        ProfScope ps(PK_UP_CHUNK, L, s, f->n[L], f->n[L - 1], 0, 0, 1);
        k_sw_up_chunk<T, PAPER><<<grid_of(nc * 64), kBlk, 0, s>>>(nc, x.chunk[L], a, ik, var, rm, eps);
      } else {
        const int64_t n = f->n[L - 1];
        if (n == 0) continue;
        ProfScope ps(PK_UP_PARENT, L, s, f->n[L], n, 0, 0, 1);
        k_sw_up_parent<T, PAPER><<<grid_of(n), kBlk, 0, s>>>(n, nullptr, a, ik, var, rm, eps);
      }
    }
  }
  {
    ProfScope ps(PK_SETUP, 1, s);
    for (int L = 1; L <= 8; ++L)
      if (f->n[L] > 0)
        k_sw_sigma_out<T><<<grid_of(f->n[L]), kBlk, 0, s>>>(f->n[L], f->parent[L], R[L],
                                                             Z[L - 1], sg[L], rm, eps);
  }
  hipError_t e = hipGetLastError();
  (void)hipFreeAsync(Zbuf, s);
  if (e != hipSuccess) {
    set_error("streaming sweeps: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  return PASUR_OK;
}

}  // namespace

bool sweep_pays(const pasur_fgt *f) {
  // Measured on full games: the persistent segment kernel runs a round at
  // about 7e10 node-updates/s once it fills the chip; the streaming sweeps
  // are bound by HBM plus ~15 launches per iteration, which only large
  // rounds amortise.
  int64_t nodes = 0;
  for (int l = 0; l <= 8; ++l) nodes += f->n[l];
  return nodes >= (int64_t)40 * 1000 * 1000;
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
