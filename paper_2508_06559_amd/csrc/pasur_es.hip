// pasur_es.hip -- external-sampling CFR on one round's unfolded tree
// (section "External Sampling", CodeSnippet ExternalSampling).
//
// One iteration is a pass for Alex, then a pass for Bob.  In the pass of
// player p the opponent keeps a single action per node, drawn from its
// current strategy, and p keeps all of its actions: the paper's boolean
// mask over the edges of the unfolded tree.  Here the mask is a pick per
// node, set level by level from the roots down:
//   kNone  the node is not reached in this pass,
//   kAll   a reached node of p: every child is reached,
//   c      a reached node of the opponent: only child c is reached.
// A reached opponent node adds its children's current strategy to their
// average sums when it draws.  Then, from the last level up, a reached node
// of p takes the strategy-weighted value of its children, adds to each
// child's regret the child's value minus its own (negated for Bob: values
// are Alex minus Bob) and regret-matches its children; a reached opponent
// node takes the value of its kept child.  Sampling weights cancel in this
// scheme, so all sums are plain.
//
// Two schedules give bit-identical results (every update is per node and
// in a fixed order, whatever order nodes are visited in):
//  - frontier (default): one persistent launch for all iterations.  Roots
//    are independent, so each workgroup takes a run of consecutive roots and
//    runs every iteration on them alone.  Per pass it keeps, for each level,
//    the list of its reached nodes (the frontier) in global scratch: the
//    reached nodes of level l + 1 are appended while level l draws (one LDS
//    counter per level, reserved once per wave), and the up sweep visits the
//    frontiers only.  Work per pass is proportional to the reached nodes
//    (about one opponent action in k per opponent level), not the tree.
//  - level: one launch per level and direction with one thread per node of
//    the level, reading the previous level's picks (no compaction).
// Arithmetic is FP64 in registers with the state stored as float or double,
// in the same order as the definition above.
#include "pasur_internal.hpp"

#include <cmath>

using namespace pasur;

namespace {

constexpr int32_t kNone = -1;
constexpr int32_t kAll = -2;
constexpr int kBlock = 256;

struct EsLevel {
  const int32_t *cb;       // child_begin of level l (n + 1 entries)
  const int32_t *par;      // parent of each level-l node (l >= 1)
  const int32_t *pick_up;  // picks of level l - 1 (l >= 1)
  int32_t *pick;           // picks of level l
  void *sigma, *R, *Sbar;  // edge arrays of level l + 1
  void *u_l;               // values of level l
  const void *u_c;         // values of level l + 1
  int64_t n;               // nodes on level l
  uint64_t seed, base;     // draw index of node h: base + h
  int l, p, rm_mode;
  double eps;
};

// Down step of a reached node h of level l in p's pass: its pick, and for
// an opponent node the average-sum update and the draw.  Returns the first
// kept child and sets *k to the number of kept children and *kids to the
// number of children.
template <class T>
__device__ __forceinline__ int32_t down_node(const EsLevel &a, int64_t h, int *k, int *kids) {
  const int32_t b = a.cb[h], e = a.cb[h + 1];
  *kids = e - b;
  if ((a.l & 1) == a.p) {
    a.pick[h] = kAll;
    *k = e - b;
    return b;
  }
  const T *sg = reinterpret_cast<const T *>(a.sigma);
  T *sb = reinterpret_cast<T *>(a.Sbar);
  for (int32_t c = b; c < e; ++c) sb[c] = (T)((double)sb[c] + (double)sg[c]);
  int j = 0;
  if (e - b > 1)
    j = choose<T>(splitmix_uniform(a.seed, a.base + (uint64_t)h), sg + b, e - b,
                  PASUR_PLAY_SIGMA_BAR);
  a.pick[h] = b + j;
  *k = 1;
  return b + j;
}

// Up step of a reached node h of level l (its pick set by the down sweep).
template <class T>
__device__ __forceinline__ void up_node(const EsLevel &a, int64_t h) {
  const int32_t pk = a.pick[h];
  const T *uc = reinterpret_cast<const T *>(a.u_c);
  T *ul = reinterpret_cast<T *>(a.u_l);
  if (pk != kAll) {
    ul[h] = uc[pk];
    return;
  }
  const int32_t b = a.cb[h], e = a.cb[h + 1];
  T *sg = reinterpret_cast<T *>(a.sigma);
  T *R = reinterpret_cast<T *>(a.R);
  double acc = 0.0;
  for (int32_t c = b; c < e; ++c) acc += (double)sg[c] * (double)uc[c];
  const T uh = (T)acc;
  ul[h] = uh;
  const double v = (double)uh;
  double sum = 0.0;
  for (int32_t c = b; c < e; ++c) {
    const double w = (double)uc[c];
    const T r = (T)((double)R[c] + (a.p == 0 ? w - v : v - w));
    R[c] = r;
    sum += a.rm_mode == PASUR_RM_FLOOR ? fmax((double)r, a.eps) : fmax((double)r, 0.0);
  }
  const double inv_k = 1.0 / (double)(e - b);
  for (int32_t c = b; c < e; ++c) {
    const double x = a.rm_mode == PASUR_RM_FLOOR ? fmax((double)R[c], a.eps)
                                                 : fmax((double)R[c], 0.0);
    sg[c] = (T)(sum > 0.0 ? x / sum : inv_k);
  }
}

template <class T>
__global__ void k_es_down(EsLevel a) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n) return;
  if (a.l > 0) {
    const int32_t pk = a.pick_up[a.par[h]];
    if (pk != kAll && pk != (int32_t)h) {
      a.pick[h] = kNone;
      return;
    }
  }
  int k, kids;
  (void)down_node<T>(a, h, &k, &kids);
}

template <class T>
__global__ void k_es_up(EsLevel a) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n) return;
  if (a.pick[h] == kNone) return;
  up_node<T>(a, h);
}

// ---- frontier schedule -------------------------------------------------------
// The state of a node sits in one record (the strategy, regret and average
// sum of the edge into it, and its value), packed from the solver's arrays
// when a call starts and unpacked when it ends: a reached node's children
// then share one or two cache lines instead of four arrays' worth.

template <class T>
struct alignas(4 * sizeof(T)) EsRec {
  T sg, R, Sb, u;
};

template <class T>
__global__ void k_es_pack(int64_t n, const T *sg, const T *R, const T *Sb, const T *u,
                          EsRec<T> *rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  EsRec<T> x;
  x.sg = sg ? sg[i] : (T)0;
  x.R = R ? R[i] : (T)0;
  x.Sb = Sb ? Sb[i] : (T)0;
  x.u = u[i];
  rec[i] = x;
}

template <class T>
__global__ void k_es_unpack(int64_t n, const EsRec<T> *rec, T *sg, T *R, T *Sb, T *u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const EsRec<T> x = rec[i];
  if (sg) {
    sg[i] = x.sg;
    R[i] = x.R;
    Sb[i] = x.Sb;
  }
  u[i] = x.u;
}

struct EsSegArgs {
  const int32_t *cb[8];
  void *rec[9];                // records of each level
  const int32_t *root_off[9];  // level-l node range of each root
  int32_t *front;              // frontier lists, level l at off[l]
  int32_t *choice;             // per frontier entry: kAll or the kept child
  int64_t off[9];
  int64_t n_roots, n_iters, t0;
  uint64_t N, seed;
  int roots_per_wg, rm_mode;
  double eps;
  unsigned long long *stats;   // optional: visits and kept children, see pasur_es_iterate
};

// Exclusive offset of this lane's k items in a wave-wide reservation of
// *counter (LDS); every lane of the wave must call it.
__device__ __forceinline__ int wave_reserve(int k, int *counter) {
  int x = k;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if ((int)(threadIdx.x & 63) >= d) x += y;
  }
  const int total = __shfl(x, 63, 64);
  int base = 0;
  if ((threadIdx.x & 63) == 63 && total > 0) base = atomicAdd(counter, total);
  base = __shfl(base, 63, 64);
  return base + x - k;
}

// Down step of reached node h of level l on records (as down_node): returns
// the first kept child, the number kept in *k, the number of children in
// *kids and the entry's choice in *ch.
template <class T>
__device__ __forceinline__ int32_t rec_down(const EsSegArgs &a, int l, int p, uint64_t base,
                                            int64_t h, int *k, int *kids, int32_t *ch) {
  const int32_t b = a.cb[l][h], e = a.cb[l][h + 1];
  *kids = e - b;
  if ((l & 1) == p) {
    *ch = kAll;
    *k = e - b;
    return b;
  }
  EsRec<T> *rc = reinterpret_cast<EsRec<T> *>(a.rec[l + 1]);
  int j = 0;
  if (e - b > 1)
    j = choose_by(splitmix_uniform(a.seed, base + (uint64_t)h), e - b, PASUR_PLAY_SIGMA_BAR,
                  [rc, b](int c) { return (double)rc[b + c].sg; });
  for (int c = b; c < e; ++c) rc[c].Sb = (T)((double)rc[c].Sb + (double)rc[c].sg);
  *ch = b + j;
  *k = 1;
  return b + j;
}

// Up step of reached node h of level l on records (as up_node).
template <class T>
__device__ __forceinline__ void rec_up(const EsSegArgs &a, int l, int p, int64_t h, int32_t ch) {
  EsRec<T> *rc = reinterpret_cast<EsRec<T> *>(a.rec[l + 1]);
  EsRec<T> *rl = reinterpret_cast<EsRec<T> *>(a.rec[l]);
  if (ch != kAll) {
    rl[h].u = rc[ch].u;
    return;
  }
  const int32_t b = a.cb[l][h], e = a.cb[l][h + 1];
  double acc = 0.0;
  for (int32_t c = b; c < e; ++c) acc += (double)rc[c].sg * (double)rc[c].u;
  const T uh = (T)acc;
  rl[h].u = uh;
  const double v = (double)uh;
  double sum = 0.0;
  for (int32_t c = b; c < e; ++c) {
    const double w = (double)rc[c].u;
    const T r = (T)((double)rc[c].R + (p == 0 ? w - v : v - w));
    rc[c].R = r;
    sum += a.rm_mode == PASUR_RM_FLOOR ? fmax((double)r, a.eps) : fmax((double)r, 0.0);
  }
  const double inv_k = 1.0 / (double)(e - b);
  for (int32_t c = b; c < e; ++c) {
    const double x = a.rm_mode == PASUR_RM_FLOOR ? fmax((double)rc[c].R, a.eps)
                                                 : fmax((double)rc[c].R, 0.0);
    rc[c].sg = (T)(sum > 0.0 ? x / sum : inv_k);
  }
}

template <class T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_es_frontier(EsSegArgs a) {
  __shared__ int cnt[9];
  __shared__ int64_t seg[9];  // where this workgroup's frontier of each level starts
  const int64_t r0 = (int64_t)blockIdx.x * a.roots_per_wg;
  const int64_t r1 = r0 + a.roots_per_wg < a.n_roots ? r0 + a.roots_per_wg : a.n_roots;
  if (threadIdx.x < 9) seg[threadIdx.x] = a.off[threadIdx.x] + a.root_off[threadIdx.x][r0];
  unsigned long long n_trav = 0, e_trav = 0, n_opp = 0, e_opp = 0;
  for (int64_t it = 0; it < a.n_iters; ++it) {
    const uint64_t t = (uint64_t)(a.t0 + it + 1);
    for (int p = 0; p < 2; ++p) {
      const uint64_t pass_base = (2 * (t - 1) + (uint64_t)p) * a.N;
      __syncthreads();  // the previous pass has finished with the counters
      if (threadIdx.x < 9) cnt[threadIdx.x] = 0;
      __syncthreads();
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        const uint64_t base = pass_base + (uint64_t)a.off[l];
        const int m = l == 0 ? (int)(r1 - r0) : cnt[l];
        for (int i0 = 0; i0 < m; i0 += BLOCK) {
          const int i = i0 + (int)threadIdx.x;
          int k = 0, kids = 0;
          int32_t first = 0;
          if (i < m) {
            const int64_t h = l == 0 ? r0 + i : (int64_t)a.front[seg[l] + i];
            int32_t ch;
            first = rec_down<T>(a, l, p, base, h, &k, &kids, &ch);
            a.choice[seg[l] + i] = ch;
            if ((l & 1) == p) {
              ++n_trav;
              e_trav += kids;
            } else {
              ++n_opp;
              e_opp += kids;
            }
          }
          if (l < 7) {
            const int pos = wave_reserve(k, &cnt[l + 1]);
            int32_t *dst = a.front + seg[l + 1] + pos;
            for (int j = 0; j < k; ++j) dst[j] = first + j;
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int l = 7; l >= 0; --l) {
        const int m = l == 0 ? (int)(r1 - r0) : cnt[l];
        for (int i = (int)threadIdx.x; i < m; i += BLOCK) {
          const int64_t h = l == 0 ? r0 + i : (int64_t)a.front[seg[l] + i];
          rec_up<T>(a, l, p, h, a.choice[seg[l] + i]);
        }
        __syncthreads();
      }
    }
  }
  if (a.stats) {
    atomicAdd(a.stats + 0, n_trav);
    atomicAdd(a.stats + 1, e_trav);
    atomicAdd(a.stats + 2, n_opp);
    atomicAdd(a.stats + 3, e_opp);
  }
}

void fill_levels(EsLevel lv[8], const pasur_fgt *f, const pasur_cfr_state *st, const int64_t off[9],
                 int32_t *picks, uint64_t seed, int rm_mode, double eps) {
  for (int l = 0; l < 8; ++l) {
    EsLevel &a = lv[l];
    a.cb = f->child_begin[l];
    a.par = l > 0 ? f->parent[l] : nullptr;
    a.pick_up = l > 0 ? picks + off[l - 1] : nullptr;
    a.pick = picks + off[l];
    a.sigma = st->sigma[l + 1];
    a.R = st->R[l + 1];
    a.Sbar = st->Sbar[l + 1];
    a.u_l = st->u[l];
    a.u_c = st->u[l + 1];
    a.n = f->n[l];
    a.seed = seed;
    a.base = (uint64_t)off[l];
    a.l = l;
    a.p = 0;
    a.rm_mode = rm_mode;
    a.eps = eps;
  }
}

constexpr int kFrontierBlock = 64;
constexpr int64_t kNodesPerWorkgroup = 4096;

template <class T>
int es_run(const pasur_fgt *f, const pasur_cfr_state *st, int64_t t0, int64_t n_iters,
           uint64_t seed, int rm_mode, double eps, int schedule, int roots_per_wg, void *ws,
           unsigned long long *stats, hipStream_t s) {
  int64_t off[9];
  off[0] = 0;
  for (int l = 0; l < 8; ++l) off[l + 1] = off[l] + f->n[l];
  const uint64_t N = (uint64_t)off[8];
  int32_t *picks = reinterpret_cast<int32_t *>(ws);
  if (f->n[0] == 0) return PASUR_OK;
  if (schedule == PASUR_ES_FRONTIER) {
    // workspace: the records of levels 0..8, then the frontier lists and
    // the entries' choices of levels 0..7
    EsRec<T> *recs = reinterpret_cast<EsRec<T> *>(ws);
    int64_t roff = 0;
    EsSegArgs a;
    for (int l = 0; l < 9; ++l) {
      a.rec[l] = recs + roff;
      const int64_t n = f->n[l];
      if (n > 0)
        k_es_pack<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            n, l > 0 ? (const T *)st->sigma[l] : nullptr, l > 0 ? (const T *)st->R[l] : nullptr,
            l > 0 ? (const T *)st->Sbar[l] : nullptr, (const T *)st->u[l], recs + roff);
      roff += n;
    }
    int32_t *lists = reinterpret_cast<int32_t *>(recs + roff);
    for (int l = 0; l < 8; ++l) a.cb[l] = f->child_begin[l];
    for (int l = 0; l < 9; ++l) {
      a.root_off[l] = f->root_off[l];
      a.off[l] = off[l];
    }
    a.front = lists;
    a.choice = lists + N;
    a.seed = seed;
    a.rm_mode = rm_mode;
    a.eps = eps;
    a.n_roots = f->n_roots;
    a.n_iters = n_iters;
    a.t0 = t0;
    a.N = N;
    int64_t total = 0;
    for (int l = 0; l < 9; ++l) total += f->n[l];
    int64_t per = kNodesPerWorkgroup * f->n_roots / (total > 0 ? total : 1);
    if (roots_per_wg > 0) per = roots_per_wg;
    a.roots_per_wg = (int)(per < 1 ? 1 : per > f->n_roots ? f->n_roots : per);
    a.stats = stats;
    const unsigned grid = (unsigned)((f->n_roots + a.roots_per_wg - 1) / a.roots_per_wg);
    k_es_frontier<T, kFrontierBlock><<<grid, kFrontierBlock, 0, s>>>(a);
    for (int l = 0; l < 9; ++l) {
      const int64_t n = f->n[l];
      if (n > 0)
        k_es_unpack<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            n, reinterpret_cast<const EsRec<T> *>(a.rec[l]), l > 0 ? (T *)st->sigma[l] : nullptr,
            l > 0 ? (T *)st->R[l] : nullptr, l > 0 ? (T *)st->Sbar[l] : nullptr, (T *)st->u[l]);
    }
    PASUR_TRY_HIP(hipGetLastError());
    return PASUR_OK;
  }
  EsLevel lv[8];
  fill_levels(lv, f, st, off, picks, seed, rm_mode, eps);
  for (int64_t it = 0; it < n_iters; ++it) {
    const uint64_t t = (uint64_t)(t0 + it + 1);
    for (int p = 0; p < 2; ++p) {
      const uint64_t pass_base = (2 * (t - 1) + (uint64_t)p) * N;
      for (int l = 0; l < 8; ++l) {
        lv[l].p = p;
        lv[l].base = pass_base + (uint64_t)off[l];
      }
      for (int l = 0; l < 8; ++l) {
        if (lv[l].n == 0) continue;
        const unsigned grid = (unsigned)((lv[l].n + kBlock - 1) / kBlock);
        k_es_down<T><<<grid, kBlock, 0, s>>>(lv[l]);
      }
      for (int l = 7; l >= 0; --l) {
        if (lv[l].n == 0) continue;
        const unsigned grid = (unsigned)((lv[l].n + kBlock - 1) / kBlock);
        k_es_up<T><<<grid, kBlock, 0, s>>>(lv[l]);
      }
      PASUR_TRY_HIP(hipGetLastError());
    }
  }
  return PASUR_OK;
}

}  // namespace

extern "C" int64_t pasur_es_workspace_bytes(const pasur_fgt *fgt, int dtype) {
  if (!fgt) {
    set_error("fgt is NULL");
    return PASUR_E_INVAL;
  }
  if (dtype != PASUR_F32 && dtype != PASUR_F64) {
    set_error("unknown dtype %d", dtype);
    return PASUR_E_RANGE;
  }
  int64_t n8 = 0;
  for (int l = 0; l < 8; ++l) n8 += fgt->n[l];
  const int64_t n9 = n8 + fgt->n[8];
  const int64_t rec = dtype == PASUR_F32 ? (int64_t)sizeof(EsRec<float>) : (int64_t)sizeof(EsRec<double>);
  return n9 * rec + 2 * n8 * (int64_t)sizeof(int32_t);
}

extern "C" int pasur_es_iterate(const pasur_fgt *fgt, const pasur_cfr_state *st, int64_t t0,
                                int64_t n_iters, uint64_t seed, int rm_mode, double eps,
                                int schedule, int roots_per_wg, void *workspace,
                                int64_t workspace_bytes, uint64_t *d_stats, void *stream) {
  if (!fgt || !st) {
    set_error("fgt or state is NULL");
    return PASUR_E_INVAL;
  }
  if (st->dtype != PASUR_F32 && st->dtype != PASUR_F64) {
    set_error("unknown dtype %d", st->dtype);
    return PASUR_E_RANGE;
  }
  if (rm_mode != PASUR_RM_FLOOR && rm_mode != PASUR_RM_POSITIVE) {
    set_error("unknown rm_mode %d", rm_mode);
    return PASUR_E_RANGE;
  }
  if (!(eps >= 0.0) || !std::isfinite(eps)) {
    set_error("eps must be finite and >= 0");
    return PASUR_E_RANGE;
  }
  if (schedule != PASUR_ES_FRONTIER && schedule != PASUR_ES_LEVEL) {
    set_error("unknown schedule %d", schedule);
    return PASUR_E_RANGE;
  }
  if (roots_per_wg < 0) {
    set_error("roots_per_wg %d must be >= 0", roots_per_wg);
    return PASUR_E_RANGE;
  }
  if (t0 < 0 || n_iters < 0) {
    set_error("t0 %lld and n_iters %lld must be >= 0", (long long)t0, (long long)n_iters);
    return PASUR_E_RANGE;
  }
  for (int l = 0; l <= 8; ++l) {
    if (!st->u[l] || (l > 0 && (!st->sigma[l] || !st->R[l] || !st->Sbar[l]))) {
      set_error("state arrays of level %d are NULL", l);
      return PASUR_E_INVAL;
    }
  }
  const int64_t need = pasur_es_workspace_bytes(fgt, st->dtype);
  if (!workspace || workspace_bytes < need) {
    set_error("workspace of %lld bytes needed, %lld given", (long long)need,
              (long long)(workspace ? workspace_bytes : 0));
    return PASUR_E_INVAL;
  }
  if (n_iters == 0) return PASUR_OK;
  if ((reinterpret_cast<uintptr_t>(workspace) & 31) != 0) {
    set_error("workspace must be 32-byte aligned");
    return PASUR_E_INVAL;
  }
  void *ws = workspace;
  unsigned long long *stats = reinterpret_cast<unsigned long long *>(d_stats);
  hipStream_t s = (hipStream_t)stream;
  if (st->dtype == PASUR_F32)
    return es_run<float>(fgt, st, t0, n_iters, seed, rm_mode, eps, schedule, roots_per_wg, ws,
                         stats, s);
  return es_run<double>(fgt, st, t0, n_iters, seed, rm_mode, eps, schedule, roots_per_wg,
                        ws, stats, s);
}
