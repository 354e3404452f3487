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
// Level-synchronous: one launch per level and direction, one thread per
// node; every launch reads the previous level's picks, so the mask never
// needs compacting.  Arithmetic is FP64 in registers with the state stored
// as float or double, in the same order as the definition above.
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

template <class T>
__global__ void k_es_down(EsLevel a) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n) return;
  bool reached = true;
  if (a.l > 0) {
    const int32_t pk = a.pick_up[a.par[h]];
    reached = pk == kAll || pk == (int32_t)h;
  }
  int32_t out = kNone;
  if (reached) {
    if ((a.l & 1) == a.p) {
      out = kAll;
    } else {
      const int32_t b = a.cb[h], e = a.cb[h + 1];
      const T *sg = reinterpret_cast<const T *>(a.sigma);
      T *sb = reinterpret_cast<T *>(a.Sbar);
      for (int32_t c = b; c < e; ++c) sb[c] = (T)((double)sb[c] + (double)sg[c]);
      int j = 0;
      if (e - b > 1)
        j = choose<T>(splitmix_uniform(a.seed, a.base + (uint64_t)h), sg + b, e - b,
                      PASUR_PLAY_SIGMA_BAR);
      out = b + j;
    }
  }
  a.pick[h] = out;
}

template <class T>
__global__ void k_es_up(EsLevel a) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n) return;
  const int32_t pk = a.pick[h];
  if (pk == kNone) return;
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
int es_run(const pasur_fgt *f, const pasur_cfr_state *st, int64_t t0, int64_t n_iters,
           uint64_t seed, int rm_mode, double eps, int32_t *picks, hipStream_t s) {
  int64_t off[9];
  off[0] = 0;
  for (int l = 0; l < 8; ++l) off[l + 1] = off[l] + f->n[l];
  const uint64_t N = (uint64_t)off[8];
  for (int64_t it = 0; it < n_iters; ++it) {
    const uint64_t t = (uint64_t)(t0 + it + 1);
    for (int p = 0; p < 2; ++p) {
      const uint64_t pass_base = (2 * (t - 1) + (uint64_t)p) * N;
      EsLevel lv[8];
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
        a.base = pass_base + (uint64_t)off[l];
        a.l = l;
        a.p = p;
        a.rm_mode = rm_mode;
        a.eps = eps;
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

extern "C" int64_t pasur_es_workspace_bytes(const pasur_fgt *fgt) {
  if (!fgt) {
    set_error("fgt is NULL");
    return PASUR_E_INVAL;
  }
  int64_t n = 0;
  for (int l = 0; l < 8; ++l) n += fgt->n[l];
  return n * (int64_t)sizeof(int32_t);
}

extern "C" int pasur_es_iterate(const pasur_fgt *fgt, const pasur_cfr_state *st, int64_t t0,
                                int64_t n_iters, uint64_t seed, int rm_mode, double eps,
                                void *workspace, int64_t workspace_bytes, void *stream) {
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
  const int64_t need = pasur_es_workspace_bytes(fgt);
  if (!workspace || workspace_bytes < need) {
    set_error("workspace of %lld bytes needed, %lld given", (long long)need,
              (long long)(workspace ? workspace_bytes : 0));
    return PASUR_E_INVAL;
  }
  if (n_iters == 0) return PASUR_OK;
  int32_t *picks = reinterpret_cast<int32_t *>(workspace);
  hipStream_t s = (hipStream_t)stream;
  if (st->dtype == PASUR_F32) return es_run<float>(fgt, st, t0, n_iters, seed, rm_mode, eps, picks, s);
  return es_run<double>(fgt, st, t0, n_iters, seed, rm_mode, eps, picks, s);
}
