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

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

using namespace pasur;

namespace {

// Optional per-launch timing of the sweep kernels (HIP events on the launch
// stream), off unless pasur_profile_enable(1) was called.
struct ProfRec {
  int kernel, level;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
bool g_prof_on = false;

void prof_clear() {
  for (auto &r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
}

struct ProfScope {
  ProfRec rec;
  hipStream_t s;
  bool on;
  ProfScope(int kernel, int level, hipStream_t stream) : s(stream), on(g_prof_on) {
    if (!on) return;
    rec.kernel = kernel;
    rec.level = level;
    (void)hipEventCreate(&rec.a);
    (void)hipEventCreate(&rec.b);
    (void)hipEventRecord(rec.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.b, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(rec);
  }
};

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

struct IterConsts {
  double dpos, dneg;  // DCFR discounts for R > 0 and R <= 0
  double avg_w;       // weight of the previous average-strategy sum
  double avg_t;       // multiplier of the new term (t for CFR+, else 1)
  double eps;
  int variant, rm_mode;
};

// FindUtility, one level, one thread per parent h (children cb[h]..cb[h+1]):
//   u(h) = sum sigma^t u;  r = s_p pi_{-p}(h) (u(q) - u(h));
//   R <- d R + r;  sigma^{t+1} = max(R, eps) / sum;  Sbar <- w Sbar + pi_p(h) sigma^t.
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
      const double d = Rq > 0.0 ? ic.dpos : ic.dneg;
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
    Sbar[q] = (T)(ic.avg_w * (double)Sbar[q] + add);
    sigma[q] = (T)s_new;
  }
  if (vacc) vacc[h] += uh;
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
                            T *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double pts = (double)base[i];
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

IterConsts consts_for(const pasur_cfr_params *p, int64_t t) {
  IterConsts ic;
  const double tm1 = (double)(t - 1);
  double pa = std::pow(tm1, p->alpha);
  double pb = std::pow(tm1, p->beta);
  ic.dpos = pa / (pa + 1.0);
  ic.dneg = pb / (pb + 1.0);
  ic.avg_w = p->variant == PASUR_DCFR ? std::pow(tm1 / (double)t, p->gamma) : 1.0;
  ic.avg_t = (double)t;
  ic.eps = p->eps;
  ic.variant = p->variant;
  ic.rm_mode = p->rm_mode;
  return ic;
}

template <class T>
int iterate_t(const pasur_fgt *f, const pasur_cfr_state *st, const pasur_cfr_params *p,
              int64_t t0, int n_iters, hipStream_t s) {
  for (int64_t t = t0; t < t0 + n_iters; ++t) {
    const IterConsts ic = consts_for(p, t);
    for (int l = 1; l <= 7; ++l) {
      ProfScope ps(0, l, s);
      k_down<T><<<grid_for(f->n[l]), kThreads, 0, s>>>(
          f->n[l], (l - 1) & 1, f->parent[l], (const T *)st->sigma[l],
          (const T *)st->reachA[l - 1], (const T *)st->reachB[l - 1], (T *)st->reachA[l],
          (T *)st->reachB[l]);
    }
    for (int l = 8; l >= 1; --l) {
      ProfScope ps(1, l, s);
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

template <class T, class L>
int values_t(const pasur_fgt *f, const L *leaf, void *const sigma[9], int mode, double *out,
             hipStream_t s) {
  int64_t mx = 1;
  for (int l = 0; l <= 7; ++l) mx = f->n[l] > mx ? f->n[l] : mx;
  double *buf[2] = {nullptr, nullptr};
  PASUR_TRY_HIP(hipMallocAsync((void **)&buf[0], mx * sizeof(double), s));
  hipError_t e = hipMallocAsync((void **)&buf[1], mx * sizeof(double), s);
  if (e != hipSuccess) {
    (void)hipFreeAsync(buf[0], s);
    set_error("hipMallocAsync: %s", hipGetErrorString(e));
    return PASUR_E_NOMEM;
  }
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
  e = hipGetLastError();
  (void)hipFreeAsync(buf[0], s);
  (void)hipFreeAsync(buf[1], s);
  if (e != hipSuccess) {
    set_error("tree values: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
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
  hipStream_t s = (hipStream_t)stream;
  return st->dtype == PASUR_F32 ? iterate_t<float>(f, st, p, t0, n_iters, s)
                                : iterate_t<double>(f, st, p, t0, n_iters, s);
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
                                    void *d_leaf, void *stream) {
  if (!f || !d_leaf) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (dtype != PASUR_F32 && dtype != PASUR_F64) {
    set_error("unknown dtype %d", dtype);
    return PASUR_E_RANGE;
  }
  if (f->round < 5 && !d_V_next) {
    set_error("rounds 0..4 need the next round's root values");
    return PASUR_E_INVAL;
  }
  const double *V = f->round < 5 ? d_V_next : nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (dtype == PASUR_F32)
    k_leaf_util<float><<<grid_for(f->n[8]), kThreads, 0, s>>>(f->n[8], f->leaf_base, f->link, V,
                                                              (float *)d_leaf);
  else
    k_leaf_util<double><<<grid_for(f->n[8]), kThreads, 0, s>>>(f->n[8], f->leaf_base, f->link, V,
                                                               (double *)d_leaf);
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
  hipStream_t s = (hipStream_t)stream;
  return dtype == PASUR_F32 ? values_t<float, double>(f, d_leaf, sigma, mode, d_out, s)
                            : values_t<double, double>(f, d_leaf, sigma, mode, d_out, s);
}

extern "C" int pasur_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_clear();
  g_prof_on = on != 0;
  return PASUR_OK;
}

extern "C" int pasur_profile_read(int64_t cap, int32_t *kernel, int32_t *level, float *ms,
                                  int64_t *n_out) {
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
  }
  return PASUR_OK;
}
