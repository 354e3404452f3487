// pasur_play.hip -- self-play with average strategies: the paper's way of
// estimating a deal's fair value (section "Experimental Evaluation").  One
// thread per game walks the unfolded trees of a solved subgame from a root:
// at each decision the player to move samples one child (inverse CDF of the
// average strategy, or uniformly at random); at a round's last level the
// game adds the leaf's round points and continues at the linked next-round
// root.  Random numbers come from a counter-based SplitMix64 stream, so any
// game can be replayed on its own.
#include "pasur_internal.hpp"

#include <cstring>

using namespace pasur;

namespace {

constexpr int kMaxRounds = 6;

struct PlayRound {
  const int32_t *cb[8];
  const void *sbar[9];
  const int32_t *link;
  const int16_t *base;
};

struct PlayArgs {
  PlayRound r[kMaxRounds];
  int n_rounds, dtype, policy[2], root;
  uint64_t seed;
  int64_t n_games;
};

// kGamesPerThread games per thread, g, g + stride, ... (stride = threads in
// the grid), stepped together so that their dependent gathers overlap (one
// game per thread: 19.3 ms per three matchups of 2^24 full games; two 17.7,
// four 16.2, eight 15.5).  A thread's games past the last one are played
// (indices stay valid) and their margins dropped.
constexpr int kGamesPerThread = 8;

template <class T>
__global__ void k_selfplay(PlayArgs a, int32_t *__restrict__ margin) {
  constexpr int G = kGamesPerThread;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g0 >= a.n_games) return;
  int64_t g[G];
  int32_t q[G], m[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    g[i] = g0 + i * stride;
    q[i] = a.root;
    m[i] = 0;
  }
  for (int r = 0; r < a.n_rounds; ++r) {
    const PlayRound &R = a.r[r];
    for (int l = 0; l < 8; ++l) {
      int32_t b[G], e[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        b[i] = R.cb[l][q[i]];
        e[i] = R.cb[l][q[i] + 1];
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int k = e[i] - b[i];
        int c = 0;
        if (k > 1) {
          const double u = splitmix_uniform(a.seed, (uint64_t)g[i] * 64u + (uint64_t)(r * 8 + l));
          c = choose<T>(u, reinterpret_cast<const T *>(R.sbar[l + 1]) + b[i], k, a.policy[l & 1]);
        }
        q[i] = b[i] + c;
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      m[i] += R.base[q[i]];
      if (r + 1 < a.n_rounds) q[i] = R.link[q[i]];
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i)
    if (g[i] < a.n_games) margin[g[i]] = m[i];
}

}  // namespace

extern "C" int pasur_selfplay(const pasur_fgt *const *fgts, int n_rounds,
                              const void *const *sigma_bar, int dtype, int root,
                              int64_t n_games, uint64_t seed, int policy_a, int policy_b,
                              int32_t *d_margin, void *stream) {
  if (!fgts || !sigma_bar || !d_margin || n_games < 0) {
    set_error("null argument or negative game count");
    return PASUR_E_INVAL;
  }
  if (n_games > (int64_t)INT32_MAX * 256) {
    set_error("n_games %lld beyond one launch (%lld)", (long long)n_games,
              (long long)INT32_MAX * 256);
    return PASUR_E_RANGE;
  }
  if (n_rounds < 1 || n_rounds > kMaxRounds) {
    set_error("n_rounds %d outside 1..%d", n_rounds, kMaxRounds);
    return PASUR_E_RANGE;
  }
  if (dtype != PASUR_F32 && dtype != PASUR_F64) {
    set_error("unknown dtype %d", dtype);
    return PASUR_E_RANGE;
  }
  for (int p : {policy_a, policy_b}) {
    if (p != PASUR_PLAY_SIGMA_BAR && p != PASUR_PLAY_UNIFORM) {
      set_error("unknown policy %d", p);
      return PASUR_E_RANGE;
    }
  }
  PlayArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int r = 0; r < n_rounds; ++r) {
    const pasur_fgt *f = fgts[r];
    if (!f) {
      set_error("fgts[%d] is NULL", r);
      return PASUR_E_INVAL;
    }
    if (r > 0 && f->round != fgts[r - 1]->round + 1) {
      set_error("rounds must be consecutive");
      return PASUR_E_INVAL;
    }
    if (r + 1 < n_rounds && f->round == 5) {
      set_error("round 5 is the last round");
      return PASUR_E_INVAL;
    }
    for (int l = 0; l < 8; ++l) a.r[r].cb[l] = f->child_begin[l];
    for (int l = 1; l <= 8; ++l) {
      a.r[r].sbar[l] = sigma_bar[r * 9 + l];
      if (!a.r[r].sbar[l]) {
        set_error("sigma_bar[%d][%d] is NULL", r, l);
        return PASUR_E_INVAL;
      }
    }
    if ((r + 1 < n_rounds && !f->link) || !f->leaf_base) {
      set_error("tree of round %d has no %s", f->round, f->leaf_base ? "link table" : "leaf scores");
      return PASUR_E_INVAL;
    }
    a.r[r].link = f->link;
    a.r[r].base = f->leaf_base;
  }
  if (root < 0 || root >= fgts[0]->n[0]) {
    set_error("root %d outside 0..%lld", root, (long long)fgts[0]->n[0] - 1);
    return PASUR_E_RANGE;
  }
  if (n_games == 0) return PASUR_OK;
  a.n_rounds = n_rounds;
  a.dtype = dtype;
  a.policy[0] = policy_a;
  a.policy[1] = policy_b;
  a.root = root;
  a.seed = seed;
  a.n_games = n_games;
  hipStream_t s = (hipStream_t)stream;
  const int64_t threads = (n_games + kGamesPerThread - 1) / kGamesPerThread;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  if (dtype == PASUR_F32)
    k_selfplay<float><<<grid, 256, 0, s>>>(a, d_margin);
  else
    k_selfplay<double><<<grid, 256, 0, s>>>(a, d_margin);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}
