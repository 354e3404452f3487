// pasur_infoset.hip -- infoset rows of unfolded-tree nodes (sections
// "Compressed Game Tensor" and "Infoset Tensors").
//
// One thread per row (staged in LDS, written out by the workgroup with
// 16-byte stores).  The node's action history is read from its GT
// ancestors (at most eight): in turn i (1-based) the mover's history gains i
// at the card he plays and 10 i at each pool card he collects.  The card
// states come from the node's own pool and hands.  Per card the compressed
// code is Alex's history minus Bob's, with the no-leg codes (100 Alex's
// hand, 105 Bob's hand, 110 pool) where that difference is 0 and 110 + d
// for a card laid and collecting in the same turn (out of play, 0 < |d| < 5).
// Columns 0..51: that code for cards in play this round, -127 for cards dealt
// earlier and out of play, 0 for cards not dealt yet; 52..54 the inherited
// score (Alex clubs or 7 if Alex owns the 7-clubs bonus, Bob clubs or 7 if
// Bob owns it, point difference); 55..57 round, turn and player of the action
// that leads to the node.
#include "pasur_internal.hpp"

using namespace pasur;

namespace {

constexpr int kRow = 58;
constexpr int kMlpIn = 192;

struct InfoArgs {
  const int32_t *edges;  // FGT nodes of the level, or NULL for all in order
  int64_t n;
  const int32_t *fgt_gt, *fgt_sid;
  const int8_t *score_tab;
  const uint8_t *act_card[9];
  const uint64_t *act_cap[9];
  const int32_t *parent[9];
  const uint64_t *pool[9];
  const uint8_t *hands[9];
  uint64_t hand_a, hand_b, dealt;  // card masks: the round's hands, all cards dealt so far
  uint8_t card[8];                 // the round's dealt cards, Alex's four then Bob's
  int level, round, format;
  void *out;
};

__device__ __forceinline__ int bit(uint64_t m, int c) { return (int)((m >> c) & 1ull); }

constexpr int kBlock = 256;

// Rows are built in LDS, one 58-byte row per thread; the workgroup then
// writes its consecutive rows with 16-byte stores.  Card bytes start from
// masks (-127 for a card dealt earlier and out of play, 0 otherwise) and
// only the cards in play this round get a code.
__global__ __launch_bounds__(kBlock) void k_infoset(InfoArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kBlock * kRow];
  const int t = (int)threadIdx.x;
  const int64_t q0 = (int64_t)blockIdx.x * kBlock;
  const int64_t q = q0 + t;
  if (q < a.n) {
    int8_t *row = lds + t * kRow;
    const int64_t e = a.edges ? (int64_t)a.edges[q] : q;
    int32_t g = a.fgt_gt[e];
    const int32_t sid = a.fgt_sid[e];
    const uint64_t pool_now = a.pool[a.level][g];
    const uint8_t h = a.hands[a.level][g];
    uint64_t held_a = 0, held_b = 0;
    for (int i = 0; i < 4; ++i) {
      if ((h >> i) & 1) held_a |= 1ull << a.card[i];
      if ((h >> (4 + i)) & 1) held_b |= 1ull << a.card[4 + i];
    }
    // per turn (0..3): the card each player laid and the cards he collected
    uint64_t lay[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    uint64_t cap[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int k = 8; k >= 1; --k) {
      if (k <= a.level) {
        lay[(k - 1) & 1][(k - 1) >> 1] = 1ull << a.act_card[k][g];
        cap[(k - 1) & 1][(k - 1) >> 1] = a.act_cap[k][g];
        g = a.parent[k][g];
      }
    }
    const uint64_t in_play = a.hand_a | a.hand_b | a.pool[0][g];
    const uint64_t gone = a.dealt & ~in_play;
    int16_t *row2 = reinterpret_cast<int16_t *>(row);  // rows start at even offsets
    for (int c = 0; c < 52; c += 2) {
      const int lo = bit(gone, c) ? 0x81 : 0, hi = bit(gone, c + 1) ? 0x81 : 0;
      row2[c >> 1] = (int16_t)(lo | (hi << 8));
    }
    for (uint64_t m = in_play; m; m &= m - 1) {
      const int c = __builtin_ctzll(m);
      int d = 0;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
        d += (tt + 1) * (bit(lay[0][tt], c) - bit(lay[1][tt], c)) +
             10 * (tt + 1) * (bit(cap[0][tt], c) - bit(cap[1][tt], c));
      if (d == 0) {
        d = bit(held_a, c) ? 100 : bit(held_b, c) ? 105 : bit(pool_now, c) ? 110 : 0;
      } else if (!bit(held_a | held_b | pool_now, c) && d > -5 && d < 5) {
        d += 110;
      }
      row[c] = (int8_t)d;
    }
    const int8_t *s = a.score_tab + 4 * (int64_t)sid;
    const int8_t s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3];
    row[52] = s3 == 1 ? (int8_t)7 : s0;
    row[53] = s3 == 2 ? (int8_t)7 : s1;
    row[54] = s2;
    row[55] = (int8_t)a.round;
    row[56] = (int8_t)((a.level - 1) >> 1);
    row[57] = (int8_t)((a.level - 1) & 1);
  }
  __syncthreads();
  const int64_t rows = a.n - q0 < kBlock ? a.n - q0 : kBlock;
  if (a.format == PASUR_INFOSET_INT8) {
    int8_t *dst = reinterpret_cast<int8_t *>(a.out) + q0 * kRow;
    const int64_t bytes = rows * kRow;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
      done = bytes & ~(int64_t)15;
      for (int64_t i = t; i < (done >> 4); i += kBlock)
        reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(lds)[i];
    }
    for (int64_t i = done + t; i < bytes; i += kBlock) dst[i] = lds[i];
  } else {
    // BF16 [rows][192]: eight columns per 16-byte store, row / 128 then zeros
    uint4 *dst = reinterpret_cast<uint4 *>(reinterpret_cast<__bf16 *>(a.out) + q0 * kMlpIn);
    constexpr int kChunks = kMlpIn / 8;
    for (int64_t i = t; i < rows * kChunks; i += kBlock) {
      const int r = (int)(i / kChunks), col0 = (int)(i % kChunks) * 8;
      uint32_t w[4];
      for (int k = 0; k < 4; ++k) {
        uint32_t pair = 0;
        for (int hh = 0; hh < 2; ++hh) {
          const int col = col0 + 2 * k + hh;
          const float v = col < kRow ? (float)lds[r * kRow + col] * (1.0f / 128.0f) : 0.0f;
          const __bf16 b = (__bf16)v;
          pair |= (uint32_t)__builtin_bit_cast(uint16_t, b) << (16 * hh);
        }
        w[k] = pair;
      }
      dst[i] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

}  // namespace

extern "C" int pasur_infoset_rows(const pasur_gt *gt, const pasur_fgt *fgt, int level,
                                  const int32_t *d_edges, int64_t n, int format, void *d_out,
                                  void *stream) {
  if (!gt || !fgt || !d_out || n < 0) {
    set_error("null argument or negative row count");
    return PASUR_E_INVAL;
  }
  if (level < 1 || level > 8) {
    set_error("level %d outside 1..8", level);
    return PASUR_E_RANGE;
  }
  if (n > (int64_t)INT32_MAX * kBlock) {
    set_error("n %lld beyond one launch", (long long)n);
    return PASUR_E_RANGE;
  }
  if (format != PASUR_INFOSET_INT8 && format != PASUR_INFOSET_MLP) {
    set_error("unknown format %d", format);
    return PASUR_E_RANGE;
  }
  if (!d_edges && n != fgt->n[level]) {
    set_error("without an edge list n must be the level size");
    return PASUR_E_INVAL;
  }
  if (gt->n[0] == 0 || fgt->round != gt->round) {
    set_error("the game tree does not belong to this unfolded tree");
    return PASUR_E_INVAL;
  }
  if (n == 0) return PASUR_OK;
  InfoArgs a;
  a.edges = d_edges;
  a.n = n;
  a.fgt_gt = fgt->gt[level];
  a.fgt_sid = fgt->sid[level];
  a.score_tab = fgt->score_tab;
  for (int k = 0; k < 9; ++k) {
    a.act_card[k] = gt->act_card[k];
    a.act_cap[k] = gt->act_cap[k];
    a.parent[k] = gt->parent[k];
    a.pool[k] = gt->pool[k];
    a.hands[k] = gt->hands[k];
  }
  a.hand_a = a.hand_b = 0;
  for (int i = 0; i < 4; ++i) {
    a.card[i] = gt->deck[4 + 8 * gt->round + i];
    a.card[4 + i] = gt->deck[8 + 8 * gt->round + i];
    a.hand_a |= 1ull << a.card[i];
    a.hand_b |= 1ull << a.card[4 + i];
  }
  a.dealt = 0;
  for (int i = 0; i < 12 + 8 * gt->round; ++i) a.dealt |= 1ull << gt->deck[i];
  a.level = level;
  a.round = gt->round;
  a.format = format;
  a.out = d_out;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  k_infoset<<<grid, kBlock, 0, (hipStream_t)stream>>>(a);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}
