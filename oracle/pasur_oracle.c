/*
 * pasur_oracle.c -- FP64 CPU oracle for the Pasur round solver.
 *
 * TEST INFRASTRUCTURE ONLY (see pasur_oracle.h).  Plain and slow on
 * purpose: every function follows the passage of the paper it cites, in the
 * order the paper gives, with no blocking, fusion or reordering.  It runs
 * single-threaded unless or_set_threads asks for more; then only the
 * per-parent loops of one tree level inside or_cfr_run are shared out
 * (each parent's sums stay sequential in child order, so every result is
 * bit-identical to the single-threaded run) -- used to time the oracle on
 * all host cores beside the GPU.
 */
#include "pasur_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Cards (figure "Mapping Cards to Indices"; table of index sets for card
 * categories and scoring): index = 4*rank + suit, rank A..10,J,Q,K = 0..12,
 * suit clubs, diamonds, hearts, spades = 0..3.
 * ---------------------------------------------------------------------- */
static int o_is_numeric(int c) { return c < 40; }
static int o_value(int c) { return c / 4 + 1; } /* A = 1 .. 10 = 10 */
static int o_is_jack(int c) { return c >= 40 && c <= 43; }
static int o_is_club(int c) { return c % 4 == 0; }
/* Scoring table: each Ace 1, each Jack 1, 2 of clubs 2, 10 of diamonds 3. */
static int o_points(int c) {
  if (c <= 3) return 1;
  if (c == 4) return 2;
  if (c == 37) return 3;
  if (o_is_jack(c)) return 1;
  return 0;
}
static int o_bit(uint64_t m, int c) { return (int)((m >> c) & 1u); }

static int o_count_clubs(uint64_t m) {
  int n = 0;
  for (int c = 0; c < 52; c++)
    if (o_bit(m, c) && o_is_club(c)) n++;
  return n;
}
static int o_count_points(uint64_t m) {
  int n = 0;
  for (int c = 0; c < 52; c++)
    if (o_bit(m, c)) n += o_points(c);
  return n;
}

/* ------------------------------------------------------------------------
 * Subset-sum table (section "Numerical Actions"): every set of numeric cards
 * whose values sum to 11.  The paper stores them as the columns of a
 * [40, 2764] tensor.  For a numeric hand card c the captures are the sets
 * T \ {c} over the table entries T that contain c.  They are kept per card in
 * ascending mask order so that captures come out in canonical order.
 * ---------------------------------------------------------------------- */
static uint64_t *g_sets = NULL;
static int64_t g_nsets = 0, g_capsets = 0;
static uint64_t *g_card_caps[40];
static int64_t g_card_ncaps[40];
static int g_table_ready = 0;

static int o_push_set(uint64_t m) {
  if (g_nsets == g_capsets) {
    int64_t nc = g_capsets ? 2 * g_capsets : 4096;
    uint64_t *p = (uint64_t *)realloc(g_sets, (size_t)nc * sizeof(uint64_t));
    if (!p) return OR_ENOMEM;
    g_sets = p;
    g_capsets = nc;
  }
  g_sets[g_nsets++] = m;
  return OR_OK;
}

static int o_enum11(int start, int sum, uint64_t mask) {
  if (sum == 11) return o_push_set(mask);
  for (int c = start; c < 40; c++) {
    if (sum + o_value(c) <= 11) {
      int st = o_enum11(c + 1, sum + o_value(c), mask | (1ull << c));
      if (st) return st;
    }
  }
  return OR_OK;
}

static int o_cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int o_table(void) {
  if (g_table_ready) return OR_OK;
  int st = o_enum11(0, 0, 0);
  if (st) return st;
  for (int c = 0; c < 40; c++) {
    int64_t k = 0;
    for (int64_t i = 0; i < g_nsets; i++)
      if (o_bit(g_sets[i], c)) k++;
    g_card_caps[c] = (uint64_t *)malloc((size_t)(k ? k : 1) * sizeof(uint64_t));
    if (!g_card_caps[c]) return OR_ENOMEM;
    k = 0;
    for (int64_t i = 0; i < g_nsets; i++)
      if (o_bit(g_sets[i], c)) g_card_caps[c][k++] = g_sets[i] & ~(1ull << c);
    qsort(g_card_caps[c], (size_t)k, sizeof(uint64_t), o_cmp_u64);
    g_card_ncaps[c] = k;
  }
  g_table_ready = 1;
  return OR_OK;
}

int or_subset11_count(int64_t by_size[16]) {
  int st = o_table();
  if (st) return st;
  for (int i = 0; i < 16; i++) by_size[i] = 0;
  for (int64_t i = 0; i < g_nsets; i++) {
    int k = 0;
    for (int c = 0; c < 40; c++) k += o_bit(g_sets[i], c);
    by_size[k]++;
  }
  return (int)g_nsets;
}

/* ------------------------------------------------------------------------
 * Legal moves (capture table, section "Pasur"): the mover plays one card.
 *   numeric: every non-empty set S of pool numerics with value(c)+sum(S)=11
 *            is a capture; a numeric card with no capture is laid.  A card
 *            that can capture must capture; the must-capture duty applies
 *            card by card (the lay of a non-capturing card stays legal while
 *            another card could capture -- the second sample game lays a 10
 *            while holding a King that could capture).
 *   Jack:    captures every pool card except Queens and Kings; with nothing
 *            to capture it is laid.
 *   Queen/King: captures a single pool card of the same rank, one action per
 *            such card; with none it is laid.
 * Moves come out ordered by (card index, capture mask).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint8_t card;
  uint64_t cap;
} o_move;

#define O_NUMERIC_MASK ((1ull << 40) - 1)
#define O_JACK_MASK (0xFull << 40)
#define O_QUEEN_MASK (0xFull << 44)
#define O_KING_MASK (0xFull << 48)

static int o_moves(uint64_t hand, uint64_t pool, o_move *out, int cap_out) {
  int n = 0;
  for (int c = 0; c < 52; c++) {
    if (!o_bit(hand, c)) continue;
    int found = 0;
    if (o_is_numeric(c)) {
      for (int64_t i = 0; i < g_card_ncaps[c]; i++) {
        uint64_t s = g_card_caps[c][i];
        if ((s & ~pool) == 0) {
          if (n < cap_out) { out[n].card = (uint8_t)c; out[n].cap = s; }
          n++;
          found = 1;
        }
      }
    } else if (o_is_jack(c)) {
      uint64_t s = pool & (O_NUMERIC_MASK | O_JACK_MASK);
      if (s) {
        if (n < cap_out) { out[n].card = (uint8_t)c; out[n].cap = s; }
        n++;
        found = 1;
      }
    } else {
      int rank = c / 4;
      for (int x = 4 * rank; x < 4 * rank + 4; x++) {
        if (o_bit(pool, x)) {
          if (n < cap_out) { out[n].card = (uint8_t)c; out[n].cap = 1ull << x; }
          n++;
          found = 1;
        }
      }
    }
    if (!found) {
      if (n < cap_out) { out[n].card = (uint8_t)c; out[n].cap = 0; }
      n++;
    }
  }
  return n;
}

/* Apply one move (CodeSnippet ApplyActions, scoring table, Sur rule).
 *   lay:     the card leaves the hand and joins the pool.
 *   capture: card and captured cards leave hand and pool; the mover counts
 *            their clubs and points and becomes the last picker.  A capture
 *            that empties the pool is a Sur (+5) unless made with a Jack or
 *            in the final round.
 * After the final ply of the final round the last picker of that round
 * takes what is left in the pool (clubs and points, no Sur); if nobody
 * picked in that round the cards stay unclaimed.  The leaf keeps the pool as
 * it was before that clean-up. */
static void o_apply(int round, int ply, uint64_t *pool, uint64_t *handA,
                    uint64_t *handB, int8_t rs[8], o_move mv) {
  int mover = ply % 2; /* 0 Alex, 1 Bob: Alex moves first every turn */
  uint64_t cbit = 1ull << mv.card;
  if (mover == 0) *handA &= ~cbit;
  else *handB &= ~cbit;
  if (mv.cap == 0) {
    *pool |= cbit;
  } else {
    uint64_t before = *pool;
    uint64_t taken = mv.cap | cbit;
    *pool &= ~mv.cap;
    int cl = o_count_clubs(taken), pt = o_count_points(taken);
    if (mover == 0) { rs[RS_ACL] += cl; rs[RS_APT] += pt; }
    else { rs[RS_BCL] += cl; rs[RS_BPT] += pt; }
    rs[RS_L] = (int8_t)(mover + 1);
    if (mv.cap == before && !o_is_jack(mv.card) && round != 5) {
      if (mover == 0) rs[RS_ASR] += 1;
      else rs[RS_BSR] += 1;
    }
  }
  if (round == 5 && ply == 7 && rs[RS_L] != 0) {
    int cl = o_count_clubs(*pool), pt = o_count_points(*pool);
    if (rs[RS_L] == 1) { rs[RS_ACL] += cl; rs[RS_APT] += pt; }
    else { rs[RS_BCL] += cl; rs[RS_BPT] += pt; }
  }
}

int or_children(int round, int ply, uint64_t pool, uint64_t handA,
                uint64_t handB, const int8_t rs[8], int max_children,
                uint8_t *act_card, uint64_t *act_cap, uint64_t *c_pool,
                uint64_t *c_handA, uint64_t *c_handB, int8_t *c_rs) {
  if (o_table()) return OR_ENOMEM;
  if (round < 0 || round > 5 || ply < 0 || ply > 7) return OR_ERANGE;
  o_move mv[512];
  int n = o_moves(ply % 2 == 0 ? handA : handB, pool, mv, 512);
  if (n > 512) return OR_ERANGE;
  for (int i = 0; i < n && i < max_children; i++) {
    uint64_t p = pool, a = handA, b = handB;
    int8_t r[8];
    memcpy(r, rs, 8);
    o_apply(round, ply, &p, &a, &b, r, mv[i]);
    act_card[i] = mv[i].card;
    act_cap[i] = mv[i].cap;
    c_pool[i] = p;
    c_handA[i] = a;
    c_handB[i] = b;
    memcpy(c_rs + 8 * i, r, 8);
  }
  return n;
}

/* ------------------------------------------------------------------------
 * Score passed between rounds (section "Score Tensors"; Between-Hand
 * update): s = (ca, cb, d, bonus) plus the round's running score.  Clubs are
 * only counted while the bonus is undecided; reaching 7 clubs gives the
 * bonus (1 Alex, 2 Bob) and resets both club counts; the point difference
 * gains (Apt + 5 Asr) - (Bpt + 5 Bsr).
 * ---------------------------------------------------------------------- */
static int o_round_points(const int8_t rs[8]) {
  return (rs[RS_APT] + 5 * rs[RS_ASR]) - (rs[RS_BPT] + 5 * rs[RS_BSR]);
}

int or_combine_score(const int8_t s[4], const int8_t rs[8], int8_t out[4]) {
  int ca = s[0], cb = s[1], d = s[2], bonus = s[3];
  if (bonus == 0) {
    ca += rs[RS_ACL];
    cb += rs[RS_BCL];
  }
  d += o_round_points(rs);
  if (bonus == 0 && ca >= 7) { bonus = 1; ca = 0; cb = 0; }
  else if (bonus == 0 && cb >= 7) { bonus = 2; ca = 0; cb = 0; }
  out[0] = (int8_t)ca;
  out[1] = (int8_t)cb;
  out[2] = (int8_t)d;
  out[3] = (int8_t)bonus;
  return OR_OK;
}

/* Sort key of a score: (bonus, ca, cb, d). */
static int64_t o_score_key(const int8_t s[4]) {
  return ((int64_t)s[3] << 24) | ((int64_t)s[0] << 16) | ((int64_t)s[1] << 8) |
         (int64_t)(s[2] + 128);
}

/* ------------------------------------------------------------------------
 * Round game tree (sections "Game Tensor" and "Actions"): level 0 holds the
 * distinct card states at the round start (pool only: the hands are the
 * round's dealt cards); level l+1 holds, parent by parent, the children of
 * every level-l node in move order.  Eight plies per round, Alex at even
 * plies.
 * ---------------------------------------------------------------------- */
struct or_gt {
  int round;
  int64_t n[9];
  uint64_t *pool[9];
  uint8_t *hands[9]; /* bit i: Alex still holds his i-th dealt card; bit 4+i: Bob */
  int8_t *rs[9];     /* 8 bytes per node */
  int32_t *parent[9];
  int32_t *child_begin[8];
  uint8_t *act_card[9];
  uint64_t *act_cap[9];
  uint8_t hand_card[8]; /* deck cards behind the 8 hand bits */
};

void or_gt_free(or_gt *g) {
  if (!g) return;
  for (int l = 0; l < 9; l++) {
    free(g->pool[l]); free(g->hands[l]); free(g->rs[l]); free(g->parent[l]);
    free(g->act_card[l]); free(g->act_cap[l]);
    if (l < 8) free(g->child_begin[l]);
  }
  free(g);
}

static uint64_t o_hand_mask(const or_gt *g, uint8_t bits, int who) {
  uint64_t m = 0;
  for (int i = 0; i < 4; i++)
    if ((bits >> (4 * who + i)) & 1) m |= 1ull << g->hand_card[4 * who + i];
  return m;
}

or_gt *or_gt_build(const uint8_t deck[52], int round, const uint64_t *pools,
                   int64_t n_pools, int *status) {
  int st_dummy;
  if (!status) status = &st_dummy;
  *status = OR_OK;
  if (o_table()) { *status = OR_ENOMEM; return NULL; }
  if (round < 0 || round > 5 || n_pools < 1) { *status = OR_ERANGE; return NULL; }
  uint64_t seen = 0;
  for (int i = 0; i < 52; i++) {
    if (deck[i] >= 52 || o_bit(seen, deck[i])) { *status = OR_EINVAL; return NULL; }
    seen |= 1ull << deck[i];
  }
  uint64_t dealt_before = 0;
  for (int i = 0; i < 4 + 8 * round; i++) dealt_before |= 1ull << deck[i];
  for (int64_t i = 0; i < n_pools; i++) {
    if ((pools[i] & ~dealt_before) != 0) { *status = OR_EINVAL; return NULL; }
    if (i > 0 && pools[i] <= pools[i - 1]) { *status = OR_EINVAL; return NULL; }
  }
  or_gt *g = (or_gt *)calloc(1, sizeof(or_gt));
  if (!g) { *status = OR_ENOMEM; return NULL; }
  g->round = round;
  for (int i = 0; i < 8; i++) g->hand_card[i] = deck[4 + 8 * round + i];

  g->n[0] = n_pools;
  g->pool[0] = (uint64_t *)malloc((size_t)n_pools * 8);
  g->hands[0] = (uint8_t *)malloc((size_t)n_pools);
  g->rs[0] = (int8_t *)calloc((size_t)n_pools, 8);
  if (!g->pool[0] || !g->hands[0] || !g->rs[0]) goto nomem;
  for (int64_t i = 0; i < n_pools; i++) {
    g->pool[0][i] = pools[i];
    g->hands[0][i] = 0xFF;
  }

  for (int l = 0; l < 8; l++) {
    int mover = l % 2;
    o_move mv[512];
    /* count pass */
    int64_t total = 0;
    g->child_begin[l] = (int32_t *)malloc((size_t)(g->n[l] + 1) * 4);
    if (!g->child_begin[l]) goto nomem;
    for (int64_t i = 0; i < g->n[l]; i++) {
      uint64_t hand = o_hand_mask(g, g->hands[l][i], mover);
      int k = o_moves(hand, g->pool[l][i], mv, 512);
      if (k > 512) { or_gt_free(g); *status = OR_ERANGE; return NULL; }
      g->child_begin[l][i] = (int32_t)total;
      total += k;
      if (total > INT32_MAX) { or_gt_free(g); *status = OR_ERANGE; return NULL; }
    }
    g->child_begin[l][g->n[l]] = (int32_t)total;
    int L = l + 1;
    g->n[L] = total;
    size_t m = (size_t)(total ? total : 1);
    g->pool[L] = (uint64_t *)malloc(m * 8);
    g->hands[L] = (uint8_t *)malloc(m);
    g->rs[L] = (int8_t *)malloc(m * 8);
    g->parent[L] = (int32_t *)malloc(m * 4);
    g->act_card[L] = (uint8_t *)malloc(m);
    g->act_cap[L] = (uint64_t *)malloc(m * 8);
    if (!g->pool[L] || !g->hands[L] || !g->rs[L] || !g->parent[L] ||
        !g->act_card[L] || !g->act_cap[L])
      goto nomem;
    /* fill pass */
    int64_t q = 0;
    for (int64_t i = 0; i < g->n[l]; i++) {
      uint64_t hA = o_hand_mask(g, g->hands[l][i], 0);
      uint64_t hB = o_hand_mask(g, g->hands[l][i], 1);
      int k = o_moves(mover == 0 ? hA : hB, g->pool[l][i], mv, 512);
      for (int j = 0; j < k; j++, q++) {
        uint64_t p = g->pool[l][i], a = hA, b = hB;
        int8_t r[8];
        memcpy(r, g->rs[l] + 8 * i, 8);
        o_apply(round, l, &p, &a, &b, r, mv[j]);
        uint8_t bits = 0;
        for (int h = 0; h < 4; h++) {
          if (o_bit(a, g->hand_card[h])) bits |= (uint8_t)(1u << h);
          if (o_bit(b, g->hand_card[4 + h])) bits |= (uint8_t)(1u << (4 + h));
        }
        g->pool[L][q] = p;
        g->hands[L][q] = bits;
        memcpy(g->rs[L] + 8 * q, r, 8);
        g->parent[L][q] = (int32_t)i;
        g->act_card[L][q] = mv[j].card;
        g->act_cap[L][q] = mv[j].cap;
      }
    }
  }
  return g;
nomem:
  or_gt_free(g);
  *status = OR_ENOMEM;
  return NULL;
}

int64_t or_gt_size(const or_gt *g, int level) {
  if (!g || level < 0 || level > 8) return -1;
  return g->n[level];
}

int or_gt_copy(const or_gt *g, int field, int level, void *dst) {
  if (!g || level < 0 || level > 8 || !dst) return OR_EINVAL;
  int64_t n = g->n[level];
  switch (field) {
    case GT_POOL: memcpy(dst, g->pool[level], (size_t)n * 8); break;
    case GT_HANDS: memcpy(dst, g->hands[level], (size_t)n); break;
    case GT_RS: memcpy(dst, g->rs[level], (size_t)n * 8); break;
    case GT_PARENT:
      if (level == 0) return OR_EINVAL;
      memcpy(dst, g->parent[level], (size_t)n * 4); break;
    case GT_CHILD_BEGIN:
      if (level == 8) return OR_EINVAL;
      memcpy(dst, g->child_begin[level], (size_t)(n + 1) * 4); break;
    case GT_ACT_CARD:
      if (level == 0) return OR_EINVAL;
      memcpy(dst, g->act_card[level], (size_t)n); break;
    case GT_ACT_CAP:
      if (level == 0) return OR_EINVAL;
      memcpy(dst, g->act_cap[level], (size_t)n * 8); break;
    default: return OR_EINVAL;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Unfolding (section "In-Hand Updates", figure "Unfolding Process"): an FGT
 * node is a pair (GT node, inherited score id).  Every FGT root is a GT root
 * tagged with a score; the children of FGT node (g, s) are the GT children
 * of g, each tagged with the same s.  Built level by level, parent-major.
 * ---------------------------------------------------------------------- */
struct or_fgt {
  int64_t n[9];
  int32_t *gt[9], *sid[9], *parent[9], *child_begin[8];
  int64_t n_scores;
  int8_t *score_tab; /* 4 bytes per score: ca, cb, d, bonus */
  int64_t n_next;
  or_root *next_roots;
  int32_t *link; /* per leaf: index of its next-round root */
  int round;
};

void or_fgt_free(or_fgt *f) {
  if (!f) return;
  for (int l = 0; l < 9; l++) {
    free(f->gt[l]); free(f->sid[l]); free(f->parent[l]);
    if (l < 8) free(f->child_begin[l]);
  }
  free(f->score_tab);
  free(f->next_roots);
  free(f->link);
  free(f);
}

static or_fgt *o_unfold_core(const int64_t gt_n[9],
                             const int32_t *const cb[8],
                             const int32_t *root_gt, const int32_t *root_sid,
                             int64_t n_roots, int *status) {
  or_fgt *f = (or_fgt *)calloc(1, sizeof(or_fgt));
  if (!f) { *status = OR_ENOMEM; return NULL; }
  f->round = -1;
  f->n[0] = n_roots;
  f->gt[0] = (int32_t *)malloc((size_t)n_roots * 4);
  f->sid[0] = (int32_t *)malloc((size_t)n_roots * 4);
  if (!f->gt[0] || !f->sid[0]) goto nomem;
  for (int64_t j = 0; j < n_roots; j++) {
    if (root_gt[j] < 0 || root_gt[j] >= gt_n[0]) {
      or_fgt_free(f); *status = OR_EINVAL; return NULL;
    }
    f->gt[0][j] = root_gt[j];
    f->sid[0][j] = root_sid[j];
  }
  for (int l = 0; l < 8; l++) {
    int64_t total = 0;
    f->child_begin[l] = (int32_t *)malloc((size_t)(f->n[l] + 1) * 4);
    if (!f->child_begin[l]) goto nomem;
    for (int64_t i = 0; i < f->n[l]; i++) {
      int32_t g = f->gt[l][i];
      f->child_begin[l][i] = (int32_t)total;
      total += cb[l][g + 1] - cb[l][g];
      if (total > INT32_MAX) { or_fgt_free(f); *status = OR_ERANGE; return NULL; }
    }
    f->child_begin[l][f->n[l]] = (int32_t)total;
    int L = l + 1;
    f->n[L] = total;
    size_t m = (size_t)(total ? total : 1);
    f->gt[L] = (int32_t *)malloc(m * 4);
    f->sid[L] = (int32_t *)malloc(m * 4);
    f->parent[L] = (int32_t *)malloc(m * 4);
    if (!f->gt[L] || !f->sid[L] || !f->parent[L]) goto nomem;
    int64_t q = 0;
    for (int64_t i = 0; i < f->n[l]; i++) {
      int32_t g = f->gt[l][i];
      for (int32_t c = cb[l][g]; c < cb[l][g + 1]; c++, q++) {
        f->gt[L][q] = c;
        f->sid[L][q] = f->sid[l][i];
        f->parent[L][q] = (int32_t)i;
      }
    }
  }
  return f;
nomem:
  or_fgt_free(f);
  *status = OR_ENOMEM;
  return NULL;
}

or_fgt *or_fgt_unfold_csr(const int64_t gt_n[9],
                          const int32_t *const gt_child_begin[8],
                          const int32_t *root_gt, const int32_t *root_sid,
                          int64_t n_roots, int *status) {
  int st_dummy;
  if (!status) status = &st_dummy;
  *status = OR_OK;
  return o_unfold_core(gt_n, gt_child_begin, root_gt, root_sid, n_roots,
                       status);
}

static int o_cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
  uint64_t pool;
  int64_t skey;
} o_pair;

static int o_cmp_pair(const void *a, const void *b) {
  const o_pair *x = (const o_pair *)a, *y = (const o_pair *)b;
  if (x->pool != y->pool) return x->pool < y->pool ? -1 : 1;
  if (x->skey != y->skey) return x->skey < y->skey ? -1 : 1;
  return 0;
}

static void o_key_to_score(int64_t k, int8_t s[4]) {
  s[3] = (int8_t)((k >> 24) & 0xFF);
  s[0] = (int8_t)((k >> 16) & 0xFF);
  s[1] = (int8_t)((k >> 8) & 0xFF);
  s[2] = (int8_t)((k & 0xFF) - 128);
}

/* Between-Hand update (CodeSnippet BetweenHands): every FGT leaf (t, s)
 * passes the pool of t and the score s combined with t's running score to
 * the next round; the next-round roots are the distinct such pairs and the
 * linkage maps each leaf to its pair.  The final round has no successor. */
or_fgt *or_fgt_unfold(const or_gt *g, const or_root *roots, int64_t n_roots,
                      int *status) {
  int st_dummy;
  if (!status) status = &st_dummy;
  *status = OR_OK;
  if (!g || !roots || n_roots < 1) { *status = OR_EINVAL; return NULL; }
  /* roots strictly ascending by (pool, bonus, ca, cb, d), pools in the GT */
  for (int64_t j = 0; j < n_roots; j++) {
    const or_root *r = &roots[j];
    if (r->bonus < 0 || r->bonus > 2 || r->ca < 0 || r->cb < 0 ||
        (r->bonus != 0 && (r->ca != 0 || r->cb != 0)) || r->ca > 6 || r->cb > 6) {
      *status = OR_EINVAL; return NULL;
    }
    if (j > 0) {
      const or_root *p = &roots[j - 1];
      int8_t sp[4] = {p->ca, p->cb, p->d, p->bonus};
      int8_t sr[4] = {r->ca, r->cb, r->d, r->bonus};
      if (r->pool < p->pool ||
          (r->pool == p->pool && o_score_key(sr) <= o_score_key(sp))) {
        *status = OR_EINVAL; return NULL;
      }
    }
  }
  /* score table: distinct root scores ascending by (bonus, ca, cb, d) */
  int64_t *keys = (int64_t *)malloc((size_t)n_roots * 8);
  int32_t *root_gt = (int32_t *)malloc((size_t)n_roots * 4);
  int32_t *root_sid = (int32_t *)malloc((size_t)n_roots * 4);
  if (!keys || !root_gt || !root_sid) {
    free(keys); free(root_gt); free(root_sid);
    *status = OR_ENOMEM; return NULL;
  }
  for (int64_t j = 0; j < n_roots; j++) {
    int8_t s[4] = {roots[j].ca, roots[j].cb, roots[j].d, roots[j].bonus};
    keys[j] = o_score_key(s);
  }
  qsort(keys, (size_t)n_roots, 8, o_cmp_i64);
  int64_t ns = 0;
  for (int64_t j = 0; j < n_roots; j++)
    if (j == 0 || keys[j] != keys[j - 1]) keys[ns++] = keys[j];
  for (int64_t j = 0; j < n_roots; j++) {
    int8_t s[4] = {roots[j].ca, roots[j].cb, roots[j].d, roots[j].bonus};
    int64_t k = o_score_key(s);
    int64_t *hit = (int64_t *)bsearch(&k, keys, (size_t)ns, 8, o_cmp_i64);
    root_sid[j] = (int32_t)(hit - keys);
    uint64_t *gh = (uint64_t *)bsearch(&roots[j].pool, g->pool[0],
                                       (size_t)g->n[0], 8, o_cmp_u64);
    if (!gh) {
      free(keys); free(root_gt); free(root_sid);
      *status = OR_EINVAL; return NULL;
    }
    root_gt[j] = (int32_t)(gh - g->pool[0]);
  }
  const int32_t *cb[8];
  for (int l = 0; l < 8; l++) cb[l] = g->child_begin[l];
  or_fgt *f = o_unfold_core(g->n, cb, root_gt, root_sid, n_roots, status);
  free(root_gt);
  free(root_sid);
  if (!f) { free(keys); return NULL; }
  f->round = g->round;
  f->n_scores = ns;
  f->score_tab = (int8_t *)malloc((size_t)ns * 4);
  if (!f->score_tab) { free(keys); or_fgt_free(f); *status = OR_ENOMEM; return NULL; }
  for (int64_t i = 0; i < ns; i++) o_key_to_score(keys[i], f->score_tab + 4 * i);
  free(keys);

  if (g->round == 5) return f;
  int64_t nl = f->n[8];
  o_pair *pairs = (o_pair *)malloc((size_t)(nl ? nl : 1) * sizeof(o_pair));
  f->link = (int32_t *)malloc((size_t)(nl ? nl : 1) * 4);
  if (!pairs || !f->link) { free(pairs); or_fgt_free(f); *status = OR_ENOMEM; return NULL; }
  for (int64_t i = 0; i < nl; i++) {
    int32_t t = f->gt[8][i];
    int8_t nxt[4];
    or_combine_score(f->score_tab + 4 * f->sid[8][i], g->rs[8] + 8 * t, nxt);
    pairs[i].pool = g->pool[8][t];
    pairs[i].skey = o_score_key(nxt);
  }
  o_pair *uniq = (o_pair *)malloc((size_t)(nl ? nl : 1) * sizeof(o_pair));
  if (!uniq) { free(pairs); or_fgt_free(f); *status = OR_ENOMEM; return NULL; }
  memcpy(uniq, pairs, (size_t)nl * sizeof(o_pair));
  qsort(uniq, (size_t)nl, sizeof(o_pair), o_cmp_pair);
  int64_t nu = 0;
  for (int64_t i = 0; i < nl; i++)
    if (nu == 0 || o_cmp_pair(&uniq[i], &uniq[nu - 1]) != 0) uniq[nu++] = uniq[i];
  for (int64_t i = 0; i < nl; i++) {
    o_pair *hit = (o_pair *)bsearch(&pairs[i], uniq, (size_t)nu, sizeof(o_pair),
                                    o_cmp_pair);
    f->link[i] = (int32_t)(hit - uniq);
  }
  f->n_next = nu;
  f->next_roots = (or_root *)calloc((size_t)(nu ? nu : 1), sizeof(or_root));
  if (!f->next_roots) { free(pairs); free(uniq); or_fgt_free(f); *status = OR_ENOMEM; return NULL; }
  for (int64_t i = 0; i < nu; i++) {
    int8_t s[4];
    o_key_to_score(uniq[i].skey, s);
    f->next_roots[i].pool = uniq[i].pool;
    f->next_roots[i].ca = s[0];
    f->next_roots[i].cb = s[1];
    f->next_roots[i].d = s[2];
    f->next_roots[i].bonus = s[3];
  }
  free(pairs);
  free(uniq);
  return f;
}

int64_t or_fgt_size(const or_fgt *f, int level) {
  if (!f || level < 0 || level > 8) return -1;
  return f->n[level];
}
int64_t or_fgt_n_scores(const or_fgt *f) { return f ? f->n_scores : -1; }
int64_t or_fgt_n_next(const or_fgt *f) { return f ? f->n_next : -1; }

int or_fgt_copy(const or_fgt *f, int field, int level, void *dst) {
  if (!f || level < 0 || level > 8 || !dst) return OR_EINVAL;
  int64_t n = f->n[level];
  switch (field) {
    case FGT_GT: memcpy(dst, f->gt[level], (size_t)n * 4); break;
    case FGT_SID: memcpy(dst, f->sid[level], (size_t)n * 4); break;
    case FGT_PARENT:
      if (level == 0) return OR_EINVAL;
      memcpy(dst, f->parent[level], (size_t)n * 4); break;
    case FGT_CHILD_BEGIN:
      if (level == 8) return OR_EINVAL;
      memcpy(dst, f->child_begin[level], (size_t)(n + 1) * 4); break;
    case FGT_SCORE_TAB: memcpy(dst, f->score_tab, (size_t)f->n_scores * 4); break;
    case FGT_NEXT_ROOTS:
      if (!f->next_roots) return OR_EINVAL;
      memcpy(dst, f->next_roots, (size_t)f->n_next * sizeof(or_root)); break;
    case FGT_LINK:
      if (!f->link) return OR_EINVAL;
      memcpy(dst, f->link, (size_t)f->n[8] * 4); break;
    default: return OR_EINVAL;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Leaf utilities (equations final_util and passuputil), Alex's point
 * difference.  Final round: the 7-club bonus (+7 Alex, -7 Bob, 0 if nobody
 * reached 7 clubs; -7 there too with OR_LITERAL_BONUS0, the equation's
 * printed 7(2(bonus mod 2) - 1)) of the combined score plus the round's
 * points.  Earlier rounds: the value of the linked next-round root plus the
 * round's points.  The inherited point difference is not part of the
 * utility: points are added round by round.
 * ---------------------------------------------------------------------- */
int or_leaf_utilities(const or_gt *g, const or_fgt *f, const double *V_next, int flags,
                      double *leaf_u) {
  if (!g || !f || !leaf_u || (flags & ~OR_LITERAL_BONUS0)) return OR_EINVAL;
  double b0 = (flags & OR_LITERAL_BONUS0) ? -7.0 : 0.0;
  int last = (g->round == 5);
  if (!last && !V_next) return OR_EINVAL;
  for (int64_t i = 0; i < f->n[8]; i++) {
    int32_t t = f->gt[8][i];
    const int8_t *rs = g->rs[8] + 8 * t;
    double pts = (double)o_round_points(rs);
    if (last) {
      int8_t nxt[4];
      or_combine_score(f->score_tab + 4 * f->sid[8][i], rs, nxt);
      double b = nxt[3] == 1 ? 7.0 : (nxt[3] == 2 ? -7.0 : b0);
      leaf_u[i] = b + pts;
    } else {
      leaf_u[i] = V_next[f->link[i]] + pts;
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * CFR on one round's unfolded tree (section "CFR Algorithm", CodeSnippets
 * CFR, FindReachProbability, FindUtility; equations reg, RM, avsigma,
 * DFCR_REG, DFCR_AVG).  Both hands are visible, so an information set is a
 * single FGT node and its actions are that node's children.  Reach of every
 * root is 1.  Alex moves at even plies (levels 0,2,4,6), Bob at odd ones.
 * Utilities are Alex's; Bob's are their negation.
 *
 * One iteration t (1-based):
 *  1. reach: pi_A, pi_B of every internal node, the mover's factor times
 *     sigma^t of the edge taken;
 *  2. levels 8..1, parent by parent:
 *       u(h)   = sum over children q of sigma^t(q) u(q)
 *       r(q)   = s_p * pi_{-p}(h) * (u(q) - u(h)),  s_Alex = +1, s_Bob = -1
 *       R(q)  <- d * R(q) + r(q)   (DCFR: d = (t-1)^a/((t-1)^a+1) if R(q)>0,
 *                                   else (t-1)^b/((t-1)^b+1))
 *       sigma^{t+1}(q) = max(R(q), eps) / sum over siblings of max(R, eps)
 *       Sbar(q) <- ((t-1)/t)^g * Sbar(q) + pi_p(h) * sigma^t(q)
 *  3. vacc(root) += u(root).
 * ---------------------------------------------------------------------- */
struct or_cfr {
  int64_t n[9];
  int32_t *cb[8];
  double *sigma[9], *R[9], *Sbar[9], *u[9], *reachA[9], *reachB[9];
  double *vacc;
};

void or_cfr_free(or_cfr *c) {
  if (!c) return;
  for (int l = 0; l < 9; l++) {
    free(c->sigma[l]); free(c->R[l]); free(c->Sbar[l]); free(c->u[l]);
    free(c->reachA[l]); free(c->reachB[l]);
    if (l < 8) free(c->cb[l]);
  }
  free(c->vacc);
  free(c);
}

or_cfr *or_cfr_create(const int64_t n[9], const int32_t *const child_begin[8],
                      const double *leaf_u, int *status) {
  int st_dummy;
  if (!status) status = &st_dummy;
  *status = OR_OK;
  or_cfr *c = (or_cfr *)calloc(1, sizeof(or_cfr));
  if (!c) { *status = OR_ENOMEM; return NULL; }
  for (int l = 0; l < 9; l++) c->n[l] = n[l];
  for (int l = 0; l < 8; l++) {
    if (child_begin[l][0] != 0 || child_begin[l][n[l]] != n[l + 1]) {
      or_cfr_free(c); *status = OR_EINVAL; return NULL;
    }
    for (int64_t i = 0; i < n[l]; i++) {
      if (child_begin[l][i + 1] <= child_begin[l][i]) {
        /* every internal node of a round has at least one move */
        or_cfr_free(c); *status = OR_EINVAL; return NULL;
      }
    }
  }
  for (int l = 0; l < 9; l++) {
    size_t m = (size_t)(n[l] ? n[l] : 1);
    c->sigma[l] = (double *)calloc(m, 8);
    c->R[l] = (double *)calloc(m, 8);
    c->Sbar[l] = (double *)calloc(m, 8);
    c->u[l] = (double *)calloc(m, 8);
    c->reachA[l] = (double *)calloc(m, 8);
    c->reachB[l] = (double *)calloc(m, 8);
    if (!c->sigma[l] || !c->R[l] || !c->Sbar[l] || !c->u[l] || !c->reachA[l] ||
        !c->reachB[l]) { or_cfr_free(c); *status = OR_ENOMEM; return NULL; }
    if (l < 8) {
      c->cb[l] = (int32_t *)malloc((size_t)(n[l] + 1) * 4);
      if (!c->cb[l]) { or_cfr_free(c); *status = OR_ENOMEM; return NULL; }
      memcpy(c->cb[l], child_begin[l], (size_t)(n[l] + 1) * 4);
    }
  }
  c->vacc = (double *)calloc((size_t)(n[0] ? n[0] : 1), 8);
  if (!c->vacc) { or_cfr_free(c); *status = OR_ENOMEM; return NULL; }
  for (int64_t i = 0; i < n[8]; i++) c->u[8][i] = leaf_u[i];
  /* sigma^1 uniform over each node's children (CodeSnippet CFR: init) */
  for (int l = 0; l < 8; l++)
    for (int64_t h = 0; h < n[l]; h++) {
      int32_t b = c->cb[l][h], e = c->cb[l][h + 1];
      for (int32_t q = b; q < e; q++) c->sigma[l + 1][q] = 1.0 / (double)(e - b);
    }
  return c;
}

static int g_threads = 1;

int or_set_threads(int n) {
  g_threads = n < 1 ? 1 : n;
  return OR_OK;
}

static double o_dcfr_factor(double t_minus_1, double expo) {
  double p = pow(t_minus_1, expo); /* pow(0, 0) = 1 */
  return p / (p + 1.0);
}

int or_cfr_run(or_cfr *c, const or_params *p, int64_t t0, int n_iters) {
  if (!c || !p || t0 < 1 || n_iters < 0) return OR_EINVAL;
  if ((p->flags & ~(OR_SNIPPET_TOL | OR_SNIPPET_AVG)) ||
      (p->flags && p->variant != CFR_DCFR)) return OR_EINVAL;
  int snip_tol = (p->flags & OR_SNIPPET_TOL) != 0;
  int snip_avg = (p->flags & OR_SNIPPET_AVG) != 0;
  for (int64_t t = t0; t < t0 + n_iters; t++) {
    /* 1. reach probabilities, levels 1..7 (FindReachProbability) */
    for (int64_t j = 0; j < c->n[0]; j++) { c->reachA[0][j] = 1.0; c->reachB[0][j] = 1.0; }
    for (int l = 1; l <= 7; l++) {
      int mover = (l - 1) % 2;
#pragma omp parallel for num_threads(g_threads) schedule(static) if (g_threads > 1)
      for (int64_t h = 0; h < c->n[l - 1]; h++) {
        for (int32_t q = c->cb[l - 1][h]; q < c->cb[l - 1][h + 1]; q++) {
          double a = c->reachA[l - 1][h], b = c->reachB[l - 1][h];
          if (mover == 0) a *= c->sigma[l][q];
          else b *= c->sigma[l][q];
          c->reachA[l][q] = a;
          c->reachB[l][q] = b;
        }
      }
    }
    /* 2. utilities, regrets, regret matching, average (FindUtility) */
    double tm1 = (double)(t - 1);
    double avg_w = snip_avg ? 1.0 - 1.0 / pow((double)t, p->gamma)
                            : pow(tm1 / (double)t, p->gamma);
    for (int l = 8; l >= 1; l--) {
      int mover = (l - 1) % 2;
      double sgn = mover == 0 ? 1.0 : -1.0;
#pragma omp parallel for num_threads(g_threads) schedule(static) if (g_threads > 1)
      for (int64_t h = 0; h < c->n[l - 1]; h++) {
        int32_t b = c->cb[l - 1][h], e = c->cb[l - 1][h + 1];
        double uh = 0.0;
        for (int32_t q = b; q < e; q++) uh += c->sigma[l][q] * c->u[l][q];
        c->u[l - 1][h] = uh;
        double opp = mover == 0 ? c->reachB[l - 1][h] : c->reachA[l - 1][h];
        double own = mover == 0 ? c->reachA[l - 1][h] : c->reachB[l - 1][h];
        for (int32_t q = b; q < e; q++) {
          double r = sgn * opp * (c->u[l][q] - uh);
          double R = c->R[l][q];
          if (p->variant == CFR_DCFR) {
            int pos = snip_tol ? R >= 1e-5 : R > 0.0;
            double d = pos ? o_dcfr_factor(tm1, p->alpha) : o_dcfr_factor(tm1, p->beta);
            R = d * R + r;
          } else if (p->variant == CFR_PLUS) {
            R = R + r;
            if (R < 0.0) R = 0.0;
          } else {
            R = R + r;
          }
          c->R[l][q] = R;
        }
        double sum = 0.0;
        for (int32_t q = b; q < e; q++) {
          double x = p->rm_mode == RM_FLOOR ? fmax(c->R[l][q], p->eps)
                                            : fmax(c->R[l][q], 0.0);
          sum += x;
        }
        for (int32_t q = b; q < e; q++) {
          double x = p->rm_mode == RM_FLOOR ? fmax(c->R[l][q], p->eps)
                                            : fmax(c->R[l][q], 0.0);
          double s_new = sum > 0.0 ? x / sum : 1.0 / (double)(e - b);
          double w;
          if (p->variant == CFR_DCFR) w = avg_w;
          else w = 1.0;
          double add = own * c->sigma[l][q];
          if (p->variant == CFR_PLUS) add *= (double)t; /* linear averaging */
          if (snip_avg) add *= s_new;
          c->Sbar[l][q] = w * c->Sbar[l][q] + add;
          c->sigma[l][q] = s_new;
        }
      }
    }
    /* 3. root utility accumulator */
    for (int64_t j = 0; j < c->n[0]; j++) c->vacc[j] += c->u[0][j];
  }
  return OR_OK;
}

int or_cfr_copy(const or_cfr *c, int field, int level, double *dst) {
  if (!c || !dst || level < 0 || level > 8) return OR_EINVAL;
  int64_t n = c->n[level];
  switch (field) {
    case CF_SIGMA: memcpy(dst, c->sigma[level], (size_t)n * 8); break;
    case CF_R: memcpy(dst, c->R[level], (size_t)n * 8); break;
    case CF_SBAR: memcpy(dst, c->Sbar[level], (size_t)n * 8); break;
    case CF_U: memcpy(dst, c->u[level], (size_t)n * 8); break;
    case CF_REACHA: memcpy(dst, c->reachA[level], (size_t)n * 8); break;
    case CF_REACHB: memcpy(dst, c->reachB[level], (size_t)n * 8); break;
    case CF_VACC: memcpy(dst, c->vacc, (size_t)c->n[0] * 8); break;
    case CF_SIGMA_BAR: {
      /* Normalise (CodeSnippet CFR): sbar / sum over siblings; uniform when
       * the sum is zero (a node its mover never reaches). */
      if (level == 0) return OR_EINVAL;
      for (int64_t h = 0; h < c->n[level - 1]; h++) {
        int32_t b = c->cb[level - 1][h], e = c->cb[level - 1][h + 1];
        double s = 0.0;
        for (int32_t q = b; q < e; q++) s += c->Sbar[level][q];
        for (int32_t q = b; q < e; q++)
          dst[q] = s > 0.0 ? c->Sbar[level][q] / s : 1.0 / (double)(e - b);
      }
      break;
    }
    default: return OR_EINVAL;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * Exact tree values for a fixed profile (not in the paper, which lists
 * exploitability as future work): expected value under sigma, best response
 * of Alex (max at his nodes) or Bob (min at his nodes) against sigma, or the
 * minimax value (max at Alex, min at Bob; exact because both hands are
 * visible and no chance move happens inside a round).
 * ---------------------------------------------------------------------- */
int or_tree_values(const int64_t n[9], const int32_t *const child_begin[8],
                   const double *leaf, const double *const sigma[9], int mode,
                   int out_level, double *out) {
  if (out_level < 0 || out_level > 8) return OR_EINVAL;
  double *cur = (double *)malloc((size_t)(n[8] ? n[8] : 1) * 8);
  if (!cur) return OR_ENOMEM;
  memcpy(cur, leaf, (size_t)n[8] * 8);
  for (int l = 8; l >= 1; l--) {
    if (l == out_level) break;
    int mover = (l - 1) % 2;
    double *up = (double *)malloc((size_t)(n[l - 1] ? n[l - 1] : 1) * 8);
    if (!up) { free(cur); return OR_ENOMEM; }
    for (int64_t h = 0; h < n[l - 1]; h++) {
      int32_t b = child_begin[l - 1][h], e = child_begin[l - 1][h + 1];
      int use_max = (mode == TV_MINIMAX && mover == 0) || (mode == TV_BR_A && mover == 0);
      int use_min = (mode == TV_MINIMAX && mover == 1) || (mode == TV_BR_B && mover == 1);
      double v;
      if (use_max) {
        v = -INFINITY;
        for (int32_t q = b; q < e; q++) v = fmax(v, cur[q]);
      } else if (use_min) {
        v = INFINITY;
        for (int32_t q = b; q < e; q++) v = fmin(v, cur[q]);
      } else {
        v = 0.0;
        for (int32_t q = b; q < e; q++) v += sigma[l][q] * cur[q];
      }
      up[h] = v;
    }
    free(cur);
    cur = up;
  }
  memcpy(out, cur, (size_t)n[out_level] * 8);
  free(cur);
  return OR_OK;
}
