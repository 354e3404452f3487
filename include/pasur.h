/*
 * pasur.h -- C ABI of the MI355X (gfx950) Pasur round solver.
 *
 * Scope: the data-parallel hot path of "Solving Pasur Using GPU-Accelerated
 * Counterfactual Regret Minimization" (arXiv 2508.06559): the round game
 * tree of card states, the Unfolding Process that pairs it with inherited
 * scores, the Between-Hand linkage to next-round roots, full-width DCFR on
 * one round's unfolded tree, and the backward round-value propagation, plus
 * exact best-response values used to measure exploitability.
 *
 * Conventions
 *  - Every function returns 0 (PASUR_OK) or a negative pasur_status; nothing
 *    aborts.  pasur_last_error() returns a message for the calling thread.
 *  - "device" pointers are HIP device memory on the current device;
 *    "host" pointers are ordinary CPU memory.  `stream` is a hipStream_t
 *    (NULL = the null stream).  Calls that take a stream enqueue work on it
 *    and return without waiting unless stated otherwise.
 *  - Tree handles (pasur_gt, pasur_fgt) own their device memory; free them
 *    with the matching *_free.  Build and unfold calls synchronise `stream`
 *    (they read level sizes back to allocate the next level).
 *  - Solver state (pasur_cfr_state) and output arrays are owned by the
 *    caller.
 *  - Results are deterministic: identical inputs give bit-identical outputs
 *    (no floating-point atomics).
 *
 * Cards: index = 4*rank + suit, rank A,2..10,J,Q,K = 0..12, suit clubs,
 * diamonds, hearts, spades = 0..3 (the paper's fixed 52-slot layout).
 * Deck layout: deck[0..3] is the initial pool; round r (0-based) deals
 * deck[4+8r..7+8r] to Alex and deck[8+8r..11+8r] to Bob.  A round has 8
 * plies (levels 0..8 of its tree); Alex moves at even plies.
 *
 * Canonical order (the paper's unique() order is unspecified): roots
 * ascending by (pool, bonus, ca, cb, d); level l+1 parent-major, siblings by
 * (played card, captured-card mask); score table ascending by
 * (bonus, ca, cb, d).
 */
#ifndef PASUR_H
#define PASUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PASUR_OK = 0,
  PASUR_E_INVAL = -1,    /* null or inconsistent argument, bad deck or roots */
  PASUR_E_RANGE = -2,    /* round outside 0..5, t0 < 1, unknown enum value */
  PASUR_E_OVERFLOW = -3, /* a tree level would exceed INT32_MAX nodes */
  PASUR_E_HIP = -4,      /* HIP runtime error (text in pasur_last_error) */
  PASUR_E_NOMEM = -5,    /* device allocation failed */
  PASUR_E_CAPACITY = -6  /* a fixed or caller-sized buffer is too small (the size
                            needed is reported where the call says so) */
} pasur_status;

typedef enum { PASUR_F32 = 0, PASUR_F64 = 1 } pasur_dtype;

/* A round root: the pool at the round start and the score inherited from
 * earlier rounds (paper tensor t_scr: Alex clubs, Bob clubs, point
 * difference, 7-club bonus 0/1 Alex/2 Bob).  Once the bonus is decided both
 * club counts are 0; an undecided bonus has ca, cb in 0..6. */
typedef struct {
  uint64_t pool;
  int8_t ca, cb, d, bonus;
  int32_t pad; /* must be 0 */
} pasur_root;

typedef struct pasur_gt pasur_gt;   /* round game tree of card states */
typedef struct pasur_fgt pasur_fgt; /* unfolded (full) game tree of a round */

const char *pasur_last_error(void);
int pasur_version(void);

/* ---- a1: round game tree --------------------------------------------------
 * Section "Actions" and the capture/scoring tables of section "Pasur".
 * Builds the game tree of round `round` from the distinct pools of
 * `d_roots` (device, n_roots entries, strictly ascending in canonical root
 * order; every pool a subset of the cards dealt before the round).  Level 0
 * holds the distinct pools ascending; every node's children are its legal
 * moves: a numeric card captures every set of pool numerics completing 11
 * (one child each) or is laid; a Jack captures all pool cards but Queens and
 * Kings or is laid; a Queen/King captures one same-rank pool card (one child
 * each) or is laid.  The must-capture duty is per card.  A capture that
 * empties the pool scores a Sur unless made with a Jack or in round 5.  In
 * round 5 the last ply's children include the clean-up by that round's last
 * picker.  `deck` is host memory (a permutation of 0..51).  On success
 * *out_gt receives a new handle.  Synchronises `stream`. */
int pasur_build_round_tree(const uint8_t deck[52], int round,
                           const pasur_root *d_roots, int64_t n_roots,
                           pasur_gt **out_gt, void *stream);
int pasur_gt_sizes(const pasur_gt *gt, int64_t n[9]);

typedef enum {
  PASUR_GT_POOL = 0,        /* uint64 per node */
  PASUR_GT_HANDS = 1,       /* uint8: bit i = Alex holds his i-th dealt card, bit 4+i Bob */
  PASUR_GT_RS = 2,          /* int8[8]: Acl, Bcl, last picker (0/1/2), Apt, Asr, Bpt, Bsr, 0 */
  PASUR_GT_PARENT = 3,      /* int32, levels 1..8 */
  PASUR_GT_CHILD_BEGIN = 4, /* int32, n+1 entries, levels 0..7 */
  PASUR_GT_ACT_CARD = 5,    /* uint8 played card, levels 1..8 */
  PASUR_GT_ACT_CAP = 6      /* uint64 captured cards (0 = lay), levels 1..8 */
} pasur_gt_field;
/* Synchronous copy of one GT array of one level into host memory. */
int pasur_gt_read(const pasur_gt *gt, int field, int level, void *host_dst);
/* Read-only device view of a game tree's arrays (no copy): the same arrays
 * as pasur_gt_read, owned by the handle and valid until pasur_gt_free.
 * Entries of levels a field does not have are NULL. */
typedef struct {
  int round;
  int64_t n[9];
  const uint64_t *pool[9];
  const uint8_t *hands[9];
  const uint64_t *rs[9];
  const int32_t *parent[9];
  const int32_t *child_begin[8];
  const uint8_t *act_card[9];
  const uint64_t *act_cap[9];
} pasur_gt_view;
int pasur_gt_get_view(const pasur_gt *gt, pasur_gt_view *out);
void pasur_gt_free(pasur_gt *gt);

/* ---- a2 + a3: unfolding and between-round linkage -------------------------
 * Sections "In-Hand Updates" (figure "Unfolding Process") and "Between-Hand
 * Updates" (CodeSnippet BetweenHands).  FGT level 0 are the roots `d_roots`
 * (the same device array given to pasur_build_round_tree for `gt`); the
 * children of FGT node (g, s) are the GT children of g tagged with the same
 * score id s, parent-major.  For rounds 0..4 every FGT leaf (t, s) links to
 * the next-round root (pool of t, normalise(s + running score of t)); the
 * distinct such roots, ascending, form the next round's root list.  The
 * handle keeps per-leaf base utilities so that `gt` may be freed afterwards.
 * Synchronises `stream`. */
int pasur_unfold_scores(const pasur_gt *gt, const pasur_root *d_roots,
                        int64_t n_roots, pasur_fgt **out_fgt, void *stream);
int pasur_fgt_sizes(const pasur_fgt *fgt, int64_t n[9], int64_t *n_scores,
                    int64_t *n_next);
typedef enum {
  PASUR_FGT_GT = 0,          /* int32 GT node per FGT node */
  PASUR_FGT_SID = 1,         /* int32 score id per FGT node */
  PASUR_FGT_PARENT = 2,      /* int32, levels 1..8 */
  PASUR_FGT_CHILD_BEGIN = 3, /* int32, n+1 entries, levels 0..7 */
  PASUR_FGT_SCORE_TAB = 4,   /* int8[4] per score: ca, cb, d, bonus (level ignored) */
  PASUR_FGT_NEXT_ROOTS = 5,  /* pasur_root per next-round root (level ignored) */
  PASUR_FGT_LINK = 6,        /* int32 per leaf: next-round root index (level ignored) */
  PASUR_FGT_LEAF_BASE = 7    /* int16 per leaf: round points (+ bonus in round 5) */
} pasur_fgt_field;
int pasur_fgt_read(const pasur_fgt *fgt, int field, int level, void *host_dst);
/* Read-only device view of an unfolded tree's arrays (no copy), owned by the
 * handle and valid until pasur_fgt_free: per level the FGT node's GT node,
 * score id, parent (levels 1..8) and child range (levels 0..7, n+1
 * entries); the score table (4 int8 per score), the next-round roots and
 * each leaf's link into them (NULL for round 5), and the leaves' round
 * points.  Callers that keep their own copies size them from `n`. */
typedef struct {
  int round;
  int64_t n[9];
  const int32_t *gt[9];
  const int32_t *sid[9];
  const int32_t *parent[9];
  const int32_t *child_begin[8];
  const int8_t *score_tab;
  int64_t n_scores;
  const pasur_root *next_roots;
  int64_t n_next;
  const int32_t *link;
  const int16_t *leaf_base;
} pasur_fgt_view;
int pasur_fgt_get_view(const pasur_fgt *fgt, pasur_fgt_view *out);
/* Device pointer to the next-round roots (owned by the handle, n_next
 * entries, canonical order); NULL for round 5. */
const pasur_root *pasur_fgt_next_roots(const pasur_fgt *fgt);
void pasur_fgt_free(pasur_fgt *fgt);

/* ---- a4: leaf utilities -----------------------------------------------------
 * Equations final_util and passuputil: Alex's point difference at every FGT
 * leaf.  Round 5: bonus (+7 Alex, -7 Bob, 0 none) of the combined score plus
 * the round's points (Apt + 5 Asr) - (Bpt + 5 Bsr); with
 * PASUR_LEAF_LITERAL_BONUS0 in `flags`, equation final_util as printed,
 * 7 (2 (bonus mod 2) - 1), which gives -7 for "none" too.  Rounds 0..4:
 * d_V_next[link] + the round's points, with d_V_next (device, double, one
 * value per next-round root) the next round's root values.  Writes n[8]
 * values of type `dtype` to d_leaf (device).  Unknown flag bits are
 * PASUR_E_RANGE. */
enum { PASUR_LEAF_LITERAL_BONUS0 = 1 };
int pasur_leaf_utilities(const pasur_fgt *fgt, const double *d_V_next, int dtype, int flags,
                         void *d_leaf, void *stream);

/* ---- a5..a10: DCFR on one round ---------------------------------------------
 * Section "CFR Algorithm" (CodeSnippets CFR, FindReachProbability,
 * FindUtility) with equations DFCR_REG, RM and DFCR_AVG.  Caller-owned
 * device arrays, all of element type `dtype` except vacc:
 *   sigma[l], R[l], Sbar[l]  levels 1..8, n[l] each (per edge);
 *   reachA[l], reachB[l]     levels 0..7, n[l] each (pi_Alex, pi_Bob);
 *   u[l]                     levels 0..8, n[l] each; u[8] = leaf utilities;
 *   vacc                     double, n[0]: sum of root utilities.
 * Arithmetic is FP64 in registers whatever `dtype` is. */
typedef struct {
  int dtype;
  void *sigma[9], *R[9], *Sbar[9];
  void *reachA[9], *reachB[9];
  void *u[9];
  double *vacc;
} pasur_cfr_state;

typedef enum { PASUR_DCFR = 0, PASUR_CFR_PLUS = 1, PASUR_CFR_VANILLA = 2 } pasur_variant;
typedef enum { PASUR_RM_FLOOR = 0, PASUR_RM_POSITIVE = 1 } pasur_rm_mode;
/* Kernel schedule of pasur_cfr_iterate (same results bit for bit, except
 * as noted for STREAM):
 * ROOT: one persistent workgroup per segment (a run of consecutive roots,
 *   see seg_nodes) runs all iterations on that segment's subtrees, its state
 *   held in LDS when it fits (else in global memory);
 * LEVEL_SYNC: one launch per level and sweep direction;
 * ROOT_GLOBAL: the persistent schedule with state always in global memory;
 * STREAM: one coalesced launch per level and sweep direction that streams
 *   the level through HBM, without a strategy array inside the call (sigma is
 *   recomputed from R and the parent's regret-matching sum) and without
 *   iterating chains of single-child nodes (their edges are forced).  Every
 *   state array ends as with the other schedules except Sbar of the edges
 *   below a node whose whole subtree is such a chain: those sums are not
 *   accumulated (their average strategy is 1 regardless).  The sigma array
 *   is read on a call's first iteration and written after its last; single-
 *   child edges must hold sigma = 1 (as pasur_cfr_init and the warm start
 *   leave them);
 * AUTO: STREAM for rounds of at least 1e7 nodes, else ROOT. */
typedef enum { PASUR_SCHED_ROOT = 0, PASUR_SCHED_LEVEL_SYNC = 1,
               PASUR_SCHED_ROOT_GLOBAL = 2, PASUR_SCHED_STREAM = 3,
               PASUR_SCHED_AUTO = 4 } pasur_schedule;
typedef struct {
  int variant;  /* pasur_variant */
  int rm_mode;  /* PASUR_RM_FLOOR: max(R, eps)/sum (the paper's executed rule);
                   PASUR_RM_POSITIVE: R+/sum, uniform if no R > 0 */
  double alpha; /* DCFR positive-regret exponent (paper: 1.5) */
  double beta;  /* DCFR negative-regret exponent (paper: 0) */
  double gamma; /* DCFR average-strategy exponent (paper: 2) */
  double eps;   /* regret floor (paper's executed rule: 1e-8) */
  int schedule; /* pasur_schedule */
  int block;    /* threads per workgroup of the persistent schedule: 0 (= 1024),
                   256, 512 or 1024 */
  int seg_nodes; /* persistent schedule: a workgroup takes a run of consecutive
                    roots of up to seg_nodes nodes (0: one root each) */
  int flags;     /* pasur_cfr_flags, 0 for the equations' DCFR */
} pasur_cfr_params;
/* The executed forms of CodeSnippet FindUtility where they differ from the
 * equations (DCFR only; honoured by PASUR_SCHED_LEVEL_SYNC, which AUTO picks
 * when any is set; the other schedules and plans reject them):
 *   SNIPPET_TOL: a regret is discounted as positive when R >= 1e-5 (the
 *     snippet's TOL) rather than R > 0;
 *   SNIPPET_AVG: Sbar <- (1 - 1/t^gamma) Sbar + pi_p(h) sigma^t(a)
 *     sigma^{t+1}(a): the snippet's weight, and its term, whose reach holds
 *     sigma^t(a) and which multiplies by the newly matched strategy. */
typedef enum { PASUR_CFR_SNIPPET_TOL = 1, PASUR_CFR_SNIPPET_AVG = 2 } pasur_cfr_flags;

/* R = 0, Sbar = 0, sigma uniform over every node's children, vacc = 0. */
int pasur_cfr_init(const pasur_fgt *fgt, const pasur_cfr_state *st, void *stream);
/* Iterations t0 .. t0+n_iters-1 (1-based t).  Each: reach down levels
 * 1..7; then levels 8..1: u(h) = sum sigma*u, regret
 * r = s_p pi_{-p}(h) (u(q) - u(h)), discounted regret update, regret
 * matching, discounted average-strategy accumulation with pi_p(h); then
 * vacc += u(root).  u[8] must hold the leaf utilities. */
int pasur_cfr_iterate(const pasur_fgt *fgt, const pasur_cfr_state *st,
                      const pasur_cfr_params *p, int64_t t0, int n_iters,
                      void *stream);
/* ---- a12: batched solve -------------------------------------------------------
 * A plan gathers n_items (unfolded tree, solver state) pairs -- e.g. one
 * round of many deals -- into one persistent launch of the segment schedule
 * and uploads everything the launch needs: item descriptors, the segment
 * list (longest first) and the DCFR constants of iterations
 * t_first..t_last (computed on the host).  pasur_plan_iterate only enqueues
 * one kernel, so it can be captured into a HIP graph; it runs iterations
 * t0..t0+n_iters-1 (within the plan's range) on every item, with results
 * bit-identical to pasur_cfr_iterate on each item.  Items keep their own
 * caller-owned arrays, which must outlive the plan.  All items share one
 * dtype.  plan_create synchronises `stream`. */
typedef struct pasur_plan pasur_plan;
int pasur_plan_create(const pasur_fgt *const *fgts, const pasur_cfr_state *const *states,
                      int n_items, const pasur_cfr_params *p, int64_t t_first,
                      int64_t t_last, pasur_plan **out, void *stream);
int pasur_plan_iterate(const pasur_plan *plan, int64_t t0, int n_iters, void *stream);
/* info: segments, LDS-resident segments, dynamic LDS bytes, threads per
 * workgroup, edges, internal nodes, roots, level-7 nodes. */
int pasur_plan_info(const pasur_plan *plan, int64_t info[8]);
void pasur_plan_free(pasur_plan *plan);

/* Normalise (CodeSnippet CFR): sigma_bar = Sbar / sum over siblings, uniform
 * where that sum is 0.  sigma_bar[l] (device, `st->dtype`, levels 1..8). */
int pasur_average_strategy(const pasur_fgt *fgt, const pasur_cfr_state *st,
                           void *const sigma_bar[9], void *stream);

typedef enum { PASUR_V_ITERATE_MEAN = 0, PASUR_V_SIGMA_BAR = 1 } pasur_value_mode;
/* Root values passed to the previous round (d_V, device double, n[0]).
 * ITERATE_MEAN: vacc / T (the paper's g_UTL / NUM_ITER).  SIGMA_BAR: the
 * expected value under sigma_bar (needs sigma_bar, else may be NULL). */
int pasur_round_values(const pasur_fgt *fgt, const pasur_cfr_state *st,
                       int value_mode, int64_t T, void *const sigma_bar[9],
                       double *d_V, void *stream);

/* ---- a11: exact values for exploitability ----------------------------------
 * Not in the paper (exploitability is its future work).  Up-sweep of
 * d_leaf (device double, n[8]) to the roots (d_out, device double, n[0]):
 * EXPECT: sum sigma * value; BR_A: max at Alex's nodes, expectation at Bob's;
 * BR_B: min at Bob's nodes, expectation at Alex's; MINIMAX: max/min.
 * sigma (type `dtype`, levels 1..8) may be NULL for MINIMAX.  Uses
 * stream-ordered scratch memory. */
typedef enum { PASUR_TV_EXPECT = 0, PASUR_TV_BR_A = 1, PASUR_TV_BR_B = 2,
               PASUR_TV_MINIMAX = 3 } pasur_tv_mode;
int pasur_tree_values(const pasur_fgt *fgt, const double *d_leaf, int dtype,
                      void *const sigma[9], int mode, double *d_out,
                      void *stream);

/* Exploitability of a subgame's average strategies, composed across its
 * rounds (the paper names exploitability as future work; the definition is
 * the standard one for two-player zero-sum games).  fgts[0..n_rounds-1] are
 * consecutive rounds, each the unfolding of the previous one's next-round
 * roots, the last being round 5; sigma_bar[r*9 + l] (device, `dtype`,
 * levels 1..8 of round slot r; entries r*9 are unused) are the average
 * strategies.  For every root of fgts[0], on the device in double:
 *   d_br_a[k]: Alex's value when he best-responds to Bob's sigma_bar,
 *   d_br_b[k]: Alex's value when Bob best-responds to Alex's sigma_bar,
 *   d_v[k]:    Alex's value when both play sigma_bar.
 * Each round's leaf value is its round points plus the later round's value
 * of the same kind at the linked root (last round: as pasur_leaf_utilities
 * with `leaf_flags`).  Any output may be NULL (not
 * computed), not all three.  Exploitability in points per game is
 * (br_a - br_b) / 2 >= 0.  Asynchronous on `stream`; uses stream-ordered
 * scratch (a level of each round, its leaves and its roots, in double).
 * PASUR_E_INVAL for null or inconsistent trees, PASUR_E_RANGE for n_rounds
 * outside 1..6 or an unknown dtype. */
int pasur_exploitability(const pasur_fgt *const *fgts, int n_rounds, void *const *sigma_bar,
                         int dtype, int leaf_flags, double *d_br_a, double *d_br_b,
                         double *d_v, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and arguments as pasur_tree_values, with its two level
 * buffers in a fixed device array instead of stream-ordered allocations.
 * Allocates nothing.  Limit: every level 0..7 of the tree at most 2^21
 * (2,097,152) nodes -- larger trees get PASUR_E_CAPACITY (use
 * pasur_tree_values).  Each GPU holds one 32 MiB array for the process's
 * lifetime, shared by every call on that GPU: calls that overlap on one GPU
 * (on any streams) race and must be serialised by the caller. */
int pasur_tree_values_noalloc(const pasur_fgt *fgt, const double *d_leaf, int dtype,
                              void *const sigma[9], int mode, double *d_out, void *stream);

/* ---- f2: self-play (section "Experimental Evaluation") ---------------------
 * n_games independent games on one solved subgame, one GPU thread each, from
 * root `root` of the first round: at each decision the player to move (Alex
 * at even levels) samples one child, by inverse CDF of the average strategy
 * (sigma_bar[r*9 + l], levels 1..8 of round slot r, dtype as the solver
 * state) or uniformly; at a round's last level the game adds the leaf's
 * round points (PASUR_FGT_LEAF_BASE) and continues at the linked next-round
 * root.  d_margin[g] = Alex's points minus Bob's over the rounds played; the
 * fair value is the fraction of games with margin > 0.  Draw i = g*64 +
 * round_slot*8 + level of a counter-based SplitMix64 stream (the published
 * finaliser of seed + (i+1)*0x9E3779B97F4A7C15) gives u = (z >> 11) / 2^53;
 * the sampled child is the first whose running FP64 sum of sigma_bar exceeds
 * u * total (uniform: floor(u * k)); forced moves draw nothing.  fgts are
 * consecutive rounds ending at the subgame's last round.  n_games above
 * 256 * (2^31 - 1), one launch, is PASUR_E_RANGE. */
enum { PASUR_PLAY_SIGMA_BAR = 0, PASUR_PLAY_UNIFORM = 1 };
int pasur_selfplay(const pasur_fgt *const *fgts, int n_rounds, const void *const *sigma_bar,
                   int dtype, int root, int64_t n_games, uint64_t seed, int policy_a,
                   int policy_b, int32_t *d_margin, void *stream);

/* ---- f3: external-sampling CFR (section "External Sampling") ---------------
 * n_iters iterations of external-sampling CFR on one round (the state as
 * pasur_cfr_init leaves it, u[8] = leaf utilities), continuing after t0
 * iterations.  An iteration is a pass for Alex, then one for Bob.  In p's
 * pass the opponent keeps one action per reached node, drawn from its
 * current strategy (CodeSnippet ExternalSampling: one multinomial draw per
 * node), and adds that strategy to the average sums Sbar of its children;
 * p keeps every action.  From the last level up, a reached node of p takes
 * u = sum of sigma * u over its children, adds u(child) - u to each child's
 * regret R (u - u(child) for Bob; values are Alex minus Bob) and
 * regret-matches its children's sigma with `rm_mode` / `eps` as in
 * pasur_cfr_params; a reached opponent node takes its kept child's value.
 * Sums are plain (sampling weights cancel); no discounting.  The draw of
 * the node h of level l in p's pass (p = 0 Alex, 1 Bob) of iteration t
 * (1-based) is index (2(t-1) + p) * N + off[l] + h of the counter-based
 * SplitMix64 stream of `seed` (as pasur_selfplay), N = n[0] + ... + n[7],
 * off[l] = n[0] + ... + n[l-1]; the kept child is the first whose running
 * FP64 sum of sigma exceeds u * total, and a node with one child draws
 * nothing.  Values u of unreached nodes are left as they were.  The average
 * strategy is pasur_average_strategy's normalisation of Sbar.
 * Schedules (bit-identical results): PASUR_ES_FRONTIER, one persistent
 * launch for all iterations, each workgroup running a run of consecutive
 * roots and visiting only the reached nodes (per-level frontier lists);
 * PASUR_ES_LEVEL, two launches per level and pass over every node.
 * roots_per_wg: consecutive roots per workgroup of the frontier schedule
 * (0 = about 4096 tree nodes per workgroup, at least one root).
 * `workspace` (device, caller-owned, 32-byte aligned): the frontier
 * schedule packs each node's sigma, R, Sbar and u into one record there for
 * the call (levels 0..8) and keeps two int32 per node of levels 0..7
 * (frontier lists and their choices); the level schedule uses one int32 per
 * node.  pasur_es_workspace_bytes(fgt, dtype) bytes (negative on error).
 * Calls on one workspace must not overlap.
 * d_stats (device, 4 uint64, or NULL; frontier schedule only) gains the
 * work done: reached nodes of the updated player, their children, reached
 * opponent nodes, their children (over all passes).
 * Asynchronous on `stream`. */
enum { PASUR_ES_FRONTIER = 0, PASUR_ES_LEVEL = 1 };
int64_t pasur_es_workspace_bytes(const pasur_fgt *fgt, int dtype);
int pasur_es_iterate(const pasur_fgt *fgt, const pasur_cfr_state *st, int64_t t0,
                     int64_t n_iters, uint64_t seed, int rm_mode, double eps, int schedule,
                     int roots_per_wg, void *workspace, int64_t workspace_bytes,
                     uint64_t *d_stats, void *stream);

/* ---- f4: infoset rows (sections "Compressed Game Tensor", "Infoset Tensors")
 * One row per FGT node of `level` (1..8): the nodes d_edges[i] (device) or,
 * with d_edges NULL, all n = n[level] nodes in order.  `gt` must be the game
 * tree `fgt` was unfolded from.  Row (58 int8): columns 0..51 per card (index
 * as everywhere in this library) the compressed code of the node's game
 * tensor for cards in play this round (held, or in the pool when the round
 * began): Alex's history minus Bob's, where in turn i (1-based) the mover's
 * history gains i at the card he plays and 10 i at each pool card he
 * collects; a difference of 0 becomes 100 / 105 / 110 for a card in Alex's
 * hand / Bob's hand / the pool, and a card out of play with 0 < |d| < 5
 * (laid and collecting in one turn) becomes 110 + d; cards dealt earlier and
 * out of play are -127, cards not yet dealt 0.  Columns 52..54: inherited
 * score as Alex clubs (7 if Alex owns the 7-clubs bonus), Bob clubs (7 if
 * Bob owns it), point difference; 55..57: round, turn (0..3) and player
 * (0 Alex, 1 Bob) of the action leading to the node.
 * format PASUR_INFOSET_INT8: d_out int8 [n][58]; PASUR_INFOSET_MLP: d_out
 * BF16 [n][192], the warm-start network's input, with row / 128 in columns
 * 0..57 and zeros after.  n above 256 * (2^31 - 1), one launch, is
 * PASUR_E_RANGE.  Asynchronous on `stream`. */
enum { PASUR_INFOSET_INT8 = 0, PASUR_INFOSET_MLP = 1 };
int pasur_infoset_rows(const pasur_gt *gt, const pasur_fgt *fgt, int level,
                       const int32_t *d_edges, int64_t n, int format, void *d_out,
                       void *stream);

/* ---- a13: learned warm start ------------------------------------------------
 * Not in the paper (its learned model is an XGBoost regressor on infoset
 * rows).  A 192-256-256-2 MLP: input = the child node's card state (Alex's
 * hand, Bob's hand, pool as 3 x 52 bits), inherited score (ca/7, cb/7, d/16,
 * +1/-1/0 bonus owner), the round's running score so far (clubs /13, last
 * picker, points /10, Surs of each side), a one-hot of the level and zero
 * padding (layout in pasur_edge_features); two ReLU hidden layers of 256; outputs a
 * policy logit (softmax over siblings = predicted average strategy) and a
 * node value.  Weights are row-major [in][out]; BF16 arrays are raw 16-bit
 * words.  All GEMMs run on MFMA (BF16 x BF16 -> FP32). */
typedef struct {
  const uint16_t *W1; const float *b1; /* [192][256], [256] */
  const uint16_t *W2; const float *b2; /* [256][256], [256] */
  const uint16_t *W3; const float *b3; /* [256][2], [2] */
  /* Optional (may be NULL): W1 and W2 transposed to [256][192] and [256][256]
   * (pasur_mlp_transpose), used by pasur_mlp_infer and the fused
   * pasur_mlp_forward instead of transposing into scratch on every call. */
  const uint16_t *W1t, *W2t;
} pasur_mlp_weights;
typedef struct {
  float *dW1, *db1, *dW2, *db2, *dW3, *db3; /* FP32, same shapes */
} pasur_mlp_grads;

/* C[M,N] = op(A) op(B) (+ bias per column, ReLU) with op(A)(m,k) =
 * A[m*sar + k*sac], op(B)(k,n) = B[k*sbr + n*sbc]; BF16 operands, FP32
 * accumulation; writes Cf (FP32) and/or Cb (BF16) with row stride ldc. */
int pasur_gemm_bf16(int M, int N, int K, const uint16_t *A, int64_t sar, int64_t sac,
                    const uint16_t *B, int64_t sbr, int64_t sbc, float *Cf, uint16_t *Cb,
                    int64_t ldc, const float *bias, int relu, void *stream);
/* Forward for M rows of X [M][192] (BF16): H1, H2 [M][256] (BF16, after
 * ReLU), Y [M][2] (FP32: logit, value).  With X, H1 and H2 16-byte aligned
 * all three layers run in the fused kernel of pasur_mlp_infer, which also
 * writes H1 and H2 (uses stream-ordered scratch for the transposed weights
 * unless w carries them); otherwise two GEMMs and the output layer (same
 * arithmetic, FP32 accumulation in another order). */
int pasur_mlp_forward(const pasur_mlp_weights *w, const uint16_t *X, int64_t M,
                      uint16_t *H1, uint16_t *H2, float *Y, void *stream);
/* Inference only: Y [M][2] (FP32) for M rows of X [M][192] (BF16), the same
 * arithmetic as pasur_mlp_forward (H1, H2 rounded to BF16; FP32 accumulation
 * in another order) in one fused launch that keeps H1 and H2 on chip.  Uses
 * stream-ordered scratch for the transposed weights (~220 KB) unless w
 * carries them. */
int pasur_mlp_infer(const pasur_mlp_weights *w, const uint16_t *X, int64_t M, float *Y,
                    void *stream);
/* W1t = W1^T [256][192], W2t = W2^T [256][256] (BF16, caller-owned). */
int pasur_mlp_transpose(const pasur_mlp_weights *w, uint16_t *W1t, uint16_t *W2t, void *stream);
/* Gradients of the loss with respect to the weights given dY [M][2] (FP32);
 * dY is rounded to BF16 for its products (db3 sums it in FP32).  H1 and H2 must be 8-byte aligned
 * (PASUR_E_INVAL otherwise).  The weight gradients reduce over the M rows in
 * FP32 partials of row chunks, summed in chunk order (deterministic).  Its
 * scratch (the two hidden gradients, BF16 [M][256] each, and up to 256
 * partial 256x256 FP32 gradients: about 0.33 GB for M = 2^18) is kept per
 * (device, stream) between calls: allocated stream-ordered when a call needs
 * more than it holds, held until the process ends.  Calls on one stream
 * from several host threads at once race on it. */
int pasur_mlp_backward(const pasur_mlp_weights *w, const uint16_t *X, const uint16_t *H1,
                       const uint16_t *H2, const float *dY, int64_t M, pasur_mlp_grads *g,
                       void *stream);
/* Rows seg[p]..seg[p+1] are the children of sampled parent p.  Policy loss:
 * cross-entropy of softmax(logits over siblings) against target_sigma,
 * averaged over parents; value loss: value_weight/2 (value - target)^2
 * averaged over rows.  Writes dY [n_rows][2] and loss [n_parents][2]. */
int pasur_mlp_loss(const float *Y, const float *target_sigma, const float *target_value,
                   const int32_t *seg, int64_t n_parents, int64_t n_rows, float value_weight,
                   float *dY, float *loss, void *stream);
/* Plain SGD on an FP32 master array, w <- w - lr g; refreshes its BF16 copy
 * when w_bf16 != NULL. */
int pasur_sgd_step(float *w, const float *g, uint16_t *w_bf16, int64_t n, float lr, void *stream);
/* Adam on an FP32 master array; refreshes its BF16 copy when w_bf16 != NULL. */
int pasur_adam_step(float *w, const float *g, float *m, float *v, uint16_t *w_bf16, int64_t n,
                    float lr, float beta1, float beta2, float eps, int64_t step, void *stream);
/* Adam over 1..8 FP32 master arrays in one launch, the same arithmetic per
 * element as pasur_adam_step: array t has n[t] elements at w[t], g[t], m[t],
 * v[t] and a BF16 copy at w_bf16[t] (w_bf16 or an entry NULL: none).  The
 * pointer arrays are host memory, the arrays they name device memory. */
int pasur_adam_step_multi(int count, float *const w[], const float *const g[], float *const m[],
                          float *const v[], uint16_t *const w_bf16[], const int64_t n[],
                          float lr, float beta1, float beta2, float eps, int64_t step,
                          void *stream);
/* Feature rows (BF16 [n][192]) of FGT nodes of `level`: the nodes d_edges[i]
 * (device) or, with d_edges NULL, all n = n[level] nodes in order.  `gt` must
 * be the game tree `fgt` was unfolded from.  Columns: 0..51 Alex's hand,
 * 52..103 Bob's hand, 104..155 pool (card bits); 156..159 ca/7, cb/7, d/16,
 * bonus owner +1/-1/0; 160..166 the GT node's running score: Acl/13, Bcl/13,
 * last picker +1 (Alex) / -1 (Bob) / 0, Apt/10, Asr, Bpt/10, Bsr; 167+level = 1;
 * other columns 0. */
int pasur_edge_features(const pasur_gt *gt, const pasur_fgt *fgt, int level,
                        const int32_t *d_edges, int64_t n, uint16_t *d_X, void *stream);
/* Training sample: decision parents (two or more children) on level-1 kept
 * when a seeded hash falls below keep_prob; d_seg (n[level-1]+1 capacity)
 * receives the offsets of their children in d_edges (n[level] capacity),
 * which receives the child indices.  Synchronises `stream`. */
int pasur_sample_parents(const pasur_fgt *fgt, int level, uint64_t seed, double keep_prob,
                         int32_t *d_seg, int32_t *d_edges, int64_t *n_parents,
                         int64_t *n_edges, void *stream);
/* Warm start of one level from predicted logits Y [n[level]][2]: sigma =
 * softmax over each node's children, R = kappa_r sigma, Sbar = kappa_s sigma.
 * Call after pasur_cfr_init; iterate from a later t0 so that the DCFR
 * discounts treat the warm start as earlier iterations. */
int pasur_cfr_warm_init(const pasur_fgt *fgt, const pasur_cfr_state *st, int level,
                        const float *Y, float kappa_r, float kappa_s, void *stream);
/* The warm start of a whole round in one call (after pasur_cfr_init): the
 * feature rows of every node of levels 1..max_level (one launch), the MLP
 * forward pass over all of them, and sigma / R / Sbar of those levels as in
 * pasur_cfr_warm_init (one launch); deeper levels keep their initial state.
 * `gt` must be the game tree `fgt` was unfolded from.  Uses stream-ordered
 * the caller's workspace when it is large enough, else stream-ordered scratch
 * (rows x 192 BF16 + rows x 2 FP32); the forward pass is pasur_mlp_infer. */
int pasur_warm_start_round(const pasur_gt *gt, const pasur_fgt *fgt, const pasur_cfr_state *st,
                           const pasur_mlp_weights *w, int max_level, float kappa_r,
                           float kappa_s, void *workspace, int64_t workspace_bytes,
                           void *stream);
/* Bytes of device workspace pasur_warm_start_round needs for max_level (a
 * smaller or NULL workspace makes it allocate stream-ordered scratch). */
int64_t pasur_warm_start_workspace_bytes(const pasur_fgt *fgt, int max_level);

/* Training-data helpers: dst[i] = (float)src[idx[i]] (idx NULL: src[i]) for
 * a `dtype` array; dst[i] = src[i] + add for int32 offsets. */
int pasur_gather_f32(const void *src, int dtype, const int32_t *idx, int64_t n, float *dst,
                     void *stream);
int pasur_shift_i32(const int32_t *src, int64_t n, int32_t add, int32_t *dst, void *stream);

/* ---- tracing ----------------------------------------------------------------
 * Per-launch timing of the sweep kernels with HIP events recorded on the
 * launch stream around every launch made by pasur_cfr_iterate.  Enabling
 * (or disabling) clears earlier records and selects every kernel;
 * pasur_profile_select restricts recording to the kernel ids whose bit is
 * set in kernel_mask.  pasur_profile_read waits for the events and copies up
 * to `cap` records into host arrays, with the work of each launch in `work`
 * (5 int64 per record); any output array may be NULL.  *n_out gets the
 * number recorded.  Kernel ids, level and work:
 *   0 reach down-sweep, 1 fused up-sweep (level-synchronous; level = child
 *     level; work = edges, internal nodes);
 *   2 / 3 persistent segment kernel, every subtree in LDS / some in global
 *     memory (level -1; work = edges, internal nodes, roots, level-7 nodes,
 *     iterations);
 *   streaming schedule (level = child level; work = nodes or children,
 *   parents, boundary-list entries): 4 tile down-sweep, 5 tile up-sweep,
 *   6 up-sweep one thread per parent, 7 up-sweep over a parent list, 8 set-up
 *   and tear-down of a call, 9 / 10 down / up sweeps of the compact tail,
 *   11 / 12 tile up / down sweeps at the tail's boundary, 13 down-sweep over
 *   a node list, 14 down-sweep one thread per parent.
 * Not thread-safe against concurrent iterate calls. */
int pasur_profile_enable(int on);
int pasur_profile_select(uint64_t kernel_mask);
int pasur_profile_read(int64_t cap, int32_t *kernel, int32_t *level, float *ms,
                       int64_t *work, int64_t *n_out);

#ifdef __cplusplus
}
#endif
#endif
