"""Pins of the FP64 oracle's rules, tree construction and unfolding.

Each test checks the oracle against something other than itself: values the
paper prints (subset-sum count, worked game traces, first-turn equilibrium
table, score normalisation and unfolding examples), independent brute force,
or closed-form combinatorics.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import card_index, cards_of, read_rows


def test_subset_sum_table_count():
    # Section "Numerical Actions": 2764 numeric subsets sum to 11.
    n, by = oracle.subset11_count()
    assert n == 2764
    # Independent count: choose how many cards of each value 1..10 (each value
    # has 4 suits), weight by binomial(4, k).
    want = {}
    for ks in itertools.product(range(5), repeat=10):
        if sum((v + 1) * k for v, k in enumerate(ks)) != 11:
            continue
        size = sum(ks)
        want[size] = want.get(size, 0) + math.prod(math.comb(4, k) for k in ks)
    assert sum(want.values()) == 2764
    for size in range(16):
        assert by[size] == want.get(size, 0)


def _moves(hand, pool, rnd=0, ply=0):
    hA = synth.mask_of(hand)
    ch = oracle.children(rnd, ply, synth.mask_of(pool), hA, 0)
    return [(c[0], c[1]) for c in ch]


@pytest.mark.parametrize("base", [44, 48])
def test_queen_king_all_81_patterns(base):
    # Section "King Actions": 3**4 = 81 hand/pool patterns of the four Kings
    # (or Queens).  Capture table: a single card of the same rank.
    seen = 0
    for pattern in itertools.product(range(3), repeat=4):  # 0 out, 1 hand, 2 pool
        hand = [base + i for i in range(4) if pattern[i] == 1]
        pool = [base + i for i in range(4) if pattern[i] == 2]
        seen += 1
        got = _moves(hand, pool)
        want = []
        for c in sorted(hand):
            if pool:
                want += [(c, 1 << x) for x in sorted(pool)]
            else:
                want.append((c, 0))
        assert got == want, (pattern, got, want)
    assert seen == 81


def test_jack_rules_from_traces():
    # Fig. game_0 stage 1_0_1: Jack onto a pool holding only a Queen is a lay.
    assert _moves([card_index("JD")], [card_index("QC")]) == [(card_index("JD"), 0)]
    # Stage 3_1_0: Jack takes every pool card except Queens and Kings, Jacks included.
    pool = cards_of("6C,6D,6S,7C,8C,8D,8S,9H,JD,QC")
    got = _moves([card_index("JS")], pool)
    assert got == [(card_index("JS"), synth.mask_of(cards_of("6C,6D,6S,7C,8C,8D,8S,9H,JD")))]


def test_must_capture_is_per_card():
    # Fig. game_9 stage 5_0_0 lays the 10 of clubs while the Ace and the Queen
    # in hand could capture: a non-capturing card may still be laid.
    hand = cards_of("AH,3S,10C,QD")
    pool = cards_of("4S,5H,10S,JH,QH")
    got = _moves(hand, pool)
    assert (card_index("10C"), 0) in got
    assert (card_index("AH"), 1 << card_index("10S")) in got
    assert (card_index("QD"), 1 << card_index("QH")) in got
    assert all(cap != 0 for c, cap in got if c in (card_index("AH"), card_index("QD")))


def test_score_normalisation_example():
    # Section "Score Tensors": [3, 8, 2, 0] is normalised to [0, 0, 2, 2].
    out = oracle.combine_score([3, 8, 2, 0], np.zeros(8, np.int8))
    assert list(out) == [0, 0, 2, 2]


def _replay(path, deck):
    """Replay a printed game: every (lay, pick) must be a generated move and
    the running columns must match the printed ones."""
    rows = read_rows(path)
    has_cl = len(rows[0]) == 15
    s = np.zeros(4, np.int8)  # ca, cb, d, bonus
    rs = np.zeros(8, np.int8)
    pool = synth.mask_of(deck[:4])
    clean = [r for r in rows if r[0] == "CleanUp"][0]
    for row in rows:
        stage = row[0]
        if stage == "CleanUp":
            continue
        rnd, turn, who = (int(x) for x in stage.split("_"))
        ply = 2 * turn + who
        if ply == 0:
            if rnd > 0:
                s = oracle.combine_score(s, rs)
            rs = np.zeros(8, np.int8)
            a, b = synth.round_hands(deck, rnd)
            handA, handB = synth.mask_of(a), synth.mask_of(b)
        assert handA == synth.mask_of(cards_of(row[1])), stage
        assert handB == synth.mask_of(cards_of(row[2])), stage
        assert pool == synth.mask_of(cards_of(row[3])), stage
        lay = card_index(row[4])
        pick = synth.mask_of(cards_of(row[5]))
        kids = oracle.children(rnd, ply, pool, handA, handB, rs)
        match = [k for k in kids if k[0] == lay and k[1] == pick]
        assert len(match) == 1, (stage, row[4], row[5])
        _, _, pool, handA, handB, rs = match[0]
        # the final-round clean-up is folded into the last ply
        ref = clean if (rnd == 5 and ply == 7) else row
        acl, bcl, apt, bpt, asr, bsr, d = (int(x) for x in ref[6:13])
        L = {"0": 0, "A": 1, "B": 2}[ref[13]]
        assert int(s[0]) + int(rs[0]) == acl, stage
        assert int(s[1]) + int(rs[1]) == bcl, stage
        assert (int(rs[3]), int(rs[5]), int(rs[4]), int(rs[6])) == (apt, bpt, asr, bsr), stage
        assert int(rs[2]) == L, stage
        if ref is row:
            assert int(s[2]) == d, stage
        if has_cl and row[14] != "-":
            assert int(s[3]) == {"A": 1, "B": 2}[row[14]], stage
    final = oracle.combine_score(s, rs)
    bonus = {0: 0, 1: 7, 2: -7}[int(final[3])]
    return int(final[2]) + bonus


def test_replay_game0(golden_dir):
    # Caption of fig. game_0: Alex ends 8 points ahead.  (Its CleanUp row
    # prints a point difference of 2 where the caption's sum gives 3: the
    # difference column is not checked on that row.)
    final = _replay(os.path.join(golden_dir, "game0_trace.txt"), synth.DECK9)
    assert final == 8


def test_replay_game9(golden_dir):
    final = _replay(os.path.join(golden_dir, "game9_trace.txt"), synth.DECK9)
    assert final == 14


def test_unfolding_edge_example():
    # Figure "Unfolding Process": GT parents 0 and 1 with 2 and 3 children and
    # 3 and 2 inherited scores (green, red, blue | orange, blue); the paper's
    # edge tensor is [0,1,2,0,1,2,3,4,3,4,3,4] over FGT roots
    # [(0,g),(0,r),(0,b),(1,o),(1,b)] and children ordered GT-node-major.
    # Scores: g=0, r=1, b=2, o=3.  Pad the 1-level GT to 8 levels with forced
    # single-child chains so that it has the shape of a round.
    gt_n = [2, 5] + [5] * 7
    cb = [np.array([0, 2, 5], np.int32)] + [np.arange(6, dtype=np.int32)] * 7
    root_gt = [0, 0, 0, 1, 1]
    root_sid = [0, 1, 2, 3, 2]
    f = oracle.FGT(None, csr=(gt_n, cb, root_gt, root_sid))
    paper_roots = list(zip(root_gt, root_sid))
    paper_children = [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2),
                      (2, 3), (2, 2), (3, 3), (3, 2), (4, 3), (4, 2)]
    paper_edg = [0, 1, 2, 0, 1, 2, 3, 4, 3, 4, 3, 4]
    want = {(c, paper_roots[p]) for c, p in zip(paper_children, paper_edg)}
    g1, s1, p1 = f.get(oracle.FGT_GT, 1), f.get(oracle.FGT_SID, 1), f.get(oracle.FGT_PARENT, 1)
    g0, s0 = f.get(oracle.FGT_GT, 0), f.get(oracle.FGT_SID, 0)
    got = {((int(g1[i]), int(s1[i])), (int(g0[p1[i]]), int(s0[p1[i]]))) for i in range(f.n[1])}
    assert len(got) == f.n[1] == 12
    assert got == want
    # parent-major canonical order: children of each FGT root are contiguous
    assert list(p1) == sorted(p1)


# --- independent brute-force round enumerator (P6) ------------------------

VAL = {c: c // 4 + 1 for c in range(40)}
POINTS = {0: 1, 1: 1, 2: 1, 3: 1, 4: 2, 37: 3, 40: 1, 41: 1, 42: 1, 43: 1}


def _bf_moves(hand, pool):
    out = []
    for c in sorted(hand):
        caps = []
        if c < 40:
            nums = sorted(x for x in pool if x < 40)
            for k in range(1, len(nums) + 1):
                for sub in itertools.combinations(nums, k):
                    if VAL[c] + sum(VAL[x] for x in sub) == 11:
                        caps.append(sum(1 << x for x in sub))
        elif c < 44:
            m = sum(1 << x for x in pool if x < 44)
            if m:
                caps.append(m)
        else:
            caps = [1 << x for x in sorted(pool) if x // 4 == c // 4]
        if caps:
            out += [(c, m) for m in sorted(caps)]
        else:
            out.append((c, 0))
    return out


def _bf_round(deck, rnd, pool_mask):
    """Depth-first enumeration of one round: per-level counts and the leaf
    multiset of (pool, running score)."""
    a, b = synth.round_hands(deck, rnd)
    counts = [0] * 9
    leaves = []

    def rec(ply, pool, hands, rs):
        counts[ply] += 1
        if ply == 8:
            leaves.append((pool, tuple(rs)))
            return
        who = ply % 2
        for c, cap in _bf_moves(hands[who], [x for x in range(52) if pool >> x & 1]):
            p = pool
            h = [set(hands[0]), set(hands[1])]
            h[who].discard(c)
            r = list(rs)
            if cap == 0:
                p |= 1 << c
            else:
                taken = [x for x in range(52) if (cap | 1 << c) >> x & 1]
                r[who] += sum(1 for x in taken if x % 4 == 0)
                r[3 + 2 * who] += sum(POINTS.get(x, 0) for x in taken)
                r[2] = who + 1
                if cap == p and not 40 <= c < 44 and rnd != 5:
                    r[4 + 2 * who] += 1
                p &= ~cap
            if rnd == 5 and ply == 7 and r[2]:
                left = [x for x in range(52) if p >> x & 1]
                w = r[2] - 1
                r[w] += sum(1 for x in left if x % 4 == 0)
                r[3 + 2 * w] += sum(POINTS.get(x, 0) for x in left)
            rec(ply + 1, p, h, r)

    rec(0, pool_mask, [set(a), set(b)], [0] * 8)
    return counts, leaves


@pytest.mark.parametrize("seed,rnd", [(3, 5), (2, 5), (7, 4)])
def test_tree_matches_brute_force(seed, rnd):
    deck, pool, ca, cb, bonus, _ = synth.subgame_start(seed, rnd, pool_max=6)
    gt = oracle.GT(deck, rnd, [pool])
    counts, leaves = _bf_round(deck, rnd, pool)
    assert list(gt.n) == counts
    lp = gt.get(oracle.GT_POOL, 8)
    lrs = gt.get(oracle.GT_RS, 8)
    got = sorted((int(lp[i]), tuple(int(x) for x in lrs[i])) for i in range(gt.n[8]))
    assert got == sorted(leaves)
    # canonical order inside each parent: (card, capture mask) ascending
    for l in range(1, 9):
        par = gt.get(oracle.GT_PARENT, l)
        key = list(zip(par.tolist(), gt.get(oracle.GT_ACT_CARD, l).tolist(),
                       gt.get(oracle.GT_ACT_CAP, l).tolist()))
        assert key == sorted(key)


def test_between_rounds_roots_and_link():
    deck, roots = synth.two_round_root(1)
    gt = oracle.GT(deck, 4, [roots[0].pool])
    f = oracle.FGT(gt, roots)
    nxt = f.get(oracle.FGT_NEXT_ROOTS)
    link = f.get(oracle.FGT_LINK)
    keys = [(int(r["pool"]), int(r["bonus"]), int(r["ca"]), int(r["cb"]), int(r["d"])) for r in nxt]
    assert keys == sorted(set(keys))
    lg = f.get(oracle.FGT_GT, 8)
    lp = gt.get(oracle.GT_POOL, 8)
    lrs = gt.get(oracle.GT_RS, 8)
    r0 = roots[0]
    for i in range(f.n[8]):
        t = lg[i]
        ca, cb, d, bonus = (int(x) for x in oracle.combine_score([r0.ca, r0.cb, r0.d, r0.bonus], lrs[t]))
        assert keys[link[i]] == (int(lp[t]), bonus, ca, cb, d)
    assert set(link.tolist()) == set(range(len(keys)))


@pytest.mark.slow
def test_deck9_first_turn_support(golden_dir):
    # Table tab:deck9_exp: the near-Nash first-turn strategies of the worked
    # deck.  Both hands are visible, so an equilibrium only plays actions of
    # maximal minimax value; the full six-round minimax must single out the
    # same actions.  The sample game of fig. game_9 (played by those
    # strategies) ends at +14 for Alex, which must equal the game value.
    deck = synth.DECK9
    roots = [synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)]
    rounds = []
    for r in range(6):
        gt = oracle.GT(deck, r, sorted({x.pool for x in roots}))
        f = oracle.FGT(gt, roots)
        rounds.append((gt, f))
        if r < 5:
            roots = [synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]),
                                int(x["bonus"])) for x in f.get(oracle.FGT_NEXT_ROOTS)]
    V = None
    for r in range(5, -1, -1):
        gt, f = rounds[r]
        leaf = f.leaf_utilities(V)
        cb = f.child_begin()
        if r == 0:
            v1 = oracle.tree_values(f.n, cb, leaf, None, oracle.TV_MINIMAX, level=1)
            v2 = oracle.tree_values(f.n, cb, leaf, None, oracle.TV_MINIMAX, level=2)
        V = oracle.tree_values(f.n, cb, leaf, None, oracle.TV_MINIMAX)
        rounds[r] = (gt, f) if r == 0 else None
    assert V.tolist() == [14.0]
    gt, f = rounds[0]
    a1 = gt.get(oracle.GT_ACT_CARD, 1).tolist()
    a2 = gt.get(oracle.GT_ACT_CARD, 2).tolist()
    c2 = gt.get(oracle.GT_ACT_CAP, 2).tolist()
    cbg = gt.get(oracle.GT_CHILD_BEGIN, 1)
    rows = read_rows(os.path.join(golden_dir, "deck9_first_turn.txt"))
    alex = {card_index(r[1]): float(r[4]) for r in rows if r[0] == "A"}
    assert sorted(alex) == sorted(a1)  # exactly the legal first moves
    best = max(v1)
    for i, c in enumerate(a1):
        assert (v1[i] == best) == (alex[c] > 0), c
        replies = {(card_index(r[2]), synth.mask_of(cards_of(r[3]))): float(r[4])
                   for r in rows if r[0] == "B" and card_index(r[1]) == c}
        kids = list(range(cbg[i], cbg[i + 1]))
        assert sorted(replies) == sorted((a2[q], c2[q]) for q in kids)
        bob_best = min(v2[q] for q in kids)
        for q in kids:
            assert (v2[q] == bob_best) == (replies[(a2[q], c2[q])] > 0), (c, a2[q])


def test_literal_bonus0_flag():
    # Equation final_util as printed gives 7(2(bonus mod 2) - 1): -7 also for
    # bonus 0 (nobody reached 7 clubs).  A last round with no club among the
    # pool and the eight hand cards cannot award the bonus, so every leaf of
    # a root with no bonus yet ends at bonus 0: the printed form lowers its
    # utility by exactly 7; a root whose bonus Alex already holds keeps +7
    # either way.
    nonclubs = [c for c in range(52) if c % 4]
    clubs = [c for c in range(52) if c % 4 == 0]
    deck = nonclubs[:4] + clubs + nonclubs[4:]
    assert all(c % 4 for c in deck[44:])
    pool = synth.mask_of(deck[:4])
    roots = [synth.Root(pool, 0, 0, 0, 0), synth.Root(pool, 0, 0, 0, 1)]
    gt = oracle.GT(deck, 5, [pool])
    f = oracle.FGT(gt, roots)
    plain = f.leaf_utilities()
    literal = f.leaf_utilities(literal_bonus0=True)
    # the two roots' leaves: root k's subtree through the level ranges
    lo, hi = [0, 1], [1, 2]
    for cb in f.child_begin():
        lo = [int(cb[x]) for x in lo]
        hi = [int(cb[x]) for x in hi]
    assert hi[0] == lo[1] and hi[1] == f.n[8]
    np.testing.assert_array_equal(literal[:hi[0]] - plain[:hi[0]], -7.0)
    np.testing.assert_array_equal(literal[lo[1]:], plain[lo[1]:])
    # with the bonus held, every leaf is +7 plus the round's points, and the
    # same round points sit under the bonus-0 root
    np.testing.assert_array_equal(plain[lo[1]:] - 7.0, plain[:hi[0]])
