"""Pins of the infoset-row reference (oracle/infoset.py).

- Every value of the paper's compressed-code table (tests/golden/
  tcmp_values.txt) comes out of the game-tensor history rule and the
  compression steps for a card with that history.
- On real rounds: the card states replayed from each node's actions agree
  with the node's own pool and hands; every code is a table value or one of
  the values the table omits (+-10 j, -36); each row has exactly as many
  cards with a lay leg as actions were taken; held and pool cards carry
  their no-leg codes; the score slots decode to the node's inherited score;
  dealt cards out of play are -127 and undealt cards 0.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import infoset as inf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tcmp_values.txt")
ALEX, BOB, POOL = [0, 1, 2, 3], [4, 5, 6, 7], [8, 9, 10, 11]


def table():
    out = []
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if line:
            out.append((int(line[0]), line[1:]))
    return out


def history(desc):
    """Game tensor of a toy round in which card X has the history `desc`
    and every other action lays a spare card of its mover."""
    kind = desc[0]
    spare = {0: [c for c in ALEX], 1: [c for c in BOB]}
    events = {}
    if kind == "hand":
        x = spare[0 if desc[1] == "A" else 1].pop(0)
        last = 6
    elif kind == "pool":
        x = POOL[0]
        last = 8
    else:
        p = 0 if desc[1] == "A" else 1
        x = spare[p].pop(0)
        lvl = 2 * int(desc[2]) + p + 1
        if kind == "same":
            events[lvl] = (x, 1 << POOL[1])
            last = lvl
        else:
            events[lvl] = (x, 0)
            last = lvl
            if len(desc) > 3:
                q = 0 if desc[4] == "A" else 1
                lq = 2 * int(desc[5]) + q + 1
                events[lq] = (spare[q].pop(0), 1 << x)
                last = lq
    acts = []
    for lvl in range(1, last + 1):
        if lvl in events:
            acts.append(events[lvl])
        else:
            acts.append((spare[(lvl - 1) % 2].pop(0), 0))
    return x, inf.game_tensor(ALEX, BOB, sum(1 << c for c in POOL), acts)


@pytest.mark.parametrize("code,desc", table())
def test_table_values(code, desc):
    x, g = history(desc)
    assert inf.compress(g)[x] == code, (desc, g[:, x])


def test_table_is_complete_up_to_the_omissions():
    """Every legal one-card history lands on a table value, except the
    omitted ones the rule still defines."""
    codes = {c for c, _ in table()}
    seen = set()
    for p in (0, 1):
        for i in range(4):
            for q in (0, 1):
                for j in range(4):
                    if 2 * j + q > 2 * i + p:  # collected after it was laid
                        x, g = history(["lay", "AB"[p], str(i), "pick", "AB"[q], str(j)])
                        seen.add(int(inf.compress(g)[x]))
    assert seen - codes == {-36}


ALLOWED = {c for c, _ in table()} | {-36} | {s * 10 * j for s in (1, -1) for j in (1, 2, 3, 4)}
NO_LAY = {100, 105, 110} | {s * 10 * j for s in (1, -1) for j in (1, 2, 3, 4)}


@pytest.mark.parametrize("seed,rnd", [(4, 5), (2, 4), (7, 0)])
def test_rows_on_real_rounds(seed, rnd):
    if rnd == 5:
        deck, roots = synth.last_round_roots(seed)
    else:
        deck, roots = synth.subgame_roots(seed, rnd)
    gt = oracle.GT(deck, rnd, sorted({x.pool for x in roots}))
    f = oracle.FGT(gt, roots)
    alex, bob = inf.round_cards(deck, rnd)
    dealt = set(int(c) for c in deck[: 12 + 8 * rnd])
    tab = f.get(oracle.FGT_SCORE_TAB)
    for level in range(1, 9):
        R = inf.rows(gt, f, level).astype(np.int64)
        g_of = f.get(oracle.FGT_GT, level)
        sid = f.get(oracle.FGT_SID, level)
        pool = gt.get(oracle.GT_POOL, level)[g_of]
        hands = gt.get(oracle.GT_HANDS, level)[g_of]
        step = max(1, len(R) // 300)
        for q in range(0, len(R), step):
            row = R[q]
            codes = row[:52]
            held_a = {alex[i] for i in range(4) if (hands[q] >> i) & 1}
            held_b = {bob[i] for i in range(4) if (hands[q] >> (4 + i)) & 1}
            in_pool = set(inf.bits(pool[q]))
            for c in range(52):
                v = codes[c]
                if c in held_a:
                    assert v == 100
                elif c in held_b:
                    assert v == 105
                elif c in in_pool:
                    assert v == 110 or 1 <= abs(v) <= 4
                elif v not in (0, -127):
                    assert v in ALLOWED and not (1 <= abs(v) <= 4) and v not in (100, 105, 110)
                if c not in dealt:
                    assert v == 0
                elif v == 0:
                    raise AssertionError(f"dealt card {c} coded 0")
            assert all(v in ALLOWED for v in codes if v not in (0, -127))
            lays = sum(1 for v in codes if v in ALLOWED and v not in NO_LAY)
            assert lays == level
            ca, cb, d, bonus = (int(x) for x in tab[int(sid[q])])
            assert tuple(row[52:55]) == inf.score_slots(ca, cb, d, bonus)
            assert tuple(row[55:58]) == (rnd, (level - 1) // 2, (level - 1) % 2)


def test_replayed_states_match_the_tree():
    deck, roots = synth.last_round_roots(5)
    gt = oracle.GT(deck, 5, sorted({x.pool for x in roots}))
    alex, bob = inf.round_cards(deck, 5)
    card = [None] + [gt.get(oracle.GT_ACT_CARD, k) for k in range(1, 9)]
    cap = [None] + [gt.get(oracle.GT_ACT_CAP, k) for k in range(1, 9)]
    par = [None] + [gt.get(oracle.GT_PARENT, k) for k in range(1, 9)]
    for level in range(1, 9):
        pool = gt.get(oracle.GT_POOL, level)
        hands = gt.get(oracle.GT_HANDS, level)
        for g0 in range(0, gt.n[level], max(1, gt.n[level] // 200)):
            g, acts = g0, []
            for k in range(level, 0, -1):
                acts.append((int(card[k][g]), int(cap[k][g])))
                g = int(par[k][g])
            acts.reverse()
            t = inf.game_tensor(alex, bob, int(gt.get(oracle.GT_POOL, 0)[g]), acts)
            want = np.zeros(52, np.int64)
            for i in range(4):
                if (hands[g0] >> i) & 1:
                    want[alex[i]] = 1
                if (hands[g0] >> (4 + i)) & 1:
                    want[bob[i]] = 2
            for c in inf.bits(pool[g0]):
                want[c] = 3
            assert np.array_equal(t[0], want), (level, g0)


def test_score_slots_are_lossless():
    seen = {}
    for ca in range(7):
        for cb in range(7):
            for d in range(-20, 21):
                seen[inf.score_slots(ca, cb, d, 0)] = (ca, cb, d, 0)
    for d in range(-20, 21):
        seen[inf.score_slots(0, 0, d, 1)] = (0, 0, d, 1)
        seen[inf.score_slots(0, 0, d, 2)] = (0, 0, d, 2)
    assert len(seen) == 7 * 7 * 41 + 2 * 41
