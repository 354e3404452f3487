"""Infoset rows of unfolded-tree nodes (test infrastructure only).

Plain definitions, in the paper's order:

1. Game tensor (section on the game tree, state-encoding table and the
   history rule, CodeSnippet ApplyActions): per card, a state (1 held by
   Alex, 2 held by Bob, 3 in the pool, 0 otherwise) and one history row per
   player.  In turn i (1-based) the mover adds i at the card he plays and
   10 i at every pool card he collects; a played card goes to the pool
   (state 3) if it collects nothing, otherwise it and the collected cards
   leave play (state 0).
2. Compressed game tensor (CodeSnippet Compressed Game Tensor and its two
   tables): cmp = Alex's row - Bob's row; a card out of play whose cmp is
   in -4..4 but not 0 (both legs in one turn) becomes 110 + cmp; a card
   with cmp 0 becomes 110 in the pool, 100 in Alex's hand, 105 in Bob's.
3. Infoset row (CodeSnippet Infoset Tensor, table of the row layout), 58
   int8: columns 0..51 the compressed code of each in-play card (held, or
   in the pool when the round began), -127 for a card dealt earlier in the
   game and no longer in play, 0 for a card not yet dealt; 52..54 the
   inherited score; 55..57 (round, turn, player) of the action leading to
   the node.

Readings where the paper is silent or inconsistent:
- Score columns: the score vector has four entries (Alex clubs, Bob clubs,
  point difference, 7-clubs bonus owner) but the row has three slots.
  Clubs are reset and no longer counted once a bonus is owned, so the three
  slots hold Alex clubs (7 if Alex owns the bonus), Bob clubs (7 if Bob
  owns it) and the difference: the four entries are recovered exactly.
- The value table omits pool cards collected later (cmp = +-10 j, which
  the same rule yields: +10 j when Alex collects at turn j, -10 j for Bob)
  and -36 (Alex's last card collected by Bob's last card); they follow from
  the rule as printed.
- Rows are those of levels 1..8 (each node is reached by one action);
  turn = (level - 1) // 2 and player = (level - 1) % 2 (0 Alex, 1 Bob) of
  that action.
Cards are indexed 0..51 as in the rest of the package (4 * rank + suit).
"""
from typing import List, Sequence, Tuple

import numpy as np

from . import (FGT_GT, FGT_SCORE_TAB, FGT_SID, GT_ACT_CAP, GT_ACT_CARD, GT_PARENT, GT_POOL)

N_ROW = 58


def bits(mask: int) -> List[int]:
    return [c for c in range(52) if (int(mask) >> c) & 1]


def round_cards(deck: Sequence[int], rnd: int) -> Tuple[List[int], List[int]]:
    """Alex's and Bob's dealt cards of round rnd: after the four-card initial
    pool, each round deals four to Alex, then four to Bob."""
    return [int(c) for c in deck[4 + 8 * rnd: 8 + 8 * rnd]], [int(c) for c in deck[8 + 8 * rnd: 12 + 8 * rnd]]


def game_tensor(alex: Sequence[int], bob: Sequence[int], root_pool: int,
                actions: Sequence[Tuple[int, int]]) -> np.ndarray:
    """t_gme [3, 52] after the actions (card, collected-card mask) of levels
    1..len(actions), the first by Alex."""
    g = np.zeros((3, 52), np.int64)
    for c in alex:
        g[0, c] = 1
    for c in bob:
        g[0, c] = 2
    for c in bits(root_pool):
        g[0, c] = 3
    for k, (card, cap) in enumerate(actions, start=1):
        mover = (k - 1) % 2
        turn = (k - 1) // 2 + 1
        g[1 + mover, card] += turn
        taken = bits(cap)
        for c in taken:
            g[1 + mover, c] += 10 * turn
        if taken:
            g[0, card] = 0
            for c in taken:
                g[0, c] = 0
        else:
            g[0, card] = 3
    return g


def compress(g: np.ndarray) -> np.ndarray:
    """t_cmp of one game-tensor slice, step by step as printed."""
    cmp = g[1] - g[2]
    lpm = (g[0] == 0) & (cmp != 0) & (np.abs(cmp) < 5)
    cmp[lpm] = 110 + cmp[lpm]
    cmp[(g[0] == 3) & (cmp == 0)] = 110
    cmp[(g[0] == 1) & (cmp == 0)] = 100
    cmp[(g[0] == 2) & (cmp == 0)] = 105
    return cmp


def score_slots(ca: int, cb: int, d: int, bonus: int) -> Tuple[int, int, int]:
    return (7 if bonus == 1 else ca, 7 if bonus == 2 else cb, d)


def infoset_row(deck: Sequence[int], rnd: int, root_pool: int,
                actions: Sequence[Tuple[int, int]], score: Sequence[int]) -> np.ndarray:
    alex, bob = round_cards(deck, rnd)
    cmp = compress(game_tensor(alex, bob, root_pool, actions))
    inp = np.zeros(52, bool)
    inp[alex + bob + bits(root_pool)] = True
    row = np.zeros(N_ROW, np.int64)
    row[:52][inp] = cmp[inp]
    row[52:55] = score_slots(*[int(x) for x in score])
    dealt = np.zeros(52, bool)
    dealt[[int(c) for c in deck[: 12 + 8 * rnd]]] = True
    cards = row[:52]
    cards[dealt & (cards == 0)] = -127
    level = len(actions)
    row[55:58] = (rnd, (level - 1) // 2, (level - 1) % 2)
    return row.astype(np.int8)


def rows(gt, fgt, level: int) -> np.ndarray:
    """Infoset rows [n, 58] of every FGT node of `level` (1..8), in order."""
    g_of = fgt.get(FGT_GT, level)
    sid = fgt.get(FGT_SID, level)
    tab = fgt.get(FGT_SCORE_TAB)
    card = [None] + [gt.get(GT_ACT_CARD, k) for k in range(1, 9)]
    cap = [None] + [gt.get(GT_ACT_CAP, k) for k in range(1, 9)]
    par = [None] + [gt.get(GT_PARENT, k) for k in range(1, 9)]
    pool0 = gt.get(GT_POOL, 0)
    out = np.zeros((len(g_of), N_ROW), np.int8)
    for q in range(len(g_of)):
        g = int(g_of[q])
        acts = []
        for k in range(level, 0, -1):
            acts.append((int(card[k][g]), int(cap[k][g])))
            g = int(par[k][g])
        acts.reverse()
        out[q] = infoset_row(gt.deck, gt.round, int(pool0[g]), acts, tab[int(sid[q])])
    return out
