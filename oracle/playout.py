"""Seeded legal playouts (test infrastructure only; imported by tests and
bench.py's CPU leg, never by the HIP path).

The start state of round ``rnd`` of a deal, reached by playing rounds
0..rnd-1 from the initial deal (section "Pasur": four pool cards, four cards
to each player per round, Alex first): each move is the legal move number
``draws[i] mod k`` in the canonical order of the move generator, and each
round's end updates the inherited score as the unfolding does (equation
passuputil's running score combined with the root score: clubs, the 7-club
bonus, the point difference).  The pool carries over between rounds (the
clean-up happens only after round 6)."""
from __future__ import annotations

import numpy as np

import synth
from . import children, combine_score


def playout_root(deck, rnd: int, draws) -> synth.Root:
    """Root (pool, ca, cb, d, bonus) at the start of round ``rnd`` (0..5)."""
    pool = synth.mask_of(deck[:4])
    score = np.zeros(4, np.int8)
    i = 0
    for r in range(rnd):
        hand_a, hand_b = synth.round_hands(deck, r)
        ha, hb = synth.mask_of(hand_a), synth.mask_of(hand_b)
        rs = np.zeros(8, np.int8)
        for ply in range(8):
            kids = children(r, ply, pool, ha, hb, rs)
            card, cap, pool, ha, hb, rs = kids[int(draws[i]) % len(kids)]
            i += 1
        score = combine_score(score, rs)
    return synth.Root(int(pool), int(score[0]), int(score[1]), int(score[2]), int(score[3]))
