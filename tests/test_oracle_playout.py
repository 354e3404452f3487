"""The oracle's seeded legal playout (oracle/playout.py), pinned against the
oracle's own unfolded trees and the game's club bookkeeping."""
import numpy as np
import pytest

import oracle
import synth
from oracle.playout import playout_root


def walk_trees(deck, rnd, draws):
    """The same playout through the oracle's level-major trees: from the
    round's root, child begin + (draw mod count) on every level, then the
    leaf's link into the next round's roots."""
    root = synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)
    i = 0
    for r in range(rnd):
        f = oracle.FGT(oracle.GT(deck, r, [root.pool]), [root])
        node = 0
        cb = f.child_begin()
        for l in range(8):
            b, e = int(cb[l][node]), int(cb[l][node + 1])
            node = b + int(draws[i]) % (e - b)
            i += 1
        x = f.get(oracle.FGT_NEXT_ROOTS)[int(f.get(oracle.FGT_LINK)[node])]
        root = synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]), int(x["bonus"]))
    return root


@pytest.mark.parametrize("seed", [1, 2, 3, 7])
def test_playout_equals_walk_through_unfolded_trees(seed):
    # two independent oracle routes: the move generator, and the trees the
    # unfolding builds (canonical child order, between-round linkage)
    deck = synth.deal(seed)
    draws = synth.playout_draws(seed, 5)
    for rnd in range(1, 6):
        assert playout_root(deck, rnd, draws) == walk_trees(deck, rnd, draws), (seed, rnd)


def test_playout_club_bookkeeping_and_reach():
    # every club dealt before the round is in the pool or counted for a side
    # while no bonus is decided; the pool holds only dealt cards; over many
    # seeds pools with a Jack occur (a legal state the old recipe never made)
    jack_pools = 0
    for seed in range(1, 41):
        deck = synth.deal(seed)
        draws = synth.playout_draws(seed, 5)
        for rnd in (4, 5):
            root = playout_root(deck, rnd, draws)
            dealt = synth.mask_of(deck[:4 + 8 * rnd])
            assert root.pool & ~dealt == 0
            clubs_dealt = sum(1 for c in deck[:4 + 8 * rnd] if c % 4 == 0)
            clubs_pool = sum(1 for c in range(0, 52, 4) if (root.pool >> c) & 1)
            if root.bonus == 0:
                assert root.ca + root.cb + clubs_pool == clubs_dealt, (seed, rnd)
                assert root.ca < 7 and root.cb < 7
            else:
                assert root.ca == 0 and root.cb == 0
            jack_pools += any((root.pool >> c) & 1 for c in synth.JACKS)
    assert jack_pools > 0


def test_playout_is_seeded():
    deck = synth.deal(5)
    a = playout_root(deck, 5, synth.playout_draws(5, 5))
    b = playout_root(deck, 5, synth.playout_draws(5, 5))
    c = playout_root(deck, 5, synth.playout_draws(6, 5))
    assert a == b and a != c
