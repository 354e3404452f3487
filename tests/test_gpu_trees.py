"""GPU parity of tree construction, unfolding and linkage: bit-exact
against the FP64 oracle, level by level, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import require_gpu, roots_from_array

pytestmark = pytest.mark.gpu

GT_FIELDS = [("GT_POOL", oracle.GT_POOL), ("GT_HANDS", oracle.GT_HANDS), ("GT_RS", oracle.GT_RS),
             ("GT_PARENT", oracle.GT_PARENT), ("GT_CHILD_BEGIN", oracle.GT_CHILD_BEGIN),
             ("GT_ACT_CARD", oracle.GT_ACT_CARD), ("GT_ACT_CAP", oracle.GT_ACT_CAP)]


def compare_round(pa, deck, rnd, roots):
    print(f"[tree parity] round={rnd} n_roots={len(roots)}", flush=True)
    d_roots = pa.roots_to_device(roots)
    gt = pa.build_round_tree(deck, rnd, d_roots, len(roots))
    ogt = oracle.GT(deck, rnd, sorted({r.pool for r in roots}))
    assert gt.n == ogt.n
    for name, fo in GT_FIELDS:
        fg = getattr(pa, name)
        for l in range(9):
            if fo == oracle.GT_PARENT and l == 0:
                continue
            if fo == oracle.GT_CHILD_BEGIN and l == 8:
                continue
            if fo in (oracle.GT_ACT_CARD, oracle.GT_ACT_CAP) and l == 0:
                continue
            a, b = gt.read(fg, l), ogt.get(fo, l)
            assert np.array_equal(a, b), (name, l)
    fgt = pa.unfold_scores(gt, d_roots, len(roots))
    of = oracle.FGT(ogt, roots)
    assert fgt.n == of.n and fgt.n_scores == of.n_scores and fgt.n_next == of.n_next
    for l in range(9):
        assert np.array_equal(fgt.read(pa.FGT_GT, l), of.get(oracle.FGT_GT, l))
        assert np.array_equal(fgt.read(pa.FGT_SID, l), of.get(oracle.FGT_SID, l))
        if l > 0:
            assert np.array_equal(fgt.read(pa.FGT_PARENT, l), of.get(oracle.FGT_PARENT, l))
        if l < 8:
            assert np.array_equal(fgt.read(pa.FGT_CHILD_BEGIN, l), of.get(oracle.FGT_CHILD_BEGIN, l))
    assert np.array_equal(fgt.read(pa.FGT_SCORE_TAB), of.get(oracle.FGT_SCORE_TAB))
    # per-leaf base utility = oracle leaf utility with zero continuation values
    if rnd == 5:
        want = of.leaf_utilities()
    else:
        want = of.leaf_utilities(np.zeros(of.n_next))
    assert np.array_equal(fgt.read(pa.FGT_LEAF_BASE).astype(np.float64), want)
    if rnd < 5:
        nr, onr = fgt.read(pa.FGT_NEXT_ROOTS), of.get(oracle.FGT_NEXT_ROOTS)
        for k in ("pool", "ca", "cb", "d", "bonus", "pad"):
            assert np.array_equal(nr[k], onr[k]), k
        assert np.array_equal(fgt.read(pa.FGT_LINK), of.get(oracle.FGT_LINK))
        nxt = roots_from_array(onr)
    else:
        nxt = None
    gt.free()
    fgt.free()
    return nxt


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_last_round_trees_bit_exact(seed):
    pa = require_gpu()
    deck, roots = synth.last_round_roots(seed)
    compare_round(pa, deck, 5, roots)


@pytest.mark.parametrize("seed", [1, 3])
def test_two_round_trees_bit_exact(seed):
    pa = require_gpu()
    deck, roots = synth.two_round_root(seed)
    nxt = compare_round(pa, deck, 4, roots)
    compare_round(pa, deck, 5, nxt)


def test_full_game_first_rounds_bit_exact():
    pa = require_gpu()
    deck, roots = synth.full_game_root(2)
    for r in range(0, 3):
        roots = compare_round(pa, deck, r, roots)


def test_worked_deck_round_chain_bit_exact():
    # The paper's worked deck: rounds 0 and 1 from the initial deal.
    pa = require_gpu()
    deck = synth.DECK9
    roots = [synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)]
    roots = compare_round(pa, deck, 0, roots)
    compare_round(pa, deck, 1, roots)


def test_device_chained_rounds_match_host_chained():
    # Next-round roots stay on the device between rounds.
    pa = require_gpu()
    deck, roots = synth.two_round_root(1)
    d_roots = pa.roots_to_device(roots)
    gt4 = pa.build_round_tree(deck, 4, d_roots, len(roots))
    f4 = pa.unfold_scores(gt4, d_roots, len(roots))
    ptr, n = f4.next_roots_device()
    gt5 = pa.build_round_tree(deck, 5, ptr, n)
    f5 = pa.unfold_scores(gt5, ptr, n)
    of4 = oracle.FGT(oracle.GT(deck, 4, [roots[0].pool]), roots)
    r5 = roots_from_array(of4.get(oracle.FGT_NEXT_ROOTS))
    of5 = oracle.FGT(oracle.GT(deck, 5, sorted({r.pool for r in r5})), r5)
    assert f5.n == of5.n
    assert np.array_equal(f5.read(pa.FGT_PARENT, 8), of5.get(oracle.FGT_PARENT, 8))


def test_invalid_inputs_are_rejected():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(1)
    d_roots = pa.roots_to_device(roots)
    with pytest.raises(pa.PasurError, match="round"):
        pa.build_round_tree(deck, 6, d_roots, len(roots))
    bad_deck = list(deck)
    bad_deck[0] = bad_deck[1]
    with pytest.raises(pa.PasurError, match="permutation"):
        pa.build_round_tree(bad_deck, 5, d_roots, len(roots))
    # roots out of canonical order
    d_rev = pa.roots_to_device(list(reversed(roots)))
    with pytest.raises(pa.PasurError, match="ascending"):
        pa.build_round_tree(deck, 5, d_rev, len(roots))
    # a pool card that is dealt in this very round
    hand_card = deck[44]
    r0 = roots[0]
    d_bad = pa.roots_to_device([synth.Root(r0.pool | (1 << hand_card), r0.ca, r0.cb, r0.d, r0.bonus)])
    with pytest.raises(pa.PasurError):
        pa.build_round_tree(deck, 5, d_bad, 1)
    # unfolding with roots whose pools are not the tree's
    gt = pa.build_round_tree(deck, 5, d_roots, len(roots))
    smaller = r0.pool & (r0.pool - 1)  # drop the lowest pool card
    d_o = pa.roots_to_device([synth.Root(smaller, r0.ca, r0.cb, r0.d, r0.bonus)])
    with pytest.raises(pa.PasurError, match="pools"):
        pa.unfold_scores(gt, d_o, 1)
    gt.free()
