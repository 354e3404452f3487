"""Subgames that start from legal states: both sides play the same seeded
moves from the initial deal with their own rules (the oracle's move
generator, the library's round trees), reach the same root, and solve its
subgame to the usual parity bars."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (assert_sigma_bar_up_to_ties, oracle_rounds, oracle_solve, require_gpu,
                        tie_groups, to_np)
from oracle.playout import playout_root as oracle_playout

pytestmark = pytest.mark.gpu


def both_roots(pa, seed, rnd):
    deck = synth.deal(seed)
    draws = synth.playout_draws(seed, 5)
    g = pa.playout_root(deck, rnd, draws)
    o = oracle_playout(deck, rnd, draws)
    return deck, synth.Root(int(g["pool"]), int(g["ca"]), int(g["cb"]), int(g["d"]),
                            int(g["bonus"])), o


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_playout_roots_match_oracle(seed):
    pa = require_gpu()
    for rnd in range(1, 6):
        deck, g, o = both_roots(pa, seed, rnd)
        assert g == o, (seed, rnd, g, o)


def last_round(root, deltas=range(-3, 4)):
    return sorted((synth.Root(root.pool, root.ca, root.cb, root.d + int(x), root.bonus)
                   for x in deltas), key=synth.Root.sort_key)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_playout_last_round_fp64_and_fp32(seed):
    pa = require_gpu()
    import torch
    deck, g, o = both_roots(pa, seed, 5)
    assert g == o
    print(f"[playout] last round seed={seed} pool={g.pool:#x} score=({g.ca},{g.cb},{g.d},{g.bonus})",
          flush=True)
    rounds = oracle_rounds(deck, 5, last_round(o))
    (c, leaf, V), = oracle_solve(rounds, 1000)
    s = pa.SubgameSolver(deck, 5, last_round(g), dtype=pa.PASUR_F64)
    s.solve(1000)
    torch.cuda.synchronize()
    st = s.rounds[0].state
    assert np.array_equal(to_np(st.u[8]), leaf)
    for l in range(1, 9):
        np.testing.assert_allclose(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l), rtol=0,
                                   atol=1e-9)
        np.testing.assert_allclose(to_np(st.R[l]), c.get(oracle.CF_R, l), rtol=0, atol=1e-9)
    np.testing.assert_allclose(to_np(s.rounds[0].V), V, rtol=0, atol=1e-9)
    s.free()
    s = pa.SubgameSolver(deck, 5, last_round(g), dtype=pa.PASUR_F32)
    s.solve(1000)
    torch.cuda.synchronize()
    gsb = [None] + [to_np(t) for t in s.rounds[0].state.sigma_bar[1:]]
    assert_sigma_bar_up_to_ties(gsb, c.sigma_bar(), tie_groups(rounds[0][1], leaf),
                                rounds[0][1].child_begin(), 1e-5, seed)
    assert np.abs(to_np(s.rounds[0].V) - V).max() <= 1e-5
    s.free()


@pytest.mark.parametrize("seed", [1, 2])
def test_playout_two_rounds_fp64_with_exploitability(seed):
    pa = require_gpu()
    import torch
    deck, g, o = both_roots(pa, seed, 4)
    assert g == o
    print(f"[playout] two rounds seed={seed}", flush=True)
    rounds = oracle_rounds(deck, 4, [o])
    res = oracle_solve(rounds, 2000)
    s = pa.SubgameSolver(deck, 4, [g], dtype=pa.PASUR_F64)
    s.solve(2000)
    torch.cuda.synchronize()
    for k in range(2):
        c, leaf, V = res[k]
        st = s.rounds[k].state
        for l in range(1, 9):
            np.testing.assert_allclose(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l),
                                       rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(s.rounds[k].V), V, rtol=0, atol=1e-9)
    from gpu_common import oracle_exploitability
    sb = [c.sigma_bar() for c, _, _ in res]
    bra, brb, v = oracle_exploitability(rounds, sb)
    gbra, gbrb, gv = (to_np(x) for x in s.exploitability())
    np.testing.assert_allclose(gbra, bra, rtol=0, atol=1e-9)
    np.testing.assert_allclose(gbrb, brb, rtol=0, atol=1e-9)
    s.free()
