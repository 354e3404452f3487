"""GPU self-play (pasur_selfplay) against the oracle: the same counter-based
draws and FP64 average strategies give the same games, so every margin must
match exactly; at the full-game scale the mean margin of 2^20 games must
agree with the exact expected margin of the profile."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import oracle_rounds, oracle_solve, require_gpu, to_np
from oracle import selfplay as sp
from test_oracle_selfplay import play_rounds

pytestmark = pytest.mark.gpu


def test_selfplay_matches_oracle_game_by_game():
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(5)
    iters = 100
    s = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F64)
    s.solve(iters)
    orr = oracle_rounds(deck, 4, roots)
    res = oracle_solve(orr, iters)
    sbars = [r[0].sigma_bar() for r in res]
    # the average strategies agree (FP64, the oracle's operation order)
    for k, rr in enumerate(s.rounds):
        for l in range(1, 9):
            np.testing.assert_allclose(to_np(rr.state.sigma_bar[l]), sbars[k][l], rtol=0, atol=1e-12)
    rounds = play_rounds(orr, sbars)
    n = 2001  # odd: a thread's second game past the end
    for seed, pa_, pb_ in ((1, pa.PLAY_SIGMA_BAR, pa.PLAY_SIGMA_BAR),
                           (2, pa.PLAY_SIGMA_BAR, pa.PLAY_UNIFORM),
                           (3, pa.PLAY_UNIFORM, pa.PLAY_SIGMA_BAR),
                           (4, pa.PLAY_UNIFORM, pa.PLAY_UNIFORM)):
        got = to_np(s.selfplay(n, seed, pa_, pb_)).astype(np.int64)
        want = sp.play(rounds, n, seed, pa_, pb_, 0)
        assert np.array_equal(got, want), (seed, np.nonzero(got != want)[0][:5])
        print(f"[selfplay] policies {pa_}/{pb_}: {n} games identical, "
              f"{len(np.unique(got))} distinct margins, Alex wins {np.mean(got > 0):.3f}", flush=True)
    # the average strategy of a two-round endgame is close to pure, so the
    # seed is seen through the uniform players: deterministic per seed,
    # different across seeds, and the games do differ from each other
    u = pa.PLAY_UNIFORM
    a = to_np(s.selfplay(n, 1, u, u))
    b = to_np(s.selfplay(n, 1, u, u))
    c = to_np(s.selfplay(n, 99, u, u))
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert len(np.unique(a)) > 3
    s.free()


def test_full_game_mean_margin_matches_expectation():
    """2^20 full games per matchup: the mean margin agrees with the exact
    expected margin of the profile being played.  For a uniform player that
    profile is built by clearing its cumulative strategy on its levels (Bob
    moves on the even levels) and normalising again, which gives uniform
    average strategies there; the exact value then comes from the same
    expected-value pass that exploitability uses."""
    pa = require_gpu()
    import torch
    deck, roots = synth.full_game_root(1)
    s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F32)
    s.solve(300)
    n = 1 << 20
    U, S = pa.PLAY_UNIFORM, pa.PLAY_SIGMA_BAR
    m = {pp: to_np(s.selfplay(n, 2024 + i, *pp)).astype(np.float64)
         for i, pp in enumerate(((S, S), (S, U), (U, U)))}

    def exact():
        return float(s.exploitability()[2][0])

    def check(pp, want):
        x = m[pp]
        se = x.std() / np.sqrt(n)
        print(f"[selfplay] full game {pp}: mean margin {x.mean():.4f} (se {se:.4f}), exact {want:.4f}, "
              f"fair value {np.mean(x > 0):.4f}", flush=True)
        assert abs(x.mean() - want) <= 5 * se + 0.01, pp

    check((S, S), exact())
    for rr in s.rounds:
        for l in (2, 4, 6, 8):
            rr.state.Sbar[l].zero_()
        pa.average_strategy(rr.state, s.stream)
    check((S, U), exact())
    for rr in s.rounds:
        for l in (1, 3, 5, 7):
            rr.state.Sbar[l].zero_()
        pa.average_strategy(rr.state, s.stream)
    check((U, U), exact())
    assert m[(S, U)].std() > 0 and m[(U, U)].std() > 0
    s.free()


def test_single_round_other_root_and_empty_call():
    """One round (the final-round subgame of seven roots), games from root 5,
    game by game against the oracle; zero games is a valid empty call."""
    pa = require_gpu()
    deck, roots = synth.last_round_roots(2)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F64)
    s.solve(60)
    gt = oracle.GT(deck, 5, sorted({x.pool for x in roots}))
    f = oracle.FGT(gt, roots)
    sb = [None] + [to_np(x).copy() for x in s.rounds[0].state.sigma_bar[1:]]
    rounds = [{"cb": f.child_begin(), "sbar": sb, "link": None, "base": f.leaf_utilities()}]
    for pp in ((pa.PLAY_SIGMA_BAR, pa.PLAY_UNIFORM), (pa.PLAY_UNIFORM, pa.PLAY_UNIFORM)):
        got = to_np(s.selfplay(1500, 7, *pp, root=5)).astype(np.int64)
        want = sp.play(rounds, 1500, 7, pp[0], pp[1], 5)
        assert np.array_equal(got, want), pp
    assert s.selfplay(0, 7).numel() == 0
    s.free()
