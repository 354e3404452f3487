"""Pins of the self-play oracle: its random stream against SplitMix64's
published outputs, the inverse-CDF choice at its edges, exact paths for
pure strategies, and the Monte Carlo mean of the margins against the exact
expectation of the strategy profile (one and two rounds)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import oracle_rounds, oracle_solve
from oracle import selfplay as sp


def test_stream_is_splitmix64():
    # first outputs of SplitMix64 seeded with 0 (the generator's reference values)
    assert [sp.splitmix64(0, i) for i in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert sp.splitmix_uniform(0, 0) == (0xE220A8397B1DCDAF >> 11) / 2.0 ** 53


def test_choose_edges():
    p = [0.0, 0.25, 0.0, 0.75, 0.0]
    assert sp.choose(0.0, p, sp.POLICY_SIGMA_BAR) == 1
    assert sp.choose(0.2499, p, sp.POLICY_SIGMA_BAR) == 1
    assert sp.choose(0.2501, p, sp.POLICY_SIGMA_BAR) == 3
    assert sp.choose(1.0 - 2 ** -53, p, sp.POLICY_SIGMA_BAR) == 3
    assert [sp.choose(u, p, sp.POLICY_UNIFORM) for u in (0.0, 0.19, 0.2, 0.99)] == [0, 0, 1, 4]
    assert sp.choose(0.7, [0.0, 0.0], sp.POLICY_SIGMA_BAR) == 1  # zero total: uniform
    assert sp.choose(0.3, [1.0], sp.POLICY_SIGMA_BAR) == 0


def play_rounds(orr, sbars):
    rounds = []
    for k, (gt, f) in enumerate(orr):
        last = k == len(orr) - 1
        base = f.leaf_utilities(None if last else np.zeros(orr[k + 1][1].n[0]))
        rounds.append({"cb": f.child_begin(), "sbar": sbars[k],
                       "link": None if last else f.get(oracle.FGT_LINK), "base": base})
    return rounds


def expected_margin(orr, sbars, root):
    V = None
    for k in range(len(orr) - 1, -1, -1):
        gt, f = orr[k]
        leaf = f.leaf_utilities(V)
        V = oracle.tree_values(f.n, f.child_begin(), leaf, sbars[k], oracle.TV_EXPECT)
    return V[root]


def uniform_sigma(f):
    cb = f.child_begin()
    out = [None]
    for l in range(1, 9):
        s = np.zeros(f.n[l])
        for h in range(f.n[l - 1]):
            s[cb[l - 1][h]:cb[l - 1][h + 1]] = 1.0 / (cb[l - 1][h + 1] - cb[l - 1][h])
        out.append(s)
    return out


def test_pure_strategies_follow_one_path():
    deck, roots = synth.last_round_roots(4)
    orr = oracle_rounds(deck, 5, roots)
    res = oracle_solve(orr, 100)
    f = orr[0][1]
    cb = f.child_begin()
    sb = res[0][0].sigma_bar()
    pure = [None]
    for l in range(1, 9):
        s = np.zeros(f.n[l])
        for h in range(f.n[l - 1]):
            b, e = cb[l - 1][h], cb[l - 1][h + 1]
            s[b + int(np.argmax(sb[l][b:e]))] = 1.0
        pure.append(s)
    rounds = play_rounds(orr, [pure])
    for root in range(len(roots)):
        q = root
        for l in range(8):
            b, e = cb[l][q], cb[l][q + 1]
            q = b + int(np.argmax(pure[l + 1][b:e]))
        want = rounds[0]["base"][q]
        got = sp.play(rounds, 50, 7, sp.POLICY_SIGMA_BAR, sp.POLICY_SIGMA_BAR, root)
        assert np.all(got == want), root


@pytest.mark.parametrize("start", [5, 4])
def test_mean_margin_matches_expectation(start):
    seed = 3
    deck, roots = synth.last_round_roots(seed) if start == 5 else synth.two_round_root(seed)
    orr = oracle_rounds(deck, start, roots)
    res = oracle_solve(orr, 100)
    sbars = [r[0].sigma_bar() for r in res]
    n = 3000
    for pa_, pb_, sb in ((sp.POLICY_SIGMA_BAR, sp.POLICY_SIGMA_BAR, sbars),
                         (sp.POLICY_UNIFORM, sp.POLICY_UNIFORM,
                          [uniform_sigma(f) for _, f in orr])):
        m = sp.play(play_rounds(orr, sb), n, 11, pa_, pb_, 0)
        want = expected_margin(orr, sb, 0)
        se = m.std() / np.sqrt(n)
        # 5 standard errors, plus a little for outcomes of probability too small
        # to be drawn in n games (a near-pure strategy profile gives se = 0)
        assert abs(m.mean() - want) <= 5 * se + 0.01, (pa_, m.mean(), want, se)
