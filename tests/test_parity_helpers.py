"""The reach-weighted comparison of average strategies used by the FP32
parity tests, checked on the CPU with planted mistakes: it must accept the
oracle's own average strategy, re-splits inside a tie group and noise at
nodes that play does not reach, and reject a small change of behaviour where
play does reach."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (assert_sigma_bar_up_to_ties, oracle_rounds, oracle_solve, path_reach,
                        tie_groups)


@pytest.fixture(scope="module")
def solved():
    deck, roots = synth.last_round_roots(1)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 300)
    f = rounds[0][1]
    return f, leaf, c.sigma_bar(), tie_groups(f, leaf)


def _parent_of(cb, l):
    b = np.asarray(cb[l - 1], np.int64)
    return np.repeat(np.arange(len(b) - 1), np.diff(b)), b


def test_path_reach_is_product_along_the_path(solved):
    f, leaf, sb, g = solved
    cb = f.child_begin()
    x = path_reach(cb, sb)
    par2, _ = _parent_of(cb, 2)
    par3, _ = _parent_of(cb, 3)
    e3 = 7
    e2 = par3[e3]
    e1 = par2[e2]
    assert x[3][e3] == pytest.approx(sb[1][e1] * sb[2][e2] * sb[3][e3], abs=0, rel=1e-15)
    # probabilities of one level sum to one (every root reached)
    for l in range(8):
        assert x[l].sum() == pytest.approx(f.n[0], rel=1e-12)


def _untied_pair(f, sb, g, want_high):
    """(level, untied edge, a sibling in another group, reach of the parent):
    at the most reached such parent, or at one reached below 1e-7."""
    cb = f.child_begin()
    x = path_reach(cb, sb)
    best = None
    for l in range(1, 9):
        par, b = _parent_of(cb, l)
        size = np.bincount(g[l])
        for e in np.nonzero(size[g[l]] == 1)[0]:
            h = par[e]
            sib = [o for o in range(b[h], b[h + 1]) if g[l][o] != g[l][e]]
            if not sib:
                continue
            w = x[l - 1][h]
            if want_high and w > 1e-3 and (best is None or w > best[3]):
                best = (l, e, sib[0], w)
            if not want_high and w < 1e-7:
                return l, e, sib[0], w
    if best is None:
        pytest.skip("no such parent in this tree")
    return best


def test_accepts_the_oracle_itself(solved):
    f, leaf, sb, g = solved
    tied, total, big = assert_sigma_bar_up_to_ties(sb, sb, g, f.child_begin(), 1e-5)
    assert big == 0 and 0 < tied < total


def test_rejects_small_change_where_mover_reaches(solved):
    f, leaf, sb, g = solved
    l, e, o, w = _untied_pair(f, sb, g, want_high=True)
    d = 3e-5 / w  # the action is played 3e-5 more (or less) often
    bad = [s.copy() for s in sb]
    sgn = 1.0 if bad[l][o] >= d else -1.0
    bad[l][e] += sgn * d
    bad[l][o] -= sgn * d
    with pytest.raises(AssertionError):
        assert_sigma_bar_up_to_ties(bad, sb, g, f.child_begin(), 1e-5)


def test_accepts_noise_where_mover_never_reaches(solved):
    f, leaf, sb, g = solved
    l, e, o, w = _untied_pair(f, sb, g, want_high=False)
    bad = [s.copy() for s in sb]
    m = min(bad[l][e], 0.3)
    bad[l][e] -= m
    bad[l][o] += m
    assert_sigma_bar_up_to_ties(bad, sb, g, f.child_begin(), 1e-5)


def test_accepts_resplit_inside_a_tie_group_but_not_across(solved):
    f, leaf, sb, g = solved
    cb = f.child_begin()
    x = path_reach(cb, sb)
    for l in range(1, 9):
        par, b = _parent_of(cb, l)
        size = np.bincount(g[l])
        cand = np.nonzero((size[g[l]] >= 2) & (x[l - 1][par] >= 0.1))[0]
        for e in cand:
            mates = np.nonzero((g[l] == g[l][e]) & (np.arange(len(g[l])) != e))[0]
            others = np.nonzero((par == par[e]) & (g[l] != g[l][e]))[0]
            if len(others) == 0:
                continue
            ok = [s.copy() for s in sb]
            m = ok[l][e] / 2
            ok[l][e] -= m
            ok[l][mates[0]] += m
            assert_sigma_bar_up_to_ties(ok, sb, g, cb, 1e-5)
            d = 3e-5 / x[l - 1][par[e]]  # the group is played 3e-5 more or less often
            sgn = 1.0 if sb[l][e] >= d else -1.0
            bad = [s.copy() for s in sb]
            bad[l][e] -= sgn * d
            bad[l][others[0]] += sgn * d
            with pytest.raises(AssertionError):
                assert_sigma_bar_up_to_ties(bad, sb, g, cb, 1e-5)
            return
    pytest.skip("no reached tie group with an untied sibling in this tree")


# ---- the element-wise MLP bounds (tests/mlp_bounds.py), with planted mistakes

def _mlp_problem(seed=3, M=900):
    from oracle import mlp as omlp
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 2, (M, omlp.N_IN)).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    dY = rng.normal(0, 1e-3, (M, 2))
    return W, X, dY


def test_mlp_forward_bounds_catch_planted_mistakes():
    from mlp_bounds import forward_bounds, layer_bounds
    from oracle import mlp as omlp
    W, X, _ = _mlp_problem()
    (H1, H2, Y), (A1, A2, bY) = forward_bounds(W, X)
    assert np.array_equal(H1, omlp.forward(W, X)[0])
    # layer by layer, only a small share of activations may round either way
    H1l, A1l = layer_bounds(X, W[0], W[1], True)
    H2l, A2l = layer_bounds(H1, W[2], W[3], True)
    Yl, bYl = layer_bounds(H2, W[4], W[5], False)
    assert np.array_equal(H1l, H1) and np.array_equal(H2l, H2)
    assert np.mean(A1l > 0) < 5e-2 and np.mean(A2l > 0) < 5e-2
    # one activation one bfloat16 step off where no rounding point is near
    i, j = map(int, np.argwhere((A2l == 0) & (H2 > 0))[0])
    bad = omlp.bf16_round(H2[i, j] * (1 + 2 ** -7))
    assert bad != H2[i, j] and abs(bad - H2[i, j]) > A2l[i, j]
    # an output off by a hundred-thousandth of the sum of its terms' sizes
    k = int(np.argmax(np.abs(Y[:, 0])))
    assert 1e-5 * (np.abs(H2[k]) @ np.abs(omlp.bf16_round(W[4][:, 0]))) > bYl[k, 0]
    # the carried (chain) bound is looser but still below a 1% error
    assert abs(Y[k, 0]) * 1e-2 > bY[k, 0]


def test_mlp_backward_bounds_catch_planted_mistakes():
    from mlp_bounds import backward_bounds
    from oracle import mlp as omlp
    W, X, dY = _mlp_problem()
    H1, H2, _ = omlp.forward(W, X)
    g = omlp.backward(W, X, H1, H2, dY)
    b = backward_bounds(W, X, H1, H2, dY)
    assert all(np.all(bi >= 0) for bi in b)
    # one dropped term of dW1 (one row of the reduction over rows)
    Xq = omlp.bf16_round(X)
    G2q = omlp.bf16_round((omlp.bf16_round(dY) @ omlp.bf16_round(W[4]).T) * (H2 > 0))
    G1q = omlp.bf16_round((G2q @ omlp.bf16_round(W[2]).T) * (H1 > 0))
    terms = np.abs(Xq[:, 0, None] * G1q)  # dW1[0, :] terms per row
    m, j = np.unravel_index(np.argmax(terms), terms.shape)
    assert terms[m, j] > b[0][0, j]
    # a column of dW2 taken from its neighbour
    assert np.any(np.abs(g[2][:, 1] - g[2][:, 0]) > b[2][:, 0])
    # a row of dW3 dropped, and db1 shifted by one row's gradient
    assert np.any(np.abs(g[4][3]) > b[4][3])
    G1 = (G2q @ omlp.bf16_round(W[2]).T) * (H1 > 0)
    r = int(np.argmax(np.abs(G1).sum(axis=1)))
    assert np.any(np.abs(G1[r]) > b[1])
