"""Pins of the external-sampling CFR reference (oracle/es.py).

- Unbiasedness: from a fixed strategy, one iteration's change of Alex's
  regrets and of Bob's average sums, averaged over many seeds, equals the
  exact full-width counterfactual quantities: Bob's reach times (child
  value - node value), and Bob's reach times Bob's strategy, with values
  computed by plain expectation over the whole tree (5 standard errors;
  edges too rarely reached to sample are bounded by their reach).
- With only forced moves for the opponent there is nothing to sample: the
  change is exactly that full-width quantity on one seed (for Alex's pass
  with Bob forced, and for Bob's pass, with its regret sign, with Alex
  forced).
- The counter-based draws continue across calls (n iterations at once equal
  n calls of one).
- Convergence: the average strategy's exploitability on a real final-round
  subgame falls far below the uniform profile's.
"""
import copy

import numpy as np
import pytest

import oracle
import synth
from oracle import es


def random_tree(rng, p_two=0.45, p_three=0.1, forced=None):
    """Eight levels from one root, 1-3 children per node (one at the levels
    of `forced`, "alex" or "bob"), integer leaf utilities in -8..8."""
    n = [1]
    cb = []
    for l in range(8):
        if (forced == "bob" and l & 1) or (forced == "alex" and not l & 1):
            k = np.ones(n[l], np.int64)
        else:
            k = rng.choice([1, 2, 3], size=n[l], p=[1 - p_two - p_three, p_two, p_three])
        cb.append(np.concatenate([[0], np.cumsum(k)]).astype(np.int64))
        n.append(int(cb[-1][-1]))
    leaf = rng.integers(-8, 9, n[8]).astype(np.float64)
    return n, cb, leaf


def random_sigma(rng, st):
    for l in range(8):
        for h in range(st.n[l]):
            b, e = st.cb[l][h], st.cb[l][h + 1]
            st.sigma[l + 1][b:e] = rng.dirichlet(np.ones(e - b))


def exact_quantities(st, leaf):
    """Full-width values under st.sigma, Bob's reach of every node, and the
    expected one-pass changes of Alex's regrets and Bob's average sums."""
    n, cb = st.n, st.cb
    val = [None] * 9
    val[8] = leaf.copy()
    for l in range(7, -1, -1):
        val[l] = np.zeros(n[l])
        for h in range(n[l]):
            for c in range(cb[l][h], cb[l][h + 1]):
                val[l][h] += st.sigma[l + 1][c] * val[l + 1][c]
    reach_b = [np.ones(n[0])]
    for l in range(8):
        r = np.zeros(n[l + 1])
        for h in range(n[l]):
            for c in range(cb[l][h], cb[l][h + 1]):
                r[c] = reach_b[l][h] * (st.sigma[l + 1][c] if l & 1 else 1.0)
        reach_b.append(r)
    dR, dS, pr = [None] * 9, [None] * 9, [None] * 9
    for l in range(8):
        d = np.zeros(n[l + 1])
        pr[l + 1] = np.zeros(n[l + 1])
        for h in range(n[l]):
            for c in range(cb[l][h], cb[l][h + 1]):
                pr[l + 1][c] = reach_b[l][h]
                if l & 1:   # Bob's node: his own reach times his strategy
                    d[c] = reach_b[l][h] * st.sigma[l + 1][c]
                else:       # Alex's node: Bob's reach times the regret
                    d[c] = reach_b[l][h] * (val[l + 1][c] - val[l][h])
        (dS if l & 1 else dR)[l + 1] = d
    return dR, dS, pr


@pytest.mark.parametrize("tree_seed", [0, 1])
def test_one_iteration_is_unbiased(tree_seed):
    rng = np.random.default_rng(tree_seed)
    n, cb, leaf = random_tree(rng)
    st0 = es.ESState(n, cb)
    random_sigma(rng, st0)
    dR, dS, pr = exact_quantities(st0, leaf)
    M = 3000
    acc = {("R", l): [] for l in (1, 3, 5, 7)}
    acc.update({("S", l): [] for l in (2, 4, 6, 8)})
    for s in range(M):
        st = copy.deepcopy(st0)
        es.es_iterate(st, leaf, 1, seed=1000 + s)
        for l in (1, 3, 5, 7):
            acc[("R", l)].append(st.R[l].copy())
        for l in (2, 4, 6, 8):
            acc[("S", l)].append(st.Sbar[l].copy())
    # an edge whose parent is expected to be reached fewer than 5 times in M
    # passes cannot be tested by its sample mean; its error is bounded by its
    # largest possible increment (16 for a regret, 1 for a strategy) times
    # the parent's reach
    tested = 0
    for (kind, l), xs in acc.items():
        xs = np.array(xs)
        mean, se = xs.mean(0), xs.std(0) / np.sqrt(M)
        want = (dR if kind == "R" else dS)[l]
        rare = pr[l] * M < 5
        tol = 5 * se + 1e-9 + np.where(rare, (16.0 if kind == "R" else 1.0) * pr[l], 0.0)
        assert np.all(np.abs(mean - want) <= tol), (kind, l, np.max(np.abs(mean - want) - tol))
        tested += int((~rare).sum())
    assert tested > 0.5 * sum(n[1:])


def test_forced_opponent_moves_are_exact():
    rng = np.random.default_rng(5)
    n, cb, leaf = random_tree(rng, p_two=0.6, p_three=0.2, forced="bob")
    st = es.ESState(n, cb)
    random_sigma(rng, st)
    dR, dS, _ = exact_quantities(st, leaf)
    es.es_iterate(st, leaf, 1, seed=3)
    for l in (1, 3, 5, 7):
        np.testing.assert_allclose(st.R[l], dR[l], rtol=0, atol=1e-12)
    for l in (2, 4, 6, 8):
        np.testing.assert_allclose(st.Sbar[l], dS[l], rtol=0, atol=1e-12)


def test_bob_pass_with_forced_alex_moves_is_exact():
    """Alex's moves all forced: his strategy stays 1, so Bob's pass is
    deterministic; Bob's regrets gain (node value - child value), the
    utilities being Alex minus Bob, and Alex's average sums gain 1."""
    rng = np.random.default_rng(9)
    n, cb, leaf = random_tree(rng, p_two=0.6, p_three=0.2, forced="alex")
    st = es.ESState(n, cb)
    random_sigma(rng, st)
    val = [None] * 9
    val[8] = leaf
    for l in range(7, -1, -1):
        val[l] = np.array([sum(st.sigma[l + 1][c] * val[l + 1][c] for c in range(cb[l][h], cb[l][h + 1]))
                           for h in range(n[l])])
    es.es_iterate(st, leaf, 1, seed=4)
    for l in (2, 4, 6, 8):
        want = np.zeros(n[l])
        for h in range(n[l - 1]):
            for c in range(cb[l - 1][h], cb[l - 1][h + 1]):
                want[c] = val[l - 1][h] - val[l][c]
        np.testing.assert_allclose(st.R[l], want, rtol=0, atol=1e-12)
    for l in (1, 3, 5, 7):
        np.testing.assert_allclose(st.Sbar[l], 1.0, rtol=0, atol=1e-12)
        np.testing.assert_allclose(st.R[l], 0.0, rtol=0, atol=1e-12)


def test_draws_continue_across_calls():
    rng = np.random.default_rng(7)
    n, cb, leaf = random_tree(rng)
    a, b = es.ESState(n, cb), es.ESState(n, cb)
    es.es_iterate(a, leaf, 5, seed=11)
    for _ in range(5):
        es.es_iterate(b, leaf, 1, seed=11)
    for l in range(1, 9):
        assert np.array_equal(a.R[l], b.R[l]) and np.array_equal(a.Sbar[l], b.Sbar[l])
    c = es.ESState(n, cb)
    es.es_iterate(c, leaf, 5, seed=12)
    assert any(not np.array_equal(a.Sbar[l], c.Sbar[l]) for l in range(1, 9))


def test_converges_on_final_round_subgame():
    deck, roots = synth.last_round_roots(4)
    gt = oracle.GT(deck, 5, sorted({x.pool for x in roots}))
    f = oracle.FGT(gt, roots[:1])
    cb = f.child_begin()
    leaf = f.leaf_utilities()
    st = es.ESState(f.n, cb)

    def expl(sig):
        bra = oracle.tree_values(f.n, cb, leaf, sig, oracle.TV_BR_A)
        brb = oracle.tree_values(f.n, cb, leaf, sig, oracle.TV_BR_B)
        return float((bra[0] - brb[0]) / 2)

    e0 = expl(st.sigma_bar())
    es.es_iterate(st, leaf, 1000, seed=1)
    e1 = expl(st.sigma_bar())
    mm = oracle.tree_values(f.n, cb, leaf, st.sigma_bar(), oracle.TV_MINIMAX)[0]
    v = oracle.tree_values(f.n, cb, leaf, st.sigma_bar(), oracle.TV_EXPECT)[0]
    print(f"[es] exploitability uniform {e0:.4f} -> {e1:.4f} after 1000 iterations; "
          f"value {v:.4f}, minimax {mm:.4f}")
    assert e1 < 0.05 * e0
    # the value and the minimax value both lie between the best responses
    assert abs(v - mm) <= 2 * e1 + 1e-9
