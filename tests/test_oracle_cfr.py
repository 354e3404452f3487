"""Pins of the FP64 oracle's DCFR, average strategy and best response.

The CFR pins are: a tiny game whose first three DCFR iterations were worked
out by hand from the paper's equations (DFCR_REG, RM, DFCR_AVG); brute-force
best responses over all pure strategies; the minimax bound and shrinking
exploitability that the convergence theorems guarantee; and structural
invariants (simplex, forced moves, the inherited point difference not
entering the utility).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def padded_tree(fanouts_l1, leaves):
    """Alex picks among len(fanouts_l1) actions at level 0, Bob then picks
    among fanouts_l1[i]; levels 2..8 are forced single-child chains so the
    tree has the 8-ply shape of a round."""
    n1 = len(fanouts_l1)
    n2 = sum(fanouts_l1)
    n = [1, n1] + [n2] * 7
    cb = [np.array([0, n1], np.int32),
          np.concatenate([[0], np.cumsum(fanouts_l1)]).astype(np.int32)]
    cb += [np.arange(n2 + 1, dtype=np.int32)] * 6
    return n, cb, np.asarray(leaves, np.float64)


def test_dcfr_three_iterations_by_hand():
    # Alex: a1, a2; Bob after a1: b1 -> 3, b2 -> -1; after a2: b1 -> 0, b2 -> 2.
    # Textbook regret matching (positive part, uniform when none is positive),
    # DCFR alpha=1.5, beta=0, gamma=2.  Hand computation (t = 1, 2, 3):
    #   t=1: u(a1)=1, u(a2)=1, u=1.  R(a1:b)=(-1,1), R(a2:b)=(1/2,-1/2), R(root)=(0,0)
    #   t=2: sigma(a1:b)=(0,1), sigma(a2:b)=(1,0), sigma(root)=(1/2,1/2);
    #        u(a1)=-1, u(a2)=0, u=-1/2; every discount is 1/2 at t=2;
    #        R(a1:b)=(-5/2,1/2), R(a2:b)=(1/4,-5/4), R(root)=(-1/2,1/2)
    #   t=3: sigma(root)=(0,1); u=0; with c = 2^1.5/(2^1.5+1):
    #        R(a1:b)=(-5/4, c/2), R(a2:b)=(c/4, -21/8), R(root)=(-5/4, c/2)
    #   Sbar(root)=(5/18, 23/18) -> avg (5/28, 23/28); Sbar(a1:b)=(1/18, 3/2)
    #   -> (1/28, 27/28); Sbar(a2:b)=(3/2, 1/18) -> (27/28, 1/28); vacc = 1/2.
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    c = oracle.CFR(n, cb, leaves)
    c.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE))
    cc = 2 ** 1.5 / (2 ** 1.5 + 1)
    np.testing.assert_allclose(c.get(oracle.CF_R, 1), [-1.25, cc / 2], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_R, 2), [-1.25, cc / 2, cc / 4, -2.625], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 1), [5 / 18, 23 / 18], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 2), [1 / 18, 1.5, 1.5, 1 / 18], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 1), [5 / 28, 23 / 28], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 2),
                               [1 / 28, 27 / 28, 27 / 28, 1 / 28], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA, 1), [0, 1], atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA, 2), [0, 1, 1, 0], atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_VACC), [0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_U, 0), [0.0], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_U, 1), [-1.0, 0.0], atol=1e-14)


def test_vanilla_cfr_three_iterations_by_hand():
    # Same game; vanilla CFR (section "CFR": R <- R + r, no discount, uniform
    # average weights), textbook regret matching.  Reaches: level-1 nodes
    # have pi_A = sigma(root), pi_B = 1; Bob's regret is -pi_A (u(q) - u(h)).
    #   t=1: sigma uniform; u(a1)=u(a2)=u=1; r(a1:b)=(-1,1), r(a2:b)=(1/2,-1/2),
    #        r(root)=(0,0); Sbar(root)=(1/2,1/2), Sbar(a1:b)=Sbar(a2:b)=(1/2,1/2)
    #   t=2: sigma(a1:b)=(0,1), sigma(a2:b)=(1,0), sigma(root)=(1/2,1/2);
    #        u(a1)=-1, u(a2)=0, u=-1/2; r(a1:b)=(-2,0), r(a2:b)=(0,-1),
    #        r(root)=(-1/2,1/2); R(a1:b)=(-3,1), R(a2:b)=(1/2,-3/2),
    #        R(root)=(-1/2,1/2); Sbar(root)=(1,1), Sbar(a1:b)=(1/2,3/2),
    #        Sbar(a2:b)=(3/2,1/2)
    #   t=3: sigma(root)=(0,1) (pi_A(a1)=0, so Bob's regrets at a1 stay);
    #        u(a1)=-1, u(a2)=0, u=0; r(a2:b)=(0,-2), r(root)=(-1,0);
    #        R(a1:b)=(-3,1), R(a2:b)=(1/2,-7/2), R(root)=(-3/2,1/2);
    #        Sbar(root)=(1,2), Sbar(a1:b)=(1/2,5/2), Sbar(a2:b)=(5/2,1/2);
    #        average (1/3,2/3), (1/6,5/6), (5/6,1/6); vacc = 1 - 1/2 + 0.
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    c = oracle.CFR(n, cb, leaves)
    c.run(3, oracle.Params(variant=oracle.CFR_VANILLA, rm_mode=oracle.RM_POSITIVE))
    np.testing.assert_allclose(c.get(oracle.CF_R, 1), [-1.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_R, 2), [-3, 1, 0.5, -3.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 1), [1, 2], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 2), [0.5, 2.5, 2.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 1), [1 / 3, 2 / 3], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 2), [1 / 6, 5 / 6, 5 / 6, 1 / 6],
                               atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA, 1), [0, 1], atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA, 2), [0, 1, 1, 0], atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_VACC), [0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_U, 1), [-1.0, 0.0], atol=1e-14)
    # forced edges keep zero regret and probability one
    for l in range(3, 9):
        np.testing.assert_allclose(c.get(oracle.CF_R, l), np.zeros(4), atol=0)
        np.testing.assert_allclose(c.get(oracle.CF_SIGMA, l), np.ones(4), atol=0)


def test_cfr_plus_three_iterations_by_hand():
    # Same game; CFR+ (section "CFR", the CFR+ rule: R <- max(R + r, 0)) with
    # the linearly weighted average of Tammelin's CFR+ (iteration t adds
    # t * pi_p * sigma^t), textbook regret matching.  Instantaneous regrets
    # are those of the vanilla run until the profiles differ (they do not here):
    #   t=1: R(a1:b)=(0,1), R(a2:b)=(1/2,0), R(root)=(0,0); Sbar as vanilla
    #   t=2: same sigma^2; R(a1:b)=(0,1), R(a2:b)=(1/2,0), R(root)=(0,1/2);
    #        Sbar(root)=(1/2+1, 1/2+1), Sbar(a1:b)=(1/2, 1/2+2), Sbar(a2:b)=(1/2+2, 1/2)
    #   t=3: sigma(root)=(0,1); R(a2:b)=(1/2, max(0-2,0)), R(root)=(max(0-1,0), 1/2);
    #        Sbar(root)=(3/2, 3/2+3), Sbar(a1:b)=(1/2, 5/2+3), Sbar(a2:b)=(5/2+3, 1/2);
    #        average (1/4,3/4), (1/12,11/12), (11/12,1/12)
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    c = oracle.CFR(n, cb, leaves)
    c.run(3, oracle.Params(variant=oracle.CFR_PLUS, rm_mode=oracle.RM_POSITIVE))
    np.testing.assert_allclose(c.get(oracle.CF_R, 1), [0, 0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_R, 2), [0, 1, 0.5, 0], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 1), [1.5, 4.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 2), [0.5, 5.5, 5.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 1), [0.25, 0.75], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 2), [1 / 12, 11 / 12, 11 / 12, 1 / 12],
                               atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA, 1), [0, 1], atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_VACC), [0.5], atol=1e-14)
    # clipped regrets are never negative
    for l in range(1, 9):
        assert (c.get(oracle.CF_R, l) >= 0).all()


def test_cfr_plus_and_vanilla_split_runs_continue_the_count():
    # t0 carries the iteration number: 3 iterations as 1 + 2 equal 3 at once
    # (the linear weight of CFR+ and the counters of both rules depend on t).
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    for variant in (oracle.CFR_PLUS, oracle.CFR_VANILLA):
        p = oracle.Params(variant=variant, rm_mode=oracle.RM_POSITIVE)
        a = oracle.CFR(n, cb, leaves)
        a.run(3, p)
        b = oracle.CFR(n, cb, leaves)
        b.run(1, p)
        b.run(2, p)  # continues at t = 2
        for l in (1, 2):
            np.testing.assert_array_equal(a.get(oracle.CF_SBAR, l), b.get(oracle.CF_SBAR, l))
            np.testing.assert_array_equal(a.get(oracle.CF_R, l), b.get(oracle.CF_R, l))


def test_threaded_cfr_is_bit_identical():
    # the per-level parent loops shared out over threads give the same
    # arrays bit for bit (each parent's sums stay sequential)
    deck, roots = synth.last_round_roots(2)
    f = oracle.FGT(oracle.GT(deck, 5, sorted({x.pool for x in roots})), roots)
    out = []
    for threads in (1, 4):
        oracle.set_threads(threads)
        try:
            c = oracle.CFR(f.n, f.child_begin(), f.leaf_utilities())
            c.run(50)
            out.append([c.get(fld, l) for fld in (oracle.CF_R, oracle.CF_SBAR, oracle.CF_SIGMA)
                        for l in range(1, 9)] + [c.get(oracle.CF_VACC)])
        finally:
            oracle.set_threads(1)
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_floor_rule_matches_textbook_when_regrets_are_large():
    # The executed rule max(R, 1e-8)/sum differs from the positive-part rule
    # only by terms of order 1e-8.
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    a = oracle.CFR(n, cb, leaves)
    b = oracle.CFR(n, cb, leaves)
    a.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE))
    b.run(3, oracle.Params(rm_mode=oracle.RM_FLOOR))
    for l in (1, 2):
        np.testing.assert_allclose(a.get(oracle.CF_SIGMA_BAR, l), b.get(oracle.CF_SIGMA_BAR, l),
                                   atol=1e-7)


def random_tree(rng, fan):
    """Random 8-level tree with the given max fan-out per level."""
    n = [1]
    cb = []
    for l in range(8):
        k = rng.integers(1, fan[l] + 1, size=n[-1])
        cb.append(np.concatenate([[0], np.cumsum(k)]).astype(np.int32))
        n.append(int(k.sum()))
    leaves = rng.integers(-6, 7, size=n[8]).astype(np.float64)
    return n, cb, leaves


def brute_force_br(n, cb, leaves, sigma, player):
    """Enumerate every pure strategy of ``player`` (0 Alex maximises, 1 Bob
    minimises) and evaluate it against ``sigma`` by plain recursion."""
    dec = [(l, h) for l in range(8) if l % 2 == player for h in range(n[l])
           if cb[l][h + 1] - cb[l][h] > 1]
    choices = [range(cb[l][h + 1] - cb[l][h]) for l, h in dec]
    best = None
    for pick in itertools.product(*choices):
        pure = dict(zip(dec, pick))

        def val(l, h):
            if l == 8:
                return leaves[h]
            b, e = cb[l][h], cb[l][h + 1]
            if l % 2 == player:
                j = pure.get((l, h), 0)
                return val(l + 1, b + j)
            return sum(sigma[l + 1][q] * val(l + 1, q) for q in range(b, e))

        v = val(0, 0)
        if best is None or (v > best if player == 0 else v < best):
            best = v
    return best


@pytest.mark.parametrize("seed", range(6))
def test_best_response_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    n, cb, leaves = random_tree(rng, [3, 2, 2, 2, 1, 2, 1, 1])
    sigma = [np.ones(1)]
    for l in range(8):
        s = np.zeros(n[l + 1])
        for h in range(n[l]):
            b, e = cb[l][h], cb[l][h + 1]
            s[b:e] = rng.dirichlet(np.ones(e - b))
        sigma.append(s)
    for player, mode in ((0, oracle.TV_BR_A), (1, oracle.TV_BR_B)):
        got = oracle.tree_values(n, cb, leaves, sigma, mode)[0]
        assert got == pytest.approx(brute_force_br(n, cb, leaves, sigma, player), abs=1e-12)


def exploitability(n, cb, leaves, sbar):
    br_a = oracle.tree_values(n, cb, leaves, sbar, oracle.TV_BR_A)
    br_b = oracle.tree_values(n, cb, leaves, sbar, oracle.TV_BR_B)
    return br_a, br_b, (br_a - br_b) / 2


def last_round_problem(seed):
    deck, roots = synth.last_round_roots(seed)
    gt = oracle.GT(deck, 5, sorted({r.pool for r in roots}))
    f = oracle.FGT(gt, roots)
    return gt, f, f.leaf_utilities()


@pytest.mark.parametrize("seed", [3, 11])
def test_dcfr_converges_to_minimax(seed):
    gt, f, leaves = last_round_problem(seed)
    cb = f.child_begin()
    M = oracle.tree_values(f.n, cb, leaves, None, oracle.TV_MINIMAX)
    c = oracle.CFR(f.n, cb, leaves)
    prev = None
    for T in (10, 90, 900):
        c.run(T)
        sbar = c.sigma_bar()
        br_a, br_b, ex = exploitability(f.n, cb, leaves, sbar)
        v = oracle.tree_values(f.n, cb, leaves, sbar, oracle.TV_EXPECT)
        assert np.all(ex >= -1e-12)
        assert np.all(br_b - 1e-9 <= M) and np.all(M <= br_a + 1e-9)
        assert np.all(np.abs(v - M) <= 2 * ex + 1e-9)
        if prev is not None:
            assert ex.max() <= prev + 1e-12
        prev = ex.max()
    assert prev < 0.05


def test_invariants_and_inherited_difference():
    gt, f, leaves = last_round_problem(3)
    cb = f.child_begin()
    c = oracle.CFR(f.n, cb, leaves)
    c.run(50)
    for l in range(1, 9):
        s = c.get(oracle.CF_SIGMA, l)
        sb = c.get(oracle.CF_SIGMA_BAR, l)
        R = c.get(oracle.CF_R, l)
        assert np.all(s >= 0) and np.all(sb >= 0)
        k = np.diff(cb[l - 1])
        par = np.repeat(np.arange(f.n[l - 1]), k)
        np.testing.assert_allclose(np.bincount(par, s, f.n[l - 1]), 1.0, atol=1e-12)
        np.testing.assert_allclose(np.bincount(par, sb, f.n[l - 1]), 1.0, atol=1e-12)
        forced = (k[par] == 1)
        assert np.all(s[forced] == 1.0) and np.all(R[forced] == 0.0)
    # reach: full reach pi_A * pi_B sums to 1 over each level per root
    for l in range(1, 8):
        ra, rb = c.get(oracle.CF_REACHA, l), c.get(oracle.CF_REACHB, l)
        root = np.arange(f.n[l])
        for up in range(l, 0, -1):
            root = f.get(oracle.FGT_PARENT, up)[root]
        np.testing.assert_allclose(np.bincount(root, ra * rb, f.n[0]), 1.0, atol=1e-12)
    # the seven roots differ only in the inherited point difference, which
    # does not enter the utility: identical subgames, identical results
    sizes = [f.n[l] // f.n[0] for l in range(9)]
    for l in range(1, 9):
        sb = c.get(oracle.CF_SIGMA_BAR, l).reshape(f.n[0], sizes[l])
        assert np.all(sb == sb[0])
    vacc = c.get(oracle.CF_VACC)
    assert np.all(vacc == vacc[0])


def test_two_round_composition():
    # Backward round propagation (CodeSnippet CFR, equation passuputil):
    # solve the last round, pass its root values to the previous round's
    # leaves, solve that round; composed best responses bracket the minimax.
    deck, roots = synth.two_round_root(3)
    gt4 = oracle.GT(deck, 4, [roots[0].pool])
    f4 = oracle.FGT(gt4, roots)
    nxt = f4.get(oracle.FGT_NEXT_ROOTS)
    roots5 = [synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]), int(x["bonus"]))
              for x in nxt]
    gt5 = oracle.GT(deck, 5, sorted({r.pool for r in roots5}))
    f5 = oracle.FGT(gt5, roots5)
    cb5, cb4 = f5.child_begin(), f4.child_begin()
    leaf5 = f5.leaf_utilities()
    M5 = oracle.tree_values(f5.n, cb5, leaf5, None, oracle.TV_MINIMAX)
    M4 = oracle.tree_values(f4.n, cb4, f4.leaf_utilities(M5), None, oracle.TV_MINIMAX)
    prev = None
    c5 = oracle.CFR(f5.n, cb5, leaf5)
    for T in (20, 180):
        c5.run(T)
        V5 = c5.get(oracle.CF_VACC) / (c5.t - 1)
        c4 = oracle.CFR(f4.n, cb4, f4.leaf_utilities(V5))
        c4.run(c5.t - 1)
        s5, s4 = c5.sigma_bar(), c4.sigma_bar()
        bra5 = oracle.tree_values(f5.n, cb5, leaf5, s5, oracle.TV_BR_A)
        brb5 = oracle.tree_values(f5.n, cb5, leaf5, s5, oracle.TV_BR_B)
        bra4 = oracle.tree_values(f4.n, cb4, f4.leaf_utilities(bra5), s4, oracle.TV_BR_A)
        brb4 = oracle.tree_values(f4.n, cb4, f4.leaf_utilities(brb5), s4, oracle.TV_BR_B)
        assert brb4[0] - 1e-9 <= M4[0] <= bra4[0] + 1e-9
        ex = (bra4[0] - brb4[0]) / 2
        if prev is not None:
            assert ex <= prev + 1e-12
        prev = ex
    assert prev < 0.1


def test_snippet_tol_flag_by_hand():
    # OR_SNIPPET_TOL: the discount's sign test is R >= 1e-5 (the snippet's
    # TOL) instead of R > 0.  The game of the hand-worked DCFR run with every
    # leaf scaled by s = 2^-20, so every regret is below 1e-5: regret matching
    # is scale-free, so sigma is as before, and the first discount that
    # differs is at t=3 (alpha and beta discounts are both 1/2 at t=2), where
    # the positive regrets (1/2 s, 1/2 s, 1/4 s) are halved instead of
    # multiplied by c = 2^1.5/(2^1.5+1); no new regret is added to them there.
    s = 2.0 ** -20
    n, cb, leaves = padded_tree([2, 2], [3 * s, -1 * s, 0, 2 * s])
    cc = 2 ** 1.5 / (2 ** 1.5 + 1)
    plain = oracle.CFR(n, cb, leaves)
    plain.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE))
    np.testing.assert_allclose(plain.get(oracle.CF_R, 1), [-1.25 * s, cc / 2 * s], rtol=1e-14, atol=0)
    c = oracle.CFR(n, cb, leaves)
    c.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE, flags=oracle.SNIPPET_TOL))
    np.testing.assert_allclose(c.get(oracle.CF_R, 1), [-1.25 * s, 0.25 * s], rtol=1e-14, atol=0)
    np.testing.assert_allclose(c.get(oracle.CF_R, 2), [-1.25 * s, 0.25 * s, 0.125 * s, -2.625 * s],
                               rtol=1e-14, atol=0)
    np.testing.assert_array_equal(c.get(oracle.CF_SIGMA, 1), plain.get(oracle.CF_SIGMA, 1))
    # unscaled, every positive regret is far above 1e-5: the flag changes nothing
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    a, b = oracle.CFR(n, cb, leaves), oracle.CFR(n, cb, leaves)
    a.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE))
    b.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE, flags=oracle.SNIPPET_TOL))
    for l in (1, 2):
        np.testing.assert_array_equal(a.get(oracle.CF_R, l), b.get(oracle.CF_R, l))


def test_snippet_avg_flag_by_hand():
    # OR_SNIPPET_AVG: Sbar <- (1 - 1/t^2) Sbar + pi_p sigma^t sigma^{t+1}.
    # Same game and regrets as the hand-worked DCFR run, so the strategies
    # are sigma^1 uniform, sigma^2 = root (1/2,1/2), a1:b (0,1), a2:b (1,0),
    # sigma^3 = sigma^4 = root (0,1), a1:b (0,1), a2:b (1,0); weights 0, 3/4,
    # 8/9; both movers' own reach at their nodes is 1:
    #   root: t=1 (1/4,1/4); t=2 (3/16, 3/16+1/2); t=3 (1/6, 11/18+1)
    #         -> average (3/32, 29/32)
    #   a1:b: t=1 (0, 1/2 * 1); t=2 (0, 3/8+1); t=3 (0, 11/9+1);  a2:b mirrored.
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    c = oracle.CFR(n, cb, leaves)
    c.run(3, oracle.Params(rm_mode=oracle.RM_POSITIVE, flags=oracle.SNIPPET_AVG))
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 1), [1 / 6, 29 / 18], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SBAR, 2), [0, 20 / 9, 20 / 9, 0], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 1), [3 / 32, 29 / 32], atol=1e-14)
    np.testing.assert_allclose(c.get(oracle.CF_SIGMA_BAR, 2), [0, 1, 1, 0], atol=1e-14)
    # the averaging does not feed back: regrets equal the plain run's
    cc = 2 ** 1.5 / (2 ** 1.5 + 1)
    np.testing.assert_allclose(c.get(oracle.CF_R, 2), [-1.25, cc / 2, cc / 4, -2.625], atol=1e-14)


def test_snippet_flags_need_dcfr():
    n, cb, leaves = padded_tree([2, 2], [3, -1, 0, 2])
    c = oracle.CFR(n, cb, leaves)
    with pytest.raises(oracle.OracleError):
        c.run(1, oracle.Params(variant=oracle.CFR_PLUS, flags=oracle.SNIPPET_AVG))
    with pytest.raises(oracle.OracleError):
        c.run(1, oracle.Params(flags=8))
