"""Full six-round solves on the GPU (rounds 1..6 built forward, solved
backward with root values passed between rounds, equation passuputil).

* The paper's worked deck (table tab:deck9_exp): after DCFR the average
  strategy of Alex's first move must sit on the printed support, and each
  of Bob's replies on the printed capture(s).
* Seeded full games at their real size, FP64 state: seed 1 (3.4e7 nodes)
  and seed 40 (8.5e8 nodes, the full-game benchmark's deal and the largest
  among seeds 1-64).  Properties that hold at any size (the composed best
  responses bracket the value, small exploitability; for seed 1 also every
  average-strategy row sums to 1), and element-by-element parity with the
  oracle on sampled subgames the oracle can solve alone: roots of the last two rounds that the game
  reaches (found by following seeded branches of the oracle's own unfolding
  from the initial deal).  A root's subgame is independent of the other
  roots of its round, so its slice of the GPU's forest must equal the
  oracle's solve of that root by itself.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import card_index, cards_of, read_rows
from gpu_common import (assert_sigma_bar_up_to_ties, oracle_rounds, oracle_solve, require_gpu,
                        roots_from_array, tie_groups, to_np)

pytestmark = pytest.mark.gpu

ITERS = 200
TOL64 = 1e-9


def _first_turn_rows(golden_dir):
    rows = read_rows(os.path.join(golden_dir, "deck9_first_turn.txt"))
    alex = {card_index(r[1]): float(r[4]) for r in rows if r[0] == "A"}
    bob = {}
    for r in rows:
        if r[0] == "B":
            bob.setdefault(card_index(r[1]), {})[(card_index(r[2]), synth.mask_of(cards_of(r[3])))] = float(r[4])
    return alex, bob


def test_worked_deck_first_turn_support(golden_dir):
    pa = require_gpu()
    import torch
    deck = synth.DECK9
    roots = [synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)]
    print("[full game] worked deck, 6 rounds, 300 DCFR iterations per round", flush=True)
    s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F32, keep_gt=True)
    s.solve(300)
    torch.cuda.synchronize()
    rr = s.rounds[0]
    assert abs(to_np(rr.V)[0] - 14.0) < 0.05  # the game value (oracle minimax pin)
    alex, bob = _first_turn_rows(golden_dir)
    sb1, sb2 = to_np(rr.state.sigma_bar[1]), to_np(rr.state.sigma_bar[2])
    a1 = rr.gt.read(pa.GT_ACT_CARD, 1)
    a2, c2 = rr.gt.read(pa.GT_ACT_CARD, 2), rr.gt.read(pa.GT_ACT_CAP, 2)
    cb = rr.gt.read(pa.GT_CHILD_BEGIN, 1)
    assert sum(sb1[i] for i, c in enumerate(a1) if alex[int(c)] > 0) > 0.98
    for i, c in enumerate(a1):
        on = sum(sb2[q] for q in range(cb[i], cb[i + 1]) if bob[int(c)][(int(a2[q]), int(c2[q]))] > 0)
        assert on > 0.98, (int(c), on)
    s.free()


def _sample_reached_roots(deck, rng, per_round=3):
    """Roots of rounds 5 and 6 that the full game from the initial deal
    reaches: follow ``per_round`` seeded next-round roots per round through
    the oracle's unfolding.  Returns {round index: [Root]}."""
    cur = [synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)]
    out = {}
    for r in range(0, 6):
        if r >= 4:
            out[r] = list(cur)
        if r == 5:
            break
        gt = oracle.GT(deck, r, sorted({x.pool for x in cur}))
        f = oracle.FGT(gt, cur)
        nxt = roots_from_array(f.get(oracle.FGT_NEXT_ROOTS))
        idx = sorted(rng.choice(len(nxt), size=min(per_round, len(nxt)), replace=False))
        cur = [nxt[i] for i in idx]
    return out


def _subtree_slices(child_begins, k):
    """[lo, hi) of root k's subtree on every level of a root-major forest."""
    lo, hi = k, k + 1
    sl = [(lo, hi)]
    for cb in child_begins:
        lo, hi = int(cb[lo]), int(cb[hi])
        sl.append((lo, hi))
    return sl


@pytest.mark.parametrize("seed,min_nodes,iters", [(1, 3e7, ITERS), (40, 8e8, 100)])
def test_full_game_at_scale_sampled_parity(seed, min_nodes, iters):
    pa = require_gpu()
    import torch
    deck, roots = synth.full_game_root(seed)
    print(f"[full game] seed {seed}, FP64 state, {iters} DCFR iterations per round", flush=True)
    s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F64)
    s.solve(iters)
    torch.cuda.synchronize()
    sizes = [sum(n) for n in s.sizes()]
    print(f"[full game] round sizes {sizes}", flush=True)
    assert sum(sizes) > min_nodes

    # properties at full size (the per-row simplex check reads every level)
    for rr in (s.rounds if sum(sizes) < 1e8 else []):
        for l in range(8):
            par = torch.from_numpy(rr.fgt.read(pa.FGT_PARENT, l + 1).astype(np.int64)).cuda()
            tot = torch.zeros(rr.fgt.n[l], dtype=torch.float64, device="cuda")
            tot.index_add_(0, par, rr.state.sigma_bar[l + 1].double())
            assert float((tot - 1).abs().max()) < 1e-12, (rr.round, l)
    bra, brb, v = (float(x[0]) for x in s.exploitability())
    print(f"[full game] BR_A {bra:.6f} v {v:.6f} BR_B {brb:.6f}", flush=True)
    assert bra >= v - 1e-9 and v >= brb - 1e-9
    assert (bra - brb) / 2 < 0.1

    # sampled parity against the oracle
    rng = np.random.default_rng(seed)
    sample = _sample_reached_roots(deck, rng)
    for r, picks in sample.items():
        rr = s.rounds[r]
        gpu_roots = s.rounds[r - 1].fgt.read(pa.FGT_NEXT_ROOTS)
        cbs = [rr.fgt.read(pa.FGT_CHILD_BEGIN, l) for l in range(8)]
        V = to_np(rr.V)
        for root in picks:
            k = np.nonzero((gpu_roots["pool"] == root.pool) & (gpu_roots["ca"] == root.ca)
                           & (gpu_roots["cb"] == root.cb) & (gpu_roots["d"] == root.d)
                           & (gpu_roots["bonus"] == root.bonus))[0]
            assert len(k) == 1, root
            k = int(k[0])
            orr = oracle_rounds(deck, r, [root])
            res = oracle_solve(orr, iters)
            c0 = res[0][0]
            osb = c0.sigma_bar()
            sl = _subtree_slices(cbs, k)
            for l in range(1, 9):
                lo, hi = sl[l]
                assert hi - lo == orr[0][1].n[l], (r, k, l)
                np.testing.assert_allclose(to_np(rr.state.sigma_bar[l][lo:hi]), osb[l], rtol=0,
                                           atol=TOL64, err_msg=f"round {r} root {k} level {l}")
            assert abs(V[k] - res[0][2][0]) < TOL64, (r, k, V[k], res[0][2][0])
            print(f"[full game] round {r} root {k}: {sum(orr[0][1].n)} nodes match", flush=True)
    s.free()


def test_full_game_fp32_sampled_parity_up_to_ties():
    # The benchmark's configuration (deal 40, FP32 state, 1000 iterations per
    # round, the default schedule): sampled roots of rounds 5 and 6 against
    # the oracle's solve of each root alone -- how often each untied action
    # and each tie group (equally good actions under one parent) is played
    # within 1e-5, root values within 1e-5.
    pa = require_gpu()
    import torch
    deck, roots = synth.full_game_root(40)
    iters = 1000
    print(f"[full game] seed 40, FP32 state, {iters} DCFR iterations per round", flush=True)
    s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F32)
    s.solve(iters)
    torch.cuda.synchronize()
    rng = np.random.default_rng(41)
    sample = _sample_reached_roots(deck, rng, per_round=3)
    for r, picks in sample.items():
        rr = s.rounds[r]
        gpu_roots = s.rounds[r - 1].fgt.read(pa.FGT_NEXT_ROOTS)
        cbs = [rr.fgt.read(pa.FGT_CHILD_BEGIN, l) for l in range(8)]
        V = to_np(rr.V)
        for root in picks:
            k = np.nonzero((gpu_roots["pool"] == root.pool) & (gpu_roots["ca"] == root.ca)
                           & (gpu_roots["cb"] == root.cb) & (gpu_roots["d"] == root.d)
                           & (gpu_roots["bonus"] == root.bonus))[0]
            assert len(k) == 1, root
            k = int(k[0])
            orr = oracle_rounds(deck, r, [root])
            res = oracle_solve(orr, iters)
            c0, leaf0, V0 = res[0]
            sl = _subtree_slices(cbs, k)
            gsb = [None] + [to_np(rr.state.sigma_bar[l][sl[l][0]:sl[l][1]]) for l in range(1, 9)]
            tied, total, big = assert_sigma_bar_up_to_ties(
                gsb, c0.sigma_bar(), tie_groups(orr[0][1], leaf0), orr[0][1].child_begin(), 1e-5,
                (r, k))
            assert abs(V[k] - V0[0]) <= 1e-5, (r, k, V[k], V0[0])
            print(f"[full game] fp32 round {r} root {k}: {total} actions ({tied} tied) match; "
                  f"largest difference at reach >= 0.5: {big:.2e}", flush=True)
    s.free()
