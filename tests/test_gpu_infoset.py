"""Infoset rows on the GPU (pasur_infoset_rows) against the oracle, byte for
byte: every level of three rounds (last, middle, first), a ragged unsorted
edge list, the network-input format, and sampled roots of the full game of
deal 1 at its real size (each root's slice of a round of thousands of roots
against the oracle's tree of that root alone)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import require_gpu, roots_from_array, to_np
from oracle import infoset as inf

pytestmark = pytest.mark.gpu


def _case(seed, rnd):
    if rnd == 5:
        return synth.last_round_roots(seed)
    return synth.subgame_roots(seed, rnd)


@pytest.mark.parametrize("seed,rnd", [(4, 5), (2, 4), (7, 0)])
def test_rows_match_oracle(seed, rnd):
    pa = require_gpu()
    import torch
    deck, roots = _case(seed, rnd)
    s = pa.SubgameSolver(deck, rnd, roots, keep_gt=True)
    rr = s.rounds[0]
    gt = oracle.GT(deck, rnd, sorted({x.pool for x in roots}))
    f = oracle.FGT(gt, roots)
    assert list(rr.fgt.n) == list(f.n)
    rng = np.random.default_rng(seed)
    for level in range(1, 9):
        n = rr.fgt.n[level]
        want = inf.rows(gt, f, level)
        out = torch.empty((n, pa.INFOSET_WIDTH), dtype=torch.int8, device="cuda")
        pa.infoset_rows(rr.gt, rr.fgt, level, None, n, out)
        got = to_np(out)
        assert np.array_equal(got, want), (level, np.argwhere(got != want)[:4])
        # an unsorted edge list with repeats and a ragged length
        m = int(rng.integers(1, 2 * n + 3))
        idx = rng.integers(0, n, m).astype(np.int32)
        d_idx = torch.from_numpy(idx).cuda()
        out2 = torch.empty((m, pa.INFOSET_WIDTH), dtype=torch.int8, device="cuda")
        pa.infoset_rows(rr.gt, rr.fgt, level, d_idx, m, out2)
        assert np.array_equal(to_np(out2), want[idx])
        # network input: row / 128 in BF16 (exact), zeros after column 57
        X = torch.empty((n, 192), dtype=torch.int16, device="cuda")
        pa.infoset_rows(rr.gt, rr.fgt, level, None, n, X, pa.INFOSET_MLP)
        Xf = X.view(torch.bfloat16).float().cpu().numpy()
        assert np.array_equal(Xf[:, :58] * 128.0, want.astype(np.float32))
        assert not Xf[:, 58:].any()
    print(f"[infoset] round {rnd} seed {seed}: {sum(f.n[1:])} rows identical", flush=True)
    s.free()


def _slices(child_begins, k):
    lo, hi = k, k + 1
    out = [(lo, hi)]
    for cb in child_begins:
        lo, hi = int(cb[lo]), int(cb[hi])
        out.append((lo, hi))
    return out


def test_full_game_sampled_roots():
    pa = require_gpu()
    import torch
    deck, roots = synth.full_game_root(1)
    s = pa.SubgameSolver(deck, 0, roots, keep_gt=True)
    rng = np.random.default_rng(11)
    checked = 0
    for r in (3, 5):
        rr = s.rounds[r]
        cbs = [rr.fgt.read(pa.FGT_CHILD_BEGIN, l) for l in range(8)]
        round_roots = roots_from_array(s.rounds[r - 1].fgt.read(pa.FGT_NEXT_ROOTS))
        assert len(round_roots) == rr.fgt.n[0]
        for k in rng.choice(len(round_roots), 3, replace=False):
            k = int(k)
            root = round_roots[k]
            gt = oracle.GT(deck, r, [root.pool])
            f = oracle.FGT(gt, [root])
            sl = _slices(cbs, k)
            for level in range(1, 9):
                lo, hi = sl[level]
                assert hi - lo == f.n[level]
                idx = torch.arange(lo, hi, dtype=torch.int32, device="cuda")
                out = torch.empty((hi - lo, pa.INFOSET_WIDTH), dtype=torch.int8, device="cuda")
                pa.infoset_rows(rr.gt, rr.fgt, level, idx, hi - lo, out)
                assert np.array_equal(to_np(out), inf.rows(gt, f, level)), (r, k, level)
                checked += hi - lo
    print(f"[infoset] full game seed 1: {checked} sampled rows identical", flush=True)
    s.free()


def test_models_on_infoset_rows():
    """The strategy models on infoset rows run end to end: the network
    trains on them (loss falls), the tree model's data holds each sampled
    decision's full average strategy (100 per parent), and the profiles both
    models predict are valid (finite, non-negative exploitability)."""
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    probs = [synth.two_round_root(s) for s in range(50000, 50006)]
    units = learn.training_units(probs, 200, 150, features="infoset")
    m = learn.WarmStartMLP(0)
    hist = learn.train(m, units, 4)
    assert hist[-1][0] < hist[0][0]
    rows, tgt, grp = learn.infoset_dataset(probs[:3], 200, 100)
    assert rows.dtype == np.int8 and rows.shape[1] == 58 and len(rows) == len(tgt) == len(grp)
    np.testing.assert_allclose(np.bincount(grp, weights=tgt), 100.0, atol=1e-3)
    tree = learn.fit_tree_model(rows, tgt, max_iter=20)
    deck, roots = synth.two_round_root(50010)
    ex = [learn.initial_profile_exploitability(deck, roots, None),
          learn.initial_profile_exploitability(deck, roots, m, "infoset"),
          learn.tree_profile_exploitability(deck, roots, tree)]
    print(f"[infoset] starting-profile exploitability uniform / network / tree: {ex}", flush=True)
    assert all(np.isfinite(ex)) and min(ex) >= 0


def test_empty_edge_list():
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(3)
    s = pa.SubgameSolver(deck, 5, roots, keep_gt=True)
    rr = s.rounds[0]
    idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.full((1, pa.INFOSET_WIDTH), 9, dtype=torch.int8, device="cuda")
    pa.infoset_rows(rr.gt, rr.fgt, 3, idx, 0, out)
    torch.cuda.synchronize()
    assert (to_np(out) == 9).all()
    s.free()
