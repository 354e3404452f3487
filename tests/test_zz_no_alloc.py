"""pasur_tree_values_noalloc (tree values with its level buffers in a fixed
device array, no allocation) against pasur_tree_values, through the C ABI:
two calls in a row on the same GPU, the second on a smaller tree, every
mode; and its capacity limit."""
import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_np

pytestmark = pytest.mark.gpu


def test_noalloc_tree_values_equal_the_allocating_call():
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(1)
    print("[noalloc] two-round subgame of deal 1, FP32 and FP64 state", flush=True)
    for dtype in (pa.PASUR_F32, pa.PASUR_F64):
        s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        s.solve(60)
        torch.cuda.synchronize()
        # round 6 (56 roots, levels up to 44,521 nodes) first, then round 5
        # (one root, 1,044 nodes): the second call reuses the array
        V = None
        for rr in (s.rounds[1], s.rounds[0]):
            assert rr.fgt.n[0] < 60
            leaf = torch.empty(rr.fgt.n[8], dtype=torch.float64, device="cuda")
            pa.leaf_utilities(rr.fgt, V, pa.PASUR_F64, leaf)
            for mode in (pa.TV_EXPECT, pa.TV_BR_A, pa.TV_BR_B, pa.TV_MINIMAX):
                sg = None if mode == pa.TV_MINIMAX else rr.state.sigma_bar
                a = torch.full((rr.fgt.n[0],), float("nan"), dtype=torch.float64, device="cuda")
                b = torch.full((rr.fgt.n[0],), float("nan"), dtype=torch.float64, device="cuda")
                pa.tree_values(rr.fgt, leaf, dtype, sg, mode, a)
                pa.tree_values_noalloc(rr.fgt, leaf, dtype, sg, mode, b)
                torch.cuda.synchronize()
                x, y = to_np(a), to_np(b)
                assert np.isfinite(y).all()
                assert np.array_equal(x, y), (rr.round, mode)
            V = rr.V
        s.free()


def test_noalloc_rejects_levels_beyond_its_array():
    pa = require_gpu()
    deck, roots = synth.full_game_root(40)
    print("[noalloc] full game of deal 40: round 4 has a level of 3.2e6 nodes", flush=True)
    s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F32)
    import torch
    rr = s.rounds[3]
    assert max(rr.fgt.n[:8]) > (1 << 21)
    leaf = torch.zeros(rr.fgt.n[8], dtype=torch.float64, device="cuda")
    out = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
    with pytest.raises(pa.PasurError, match="exceeds"):
        pa.tree_values_noalloc(rr.fgt, leaf, pa.PASUR_F32, None, pa.TV_MINIMAX, out)
    s.free()
