"""Device views of the tree handles (no copy) equal the arrays the read calls
copy out, and the plain SGD step equals its FP32 definition."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_np
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def dev_copy(ptr, nbytes, dtype):
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    out = np.empty(nbytes // np.dtype(dtype).itemsize, dtype)
    assert hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0  # device to host
    return out


def test_views_equal_read_copies():
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(3)
    s = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F32, keep_gt=True)
    torch.cuda.synchronize()
    for rr in s.rounds:
        v = pa.fgt_view(rr.fgt)
        assert v.round == rr.round
        for l in range(9):
            assert v.n[l] == rr.fgt.n[l]
            for field, arr in ((pa.FGT_GT, v.gt), (pa.FGT_SID, v.sid)):
                got = dev_copy(arr[l], 4 * v.n[l], np.int32)
                assert np.array_equal(got, rr.fgt.read(field, l)), (field, l)
            if l >= 1:
                assert np.array_equal(dev_copy(v.parent[l], 4 * v.n[l], np.int32),
                                      rr.fgt.read(pa.FGT_PARENT, l))
            if l < 8:
                assert np.array_equal(dev_copy(v.child_begin[l], 4 * (v.n[l] + 1), np.int32),
                                      rr.fgt.read(pa.FGT_CHILD_BEGIN, l))
        assert np.array_equal(dev_copy(v.leaf_base, 2 * v.n[8], np.int16),
                              rr.fgt.read(pa.FGT_LEAF_BASE))
        assert np.array_equal(dev_copy(v.score_tab, 4 * v.n_scores, np.int8),
                              rr.fgt.read(pa.FGT_SCORE_TAB).reshape(-1))
        if v.next_roots:
            assert np.array_equal(dev_copy(v.link, 4 * v.n[8], np.int32), rr.fgt.read(pa.FGT_LINK))
            assert np.array_equal(dev_copy(v.next_roots, 16 * v.n_next, np.uint8),
                                  rr.fgt.read(pa.FGT_NEXT_ROOTS).view(np.uint8))
        else:
            assert rr.round == 5 and not v.link
        g = pa.gt_view(rr.gt)
        for l in range(9):
            assert np.array_equal(dev_copy(g.pool[l], 8 * g.n[l], np.uint64),
                                  rr.gt.read(pa.GT_POOL, l))
            if l < 8:
                assert np.array_equal(dev_copy(g.child_begin[l], 4 * (g.n[l] + 1), np.int32),
                                      rr.gt.read(pa.GT_CHILD_BEGIN, l))
    s.free()


def test_sgd_step_matches_definition():
    pa = require_gpu()
    import torch
    rng = np.random.default_rng(5)
    n = 100_003
    w = rng.normal(0, 1, n).astype(np.float32)
    g = rng.normal(0, 1, n).astype(np.float32)
    lr = np.float32(0.0375)
    dw, dg = torch.from_numpy(w).cuda(), torch.from_numpy(g).cuda()
    wb = torch.empty(n, dtype=torch.int16, device="cuda")
    pa.sgd_step(dw, dg, wb, float(lr))
    torch.cuda.synchronize()
    want = w - lr * g  # float32 product, then float32 difference
    assert np.array_equal(to_np(dw), want)
    assert np.array_equal(to_np(wb).view(np.uint16), omlp.bf16_bits(want))
