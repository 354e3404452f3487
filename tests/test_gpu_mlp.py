"""GPU parity of the learned part: the BF16 MFMA GEMM, the MLP forward and
backward passes, the loss and the features, against the FP64 oracle with
bfloat16 rounding at the same points (oracle/mlp.py).  Every comparison is
element by element: products of bfloat16 values are exact in FP32, so a
product differs from the FP64 sum only by FP32 accumulation (2e-6 of the sum
of |terms|); a value rounded to bfloat16 (hidden activation or gradient) may
differ from the oracle's only where its FP64 value lies within that band of a
rounding point, and that allowance is carried through the later products
(tests/mlp_bounds.py)."""
import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_np
from mlp_bounds import backward_bounds, forward_bounds, layer_bounds
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def bf16_tensor(x):
    import torch
    return torch.from_numpy(omlp.bf16_bits(x).view(np.int16).copy()).cuda()


def from_bf16(t):
    u = to_np(t).view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,transA,transB", [(100, 70, 45, False, False), (64, 64, 32, False, False),
                                                  (33, 257, 160, False, True), (160, 256, 1000, True, False),
                                                  (1, 2, 256, False, False), (515, 2, 256, False, False),
                                                  # 128x128 tiles: ragged, both operand orientations, long K
                                                  (300, 200, 100, False, False), (257, 384, 64, True, True),
                                                  (1024, 256, 192, False, False), (130, 129, 33, False, True),
                                                  (256, 256, 2048, True, False)])
def test_gemm_matches_fp64(M, N, K, transA, transB):
    pa = require_gpu()
    import torch
    rng = np.random.default_rng(M * 7 + N)
    A = omlp.bf16_round(rng.normal(0, 1, (K, M) if transA else (M, K)))
    B = omlp.bf16_round(rng.normal(0, 1, (N, K) if transB else (K, N)))
    opA = A.T if transA else A
    opB = B.T if transB else B
    want = opA @ opB
    bound = np.abs(opA) @ np.abs(opB) * 2e-6 + 1e-30
    dA, dB = bf16_tensor(A), bf16_tensor(B)
    C = torch.empty((M, N), dtype=torch.float32, device="cuda")
    sar, sac = (1, M) if transA else (K, 1)
    sbr, sbc = (1, K) if transB else (N, 1)
    print(f"[gemm] M={M} N={N} K={K} transA={transA} transB={transB}", flush=True)
    pa.gemm_bf16(M, N, K, dA, sar, sac, dB, sbr, sbc, Cf=C)
    torch.cuda.synchronize()
    assert np.all(np.abs(to_np(C) - want) <= bound)


def make_problem(seed, n_par=300):
    rng = np.random.default_rng(seed)
    fan = rng.integers(1, 6, n_par)
    seg = np.concatenate([[0], np.cumsum(fan)]).astype(np.int32)
    M = int(seg[-1])
    X = rng.integers(0, 2, (M, omlp.N_IN)).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    tsig = np.concatenate([rng.dirichlet(np.ones(k)) for k in fan]).astype(np.float32)
    tval = rng.normal(0, 3, M).astype(np.float32)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    return X, seg, tsig, tval, W


# about 900 rows (one row chunk per weight gradient, ragged in its last K
# step) and about 6000 (six chunks, the last ragged); with X and W2 8 bytes
# off a 16-byte boundary the forward and dW1 take the GEMM path (element-wise
# operand loads) instead of the fused forward and the whole-gradient kernel
@pytest.mark.parametrize("n_par,x_off", [(300, 0), (2000, 0), (300, 4)])
def test_mlp_forward_backward_match_oracle(n_par, x_off):
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    X, seg, tsig, tval, W = make_problem(3, n_par)
    M = X.shape[0]
    print(f"[mlp] forward/backward M={M} x_off={x_off}", flush=True)
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    # the host-side bfloat16 conversion of the binding equals the oracle's
    for k in (0, 2, 4):
        assert np.array_equal(to_np(model.bf[k]).view(np.uint16), omlp.bf16_bits(W[k]))
    dX = bf16_tensor(X)
    if x_off:
        buf = torch.zeros(dX.numel() + x_off, dtype=dX.dtype, device="cuda")
        buf[x_off:] = dX.flatten()
        dX = buf[x_off:].view(dX.shape)
        assert dX.data_ptr() % 16 == 2 * x_off
    b = model._buffers(M)
    w = model.weights()
    if x_off:
        w2 = model.bf[2].view(torch.int16)
        wbuf = torch.zeros(w2.numel() + x_off, dtype=w2.dtype, device="cuda")
        wbuf[x_off:] = w2.flatten()
        w.W2 = wbuf[x_off:].data_ptr()
        assert w.W2 % 16 == 2 * x_off
    pa.mlp_forward(w, dX, M, b["H1"], b["H2"], b["Y"])
    dseg = torch.from_numpy(seg).cuda()
    dts, dtv = torch.from_numpy(tsig).cuda(), torch.from_numpy(tval).cuda()
    loss = torch.empty((len(seg) - 1, 2), dtype=torch.float32, device="cuda")
    pa.mlp_loss(b["Y"], dts, dtv, dseg, len(seg) - 1, M, 0.5, b["dY"], loss)
    pa.mlp_backward(w, dX, b["H1"], b["H2"], b["dY"], M, model.grads())
    torch.cuda.synchronize()
    H1g, H2g = from_bf16(b["H1"][:M]), from_bf16(b["H2"][:M])
    Yg = to_np(b["Y"][:M]).astype(np.float64)
    # each layer on the GPU's own input: equal to the oracle's layer except
    # within the rounding allowance (Y: FP32 accumulation only)
    for name, got, (want, bound) in (("H1", H1g, layer_bounds(X, W[0], W[1], True)),
                                     ("H2", H2g, layer_bounds(H1g, W[2], W[3], True)),
                                     ("Y", Yg, layer_bounds(H2g, W[4], W[5], False))):
        assert np.all(np.abs(got - want) <= bound), name
    # and the whole pass against the oracle's, allowances carried through
    (H1o, H2o, Yo), (A1, A2, bY) = forward_bounds(W, X)
    assert np.all(np.abs(H2g - H2o) <= A2) and np.all(np.abs(Yg - Yo) <= bY)
    assert np.mean(H1g != H1o) < 1e-3 and np.mean(H2g != H2o) < 1e-3
    # loss gradient from the GPU's Y; weight gradients from its activations
    lo, dYo = omlp.loss_and_dY(Yg, seg, tsig.astype(np.float64), tval.astype(np.float64), 0.5)
    dYg = to_np(b["dY"][:M]).astype(np.float64)
    assert np.abs(dYg - dYo).max() <= 1e-6 * (np.abs(dYo).max() + 1e-12) + 1e-9
    assert float(loss.sum()) == pytest.approx(lo, rel=1e-4)
    check_gradients(model, W, X, H1g, H2g, dYg)


def check_gradients(model, W, X, H1g, H2g, dY):
    go = omlp.backward(W, X, H1g, H2g, dY, bf16=True)
    bounds = backward_bounds(W, X, H1g, H2g, dY)
    names = ("dW1", "db1", "dW2", "db2", "dW3", "db3")
    for name, gg, gref, bound in zip(names, model.g, go, bounds):
        gg = to_np(gg).astype(np.float64).reshape(gref.shape)
        assert np.all(np.abs(gg - gref) <= bound + 1e-30), (name, float(np.max(np.abs(gg - gref) - bound)))


def test_features_encode_state_and_score():
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(2)
    s = pa.SubgameSolver(deck, 5, roots, keep_gt=True)
    rr = s.rounds[0]
    l = 3
    n = rr.fgt.n[l]
    X = torch.empty((n, omlp.N_IN), dtype=torch.int16, device="cuda")
    pa.edge_features(rr.gt, rr.fgt, l, None, n, X)
    torch.cuda.synchronize()
    Xf = from_bf16(X)
    g = rr.fgt.read(pa.FGT_GT, l)
    sid = rr.fgt.read(pa.FGT_SID, l)
    tab = rr.fgt.read(pa.FGT_SCORE_TAB)
    pool = rr.gt.read(pa.GT_POOL, l)
    hands = rr.gt.read(pa.GT_HANDS, l)
    rs = rr.gt.read(pa.GT_RS, l)
    a, b = synth.round_hands(deck, 5)
    for i in range(0, n, max(1, n // 50)):
        t = g[i]
        ha = [a[k] for k in range(4) if (hands[t] >> k) & 1]
        hb = [b[k] for k in range(4) if (hands[t] >> (4 + k)) & 1]
        want = np.zeros(omlp.N_IN)
        want[ha] = 1
        want[[52 + c for c in hb]] = 1
        want[[104 + c for c in range(52) if (int(pool[t]) >> c) & 1]] = 1
        ca, cb, d, bo = tab[sid[i]]
        want[156:160] = omlp.bf16_round([ca / 7, cb / 7, d / 16, {0: 0, 1: 1, 2: -1}[int(bo)]])
        acl, bcl, lp, apt, asr, bpt, bsr = (int(v) for v in rs[t][:7])
        want[160:167] = omlp.bf16_round([acl / 13, bcl / 13, {0: 0, 1: 1, 2: -1}[lp],
                                         apt / 10, asr, bpt / 10, bsr])
        want[167 + l] = 1
        assert np.array_equal(Xf[i], want), i
    s.free()


@pytest.mark.parametrize("M", [1, 127, 128, 129, 1000, 4099])
def test_mlp_infer_matches_oracle_and_forward(M):
    """The fused inference kernel against the oracle's BF16-rounded forward
    pass (ragged row counts around the 128-row tile) and against the
    forward pass (two GEMMs and the output layer) of the same weights."""
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    rng = np.random.default_rng(M)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    X = rng.integers(0, 2, (M, omlp.N_IN)).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    dX = bf16_tensor(X)
    Y = torch.empty((M, 2), dtype=torch.float32, device="cuda")
    pa.mlp_infer(model.weights(), dX, M, Y)
    # with the model's cached transposed weights: the same result
    Y2 = torch.empty((M, 2), dtype=torch.float32, device="cuda")
    pa.mlp_infer(model.infer_weights(), dX, M, Y2)
    b = model._buffers(M)
    pa.mlp_forward(model.weights(), dX, M, b["H1"], b["H2"], b["Y"])
    torch.cuda.synchronize()
    (_, _, Yo), (_, _, bY) = forward_bounds(W, X)
    Yi = to_np(Y).astype(np.float64)
    assert np.array_equal(Yi, to_np(Y2).astype(np.float64))
    Yf = to_np(b["Y"][:M]).astype(np.float64)
    # both within the element-wise bound of the oracle's forward pass
    assert np.all(np.abs(Yi - Yo) <= bY)
    assert np.all(np.abs(Yf - Yo) <= bY)


def test_forward_output_layer_both_paths():
    """The forward pass's output layer as per-row dot products (H2 16-byte
    aligned) and as a GEMM (H2 8 bytes off): the same hidden activations, Y
    equal up to FP32 accumulation order, both near the oracle."""
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    X, seg, tsig, tval, W = make_problem(5, 400)
    M = X.shape[0]
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    dX = bf16_tensor(X)
    w = model.weights()
    H1 = torch.empty((M, 256), dtype=torch.int16, device="cuda")
    H2 = torch.empty((M, 256), dtype=torch.int16, device="cuda")
    H2off = torch.empty(M * 256 + 4, dtype=torch.int16, device="cuda")[4:]
    assert H2.data_ptr() % 16 == 0 and H2off.data_ptr() % 16 == 8
    Ya = torch.empty((M, 2), dtype=torch.float32, device="cuda")
    Yb = torch.empty((M, 2), dtype=torch.float32, device="cuda")
    pa.mlp_forward(w, dX, M, H1, H2, Ya)
    pa.mlp_forward(w, dX, M, H1, H2off, Yb)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(H2), to_np(H2off).reshape(M, 256))
    Yo, bY = layer_bounds(from_bf16(H2), W[4], W[5], False)
    Ya, Yb = to_np(Ya).astype(np.float64), to_np(Yb).astype(np.float64)
    # each side within 2e-6 of the sum of |terms| of the exact result (FP32
    # accumulation), so within twice that of each other
    terms = np.abs(from_bf16(H2)) @ np.abs(omlp.bf16_round(W[4])) + np.abs(W[5])
    assert np.all(np.abs(Ya - Yb) <= 4e-6 * terms + 1e-30)
    assert np.all(np.abs(Ya - Yo) <= bY)


# one row; 33 rows (one chunk of two K steps, the second ragged); and row
# counts just past the weight-gradient chunk size (1025 rows: chunks of 544
# and 481; 4097: four of 832 and one of 769)
@pytest.mark.parametrize("M", [1, 33, 1025, 4097])
def test_mlp_backward_edge_sizes(M):
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    print(f"[mlp] backward edge size M={M}", flush=True)
    rng = np.random.default_rng(100 + M)
    X = (rng.random((M, omlp.N_IN)) < 0.25).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    dX = bf16_tensor(X)
    b = model._buffers(M)
    w = model.weights()
    pa.mlp_forward(w, dX, M, b["H1"], b["H2"], b["Y"])
    dY = rng.normal(0, 1e-2, (M, 2)).astype(np.float32)
    pa.mlp_backward(w, dX, b["H1"], b["H2"], torch.from_numpy(dY).cuda(), M, model.grads())
    torch.cuda.synchronize()
    H1g, H2g = from_bf16(b["H1"][:M]), from_bf16(b["H2"][:M])
    check_gradients(model, W, X, H1g, H2g, dY.astype(np.float64))


def test_mlp_backward_full_size():
    """At the size the benchmark trains on (2^18 rows): the weight gradients
    take 256 row chunks of 1024, db1 the 2048 row tiles of the dH1 product, db2, dW3
    and db3 2048 full row chunks.  All six gradients against the oracle's
    backward on the GPU's own activations."""
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    M = 1 << 18
    rng = np.random.default_rng(18)
    X = (rng.random((M, omlp.N_IN)) < 0.25).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    dX = bf16_tensor(X)
    b = model._buffers(M)
    w = model.weights()
    pa.mlp_forward(w, dX, M, b["H1"], b["H2"], b["Y"])
    dY = rng.normal(0, 1e-3, (M, 2)).astype(np.float32)
    pa.mlp_backward(w, dX, b["H1"], b["H2"], torch.from_numpy(dY).cuda(), M, model.grads())
    torch.cuda.synchronize()
    print(f"[mlp] backward at {M} rows done, oracle next", flush=True)
    H1g, H2g = from_bf16(b["H1"][:M]), from_bf16(b["H2"][:M])
    check_gradients(model, W, X, H1g, H2g, dY.astype(np.float64))


def test_mlp_infer_full_size_sampled():
    """The fused inference at the benchmark's call size (2^20 rows, 8192
    workgroups): 4096 sampled rows against the oracle's forward pass."""
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    import torch
    M = 1 << 20
    rng = np.random.default_rng(20)
    X = (rng.random((M, omlp.N_IN)) < 0.25).astype(np.float32)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    X = omlp.bf16_round(X)
    W = omlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    W = [np.asarray(w, np.float32).astype(np.float64) for w in W]
    model = learn.WarmStartMLP(0)
    model.set_weights(W)
    Y = torch.empty((M, 2), dtype=torch.float32, device="cuda")
    pa.mlp_infer(model.infer_weights(), bf16_tensor(X), M, Y)
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(M, 4096, replace=False))
    idx[-1] = M - 1  # the last row of the last tile
    (_, _, Yo), (_, _, bY) = forward_bounds(W, X[idx].astype(np.float64))
    Yi = to_np(Y)[idx].astype(np.float64)
    assert np.all(np.abs(Yi - Yo) <= bY)


def test_adam_multi_equals_per_array_steps():
    """One multi-array Adam launch gives every array exactly what its own
    pasur_adam_step call gives (moments, master weights, BF16 copies),
    arrays of uneven sizes, one without a BF16 copy."""
    pa = require_gpu()
    import torch
    g = torch.Generator(device="cpu").manual_seed(5)
    sizes = [192 * 256, 256, 7, 256 * 256 + 3]
    def mk():
        return [torch.randn(n, generator=g).cuda() for n in sizes]
    w, gr, m = mk(), mk(), mk()
    v = [x.abs() for x in mk()]
    wb = [torch.zeros(n, dtype=torch.int16, device="cuda") for n in sizes]
    wb[2] = None
    a = [[t.clone() if t is not None else None for t in ts] for ts in (w, m, v, wb)]
    b = [[t.clone() if t is not None else None for t in ts] for ts in (w, m, v, wb)]
    for k in range(len(sizes)):
        pa.adam_step(a[0][k], gr[k], a[1][k], a[2][k], a[3][k], 1e-3, 0.9, 0.999, 1e-8, 7)
    pa.adam_step_multi(b[0], gr, b[1], b[2], b[3], 1e-3, 0.9, 0.999, 1e-8, 7)
    torch.cuda.synchronize()
    for ta, tb in zip(a, b):
        for x, y in zip(ta, tb):
            if x is None:
                assert y is None
            else:
                assert torch.equal(x, y)
