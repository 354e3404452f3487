"""The learned warm start end to end: training on this solver's own DCFR
solutions lowers the loss, the warm-start initialisation sets exactly the
softmax of the predicted logits, and the trained network's starting
profile is less exploitable than the uniform profile plain DCFR starts from
(what the network gains over the method without it)."""
import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    print("[learn] training data from 48 deals", flush=True)
    units = learn.training_units([synth.two_round_root(s) for s in range(10000, 10048)], 500)
    model = learn.WarmStartMLP(0)
    hist = learn.train(model, units, 12)
    return model, hist


def test_training_lowers_loss(trained):
    model, hist = trained
    assert hist[-1][0] < hist[0][0] and hist[-1][1] < hist[0][1]


def test_warm_init_sets_softmax_of_logits(trained):
    pa = require_gpu()
    import torch
    from paper_2508_06559_amd import learn
    model, _ = trained
    deck, roots = synth.two_round_root(20001)
    sv = pa.SubgameSolver(deck, 4, roots, keep_gt=True)
    rr = sv.rounds[1]
    rr.state = pa.CfrState(rr.fgt, pa.PASUR_F64)
    pa.cfr_init(rr.state)
    l = 2
    n = rr.fgt.n[l]
    X = torch.empty((n, learn.N_IN), dtype=torch.int16, device="cuda")
    pa.edge_features(rr.gt, rr.fgt, l, None, n, X)
    Y = to_np(model.forward(X, n)).astype(np.float64)
    pa.cfr_warm_init(rr.state, l, model.forward(X, n), 0.5, 2.0)
    torch.cuda.synchronize()
    cb = rr.fgt.read(pa.FGT_CHILD_BEGIN, l - 1)
    want = np.zeros(n)
    for h in range(rr.fgt.n[l - 1]):
        z = Y[cb[h]:cb[h + 1], 0]
        e = np.exp(z - z.max())
        want[cb[h]:cb[h + 1]] = e / e.sum()
    np.testing.assert_allclose(to_np(rr.state.sigma[l]), want, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(to_np(rr.state.R[l]), 0.5 * want, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(to_np(rr.state.Sbar[l]), 2.0 * want, rtol=1e-12, atol=1e-15)
    sv.free()


def test_network_profile_beats_uniform_start(trained):
    pa = require_gpu()
    from paper_2508_06559_amd import learn
    model, _ = trained
    ex_u, ex_n, it_p, it_w = [], [], [], []
    for s in range(20000, 20006):
        deck, roots = synth.two_round_root(s)
        ex_u.append(learn.initial_profile_exploitability(deck, roots, None))
        ex_n.append(learn.initial_profile_exploitability(deck, roots, model))
        grid = (8, 16, 32, 64, 128, 256)
        it_p.append(learn.seconds_to_target(deck, 4, roots, 1e-3, grid, None)["iters"])
        it_w.append(learn.seconds_to_target(deck, 4, roots, 1e-3, grid, model)["iters"])
    print(f"[learn] initial exploitability uniform {np.median(ex_u):.3f} network {np.median(ex_n):.3f}; "
          f"iterations to 1e-3 plain {it_p} warm {it_w}", flush=True)
    assert np.median(ex_n) < np.median(ex_u)
    assert all(i is not None for i in it_p + it_w)


@pytest.mark.parametrize("max_level", [8, 3])
def test_round_warm_start_matches_per_level_calls(trained, max_level):
    """The one-call round warm start (features of all levels, one forward
    pass, one initialisation launch) sets exactly what the per-level calls
    set on levels 1..max_level and leaves deeper levels as cfr_init left them."""
    pa = require_gpu()
    import torch
    from paper_2508_06559_amd import learn
    model, _ = trained
    deck, roots = synth.two_round_root(20003)
    sv = pa.SubgameSolver(deck, 4, roots, keep_gt=True)
    rr = sv.rounds[1]
    got = pa.CfrState(rr.fgt, pa.PASUR_F64)
    ref = pa.CfrState(rr.fgt, pa.PASUR_F64)
    pa.cfr_init(got)
    pa.cfr_init(ref)
    init = [None] + [to_np(x).copy() for x in ref.sigma[1:]]
    rr.state = ref
    learn.warm_start_round_by_level(model, rr, 0.5, 2.0)
    rr.state = got
    learn.warm_start_round(model, rr, 0.5, 2.0, max_level)
    torch.cuda.synchronize()
    for l in range(1, 9):
        g_s, g_r, g_b = to_np(got.sigma[l]), to_np(got.R[l]), to_np(got.Sbar[l])
        if l <= max_level:
            assert np.array_equal(g_s, to_np(ref.sigma[l])), l
            assert np.array_equal(g_r, to_np(ref.R[l])), l
            assert np.array_equal(g_b, to_np(ref.Sbar[l])), l
        else:
            assert np.array_equal(g_s, init[l]), l
            assert not g_r.any() and not g_b.any(), l
    sv.free()


@pytest.mark.parametrize("warm", [False, True])
def test_reused_solver_equals_fresh_solve(trained, warm):
    """solve_built on one solver reused over an iteration grid (the whole-game
    warm-start measurement) leaves exactly the states, average strategies and
    round values of a fresh solve of the last count: cfr_init resets every
    array a longer earlier solve wrote."""
    pa = require_gpu()
    import torch
    from paper_2508_06559_amd import learn
    model, _ = trained
    m = model if warm else None
    wp = learn.WarmParams(max_level=3)
    deck, roots = synth.two_round_root(20004)
    sv = pa.SubgameSolver(deck, 4, roots, keep_gt=True)
    learn.solve_built(sv, 20, m, wp)
    learn.solve_built(sv, 12, m, wp)
    ref = learn.solve_subgame(deck, 4, roots, 12, model=m, warm=wp)
    torch.cuda.synchronize()
    for a, b in zip(sv.rounds, ref.rounds):
        assert np.array_equal(to_np(a.V), to_np(b.V)), a.round
        for l in range(1, 9):
            for name in ("sigma", "R", "Sbar", "sigma_bar"):
                assert np.array_equal(to_np(getattr(a.state, name)[l]),
                                      to_np(getattr(b.state, name)[l])), (a.round, name, l)
    assert learn.exploitability(sv) == learn.exploitability(ref)
    sv.free()
    ref.free()
