"""External-sampling CFR on the GPU (pasur_es_iterate) against the oracle.

With FP64 state both sides draw the same counter-based numbers from the same
strategies, so every regret, strategy and average sum must agree element by
element after many iterations (every pick and every draw the same).  With
FP32 state and at the full-game scale the checks are properties:
exploitability falls, average strategies are valid profiles, a seed
reproduces its run."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import require_gpu, to_np
from oracle import es

pytestmark = pytest.mark.gpu


def oracle_round(deck, roots):
    gt = oracle.GT(deck, 5, sorted({x.pool for x in roots}))
    f = oracle.FGT(gt, roots)
    return f, f.child_begin(), f.leaf_utilities()


def gpu_round(pa, deck, roots, dtype):
    s = pa.SubgameSolver(deck, 5, roots, dtype=dtype)
    rr = s.rounds[0]
    st = pa.CfrState(rr.fgt, dtype)
    pa.leaf_utilities(rr.fgt, None, dtype, st.u[8])
    pa.cfr_init(st)
    return s, rr, st


@pytest.mark.parametrize("seed,rm,schedule,per_wg", [
    (4, "floor", "frontier", 0), (5, "floor", "level", 0), (1, "positive", "frontier", 3),
    (4, "positive", "level", 0), (5, "floor", "frontier", 2)])
def test_es_matches_oracle_element_by_element(seed, rm, schedule, per_wg):
    """Both schedules; the frontier schedule also with several roots per
    workgroup (7 roots in groups of 3 or 2: a ragged last group)."""
    pa = require_gpu()
    deck, roots = synth.last_round_roots(seed)
    f, cb, leaf = oracle_round(deck, roots)
    s, rr, st = gpu_round(pa, deck, roots, pa.PASUR_F64)
    assert list(rr.fgt.n) == list(f.n)
    rm_mode = pa.RM_FLOOR if rm == "floor" else pa.RM_POSITIVE
    iters, draw_seed = 40, 77 + seed
    # two calls (the second continues the draw stream) against one oracle call
    sch = pa.ES_FRONTIER if schedule == "frontier" else pa.ES_LEVEL
    pa.es_iterate(st, 15, draw_seed, rm_mode, schedule=sch, roots_per_wg=per_wg)
    pa.es_iterate(st, iters - 15, draw_seed, rm_mode, schedule=sch, roots_per_wg=per_wg)
    ost = es.ESState(f.n, cb)
    es.es_iterate(ost, leaf, iters, draw_seed, rm_mode=rm)
    print(f"[es] seed {seed} ({rm}, {schedule}, {per_wg} roots per workgroup): {sum(f.n)} nodes, "
          f"{iters} iterations", flush=True)
    for l in range(1, 9):
        for name, want in (("sigma", ost.sigma[l]), ("R", ost.R[l]), ("Sbar", ost.Sbar[l])):
            got = to_np(getattr(st, name)[l])
            assert np.array_equal(got, want), (name, l, np.max(np.abs(got - want)))
    sb = pa.average_strategy(st)
    for l in range(1, 9):
        np.testing.assert_allclose(to_np(sb[l]), ost.sigma_bar()[l], rtol=0, atol=1e-12)
    s.free()


def test_es_fp32_converges():
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(4)
    s, rr, st = gpu_round(pa, deck, roots, pa.PASUR_F32)

    def expl():
        sb = pa.average_strategy(st)
        leaf = torch.empty(rr.fgt.n[8], dtype=torch.float64, device="cuda")
        pa.leaf_utilities(rr.fgt, None, pa.PASUR_F64, leaf)
        out = []
        for mode in (pa.TV_BR_A, pa.TV_BR_B):
            v = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
            pa.tree_values(rr.fgt, leaf, pa.PASUR_F32, sb, mode, v)
            out.append(to_np(v))
        return float(np.max((out[0] - out[1]) / 2))

    e0 = expl()
    pa.es_iterate(st, 2000, 5)
    e1 = expl()
    print(f"[es] FP32 final round: exploitability {e0:.4f} -> {e1:.5f} after 2000 iterations", flush=True)
    assert e1 < 0.05 * e0
    sb = pa.average_strategy(st)
    for l in range(1, 9):
        x = to_np(sb[l]).astype(np.float64)
        cbl = rr.fgt.read(pa.FGT_CHILD_BEGIN, l - 1)
        sums = np.add.reduceat(x, cbl[:-1]) if len(x) else x
        np.testing.assert_allclose(sums, 1.0, atol=1e-5)
    s.free()


def test_es_full_game():
    """All six rounds of seeded deal 1 solved backward with external
    sampling: a seed reproduces the run bit for bit, the level-synchronous
    schedule gives the frontier schedule's results bit for bit at this size,
    and the composed exploitability of the average strategies falls as
    iterations grow."""
    pa = require_gpu()
    deck, roots = synth.full_game_root(1)
    res = {}
    for iters, seed, sch in ((50, 1, pa.ES_FRONTIER), (50, 1, pa.ES_LEVEL), (400, 1, pa.ES_FRONTIER)):
        s = pa.SubgameSolver(deck, 0, roots, dtype=pa.PASUR_F32)
        s.solve_es(iters, seed, schedule=sch)
        bra, brb, v = s.exploitability()
        ex = float(((bra - brb) / 2).max().item())
        sb = [to_np(x).copy() for rr in s.rounds for x in rr.state.sigma_bar[1:]]
        res.setdefault(iters, []).append((ex, sb, float(v[0].item())))
        print(f"[es] full game seed 1: {iters} iterations per round, exploitability {ex:.4f}, "
              f"value {float(v[0].item()):.3f}", flush=True)
        s.free()
    a, b = res[50]
    assert all(np.array_equal(x, y) for x, y in zip(a[1], b[1])) and a[2] == b[2]
    assert res[400][0][0] < 0.5 * a[0]


def test_es_zero_iterations_and_empty_rounds_change_nothing():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    s, rr, st = gpu_round(pa, deck, roots, pa.PASUR_F64)
    before = [to_np(x).copy() for x in st.sigma[1:] + st.R[1:] + st.Sbar[1:]]
    for sch in (pa.ES_FRONTIER, pa.ES_LEVEL):
        pa.es_iterate(st, 0, 5, schedule=sch)
    after = [to_np(x) for x in st.sigma[1:] + st.R[1:] + st.Sbar[1:]]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    s.free()
