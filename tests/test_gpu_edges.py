"""Edge cases of the round path, through the C ABI: an empty root list is
refused, zero iterations leave the state untouched under every schedule,
averaging before any iteration gives the uniform strategy, the iterate-mean
value needs at least one iteration, the smallest subgame (one root of the
final round) matches the FP64 oracle under every schedule, and the solver's
per-round hook sees the rounds in order."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import oracle_rounds, oracle_solve, require_gpu, to_np

pytestmark = pytest.mark.gpu

SCHEDS = ["SCHED_ROOT", "SCHED_LEVEL_SYNC", "SCHED_ROOT_GLOBAL", "SCHED_STREAM"]


def fresh_round(pa, deck, start, roots, k, dtype):
    s = pa.SubgameSolver(deck, start, roots, dtype=dtype)
    rr = s.rounds[k]
    st = pa.CfrState(rr.fgt, dtype)
    pa.leaf_utilities(rr.fgt, None, dtype, st.u[8])
    pa.cfr_init(st)
    return s, rr, st


def snapshot(st):
    arrs = st.sigma[1:] + st.R[1:] + st.Sbar[1:] + st.u + st.reachA[:8] + st.reachB[:8]
    return [to_np(x).copy() for x in arrs] + [to_np(st.vacc).copy()]


def test_empty_root_list_is_refused():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(2)
    d = pa.roots_to_device(roots)
    with pytest.raises(pa.PasurError, match="at least one root"):
        pa.build_round_tree(deck, 5, d, 0)
    gt = pa.build_round_tree(deck, 5, d, len(roots))
    with pytest.raises(pa.PasurError, match="at least one root"):
        pa.unfold_scores(gt, d, 0)
    gt.free()


@pytest.mark.parametrize("sched", SCHEDS)
def test_zero_iterations_change_nothing(sched):
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(3)
    print(f"[edges] zero iterations, {sched}", flush=True)
    s, rr, st = fresh_round(pa, deck, 4, roots, 1, pa.PASUR_F64)
    params = pa.paper_params(getattr(pa, sched))
    pa.cfr_iterate(st, 5, params)
    torch.cuda.synchronize()
    before = snapshot(st)
    pa.cfr_iterate(st, 0, params)
    torch.cuda.synchronize()
    assert st.t == 6
    for a, b in zip(before, snapshot(st)):
        assert np.array_equal(a, b)
    s.free()


@pytest.mark.parametrize("dtype_name", ["PASUR_F32", "PASUR_F64"])
def test_average_before_any_iteration_is_uniform(dtype_name):
    pa = require_gpu()
    import torch
    dtype = getattr(pa, dtype_name)
    deck, roots = synth.last_round_roots(4)
    s, rr, st = fresh_round(pa, deck, 5, roots, 0, dtype)
    pa.average_strategy(st)
    torch.cuda.synchronize()
    ft = np.float32 if dtype == pa.PASUR_F32 else np.float64
    for l in range(1, 9):
        cb = rr.fgt.read(pa.FGT_CHILD_BEGIN, l - 1).astype(np.int64)
        k = np.diff(cb)
        want = np.repeat((1.0 / k).astype(ft), k)
        assert np.array_equal(to_np(st.sigma_bar[l]), want), l
    # the iterate mean of zero iterations is undefined: refused
    V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
    with pytest.raises(pa.PasurError, match="T must be"):
        pa.round_values(st, pa.V_ITERATE_MEAN, V)
    s.free()


@pytest.mark.parametrize("sched", SCHEDS)
def test_one_root_final_round_matches_oracle(sched):
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(6, deltas=[0])
    assert len(roots) == 1
    print(f"[edges] one root, {sched}", flush=True)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F64)
    s.solve(200, pa.paper_params(getattr(pa, sched)))
    torch.cuda.synchronize()
    (c, leaf, V), = oracle_solve(oracle_rounds(deck, 5, roots), 200)
    st = s.rounds[0].state
    for l in range(1, 9):
        assert np.max(np.abs(to_np(st.sigma_bar[l]) - c.get(oracle.CF_SIGMA_BAR, l))) <= 1e-9, l
        assert np.max(np.abs(to_np(st.R[l]) - c.get(oracle.CF_R, l))) <= 1e-9, l
    assert np.max(np.abs(to_np(s.rounds[0].V) - V)) <= 1e-9
    s.free()


def test_solve_round_hook_and_profile_count():
    """SubgameSolver.solve calls on_round once per round, last round first,
    after the round's iterations are enqueued; the profile's record count
    (read without waiting for the GPU) grows with every round's sweeps."""
    pa = require_gpu()
    deck, roots = synth.two_round_root(1)
    print("[edges] on_round hook, two-round subgame of deal 1", flush=True)
    s = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F32)
    seen = []
    pa.profile_enable(True)
    try:
        s.solve(5, on_round=lambda r: seen.append((r, pa.profile_count())))
        total = len(pa.profile_read()[0])
    finally:
        pa.profile_enable(False)
        s.free()
    assert [r for r, _ in seen] == [5, 4]
    counts = [c for _, c in seen]
    assert 0 < counts[0] < counts[1] <= total
