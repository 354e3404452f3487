"""GPU parity of DCFR, leaf utilities, round values, average strategies and
exploitability against the FP64 oracle, through the C ABI.

FP64 state: every array must match the oracle within 1e-9 (the kernels keep
the oracle's operation order, so in practice they agree exactly).
FP32 state: root values must match within 1e-5, and average strategies
within 1e-5 as play frequencies (each action's sigma-bar difference times the
probability that play reaches its parent), with equally good actions
compared by their total: ties make the split among them depend on rounding
(FP32 noise in the regrets exceeds the regret floor), and behaviour where
play does not go is not fixed by an equilibrium.  That behaviour is checked
through quality instead (exploitability no worse than the oracle's)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (assert_sigma_bar_up_to_ties, oracle_exploitability, oracle_rounds,
                        oracle_solve, require_gpu, tie_groups, to_np)

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32_VALUES = 1e-5


def gpu_solver(pa, deck, start, roots, dtype, iters, params=None):
    s = pa.SubgameSolver(deck, start, roots, dtype=dtype)
    s.solve(iters, params)
    import torch
    torch.cuda.synchronize()
    return s


def max_diff(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))))


@pytest.mark.parametrize("seed", [1, 2])
def test_fp64_state_matches_oracle_last_round(seed):
    pa = require_gpu()
    deck, roots = synth.last_round_roots(seed)
    print(f"[cfr fp64] last round seed={seed} T=1000", flush=True)
    s = gpu_solver(pa, deck, 5, roots, pa.PASUR_F64, 1000)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 1000)
    st = s.rounds[0].state
    assert max_diff(to_np(st.u[8]), leaf) == 0.0
    for l in range(1, 9):
        assert max_diff(to_np(st.sigma[l]), c.get(oracle.CF_SIGMA, l)) <= TOL64, l
        assert max_diff(to_np(st.R[l]), c.get(oracle.CF_R, l)) <= TOL64, l
        assert max_diff(to_np(st.Sbar[l]), c.get(oracle.CF_SBAR, l)) <= TOL64, l
        assert max_diff(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l)) <= TOL64, l
    for l in range(0, 8):
        assert max_diff(to_np(st.u[l]), c.get(oracle.CF_U, l)) <= TOL64, l
        assert max_diff(to_np(st.reachA[l]), c.get(oracle.CF_REACHA, l)) <= TOL64, l
        assert max_diff(to_np(st.reachB[l]), c.get(oracle.CF_REACHB, l)) <= TOL64, l
    assert max_diff(to_np(s.rounds[0].V), V) <= TOL64


@pytest.mark.parametrize("seed", [1, 3])
def test_fp64_two_round_solve_matches_oracle(seed):
    # Rounds 5-6 of a seeded deal at full size, 2000 iterations per round,
    # round values passed backward (the benchmark's workload for seed 1).
    pa = require_gpu()
    deck, roots = synth.two_round_root(seed)
    print(f"[cfr fp64] two rounds seed={seed} T=2000", flush=True)
    s = gpu_solver(pa, deck, 4, roots, pa.PASUR_F64, 2000)
    rounds = oracle_rounds(deck, 4, roots)
    res = oracle_solve(rounds, 2000)
    for k in range(2):
        c, leaf, V = res[k]
        st = s.rounds[k].state
        assert max_diff(to_np(st.u[8]), leaf) <= TOL64
        assert max_diff(to_np(s.rounds[k].V), V) <= TOL64
        for l in range(1, 9):
            assert max_diff(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l)) <= TOL64, (k, l)
            assert max_diff(to_np(st.sigma[l]), c.get(oracle.CF_SIGMA, l)) <= TOL64, (k, l)
    # exploitability of the GPU's average strategies, composed across rounds
    sb = [[np.ones(1)] + [to_np(t) for t in rr.state.sigma_bar[1:]] for rr in s.rounds]
    bra, brb, v = oracle_exploitability(rounds, sb)
    gbra, gbrb, gv = (to_np(x) for x in s.exploitability())
    assert max_diff(gbra, bra) <= TOL64
    assert max_diff(gbrb, brb) <= TOL64
    assert max_diff(gv, v) <= TOL64
    assert np.all(gbra >= gbrb - 1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fp32_state_values_and_strategy_quality(seed):
    pa = require_gpu()
    deck, roots = synth.last_round_roots(seed)
    print(f"[cfr fp32] last round seed={seed} T=1000", flush=True)
    s = gpu_solver(pa, deck, 5, roots, pa.PASUR_F32, 1000)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 1000)
    assert max_diff(to_np(s.rounds[0].V), V) <= TOL32_VALUES
    st = s.rounds[0].state
    f = rounds[0][1]
    for l in range(1, 9):
        sb = to_np(st.sigma_bar[l]).astype(np.float64)
        assert np.all(sb >= 0)
        par = np.repeat(np.arange(f.n[l - 1]), np.diff(f.get(oracle.FGT_CHILD_BEGIN, l - 1)))
        np.testing.assert_allclose(np.bincount(par, sb, f.n[l - 1]), 1.0, atol=1e-5)
    gsb = [[np.ones(1)] + [to_np(t).astype(np.float64) for t in st.sigma_bar[1:]]]
    bra, brb, _ = oracle_exploitability(rounds, gsb)
    obra, obrb, _ = oracle_exploitability(rounds, [c.sigma_bar()])
    ex_gpu, ex_or = (bra - brb) / 2, (obra - obrb) / 2
    M = oracle.tree_values(f.n, f.child_begin(), leaf, None, oracle.TV_MINIMAX)
    # FP32 sigma_bar sums to 1 only up to float rounding (~1e-7 relative)
    assert np.all(brb - TOL32_VALUES <= M) and np.all(M <= bra + TOL32_VALUES)
    # equally good actions may split differently, but the profile must be as
    # good as the oracle's
    assert ex_gpu.max() <= 1.5 * ex_or.max() + 1e-6


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fp32_sigma_bar_matches_oracle_up_to_ties_last_round(seed):
    # FP32 state against the FP64 oracle: how often each action is played
    # (its sigma-bar difference times the probability that play under the
    # average profile reaches its parent) within 1e-5, and among equally good
    # actions (same minimax value under one parent) only their total, since
    # FP32 rounding noise in the regrets exceeds the regret floor and may
    # split that total differently.
    pa = require_gpu()
    deck, roots = synth.last_round_roots(seed)
    print(f"[cfr fp32] sigma-bar up to ties, last round seed={seed} T=1000", flush=True)
    s = gpu_solver(pa, deck, 5, roots, pa.PASUR_F32, 1000)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 1000)
    groups = tie_groups(rounds[0][1], leaf)
    gsb = [None] + [to_np(t) for t in s.rounds[0].state.sigma_bar[1:]]
    tied, total, big = assert_sigma_bar_up_to_ties(gsb, c.sigma_bar(), groups,
                                                   rounds[0][1].child_begin(), TOL32_VALUES, seed)
    print(f"[cfr fp32] {tied} of {total} actions in tie groups; largest difference at parents "
          f"reached with probability >= 0.5: {big:.2e}", flush=True)
    assert tied < total


@pytest.mark.parametrize("seed", [1, 13])
def test_fp32_sigma_bar_matches_oracle_up_to_ties_two_rounds(seed):
    # round 5's leaves are round 6's values, FP32 on the GPU: actions whose
    # minimax values differ by less than 1e-3 count as tied there
    pa = require_gpu()
    deck, roots = synth.two_round_root(seed)
    print(f"[cfr fp32] sigma-bar up to ties, two rounds seed={seed} T=2000", flush=True)
    s = gpu_solver(pa, deck, 4, roots, pa.PASUR_F32, 2000)
    rounds = oracle_rounds(deck, 4, roots)
    res = oracle_solve(rounds, 2000)
    for k in (1, 0):
        c, leaf, V = res[k]
        groups = tie_groups(rounds[k][1], leaf)
        gsb = [None] + [to_np(t) for t in s.rounds[k].state.sigma_bar[1:]]
        tied, total, big = assert_sigma_bar_up_to_ties(gsb, c.sigma_bar(), groups,
                                                       rounds[k][1].child_begin(), TOL32_VALUES, k)
        print(f"[cfr fp32] round {k + 5}: {tied} of {total} actions in tie groups; largest "
              f"difference at parents reached with probability >= 0.5: {big:.2e}", flush=True)
        assert max_diff(to_np(s.rounds[k].V), V) <= TOL32_VALUES


def test_fp32_two_round_values():
    pa = require_gpu()
    deck, roots = synth.two_round_root(1)
    s = gpu_solver(pa, deck, 4, roots, pa.PASUR_F32, 2000)
    res = oracle_solve(oracle_rounds(deck, 4, roots), 2000)
    assert max_diff(to_np(s.rounds[0].V), res[0][2]) <= TOL32_VALUES
    assert max_diff(to_np(s.rounds[1].V), res[1][2]) <= TOL32_VALUES


@pytest.mark.parametrize("variant,rm", [(oracle.CFR_PLUS, oracle.RM_POSITIVE),
                                        (oracle.CFR_VANILLA, oracle.RM_POSITIVE),
                                        (oracle.CFR_DCFR, oracle.RM_POSITIVE)])
def test_fp64_variants_match_oracle(variant, rm):
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    params = pa.CfrParams(variant, rm, 1.5, 0.0, 2.0, 1e-8)
    s = gpu_solver(pa, deck, 5, roots, pa.PASUR_F64, 300, params)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 300, oracle.Params(variant=variant, rm_mode=rm))
    st = s.rounds[0].state
    for l in range(1, 9):
        assert max_diff(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l)) <= TOL64
        assert max_diff(to_np(st.R[l]), c.get(oracle.CF_R, l)) <= TOL64
    assert max_diff(to_np(s.rounds[0].V), V) <= TOL64


def test_minimax_and_sigma_bar_values():
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(3)
    s = gpu_solver(pa, deck, 4, roots, pa.PASUR_F64, 200)
    rounds = oracle_rounds(deck, 4, roots)
    Vg, Vo = None, None
    for k in (1, 0):
        rr = s.rounds[k]
        f = rounds[k][1]
        leaf_o = f.leaf_utilities(Vo)
        Vo = oracle.tree_values(f.n, f.child_begin(), leaf_o, None, oracle.TV_MINIMAX)
        leaf_g = torch.empty(rr.fgt.n[8], dtype=torch.float64, device="cuda")
        pa.leaf_utilities(rr.fgt, Vg, pa.PASUR_F64, leaf_g)
        assert max_diff(to_np(leaf_g), leaf_o) == 0.0
        Vg = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
        pa.tree_values(rr.fgt, leaf_g, pa.PASUR_F64, None, pa.TV_MINIMAX, Vg)
        assert max_diff(to_np(Vg), Vo) == 0.0
    # SIGMA_BAR value mode = expectation under sigma_bar
    rr = s.rounds[1]
    V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
    pa.round_values(rr.state, pa.V_SIGMA_BAR, V)
    f = rounds[1][1]
    sb = [np.ones(f.n[0])] + [to_np(t) for t in rr.state.sigma_bar[1:]]
    want = oracle.tree_values(f.n, f.child_begin(), f.leaf_utilities(), sb, oracle.TV_EXPECT)
    assert max_diff(to_np(V), want) <= TOL64


def test_split_iterations_equal_single_call_and_determinism():
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(2)
    outs = []
    for split in (False, True, False):
        s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F32)
        rr = s.rounds[0]
        st = pa.CfrState(rr.fgt, pa.PASUR_F32)
        pa.leaf_utilities(rr.fgt, None, pa.PASUR_F32, st.u[8])
        pa.cfr_init(st)
        if split:
            pa.cfr_iterate(st, 123)
            pa.cfr_iterate(st, 377)
        else:
            pa.cfr_iterate(st, 500)
        torch.cuda.synchronize()
        outs.append([to_np(t).copy() for t in st.sigma[1:] + st.R[1:] + st.Sbar[1:]] +
                    [to_np(st.vacc).copy()])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0], outs[2]):
        assert np.array_equal(a, b)


def test_cfr_rejects_bad_arguments():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F32)
    st = pa.CfrState(s.rounds[0].fgt, pa.PASUR_F32)
    with pytest.raises(pa.PasurError, match="t0"):
        pa.cfr_iterate(st, 1, t0=0)
    bad = pa.CfrParams(7, 0, 1.5, 0.0, 2.0, 1e-8)
    with pytest.raises(pa.PasurError, match="variant"):
        pa.cfr_iterate(st, 1, bad)
    deck2, roots2 = synth.two_round_root(3)
    s2 = pa.SubgameSolver(deck2, 4, roots2, dtype=pa.PASUR_F32)
    import torch
    buf = torch.empty(s2.rounds[0].fgt.n[8], dtype=torch.float32, device="cuda")
    with pytest.raises(pa.PasurError, match="next round"):
        pa.leaf_utilities(s2.rounds[0].fgt, None, pa.PASUR_F32, buf)


@pytest.mark.parametrize("dtype_name", ["PASUR_F32", "PASUR_F64"])
def test_schedules_are_bit_identical(dtype_name):
    # Per-root persistent kernels (LDS-resident or global memory) and the
    # level-synchronous kernels run the same per-parent arithmetic.
    pa = require_gpu()
    import torch
    dtype = getattr(pa, dtype_name)
    results = []
    for sched, block in ((pa.SCHED_LEVEL_SYNC, 0), (pa.SCHED_ROOT, 256), (pa.SCHED_ROOT, 512),
                         (pa.SCHED_ROOT, 1024), (pa.SCHED_ROOT_GLOBAL, 256)):
        print(f"[schedules] {dtype_name} schedule={sched} block={block}", flush=True)
        for deck, start, roots in ((*synth.two_round_root(1)[:1], 4, synth.two_round_root(1)[1]),
                                   (*synth.last_round_roots(2)[:1], 5, synth.last_round_roots(2)[1])):
            s = pa.SubgameSolver(deck, start, roots, dtype=dtype)
            s.solve(300, pa.paper_params(sched, block))
            torch.cuda.synchronize()
            arrs = []
            for rr in s.rounds:
                st = rr.state
                arrs += [to_np(t).copy() for t in st.sigma[1:] + st.R[1:] + st.Sbar[1:]
                         + st.reachA[:8] + st.reachB[:8] + st.u[:8]] + [to_np(st.vacc).copy()]
            results.append(arrs)
            s.free()
    ref = results[0:2]
    for k in range(2, len(results)):
        for a, b in zip(results[k], ref[k % 2]):
            assert np.array_equal(a, b)


def test_exploitability_entry_point():
    # pasur_exploitability against the oracle's composition, with outputs
    # requested one at a time, and its consistency checks on real trees
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(3)
    s = gpu_solver(pa, deck, 4, roots, pa.PASUR_F32, 300)
    rounds = oracle_rounds(deck, 4, roots)
    sb = [[np.ones(1)] + [to_np(t).astype(np.float64) for t in rr.state.sigma_bar[1:]]
          for rr in s.rounds]
    ref = oracle_exploitability(rounds, sb)
    fg = [rr.fgt for rr in s.rounds]
    sbs = [rr.state.sigma_bar for rr in s.rounds]
    n0 = fg[0].n[0]
    for i in range(3):
        outs = [None, None, None]
        outs[i] = torch.full((n0,), float("nan"), dtype=torch.float64, device="cuda")
        pa.exploitability(fg, sbs, pa.PASUR_F32, *outs)
        torch.cuda.synchronize()
        assert max_diff(to_np(outs[i]), ref[i]) <= TOL64, i
    assert np.all(ref[0] >= ref[1])
    out = torch.empty(n0, dtype=torch.float64, device="cuda")
    with pytest.raises(pa.PasurError, match="round 5"):
        pa.exploitability(fg[:1], sbs[:1], pa.PASUR_F32, out)
    with pytest.raises(pa.PasurError, match="not the unfolding"):
        pa.exploitability(fg[::-1], sbs[::-1], pa.PASUR_F32, out)
    d2, r2 = synth.two_round_root(1)
    s2 = pa.SubgameSolver(d2, 4, r2, dtype=pa.PASUR_F32)
    if s2.rounds[1].fgt.n[0] != fg[1].n[0]:
        with pytest.raises(pa.PasurError, match="not the unfolding"):
            pa.exploitability([fg[0], s2.rounds[1].fgt], sbs, pa.PASUR_F32, out)
    s2.free()
    s.free()
