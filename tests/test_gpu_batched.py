"""Batched solve (many deals in one persistent launch per round, a plan)
and its HIP-graph capture: bit-identical to solving every deal alone."""
import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_np

pytestmark = pytest.mark.gpu


def state_arrays(rounds):
    out = []
    for rr in rounds:
        st = rr.state
        out += [to_np(t).copy() for t in st.sigma[1:] + st.R[1:] + st.Sbar[1:] + st.u[:8]]
        out += [to_np(st.vacc).copy(), to_np(rr.V).copy()]
        out += [to_np(t).copy() for t in st.sigma_bar[1:]]
    return out


def problems(seeds):
    return [synth.two_round_root(s) for s in seeds]


@pytest.mark.parametrize("dtype_name,seg_nodes", [("PASUR_F32", 0), ("PASUR_F32", 6000),
                                                  ("PASUR_F64", 0)])
def test_batched_equals_individual_solves(dtype_name, seg_nodes):
    pa = require_gpu()
    import torch
    dtype = getattr(pa, dtype_name)
    probs = problems([1, 2, 3, 5])
    print(f"[batched] {dtype_name} seg_nodes={seg_nodes} deals={len(probs)}", flush=True)
    b = pa.BatchSolver(probs, 4, 300, dtype=dtype, params=pa.paper_params(seg_nodes=seg_nodes))
    b.solve()
    torch.cuda.synchronize()
    for (deck, roots), sv in zip(probs, b.deals):
        ref = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        ref.solve(300)
        torch.cuda.synchronize()
        for x, y in zip(state_arrays(sv.rounds), state_arrays(ref.rounds)):
            assert np.array_equal(x, y)
        ref.free()
    assert all(p.n_segs >= 1 for p in b.plans)
    b.free()


@pytest.mark.parametrize("which", ["all", "largest"])
def test_batched_streamed_rounds_equal_per_round_schedules(which):
    """Rounds at or above stream_min_nodes leave the round's plan and run the
    streaming schedule deal by deal; every deal then equals its own backward
    solve with the same schedule per round (streaming sweeps for those
    rounds, persistent segments for the rest), bit for bit, and such a
    batch refuses HIP-graph capture."""
    pa = require_gpu()
    import torch
    dtype, iters = pa.PASUR_F32, 300
    probs = problems([1, 2, 3, 5])
    sizes = []
    for deck, roots in probs:
        sv = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        sizes.append([sum(rr.fgt.n) for rr in sv.rounds])
        sv.free()
    # "largest": only the round-6 tree of the largest deal is streamed
    thr = 1 if which == "all" else max(sz[1] for sz in sizes)
    print(f"[batched] streamed rounds ({which}): threshold {thr}, sizes {sizes}", flush=True)
    b = pa.BatchSolver(probs, 4, iters, dtype=dtype, stream_min_nodes=thr)
    assert any(any(st) for st in b.streamed)
    b.solve()
    torch.cuda.synchronize()
    for (deck, roots), sv, sz in zip(probs, b.deals, sizes):
        ref = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        V = None
        for k in (1, 0):
            rr = ref.rounds[k]
            rr.state = pa.CfrState(rr.fgt, dtype)
            pa.leaf_utilities(rr.fgt, V, dtype, rr.state.u[8])
            pa.cfr_init(rr.state)
            sched = pa.SCHED_STREAM if sz[k] >= thr else pa.SCHED_AUTO
            pa.cfr_iterate(rr.state, iters, pa.paper_params(sched))
            pa.average_strategy(rr.state)
            rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
            pa.round_values(rr.state, pa.V_ITERATE_MEAN, rr.V)
            V = rr.V
        torch.cuda.synchronize()
        for x, y in zip(state_arrays(sv.rounds), state_arrays(ref.rounds)):
            assert np.array_equal(x, y)
        ref.free()
    with pytest.raises(ValueError, match="captured"):
        b.capture()
    b.free()


def test_autotune_keeps_fastest_and_results():
    """The autotuner times every candidate of every round, keeps the
    fastest, and the batch solved with its schedule equals the deals solved
    one by one (every segment schedule gives the same bits)."""
    pa = require_gpu()
    import torch
    from paper_2508_06559_amd import autotune
    probs = problems([1, 2, 3, 5])
    b = pa.BatchSolver(probs, 4, 200, dtype=pa.PASUR_F32)
    cands = ((256, 0), (1024, 0), (1024, 4096), (512, 2048))
    res = autotune.autotune(b.round_states(), candidates=cands, iters=3)
    assert len(res["rounds"]) == 2
    for r in res["rounds"]:
        assert len(r["timings"]) == len(cands)
        assert r["best"] == min(r["timings"], key=lambda x: x["ms_per_iter"])
        assert all(t["ms_per_iter"] > 0 for t in r["timings"])
    b.set_params(autotune.params_from(res))
    for k, r in enumerate(res["rounds"]):
        assert (b.params[k].block, b.params[k].seg_nodes) == (r["best"]["block"],
                                                             r["best"]["seg_nodes"])
    b.solve()
    torch.cuda.synchronize()
    for (deck, roots), sv in zip(probs, b.deals):
        ref = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F32)
        ref.solve(200)
        torch.cuda.synchronize()
        for x, y in zip(state_arrays(sv.rounds), state_arrays(ref.rounds)):
            assert np.array_equal(x, y)
        ref.free()
    assert len(autotune.DEFAULT_CANDIDATES) == 18
    b.free()


def test_graph_replays_match_eager():
    pa = require_gpu()
    import torch
    probs = problems([1, 3])
    b = pa.BatchSolver(probs, 4, 200, dtype=pa.PASUR_F32)
    b.solve()
    torch.cuda.synchronize()
    eager = [state_arrays(sv.rounds) for sv in b.deals]
    b.capture()
    torch.cuda.synchronize()
    for rep in range(3):
        print(f"[graph] replay {rep}", flush=True)
        # the program's own eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        got = [state_arrays(sv.rounds) for sv in b.deals]
        for ge, gg in zip(eager, got):
            for x, y in zip(ge, gg):
                assert np.array_equal(x, y)
        del junk
    b.free()


def test_plan_rejects_bad_ranges():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F32)
    st = pa.CfrState(s.rounds[0].fgt, pa.PASUR_F32)
    with pytest.raises(pa.PasurError, match="t_first"):
        pa.Plan([st], t_first=0, t_last=10)
    p = pa.Plan([st], t_first=1, t_last=10)
    with pytest.raises(pa.PasurError, match="outside"):
        p.iterate(5, 10)
    st64 = pa.CfrState(s.rounds[0].fgt, pa.PASUR_F64)
    with pytest.raises(pa.PasurError, match="dtype"):
        pa.Plan([st, st64], t_first=1, t_last=10)
    p.free()


def test_batched_fp64_matches_oracle():
    # every deal of an FP64 batched solve against the oracle's solve of that
    # deal alone: state, average strategies and round values within 1e-9
    pa = require_gpu()
    import torch
    import oracle
    from gpu_common import oracle_rounds, oracle_solve
    seeds = [1, 3, 13]
    probs = problems(seeds)
    print(f"[batched] FP64 vs oracle, deals {seeds}, 300 iterations", flush=True)
    b = pa.BatchSolver(probs, 4, 300, dtype=pa.PASUR_F64)
    b.solve()
    torch.cuda.synchronize()
    for seed, (deck, roots), sv in zip(seeds, probs, b.deals):
        res = oracle_solve(oracle_rounds(deck, 4, roots), 300)
        for k, rr in enumerate(sv.rounds):
            c, leaf, V = res[k]
            st = rr.state
            assert np.array_equal(to_np(st.u[8]), leaf), (seed, k)
            for l in range(1, 9):
                for name, mine, field in (("sigma", st.sigma, oracle.CF_SIGMA),
                                          ("R", st.R, oracle.CF_R),
                                          ("Sbar", st.Sbar, oracle.CF_SBAR),
                                          ("sigma_bar", st.sigma_bar, oracle.CF_SIGMA_BAR)):
                    np.testing.assert_allclose(to_np(mine[l]), c.get(field, l), rtol=0, atol=1e-9,
                                               err_msg=f"deal {seed} round {k + 5} {name} {l}")
            for l in range(8):
                np.testing.assert_allclose(to_np(st.u[l]), c.get(oracle.CF_U, l), rtol=0, atol=1e-9)
            np.testing.assert_allclose(to_np(rr.V), V, rtol=0, atol=1e-9)
    b.free()


def test_plans_launch_in_any_order():
    # A plan with a larger LDS footprint, created before one with a smaller
    # footprint, must still launch (the dynamic-LDS ceiling is not the last
    # plan's), and give the same state as when built alone.
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(1)
    big = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F32).rounds[1]
    sdeck, sroots = synth.last_round_roots(3)
    small = pa.SubgameSolver(sdeck, 5, sroots, dtype=pa.PASUR_F32).rounds[0]
    outs = []
    for with_small in (False, True):
        st = pa.CfrState(big.fgt, pa.PASUR_F32)
        pa.leaf_utilities(big.fgt, None, pa.PASUR_F32, st.u[8])
        pa.cfr_init(st)
        pa_big = pa.Plan([st], t_first=1, t_last=50)
        if with_small:
            st2 = pa.CfrState(small.fgt, pa.PASUR_F32)
            pa_small = pa.Plan([st2], t_first=1, t_last=50)
            assert pa_small.lds_bytes < pa_big.lds_bytes
        pa_big.iterate(1, 50)
        torch.cuda.synchronize()
        outs.append([to_np(t).copy() for t in st.sigma[1:] + st.R[1:] + st.Sbar[1:]])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
