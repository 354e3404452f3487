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
