"""The paper's executed readings as flags, through the C ABI against the
FP64 oracle run with the same flags: literal_bonus0 (equation final_util as
printed), snippet_tol and snippet_avg (CodeSnippet FindUtility's sign test
and average update).  The CFR flags run on the level-synchronous schedule,
which AUTO picks for them; other schedules and plans reject them."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import oracle_rounds, require_gpu, to_np

pytestmark = pytest.mark.gpu


def no_club_deal():
    # the last round's hands and pool hold no club, so no leaf can win the
    # 7-club bonus: a root without it ends at bonus 0 everywhere
    nonclubs = [c for c in range(52) if c % 4]
    clubs = [c for c in range(52) if c % 4 == 0]
    deck = nonclubs[:4] + clubs + nonclubs[4:]
    pool = synth.mask_of(deck[:4])
    return deck, [synth.Root(pool, 0, 0, 0, 0), synth.Root(pool, 0, 0, 0, 1)]


@pytest.mark.parametrize("dtype_name", ["PASUR_F32", "PASUR_F64"])
def test_literal_bonus0_leaf_utilities(dtype_name):
    pa = require_gpu()
    import torch
    deck, roots = no_club_deal()
    dtype = getattr(pa, dtype_name)
    print(f"[readings] literal_bonus0 leaf utilities {dtype_name}", flush=True)
    s = pa.SubgameSolver(deck, 5, roots, dtype=dtype)
    (gt, f), = oracle_rounds(deck, 5, roots)
    rr = s.rounds[0]
    tdt = torch.float32 if dtype == pa.PASUR_F32 else torch.float64
    for literal in (False, True):
        out = torch.empty(rr.fgt.n[8], dtype=tdt, device="cuda")
        pa.leaf_utilities(rr.fgt, None, dtype, out, literal_bonus0=literal)
        torch.cuda.synchronize()
        want = f.leaf_utilities(literal_bonus0=literal)
        np.testing.assert_array_equal(to_np(out).astype(np.float64), want)
    assert (f.leaf_utilities(literal_bonus0=True) != f.leaf_utilities()).any()
    s.free()


def test_literal_bonus0_solve_and_exploitability():
    pa = require_gpu()
    import torch
    deck, roots = no_club_deal()
    print("[readings] literal_bonus0 solve, FP64, 200 iterations", flush=True)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F64, literal_bonus0=True)
    s.solve(200)
    torch.cuda.synchronize()
    (gt, f), = oracle_rounds(deck, 5, roots)
    leaf = f.leaf_utilities(literal_bonus0=True)
    c = oracle.CFR(f.n, f.child_begin(), leaf)
    c.run(200)
    np.testing.assert_allclose(to_np(s.rounds[0].V), c.get(oracle.CF_VACC) / 200, rtol=0, atol=1e-9)
    sb = c.sigma_bar()
    gbra, gbrb, gv = (to_np(x) for x in s.exploitability())
    for got, mode in ((gbra, oracle.TV_BR_A), (gbrb, oracle.TV_BR_B), (gv, oracle.TV_EXPECT)):
        np.testing.assert_allclose(got, oracle.tree_values(f.n, f.child_begin(), leaf, sb, mode),
                                   rtol=0, atol=1e-9)
    s.free()


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("flags", [1, 2, 3])
@pytest.mark.parametrize("sched_name", ["SCHED_LEVEL_SYNC", "SCHED_AUTO"])
def test_snippet_flags_match_oracle(seed, flags, sched_name):
    pa = require_gpu()
    import torch
    deck, roots = synth.last_round_roots(seed)
    print(f"[readings] snippet flags {flags} {sched_name} seed {seed}, FP64, 300 iterations",
          flush=True)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F64)
    s.solve(300, pa.paper_params(getattr(pa, sched_name), flags=flags))
    torch.cuda.synchronize()
    (gt, f), = oracle_rounds(deck, 5, roots)
    c = oracle.CFR(f.n, f.child_begin(), f.leaf_utilities())
    c.run(300, oracle.Params(flags=flags))
    st = s.rounds[0].state
    for l in range(1, 9):
        for name, mine, field in (("sigma", st.sigma, oracle.CF_SIGMA), ("R", st.R, oracle.CF_R),
                                  ("Sbar", st.Sbar, oracle.CF_SBAR),
                                  ("sigma_bar", st.sigma_bar, oracle.CF_SIGMA_BAR)):
            np.testing.assert_allclose(to_np(mine[l]), c.get(field, l), rtol=0, atol=1e-9,
                                       err_msg=f"{name} level {l}")
    for l in range(8):
        np.testing.assert_allclose(to_np(st.u[l]), c.get(oracle.CF_U, l), rtol=0, atol=1e-9)
    np.testing.assert_allclose(to_np(s.rounds[0].V), c.get(oracle.CF_VACC) / 300, rtol=0, atol=1e-9)
    s.free()


def test_snippet_flags_rejected_elsewhere():
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    s = pa.SubgameSolver(deck, 5, roots, dtype=pa.PASUR_F32)
    rr = s.rounds[0]
    st = pa.CfrState(rr.fgt, pa.PASUR_F32)
    pa.leaf_utilities(rr.fgt, None, pa.PASUR_F32, st.u[8])
    pa.cfr_init(st)
    for sched in (pa.SCHED_ROOT, pa.SCHED_STREAM, pa.SCHED_ROOT_GLOBAL):
        with pytest.raises(pa.PasurError, match="LEVEL_SYNC"):
            pa.cfr_iterate(st, 1, pa.paper_params(sched, flags=pa.SNIPPET_AVG))
    p = pa.CfrParams(pa.CFR_PLUS, pa.RM_POSITIVE, 0.0, 0.0, 0.0, 0.0, pa.SCHED_LEVEL_SYNC, 0, 0,
                     pa.SNIPPET_TOL)
    with pytest.raises(pa.PasurError, match="DCFR only"):
        pa.cfr_iterate(st, 1, p)
    with pytest.raises(pa.PasurError, match="flags"):
        pa.cfr_iterate(st, 1, pa.paper_params(pa.SCHED_LEVEL_SYNC, flags=4))
    with pytest.raises(pa.PasurError, match="plans"):
        pa.Plan([st], pa.paper_params(pa.SCHED_ROOT, flags=pa.SNIPPET_TOL), 1, 10)
    s.free()
