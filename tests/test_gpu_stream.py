"""The HBM-streaming schedule (PASUR_SCHED_STREAM) against the persistent
segment schedule and the FP64 oracle.

The streaming sweeps keep no strategy array inside a call and do not iterate
chains of single-child nodes.  Every state array must equal the other
schedules' bit for bit, except the average-strategy sums of edges below a
node whose subtree is such a chain ("passive"): those are not accumulated,
and their average strategy must still be exactly 1."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import oracle_rounds, oracle_solve, require_gpu, to_np

pytestmark = pytest.mark.gpu


def skipped_edges(child_begin):
    """Per level 1..8, True for edges whose parent is passive (one child, and
    that child a leaf or passive), computed on the host from the CSR."""
    cb = [np.asarray(c, np.int64) for c in child_begin]  # levels 0..7
    passive = [None] * 8  # levels 1..7
    for l in range(7, 0, -1):
        first = cb[l][:-1]
        k = cb[l][1:] - first
        below = np.ones(len(k), bool)
        if l < 7:
            has = k >= 1
            below = np.zeros(len(k), bool)
            below[has] = passive[l + 1][first[has]]
        passive[l] = (k == 1) & below
    out = [None, np.zeros(int(cb[0][-1]), bool)]  # level 1: parents are roots
    for L in range(2, 9):
        out.append(np.repeat(passive[L - 1], cb[L - 1][1:] - cb[L - 1][:-1]))
    return out


def state_arrays(st):
    return {"sigma": [to_np(t).copy() for t in st.sigma[1:]],
            "R": [to_np(t).copy() for t in st.R[1:]],
            "Sbar": [to_np(t).copy() for t in st.Sbar[1:]],
            "sigma_bar": [to_np(t).copy() for t in st.sigma_bar[1:]],
            "reachA": [to_np(t).copy() for t in st.reachA[:8]],
            "reachB": [to_np(t).copy() for t in st.reachB[:8]],
            "u": [to_np(t).copy() for t in st.u],
            "vacc": [to_np(st.vacc).copy()]}


def solve(pa, deck, start, roots, dtype, iters, sched, params=None):
    import torch
    s = pa.SubgameSolver(deck, start, roots, dtype=dtype)
    p = params if params is not None else pa.paper_params(sched)
    p.schedule = sched
    s.solve(iters, p)
    torch.cuda.synchronize()
    return s


# deals whose trees have non-chain nodes on levels 6 and 7 (so the compact
# tail has two levels), one whose level 6 is all chains, and ones with
# sibling groups of 8 to 22 children (the up sweep's per-child form for wide
# levels: seeds 1 and 22)
CASES = [("two-round 1", lambda: (4, synth.two_round_root(1))),
         ("two-round 13", lambda: (4, synth.two_round_root(13))),
         ("two-round 38", lambda: (4, synth.two_round_root(38))),
         ("two-round 22", lambda: (4, synth.two_round_root(22))),
         ("last-round 2", lambda: (5, synth.last_round_roots(2)))]


@pytest.mark.parametrize("dtype_name", ["PASUR_F32", "PASUR_F64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_stream_equals_segment_schedule(dtype_name, case):
    pa = require_gpu()
    name, mk = CASES[case]
    start, (deck, roots) = mk()
    dtype = getattr(pa, dtype_name)
    print(f"[stream] {name} {dtype_name} 300 iterations", flush=True)
    a = solve(pa, deck, start, roots, dtype, 300, pa.SCHED_ROOT)
    b = solve(pa, deck, start, roots, dtype, 300, pa.SCHED_STREAM)
    for ra, rb in zip(a.rounds, b.rounds):
        cb = [ra.fgt.read(pa.FGT_CHILD_BEGIN, l) for l in range(8)]
        skip = skipped_edges(cb)
        A, B = state_arrays(ra.state), state_arrays(rb.state)
        for key in ("sigma", "R", "sigma_bar", "reachA", "reachB", "u", "vacc"):
            for l, (x, y) in enumerate(zip(A[key], B[key])):
                assert np.array_equal(x, y), (name, key, l)
        for l in range(1, 9):
            m = skip[l]
            assert np.array_equal(A["Sbar"][l - 1][~m], B["Sbar"][l - 1][~m]), (name, l)
            assert (B["Sbar"][l - 1][m] == 0).all()
            assert (B["sigma_bar"][l - 1][m] == 1).all()
        assert np.array_equal(to_np(ra.V), to_np(rb.V))
    # the last round of these subgames has passive chains to skip
    assert skipped_edges([b.rounds[-1].fgt.read(pa.FGT_CHILD_BEGIN, l) for l in range(8)])[8].any()


def test_stream_fp64_two_round_matches_oracle():
    # a two-round subgame whose compact tail has non-chain nodes on levels 6
    # and 7 in both rounds, 300 iterations per round, against the oracle
    pa = require_gpu()
    deck, roots = synth.two_round_root(13)
    print("[stream] fp64 two-round 13 vs oracle", flush=True)
    s = solve(pa, deck, 4, roots, pa.PASUR_F64, 300, pa.SCHED_STREAM)
    rounds = oracle_rounds(deck, 4, roots)
    res = oracle_solve(rounds, 300)
    for k in (0, 1):
        c, leaf, V = res[k]
        st = s.rounds[k].state
        skip = skipped_edges(rounds[k][1].child_begin())
        for l in range(1, 9):
            m = ~skip[l]
            np.testing.assert_allclose(to_np(st.R[l]), c.get(oracle.CF_R, l), rtol=0, atol=1e-9)
            np.testing.assert_allclose(to_np(st.Sbar[l])[m], c.get(oracle.CF_SBAR, l)[m], rtol=0,
                                       atol=1e-9)
            np.testing.assert_allclose(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l),
                                       rtol=0, atol=1e-9)
        for l in range(8):
            np.testing.assert_allclose(to_np(st.u[l]), c.get(oracle.CF_U, l), rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(s.rounds[k].V), V, rtol=0, atol=1e-9)


@pytest.mark.parametrize("variant,rm", [(oracle.CFR_DCFR, oracle.RM_FLOOR),
                                        (oracle.CFR_PLUS, oracle.RM_POSITIVE),
                                        (oracle.CFR_VANILLA, oracle.RM_POSITIVE)])
def test_stream_fp64_matches_oracle(variant, rm):
    pa = require_gpu()
    deck, roots = synth.last_round_roots(3)
    print(f"[stream] fp64 vs oracle variant={variant} rm={rm}", flush=True)
    params = pa.CfrParams(variant, rm, 1.5, 0.0, 2.0, 1e-8, pa.SCHED_STREAM, 0, 0)
    s = solve(pa, deck, 5, roots, pa.PASUR_F64, 400, pa.SCHED_STREAM, params)
    rounds = oracle_rounds(deck, 5, roots)
    (c, leaf, V), = oracle_solve(rounds, 400, oracle.Params(variant=variant, rm_mode=rm))
    st = s.rounds[0].state
    skip = skipped_edges(rounds[0][1].child_begin())
    for l in range(1, 9):
        m = ~skip[l]
        np.testing.assert_allclose(to_np(st.sigma[l]), c.get(oracle.CF_SIGMA, l), rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(st.R[l]), c.get(oracle.CF_R, l), rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(st.Sbar[l])[m], c.get(oracle.CF_SBAR, l)[m], rtol=0,
                                   atol=1e-9)
        np.testing.assert_allclose(to_np(st.sigma_bar[l]), c.get(oracle.CF_SIGMA_BAR, l), rtol=0,
                                   atol=1e-9)
    for l in range(8):
        np.testing.assert_allclose(to_np(st.u[l]), c.get(oracle.CF_U, l), rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(st.reachA[l]), c.get(oracle.CF_REACHA, l), rtol=0, atol=1e-9)
        np.testing.assert_allclose(to_np(st.reachB[l]), c.get(oracle.CF_REACHB, l), rtol=0, atol=1e-9)
    np.testing.assert_allclose(to_np(s.rounds[0].V), V, rtol=0, atol=1e-9)


def test_stream_split_calls_equal_one_call():
    # sigma is read on a call's first iteration and written after its last,
    # so 1 + 122 + 377 iterations must equal 500 at once, bit for bit.
    pa = require_gpu()
    import torch
    deck, roots = synth.two_round_root(2)
    outs = []
    for split in ((500,), (1, 122, 377)):
        s = pa.SubgameSolver(deck, 4, roots, dtype=pa.PASUR_F32)
        rr = s.rounds[1]
        st = pa.CfrState(rr.fgt, pa.PASUR_F32)
        pa.leaf_utilities(rr.fgt, None, pa.PASUR_F32, st.u[8])
        pa.cfr_init(st)
        for k in split:
            pa.cfr_iterate(st, k, pa.paper_params(pa.SCHED_STREAM))
        torch.cuda.synchronize()
        outs.append([to_np(t).copy() for t in st.sigma[1:] + st.R[1:] + st.Sbar[1:] + st.u[:8]]
                    + [to_np(st.vacc).copy()])
        s.free()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_auto_schedule_picks_stream_only_for_large_rounds():
    # AUTO equals ROOT on a small subgame (every Sbar accumulated).
    pa = require_gpu()
    deck, roots = synth.last_round_roots(4)
    a = solve(pa, deck, 5, roots, pa.PASUR_F32, 200, pa.SCHED_ROOT)
    b = solve(pa, deck, 5, roots, pa.PASUR_F32, 200, pa.SCHED_AUTO)
    for x, y in zip(state_arrays(a.rounds[0].state)["Sbar"], state_arrays(b.rounds[0].state)["Sbar"]):
        assert np.array_equal(x, y)
