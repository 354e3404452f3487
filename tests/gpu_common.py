"""Helpers shared by the GPU parity tests: run the HIP path through its C ABI
and the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False


def require_gpu():
    if not HAVE_GPU:
        pytest.fail("GPU test run without a GPU")
    import paper_2508_06559_amd as pa
    pa.lib()
    return pa


def roots_from_array(arr):
    return [synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]), int(x["bonus"]))
            for x in arr]


def oracle_rounds(deck, start, roots):
    """Oracle GT/FGT of every round from ``start`` to 5."""
    out = []
    for r in range(start, 6):
        gt = oracle.GT(deck, r, sorted({x.pool for x in roots}))
        f = oracle.FGT(gt, roots)
        out.append((gt, f))
        if r < 5:
            roots = roots_from_array(f.get(oracle.FGT_NEXT_ROOTS))
    return out


def oracle_solve(rounds, iters, params=None):
    """Backward DCFR with the oracle; returns per round (CFR, leaf_u, V)."""
    params = params or oracle.Params()
    res = [None] * len(rounds)
    V = None
    for k in range(len(rounds) - 1, -1, -1):
        gt, f = rounds[k]
        leaf = f.leaf_utilities(V)
        c = oracle.CFR(f.n, f.child_begin(), leaf)
        c.run(iters, params)
        V = c.get(oracle.CF_VACC) / iters
        res[k] = (c, leaf, V)
    return res


def oracle_exploitability(rounds, sbars):
    """Composed BR_A, BR_B, v at the first round's roots for the given
    per-round average strategies."""
    vals = {}
    for mode in (oracle.TV_BR_A, oracle.TV_BR_B, oracle.TV_EXPECT):
        V = None
        for k in range(len(rounds) - 1, -1, -1):
            gt, f = rounds[k]
            leaf = f.leaf_utilities(V)
            V = oracle.tree_values(f.n, f.child_begin(), leaf, sbars[k], mode)
        vals[mode] = V
    return vals[oracle.TV_BR_A], vals[oracle.TV_BR_B], vals[oracle.TV_EXPECT]


def to_np(t):
    return t.detach().cpu().numpy()
