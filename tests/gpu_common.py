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


NEAR_TIE = 1e-3


def tie_groups(f, leaf, tol=NEAR_TIE):
    """Per level l = 1..8, a group id for every edge: the children of one
    parent whose minimax values (oracle, exact tree values) agree within tol
    share an id.  Such actions are equally good, or so nearly equal that
    DCFR has not separated them after a few thousand iterations; the split
    of the average strategy among them is not unique (in the last round the
    leaf values are integers, so only exact ties group)."""
    cb = f.child_begin()
    groups = [None]
    for l in range(1, 9):
        mm = oracle.tree_values(f.n, cb, leaf, None, oracle.TV_MINIMAX, level=l)
        b = np.asarray(cb[l - 1], np.int64)
        gid = np.empty(len(mm), np.int64)
        nxt = 0
        for h in range(len(b) - 1):
            vals = mm[b[h]:b[h + 1]]
            seen = []
            for j, v in enumerate(vals):
                for gv, g in seen:
                    if abs(gv - v) <= tol:
                        gid[b[h] + j] = g
                        break
                else:
                    seen.append((v, nxt))
                    gid[b[h] + j] = nxt
                    nxt += 1
        groups.append(gid)
    return groups


def path_reach(child_begin, sigma_bar):
    """Per level l = 0..7, the probability that play under the average
    profile passes through each node: the product of sigma-bar along the
    path from the root (both players' moves)."""
    cb = [np.asarray(c, np.int64) for c in child_begin]
    out = [np.ones(len(cb[0]) - 1)]
    for l in range(1, 8):
        par = np.repeat(np.arange(len(cb[l - 1]) - 1), np.diff(cb[l - 1]))
        out.append(out[-1][par] * np.asarray(sigma_bar[l], np.float64))
    return out


def assert_sigma_bar_up_to_ties(gpu_sb, oracle_sb, groups, child_begin, tol, what=""):
    """Average strategies compared by how often each action is played: for
    every untied action, |gpu - oracle| times the probability that play
    under the average profile reaches its parent (the smaller of the two
    profiles' probabilities) within tol, and the same for the total of every
    tie group.  Behaviour at a node that play does not reach is not fixed by
    an equilibrium (it rests on regrets scaled by a vanishing reach and is
    set by rounding); its effect is what exploitability measures.  Returns
    (actions in tie groups, actions, largest unweighted difference at
    parents reached with probability >= 0.5)."""
    xo = path_reach(child_begin, oracle_sb)
    xg = path_reach(child_begin, gpu_sb)
    cb = [np.asarray(c, np.int64) for c in child_begin]
    tied, total, big = 0, 0, 0.0
    for l in range(1, 9):
        g = groups[l]
        a = np.asarray(gpu_sb[l], np.float64)
        b = np.asarray(oracle_sb[l], np.float64)
        par = np.repeat(np.arange(len(cb[l - 1]) - 1), np.diff(cb[l - 1]))
        w = np.minimum(xo[l - 1], xg[l - 1])[par]
        size = np.bincount(g)
        single = size[g] == 1
        tied += int((~single).sum())
        total += len(g)
        d = np.abs(a - b)
        if single.any():
            dw = d[single] * w[single]
            assert dw.max() <= tol, (what, l, int(np.nonzero(single)[0][np.argmax(dw)]),
                                     float(dw.max()))
            hi = single & (w >= 0.5)
            if hi.any():
                big = max(big, float(d[hi].max()))
        sa = np.bincount(g, a, len(size))
        sb = np.bincount(g, b, len(size))
        gw = np.zeros(len(size))
        gw[g] = w
        dg = np.abs(sa - sb) * gw
        assert dg.max() <= tol, (what, l, "group sums", float(dg.max()))
    return tied, total, big
