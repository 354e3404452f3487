"""External-sampling CFR on one round's unfolded tree (test infrastructure only).

Section "External Sampling" (figures on the sampled t_edg / t_fgm and
CodeSnippet ExternalSampling): while the tree is unfolded, the opponent of
the player being updated keeps a single action per node, drawn from its
current strategy, while the updated player keeps all of its actions.  The
paper gives only this sampling step; the CFR around it here is the standard
external-sampling scheme (Lanctot et al., "Monte Carlo Sampling for Regret
Minimization in Extensive Games", 2009) with alternating updates:

  for t = t0+1 .. t0+n, for p in (Alex, Bob):
    walk the tree from every root;
    at a node of p: visit every child; the node's value is the sum over
      children of sigma * value; each child's regret gains its value minus
      the node's value (from p's side: negated for Bob, since utilities are
      Alex minus Bob); the children's strategy is then regret-matched;
    at a node of the opponent: add the current strategy of its children to
      their average sums; draw one child from that strategy and return its
      value;
    a leaf returns its utility.

Sampling weights cancel in this scheme (the opponent's reach is the sampling
probability), so regrets and average sums are plain, unweighted sums.

Draws: SplitMix64 as a counter-based generator (the published finaliser
applied to seed + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64), uniform u = top
53 bits * 2^-53.  The opponent node h of level l (0..7) in the pass of
player p (0 Alex, 1 Bob) at iteration t (1-based) uses draw
  i = (2 (t - 1) + p) * N + off[l] + h,   N = n_0 + ... + n_7,
  off[l] = n_0 + ... + n_(l-1).
The child taken is the first whose running FP64 sum of sigma exceeds
u * (sum of the siblings' sigma); a node with one child draws nothing.

Regret matching: sigma = max(R, eps) / sum over siblings (the paper's
floor, rm_mode "floor") or max(R, 0) / sum ("positive"), uniform where the
sum is 0.  Alex moves at even levels, Bob at odd levels.  Arithmetic is
FP64.
"""
from typing import List, Sequence

import numpy as np

from .selfplay import POLICY_SIGMA_BAR, choose, splitmix_uniform


def _match(R: np.ndarray, rm_mode: str, eps: float) -> np.ndarray:
    k = len(R)
    xs = [max(float(r), eps) if rm_mode == "floor" else max(float(r), 0.0) for r in R]
    s = 0.0
    for x in xs:
        s += x
    if s > 0.0:
        return np.array([x / s for x in xs])
    return np.full(k, 1.0 / k)


class ESState:
    """Current strategy, cumulative regret and cumulative strategy per edge
    (arrays of levels 1..8, index = child node), initialised as plain CFR
    starts: uniform strategy, zero sums."""

    def __init__(self, n: Sequence[int], child_begin: List[np.ndarray]):
        self.n = [int(x) for x in n]
        self.cb = [np.asarray(c, np.int64) for c in child_begin]
        self.sigma = [None] + [np.zeros(self.n[l]) for l in range(1, 9)]
        self.R = [None] + [np.zeros(self.n[l]) for l in range(1, 9)]
        self.Sbar = [None] + [np.zeros(self.n[l]) for l in range(1, 9)]
        for l in range(8):
            cb = self.cb[l]
            for h in range(self.n[l]):
                b, e = int(cb[h]), int(cb[h + 1])
                if e > b:
                    self.sigma[l + 1][b:e] = 1.0 / (e - b)
        self.t = 0

    def sigma_bar(self) -> List[np.ndarray]:
        """Average strategy: Sbar normalised over siblings, uniform where the
        sum is 0."""
        out = [np.ones(self.n[0])]
        for l in range(1, 9):
            sb = np.zeros(self.n[l])
            cb = self.cb[l - 1]
            for h in range(self.n[l - 1]):
                b, e = int(cb[h]), int(cb[h + 1])
                s = 0.0
                for q in range(b, e):
                    s += self.Sbar[l][q]
                for q in range(b, e):
                    sb[q] = self.Sbar[l][q] / s if s > 0.0 else 1.0 / (e - b)
            out.append(sb)
        return out


def es_iterate(st: ESState, leaf_u: np.ndarray, n_iters: int, seed: int,
               rm_mode: str = "floor", eps: float = 1e-8) -> None:
    """n_iters external-sampling iterations (both players' passes each),
    continuing from iteration st.t."""
    n, cb = st.n, st.cb
    N = sum(n[:8])
    off = [sum(n[:l]) for l in range(9)]

    def walk(l: int, h: int, p: int, base: int) -> float:
        if l == 8:
            return float(leaf_u[h])
        b, e = int(cb[l][h]), int(cb[l][h + 1])
        sig = st.sigma[l + 1]
        if (l & 1) == p:
            vals = [walk(l + 1, c, p, base) for c in range(b, e)]
            v = 0.0
            for j, c in enumerate(range(b, e)):
                v += sig[c] * vals[j]
            R = st.R[l + 1]
            for j, c in enumerate(range(b, e)):
                R[c] = R[c] + ((vals[j] - v) if p == 0 else (v - vals[j]))
            sig[b:e] = _match(R[b:e], rm_mode, eps)
            return v
        Sb = st.Sbar[l + 1]
        for c in range(b, e):
            Sb[c] = Sb[c] + sig[c]
        u = splitmix_uniform(seed, base + off[l] + h) if e - b > 1 else 0.0
        j = choose(u, sig[b:e], POLICY_SIGMA_BAR)
        return walk(l + 1, b + j, p, base)

    for _ in range(n_iters):
        st.t += 1
        for p in (0, 1):
            base = (2 * (st.t - 1) + p) * N
            for r in range(n[0]):
                walk(0, r, p, base)
