"""Self-play with average strategies (test infrastructure only).

Plain Python definition of the self-play the paper uses to estimate a
deck's fair value (section "Experimental Evaluation"): many games on one
deal, each walking the unfolded trees from the root; at each decision the
player to move samples an action from its strategy (the average strategy
of that node's children, or uniformly at random), at the end of a round the
game adds the round's points at the leaf reached and continues at the
linked next-round root.  The fair value is the fraction of games Alex wins
(final margin > 0).  One sampled action per game and decision, as the
paper's grouped multinomial sampling draws one child per row.

Random numbers: a counter-based SplitMix64 stream (the published SplitMix64
finaliser applied to seed + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64, the
generator's i-th state), so any draw can be computed on its own:
uniform(seed, i) = (z >> 11) * 2^-53 for draw i = game * 64 + round * 8 +
level.  A draw is used by inverse CDF: the first child whose running sum of
sigma-bar (FP64, in child order) exceeds u * total; uniform players take
child floor(u * k).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1
POLICY_SIGMA_BAR, POLICY_UNIFORM = 0, 1


def splitmix64(seed: int, i: int) -> int:
    """The i-th 64-bit output of SplitMix64 started at seed."""
    z = (seed + (i + 1) * GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix_uniform(seed: int, i: int) -> float:
    return (splitmix64(seed, i) >> 11) * (1.0 / (1 << 53))


def choose(u: float, probs: Sequence[float], policy: int) -> int:
    """Index of the sampled child."""
    k = len(probs)
    if k == 1:
        return 0
    if policy == POLICY_UNIFORM:
        return min(int(u * k), k - 1)
    total = 0.0
    for p in probs:
        total += float(p)
    if not total > 0.0:
        return min(int(u * k), k - 1)
    x = u * total
    acc = 0.0
    last = 0
    for c, p in enumerate(probs):
        acc += float(p)
        if float(p) > 0.0:
            last = c
        if acc > x:
            return c
    return last


def play(rounds: List[dict], n_games: int, seed: int, policy_a: int, policy_b: int,
         root: int = 0) -> np.ndarray:
    """rounds[r]: {"cb": [child_begin of levels 0..7], "sbar": [None, sigma-bar
    of levels 1..8], "link": next-root index per leaf (unused in the last
    round), "base": the round's points per leaf}.  Returns the final margin
    (Alex minus Bob, points) of every game."""
    out = np.zeros(n_games, np.int64)
    pol = (policy_a, policy_b)
    for g in range(n_games):
        q, m = root, 0
        for r, R in enumerate(rounds):
            for l in range(8):
                b, e = int(R["cb"][l][q]), int(R["cb"][l][q + 1])
                u = splitmix_uniform(seed, g * 64 + r * 8 + l)
                q = b + choose(u, R["sbar"][l + 1][b:e], pol[l & 1])
            m += int(round(R["base"][q]))
            if r + 1 < len(rounds):
                q = int(R["link"][q])
        out[g] = m
    return out
