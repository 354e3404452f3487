"""Seeded synthetic inputs for the Pasur round solver.

This module is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path (``paper_2508_06559_amd``).  It holds no game arithmetic: it only
draws random numbers and turns them into inputs (a 52-card deal and the
start states of a round subgame).  Every function is deterministic in its
seed.

Card indices follow the paper's fixed 52-slot layout (section "PyTorch-Based
Framework", figure "Mapping Cards to Indices"): index = 4*rank + suit with
rank A,2..10,J,Q,K = 0..12 and suit clubs, diamonds, hearts, spades = 0..3.

Deal layout (section "Pasur"): four face-up pool cards, then every round
four cards to Alex and four to Bob.  Here ``deck[0:4]`` is the initial pool
and round r (0-based) deals ``deck[4+8r : 8+8r]`` to Alex and
``deck[8+8r : 12+8r]`` to Bob.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

MASK64 = (1 << 64) - 1
JACKS = (40, 41, 42, 43)


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        return self.next() % n


def _fisher_yates(cards: List[int], rng: SplitMix64) -> None:
    for i in range(len(cards) - 1, 0, -1):
        j = rng.below(i + 1)
        cards[i], cards[j] = cards[j], cards[i]


def deal(seed: int) -> List[int]:
    """Seeded 52-card deal that satisfies the initial-pool Jack rule.

    The pool may hold no Jack (section "Pasur"): a single Jack among the first
    four cards goes to the bottom of the deck and the next card takes its
    place; two or more Jacks, or a Jack as the replacement, mean a reshuffle
    (Fisher-Yates again, continuing the same random stream).
    """
    rng = SplitMix64(seed)
    cards = list(range(52))
    while True:
        _fisher_yates(cards, rng)
        jacks = [i for i in range(4) if cards[i] in JACKS]
        if not jacks:
            return list(cards)
        if len(jacks) > 1:
            continue
        j = cards.pop(jacks[0])
        cards.append(j)
        if cards[3] in JACKS:
            continue
        return list(cards)


def round_hands(deck: List[int], rnd: int) -> Tuple[List[int], List[int]]:
    """Alex's and Bob's four dealt cards of round ``rnd`` (0-based)."""
    a = deck[4 + 8 * rnd: 8 + 8 * rnd]
    b = deck[8 + 8 * rnd: 12 + 8 * rnd]
    return list(a), list(b)


def mask_of(cards) -> int:
    m = 0
    for c in cards:
        m |= 1 << int(c)
    return m


@dataclass(frozen=True)
class Root:
    """A round root: the pool at the round start plus the inherited score.

    ``ca``/``cb``: clubs collected so far by Alex/Bob (0 once the bonus is
    decided), ``d``: point difference Alex-Bob so far, ``bonus``: 0 undecided,
    1 Alex has the 7-club bonus, 2 Bob has it.
    """
    pool: int
    ca: int
    cb: int
    d: int
    bonus: int

    def sort_key(self):
        return (self.pool, self.bonus, self.ca, self.cb, self.d)


def subgame_start(seed: int, rnd: int, deck: List[int] | None = None,
                  pool_min: int = 4, pool_max: int = 8):
    """Synthetic start state of round ``rnd`` >= 1 for a seeded deal.

    Recipe (no game rules are applied): the pool is a uniformly drawn subset
    of ``pool_min..pool_max`` non-Jack cards among those dealt before round
    ``rnd``; every other earlier-dealt club is credited to Alex or Bob by a
    fair coin, and a side holding 7 or more clubs gets the bonus (clubs then
    reset to 0, the paper's score normalisation).  Returns
    ``(deck, pool_mask, ca, cb, bonus, rng)``; ``rng`` continues the stream
    for further draws (e.g. the inherited point difference).
    """
    if deck is None:
        deck = deal(seed)
    if not 1 <= rnd <= 5:
        raise ValueError("subgame rounds are 1..5")
    rng = SplitMix64(seed ^ 0xA5A5A5A5A5A5A5A5)
    prior = deck[: 4 + 8 * rnd]
    cand = [c for c in prior if c not in JACKS]
    k = pool_min + rng.below(pool_max - pool_min + 1)
    k = min(k, len(cand))
    cand = list(cand)
    _fisher_yates(cand, rng)
    pool_cards = sorted(cand[:k])
    pool = mask_of(pool_cards)
    ca = cb = 0
    for c in prior:
        if c % 4 == 0 and not (pool >> c) & 1:
            if rng.below(2) == 0:
                ca += 1
            else:
                cb += 1
    bonus = 0
    if ca >= 7:
        bonus, ca, cb = 1, 0, 0
    elif cb >= 7:
        bonus, ca, cb = 2, 0, 0
    return deck, pool, ca, cb, bonus, rng


def last_round_roots(seed: int, deltas=range(-3, 4)):
    """Roots of a final-round-only subgame: one pool, one club state and one
    root per inherited point difference in ``deltas``."""
    deck, pool, ca, cb, bonus, _ = subgame_start(seed, 5)
    roots = sorted((Root(pool, ca, cb, int(d), bonus) for d in deltas),
                   key=Root.sort_key)
    return deck, roots


def two_round_root(seed: int):
    """Single root of a two-round subgame (the last two rounds) with a
    seeded inherited point difference in -5..5."""
    deck, pool, ca, cb, bonus, rng = subgame_start(seed, 4)
    d = rng.below(11) - 5
    return deck, [Root(pool, ca, cb, d, bonus)]


def full_game_root(seed: int):
    """Root of a full six-round game: the initial pool, score all zero."""
    deck = deal(seed)
    return deck, [Root(mask_of(deck[:4]), 0, 0, 0, 0)]


def subgame_roots(seed: int, rnd: int):
    """Single root of a subgame that starts at round ``rnd``."""
    if rnd == 0:
        return full_game_root(seed)
    deck, pool, ca, cb, bonus, rng = subgame_start(seed, rnd)
    d = rng.below(11) - 5
    return deck, [Root(pool, ca, cb, d, bonus)]


def playout_draws(seed: int, rounds: int) -> List[int]:
    """Random 64-bit draws for a seeded playout of ``rounds`` rounds from the
    initial deal (eight moves per round): move i takes the legal move number
    ``draws[i] mod k`` among the k legal moves in canonical order.  Only the
    random numbers live here; each side plays the moves with its own rules."""
    rng = SplitMix64(seed ^ 0x3C6EF372FE94F82B)
    return [rng.next() for _ in range(8 * rounds)]


# Deck of the paper's worked example (table "Initial setup for a single game
# instance" and the first row of every round of the step-by-step gameplay
# figure): pool, then per round Alex's and Bob's four cards.
DECK9 = [0, 3, 33, 49,
         12, 13, 25, 44, 9, 10, 16, 51,
         20, 21, 34, 40, 22, 24, 41, 50,
         17, 32, 38, 48, 1, 23, 28, 31,
         4, 8, 43, 47, 27, 29, 30, 46,
         14, 15, 26, 42, 5, 18, 35, 39,
         2, 11, 36, 45, 6, 7, 19, 37]
