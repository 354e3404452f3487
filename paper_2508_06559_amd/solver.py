"""Round-by-round driver over the libpasur calls (CodeSnippet CFR, runcfr).

Forward: build and unfold every round from the start round to round 5,
chaining each round's next-round roots (device memory) into the next build.
Backward: solve round 5 first; each solved round passes its root values to
the previous round's leaves (equation passuputil).  Exploitability composes
best responses across rounds the same way.  Control flow only: every step is
a libpasur kernel.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

from . import (PASUR_F32, PASUR_F64, PLAY_SIGMA_BAR, RM_FLOOR, SCHED_STREAM, V_ITERATE_MEAN,
               V_SIGMA_BAR, ES_FRONTIER, CfrParams, FGT_CHILD_BEGIN, FGT_LINK, FGT_NEXT_ROOTS, ROOT_DTYPE, CfrState,
               es_iterate, exploitability, selfplay, Plan, UnfoldedTree,
               average_strategy, build_round_tree, cfr_init, cfr_iterate, leaf_utilities,
               paper_params, round_values, roots_to_device, unfold_scores, _torch)


@dataclass
class RoundResult:
    round: int
    fgt: UnfoldedTree
    state: Optional[CfrState] = None
    V: Optional[object] = None  # device double tensor, one value per root
    gt: Optional[object] = None  # the round's game tree, kept when features are needed


class SubgameSolver:
    """All rounds from ``start_round`` to 5 of one deal."""

    def __init__(self, deck, start_round: int, roots, dtype: int = PASUR_F32, stream=None,
                 keep_gt: bool = False, literal_bonus0: bool = False):
        torch = _torch()
        self.deck = list(int(c) for c in deck)
        self.start = start_round
        self.dtype = dtype
        self.literal_bonus0 = literal_bonus0  # leaf utilities: the printed final_util
        self.stream = stream
        self.rounds: List[RoundResult] = []
        d_roots = roots_to_device(roots)
        self._root_tensor = d_roots
        ptr, n = d_roots.data_ptr(), len(roots)
        for r in range(start_round, 6):
            gt = build_round_tree(self.deck, r, ptr, n, stream)
            fgt = unfold_scores(gt, ptr, n, stream)
            if not keep_gt:
                gt.free()
                gt = None
            self.rounds.append(RoundResult(r, fgt, gt=gt))
            if r < 5:
                ptr, n = fgt.next_roots_device()
        self.torch = torch

    def sizes(self):
        return [rr.fgt.n for rr in self.rounds]

    def edges(self) -> int:
        return sum(rr.fgt.edges() for rr in self.rounds)

    def solve(self, iters: int, params=None, value_mode: int = V_ITERATE_MEAN,
              round_events=None, on_round=None):
        """Backward DCFR: ``iters`` iterations per round.  If ``round_events``
        is a list, a (start, end) pair of CUDA events around each round's
        iterations is appended to it (last round first).  ``on_round(r)``,
        if given, is called on the host once round r's iterations are
        enqueued (last round first)."""
        torch = self.torch
        params = params if params is not None else paper_params()
        V = None
        for rr in reversed(self.rounds):
            st = rr.state if rr.state is not None else CfrState(rr.fgt, self.dtype)
            rr.state = st
            leaf_utilities(rr.fgt, V, self.dtype, st.u[8], self.stream, self.literal_bonus0)
            cfr_init(st, self.stream)
            if round_events is not None:
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                ev[0].record()
            cfr_iterate(st, iters, params, stream=self.stream)
            if round_events is not None:
                ev[1].record()
                round_events.append(ev)
            if on_round is not None:
                on_round(rr.round)
            average_strategy(st, self.stream)
            rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
            round_values(st, value_mode, rr.V, self.stream)
            V = rr.V
        return self.rounds[0].V

    def solve_es(self, iters: int, seed: int, rm_mode: int = RM_FLOOR, eps: float = 1e-8,
                 schedule: int = ES_FRONTIER):
        """Backward solve with external-sampling CFR (pasur_es_iterate):
        ``iters`` iterations per round, last round first; each round passes
        back the value of its average strategy, v(sigma-bar), as the next
        earlier round's leaf values."""
        torch = self.torch
        V = None
        for rr in reversed(self.rounds):
            st = rr.state if rr.state is not None else CfrState(rr.fgt, self.dtype)
            rr.state = st
            leaf_utilities(rr.fgt, V, self.dtype, st.u[8], self.stream, self.literal_bonus0)
            cfr_init(st, self.stream)
            es_iterate(st, iters, seed, rm_mode, eps, schedule=schedule, stream=self.stream)
            average_strategy(st, self.stream)
            rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
            round_values(st, V_SIGMA_BAR, rr.V, self.stream)
            V = rr.V
        return self.rounds[0].V

    def exploitability(self):
        """Composed best responses of both players against the average
        strategies of every round (pasur_exploitability); returns (BR_A, BR_B,
        v) at the start round's roots as device double tensors.
        Exploitability (points per game) is (BR_A - BR_B) / 2."""
        torch = self.torch
        n0 = self.rounds[0].fgt.n[0]
        out = [torch.empty(n0, dtype=torch.float64, device="cuda") for _ in range(3)]
        exploitability([rr.fgt for rr in self.rounds], [rr.state.sigma_bar for rr in self.rounds],
                       self.dtype, out[0], out[1], out[2], self.stream, self.literal_bonus0)
        return tuple(out)

    def selfplay(self, n_games: int, seed: int, policy_a: int = PLAY_SIGMA_BAR,
                 policy_b: int = PLAY_SIGMA_BAR, root: int = 0, strategies=None):
        """Margins (Alex minus Bob, int32 device tensor) of n_games self-play
        games from start-round root `root` (pasur_selfplay).  A non-uniform
        player samples from the solved average strategies, or from
        `strategies[r][l]` (per round, levels 1..8, the solver's dtype: any
        per-edge strategy, e.g. a network's prediction) when given."""
        torch = self.torch
        margin = torch.empty(max(n_games, 1), dtype=torch.int32, device="cuda")
        sb = strategies if strategies is not None else [rr.state.sigma_bar for rr in self.rounds]
        selfplay([rr.fgt for rr in self.rounds], sb, self.dtype, root, n_games, seed, policy_a,
                 policy_b, margin, self.stream)
        return margin[:n_games]

    def free(self):
        for rr in self.rounds:
            rr.fgt.free()
            if rr.gt is not None:
                rr.gt.free()
        self.rounds = []


def playout_root(deck, rnd: int, draws, stream=None):
    """Start state of round ``rnd`` reached by a seeded legal playout from the
    initial deal (section "Pasur"): each round's tree is built and unfolded
    by the library from the current root alone (pasur_build_round_tree,
    pasur_unfold_scores), move i takes the child ``draws[i] mod k`` of the
    current node among its k children (canonical order), and the leaf's link
    gives the next round's root.  Returns (pool, ca, cb, d, bonus) as a
    ROOT_DTYPE record."""
    import numpy as np
    root = np.zeros(1, ROOT_DTYPE)
    root[0] = (_initial_pool(deck), 0, 0, 0, 0, 0)
    i = 0
    for r in range(rnd):
        d_root = roots_to_device(root)
        gt = build_round_tree(deck, r, d_root, 1, stream)
        f = unfold_scores(gt, d_root, 1, stream)
        gt.free()
        node = 0
        for l in range(8):
            cb = f.read(FGT_CHILD_BEGIN, l)
            b, e = int(cb[node]), int(cb[node + 1])
            node = b + int(draws[i]) % (e - b)
            i += 1
        link = f.read(FGT_LINK)
        root = f.read(FGT_NEXT_ROOTS)[int(link[node]):int(link[node]) + 1].copy()
        f.free()
    return root[0]


def _initial_pool(deck) -> int:
    m = 0
    for c in deck[:4]:
        m |= 1 << int(c)
    return m


class BatchSolver:
    """Many deals solved together (a12): every round of every deal is built
    and unfolded as in SubgameSolver; the backward solve then runs one
    persistent launch per round over the trees of all deals (a plan), with
    per-deal leaf utilities, initialisation, average strategies and round
    values around it.  ``capture()`` records the whole backward solve into a
    HIP graph (torch.cuda.CUDAGraph) so that ``replay()`` is one graph launch.

    ``stream_min_nodes``: a deal's round with at least this many FGT nodes
    is left out of the round's plan and solved on its own with the streaming
    schedule (whole games, whose late rounds are far larger than a
    persistent launch keeps busy); such a batch cannot be captured."""

    def __init__(self, problems, start_round: int, iters: int, dtype: int = PASUR_F32,
                 params=None, value_mode: int = V_ITERATE_MEAN,
                 stream_min_nodes: Optional[int] = None):
        torch = _torch()
        self.torch = torch
        self.iters = iters
        self.value_mode = value_mode
        self.deals = [SubgameSolver(deck, start_round, roots, dtype=dtype) for deck, roots in problems]
        self.n_rounds = 6 - start_round
        # per round slot: the deals whose round is streamed (not in the plan)
        self.streamed = [[stream_min_nodes is not None and sum(sv.rounds[k].fgt.n) >= stream_min_nodes
                          for sv in self.deals] for k in range(self.n_rounds)]
        for sv in self.deals:
            for rr in sv.rounds:
                rr.state = CfrState(rr.fgt, dtype)
                rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
        self.plans = []
        self.set_params(params)

    def round_states(self):
        """States covered by each round's plan (round slot k = start_round + k)."""
        return [[sv.rounds[k].state for sv, st in zip(self.deals, self.streamed[k]) if not st]
                for k in range(self.n_rounds)]

    def set_params(self, params=None):
        """One CfrParams for every round, or a list with one per round slot;
        (re)creates the per-round plans."""
        for p in self.plans:
            if p is not None:
                p.free()
        if params is None:
            params = paper_params()
        plist = list(params) if isinstance(params, (list, tuple)) else [params] * self.n_rounds
        self.params = plist
        self.plans = [Plan(states, plist[k], 1, self.iters) if states else None
                      for k, states in enumerate(self.round_states())]
        self.stream_params = []
        for p in plist:
            q = CfrParams.from_buffer_copy(p)
            q.schedule = SCHED_STREAM
            self.stream_params.append(q)
        self.graph = None

    def edges(self) -> int:
        return sum(sv.edges() for sv in self.deals)

    def _backward(self, stream=None):
        for k in range(self.n_rounds - 1, -1, -1):
            for sv in self.deals:
                rr = sv.rounds[k]
                V = None if k == self.n_rounds - 1 else sv.rounds[k + 1].V
                leaf_utilities(rr.fgt, V, rr.state.dtype, rr.state.u[8], stream)
                cfr_init(rr.state, stream)
            if self.plans[k] is not None:
                self.plans[k].iterate(1, self.iters, stream)
            for sv, st in zip(self.deals, self.streamed[k]):
                if st:
                    cfr_iterate(sv.rounds[k].state, self.iters, self.stream_params[k], stream=stream)
            for sv in self.deals:
                rr = sv.rounds[k]
                average_strategy(rr.state, stream)
                round_values(rr.state, self.value_mode, rr.V, stream)

    def solve(self):
        self._backward()

    def capture(self):
        if any(any(st) for st in self.streamed):
            raise ValueError("a batch with streamed rounds cannot be captured (the streaming "
                             "schedule builds its index and allocates on first use)")
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self._backward(s)
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def exploitability(self):
        return [sv.exploitability() for sv in self.deals]

    def free(self):
        for p in self.plans:
            if p is not None:
                p.free()
        self.plans = []
        self.graph = None
        for sv in self.deals:
            sv.free()
