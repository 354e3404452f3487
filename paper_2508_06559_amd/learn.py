"""Learned warm start for DCFR (a13): driver over the libpasur MLP kernels.

Training data come from this solver's own DCFR runs: for sampled decision
nodes of every level, the feature rows of their children (card masks and
inherited score, ``pasur_edge_features``), the average strategy of those
children (policy target) and their node values (value target).  Training
runs forward, loss, backward and Adam in libpasur kernels (BF16 MFMA GEMMs
with FP32 accumulation, FP32 master weights).  The warm start predicts
every node's policy logit, sets sigma = softmax over siblings, seeds the
regrets and average-strategy sums with that profile, and iterates from a
later t0 so that the DCFR discounts treat it as earlier iterations.  Plain
DCFR is the fallback when the warm start does not reach the target.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import (FGT_PARENT, INFOSET_MLP, INFOSET_WIDTH, PASUR_F32, PASUR_F64, MlpGrads, MlpWeights,
               CfrState, adam_step_multi, average_strategy, infoset_rows,
               cfr_init, cfr_iterate, cfr_warm_init, edge_features, gather_f32, leaf_utilities,
               mlp_backward, mlp_forward, mlp_infer, mlp_loss, paper_params, round_values, sample_parents,
               shift_i32, mlp_transpose, warm_start_round as _warm_start_round,
               warm_start_workspace_bytes, _torch)
from .solver import SubgameSolver

N_IN, N_HID, N_OUT = 192, 256, 2


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even (host-side init)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


@dataclass
class Unit:
    """One training unit: sampled parents of one round of one deal."""
    X: object      # [rows, N_IN] BF16 bits (int16)
    seg: object    # [parents + 1] int32 row offsets
    tsig: object   # [rows] float32 target average strategy
    tval: object   # [rows] float32 target node value
    n_par: int
    n_rows: int


class WarmStartMLP:
    """192-256-256-2 MLP; FP32 master weights with BF16 copies for the GEMMs."""

    def __init__(self, seed: int = 0):
        torch = _torch()
        self.torch = torch
        rng = np.random.default_rng(seed)
        shapes = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,)]
        init = [rng.normal(0, math.sqrt(2.0 / N_IN), shapes[0]), np.zeros(N_HID),
                rng.normal(0, math.sqrt(2.0 / N_HID), shapes[2]), np.zeros(N_HID),
                rng.normal(0, math.sqrt(1.0 / N_HID), shapes[4]), np.zeros(N_OUT)]
        self.master = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in init]
        self.bf = {k: torch.from_numpy(_bf16_bits(init[k]).copy()).cuda() for k in (0, 2, 4)}
        self.m = [torch.zeros_like(t) for t in self.master]
        self.v = [torch.zeros_like(t) for t in self.master]
        self.g = [torch.zeros_like(t) for t in self.master]
        self.step = 0
        self._bufs = {}
        self._version = 0      # bumped whenever the BF16 weights change
        self._tversion = -1    # version the transposed copies were made from
        self._wt = None
        self._ws = None

    def set_weights(self, W: Sequence[np.ndarray]):
        """Load FP32 weights (W1, b1, W2, b2, W3, b3) and their BF16 copies."""
        torch = self.torch
        self.master = [torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda") for a in W]
        self.bf = {k: torch.from_numpy(_bf16_bits(np.asarray(W[k], np.float32)).copy()).cuda()
                   for k in (0, 2, 4)}
        self._version += 1

    def weights(self) -> MlpWeights:
        m, b = self.master, self.bf
        return MlpWeights(b[0].data_ptr(), m[1].data_ptr(), b[2].data_ptr(), m[3].data_ptr(),
                          b[4].data_ptr(), m[5].data_ptr(), None, None)

    def infer_weights(self) -> MlpWeights:
        """Weights with transposed W1/W2 copies for pasur_mlp_infer, refreshed
        when the weights changed since they were made."""
        torch = self.torch
        if self._wt is None:
            self._wt = (torch.empty((N_HID, N_IN), dtype=torch.int16, device="cuda"),
                        torch.empty((N_HID, N_HID), dtype=torch.int16, device="cuda"))
        if self._tversion != self._version:
            mlp_transpose(self.weights(), self._wt[0], self._wt[1])
            self._tversion = self._version
        w = self.weights()
        w.W1t, w.W2t = self._wt[0].data_ptr(), self._wt[1].data_ptr()
        return w

    def workspace(self, nbytes: int):
        """A reused device buffer of at least nbytes (grown by doubling)."""
        if self._ws is None or self._ws.numel() < nbytes:
            cap = max(nbytes, 2 * (self._ws.numel() if self._ws is not None else 0))
            self._ws = self.torch.empty(cap, dtype=self.torch.uint8, device="cuda")
        return self._ws

    def grads(self) -> MlpGrads:
        g = self.g
        return MlpGrads(*[t.data_ptr() for t in g])

    def _buffers(self, M: int):
        torch = self.torch
        cap = self._bufs.get("cap", 0)
        if M > cap:
            cap = max(M, 2 * cap)
            self._bufs = {"cap": cap,
                          "H1": torch.empty((cap, N_HID), dtype=torch.int16, device="cuda"),
                          "H2": torch.empty((cap, N_HID), dtype=torch.int16, device="cuda"),
                          "Y": torch.empty((cap, N_OUT), dtype=torch.float32, device="cuda"),
                          "dY": torch.empty((cap, N_OUT), dtype=torch.float32, device="cuda")}
        return self._bufs

    def forward(self, X, M: int):
        """Y [M, 2] (a view into a reused buffer) for feature rows X."""
        b = self._buffers(M)
        w = self.weights()
        mlp_forward(w, X, M, b["H1"], b["H2"], b["Y"])
        return b["Y"][:M]

    def train_unit(self, u: Unit, lr: float, value_weight: float = 0.05,
                   betas=(0.9, 0.999), eps=1e-8):
        torch = self.torch
        b = self._buffers(u.n_rows)
        # the transposed W1/W2 copies the fused forward reads (made in place,
        # so that the step allocates nothing for them)
        w = self.infer_weights()
        mlp_forward(w, u.X, u.n_rows, b["H1"], b["H2"], b["Y"])
        loss = torch.empty((u.n_par, 2), dtype=torch.float32, device="cuda")
        mlp_loss(b["Y"], u.tsig, u.tval, u.seg, u.n_par, u.n_rows, value_weight, b["dY"], loss)
        mlp_backward(w, u.X, b["H1"], b["H2"], b["dY"], u.n_rows, self.grads())
        self.step += 1
        adam_step_multi(self.master, self.g, self.m, self.v, [self.bf.get(k) for k in range(6)], lr,
                        betas[0], betas[1], eps, self.step)
        self._version += 1
        return loss

    def state_dict(self):
        return [t.detach().cpu().numpy().copy() for t in self.master]


def features_into(rr, level: int, edges, n: int, X, features: str = "edge"):
    """Network input rows of FGT nodes of `level` (edges None: all, in
    order): the edge features (pasur_edge_features) or the paper's infoset
    rows scaled into the same input width (pasur_infoset_rows)."""
    if features == "edge":
        edge_features(rr.gt, rr.fgt, level, edges, n, X)
    elif features == "infoset":
        infoset_rows(rr.gt, rr.fgt, level, edges, n, X, INFOSET_MLP)
    else:
        raise ValueError(f"unknown feature set {features!r}")


def make_units(solver: SubgameSolver, seed: int, parents_per_level: int = 400,
               features: str = "edge") -> List[Unit]:
    """Training units from a solved SubgameSolver built with keep_gt=True:
    one unit per round, sampled decision parents of every level."""
    torch = _torch()
    units = []
    for rr in solver.rounds:
        f, st = rr.fgt, rr.state
        parts = []
        for l in range(1, 9):
            seg = torch.empty(f.n[l - 1] + 1, dtype=torch.int32, device="cuda")
            edges = torch.empty(f.n[l], dtype=torch.int32, device="cuda")
            keep = min(1.0, parents_per_level / max(1, f.n[l - 1]))
            npar, ne = sample_parents(f, l, (seed << 8) ^ (rr.round << 4) ^ l, keep, seg, edges)
            if npar:
                parts.append((l, seg, edges, npar, ne))
        rows = sum(p[4] for p in parts)
        pars = sum(p[3] for p in parts)
        if rows == 0:
            continue
        X = torch.empty((rows, N_IN), dtype=torch.int16, device="cuda")
        tsig = torch.empty(rows, dtype=torch.float32, device="cuda")
        tval = torch.empty(rows, dtype=torch.float32, device="cuda")
        useg = torch.empty(pars + 1, dtype=torch.int32, device="cuda")
        off = poff = 0
        for l, seg, edges, npar, ne in parts:
            features_into(rr, l, edges, ne, X[off:], features)
            gather_f32(st.sigma_bar[l], st.dtype, edges, ne, tsig[off:])
            gather_f32(st.u[l], st.dtype, edges, ne, tval[off:])
            shift_i32(seg, npar + 1, off, useg[poff:])
            off += ne
            poff += npar
        units.append(Unit(X, useg, tsig, tval, pars, rows))
    return units


def warm_start_round(model: WarmStartMLP, rr, kappa_r: float, kappa_s: float,
                     max_level: int = 8):
    """Predict the logits of levels 1..max_level and seed sigma, R and Sbar
    (after cfr_init): one libpasur call (features, fused forward pass, warm
    init) with the model's cached transposed weights and reused workspace."""
    ws = model.workspace(warm_start_workspace_bytes(rr.fgt, max_level))
    _warm_start_round(rr.gt, rr.state, model.infer_weights(), max_level, kappa_r, kappa_s, ws)


def warm_start_round_by_level(model: WarmStartMLP, rr, kappa_r: float, kappa_s: float,
                              features: str = "edge"):
    """The same as warm_start_round with max_level 8, one level at a time
    through the per-level calls (a cross-check, and the path for networks
    trained on infoset rows)."""
    torch = _torch()
    f = rr.fgt
    for l in range(1, 9):
        n = f.n[l]
        X = torch.empty((n, N_IN), dtype=torch.int16, device="cuda")
        features_into(rr, l, None, n, X, features)
        Y = torch.empty((n, N_OUT), dtype=torch.float32, device="cuda")
        mlp_infer(model.weights(), X, n, Y)
        cfr_warm_init(rr.state, l, Y, kappa_r, kappa_s)


@dataclass
class WarmParams:
    """kappa_r, kappa_s: regret and average-sum seeds (multiples of the
    predicted profile); t_virtual: iterations the seeds stand for.  The
    default uses the prediction as the first iterate only (seeds 0, t0 = 1):
    on held-out two-round deals seeding regrets or averages with a profile
    this exploitable slowed convergence, while starting from it did not.
    max_level: the levels whose strategies are predicted (1..max_level)."""
    kappa_r: float = 0.0
    kappa_s: float = 0.0
    t_virtual: int = 0
    max_level: int = 8


def solve_subgame(deck, start_round: int, roots, iters: int, dtype: int = PASUR_F32,
                  model: Optional[WarmStartMLP] = None, warm: WarmParams = WarmParams(),
                  params=None):
    """Backward solve of a subgame, plain or warm-started; returns the solver
    (states and round values filled; build_seconds: building and unfolding
    the trees)."""
    torch = _torch()
    t_build = time.perf_counter()
    # both arms keep the game trees (the warm start needs them; freeing them
    # inside the timed solve would charge the plain arm alone)
    sv = SubgameSolver(deck, start_round, roots, dtype=dtype, keep_gt=True)
    torch.cuda.synchronize()
    sv.build_seconds = time.perf_counter() - t_build
    return solve_built(sv, iters, model, warm, params, fresh_state=True)


def solve_built(sv: SubgameSolver, iters: int, model: Optional[WarmStartMLP] = None,
                warm: WarmParams = WarmParams(), params=None, fresh_state: bool = False):
    """The backward solve of solve_subgame on a solver whose trees are built
    (keep_gt=True); a round's state is allocated when it has none (or when
    fresh_state) and re-initialised otherwise, so one solver serves a grid
    of iteration counts."""
    torch = _torch()
    params = params if params is not None else paper_params()
    dtype = sv.dtype
    V = None
    for rr in reversed(sv.rounds):
        if fresh_state or rr.state is None:
            rr.state = CfrState(rr.fgt, dtype)
        leaf_utilities(rr.fgt, V, dtype, rr.state.u[8])
        cfr_init(rr.state)
        rr.state.t = 1
        t0 = 1
        if model is not None:
            warm_start_round(model, rr, warm.kappa_r, warm.kappa_s, warm.max_level)
            t0 = warm.t_virtual + 1
        cfr_iterate(rr.state, iters, params, t0=t0)
        average_strategy(rr.state)
        if fresh_state or rr.V is None:
            rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
        # round value: mean of the iterate values of the iterations run (the
        # paper's g_UTL / NUM_ITER); vacc holds exactly `iters` terms
        rr.state.t = 1 + iters
        round_values(rr.state, 0, rr.V)
        rr.state.t = t0 + iters
        V = rr.V
    return sv


def exploitability(sv: SubgameSolver) -> float:
    bra, brb, _ = sv.exploitability()
    return float(((bra - brb) / 2).max().item())


def seconds_to_target(deck, start_round: int, roots, target: float, grid: Sequence[int],
                      model: Optional[WarmStartMLP] = None, warm: WarmParams = WarmParams(),
                      fallback: bool = True):
    """Smallest iteration count of ``grid`` whose solve reaches exploitability
    <= target, and the wall-clock seconds of that solve (exploitability checks
    excluded), also without building the trees (solve_seconds: warm start,
    iterations, values).  A warm start that misses the target on the whole
    grid falls back to plain DCFR; its seconds then include the failed warm
    attempts."""
    torch = _torch()
    spent = spent_solve = 0.0
    for T in grid:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv = solve_subgame(deck, start_round, roots, T, model=model, warm=warm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        solve = el - sv.build_seconds
        ex = exploitability(sv)
        sv.free()
        if ex <= target:
            return {"iters": T, "seconds": el, "solve_seconds": solve, "exploitability": ex,
                    "fallback": False}
        if model is not None:
            spent += el
            spent_solve += solve
    if model is not None and fallback:
        r = seconds_to_target(deck, start_round, roots, target, grid, None)
        r["seconds"] += spent
        r["solve_seconds"] += spent_solve
        r["fallback"] = True
        return r
    return {"iters": None, "seconds": None, "solve_seconds": None, "exploitability": ex,
            "fallback": False}


def iterations_to_target(sv: SubgameSolver, target: float, grid: Sequence[int],
                         model: Optional[WarmStartMLP] = None, warm: WarmParams = WarmParams()):
    """seconds_to_target on one built solver (keep_gt=True) reused for every
    iteration count of the grid: the smallest count whose solve reaches
    exploitability <= target, and the seconds of that solve (warm start,
    iterations, average strategies, values; trees and exploitability checks
    excluded).  A warm start that misses the target on the whole grid falls
    back to plain DCFR and is charged both."""
    torch = _torch()
    spent = 0.0
    for T in grid:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve_built(sv, T, model, warm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ex = exploitability(sv)
        if ex <= target:
            return {"iters": T, "solve_seconds": el, "exploitability": ex, "fallback": False}
        if model is not None:
            spent += el
    if model is not None:
        r = iterations_to_target(sv, target, grid, None)
        if r["iters"] is not None:
            r["solve_seconds"] += spent
            r["fallback"] = True
        return r
    return {"iters": None, "solve_seconds": None, "exploitability": ex, "fallback": False}


def train(model: WarmStartMLP, units: List[Unit], epochs: int, seed: int = 0, lr: float = 2e-3,
          log=None):
    """Adam over shuffled units; lr stepped down at 1/2 and 3/4 of the epochs."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        r = lr if ep < epochs // 2 else (lr * 0.3 if ep < 3 * epochs // 4 else lr * 0.1)
        tot = np.zeros(2)
        for i in rng.permutation(len(units)):
            tot += model.train_unit(units[i], lr=r).sum(0).cpu().numpy()
        hist.append((tot / max(1, len(units))).tolist())
        if log:
            log(f"[train] epoch {ep}: policy {hist[-1][0]:.4f} value {hist[-1][1]:.4f}")
    return hist


def training_units(problems, iters: int, parents_per_level: int = 600, seed0: int = 0,
                   features: str = "edge", start_round: int = 4):
    """Solve every (deck, roots) problem (two-round by default; start_round 0:
    full games) with plain DCFR and sample training units from the solution."""
    units = []
    for k, (deck, roots) in enumerate(problems):
        sv = SubgameSolver(deck, start_round, roots, keep_gt=True)
        sv.solve(iters)
        units += make_units(sv, seed0 + k, parents_per_level, features)
        sv.free()
    return units


def initial_profile_exploitability(deck, roots, model: Optional[WarmStartMLP],
                                   features: str = "edge", start_round: int = 4):
    """Exploitability of the profile DCFR starts from: uniform, or the
    network's prediction."""
    sv = SubgameSolver(deck, start_round, roots, keep_gt=True)
    for rr in sv.rounds:
        rr.state = CfrState(rr.fgt, PASUR_F32)
        cfr_init(rr.state)
        if model is not None and features == "edge":
            warm_start_round(model, rr, 0.0, 0.0)
        elif model is not None:
            warm_start_round_by_level(model, rr, 0.0, 0.0, features)
        for l in range(1, 9):
            rr.state.sigma_bar[l].copy_(rr.state.sigma[l])
    ex = exploitability(sv)
    sv.free()
    return ex


# ---- tree-model baseline on infoset rows -------------------------------------
# The paper fits a gradient-boosted tree model (XGBoost, RMSE, gamma = 1) to
# 100 x sigma on 58-byte infoset rows.  XGBoost is not available here; the
# baseline is scikit-learn's histogram gradient boosting with the squared
# error, on the same rows and target, on the CPU.


def infoset_dataset(problems, iters: int, parents_per_level: int = 600, seed0: int = 0):
    """(rows int8 [N, 58], 100 x average strategy [N], parent id [N]) of
    sampled decision parents of the solved two-round problems."""
    torch = _torch()
    rows, tgt, grp = [], [], []
    gid = 0
    for k, (deck, roots) in enumerate(problems):
        sv = SubgameSolver(deck, 4, roots, keep_gt=True)
        sv.solve(iters)
        for rr in sv.rounds:
            f, st = rr.fgt, rr.state
            for l in range(1, 9):
                seg = torch.empty(f.n[l - 1] + 1, dtype=torch.int32, device="cuda")
                edges = torch.empty(f.n[l], dtype=torch.int32, device="cuda")
                keep = min(1.0, parents_per_level / max(1, f.n[l - 1]))
                npar, ne = sample_parents(f, l, ((seed0 + k) << 8) ^ (rr.round << 4) ^ l, keep,
                                          seg, edges)
                if not ne:
                    continue
                R = torch.empty((ne, INFOSET_WIDTH), dtype=torch.int8, device="cuda")
                infoset_rows(rr.gt, f, l, edges, ne, R)
                t = torch.empty(ne, dtype=torch.float32, device="cuda")
                gather_f32(st.sigma_bar[l], st.dtype, edges, ne, t)
                sg = seg[: npar + 1].cpu().numpy()
                g = np.repeat(np.arange(npar), np.diff(sg)) + gid
                gid += npar
                rows.append(R.cpu().numpy())
                tgt.append(100.0 * t.cpu().numpy())
                grp.append(g)
        sv.free()
    return np.concatenate(rows), np.concatenate(tgt), np.concatenate(grp)


def fit_tree_model(rows: np.ndarray, target: np.ndarray, seed: int = 0, max_iter: int = 300):
    from sklearn.ensemble import HistGradientBoostingRegressor
    m = HistGradientBoostingRegressor(loss="squared_error", max_iter=max_iter, learning_rate=0.1,
                                      max_leaf_nodes=63, random_state=seed)
    m.fit(rows.astype(np.float32), target)
    return m


def tree_profile_exploitability(deck, roots, tree) -> float:
    """Exploitability of the profile the tree model predicts: 100 x sigma
    clipped at 0 and normalised over siblings (uniform where all are 0)."""
    torch = _torch()
    sv = SubgameSolver(deck, 4, roots, keep_gt=True)
    for rr in sv.rounds:
        f = rr.fgt
        rr.state = CfrState(f, PASUR_F32)
        for l in range(1, 9):
            n = f.n[l]
            R = torch.empty((n, INFOSET_WIDTH), dtype=torch.int8, device="cuda")
            infoset_rows(rr.gt, f, l, None, n, R)
            p = np.maximum(tree.predict(R.cpu().numpy().astype(np.float32)), 0.0)
            par = f.read(FGT_PARENT, l).astype(np.int64)
            tot = np.bincount(par, weights=p, minlength=f.n[l - 1])
            cnt = np.bincount(par, minlength=f.n[l - 1])
            sig = np.where(tot[par] > 0, p / np.where(tot[par] > 0, tot[par], 1.0), 1.0 / cnt[par])
            rr.state.sigma_bar[l].copy_(torch.from_numpy(sig.astype(np.float32)))
    ex = exploitability(sv)
    sv.free()
    return ex
