"""Python binding of libpasur (the MI355X Pasur round solver, include/pasur.h).

Argument marshalling only: every step runs in the HIP kernels of libpasur.so.
PyTorch provides device memory and the stream.  Importing this module on a
machine without the built library or without a GPU raises; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpasur.so")

PASUR_F32, PASUR_F64 = 0, 1
DCFR, CFR_PLUS, CFR_VANILLA = 0, 1, 2
RM_FLOOR, RM_POSITIVE = 0, 1
V_ITERATE_MEAN, V_SIGMA_BAR = 0, 1
TV_EXPECT, TV_BR_A, TV_BR_B, TV_MINIMAX = 0, 1, 2, 3
GT_POOL, GT_HANDS, GT_RS, GT_PARENT, GT_CHILD_BEGIN, GT_ACT_CARD, GT_ACT_CAP = range(7)
(FGT_GT, FGT_SID, FGT_PARENT, FGT_CHILD_BEGIN, FGT_SCORE_TAB, FGT_NEXT_ROOTS, FGT_LINK,
 FGT_LEAF_BASE) = range(8)

ROOT_DTYPE = np.dtype([("pool", "<u8"), ("ca", "i1"), ("cb", "i1"), ("d", "i1"),
                       ("bonus", "i1"), ("pad", "<i4")])


class PasurError(RuntimeError):
    pass


SCHED_ROOT, SCHED_LEVEL_SYNC, SCHED_ROOT_GLOBAL, SCHED_STREAM, SCHED_AUTO = 0, 1, 2, 3, 4


class CfrParams(C.Structure):
    _fields_ = [("variant", C.c_int), ("rm_mode", C.c_int), ("alpha", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("schedule", C.c_int), ("block", C.c_int), ("seg_nodes", C.c_int),
                ("flags", C.c_int)]


SNIPPET_TOL, SNIPPET_AVG = 1, 2  # CfrParams.flags (pasur_cfr_flags)
LEAF_LITERAL_BONUS0 = 1          # leaf-utility flags


def paper_params(schedule: int = SCHED_AUTO, block: int = 0, seg_nodes: int = 0,
                 flags: int = 0) -> CfrParams:
    """DCFR with the paper's constants (alpha 1.5, beta 0, gamma 2) and its
    regret-matching floor (1e-8); by default the library picks the schedule
    per round (persistent segments, or streaming sweeps for large rounds).
    ``flags``: SNIPPET_TOL / SNIPPET_AVG, the snippet's executed forms."""
    return CfrParams(DCFR, RM_FLOOR, 1.5, 0.0, 2.0, 1e-8, schedule, block, seg_nodes, flags)


class _State(C.Structure):
    _fields_ = [("dtype", C.c_int), ("sigma", C.c_void_p * 9), ("R", C.c_void_p * 9),
                ("Sbar", C.c_void_p * 9), ("reachA", C.c_void_p * 9),
                ("reachB", C.c_void_p * 9), ("u", C.c_void_p * 9), ("vacc", C.c_void_p)]


_lib = None


def lib():
    """Load libpasur.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PasurError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.pasur_last_error.restype = C.c_char_p
        L.pasur_build_round_tree.argtypes = [vp, i32, vp, i64, C.POINTER(vp), vp]
        L.pasur_gt_sizes.argtypes = [vp, vp]
        L.pasur_gt_read.argtypes = [vp, i32, i32, vp]
        L.pasur_gt_free.argtypes = [vp]
        L.pasur_gt_free.restype = None
        L.pasur_unfold_scores.argtypes = [vp, vp, i64, C.POINTER(vp), vp]
        L.pasur_fgt_sizes.argtypes = [vp, vp, vp, vp]
        L.pasur_fgt_read.argtypes = [vp, i32, i32, vp]
        L.pasur_fgt_next_roots.argtypes = [vp]
        L.pasur_fgt_next_roots.restype = vp
        L.pasur_fgt_free.argtypes = [vp]
        L.pasur_fgt_free.restype = None
        L.pasur_leaf_utilities.argtypes = [vp, vp, i32, i32, vp, vp]
        L.pasur_cfr_init.argtypes = [vp, vp, vp]
        L.pasur_cfr_iterate.argtypes = [vp, vp, vp, i64, i32, vp]
        L.pasur_average_strategy.argtypes = [vp, vp, vp, vp]
        L.pasur_round_values.argtypes = [vp, vp, i32, i64, vp, vp, vp]
        L.pasur_tree_values.argtypes = [vp, vp, i32, vp, i32, vp, vp]
        L.pasur_tree_values_noalloc.argtypes = [vp, vp, i32, vp, i32, vp, vp]
        L.pasur_exploitability.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp, vp]
        L.pasur_gt_get_view.argtypes = [vp, vp]
        L.pasur_fgt_get_view.argtypes = [vp, vp]
        L.pasur_sgd_step.argtypes = [vp, vp, vp, i64, C.c_float, vp]
        L.pasur_plan_create.argtypes = [vp, vp, i32, vp, i64, i64, C.POINTER(vp), vp]
        L.pasur_plan_iterate.argtypes = [vp, i64, i32, vp]
        L.pasur_plan_info.argtypes = [vp, vp]
        L.pasur_plan_free.argtypes = [vp]
        L.pasur_plan_free.restype = None
        L.pasur_gemm_bf16.argtypes = [i32, i32, i32, vp, i64, i64, vp, i64, i64, vp, vp, i64, vp,
                                      i32, vp]
        L.pasur_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.pasur_mlp_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.pasur_mlp_loss.argtypes = [vp, vp, vp, vp, i64, i64, C.c_float, vp, vp, vp]
        L.pasur_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float,
                                      C.c_float, i64, vp]
        L.pasur_adam_step_multi.argtypes = [i32, vp, vp, vp, vp, vp, vp, C.c_float, C.c_float,
                                            C.c_float, C.c_float, i64, vp]
        L.pasur_edge_features.argtypes = [vp, vp, i32, vp, i64, vp, vp]
        L.pasur_sample_parents.argtypes = [vp, i32, C.c_uint64, C.c_double, vp, vp,
                                           C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp]
        L.pasur_cfr_warm_init.argtypes = [vp, vp, i32, vp, C.c_float, C.c_float, vp]
        L.pasur_warm_start_round.argtypes = [vp, vp, vp, vp, i32, C.c_float, C.c_float, vp, i64,
                                             vp]
        L.pasur_warm_start_workspace_bytes.restype = i64
        L.pasur_warm_start_workspace_bytes.argtypes = [vp, i32]
        L.pasur_mlp_infer.argtypes = [vp, vp, i64, vp, vp]
        L.pasur_mlp_transpose.argtypes = [vp, vp, vp, vp]
        L.pasur_selfplay.argtypes = [vp, i32, vp, i32, i32, i64, C.c_uint64, i32, i32, vp, vp]
        L.pasur_infoset_rows.argtypes = [vp, vp, i32, vp, i64, i32, vp, vp]
        L.pasur_es_workspace_bytes.restype = i64
        L.pasur_es_workspace_bytes.argtypes = [vp, i32]
        L.pasur_es_iterate.argtypes = [vp, vp, i64, i64, C.c_uint64, i32, C.c_double, i32, i32, vp,
                                       i64, vp, vp]
        L.pasur_gather_f32.argtypes = [vp, i32, vp, i64, vp, vp]
        L.pasur_shift_i32.argtypes = [vp, i64, i32, vp, vp]
        L.pasur_profile_enable.argtypes = [i32]
        L.pasur_profile_select.argtypes = [C.c_uint64]
        L.pasur_profile_read.argtypes = [i64, vp, vp, vp, vp, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != 0:
        msg = lib().pasur_last_error().decode(errors="replace")
        raise PasurError(f"{what} failed ({status}): {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise PasurError("no GPU: libpasur runs on an MI355X (gfx950) only")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def roots_to_device(roots) -> "torch.Tensor":
    """Roots (objects with pool, ca, cb, d, bonus, or a ROOT_DTYPE array) ->
    device byte tensor laid out as pasur_root[]."""
    torch = _torch()
    if isinstance(roots, np.ndarray) and roots.dtype == ROOT_DTYPE:
        a = roots
    else:
        a = np.zeros(len(roots), ROOT_DTYPE)
        for i, r in enumerate(roots):
            a[i] = (r.pool, r.ca, r.cb, r.d, r.bonus, 0)
    return torch.from_numpy(a.view(np.uint8).copy()).cuda()


class GameTree:
    """Handle of a round game tree (pasur_gt)."""

    def __init__(self, handle, rnd: int):
        self.h = handle
        self.round = rnd
        n = (C.c_int64 * 9)()
        _check(lib().pasur_gt_sizes(self.h, n), "pasur_gt_sizes")
        self.n = list(n)

    def free(self):
        if self.h:
            lib().pasur_gt_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def read(self, field: int, level: int) -> np.ndarray:
        n = self.n[level]
        dt, size = {GT_POOL: (np.uint64, n), GT_HANDS: (np.uint8, n), GT_RS: (np.int8, 8 * n),
                    GT_PARENT: (np.int32, n), GT_CHILD_BEGIN: (np.int32, n + 1),
                    GT_ACT_CARD: (np.uint8, n), GT_ACT_CAP: (np.uint64, n)}[field]
        out = np.zeros(max(size, 1), dt)
        _check(lib().pasur_gt_read(self.h, field, level, out.ctypes.data_as(C.c_void_p)),
               "pasur_gt_read")
        out = out[:size]
        return out.reshape(n, 8) if field == GT_RS else out


class UnfoldedTree:
    """Handle of a round's unfolded tree (pasur_fgt)."""

    def __init__(self, handle, rnd: int):
        self.h = handle
        self.round = rnd
        n = (C.c_int64 * 9)()
        ns, nn = C.c_int64(), C.c_int64()
        _check(lib().pasur_fgt_sizes(self.h, n, C.byref(ns), C.byref(nn)), "pasur_fgt_sizes")
        self.n = list(n)
        self.n_scores = ns.value
        self.n_next = nn.value

    def free(self):
        if self.h:
            lib().pasur_fgt_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def read(self, field: int, level: int = 0) -> np.ndarray:
        if field == FGT_SCORE_TAB:
            out = np.zeros(max(4 * self.n_scores, 1), np.int8)
        elif field == FGT_NEXT_ROOTS:
            out = np.zeros(max(self.n_next, 1), ROOT_DTYPE)
        elif field == FGT_LEAF_BASE:
            out = np.zeros(max(self.n[8], 1), np.int16)
        else:
            n = self.n[8] if field == FGT_LINK else self.n[level]
            out = np.zeros(max(n + 1 if field == FGT_CHILD_BEGIN else n, 1), np.int32)
        _check(lib().pasur_fgt_read(self.h, field, level, out.ctypes.data_as(C.c_void_p)),
               "pasur_fgt_read")
        if field == FGT_SCORE_TAB:
            return out[: 4 * self.n_scores].reshape(-1, 4)
        if field == FGT_NEXT_ROOTS:
            return out[: self.n_next]
        if field == FGT_LEAF_BASE or field == FGT_LINK:
            return out[: self.n[8]]
        n = self.n[level]
        return out[: n + 1 if field == FGT_CHILD_BEGIN else n]

    def next_roots_device(self):
        """(device pointer, count) of the next-round roots owned by this handle."""
        return lib().pasur_fgt_next_roots(self.h), self.n_next

    def edges(self) -> int:
        """Non-root nodes: one per action edge, updated once per iteration."""
        return int(sum(self.n[1:]))


def build_round_tree(deck: Sequence[int], rnd: int, d_roots, n_roots: int, stream=None) -> GameTree:
    """pasur_build_round_tree: ``d_roots`` is a device tensor (or int device
    pointer) of pasur_root in canonical order."""
    dk = (C.c_uint8 * 52)(*[int(c) for c in deck])
    h = C.c_void_p()
    ptr = C.c_void_p(d_roots if isinstance(d_roots, int) else d_roots.data_ptr())
    _check(lib().pasur_build_round_tree(dk, rnd, ptr, n_roots, C.byref(h), _stream(stream)),
           "pasur_build_round_tree")
    return GameTree(h, rnd)


def unfold_scores(gt: GameTree, d_roots, n_roots: int, stream=None) -> UnfoldedTree:
    h = C.c_void_p()
    ptr = C.c_void_p(d_roots if isinstance(d_roots, int) else d_roots.data_ptr())
    _check(lib().pasur_unfold_scores(gt.h, ptr, n_roots, C.byref(h), _stream(stream)),
           "pasur_unfold_scores")
    return UnfoldedTree(h, gt.round)


class CfrState:
    """Caller-owned solver state of one round (torch device tensors)."""

    def __init__(self, fgt: UnfoldedTree, dtype: int = PASUR_F32):
        torch = _torch()
        self.fgt = fgt
        self.dtype = dtype
        tdt = torch.float32 if dtype == PASUR_F32 else torch.float64
        n = fgt.n
        dev = torch.device("cuda")
        self.sigma = [None] + [torch.empty(n[l], dtype=tdt, device=dev) for l in range(1, 9)]
        self.R = [None] + [torch.empty(n[l], dtype=tdt, device=dev) for l in range(1, 9)]
        self.Sbar = [None] + [torch.empty(n[l], dtype=tdt, device=dev) for l in range(1, 9)]
        self.reachA = [torch.empty(n[l], dtype=tdt, device=dev) for l in range(8)] + [None]
        self.reachB = [torch.empty(n[l], dtype=tdt, device=dev) for l in range(8)] + [None]
        self.u = [torch.empty(n[l], dtype=tdt, device=dev) for l in range(9)]
        self.vacc = torch.zeros(n[0], dtype=torch.float64, device=dev)
        self.sigma_bar = [None] + [torch.empty(n[l], dtype=tdt, device=dev) for l in range(1, 9)]
        st = _State()
        st.dtype = dtype
        for name in ("sigma", "R", "Sbar", "reachA", "reachB", "u"):
            arr = getattr(st, name)
            for l, t in enumerate(getattr(self, name)):
                arr[l] = t.data_ptr() if t is not None else None
        st.vacc = self.vacc.data_ptr()
        self.c = st
        self.sb_ptrs = (C.c_void_p * 9)(*([None] + [t.data_ptr() for t in self.sigma_bar[1:]]))
        self.t = 1
        self.es_t = 0
        self.es_ws = None

    def bytes(self) -> int:
        ts = [*self.sigma[1:], *self.R[1:], *self.Sbar[1:], *self.reachA[:8], *self.reachB[:8],
              *self.u, self.vacc]
        return int(sum(t.numel() * t.element_size() for t in ts))


def leaf_utilities(fgt: UnfoldedTree, d_V_next, dtype: int, d_out, stream=None,
                   literal_bonus0: bool = False):
    vp = None if d_V_next is None else _p(d_V_next)
    flags = LEAF_LITERAL_BONUS0 if literal_bonus0 else 0
    _check(lib().pasur_leaf_utilities(fgt.h, vp, dtype, flags, _p(d_out), _stream(stream)),
           "pasur_leaf_utilities")


def cfr_init(st: CfrState, stream=None):
    _check(lib().pasur_cfr_init(st.fgt.h, C.byref(st.c), _stream(stream)), "pasur_cfr_init")
    st.t = 1
    st.es_t = 0


def cfr_iterate(st: CfrState, n_iters: int, params: Optional[CfrParams] = None, t0: Optional[int] = None,
                stream=None):
    p = params if params is not None else paper_params()
    t = st.t if t0 is None else t0
    _check(lib().pasur_cfr_iterate(st.fgt.h, C.byref(st.c), C.byref(p), t, n_iters,
                                   _stream(stream)), "pasur_cfr_iterate")
    st.t = t + n_iters


def average_strategy(st: CfrState, stream=None):
    _check(lib().pasur_average_strategy(st.fgt.h, C.byref(st.c), st.sb_ptrs, _stream(stream)),
           "pasur_average_strategy")
    return st.sigma_bar


def round_values(st: CfrState, value_mode: int, d_V, stream=None):
    T = st.t - 1
    _check(lib().pasur_round_values(st.fgt.h, C.byref(st.c), value_mode, T, st.sb_ptrs, _p(d_V),
                                    _stream(stream)), "pasur_round_values")
    return d_V


def tree_values(fgt: UnfoldedTree, d_leaf, dtype: int, sigma: Optional[List], mode: int, d_out,
                stream=None):
    if sigma is None:
        sp = None
    else:
        sp = (C.c_void_p * 9)(*([None] + [t.data_ptr() for t in sigma[1:]]))
    _check(lib().pasur_tree_values(fgt.h, _p(d_leaf), dtype, sp, mode, _p(d_out),
                                   _stream(stream)), "pasur_tree_values")
    return d_out


def tree_values_noalloc(fgt: UnfoldedTree, d_leaf, dtype: int, sigma: Optional[List], mode: int,
                        d_out, stream=None):
    """pasur_tree_values_noalloc: tree_values with no device allocation
    (levels of at most 2^21 nodes)."""
    if sigma is None:
        sp = None
    else:
        sp = (C.c_void_p * 9)(*([None] + [t.data_ptr() for t in sigma[1:]]))
    _check(lib().pasur_tree_values_noalloc(fgt.h, _p(d_leaf), dtype, sp, mode, _p(d_out),
                                           _stream(stream)), "pasur_tree_values_noalloc")
    return d_out


def exploitability(fgts, sigma_bars, dtype: int, br_a=None, br_b=None, v=None, stream=None,
                   literal_bonus0: bool = False):
    """pasur_exploitability: fgts are consecutive rounds ending at round 5,
    sigma_bars[r][l] (l = 1..8) device tensors of their average strategies;
    br_a, br_b, v: device double tensors of fgts[0]'s root count (None: not
    computed)."""
    n = len(fgts)
    hs = (C.c_void_p * n)(*[f.h for f in fgts])
    sb = (C.c_void_p * (9 * n))()
    for r in range(n):
        for l in range(1, 9):
            sb[9 * r + l] = _p(sigma_bars[r][l])
    flags = LEAF_LITERAL_BONUS0 if literal_bonus0 else 0
    _check(lib().pasur_exploitability(hs, n, sb, dtype, flags, _p(br_a), _p(br_b), _p(v),
                                      _stream(stream)), "pasur_exploitability")


class GtView(C.Structure):
    """pasur_gt_view: device pointers of a game tree's arrays (borrowed)."""
    _fields_ = [("round", C.c_int), ("n", C.c_int64 * 9), ("pool", C.c_void_p * 9),
                ("hands", C.c_void_p * 9), ("rs", C.c_void_p * 9), ("parent", C.c_void_p * 9),
                ("child_begin", C.c_void_p * 8), ("act_card", C.c_void_p * 9),
                ("act_cap", C.c_void_p * 9)]


class FgtView(C.Structure):
    """pasur_fgt_view: device pointers of an unfolded tree's arrays (borrowed,
    valid until the tree is freed)."""
    _fields_ = [("round", C.c_int), ("n", C.c_int64 * 9), ("gt", C.c_void_p * 9),
                ("sid", C.c_void_p * 9), ("parent", C.c_void_p * 9),
                ("child_begin", C.c_void_p * 8), ("score_tab", C.c_void_p),
                ("n_scores", C.c_int64), ("next_roots", C.c_void_p), ("n_next", C.c_int64),
                ("link", C.c_void_p), ("leaf_base", C.c_void_p)]


def gt_view(gt) -> GtView:
    v = GtView()
    _check(lib().pasur_gt_get_view(gt.h, C.byref(v)), "pasur_gt_get_view")
    return v


def fgt_view(fgt) -> FgtView:
    v = FgtView()
    _check(lib().pasur_fgt_get_view(fgt.h, C.byref(v)), "pasur_fgt_get_view")
    return v


def sgd_step(w, g, wb, lr, stream=None):
    """pasur_sgd_step on torch tensors (wb: int16 BF16 bit patterns or None)."""
    _check(lib().pasur_sgd_step(_p(w), _p(g), _p(wb), w.numel(), lr, _stream(stream)),
           "pasur_sgd_step")


class Plan:
    """pasur_plan: a batch of (unfolded tree, solver state) items iterated by
    one persistent launch per call (a12).  Keeps the items alive."""

    def __init__(self, states: Sequence[CfrState], params: Optional[CfrParams] = None,
                 t_first: int = 1, t_last: int = 1000, stream=None):
        self.states = list(states)
        self.params = params if params is not None else paper_params()
        fg = (C.c_void_p * len(self.states))(*[st.fgt.h for st in self.states])
        sp = (C.c_void_p * len(self.states))(*[C.addressof(st.c) for st in self.states])
        h = C.c_void_p()
        _check(lib().pasur_plan_create(fg, sp, len(self.states), C.byref(self.params), t_first,
                                       t_last, C.byref(h), _stream(stream)), "pasur_plan_create")
        self.h = h
        self.t_first, self.t_last = t_first, t_last
        info = (C.c_int64 * 8)()
        _check(lib().pasur_plan_info(self.h, info), "pasur_plan_info")
        (self.n_segs, self.n_lds_segs, self.lds_bytes, self.block, self.edges, self.internal,
         self.roots, self.n7) = list(info)

    def iterate(self, t0: int, n_iters: int, stream=None):
        _check(lib().pasur_plan_iterate(self.h, t0, n_iters, _stream(stream)), "pasur_plan_iterate")
        for st in self.states:
            st.t = t0 + n_iters

    def free(self):
        if getattr(self, "h", None):
            lib().pasur_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class MlpWeights(C.Structure):
    _fields_ = [("W1", C.c_void_p), ("b1", C.c_void_p), ("W2", C.c_void_p), ("b2", C.c_void_p),
                ("W3", C.c_void_p), ("b3", C.c_void_p), ("W1t", C.c_void_p), ("W2t", C.c_void_p)]


class MlpGrads(C.Structure):
    _fields_ = [("dW1", C.c_void_p), ("db1", C.c_void_p), ("dW2", C.c_void_p),
                ("db2", C.c_void_p), ("dW3", C.c_void_p), ("db3", C.c_void_p)]


def _p(t):
    """Device pointer of a tensor (None stays NULL)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def gemm_bf16(M, N, K, A, sar, sac, B, sbr, sbc, Cf=None, Cb=None, ldc=None, bias=None,
              relu=False, stream=None):
    """pasur_gemm_bf16 on torch tensors (A, B, Cb as int16 bit patterns)."""
    _check(lib().pasur_gemm_bf16(M, N, K, _p(A), sar, sac, _p(B), sbr, sbc, _p(Cf), _p(Cb),
                                 N if ldc is None else ldc, _p(bias), 1 if relu else 0,
                                 _stream(stream)), "pasur_gemm_bf16")


def mlp_forward(w: MlpWeights, X, M, H1, H2, Y, stream=None):
    _check(lib().pasur_mlp_forward(C.byref(w), _p(X), M, _p(H1), _p(H2), _p(Y), _stream(stream)),
           "pasur_mlp_forward")


def mlp_infer(w: MlpWeights, X, M, Y, stream=None):
    _check(lib().pasur_mlp_infer(C.byref(w), _p(X), M, _p(Y), _stream(stream)), "pasur_mlp_infer")


def mlp_backward(w: MlpWeights, X, H1, H2, dY, M, g: MlpGrads, stream=None):
    _check(lib().pasur_mlp_backward(C.byref(w), _p(X), _p(H1), _p(H2), _p(dY), M, C.byref(g),
                                    _stream(stream)), "pasur_mlp_backward")


def mlp_loss(Y, tsig, tval, seg, n_par, n_rows, value_weight, dY, loss, stream=None):
    _check(lib().pasur_mlp_loss(_p(Y), _p(tsig), _p(tval), _p(seg), n_par, n_rows,
                                value_weight, _p(dY), _p(loss), _stream(stream)), "pasur_mlp_loss")


def adam_step(w, g, m, v, wb, lr, b1, b2, eps, step, stream=None):
    _check(lib().pasur_adam_step(_p(w), _p(g), _p(m), _p(v), _p(wb), w.numel(), lr, b1, b2, eps,
                                 step, _stream(stream)), "pasur_adam_step")


def adam_step_multi(ws, gs, ms, vs, wbs, lr, b1, b2, eps, step, stream=None):
    """pasur_adam_step_multi: one launch over the arrays of the lists (wbs
    entries may be None)."""
    k = len(ws)
    arr = lambda ts: (C.c_void_p * k)(*[None if t is None else t.data_ptr() for t in ts])
    n = (C.c_int64 * k)(*[t.numel() for t in ws])
    _check(lib().pasur_adam_step_multi(k, arr(ws), arr(gs), arr(ms), arr(vs), arr(wbs), n, lr, b1,
                                       b2, eps, step, _stream(stream)), "pasur_adam_step_multi")


def edge_features(gt: GameTree, fgt: UnfoldedTree, level: int, edges, n: int, X, stream=None):
    _check(lib().pasur_edge_features(gt.h, fgt.h, level, _p(edges), n, _p(X), _stream(stream)),
           "pasur_edge_features")


def sample_parents(fgt: UnfoldedTree, level: int, seed: int, keep_prob: float, seg, edges,
                   stream=None):
    npar, ne = C.c_int64(), C.c_int64()
    _check(lib().pasur_sample_parents(fgt.h, level, seed, keep_prob, _p(seg), _p(edges),
                                      C.byref(npar), C.byref(ne), _stream(stream)),
           "pasur_sample_parents")
    return npar.value, ne.value


def cfr_warm_init(st: CfrState, level: int, Y, kappa_r: float, kappa_s: float, stream=None):
    _check(lib().pasur_cfr_warm_init(st.fgt.h, C.byref(st.c), level, _p(Y), kappa_r, kappa_s,
                                     _stream(stream)), "pasur_cfr_warm_init")


def warm_start_workspace_bytes(fgt: UnfoldedTree, max_level: int) -> int:
    return int(lib().pasur_warm_start_workspace_bytes(fgt.h, max_level))


def warm_start_round(gt: GameTree, st: CfrState, w: MlpWeights, max_level: int, kappa_r: float,
                     kappa_s: float, workspace=None, stream=None):
    nbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().pasur_warm_start_round(gt.h, st.fgt.h, C.byref(st.c), C.byref(w), max_level,
                                        kappa_r, kappa_s, _p(workspace), nbytes, _stream(stream)),
           "pasur_warm_start_round")


def mlp_transpose(w: MlpWeights, W1t, W2t, stream=None):
    _check(lib().pasur_mlp_transpose(C.byref(w), _p(W1t), _p(W2t), _stream(stream)),
           "pasur_mlp_transpose")


PLAY_SIGMA_BAR, PLAY_UNIFORM = 0, 1


def es_workspace_bytes(fgt: UnfoldedTree, dtype: int) -> int:
    n = lib().pasur_es_workspace_bytes(fgt.h, dtype)
    if n < 0:
        _check(int(n), "pasur_es_workspace_bytes")
    return int(n)


ES_FRONTIER, ES_LEVEL = 0, 1
INFOSET_INT8, INFOSET_MLP = 0, 1
INFOSET_WIDTH = 58


def infoset_rows(gt: GameTree, fgt: UnfoldedTree, level: int, d_edges, n: int, out,
                 fmt: int = INFOSET_INT8, stream=None):
    """Infoset rows of FGT nodes of `level` (pasur_infoset_rows): out is an
    int8 [n, 58] device tensor (INFOSET_INT8) or int16 [n, 192] holding BF16
    network input (INFOSET_MLP); d_edges None means every node in order."""
    _check(lib().pasur_infoset_rows(gt.h, fgt.h, level, None if d_edges is None else _p(d_edges), n,
                                    fmt, _p(out), _stream(stream)), "pasur_infoset_rows")
    return out


def es_iterate(st: CfrState, n_iters: int, seed: int, rm_mode: int = RM_FLOOR, eps: float = 1e-8,
               t0: Optional[int] = None, schedule: int = ES_FRONTIER, roots_per_wg: int = 0,
               stats=None, stream=None):
    """n_iters external-sampling CFR iterations on st (pasur_es_iterate),
    continuing after st.es_t iterations (or t0); the pick workspace is kept
    on the state.  stats: optional int64 device tensor of 4 counters (frontier
    schedule) that gains the work done (see pasur_es_iterate)."""
    torch = _torch()
    nb = es_workspace_bytes(st.fgt, st.dtype)
    if st.es_ws is None or st.es_ws.numel() < max(nb, 1):
        st.es_ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    t = st.es_t if t0 is None else t0
    _check(lib().pasur_es_iterate(st.fgt.h, C.byref(st.c), t, n_iters, seed & ((1 << 64) - 1),
                                  rm_mode, eps, schedule, roots_per_wg, _p(st.es_ws), st.es_ws.numel(),
                                  None if stats is None else _p(stats), _stream(stream)),
           "pasur_es_iterate")
    st.es_t = t + n_iters


def selfplay(fgts, sigma_bars, dtype: int, root: int, n_games: int, seed: int, policy_a: int,
             policy_b: int, margin, stream=None):
    """fgts: UnfoldedTree of consecutive rounds; sigma_bars[r][l] (l = 1..8)
    device tensors of the average strategies; margin: int32 device tensor of
    n_games entries (pasur_selfplay)."""
    n = len(fgts)
    hs = (C.c_void_p * n)(*[f.h for f in fgts])
    sb = (C.c_void_p * (9 * n))()
    for r in range(n):
        for l in range(1, 9):
            sb[9 * r + l] = _p(sigma_bars[r][l])
    _check(lib().pasur_selfplay(hs, n, sb, dtype, root, n_games, seed & ((1 << 64) - 1), policy_a,
                                policy_b, _p(margin), _stream(stream)), "pasur_selfplay")


def gather_f32(src, dtype: int, idx, n: int, dst, stream=None):
    _check(lib().pasur_gather_f32(_p(src), dtype, _p(idx), n, _p(dst), _stream(stream)),
           "pasur_gather_f32")


def shift_i32(src, n: int, add: int, dst, stream=None):
    _check(lib().pasur_shift_i32(_p(src), n, add, _p(dst), _stream(stream)), "pasur_shift_i32")


def profile_enable(on: bool):
    _check(lib().pasur_profile_enable(1 if on else 0), "pasur_profile_enable")


def profile_select(kernels):
    """Record only the given kernel ids (see pasur_profile_read)."""
    mask = 0
    for k in kernels:
        mask |= 1 << int(k)
    _check(lib().pasur_profile_select(mask), "pasur_profile_select")


def profile_count() -> int:
    """Number of sweep launches recorded so far (reads no timings, so it
    does not wait for the GPU)."""
    n = C.c_int64()
    _check(lib().pasur_profile_read(0, None, None, None, None, C.byref(n)), "pasur_profile_read")
    return n.value


def profile_read():
    """Recorded sweep launches: arrays (kernel, level, milliseconds, work)
    with work[i] = (edges, internal nodes, roots, level-7 nodes, iterations)."""
    n = C.c_int64()
    _check(lib().pasur_profile_read(0, None, None, None, None, C.byref(n)), "pasur_profile_read")
    m = max(n.value, 1)
    k = np.zeros(m, np.int32)
    lv = np.zeros(m, np.int32)
    ms = np.zeros(m, np.float32)
    work = np.zeros((m, 5), np.int64)
    _check(lib().pasur_profile_read(n.value, k.ctypes.data_as(C.c_void_p),
                                    lv.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p),
                                    work.ctypes.data_as(C.c_void_p), C.byref(n)),
           "pasur_profile_read")
    return k[: n.value], lv[: n.value], ms[: n.value], work[: n.value]


from .solver import SubgameSolver, RoundResult, BatchSolver, playout_root  # noqa: E402  (drivers over the calls above)
