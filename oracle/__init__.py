"""FP64 CPU oracle for the Pasur round solver (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py`` -- never by the HIP product path, with which
it shares no code.  The arithmetic lives in ``pasur_oracle.c``; this module
only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pasur_oracle.c")
_LIB = os.path.join(_HERE, "libpasur_oracle.so")

GT_POOL, GT_HANDS, GT_RS, GT_PARENT, GT_CHILD_BEGIN, GT_ACT_CARD, GT_ACT_CAP = range(7)
FGT_GT, FGT_SID, FGT_PARENT, FGT_CHILD_BEGIN, FGT_SCORE_TAB, FGT_NEXT_ROOTS, FGT_LINK = range(7)
CF_SIGMA, CF_R, CF_SBAR, CF_U, CF_REACHA, CF_REACHB, CF_VACC, CF_SIGMA_BAR = range(8)
TV_EXPECT, TV_BR_A, TV_BR_B, TV_MINIMAX = range(4)
LITERAL_BONUS0 = 1  # leaf utilities: the printed final_util (-7 when nobody reached 7 clubs)
SNIPPET_TOL, SNIPPET_AVG = 1, 2  # Params.flags: the executed forms of CodeSnippet FindUtility
CFR_DCFR, CFR_PLUS, CFR_VANILLA = range(3)
RM_FLOOR, RM_POSITIVE = range(2)

ROOT_DTYPE = np.dtype([("pool", "<u8"), ("ca", "i1"), ("cb", "i1"), ("d", "i1"),
                       ("bonus", "i1"), ("pad", "<i4")])


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O2; OpenMP only for the
    optional multi-threaded CFR loops, single-threaded by default)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.or_subset11_count.argtypes = [vp]
        L.or_children.argtypes = [i32, i32, C.c_uint64, C.c_uint64, C.c_uint64, vp, i32,
                                  vp, vp, vp, vp, vp, vp]
        L.or_combine_score.argtypes = [vp, vp, vp]
        L.or_gt_build.restype = vp
        L.or_gt_build.argtypes = [vp, i32, vp, i64, C.POINTER(C.c_int)]
        L.or_gt_size.restype = i64
        L.or_gt_size.argtypes = [vp, i32]
        L.or_gt_copy.argtypes = [vp, i32, i32, vp]
        L.or_gt_free.argtypes = [vp]
        L.or_fgt_unfold.restype = vp
        L.or_fgt_unfold.argtypes = [vp, vp, i64, C.POINTER(C.c_int)]
        L.or_fgt_unfold_csr.restype = vp
        L.or_fgt_unfold_csr.argtypes = [vp, vp, vp, vp, i64, C.POINTER(C.c_int)]
        L.or_fgt_size.restype = i64
        L.or_fgt_size.argtypes = [vp, i32]
        L.or_fgt_n_scores.restype = i64
        L.or_fgt_n_scores.argtypes = [vp]
        L.or_fgt_n_next.restype = i64
        L.or_fgt_n_next.argtypes = [vp]
        L.or_fgt_copy.argtypes = [vp, i32, i32, vp]
        L.or_fgt_free.argtypes = [vp]
        L.or_leaf_utilities.argtypes = [vp, vp, vp, C.c_int, vp]
        L.or_cfr_create.restype = vp
        L.or_cfr_create.argtypes = [vp, vp, vp, C.POINTER(C.c_int)]
        L.or_cfr_run.argtypes = [vp, vp, i64, i32]
        L.or_set_threads.argtypes = [i32]
        L.or_cfr_copy.argtypes = [vp, i32, i32, vp]
        L.or_cfr_free.argtypes = [vp]
        L.or_tree_values.argtypes = [vp, vp, vp, vp, i32, i32, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(st: int, what: str):
    if st < 0:
        raise OracleError(f"{what} failed with status {st}")


class _Params(C.Structure):
    _fields_ = [("variant", C.c_int), ("rm_mode", C.c_int), ("alpha", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("flags", C.c_int)]


@dataclass
class Params:
    """DCFR constants of the paper's experiments (gamma=2, alpha=1.5, beta=0)
    and the regret-matching floor of its executed rule (eps = 1e-8)."""
    variant: int = CFR_DCFR
    rm_mode: int = RM_FLOOR
    alpha: float = 1.5
    beta: float = 0.0
    gamma: float = 2.0
    eps: float = 1e-8
    flags: int = 0  # SNIPPET_TOL | SNIPPET_AVG (DCFR only)

    def c(self):
        return _Params(self.variant, self.rm_mode, self.alpha, self.beta, self.gamma, self.eps,
                       self.flags)


def subset11_count():
    by = np.zeros(16, np.int64)
    n = lib().or_subset11_count(_ptr(by))
    _check(n, "subset11_count")
    return n, by


def children(rnd: int, ply: int, pool: int, handA: int, handB: int, rs=None):
    """Legal children of a card state: list of (card, cap, pool, handA, handB, rs)."""
    rs = np.zeros(8, np.int8) if rs is None else np.asarray(rs, np.int8)
    m = 600
    ac = np.zeros(m, np.uint8); cap = np.zeros(m, np.uint64)
    cp = np.zeros(m, np.uint64); ca = np.zeros(m, np.uint64); cbh = np.zeros(m, np.uint64)
    crs = np.zeros(8 * m, np.int8)
    n = lib().or_children(rnd, ply, pool, handA, handB, _ptr(rs), m, _ptr(ac), _ptr(cap),
                          _ptr(cp), _ptr(ca), _ptr(cbh), _ptr(crs))
    _check(n, "children")
    return [(int(ac[i]), int(cap[i]), int(cp[i]), int(ca[i]), int(cbh[i]),
             crs[8 * i: 8 * i + 8].copy()) for i in range(n)]


def combine_score(s, rs):
    s = np.asarray(s, np.int8); rs = np.asarray(rs, np.int8)
    out = np.zeros(4, np.int8)
    lib().or_combine_score(_ptr(s), _ptr(rs), _ptr(out))
    return out


def roots_array(roots) -> np.ndarray:
    a = np.zeros(len(roots), ROOT_DTYPE)
    for i, r in enumerate(roots):
        a[i] = (r.pool, r.ca, r.cb, r.d, r.bonus, 0)
    return a


class GT:
    """Round game tree (levels 0..8, canonical order)."""

    def __init__(self, deck, rnd: int, pools):
        self.deck = np.asarray(deck, np.uint8)
        self.round = rnd
        p = np.ascontiguousarray(np.asarray(pools, np.uint64))
        st = C.c_int(0)
        self.h = lib().or_gt_build(_ptr(self.deck), rnd, _ptr(p), len(p), C.byref(st))
        if not self.h:
            raise OracleError(f"or_gt_build failed with status {st.value}")
        self.n = [lib().or_gt_size(self.h, l) for l in range(9)]

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_gt_free(self.h)
            self.h = None

    def get(self, field: int, level: int) -> np.ndarray:
        n = self.n[level]
        dt = {GT_POOL: np.uint64, GT_HANDS: np.uint8, GT_RS: np.int8, GT_PARENT: np.int32,
              GT_CHILD_BEGIN: np.int32, GT_ACT_CARD: np.uint8, GT_ACT_CAP: np.uint64}[field]
        size = n + 1 if field == GT_CHILD_BEGIN else (8 * n if field == GT_RS else n)
        out = np.zeros(max(size, 1), dt)
        _check(lib().or_gt_copy(self.h, field, level, _ptr(out)), "gt_copy")
        out = out[:size]
        return out.reshape(n, 8) if field == GT_RS else out


class FGT:
    """Unfolded tree of one round plus the next-round roots and linkage."""

    def __init__(self, gt: Optional[GT], roots=None, *, csr=None):
        st = C.c_int(0)
        self.gt = gt
        if csr is not None:
            gt_n, gt_cb, root_gt, root_sid = csr
            n_arr = np.asarray(gt_n, np.int64)
            self._keep = [np.ascontiguousarray(np.asarray(x, np.int32)) for x in gt_cb]
            ptrs = (C.c_void_p * 8)(*[x.ctypes.data for x in self._keep])
            rg = np.ascontiguousarray(np.asarray(root_gt, np.int32))
            rsd = np.ascontiguousarray(np.asarray(root_sid, np.int32))
            self.h = lib().or_fgt_unfold_csr(_ptr(n_arr), ptrs, _ptr(rg), _ptr(rsd), len(rg),
                                             C.byref(st))
        else:
            ra = roots_array(roots)
            self.h = lib().or_fgt_unfold(gt.h, _ptr(ra), len(ra), C.byref(st))
        if not self.h:
            raise OracleError(f"or_fgt_unfold failed with status {st.value}")
        self.n = [lib().or_fgt_size(self.h, l) for l in range(9)]
        self.n_scores = lib().or_fgt_n_scores(self.h)
        self.n_next = lib().or_fgt_n_next(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_fgt_free(self.h)
            self.h = None

    def get(self, field: int, level: int = 0) -> np.ndarray:
        if field == FGT_SCORE_TAB:
            out = np.zeros(max(4 * self.n_scores, 1), np.int8)
            _check(lib().or_fgt_copy(self.h, field, 0, _ptr(out)), "fgt_copy")
            return out[: 4 * self.n_scores].reshape(-1, 4)
        if field == FGT_NEXT_ROOTS:
            out = np.zeros(max(self.n_next, 1), ROOT_DTYPE)
            _check(lib().or_fgt_copy(self.h, field, 0, _ptr(out)), "fgt_copy")
            return out[: self.n_next]
        n = self.n[8] if field == FGT_LINK else self.n[level]
        size = n + 1 if field == FGT_CHILD_BEGIN else n
        out = np.zeros(max(size, 1), np.int32)
        _check(lib().or_fgt_copy(self.h, field, 8 if field == FGT_LINK else level, _ptr(out)),
               "fgt_copy")
        return out[:size]

    def child_begin(self) -> List[np.ndarray]:
        return [self.get(FGT_CHILD_BEGIN, l) for l in range(8)]

    def leaf_utilities(self, V_next=None, literal_bonus0: bool = False) -> np.ndarray:
        out = np.zeros(max(self.n[8], 1), np.float64)
        vn = None if V_next is None else np.ascontiguousarray(np.asarray(V_next, np.float64))
        _check(lib().or_leaf_utilities(self.gt.h, self.h, None if vn is None else _ptr(vn),
                                       LITERAL_BONUS0 if literal_bonus0 else 0, _ptr(out)),
               "leaf_utilities")
        return out[: self.n[8]]


class CFR:
    """DCFR state of one round (FP64)."""

    def __init__(self, n, child_begin, leaf_u):
        self.n = [int(x) for x in n]
        n_arr = np.asarray(self.n, np.int64)
        self._cb = [np.ascontiguousarray(np.asarray(x, np.int32)) for x in child_begin]
        ptrs = (C.c_void_p * 8)(*[x.ctypes.data for x in self._cb])
        lu = np.ascontiguousarray(np.asarray(leaf_u, np.float64))
        st = C.c_int(0)
        self.h = lib().or_cfr_create(_ptr(n_arr), ptrs, _ptr(lu), C.byref(st))
        if not self.h:
            raise OracleError(f"or_cfr_create failed with status {st.value}")
        self.t = 1

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_cfr_free(self.h)
            self.h = None

    def run(self, n_iters: int, params: Params = Params()):
        p = params.c()
        _check(lib().or_cfr_run(self.h, C.byref(p), self.t, n_iters), "cfr_run")
        self.t += n_iters

    def get(self, field: int, level: int = 0) -> np.ndarray:
        n = self.n[0] if field == CF_VACC else self.n[level]
        out = np.zeros(max(n, 1), np.float64)
        _check(lib().or_cfr_copy(self.h, field, level, _ptr(out)), "cfr_copy")
        return out[:n]

    def sigma_bar(self) -> List[np.ndarray]:
        return [np.ones(self.n[0])] + [self.get(CF_SIGMA_BAR, l) for l in range(1, 9)]


def set_threads(n: int) -> None:
    """Threads for the per-level parent loops of CFR.run (1 = the plain
    single-threaded oracle; results are bit-identical for any count)."""
    _check(lib().or_set_threads(int(n)), "set_threads")


def tree_values(n, child_begin, leaf, sigma, mode: int, level: int = 0) -> np.ndarray:
    n_arr = np.asarray([int(x) for x in n], np.int64)
    cb = [np.ascontiguousarray(np.asarray(x, np.int32)) for x in child_begin]
    cbp = (C.c_void_p * 8)(*[x.ctypes.data for x in cb])
    if sigma is None:
        sg = [np.zeros(max(int(n[l]), 1)) for l in range(9)]
    else:
        sg = [np.ascontiguousarray(np.asarray(s, np.float64)) for s in sigma]
    sp = (C.c_void_p * 9)(*[x.ctypes.data for x in sg])
    lf = np.ascontiguousarray(np.asarray(leaf, np.float64))
    out = np.zeros(max(int(n[level]), 1), np.float64)
    _check(lib().or_tree_values(_ptr(n_arr), cbp, _ptr(lf), sp, mode, level, _ptr(out)),
           "tree_values")
    return out[: int(n[level])]
