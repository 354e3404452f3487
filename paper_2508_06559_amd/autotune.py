"""Autotuner for the persistent segment schedule (a12).

For every round of a batch it times each candidate schedule -- threads per
workgroup x root-run length (seg_nodes) -- on a short run of the real plan
and keeps the fastest.  Timing uses HIP events on the launch stream.  The
chosen schedule is returned and can be written as JSON.  Tuning runs DCFR
iterations on the solver states; callers re-initialise them (cfr_init)
before solving, as BatchSolver.solve does.
"""
from __future__ import annotations

import json
from typing import Dict, List, Optional, Sequence, Tuple

from . import CfrState, Plan, paper_params, _torch

# threads per workgroup x root-run length (0: one root per segment; a run
# also stops at the workgroup's thread count and at its LDS budget)
BLOCKS: Tuple[int, ...] = (256, 512, 1024)
SEG_NODES: Tuple[int, ...] = (0, 2048, 4096, 8192, 16384, 32768)
DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = tuple((b, g) for b in BLOCKS for g in SEG_NODES)


def time_plan(states: Sequence[CfrState], block: int, seg_nodes: int, iters: int) -> float:
    """Milliseconds per iteration of one plan over ``states``."""
    torch = _torch()
    plan = Plan(states, paper_params(block=block, seg_nodes=seg_nodes), 1, iters + 1)
    plan.iterate(1, 1)  # warm-up (first launch, caches)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    plan.iterate(2, iters)
    b.record()
    b.synchronize()
    plan.free()
    return a.elapsed_time(b) / iters


def autotune(rounds_states: List[Sequence[CfrState]], candidates=DEFAULT_CANDIDATES,
             iters: int = 20, out_json: Optional[str] = None, log=None) -> Dict:
    """rounds_states[k] = the states one plan of round k covers."""
    result = {"candidates": [list(c) for c in candidates], "iters_timed": iters, "rounds": []}
    for k, states in enumerate(rounds_states):
        if not states:  # every tree of the round is streamed: no plan to tune
            result["rounds"].append({"slot": k, "best": None, "timings": []})
            continue
        timings = []
        for block, seg in candidates:
            ms = time_plan(states, block, seg, iters)
            timings.append({"block": block, "seg_nodes": seg, "ms_per_iter": ms})
            if log:
                log(f"[autotune] round-slot {k}: block={block} seg_nodes={seg} {ms * 1e3:.1f} us/iter")
        best = min(timings, key=lambda x: x["ms_per_iter"])
        result["rounds"].append({"slot": k, "best": best, "timings": timings})
    if out_json:
        with open(out_json, "w") as fh:
            json.dump(result, fh, indent=1)
    return result


def params_from(result: Dict) -> List:
    return [paper_params(block=r["best"]["block"], seg_nodes=r["best"]["seg_nodes"])
            if r["best"] is not None else paper_params() for r in result["rounds"]]
