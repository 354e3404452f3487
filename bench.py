#!/usr/bin/env python3
"""Benchmark: full-width DCFR node-updates/s on one MI355X.

One step = the whole hot path on one seeded two-round subgame (the last two
rounds of deal 1, every round-6 card state times every inherited score):
build both rounds' game trees, unfold them, link the leaves to next-round
roots, leaf utilities, 2000 DCFR iterations per round (last round first),
average strategies, round values passed backward, and the composed
exploitability of the average strategies.  Inputs are resident on the GPU
before the timed region; K steps are timed between device synchronisations.

Prints one JSON line ("Measurement").
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFR node-updates/s at 1 GPU; secs to exploitability 1e-3, warm-start vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def up_bytes(n, l, T):
    """Algorithmic bytes of one fused up-sweep launch for child level l:
    per edge sigma, u, R, Sbar read and R, Sbar, sigma written (7 T); per
    parent the CSR offset, both reaches read and u written (4 + 3 T);
    vacc read and written at the roots."""
    b = n[l] * 7 * T + n[l - 1] * (4 + 3 * T) + 4
    if l == 1:
        b += 16 * n[0]
    return b


def down_bytes(n, l, T):
    """Reach down-sweep, child level l: parent index, sigma, two reaches
    written per child; two parent reaches read per parent."""
    return n[l] * (4 + 3 * T) + n[l - 1] * 2 * T


def cpu_baseline(deck, roots, iters):
    """The FP64 oracle on the same workload, single-threaded on a host core."""
    import numpy as np
    import oracle
    import synth

    t0 = time.perf_counter()
    rounds = []
    rr = roots
    for r in (4, 5):
        gt = oracle.GT(deck, r, sorted({x.pool for x in rr}))
        f = oracle.FGT(gt, rr)
        rounds.append((gt, f))
        if r == 4:
            rr = [synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]),
                             int(x["bonus"])) for x in f.get(oracle.FGT_NEXT_ROOTS)]
    V = None
    sbars = [None, None]
    edges = 0
    for k in (1, 0):
        gt, f = rounds[k]
        c = oracle.CFR(f.n, f.child_begin(), f.leaf_utilities(V))
        c.run(iters)
        V = c.get(oracle.CF_VACC) / iters
        sbars[k] = c.sigma_bar()
        edges += sum(f.n[1:])
    for mode in (oracle.TV_BR_A, oracle.TV_BR_B):
        W = None
        for k in (1, 0):
            gt, f = rounds[k]
            W = oracle.tree_values(f.n, f.child_begin(), f.leaf_utilities(W), sbars[k], mode)
    el = time.perf_counter() - t0
    return {"value": edges * iters / el, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the full workload once (both rounds, {iters} iterations each, trees, "
                      f"values and exploitability), {el:.1f} s single-threaded FP64",
            "seconds": el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--state", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this solver is a single-GPU build "
              "(see DESIGN.md, 'More than one GPU'); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2508_06559_amd as pa
    import synth

    torch.cuda.set_device(0)
    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    deck, roots = synth.two_round_root(args.seed)
    d_roots = pa.roots_to_device(roots)  # resident before timing
    torch.cuda.synchronize()

    def step():
        s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        s.solve(args.iters)
        bra, brb, v = s.exploitability()
        torch.cuda.synchronize()
        ex = float(((bra - brb) / 2).max().item())
        sizes = s.sizes()
        s.free()
        return sizes, ex

    for w in range(args.warmup):
        sizes, ex = step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done, exploitability {ex:.3e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sizes, ex = step()
        log(f"[bench] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    edges = sum(sum(n[1:]) for n in sizes)
    nodes = sum(sum(n) for n in sizes)
    value = edges * args.iters * args.steps / el

    # Dominant kernel: the fused up-sweep.  Average launch duration measured
    # live with HIP events on the launch stream over one step's iterations.
    s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
    pa.profile_enable(True)
    s.solve(args.iters)
    torch.cuda.synchronize()
    kern, lev, ms = pa.profile_read()
    pa.profile_enable(False)
    # records come round by round (last round first), iteration by iteration
    order = [s.rounds[1].fgt.n, s.rounds[0].fgt.n]
    recs_per_round = 15 * args.iters
    up_b = up_t = dn_b = dn_t = 0.0
    n_up = 0
    for idx in range(len(kern)):
        n = order[idx // recs_per_round]
        if kern[idx] == 1:
            up_b += up_bytes(n, int(lev[idx]), T)
            up_t += float(ms[idx]) * 1e-3
            n_up += 1
        else:
            dn_b += down_bytes(n, int(lev[idx]), T)
            dn_t += float(ms[idx]) * 1e-3
    s.free()
    achieved = up_b / up_t / 1e9
    log(f"[bench] up-sweep: {n_up} launches, avg {up_t / n_up * 1e6:.2f} us, "
        f"{up_b / n_up / 1e6:.3f} MB/launch; down-sweep avg {dn_t / (len(kern) - n_up) * 1e6:.2f} us")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"last two rounds of seeded deal {args.seed}: full unfolded trees "
                        f"({nodes} nodes, {edges} edges), {args.iters} DCFR iterations per round, "
                        f"backward round values, composed exploitability",
            "state": args.state,
            "arithmetic": "f64 registers",
            "iters_per_round": args.iters,
            "level_sizes": sizes,
            "exploitability_points": ex,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_up<{'float' if T == 4 else 'double'}> (fused up-sweep)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": up_t / n_up * 1e6,
            "algorithmic_bytes_per_launch": up_b / n_up,
            "iteration_effective_GBs": (up_b + dn_b) / (up_t + dn_t) / 1e9,
        },
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(deck, roots, args.iters)
        log(f"[bench] cpu baseline done in {out['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
