#!/usr/bin/env python3
"""Benchmark: full-width DCFR node-updates/s on one MI355X.

Default workload (full-game): one step = the whole hot path on the full game
of seeded deal 40 (all six rounds from the initial deal, 8.5e8 unfolded
nodes): build every round's game tree, unfold it, link the leaves to
next-round roots, leaf utilities, 1000 DCFR iterations per round (last round
first), average strategies, round values passed backward, and the composed
exploitability of the average strategies.  The deal's roots are resident on
the GPU before the timed region; K steps are timed between device
synchronisations.  Other workloads (--workload): two-round (the last two
rounds of one deal from a seeded legal playout), batched (64 deals from
playouts, rounds 4-6, one persistent launch per round, HIP-graph replay),
paper-scale (32 full games as one batch), warm-start (learned warm start vs
plain DCFR), selfplay (games/s and fair values on a solved full game), es
(external-sampling CFR on a full game), infoset (infoset rows of a full
game; strategy models on them), mlp (the network's MFMA kernels alone),
variants (DCFR, CFR+ and vanilla CFR convergence), copy (counter
calibration), copy-rate (the HBM rate of a plain device copy).

Prints one JSON line: the metric and its value, the step time, the
dominant kernel's roofline (achieved algorithmic bytes or FLOPs per second
against the MI355X peak, with counter-measured HBM traffic per launch and
its rate, `traffic_GBs`, when recorded for this kernel source) and, for the
full-game and two-round workloads, the FP64 CPU oracle's rate on the host
(cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFR node-updates/s at 1 GPU; secs to exploitability 1e-3, warm-start vs plain"

# HBM bytes per launch of each workload's dominant kernel, from rocprofv3
# FETCH_SIZE / WRITE_SIZE counters scaled by a plain-copy calibration (the
# counter summaries under profiles/).  Valid only while the kernel's source
# file is unchanged (sha256 recorded with the counters).
TRAFFIC = {
    # k_cfr_seg, two-round subgame of deal 1 (average of its two launches)
    "two-round": {"source": "paper_2508_06559_amd/csrc/pasur_cfr.hip",
                  "sha256": "8a5ddb5c77265daad665dce4f88b4a8561c5daf99c8fbfcfc7c9ae652406889c",
                  "bytes": 4.60e6},
    # k_cfr_seg, the batched solve's largest launch (round 6 of all 64 deals)
    "batched": {"source": "paper_2508_06559_amd/csrc/pasur_cfr.hip",
                "sha256": "8a5ddb5c77265daad665dce4f88b4a8561c5daf99c8fbfcfc7c9ae652406889c",
                "bytes": 1.226e12},
    # the full game's dominant streaming kernel (average over its launches)
    "full-game": {"source": "paper_2508_06559_amd/csrc/pasur_sweep.hip",
                  "sha256": "b709966b880899046598e783d0007aaedb0aeb2b4c2c72f3c58875b6926fa956",
                  "bytes": 2.134e9},
}


def counted_traffic(args, workload="two-round"):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters (copy
    calibrated), valid only for the kernel source they were taken on."""
    import hashlib
    rec = TRAFFIC[workload]
    if rec["sha256"] is None or args.state != "f32":
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != rec["sha256"]:
            return None
    if workload == "two-round" and (args.sched not in ("root", "auto") or
                                    args.block not in (0, 1024)):
        return None
    if workload == "full-game" and args.sched != "auto":
        return None
    return rec["bytes"]


def playout_problem(seed, rnd):
    """Deal ``seed`` and the root of round ``rnd`` reached by the seeded legal
    playout (synth.playout_draws), played by the library's own round trees."""
    import paper_2508_06559_amd as pa
    import synth
    deck = synth.deal(seed)
    g = pa.playout_root(deck, rnd, synth.playout_draws(seed, 5))
    return deck, [synth.Root(int(g["pool"]), int(g["ca"]), int(g["cb"]), int(g["d"]),
                             int(g["bonus"]))]


def oracle_playout_problem(seed, rnd):
    """The same start state played by the oracle's own move generator (for
    the CPU baseline: no oracle input comes from the HIP path)."""
    import synth
    from oracle.playout import playout_root
    deck = synth.deal(seed)
    return deck, [playout_root(deck, rnd, synth.playout_draws(seed, 5))]


HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def launch_bytes(kernel, level, work, T):
    """Algorithmic bytes moved by one recorded sweep launch.

    Per edge and iteration the fused up-sweep reads sigma, u, R, Sbar and
    writes R, Sbar, sigma (7 T bytes); per parent it reads its CSR offset and
    both reaches and writes u (4 + 3 T); every root reads and writes vacc
    (16) and its two CSR ends add 4 per level.  The reach down-sweep reads
    the parent index and sigma and writes two reaches per child (4 + 3 T)
    and reads two reaches per parent (2 T).  The per-root schedule performs
    both sweeps over all levels of each root's subtree every iteration.
    """
    edges, internal, roots, n7, iters = (int(x) for x in work)
    if kernel == 1:  # one level of the up-sweep
        return edges * 7 * T + internal * (4 + 3 * T) + 4 + (16 * internal if level == 1 else 0)
    if kernel == 0:  # one level of the down-sweep
        return edges * (4 + 3 * T) + internal * 2 * T
    up = 7 * T * edges + (4 + 3 * T) * internal + 48 * roots
    down = (4 + 3 * T) * (internal - roots) + 2 * T * (internal - n7)
    return iters * (up + down)


def sweep_bytes(kernel, level, work, T):
    """Algorithmic bytes of one launch of the streaming schedule (kernel ids
    of pasur_profile_read; work = nodes or children, parents, boundary-list
    entries).  Per child of a tile up sweep: R and Sbar read and written, u
    read (5 T); per parent: two CSR ends, both reaches read, u written
    (4 + 3 T); per head of the compact tail at its boundary: its index, its
    utility and its next strategy (4 + 2 T).  Per node of a tile down sweep:
    R read, both reaches written (3 T); per parent: CSR, both reaches read
    (4 + 2 T); per boundary parent: two reach copies (2 T).  List and tail
    sweeps add their index reads (4 or 8 per node) and the stored sums of
    the tail's parents (8 read and written)."""
    n0, n1, n2 = int(work[0]), int(work[1]), int(work[2])
    if kernel in (5, 6):      # up, tiles / one thread per parent
        return n0 * 5 * T + n1 * (4 + 3 * T) + (16 * n1 if level == 1 else 0)
    if kernel == 11:          # up, tiles, the tail's first level
        return n0 * 5 * T + n1 * (4 + 3 * T) + n2 * (4 + 2 * T)
    if kernel in (4, 14):     # down, tiles / one thread per parent
        return n0 * 3 * T + n1 * (4 + 2 * T)
    if kernel == 12:          # down, tiles, the level above the tail
        return n0 * 3 * T + n1 * (4 + 2 * T) + n2 * (4 + 2 * T)
    if kernel == 13:          # down over a node list (first iteration)
        return n0 * (8 + 3 * T + 8 + 2 * T)
    if kernel == 7:           # up over a parent list
        return n0 * 5 * T + n1 * (4 + 8 + 3 * T)
    if kernel == 9:           # tail down
        return n0 * (8 + 3 * T + 8 + 2 * T)
    if kernel == 10:          # tail up
        return n0 * 5 * T + n1 * (4 + 4 + 16 + 3 * T)
    return 0


KERNEL_NAMES = {0: "k_down", 1: "k_up", 2: "k_cfr_seg (all LDS)", 3: "k_cfr_seg (LDS + global)",
                4: "k_sw_down_tile", 5: "k_sw_up_tile", 6: "k_sw_up_parent (dense)",
                7: "k_sw_up_parent (list)", 8: "streaming set-up", 9: "k_sw_down_list (tail)",
                10: "k_sw_up_parent (tail)", 11: "k_sw_up_tile (tail boundary)",
                12: "k_sw_down_tile (tail boundary)", 13: "k_sw_down_list", 14: "k_sw_down_parent"}
# rocprofv3 names of the kernel ids (FP32 state, the paper's variant)
KERNEL_SYMBOLS = {2: "k_cfr_seg<float, 1024, true>", 3: "k_cfr_seg<float, 1024, true>",
                  4: "k_sw_down_tile<float, true, false>", 5: "k_sw_up_tile<float, true, false>",
                  11: "k_sw_up_tile<float, true, true>", 12: "k_sw_down_tile<float, true, true>"}


def all_launch_bytes(kernel, level, work, T):
    if kernel in (0, 1, 2, 3):
        return launch_bytes(kernel, level, work, T)
    return sweep_bytes(kernel, level, work, T)


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


def bench_batched(args):
    """64 seeded deals (seeds 100..163), rounds 4-6 from the round-4 start of
    a seeded legal playout, 1000 DCFR iterations per round; the backward solve of all deals is
    captured in one HIP graph and replayed.  Schedules are autotuned first."""
    import torch
    import paper_2508_06559_amd as pa
    from paper_2508_06559_amd import autotune
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    iters = 1000 if args.iters == 2000 else args.iters
    probs = [playout_problem(seed, 3) for seed in range(100, 164)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = pa.BatchSolver(probs, 3, iters, dtype=dtype)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    edges = b.edges()
    sizes = [sum(sum(rr.fgt.n) for rr in sv.rounds) for sv in b.deals]
    log(f"[bench] batched: {len(probs)} deals, {sum(sizes)} nodes ({min(sizes)}..{max(sizes)}), "
        f"built in {build_s:.2f} s")
    sched = autotune.autotune(b.round_states(), iters=10, out_json=args.schedule_json, log=log)
    b.set_params(autotune.params_from(sched))
    for w in range(args.warmup):
        b.solve()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    b.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.replay()
        torch.cuda.synchronize()
        log(f"[bench] step {k + 1}/{args.steps} done")
    el = time.perf_counter() - t0
    value = edges * iters * args.steps / el
    # roofline: per-launch timing of the plans over one eager solve
    pa.profile_enable(True)
    b.solve()
    torch.cuda.synchronize()
    kern, lev, ms, work = pa.profile_read()
    pa.profile_enable(False)
    tot_b = sum(launch_bytes(int(kern[i]), int(lev[i]), work[i], T) for i in range(len(kern)))
    tot_t = sum(float(x) for x in ms) * 1e-3
    dom = int(np.argmax(ms))
    db = launch_bytes(int(kern[dom]), int(lev[dom]), work[dom], T)
    dt = float(ms[dom]) * 1e-3
    ex = [float(((x[0] - x[1]) / 2).max().item()) for x in b.exploitability()[:4]]
    out = {
        "metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: 64 seeded deals (seeds 100-163), rounds 4-6 from seeded legal playouts, {sum(sizes)} "
                               f"nodes ({min(sizes)}..{max(sizes)} per deal), {iters} DCFR iterations "
                               f"per round, backward solve of all deals replayed as one HIP graph",
                   "state": args.state, "build_seconds": build_s,
                   "schedule": [r["best"] for r in sched["rounds"]],
                   "exploitability_points_first_deals": ex},
        "roofline": {"bound": "hbm", "kernel": f"k_cfr_seg ({'float' if T == 4 else 'double'} state), "
                                             f"largest launch",
                     "achieved": db / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": db / dt / 1e9 / HBM_PEAK_GBS, "traffic": counted_traffic(args, "batched"),
                     "traffic_GBs": (counted_traffic(args, "batched") / dt / 1e9
                                     if counted_traffic(args, "batched") is not None else None),
                     "avg_launch_us": dt * 1e6, "algorithmic_bytes_per_launch": db,
                     "all_sweeps_GBs": tot_b / tot_t / 1e9},
    }
    print(json.dumps(out), flush=True)
    b.free()


def oracle_sample_roots(deck, per_round, seed):
    """Roots of every round that the full game from the initial deal
    reaches, found by following seeded picks through the oracle's own
    unfolding (up to per_round roots per round)."""
    import oracle
    import synth
    rng = np.random.default_rng(seed)
    cur = [synth.Root(synth.mask_of(deck[:4]), 0, 0, 0, 0)]
    out = []
    for r in range(6):
        out.append(cur)
        if r == 5:
            break
        f = oracle.FGT(oracle.GT(deck, r, sorted({x.pool for x in cur})), cur)
        nxt = [synth.Root(int(x["pool"]), int(x["ca"]), int(x["cb"]), int(x["d"]), int(x["bonus"]))
               for x in f.get(oracle.FGT_NEXT_ROOTS)]
        idx = sorted(rng.choice(len(nxt), size=min(per_round, len(nxt)), replace=False))
        cur = [nxt[i] for i in idx]
    return out


def cpu_baseline_full(deck, round_edges, iters, threads, per_round=32, seed=7, min_s=1.0):
    """The FP64 oracle's DCFR rate on seeded samples of every round of the
    full game (roots reached through the oracle's own unfolding), each round
    iterated until at least min_s seconds have passed, extrapolated per
    node-update to the whole workload (round_edges[r] edges per round,
    iters iterations each).  threads > 1 shares each level's parent loops."""
    import oracle
    sample = oracle_sample_roots(deck, per_round, seed)
    oracle.set_threads(threads)
    try:
        rates, desc = [], []
        for r, roots in enumerate(sample):
            f = oracle.FGT(oracle.GT(deck, r, sorted({x.pool for x in roots})), roots)
            leaf = f.leaf_utilities(None if r == 5 else np.zeros(max(f.n_next, 1)))
            c = oracle.CFR(f.n, f.child_begin(), leaf)
            edges = sum(f.n[1:])
            done, t0 = 0, time.perf_counter()
            while True:
                c.run(5)
                done += 5
                el = time.perf_counter() - t0
                if el >= min_s:
                    break
            rates.append(edges * done / el)
            desc.append(f"round {r + 1}: {len(roots)} roots, {sum(f.n)} nodes, {done} iterations")
    finally:
        oracle.set_threads(1)
    total_t = sum(e * iters / rt for e, rt in zip(round_edges, rates))
    value = sum(round_edges) * iters / total_t
    return value, rates, desc, total_t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_full(args):
    """All six rounds of seeded deal --full-seed from the initial deal, one
    step = the whole hot path: build and unfold every round, leaf
    utilities, DCFR round by round from round 6 backward (--iters per round,
    default 1000), average strategies, round values passed back, and the
    composed exploitability.  The default deal, seed 40, is the largest full
    game among seeds 1-64 (8.5e8 FGT nodes; the paper reports about 1e9 per
    deck on average)."""
    import torch
    import paper_2508_06559_amd as pa
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    iters = 1000 if args.iters == 2000 else args.iters
    deck, roots = synth.full_game_root(args.full_seed)
    d_roots = pa.roots_to_device(roots)  # resident before timing
    params = pa.paper_params({"root": pa.SCHED_ROOT, "level": pa.SCHED_LEVEL_SYNC,
                              "root-global": pa.SCHED_ROOT_GLOBAL, "stream": pa.SCHED_STREAM,
                              "auto": pa.SCHED_AUTO}[args.sched], args.block)
    round_ms = []

    def step(record_rounds=False, on_round=None):
        s = pa.SubgameSolver(deck, 0, roots, dtype=dtype)
        ev = [] if record_rounds else None
        s.solve(iters, params, round_events=ev, on_round=on_round)
        bra, brb, _ = s.exploitability()
        torch.cuda.synchronize()
        if ev is not None:
            round_ms[:] = [a.elapsed_time(b) for a, b in ev]
        ex = float(((bra - brb) / 2).max().item())
        sizes = s.sizes()
        V0 = float(s.rounds[0].V[0].item())
        s.free()
        return sizes, ex, V0

    def read_records():
        """The recorded sweep launches as (kernel id, algorithmic bytes,
        seconds from HIP events on the launch stream); the streaming
        schedule's per-call set-up (id 8) is not a sweep and is left out."""
        kern, lev, ms, work = pa.profile_read()
        return [(int(kern[i]), all_launch_bytes(int(kern[i]), int(lev[i]), work[i], T),
                 float(ms[i]) * 1e-3) for i in range(len(kern)) if int(kern[i]) != 8]

    def per_kernel(recs=None):
        """Algorithmic bytes, seconds and launches per kernel id."""
        per = {}
        for k, b1, t1 in (read_records() if recs is None else recs):
            b, t, c = per.get(k, (0.0, 0.0, 0))
            per[k] = (b + b1, t + t1, c + 1)
        return per

    # launch records per round in the first warm-up step: the count of
    # records (sweep launches enqueued, id 8 included) after each round
    bounds = []

    def mark(r):
        bounds.append((r, pa.profile_count()))

    # Warm-up steps time every sweep launch, which picks the dominant kernel
    # (the largest share of time) and gives the whole-sweep figures; the
    # timed steps then record only the dominant kernel's launches.  Without
    # warm-up, the timed steps record every launch.
    pa.profile_enable(True)
    per_all = None
    round_alg = {}
    for w in range(args.warmup):
        sizes, ex, V0 = step(on_round=mark if w == 0 else None)
        log(f"[bench] warmup {w + 1}/{args.warmup} done, exploitability {ex:.3e}")
    if args.warmup:
        kern, lev, ms, work = pa.profile_read()
        recs_all = [(int(kern[i]), all_launch_bytes(int(kern[i]), int(lev[i]), work[i], T),
                     float(ms[i]) * 1e-3) for i in range(len(kern))]
        prev = 0
        for r, cnt in bounds:
            part = [x for x in recs_all[prev:cnt] if x[0] != 8]
            b = sum(x[1] for x in part)
            t = sum(x[2] for x in part)
            lds = sum(x[1] for x in part if x[0] == 2)  # k_cfr_seg, every segment in LDS
            seg = sum(x[1] for x in part if x[0] in (2, 3))
            round_alg[r] = (b, t, lds / seg if seg else None)
            prev = cnt
        per_all = per_kernel([x for x in recs_all if x[0] != 8])
        dom = max(per_all, key=lambda k: per_all[k][1])
        pa.profile_enable(True)
        pa.profile_select([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sizes, ex, V0 = step(record_rounds=k == args.steps - 1)
        log(f"[bench] step {k + 1}/{args.steps} done ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    per_t = per_kernel()
    pa.profile_enable(False)
    if per_all is None:
        per_all = per_t
        dom = max(per_all, key=lambda k: per_all[k][1])
    for k, (b, t, c) in sorted(per_all.items(), key=lambda kv: -kv[1][1]):
        log(f"[bench] {KERNEL_NAMES.get(k, k)}: {c} launches, {t:.3f} s, avg {t / c * 1e6:.1f} us, "
            f"{b / c / 1e6:.3f} MB/launch, {b / t / 1e9:.1f} GB/s")
    all_b = sum(v[0] for v in per_all.values())
    all_t = sum(v[1] for v in per_all.values())
    db, dt, dc = per_t[dom]
    achieved = db / dt / 1e9
    edges = sum(sum(n[1:]) for n in sizes)
    nodes = sum(sum(n) for n in sizes)
    value = edges * iters * args.steps / el
    tr = counted_traffic(args, "full-game")
    rounds = []
    for r, n in enumerate(sizes):
        e_r = sum(n[1:])
        ms_r = round_ms[5 - r] if len(round_ms) == 6 else None
        b_r, t_r, lds_r = round_alg.get(r, (0.0, 0.0, None))
        rounds.append({"round": r + 1, "nodes": int(sum(n)), "edges": int(e_r),
                       "schedule": (("stream" if sum(n) >= 9_000_000 else "persistent segments")
                                    if args.sched == "auto" else args.sched),
                       "dcfr_ms": ms_r,
                       "node_updates_per_s": e_r * iters / (ms_r * 1e-3) if ms_r else None,
                       # algorithmic bytes of the round's sweep launches over
                       # their summed launch time (first warm-up step)
                       "alg_GBs": b_r / t_r / 1e9 if t_r else None,
                       "alg_frac": b_r / t_r / 1e9 / HBM_PEAK_GBS if t_r else None,
                       # share of the persistent kernel's algorithmic bytes in
                       # launches that kept every segment's state in LDS
                       "lds_resident_share": lds_r})
    out = {"metric": METRIC, "value": value, "unit": "node-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"full game of seeded deal {args.full_seed}: all 6 rounds "
                                  f"({nodes} FGT nodes, {edges} edges), {iters} DCFR iterations per "
                                  f"round, trees built and unfolded, round values passed back, "
                                  f"composed exploitability",
                      "state": args.state, "arithmetic": "f64 registers",
                      "schedule": args.sched, "iters_per_round": iters,
                      "rounds": rounds, "exploitability_points": ex, "game_value": V0},
           "roofline": {"bound": "hbm",
                        "kernel": f"{KERNEL_SYMBOLS.get(dom, KERNEL_NAMES.get(dom, dom))}",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": tr,
                        "traffic_GBs": tr / (dt / dc) / 1e9 if tr is not None else None,
                        "avg_launch_us": dt / dc * 1e6, "launches": dc,
                        "algorithmic_bytes_per_launch": db / dc,
                        "all_sweeps_GBs": all_b / all_t / 1e9,
                        "all_sweeps_frac": all_b / all_t / 1e9 / HBM_PEAK_GBS}}
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        round_edges = [sum(n[1:]) for n in sizes]
        log("[bench] cpu baseline (oracle, 1 thread) ...")
        v1, r1, desc, t1 = cpu_baseline_full(deck, round_edges, iters, 1)
        log(f"[bench] cpu baseline (oracle, {threads} threads) ...")
        vn, rn, _, tn = cpu_baseline_full(deck, round_edges, iters, threads)
        out["cpu_baseline"] = {
            "value": vn, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"the FP64 oracle's DCFR on seeded samples of every round (up to 32 roots "
                       f"per round, reached through the oracle's own unfolding; "
                       f"{'; '.join(desc)}), each round iterated >= 1 s, per-round rates "
                       f"extrapolated to the whole workload ({t1:.0f} s single-threaded, "
                       f"{tn:.0f} s on {threads} threads per step)"),
            "per_round_rates": rn,
            "single_thread": {"value": v1, "cores": 1, "per_round_rates": r1},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    print(json.dumps(out), flush=True)


def bench_paper_scale(args):
    """Full games of --deals seeded deals (seeds 1..N) solved together: every
    round of every game built and unfolded, then per round one persistent
    launch over the games' trees below --stream-min-nodes (a batched plan)
    and the streaming sweeps for each game's larger tree of that round, 1000
    DCFR iterations per round.  With the default 32 deals this is about 4e9
    FGT nodes (1.3e8 per deck on average; the paper reports about 1e9 per
    deck), all resident in HBM at once.  --stream-min-nodes 0 puts every
    round in the plan."""
    import torch
    import paper_2508_06559_amd as pa
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    iters = 1000 if args.iters == 2000 else args.iters
    probs = [synth.full_game_root(s) for s in range(1, args.deals + 1)]
    free0, total = torch.cuda.mem_get_info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = pa.BatchSolver(probs, 0, iters, dtype=dtype,
                       stream_min_nodes=args.stream_min_nodes if args.stream_min_nodes > 0 else None)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    n_streamed = sum(sum(st) for st in b.streamed)
    used = free0 - torch.cuda.mem_get_info()[0]
    per_deal = [sum(sum(rr.fgt.n) for rr in sv.rounds) for sv in b.deals]
    nodes = sum(per_deal)
    edges = b.edges()
    log(f"[bench] paper scale: {args.deals} full games, {nodes} nodes, built in {build_s:.1f} s, "
        f"{used / 2**30:.1f} GiB of HBM, {n_streamed} round trees streamed")
    for w in range(args.warmup):
        b.solve()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.solve()
        torch.cuda.synchronize()
        log(f"[bench] step {k + 1}/{args.steps} done ({time.perf_counter() - t0:.1f} s)")
    el = time.perf_counter() - t0
    ex = [float(((x[0] - x[1]) / 2).max().item()) for x in b.exploitability()[:2]]
    b.free()
    out = {"metric": METRIC, "value": edges * iters * args.steps / el, "unit": "node-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"paper scale: full games of {args.deals} seeded deals (seeds 1-"
                                  f"{args.deals}) solved as one batch, {nodes} FGT nodes, {iters} DCFR "
                                  f"iterations per round; round trees of at least "
                                  f"{args.stream_min_nodes} nodes ({n_streamed} of "
                                  f"{args.deals * 6}) on the streaming sweeps, the rest in one "
                                  f"persistent launch per round",
                      "state": args.state, "nodes": nodes, "nodes_per_deal": per_deal,
                      "hbm_bytes_in_use": used,
                      "build_seconds": build_s, "exploitability_points_first_deals": ex}}
    print(json.dumps(out), flush=True)


def bench_warm(args):
    """Learned warm start: train the MLP on DCFR solutions of --train-deals
    seeded two-round deals (seeds 10000..), then on --test-deals held-out
    deals (seeds 20000..) measure the seconds (and iterations) DCFR needs to
    reach exploitability <= 1e-3 at the round-5 root, plain vs warm-started
    (inference included, exploitability checks excluded, plain DCFR as the
    fallback).  Also reports the MFMA throughput of the network's GEMMs, and
    plain DCFR's exploitability after 1..16 iterations on the first 32
    held-out deals (what the network's starting profile is worth in
    iterations)."""
    import torch
    import paper_2508_06559_amd as pa
    from paper_2508_06559_amd import learn
    import synth

    t0 = time.perf_counter()
    train = [playout_problem(s, 4) for s in range(10000, 10000 + args.train_deals)]
    units = learn.training_units(train, 1000)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    rows = sum(u.n_rows for u in units)
    log(f"[bench] training data: {len(units)} units, {rows} rows, {data_s:.1f} s")
    model = learn.WarmStartMLP(0)
    # MFMA throughput: one epoch of training steps timed with events
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    hist = learn.train(model, units, 1, seed=99, log=log)
    b.record()
    b.synchronize()
    train_ms = a.elapsed_time(b)
    per_row = MLP_FWD_FLOP
    train_tflops = MLP_TRAIN_FLOP * rows / (train_ms * 1e-3) / 1e12
    hist += learn.train(model, units, args.epochs - 1, seed=0, log=log)
    big = torch.zeros((1 << 20, learn.N_IN), dtype=torch.int16, device="cuda")
    Yb = torch.empty((big.shape[0], 2), dtype=torch.float32, device="cuda")
    pa.mlp_infer(model.infer_weights(), big, big.shape[0], Yb)
    a.record()
    for _ in range(5):
        pa.mlp_infer(model.infer_weights(), big, big.shape[0], Yb)
    b.record()
    b.synchronize()
    inf_tflops = 5 * per_row * big.shape[0] / (a.elapsed_time(b) * 1e-3) / 1e12
    a.record()
    for _ in range(5):
        model.forward(big, big.shape[0])
    b.record()
    b.synchronize()
    fwd_tflops = 5 * per_row * big.shape[0] / (a.elapsed_time(b) * 1e-3) / 1e12
    del big, Yb
    grid = tuple(range(6, 64, 2)) + (64, 80, 96, 128, 192, 256)
    test = [playout_problem(s, 4) for s in range(20000, 20000 + args.test_deals)]
    levels = [int(x) for x in args.warm_levels.split(",")]
    res = {"plain": [], "warm": []}
    res.update({f"warm_levels_{L}": [] for L in levels[1:]})
    ex0 = {"uniform": [], "network": []}
    # plain DCFR's exploitability after a few iterations: how many iterations
    # the network's starting profile is worth
    early = (1, 2, 3, 4, 6, 8, 10, 12, 16)
    ex_early = {T: [] for T in early}
    for k, (deck, roots) in enumerate(test):
        res["plain"].append(learn.seconds_to_target(deck, 4, roots, 1e-3, grid, None))
        res["warm"].append(learn.seconds_to_target(deck, 4, roots, 1e-3, grid, model,
                                                   learn.WarmParams(max_level=levels[0])))
        for L in levels[1:]:
            res[f"warm_levels_{L}"].append(learn.seconds_to_target(
                deck, 4, roots, 1e-3, grid, model, learn.WarmParams(max_level=L)))
        if k < 32:
            ex0["uniform"].append(learn.initial_profile_exploitability(deck, roots, None))
            ex0["network"].append(learn.initial_profile_exploitability(deck, roots, model))
            for T in early:
                sv = learn.solve_subgame(deck, 4, roots, T)
                ex_early[T].append(learn.exploitability(sv))
                sv.free()
        if k % 32 == 31:
            log(f"[bench] evaluated {k + 1}/{len(test)} held-out deals")

    def summ(rs):
        sec = np.array([r["seconds"] for r in rs if r["seconds"] is not None])
        sol = np.array([r["solve_seconds"] for r in rs if r["solve_seconds"] is not None])
        it = np.array([r["iters"] for r in rs if r["iters"] is not None])
        return {"median_seconds": float(np.median(sec)), "p25_seconds": float(np.percentile(sec, 25)),
                "p75_seconds": float(np.percentile(sec, 75)), "median_iters": float(np.median(it)),
                "mean_iters": float(np.mean(it)), "reached": int(len(sec)),
                "fallbacks": int(sum(r["fallback"] for r in rs)),
                "median_solve_seconds_without_trees": float(np.median(sol))}

    def paired(rs):
        # per-deal warm / plain seconds (same deal, same grid), with and
        # without building the trees (common to both)
        r = np.array([w["seconds"] / p["seconds"] for w, p in zip(rs, res["plain"])
                      if w["seconds"] is not None and p["seconds"] is not None])
        q = np.array([w["solve_seconds"] / p["solve_seconds"] for w, p in zip(rs, res["plain"])
                      if w["solve_seconds"] is not None and p["solve_seconds"] is not None])
        return {"median_ratio_warm_over_plain": float(np.median(r)),
                "fraction_of_deals_warm_faster": float(np.mean(r < 1.0)),
                "median_ratio_without_trees": float(np.median(q)),
                "fraction_faster_without_trees": float(np.mean(q < 1.0))}

    sp, sw = summ(res["plain"]), summ(res["warm"])
    sw.update(paired(res["warm"]))
    full = bench_warm_full_games(args, levels[0], log) if args.full_test_games > 0 else None
    out = {
        "metric": METRIC, "value": sw["median_seconds"], "unit": "s to exploitability 1e-3 (warm start)",
        "n_gpus": 1, "steps": len(test), "warmup": 0, "ms_per_step": sw["median_seconds"] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"learned warm start: MLP 192-256-256-2 trained on DCFR solutions of "
                               f"{len(train)} seeded two-round deals ({rows} rows, {args.epochs} epochs); "
                               f"seconds to exploitability 1e-3 on {len(test)} held-out deals, "
                               f"iteration grid {list(grid)}",
                   "plain": sp, "warm": sw, "warm_levels": levels[0],
                   "other_warm_levels": {k: {**summ(v), **paired(v)} for k, v in res.items()
                                         if k.startswith("warm_levels_")},
                   "speedup_median_seconds": sp["median_seconds"] / sw["median_seconds"],
                   "initial_profile_exploitability_median": {k: float(np.median(v)) for k, v in ex0.items()},
                   "plain_exploitability_after_iterations": {
                       str(T): {"median": float(np.median(v)), "p25": float(np.percentile(v, 25)),
                                "p75": float(np.percentile(v, 75))} for T, v in ex_early.items()},
                   "final_train_loss": hist[-1], "data_seconds": data_s,
                   "full_games": full},
        "roofline": {"bound": "mfma", "kernel": "k_mlp_infer (fused 3-layer inference, BF16 MFMA "
                                                "16x16x32, FP32 accumulate), 2^20 rows",
                     "achieved": inf_tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": inf_tflops / 2500.0, "traffic": None,
                     "forward_pass_TFLOPs": fwd_tflops,
                     # one epoch over units of ~8,000 rows: launch-bound, not
                     # the GEMM rate (the mlp workload times 2^18-row steps)
                     "training_epoch_TFLOPs": train_tflops},
    }
    print(json.dumps(out), flush=True)


def bench_warm_full_games(args, max_level, log):
    """The warm start on whole games: a network trained on DCFR solutions
    (--full-iters iterations per round) of --full-train-games seeded full
    games (seeds 10000..), then on --full-test-games held-out full games
    (seeds 20000..) the iterations and seconds DCFR needs to reach
    exploitability <= 1e-3 at the initial deal, plain vs warm-started (levels
    1..max_level of every round), trees built once per deal outside the
    timed solves.  Also plain DCFR's exploitability after its first
    iterations and that of the network's starting profile."""
    import torch
    from paper_2508_06559_amd import learn
    from paper_2508_06559_amd.solver import SubgameSolver
    import synth

    t0 = time.perf_counter()
    train = [synth.full_game_root(s_) for s_ in range(10000, 10000 + args.full_train_games)]
    units = learn.training_units(train, args.full_iters, start_round=0)
    rows = sum(u.n_rows for u in units)
    log(f"[bench] full-game training data: {len(units)} units, {rows} rows, "
        f"{time.perf_counter() - t0:.1f} s")
    model = learn.WarmStartMLP(1)
    hist = learn.train(model, units, args.epochs, seed=1, log=log)
    del units
    grid = tuple(range(8, 64, 2)) + (64, 72, 80, 96, 112, 128, 160, 192, 256)
    early = (1, 2, 4, 8, 16, 32)
    warm = learn.WarmParams(max_level=max_level)
    res = {"plain": [], "warm": []}
    ex_early = {T: [] for T in early}
    ex0 = {"uniform": [], "network": []}
    build = []
    nodes = []
    for k, s_ in enumerate(range(20000, 20000 + args.full_test_games)):
        deck, roots = synth.full_game_root(s_)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        sv = SubgameSolver(deck, 0, roots, keep_gt=True)
        torch.cuda.synchronize()
        build.append(time.perf_counter() - tb)
        nodes.append(sum(sum(n) for n in sv.sizes()))
        res["plain"].append(learn.iterations_to_target(sv, 1e-3, grid, None))
        res["warm"].append(learn.iterations_to_target(sv, 1e-3, grid, model, warm))
        for T in early:
            learn.solve_built(sv, T)
            ex_early[T].append(learn.exploitability(sv))
        sv.free()
        ex0["uniform"].append(learn.initial_profile_exploitability(deck, roots, None, start_round=0))
        ex0["network"].append(learn.initial_profile_exploitability(deck, roots, model, start_round=0))
        log(f"[bench] full game {s_}: {nodes[-1]:.3g} nodes, plain {res['plain'][-1]['iters']} "
            f"iterations {res['plain'][-1]['solve_seconds']:.3f} s, warm {res['warm'][-1]['iters']} "
            f"iterations {res['warm'][-1]['solve_seconds']:.3f} s")

    def q(v):
        v = np.asarray(v, dtype=float)
        return {"median": float(np.median(v)), "p25": float(np.percentile(v, 25)),
                "p75": float(np.percentile(v, 75))}

    ok = [(w, p_) for w, p_ in zip(res["warm"], res["plain"])
          if w["iters"] is not None and p_["iters"] is not None]
    ratio = [w["solve_seconds"] / p_["solve_seconds"] for w, p_ in ok]
    return {"workload": f"{args.full_train_games} seeded full games for training ({rows} rows, "
                        f"{args.full_iters} DCFR iterations per round), {args.full_test_games} "
                        f"held-out full games, iteration grid {list(grid)}, warm levels 1..{max_level}",
            "nodes": q(nodes), "tree_build_seconds": q(build),
            "plain_iters": q([p_["iters"] for _, p_ in ok]),
            "warm_iters": q([w["iters"] for w, _ in ok]),
            "plain_solve_seconds": q([p_["solve_seconds"] for _, p_ in ok]),
            "warm_solve_seconds": q([w["solve_seconds"] for w, _ in ok]),
            "per_deal_ratio_warm_over_plain": q(ratio),
            "fraction_of_deals_warm_faster": float(np.mean(np.array(ratio) < 1.0)),
            "warm_fallbacks": int(sum(w["fallback"] for w in res["warm"])),
            "reached": len(ok),
            "initial_profile_exploitability": {k_: q(v) for k_, v in ex0.items()},
            "plain_exploitability_after_iterations": {str(T): q(v) for T, v in ex_early.items()},
            "final_train_loss": hist[-1]}


def bench_selfplay(args):
    """Self-play on the solved full game of seeded deal --full-seed: after an
    untimed build and solve (--iters per round, default 1000), one step
    plays --games games in each of three matchups (average strategy vs
    average strategy, average strategy vs uniform random, uniform random vs
    average strategy), one pasur_selfplay launch per matchup.  Reports
    games/s, each matchup's fair value (fraction of games Alex wins) and
    mean margin, and the exact expected margins of the played profiles."""
    import torch
    import paper_2508_06559_amd as pa
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    iters = 1000 if args.iters == 2000 else args.iters
    deck, roots = synth.full_game_root(args.full_seed)
    stream = torch.cuda.Stream()
    s = pa.SubgameSolver(deck, 0, roots, dtype=dtype, stream=stream)
    s.solve(iters, pa.paper_params(block=args.block))
    torch.cuda.synchronize()
    v_ss = float(s.exploitability()[2][0].item())
    S, U = pa.PLAY_SIGMA_BAR, pa.PLAY_UNIFORM
    matchups = {"avg_vs_avg": (S, S), "avg_vs_uniform": (S, U), "uniform_vs_avg": (U, S)}
    n = args.games
    margin = {k: torch.empty(n, dtype=torch.int32, device="cuda") for k in matchups}
    fgts = [rr.fgt for rr in s.rounds]
    sbars = [rr.state.sigma_bar for rr in s.rounds]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(matchups))]
    kernel_ms = []

    def play(k, timed):
        for i, (name, (p_a, p_b)) in enumerate(matchups.items()):
            ev[2 * i].record(stream)
            pa.selfplay(fgts, sbars, dtype, 0, n, 1000 * k + i, p_a, p_b, margin[name], stream)
            ev[2 * i + 1].record(stream)
        torch.cuda.synchronize()
        if timed:
            kernel_ms.extend(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(len(matchups)))
        log(f"[bench] self-play step {k + 1} done")

    for k in range(args.warmup):
        play(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        play(k, True)
    el = time.perf_counter() - t0
    stats = {}
    for name in matchups:
        m = margin[name].double()
        stats[name] = {"fair_value": float((m > 0).double().mean().item()),
                       "mean_margin": float(m.mean().item()),
                       "stderr": float(m.std().item() / np.sqrt(n))}
    stats["avg_vs_avg"]["exact_expected_margin"] = v_ss
    rounds = len(fgts)
    # algorithmic bytes per game: the path's index reads (a child-begin pair
    # per level, a leaf score and a link per round) and the margin written;
    # average-strategy reads come on top and depend on the policy
    per_game = rounds * (8 * 8 + 4) + (rounds - 1) * 4 + 4
    dt = float(np.mean(kernel_ms)) * 1e-3
    achieved = per_game * n / dt / 1e9
    sizes = s.sizes()
    s.free()
    out = {"metric": "self-play games/s at 1 GPU", "value": 3 * n * args.steps / el,
           "unit": "games/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"self-play on the solved full game of seeded deal {args.full_seed} "
                                  f"({sum(sum(x) for x in sizes)} nodes, {iters} DCFR iterations per "
                                  f"round): {n} games per matchup, 3 matchups per step",
                      "state": args.state, "matchups": stats},
           "roofline": {"bound": "hbm", "kernel": "k_selfplay (one thread per game, dependent "
                                                  "child-begin gathers down one path)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "bytes_per_game": per_game, "kernel_ms_per_launch": dt * 1e3,
                        "dependent_gathers_per_game": rounds * 8}}
    print(json.dumps(out), flush=True)


def es_bytes(stats, T):
    """Algorithmic bytes of the frontier schedule's work counters: per
    reached node of the updated player its frontier entry (read down and
    up), child-begin pair (down and up), pick (written, read) and value
    written; per child of such a node a frontier append and sigma, value,
    regret (read and written) and new sigma; per reached opponent node its
    frontier entry (twice), child-begin pair, pick (twice), one frontier
    append and the kept child's value read and its own written; per child of
    an opponent node sigma read and the average sum read and written."""
    n_t, e_t, n_o, e_o = (float(x) for x in stats)
    return n_t * (32 + T) + e_t * (4 + 5 * T) + n_o * (28 + 2 * T) + e_o * 3 * T


def bench_es(args):
    """External-sampling CFR on the full game of seeded deal --full-seed:
    each step solves all six rounds backward with --iters external-sampling
    iterations per round (default 1000; frontier schedule, one launch per
    round), average strategies and values of the average strategies passed
    back, then the composed exploitability.  Reports node visits/s (reached
    nodes of both passes), the frontier kernel's roofline from its exact work
    counters, and full-width DCFR on the same game at a few iteration counts
    (seconds and exploitability) for comparison."""
    import torch
    import paper_2508_06559_amd as pa
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    iters = 1000 if args.iters == 2000 else args.iters
    deck, roots = synth.full_game_root(args.full_seed)
    stream = torch.cuda.Stream()
    s = pa.SubgameSolver(deck, 0, roots, dtype=dtype, stream=stream)
    sizes = s.sizes()
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")

    def step(k, timed):
        V = None
        evs = []
        for rr in reversed(s.rounds):
            st = rr.state if rr.state is not None else pa.CfrState(rr.fgt, dtype)
            rr.state = st
            pa.leaf_utilities(rr.fgt, V, dtype, st.u[8], stream)
            pa.cfr_init(st, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pa.es_iterate(st, iters, 1 + k, stats=stats if timed else None, stream=stream)
            e1.record(stream)
            evs.append((e0, e1))
            pa.average_strategy(st, stream)
            rr.V = torch.empty(rr.fgt.n[0], dtype=torch.float64, device="cuda")
            pa.round_values(st, pa.V_SIGMA_BAR, rr.V, stream)
            V = rr.V
        torch.cuda.synchronize()
        log(f"[bench] es step {k + 1} done")
        return sum(a.elapsed_time(b) for a, b in evs)

    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms = sum(step(args.warmup + k, True) for k in range(args.steps))
    el = time.perf_counter() - t0
    bra, brb, v = s.exploitability()
    ex = float(((bra - brb) / 2).max().item())
    st_np = stats.cpu().numpy()
    visits = float(st_np[0] + st_np[2])
    nbytes = es_bytes(st_np, T)
    achieved = nbytes / (kern_ms * 1e-3) / 1e9
    dcfr = []
    for it in (10, 30, 100):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.solve(it)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        a, b, _ = s.exploitability()
        dcfr.append({"iterations": it, "seconds": dt, "exploitability": float(((a - b) / 2).max().item())})
        log(f"[bench] dcfr {it} iterations: {dt:.3f} s")
    s.free()
    per_iter = visits / (args.steps * iters)
    out = {"metric": "external-sampling CFR node visits/s at 1 GPU", "value": visits / el,
           "unit": "node visits/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"external-sampling CFR, full game of seeded deal {args.full_seed} "
                                  f"({sum(sum(n) for n in sizes)} nodes), {iters} iterations per round",
                      "state": args.state, "visits_per_iteration": per_iter,
                      "fraction_of_tree_per_iteration": per_iter / sum(sum(n) for n in sizes),
                      "exploitability_points": ex, "game_value": float(v[0].item()),
                      "dcfr_same_game": dcfr},
           "roofline": {"bound": "hbm", "kernel": "k_es_frontier (persistent, one wave per run of roots, "
                                                  "per-level frontiers of reached nodes)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel_ms_per_step": kern_ms / args.steps, "launches_per_step": len(sizes),
                        "work_counters": [int(x) for x in st_np]}}
    print(json.dumps(out), flush=True)


def infoset_bytes(level, rows):
    """Algorithmic bytes of pasur_infoset_rows (int8 rows) for `rows` nodes
    of `level`: the row written (58) and, read, the node's GT index and
    score id (8), pool and hands (9), per ancestor action its played card,
    collected mask and parent (13 each), the root's pool (8) and the score
    entry (4)."""
    return rows * (58 + 8 + 9 + 13 * level + 8 + 4)


def bench_infoset(args):
    """Infoset rows (section "Infoset Tensors") for every FGT node of the
    full game of seeded deal --full-seed, level by level (one launch each,
    into a reused buffer), timed with HIP events; then the paper's strategy
    model design against the warm-start network: a network trained on
    infoset rows, one on the edge features, and a gradient-boosted tree model
    on infoset rows (the paper's XGBoost analogue, CPU), all on DCFR
    solutions of --model-train-deals two-round deals, evaluated on
    --model-test-deals held-out deals (RMSE of 100 x sigma on sampled
    decisions, exploitability of the predicted starting profile)."""
    import torch
    import paper_2508_06559_amd as pa
    from paper_2508_06559_amd import learn
    import synth

    deck, roots = synth.full_game_root(args.full_seed)
    stream = torch.cuda.Stream()
    s = pa.SubgameSolver(deck, 0, roots, keep_gt=True, stream=stream)
    sizes = s.sizes()
    nmax = max(max(n[1:]) for n in sizes)
    out = torch.empty((nmax, pa.INFOSET_WIDTH), dtype=torch.int8, device="cuda")
    rows_total = sum(sum(n[1:]) for n in sizes)
    nbytes = sum(infoset_bytes(l, n[l]) for n in sizes for l in range(1, 9))

    def step(k):
        evs = []
        for rr in s.rounds:
            for l in range(1, 9):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                pa.infoset_rows(rr.gt, rr.fgt, l, None, rr.fgt.n[l], out, stream=stream)
                e1.record(stream)
                evs.append((e0, e1))
        torch.cuda.synchronize()
        log(f"[bench] infoset step {k + 1} done")
        return sum(a.elapsed_time(b) for a, b in evs)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms = sum(step(args.warmup + k) for k in range(args.steps))
    el = time.perf_counter() - t0
    s.free()
    achieved = nbytes * args.steps / (kern_ms * 1e-3) / 1e9

    res = {"metric": "infoset rows/s at 1 GPU", "value": rows_total * args.steps / el, "unit": "rows/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
           "data": "synthetic",
           "config": {"workload": f"infoset rows of every node of the full game of seeded deal "
                                  f"{args.full_seed} ({rows_total} rows of 58 bytes, 48 launches per step)"},
           "roofline": {"bound": "hbm", "kernel": "k_infoset (one thread per row, history from up to "
                                                  "eight ancestors)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel_ms_per_step": kern_ms / args.steps,
                        "algorithmic_bytes_per_step": nbytes}}
    if args.no_models:
        print(json.dumps(res), flush=True)
        return

    # strategy models
    ntr, nte = args.model_train_deals, args.model_test_deals
    train = [playout_problem(s_, 4) for s_ in range(30000, 30000 + ntr)]
    test = [playout_problem(s_, 4) for s_ in range(40000, 40000 + nte)]
    tm = time.perf_counter()
    models = {}
    for feats in ("edge", "infoset"):
        units = learn.training_units(train, 500, 300, features=feats)
        m = learn.WarmStartMLP(0)
        hist = learn.train(m, units, args.epochs)
        models[feats] = (m, hist[-1])
        log(f"[bench] network on {feats} features trained: loss {hist[-1]}")
    rows, tgt, _ = learn.infoset_dataset(train, 500, 150)
    tree = learn.fit_tree_model(rows, tgt)
    log(f"[bench] tree model fitted on {len(rows)} rows")
    t_models = time.perf_counter() - tm

    def net_rmse(m, feats):
        errs = []
        for u in learn.training_units(test, 500, 300, seed0=7, features=feats):
            Y = m.forward(u.X, u.n_rows)[:, 0].float().cpu().numpy().astype(np.float64)
            seg = u.seg.cpu().numpy()
            sig = np.empty_like(Y)
            for p in range(u.n_par):
                z = Y[seg[p]:seg[p + 1]]
                e = np.exp(z - z.max())
                sig[seg[p]:seg[p + 1]] = e / e.sum()
            errs.append(100.0 * sig - 100.0 * u.tsig.cpu().numpy())
        e = np.concatenate(errs)
        return float(np.sqrt(np.mean(e * e)))

    trows, ttgt, tgrp = learn.infoset_dataset(test, 500, 300, seed0=7)
    p = np.maximum(tree.predict(trows.astype(np.float32)), 0.0)
    tot = np.bincount(tgrp, weights=p)
    cnt = np.bincount(tgrp)
    pos = tot[tgrp] > 0
    sig = 100.0 * np.where(pos, p / np.where(pos, tot[tgrp], 1.0), 1.0 / cnt[tgrp])
    tree_rmse = float(np.sqrt(np.mean((sig - ttgt) ** 2)))
    ex = {"uniform": [], "network_edge": [], "network_infoset": [], "tree_infoset": []}
    for deck_, roots_ in test:
        ex["uniform"].append(learn.initial_profile_exploitability(deck_, roots_, None))
        ex["network_edge"].append(learn.initial_profile_exploitability(deck_, roots_, models["edge"][0]))
        ex["network_infoset"].append(learn.initial_profile_exploitability(deck_, roots_, models["infoset"][0],
                                                                          "infoset"))
        ex["tree_infoset"].append(learn.tree_profile_exploitability(deck_, roots_, tree))
    cmp = {"rmse_100sigma_heldout": {"network_edge": net_rmse(models["edge"][0], "edge"),
                                     "network_infoset": net_rmse(models["infoset"][0], "infoset"),
                                     "tree_infoset": tree_rmse},
           "initial_exploitability_median": {k: float(np.median(v)) for k, v in ex.items()},
           "final_train_loss": {k: v[1] for k, v in models.items()},
           "tree_rows": int(len(rows)), "train_deals": ntr, "test_deals": nte, "epochs": args.epochs,
           "seconds": t_models}
    res["config"]["models"] = cmp
    print(json.dumps(res), flush=True)


MLP_FWD_FLOP = 2 * (192 * 256 + 256 * 256 + 256 * 2)          # per row
# per row of a training step: forward, then the weight gradients of all
# three layers and the input gradients of layers 2 and 3 (layer 1 needs none)
MLP_TRAIN_FLOP = MLP_FWD_FLOP + 2 * 192 * 256 + 2 * (2 * 256 * 256) + 2 * (2 * 256 * 2)


def bench_mlp(args):
    """The warm-start network's MFMA kernels on their own, on synthetic
    feature rows (card bits set with probability 1/4, score and level
    columns as the feature layout fills them): --steps timed calls of the
    fused inference (k_mlp_infer) over 2^20 rows, and --steps training steps
    (forward: the fused kernel, which also writes H1 and H2; loss, backward, Adam) over 2^18 rows
    in groups of four siblings, each timed with HIP events on the launch stream."""
    import torch
    from paper_2508_06559_amd import learn
    import paper_2508_06559_amd as pa

    rng = np.random.default_rng(5)

    def rows(n):
        x = np.zeros((n, learn.N_IN), np.float32)
        x[:, :156] = rng.random((n, 156)) < 0.25
        x[:, 156:167] = rng.random((n, 11)) * 2 - 1
        x[np.arange(n), 167 + rng.integers(1, 9, n)] = 1.0
        return torch.from_numpy(x).cuda().bfloat16().view(torch.int16)

    model = learn.WarmStartMLP(0)
    n_inf, n_tr = 1 << 20, 1 << 18
    X = rows(n_inf)
    Y = torch.empty((n_inf, 2), dtype=torch.float32, device="cuda")
    w = model.infer_weights()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(args.warmup):
        pa.mlp_infer(w, X, n_inf, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(args.steps):
        pa.mlp_infer(w, X, n_inf, Y)
    ev[1].record()
    ev[1].synchronize()
    el = time.perf_counter() - t0
    inf_ms = ev[0].elapsed_time(ev[1]) / args.steps
    inf_tf = MLP_FWD_FLOP * n_inf / (inf_ms * 1e-3) / 1e12

    Xt = rows(n_tr)
    seg = torch.arange(0, n_tr + 1, 4, dtype=torch.int32, device="cuda")
    tsig = torch.full((n_tr,), 0.25, dtype=torch.float32, device="cuda")
    tval = torch.from_numpy(rng.normal(0, 3, n_tr).astype(np.float32)).cuda()
    unit = learn.Unit(Xt, seg, tsig, tval, n_tr // 4, n_tr)
    for _ in range(args.warmup):
        model.train_unit(unit, 1e-3)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        model.train_unit(unit, 1e-3)
    ev[1].record()
    ev[1].synchronize()
    tr_ms = ev[0].elapsed_time(ev[1]) / args.steps
    tr_tf = MLP_TRAIN_FLOP * n_tr / (tr_ms * 1e-3) / 1e12
    out = {"metric": "warm-start MLP inference TFLOP/s at 1 GPU", "value": inf_tf, "unit": "TFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": f"192-256-256-2 MLP: fused inference over {n_inf} rows per call; "
                                  f"training steps over {n_tr} rows",
                      "inference_ms_per_call": inf_ms, "training_ms_per_step": tr_ms,
                      "training_TFLOPs": tr_tf, "flop_per_row_inference": MLP_FWD_FLOP,
                      "flop_per_row_training": MLP_TRAIN_FLOP},
           "roofline": {"bound": "mfma", "kernel": "k_mlp_infer (three layers fused, BF16 MFMA 16x16x32, "
                                                   "FP32 accumulate)",
                        "achieved": inf_tf, "peak": 2500.0, "unit": "TFLOP/s", "frac": inf_tf / 2500.0,
                        "traffic": None}}
    print(json.dumps(out), flush=True)


def bench_variants(args):
    """Convergence of the three CFR update rules built into the sweep kernel
    (DCFR with the paper's constants and regret floor; CFR+ with R+ and
    linearly weighted averages; vanilla CFR), on the two-round subgame of
    seeded deal --seed: for each rule and each iteration count of a grid, a
    whole solve (trees, iterations, values) timed end to end, then the
    composed exploitability of its average strategies.  The roofline object
    is the segment kernel's, measured live on the 2000-iteration CFR+ solve
    (the generic, non-DCFR instance of the kernel)."""
    import torch
    import paper_2508_06559_amd as pa
    import synth

    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    deck, roots = playout_problem(args.seed, 4)
    rules = {"dcfr": pa.paper_params(),
             "cfr_plus": pa.CfrParams(pa.CFR_PLUS, pa.RM_POSITIVE, 0.0, 0.0, 0.0, 0.0, pa.SCHED_ROOT, 0, 0),
             "vanilla": pa.CfrParams(pa.CFR_VANILLA, pa.RM_POSITIVE, 0.0, 0.0, 0.0, 0.0, pa.SCHED_ROOT, 0, 0)}
    grid = (5, 10, 20, 30, 50, 100, 200, 500, 1000, 2000)
    res = {}
    for name, p in rules.items():
        rows = []
        for it in grid:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
            s.solve(it, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            bra, brb, _ = s.exploitability()
            ex = float(((bra - brb) / 2).max().item())
            s.free()
            rows.append({"iterations": it, "seconds": dt, "exploitability": ex})
        hit = next((r for r in rows if r["exploitability"] <= 1e-3), None)
        res[name] = {"grid": rows, "iterations_to_1e-3": hit["iterations"] if hit else None,
                     "seconds_to_1e-3": hit["seconds"] if hit else None}
        log(f"[bench] {name}: to 1e-3 in {res[name]['iterations_to_1e-3']} iterations")
    # live roofline of the generic kernel instance (CFR+, 2000 iterations)
    s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
    pa.profile_enable(True)
    s.solve(2000, rules["cfr_plus"])
    torch.cuda.synchronize()
    kern, lev, ms, work = pa.profile_read()
    pa.profile_enable(False)
    s.free()
    db = sum(launch_bytes(int(kern[i]), int(lev[i]), work[i], T) for i in range(len(kern)))
    dt = sum(float(x) for x in ms) * 1e-3
    dcfr = res["dcfr"]
    out = {"metric": "seconds to exploitability 1e-3 by CFR update rule at 1 GPU",
           "value": dcfr["seconds_to_1e-3"], "unit": "s (DCFR; other rules in config)",
           "n_gpus": 1, "steps": len(grid) * len(rules), "warmup": 0,
           "ms_per_step": (dcfr["seconds_to_1e-3"] or 0.0) * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"last two rounds of seeded deal {args.seed}, each CFR update rule over "
                                  f"the iteration grid {list(grid)}; seconds include building the trees",
                      "state": args.state, "rules": res},
           "roofline": {"bound": "hbm", "kernel": "k_cfr_seg, generic variant instance (CFR+), "
                                                  f"{'float' if T == 4 else 'double'} state",
                        "achieved": db / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": db / dt / 1e9 / HBM_PEAK_GBS, "traffic": None,
                        "avg_launch_us": dt / len(kern) * 1e6, "launches": len(kern)}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--state", choices=["f32", "f64"], default="f32")
    ap.add_argument("--sched", choices=["auto", "root", "level", "root-global", "stream"],
                    default="auto")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["two-round", "batched", "warm-start", "full-game",
                                           "paper-scale", "selfplay", "es", "infoset", "mlp", "variants", "copy",
                                           "copy-rate"],
                    default="full-game",
                    help="full-game: the headline configuration (all six rounds of one deal); "
                         "two-round: rounds 5-6 of one deal; batched: 64 deals, rounds 4-6; "
                         "warm-start: learned warm start vs plain DCFR")
    ap.add_argument("--train-deals", type=int, default=512)
    ap.add_argument("--test-deals", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--stream-min-nodes", type=int, default=9_000_000,
                    help="paper-scale: round trees this large run the streaming sweeps "
                         "(0: every round in the batched plan)")
    ap.add_argument("--full-train-games", type=int, default=48,
                    help="warm-start: seeded full games the full-game network trains on")
    ap.add_argument("--full-test-games", type=int, default=16,
                    help="warm-start: held-out full games (0 skips the full-game arm)")
    ap.add_argument("--full-iters", type=int, default=200,
                    help="warm-start: DCFR iterations per round of the full-game training solves")
    ap.add_argument("--deals", type=int, default=32, help="paper-scale: number of full games")
    ap.add_argument("--model-train-deals", type=int, default=64, help="infoset: deals the models learn from")
    ap.add_argument("--model-test-deals", type=int, default=16, help="infoset: held-out deals")
    ap.add_argument("--no-models", action="store_true", help="infoset: rows only, no model comparison")
    ap.add_argument("--games", type=int, default=1 << 24, help="selfplay: games per matchup")
    ap.add_argument("--full-seed", type=int, default=40, help="full-game: the seeded deal")
    ap.add_argument("--warm-levels", default="3,2,4,8",
                    help="warm-start: comma list of max_level values (levels 1..L predicted); the first is reported")
    ap.add_argument("--schedule-json", default=None, help="where the batched autotuner writes its schedule")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver shards by roots across GPUs only "
              "by design, it is not built for several; rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2508_06559_amd as pa
    import synth

    torch.cuda.set_device(0)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "warm-start":
        return bench_warm(args)
    if args.workload == "full-game":
        return bench_full(args)
    if args.workload == "paper-scale":
        return bench_paper_scale(args)
    if args.workload == "selfplay":
        return bench_selfplay(args)
    if args.workload == "es":
        return bench_es(args)
    if args.workload == "infoset":
        return bench_infoset(args)
    if args.workload == "mlp":
        return bench_mlp(args)
    if args.workload == "variants":
        return bench_variants(args)
    if args.workload == "copy":
        # calibration for hardware byte counters: a plain device copy of a
        # known size (256 MiB read + 256 MiB written per launch, 4 launches)
        x = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_per_launch_each_way": 1 << 28, "launches": 4}))
        return
    if args.workload == "copy-rate":
        # the HBM rate a plain device copy reaches (2 GiB each way per launch)
        x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            y.copy_(x)
        b.record()
        b.synchronize()
        s_ = a.elapsed_time(b) * 1e-3 / 20
        print(json.dumps({"workload": "copy-rate", "bytes_per_launch": 2 * x.numel() * 4,
                          "seconds_per_launch": s_, "TB_per_s": 2 * x.numel() * 4 / s_ / 1e12}))
        return
    dtype = pa.PASUR_F32 if args.state == "f32" else pa.PASUR_F64
    T = 4 if args.state == "f32" else 8
    params = pa.paper_params({"root": pa.SCHED_ROOT, "level": pa.SCHED_LEVEL_SYNC,
                              "root-global": pa.SCHED_ROOT_GLOBAL, "stream": pa.SCHED_STREAM,
                              "auto": pa.SCHED_AUTO}[args.sched], args.block)
    deck, roots = playout_problem(args.seed, 4)
    d_roots = pa.roots_to_device(roots)  # resident before timing
    torch.cuda.synchronize()

    def step():
        s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
        s.solve(args.iters, params)
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

    # Dominant kernel: the sweep kernel with the largest share of time.  Its
    # average launch duration is measured live with HIP events on the launch
    # stream over one step's solve (the library's per-launch profiling).
    s = pa.SubgameSolver(deck, 4, roots, dtype=dtype)
    pa.profile_enable(True)
    s.solve(args.iters, params)
    torch.cuda.synchronize()
    kern, lev, ms, work = pa.profile_read()
    pa.profile_enable(False)
    s.free()
    per = {}
    for i in range(len(kern)):
        k = int(kern[i])
        b, t, c = per.get(k, (0.0, 0.0, 0))
        per[k] = (b + launch_bytes(k, int(lev[i]), work[i], T), t + float(ms[i]) * 1e-3, c + 1)
    dom = max(per, key=lambda k: per[k][1])
    db, dt, dc = per[dom]
    achieved = db / dt / 1e9
    all_b = sum(v[0] for v in per.values())
    all_t = sum(v[1] for v in per.values())
    for k, (b, t, c) in sorted(per.items()):
        log(f"[bench] {KERNEL_NAMES[k]}: {c} launches, avg {t / c * 1e6:.1f} us, "
            f"{b / c / 1e6:.3f} MB/launch, {b / t / 1e9:.1f} GB/s")

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
            "workload": f"last two rounds of seeded deal {args.seed} from a seeded legal playout "
                        f"of rounds 1-4: full unfolded trees "
                        f"({nodes} nodes, {edges} edges), {args.iters} DCFR iterations per round, "
                        f"backward round values, composed exploitability",
            "state": args.state,
            "schedule": args.sched,
            "block": args.block,
            "arithmetic": "f64 registers",
            "iters_per_round": args.iters,
            "level_sizes": sizes,
            "exploitability_points": ex,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{KERNEL_NAMES[dom]}, {'float' if T == 4 else 'double'} state",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counted_traffic(args),
            "traffic_GBs": (counted_traffic(args) / (dt / dc) / 1e9
                            if counted_traffic(args) is not None else None),
            "avg_launch_us": dt / dc * 1e6,
            "launches": dc,
            "algorithmic_bytes_per_launch": db / dc,
            "all_sweeps_GBs": all_b / all_t / 1e9,
        },
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        odeck, oroots = oracle_playout_problem(args.seed, 4)
        out["cpu_baseline"] = cpu_baseline(odeck, oroots, args.iters)
        log(f"[bench] cpu baseline done in {out['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
