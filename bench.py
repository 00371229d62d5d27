#!/usr/bin/env python3
"""Benchmark of the compact-fractal automaton step on one MI355X.

Workload (default): Sierpinski triangle F^{3,2} at level r = 16 (n = 65,536,
43,046,721 compact cells), Bernoulli(0.3) initial state from seed 12952,
Game of Life B3/S23.  A timed step is one generation of the compact step
over the whole fractal (one kernel launch).  The same run also times the
bounding-box step over the full 65,536^2 box (the paper's baseline) and the
lambda / nu maps over all 43M indices, checks that the compact and box
results agree, times the 512-instance batched workload against one launch
per instance (and its small instances run in LDS against the per-generation
launches), serves Poisson-arriving requests for p50/p99 latency, and
times the CPU oracle on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
STRATEGY_NAMES = {1: "tiled", 2: "direct", 3: "tiled_wave", 5: "temporal"}
FORM_NAMES = {0: None, 1: "edge_records", 2: "byte_scatter", 3: "temporal"}
COUNTERS = os.path.join(ROOT, "profiles", "compact_step_triangle_r16_counters.txt")
CSRC = os.path.join(ROOT, "paper_2110_12952_amd", "csrc")
# the device code of the step kernels: a counter summary taken on other sources is stale
KERNEL_SOURCES = ("kernels.hip", "device_common.hpp", "params.hpp", "edges.hpp", "edges_inst.hip", "tiled.hpp",
                  "tiled_inst.hip")


def kernel_sources_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def warm_up(torch, run, steps, min_ms):
    """Runs run(steps), then run(chunk) until min_ms of GPU time have passed
    since the start; returns the number of steps run."""
    done = 0
    if steps:
        run(steps)
        done += steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = max(steps, 20)
    while min_ms > 0 and (time.perf_counter() - t0) * 1e3 < min_ms:
        run(chunk)
        torch.cuda.synchronize()
        done += chunk
    return done


def time_events(torch, fn, reps=1):
    """Milliseconds of fn() on the current stream, bracketed by HIP events."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    out = None
    for _ in range(reps):
        out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def measured_traffic(per_launch_alg_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


LARGE_COUNTERS = os.path.join(ROOT, "profiles", "large_steps_carpet_r9_hfractal_r10_counters.txt")
LARGE_ROWS = {"carpet_r9": "carpet r9", "hfractal_r10": "H r10"}


def measured_large_traffic(name):
    """(compact, box) HBM traffic over algorithmic bytes of an HBM-sized
    workload from the committed counter summary, if it was taken on the
    current kernel source; else (None, None)."""
    if name not in LARGE_ROWS or not os.path.exists(LARGE_COUNTERS):
        return None, None
    lines = open(LARGE_COUNTERS).read().splitlines()
    if f"kernel_sources_sha256_16: {kernel_sources_hash()}" not in lines:
        return None, None
    got = {}
    for line in lines:
        for form in ("compact", "box"):
            if line.startswith(f"{LARGE_ROWS[name]} {form} "):
                try:
                    got[form] = float(line.rsplit("|", 1)[1])
                except ValueError:
                    pass
    return got.get("compact"), got.get("box")


def cpu_baseline(W, wl, seconds, one_thread=True):
    from oracle import oracle as O
    fd = wl.fractal
    o = O.Fractal(fd.s, fd.offsets, wl.r)
    st = o.init_compact(wl.seeds[0], wl.p)
    rule = W.rule_mask(wl.rule)
    steps, t = 0, 0.0
    while t < seconds or steps == 0:
        t0 = time.perf_counter()
        st = o.compact_steps(st, rule, 1)
        t += time.perf_counter() - t0
        steps += 1
        log(f"oracle step {steps}: {t:.1f} s")
    out = {"value": o.cells * steps / t, "unit": "cell-updates/s", "cores": O.threads(), "kind": "oracle",
           "sample": f"{steps} generation(s) of the oracle's compact step (lambda, 8 x nu per cell) over "
                     f"the full {o.cells}-cell state, {t:.1f} s"}
    if one_thread:
        # the same step on one host thread: one generation of the full state
        cores = O.threads()
        O.set_threads(1)
        try:
            t0 = time.perf_counter()
            o.compact_steps(st, rule, 1)
            t1 = time.perf_counter() - t0
        finally:
            O.set_threads(cores)
        out["one_thread"] = {"value": o.cells / t1, "unit": "cell-updates/s", "cores": 1,
                             "sample": f"1 generation of the full {o.cells}-cell state, {t1:.1f} s"}
        log(f"oracle on one thread: {o.cells / t1:.3e} cell-updates/s")
    return out


def small_case(torch, N, W, rule):
    """Triangle r = 10 (59,049 cells), 100 generations: one launch per
    generation is launch-bound, so the same 100 launches are also captured
    in a HIP graph and replayed.  Also times the initial-state kernel."""
    wl = W.SMALL_TRIANGLE
    fd = wl.fractal
    g = N.Fractal(fd.s, fd.offsets, wl.r)
    a0 = g.init_compact(wl.seeds[0], wl.p)
    a, b = a0.clone(), torch.empty_like(a0)
    T = wl.steps
    g.step_compact(a, b, 2, rule)
    a.copy_(a0)
    ms_eager, res = time_events(torch, lambda: g.step_compact(a, b, T, rule))
    eager = res.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.step_compact(a, b, 2, rule)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    a.copy_(a0)
    with torch.cuda.graph(graph):
        gres = g.step_compact(a, b, T, rule)
    a.copy_(a0)
    graph.replay()
    a.copy_(a0)
    ms_graph, _ = time_events(torch, graph.replay)
    same = bool(torch.equal(gres, eager))
    # several generations per launch (temporal blocking), automatic plan
    gt = N.Fractal(fd.s, fd.offsets, wl.r)
    gt.configure_temporal(0, 0)
    tinf = gt.info()
    ta, tb = a0.clone(), torch.empty_like(a0)
    gt.step_compact(ta.clone(), tb, 2, rule)
    ms_temp, tres = time_events(torch, lambda: gt.step_compact(ta, tb, T, rule))
    temporal = {"us_per_step": ms_temp / T * 1e3, "tile_level": int(tinf.tile_level),
                "depth": int(tinf.temporal_depth), "launches": -(-T // int(tinf.temporal_depth)),
                "equals_tiled": bool(torch.equal(tres, eager))}
    # the initial-state kernel on the large triangle (1 byte written per cell)
    big = W.LARGE_TRIANGLE
    gb = N.Fractal(big.fractal.s, big.fractal.offsets, big.r)
    st = gb.new_compact()
    gb.init_compact(big.seeds[0], big.p, out=st)
    ms_init, _ = time_events(torch, lambda: gb.init_compact(big.seeds[0], big.p, out=st), 10)
    out = {"cells": g.cells, "steps": T, "eager_us_per_step": ms_eager / T * 1e3,
           "graph_us_per_step": ms_graph / T * 1e3, "graph_equals_eager": same, "temporal": temporal,
           "init_triangle_r16_us": ms_init / 10 * 1e3,
           "init_triangle_r16_gbps": gb.cells / (ms_init / 10 * 1e-3) / 1e9}
    log(f"small triangle r10: eager {out['eager_us_per_step']:.2f} us/step, graph "
        f"{out['graph_us_per_step']:.2f} us/step, same={same}; temporal (m={temporal['tile_level']}, "
        f"h={temporal['depth']}) {temporal['us_per_step']:.2f} us/step, same={temporal['equals_tiled']}; "
        f"init r16 {out['init_triangle_r16_us']:.1f} us")
    return out


def batch_run(torch, N, W, args):
    """The 512-instance batched workload: all instances stepped together, one
    launch per fractal group per generation, against one launch per instance
    per generation."""
    bw = W.BATCH512
    items = bw.items()
    frs = N.shared_descriptors([(it.fractal.s, it.fractal.offsets, it.r) for it in items])
    batch = N.Batch(frs)
    inf = batch.info()
    rule = W.rule_mask(bw.rule)
    a, b = batch.new_arena(), batch.new_arena()

    def init_states(bt):
        for i, (it, f) in enumerate(zip(items, frs)):
            f.init_compact(it.seed, it.p, out=bt.state(a, i))

    init_states(batch)
    tune_s = None
    if not args.no_batch_autotune:
        # tile plans per fractal chosen by timing them on the batch's own
        # instances (the arenas are stepped, then initialised afresh)
        offsets = batch.offsets
        del batch  # rebuilt below from the retuned descriptors
        t0 = time.perf_counter()
        N.batch_autotune(frs, offsets, a, b, steps=args.batch_tune_steps, rule=rule, use_cache=False)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
        batch = N.Batch(frs)
        inf = batch.info()
        log(f"batch autotune: {tune_s:.1f} s")
        init_states(batch)
    init = a.clone()
    Kb = args.batch_steps or bw.steps
    batch.step(a.clone(), b, 2, rule)
    ms, _ = time_events(torch, lambda: batch.step(a, b, Kb, rule))
    ms_step = ms / Kb
    # one launch per instance and generation, from the same initial states
    Ts = args.batch_seq_steps
    sa, sb = init.clone(), torch.empty_like(init)
    va = [batch.state(sa, i) for i in range(len(frs))]
    vb = [batch.state(sb, i) for i in range(len(frs))]

    def sequential():
        for f, x, y in zip(frs, va, vb):
            f.step_compact(x, y, Ts, rule)
    ms_seq, _ = time_events(torch, sequential)
    seq_res = sb if Ts & 1 else sa
    ba = init.clone()
    bres = batch.step(ba, torch.empty_like(ba), Ts, rule)
    same = all(torch.equal(batch.state(bres, i), batch.state(seq_res, i)) for i in range(len(frs)))
    levels = sorted({(it.fractal.name, f.info().tile_level, STRATEGY_NAMES[f.info().strategy],
                      FORM_NAMES[f.info().tiled_form]) for it, f in zip(items, frs)})
    out = {"workload": bw.name, "instances": len(items), "cells": int(inf.cells), "groups": int(inf.groups),
           "autotune_s": tune_s,
           "tiles": int(inf.tiles), "plans": [list(x) for x in levels], "steps": Kb, "ms_per_step": ms_step,
           "cell_updates_per_s": inf.cells * Kb / (ms * 1e-3),
           "alg_gbps": 2 * inf.cells / (ms_step * 1e-3) / 1e9,
           "sequential_ms_per_step": ms_seq / Ts, "sequential_steps": Ts,
           "speedup_vs_sequential": (ms_seq / Ts) / ms_step, "matches_sequential": bool(same)}
    out["roofline_frac"] = out["alg_gbps"] / HBM_PEAK_GBPS
    log(f"batch: {ms_step * 1e3:.1f} us/step, {out['cell_updates_per_s']:.3e} cell-updates/s, "
        f"{out['alg_gbps']:.0f} GB/s; one launch per instance {ms_seq / Ts * 1e3:.1f} us/step; same={same}")
    if not args.no_small_batch:
        out["small_instances"] = small_batch_run(torch, N, items, frs, init, batch, rule, Kb)
    return out


def small_batch_run(torch, N, items, frs, init, big_batch, rule, steps):
    """The batch's small instances (those a work-group's LDS holds) on their
    own: every generation in LDS, one launch for all of them, against the
    per-generation group launches."""
    idx = [i for i, f in enumerate(frs) if 2 * f.cells < 65536]
    sub = [frs[i] for i in idx]
    out = {"instances": len(idx), "cells": int(sum(f.cells for f in sub)), "steps": steps}
    res = {}
    for resident in (True, False):
        bt = N.Batch(sub, resident=resident)
        a, b = bt.new_arena(), bt.new_arena()
        for j, i in enumerate(idx):
            bt.state(a, j).copy_(big_batch.state(init, i))
        a0 = a.clone()
        bt.step(a, b, 2, rule)
        a.copy_(a0)
        ms, _ = time_events(torch, lambda: bt.step(a, b, steps, rule))
        res[resident] = (b if steps & 1 else a).clone()
        key = "lds_resident" if resident else "group_launches"
        out[key] = {"us_per_step": ms / steps * 1e3, "cell_updates_per_s": out["cells"] * steps / (ms * 1e-3),
                    "resident_instances": int(bt.info().resident), "groups": int(bt.info().groups)}
        del bt
    out["same"] = bool(torch.equal(res[True], res[False]))
    out["speedup"] = out["group_launches"]["us_per_step"] / out["lds_resident"]["us_per_step"]
    log(f"batch, {len(idx)} small instances alone: in LDS {out['lds_resident']['us_per_step']:.1f} us/step, "
        f"group launches {out['group_launches']['us_per_step']:.1f} us/step, same={out['same']}")
    return out


def serve_run(torch, W, args):
    """The served workload: Poisson arrivals (2000 per second), each request
    one automaton run on a carpet or H fractal, served from states resident
    in HBM by the request loop; p50/p99 latency from arrival to the result
    being in HBM."""
    from paper_2110_12952_amd.serve import Server
    sw = W.SERVE2000
    reqs = sw.requests(args.serve_seconds)
    srv = Server(8 << 30, rule=W.rule_mask(sw.rule), deadline_s=args.serve_deadline, round_s=0.02,
                 max_gens=64, throughput0=1.5e12, tile_levels={"carpet": 4, "hfractal": 4})
    # warm the descriptor cache and the kernels outside the measured run
    srv.run([type(q)(q.rid, 0.0, q.fractal, q.r, 10, q.p, q.seed) for q in reqs[:64]])
    st = srv.run(reqs, log=log)
    out = {"workload": sw.name, "rate_per_s": sw.rate, "arrival_window_s": args.serve_seconds,
           "deadline_s": args.serve_deadline,
           "offered_cell_updates_per_s": sum(q.cells * q.steps for q in reqs) / args.serve_seconds}
    out.update(st.summary())
    log(f"serve: {out['completed']}/{out['offered']} completed, p50 {out['latency_p50_ms']:.1f} ms, "
        f"p99 {out['latency_p99_ms']:.1f} ms, {out['cell_updates_per_s']:.3e} cell-updates/s")
    del srv
    torch.cuda.empty_cache()
    return out


def large_case(torch, N, W, name, rule, steps, warm_ms=50.0):
    """One of the HBM-sized workloads (carpet r = 9: 134M cells, H r = 10:
    282M cells; their double buffers exceed the 256 MB Infinity Cache): the
    compact step and the box step for `steps` generations each, per-generation
    times, roofline fractions and whether the two results agree."""
    wl = W.WORKLOADS[name]
    fd = wl.fractal
    g = N.Fractal(fd.s, fd.offsets, wl.r)
    # the two states as the halves of one allocation: with separate
    # allocations the step's time depended on where the allocator placed them
    # (carpet r9: 51 us per generation in a fresh process, 59 after the
    # other workloads' allocations)
    span = (g.cells + 4095) // 4096 * 4096
    pair = torch.empty(2 * span, dtype=torch.uint8, device="cuda")
    a, b = pair[:g.cells], pair[span:span + g.cells]
    g.init_compact(wl.seeds[0], wl.p, out=a)
    warm_up(torch, lambda n: g.step_compact(a.clone(), b, n, rule), 2, warm_ms)
    ms, res = time_events(torch, lambda: g.step_compact(a, b, steps, rule))
    alg = 2 * g.cells
    out = {"cells": g.cells, "n": g.n, "steps": steps, "tile_level": g.info().tile_level,
           "ms_per_step": ms / steps, "cell_updates_per_s": g.cells * steps / (ms * 1e-3),
           "alg_gbps": alg / (ms / steps * 1e-3) / 1e9}
    out["roofline_frac"] = out["alg_gbps"] / HBM_PEAK_GBPS
    out["traffic_over_alg"], box_traffic = measured_large_traffic(name)
    res = res.clone()
    del a, b, pair
    box = g.init_bbox(wl.seeds[0], wl.p)
    box2 = torch.empty_like(box)
    g.step_bbox(box.clone(), box2, 2, rule)
    msb, resb = time_events(torch, lambda: g.step_bbox(box, box2, steps, rule))
    out["bbox_ms_per_step"] = msb / steps
    out["bbox_alg_gbps"] = 2 * g.n * g.n / (msb / steps * 1e-3) / 1e9
    out["bbox_roofline_frac"] = out["bbox_alg_gbps"] / HBM_PEAK_GBPS
    out["bbox_traffic_over_alg"] = box_traffic
    out["speedup_vs_bbox"] = msb / ms
    out["compact_equals_bbox"] = bool(torch.equal(g.gather(resb), res))
    log(f"{name}: compact {ms / steps * 1e3:.1f} us/step ({out['roofline_frac']:.3f} of HBM peak), box "
        f"{msb / steps * 1e3:.1f} us/step, same={out['compact_equals_bbox']}")
    del box, box2, resb, res
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-ms", type=float, default=100.0,
                    help="after --warmup steps, keep warming up until this much time has passed")
    ap.add_argument("--workload", default="triangle_r16")
    ap.add_argument("--bbox-steps", type=int, default=None, help="box-step generations (default: --steps)")
    ap.add_argument("--map-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bbox", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=None,
                    help="generations of the 512-instance batch (default: the workload's 500)")
    ap.add_argument("--batch-seq-steps", type=int, default=10,
                    help="generations of the one-launch-per-instance comparison")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="keep the batch's heuristic tile plans instead of timing the candidates")
    ap.add_argument("--batch-tune-steps", type=int, default=10,
                    help="generations each candidate plan of the batch autotuner is timed over")
    ap.add_argument("--no-cpu-one-thread", action="store_true",
                    help="skip the oracle's one-thread figure (one generation, ~10 s)")
    ap.add_argument("--repeats", type=int, default=10,
                    help="extra timed runs of the compact step for median / mean per-generation times")
    ap.add_argument("--no-small-batch", action="store_true",
                    help="skip timing the batch's small instances alone (in LDS and in group launches)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the served workload (the workload's full 60 s); 0 skips it")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="generations of each HBM-sized workload (carpet r9, H r10); 0 skips them")
    ap.add_argument("--serve-deadline", type=float, default=0.5,
                    help="admission: predicted drain time limit, seconds")
    ap.add_argument("--packed", action="store_true",
                    help="also time the bit-packed state (a capacity form: 8x smaller state, slower step)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference for byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_12952_amd import nbbfrac as N
    from paper_2110_12952_amd import workloads as W

    wl = W.WORKLOADS[args.workload]
    fd = wl.fractal
    torch.cuda.set_device(0)
    g = N.Fractal(fd.s, fd.offsets, wl.r)
    info = g.info()
    rule = W.rule_mask(wl.rule)
    K, Wu = args.steps, args.warmup
    log(f"{wl.name}: n={g.n} cells={g.cells} strategy={info.strategy} tile_level={info.tile_level}")

    if args.copy_probe_mib:
        src = torch.zeros(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- compact step -----------------------------------------------------
    a = g.init_compact(wl.seeds[0], wl.p)
    b = torch.empty_like(a)
    init = a.clone()
    # untimed warm-up: the W steps asked for, then more until the GPU has run
    # this step for --warmup-ms (its clocks ramp up over the first ~10 ms of
    # sustained work; warmup_total_steps in the JSON line counts them all)
    warm_steps = warm_up(torch, lambda n: g.step_compact(a.clone(), b, n, rule), Wu, args.warmup_ms)
    ms, res = time_events(torch, lambda: g.step_compact(a, b, K, rule))
    ms_step = ms / K
    value = g.cells * K / (ms * 1e-3)
    alg_bytes = 2 * g.cells  # read + write one byte per cell per generation
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    log(f"compact: {ms_step * 1e3:.2f} us/step, {value:.3e} cell-updates/s, {achieved:.0f} GB/s")
    # repeats: R more timed runs of at least 100 generations each (the
    # per-generation spread; shorter runs would mostly time events and syncs)
    repeats = None
    if args.repeats > 0:
        Kr = max(100, K // args.repeats)
        ra, rb = init.clone(), torch.empty_like(init)  # the timed result above stays intact
        per = []
        for _ in range(args.repeats):
            msr, _ = time_events(torch, lambda: g.step_compact(ra, rb, Kr, rule))
            per.append(msr / Kr * 1e3)
        del ra, rb
        per.sort()
        mid = len(per) // 2
        repeats = {"runs": len(per), "steps_each": Kr,
                   "median_us": per[mid] if len(per) % 2 else 0.5 * (per[mid - 1] + per[mid]),
                   "mean_us": sum(per) / len(per), "min_us": per[0], "max_us": per[-1]}
        log(f"compact, {len(per)} runs of {Kr}: median {repeats['median_us']:.2f} us, "
            f"mean {repeats['mean_us']:.2f} us")

    # ---- the same step in the byte-scatter form (the tile scattered into an
    # LDS box) at the same tile level, for comparison with the edge-record form
    box_form = None
    if info.strategy == N.STRATEGY_TILED and info.tiled_form == 1:
        Kf = max(100, min(K, 200))
        g.configure(N.STRATEGY_TILED_BOX, info.tile_level)
        fa, fb = init.clone(), torch.empty_like(init)
        g.step_compact(fa.clone(), fb, 2, rule)
        msf, resf = time_events(torch, lambda: g.step_compact(fa, fb, Kf, rule))
        g.configure(N.STRATEGY_TILED, info.tile_level)
        refe = g.step_compact(init.clone(), torch.empty_like(init), Kf, rule)
        box_form = {"us_per_step": msf / Kf * 1e3, "steps": Kf,
                    "alg_gbps": alg_bytes / (msf / Kf * 1e-3) / 1e9,
                    "equals_edge_form": bool(torch.equal(resf, refe))}
        log(f"byte-scatter form: {box_form['us_per_step']:.2f} us/step, same: {box_form['equals_edge_form']}")
        del fa, fb, resf, refe

    # ---- the same generations on the bit-packed state (1 bit per cell; a
    # capacity form, slower than the byte step, timed only when asked for) --
    packed = None
    if args.packed and info.strategy != N.STRATEGY_DIRECT:
        Kp = min(K, 200)
        pa = g.pack(init)
        pb = torch.zeros_like(pa)
        g.step_packed(pa.clone(), pb, 2, rule)
        pa2 = pa.clone()
        msp, resp = time_events(torch, lambda: g.step_packed(pa2, pb, Kp, rule))
        refp = g.step_compact(init.clone(), torch.empty_like(init), Kp, rule)
        packed = {"ms_per_step": msp / Kp, "steps": Kp, "bytes": pa.numel(),
                  "cell_updates_per_s": g.cells * Kp / (msp * 1e-3),
                  "alg_gbps": 2 * pa.numel() / (msp / Kp * 1e-3) / 1e9,
                  "equals_byte_step": bool(torch.equal(g.unpack(resp), refp))}
        log(f"packed state: {msp / Kp * 1e3:.1f} us/step over {pa.numel()} B, same as byte step: "
            f"{packed['equals_byte_step']}")
        del pa, pb, pa2, resp, refp

    # ---- box step (baseline) ----------------------------------------------
    bbox = None
    parity = None
    if not args.no_bbox:
        Kb = args.bbox_steps or K
        box = g.init_bbox(wl.seeds[0], wl.p)
        box2 = torch.empty_like(box)
        if Wu:
            g.step_bbox(box.clone(), box2, min(Wu, 5), rule)
        msb, resb = time_events(torch, lambda: g.step_bbox(box, box2, Kb, rule))
        msb_step = msb / Kb
        box_cells = g.n * g.n
        bbox = {"ms_per_step": msb_step, "steps": Kb,
                "cell_updates_per_s": g.cells * Kb / (msb * 1e-3),
                "box_cell_updates_per_s": box_cells * Kb / (msb * 1e-3),
                "alg_gbps": 2 * box_cells / (msb_step * 1e-3) / 1e9}
        bbox["roofline_frac"] = bbox["alg_gbps"] / HBM_PEAK_GBPS
        log(f"bbox: {msb_step * 1e3:.1f} us/step, {bbox['alg_gbps']:.0f} GB/s")
        if Kb == K:
            parity = bool(torch.equal(g.gather(resb), res))
            log(f"compact == gathered box after {K} steps: {parity}")
        # the paper's lambda approach on the same box (threads over fractal cells)
        Kl = min(Kb, 50)
        box = g.init_bbox(wl.seeds[0], wl.p)
        ref = g.step_bbox(box.clone(), box2, Kl, rule).clone()
        msl, resl = time_events(torch, lambda: g.step_lambda(box, box2, Kl, rule))
        bbox["lambda_approach"] = {"ms_per_step": msl / Kl, "steps": Kl,
                                   "cell_updates_per_s": g.cells * Kl / (msl * 1e-3),
                                   "equals_box_step": bool(torch.equal(resl, ref))}
        log(f"lambda approach: {msl / Kl * 1e3:.1f} us/step, same as box step: "
            f"{bbox['lambda_approach']['equals_box_step']}")
        del box, box2, resb, ref, resl
        # the blocked layout (each tile stored as its S x S square)
        if info.strategy != N.STRATEGY_DIRECT:
            blk = g.to_blocked(init)
            blk2 = torch.empty_like(blk)
            refc = g.step_compact(init.clone(), torch.empty_like(init), Kl, rule)
            msk, resk = time_events(torch, lambda: g.step_blocked(blk, blk2, Kl, rule))
            bbox["blocked_layout"] = {"ms_per_step": msk / Kl, "steps": Kl, "bytes": blk.numel(),
                                      "cell_updates_per_s": g.cells * Kl / (msk * 1e-3),
                                      "equals_compact_step": bool(torch.equal(g.from_blocked(resk), refc))}
            log(f"blocked layout: {msk / Kl * 1e3:.1f} us/step over {blk.numel()} B, same as compact: "
                f"{bbox['blocked_layout']['equals_compact_step']}")
            del blk, blk2, refc, resk

    # ---- the small case: launch-bound, eager launches against a HIP graph ------
    small = small_case(torch, N, W, rule)

    # ---- maps ---------------------------------------------------------------
    x = torch.empty(g.cells, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    idx = torch.empty_like(x)
    g.lam(out=(x, y))
    g.nu(x, y, out=idx)
    msl, _ = time_events(torch, lambda: g.lam(out=(x, y)), args.map_reps)
    msn, _ = time_events(torch, lambda: g.nu(x, y, out=idx), args.map_reps)
    maps_ok = bool(torch.equal(idx.to(torch.int64), torch.arange(g.cells, device="cuda")))
    maps = {"lambda_items_per_s": g.cells * args.map_reps / (msl * 1e-3),
            "lambda_gbps": 8 * g.cells * args.map_reps / (msl * 1e-3) / 1e9,
            "nu_items_per_s": g.cells * args.map_reps / (msn * 1e-3),
            "nu_gbps": 12 * g.cells * args.map_reps / (msn * 1e-3) / 1e9,
            "nu_of_lambda_is_identity": maps_ok}
    # The same maps one level per step (the paper's per-thread maps) and the
    # lambda sum on the matrix cores (the paper's tensor-core encoding).
    x2, y2 = torch.empty_like(x), torch.empty_like(y)
    for name, method in (("digits", N.MAP_DIGITS), ("mfma", N.MAP_MFMA)):
        try:
            g.lam(out=(x2, y2), method=method)
        except N.NbbError:
            continue
        ms_m, _ = time_events(torch, lambda: g.lam(out=(x2, y2), method=method), args.map_reps)
        maps[f"lambda_{name}_gbps"] = 8 * g.cells * args.map_reps / (ms_m * 1e-3) / 1e9
        maps[f"lambda_{name}_matches_lut"] = bool(torch.equal(x2, x) and torch.equal(y2, y))
    idx2 = torch.empty_like(idx)
    for name, method in (("digits", N.MAP_DIGITS), ("mfma", N.MAP_MFMA)):
        try:
            g.nu(x, y, out=idx2, method=method)
        except N.NbbError:
            continue
        ms_n, _ = time_events(torch, lambda: g.nu(x, y, out=idx2, method=method), args.map_reps)
        maps[f"nu_{name}_gbps"] = 12 * g.cells * args.map_reps / (ms_n * 1e-3) / 1e9
        maps[f"nu_{name}_matches_lut"] = bool(torch.equal(idx2, idx))
    del x2, y2, idx2
    log("maps: " + ", ".join(f"{k} {v:.0f}" if isinstance(v, float) else f"{k} {v}" for k, v in maps.items()))
    del x, y, idx

    large = None
    if args.large_steps > 0:
        large = {nm: large_case(torch, N, W, nm, W.rule_mask(W.WORKLOADS[nm].rule), args.large_steps)
                 for nm in ("carpet_r9", "hfractal_r10")}

    batch = None if args.no_batch else batch_run(torch, N, W, args)
    serve = serve_run(torch, W, args) if args.serve_seconds > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, wl, args.cpu_seconds, not args.no_cpu_one_thread)
        log(f"oracle: {cpu['value']:.3e} cell-updates/s on {cpu['cores']} threads")

    # the committed counter summary covers the triangle r = 16 workload only
    traffic = measured_traffic(alg_bytes) if wl.name == "triangle_r16" else None
    out = {
        "metric": "compact cell-updates/sec + % HBM roofline vs bbox; batched p50/p99 latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "warmup_total_steps": warm_steps,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.name, "fractal": f"F^{{{fd.k},{fd.s}}} {fd.name}", "r": wl.r, "n": g.n,
                   "cells": g.cells, "p": wl.p, "seed": wl.seeds[0], "rule": wl.rule,
                   "strategy": STRATEGY_NAMES[info.strategy],
                   "tiled_form": FORM_NAMES[info.tiled_form],
                   "tile_level": info.tile_level},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": ("k_step_direct" if info.strategy == N.STRATEGY_DIRECT else
                                "k_step_edges" if info.tiled_form == 1 else "k_step_tiled"),
                     "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "compact_repeats": repeats,
        "bbox": bbox,
        "speedup_vs_bbox": (bbox["ms_per_step"] / ms_step) if bbox else None,
        "compact_equals_bbox": parity,
        "memory_ratio_bbox_over_compact": g.n * g.n / g.cells,
        "maps": maps,
        "byte_scatter_form": box_form,
        "small_triangle_r10": small,
        "large_workloads": large,
        "packed_state": packed,
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
