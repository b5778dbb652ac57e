"""Benchmark: leaf-parallel random-playout throughput on one MI355X.

Workload (leaf-parallel rollout): 4096 synthetic mid-game two-player leaf
states (pool 0-16 tiles, 0-8 tiles revealed per row, turn start), 256
uniform-random playouts each = 1,048,576 playouts per step.  One step is one
pass of the hot path over that batch: generate the leaf states on the GPU
(dvc_init_states), then run every playout with per-playout winner (int8),
game length (int16) and per-leaf seat wins (dvc_rollout).  Inputs are
synthetic and resident in HBM before timing starts.

By default 400 steps (about 45 ms) are timed: the first milliseconds after
the synchronize before the timed region run slower (a 50-step region
measures about 4 % less throughput, with the kernel itself slower), so a
longer region measures the steady state.

Prints one JSON line.  `value` is playouts/s of the whole step; `roofline`
prices the dominant kernel (the rollout kernel, one playout per lane at this
size) against the integer-VALU issue peak of the chip, from its average
duration between HIP events around it in every fourth timed step
(`--event-every`: a pair of events costs a step a few microseconds); `cpu_baseline` is the
CPU oracle timed on this host's cores on a bounded sample of the same
workload.  Side figures: batched search (as configured, with two leaves per
pass, also pipelined, and with the shape the library's search autotuner
picks under its agreement guard, each with its `critical_path`: the launch
against the per-wavefront instruction-issue bound), root-parallel search and
a single tree (also four leaves per pass, plain and pipelined), timed with
HIP events;
`value_vs_rollout`: value-network training on
pairs the rollout kernel labels (step time, TFLOP/s) and the value-network
search against the pure-playout search on 1024 fresh deals x 4096 iterations
(decisions/s of both, GPU-seconds ratio, root-move agreement).

--copy-mib N additionally copies an N MiB device buffer three times after the
timed steps: a kernel of known traffic, used to scale the HBM byte counters
of a profiler run.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_LEAVES, PPL, SEED = 4096, 256, 2
DEAL = dict(p_min=2, p_max=2, pile_min=0, pile_max=16, revealed_max=8)

# Integer VALU peak of MI355X, from its unit counts and clock: 256 CUs x 4
# SIMDs x 32 lanes per clock x 2.4 GHz = 78.6 T lane-ops/s (the published
# 157.3 TFLOP/s vector FP32 rate counts the same 32 lanes, an FMA as two).
# The chip's own issue-rate probe (measure.probe_valu: v_xor_b32 at 58 T/s) rules
# out the 16-lanes-per-clock figure (39.3 T).
INT_VALU_PEAK = 256 * 4 * 32 * 2.4e9          # lane-ops/s
# Algorithmic integer operations of one guess step, each weighted by its
# issue cost relative to a 32-bit xor as measured by that probe (xor 58.1,
# add 54.5, 32x32->64 multiply-add 32.7, high multiply 34.7, bit count 36.7
# T/s): one Philox4x32-10 block = 20 multiplies (x1.78) + 40 xors + 18 adds
# (x1.07) = 94.7; four uniform picks (high multiplies, x1.67) = 6.7; four bit
# counts (x1.58) = 6.3; three k-th-set-bit selections (about 30 operations
# each as a bit-count search) = 90; about 24 mask operations on the 24-bit
# rows.  Total ~222 xor-equivalent lane-operations per guess step.
OPS_PER_GUESS = 222

# HBM traffic of one launch of the rollout kernel at this workload, from two
# profiler counter passes (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each
# scaled by what the same counter reads for a plain 256 MiB device copy
# (FETCH_SIZE reads half the bytes moved, WRITE_SIZE all of them).  Valid
# only for the kernel sources it was taken on: reported as null otherwise.
PROFILED_TRAFFIC = {"fetch_kib": 400.5, "fetch_scale": 2.0, "write_kib": 3200.0,
                    "write_scale": 1.0,
                    "sources_sha256": "8f5c798da1bdf421cc7236fcff008f8315034d9863134c491d75a1da3f598c77"}
# Instructions one tree issues per iteration in the batched search (both
# wavefronts of a pipelined tree), from the SQ instruction counters of a
# profiler pass over `experiments --what phases` (VALU + SALU + LDS + SMEM +
# VMEM + branch), keyed by (playouts per leaf, leaves per pass, pipeline);
# valid only for the tree-kernel sources they were taken on.
PROFILED_SEARCH = {"instructions_per_tree_iteration": {(32, 1, 0): 4749, (32, 2, 1): 3465},
                   "sources_sha256": "eeecd58f2c4c6f297fc5597b0d03fd7363da26774ab592b43d6eada116c10273"}
SEARCH_SOURCES = ["paper_2403_10720_amd/csrc/dvc_core.hpp",
                  "paper_2403_10720_amd/csrc/dvc_internal.hpp",
                  "paper_2403_10720_amd/csrc/search.hip"]
KERNEL_SOURCES = ["paper_2403_10720_amd/csrc/dvc_core.hpp",
                  "paper_2403_10720_amd/csrc/dvc_internal.hpp",
                  "paper_2403_10720_amd/csrc/rollout.hip"]


def sources_sha256(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def search_critical_path(ms, iterations, ppl, lpp, pipeline):
    """The tree kernel against its bound: a wavefront issues at most one
    instruction per 4-cycle slot, so a tree whose W wavefronts issued every
    slot would need instructions x 4 / W cycles per iteration; the launch
    takes ms x 2.4 GHz / iterations (every tree runs concurrently, the
    slowest sets the time).  frac = the first over the second.  None when
    the profiled count does not cover this shape or these sources."""
    n_inst = PROFILED_SEARCH["instructions_per_tree_iteration"].get((ppl, lpp, pipeline))
    if n_inst is None or sources_sha256(SEARCH_SOURCES) != PROFILED_SEARCH["sources_sha256"]:
        return None
    waves = 2 if pipeline else 1
    bound = n_inst * 4.0 / waves
    launch = ms * 1e-3 * 2.4e9 / iterations
    return {"bound": "per-wavefront instruction issue (one per 4-cycle slot)",
            "instructions_per_tree_iteration": n_inst, "wavefronts_per_tree": waves,
            "issue_bound_cycles_per_iteration": bound,
            "launch_cycles_per_iteration_at_2.4GHz": launch, "frac": bound / launch}


def profiled_traffic_bytes():
    t = PROFILED_TRAFFIC
    if sources_sha256() != t["sources_sha256"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-search", action="store_true", help="skip the tree-search figures")
    ap.add_argument("--no-value", action="store_true",
                    help="skip value-network training and the value-vs-playout search")
    ap.add_argument("--copy-mib", type=int, default=0, help="copy a buffer of this size (MiB)")
    ap.add_argument("--event-every", type=int, default=4,
                    help="bracket the rollout kernel of every N-th timed step with HIP events "
                         "(each pair costs the step a few microseconds of GPU time)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="also measure the issue rate of the integer operations of a guess step")
    ap.add_argument("--cpu-sweep", action="store_true",
                    help="also time the CPU oracle at 1, 2, 4, ... threads (the paper's CPU sweep)")
    return ap.parse_args()


SEARCH_DEAL = dict(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), pile_min=0, pile_max=16,
                   revealed_max=8, root_draw=1)


def batched_search(D, torch, reps=3, leaves_per_pass=1, pipeline=0):
    """Batched search: 2048 mixed 2/3/4-player roots, 1024 iterations x 32 playouts,
    depth 4, one launch; decisions/s from HIP events.  leaves_per_pass 2: two
    leaves' playouts share each tree's 64 lanes; pipeline 1: a pass's wins are
    credited after the next pass's descents, one wavefront per tree descending
    while another plays out."""
    n, iters, ppl = 2048, 1024, 32
    roots = D.dvc_init_states(n, D.deal_params(**SEARCH_DEAL), 3)
    mp = D.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=4,
                       leaves_per_pass=leaves_per_pass, pipeline=pipeline)
    ws = torch.empty(D.dvc_mcts_workspace_bytes(n, mp), dtype=torch.uint8, device=roots.device)
    D.mcts_search(roots, mp, 3, workspace=ws, want_children=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        D.mcts_search(roots, mp, 3, workspace=ws, want_children=False)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    best = min(ms)
    return {"critical_path": search_critical_path(best, iters, ppl, leaves_per_pass, pipeline),
            "workload": "2048 trees (2-4 players, mid-game, root draw) x 1024 iterations x 32 "
                        "playouts, depth 4" + (f", {leaves_per_pass} leaves per pass"
                                               if leaves_per_pass > 1 else "") +
                        (", pipelined passes" if pipeline else ""),
            "ms_per_launch": best,
            "decisions_per_s": n / (best / 1e3), "playouts_per_s": n * iters * ppl / (best / 1e3)}


def autotuned_search(D, torch, reps=3, tolerance=0.02):
    """The batched search with the shape the library's search autotuner picks
    for it: dvc_mcts_autotune times every (playouts per leaf, leaves per pass,
    pipelined or not) candidate on these roots and admits those whose
    decisions agree with the sequential 32-playout search at least as often as
    a second seed of that search does, less `tolerance`; the fastest admitted
    shape then runs as the automatic shape (playouts per leaf, leaves per pass
    and pipeline all 0)."""
    n, iters, ppl = 2048, 1024, 32
    roots = D.dvc_init_states(n, D.deal_params(**SEARCH_DEAL), 3)
    ref = D.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=4)
    auto = D.mcts_params(iterations=iters, playouts_per_leaf=0, max_depth=4, leaves_per_pass=0)
    ws = torch.empty(max(D.dvc_mcts_workspace_bytes(n, ref), D.dvc_mcts_workspace_bytes(n, auto)),
                     dtype=torch.uint8, device=roots.device)
    choice, _ = D.dvc_mcts_autotune(roots, ref, 3, workspace=ws, tolerance=tolerance)
    D.mcts_search(roots, auto, 3, workspace=ws, want_children=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        D.mcts_search(roots, auto, 3, workspace=ws, want_children=False)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    best = min(ms)
    return {"critical_path": search_critical_path(best, iters, choice["playouts_per_leaf"],
                                                  choice["leaves_per_pass"], choice["pipeline"]),
            "workload": "2048 trees (2-4 players, mid-game, root draw) x 1024 iterations, depth 4, "
                        "autotuned playouts per leaf x leaves per pass x pipelined passes "
                        "(agreement guard: within "
                        f"{tolerance} of the 32-playout search's seed-to-seed agreement)",
            "choice": choice, "ms_per_launch": best, "decisions_per_s": n / (best / 1e3),
            "playouts_per_s": n * iters * choice["playouts_per_leaf"] / (best / 1e3)}


def root_parallel_search(D, torch, reps=3, leaves_per_pass=1, pipeline=0):
    """The paper's decomposition: 64 fresh 2-4 player deals, 32 independent
    trees each (1024 iterations x 32 playouts, depth 4), amalgamated at the
    root; optionally each tree with two leaves per pass, pipelined."""
    n, K, iters, ppl = 64, 32, 1024, 32
    roots = D.dvc_init_states(n, D.deal_params(p_min=2, p_max=4, hand=(0, 0, 4, 4, 3), fresh=1,
                                               root_draw=1), 6)
    mp = D.mcts_params(iterations=iters, playouts_per_leaf=ppl, max_depth=4,
                       leaves_per_pass=leaves_per_pass, pipeline=pipeline)
    ws = torch.empty(D.dvc_mcts_workspace_bytes(n * K, mp), dtype=torch.uint8, device=roots.device)
    D.mcts_search_root_parallel(roots, K, mp, 6, workspace=ws, want_children=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        D.mcts_search_root_parallel(roots, K, mp, 6, workspace=ws, want_children=False)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    best = min(ms)
    return {"workload": "64 fresh 2-4 player deals x 32 trees x 1024 iterations x 32 playouts, "
                        "depth 4, merged at the root" +
                        (f", {leaves_per_pass} leaves per pass" if leaves_per_pass > 1 else "") +
                        (", pipelined passes" if pipeline else ""), "ms_per_launch": best,
            "decisions_per_s": n / (best / 1e3), "playouts_per_s": n * K * iters * ppl / (best / 1e3)}


def single_tree_search(D, torch, leaves_per_pass=1, pipeline=0, reps=5):
    """Plain search: one fresh two-player deal, 2000 iterations x 16 playouts.
    leaves_per_pass 4: four descents per pass, their 64 playouts filling the
    wavefront (a different, batched schedule of the same iterations);
    pipeline 1: pipelined passes (two wavefronts)."""
    roots = D.dvc_init_states(1, D.deal_params(p_min=2, p_max=2, fresh=1, root_draw=1), 1)
    mp = D.mcts_params(iterations=2000, playouts_per_leaf=16, max_depth=4,
                       leaves_per_pass=leaves_per_pass, pipeline=pipeline)
    ws = torch.empty(D.dvc_mcts_workspace_bytes(1, mp), dtype=torch.uint8, device=roots.device)
    D.mcts_search(roots, mp, 1, workspace=ws, want_children=False)
    torch.cuda.synchronize()
    gpu, wall = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        best, _ = D.mcts_search(roots, mp, 1, workspace=ws, want_children=False)
        e1.record()
        int(best[0].item())   # the decision on the host
        wall.append((time.perf_counter() - t0) * 1e3)
        gpu.append(e0.elapsed_time(e1))
    ms = sorted(gpu)[len(gpu) // 2]
    return {"workload": "1 tree, fresh 2-player deal, 2000 iterations x 16 playouts" +
                        (f", {leaves_per_pass} leaves per pass" if leaves_per_pass > 1 else "") +
                        (", pipelined passes" if pipeline else ""),
            "ms_per_decision": ms, "decisions_per_s": 1e3 / ms,
            "ms_per_decision_mean": sum(gpu) / len(gpu),
            "wall_ms_per_decision": sorted(wall)[len(wall) // 2],
            "timing": f"HIP events, median of {reps} launches after one warm-up; wall: host call "
                      f"to the decision read back, median"}


def value_vs_rollout():
    """The learned evaluator end to end: 2^23 training pairs (2-4 player
    mid-game states, labels = 256-playout win rates) generated by the rollout
    kernel, 20 epochs of batch 8192 on the library's training kernels (Adam,
    lr 1e-3), the network's MSE against 4096-playout estimates on 4096
    held-out states, then 1024 fresh 2-4 player deals searched for 4096
    iterations with the network at the leaves (64 fallback playouts when the
    root player's value is within 0.05 of 1/2) and with 64 playouts per leaf:
    decisions/s of both, the GPU-seconds ratio, root-move agreement next to
    the agreement of two playout searches with different seeds.  Every search
    is timed with HIP events, median of three launches after a warm-up."""
    from paper_2403_10720_amd.experiments import compare
    out, _ = compare(log=lambda m: None)
    return out


def gpu_info(torch):
    """The device and its clocks as rocm-smi reports them after the timed steps
    (best effort: None where the tool is missing or prints something else)."""
    import subprocess
    p = torch.cuda.get_device_properties(0)
    out = {"name": p.name, "compute_units": p.multi_processor_count,
           "gcn_arch": getattr(p, "gcnArchName", None), "clocks": None}
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=20)
        card = next(iter(json.loads(r.stdout).values()))
        out["clocks"] = {k: v for k, v in card.items() if "clock" in k.lower()}
    except Exception:
        pass
    return out


def host_cpu():
    """(CPU model, physical cores among the CPUs this process may run on)."""
    model, cores, phys, core = "unknown", set(), None, None
    allowed = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    cpu = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    cpu = int(v)
                elif k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                if k == "core id" and (allowed is None or cpu in allowed):
                    cores.add((phys, core))
    except OSError:
        pass
    n = len(cores) or len(allowed or []) or (os.cpu_count() or 1)
    return model, n


def _median_rate(fn, n_items, reps):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return n_items / ts[len(ts) // 2], ts


def cpu_baseline(states_np, reps=10):
    """The oracle, as it stands, on this host.  Playouts/s on the full batch
    (4096 leaves x 256 playouts) with the leaves split over one thread per
    physical core (at most 16, this GPU's share of the host), and on 512 of
    the leaves with one thread; median of `reps` runs each.  Also the single
    tree search (one fresh two-player deal, 2000 iterations x 16 playouts), one
    thread, median of 5."""
    import oracle
    model, phys = host_cpu()
    threads = max(1, min(16, phys))
    oracle.rollout(states_np[:64], 16, SEED)          # load + warm
    n = states_np.shape[0] * PPL
    rate, ts = _median_rate(lambda: oracle.rollout(states_np, PPL, SEED, threads=threads,
                                                   want_winner=False, want_length=False),
                            n, reps)
    sample = states_np[:512]
    rate1, ts1 = _median_rate(lambda: oracle.rollout(sample, PPL, SEED, threads=1,
                                                     want_winner=False, want_length=False),
                              sample.shape[0] * PPL, reps)
    root = oracle.init_states(1, oracle.deal_params(p_min=2, p_max=2, fresh=1, root_draw=1), 1)
    mp = oracle.mcts_params(iterations=2000, playouts_per_leaf=16, max_depth=4)
    rate_t, _ = _median_rate(lambda: oracle.mcts_search(root, mp, 1, 0), 1, 5)
    return {"value": rate, "unit": "playouts/s", "cores": threads, "kind": "oracle",
            "sample": f"{states_np.shape[0]} leaves x {PPL} playouts (the full batch), "
                      f"{threads} threads, median of {reps} runs ({ts[len(ts) // 2]:.3f} s)",
            "cpu_model": model, "physical_cores": phys,
            "single_thread": {"value": rate1, "unit": "playouts/s",
                              "sample": f"512 leaves x {PPL} playouts, 1 thread, median of "
                                        f"{reps} runs ({ts1[len(ts1) // 2]:.3f} s)"},
            "single_tree_ms_per_decision": 1e3 / rate_t,
            "single_tree_sample": "1 fresh 2-player deal, 2000 iterations x 16 playouts, "
                                  "1 thread, median of 5"}


def valu_probe(torch, iters=4096):
    """Issue rate (T lane-ops/s) of each integer operation of a guess step,
    eight waves per SIMD, eight independent chains per lane."""
    from paper_2403_10720_amd import measure
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * 8
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    out = {}
    for op, name in enumerate(measure.OPS):
        measure.probe_valu(op, blocks, 16, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        measure.probe_valu(op, blocks, iters, sink)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        out[name] = blocks * 256 * iters * 64 / t / 1e12
    return out


def cpu_thread_sweep(states_np, max_threads):
    """Oracle playouts/s against host threads on 512 leaves x 256 playouts."""
    import oracle
    sample = states_np[:512]
    out = []
    t = 1
    while t <= max_threads:
        t0 = time.perf_counter()
        oracle.rollout(sample, PPL, SEED, threads=t, want_winner=False, want_length=False)
        dt = time.perf_counter() - t0
        out.append({"threads": t, "playouts_per_s": sample.shape[0] * PPL / dt})
        t *= 2
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2403_10720_amd as D

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    params = D.deal_params(**DEAL)
    total = N_LEAVES * PPL
    states = torch.empty((N_LEAVES, 4), dtype=torch.int32, device=dev)
    winner = torch.empty(total, dtype=torch.int8, device=dev)
    length = torch.empty(total, dtype=torch.int16, device=dev)
    wins = torch.empty((N_LEAVES, 4), dtype=torch.int32, device=dev)

    # The automatic shape at this size (variant 7) stores each leaf's seat
    # wins over the table, as variants 7 and 9 do when a workgroup holds
    # whole leaves; other shapes add to a table zeroed here first.  Either
    # way the events bracket the rollout kernel alone.
    stores_wins = args.variant in (0, 7, 9)

    def step(ev=None):
        D.dvc_init_states(N_LEAVES, params, SEED, out=states)
        if not stores_wins:
            wins.zero_()
        if ev is not None:
            ev[0].record(stream)
        D.dvc_rollout(states, PPL, SEED, 0, 0, winner=winner, length=length, seat_wins=wins,
                      variant=args.variant, block=args.block, grid=args.grid,
                      accumulate=not stores_wins)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rc = D.dvc_check()
    if rc != 0:
        raise RuntimeError(f"device error {rc}")
    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
    guesses = int(length.to(torch.int64).sum().item())
    lens = length.float()
    every = max(1, args.event_every)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           if k % every == 0 else None for k in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # torch creates a HIP event at its first record: create them all here,
    # outside the timed region
    for e in [(start, stop)] + [e for e in evs if e is not None]:
        e[0].record(stream)
        e[1].record(stream)
    torch.cuda.synchronize()
    start.record(stream)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.copy_mib > 0:
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    kern_ms = [e[0].elapsed_time(e[1]) for e in evs if e is not None]
    ms_step = ms_total / args.steps
    kern_avg_s = sum(kern_ms) / len(kern_ms) / 1e3
    value = total / (ms_step / 1e3)
    achieved = guesses * OPS_PER_GUESS / kern_avg_s
    out = {
        "metric": "playouts/sec (leaf-parallel random playouts, Da Vinci Code MCTS simulation step)",
        "value": value,
        "unit": "playouts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (Philox-generated game states)",
        "config": {"workload": "leaf-parallel rollout: 4096 two-player mid-game leaves x 256 "
                               "playouts (pool 0-16, 0-8 revealed per row)",
                   "leaves": N_LEAVES, "playouts_per_leaf": PPL, "seed": SEED,
                   # 0/0/0 is the library's automatic shape at this size: variant 7
                   # (compacted at steps 5, 8, 11, 14, 17)
                   "variant": args.variant or 7, "block": args.block,
                   "grid": args.grid if args.variant else 2},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_VALU_PEAK / 1e12,
                     "unit": "TOP/s", "frac": achieved / INT_VALU_PEAK,
                     "traffic": profiled_traffic_bytes()},
        "rollout_kernel_ms": kern_avg_s * 1e3,
        "rollout_kernel_timing": f"HIP events on the launch stream around the rollout kernel of "
                                 f"{len(kern_ms)} of the {args.steps} timed steps (every {every}th)",
        "guess_steps_per_launch": guesses,
        "mean_game_length": float(lens.mean().item()),
        "wall_s": wall,
        "gpu": gpu_info(torch),
    }
    if args.valu_probe:
        out["roofline"]["probe_TOPs"] = valu_probe(torch)
    if not args.no_search:
        out["batched_search"] = batched_search(D, torch)
        out["batched_search_leaf_batched"] = batched_search(D, torch, leaves_per_pass=2)
        out["batched_search_pipelined"] = batched_search(D, torch, leaves_per_pass=2, pipeline=1)
        out["batched_search_autotuned"] = autotuned_search(D, torch)
        out["root_parallel_search"] = root_parallel_search(D, torch)
        out["root_parallel_search_pipelined"] = root_parallel_search(D, torch, leaves_per_pass=2,
                                                                     pipeline=1)
        out["single_tree_search"] = single_tree_search(D, torch)
        out["single_tree_search_leaf_batched"] = single_tree_search(D, torch, leaves_per_pass=4)
        out["single_tree_search_pipelined"] = single_tree_search(D, torch, leaves_per_pass=4,
                                                                 pipeline=1)
    if not args.no_value:
        out["value_vs_rollout"] = value_vs_rollout()
    if not args.no_cpu:
        host_states = states.cpu().numpy().view(np.uint32)
        out["cpu_baseline"] = cpu_baseline(host_states)
        if args.cpu_sweep:
            out["cpu_baseline"]["thread_sweep"] = cpu_thread_sweep(
                host_states, 2 * (os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
