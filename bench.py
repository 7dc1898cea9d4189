#!/usr/bin/env python3
"""Throughput of the batched push transition on one MI355X.

One step = one pass of the batched expansion/simulation hot path over the
benchmark workload: load every environment from the device state pool
(batch expansion, Sec. IV-C), one 5 cm push per environment (Sec. V-A:
120 substeps of 1/240 s, 10 Jacobi iterations each) through the fused step
kernel (with more environments than resident workgroups a cost pass at the
start poses first orders each XCD's environments largest first, and
persistent workgroups take them from per-XCD queues), then the retrieval
reward of every environment.  Workload: 4096
environments x 15 cuboids (edges U[3,6] cm, mass U[0.05,0.2] kg, mu
U[0.3,0.7]) on a 0.3 m table, one circle push each; seeded and synthetic.

Prints one JSON line: env-substeps/s, the step kernel against the FP32
vector-ALU roofline, the algorithmic HBM fraction, and the FP64 oracle's
throughput on the host cores for the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (counts packed FP32: two operations per lane per cycle)
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # the same without packed FP32 (256 CUs x 2.4 GHz x 128 flop/cycle)
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E


def flops_per_env_substep(nc: float, npairs: float, nb: float, iters: int) -> float:
    """Algorithmic FP32 operations of one substep of one environment, the
    work model F = N_c (250 + 144 I) + 300 n_b + 500 N_cand + 1000 (FMA = 2):
    per contact and Jacobi iteration 144 (relative velocity at both lever
    arms, normal and friction-cone update, impulse, its two torques, the
    per-body sums and velocity updates), per contact 250 of preparation
    (lever arms, tangent basis, three effective masses, bias), per body 300
    (velocity and position stages, frames, world inverse inertia, AABB,
    plane vertices), per candidate pair 500 (separating-axis test) and
    1000 per environment (broadphase pair tests, push begin)."""
    return nc * (250.0 + 144.0 * iters) + 300.0 * nb + 500.0 * npairs + 1000.0


def flops_counted(nc: float, npairs: float, nb: float, iters: int) -> float:
    """The same work counted from the kernel's own arithmetic (FMA = 2):
    per Jacobi iteration 108 per contact and 21 per body; per substep 230
    per contact, 880 per candidate pair (15 axes) and 190 per body."""
    return iters * (108.0 * nc + 21.0 * nb) + 230.0 * nc + 880.0 * npairs + 190.0 * nb


def hbm_bytes_per_call(n_bodies: int, n_envs: int) -> float:
    """State in (52 B) + geometry/material (32 B) + state out (52 B) per
    body; env offsets, push and status (28 B) per environment."""
    return 136.0 * n_bodies + 28.0 * n_envs


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_4096x15_traffic.md")
KERNEL_SOURCES = ("paper_2207_06649_amd/csrc/pmbs_kernels.hip", "paper_2207_06649_amd/csrc/pmbs_kernels.h")


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code: comments and whitespace removed, so
    an edit to a comment keeps the recorded counters valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            src = f.read()
        # string and character literals are kept whole; comments go
        tokens = re.findall(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/|\S+', src, re.S)
        code = " ".join(t for t in tokens if not t.startswith(("//", "/*")))
        h.update(rel.encode() + b"\0" + code.encode())
    return h.hexdigest()


def measured_traffic(n_envs: int, n_bodies: int, substeps: int):
    """HBM bytes per step-kernel launch from the recorded FETCH_SIZE and
    WRITE_SIZE counter runs (each scaled by the same counter's reading for a
    plain device copy of known size; the record is written by
    bench_traffic.py), or None when the counters were taken on other kernel
    sources or another workload."""
    rec = {}
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    rec[k.strip()] = v.strip()
    except OSError:
        return None
    try:
        if rec.get("kernel_source_sha256") != kernel_source_hash():
            return None
        if (int(rec["envs"]), int(rec["bodies_per_env"]), int(rec["substeps"])) != (n_envs, n_bodies, substeps):
            return None
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_threads() -> int:
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        n = min(n, int(omp))
    return max(1, n)


def plan_latency(pmbs, scenes, args) -> dict:
    """MCTS object retrieval: 20 cuboids + a target at the centre of a
    0.4 m square; UCT c = 1.4, leaves per iteration, depth <= 5 pushes,
    30 iterations.  Wall time of pmbs_plan per seeded scene (p50/p99), and
    serial one-leaf-at-a-time MCTS on the same scene, timed for a bounded
    number of iterations and projected to the same number of simulations."""
    import torch
    n_bodies, depth = 21, 5
    times, values, subs = [], [], []

    def sim_for(n_envs, max_nodes):
        return pmbs.Sim(max_envs=n_envs, max_bodies=n_envs * n_bodies, pool_slots=max_nodes, pool_stride=n_bodies,
                        max_horizon=depth)

    def root_reward(st, bd):
        s1 = pmbs.Sim(max_envs=1, max_bodies=n_bodies)
        s1.set_state([0, n_bodies], st, bd)
        return float(s1.eval_reward([0], 0.08)[0][0])

    leaves, iters = args.plan_leaves, args.plan_iters
    max_nodes = leaves * iters + 2
    sim = sim_for(leaves, max_nodes)
    # launch plan (workgroup shape, workgroups per CU, order) chosen by the
    # autotuner on a rollout of the planning workload's shape: every leaf a
    # copy of the first scene with depth-many random contour pushes
    sc0 = scenes.retrieval_scene(100, n_others=20, region=0.4)
    tb = scenes.concat([scenes.Batch(np.array([0, n_bodies], np.int32), sc0.state, sc0.body, np.zeros((1, 4)),
                                     np.zeros(1, np.int32))] * leaves)
    sim.set_state(tb.env_offset, tb.state, tb.body)
    t_acts, t_off = scenes.contour_actions(7, tb.counts(), np.full(leaves, depth))
    t0 = time.perf_counter()
    tuned, tuned_ms, _ = sim.autotune(t_acts, t_off, np.zeros(leaves, np.int32), n_substeps=120, max_h=depth, reps=3,
                                      flags=pmbs.ROLLOUT_QUEUE)
    tune_s = time.perf_counter() - t0
    print(f"# plan launch plan {tuned} ({tuned_ms:.1f} ms per rollout, {tune_s:.1f} s of tuning)", file=sys.stderr,
          flush=True)
    for k in range(args.plan_scenes):
        sc = scenes.retrieval_scene(100 + k, n_others=20, region=0.4)
        tree = pmbs.Tree(n_bodies, root_reward(sc.state, sc.body), n_envs=leaves, max_depth=depth, c=1.4,
                         gamma=0.8, seed=100 + k, max_nodes=max_nodes)
        res = pmbs.plan(sim, tree, sc.state, sc.body, 0, iters, n_substeps=120)
        times.append(res["seconds"])
        values.append(res["value"])
        subs.append(res["env_substeps"])
        print(f"# plan scene {k}: {res['seconds']:.3f} s, action {res['action']}, value {res['value']:.3f}, "
              f"{res['nodes']} nodes", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # serial baseline: same scene as the first plan, one leaf per iteration
    sc = scenes.retrieval_scene(100, n_others=20, region=0.4)
    ssim = sim_for(1, args.serial_iters + 2)
    ssim.set_launch_plan(**tuned)   # the same launch shape for the one-leaf search
    tree = pmbs.Tree(n_bodies, root_reward(sc.state, sc.body), n_envs=1, max_depth=depth, c=1.4, gamma=0.8,
                     seed=100, max_nodes=args.serial_iters + 2)
    sres = pmbs.plan(ssim, tree, sc.state, sc.body, 0, args.serial_iters, n_substeps=120)
    per_iter = sres["seconds"] / max(1, sres["iterations"])
    projected = per_iter * leaves * iters
    t = np.array(times)
    return {
        "workload": f"{n_bodies - 1} cuboids + target in 0.4 m square, c=1.4, {leaves} leaves/iteration, "
                    f"depth <= {depth}, {iters} iterations, 120 substeps per push",
        "scenes": len(times),
        "p50_s": round(float(np.percentile(t, 50)), 4),
        "p99_s": round(float(np.percentile(t, 99)), 4),
        "mean_s": round(float(t.mean()), 4),
        "env_substeps_per_s": round(float(np.sum(subs) / t.sum()), 1),
        "serial": {"iterations_timed": int(sres["iterations"]), "s_per_iteration": round(per_iter, 5),
                   "projected_s_same_simulations": round(projected, 3)},
        "speedup_vs_serial": round(projected / float(np.percentile(t, 50)), 2),
        "launch_plan": tuned,
    }


def batched_1024(pmbs, scenes, args) -> dict:
    """The batched-step workload at 1024 envs x 15 cuboids (seed 1): the same
    step (pool gather + fused push step + reward) timed over args.steps, for
    one and two waves per environment (about one environment per SIMD, so
    the shape matters); the faster shape is reported."""
    import torch
    b = scenes.clutter_batch(1, args.small_envs, args.bodies)
    E = b.n_envs
    dev = torch.device("cuda:0")
    sim = pmbs.Sim(max_envs=E, max_bodies=b.n_bodies, pool_slots=E, pool_stride=int(b.counts().max()))
    sim.set_state(b.env_offset, b.state, b.body)
    slots = torch.arange(E, dtype=torch.int32, device=dev)
    sim.pool_scatter(slots)
    push = torch.tensor(b.push.astype(np.float32), device=dev).contiguous()
    target = torch.zeros(E, dtype=torch.int32, device=dev)
    rew = torch.empty(E, dtype=torch.float32, device=dev)
    clr = torch.empty(E, dtype=torch.float32, device=dev)

    def one():
        sim.pool_gather(slots)
        sim.step(push, args.substeps)
        sim.eval_reward(target, 0.08, rew, clr, sync=False)

    per_shape = {}
    for waves in (1, 2):
        sim.set_launch_plan(small_waves=waves, large_waves=waves)
        for _ in range(args.warmup):
            one()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(sim.stream)
        for _ in range(args.steps):
            one()
        ev[1].record(sim.stream)
        torch.cuda.synchronize()
        per_shape[waves] = ev[0].elapsed_time(ev[1]) / args.steps
    waves = min(per_shape, key=per_shape.get)
    ms = per_shape[waves]
    status = sim.env_status()
    return {"workload": f"{E} envs x {args.bodies} cuboids, one 5 cm circle push each, {args.substeps} substeps "
                        "(seed 1)",
            "env_substeps_per_s": round(E * args.substeps / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
            "waves_per_env": waves, "ms_per_step_by_waves": {str(k): round(v, 4) for k, v in per_shape.items()},
            "valid_pushes": int(np.sum((status & pmbs.PMBS_ENV_PUSH_INVALID) == 0))}


def plain_per_push(sim, acts, off, tgt, n_substeps, width=0.08, rewards=None, counts=None):
    """The plain form of uneven rollouts: one launch per push index over a
    fixed-shape batch (the caller pads every env to the same body count),
    one workgroup per env, the state kept in the env slots, and a
    synchronous read-back after every launch to apply the rollout rules on
    the host (a discarded expansion push ends the env, a later discarded
    push repeats the previous reward, a reward of 1 ends the env).
    Returns (rewards [E, H], counts [E], status [E])."""
    from paper_2207_06649_amd import pmbs
    off = np.asarray(off)
    h = np.diff(off)
    E, H = len(h), int(h.max()) if len(h) else 0
    rew = np.zeros((E, max(H, 1)), np.float32)
    cnt = np.zeros(E, np.int32)
    status = np.zeros(E, np.uint32)
    last = np.zeros(E, np.float32)
    ended = np.zeros(E, bool)
    for t in range(H):
        go = (~ended) & (t < h)
        a1 = acts[(off[:-1] + t)[go]] if go.any() else np.zeros(0, np.int32)
        o1 = np.zeros(E + 1, np.int32)
        o1[1:] = np.cumsum(go)
        r1, c1 = sim.rollout(a1, o1, tgt, n_substeps=n_substeps, width=width, max_h=1,
                             flags=pmbs.ROLLOUT_WRITE_STATE, rewards=rewards, counts=counts)
        st = sim.env_status()
        took = go & (c1 > 0)
        dropped = go & (c1 == 0)
        rew[took, t] = r1[took, 0]
        last[took] = r1[took, 0]
        cnt[took] = t + 1
        if t == 0:
            ended |= dropped
            status[dropped] |= pmbs.PMBS_ENV_PUSH_INVALID
        else:
            rew[dropped, t] = last[dropped]
            cnt[dropped] = t + 1
        status[go] |= st[go] & ~np.uint32(pmbs.PMBS_ENV_PUSH_INVALID)
        ended |= took & (r1[:, 0] >= 1.0)
    return rew, cnt, status


def uneven_batching(pmbs, scenes, args) -> dict:
    """Uneven batch: envs of 5-30 cuboids, 1-5 contour pushes each, 120
    substeps per push.  Packed form: one graph-captured launch of persistent
    work-queue kernels per contact class, envs loaded from pool slots,
    launch plan chosen by the autotuner, batches launched back to back.
    Plain form: every env padded to 30 bodies, one launch per push index
    with a host round trip between launches.  Both report useful
    env-substeps (real bodies, pushes actually simulated) per second of
    wall time."""
    import torch
    E, sub, H = args.uneven_envs, args.substeps, 5
    t0 = time.time()
    b = scenes.clutter_batch(3, E, (5, 30))
    hz = scenes.horizons(3, E)
    acts, off = scenes.contour_actions(3, b.counts(), hz)
    tgt = np.zeros(E, np.int32)
    print(f"# uneven workload ready: {E} envs, {b.n_bodies} bodies, {int(off[-1])} pushes "
          f"({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    sim = pmbs.Sim(max_envs=E, max_bodies=b.n_bodies, max_contacts=256, pool_slots=2 * E, pool_stride=31,
                   max_horizon=H)
    sim.set_state(b.env_offset, b.state, b.body)
    src = np.arange(E, dtype=np.int32)
    child = src + E
    sim.pool_scatter(src)
    rew = torch.empty((E, H), dtype=torch.float32, device=dev)
    cnt = torch.empty(E, dtype=torch.int32, device=dev)
    t1 = time.perf_counter()
    plan, tune_ms, _ = sim.autotune(acts, off, tgt, n_substeps=sub, src_slot=src, child_slot=child, max_h=H,
                                    reps=5, rewards=rew, counts=cnt, flags=pmbs.ROLLOUT_QUEUE | pmbs.ROLLOUT_GRAPH)
    tune_s = time.perf_counter() - t1
    print(f"# autotuned plan {plan} ({tune_ms:.1f} ms per launch, {tune_s:.1f} s of tuning)",
          file=sys.stderr, flush=True)
    flags = pmbs.ROLLOUT_QUEUE | pmbs.ROLLOUT_GRAPH
    sim.rollout(acts, off, tgt, n_substeps=sub, src_slot=src, child_slot=child, max_h=H, flags=flags,
                rewards=rew, counts=cnt, sync=True)   # capture
    useful = int(sim.stats()[:, 2].sum())
    reps = args.uneven_reps
    for _ in range(3):   # untimed replays after the capture
        sim.rollout(acts, off, tgt, n_substeps=sub, src_slot=src, child_slot=child, max_h=H, flags=flags,
                    rewards=rew, counts=cnt, sync=False)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    # batches launched back to back: the host stages batch k + 1 while the
    # device runs batch k (the inputs go through the simulator's pinned
    # staging, so nothing waits for the device until the end)
    for _ in range(reps):
        sim.rollout(acts, off, tgt, n_substeps=sub, src_slot=src, child_slot=child, max_h=H, flags=flags,
                    rewards=rew, counts=cnt, sync=False)
    sim.sync()
    packed_s = (time.perf_counter() - tw) / reps
    packed_rew, packed_cnt = rew.cpu().numpy(), cnt.cpu().numpy()
    del sim
    # plain form
    pb = scenes.pad_batch(b, 30)
    psim = pmbs.Sim(max_envs=E, max_bodies=pb.n_bodies, max_contacts=256, max_horizon=H)
    prew = torch.empty((E, 1), dtype=torch.float32, device=dev)
    pcnt = torch.empty(E, dtype=torch.int32, device=dev)
    plain = []
    for _ in range(max(1, reps // 2)):
        psim.set_state(pb.env_offset, pb.state, pb.body)
        torch.cuda.synchronize()
        tw = time.perf_counter()
        r_p, c_p, _ = plain_per_push(psim, acts, off, tgt, sub, rewards=prew, counts=pcnt)
        plain.append(time.perf_counter() - tw)
    plain_s = float(np.median(plain))
    same_counts = float(np.mean(c_p == packed_cnt))
    return {
        "workload": f"{E} envs x U{{5..30}} cuboids, U{{1..5}} contour pushes, {sub} substeps each",
        "useful_env_substeps": useful,
        "packed": {"env_substeps_per_s": round(useful / packed_s, 1), "s_per_batch": round(packed_s, 4),
                   "plan": plan, "autotune_s": round(tune_s, 2), "graph": True},
        "plain_padded_per_push": {"env_substeps_per_s": round(useful / plain_s, 1), "s_per_batch": round(plain_s, 4),
                                  "padded_to": 30},
        "speedup": round(plain_s / packed_s, 2),
        "envs_with_equal_reward_counts": round(same_counts, 4),
    }


def serving(pmbs, scenes, args) -> dict:
    """Planning requests arriving as a Poisson stream: scenes of 5-30 cuboids
    (a target at the centre), leaf batches of 64, 256 or 1024, 10-30
    iterations, depth <= 5, 120 substeps per push.  Continuous batching
    (every request in flight advances one iteration per packed,
    graph-replayed launch; admission by free env slots, request slots and
    node-pool bytes; two launch lanes, so one lane's tree work overlaps the
    other lane's device work) against the plain form: one request at a
    time in arrival order, each with its own batched launches.  Capacity
    comes from saturated runs (all requests at t = 0; continuous batching
    also with one lane); latency from Poisson runs at 0.7x each form's own
    capacity, and of continuous batching at the plain form's rate too (the
    nominal 50 requests/s saturates both forms)."""
    rng = np.random.default_rng([4, 2024])
    n = args.serve_requests
    reqs = []
    for k in range(n):
        nb = int(rng.integers(5, 31))
        sc = scenes.retrieval_scene(500 + k, n_others=nb - 1, region=0.4)
        reqs.append(dict(state=sc.state, body=sc.body, target=0, leaves=int(rng.choice([64, 256, 1024])),
                         iterations=int(rng.integers(10, 31)), seed=1000 + k))
    gaps = rng.exponential(1.0, size=n)

    def run(continuous: bool, rate: float | None, lanes: int = 2) -> dict:
        srv = pmbs.Server(max_envs=4096, max_requests=16 if continuous else 1, pool_slots=262144,
                          n_substeps=args.substeps, graph=1 if continuous else 0, lanes=lanes if continuous else 1)
        t0 = time.perf_counter()
        arrivals = np.cumsum(gaps / rate) - gaps[0] / rate if rate else np.zeros(n)
        ids = []
        for k, q in enumerate(reqs):
            delay = t0 + arrivals[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(**q))
        res = [srv.wait(i) for i in ids]
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.array([r["latency_seconds"] for r in res])
        useful = sum(r["env_substeps"] for r in res)
        return {"requests": n, "offered_per_s": round(rate, 3) if rate else None, "wall_s": round(wall, 3),
                "env_substeps_per_s": round(useful / wall, 1),
                "requests_per_s": round(n / wall, 3), "p50_s": round(float(np.percentile(lat, 50)), 4),
                "p99_s": round(float(np.percentile(lat, 99)), 4), "launches": st["launches"],
                "peak_in_flight": st["peak_in_flight"], "peak_held_mb": round(st["peak_held_bytes"] / 2**20, 1),
                "failed": int(sum(r["status"] != 0 for r in res)),
                "results": [(r["action"], round(r["value"], 6)) for r in res]}

    plain_sat = run(False, None)
    print(f"# serving plain saturated: {plain_sat['requests_per_s']} req/s", file=sys.stderr, flush=True)
    cont_sat = run(True, None)
    print(f"# serving continuous saturated: {cont_sat['requests_per_s']} req/s", file=sys.stderr, flush=True)
    cont1_sat = run(True, None, lanes=1)
    print(f"# serving continuous, one lane, saturated: {cont1_sat['requests_per_s']} req/s", file=sys.stderr,
          flush=True)
    rate_plain = min(50.0, 0.7 * plain_sat["requests_per_s"])
    rate_cont = min(50.0, 0.7 * cont_sat["requests_per_s"])
    plain = run(False, rate_plain)
    cont = run(True, rate_cont)
    cont_same_rate = run(True, rate_plain)
    res = [d.pop("results") for d in (plain, cont, cont_same_rate, plain_sat, cont_sat, cont1_sat)]
    same = all(r == res[0] for r in res[1:])
    return {
        "workload": f"{n} requests: 5-30 cuboids (target at the centre, 0.4 m square), leaves U{{64,256,1024}}, "
                    f"10-30 iterations, depth <= 5, {args.substeps} substeps per push",
        "nominal_rate_per_s": 50.0,
        "nominal_rate_saturates_both": bool(cont_sat["requests_per_s"] < 50.0 and plain_sat["requests_per_s"] < 50.0),
        "continuous": cont, "plain_per_request": plain, "continuous_at_plain_rate": cont_same_rate,
        "capacity": {"continuous": cont_sat, "continuous_one_lane": cont1_sat, "plain_per_request": plain_sat},
        "same_results_alone_and_mixed": same,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--bodies", type=int, default=15)
    ap.add_argument("--substeps", type=int, default=120)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan-scenes", type=int, default=5, help="seeded retrieval scenes for plan latency (0: skip)")
    ap.add_argument("--plan-iters", type=int, default=30)
    ap.add_argument("--plan-leaves", type=int, default=256)
    ap.add_argument("--serial-iters", type=int, default=64, help="one-leaf iterations timed for the serial baseline")
    ap.add_argument("--uneven-envs", type=int, default=4096, help="envs of the uneven batch (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=48, help="requests of the serving runs (0: skip)")
    ap.add_argument("--uneven-reps", type=int, default=16)
    ap.add_argument("--small-envs", type=int, default=1024, help="envs of the 1024 x 15 batched line (0: skip)")
    ap.add_argument("--no-peaks", dest="peaks", action="store_false", help="skip the FMA / copy peak probes")
    ap.add_argument("--copy-mb", type=int, default=256,
                    help="size of a plain device copy run after the timed region (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(environments would shard across GPUs with no exchange inside a step)",
              file=sys.stderr)
        return 2

    import torch

    from paper_2207_06649_amd import pmbs, scenes

    t0 = time.time()
    batch = scenes.clutter_batch(args.seed, args.envs, args.bodies)
    E, N = batch.n_envs, batch.n_bodies
    print(f"# workload ready: {E} envs, {N} bodies ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    sim = pmbs.Sim(max_envs=E, max_bodies=N, pool_slots=E, pool_stride=int(batch.counts().max()))
    sim.set_state(batch.env_offset, batch.state, batch.body)
    slots = torch.arange(E, dtype=torch.int32, device=dev)
    sim.pool_scatter(slots)                       # the leaf states live in the pool
    push = torch.tensor(batch.push.astype(np.float32), device=dev).contiguous()
    target = torch.zeros(E, dtype=torch.int32, device=dev)
    rew = torch.empty(E, dtype=torch.float32, device=dev)
    clr = torch.empty(E, dtype=torch.float32, device=dev)
    stream = sim.stream

    def one_step(k_ev=None):
        sim.pool_gather(slots)
        if k_ev is not None:
            k_ev[0].record(stream)
        sim.step(push, args.substeps)
        if k_ev is not None:
            k_ev[1].record(stream)
        sim.eval_reward(target, 0.08, rew, clr, sync=False)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        one_step(kev[k])
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    kernel_ms = [a.elapsed_time(b) for a, b in kev]   # the whole step call: cost pass, order, step kernel
    k_avg_ms = float(np.mean(kernel_ms))

    status = sim.env_status()
    stats = sim.stats().astype(np.float64)[:, :2]
    n_valid = int(np.sum((status & pmbs.PMBS_ENV_PUSH_INVALID) == 0))
    # push mix: a valid push that moved some box by more than 1 mm touched it
    after = sim.get_state()
    moved = np.linalg.norm(after[:, :3] - batch.state[:, :3].astype(np.float32), axis=1) > 1e-3
    n_touch = int(np.add.reduceat(moved.astype(np.int64), batch.env_offset[:-1]).astype(bool).sum())
    n_overflow = int(np.sum((status & pmbs.PMBS_ENV_CONTACT_OVERFLOW) != 0))
    if np.any(status & (pmbs.PMBS_ENV_NONFINITE | pmbs.PMBS_ENV_CONTACT_OVERFLOW)):
        print("# warning: non-finite or overflowing environments", file=sys.stderr)
    env_substeps = E * args.substeps
    nc = stats[:, 0].sum() / env_substeps
    npairs = stats[:, 1].sum() / env_substeps
    nb = N / E
    iters = int(sim.cfg.solver_iters)
    f_unit = flops_per_env_substep(nc, npairs, nb, iters)
    flops_launch = f_unit * env_substeps
    achieved_tflops = flops_launch / (k_avg_ms * 1e-3) / 1e12
    f_counted = flops_counted(nc, npairs, nb, iters)
    bytes_launch = hbm_bytes_per_call(N, E)
    achieved_gbs = bytes_launch / (k_avg_ms * 1e-3) / 1e9

    # plain copy for counter calibration (outside the timed region)
    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms_per_step = total_ms / args.steps
    value = env_substeps * args.steps / (total_ms * 1e-3)
    peaks = pmbs.measure_peaks() if args.peaks else None
    configs1 = batched_1024(pmbs, scenes, args) if args.small_envs > 0 else None
    out = {
        "metric": "env-substeps/sec (4096 envs x 15 boxes) + %HBM peak; p50/p99 MCTS plan latency",
        "value": round(value, 1),
        "unit": "env-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{E} envs x {args.bodies} cuboids, one 5 cm circle push each "
                        f"({args.substeps} substeps of 1/240 s, {iters} Jacobi iterations); "
                        "step = pool gather + fused push step + reward",
            "envs": E, "bodies_per_env": args.bodies, "substeps": args.substeps,
            "solver_iters": iters, "seed": args.seed, "valid_pushes": n_valid,
            "max_contacts": int(sim.cfg.max_contacts), "overflow_envs": n_overflow,
            "push_mix": {"discarded": E - n_valid, "valid_touching": n_touch, "valid_missing": n_valid - n_touch},
        },
        "roofline": {
            "kernel": "step_kernel",
            "bound": "alu",
            "achieved": round(achieved_tflops, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 5),
            "traffic": measured_traffic(E, args.bodies, args.substeps),
            "kernel_ms": round(k_avg_ms, 4),
            "flop_per_env_substep": round(f_unit, 1),
            "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": round(achieved_tflops / PEAK_FP32_NONPACKED_TFLOPS, 5),
            "measured_fma_peak": peaks["fma_tflops"] if peaks else None,
            "frac_measured_peak": round(achieved_tflops / peaks["fma_tflops"], 5) if peaks else None,
            "flop_per_env_substep_counted": round(f_counted, 1),
            "contacts_per_env_substep": round(nc, 3),
            "pairs_per_env_substep": round(npairs, 3),
        },
        "hbm": {
            "algorithmic_bytes_per_launch": bytes_launch,
            "achieved": round(achieved_gbs, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / PEAK_HBM_GBS, 6),
            "measured_copy_peak": peaks["copy_gbs"] if peaks else None,
        },
    }
    if peaks:
        out["peaks"] = peaks
    if configs1:
        out["batched_1024"] = configs1

    if args.plan_scenes > 0:
        out["plan"] = plan_latency(pmbs, scenes, args)
    if args.uneven_envs > 0:
        out["uneven"] = uneven_batching(pmbs, scenes, args)
    if args.serve_requests > 0:
        out["serving"] = serving(pmbs, scenes, args)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        th = cpu_threads()
        cfg = O.make_config()
        st = batch.state.astype(np.float32).astype(np.float64)
        bd = batch.body.astype(np.float32).astype(np.float64)
        ps = batch.push.astype(np.float32).astype(np.float64)
        t1 = time.perf_counter()
        O.step(cfg, batch.env_offset, st, bd, ps, args.substeps, n_threads=th)
        dt = time.perf_counter() - t1
        # one host thread on the first 256 envs (envs are independent)
        n1 = min(256, E)
        o1 = int(batch.env_offset[n1])
        t2 = time.perf_counter()
        O.step(cfg, batch.env_offset[:n1 + 1], st[:o1], bd[:o1], ps[:n1], args.substeps, n_threads=1)
        dt1 = time.perf_counter() - t2
        out["cpu_baseline"] = {
            "value": round(env_substeps / dt, 1),
            "unit": "env-substeps/s",
            "cores": th,
            "kind": "oracle",
            "sample": f"the full workload once ({E} envs x {args.bodies} cuboids, one {args.substeps}-substep "
                      f"push each) in the FP64 oracle on {th} host threads, {dt:.2f} s wall",
            "single_core": {"value": round(n1 * args.substeps / dt1, 1), "unit": "env-substeps/s",
                            "sample": f"the first {n1} envs on 1 host thread, {dt1:.2f} s wall"},
        }

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
