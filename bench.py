#!/usr/bin/env python3
"""Benchmark of the F.A.S.T. planning phase on one MI355X.

Headline workload: the 400 x 400 room with 40,000 agents at v_m = 4,
k_S = 1.2, k_other = 0 (paper Sec. 2 parameters; the paper times 396 steps of
40,000 agents).  A step is one planning phase plus one motion phase; the
`warmup` first steps of the run are untimed, the next `steps` are timed (the
defaults cover the paper's 396 steps).  `value` is planning agent-updates/s:
agents planned over the timed steps divided by the summed duration of the
planning kernel, recorded by HIP events that the kernel launch itself stamps
at the kernel's start and end (the interval a kernel trace reports).  Events
recorded on the stream around each launch, which add the dispatch latency,
give the `_bracketed` figures; `ms_per_step` is the whole step (plan + move).
Events cost the stream time of their own, so the room runs three times
from the same seed (the same trajectory step for step, which is checked):
run 1 times the whole steps with nothing recorded between the launches,
run 2 takes the kernel stamps (events created without the system-scope
fence, which otherwise writes back and invalidates the caches and slows the
next launch), run 3 the bracketing events.

Also printed on the same JSON line:
  roofline      the planning kernel's algorithmic bytes per launch (5 B per
                cell inside some agent's reach window: occupancy 1 B + exp
                table 4 B; 12 B per agent: position 8 B + desired cell 4 B)
                over its average kernel duration, against 8 TB/s of HBM;
                `traffic` is the HBM bytes per launch measured with hardware
                counters (profiles/plan_traffic.json), or null when the
                planning sources have changed since it was measured.
  large         the same for 16 scenarios of 1000 x 1000 cells (200,000
                agents each) planned in one launch, the throughput regime.
  ensemble      the 256-scenario ensemble workload run as one batch (one
                planning and one motion launch per step, replayed from a HIP
                graph), scenario-steps/s, next to the same scenarios stepped
                one at a time with plain launches.
  serving       the continuous-batching server on Poisson arrivals: p50 / p99
                latency and scenarios/s, open and closed loop.
  cpu_baseline  the CPU oracle's threaded planning loop (chunks as in the paper)
                on the host's cores, on the first steps of the same run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PLAN_SOURCES = ("paper_0911_2900_amd/csrc/plan_tile.h", "paper_0911_2900_amd/csrc/plan_one.hip",
                "paper_0911_2900_amd/csrc/plan_batch.hip", "paper_0911_2900_amd/csrc/plan_fixed.hip",
                "paper_0911_2900_amd/csrc/fast_dev.h")


def plan_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in PLAN_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per planning launch from the hardware counters summarised in
    profiles/plan_traffic.json, or None if that file is missing or was taken
    on other planning sources than these."""
    path = os.path.join(ROOT, "profiles", "plan_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("plan_sources_sha256") != plan_sources_digest() or workload not in t:
        return None
    return t[workload]["hbm_bytes_per_launch"]


def window_cells(cell_type: np.ndarray, xy: np.ndarray, v: int) -> int:
    """Cells of the grid inside the reach disc of at least one agent (the
    planning phase's algorithmic footprint)."""
    from scipy.ndimage import binary_dilation

    H, W = cell_type.shape
    occ = np.zeros((H, W), dtype=bool)
    occ[xy[:, 1], xy[:, 0]] = True
    yy, xx = np.mgrid[-v:v + 1, -v:v + 1]
    disc = xx * xx + yy * yy <= v * v
    return int(binary_dilation(occ, structure=disc).sum())


def bench_room(ctx, torch, warmup: int, steps: int, v: int = 4, n_agents: int = 40000,
               agent_v=None, scenario=None, trail=None):
    from paper_0911_2900_amd import scenarios as sc

    s = sc.room(v=v, n_agents=n_agents) if scenario is None else scenario

    def start():
        if agent_v is None and trail is None:
            h = ctx.init_from(s)
        else:
            h = ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn,
                                  agent_v=agent_v, trail=trail)
        for _ in range(warmup):
            ctx.plan(h)
            ctx.move(h)
        return h

    stream = ctx.stream
    # run 1: the whole steps, nothing recorded between the launches
    h1 = start()
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(stream)
    for _ in range(steps):
        ctx.plan(h1)
        ctx.move(h1)
    e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e_start.elapsed_time(e_end)
    # run 2: the same steps of the same scenario, each planning launch stamped
    h = start()
    st = ctx.state(h)
    alive = st["alive"].astype(bool)
    cells = window_cells(s.cell_type, st["xy"][alive], v)
    planned0 = ctx.stats(h)["planned"]
    torch.cuda.synchronize()
    ctx.timing_start(steps)
    for _ in range(steps):
        ctx.plan(h)
        ctx.move(h)
    torch.cuda.synchronize()
    kernel_ms = ctx.timing_read()
    assert len(kernel_ms) == steps
    stt = ctx.stats(h)
    planned = stt["planned"] - planned0
    # run 3: the same again, events recorded on the stream around each launch
    h3 = start()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        ctx.plan(h3)
        ev[k][1].record(stream)
        ctx.move(h3)
    torch.cuda.synchronize()
    bracket_ms = [a.elapsed_time(b) for a, b in ev]
    s1 = ctx.state(h1)
    for other in (h, h3):
        so = ctx.state(other)
        assert np.array_equal(s1["xy"], so["xy"]) and np.array_equal(s1["alive"], so["alive"]), \
            "the runs of the room diverged"
    res = {
        "planned": planned, "plan_ms": [float(x) for x in kernel_ms], "bracket_ms": bracket_ms,
        "total_ms": total_ms, "wall_s": wall, "cells": cells, "stats": stt, "handle": h,
    }
    for x in (h1, h, h3):
        ctx.destroy(x)
    return res


def bench_ensemble(ctx, torch, warmup: int, steps: int, plain_steps: int):
    from paper_0911_2900_amd import scenarios as sc

    ens = sc.ensemble(256)
    t0 = time.perf_counter()
    hs = [ctx.init_from(m, batched=True) for m in ens]
    init_s = time.perf_counter() - t0
    ctx.run(hs, warmup)                    # the first step also captures the step graph
    planned0 = sum(ctx.stats(h)["planned"] for h in hs)
    stream = ctx.stream
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    ctx.run(hs, steps)
    b.record(stream)
    torch.cuda.synchronize()
    batched_ms = a.elapsed_time(b)
    planned = sum(ctx.stats(h)["planned"] for h in hs) - planned0
    # the same scenarios, one at a time, with plain (non-graph) launches
    a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a2.record(stream)
    for _ in range(plain_steps):
        for h in hs:
            ctx.plan(h)
            ctx.move(h)
    b2.record(stream)
    torch.cuda.synchronize()
    plain_ms = a2.elapsed_time(b2)
    for h in hs:
        ctx.destroy(h)
    n = len(hs)
    return {
        "workload": "ensemble: 256 scenarios, grids 30..300 cells a side, 0-15 % pillars, "
                    "1-4 exits, 50-20,000 agents each, v_m 1..5",
        "scenarios": n, "cells": int(sum(m.W * m.H for m in ens)),
        "agents": int(sum(m.n_agents for m in ens)),
        "steps": steps,
        "timed_steps": f"{warmup}..{warmup + steps - 1} of each scenario's 396-step run "
                       f"(steps 0..{warmup - 1} untimed: graph capture and warmup)",
        "plain_loop_timed_steps": f"{warmup + steps}..{warmup + steps + plain_steps - 1}",
        "batched_scenario_steps_per_s": n * steps / (batched_ms / 1e3),
        "batched_agent_updates_per_s": planned / (batched_ms / 1e3),
        "plain_loop_scenario_steps_per_s": n * plain_steps / (plain_ms / 1e3),
        "batched_over_plain": (n * steps / batched_ms) / (n * plain_steps / plain_ms),
        "ms_per_batched_step": batched_ms / steps,
        "init_s": init_s,
    }


def bench_batch_plan(ctx, torch, scenarios, name: str, warmup: int, steps: int,
                     traffic_key: str = ""):
    """Planning kernel of many scenarios in one launch (fast_plan_batch), the
    throughput regime: kernel-stamped events on each launch over the timed
    steps, motion between them; then as many steps again with events
    recorded around each launch (the bracketed figure)."""
    t0 = time.perf_counter()
    hs = [ctx.init_from(m, batched=True) for m in scenarios]
    init_s = time.perf_counter() - t0
    tile = [ctx.stats(hs[0])["tile_w"], ctx.stats(hs[0])["tile_h"]]
    uniform = all(m.v == scenarios[0].v for m in scenarios) and all(
        [ctx.stats(h)["tile_w"], ctx.stats(h)["tile_h"]] == tile for h in hs)
    kernel = f"plan_kernel_fixed<{scenarios[0].v}, {tile[0]}>" if uniform else "plan_kernel"
    for _ in range(warmup):
        ctx.plan_batch(hs)
        ctx.move_batch(hs)
    cells = 0
    for m, h in zip(scenarios, hs):
        st = ctx.state(h)
        cells += window_cells(m.cell_type, st["xy"][st["alive"].astype(bool)], m.v)
    planned0 = sum(ctx.stats(h)["planned"] for h in hs)
    stream = ctx.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    ctx.timing_start(steps)
    for _ in range(steps):
        ctx.plan_batch(hs)
        ctx.move_batch(hs)
    torch.cuda.synchronize()
    plan_ms = [float(x) for x in ctx.timing_read()]
    assert len(plan_ms) == steps
    planned = sum(ctx.stats(h)["planned"] for h in hs) - planned0
    for k in range(steps):
        ev[k][0].record(stream)
        ctx.plan_batch(hs)
        ev[k][1].record(stream)
        ctx.move_batch(hs)
    torch.cuda.synchronize()
    bracket_ms = [a.elapsed_time(b) for a, b in ev]
    for h in hs:
        ctx.destroy(h)
    avg_ms = float(np.mean(plan_ms))
    bytes_per_launch = 5.0 * cells + 12.0 * planned / steps
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    return {
        "workload": name, "scenarios": len(scenarios), "agents": int(sum(m.n_agents for m in scenarios)),
        "tile": tile,
        "planning_agent_updates_per_s": planned / (sum(plan_ms) / 1e3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_key),
                     "kernel": kernel,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_ms * 1e3},
        "plan_us_bracketed": float(np.mean(bracket_ms)) * 1e3,
        "init_s": init_s,
    }


def bench_serving(fast, n_req: int, rate: float, steps: int = 396, plain_sample: int = 16,
                  small_budget_mb: int = 64):
    """Continuous-batching server on Poisson arrivals (mean `rate` requests/s)
    of scenarios drawn from the ensemble distribution (scenario ids 1000 + k),
    `steps` steps each: an open-loop run whose budget admits everything, an
    open-loop run on a quarter of the requests with a small forced budget so
    admission binds, and a closed-loop run (all submitted at once) on half of
    them for the saturation rate; next to the same requests run one at a time
    with plain single-scenario launches (on a sample)."""
    from paper_0911_2900_amd import scenarios as sc

    t0 = time.perf_counter()
    reqs = [sc.ensemble_member(k, base_seed=4, scn_base=1000) for k in range(n_req)]
    gen_s = time.perf_counter() - t0
    gaps = np.random.default_rng([4, 1]).exponential(1.0 / rate, n_req)

    def run(members, budget, closed):
        ctx = fast.Context(device=0, torch_alloc=False)
        try:
            ctx.serve_start(budget=budget)
            arrive = np.zeros(len(members)) if closed else np.cumsum(gaps[: len(members)])
            tickets = []
            t_start = time.perf_counter()
            for m, ta in zip(members, arrive):
                dt = t_start + ta - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets.append(ctx.serve_submit(m.cell_type, m.n_agents, m.v, m.k_s, m.seed,
                                                m.scn, steps=steps))
            ctx.serve_stop()                  # returns once every request has finished
            wall = time.perf_counter() - t_start
            lat = np.array([ctx.serve_poll(t)[1] for t in tickets])
        finally:
            ctx.close()
        return {"requests": len(members), "wall_s": wall,
                "scenarios_per_s": len(members) / wall,
                "agent_steps_per_s": sum(m.n_agents for m in members) * steps / wall,
                "latency_p50_s": float(np.percentile(lat, 50)),
                "latency_p99_s": float(np.percentile(lat, 99)),
                "latency_max_s": float(lat.max())}

    log(f"serving: open loop, {n_req} requests at {rate}/s ...")
    open_loop = run(reqs, 0, False)
    log(f"serving: {open_loop}")
    nb = max(1, n_req // 4)
    log(f"serving: open loop, {nb} requests, {small_budget_mb} MB budget ...")
    small = run(reqs[:nb], small_budget_mb << 20, False)
    log(f"serving: {small}")
    nc = max(1, n_req // 2)
    log(f"serving: closed loop, {nc} requests ...")
    closed = run(reqs[:nc], 0, True)
    log(f"serving: {closed}")
    # the plain single-scenario loop, one request after another
    ctx = fast.Context(device=0, torch_alloc=False)
    t_p = time.perf_counter()
    for m in reqs[:plain_sample]:
        h = ctx.init_from(m, tile="auto")
        for _ in range(steps):
            ctx.plan(h)
            ctx.move(h)
        ctx.state(h)
        ctx.destroy(h)
    plain_s = time.perf_counter() - t_p
    ctx.close()
    plain_rate = plain_sample / plain_s
    return {
        "workload": f"Poisson arrivals, mean {rate:g}/s, of ensemble-distribution scenarios "
                    f"(ids 1000+k), {steps} steps each",
        "open_loop": open_loop, "small_budget": dict(small, budget_mb=small_budget_mb),
        "closed_loop": closed,
        "plain_one_at_a_time_scenarios_per_s": plain_rate, "plain_sample": plain_sample,
        "closed_over_plain": closed["scenarios_per_s"] / plain_rate,
        "request_generation_s": gen_s,
    }


def cpu_baseline(budget_s: float = 15.0, max_steps: int = 396, v: int = 4):
    """The oracle as it stands: its threaded planning loop (threads claim
    chunks of N / threads agents, at most 32767, as in paper Sec. 2) on every
    host thread, sequential motion, on the room workload."""
    import oracle
    from paper_0911_2900_amd import scenarios as sc

    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    s = sc.room(v=v)
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    planned, plan_s, steps = 0, 0.0, 0
    t_all = time.perf_counter()
    while steps < max_steps and time.perf_counter() - t_all < budget_s:
        n = sim.n_alive()
        t0 = time.perf_counter()
        sim.plan_threads(cores)
        plan_s += time.perf_counter() - t0
        planned += n
        sim.move()
        sim.end_step()
        steps += 1
    return {
        "value": planned / plan_s, "unit": "agent-updates/s", "cores": cores, "kind": "oracle",
        "sample": f"first {steps} steps of the 400x400 room, 40,000 agents, v_m={v}: FP64 "
                  f"planning loop, threads claiming chunks of max(min(N/threads, 32767), 1) "
                  f"agents, on {cores} threads (timed), sequential motion (untimed)",
        "whole_steps_s": time.perf_counter() - t_all,
    }


def sweep_v(ctx, torch, warmup: int, steps: int):
    """The room at v_m = 1..5 (40,000 agents): planning agent-updates/s from
    the kernel times, and the whole step."""
    out = []
    from paper_0911_2900_amd import scenarios as sc

    for v in (1, 2, 3, 4, 5):
        r = bench_room(ctx, torch, warmup, steps, v=v)
        out.append({"v_m": v, "planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                    "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                    "whole_step_us": r["total_ms"] / steps * 1e3,
                    "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]],
                    "flagged_per_step": r["stats"]["flagged"] / (warmup + steps)})
        log(f"v_m={v}: {out[-1]}")
    return out


def sweep_n(ctx, torch, warmup: int, steps: int):
    """The room at v_m = 4 with 5,000 .. 150,000 agents (160,000 would exceed
    its 158,404 free interior cells): planning agent-updates/s and the whole
    step."""
    out = []
    for n in (5000, 10000, 20000, 40000, 80000, 150000):
        r = bench_room(ctx, torch, warmup, steps, v=4, n_agents=n)
        out.append({"agents": n, "planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                    "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                    "whole_step_us": r["total_ms"] / steps * 1e3,
                    "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]]})
        log(f"N={n}: {out[-1]}")
    return out


def sweep_cu(torch, warmup: int, steps: int, cus=(8, 16, 32, 64, 128, 256),
             agents=(10000, 40000, 150000), batch: bool = True):
    """The room at v_m = 4 with 10,000 / 40,000 / 150,000 agents on streams
    confined to 8 .. 256 CUs (n / 8 on each XCD): how planning and the whole
    step speed up with more of the chip, the counterpart of the paper's speed
    factor over the number of cores (Sec. 3).  A batched planning launch of
    16 rooms (640,000 agents) shows the same with enough tiles to fill every
    CU.  Speed-ups are relative to the fewest CUs timed (8 by default)."""
    from paper_0911_2900_amd import fast
    from paper_0911_2900_amd import scenarios as sc

    rooms = [sc.room(v=4, scn=k) for k in range(16)] if batch else []
    out = []
    for n_cu in cus:
        cs = fast.CUStream(n_cu)
        log(f"{n_cu} CUs: probe reached {cs.n_cus_run}, per XCD {cs.per_xcd}")
        ctx = fast.Context(stream=cs.torch)
        try:
            for n in agents:
                r = bench_room(ctx, torch, warmup, steps, v=4, n_agents=n)
                out.append({"cus": n_cu, "cus_reached": cs.n_cus_run, "ctx_cus": ctx.cus(),
                            "agents": n,
                            "planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                            "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                            "whole_step_us": r["total_ms"] / steps * 1e3})
                log(f"{n_cu} CUs, N={n}: {out[-1]}")
            if not batch:
                continue
            r = bench_batch_plan(ctx, torch, rooms, "16 x room", 2, steps)
            out.append({"cus": n_cu, "cus_reached": cs.n_cus_run, "ctx_cus": ctx.cus(),
                        "agents": r["agents"], "batch": "16 rooms, one planning launch",
                        "planning_agent_updates_per_s": r["planning_agent_updates_per_s"],
                        "plan_us": r["roofline"]["avg_launch_us"], "whole_step_us": None})
            log(f"{n_cu} CUs, 16 rooms: {out[-1]}")
        finally:
            ctx.close()
            cs.close()
    base = {o["agents"]: o for o in out if o["cus"] == min(cus)}
    for o in out:
        b = base[o["agents"]]
        o["plan_speedup_vs_8"] = b["plan_us"] / o["plan_us"]
        if o["whole_step_us"] is not None:
            o["step_speedup_vs_8"] = b["whole_step_us"] / o["whole_step_us"]
    return out


def bench_fd(ctx, torch, steps: int = 396, per_density: int = 16):
    """Fundamental-diagram ensemble: the corridor at 11 initial densities
    (0.5 .. 5.5 P/m^2) x per_density seeds, all run together as one
    graph-replayed batch for `steps` steps.  Timed twice over steps 2 ..
    `steps` (the first step captures the graph): without region counts, and
    with the measurement area's and the upstream region's counts recorded
    after every step.  The counted run gives the diagram, binned by density,
    with Weidmann's published fit beside it as context.  Then, untimed,
    bottleneck corridors (exits of 1 or 2 of the 10 cells) sample the
    congested branch that the open corridors never reach."""
    from paper_0911_2900_amd import fd
    from paper_0911_2900_amd import scenarios as sc

    members = sc.fd_ensemble(per_density=per_density)
    out = {"workload": f"{len(members)} corridors 100x10 cells, v_m=4, {steps} steps, batched",
           "scenarios": len(members), "agents": int(sum(m.n_agents for m in members))}
    rho_all, flow_all = [], []
    for counted in (False, True):
        hs = [ctx.init_scenario(m.cell_type, 0, m.v, m.k_s, m.seed, m.scn,
                                agent_xy=m.meta["agent_xy"], tile="auto", batched=True)
              for m in members]
        if counted:
            for m, h in zip(members, hs):
                ctx.set_regions(h, [m.meta["area"], m.meta["upstream"]], steps)
        ctx.run(hs, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.run(hs, steps - 1)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        key = "counted" if counted else "plain"
        out[key] = {"ms_per_step": ms / (steps - 1),
                    "scenario_steps_per_s": len(hs) * (steps - 1) / (ms / 1e3)}
        if counted:
            for m, h in zip(members, hs):
                rho, flow = fd.samples(ctx.regions(h), m.meta["area_m2"], m.meta["width_m"])
                rho_all.append(rho)
                flow_all.append(flow)
        exited = sum(ctx.stats(h)["exited"] for h in hs)
        out[key]["exited"] = int(exited)
        out["tile"] = [ctx.stats(hs[0])["tile_w"], ctx.stats(hs[0])["tile_h"]]
        for h in hs:
            ctx.destroy(h)
        log(f"fd {key}: {out[key]}")
    out["count_overhead"] = out["counted"]["ms_per_step"] / out["plain"]["ms_per_step"] - 1.0
    bins = fd.diagram(np.concatenate(rho_all), np.concatenate(flow_all))
    for b in bins:
        b["weidmann_flow"] = float(fd.weidmann_flow(np.array([b["rho_mean"]]))[0])
    out["diagram"] = bins
    if bins:
        top = max(bins, key=lambda b: b["flow_mean"])
        out["capacity"] = {"flow": top["flow_mean"], "at_density": top["rho_mean"]}
    # The congested branch: bottleneck corridors, whose queue covers the
    # measurement area; there the flow across the line is the bottleneck's
    # outflow and the density that of the queue.
    bm = sc.fd_bottleneck_ensemble()
    hs = [ctx.init_scenario(m.cell_type, 0, m.v, m.k_s, m.seed, m.scn, agent_xy=m.meta["agent_xy"],
                            tile="auto", batched=True) for m in bm]
    for m, h in zip(bm, hs):
        ctx.set_regions(h, [m.meta["area"], m.meta["upstream"]], steps)
    ctx.run(hs, steps)
    per_width, rho_b, flow_b = {}, [], []
    for m, h in zip(bm, hs):
        rho, flow = fd.samples(ctx.regions(h), m.meta["area_m2"], m.meta["width_m"])
        rho_b.append(rho)
        flow_b.append(flow)
        w = per_width.setdefault(m.meta["exit_cells"], [[], []])
        w[0].append(rho)
        w[1].append(flow)
    for h in hs:
        ctx.destroy(h)
    bins_b = fd.diagram(np.concatenate(rho_b), np.concatenate(flow_b))
    for b in bins_b:
        b["weidmann_flow"] = float(fd.weidmann_flow(np.array([b["rho_mean"]]))[0])
    out["bottleneck"] = {
        "workload": f"{len(bm)} corridors 100x10 cells with exits of 1 or 2 cells, "
                    f"initial 4/5/6 P/m^2, measurement area x = 81..90, {steps} steps",
        "scenarios": len(bm),
        "by_exit_width": [{"exit_cells": w, "exit_m": 0.4 * w,
                           "rho_mean": float(np.concatenate(v[0]).mean()),
                           "flow_mean": float(np.concatenate(v[1]).mean()),
                           "samples": int(sum(len(x) for x in v[0]))}
                          for w, v in sorted(per_width.items())],
        "diagram": bins_b,
    }
    log(f"fd bottleneck: {out['bottleneck']['by_exit_width']}")
    return out


def bench_het(ctx, torch, warmup: int, steps: int):
    """The room (40,000 agents) with a maximum speed per agent drawn
    uniformly from 1..5 (v_max = 5), on the FP32 table path with each agent's
    own disc.  Beside it the same room with v_m = 5 for everybody."""
    vi = np.random.default_rng(11).integers(1, 6, size=40000)
    out = {}
    for key, av in (("per_agent_speeds", vi), ("uniform_v5", None)):
        r = bench_room(ctx, torch, warmup, steps, v=5, agent_v=av)
        out[key] = {"planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                    "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                    "whole_step_us": r["total_ms"] / steps * 1e3,
                    "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]],
                    "fp64_draws_per_step": r["stats"]["fallback"] / (warmup + steps)}
        log(f"het {key}: {out[key]}")
    out["workload"] = "room 400x400, 40,000 agents, speeds U{1..5} (v_max = 5)"
    return out


def bench_fields(ctx, torch, warmup: int, steps: int):
    """A 400 x 400 counterflow hall, 40,000 agents at v_m = 4 in two groups,
    each following the floor field of its own exits (left or right wall),
    on the FP32 table path with one exp table per field.  Beside it the
    400 x 400 room with one exit and one field."""
    from paper_0911_2900_amd import scenarios as sc

    out = {}
    for key, scn in (("two_fields", sc.counterflow(n_agents=40000, v=4, W=400, H=400)),
                     ("one_field_room", None)):
        r = bench_room(ctx, torch, warmup, steps, v=4, scenario=scn)
        out[key] = {"planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                    "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                    "whole_step_us": r["total_ms"] / steps * 1e3,
                    "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]],
                    "exited": r["stats"]["exited"],
                    "fp64_draws_per_step": r["stats"]["fallback"] / (warmup + steps)}
        log(f"fields {key}: {out[key]}")
    out["workload"] = ("counterflow hall 400x400, exits 4 cells on the left and right walls, "
                       "40,000 agents in two even groups, v_m=4, k_S=1.2")
    return out


def bench_trail(ctx, torch, warmup: int, steps: int):
    """The room (40,000 agents, v_m = 4) with a dynamic floor field (a trail
    that departing agents leave, decayed and diffused after every motion
    phase, weighted by exp(k_D (T(t) - T(c)))), beside the plain room.  The
    whole step includes the two launches that update the trail and rebuild
    the exp table."""
    out = {}
    for key, tr in (("trail", (1.0, 0.3, 0.2)), ("plain_room", None)):
        r = bench_room(ctx, torch, warmup, steps, v=4, trail=tr)
        out[key] = {"planning_agent_updates_per_s": r["planned"] / (sum(r["plan_ms"]) / 1e3),
                    "plan_us": float(np.mean(r["plan_ms"])) * 1e3,
                    "whole_step_us": r["total_ms"] / steps * 1e3,
                    "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]],
                    "exited": r["stats"]["exited"],
                    "fp64_draws_per_step": r["stats"]["fallback"] / (warmup + steps),
                    "flagged_per_step": r["stats"]["flagged"] / (warmup + steps)}
        log(f"trail {key}: {out[key]}")
    out["workload"] = ("room 400x400, 40,000 agents, v_m=4, k_S=1.2, trail k_D=1, decay 0.3, "
                       "diffusion 0.2")
    return out


def achievable(ctx, achieved_gbs: float, footprint: float, stream_4g: float) -> dict:
    """The planning launch's algorithmic rate against what the streaming
    kernel reaches beyond the cache (4 GiB) and at the launch's own
    footprint (cache-resident)."""
    same, same_us = ctx.stream_bandwidth(int(footprint), 50)
    return {"stream_4GiB_GBs": stream_4g, "stream_same_footprint_GBs": same,
            "stream_same_footprint_us": same_us,
            "frac_of_stream_4GiB": achieved_gbs / stream_4g,
            "frac_of_stream_same_footprint": achieved_gbs / same}


def cpu_table(budget_steps: int = 5):
    """The oracle on the host: one thread, and its threaded planning loop on
    every host thread, per workload (planning agent-updates/s and whole steps
    per second; the room, ensemble and 1000 x 1000 rows time the first
    `budget_steps` steps, the corridor its full 396)."""
    import oracle
    from paper_0911_2900_amd import scenarios as sc

    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    rows = []

    def time_sim(name, members, steps, extrapolate=1.0):
        for threads in (1, cores):
            sims = [oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents) for m in members]
            planned, plan_s, t0 = 0, 0.0, time.perf_counter()
            for _ in range(steps):
                for sim in sims:
                    n = sim.n_alive()
                    t1 = time.perf_counter()
                    if threads == 1:
                        sim.plan()
                    else:
                        sim.plan_threads(threads)
                    plan_s += time.perf_counter() - t1
                    planned += n
                    sim.move()
                    sim.end_step()
            whole = time.perf_counter() - t0
            rows.append({"workload": name, "threads": threads, "steps": steps,
                         "planning_agent_updates_per_s": planned / plan_s,
                         "whole_steps_per_s": steps / whole / extrapolate,
                         "extrapolated_from": f"{len(members)} of {int(len(members) * extrapolate)} "
                                              "scenarios" if extrapolate != 1.0 else None})
            log(rows[-1])

    time_sim("corridor 60x25, 200 agents, v_m=4", [sc.corridor()], 396)
    for v in (1, 2, 3, 4, 5):
        time_sim(f"room 400x400, 40,000 agents, v_m={v}", [sc.room(v=v)], budget_steps)
    time_sim("ensemble, 256 scenarios", sc.ensemble(256), budget_steps)
    time_sim("16 x 1000x1000, 200,000 agents each", [sc.large_member(0)], budget_steps, 16.0)
    return {"cores": cores, "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=386)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--ensemble-steps", type=int, default=395,
                    help="batched ensemble steps timed after one untimed step (395: the rest "
                         "of the 396-step run)")
    ap.add_argument("--plain-steps", type=int, default=4)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 5 times (the reference "
                         "kernel for scaling the HBM traffic counters) and exit")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--room-replicas", type=int, default=64,
                    help="also time the planning launch over this many copies of the room")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests in the open-loop serving run (0 = no serving run)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--sweep-n", action="store_true",
                    help="only the room at v_m = 4 with 5k .. 150k agents")
    ap.add_argument("--sweep-v", action="store_true",
                    help="only time the room at v_m = 1..5 and print one JSON line")
    ap.add_argument("--sweep-cu", action="store_true",
                    help="only the room at v_m = 4 (10k / 40k / 150k agents) and a 16-room "
                         "planning launch on 8 .. 256 CUs")
    ap.add_argument("--cus", default="8,16,32,64,128,256",
                    help="--sweep-cu: CU counts (multiples of 8), comma-separated")
    ap.add_argument("--sweep-agents", default="10000,40000,150000",
                    help="--sweep-cu: room agent counts, comma-separated (empty: none)")
    ap.add_argument("--het", action="store_true",
                    help="only the room with a maximum speed per agent (FP64 planning path)")
    ap.add_argument("--fields", action="store_true",
                    help="only the counterflow hall with a floor field per exit group "
                         "(FP64 planning path)")
    ap.add_argument("--trail", action="store_true",
                    help="only the room with a dynamic floor field (trail) beside the plain room")
    ap.add_argument("--no-fd", action="store_true",
                    help="leave the fundamental-diagram ensemble out of the default run")
    ap.add_argument("--fd", action="store_true",
                    help="only the fundamental-diagram ensemble (176 corridors, region counts)")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the oracle on the host (one thread and all threads) per "
                         "workload and print one JSON line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs each scenario on a single MI355X and "
              "has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.cpu_table:
        print(json.dumps(cpu_table()), flush=True)
        return
    import torch
    from paper_0911_2900_amd import fast

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * 1024 * 1024
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n} bytes 5 times")
        return
    if args.sweep_cu:
        cus = [int(x) for x in args.cus.split(",") if x]
        agents = [int(x) for x in args.sweep_agents.split(",") if x]
        print(json.dumps({"sweep_cu": sweep_cu(torch, args.warmup, args.steps, cus, agents,
                                               batch=not args.no_large)}), flush=True)
        return
    ctx = fast.Context(device=0)
    if args.fd:
        print(json.dumps({"fd": bench_fd(ctx, torch)}), flush=True)
        ctx.close()
        return
    if args.het:
        print(json.dumps({"het": bench_het(ctx, torch, args.warmup, args.steps)}), flush=True)
        ctx.close()
        return
    if args.trail:
        print(json.dumps({"trail": bench_trail(ctx, torch, args.warmup, args.steps)}), flush=True)
        ctx.close()
        return
    if args.fields:
        print(json.dumps({"fields": bench_fields(ctx, torch, args.warmup, args.steps)}), flush=True)
        ctx.close()
        return
    if args.sweep_v:
        print(json.dumps({"sweep_v": sweep_v(ctx, torch, args.warmup, args.steps)}), flush=True)
        ctx.close()
        return
    if args.sweep_n:
        print(json.dumps({"sweep_n": sweep_n(ctx, torch, args.warmup, args.steps)}), flush=True)
        ctx.close()
        return
    log(f"room: warmup {args.warmup}, timed {args.steps} steps")
    r = bench_room(ctx, torch, args.warmup, args.steps)
    plan_s = sum(r["plan_ms"]) / 1e3
    value = r["planned"] / plan_s
    avg_plan_ms = float(np.mean(r["plan_ms"]))
    bytes_per_launch = 5.0 * r["cells"] + 12.0 * r["planned"] / args.steps
    achieved = bytes_per_launch / (avg_plan_ms / 1e3) / 1e9
    log(f"room: planning {value:.4g} agent-updates/s, plan {avg_plan_ms * 1e3:.2f} us/step, "
        f"whole step {r['total_ms'] / args.steps * 1e3:.1f} us, stats {r['stats']}")

    large = None
    if not args.no_large:
        from paper_0911_2900_amd import scenarios as sc
        log("large: 16 x 1000x1000, 200,000 agents each ...")
        large = bench_batch_plan(ctx, torch, sc.large(16),
                                 "16 scenarios of 1000x1000 cells, 10 % pillars, 4 exits, "
                                 "200,000 agents each, v_m=4, one planning launch", 2,
                                 args.large_steps, traffic_key="large")
        log(f"large: {large}")
    replicas = None
    if args.room_replicas:
        from paper_0911_2900_amd import scenarios as sc
        rooms = [sc.room(v=4, scn=k) for k in range(args.room_replicas)]
        replicas = bench_batch_plan(ctx, torch, rooms, f"{args.room_replicas} x room 400x400, "
                                    "40,000 agents, v_m=4, one planning launch", 2, args.large_steps)
        log(f"replicas: {replicas}")

    room_ach = None
    if not args.no_stream:
        stream4, _ = ctx.stream_bandwidth(4 << 30, 20)
        log(f"stream kernel, 4 GiB footprint: {stream4:.1f} GB/s")
        room_ach = achievable(ctx, achieved, bytes_per_launch, stream4)
        for x in (large, replicas):
            if x is not None:
                x["roofline"]["achievable"] = achievable(ctx, x["roofline"]["achieved"],
                                                         x["roofline"]["bytes_per_launch"], stream4)
        log(f"achievable: room {room_ach}")

    ens = None
    if not args.no_ensemble:
        log("ensemble ...")
        ens = bench_ensemble(ctx, torch, 1, args.ensemble_steps, args.plain_steps)
        log(f"ensemble: {ens}")
    fdr = None
    if not args.no_fd:
        log("fundamental-diagram ensemble ...")
        f = bench_fd(ctx, torch)
        fdr = {k: f[k] for k in ("workload", "scenarios", "agents", "plain", "counted",
                                 "count_overhead", "capacity") if k in f}
        log(f"fd: {fdr}")
    ctx.close()

    serving = None
    if args.serve_requests:
        serving = bench_serving(fast, args.serve_requests, args.serve_rate)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline ...")
        cpu = cpu_baseline()
        log(f"cpu: {cpu}")

    out = {
        "metric": "planning agent-updates/s (40k agents, v_m=4) + batched ensemble steps/s",
        "value": value,
        "unit": "agent-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["total_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "room 400x400 cells, 10-cell exit, 40,000 agents, v_m=4, k_S=1.2, "
                        f"k_other=0; timed steps {args.warmup}..{args.warmup + args.steps - 1} "
                        f"of a 396-step run (steps 0..{args.warmup - 1} untimed warmup)",
            "agents": 40000, "grid": [400, 400], "v_m": 4, "k_S": 1.2,
            "tile": [r["stats"]["tile_w"], r["stats"]["tile_h"]],
            "parallelism": "1 GPU",
        },
        "whole_step_agent_updates_per_s": r["planned"] / (r["total_ms"] / 1e3),
        "plan_us_per_step": avg_plan_ms * 1e3,
        "plan_us_bracketed": float(np.mean(r["bracket_ms"])) * 1e3,
        "planning_agent_updates_per_s_bracketed": r["planned"] / (sum(r["bracket_ms"]) / 1e3),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("room"),
            "kernel": f"plan_kernel_one_fixed<4, {r['stats']['tile_w']}>",
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": avg_plan_ms * 1e3, "achievable": room_ach,
        },
        "ensemble": ens,
        "fundamental_diagram": fdr,
        "large": large,
        "room_replicas": replicas,
        "serving": serving,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in
                                                 ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
