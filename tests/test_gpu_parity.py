"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bar: desired cells, positions, alive flags and exit counts bit-identical to
the oracle on the same seeded inputs.  Weights, compared as ratios to the
largest weight of the agent's reach set (the draw depends on ratios only),
within 1e-6 relative of the oracle's FP64 ratios wherever the FP64 weight is
at least 2^-60 W; smaller ones may be 0 in FP32 (cross-wall underflow).  The
FP32 CDF over W within half the guard band of the FP64 CDF over W, and every
draw within 1e-6 W of a boundary of its chosen slot re-resolved in FP64.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_2900_amd import fast
    c = fast.Context()
    yield c
    c.close()


def make_pair(ctx, s, tile=None, agent_xy=None):
    if agent_xy is None:
        sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
        h = ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=tile)
    else:
        sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, agent_xy=agent_xy)
        h = ctx.init_scenario(s.cell_type, 0, s.v, s.k_s, s.seed, s.scn, agent_xy=agent_xy, tile=tile)
    st = ctx.state(h)
    assert np.array_equal(st["xy"], sim.positions())
    return sim, h


def compare_state(ctx, sim, h, check_desired=False, where=""):
    st = ctx.state(h)
    n = sim.n
    alive_o = sim.alive[:n].astype(bool)
    assert np.array_equal(st["alive"].astype(bool), alive_o), f"alive differs {where}"
    assert np.array_equal(st["xy"], sim.positions()), f"positions differ {where}"
    assert st["n_active"] == int(alive_o.sum())
    if check_desired:
        d_o = sim.desired[:n]
        bad = np.nonzero(st["desired"][alive_o] != d_o[alive_o])[0]
        assert len(bad) == 0, f"desired differs for {len(bad)} agents {where}: first ids " \
                              f"{np.nonzero(alive_o)[0][bad[:5]]}"
    return st


def step_both(ctx, sim, h, steps, check_every=1, where=""):
    for s in range(steps):
        ctx.plan(h)
        sim.plan()
        if check_every and s % check_every == 0:
            st = ctx.state(h)
            alive = sim.alive[: sim.n].astype(bool)
            bad = np.nonzero(st["desired"][alive] != sim.desired[: sim.n][alive])[0]
            assert len(bad) == 0, f"plan of step {s} differs for {len(bad)} agents {where}"
        ctx.move(h)
        sim.move()
        sim.end_step()
        if check_every and s % check_every == 0:
            compare_state(ctx, sim, h, where=f"after step {s} {where}")
    compare_state(ctx, sim, h, where=f"at the end {where}")


def disc_slots(v):
    side = 2 * v + 1
    dy, dx = np.divmod(np.arange(side * side), side)
    return (dx - v) ** 2 + (dy - v) ** 2 <= v * v


def check_weights(ctx, sim, h, sample=None):
    """One debug plan against the oracle's FP64 draw of every (or `sample`)
    agent.  Returns (worst weight error, worst CDF error over W, flags,
    near-tie draws seen).

    - weights w / max(w) over the reach set: |w32 - w64| <= 1e-6 w64 wherever
      w64 >= 2^-60 W64 (on range-fallback tiles too); below that w32 is at
      most 2^-60 W64 / max(w64);
    - the FP32 CDF over W32 at every disc slot within eps / 2 of the FP64 CDF
      over W64 (eps: the guard band), on every tile with an FP32 CDF;
    - every draw whose FP64 tau lies within 1e-6 W64 of either boundary of its
      chosen slot is flagged (re-resolved in FP64), and the choices agree.
    """
    from paper_0911_2900_amd import fast
    w32, flag, margin, cdf32 = ctx.debug_plan(h)
    sim.plan()
    eps = fast.guard_band(sim.v)
    disc = disc_slots(sim.v)
    alive = np.nonzero(sim.alive[: sim.n])[0]
    ids = alive if sample is None else np.random.default_rng(0).choice(alive, min(sample, len(alive)),
                                                                       replace=False)
    worst_w = worst_c = 0.0
    near = 0
    for i in ids:
        d, w64, C, u, slot = sim.plan_agent(int(i))
        W64 = C[-1]
        wmax = w64.max()
        w = w32[i].astype(np.float64)
        big = w64 >= 2.0 ** -60 * W64
        rel = np.abs(w[big] - w64[big] / wmax) / (w64[big] / wmax)
        worst_w = max(worst_w, float(rel.max()))
        assert rel.max() <= 1e-6, f"agent {i} (flag {flag[i]}): weight rel err {rel.max():.3e}"
        assert np.all(w[~big] <= 2.0 ** -60 * W64 / wmax), f"agent {i}: small weight too large"
        if flag[i] != 2:
            c = cdf32[i].astype(np.float64)
            err = np.abs(c[disc] / c[-1] - C[disc] / W64).max()
            worst_c = max(worst_c, float(err))
            assert err < eps / 2, f"agent {i}: FP32 CDF error {err:.3e} W, band {eps:.3e}"
        tau = u * W64
        lo = C[slot - 1] if slot > 0 else 0.0
        m64 = min(abs(tau - lo), abs(tau - C[slot])) / W64
        if m64 <= 1e-6:
            near += 1
            assert flag[i] in (1, 2), f"agent {i}: tau {m64:.2e} W from a boundary, not flagged"
    st = ctx.state(h)
    a = sim.alive[: sim.n].astype(bool)
    assert np.array_equal(st["desired"][a], sim.desired[: sim.n][a])
    return worst_w, worst_c, flag, near


# ---------------------------------------------------------------------------
# corridor 60 x 25, 200 agents, v_m = 4, 396 steps
# ---------------------------------------------------------------------------

def test_corridor_plan_weights(ctx):
    s = sc.corridor()
    sim, h = make_pair(ctx, s)
    worst, worst_c, flag, near = check_weights(ctx, sim, h)
    say("corridor worst weight rel err", worst, "CDF err", worst_c)
    ctx.move(h)
    sim.move()
    sim.end_step()
    compare_state(ctx, sim, h)
    ctx.destroy(h)


def test_corridor_396_steps_bit_exact(ctx):
    s = sc.corridor()
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 396, check_every=1, where="corridor")
    st = ctx.stats(h)
    say("corridor stats", st)
    assert st["step"] == 396 and st["exited"] == sim.exited
    ctx.destroy(h)


# ---------------------------------------------------------------------------
# room 400 x 400, 40,000 agents
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("v", [1, 2, 3, 4, 5])
def test_room_plan_weights_and_cdf(ctx, v):
    """Weights, the measured FP32 CDF error against the guard band, and the
    near-tie flags on the 400 x 400 room (3,000 sampled agents, two plans)."""
    from paper_0911_2900_amd import fast
    s = sc.room(v=v)
    sim, h = make_pair(ctx, s)
    for k in range(2):
        worst, worst_c, flag, near = check_weights(ctx, sim, h, sample=3000)
        say(f"room v{v} plan {k}: worst weight rel err {worst:.2e}, CDF err {worst_c:.2e} W "
            f"(band {fast.guard_band(v):.2e}), flagged {int((flag == 1).sum())}, near ties {near}")
        ctx.move(h)
        sim.move()
        sim.end_step()
        compare_state(ctx, sim, h, where=f"room v{v} after plan {k}")
    ctx.destroy(h)


def test_near_ties_flagged_k_s_zero(ctx):
    """k_S = 0 makes every weight 1, so the CDF holds small integers and
    u*W lands within 1e-6 W of a boundary for about one draw in 10^4: every
    such draw must be flagged and re-resolved (all 40,000 agents, 3 plans)."""
    s = sc.room(v=4)
    s.k_s = 0.0
    sim, h = make_pair(ctx, s)
    seen = 0
    for k in range(3):
        worst, worst_c, flag, near = check_weights(ctx, sim, h)
        seen += near
        say(f"k_S = 0 plan {k}: near ties {near}, flagged {int((flag == 1).sum())}, CDF err {worst_c:.2e}")
        assert worst_c == 0.0                    # integer sums are exact in FP32
        ctx.move(h)
        sim.move()
        sim.end_step()
    assert seen > 0
    ctx.destroy(h)


def test_room_v4_396_steps_bit_exact(ctx):
    s = sc.room(v=4)
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 396, check_every=11, where="room v4")
    st = ctx.stats(h)
    say("room v4 stats", st)
    assert st["exited"] == sim.exited
    ctx.destroy(h)


@pytest.mark.parametrize("v", [1, 2, 3, 5])
def test_room_other_speeds(ctx, v):
    s = sc.room(v=v)
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 25, check_every=1, where=f"room v{v}")
    ctx.destroy(h)


# ---------------------------------------------------------------------------
# tiles, geometry, fallback tiles, edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", range(12))
def test_random_small_scenarios(ctx, case):
    rng = np.random.default_rng(900 + case)
    v = int(rng.integers(1, 6))
    W, H = int(rng.integers(5, 90)), int(rng.integers(5, 90))
    s = sc.random_small(rng, W, H, float(rng.uniform(0, 0.2)), int(rng.integers(1, 1500)), v,
                        seed=int(rng.integers(0, 2**63)), scn=int(rng.integers(0, 2**31)),
                        n_exits=int(rng.integers(1, 4)))
    tiles = [(8, 8), (16, 8), (8, 16), (16, 16), (32, 16), (32, 32), (64, 16), (16, 64), (64, 8)]
    tile = tiles[case % len(tiles)]
    say(f"case {case}: {W}x{H} v={v} n={s.n_agents} tile={tile}")
    sim, h = make_pair(ctx, s, tile=tile)
    step_both(ctx, sim, h, 30, check_every=1, where=f"case {case}")
    ctx.destroy(h)


@pytest.mark.parametrize("k_s", [0.0, 4.0, 9.0])
def test_extreme_k_s_and_fallback_tiles(ctx, k_s):
    rng = np.random.default_rng(77)
    s = sc.random_small(rng, 70, 50, 0.15, 900, 4, k_s=k_s, seed=5, scn=3, n_exits=2)
    sim, h = make_pair(ctx, s, tile=(32, 32))
    st = ctx.stats(h)
    say("k_s", k_s, "fallback tiles", st["n_fallback_tiles"], "of", st["n_tiles"])
    if k_s >= 4.0:
        assert st["n_fallback_tiles"] > 0
    worst, worst_c, flag, near = check_weights(ctx, sim, h)
    say("k_s", k_s, "worst weight rel err", worst, "CDF err", worst_c, "fallback draws",
        int((flag == 2).sum()))
    if k_s >= 4.0:
        assert (flag == 2).any()
    ctx.move(h)
    sim.move()
    sim.end_step()
    step_both(ctx, sim, h, 20, check_every=1, where=f"k_s={k_s}")
    ctx.destroy(h)


def test_no_agents_and_single_agent(ctx):
    s = sc.corridor(n_agents=0)
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 5)
    ctx.destroy(h)
    s1 = sc.corridor(n_agents=1)
    sim, h = make_pair(ctx, s1)
    step_both(ctx, sim, h, 40)
    ctx.destroy(h)


def test_dense_room_all_cells_but_one(ctx):
    t = sc.walled_box(12, 10)
    t[5, 11] = sc.EXIT
    free = [(x, y) for y in range(1, 9) for x in range(1, 11)]
    agents = free[:-1]                       # every free cell but one is occupied
    s = sc.Scenario("dense", t, len(agents), 3, 1.2, 4, 1)
    sim, h = make_pair(ctx, s, tile=(8, 8), agent_xy=agents)
    step_both(ctx, sim, h, 60)
    ctx.destroy(h)


def test_maximum_agent_count(ctx):
    """The most agents the boundary accepts, 2^20 - 1 (ids fill the 20-bit id
    fields), in a 1100 x 1100 room at 87 % density: plans and positions equal
    the oracle's, through the single-scenario launch and through a batched
    launch of the scenario."""
    s = sc.room(n_agents=(1 << 20) - 1, size=1100)
    say("max agents: single-scenario launches")
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 2, where="max agents")
    ctx.destroy(h)
    say("max agents: batched launches")
    sim, h = make_pair(ctx, s)
    for step in range(2):
        ctx.plan_batch([h])
        sim.plan()
        st = ctx.state(h)
        alive = sim.alive[: sim.n].astype(bool)
        bad = np.nonzero(st["desired"][alive] != sim.desired[: sim.n][alive])[0]
        assert len(bad) == 0, f"batched plan of step {step} differs for {len(bad)} agents"
        ctx.move_batch([h])
        sim.move()
        sim.end_step()
        compare_state(ctx, sim, h, where=f"batched step {step}")
    ctx.destroy(h)


def test_many_tiles_motion_split(ctx):
    """More tiles than the motion phase splits by records (4,096): a 600 x 600
    room in 8 x 8 tiles (5,625), where the motion workgroups take runs of
    tiles instead; plans and positions equal the oracle's."""
    s = sc.room(n_agents=60000, v=4, size=600)
    say("many tiles: 600 x 600 in 8 x 8 tiles")
    sim, h = make_pair(ctx, s, tile=(8, 8))
    assert ctx.stats(h)["n_tiles"] > 4096
    step_both(ctx, sim, h, 6, where="many tiles")
    ctx.destroy(h)


def test_plan_twice_then_move(ctx):
    s = sc.corridor()
    sim, h = make_pair(ctx, s)
    ctx.plan(h)
    ctx.plan(h)             # a second plan of the same step resets the mover list
    sim.plan()
    ctx.move(h)
    sim.move()
    sim.end_step()
    compare_state(ctx, sim, h)
    ctx.destroy(h)


def test_state_errors(ctx):
    from paper_0911_2900_amd import fast
    s = sc.corridor()
    h = ctx.init_from(s)
    with pytest.raises(fast.FastError):
        ctx.move(h)                              # motion without a plan
    with pytest.raises(fast.FastError):
        ctx.plan(h + 1000)                       # unknown handle
    bad = s.cell_type.copy()
    bad[bad == sc.EXIT] = sc.WALL
    with pytest.raises(fast.FastError):
        ctx.init_scenario(bad, 10, 4)            # no exit
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, 10, 6)    # v_max out of range
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, 10, 4, k_s=-1.0)
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, 5000, 4)  # more agents than cells
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, 0, 4, agent_xy=[(3, 3), (3, 3)])
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, 0, 4, agent_xy=[(0, 0)])       # on a wall
    ctx.destroy(h)



def test_stream_bandwidth_yardstick(ctx):
    """The bandwidth yardstick runs at a small and a cache-exceeding
    footprint, reports a plausible rate, and rejects bad sizes."""
    from paper_0911_2900_amd import fast
    say("stream bandwidth: 1 MiB and 512 MiB footprints")
    small, us_small = ctx.stream_bandwidth(1 << 20, 5)
    big, us_big = ctx.stream_bandwidth(512 << 20, 5)
    assert 0.0 < small and 0.0 < us_small
    assert 100.0 < big < 20000.0 and us_big > us_small
    for bad in (0, 95, (64 << 30) + 1):
        with pytest.raises(fast.FastError):
            ctx.stream_bandwidth(bad, 5)
    with pytest.raises(fast.FastError):
        ctx.stream_bandwidth(1 << 20, 0)

# ---------------------------------------------------------------------------
# batched runs: every scenario in the mix equals the oracle and itself alone
# ---------------------------------------------------------------------------

def test_batched_ensemble_members_match_oracle(ctx):
    members = [sc.ensemble_member(k) for k in (0, 1, 2, 5, 8, 13, 21, 34)]
    sims, hs = [], []
    for m in members:
        sim, h = make_pair(ctx, m)
        sims.append(sim)
        hs.append(h)
    steps = 40
    ctx.run(hs, steps)
    for m, sim, h in zip(members, sims, hs):
        sim.run(steps)
        compare_state(ctx, sim, h, where=m.name)
        ctx.destroy(h)


def test_batched_large_grid_sampled(ctx):
    """The 1000 x 1000, 200,000-agent workload at full size: one plan step
    checked on 4,000 sampled agents against the oracle's per-agent draw, then
    one full motion phase compared cell by cell."""
    s = sc.large_member(0)
    sim, h = make_pair(ctx, s)
    ctx.plan(h)
    st = ctx.state(h)
    alive = np.nonzero(sim.alive[: sim.n])[0]
    pick = np.random.default_rng(1).choice(alive, 4000, replace=False)
    for i in pick:
        d = sim.plan_agent(int(i))[0]
        assert st["desired"][i] == d, f"agent {i}"
    sim.plan()
    assert np.array_equal(st["desired"], sim.desired[: sim.n])
    ctx.move(h)
    sim.move()
    sim.end_step()
    compare_state(ctx, sim, h, where="large step 0")
    ctx.destroy(h)


def test_batched_ensemble_16_members_396_steps(ctx):
    """Sixteen members of the 256-scenario ensemble (uneven grids, agent
    counts and v_m) run together for the full 396 steps through the
    graph-replayed batched step; each final state equals the oracle's run of
    that scenario alone."""
    picks = np.random.default_rng(16).choice(256, 16, replace=False)
    members = [sc.ensemble_member(int(k)) for k in picks]
    hs = [ctx.init_from(m, batched=True) for m in members]
    ctx.run(hs, 396)
    for m, h in zip(members, hs):
        sim = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents)
        sim.run(396)
        compare_state(ctx, sim, h, where=m.name)
        st = ctx.stats(h)
        assert st["step"] == 396 and st["exited"] == sim.exited
        ctx.destroy(h)
    say("ensemble members", sorted(int(k) for k in picks))


def test_eight_step_graph_replays_between_eager_steps(ctx):
    """Runs of eight or more steps replay a graph of eight steps.  Its
    replays are interleaved with eager batched steps, state reads (stream
    synchronisations) and one-step replays; after every run each member
    equals the oracle stepped as far."""
    members = [sc.ensemble_member(k) for k in (1, 4, 12, 33)]
    hs = [ctx.init_from(m, batched=True) for m in members]
    sims = [oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents)
            for m in members]
    for k, n in enumerate((8, 3, 16, 8, 11, 24)):
        ctx.run(hs, n)
        for sim in sims:
            sim.run(n)
        for m, sim, h in zip(members, sims, hs):
            compare_state(ctx, sim, h, where=f"{m.name} after run {k} ({n} steps)")
        ctx.plan_batch(hs)                            # one eager step between the replays
        ctx.move_batch(hs)
        for sim in sims:
            sim.step_once()
    for m, sim, h in zip(members, sims, hs):
        compare_state(ctx, sim, h, where=f"{m.name} at the end")
        ctx.destroy(h)


def test_single_scenario_run_matches_eager_steps_and_oracle(ctx):
    """fast_run on one scenario plans with the single-scenario kernel inside
    its graphs: 19 steps (two eight-step replays, three one-step replays),
    then 5 more, equal the oracle and the same scenario stepped eagerly."""
    s = sc.room(n_agents=12000, v=4, size=200)
    sim, h = make_pair(ctx, s)
    he = ctx.init_from(s)
    for n in (19, 5):
        ctx.run([h], n)
        for _ in range(n):
            ctx.plan(he)
            ctx.move(he)
        sim.run(n)
        compare_state(ctx, sim, h, where=f"fast_run, {n} steps")
        assert np.array_equal(ctx.state(h)["xy"], ctx.state(he)["xy"])
    ctx.destroy(h)
    ctx.destroy(he)


def test_large_grid_396_steps_bit_exact(ctx):
    """One 1000 x 1000, 200,000-agent instance for the full 396 steps against
    the oracle (its planning loop on all host threads), final state and the
    exit count compared, positions also at steps 99 and 249."""
    s = sc.large_member(1)
    sim, h = make_pair(ctx, s)
    cores = oracle.num_threads()
    for step in range(396):
        ctx.plan(h)
        ctx.move(h)
        sim.plan_threads(cores)
        sim.move()
        sim.end_step()
        if step in (99, 249):
            compare_state(ctx, sim, h, where=f"after step {step}")
            say("large: step", step, "agents left", sim.n_alive())
    compare_state(ctx, sim, h, where="after 396 steps")
    assert ctx.stats(h)["exited"] == sim.exited
    ctx.destroy(h)


@pytest.mark.parametrize("v", [4, 5])
def test_sequential_fp64_resolve_path(ctx, monkeypatch, v):
    """The FP64 re-resolve normally accepts a wavefront scan when no prefix is
    near tau; FAST_FP64_SEQUENTIAL=1 sends every flagged draw through the
    strictly sequential sum instead.  Both the single-scenario launch (floor
    field staged in LDS) and the batched launch (floor field from global
    memory) must stay bit-exact on that path too."""
    monkeypatch.setenv("FAST_FP64_SEQUENTIAL", "1")
    s = sc.room(v=v, n_agents=20000, scn=7)
    sim, h = make_pair(ctx, s)
    step_both(ctx, sim, h, 12, check_every=4, where=f"sequential resolve v={v}")
    assert ctx.stats(h)["flagged"] > 0
    ctx.destroy(h)
    members = [m for m in (sc.ensemble_member(k) for k in range(40)) if m.v == v][:3]
    hs = [ctx.init_from(m, batched=True) for m in members]
    ctx.run(hs, 15)
    for m, h in zip(members, hs):
        o = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents)
        o.run(15)
        compare_state(ctx, o, h, where=m.name)
        ctx.destroy(h)


def _uniform_batch_vs_oracle(ctx, members, tile, steps):
    hs = [ctx.init_from(m, tile=tile, batched=True) for m in members]
    sims = [oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents) for m in members]
    cores = oracle.num_threads()
    for step in range(steps):
        ctx.plan_batch(hs)
        for sim in sims:
            sim.plan_threads(cores)
        for m, sim, h in zip(members, sims, hs):
            st = ctx.state(h)
            alive = sim.alive[: sim.n].astype(bool)
            bad = np.nonzero(st["desired"][alive] != sim.desired[: sim.n][alive])[0]
            assert len(bad) == 0, f"{m.name} step {step}: {len(bad)} desired cells differ"
        ctx.move_batch(hs)
        for sim in sims:
            sim.move()
            sim.end_step()
    for m, sim, h in zip(members, sims, hs):
        compare_state(ctx, sim, h, where=m.name)
        ctx.destroy(h)


def test_uniform_batch_large(ctx):
    """Four 1000 x 1000 instances (v_m = 4, 64 x 16 tiles) planned in one
    launch: a batch whose members share v_m and the tile shape takes the
    planning kernel specialised for them."""
    _uniform_batch_vs_oracle(ctx, [sc.large_member(k) for k in range(4)], (64, 16), 3)


@pytest.mark.parametrize("v,tile", [(2, (16, 16)), (5, (32, 8))])
def test_uniform_batch_rooms(ctx, v, tile):
    """Eight 400 x 400 rooms sharing v_m and the tile shape, planned in one
    launch by the specialised planning kernel."""
    members = [sc.room(n_agents=12000, v=v, scn=20 + k) for k in range(8)]
    _uniform_batch_vs_oracle(ctx, members, tile, 3)


# ---- part of the chip: streams confined to n CUs ---------------------------

def test_ordinary_stream_uses_every_cu(ctx):
    import torch
    assert ctx.cus() == torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("n", [8, 32, 128])
def test_cu_stream_reaches_its_cus(ctx, n):
    """A stream made for n CUs runs a probe launch on exactly n distinct CUs,
    n / 8 on each XCD."""
    from paper_0911_2900_amd import fast
    say(f"CU stream of {n} CUs")
    cs = fast.CUStream(n)
    try:
        say("  reached", cs.n_cus_run, "per XCD", cs.per_xcd)
        assert cs.n_cus_run == n
        assert cs.per_xcd == [n // 8] * 8
    finally:
        cs.close()


@pytest.mark.parametrize("n", [8, 64])
def test_part_of_the_chip_matches_oracle(ctx, n):
    """A context on a stream of n CUs sizes its motion groups for those CUs
    and steps a 20,000-agent room, and a batch of ensemble members, exactly as
    the oracle does."""
    from paper_0911_2900_amd import fast
    say(f"context on {n} CUs")
    cs = fast.CUStream(n)
    c = fast.Context(stream=cs.torch)
    try:
        assert c.cus() == n
        s = sc.room(n_agents=20000, v=4)
        sim, h = make_pair(c, s)
        step_both(c, sim, h, 8, check_every=3, where=f"room on {n} CUs")
        c.destroy(h)
        members = [sc.ensemble_member(k) for k in (3, 4, 6, 7)]
        pairs = [make_pair(c, m) for m in members]
        c.run([h for _, h in pairs], 12)
        for m, (sim, h) in zip(members, pairs):
            sim.run(12)
            compare_state(c, sim, h, where=f"{m.name} on {n} CUs")
            c.destroy(h)
    finally:
        c.close()
        cs.close()


# ---- region counts (fundamental-diagram measurements) ---------------------

def _fd_pair(ctx, m):
    xy = m.meta["agent_xy"]
    sim = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, agent_xy=xy)
    h = ctx.init_scenario(m.cell_type, 0, m.v, m.k_s, m.seed, m.scn, agent_xy=xy, tile=None)
    return sim, h


def test_region_counts_bottleneck_corridor(ctx):
    """A corridor whose exit is 2 of its 10 cells wide (the congested-branch
    workload): the queue's counts and every position equal the oracle's over
    60 graph-replayed steps."""
    steps = 60
    m = sc.fd_corridor(5.0, 50123, exit_cells=2)
    sim, h = _fd_pair(ctx, m)
    rects = [m.meta["area"], m.meta["upstream"]]
    ctx.set_regions(h, rects, steps)
    want = [sim.region_counts(rects)]
    for _ in range(steps):
        sim.step_once()
        want.append(sim.region_counts(rects))
    ctx.run([h], steps)
    got = ctx.regions(h)
    assert got.shape == (steps + 1, 2)
    assert got.tolist() == [w.tolist() for w in want]
    compare_state(ctx, sim, h, where="bottleneck corridor")
    assert got[-1, 0] > 0                          # the queue still covers the area
    ctx.destroy(h)


def test_region_counts_match_oracle(ctx):
    """Agents in the measurement area and upstream of the flow line, recorded
    after every motion phase, equal the oracle's counts step by step: one
    corridor stepped alone, two in a graph-replayed batch beside a member that
    has no regions (whose state must stay exact too)."""
    steps = 80
    ms = [sc.fd_corridor(d, 900 + i) for i, d in enumerate((1.0, 3.0, 5.5))]
    pairs = [_fd_pair(ctx, m) for m in ms]
    other = sc.ensemble_member(3)
    other_sim, other_h = make_pair(ctx, other)
    rects = [[m.meta["area"], m.meta["upstream"]] for m in ms]
    for r, (sim, h) in zip(rects, pairs):
        ctx.set_regions(h, r, steps)
    want = [[sim.region_counts(r)] for r, (sim, h) in zip(rects, pairs)]
    sim0, h0 = pairs[0]
    for _ in range(steps):
        ctx.plan(h0)
        ctx.move(h0)
        sim0.step_once()
        want[0].append(sim0.region_counts(rects[0]))
    ctx.run([pairs[1][1], pairs[2][1], other_h], steps)
    for i in (1, 2):
        for _ in range(steps):
            pairs[i][0].step_once()
            want[i].append(pairs[i][0].region_counts(rects[i]))
    for i, (sim, h) in enumerate(pairs):
        got = ctx.regions(h)
        say(ms[i].name, "area/upstream at steps 0, 20, 40, 80:", got[[0, 20, 40, 80]].tolist())
        assert got.shape == (steps + 1, 2)
        assert np.array_equal(got, np.array(want[i])), f"{ms[i].name}: counts differ"
        compare_state(ctx, sim, h, where=ms[i].name)
        ctx.destroy(h)
    other_sim.run(steps)
    compare_state(ctx, other_sim, other_h, where="member without regions")
    ctx.destroy(other_h)


def test_region_counts_set_mid_run_and_errors(ctx):
    s = sc.corridor()
    sim, h = make_pair(ctx, s)
    for _ in range(4):
        ctx.plan(h)
        ctx.move(h)
        sim.step_once()
    rects = [(0, 0, 30, 25), (30, 0, 60, 25), (50, 8, 60, 17)]
    ctx.set_regions(h, rects, 10)
    want = {4: sim.region_counts(rects)}
    ctx.run([h], 8)                      # two steps past the last row
    for k in range(5, 13):
        sim.step_once()
        want[k] = sim.region_counts(rects)
    got = ctx.regions(h)
    assert got.shape == (11, 3)
    assert (got[:4] == -1).all()
    for k in range(4, 11):
        assert got[k].tolist() == want[k].tolist(), f"step {k}"
    from paper_0911_2900_amd import fast
    for bad in ([(0, 0, 61, 25)], [(5, 5, 5, 9)], [(-1, 0, 3, 3)], [(0, 0, 2, 2)] * 9):
        with pytest.raises(fast.FastError):
            ctx.set_regions(h, bad, 10)
    ctx.set_regions(h, [], 0)
    assert ctx.regions(h).shape == (0, 0)
    ctx.run([h], 2)
    for _ in range(2):
        sim.step_once()
    compare_state(ctx, sim, h, where="after regions removed")
    ctx.destroy(h)


# ---- per-agent maximum speeds ------------------------------------------------

def _het_pair(ctx, s, vi, tile=None, k_s=None):
    k_s = s.k_s if k_s is None else k_s
    sim = oracle.Sim(s.cell_type, s.v, k_s, s.seed, s.scn, n_agents=s.n_agents, agent_v=vi)
    h = ctx.init_scenario(s.cell_type, s.n_agents, s.v, k_s, s.seed, s.scn, tile=tile, agent_v=vi)
    return sim, h


@pytest.mark.parametrize("v,tile", [(5, (16, 8)), (3, (16, 16)), (4, (32, 8)), (4, (64, 16)),
                                    (2, (8, 32)), (1, (32, 32))])
def test_per_agent_speeds_match_oracle(ctx, v, tile):
    """A room of 20,000 agents with speeds drawn from 1..v, planned on the
    FP32 table path: the first plan's weights (ratios to the reach set's
    largest) and FP32 CDF against the oracle's FP64 ones, then every plan and
    every position equal the oracle's, step by step."""
    s = sc.room(n_agents=20000, v=v)
    vi = np.random.default_rng(v).integers(1, v + 1, size=s.n_agents)
    say(f"per-agent speeds 1..{v}, tile {tile}")
    sim, h = _het_pair(ctx, s, vi, tile)
    worst, worst_c, flag, near = check_weights(ctx, sim, h, sample=3000)
    say(f"  weights rel err {worst:.2e}, CDF err {worst_c:.2e} W, flagged {int((flag == 1).sum())}")
    ctx.move(h)
    sim.move()
    sim.end_step()
    step_both(ctx, sim, h, 11, check_every=1, where=f"speeds 1..{v}")
    assert ctx.stats(h)["fallback"] == 0          # FP32 table path, no range fallback
    ctx.destroy(h)


@pytest.mark.parametrize("k_s", [0.0, 9.0])
def test_per_agent_speeds_near_ties_and_fallback_tiles(ctx, k_s):
    """Speeds 1..4 at k_S = 0 (integer CDF: many exact near ties, every one
    re-resolved in FP64 with the agent's own reach) and at k_S = 9 (tiles
    whose range does not fit the FP32 table draw in FP64, lane by lane)."""
    s = sc.room(n_agents=8000, v=4, size=200)
    vi = np.random.default_rng(int(k_s) + 3).integers(1, 5, size=s.n_agents)
    say(f"per-agent speeds, k_S = {k_s}")
    sim, h = _het_pair(ctx, s, vi, (16, 16), k_s=k_s)
    worst, worst_c, flag, near = check_weights(ctx, sim, h, sample=2000)
    say(f"  flagged {int((flag == 1).sum())}, fallback draws {int((flag == 2).sum())}, near ties {near}")
    if k_s == 0.0:
        assert (flag == 1).sum() > 0
    else:
        assert (flag == 2).sum() > 0
    ctx.move(h)
    sim.move()
    sim.end_step()
    step_both(ctx, sim, h, 6, check_every=1, where=f"speeds k_S={k_s}")
    ctx.destroy(h)


def test_speeds_all_v_max_match_the_uniform_kernels(ctx):
    """Speeds that are all v_max give the trajectories of the uniform
    kernels (two GPU paths, then the oracle at the end)."""
    s = sc.corridor()
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    hu = ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=None)
    hh = ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=None,
                           agent_v=np.full(s.n_agents, s.v))
    for k in range(60):
        for h in (hu, hh):
            ctx.plan(h)
            ctx.move(h)
        if k % 10 == 0:
            a, b = ctx.state(hu), ctx.state(hh)
            assert np.array_equal(a["xy"], b["xy"]), f"step {k}"
    sim.run(60)
    compare_state(ctx, sim, hh, where="speeds all v_max")
    ctx.destroy(hu)
    ctx.destroy(hh)


def test_per_agent_speeds_in_a_batch(ctx):
    """A graph-replayed batch of two scenarios with per-agent speeds and two
    without (their own planning launches beside the shared one), then plain
    batched steps: every member ends where the oracle does."""
    members = [sc.ensemble_member(k) for k in (5, 6, 9, 10)]
    speeds = [np.random.default_rng(40 + i).integers(1, m.v + 1, size=m.n_agents) if i % 2 == 0
              else None for i, m in enumerate(members)]
    pairs = []
    for m, vi in zip(members, speeds):
        if vi is None:
            pairs.append(make_pair(ctx, m))
        else:
            pairs.append(_het_pair(ctx, m, vi))
    hs = [h for _, h in pairs]
    ctx.run(hs, 15)
    for _ in range(3):
        ctx.plan_batch(hs)
        ctx.move_batch(hs)
    for m, (sim, h) in zip(members, pairs):
        sim.run(18)
        compare_state(ctx, sim, h, where=f"{m.name} in a mixed batch")
        ctx.destroy(h)


def test_per_agent_speeds_refused_where_invalid(ctx):
    from paper_0911_2900_amd import fast
    s = sc.corridor()
    for bad in (np.zeros(s.n_agents), np.full(s.n_agents, 5)):
        with pytest.raises(fast.FastError):
            ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=None,
                              agent_v=bad)


def test_per_agent_speeds_sequential_rebuild(ctx, monkeypatch):
    """FAST_FP64_SEQUENTIAL=1 sends every flagged per-agent-speed draw
    through the strictly sequential prefix rebuild; plans and positions stay
    the oracle's."""
    monkeypatch.setenv("FAST_FP64_SEQUENTIAL", "1")
    s = sc.room(n_agents=8000, v=5, size=200)
    vi = np.random.default_rng(17).integers(1, 6, size=s.n_agents)
    sim, h = _het_pair(ctx, s, vi, (32, 8), k_s=0.0)    # k_S = 0: many near ties
    step_both(ctx, sim, h, 6, check_every=1, where="sequential rebuild")
    assert ctx.stats(h)["flagged"] > 0
    ctx.destroy(h)


# ---- several floor fields (one per exit group) ---------------------------------

def _field_pair(ctx, s, tile=None, vi=None):
    ef, af = s.meta["exit_field"], s.meta["agent_field"]
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents, agent_v=vi,
                     exit_field=ef, agent_field=af)
    h = ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=tile,
                          agent_v=vi, exit_field=ef, agent_field=af)
    return sim, h


@pytest.mark.parametrize("v,tile", [(4, (16, 8)), (5, (32, 8)), (2, (16, 16))])
def test_counterflow_fields_match_oracle(ctx, v, tile):
    """Two groups crossing a 200 x 80 hall toward opposite walls, each by
    its own floor field: every plan and position equal the oracle's."""
    s = sc.counterflow(n_agents=5000, v=v, W=200, H=80)
    say(f"counterflow v={v}, tile {tile}")
    sim, h = _field_pair(ctx, s, tile)
    step_both(ctx, sim, h, 10, check_every=1, where=f"counterflow v={v}")
    ctx.run([h], 60)
    sim.run(60)
    compare_state(ctx, sim, h, where=f"counterflow v={v} after 70 steps")
    assert ctx.stats(h)["fallback"] == 0          # FP32 table path, no range fallback
    ctx.destroy(h)


@pytest.mark.parametrize("v,tile", [(4, (32, 16)), (3, (64, 8)), (1, (8, 16)), (5, (8, 64))])
def test_counterflow_field_weights(ctx, v, tile):
    """The debug dump of a counterflow hall (each agent's window from its own
    field's table) against the oracle's FP64 weights, FP32 CDF and near
    ties; then plans and positions for a few steps."""
    s = sc.counterflow(n_agents=4000, v=v, W=160, H=64, scn=11)
    say(f"counterflow weights v={v}, tile {tile}")
    sim, h = _field_pair(ctx, s, tile)
    worst, worst_c, flag, near = check_weights(ctx, sim, h, sample=2000)
    say(f"  weights rel err {worst:.2e}, CDF err {worst_c:.2e} W, flagged {int((flag == 1).sum())}")
    ctx.move(h)
    sim.move()
    sim.end_step()
    step_both(ctx, sim, h, 8, check_every=1, where=f"counterflow weights v={v}")
    ctx.destroy(h)


def test_fields_with_per_agent_speeds_match_oracle(ctx):
    s = sc.counterflow(n_agents=3000, v=5, W=150, H=60, scn=3)
    vi = np.random.default_rng(8).integers(1, 6, size=s.n_agents)
    say("counterflow with per-agent speeds")
    sim, h = _field_pair(ctx, s, (16, 8), vi)
    worst, worst_c, flag, near = check_weights(ctx, sim, h)
    say(f"  weights rel err {worst:.2e}, CDF err {worst_c:.2e} W")
    ctx.move(h)
    sim.move()
    sim.end_step()
    step_both(ctx, sim, h, 7, check_every=1, where="fields + speeds")
    ctx.destroy(h)


def test_fields_in_a_batch(ctx):
    """A counterflow hall planned by its own launch beside two uniform
    members of one graph-replayed batch."""
    members = [sc.ensemble_member(5), sc.counterflow(n_agents=1500, v=3, W=100, H=40, scn=9),
               sc.ensemble_member(6)]
    say("counterflow in a mixed batch")
    pairs = [(_field_pair(ctx, m) if "exit_field" in m.meta else make_pair(ctx, m)) for m in members]
    hs = [h for _, h in pairs]
    ctx.run(hs, 20)
    for m, (sim, h) in zip(members, pairs):
        sim.run(20)
        compare_state(ctx, sim, h, where=f"{m.name} in a mixed batch")
        ctx.destroy(h)


def test_fields_refused_where_invalid(ctx):
    from paper_0911_2900_amd import fast
    s = sc.counterflow(n_agents=100, v=3)
    ef, af = s.meta["exit_field"], s.meta["agent_field"]
    bad_af = af.copy()
    bad_af[0] = 2                                # field 2 has no exit cell
    with pytest.raises(fast.FastError):
        ctx.init_scenario(s.cell_type, s.n_agents, s.v, s.k_s, s.seed, s.scn, tile=None,
                          exit_field=ef, agent_field=bad_af)
    # a room split by a wall: the right group's exits do not reach the left half
    t = sc.walled_box(30, 12)
    t[:, 15] = 1
    t[5:7, 0] = 2
    t[5:7, 29] = 2
    e = np.zeros_like(t)
    e[5:7, 29] = 1
    with pytest.raises(fast.FastError):
        ctx.init_scenario(t, 0, 3, 1.2, 1, 0, agent_xy=[[3, 3]], tile=None,
                          exit_field=e, agent_field=[1])


def _eight_exit_groups(size=240, n_agents=12000, v=5, scn=21):
    """A walled square hall with eight 3-cell exits, two per wall, each its
    own group; agents tagged with a seeded field in 0..7."""
    t = sc.walled_box(size, size)
    ef = np.zeros_like(t)
    q = [size // 3, 2 * size // 3]
    spots = [((0, y), 0) for y in q] + [((size - 1, y), 0) for y in q] + \
            [((x, 0), 1) for x in q] + [((x, size - 1), 1) for x in q]
    for g, ((x, y), horiz) in enumerate(spots):
        if horiz:
            t[y, x - 1:x + 2] = 2
            ef[y, x - 1:x + 2] = g
        else:
            t[y - 1:y + 2, x] = 2
            ef[y - 1:y + 2, x] = g
    af = np.random.default_rng([scn, 8]).integers(0, 8, size=n_agents).astype(np.uint8)
    return sc.Scenario(f"hall_{size}_8_fields", t, n_agents, v, 1.2, 6, scn,
                       meta={"exit_field": ef, "agent_field": af})


def test_eight_floor_fields_match_oracle(ctx):
    """The largest number of fields (8), one per exit, at v = 5."""
    s = _eight_exit_groups()
    say("eight floor fields")
    sim, h = _field_pair(ctx, s, (16, 8))
    step_both(ctx, sim, h, 5, check_every=1, where="eight fields")
    ctx.run([h], 40)
    sim.run(40)
    compare_state(ctx, sim, h, where="eight fields after 45 steps")
    ctx.destroy(h)


def test_fields_with_no_agents(ctx):
    s = sc.counterflow(n_agents=0, v=3)
    say("fields, no agents")
    sim, h = _field_pair(ctx, s)
    ctx.run([h], 3)
    st = ctx.stats(h)
    assert st["step"] == 3 and st["n_active"] == 0
    ctx.destroy(h)


def test_one_exit_group_runs_the_single_field_model(ctx):
    """Every exit and agent tagged 0: the binding sends one field, the
    uniform kernels plan, and the oracle with the group field agrees."""
    s = sc.counterflow(n_agents=2000, v=4, W=120, H=50, scn=5)
    s.meta["exit_field"] = np.zeros_like(s.meta["exit_field"])
    s.meta["agent_field"] = np.zeros_like(s.meta["agent_field"])
    say("one exit group")
    sim, h = _field_pair(ctx, s)
    ctx.run([h], 30)
    sim.run(30)
    compare_state(ctx, sim, h, where="one exit group")
    assert ctx.stats(h)["fallback"] == 0          # FP32 table path
    ctx.destroy(h)
