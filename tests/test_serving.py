"""Serving (continuous batching) through the C-ABI: requests that arrive while
others run are admitted as slots free up, and every request's final state is
bit-identical to the oracle's run of the same scenario alone."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fast_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_2900_amd import fast
    return fast


def _requests(k0, count, steps):
    reqs = []
    for k in range(k0, k0 + count):
        m = sc.ensemble_member(k, base_seed=4, scn_base=1000)
        reqs.append((m, steps))
    return reqs


def _oracle_final(m, steps):
    sim = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents)
    sim.run(steps)
    return sim.positions(), sim.alive[: sim.n].astype(bool)


def _serve(fast, reqs, budget, max_active, gap_s, speeds=None):
    ctx = fast.Context(device=0, torch_alloc=False)
    try:
        ctx.serve_start(budget=budget, max_active=max_active)
        tickets = []
        for i, (m, steps) in enumerate(reqs):
            tickets.append(ctx.serve_submit(m.cell_type, m.n_agents, m.v, m.k_s, m.seed, m.scn,
                                            steps=steps,
                                            agent_v=None if speeds is None else speeds[i],
                                            exit_field=m.meta.get("exit_field"),
                                            agent_field=m.meta.get("agent_field")))
            time.sleep(gap_s)                      # later requests arrive while others run
        deadline = time.time() + 120
        lat = {}
        while len(lat) < len(tickets):
            assert time.time() < deadline, "serving did not finish"
            for t in tickets:
                if t not in lat:
                    done, l = ctx.serve_poll(t)
                    if done:
                        lat[t] = l
            time.sleep(0.002)
        results = [ctx.serve_result(t) for t in tickets]
        ctx.serve_stop()
        return results, [lat[t] for t in tickets]
    finally:
        ctx.close()


def test_served_results_equal_oracle_alone(fast_mod):
    reqs = _requests(0, 10, 30)
    results, lat = _serve(fast_mod, reqs, budget=0, max_active=4, gap_s=0.003)
    say("latencies", np.round(lat, 4))
    for (m, steps), r in zip(reqs, results):
        xy, alive = _oracle_final(m, steps)
        assert r["step"] == steps
        assert np.array_equal(r["alive"].astype(bool), alive), m.name
        assert np.array_equal(r["xy"], xy), m.name


def test_served_per_agent_speeds_equal_oracle(fast_mod):
    """Requests with a speed per agent, served beside requests without: every
    final state equals the oracle's run alone."""
    reqs = _requests(40, 6, 25)
    speeds = [np.random.default_rng(70 + i).integers(1, m.v + 1, size=m.n_agents) if i % 2 == 0
              else None for i, (m, _) in enumerate(reqs)]
    results, lat = _serve(fast_mod, reqs, budget=0, max_active=3, gap_s=0.002, speeds=speeds)
    for (m, steps), vi, r in zip(reqs, speeds, results):
        sim = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents, agent_v=vi)
        sim.run(steps)
        assert r["step"] == steps
        assert np.array_equal(r["xy"], sim.positions()), m.name


def test_served_counterflow_fields_equal_oracle(fast_mod):
    """Counterflow halls (a floor field per exit group) served between
    ordinary requests: every final state equals the oracle's run alone."""
    reqs = _requests(60, 4, 20)
    reqs[1] = (sc.counterflow(n_agents=800, v=4, W=80, H=30, scn=61), 30)
    reqs[3] = (sc.counterflow(n_agents=400, v=2, W=50, H=24, scn=63), 40)
    results, lat = _serve(fast_mod, reqs, budget=0, max_active=2, gap_s=0.002)
    for (m, steps), r in zip(reqs, results):
        sim = oracle.Sim(m.cell_type, m.v, m.k_s, m.seed, m.scn, n_agents=m.n_agents,
                         exit_field=m.meta.get("exit_field"), agent_field=m.meta.get("agent_field"))
        sim.run(steps)
        assert r["step"] == steps
        assert np.array_equal(r["xy"], sim.positions()), m.name


def test_small_budget_forces_queueing_and_stays_exact(fast_mod):
    reqs = _requests(20, 6, 20)
    probe = fast_mod.Context(device=0, torch_alloc=False)
    sizes = []
    for m, _ in reqs:
        h = probe.init_from(m)
        sizes.append(probe.stats(h)["device_bytes"])
        probe.destroy(h)
    probe.close()
    # room for the largest request and a little more: admission must queue
    budget = int(max(sizes) * 1.5) + (1 << 20)
    assert budget < sum(sizes)
    results, lat = _serve(fast_mod, reqs, budget=budget, max_active=0, gap_s=0.0)
    say("latencies (queued)", np.round(lat, 4))
    assert max(lat) > min(lat)
    for (m, steps), r in zip(reqs, results):
        xy, alive = _oracle_final(m, steps)
        assert np.array_equal(r["xy"], xy), m.name


def test_submit_without_start_fails(fast_mod):
    ctx = fast_mod.Context(device=0)
    try:
        m = sc.corridor()
        with pytest.raises(fast_mod.FastError):
            ctx.serve_submit(m.cell_type, m.n_agents, m.v)
    finally:
        ctx.close()


def test_unplaceable_request_is_rejected_and_others_finish(fast_mod):
    """A request whose agents do not fit the grid fails in its host build; it is
    reported as rejected and the requests around it still finish exactly."""
    good = _requests(40, 3, 10)
    bad = sc.corridor()
    ctx = fast_mod.Context(device=0, torch_alloc=False)
    try:
        ctx.serve_start()
        t0 = ctx.serve_submit(good[0][0].cell_type, good[0][0].n_agents, good[0][0].v,
                              good[0][0].k_s, good[0][0].seed, good[0][0].scn, steps=10)
        tb = ctx.serve_submit(bad.cell_type, 5000, bad.v, steps=10)   # corridor holds < 5000
        rest = [ctx.serve_submit(m.cell_type, m.n_agents, m.v, m.k_s, m.seed, m.scn, steps=10)
                for m, _ in good[1:]]
        ctx.serve_stop()
        with pytest.raises(fast_mod.FastError):
            ctx.serve_poll(tb)
        for t, (m, steps) in zip([t0] + rest, good):
            done, _ = ctx.serve_poll(t)
            assert done
            xy, alive = _oracle_final(m, steps)
            assert np.array_equal(ctx.serve_result(t)["xy"], xy), m.name
    finally:
        ctx.close()
