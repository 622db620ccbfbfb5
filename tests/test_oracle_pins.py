"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each test checks the oracle against a closed form, an independent algorithm or
library, a statistical law of the model, or a hand-worked case, chosen so that
a dropped term, a wrong sign, index or operand order in the oracle fails one
of them.
"""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_0911_2900_amd import scenarios as sc

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11): against rocRAND's independent engine.
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    gxx = shutil.which("g++")
    inc = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if gxx is None or not os.path.exists(inc):
        pytest.skip("rocRAND headers or g++ not available")
    out = tmp_path_factory.mktemp("rr") / "philox_ref"
    subprocess.run([gxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", str(out)], check=True)
    return str(out)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    rows = []
    for k in range(300):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (2**30)            # rocRAND's offset argument is 4 * (c0 | c1 << 32)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        if k < 8:                         # include small and structured counters
            c = np.array([k, 0, 0, k % 5], dtype=np.uint64)
            key = np.array([k % 2, 0], dtype=np.uint64)
        rows.append((c, key))
    inp = "\n".join(" ".join(str(int(x)) for x in list(c) + list(kk)) for c, kk in rows) + "\n"
    res = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    ref = [list(map(int, line.split())) for line in res.stdout.strip().splitlines()]
    assert len(ref) == len(rows)
    for (c, kk), r in zip(rows, ref):
        got = oracle.philox4x32_10(c.astype(np.uint32), kk.astype(np.uint32))
        assert list(map(int, got)) == r


def test_philox_counter_sensitivity():
    # every counter word and key word changes the output (no dropped input)
    base = oracle.philox4x32_10([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] += 1
        assert not np.array_equal(oracle.philox4x32_10(c, [5, 6]), base)
    for i in range(2):
        k = [5, 6]
        k[i] += 1
        assert not np.array_equal(oracle.philox4x32_10([1, 2, 3, 4], k), base)


# --------------------------------------------------------------------------
# Floor field: closed form and an independent exact shortest-path algorithm.
# --------------------------------------------------------------------------

def _octile_pair(dx, dy):
    dx, dy = abs(dx), abs(dy)
    return max(dx, dy) - min(dx, dy), min(dx, dy)


def test_floor_field_open_grid_is_octile_distance():
    """No walls at all: the exact length to the nearest exit cell is the
    octile distance (|d|max - |d|min) + |d|min * sqrt 2."""
    W, H = 23, 17
    t = np.zeros((H, W), dtype=np.uint8)
    exits = [(5, 4), (17, 12), (18, 12)]
    for x, y in exits:
        t[y, x] = sc.EXIT
    _, S, a, b = oracle.floor_field(t)
    sq2 = Decimal(2).sqrt()
    for y in range(H):
        for x in range(W):
            best = None
            for ex, ey in exits:
                p = _octile_pair(x - ex, y - ey)
                val = Decimal(p[0]) + Decimal(p[1]) * sq2
                if best is None or val < best[0]:
                    best = (val, p)
            assert (a[y, x], b[y, x]) == best[1], (x, y)
            # canonical double: fl(fl(b * sqrt2) + a)
            assert S[y, x] == float(best[1][1]) * math.sqrt(2.0) + float(best[1][0])


def _bellman_ford_exact(t):
    """Exact shortest lengths a + b*sqrt2 by Bellman-Ford relaxation with
    60-digit decimals (an algorithm and comparison independent of the
    oracle's Dijkstra with integer sign tests)."""
    getcontext().prec = 60
    sq2 = Decimal(2).sqrt()
    H, W = t.shape
    INF = None
    dist = [[INF] * W for _ in range(H)]
    pair = [[None] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            if t[y, x] == sc.EXIT:
                dist[y][x] = Decimal(0)
                pair[y][x] = (0, 0)
    changed = True
    while changed:
        changed = False
        for y in range(H):
            for x in range(W):
                if t[y, x] == sc.WALL or dist[y][x] is None:
                    continue
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if dx == 0 and dy == 0:
                            continue
                        nx, ny = x + dx, y + dy
                        if not (0 <= nx < W and 0 <= ny < H) or t[ny, nx] == sc.WALL:
                            continue
                        if dx and dy and (t[y, nx] == sc.WALL or t[ny, x] == sc.WALL):
                            continue
                        pa, pb = pair[y][x]
                        cand = (pa + (0 if (dx and dy) else 1), pb + (1 if (dx and dy) else 0))
                        cv = Decimal(cand[0]) + Decimal(cand[1]) * sq2
                        if dist[ny][nx] is None or cv < dist[ny][nx]:
                            dist[ny][nx] = cv
                            pair[ny][nx] = cand
                            changed = True
    return pair


@pytest.mark.parametrize("seed", range(6))
def test_floor_field_matches_bellman_ford_with_walls(seed):
    rng = np.random.default_rng(100 + seed)
    W, H = 11, 9
    t = sc.walled_box(W, H)
    t[1:-1, 1:-1][rng.random((H - 2, W - 2)) < 0.3] = sc.WALL
    t[int(rng.integers(1, H - 1)), W - 1] = sc.EXIT
    t[0, int(rng.integers(1, W - 1))] = sc.EXIT
    after, S, a, b = oracle.floor_field(t)
    ref = _bellman_ford_exact(t)
    for y in range(H):
        for x in range(W):
            if t[y, x] == sc.WALL:
                assert after[y, x] == sc.WALL and np.isinf(S[y, x])
            elif ref[y][x] is None:
                # free cell no exit reaches: turned into a wall
                assert after[y, x] == sc.WALL and np.isinf(S[y, x])
            else:
                assert after[y, x] == t[y, x]
                assert (a[y, x], b[y, x]) == ref[y][x], (x, y)


def test_floor_field_no_corner_cutting():
    # exit at (2,0); the diagonal from (1,1) into (2,0) would cut the wall (1,0)|(2,1)
    t = np.array([[1, 1, 2, 1],
                  [1, 0, 1, 1],
                  [1, 0, 0, 1],
                  [1, 1, 1, 1]], dtype=np.uint8)
    after, S, a, b = oracle.floor_field(t)
    # (2,0) exit is reachable from (1,1)? Only via a diagonal with wall (1,0) and (2,1):
    # not allowed, so (1,1),(1,2),(2,2) are unreachable -> walls.
    assert after[1, 1] == sc.WALL and after[2, 1] == sc.WALL and after[2, 2] == sc.WALL
    t2 = t.copy()
    t2[1, 2] = 0           # open (2,1): now (1,1) -> (2,1) -> (2,0) orthogonally, or diagonal
    after, S, a, b = oracle.floor_field(t2)
    # diagonal (1,1)->(2,0) still needs (1,0) non-wall; it is a wall, so length is 2
    assert (a[1, 1], b[1, 1]) == (2, 0)
    assert (a[1, 2], b[1, 2]) == (1, 0)
    # (2,2) -> (2,1) -> (2,0): 2 ; (1,2) -> diagonal to (2,1) needs (2,2),(1,1) free: yes
    assert (a[2, 1], b[2, 1]) == (1, 1)


def test_corridor_floor_field_rows():
    """Hand-worked cells of the 60 x 25 corridor (exit x = 59, y = 11..13)."""
    s = sc.corridor()
    after, S, a, b = oracle.floor_field(s.cell_type)
    # along the exit rows the field is the plain distance to the right wall
    for y in (11, 12, 13):
        for x in range(1, 59):
            assert S[y, x] == 59 - x
    # (58,10) -> (59,11) would cut the corner of the border wall (59,10): the
    # walk goes (58,10) -> (58,11) -> (59,11), length 2
    assert (a[10, 58], b[10, 58]) == (2, 0)
    # (57,10) -> (58,11) diagonally (both neighbours free), then one step: 1 + sqrt2
    assert (a[10, 57], b[10, 57]) == (1, 1)
    # (57,9): the octile 2*sqrt2 route is cut by the wall corner; best is 2 + sqrt2
    assert (a[9, 57], b[9, 57]) == (2, 1)
    # (58,9): straight down to (58,11), then right: 3
    assert (a[9, 58], b[9, 58]) == (3, 0)


# --------------------------------------------------------------------------
# Placement (reading R8).
# --------------------------------------------------------------------------

def test_placement_distinct_and_eligible():
    s = sc.room(n_agents=5000, size=100)
    after, S, _, _ = oracle.floor_field(s.cell_type)
    x, y = oracle.place(after, S, s.n_agents, seed=3, scn=5)
    cells = y.astype(np.int64) * s.W + x
    assert len(np.unique(cells)) == s.n_agents
    assert np.all(after[y, x] == sc.FREE)


def test_placement_uniform_chi_square():
    W, H = 8, 8
    t = sc.walled_box(W, H)
    t[3, W - 1] = sc.EXIT
    after, S, _, _ = oracle.floor_field(t)
    eligible = np.argwhere(after == sc.FREE)
    counts = np.zeros((H, W))
    trials, n = 3000, 7
    for seed in range(trials):
        x, y = oracle.place(after, S, n, seed=seed, scn=1)
        np.add.at(counts, (y, x), 1)
    obs = counts[after == sc.FREE]
    exp = np.full(len(eligible), trials * n / len(eligible))
    p = stats.chisquare(obs, exp).pvalue
    assert p > 1e-4


def test_placement_rejects_too_many():
    t = sc.walled_box(5, 5)
    t[2, 4] = sc.EXIT
    after, S, _, _ = oracle.floor_field(t)
    with pytest.raises(ValueError):
        oracle.place(after, S, 10, 1, 0)


# --------------------------------------------------------------------------
# Planning (readings R1-R3).
# --------------------------------------------------------------------------

GAUSS_CIRCLE = {1: 5, 2: 13, 3: 29, 4: 49, 5: 81}   # lattice points with x^2 + y^2 <= r^2


def _open_sim(v, k_s, agent_xy, size=15, seed=1):
    t = np.zeros((size, size), dtype=np.uint8)
    t[0, 0] = sc.EXIT          # exit far in a corner of a wall-less grid
    return oracle.Sim(t, v, k_s, seed, 0, agent_xy=agent_xy)


@pytest.mark.parametrize("v", [1, 2, 3, 4, 5])
def test_reach_set_is_the_lattice_disc(v):
    sim = _open_sim(v, 1.2, [(7, 7)])
    d, w, C, u, slot = sim.plan_agent(0)
    assert int((w > 0).sum()) == GAUSS_CIRCLE[v]
    side = 2 * v + 1
    assert w[v * side + v] == 1.0                 # own cell, weight exp(0)
    assert C[-1] == pytest.approx(w.sum(), rel=1e-15)


def test_occupied_and_wall_cells_excluded():
    t = np.zeros((9, 9), dtype=np.uint8)
    t[0, 0] = sc.EXIT
    t[4, 5] = sc.WALL
    sim = oracle.Sim(t, 1, 1.2, 1, 0, agent_xy=[(4, 4), (4, 3)])
    d, w, C, u, slot = sim.plan_agent(0)
    side = 3
    assert w[1 * side + 2] == 0.0          # (5,4) wall
    assert w[0 * side + 1] == 0.0          # (4,3) occupied by agent 1
    assert w[1 * side + 1] == 1.0          # own cell
    assert w[2 * side + 1] > 0.0 and w[1 * side + 0] > 0.0


@pytest.mark.parametrize("v", [1, 3, 5])
def test_uniform_choice_when_k_s_zero(v):
    """k_S = 0: every reachable cell has weight 1, draws are uniform (chi-square)."""
    sim = _open_sim(v, 0.0, [(7, 7)], size=15)
    side = 2 * v + 1
    counts = np.zeros(side * side)
    steps = 6000
    for s in range(steps):
        sim._st.step = s
        d, w, C, u, slot = sim.plan_agent(0)
        counts[slot] += 1
    mask = w > 0
    assert mask.sum() == GAUSS_CIRCLE[v]
    assert counts[~mask].sum() == 0
    p = stats.chisquare(counts[mask]).pvalue
    assert p > 1e-4


def test_descent_as_k_s_grows():
    """k_S -> infinity: the draw is the cell of least S in the reach set, with
    probability >= 1 - |D| exp(-k_S * gap); the field is the closed-form
    octile distance of a wall-less grid, so the argmin is known exactly."""
    sim = _open_sim(4, 110.0, [(9, 13)], size=20)
    getcontext().prec = 40
    sq2 = Decimal(2).sqrt()
    vals = []
    for ddy in range(-4, 5):
        for ddx in range(-4, 5):
            if ddx * ddx + ddy * ddy <= 16:
                p = _octile_pair(9 + ddx, 13 + ddy)
                vals.append((Decimal(p[0]) + Decimal(p[1]) * sq2, ddx, ddy))
    vals.sort()
    gap = float(vals[1][0] - vals[0][0])
    assert gap > 0.1                                  # unique argmin
    assert 49 * math.exp(-110.0 * gap) < 1e-6
    side = 9
    for s in range(300):
        sim._st.step = s
        d, w, C, u, slot = sim.plan_agent(0)
        dx, dy = slot % side - 4, slot // side - 4
        assert (dx, dy) == (vals[0][1], vals[0][2])


def test_odds_ratio_follows_exp_k_delta_s():
    """Two-candidate world: the odds of the better cell over the own cell are
    exp(k_S * (S(c) - S(t))); checked against the closed-form S of an open grid."""
    # a 1-wide horizontal strip: reach set = own cell + left + right (v = 1)
    t = np.full((3, 12), sc.WALL, dtype=np.uint8)
    t[1, 1:11] = sc.FREE
    t[1, 11] = sc.EXIT
    k_s = 0.7
    sim = oracle.Sim(t, 1, k_s, 9, 0, agent_xy=[(5, 1)])
    counts = {}
    steps = 20000
    for s in range(steps):
        sim._st.step = s
        d, w, C, u, slot = sim.plan_agent(0)
        counts[slot] = counts.get(slot, 0) + 1
    # S(x) = 11 - x along the strip
    p_right = math.exp(k_s * 1) / (math.exp(k_s * -1) + 1 + math.exp(k_s * 1))
    p_left = math.exp(-k_s) / (math.exp(-k_s) + 1 + math.exp(k_s))
    n_right, n_left = counts.get(5, 0), counts.get(3, 0)
    n_stay = counts.get(4, 0)
    assert n_right + n_left + n_stay == steps
    for n_obs, p in ((n_right, p_right), (n_left, p_left)):
        sd = math.sqrt(steps * p * (1 - p))
        assert abs(n_obs - steps * p) < 5 * sd


def test_draw_matches_brute_force_enumeration():
    """Exact enumeration of p(t) = w(t)/W on a 7x7 grid (weights from the
    closed-form octile field) against 60,000 oracle draws (chi-square)."""
    t = np.zeros((7, 7), dtype=np.uint8)
    t[0, 6] = sc.EXIT
    t[3, 1] = sc.WALL
    k_s, v = 0.8, 2
    sim = oracle.Sim(t, v, k_s, 4, 3, agent_xy=[(3, 3), (2, 4)])
    getcontext().prec = 40
    sq2 = Decimal(2).sqrt()

    def s_exact(x, y):
        a_, b_ = _octile_pair(x - 6, y - 0)
        return float(Decimal(a_) + Decimal(b_) * sq2)

    side = 5
    p = np.zeros(side * side)
    for dy in range(-v, v + 1):
        for dx in range(-v, v + 1):
            x, y = 3 + dx, 3 + dy
            if dx * dx + dy * dy > v * v or (x, y) in ((1, 3), (2, 4)):
                continue   # outside the disc, the wall, the other agent
            p[(dy + v) * side + dx + v] = math.exp(k_s * (s_exact(3, 3) - s_exact(x, y)))
    p /= p.sum()
    counts = np.zeros(side * side)
    n = 60000
    for s in range(n):
        sim._st.step = s
        _, w, C, u, slot = sim.plan_agent(0)
        counts[slot] += 1
    np.testing.assert_allclose(w / w.sum(), p, rtol=1e-12, atol=1e-15)
    m = p > 0
    assert counts[~m].sum() == 0
    assert stats.chisquare(counts[m], n * p[m]).pvalue > 1e-4


def test_u_is_24_bit_and_selection_rule():
    sim = _open_sim(2, 1.2, [(7, 7)])
    for s in range(50):
        sim._st.step = s
        d, w, C, u, slot = sim.plan_agent(0)
        x0 = int(oracle.philox4x32_10([0, s, 0, 0], [1, 0])[0])
        assert u == (x0 >> 8) / 2**24
        assert float(np.float32(u)) == u          # exact in both precisions
        tau = u * C[-1]
        assert tau < C[slot] and (slot == 0 or C[slot - 1] <= tau)
        assert w[slot] > 0


# --------------------------------------------------------------------------
# Motion (readings R4-R6).
# --------------------------------------------------------------------------

def _order_key(i, step, scn, seed):
    return int(oracle.philox4x32_10([i, step, scn, 1], [seed & 0xFFFFFFFF, seed >> 32])[0]), i


def _empty_room(W=15, H=15):
    t = sc.walled_box(W, H)
    t[H // 2, W - 1] = sc.EXIT
    return t


def _round_half_away(fr):
    return int(math.floor(fr + Fraction(1, 2))) if fr >= 0 else -int(math.floor(-fr + Fraction(1, 2)))


def test_single_agent_reaches_target_exactly():
    t = _empty_room()
    for (dx, dy) in [(3, 2), (-4, 0), (0, -4), (2, -3), (-3, -3), (1, 0)]:
        sim = oracle.Sim(t, 5, 1.2, 1, 0, agent_xy=[(7, 7)])
        sim.desired[0] = (7 + dy) * sim.W + 7 + dx
        sim.move()
        assert (sim.x[0], sim.y[0]) == (7 + dx, 7 + dy)
        assert sim.occ[7 + dy, 7 + dx] == 0 and sim.occ[7, 7] == -1


@pytest.mark.parametrize("dx,dy", [(4, 1), (3, 2), (-2, 3), (1, -4), (-4, -2), (3, 3)])
def test_dda_path_stops_before_blocker(dx, dy):
    """The path cells are the real line c + k/m (dx, dy) rounded half away from
    zero; a standing agent on cell p_k stops the mover on p_(k-1)."""
    m = max(abs(dx), abs(dy))
    path = [(7 + _round_half_away(Fraction(k * dx, m)), 7 + _round_half_away(Fraction(k * dy, m)))
            for k in range(1, m + 1)]
    assert path[-1] == (7 + dx, 7 + dy)
    for kb in range(m):
        bx, by = path[kb]
        sim = oracle.Sim(_empty_room(), 5, 1.2, 1, 0, agent_xy=[(7, 7), (bx, by)])
        sim.desired[0] = (7 + dy) * sim.W + 7 + dx
        sim.desired[1] = by * sim.W + bx          # the blocker stays
        sim.move()
        expect = path[kb - 1] if kb > 0 else (7, 7)
        assert (sim.x[0], sim.y[0]) == expect


def test_earlier_agent_wins_contested_cell():
    t = _empty_room()
    for step in range(20):
        sim = oracle.Sim(t, 3, 1.2, 5, 2, agent_xy=[(5, 7), (9, 7)])
        sim._st.step = step
        target = 7 * sim.W + 7
        sim.desired[0] = target
        sim.desired[1] = target
        sim.move()
        first = min((_order_key(0, step, 2, 5), _order_key(1, step, 2, 5)))[1]
        other = 1 - first
        assert sim.occ[7, 7] == first
        # the other one stops next to the target on its own side
        assert (sim.x[other], sim.y[other]) == ((6, 7) if other == 0 else (8, 7))


def _move_one(t, start, target, v=2):
    sim = oracle.Sim(t, v, 1.2, 1, 0, agent_xy=[start])
    sim.desired[0] = target[1] * sim.W + target[0]
    sim.move()
    return (int(sim.x[0]), int(sim.y[0]))


def test_corner_cut_blocked_and_wall_stop():
    t = _empty_room()
    t[6, 8] = sc.WALL                                   # wall at (8,6)
    assert _move_one(t, (7, 7), (9, 5)) == (7, 7)       # first path cell (8,6) is the wall
    assert _move_one(t, (7, 7), (8, 5)) == (7, 7)       # p_1 = (7 + round(1/2), 6) = (8,6)
    assert _move_one(t, (7, 7), (6, 6)) == (6, 6)       # free diagonal
    assert _move_one(t, (7, 7), (9, 7)) == (9, 7)       # straight past the wall's row
    t2 = _empty_room()
    t2[7, 8] = sc.WALL                                  # wall at (8,7)
    assert _move_one(t2, (7, 7), (8, 6)) == (7, 7)      # diagonal would cut its corner
    assert _move_one(t2, (7, 7), (7, 5)) == (7, 5)      # straight up is fine
    assert _move_one(t2, (7, 7), (9, 5)) == (7, 7)      # (8,6) diagonal cuts (8,7)


def test_exit_removes_agent_and_frees_cell():
    t = _empty_room()
    sim = oracle.Sim(t, 3, 1.2, 1, 0, agent_xy=[(12, 7)])
    sim.desired[0] = 7 * sim.W + 14        # exit cell (14,7)
    sim.move()
    assert sim.alive[0] == 0 and sim.exited == 1 and sim.x[0] == -1
    assert (sim.occ == -1).all()


def _check_invariants(sim, prev_xy, prev_alive, v):
    occ = sim.occ
    alive = sim.alive[: sim.n].astype(bool)
    assert int(alive.sum()) + sim.exited == sim.n
    xs, ys = sim.x[: sim.n][alive], sim.y[: sim.n][alive]
    assert len(set(zip(xs.tolist(), ys.tolist()))) == len(xs)        # one agent per cell
    assert np.all(sim.type[ys, xs] == sc.FREE)                       # not in walls or exits
    assert int((occ >= 0).sum()) == len(xs)
    ids = np.nonzero(alive)[0]
    assert np.all(occ[ys, xs] == ids)
    assert np.all(~alive | prev_alive)                               # no resurrection
    moved = alive & prev_alive
    d = prev_xy[moved] - np.stack([sim.x[: sim.n], sim.y[: sim.n]], 1)[moved]
    assert np.all((d ** 2).sum(1) <= v * v)                          # no move longer than v_m


@pytest.mark.parametrize("case", range(8))
def test_model_invariants_random_small(case):
    rng = np.random.default_rng(500 + case)
    v = int(rng.integers(1, 6))
    s = sc.random_small(rng, int(rng.integers(8, 25)), int(rng.integers(8, 25)),
                        float(rng.uniform(0, 0.15)), int(rng.integers(1, 120)), v,
                        seed=int(rng.integers(0, 2**40)), scn=case, n_exits=int(rng.integers(1, 3)))
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    for step in range(40):
        prev_xy = sim.positions()
        prev_alive = sim.alive[: sim.n].astype(bool).copy()
        sim.plan()
        alive = sim.alive[: sim.n].astype(bool)
        for i in np.nonzero(alive)[0]:
            dxy = (sim.desired[i] % sim.W - sim.x[i], sim.desired[i] // sim.W - sim.y[i])
            assert dxy[0] ** 2 + dxy[1] ** 2 <= v * v
        sim.move()
        sim.end_step()
        _check_invariants(sim, prev_xy, prev_alive, v)


def test_deterministic_runs():
    s = sc.corridor()
    a = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    b = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    a.run(60)
    for _ in range(60):
        b.step_once()
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.occ, b.occ)


@pytest.mark.parametrize("n,threads", [(3000, 4), (3000, 7), (5, 16), (1, 3)])
def test_threaded_plan_gives_same_draws(n, threads):
    """The CPU baseline's threaded loop (chunks claimed from a counter) plans
    every agent exactly once, with the serial loop's draws."""
    s = sc.room(n_agents=n, size=80)
    a = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    a.plan()
    d1 = a.desired.copy()
    a.desired[:] = -7
    a.plan_threads(threads)
    assert np.array_equal(d1, a.desired)


def test_corridor_evacuates_and_conserves():
    s = sc.corridor()
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    sim.run(396)
    assert sim.n_alive() + sim.exited == 200
    assert sim.exited == 200
