"""Fundamental-diagram measurements on the host: the oracle's region counts,
the corridor inputs and the reduction of counts to density and flow."""
import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import fd
from paper_0911_2900_amd import scenarios as sc


def test_oracle_region_counts_hand_case():
    t = sc.walled_box(8, 6)
    t[2:4, 7] = sc.EXIT
    xy = np.array([[1, 1], [2, 1], [6, 4], [3, 3], [1, 4]], dtype=np.int32)
    sim = oracle.Sim(t, 2, 1.2, 1, 0, agent_xy=xy)
    rects = [(0, 0, 8, 6), (1, 1, 3, 2), (3, 3, 7, 5), (0, 0, 1, 6), (1, 4, 2, 5)]
    assert sim.region_counts(rects).tolist() == [5, 2, 2, 0, 1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_region_counts_against_a_histogram(seed):
    """After some steps (agents leave by the exit), counts on the cells of a
    3 x 2 partition of the grid equal numpy's 2-D histogram of the alive
    agents, and they add up to the agents present."""
    rng = np.random.default_rng(seed)
    s = sc.random_small(rng, 30, 20, 0.1, 150, 3, n_exits=2)
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    sim.run(12)
    xs, ys = [0, 11, 23, 30], [0, 9, 20]
    rects = [(xs[i], ys[j], xs[i + 1], ys[j + 1]) for i in range(3) for j in range(2)]
    got = sim.region_counts(rects)
    alive = sim.alive[: sim.n].astype(bool)
    h, _, _ = np.histogram2d(sim.x[: sim.n][alive], sim.y[: sim.n][alive], bins=[xs, ys])
    assert got.tolist() == [int(h[i, j]) for i in range(3) for j in range(2)]
    assert got.sum() == sim.n_alive() == s.n_agents - sim.exited


def test_fd_corridor_inputs():
    for d in (0.5, 3.0, 6.25):
        m = sc.fd_corridor(d, 7)
        xy = m.meta["agent_xy"]
        assert len(xy) == m.n_agents == min(round(d * 50 * 10 * 0.16), 500)
        assert len({(int(x), int(y)) for x, y in xy}) == len(xy)
        assert xy[:, 0].min() >= 1 and xy[:, 0].max() <= 50
        assert xy[:, 1].min() >= 1 and xy[:, 1].max() <= 10
        assert (m.cell_type[xy[:, 1], xy[:, 0]] == sc.FREE).all()
        assert (m.cell_type[1:11, 101] == sc.EXIT).all()


def test_fd_bottleneck_corridor_inputs():
    """A bottleneck corridor: only exit_cells cells in the middle of the right
    wall are exit, the rest of it wall; agents as in the open corridor."""
    for w, y0 in ((1, 5), (2, 5), (3, 4), (4, 4), (6, 3)):
        m = sc.fd_corridor(4.0, 7, exit_cells=w)
        col = m.cell_type[:, 101]
        assert (col == sc.EXIT).sum() == w == m.meta["exit_cells"]
        assert (col[y0:y0 + w] == sc.EXIT).all()
        assert ((col == sc.EXIT) | (col == sc.WALL)).all()
        open_ = sc.fd_corridor(4.0, 7)
        assert open_.meta["area"] == (61, 1, 71, 11) and open_.meta["upstream"] == (0, 0, 71, 12)
        assert m.meta["area"] == (81, 1, 91, 11) and m.meta["upstream"] == (0, 0, 91, 12)
        assert np.array_equal(m.meta["agent_xy"], open_.meta["agent_xy"])
        assert np.array_equal(m.cell_type[:, :101], open_.cell_type[:, :101])
    ens = sc.fd_bottleneck_ensemble()
    assert len({m.scn for m in ens}) == len(ens)
    assert not {m.scn for m in ens} & {m.scn for m in sc.fd_ensemble()}


def test_fd_samples_from_a_known_series():
    # area counts and upstream counts over 5 recorded steps (-1: not reached)
    series = np.array([[0, 50], [4, 50], [8, 47], [6, 43], [0, 43], [-1, -1]])
    rho, flow = fd.samples(series, area_m2=16.0, width_m=4.0)
    # step 1: area 4, flow 0; step 2: 8, 3; step 3: 6, 4; step 4: empty area, left out
    assert rho.tolist() == [0.25, 0.5, 0.375]
    assert flow.tolist() == [0.0, 0.75, 1.0]
    bins = fd.diagram(rho, flow, bin_width=0.25, min_samples=1)
    assert [b["samples"] for b in bins] == [2, 1]
    assert bins[0]["flow_mean"] == pytest.approx(0.5)


def test_weidmann_fit_shape():
    rho = np.linspace(0.1, 5.4, 200)
    j = fd.weidmann_flow(rho)
    assert j[-1] == pytest.approx(0.0, abs=1e-12)          # jammed at rho_max
    k = int(np.argmax(j))
    assert 1.5 < rho[k] < 2.0 and 1.1 < j[k] < 1.3         # capacity near 1.75 P/m^2
    assert fd.weidmann_flow(np.array([0.0]))[0] == 0.0
