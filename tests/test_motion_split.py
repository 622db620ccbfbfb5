"""Host-side check of how the motion phase splits a scenario's planned
records over its G workgroups (motion.hip, move_group's gather and
list_capacity), restated here: every record goes to exactly one workgroup,
and no workgroup gets more than its list room; the lists of all workgroups
fit the arrays the runtime allocates (tiles + 2 * 64 tiles' worth)."""
import numpy as np

DIES = 8
GROUP_MAX = 64
TILES_MAX = 4096


def capacity_tiles(T, G):
    tiles = (T + G - 1) // G
    if G % DIES == 0:
        m = G // DIES
        tiles = max(tiles, ((T + DIES - 1) // DIES + m - 1) // m)
    return tiles


def split(counts, G):
    """Records (tile, k) per workgroup, as the gather takes them."""
    T = len(counts)
    out = [[] for _ in range(G)]
    for g in range(G):
        if T <= TILES_MAX:
            by_die = G % DIES == 0
            c, stride = (g % DIES, DIES) if by_die else (0, 1)
            m, w = (G // DIES, g // DIES) if by_die else (G, g)
            tiles = list(range(c, T, stride))
            recs = [(t, k) for t in tiles for k in range(counts[t])]
            r0, r1 = len(recs) * w // m, len(recs) * (w + 1) // m
            out[g] = recs[r0:r1]
        else:
            t0, t1 = T * g // G, T * (g + 1) // G
            out[g] = [(t, k) for t in range(t0, t1) for k in range(counts[t])]
    return out


def test_every_record_once_and_within_room():
    rng = np.random.default_rng(5)
    for _ in range(120):
        T = int(rng.integers(1, 120))
        G = int(rng.integers(1, GROUP_MAX + 1))
        TC = int(rng.choice([64, 128, 256, 512, 1024]))
        counts = rng.integers(0, TC + 1, size=T)
        if rng.random() < 0.3:
            counts[:] = TC                      # every cell planned
        parts = split(counts, G)
        flat = [r for p in parts for r in p]
        assert len(flat) == int(counts.sum()) and len(set(flat)) == len(flat)
        room = capacity_tiles(T, G) * TC
        assert max(len(p) for p in parts) <= room
        assert G * capacity_tiles(T, G) <= T + 2 * GROUP_MAX


def test_many_tiles_split_by_runs_of_tiles():
    counts = np.full(5000, 3)
    for G in (1, 7, 8, 40, 64):
        parts = split(counts, G)
        assert sum(len(p) for p in parts) == 3 * 5000
        assert max(len(p) for p in parts) <= capacity_tiles(5000, G) * 64
