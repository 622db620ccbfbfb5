"""C-ABI library (no GPU): it loads, exports every function the header
declares, and its host-side setup -- floor field, seeded placement, guard
band -- agrees with the oracle bit for bit on the workloads' grids."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fast.h")


@pytest.fixture(scope="module")
def fast():
    from paper_0911_2900_amd import fast as f
    try:
        f.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return f


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fast_[a-z_0-9]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["fast_ctx_create", "fast_init_scenario", "fast_plan_step", "fast_move_step",
                     "fast_run", "fast_get_state", "fast_debug_plan", "fast_serve_submit",
                     "fast_serve_poll", "fast_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(fast):
    lib = fast.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _grids():
    yield sc.corridor().cell_type
    yield sc.room(size=400).cell_type
    for k in (0, 3, 17, 101):
        yield sc.ensemble_member(k).cell_type
    rng = np.random.default_rng(3)
    for _ in range(5):
        yield sc.random_small(rng, int(rng.integers(5, 40)), int(rng.integers(5, 40)),
                              float(rng.uniform(0, 0.3)), 10, 3, n_exits=2).cell_type


@pytest.mark.parametrize("k", range(11))
def test_host_floor_field_equals_oracle(fast, k):
    grid = list(_grids())[k]
    t_o, S_o, _, _ = oracle.floor_field(grid)
    t_f, S_f = fast.floor_field(grid)
    assert np.array_equal(t_o, t_f)
    assert np.array_equal(S_o, S_f)           # bit-identical, inf on walls


def test_host_floor_field_large_member(fast):
    grid = sc.large_member(0).cell_type
    t_o, S_o, _, _ = oracle.floor_field(grid)
    t_f, S_f = fast.floor_field(grid)
    assert np.array_equal(t_o, t_f) and np.array_equal(S_o, S_f)


@pytest.mark.parametrize("k", range(6))
def test_host_placement_equals_oracle(fast, k):
    grid = list(_grids())[k]
    free = int((oracle.floor_field(grid)[0] == sc.FREE).sum())
    n = min(free, [200, 40000, 500, 1000, 50, 5000][k])
    t_o, S_o, _, _ = oracle.floor_field(grid)
    x, y = oracle.place(t_o, S_o, n, seed=1 + k, scn=k)
    xy = fast.place(grid, n, seed=1 + k, scn=k)
    assert np.array_equal(xy[:, 0], x) and np.array_equal(xy[:, 1], y)


def test_placement_rejects_overfull(fast):
    grid = sc.walled_box(5, 5)
    grid[2, 4] = sc.EXIT
    with pytest.raises(fast.FastError):
        fast.place(grid, 10, 1, 0)


def test_floor_field_rejects_bad_types(fast):
    grid = sc.walled_box(5, 5)
    grid[2, 2] = 7
    with pytest.raises(fast.FastError):
        fast.floor_field(grid)


def test_guard_band_covers_the_fp32_rounding_bound(fast):
    u = 2.0 ** -24
    for v in range(1, 6):
        band = fast.guard_band(v)
        assert band >= 1e-6
        # depth of a CDF value: pairwise row sums plus sequential row/in-row prefixes
        d = int(np.ceil(np.log2(2 * v + 1))) + 2 * v
        assert band > (2 * d + 3) * u
        assert band < 5e-6
    assert fast.guard_band(0) < 0 and fast.guard_band(6) < 0


@pytest.mark.parametrize("device_cus", [64, 256, 512])
def test_cu_mask_is_balanced_under_either_xcd_rule(fast, device_cus):
    """Every mask gives each of the eight XCDs n / 8 CUs, whether the driver
    assigns mask bit b to XCD b // (device_cus / 8) or to XCD b mod 8."""
    per = device_cus // 8
    for n in range(8, device_cus + 1, 8):
        m = fast.cu_mask(n, device_cus)
        bits = np.array([(int(m[b // 32]) >> (b % 32)) & 1 for b in range(device_cus)])
        assert bits.sum() == n
        assert [int(bits[per * j: per * (j + 1)].sum()) for j in range(8)] == [n // 8] * 8
        assert [int(bits[j::8].sum()) for j in range(8)] == [n // 8] * 8


def test_cu_mask_rejects_bad_counts(fast):
    for n, cus in [(0, 256), (4, 256), (12, 256), (264, 256), (8, 96), (8, 0)]:
        with pytest.raises(fast.FastError):
            fast.cu_mask(n, cus)


def _c_offsets(struct: str, fields, tmp_path):
    """offsetof of each field and sizeof of `struct`, from gcc and the header."""
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fast.h"\nint main(void) {\n'
                   + body + f'    printf("%zu\\n", sizeof({struct}));\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(x) for x in out]


@pytest.mark.parametrize("struct,py", [("fast_scenario_desc", "ScenarioDesc"),
                                       ("fast_stats", "Stats")])
def test_binding_structs_match_the_header_layout(fast, tmp_path, struct, py):
    cls = getattr(fast, py)
    names = [n for n, _ in cls._fields_]
    c = _c_offsets(struct, names, tmp_path)
    import ctypes
    assert c[:-1] == [getattr(cls, n).offset for n in names]
    assert c[-1] == ctypes.sizeof(cls)


def test_descriptor_takes_floor_field_groups(fast):
    s = sc.counterflow(n_agents=50, v=3)
    ef, af = s.meta["exit_field"], s.meta["agent_field"]
    d, keep = fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=ef, agent_field=af)
    assert d.n_fields == 2 and d.exit_field and d.agent_field
    d, _ = fast.make_desc(s.cell_type, s.n_agents, s.v)
    assert d.n_fields == 0 and not d.exit_field and not d.agent_field
    # every exit and agent in group 0: the single-field model
    d, _ = fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=np.zeros_like(ef),
                          agent_field=np.zeros_like(af))
    assert d.n_fields == 1 and not d.exit_field and not d.agent_field
    # one tag other than 0 on every exit and agent: still the single-field model
    d, _ = fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=np.ones_like(ef),
                          agent_field=np.ones_like(af))
    assert d.n_fields == 1 and not d.exit_field and not d.agent_field
    # two tags in use: field g is the group tagged g (group 0 must then have exits)
    d, _ = fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=ef + 1, agent_field=af + 1)
    assert d.n_fields == 3 and d.exit_field and d.agent_field
    with pytest.raises(ValueError):
        fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=ef)
    with pytest.raises(ValueError):
        fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=ef[:, 1:], agent_field=af)
    with pytest.raises(ValueError):
        fast.make_desc(s.cell_type, s.n_agents, s.v, exit_field=ef, agent_field=af[1:])
