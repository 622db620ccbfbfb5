"""Plain CPU oracle of the F.A.S.T. time step (ctypes wrapper of fast_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg import this package; the product path (``paper_0911_2900_amd``)
never does, and shares no code with it.

Paper: T. Kretz, "Computation Speed of the F.A.S.T. Model" (arXiv:0911.2900),
Sec. 1 (planning phase reads shared data and holds the exp math; motion is
sequential and writes shared data) and Sec. 2 (k_S = 1.2, k_other = 0, one v_m
for all agents, 396 steps; the planning loop is the parallel part).  The
readings the C file takes where the paper is silent are listed at its top.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fast_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CELL_FREE, CELL_WALL, CELL_EXIT = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile fast_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _State(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("H", ctypes.c_int32),
        ("type", ctypes.c_void_p), ("S", ctypes.c_void_p),
        ("v", ctypes.c_int32), ("k_s", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("scn", ctypes.c_uint32),
        ("step", ctypes.c_int32), ("n", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("alive", ctypes.c_void_p), ("desired", ctypes.c_void_p),
        ("occ", ctypes.c_void_p), ("exited", ctypes.c_int64),
        ("vi", ctypes.c_void_p),
        ("Sf", ctypes.c_void_p), ("fi", ctypes.c_void_p),
        ("Tr", ctypes.c_void_p), ("dep", ctypes.c_void_p),
        ("k_d", ctypes.c_double), ("decay", ctypes.c_double), ("diffusion", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.oracle_philox4x32_10.argtypes = [P, P, P]
        _lib.oracle_floor_field.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        _lib.oracle_floor_field_of.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32, P]
        _lib.oracle_place.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_uint32, P, P]
        _lib.oracle_reset_occ.argtypes = [P]
        _lib.oracle_plan_agent.argtypes = [P, ctypes.c_int32, P, P, P, P]
        _lib.oracle_plan_agent.restype = ctypes.c_int32
        _lib.oracle_plan_step.argtypes = [P]
        _lib.oracle_plan_step_threads.argtypes = [P, ctypes.c_int32]
        _lib.oracle_move_step.argtypes = [P]
        _lib.oracle_run.argtypes = [P, ctypes.c_int32]
        _lib.oracle_count_alive.argtypes = [P]
        _lib.oracle_count_alive.restype = ctypes.c_int32
        _lib.oracle_num_threads.restype = ctypes.c_int32
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for a 4-word counter and 2-word key (Salmon et al. 2011)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def floor_field(cell_type: np.ndarray):
    """Exact Dijkstra floor field.  Returns (type_after, S, a, b); see reading R7."""
    t = np.ascontiguousarray(cell_type, dtype=np.uint8).copy()
    H, W = t.shape
    S = np.zeros((H, W), dtype=np.float64)
    a = np.zeros((H, W), dtype=np.int64)
    b = np.zeros((H, W), dtype=np.int64)
    if lib().oracle_floor_field(W, H, _ptr(t), _ptr(S), _ptr(a), _ptr(b)) != 0:
        raise ValueError("floor field failed")
    return t, S, a, b


def place(cell_type_after: np.ndarray, S: np.ndarray, n: int, seed: int, scn: int):
    """Seeded placement of n agents (reading R8).  Returns int32 arrays (x, y)."""
    H, W = cell_type_after.shape
    t = np.ascontiguousarray(cell_type_after, dtype=np.uint8)
    S = np.ascontiguousarray(S, dtype=np.float64)
    x = np.zeros(max(n, 1), dtype=np.int32)
    y = np.zeros(max(n, 1), dtype=np.int32)
    if lib().oracle_place(W, H, _ptr(t), _ptr(S), n, seed, scn, _ptr(x), _ptr(y)) != 0:
        raise ValueError("placement failed: more agents than eligible cells")
    return x[:n].copy(), y[:n].copy()


def floor_field_of(cell_type_after: np.ndarray, exit_field: np.ndarray, g: int) -> np.ndarray:
    """Floor field g of a scenario with several fields (reading R13): the exact
    field from the exit cells whose exit_field value is g, +inf where they do
    not reach."""
    t = np.ascontiguousarray(cell_type_after, dtype=np.uint8)
    ef = np.ascontiguousarray(exit_field, dtype=np.uint8)
    H, W = t.shape
    if ef.shape != t.shape:
        raise ValueError("exit_field must have the grid's shape")
    S = np.zeros((H, W), dtype=np.float64)
    if lib().oracle_floor_field_of(W, H, _ptr(t), _ptr(ef), int(g), _ptr(S)) != 0:
        raise ValueError("floor field failed")
    return S


class Sim:
    """Oracle model state: one scenario, stepped on the CPU."""

    def __init__(self, cell_type: np.ndarray, v: int, k_s: float, seed: int, scn: int,
                 n_agents: int | None = None, agent_xy=None, agent_v=None,
                 exit_field=None, agent_field=None, trail=None):
        self.type, self.S, self.a, self.b = floor_field(cell_type)
        self.H, self.W = self.type.shape
        if agent_xy is None:
            self.x, self.y = place(self.type, self.S, int(n_agents), seed, scn)
        else:
            xy = np.asarray(agent_xy, dtype=np.int32).reshape(-1, 2)
            self.x = np.ascontiguousarray(xy[:, 0]).copy()
            self.y = np.ascontiguousarray(xy[:, 1]).copy()
        self.n = len(self.x)
        m = max(self.n, 1)
        if self.n == 0:
            self.x = np.zeros(m, dtype=np.int32)
            self.y = np.zeros(m, dtype=np.int32)
        self.alive = np.zeros(m, dtype=np.uint8)
        self.alive[: self.n] = 1
        self.desired = np.full(m, -1, dtype=np.int32)
        self.occ = np.full((self.H, self.W), -1, dtype=np.int32)
        self._st = _State()
        self._st.W, self._st.H = self.W, self.H
        self._st.type, self._st.S = _ptr(self.type), _ptr(self.S)
        self._st.v, self._st.k_s = int(v), float(k_s)
        self._st.seed, self._st.scn = int(seed), int(scn)
        self._st.step, self._st.n = 0, self.n
        self._st.x, self._st.y = _ptr(self.x), _ptr(self.y)
        self._st.alive, self._st.desired = _ptr(self.alive), _ptr(self.desired)
        self._st.occ, self._st.exited = _ptr(self.occ), 0
        # per-agent speeds: agent i reaches only its own disc dx^2 + dy^2 <= v_i^2
        # inside the (2v+1)^2 window (v = the largest speed)
        self.agent_v = None
        if agent_v is not None:
            self.agent_v = np.ascontiguousarray(np.asarray(agent_v, dtype=np.uint8)).copy()
            if len(self.agent_v) != self.n or (self.n and (self.agent_v.min() < 1
                                                           or self.agent_v.max() > v)):
                raise ValueError("agent_v: one speed in 1..v per agent")
            self._st.vi = _ptr(self.agent_v) if self.n else None
        # several floor fields (reading R13): agent i follows field agent_field[i]
        self.Sf = self.agent_field = None
        if (exit_field is None) != (agent_field is None):
            raise ValueError("exit_field and agent_field go together")
        if agent_field is not None:
            self.agent_field = np.ascontiguousarray(np.asarray(agent_field, dtype=np.uint8)).copy()
            if len(self.agent_field) != self.n:
                raise ValueError("agent_field needs one field per agent")
            G = int(self.agent_field.max()) + 1 if self.n else 1
            ef = np.asarray(exit_field, dtype=np.uint8)
            G = max(G, int(ef[self.type == 2].max()) + 1)
            self.Sf = np.ascontiguousarray(
                np.stack([floor_field_of(self.type, ef, g) for g in range(G)]))
            self._st.Sf = _ptr(self.Sf)
            self._st.fi = _ptr(self.agent_field) if self.n else None
        # dynamic floor field (reading R14): trail = (k_D, delta, alpha)
        self.Tr = self.dep = None
        if trail is not None:
            k_d, decay, diffusion = (float(x) for x in trail)
            self.Tr = np.zeros((self.H, self.W), dtype=np.float64)
            self.dep = np.zeros((self.H, self.W), dtype=np.int32)
            self._st.Tr, self._st.dep = _ptr(self.Tr), _ptr(self.dep)
            self._st.k_d, self._st.decay, self._st.diffusion = k_d, decay, diffusion
        if lib().oracle_reset_occ(ctypes.byref(self._st)) != 0:
            raise ValueError("invalid agent positions")

    # --- properties -------------------------------------------------------
    @property
    def step(self) -> int:
        return self._st.step

    @property
    def exited(self) -> int:
        return self._st.exited

    @property
    def v(self) -> int:
        return self._st.v

    def n_alive(self) -> int:
        return lib().oracle_count_alive(ctypes.byref(self._st))

    def positions(self) -> np.ndarray:
        return np.stack([self.x[: self.n], self.y[: self.n]], axis=1).copy()

    # --- phases -----------------------------------------------------------
    def plan_agent(self, i: int):
        """(desired, w, C, u, slot) for agent i against the current snapshot."""
        side = 2 * self.v + 1
        w = np.zeros(side * side, dtype=np.float64)
        C = np.zeros(side * side, dtype=np.float64)
        u = ctypes.c_double(0.0)
        slot = ctypes.c_int32(-1)
        d = lib().oracle_plan_agent(ctypes.byref(self._st), i, _ptr(w), _ptr(C),
                                    ctypes.byref(u), ctypes.byref(slot))
        return d, w, C, u.value, slot.value

    def plan(self):
        if lib().oracle_plan_step(ctypes.byref(self._st)) != 0:
            raise RuntimeError("plan failed")

    def plan_threads(self, threads: int):
        """The planning phase on `threads` host threads claiming chunks of
        agents (the CPU baseline's loop); same draws as plan()."""
        if lib().oracle_plan_step_threads(ctypes.byref(self._st), int(threads)) != 0:
            raise RuntimeError("plan failed")

    def move(self):
        """One motion phase (with a trail field, R14's update closes it)."""
        if lib().oracle_move_step(ctypes.byref(self._st)) != 0:
            raise RuntimeError("move failed")

    def trail_update(self):
        """R14's update of the trail field alone (deposits in self.dep)."""
        if self.Tr is None or lib().oracle_trail_update(ctypes.byref(self._st)) != 0:
            raise RuntimeError("no trail field")

    def end_step(self):
        self._st.step += 1

    def step_once(self):
        self.plan()
        self.move()
        self._st.step += 1

    def run(self, steps: int):
        if lib().oracle_run(ctypes.byref(self._st), int(steps)) != 0:
            raise RuntimeError("run failed")

    def region_counts(self, rects) -> np.ndarray:
        """Agents present on each rectangle (x0, y0, x1, y1), half-open: the
        counts a fundamental diagram is measured from (Sec. 2 ties v_m = 4 to
        Weidmann's diagram).  Written out as the plain definition: one
        comparison per agent and rectangle."""
        rects = np.asarray(rects, dtype=np.int64).reshape(-1, 4)
        out = np.zeros(len(rects), dtype=np.int64)
        for r, (x0, y0, x1, y1) in enumerate(rects):
            for i in range(self.n):
                if self.alive[i] and x0 <= self.x[i] < x1 and y0 <= self.y[i] < y1:
                    out[r] += 1
        return out


def num_threads() -> int:
    return lib().oracle_num_threads()
