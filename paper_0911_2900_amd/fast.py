"""Thin Python binding of libfast (include/fast.h): argument marshalling only.

Every step of the method runs in libfast's HIP kernels; PyTorch supplies the
device allocator (its caching allocator) and the HIP stream.  Importing this
module fails loudly when libfast.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfast.so")

FAST_OK = 0
ERRORS = {-1: "FAST_E_INVALID", -2: "FAST_E_NOMEM", -3: "FAST_E_BUDGET", -4: "FAST_E_DEVICE",
          -5: "FAST_E_STATE", -6: "FAST_E_NOTFOUND"}


class FastError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ScenarioDesc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("cell_type", ctypes.c_void_p),
        ("n_agents", ctypes.c_int32), ("agent_xy", ctypes.c_void_p),
        ("v_max", ctypes.c_int32), ("k_s", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("scenario_id", ctypes.c_uint32),
        ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
        ("agent_v", ctypes.c_void_p),
        ("n_fields", ctypes.c_int32), ("exit_field", ctypes.c_void_p),
        ("agent_field", ctypes.c_void_p),
        ("k_d", ctypes.c_double), ("trail_decay", ctypes.c_double),
        ("trail_diffusion", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int32), ("n_agents", ctypes.c_int32), ("n_active", ctypes.c_int32),
        ("exited", ctypes.c_int32), ("flagged", ctypes.c_int64), ("fallback", ctypes.c_int64),
        ("last_rounds", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
        ("n_tiles", ctypes.c_int32), ("n_fallback_tiles", ctypes.c_int32),
        ("guard_band", ctypes.c_double), ("device_bytes", ctypes.c_int64),
        ("planned", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0911_2900_amd.build`"
                          " (the HIP library is required; there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "fast_ctx_create": [ctypes.c_int, P, ctypes.c_size_t, ALLOC_FN, FREE_FN, P, P],
        "fast_ctx_destroy": [P],
        "fast_init_scenario": [P, P, P],
        "fast_destroy_scenario": [P, I32],
        "fast_plan_step": [P, I32],
        "fast_move_step": [P, I32],
        "fast_run": [P, P, I32, I32],
        "fast_run_noalloc": [P, P, I32, I32],
        "fast_plan_batch": [P, P, I32],
        "fast_move_batch": [P, P, I32],
        "fast_get_state": [P, I32, P, P, P, P, P],
        "fast_get_stats": [P, I32, P],
        "fast_get_trail": [P, I32, P, ctypes.c_int64],
        "fast_debug_plan": [P, I32, P, P, P, P],
        "fast_timing_start": [P, I32],
        "fast_timing_read": [P, P, I32, P],
        "fast_stream_bandwidth": [P, ctypes.c_size_t, I32, P, P],
        "fast_cu_mask": [I32, I32, P, I32],
        "fast_cu_stream_create": [I32, I32, P, P, P],
        "fast_cu_stream_destroy": [P],
        "fast_ctx_cus": [P, P],
        "fast_set_regions": [P, I32, P, I32, I32],
        "fast_get_regions": [P, I32, P, ctypes.c_int64, P, P],
        "fast_serve_start": [P, ctypes.c_size_t, I32],
        "fast_serve_submit": [P, P, I32, P],
        "fast_serve_poll": [P, U64, P, P],
        "fast_serve_result": [P, U64, P, P, P, P],
        "fast_serve_stop": [P],
    }
    sig["fast_floor_field"] = [I32, I32, P, P, P]
    sig["fast_place"] = [I32, I32, P, I32, U64, ctypes.c_uint32, P]
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.fast_guard_band.restype = ctypes.c_double
    L.fast_guard_band.argtypes = [I32]
    L.fast_last_error.restype = ctypes.c_char_p
    L.fast_last_error.argtypes = []
    _lib = L
    return L


def _check(code: int):
    if code != FAST_OK:
        raise FastError(code, lib().fast_last_error().decode())


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def floor_field(cell_type: np.ndarray):
    """Host floor field of the library: (types after, S)."""
    ct = np.ascontiguousarray(cell_type, dtype=np.uint8)
    H, W = ct.shape
    t = np.zeros_like(ct)
    S = np.zeros((H, W), dtype=np.float64)
    _check(lib().fast_floor_field(W, H, _ptr(ct), _ptr(t), _ptr(S)))
    return t, S


def place(cell_type: np.ndarray, n: int, seed: int, scn: int) -> np.ndarray:
    """Host seeded placement of the library: (n, 2) int32 (x, y)."""
    ct = np.ascontiguousarray(cell_type, dtype=np.uint8)
    H, W = ct.shape
    xy = np.zeros((max(n, 1), 2), dtype=np.int32)
    _check(lib().fast_place(W, H, _ptr(ct), int(n), int(seed), int(scn), _ptr(xy)))
    return xy[:n]


def guard_band(v: int) -> float:
    return lib().fast_guard_band(int(v))


def cu_mask(n_cus: int, device_cus: int = 256) -> np.ndarray:
    """The library's CU mask for n_cus CUs, n_cus / 8 per XCD (uint32 words)."""
    mask = np.zeros(max(device_cus // 32, 1), dtype=np.uint32)
    _check(lib().fast_cu_mask(int(n_cus), int(device_cus), _ptr(mask), len(mask)))
    return mask


class CUStream:
    """A HIP stream whose kernels run on n_cus CUs of the device (n_cus / 8 on
    each XCD); `torch` is the same stream for PyTorch, `n_cus_run` the CUs a
    probe launch reached and `per_xcd` how they split over the XCDs.  Pass
    `torch` as a Context's stream; close() after the contexts are destroyed."""

    def __init__(self, n_cus: int, device: int = 0):
        import torch

        ptr = ctypes.c_void_p()
        run = ctypes.c_int32(0)
        per = np.zeros(8, dtype=np.int32)
        _check(lib().fast_cu_stream_create(int(device), int(n_cus), ctypes.byref(ptr),
                                           ctypes.byref(run), _ptr(per)))
        self.ptr = ptr.value
        self.n_cus = int(n_cus)
        self.n_cus_run = run.value
        self.per_xcd = per.tolist()
        self.torch = torch.cuda.ExternalStream(self.ptr, device=device)

    def close(self):
        if self.ptr:
            _check(lib().fast_cu_stream_destroy(ctypes.c_void_p(self.ptr)))
            self.ptr = None


def make_desc(cell_type: np.ndarray, n_agents: int, v: int, k_s: float = 1.2, seed: int = 1,
              scn: int = 0, agent_xy=None, tile=None, agent_v=None, exit_field=None,
              agent_field=None, trail=None):
    """Descriptor plus the host arrays it points to (keep both alive).
    exit_field (H, W) and agent_field (n,) give several floor fields: exit
    cells tagged g lead field g, and agent i follows field agent_field[i].
    trail = (k_d, decay, diffusion): the dynamic floor field."""
    ct = np.ascontiguousarray(cell_type, dtype=np.uint8)
    H, W = ct.shape
    xy = None
    if agent_xy is not None:
        xy = np.ascontiguousarray(np.asarray(agent_xy, dtype=np.int32).reshape(-1, 2))
        n_agents = len(xy)
    d = ScenarioDesc()
    d.width, d.height = W, H
    d.cell_type = _ptr(ct)
    d.n_agents = int(n_agents)
    d.agent_xy = _ptr(xy) if xy is not None and len(xy) else None
    d.v_max, d.k_s = int(v), float(k_s)
    d.seed, d.scenario_id = int(seed), int(scn)
    d.tile_w, d.tile_h = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    sv = None
    if agent_v is not None:
        sv = np.ascontiguousarray(np.asarray(agent_v, dtype=np.uint8))
        if len(sv) != d.n_agents:
            raise ValueError("agent_v needs one speed per agent")
        d.agent_v = _ptr(sv) if len(sv) else None
    ef = af = None
    if (exit_field is None) != (agent_field is None):
        raise ValueError("exit_field and agent_field go together")
    if exit_field is not None:
        ef = np.ascontiguousarray(np.asarray(exit_field, dtype=np.uint8))
        af = np.ascontiguousarray(np.asarray(agent_field, dtype=np.uint8))
        if ef.shape != ct.shape or len(af) != d.n_agents:
            raise ValueError("exit_field needs the grid's shape, agent_field one entry per agent")
        tags = np.union1d(np.unique(ef[ct == 2]), np.unique(af))
        # one tag in use (whatever its value) is the single-field model;
        # otherwise field g is the group tagged g
        nf = int(tags.max()) + 1 if len(tags) > 1 else 1
        d.n_fields = nf
        if nf >= 2:
            d.exit_field = _ptr(ef)
            d.agent_field = _ptr(af) if len(af) else None
    if trail is not None:
        d.k_d, d.trail_decay, d.trail_diffusion = (float(x) for x in trail)
    return d, (ct, xy, sv, ef, af)


class Context:
    """A libfast context on one GPU, issuing work on a PyTorch stream."""

    def __init__(self, device: int = 0, stream=None, budget: int = 0, torch_alloc: bool = True):
        import torch

        self._torch = torch
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._keep = []
        alloc_cb, free_cb = ALLOC_FN(), FREE_FN()
        if torch_alloc:
            tstream = self.stream

            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, tstream)
                except Exception:          # out of memory: report NULL to the library
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            alloc_cb, free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
        self._alloc_cb, self._free_cb = alloc_cb, free_cb
        ctx = ctypes.c_void_p()
        _check(lib().fast_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), int(budget),
                                     alloc_cb, free_cb, None, ctypes.byref(ctx)))
        self.ctx = ctx
        self.n_agents = {}
        self.v = {}
        self.shape = {}

    def cus(self) -> int:
        """CUs this context's stream reaches (see fast_ctx_cus)."""
        n = ctypes.c_int32(0)
        _check(lib().fast_ctx_cus(self.ctx, ctypes.byref(n)))
        return n.value

    # -- scenarios ---------------------------------------------------------
    def init_scenario(self, cell_type, n_agents=0, v=4, k_s=1.2, seed=1, scn=0, agent_xy=None,
                      tile="auto", batched=False, agent_v=None, exit_field=None,
                      agent_field=None, trail=None) -> int:
        """tile: (tx, ty); "auto" = the autotuner's table (planned alone, or in
        a batched launch when `batched`), None = the library's own rule.
        trail: (k_d, decay, diffusion) of the dynamic floor field, or None."""
        if isinstance(tile, str):
            from . import autotune
            ct = np.asarray(cell_type)
            n = len(agent_xy) if agent_xy is not None else int(n_agents)
            tile = autotune.choose_tile(int(v), int(ct.shape[1]), int(ct.shape[0]), n, batched,
                                        het=agent_v is not None or agent_field is not None)
        d, keep = make_desc(cell_type, n_agents, v, k_s, seed, scn, agent_xy, tile, agent_v,
                            exit_field, agent_field, trail)
        h = ctypes.c_int32(-1)
        _check(lib().fast_init_scenario(self.ctx, ctypes.byref(d), ctypes.byref(h)))
        self.n_agents[h.value] = d.n_agents
        self.v[h.value] = int(v)
        self.shape[h.value] = (int(d.height), int(d.width))
        return h.value

    def init_from(self, sc, tile="auto", batched=False) -> int:
        """From a paper_0911_2900_amd.scenarios.Scenario."""
        return self.init_scenario(sc.cell_type, sc.n_agents, sc.v, sc.k_s, sc.seed, sc.scn,
                                  tile=tile, batched=batched,
                                  exit_field=sc.meta.get("exit_field"),
                                  agent_field=sc.meta.get("agent_field"))

    def destroy(self, h: int):
        _check(lib().fast_destroy_scenario(self.ctx, h))
        self.n_agents.pop(h, None)

    # -- steps -------------------------------------------------------------
    def plan(self, h: int):
        _check(lib().fast_plan_step(self.ctx, h))

    def move(self, h: int):
        _check(lib().fast_move_step(self.ctx, h))

    def plan_batch(self, handles):
        hs = np.ascontiguousarray(np.asarray(list(handles), dtype=np.int32))
        _check(lib().fast_plan_batch(self.ctx, _ptr(hs), len(hs)))

    def move_batch(self, handles):
        hs = np.ascontiguousarray(np.asarray(list(handles), dtype=np.int32))
        _check(lib().fast_move_batch(self.ctx, _ptr(hs), len(hs)))

    def run(self, handles, steps: int):
        hs = np.ascontiguousarray(np.asarray(list(handles), dtype=np.int32))
        _check(lib().fast_run(self.ctx, _ptr(hs), len(hs), int(steps)))

    def run_noalloc(self, handles, steps: int):
        hs = np.ascontiguousarray(np.asarray(list(handles), dtype=np.int32))
        _check(lib().fast_run_noalloc(self.ctx, _ptr(hs), len(hs), int(steps)))

    # -- region counts -----------------------------------------------------

    def set_regions(self, h: int, rects, max_step: int):
        """Rectangles (x0, y0, x1, y1), half-open, whose agent counts are
        recorded after every motion phase for steps 0 .. max_step."""
        r = np.ascontiguousarray(np.asarray(rects, dtype=np.int32).reshape(-1, 4))
        _check(lib().fast_set_regions(self.ctx, h, _ptr(r) if len(r) else None, len(r), int(max_step)))

    def regions(self, h: int) -> np.ndarray:
        """(rows, n_regions) int32: agents per rectangle when the step counter
        was k (row k), -1 for steps not reached."""
        n, rows = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().fast_get_regions(self.ctx, h, None, 0, ctypes.byref(n), ctypes.byref(rows)))
        out = np.zeros((rows.value, n.value), dtype=np.int32)
        if out.size:
            _check(lib().fast_get_regions(self.ctx, h, _ptr(out), out.size, None, None))
        return out

    # -- state -------------------------------------------------------------
    def state(self, h: int) -> dict:
        n = self.n_agents[h]
        m = max(n, 1)
        xy = np.zeros((m, 2), dtype=np.int32)
        alive = np.zeros(m, dtype=np.uint8)
        desired = np.zeros(m, dtype=np.int32)
        step, n_active = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().fast_get_state(self.ctx, h, _ptr(xy), _ptr(alive), _ptr(desired),
                                    ctypes.byref(step), ctypes.byref(n_active)))
        return {"xy": xy[:n], "alive": alive[:n], "desired": desired[:n], "step": step.value,
                "n_active": n_active.value}

    def trail(self, h: int) -> np.ndarray:
        """(height, width) float64: the trail field T for the next planning
        phase of a scenario that keeps one."""
        out = np.zeros(self.shape[h], dtype=np.float64)
        _check(lib().fast_get_trail(self.ctx, h, _ptr(out), out.size))
        return out

    def stats(self, h: int) -> dict:
        st = Stats()
        _check(lib().fast_get_stats(self.ctx, h, ctypes.byref(st)))
        return st.as_dict()

    def debug_plan(self, h: int):
        """(w, flag, margin, cdf) of one debug planning phase (see fast.h)."""
        n, v = self.n_agents[h], self.v[h]
        side = 2 * v + 1
        m = max(n, 1)
        w = np.zeros((m, side * side), dtype=np.float32)
        flag = np.zeros(m, dtype=np.uint8)
        margin = np.zeros(m, dtype=np.float32)
        cdf = np.zeros((m, side * side), dtype=np.float32)
        _check(lib().fast_debug_plan(self.ctx, h, _ptr(w), _ptr(flag), _ptr(margin), _ptr(cdf)))
        return w[:n], flag[:n], margin[:n], cdf[:n]

    # -- kernel timing -----------------------------------------------------
    def timing_start(self, max_launches: int):
        """The next max_launches planning launches record their kernel time."""
        _check(lib().fast_timing_start(self.ctx, int(max_launches)))
        self._timing_cap = int(max_launches)

    def timing_read(self) -> np.ndarray:
        """Kernel durations (ms) of the timed planning launches; stops timing."""
        cap = getattr(self, "_timing_cap", 0)
        ms = np.zeros(max(cap, 1), dtype=np.float32)
        n = ctypes.c_int32(0)
        _check(lib().fast_timing_read(self.ctx, _ptr(ms), cap, ctypes.byref(n)))
        return ms[: min(n.value, cap)].copy()

    def stream_bandwidth(self, footprint: int, reps: int = 20) -> tuple:
        """(GB/s, us per launch) of the 5-read/1-write streaming kernel at
        this footprint in bytes."""
        gbs, us = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(lib().fast_stream_bandwidth(self.ctx, int(footprint), int(reps), ctypes.byref(gbs),
                                           ctypes.byref(us)))
        return gbs.value, us.value

    # -- serving -----------------------------------------------------------
    def serve_start(self, budget: int = 0, max_active: int = 0):
        _check(lib().fast_serve_start(self.ctx, int(budget), int(max_active)))

    def serve_submit(self, cell_type, n_agents, v, k_s=1.2, seed=1, scn=0, steps=396,
                     agent_v=None, exit_field=None, agent_field=None, trail=None) -> int:
        d, keep = make_desc(cell_type, n_agents, v, k_s, seed, scn, agent_v=agent_v,
                            exit_field=exit_field, agent_field=agent_field, trail=trail)
        t = ctypes.c_uint64(0)
        _check(lib().fast_serve_submit(self.ctx, ctypes.byref(d), int(steps), ctypes.byref(t)))
        self.n_agents[("ticket", t.value)] = d.n_agents
        return t.value

    def serve_poll(self, ticket: int):
        done, lat = ctypes.c_int32(0), ctypes.c_double(0.0)
        _check(lib().fast_serve_poll(self.ctx, ticket, ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def serve_result(self, ticket: int) -> dict:
        n = self.n_agents[("ticket", ticket)]
        m = max(n, 1)
        xy = np.zeros((m, 2), dtype=np.int32)
        alive = np.zeros(m, dtype=np.uint8)
        step, n_active = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().fast_serve_result(self.ctx, ticket, _ptr(xy), _ptr(alive), ctypes.byref(step),
                                       ctypes.byref(n_active)))
        return {"xy": xy[:n], "alive": alive[:n], "step": step.value, "n_active": n_active.value}

    def serve_stop(self):
        _check(lib().fast_serve_stop(self.ctx))

    def close(self):
        if self.ctx:
            _check(lib().fast_ctx_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
