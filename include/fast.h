/*
 * fast.h -- C-ABI of libfast, an MI355X (gfx950) implementation of the
 * F.A.S.T. pedestrian model's time step: the data-parallel planning phase
 * (every agent chooses a desired cell) followed by the sequential motion phase.
 *
 * Paper: T. Kretz, "Computation Speed of the F.A.S.T. Model", arXiv:0911.2900.
 *   Sec. 1  A time step is a planning phase that only reads data common to all
 *           agents and holds the costly exp evaluations, then a motion phase
 *           that moves agents one after another and writes the shared data;
 *           agents never overlap (one agent per cell).
 *   Sec. 2  k_S = 1.2, k_other = 0; one maximum speed v_m for all agents,
 *           v_m = 1..5; runs of 396 steps of one simulated second; the
 *           planning loop "choose_desired_cell(i) for every agent i" is the
 *           parallel part.
 * The model details the paper leaves open are fixed as follows (the same
 * readings the test oracle takes):
 *   - reach set of an agent on cell c: cells c + (dx, dy) with
 *     dx^2 + dy^2 <= v_m^2, inside the grid, not a wall, and free at the start
 *     of the step; the agent's own cell is always a candidate;
 *   - weight exp(k_S * (S(c) - S(t))) with S the static floor field (exact
 *     8-neighbour distance to the nearest exit, orthogonal step 1, diagonal
 *     step sqrt 2, no cutting of wall corners), S in cell units;
 *   - candidates in raster order (dy outer, dx inner, from -v_m), sequential
 *     prefix sum C, W = last C, u = (x0 >> 8) * 2^-24 with x0 word 0 of
 *     Philox4x32-10 at counter (agent id, step, scenario id, 0) and key
 *     (seed low word, seed high word); the choice is the first cell with
 *     u * W < C;
 *   - motion order: ascending (x0 at counter (id, step, scenario, 1), id);
 *     each agent walks the DDA line to its cell, cell by cell, and stops
 *     before a wall, an occupied cell or a diagonal step past a wall corner;
 *     entering an exit removes it at once.
 *   - seeded placement: partial Fisher-Yates over the eligible cells in raster
 *     order with index k + ((x0 * (M - k)) >> 32), x0 at counter (k, 0, scn, 2).
 *
 * Results are bit-identical to a double-precision evaluation of these rules:
 * the GPU draws in FP32 from a per-cell exp table and re-resolves, in FP64,
 * every draw whose u*W lies within a guard band (>= 1e-6 * W, sized from the
 * FP32 rounding bound) of a CDF boundary, and every agent on a grid tile whose
 * floor-field range does not fit the FP32 table.
 *
 * Conventions
 *   - Every function returns FAST_OK (0) or a negative status; nothing aborts
 *     or throws across this boundary.  On error the state is unchanged and
 *     fast_last_error() describes the cause (thread-local string).
 *   - Host pointers are read during the call only and deep-copied; the caller
 *     keeps ownership.  Device memory belongs to the context and comes from
 *     the allocator given to fast_ctx_create (hipMalloc when NULL).
 *   - Calls that launch work (plan, move, run) are asynchronous on the
 *     context's HIP stream; calls that return state synchronise that stream.
 *   - Cells are addressed row-major: index y * width + x.
 *   - Limits: 3 <= width, height <= 16384; v_max in 1..5; at most 2^20 - 1
 *     agents per scenario; at most FAST_MAX_SLOTS live scenarios per context.
 */
#ifndef FAST_H
#define FAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fast_status;

#define FAST_OK            0
#define FAST_E_INVALID    (-1)   /* an argument or the scenario is invalid           */
#define FAST_E_NOMEM      (-2)   /* host or device allocation failed                 */
#define FAST_E_BUDGET     (-3)   /* the context's HBM budget would be exceeded       */
#define FAST_E_DEVICE     (-4)   /* a HIP runtime call failed                        */
#define FAST_E_STATE      (-5)   /* call not valid in the current state              */
#define FAST_E_NOTFOUND   (-6)   /* unknown scenario handle or serving ticket        */

#define FAST_CELL_FREE 0
#define FAST_CELL_WALL 1
#define FAST_CELL_EXIT 2

#define FAST_MAX_SLOTS     4096
#define FAST_MAX_AGENTS    1048575

typedef struct fast_ctx fast_ctx;

/* Device allocator hooks (e.g. PyTorch's caching allocator).  alloc returns a
 * device pointer of at least `bytes` bytes aligned to 256 B, or NULL. */
typedef void *(*fast_alloc_fn)(size_t bytes, void *user);
typedef void (*fast_free_fn)(void *ptr, void *user);

/* One scenario (Sec. 2 parameters plus the geometry the paper leaves open). */
typedef struct {
    int32_t width, height;       /* cells of 0.4 m                                   */
    const uint8_t *cell_type;    /* host, width*height: 0 free, 1 wall, 2 exit;
                                    free cells no exit reaches are treated as walls  */
    int32_t n_agents;            /* agents, ids 0..n_agents-1                        */
    const int32_t *agent_xy;     /* host, 2*n_agents (x, y) pairs, or NULL for the
                                    seeded placement                                 */
    int32_t v_max;               /* v_m, 1..5                                        */
    double k_s;                  /* k_S >= 0 and finite (paper: 1.2)                 */
    uint64_t seed;               /* Philox key                                       */
    uint32_t scenario_id;        /* Philox counter word 2                            */
    int32_t tile_w, tile_h;      /* planning tile in cells; 0, 0 = tuned choice;
                                    otherwise powers of two in 8..64 with
                                    tile_w * tile_h <= 1024                          */
    const uint8_t *agent_v;      /* host, n_agents speeds in 1..v_max (agent i reaches
                                    dx^2 + dy^2 <= agent_v[i]^2), or NULL: all v_max.
                                    Such a scenario is planned by a kernel of its
                                    own (the FP32 table path with each agent's
                                    disc as a mask); in a batch (and when served)
                                    it gets a planning launch of its own beside
                                    the shared one                                   */
    int32_t n_fields;            /* floor fields: 0 or 1 = one field from every exit;
                                    2..8 = route choice / counterflow (Sec. 3's richer
                                    situations): field g is the exact floor field
                                    from the exit cells tagged g alone, and agent i
                                    weighs its window with field agent_field[i].
                                    Walls stay those of the all-exit field and an
                                    agent leaves at any exit cell.  Each field has
                                    its own FP32 exp table; planned like per-agent
                                    speeds (a launch of its own in a batch)         */
    const uint8_t *exit_field;   /* host, width*height, read at exit cells: the field
                                    (0..n_fields-1) the exit belongs to; every field
                                    needs an exit.  NULL when n_fields <= 1          */
    const uint8_t *agent_field;  /* host, n_agents fields in 0..n_fields-1; an agent
                                    must stand where its field is finite.  NULL when
                                    n_fields <= 1                                    */
    double k_d;                  /* dynamic floor field, one of the couplings k_other
                                    that Sec. 2 sets to 0 (this library's reading of
                                    it): every cell holds a trail value T, zero at
                                    the start; an agent that leaves the cell it
                                    started the step on deposits 1 there; after each
                                    motion phase every non-wall cell takes
                                    T' = (1 - trail_decay) ((1 - trail_diffusion) T
                                    + (trail_diffusion / 8) N) + deposits, N the sum
                                    of its 8 neighbours (walls 0); the planning
                                    weight becomes exp(k_S (S(c) - S(t)) +
                                    k_d (T(t) - T(c))).  The field is kept when any of
                                    k_d, trail_decay, trail_diffusion is nonzero
                                    (k_d = 0 then gives the static model's weights).
                                    k_d >= 0 and finite; not with n_fields >= 2    */
    double trail_decay;          /* delta in 0..1                                    */
    double trail_diffusion;      /* alpha in 0..1                                    */
} fast_scenario_desc;

/* Counters of one scenario. */
typedef struct {
    int32_t step;                /* steps completed (the next step's number)         */
    int32_t n_agents;            /* agents at creation                               */
    int32_t n_active;            /* agents still in the simulation                   */
    int32_t exited;              /* agents that left through an exit                 */
    int64_t flagged;             /* draws re-resolved in FP64 (near-tie band)        */
    int64_t fallback;            /* draws resolved in FP64 on range-fallback tiles   */
    int32_t last_rounds;         /* reservation rounds of the last motion phase      */
    int32_t tile_w, tile_h;      /* planning tile in use                             */
    int32_t n_tiles, n_fallback_tiles;
    double guard_band;           /* relative half-width of the FP64 re-resolve band  */
    int64_t device_bytes;        /* device memory held by the scenario               */
    int64_t planned;             /* agent plans made so far (sum of N_active)        */
} fast_stats;

/* Creates a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = a non-blocking stream the context creates and owns).  hbm_budget caps the device bytes
 * held by all scenarios of the context (0 = no cap).  alloc/free_fn may both
 * be NULL (hipMalloc/hipFree). */
fast_status fast_ctx_create(int device, void *hip_stream, size_t hbm_budget,
                            fast_alloc_fn alloc, fast_free_fn free_fn, void *user,
                            fast_ctx **out);

/* Destroys all scenarios, stops serving and frees the context. */
fast_status fast_ctx_destroy(fast_ctx *ctx);

/* Builds a scenario on the host (validation, exact floor field, placement,
 * per-tile FP32 exp table) and copies it to the device.  Step counter 0.
 * Errors: FAST_E_INVALID for width/height < 3, v_max outside 1..5, k_s < 0 or
 * not finite, no exit, an agent off-grid, on a wall/exit or sharing a cell,
 * n_agents above the eligible cells or FAST_MAX_AGENTS; FAST_E_BUDGET when the
 * device bytes exceed the budget; FAST_E_NOMEM, FAST_E_DEVICE. */
fast_status fast_init_scenario(fast_ctx *ctx, const fast_scenario_desc *desc, int32_t *handle);

/* Frees a scenario's device memory (after its queued work). */
fast_status fast_destroy_scenario(fast_ctx *ctx, int32_t handle);

/* One planning phase (Sec. 1 / Sec. 2: choose_desired_cell for every agent
 * against the occupancy at the start of the step).  Writes the desired cells
 * on the device; does not advance the step. */
fast_status fast_plan_step(fast_ctx *ctx, int32_t handle);

/* One motion phase (Sec. 1: agents move one after another in the step's
 * priority order); advances the scenario's step counter.  Must follow a plan
 * of the same step (FAST_E_STATE otherwise). */
fast_status fast_move_step(fast_ctx *ctx, int32_t handle);

/* `steps` full time steps of each of the n scenarios (Sec. 2: a run is 396
 * steps of one simulated second, each a planning phase then a motion phase),
 * run as one batch: each step is one planning launch over the tiles of all
 * scenarios and one motion launch, replayed from captured HIP graphs (one of
 * eight steps while at least eight are left, then one of a single step).
 * Every scenario keeps its own step counter.  n >= 1, steps >= 0. */
fast_status fast_run(fast_ctx *ctx, const int32_t *handles, int32_t n, int32_t steps);

/* For callers that cannot allocate device memory during the call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same `steps` time steps of the n scenarios as fast_run, with the same
 * results bit for bit, run as plain launches (one planning launch, one motion
 * launch and, when a member has regions, one count launch per step) whose
 * work items -- the planning launch's tile items, the motion launch's
 * workgroup items, the region-count jobs -- live in the library's static
 * device scratch instead of a per-batch allocation.  The call allocates no
 * device memory: the items are built on the host into a pinned staging buffer
 * the context set up at creation and copied into the scratch on the context
 * stream.  Limit: the items must fit the scratch, 1 MiB per GPU (about
 * 250,000 tiles over all members); larger batches return FAST_E_INVALID with
 * the size they need.  Every call on one GPU uses that GPU's single scratch,
 * which keeps the last call's items: calls from contexts on different streams
 * of the same GPU that overlap in time race on it (calls on one context are
 * ordered by its stream).  Errors as fast_run (FAST_E_STATE for a member
 * planned without its motion phase). */
fast_status fast_run_noalloc(fast_ctx *ctx, const int32_t *handles, int32_t n, int32_t steps);

/* One planning phase of each of the n scenarios in a single launch over all
 * their tiles (the batched form of fast_plan_step).  The batched calls
 * (fast_run, fast_plan_batch, fast_move_batch) return FAST_E_INVALID for a
 * scenario of more than 2^20 tiles. */
fast_status fast_plan_batch(fast_ctx *ctx, const int32_t *handles, int32_t n);

/* One motion phase of each of the n scenarios in a single launch (the batched
 * form of fast_move_step); each must have been planned for this step. */
fast_status fast_move_batch(fast_ctx *ctx, const int32_t *handles, int32_t n);

/* Copies the state back (synchronises the stream): the agents' cells after
 * the last motion phase and the desired cells of the last planning phase
 * (Sec. 1's two phases).  Any pointer may be NULL.
 * xy: 2*n_agents (x, y), (-1, -1) for agents that left; alive: n_agents;
 * desired: n_agents cells y*width + x chosen by the last planning phase while
 * its motion phase has not run yet (-1 for agents that left, and for every
 * agent once that motion phase has run: the device keeps each plan only as
 * the chosen window slot of the agent's start cell). */
fast_status fast_get_state(fast_ctx *ctx, int32_t handle, int32_t *xy, uint8_t *alive,
                           int32_t *desired, int32_t *step, int32_t *n_active);

/* Copies the trail field T of a scenario that keeps one (descriptor fields
 * k_d, trail_decay, trail_diffusion; the dynamic floor field that the paper
 * counts among the couplings k_other of Sec. 2) as it stands for the next
 * planning phase: out[y*width + x], FP64, capacity >= width*height.  Each
 * motion phase's deposits and the update that follows are included.
 * Synchronises the stream.  FAST_E_INVALID for a scenario without the field
 * or a short buffer. */
fast_status fast_get_trail(fast_ctx *ctx, int32_t handle, double *out, int64_t capacity);

/* Counters of a scenario (synchronises the stream). */
fast_status fast_get_stats(fast_ctx *ctx, int32_t handle, fast_stats *out);

/* Debug planning phase: as fast_plan_step, and also returns, per agent id:
 *   w32[id * (2v+1)^2 + slot]   the weight of each raster slot of the window
 *       (Sec. 1's planning weight exp(k_S (S(c) - S(t))), 0 outside the reach
 *       set) divided by the largest weight of the agent's reach set, so that
 *       every value lies in [0, 1] and FP32 holds it: the kernel's table
 *       values e_t / e_max on ordinary tiles, the FP64 ratio rounded to FP32
 *       on range-fallback tiles (the draw depends on these ratios only);
 *   flag[id] = 1 if the draw was re-resolved in FP64 (2 on a fallback tile);
 *   margin[id] = distance of u*W to the nearest CDF boundary the draw
 *       examined, over W (FP32; -1 on fallback tiles);
 *   cdf32[id * (2v+1)^2 + slot]   the FP32 CDF the draw searches, at every
 *       slot of the reach disc, in the kernel's scale (row prefix plus the
 *       in-row running sum); the window's last slot, a corner outside every
 *       disc, holds the FP32 total W.  All zero on fallback tiles, which have
 *       no FP32 CDF.
 * Host buffers sized for n_agents; any may be NULL.  With per-agent speeds
 * the reach set is the agent's own disc; with several fields the weights are
 * those of the agent's field.  Synchronises. */
fast_status fast_debug_plan(fast_ctx *ctx, int32_t handle, float *w32, uint8_t *flag,
                            float *margin, float *cdf32);

/* ---- Kernel timing ------------------------------------------------------ */

/* Starts timing planning kernels: the next `max_launches` planning launches
 * of fast_plan_step and fast_plan_batch (not those inside fast_run graphs)
 * record the kernel's own start and end on the device, the same interval a
 * kernel trace reports, without waiting on the host.  The events behind this
 * carry no system-scope fence (no cache writeback and invalidation after the
 * launch), so they barely disturb the launches that follow.  Restarting
 * discards earlier records.  FAST_E_INVALID unless 1 <= max_launches <= 2^20. */
fast_status fast_timing_start(fast_ctx *ctx, int32_t max_launches);

/* Synchronises the context stream, writes the durations (milliseconds) of
 * the timed launches in launch order to ms[0 .. min(n, cap)), sets *n to the
 * number timed, and stops timing. */
fast_status fast_timing_read(fast_ctx *ctx, float *ms, int32_t cap, int32_t *n);

/* ---- Region counts: the measurements behind a fundamental diagram -------- */

/* The paper settles on v_m = 4 because the model then reproduces Weidmann's
 * fundamental diagram of walking (Sec. 2).  Such a diagram is measured from
 * counts: agents inside a measurement area give the density, and since agents
 * only move, the drop in the number upstream of a line (with a closed
 * upstream end) is the net flow across it.  FAST_MAX_REGIONS rectangles per
 * scenario at most. */
#define FAST_MAX_REGIONS 8

/* Gives scenario `handle` n_regions rectangles, rects[4 r .. 4 r + 3] =
 * (x0, y0, x1, y1) in grid cells, half-open: x0 <= x < x1, y0 <= y < y1.
 * From now on every motion phase of the scenario (fast_move_step,
 * fast_move_batch, fast_run) is followed by a count kernel that stores the
 * number of agents on each rectangle's cells as row k of a series, k being
 * the scenario's completed steps; rows 0 .. max_step exist, the row of the
 * current step is filled during this call (which synchronises the context
 * stream), rows of steps not reached hold -1.  The series lives in device
 * memory from the context allocator (counted against the budget) and is
 * freed with the scenario or by a new call; n_regions = 0 removes it.
 * FAST_E_INVALID for n_regions outside 0..FAST_MAX_REGIONS, an empty
 * rectangle or one outside the grid, or max_step outside 0..2^24 - 1.  On a
 * device error the scenario is left without regions. */
fast_status fast_set_regions(fast_ctx *ctx, int32_t handle, const int32_t *rects, int32_t n_regions,
                             int32_t max_step);

/* Copies the series of fast_set_regions into counts (row-major,
 * rows x n_regions int32; capacity = ints available) after synchronising the
 * context stream; *n_regions and *rows (either may be NULL) give its shape,
 * 0 x 0 when the scenario has no regions (counts may then be NULL).
 * FAST_E_INVALID if capacity is smaller than rows * n_regions. */
fast_status fast_get_regions(fast_ctx *ctx, int32_t handle, int32_t *counts, int64_t capacity,
                             int32_t *n_regions, int32_t *rows);

/* ---- Bandwidth yardstick ------------------------------------------------- */

/* Measures what a streaming kernel reaches at a given footprint: six arrays
 * of footprint/96 float4 each (rounded down), out = a + b + c + d + e, five
 * reads for each write.  The arrays come from the context allocator and are
 * freed before returning.  After two untimed launches, `reps` launches are
 * timed by the kernel's own start and end events; *gb_per_s = bytes moved
 * per launch / average duration, *us_per_launch (may be NULL) = that
 * duration in microseconds.  Synchronises the context stream.
 * FAST_E_INVALID unless 96 <= footprint <= 64 GiB and 1 <= reps <= 10000;
 * FAST_E_BUDGET / FAST_E_NOMEM if the arrays do not fit. */
fast_status fast_stream_bandwidth(fast_ctx *ctx, size_t footprint, int32_t reps, double *gb_per_s,
                                  double *us_per_launch);

/* ---- Running on part of the chip (CU scaling) ----------------------------- */

/* Sec. 3 of the paper measures how the step time falls as the planning loop
 * gets more of the machine's cores (1..8 cores of two quad-core Xeons).  The
 * calls below give the same study on CUs: a context created on a stream from
 * fast_cu_stream_create runs every kernel on that stream's CUs only. */

/* Bits of a CU mask (n_words 32-bit words, bit b = CU b, as the HIP runtime
 * numbers them) that enable n_cus of a device's device_cus CUs, n_cus / 8 on
 * each of its eight XCDs whether the driver gives mask bit b to XCD
 * b / (device_cus / 8) or to XCD b mod 8: no XCD is left without CUs for its
 * share of a launch's workgroups.  Host only.  FAST_E_INVALID unless
 * device_cus is a multiple of 64, n_words >= device_cus / 32 and n_cus is a
 * multiple of 8 in 8..device_cus. */
fast_status fast_cu_mask(int32_t n_cus, int32_t device_cus, uint32_t *mask, int32_t n_words);

/* Creates a HIP stream (returned as a hipStream_t in *stream) whose kernels
 * run on the n_cus CUs of fast_cu_mask, then launches a probe kernel on it
 * that records where its workgroups run: *n_cus_run (may be NULL) receives
 * the distinct CUs it reached, per_xcd (8 entries, may be NULL) how many of
 * them lie on each XCD.  The caller owns the stream and releases it with
 * fast_cu_stream_destroy after every context using it is destroyed.
 * FAST_E_INVALID for a bad device or n_cus (as fast_cu_mask, on the device's
 * CU count); FAST_E_DEVICE if the runtime refuses the mask. */
fast_status fast_cu_stream_create(int32_t device, int32_t n_cus, void **stream, int32_t *n_cus_run,
                                  int32_t *per_xcd);

/* Synchronises and destroys a stream from fast_cu_stream_create. */
fast_status fast_cu_stream_destroy(void *stream);

/* CUs the context's stream can fill with co-resident workgroups: the
 * device's count for an ordinary stream; for a CU-masked one eight times the
 * fewest CUs that a probe launch at fast_ctx_create reached on any XCD (a
 * dispatch deals its workgroups to the eight XCDs in turn), at most the
 * mask's bit count and at least 1.  The motion phase sizes its groups of
 * co-resident workgroups from this count. */
fast_status fast_ctx_cus(fast_ctx *ctx, int32_t *n_cus);

/* ---- Serving: continuous batching of scenario requests ------------------ */

/* Starts serving on host threads of the context.  Builder threads (half the
 * host's hardware threads, 1..8) do each request's host setup as soon as it
 * is submitted; the server thread admits built requests in submission order
 * as slots while the device bytes stay within `budget` (0 = the context's
 * budget) and at most `max_active` (0 = no cap) scenarios run at once, steps
 * all admitted scenarios together with batched launches of up to 8 steps,
 * retires finished ones and copies their results back.  A request that fits
 * no budget even alone is rejected.  FAST_E_STATE if already serving. */
fast_status fast_serve_start(fast_ctx *ctx, size_t budget, int32_t max_active);

/* Queues a request for `steps` time steps of the scenario; returns a ticket.
 * The descriptor's host arrays are copied during the call. */
fast_status fast_serve_submit(fast_ctx *ctx, const fast_scenario_desc *desc, int32_t steps,
                              uint64_t *ticket);

/* done = 1 once the request has finished; latency_s = completion time minus
 * submission time (seconds).  FAST_E_INVALID if the request was rejected. */
fast_status fast_serve_poll(fast_ctx *ctx, uint64_t ticket, int32_t *done, double *latency_s);

/* Final state of a finished request (as fast_get_state; n_agents sized). */
fast_status fast_serve_result(fast_ctx *ctx, uint64_t ticket, int32_t *xy, uint8_t *alive,
                              int32_t *step, int32_t *n_active);

/* Finishes every submitted request, then joins the serving threads. */
fast_status fast_serve_stop(fast_ctx *ctx);

/* ---- Host-only helpers (no device work) --------------------------------- */

/* The static floor field exactly as fast_init_scenario computes it: type_out
 * (width*height) receives the cell types with unreachable free cells turned
 * into walls, S_out (width*height) the exact walking distance to the nearest
 * exit rounded to double (+inf on walls).  FAST_E_INVALID on bad sizes/types. */
fast_status fast_floor_field(int32_t width, int32_t height, const uint8_t *cell_type,
                             uint8_t *type_out, double *S_out);

/* The seeded placement of fast_init_scenario (agent_xy == NULL): xy_out gets
 * 2*n_agents (x, y).  cell_type is the raw grid; FAST_E_INVALID if n_agents
 * exceeds the eligible cells. */
fast_status fast_place(int32_t width, int32_t height, const uint8_t *cell_type, int32_t n_agents,
                       uint64_t seed, uint32_t scenario_id, int32_t *xy_out);

/* Relative half-width of the FP64 re-resolve band used for v_max. */
double fast_guard_band(int32_t v_max);

/* Thread-local description of the last error (never NULL). */
const char *fast_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FAST_H */
