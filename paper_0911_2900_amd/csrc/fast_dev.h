// fast_dev.h -- data layout shared by libfast's host runtime and its gfx950
// kernels: the per-scenario slot descriptor, counters, and Philox4x32-10.
//
// Layout of one scenario (a "slot") in HBM.  The grid is padded by
// pad = round4(v) cells of wall on every side and rounded up to whole planning
// tiles, so that a tile's staged window -- tx + 2 pad columns (whole 4-cell
// chunks, each inside one tile column) by ty + 2v rows -- needs no bounds check:
//   padded width  Wp = ntx * tx + 2 pad rounded up to a multiple of 32 cells,
//   padded height Hp = nty * ty + 2 pad,
//   cell (x, y) of the scenario lives at index (y + pad) * Wp + (x + pad).
// Per cell:  cell u8 (static: type and corner-cut bits, see cut_bit),
//            D u32 (the exp table entry G(t) of the cell as FP32 bits, with
//            bit 31 set while an agent stands on it: the planning phase's one
//            per-cell read), S f64 (static floor field, read only by the FP64
//            re-resolve), occ i32 (agent id or -1), res0/res1 u64 (motion
//            reservations of even / odd rounds).
// Per tile:  m i32 (power-of-two scale of the exp table), fallback u8, and the
//            agents planned on the tile: a count and one 4-byte record each
//            (the agent's cell inside the tile and the window slot it chose,
//            see plan_rec), written by the planning kernel, read by the
//            motion kernel, which finds the agent's id in occ; the motion
//            rounds keep two mover lists.  Positions live only in occ (the
//            host rebuilds per-agent arrays from occ and the records when
//            asked).
//
// Exp table: G(t) = fl32(exp(m_T(t) ln 2 - k_S S(t))) where T(t) is the tile
// holding t.  A tile T staging a halo cell t of tile T' rescales it by
// 2^(m_T - m_T'), which is exact, so every value an agent of T sees equals
// fl32(exp(-k_S (S(t) - beta_T))) with beta_T = m_T ln 2 / k_S.  The weight
// ratio e_t / e_c is then exp(k_S (S(c) - S(t))) to within 2 roundings.
// Tiles whose window does not fit [e^-80, e^80] are "fallback" tiles: their
// agents are drawn directly in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

enum : int { CELL_FREE = 0, CELL_WALL = 1, CELL_EXIT = 2 };
// Device cell bytes: the type in bits 0-1, and in bits 2-5 whether a diagonal
// step into the cell cuts a wall corner, one bit per direction (sx, sy).
constexpr int CELL_TYPE_MASK = 3, CUT_SHIFT = 2;
__host__ __device__ inline int cut_bit(int sx, int sy) { return CUT_SHIFT + (sx < 0 ? 2 : 0) + (sy < 0 ? 1 : 0); }

constexpr int MAX_V = 5;
constexpr int MAX_TILE_CELLS = 1024;   // tx * ty
constexpr int MAX_STAGE = 2368;        // (tx + 2 pad) * (ty + 2v) over the allowed tiles
constexpr int PLAN_THREADS = 256;
constexpr int ONE_MAX_THREADS = 1024;     // single-scenario planning launches: up to one thread per tile cell
constexpr int MOVE_THREADS = 1024;
constexpr int MOVE_GROUP_MAX = 64;        // workgroups per scenario in the motion phase
constexpr int GATHER_TILES_MAX = 4096;    // motion splits records evenly up to this many tiles
constexpr int DIES = 8;                   // compute dies (XCDs), each with its own L2
constexpr int MOVE_SOLO_MAX = 256;        // movers left at which one workgroup takes over
constexpr int MOVE_AGENTS_PER_WG = 1024;  // group size = ceil(agents / this), capped
constexpr uint32_t SPIN_LIMIT = 1u << 22; // bound on a group-barrier wait (never hangs)

// Motion reservation words: [tag:12][~x0:32][~id:20]; the largest word on a
// cell is the earliest agent of the current round (tags grow every round).
constexpr int ID_BITS = 20;
constexpr uint32_t ID_MASK = (1u << ID_BITS) - 1u;
constexpr int TAG_SHIFT = 52;
constexpr uint32_t TAG_LIMIT = 4095u;

// int32 counters per slot
enum : int {
    C_STEP = 0,      // steps completed
    C_NACTIVE = 1,   // agents still present
    C_EXITED = 2,    // agents that left
    C_TAG = 4,       // last reservation tag used
    C_ROUNDS = 5,    // reservation rounds of the last motion phase
    C_LIMIT = 6,     // kernels act while step < limit
    C_BAR = 12,      // 2 x uint64 (C_BAR..C_BAR+3): group-barrier words of even / odd
                     // rounds, [arrivals:32][movers left:32], zeroed by the plan kernel
    C_ERR = 10,      // nonzero: a group barrier timed out, the state is invalid
    C_SOLO = 16,     // MOVE_GROUP_MAX entries: movers left per workgroup of the group
    C_NCTR = 16 + 64
};

// A mover of the running motion phase: priority word and packed coordinates
// (x | y << 16, padded) of its start and desired cells.
// key: bits 0..51 the priority word [~x0:32][~id:20] (larger = earlier);
// bits 52..54 the reach m_eff of the line; bits 55..59 flag the line cells
// k = 1..5 that hold a higher-priority mover at the start of the phase; bit
// 60 marks a line that ends on an exit.
struct Mover {
    unsigned long long key;
    uint32_t cxy, dxy;
};
constexpr unsigned long long KEY_MASK = (1ull << 52) - 1ull;
constexpr int MEFF_SHIFT = 52, HP_SHIFT = 55, EXIT_BIT = 60;

// A planned agent's record: bits 0..9 its cell inside the tile (row-major,
// ly * tx + lx), bits 10..16 the slot of its (2 v_max + 1)^2 window that it
// chose (raster order: (dy + v_max) * (2 v_max + 1) + dx + v_max; the middle
// slot when it stays).  The agent's id is occ of that cell until the motion
// phase runs.
constexpr int REC_SLOT_SHIFT = 10;
__host__ __device__ inline uint32_t plan_rec(int lcell, int slot)
{
    return (uint32_t)lcell | ((uint32_t)slot << REC_SLOT_SHIFT);
}
// Tiles of a single-scenario launch.  A dispatch deals its workgroups to
// the XCDs in turn (workgroup i to XCD i mod DIES), and each XCD has an L2
// of its own: XCD x plans the tile rows x, x + DIES, x + 2 DIES, ..., each
// row in order, so that a tile's left and right neighbours share their
// window columns through one L2 (the crowded rows of a scenario still spread
// over all the XCDs).  Workgroup i plans row_tile(i, ntx, nty) of the
// ntx x nty tiles, or nothing (-1, past the last row); the launch has
// row_grid(ntx, nty) workgroups.
__host__ __device__ inline int row_tile(int i, int ntx, int nty)
{
    const int x = i % DIES, j = i / DIES;
    const int row = x + DIES * (j / ntx);
    return row < nty ? row * ntx + j % ntx : -1;
}
__host__ __device__ inline int row_grid(int ntx, int nty)
{
    return DIES * ntx * ((nty + DIES - 1) / DIES);
}
// A batched planning item, (slot << 20) | tile, that plans nothing (padding).
constexpr uint32_t PLAN_ITEM_NONE = 0xFFFFFFFFu;
// Bit 31 of a D entry: the cell is occupied.
constexpr uint32_t D_OCC = 0x80000000u;
// uint64 statistics per slot
enum : int { S_FLAGGED = 0, S_FALLBACK = 1, S_PLANNED = 2, S_NSTAT = 4 };

struct SlotDev {
    int32_t W, H;            // scenario size
    int32_t Wp, Hp;          // padded size
    int32_t v;               // v_m
    int32_t pad;             // wall border, round4(v)
    int32_t tx, ty;          // planning tile
    int32_t ntx, nty;        // tiles per row / column
    int32_t n_agents;
    uint32_t seed_lo, seed_hi, scn;
    float eps;               // guard band, relative to W
    double k_s;
    double near64;           // FP64 re-resolve: scanned prefixes this close to tau (relative
                             // to W) send the draw to the sequential sum
    const uint8_t *cell;     // Wp*Hp: type | corner-cut bits (see cut_bit)
    uint32_t *D;             // Wp*Hp: exp table bits | D_OCC while occupied
    const double *S;         // Wp*Hp
    const int32_t *tile_m;   // (ntx+2)*(nty+2), a ring of zeros around
    uint8_t *tile_fb;        // ntx*nty (rewritten every step with a trail field)
    int32_t *occ;            // Wp*Hp
    unsigned long long *res0;// Wp*Hp, reservations of even rounds
    unsigned long long *res1;// Wp*Hp, reservations of odd rounds
    int32_t *seg_cnt;        // ntx*nty: agents planned per tile
    uint32_t *seg;           // ntx*nty*tx*ty: their records (plan_rec), tile by tile
    Mover *mv_a, *mv_b;      // (ntx*nty + 2 MOVE_GROUP_MAX)*tx*ty each: movers of the current / next round
    Mover *hand;             // (motion workgroups)*MOVE_SOLO_MAX: movers handed to workgroup 0
    int32_t *ctr;            // C_NCTR
    unsigned long long *stat;// S_NSTAT
    // dynamic floor field (trail; null when the scenario has none): the trail
    // of step s in Tr + (s & 1) Wp Hp, deposits of the running motion phase
    double *Tr;              // 2 Wp*Hp
    int32_t *dep;            // Wp*Hp
    double k_d, t_decay, t_diff;
    float *dbg_w;            // optional debug outputs (null in normal runs)
    uint8_t *dbg_flag;
    float *dbg_margin;
    float *dbg_cdf;
};

// Per-agent speeds and several floor fields of a scenario (the richer
// situations of Sec. 3).  Each field has its own exp table, tile scales and
// fallback flags, laid out like the scenario's own, field_cells apart.
struct HetDev {
    const uint8_t *vi;       // n_agents maximum speeds in 1..v, or null (all v)
    const uint8_t *fi;       // n_agents field indices, or null (one field: the scenario's own)
    const uint32_t *Gf;      // nf exp tables as FP32 bits (nf >= 2)
    const double *Sf;        // nf floor fields (nf >= 2)
    const int32_t *tile_mf;  // nf x (ntx+2)*(nty+2) tile scales (nf >= 2)
    const uint8_t *tile_fbf; // nf x ntx*nty fallback flags (nf >= 2)
    long field_cells;        // Wp*Hp
    int nf;                  // fields; 1 = the scenario's own (D, S, tile_m, tile_fb)
};
constexpr int MAX_FIELDS = 8;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), word 0 of the output
// block for counter (c0, c1, c2, c3) and key (k0, k1).
__host__ __device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// Philox streams (counter word 3)
enum : uint32_t { STREAM_PLAN = 0, STREAM_ORDER = 1, STREAM_PLACE = 2 };

}  // namespace fk
