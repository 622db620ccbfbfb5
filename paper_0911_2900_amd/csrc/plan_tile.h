// plan_tile.h -- device code of the planning phase (choose_desired_cell for
// every agent, paper Sec. 1 and Sec. 2), shared by the planning kernels.
//
// One workgroup plans one grid tile: the tile's (tx + 2 round4(v)) x (ty + 2v)
// window of the exp table, masked by the occupancy snapshot, is staged in
// LDS; the tile's agents are found by scanning its occupancy; one lane per
// agent forms the weights, the CDF over the reach disc and the Philox draw in
// FP32; draws inside the guard band are re-resolved in FP64 by a whole
// wavefront.  Each agent's (id, cell, chosen cell) record is written to its
// slot of the tile's own segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "fast_dev.h"

namespace fk {

// ---------------------------------------------------------------------------
// Compile-time geometry of the reach disc dx^2 + dy^2 <= V^2.
// ---------------------------------------------------------------------------
constexpr int isqrt_c(int n) { int r = 0; while ((r + 1) * (r + 1) <= n) ++r; return r; }
constexpr int half_width(int V, int dy) { return isqrt_c(V * V - dy * dy); }

// Pairwise (balanced) sum of x[O .. O+N): rounding depth ceil(log2 N).
template <int N, int O>
struct Tree {
    static __device__ __forceinline__ float sum(const float *x)
    {
        constexpr int h = (N + 1) / 2;
        return Tree<h, O>::sum(x) + Tree<N - h, O + h>::sum(x);
    }
};
template <int O>
struct Tree<1, O> {
    static __device__ __forceinline__ float sum(const float *x) { return x[O]; }
};

// An agent's (2V+1)-row window in the staged table (pitch P), from its
// origin (row -V, column -V) at LDS index eo >= 0.  Rows are grouped under
// separate base registers so that every read is a non-negative immediate
// offset of at most 255 words from its group's base, the reach of a paired
// LDS read; the empty asm keeps the compiler from folding the bases back
// into one address with negative or out-of-range offsets.
template <int V, int P>
struct Window {
    static constexpr int G = (255 - 2 * V) / P + 1;          // rows per base
    static constexpr int NB = (2 * V + G) / G;                // ceil((2V + 1) / G)
    const float *b[NB];
    __device__ __forceinline__ Window(const float *Em, int eo)
    {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            int o = eo + i * G * P;
            asm volatile("" : "+v"(o));
            b[i] = Em + o;
        }
    }
    template <int R>
    __device__ __forceinline__ const float *row() const { return b[R / G] + (R % G) * P; }
};

// Row R (dy = R - V) of the reach disc: its 2a+1 masked exp values; the
// agent's own cell takes e_c.  MASK (an agent whose own maximum speed vr may
// be below V): slots with dx^2 + dy^2 > vr2 = vr^2 take an exact 0, so the
// sums keep their rounding structure.
template <int V, int P, int R, bool MASK>
__device__ __forceinline__ void load_row(const Window<V, P> &w, float ec, int vr2, float (&x)[2 * V + 1])
{
    constexpr int a = half_width(V, R - V);
    const float *rp = w.template row<R>();
#pragma unroll
    for (int k = 0; k <= 2 * a; ++k) {
        if (R == V && k == a) x[k] = ec;
        else x[k] = rp[(V - a) + k];
        if constexpr (MASK) {
            constexpr int dy = R - V;
            const int dx = k - a;
            if (dx * dx + dy * dy > 0) x[k] = dx * dx + dy * dy <= vr2 ? x[k] : 0.0f;
        }
    }
}

// Row sums, software-pipelined by two rows: the loads of row R+2 are issued
// before row R is summed, and the scheduling barrier keeps later rows from
// being hoisted, so at most three rows of values are live.
template <int V, int P, int R, bool MASK>
struct RowPipe {
    static __device__ __forceinline__ void run(const Window<V, P> &w, float ec, int vr2, float *Rs,
                                               const float (&cur)[2 * V + 1],
                                               const float (&nx1)[2 * V + 1])
    {
        constexpr int a = half_width(V, R - V);
        float nx2[2 * V + 1];
        if constexpr (R + 2 < 2 * V + 1) load_row<V, P, R + 2, MASK>(w, ec, vr2, nx2);
        Rs[R] = Tree<2 * a + 1, 0>::sum(cur);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (R + 1 < 2 * V + 1) RowPipe<V, P, R + 1, MASK>::run(w, ec, vr2, Rs, nx1, nx2);
    }
};

// ---------------------------------------------------------------------------
// FP64 draw, the test oracle's arithmetic: weights exp(k_S (S(c) - S(t))) over
// the square window in raster order (zero outside the reach set), sequential
// sum, tau = u * W, first slot with tau < C.  One lane does one agent.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool reach_ok(const SlotDev &s, int gc, int t, int dx, int dy, int vr)
{
    if (dx * dx + dy * dy > vr * vr) return false;
    if ((s.cell[t] & CELL_TYPE_MASK) == CELL_WALL) return false;
    const int o = s.occ[t];
    return o < 0 || t == gc;
}

// (The loops stay rolled: this path is rare, and unrolled FP64 exp code would
// raise the register count of the whole planning kernel.)  The debug form
// also writes each slot's weight over the largest weight of the reach set,
// rounded to FP32 (every such ratio lies in [0, 1], so FP32 holds it whatever
// the range of the weights themselves).
// S: the agent's floor field (the scenario's, or its exit group's); vr: its
// maximum speed (V unless it has one of its own).
// The FP64 weight of window cell t for an agent on cell gc: exp(k_S (S(c) -
// S(t))), times exp(k_D (T(t) - T(c))) with a trail field T (evaluated as
// one exponent, in the order the model's definition writes it).
__device__ __forceinline__ double weight64(const SlotDev &s, const double *__restrict__ S,
                                           const double *__restrict__ T, int gc, int t)
{
    if (T) return exp(s.k_s * (S[gc] - S[t]) + s.k_d * (T[t] - T[gc]));
    return exp(s.k_s * (S[gc] - S[t]));
}

template <int V, bool DEBUG>
__device__ int resolve64_lane(const SlotDev &s, const double *__restrict__ S,
                              const double *__restrict__ T, int gc, int id, float u32, int vr)
{
    constexpr int SIDE = 2 * V + 1;
    double C = 0.0, wmax = 0.0;
#pragma unroll 1
    for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok(s, gc, t, dx, dy, vr)) {
                const double w = weight64(s, S, T, gc, t);
                C = C + w;
                wmax = fmax(wmax, w);
            }
        }
    if (DEBUG && s.dbg_w) {
#pragma unroll 1
        for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
            for (int dx = -V; dx <= V; ++dx) {
                const int t = gc + dy * s.Wp + dx;
                if (reach_ok(s, gc, t, dx, dy, vr))
                    s.dbg_w[(size_t)id * SIDE * SIDE + (dy + V) * SIDE + dx + V] =
                        (float)(weight64(s, S, T, gc, t) / wmax);
            }
    }
    const double tau = (double)u32 * C;
    double C2 = 0.0;
#pragma unroll 1
    for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok(s, gc, t, dx, dy, vr)) {
                C2 = C2 + weight64(s, S, T, gc, t);
                if (tau < C2) return (dy + V) * SIDE + dx + V;
            }
        }
    return V * SIDE + V;   // not reached: the own cell has weight 1 and tau < W
}

// Half widths of the disc's rows, 4 bits per row, row 0 (dy = -V) lowest.
constexpr unsigned long long row_half_widths(int V)
{
    unsigned long long t = 0;
    for (int r = 0; r <= 2 * V; ++r) t |= (unsigned long long)half_width(V, r - V) << (4 * r);
    return t;
}

// The largest |dy| whose disc row holds slot d of its row (0 <= d <= 2V),
// i.e. whose half width a satisfies 2a >= d.
constexpr int max_dy_of_slot(int V, int d)
{
    for (int dy = V; dy > 0; --dy)
        if (2 * half_width(V, dy) >= d) return dy;
    return 0;
}

// Number of slots of the reach disc (5, 13, 29, 49, 81 for v = 1..5).
constexpr int disc_count(int V)
{
    int n = 0;
    for (int dy = -V; dy <= V; ++dy) n += 2 * half_width(V, dy) + 1;
    return n;
}

// (dx, dy) of the j-th slot of the disc in raster order (j < disc_count(V)).
template <int V>
__device__ __forceinline__ void disc_slot(int j, int &dx, int &dy)
{
    int start = 0;
    dy = -V;
    dx = 0;
#pragma unroll
    for (int r = -V; r <= V; ++r) {
        const int a = half_width(V, r);
        const bool in = j >= start;
        dy = in ? r : dy;
        dx = in ? j - start - a : dx;
        start += 2 * a + 1;
    }
}

// Inclusive prefix sum over the 64 lanes of a wavefront in FP64 with DPP
// moves: row shifts by 1, 2, 4, 8 within each 16-lane row, then the row
// broadcasts of lanes 15 and 31.  Every prefix is a sum of depth <= 6.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_take(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_scan64(double x)
{
    x = x + dpp_take<0x111, 0xF>(x);      // row_shr:1
    x = x + dpp_take<0x112, 0xF>(x);      // row_shr:2
    x = x + dpp_take<0x114, 0xF>(x);      // row_shr:4
    x = x + dpp_take<0x118, 0xF>(x);      // row_shr:8
    x = x + dpp_take<0x142, 0xA>(x);      // row_bcast:15 into rows 1, 3
    x = x + dpp_take<0x143, 0xC>(x);      // row_bcast:31 into rows 2, 3
    return x;
}

__device__ __forceinline__ double lane_value(double x, int j)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), j),
                            __builtin_amdgcn_readlane(__double2loint(x), j));
}

// The same draw by a whole wavefront: lane j takes the j-th slot of the reach
// disc in raster order (v <= 4: at most 49 slots) or raster slots j and j + 64
// of the square window (v = 5), and evaluates its weight.
//
// The oracle sums the weights sequentially; a wavefront scan rounds
// differently, but for n <= 128 non-negative terms every scanned prefix and
// W lie within (gamma_n + gamma_7) W < 1.5e-14 W of the sequential ones, and
// tau within that plus two roundings.  So when no prefix lies within
// s.near64 W = 1e-12 W of tau (a 30-fold margin), every comparison tau < C_j,
// and with it the chosen slot, is the same as in the sequential sum;
// otherwise the prefix is rebuilt strictly sequentially, slot by slot (slots
// outside the reach set add exactly nothing), which is bit-identical to
// resolve64_lane.
//
// Reachability is read from the tile's staged window (Em, agent cell l, pitch
// P): on a fast tile a cell is zero there exactly when it is a wall, padding
// or occupied, so only the floor field is read, from global memory (the draws
// that come here are rare).  Returns the chosen raster slot of the window.
template <int V>
__device__ int resolve64_wave(const SlotDev &s, const double *__restrict__ S,
                              const double *__restrict__ T, int gc, float u32, int lane,
                              const float *Em, int l, int P, int vr)
{
    // The lane index passes through an empty asm here, inside the rare branch
    // that calls this: otherwise the compiler hoists the lane-dependent set-up
    // below (slot decoding, one compare per slot) out of the agent loop, and
    // every wavefront pays for it whether or not it has a flagged draw.
    asm volatile("" : "+v"(lane));
    constexpr int SIDE = 2 * V + 1;
    const double NEAR = s.near64;
    const double u = (double)u32;
    if constexpr (disc_count(V) <= 64) {
        constexpr int ND = disc_count(V);
        double w = 0.0;
        int dx = 0, dy = 0;
        disc_slot<V>(lane, dx, dy);
        if (lane < ND && dx * dx + dy * dy <= vr * vr &&
            ((dx == 0 && dy == 0) || Em[l + dy * P + dx] != 0.0f))
            w = weight64(s, S, T, gc, gc + dy * s.Wp + dx);
        const double Cp = wave_scan64(w);
        const double Wp = lane_value(Cp, ND - 1);
        const double tp = u * Wp;
        const bool in = lane < ND;
        unsigned long long m;
        if (__ballot(in && fabs(tp - Cp) <= NEAR * Wp) == 0) {
            m = __ballot(in && tp < Cp);
        } else {
            double C = 0.0, myC = 0.0;
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                C = C + lane_value(w, j);
                if (lane == j) myC = C;
            }
            const double tau = u * C;
            m = __ballot(in && tau < myC);
        }
        const int jw = m ? __builtin_ctzll(m) : (ND - 1) / 2;   // own cell if unreached
        int wx, wy;
        disc_slot<V>(jw, wx, wy);
        return (wy + V) * SIDE + wx + V;
    } else {
        constexpr int NS = SIDE * SIDE;           // 121
        double w[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j < NS) {
                const int dy = j / SIDE - V, dx = j % SIDE - V;
                const bool own = dx == 0 && dy == 0;
                if (dx * dx + dy * dy <= vr * vr && (own || Em[l + dy * P + dx] != 0.0f))
                    w[h] = weight64(s, S, T, gc, gc + dy * s.Wp + dx);
            }
        }
        const double C0 = wave_scan64(w[0]);
        const double C1 = wave_scan64(w[1]) + lane_value(C0, 63);
        const double Wp = lane_value(C1, NS - 65);
        const double tp = u * Wp;
        const bool in1 = lane + 64 < NS;
        unsigned long long m0, m1;
        if (__ballot(fabs(tp - C0) <= NEAR * Wp || (in1 && fabs(tp - C1) <= NEAR * Wp)) == 0) {
            m0 = __ballot(tp < C0);
            m1 = __ballot(in1 && tp < C1);
        } else {
            double C = 0.0, myC0 = 0.0, myC1 = 0.0;
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                C = C + lane_value(w[j / 64], j % 64);
                if (j < 64) { if (lane == j) myC0 = C; }
                else { if (lane == j - 64) myC1 = C; }
            }
            const double tau = u * C;
            m0 = __ballot(tau < myC0);
            m1 = __ballot(in1 && tau < myC1);
        }
        if (m0) return __builtin_ctzll(m0);
        if (m1) return 64 + __builtin_ctzll(m1);
        return V * SIDE + V;                     // not reached
    }
}

// ---------------------------------------------------------------------------
// Planning kernel.
// ---------------------------------------------------------------------------
// A staged tile's agent list and bookkeeping (LDS).
struct TileLists {
    uint32_t a_pk[MAX_TILE_CELLS];      // agents of the tile: id << 12 | LDS cell (id < 2^20)
    float a_ec[MAX_TILE_CELLS];         // e_c of their own cell
    int32_t m_nb[9];                    // exponents of the 3 x 3 tiles around it
    int n_agents, n_flag, fb;
};
struct PlanShared {
    alignas(16) float Em[MAX_STAGE];    // masked exp table window, pitch P = tx + 2 round4(v)
    TileLists L;
};

__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Philox word 0 for the planning draw.  The empty asm marks the key as
// rewritten on every call, so the ten round keys are formed by scalar adds at
// the point of use instead of being kept live across the agent loop (twenty
// scalar registers the kernel cannot spare).
__device__ __forceinline__ uint32_t plan_draw_word(uint32_t id, uint32_t step, uint32_t scn,
                                                   uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);                  // uniform: the scenario's seed
    k1 = __builtin_amdgcn_readfirstlane(k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
    return philox_word0(id, step, scn, STREAM_PLAN, k0, k1);
}

// Geometry of one tile's window: (TX + 2 Hc) x (ty + 2V) cells in 4-cell
// chunks, chunk j = row * cpr + cc (row-major), so that chunk j sits at LDS
// float 4j of the window's table.  The tile's own cells are rows V .. V+ty-1,
// chunk columns hc4 .. hc4+cw-1; interior chunk i (row-major over the tile,
// cw per row) is window chunk in_chunk(i).
template <int V, int TX>
struct TileGeom {
    static constexpr int SIDE = 2 * V + 1;
    static constexpr int Hc = (V + 3) & ~3;                   // column halo, a multiple of 4 >= V
    static constexpr int P = TX + 2 * Hc;                     // LDS pitch = staged width
    static constexpr int cpr = P >> 2;                        // 4-cell chunks per row
    static constexpr int hc4 = Hc >> 2;
    static constexpr int cw = TX >> 2;                        // interior chunks per row
    static constexpr int cw_log = __builtin_ctz(cw);
    int ty, tile_x, tile_y, gx0, gy0, n_win, n_in, n_halo;

    __device__ __forceinline__ TileGeom(const SlotDev &s, int tile)
    {
        ty = s.ty;
        tile_y = tile / s.ntx;
        tile_x = tile - tile_y * s.ntx;
        gx0 = tile_x * TX;                                    // padded column of window column 0
        gy0 = tile_y * ty + Hc - V;                           // padded row of window row 0
        n_win = cpr * (ty + 2 * V);
        n_in = cw * ty;                                       // <= 256
        n_halo = n_win - n_in;
    }
    static __device__ __forceinline__ int in_chunk(int i)
    {
        return (V + (i >> cw_log)) * cpr + hc4 + (i & (cw - 1));
    }
    // halo chunk h: the V rows above, the V rows below, then the hc4 chunks
    // left and right of each interior row
    __device__ __forceinline__ int halo_chunk(int h) const
    {
        constexpr int n_top = V * cpr;
        if (h < 2 * n_top) return h < n_top ? h : h + ty * cpr;
        const int hh = h - 2 * n_top;
        const int rr = (int)((unsigned)hh / (2 * hc4));
        const int c = hh - rr * 2 * hc4;
        return (V + rr) * cpr + (c < hc4 ? c : c + cw);
    }
};

// A buffer resource over `bytes` bytes from p, for loads that go straight to
// LDS (gfx950: buffer_load_dwordx4 ... lds).  Loads past `bytes` read zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lds_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
typedef __attribute__((address_space(3))) void *lds_ptr_t;

// A load through a global (not generic) address: the access is a global_load,
// counted by vmcnt only, so waits for LDS results do not also wait for it.
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
__device__ __forceinline__ int4 gload_i4(const int32_t *p)
{
    typedef int v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(1))) v4 *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
// A D-plane word as a table value: an occupied cell (bit 31 set) reads 0.
// Table values are non-negative floats, so as signed integers they are
// non-negative and the flagged words negative: one integer max does it.
__device__ __forceinline__ float fmask(uint32_t d) { return __int_as_float(max((int)d, 0)); }

// What a thread loads into registers to stage a tile: its interior chunk of
// occupancy (agent ids), and for threads 0..8 / 9 a neighbour tile's exponent
// / the fallback flag.
struct StageRegs {
    int4 oc;
    int mnb, fb;
};

// Issues every load of tile `tile`'s staging without waiting for any: the
// window of D goes straight from memory into the LDS table Em (one 16-byte
// chunk per lane, no registers), the rest into registers.
// Issues the loads of a tile's window of a per-cell 4-byte array `src`
// (Wp x Hp) straight into LDS at Em, chunk j at float 4j.
template <int V, int TX>
__device__ __forceinline__ void issue_window(const void *src, int Wp, int Hp,
                                             const TileGeom<V, TX> &tg, float *Em)
{
    constexpr int cpr = TileGeom<V, TX>::cpr;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    const int wbase = tid - lane;
    const int base = tg.gy0 * Wp + tg.gx0;                    // padded cell of window (0, 0)
    const __amdgpu_buffer_rsrc_t rs = lds_rsrc(src, (uint32_t)((size_t)Wp * Hp * 4));
    for (int j0 = 0; j0 < tg.n_win; j0 += nthr) {
        const int j = j0 + tid;
        if (j < tg.n_win) {
            const int row = (int)((unsigned)j / cpr), cc = j - row * cpr;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (lds_ptr_t)(&Em[4 * (j0 + wbase)]), 16, (uint32_t)(base + row * Wp + 4 * cc) * 4u,
                0, 0, 0);
        }
    }
}

template <int V, int TX>
__device__ __forceinline__ void stage_issue(const SlotDev &s, const TileGeom<V, TX> &tg, int tile,
                                            float *Em, StageRegs &r)
{
    using T = TileGeom<V, TX>;
    const int tid = threadIdx.x;
    const int Wp = s.Wp;
    const int base = tg.gy0 * Wp + tg.gx0;                    // padded cell of window (0, 0)
    issue_window<V, TX>(s.D, Wp, s.Hp, tg, Em);
    r.oc = make_int4(-1, -1, -1, -1);
    if (tid < tg.n_in)
        r.oc = gload_i4(s.occ + base + (V + (tid >> T::cw_log)) * Wp + T::Hc + 4 * (tid & (T::cw - 1)));
    const int tstride = s.ntx + 2;
    r.mnb = 0;
    r.fb = 0;
    if (tid < 9) r.mnb = gload(&s.tile_m[(tg.tile_y + tid / 3) * tstride + tg.tile_x + tid % 3]);
    if (tid == 9) r.fb = gload(&s.tile_fb[tile]);
}

// Turns a tile's loaded window into table values in place -- occupied cells
// (bit 31 set, a negative float) become 0, halo chunks are rescaled by
// 2^(m_T - m_T') to this tile's exponent -- and lists the tile's agents with
// their id and own-cell value.  Every load of the tile's stage_issue must
// have completed.  Ends with a workgroup barrier.
template <int V, int TX>
__device__ __forceinline__ void stage_commit(const TileGeom<V, TX> &tg, float *Em, TileLists &L,
                                             const StageRegs &r)
{
    using T = TileGeom<V, TX>;
    constexpr int cpr = T::cpr;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    if (tid < 9) L.m_nb[tid] = r.mnb;
    if (tid == 9) L.fb = r.fb;
    if (tid == 0) { L.n_agents = 0; L.n_flag = 0; }
    __syncthreads();                                          // raw window, exponents, counters

    // interior chunks: mask in place, list the agents (lane-major order: the
    // list follows the cells in raster order, so a wavefront's agents gather
    // from consecutive LDS banks)
    {
        const bool live = tid < tg.n_in;
        const int j = T::in_chunk(live ? tid : 0);
        uint4 d = make_uint4(0, 0, 0, 0);
        if (live) {
            d = *(const uint4 *)&Em[4 * j];
            *(float4 *)&Em[4 * j] = make_float4(fmask(d.x), fmask(d.y), fmask(d.z), fmask(d.w));
        }
        const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
        const int ov[4] = {r.oc.x, r.oc.y, r.oc.z, r.oc.w};
        unsigned long long m[4];
        int tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) { m[k] = __ballot(live && (dv[k] & D_OCC)); tot += __popcll(m[k]); }
        if (tot) {
            int idx0 = 0;
            if (lane == 0) idx0 = atomicAdd(&L.n_agents, tot);
            int idx = __shfl(idx0, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) idx += lanes_below(m[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (live && (dv[k] & D_OCC)) {
                    L.a_pk[idx] = ((uint32_t)ov[k] << 12) | (uint32_t)(4 * j + k);
                    L.a_ec[idx] = __uint_as_float(dv[k] & ~D_OCC);
                    ++idx;
                }
            }
        }
    }
    // halo chunks: mask and rescale in place
    const int mT = L.m_nb[4];
    for (int h = tid; h < tg.n_halo; h += nthr) {
        const int j = tg.halo_chunk(h);
        const int row = (int)((unsigned)j / cpr), cc = j - row * cpr;
        const int nby = (row >= V) + (row >= V + tg.ty);
        const int nbx = (cc >= T::hc4) + (cc >= T::hc4 + T::cw);   // a chunk lies inside one tile column
        const int dm = mT - L.m_nb[nby * 3 + nbx];
        const uint4 d = *(const uint4 *)&Em[4 * j];
        *(float4 *)&Em[4 * j] = make_float4(ldexpf(fmask(d.x), dm), ldexpf(fmask(d.y), dm),
                                             ldexpf(fmask(d.z), dm), ldexpf(fmask(d.w), dm));
    }
    __syncthreads();
}

// The step counter of scenario s and whether its kernels still act.
__device__ __forceinline__ bool scenario_live(const SlotDev &s, int &step)
{
    step = gload(&s.ctr[C_STEP]);
    return step < gload(&s.ctr[C_LIMIT]);
}

// Stages tile `tile` of scenario s (stage_issue, then stage_commit).  Returns
// false, having waited for its loads, when the scenario has finished its
// steps.
template <int V, int TX>
__device__ __forceinline__ bool stage_tile(const SlotDev &s, const TileGeom<V, TX> &tg, int tile,
                                           float *Em, TileLists &L, int &step)
{
    const bool live = scenario_live(s, step);
    StageRegs r;
    stage_issue<V, TX>(s, tg, tile, Em, r);
    __builtin_amdgcn_s_waitcnt(0);                            // loads into LDS and registers done
    if (!live) return false;                                  // scenario finished: nothing to do
    stage_commit<V, TX>(tg, Em, L, r);
    return true;
}

// What the draws of a tile need for per-agent speeds and several floor fields
// (the richer situations of Sec. 3; see plan_het.hip): each listed agent's
// field and maximum speed, one staged window per field, per-field fallback
// flags, and the fields themselves for the FP64 paths.
struct HetView {
    const uint8_t *a_gv;      // LDS, per listed agent: field << 4 | maximum speed
    const int *fbf;           // LDS, per field: the tile is a range-fallback tile for it
    const double *Sf;         // floor fields field_cells apart, or null: the scenario's S
    long field_cells;
    int win;                  // floats per staged window
};

// The draws of a staged tile: one lane per agent (FP32 from the LDS table,
// flagged draws re-resolved in FP64 by their wavefront), or every draw in
// FP64 on a fallback tile.  The record of the tile's k-th agent (its cell in
// the tile and the window slot it chose; the middle slot when it stays) goes
// to slot k of the tile's segment, and the segment count is the tile's agent
// count.  HET: agent k reads its field's window (Em + field * win) and
// reaches only its own disc dx^2 + dy^2 <= vr^2 (the other slots weigh an
// exact 0); a field for which the tile is a fallback tile draws in FP64.
// Ends with a workgroup barrier after which only thread 0 touches the LDS
// counters.
template <int V, int TX, bool DEBUG, bool HET>
__device__ __forceinline__ void plan_agents(const SlotDev &s, const TileGeom<V, TX> &tg, int tile,
                                            const float *Em, TileLists &sh, int step,
                                            const HetView &hv)
{
    using T = TileGeom<V, TX>;
    constexpr int SIDE = T::SIDE, P = T::P, Hc = T::Hc;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    uint32_t *seg = s.seg + (long)tile * (TX * tg.ty);
    const int na = sh.n_agents;
    const uint32_t kseed0 = s.seed_lo, kseed1 = s.seed_hi;
    const uint32_t scn = s.scn;          // held in registers: the loops below store to memory
    const float eps = s.eps;
    // the tile-local cell of LDS cell l (window row ly, column lx)
    auto lcell_of = [&](int l) {
        const int ly = (int)((unsigned)l / P);
        return (ly - V) * TX + (l - ly * P - Hc);
    };
    // the trail of this step, when the scenario keeps one
    const double *Tcur = s.Tr ? s.Tr + (long)(step & 1) * ((long)s.Wp * s.Hp) : nullptr;
    auto cell_of = [&](int l) {
        const int ly = (int)((unsigned)l / P);
        return (tg.gy0 + ly) * s.Wp + tg.gx0 + (l - ly * P);
    };
    // agent k's field, window, floor field, reach and fallback flag
    auto agent_view = [&](int k, int &vr, const float *&E, const double *&S, bool &fb) {
        vr = V;
        E = Em;
        S = s.S;
        fb = false;
        if constexpr (HET) {
            const int gv = hv.a_gv[k], g = gv >> 4;
            vr = gv & 15;
            E = Em + g * hv.win;
            if (hv.Sf) S = hv.Sf + g * hv.field_cells;
            fb = hv.fbf[g] != 0;
        }
    };

    if (!HET && sh.fb) {
        // every draw of this tile in FP64, one lane per agent
        for (int base = 0; base < na; base += nthr) {
            const int k = base + tid;
            if (k < na) {
                const int id = (int)(sh.a_pk[k] >> 12);
                const int l = (int)(sh.a_pk[k] & 0xFFFu);
                const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int slot = resolve64_lane<V, DEBUG>(s, s.S, Tcur, cell_of(l), id, u, V);
                seg[k] = plan_rec(lcell_of(l), slot);
                if (DEBUG && s.dbg_flag) s.dbg_flag[id] = 2;
                if (DEBUG && s.dbg_margin) s.dbg_margin[id] = -1.0f;
            }
        }
        if (tid == 0) {
            s.seg_cnt[tile] = na;
            if (na > 0) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)na);
        }
        __syncthreads();
        return;
    }

    // --- one lane per agent, FP32 from the LDS table
    int n_fb = 0;                        // HET: draws of this thread on fallback fields
    for (int base = 0; base < na; base += nthr) {
        const int k = base + tid;
        bool flagged = false;
        if (k < na) {
            const int id = (int)(sh.a_pk[k] >> 12);
            const int l = (int)(sh.a_pk[k] & 0xFFFu);
            const float ec = sh.a_ec[k];
            int vr;
            const float *E;
            const double *S;
            bool fbk;
            agent_view(k, vr, E, S, fbk);
            if (HET && fbk) {
                const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int slot = resolve64_lane<V, DEBUG>(s, S, Tcur, cell_of(l), id, u, vr);
                seg[k] = plan_rec(lcell_of(l), slot);
                if (DEBUG && s.dbg_flag) s.dbg_flag[id] = 2;
                if (DEBUG && s.dbg_margin) s.dbg_margin[id] = -1.0f;
                ++n_fb;
            } else {
            const int vr2 = vr * vr;
            const Window<V, P> win(E, l - V * P - V);         // origin (dy, dx) = (-V, -V)
            float Rs[SIDE], row0[SIDE], row1[SIDE];
            load_row<V, P, 0, HET>(win, ec, vr2, row0);
            load_row<V, P, 1, HET>(win, ec, vr2, row1);
            __builtin_amdgcn_sched_barrier(0);
            // the draw's counter-based word overlaps the first rows' LDS reads
            const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0, kseed1);
            __builtin_amdgcn_sched_barrier(0);
            RowPipe<V, P, 0, HET>::run(win, ec, vr2, Rs, row0, row1);
            float Pr[SIDE + 1];
            Pr[0] = 0.0f;
            Pr[1] = Rs[0];
#pragma unroll
            for (int r = 1; r < SIDE; ++r) Pr[r + 1] = Pr[r] + Rs[r];
            const float Wsum = Pr[SIDE];

            const float u = (float)(x0 >> 8) * 0x1p-24f;
            const float tau = u * Wsum;

            // row: the last r with Pr_r <= tau (the row prefixes never
            // decrease, so that is the number of them <= tau)
            int rs = 0;
            float Ps = 0.0f;
#pragma unroll
            for (int r = 1; r < SIDE; ++r) {
                const bool le = Pr[r] <= tau;
                rs += le ? 1 : 0;
                Ps = le ? Pr[r] : Ps;
            }
            const int as = (int)((row_half_widths(V) >> (4 * rs)) & 15u);
            // slot within the row: count of in-row boundaries <= tau.  The
            // row's cells are read at once (slots past 2a stay inside the
            // LDS block and are not used).
            const float *rb = win.b[0] + rs * P + (V - as);
            float rv[SIDE];
#pragma unroll
            for (int d = 0; d < SIDE; ++d) rv[d] = rb[d];
            // (the own cell is the middle slot, d = V, of the middle row).
            // Slots past the row's end (d > 2a) add an exact 0, so their C
            // repeats the row's last boundary: if that boundary is <= tau,
            // ks > 2a flags the draw whatever they add to ks; otherwise they
            // add nothing to ks, and the near test sees the same value again.
            // So every lane runs all SIDE slots without branching.
            const bool own_row = rs == V;
            const int rdy2 = (rs - V) * (rs - V);
            const int ady = rs < V ? V - rs : rs - V;        // |dy| of the chosen row
            const float thr = eps * Wsum;
            float Q = 0.0f;
            float margin = fabsf(tau - Ps);                  // smallest |tau - C| (debug output)
            bool near = margin <= thr;
            int ks = 0;
#pragma unroll
            for (int d = 0; d < SIDE; ++d) {
                float val = (d == V && own_row) ? ec : rv[d];
                if (d > 0) val = ady <= max_dy_of_slot(V, d) ? val : 0.0f;
                if constexpr (HET) val = (d - as) * (d - as) + rdy2 <= vr2 ? val : 0.0f;
                Q = Q + val;
                const float C = Ps + Q;
                const float diff = tau - C;
                ks += diff >= 0.0f ? 1 : 0;
                near = near || fabsf(diff) <= thr;
                if constexpr (DEBUG) margin = fminf(margin, fabsf(diff));
            }
            const bool flag = near || (ks > 2 * as);

            if constexpr (DEBUG) {
                // weights over the largest weight of the reach set (the CDF
                // depends on ratios only, and these all lie in [0, 1]); the
                // FP32 CDF at every disc slot exactly as the draw forms it
                // (row prefix Pr plus the sequential in-row sum), and the
                // total W in the window's last slot, a corner outside the disc
                auto wt = [&](int dx, int dy) {
                    if (dx == 0 && dy == 0) return ec;
                    return dx * dx + dy * dy <= vr2 ? E[l + dy * P + dx] : 0.0f;
                };
                float emax = ec;
                for (int dy = -V; dy <= V; ++dy)
                    for (int dx = -V; dx <= V; ++dx)
                        if (dx * dx + dy * dy <= V * V) emax = fmaxf(emax, wt(dx, dy));
                if (s.dbg_w) {
                    float *wd = s.dbg_w + (size_t)id * SIDE * SIDE;
                    for (int dy = -V; dy <= V; ++dy)
                        for (int dx = -V; dx <= V; ++dx)
                            wd[(dy + V) * SIDE + dx + V] =
                                dx * dx + dy * dy <= V * V ? wt(dx, dy) / emax : 0.0f;
                }
                if (s.dbg_cdf) {
                    float *cd = s.dbg_cdf + (size_t)id * SIDE * SIDE;
                    for (int r = 0; r < SIDE; ++r) {
                        const int a = (int)((row_half_widths(V) >> (4 * r)) & 15u);
                        float q = 0.0f;
                        for (int d = 0; d <= 2 * a; ++d) {
                            q = q + wt(d - a, r - V);
                            cd[r * SIDE + (V - a) + d] = Pr[r] + q;
                        }
                    }
                    cd[SIDE * SIDE - 1] = Wsum;
                }
                if (s.dbg_flag) s.dbg_flag[id] = flag ? 1 : 0;
                if (s.dbg_margin) s.dbg_margin[id] = margin / Wsum;
            }
            if (!flag) seg[k] = plan_rec(lcell_of(l), rs * SIDE + (ks - as + V));
            flagged = flag;
            }
        }

        // FP64 re-resolve of this wavefront's flagged draws, one draw at a
        // time by the whole wavefront, without waiting for the other waves
        unsigned long long fm = __ballot(flagged);
        if (fm) {
            if (lane == 0) atomicAdd(&sh.n_flag, __popcll(fm));
            while (fm) {
                const int src = __builtin_ctzll(fm);
                fm &= fm - 1ull;
                const int kk = base + (tid & ~63) + src;
                const int fid = (int)(sh.a_pk[kk] >> 12);
                const int l = (int)(sh.a_pk[kk] & 0xFFFu);
                int vr;
                const float *E;
                const double *S;
                bool fbk;
                agent_view(kk, vr, E, S, fbk);
                const uint32_t x0 = plan_draw_word((uint32_t)fid, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int slot = resolve64_wave<V>(s, S, Tcur, cell_of(l), u, lane, E, l, P, vr);
                if (lane == 0) seg[kk] = plan_rec(lcell_of(l), slot);
            }
        }
    }
    if (HET && n_fb) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)n_fb);
    __syncthreads();
    if (tid == 0) {
        const int nf = sh.n_flag;
        s.seg_cnt[tile] = na;
        if (nf) atomicAdd(&s.stat[S_FLAGGED], (unsigned long long)nf);
    }
}


// One tile, V = v_max, TX = tile width (a power of two, 8..64): both fix the
// LDS pitch, so every window offset of the agent loop is a compile-time
// constant.
template <int V, int TX, bool DEBUG>
__device__ __forceinline__ void plan_tile(const SlotDev &s, int tile, PlanShared &sh)
{
    const TileGeom<V, TX> tg(s, tile);
    int step = 0;
    if (!stage_tile<V, TX>(s, tg, tile, sh.Em, sh.L, step)) return;
    if (tile == 0 && threadIdx.x < 4) s.ctr[C_BAR + threadIdx.x] = 0;   // fresh motion barriers
    plan_agents<V, TX, DEBUG, false>(s, tg, tile, sh.Em, sh.L, step, HetView{});
}

template <int V, bool DEBUG>
__device__ __forceinline__ void plan_dispatch_tx(const SlotDev &s, int tile, PlanShared &sh)
{
    switch (s.tx) {
        case 8: plan_tile<V, 8, DEBUG>(s, tile, sh); break;
        case 16: plan_tile<V, 16, DEBUG>(s, tile, sh); break;
        case 32: plan_tile<V, 32, DEBUG>(s, tile, sh); break;
        case 64: plan_tile<V, 64, DEBUG>(s, tile, sh); break;
        default: break;
    }
}

// Device-side dispatch over (v_max, tile width): one launch can mix scenarios.
template <bool DEBUG>
__device__ __forceinline__ void plan_dispatch(const SlotDev &s, int tile, PlanShared &sh)
{
    switch (s.v) {
        case 1: plan_dispatch_tx<1, DEBUG>(s, tile, sh); break;
        case 2: plan_dispatch_tx<2, DEBUG>(s, tile, sh); break;
        case 3: plan_dispatch_tx<3, DEBUG>(s, tile, sh); break;
        case 4: plan_dispatch_tx<4, DEBUG>(s, tile, sh); break;
        case 5: plan_dispatch_tx<5, DEBUG>(s, tile, sh); break;
        default: break;
    }
}

}  // namespace fk
