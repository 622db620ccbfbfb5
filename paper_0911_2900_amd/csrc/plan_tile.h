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
// agent's own cell takes e_c.
template <int V, int P, int R>
__device__ __forceinline__ void load_row(const Window<V, P> &w, float ec, float (&x)[2 * V + 1])
{
    constexpr int a = half_width(V, R - V);
    const float *rp = w.template row<R>();
#pragma unroll
    for (int k = 0; k <= 2 * a; ++k) {
        if (R == V && k == a) x[k] = ec;
        else x[k] = rp[(V - a) + k];
    }
}

// Row sums, software-pipelined by two rows: the loads of row R+2 are issued
// before row R is summed, and the scheduling barrier keeps later rows from
// being hoisted, so at most three rows of values are live.
template <int V, int P, int R>
struct RowPipe {
    static __device__ __forceinline__ void run(const Window<V, P> &w, float ec, float *Rs,
                                               const float (&cur)[2 * V + 1],
                                               const float (&nx1)[2 * V + 1])
    {
        constexpr int a = half_width(V, R - V);
        float nx2[2 * V + 1];
        if constexpr (R + 2 < 2 * V + 1) load_row<V, P, R + 2>(w, ec, nx2);
        Rs[R] = Tree<2 * a + 1, 0>::sum(cur);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (R + 1 < 2 * V + 1) RowPipe<V, P, R + 1>::run(w, ec, Rs, nx1, nx2);
    }
};

// ---------------------------------------------------------------------------
// FP64 draw, the test oracle's arithmetic: weights exp(k_S (S(c) - S(t))) over
// the square window in raster order (zero outside the reach set), sequential
// sum, tau = u * W, first slot with tau < C.  One lane does one agent.
// ---------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ bool reach_ok(const SlotDev &s, int gc, int t, int dx, int dy)
{
    if (dx * dx + dy * dy > V * V) return false;
    if ((s.cell[t] & CELL_TYPE_MASK) == CELL_WALL) return false;
    const int o = s.occ[t];
    return o < 0 || t == gc;
}

// (The loops stay rolled: this path is rare, and unrolled FP64 exp code would
// raise the register count of the whole planning kernel.)  The debug form
// also writes each slot's weight over the largest weight of the reach set,
// rounded to FP32 (every such ratio lies in [0, 1], so FP32 holds it whatever
// the range of the weights themselves).
template <int V, bool DEBUG>
__device__ int resolve64_lane(const SlotDev &s, int gc, int id, float u32)
{
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    double C = 0.0, wmax = 0.0;
#pragma unroll 1
    for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok<V>(s, gc, t, dx, dy)) {
                const double w = exp(ks * (Sc - s.S[t]));
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
                if (reach_ok<V>(s, gc, t, dx, dy))
                    s.dbg_w[(size_t)id * (2 * V + 1) * (2 * V + 1) + (dy + V) * (2 * V + 1) + dx + V] =
                        (float)(exp(ks * (Sc - s.S[t])) / wmax);
            }
    }
    const double tau = (double)u32 * C;
    double C2 = 0.0;
#pragma unroll 1
    for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok<V>(s, gc, t, dx, dy)) {
                C2 = C2 + exp(ks * (Sc - s.S[t]));
                if (tau < C2) return t;
            }
        }
    return gc;   // not reached: the own cell has weight 1 and tau < W
}

// Half widths of the disc's rows, 4 bits per row, row 0 (dy = -V) lowest.
constexpr unsigned long long row_half_widths(int V)
{
    unsigned long long t = 0;
    for (int r = 0; r <= 2 * V; ++r) t |= (unsigned long long)half_width(V, r - V) << (4 * r);
    return t;
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
// or occupied, so only the floor field needs reads: from LDS with SS (Sw, the
// same layout as Em), else from global memory.
template <int V, bool SS>
__device__ int resolve64_wave(const SlotDev &s, int gc, float u32, int lane, const float *Em,
                              const double *Sw, int l, int P)
{
    const double NEAR = s.near64;
    auto S_at = [&](int dx, int dy) -> double {
        if constexpr (SS) return Sw[l + dy * P + dx];
        else return s.S[gc + dy * s.Wp + dx];
    };
    const double Sc = S_at(0, 0);
    const double ks = s.k_s;
    const double u = (double)u32;
    if constexpr (disc_count(V) <= 64) {
        constexpr int ND = disc_count(V);
        double w = 0.0;
        int dx = 0, dy = 0;
        disc_slot<V>(lane, dx, dy);
        if (lane < ND && ((dx == 0 && dy == 0) || Em[l + dy * P + dx] != 0.0f))
            w = exp(ks * (Sc - S_at(dx, dy)));
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
        return gc + wy * s.Wp + wx;
    } else {
        constexpr int SIDE = 2 * V + 1;
        constexpr int NS = SIDE * SIDE;           // 121
        double w[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j < NS) {
                const int dy = j / SIDE - V, dx = j % SIDE - V;
                const bool own = dx == 0 && dy == 0;
                if (dx * dx + dy * dy <= V * V && (own || Em[l + dy * P + dx] != 0.0f))
                    w[h] = exp(ks * (Sc - S_at(dx, dy)));
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
        int j;
        if (m0) j = __builtin_ctzll(m0);
        else if (m1) j = 64 + __builtin_ctzll(m1);
        else j = V * SIDE + V;                   // not reached
        return gc + (j / SIDE - V) * s.Wp + (j % SIDE - V);
    }
}

// ---------------------------------------------------------------------------
// Planning kernel.
// ---------------------------------------------------------------------------
struct PlanSharedBase {
    alignas(16) float Em[MAX_STAGE];    // masked exp table window, pitch P = tx + 2 round4(v)
    uint32_t a_pk[MAX_TILE_CELLS];      // agents of the tile: id << 12 | LDS cell (id < 2^20)
    float a_ec[MAX_TILE_CELLS];         // e_c of their own cell
    int32_t m_nb[9];
    int n_agents, n_flag;
};
template <bool SS>
struct PlanShared : PlanSharedBase {};
template <>
struct PlanShared<true> : PlanSharedBase {
    alignas(16) double Sw[MAX_STAGE];   // floor-field window, same layout as Em
};

__device__ __forceinline__ uint32_t pack_xy(int x, int y) { return (uint32_t)x | ((uint32_t)y << 16); }

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

// Geometry of one tile's staging: tile (tile_x, tile_y), the padded origin of
// its window, and the 16-byte chunks of the window this thread stages (one
// interior chunk, up to two halo chunks: V rows above and below, then hc4
// chunks left and right of the interior).
template <int V, int TX>
struct TileGeom {
    static constexpr int SIDE = 2 * V + 1;
    static constexpr int Hc = (V + 3) & ~3;                   // column halo, a multiple of 4 >= V
    static constexpr int P = TX + 2 * Hc;                     // LDS pitch = staged width
    static constexpr int cpr = P >> 2;                        // 4-cell chunks per row
    static constexpr int hc4 = Hc >> 2;
    static constexpr int cw = TX >> 2;                        // interior chunks per row
    static constexpr int cw_log = __builtin_ctz(cw);
    int n_in, n_top, n_halo, tile_x, tile_y, gx0, gy0, ly_in, cc_in, ly_h[2], cc_h[2];

    __device__ __forceinline__ TileGeom(const SlotDev &s, int tile)
    {
        const int tid = threadIdx.x, nthr = blockDim.x;
        n_in = cw * s.ty;                                     // interior chunks (<= nthr)
        n_top = V * cpr;
        n_halo = 2 * n_top + s.ty * 2 * hc4;
        tile_y = tile / s.ntx;
        tile_x = tile - tile_y * s.ntx;
        gx0 = tile_x * TX;
        gy0 = tile_y * s.ty + Hc - V;
        ly_in = V + (tid >> cw_log);
        cc_in = hc4 + (tid & (cw - 1));
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int h = tid + j * nthr;
            int ly, cc;
            if (h < 2 * n_top) {                              // rows above, then rows below
                const int hh = h < n_top ? h : h - n_top;
                ly = (int)((unsigned)hh / cpr);
                cc = hh - ly * cpr;
                if (h >= n_top) ly += V + s.ty;
            } else {                                          // left / right columns
                const int hh = h - 2 * n_top;
                const int rr = (int)((unsigned)hh / (2 * hc4));
                const int c = hh - rr * 2 * hc4;
                ly = V + rr;
                cc = c < hc4 ? c : c + cw;
            }
            ly_h[j] = ly;
            cc_h[j] = cc;
        }
    }
};

// A load through a global (not generic) address: the access is a global_load,
// counted by vmcnt only, so waits for LDS results do not also wait for it.
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
// 16-byte forms (through the native vector types: the HIP vector classes
// cannot be copied out of another address space).
__device__ __forceinline__ int4 gload_i4(const int32_t *p)
{
    typedef int v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(1))) v4 *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 gload_f4(const float *p)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(1))) v4 *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gload_d2(const double *p)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2 *)p;
    return double2{v.x, v.y};
}
// A planned record, stored through a global address.
__device__ __forceinline__ void gstore_rec(MoveRec *p, uint32_t id, uint32_t cxy, uint32_t dxy)
{
    typedef uint32_t v3 __attribute__((ext_vector_type(3)));
    v3 v;
    v.x = id;
    v.y = cxy;
    v.z = dxy;
    *(__attribute__((address_space(1))) v3 *)p = v;
}

// What a thread loads from global memory to stage one tile.
template <bool SS>
struct StageRegs {
    int4 o_in, o_h0, o_h1;
    float4 g_in, g_h0, g_h1;
    double4 s_in, s_h0, s_h1;                                 // floor field (SS only)
    int mnb;                                                  // scale exponent of a neighbour tile
    int fb;                                                   // the tile is a fallback tile
};

// Issues every global load of a tile's staging (16-byte chunks of occupancy,
// exp table and, with SS, floor field; the 3x3 tile scale exponents; the
// fallback flag) without waiting for any of them.
template <int V, int TX, bool SS>
__device__ __forceinline__ void stage_issue(const SlotDev &s, const TileGeom<V, TX> &tg,
                                            StageRegs<SS> &r)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int tstride = s.ntx + 2;
    const int *tm = &s.tile_m[(tg.tile_y + tid / 3) * tstride + tg.tile_x + tid % 3];
    const uint8_t *tf = &s.tile_fb[tg.tile_y * s.ntx + tg.tile_x];
    r.mnb = tid < 9 ? (SS ? *tm : gload(tm)) : 0;
    r.fb = SS ? *tf : gload(tf);
    r.o_in = r.o_h0 = r.o_h1 = make_int4(-1, -1, -1, -1);
    r.g_in = r.g_h0 = r.g_h1 = make_float4(0.f, 0.f, 0.f, 0.f);
    // Launches that stage the floor field (single scenarios, descriptor by
    // value: the compiler already knows the arrays are global) use plain
    // loads; the others read descriptors from memory, where plain loads would
    // be generic (flat) ones, counted against the LDS wait counter too.
    auto load = [&](int g, int4 &o, float4 &gv, double4 &d) {
        if constexpr (SS) {
            o = *(const int4 *)(s.occ + g);
            gv = *(const float4 *)(s.G + g);
            const double2 x = *(const double2 *)(s.S + g), y = *(const double2 *)(s.S + g + 2);
            d = double4{x.x, x.y, y.x, y.y};
        } else {
            o = gload_i4(s.occ + g);
            gv = gload_f4(s.G + g);
        }
    };
    if (tid < tg.n_in) load((tg.gy0 + tg.ly_in) * s.Wp + tg.gx0 + 4 * tg.cc_in, r.o_in, r.g_in, r.s_in);
    if (tid < tg.n_halo)
        load((tg.gy0 + tg.ly_h[0]) * s.Wp + tg.gx0 + 4 * tg.cc_h[0], r.o_h0, r.g_h0, r.s_h0);
    if (tid + nthr < tg.n_halo)
        load((tg.gy0 + tg.ly_h[1]) * s.Wp + tg.gx0 + 4 * tg.cc_h[1], r.o_h1, r.g_h1, r.s_h1);
}

// Writes the staged tile into LDS (halo chunks rescaled to the tile's
// exponent, occupied cells masked) and lists the tile's agents.  Only thread 0
// may have touched the LDS counters since the workgroup's last barrier.
template <int V, int TX, bool SS>
__device__ __forceinline__ void stage_commit(const SlotDev &s, const TileGeom<V, TX> &tg,
                                             PlanShared<SS> &sh, const StageRegs<SS> &r)
{
    using T = TileGeom<V, TX>;
    constexpr int P = T::P, hc4 = T::hc4, cw = T::cw;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    const int ci = tid, n_in = tg.n_in, n_halo = tg.n_halo, ly_in = tg.ly_in, cc_in = tg.cc_in;
    const int *ly_h = tg.ly_h, *cc_h = tg.cc_h;
    if (tid < 9) sh.m_nb[tid] = r.mnb;
    if (tid == 0) { sh.n_agents = 0; sh.n_flag = 0; }
    __syncthreads();                                          // m_nb, counters ready
    const int mT = sh.m_nb[4];

    // halo chunks: rescale to this tile's exponent, mask occupied cells
    auto stage_S = [&](int l0, const double4 &d) {
        if constexpr (SS) {
            *(double2 *)&sh.Sw[l0] = double2{d.x, d.y};
            *(double2 *)&sh.Sw[l0 + 2] = double2{d.z, d.w};
        }
    };
    auto stage_halo = [&](int ly, int cc, int4 o, float4 gv) {
        const int nby = (ly >= V) + (ly >= V + s.ty);
        const int nbx = (cc >= hc4) + (cc >= hc4 + cw);       // a chunk lies inside one tile column
        const int dm = mT - sh.m_nb[nby * 3 + nbx];
        *(float4 *)&sh.Em[ly * P + 4 * cc] =
            make_float4(o.x < 0 ? ldexpf(gv.x, dm) : 0.f, o.y < 0 ? ldexpf(gv.y, dm) : 0.f,
                        o.z < 0 ? ldexpf(gv.z, dm) : 0.f, o.w < 0 ? ldexpf(gv.w, dm) : 0.f);
    };
    if (tid < n_halo) {
        stage_halo(ly_h[0], cc_h[0], r.o_h0, r.g_h0);
        stage_S(ly_h[0] * P + 4 * cc_h[0], r.s_h0);
    }
    if (tid + nthr < n_halo) {
        stage_halo(ly_h[1], cc_h[1], r.o_h1, r.g_h1);
        stage_S(ly_h[1] * P + 4 * cc_h[1], r.s_h1);
    }

    // interior chunk: already in the tile's scale; its occupied cells are the
    // tile's agents (one LDS atomic per wavefront to list them)
    {
        const int4 o_in = r.o_in;
        const float4 g_in = r.g_in;
        const bool live = ci < n_in;
        const int l0 = ly_in * P + 4 * cc_in;
        if (live) {
            *(float4 *)&sh.Em[l0] = make_float4(o_in.x < 0 ? g_in.x : 0.f, o_in.y < 0 ? g_in.y : 0.f,
                                                o_in.z < 0 ? g_in.z : 0.f, o_in.w < 0 ? g_in.w : 0.f);
            stage_S(l0, r.s_in);
        }
        const int ov[4] = {o_in.x, o_in.y, o_in.z, o_in.w};
        const float gv[4] = {g_in.x, g_in.y, g_in.z, g_in.w};
        unsigned long long m[4];
        int tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) { m[k] = __ballot(live && ov[k] >= 0); tot += __popcll(m[k]); }
        if (tot) {
            // lane-major order: the list follows the cells in raster order, so
            // a wavefront's agents gather from consecutive LDS banks
            int base = 0;
            if (lane == 0) base = atomicAdd(&sh.n_agents, tot);
            int idx = __shfl(base, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) idx += lanes_below(m[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (live && ov[k] >= 0) {
                    sh.a_pk[idx] = ((uint32_t)ov[k] << 12) | (uint32_t)(l0 + k);
                    sh.a_ec[idx] = gv[k];
                    ++idx;
                }
            }
        }
    }
    __syncthreads();
}

// The draws of a staged tile: one lane per agent (FP32 from the LDS table,
// flagged draws re-resolved in FP64 by their wavefront), or every draw in
// FP64 on a fallback tile.  The record of the tile's k-th agent (id, cell,
// chosen cell; the chosen cell is its own when it stays) goes to slot k of
// the tile's segment, and the segment count is the tile's agent count.  Ends
// with a workgroup barrier after which only thread 0 touches the LDS counters.
template <int V, int TX, bool DEBUG, bool SS>
__device__ __forceinline__ void plan_agents(const SlotDev &s, const TileGeom<V, TX> &tg, int tile,
                                            PlanShared<SS> &sh, int step, bool fallback)
{
    using T = TileGeom<V, TX>;
    constexpr int SIDE = T::SIDE, P = T::P, Hc = T::Hc;
    (void)Hc;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    const int gx0 = tg.gx0, gy0 = tg.gy0;
    MoveRec *seg = s.seg + (long)tile * (TX * s.ty);
    const int na = sh.n_agents;
    const uint32_t kseed0 = s.seed_lo, kseed1 = s.seed_hi;
    const uint32_t scn = s.scn;          // held in registers: the loops below store to memory
    const float eps = s.eps;

    if (fallback) {
        // every draw of this tile in FP64, one lane per agent
        for (int base = 0; base < na; base += nthr) {
            const int k = base + tid;
            if (k < na) {
                const int id = (int)(sh.a_pk[k] >> 12);
                const int l = (int)(sh.a_pk[k] & 0xFFFu);
                const int ly = (int)((unsigned)l / P);
                const int cx = gx0 + (l - ly * P), cy = gy0 + ly;
                const int gc = cy * s.Wp + cx;
                const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int t = resolve64_lane<V, DEBUG>(s, gc, id, u);
                const int d = t - gc;                       // |dx|, |dy| <= V < Wp / 2
                const int ddy = (d + V * s.Wp + V) / s.Wp - V, ddx = d - ddy * s.Wp;
                gstore_rec(seg + k, (uint32_t)id, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy));
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
    for (int base = 0; base < na; base += nthr) {
        const int k = base + tid;
        bool flagged = false;
        if (k < na) {
            const int id = (int)(sh.a_pk[k] >> 12);
            const int l = (int)(sh.a_pk[k] & 0xFFFu);
            const float ec = sh.a_ec[k];
            const int ly = (int)((unsigned)l / P);
            const int cx = gx0 + (l - ly * P), cy = gy0 + ly;

            const Window<V, P> win(sh.Em, l - V * P - V);     // origin (dy, dx) = (-V, -V)
            float Rs[SIDE], row0[SIDE], row1[SIDE];
            load_row<V, P, 0>(win, ec, row0);
            load_row<V, P, 1>(win, ec, row1);
            __builtin_amdgcn_sched_barrier(0);
            // the draw's counter-based word overlaps the first rows' LDS reads
            const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0, kseed1);
            __builtin_amdgcn_sched_barrier(0);
            RowPipe<V, P, 0>::run(win, ec, Rs, row0, row1);
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
            // (the own cell is the middle slot, d = V, of the middle row)
            const bool own_row = rs == V;
            const float thr = eps * Wsum;
            float Q = 0.0f;
            float margin = fabsf(tau - Ps);                  // smallest |tau - C| (debug output)
            bool near = margin <= thr;
            int ks = 0;
#pragma unroll
            for (int d = 0; d < SIDE; ++d) {
                if (d <= 2 * as) {
                    const float val = (d == V && own_row) ? ec : rv[d];
                    Q = Q + val;
                    const float C = Ps + Q;
                    const float diff = tau - C;
                    ks += diff >= 0.0f ? 1 : 0;
                    near = near || fabsf(diff) <= thr;
                    if constexpr (DEBUG) margin = fminf(margin, fabsf(diff));
                }
            }
            const bool flag = near || (ks > 2 * as);

            if constexpr (DEBUG) {
                // weights over the largest weight of the reach set (the CDF
                // depends on ratios only, and these all lie in [0, 1]); the
                // FP32 CDF at every disc slot exactly as the draw forms it
                // (row prefix Pr plus the sequential in-row sum), and the
                // total W in the window's last slot, a corner outside the disc
                float emax = ec;
                for (int dy = -V; dy <= V; ++dy)
                    for (int dx = -V; dx <= V; ++dx)
                        if (dx * dx + dy * dy <= V * V && !(dx == 0 && dy == 0))
                            emax = fmaxf(emax, sh.Em[l + dy * P + dx]);
                if (s.dbg_w) {
                    float *wd = s.dbg_w + (size_t)id * SIDE * SIDE;
                    for (int dy = -V; dy <= V; ++dy)
                        for (int dx = -V; dx <= V; ++dx) {
                            float wv = 0.0f;
                            if (dx * dx + dy * dy <= V * V)
                                wv = ((dx == 0 && dy == 0) ? ec : sh.Em[l + dy * P + dx]) / emax;
                            wd[(dy + V) * SIDE + dx + V] = wv;
                        }
                }
                if (s.dbg_cdf) {
                    float *cd = s.dbg_cdf + (size_t)id * SIDE * SIDE;
                    for (int r = 0; r < SIDE; ++r) {
                        const int a = (int)((row_half_widths(V) >> (4 * r)) & 15u);
                        float q = 0.0f;
                        for (int d = 0; d <= 2 * a; ++d) {
                            const int dx = d - a, dy = r - V;
                            q = q + ((dx == 0 && dy == 0) ? ec : sh.Em[l + dy * P + dx]);
                            cd[r * SIDE + (V - a) + d] = Pr[r] + q;
                        }
                    }
                    cd[SIDE * SIDE - 1] = Wsum;
                }
                if (s.dbg_flag) s.dbg_flag[id] = flag ? 1 : 0;
                if (s.dbg_margin) s.dbg_margin[id] = margin / Wsum;
            }
            if (!flag) {
                const int ddx = ks - as, ddy = rs - V;
                gstore_rec(seg + k, (uint32_t)id, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy));
            }
            flagged = flag;
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
                const int ly = (int)((unsigned)l / P);
                const int cx = gx0 + (l - ly * P), cy = gy0 + ly;
                const int gc = cy * s.Wp + cx;
                const uint32_t x0 = plan_draw_word((uint32_t)fid, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const double *Sw = nullptr;
                if constexpr (SS) Sw = sh.Sw;
                const int t = resolve64_wave<V, SS>(s, gc, u, lane, sh.Em, Sw, l, P);
                if (lane == 0) {
                    const int d = t - gc;
                    const int ddy = (d + V * s.Wp + V) / s.Wp - V, ddx = d - ddy * s.Wp;
                    gstore_rec(seg + kk, (uint32_t)fid, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy));
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int nf = sh.n_flag;
        s.seg_cnt[tile] = na;
        if (nf) atomicAdd(&s.stat[S_FLAGGED], (unsigned long long)nf);
    }
}


// One tile, V = v_max, TX = tile width (a power of two, 8..64): both fix the
// LDS pitch, so every window offset of the agent loop is a compile-time
// constant.  SS stages the floor-field window too (launches too small to hide
// the global latency of the rare FP64 re-resolve).
template <int V, int TX, bool DEBUG, bool SS>
__device__ __forceinline__ void plan_tile(const SlotDev &s, int tile, PlanShared<SS> &sh)
{
    // the step counter is loaded first and read once the staging loads are
    // in flight
    const int step = SS ? s.ctr[C_STEP] : gload(&s.ctr[C_STEP]);
    const int limit = SS ? s.ctr[C_LIMIT] : gload(&s.ctr[C_LIMIT]);
    const TileGeom<V, TX> tg(s, tile);
    StageRegs<SS> r;
    stage_issue<V, TX, SS>(s, tg, r);
    if (step >= limit) return;                                // scenario finished: nothing to do
    if (tile == 0 && threadIdx.x < 4) s.ctr[C_BAR + threadIdx.x] = 0;   // fresh motion barriers
    stage_commit<V, TX, SS>(s, tg, sh, r);
    plan_agents<V, TX, DEBUG, SS>(s, tg, tile, sh, step, r.fb != 0);
}

template <int V, bool DEBUG, bool SS>
__device__ __forceinline__ void plan_dispatch_tx(const SlotDev &s, int tile, PlanShared<SS> &sh)
{
    switch (s.tx) {
        case 8: plan_tile<V, 8, DEBUG, SS>(s, tile, sh); break;
        case 16: plan_tile<V, 16, DEBUG, SS>(s, tile, sh); break;
        case 32: plan_tile<V, 32, DEBUG, SS>(s, tile, sh); break;
        case 64: plan_tile<V, 64, DEBUG, SS>(s, tile, sh); break;
        default: break;
    }
}

// Device-side dispatch over (v_max, tile width): one launch can mix scenarios.
template <bool DEBUG, bool SS>
__device__ __forceinline__ void plan_dispatch(const SlotDev &s, int tile, PlanShared<SS> &sh)
{
    switch (s.v) {
        case 1: plan_dispatch_tx<1, DEBUG, SS>(s, tile, sh); break;
        case 2: plan_dispatch_tx<2, DEBUG, SS>(s, tile, sh); break;
        case 3: plan_dispatch_tx<3, DEBUG, SS>(s, tile, sh); break;
        case 4: plan_dispatch_tx<4, DEBUG, SS>(s, tile, sh); break;
        case 5: plan_dispatch_tx<5, DEBUG, SS>(s, tile, sh); break;
        default: break;
    }
}

}  // namespace fk
