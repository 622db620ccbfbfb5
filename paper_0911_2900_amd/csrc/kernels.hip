// kernels.hip -- gfx950 kernels of the F.A.S.T. time step.
//
//   plan_kernel   the planning phase, choose_desired_cell for every agent
//                 (paper Sec. 1 and Sec. 2): one workgroup per grid tile; the
//                 tile's (tx+2v) x (ty+2v) window of the exp table, masked by
//                 the occupancy snapshot, is staged in LDS; agents are found
//                 by scanning the tile's occupancy; one lane per agent forms
//                 the weights, the CDF over the reach disc, and the Philox
//                 draw in FP32; draws inside the guard band are re-resolved
//                 in FP64 by a whole wavefront.  The tile's movers are written
//                 as (id, start, target) records to the tile's own segment.
//   move_kernel   the motion phase with the model's sequential semantics
//                 (Sec. 1), run as deterministic reservations: one workgroup
//                 per scenario; every round each pending agent reserves its
//                 path cells with atomicMax of its priority word, and the
//                 agents holding all their cells move.  Agents that commit in
//                 one round have disjoint paths and commute, and an agent
//                 only moves once every earlier agent sharing a cell with it
//                 has moved, so the result equals moving them one by one in
//                 priority order.
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

// Row R (dy = R - V) of the reach disc: its 2a+1 masked exp values, read
// from Eb = the agent's window origin (row -V, column -V) with pitch P; the
// agent's own cell takes e_c.
template <int V, int P, int R>
__device__ __forceinline__ void load_row(const float *Eb, float ec, float (&x)[2 * V + 1])
{
    constexpr int a = half_width(V, R - V);
#pragma unroll
    for (int k = 0; k <= 2 * a; ++k) {
        if (R == V && k == a) x[k] = ec;
        else x[k] = Eb[R * P + (V - a) + k];
    }
}

// Row sums, software-pipelined by one row: the loads of row R+1 are issued
// before row R is summed, and the scheduling barrier keeps later rows from
// being hoisted, so at most two rows of values are live.
template <int V, int P, int R>
struct RowPipe {
    static __device__ __forceinline__ void run(const float *Eb, float ec, float *Rs,
                                               const float (&cur)[2 * V + 1])
    {
        constexpr int a = half_width(V, R - V);
        float nxt[2 * V + 1];
        if constexpr (R + 1 < 2 * V + 1) load_row<V, P, R + 1>(Eb, ec, nxt);
        Rs[R] = Tree<2 * a + 1, 0>::sum(cur);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (R + 1 < 2 * V + 1) RowPipe<V, P, R + 1>::run(Eb, ec, Rs, nxt);
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
    if (s.type[t] == CELL_WALL) return false;
    const int o = s.occ[t];
    return o < 0 || t == gc;
}

// (The loops stay rolled: this path is rare, and unrolled FP64 exp code would
// raise the register count of the whole planning kernel.)
template <int V, bool DEBUG>
__device__ int resolve64_lane(const SlotDev &s, int gc, int id, float u32)
{
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    double C = 0.0;
#pragma unroll 1
    for (int dy = -V; dy <= V; ++dy)
#pragma unroll 1
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok<V>(s, gc, t, dx, dy)) {
                const double w = exp(ks * (Sc - s.S[t]));
                C = C + w;
                if (DEBUG && s.dbg_w)
                    s.dbg_w[(size_t)id * (2 * V + 1) * (2 * V + 1) + (dy + V) * (2 * V + 1) + dx + V] =
                        (float)w;
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

// The same draw by a whole wavefront: lane j evaluates raster slots j and
// j + 64 of the square window; the prefix sum is still taken sequentially,
// slot by slot, in raster order, so the result is bit-identical to
// resolve64_lane (slots outside the reach set add nothing).
// Reachability is read from the tile's staged window (Em, agent cell l, pitch
// P): on a fast tile a cell is zero there exactly when it is a wall, padding
// or occupied, so only the floor field needs global reads.  For v <= 4 the
// reach disc has at most 49 slots: lane j takes the j-th disc slot in raster
// order and the sequential sum runs over the disc only (the slots it skips add
// nothing in the raster-order sum); v = 5 uses the square window.
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

template <int V>
__device__ int resolve64_wave(const SlotDev &s, int gc, float u32, int lane, const float *Em,
                              int l, int P)
{
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    if constexpr (disc_count(V) <= 64) {
        constexpr int ND = disc_count(V);
        double w = 0.0;
        int dx = 0, dy = 0;
        disc_slot<V>(lane, dx, dy);
        if (lane < ND && ((dx == 0 && dy == 0) || Em[l + dy * P + dx] != 0.0f))
            w = exp(ks * (Sc - s.S[gc + dy * s.Wp + dx]));
        double C = 0.0, myC = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const int lo = __builtin_amdgcn_readlane(__double2loint(w), j);
            const int hi = __builtin_amdgcn_readlane(__double2hiint(w), j);
            C = C + __hiloint2double(hi, lo);
            if (lane == j) myC = C;
        }
        const double tau = (double)u32 * C;
        const unsigned long long m = __ballot(lane < ND && tau < myC);
        const int jw = m ? __builtin_ctzll(m) : V * 0 + (ND - 1) / 2;   // own cell if unreached
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
                    w[h] = exp(ks * (Sc - s.S[gc + dy * s.Wp + dx]));
            }
        }
        double C = 0.0, myC0 = 0.0, myC1 = 0.0;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const double wj = w[j / 64];
            const int lo = __builtin_amdgcn_readlane(__double2loint(wj), j % 64);
            const int hi = __builtin_amdgcn_readlane(__double2hiint(wj), j % 64);
            C = C + __hiloint2double(hi, lo);
            if (j < 64) { if (lane == j) myC0 = C; }
            else { if (lane == j - 64) myC1 = C; }
        }
        const double tau = (double)u32 * C;
        const unsigned long long m0 = __ballot(lane < NS && tau < myC0);
        const unsigned long long m1 = __ballot(lane + 64 < NS && tau < myC1);
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
struct PlanShared {
    alignas(16) float Em[MAX_STAGE];    // masked exp table window, pitch P = round4(tx + 2v)
    int32_t a_pk[MAX_TILE_CELLS];       // agents of the tile: id << 12 | LDS cell
    float a_ec[MAX_TILE_CELLS];         // e_c of their own cell
    int32_t m_nb[9];
    int n_agents, n_flag, n_mov;
};

// Appends movers (target != own cell) to the tile's record segment, one LDS
// atomic per wavefront.
__device__ __forceinline__ void emit_movers(MoveRec *seg, PlanShared &sh, bool mover, MoveRec rec)
{
    const unsigned long long mask = __ballot(mover);
    if (mask == 0) return;
    const int lane = __lane_id();
    const int leader = __builtin_ctzll(mask);
    int base = 0;
    if (lane == leader) base = atomicAdd(&sh.n_mov, __popcll(mask));
    base = __shfl(base, leader);
    if (mover) seg[base + __popcll(mask & ((1ull << lane) - 1ull))] = rec;
}

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
    asm volatile("" : "+s"(k0), "+s"(k1));
    return philox_word0(id, step, scn, STREAM_PLAN, k0, k1);
}

// V = v_max, TX = tile width (a power of two, 8..64): both fix the LDS pitch,
// so every window offset of the agent loop is a compile-time constant.
template <int V, int TX, bool DEBUG>
__device__ void plan_tile(const SlotDev &s, int tile, PlanShared &sh)
{
    constexpr int SIDE = 2 * V + 1;
    constexpr int Hc = (V + 3) & ~3;                          // column halo, a multiple of 4 >= V
    constexpr int P = TX + 2 * Hc;                            // LDS pitch = staged width
    constexpr int cpr = P >> 2;                               // 4-cell chunks per row
    constexpr int hc4 = Hc >> 2;
    constexpr int cw = TX >> 2;                               // interior chunks per row
    constexpr int cw_log = __builtin_ctz(cw);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = __lane_id();
    const int LY = s.ty + 2 * V;
    const int n_in = cw * s.ty;                               // interior chunks (<= nthr)
    const int n_top = V * cpr;                                // halo chunks: V rows above / below,
    const int n_halo = 2 * n_top + s.ty * 2 * hc4;            // then hc4 chunks left and right
    const int tile_y = tile / s.ntx, tile_x = tile - tile_y * s.ntx;
    const int gx0 = tile_x * TX, gy0 = tile_y * s.ty + Hc - V;     // padded origin of the window
    const int tstride = s.ntx + 2;
    const bool fallback = s.tile_fb[tile_y * s.ntx + tile_x] != 0;

    if (tid < 9) sh.m_nb[tid] = s.tile_m[(tile_y + tid / 3) * tstride + tile_x + tid % 3];
    if (tid == 0) { sh.n_agents = 0; sh.n_flag = 0; sh.n_mov = 0; }
    MoveRec *seg = s.seg + (long)tile * (TX * s.ty);

    // --- stage the window: one interior chunk and up to two halo chunks per
    // thread, 16-byte loads of occupancy and exp table, all issued first
    const int ci = tid;
    const int ly_in = V + (ci >> cw_log), cc_in = hc4 + (ci & (cw - 1));
    int ly_h[2], cc_h[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int h = tid + j * nthr;
        int ly, cc;
        if (h < 2 * n_top) {                                  // rows above, then rows below
            const int hh = h < n_top ? h : h - n_top;
            ly = (int)((unsigned)hh / cpr);
            cc = hh - ly * cpr;
            if (h >= n_top) ly += V + s.ty;
        } else {                                              // left / right columns
            const int hh = h - 2 * n_top;
            const int r = (int)((unsigned)hh / (2 * hc4));
            const int c = hh - r * 2 * hc4;
            ly = V + r;
            cc = c < hc4 ? c : c + cw;
        }
        ly_h[j] = ly;
        cc_h[j] = cc;
    }
    int4 o_in = make_int4(-1, -1, -1, -1), o_h0 = o_in, o_h1 = o_in;
    float4 g_in = make_float4(0.f, 0.f, 0.f, 0.f), g_h0 = g_in, g_h1 = g_in;
    if (ci < n_in) {
        const int g = (gy0 + ly_in) * s.Wp + gx0 + 4 * cc_in;
        o_in = *(const int4 *)(s.occ + g);
        g_in = *(const float4 *)(s.G + g);
    }
    if (tid < n_halo) {
        const int g = (gy0 + ly_h[0]) * s.Wp + gx0 + 4 * cc_h[0];
        o_h0 = *(const int4 *)(s.occ + g);
        g_h0 = *(const float4 *)(s.G + g);
    }
    if (tid + nthr < n_halo) {
        const int g = (gy0 + ly_h[1]) * s.Wp + gx0 + 4 * cc_h[1];
        o_h1 = *(const int4 *)(s.occ + g);
        g_h1 = *(const float4 *)(s.G + g);
    }
    // the step counter is read while the staging loads are in flight
    const int step = s.ctr[C_STEP];
    if (step >= s.ctr[C_LIMIT]) return;                       // scenario finished: nothing to do
    if (tile == 0 && tid < 4) s.ctr[C_BAR + tid] = 0;          // fresh motion barriers
    __syncthreads();                                          // m_nb, counters ready
    const int mT = sh.m_nb[4];

    // halo chunks: rescale to this tile's exponent, mask occupied cells
    auto stage_halo = [&](int ly, int cc, int4 o, float4 gv) {
        const int nby = (ly >= V) + (ly >= V + s.ty);
        const int nbx = (cc >= hc4) + (cc >= hc4 + cw);       // a chunk lies inside one tile column
        const int dm = mT - sh.m_nb[nby * 3 + nbx];
        *(float4 *)&sh.Em[ly * P + 4 * cc] =
            make_float4(o.x < 0 ? ldexpf(gv.x, dm) : 0.f, o.y < 0 ? ldexpf(gv.y, dm) : 0.f,
                        o.z < 0 ? ldexpf(gv.z, dm) : 0.f, o.w < 0 ? ldexpf(gv.w, dm) : 0.f);
    };
    if (tid < n_halo) stage_halo(ly_h[0], cc_h[0], o_h0, g_h0);
    if (tid + nthr < n_halo) stage_halo(ly_h[1], cc_h[1], o_h1, g_h1);

    // interior chunk: already in the tile's scale; its occupied cells are the
    // tile's agents (one LDS atomic per wavefront to list them)
    {
        const bool live = ci < n_in;
        const int l0 = ly_in * P + 4 * cc_in;
        if (live)
            *(float4 *)&sh.Em[l0] = make_float4(o_in.x < 0 ? g_in.x : 0.f, o_in.y < 0 ? g_in.y : 0.f,
                                                o_in.z < 0 ? g_in.z : 0.f, o_in.w < 0 ? g_in.w : 0.f);
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
                    sh.a_pk[idx] = (ov[k] << 12) | (l0 + k);
                    sh.a_ec[idx] = gv[k];
                    ++idx;
                }
            }
        }
    }
    __syncthreads();
    const int na = sh.n_agents;
    const uint32_t kseed0 = s.seed_lo, kseed1 = s.seed_hi;
    const uint32_t scn = s.scn;          // held in registers: the loops below store to memory
    const float eps = s.eps;

    if (fallback) {
        // every draw of this tile in FP64, one lane per agent
        for (int base = 0; base < na; base += nthr) {
            const int k = base + tid;
            bool mover = false;
            MoveRec rec{};
            if (k < na) {
                const int id = sh.a_pk[k] >> 12;
                const int l = sh.a_pk[k] & 0xFFF;
                const int ly = (int)((unsigned)l / P);
                const int cx = gx0 + (l - ly * P), cy = gy0 + ly;
                const int gc = cy * s.Wp + cx;
                const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int t = resolve64_lane<V, DEBUG>(s, gc, id, u);
                mover = t != gc;
                const int d = t - gc;                       // |dx|, |dy| <= V < Wp / 2
                const int ddy = (d + V * s.Wp + V) / s.Wp - V, ddx = d - ddy * s.Wp;
                rec = MoveRec{(uint32_t)id, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy)};
                if (DEBUG && s.dbg_flag) s.dbg_flag[id] = 2;
                if (DEBUG && s.dbg_margin) s.dbg_margin[id] = -1.0f;
            }
            emit_movers(seg, sh, mover, rec);
        }
        __syncthreads();
        if (tid == 0) {
            s.seg_cnt[tile] = sh.n_mov;
            if (na > 0) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)na);
        }
        return;
    }

    // --- one lane per agent, FP32 from the LDS table
    for (int base = 0; base < na; base += nthr) {
        const int k = base + tid;
        bool mover = false, flagged = false;
        MoveRec rec{};
        if (k < na) {
            const int id = sh.a_pk[k] >> 12;
            const int l = sh.a_pk[k] & 0xFFF;
            const float ec = sh.a_ec[k];
            const int ly = (int)((unsigned)l / P);
            const int cx = gx0 + (l - ly * P), cy = gy0 + ly;

            const float *Eb = sh.Em + (l - V * P - V);      // window origin (dy, dx) = (-V, -V)
            float Rs[SIDE], row0[SIDE];
            load_row<V, P, 0>(Eb, ec, row0);
            __builtin_amdgcn_sched_barrier(0);
            // the draw's counter-based word overlaps the first row's LDS reads
            const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, scn, kseed0, kseed1);
            __builtin_amdgcn_sched_barrier(0);
            RowPipe<V, P, 0>::run(Eb, ec, Rs, row0);
            float Pr[SIDE + 1];
            Pr[0] = 0.0f;
            Pr[1] = Rs[0];
#pragma unroll
            for (int r = 1; r < SIDE; ++r) Pr[r + 1] = Pr[r] + Rs[r];
            const float Wsum = Pr[SIDE];

            const float u = (float)(x0 >> 8) * 0x1p-24f;
            const float tau = u * Wsum;

            // row: the last r with Pr_r <= tau
            int rs = 0, as = half_width(V, -V);
            float Ps = 0.0f;
#pragma unroll
            for (int r = 1; r < SIDE; ++r) {
                const bool le = Pr[r] <= tau;
                rs = le ? r : rs;
                Ps = le ? Pr[r] : Ps;
                as = le ? half_width(V, r - V) : as;
            }
            // slot within the row: count of in-row boundaries <= tau.  The
            // row's cells are read at once (slots past 2a stay inside the
            // LDS block and are not used).
            const float *rb = Eb + rs * P + (V - as);
            float rv[SIDE];
#pragma unroll
            for (int d = 0; d < SIDE; ++d) rv[d] = rb[d];
            float Q = 0.0f;
            float margin = fabsf(tau - Ps);
            int ks = 0;
#pragma unroll
            for (int d = 0; d < SIDE; ++d) {
                if (d <= 2 * as) {
                    const float val = (rs == V && d == as) ? ec : rv[d];
                    Q = Q + val;
                    const float C = Ps + Q;
                    const float diff = tau - C;
                    ks += diff >= 0.0f ? 1 : 0;
                    margin = fminf(margin, fabsf(diff));
                }
            }
            const bool flag = (margin <= eps * Wsum) || (ks > 2 * as);

            if (DEBUG) {
                if (s.dbg_w) {
                    float *wd = s.dbg_w + (size_t)id * SIDE * SIDE;
                    for (int dy = -V; dy <= V; ++dy)
                        for (int dx = -V; dx <= V; ++dx) {
                            float wv = 0.0f;
                            if (dx * dx + dy * dy <= V * V)
                                wv = (dx == 0 && dy == 0) ? 1.0f : sh.Em[l + dy * P + dx] / ec;
                            wd[(dy + V) * SIDE + dx + V] = wv;
                        }
                }
                if (s.dbg_flag) s.dbg_flag[id] = flag ? 1 : 0;
                if (s.dbg_margin) s.dbg_margin[id] = margin / Wsum;
            }
            if (!flag) {
                const int ddx = ks - as, ddy = rs - V;
                mover = ddx != 0 || ddy != 0;
                rec = MoveRec{(uint32_t)id, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy)};
            }
            flagged = flag;
        }
        emit_movers(seg, sh, mover, rec);

        // FP64 re-resolve of this wavefront's flagged draws, one draw at a
        // time by the whole wavefront, without waiting for the other waves
        unsigned long long fm = __ballot(flagged);
        if (fm) {
            if (lane == 0) atomicAdd(&sh.n_flag, __popcll(fm));
            while (fm) {
                const int src = __builtin_ctzll(fm);
                fm &= fm - 1ull;
                const int kk = base + (tid & ~63) + src;
                const int fid = sh.a_pk[kk] >> 12;
                const int l = sh.a_pk[kk] & 0xFFF;
                const int ly = (int)((unsigned)l / P);
                const int cx = gx0 + (l - ly * P), cy = gy0 + ly;
                const int gc = cy * s.Wp + cx;
                const uint32_t x0 = plan_draw_word((uint32_t)fid, (uint32_t)step, scn, kseed0,
                                                   kseed1);
                const float u = (float)(x0 >> 8) * 0x1p-24f;
                const int t = resolve64_wave<V>(s, gc, u, lane, sh.Em, l, P);
                if (lane == 0 && t != gc) {
                    const int d = t - gc;
                    const int ddy = (d + V * s.Wp + V) / s.Wp - V, ddx = d - ddy * s.Wp;
                    seg[atomicAdd(&sh.n_mov, 1)] =
                        MoveRec{(uint32_t)fid, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy)};
                }
            }
        }
    }
    __syncthreads();
    const int nf = sh.n_flag;
    if (tid == 0) {
        s.seg_cnt[tile] = sh.n_mov;
        if (nf) atomicAdd(&s.stat[S_FLAGGED], (unsigned long long)nf);
    }
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

// Batched form: items[i] = (slot << 20) | tile index (row-major over the
// slot's tiles); descriptors come from the device table.
template <bool DEBUG>
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(7)))
void plan_kernel(const SlotDev *__restrict__ table,
                                                            const uint32_t *__restrict__ items)
{
    __shared__ PlanShared sh;
    const uint32_t it = items[blockIdx.x];
    plan_dispatch<DEBUG>(table[it >> 20], (int)(it & 0xFFFFFu), sh);
}

// One scenario: its descriptor arrives by value with the kernel arguments and
// workgroup i plans tile i, which saves two dependent memory round trips.
template <bool DEBUG>
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(8)))
void plan_kernel_one(const SlotDev s)
{
    __shared__ PlanShared sh;
    plan_dispatch<DEBUG>(s, (int)blockIdx.x, sh);
}

// ---------------------------------------------------------------------------
// Motion kernel: deterministic reservations.  The movers of a scenario are
// split over a group of G workgroups; each keeps its share in a private list.
// Round r reserves into res[r & 1] with tag r (tags grow, so stale words of
// earlier rounds always lose), so the checks of round r and the reservations
// of round r + 1 never touch the same array and one group barrier per round
// suffices:
//     reserve r+1 (own losers) | count | barrier | check r+1, commit, ...
// ---------------------------------------------------------------------------
__device__ __forceinline__ int isgn(int a) { return (a > 0) - (a < 0); }

__device__ __forceinline__ int ld_agent(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_res(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cells of the DDA line from (cx, cy) towards (cx + dx, cy + dy):
// p_k = (cx + sgn dx floor((2k|dx| + m) / 2m), cy + sgn dy floor((2k|dy| + m) / 2m)),
// k = 0..m, m = max(|dx|, |dy|) <= v.
struct Line {
    int cx, cy, sx, sy, adx, ady, m;
    __device__ __forceinline__ void at(int k, int &x, int &y) const
    {
        x = cx + sx * ((2 * k * adx + m) / (2 * m));
        y = cy + sy * ((2 * k * ady + m) / (2 * m));
    }
};

__device__ __forceinline__ Line make_line(uint32_t cxy, uint32_t dxy)
{
    Line L;
    L.cx = (int)(cxy & 0xFFFFu);
    L.cy = (int)(cxy >> 16);
    const int dx = (int)(dxy & 0xFFFFu) - L.cx, dy = (int)(dxy >> 16) - L.cy;
    L.sx = isgn(dx);
    L.sy = isgn(dy);
    L.adx = abs(dx);
    L.ady = abs(dy);
    L.m = max(L.adx, L.ady);
    return L;
}

// Barrier of the G workgroups of one scenario that also sums their mover
// counts.  Round r uses the 64-bit word bar[r & 1] = [arrivals:32][count:32]
// (both zeroed by the planning kernel): each workgroup adds (1 << 32) | n and
// waits until the arrivals reach (r / 2 + 1) * G.  A word is touched again only
// two barriers later, after every workgroup has read it, so the count part
// minus its value at the previous barrier of the same parity is this round's
// total.  All data shared between the workgroups moves through agent-scope
// atomics; the fences of thread 0 order them around the arrival.  A wait
// longer than SPIN_LIMIT polls marks the scenario as failed (C_ERR) instead of
// hanging; the function then returns -1.
__device__ int group_sync_count(const SlotDev &s, int G, int r, int n, unsigned long long &seen0,
                                unsigned long long &seen1)
{
    __shared__ int sh_total;
    __syncthreads();
    if (G == 1) return n;
    if (threadIdx.x == 0) {
        unsigned long long *bar = (unsigned long long *)&s.ctr[C_BAR] + (r & 1);
        unsigned long long &seen = (r & 1) ? seen1 : seen0;
        __threadfence();
        atomicAdd(bar, (1ull << 32) | (unsigned long long)(uint32_t)n);
        const unsigned long long target = (unsigned long long)(r / 2 + 1) * (unsigned long long)G;
        uint32_t spins = 0;
        unsigned long long w;
        int total = -1;
        for (;;) {
            w = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((w >> 32) >= target) { total = (int)((uint32_t)w - (uint32_t)seen); seen = w; break; }
            if (++spins > SPIN_LIMIT) { atomicOr(&s.ctr[C_ERR], 1); break; }
        }
        __threadfence();
        sh_total = total;
    }
    __syncthreads();
    return sh_total;
}

template <int V>
__device__ __forceinline__ void reserve_list(const SlotDev &s, unsigned long long *res,
                                             const Mover *list, int n, unsigned long long tagw)
{
    const int Wp = s.Wp;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const Mover mv = list[i];
        const Line L = make_line(mv.cxy, mv.dxy);
        const unsigned long long key = mv.key | tagw;
#pragma unroll
        for (int k = 0; k <= V; ++k) {
            if (k <= L.m) {
                int x, y;
                L.at(k, x, y);
                atomicMax(&res[y * Wp + x], key);
            }
        }
    }
}

// Check-and-commit for the workgroup's list: a mover holding every cell of
// its line walks it (stopping before a wall, an occupied cell, or a diagonal
// step past a wall corner; leaving at an exit); the others are appended to
// `nxt`.  Returns the number appended.
template <int V>
__device__ int commit_list(const SlotDev &s, const unsigned long long *res, const Mover *cur,
                           Mover *nxt, int n, unsigned long long tagw)
{
    __shared__ int sh_cnt;
    const int Wp = s.Wp;
    if (threadIdx.x == 0) sh_cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const Mover mv = cur[i];
        const Line L = make_line(mv.cxy, mv.dxy);
        const unsigned long long key = mv.key | tagw;
        int cell[V + 1];
        unsigned long long w[V + 1];
        int o[V + 1];
#pragma unroll
        for (int k = 0; k <= V; ++k) {
            int x = L.cx, y = L.cy;
            if (k <= L.m) L.at(k, x, y);
            cell[k] = y * Wp + x;
            w[k] = k <= L.m ? ld_res(&res[cell[k]]) : key;
            o[k] = (k >= 1 && k <= L.m) ? ld_agent(&s.occ[cell[k]]) : -1;
        }
        bool holds = true;
#pragma unroll
        for (int k = 0; k <= V; ++k) holds &= (w[k] == key);
        if (!holds) {
            nxt[atomicAdd(&sh_cnt, 1)] = mv;
            continue;
        }
        const int id = (int)(~(uint32_t)mv.key & ID_MASK);
        const int c = cell[0];
        int at = c, px = L.cx, py = L.cy;
        bool gone = false, stop = false;
#pragma unroll
        for (int k = 1; k <= V; ++k) {
            if (k > L.m || stop) break;
            int qx, qy;
            L.at(k, qx, qy);
            const int q = cell[k];
            const uint8_t tq = s.type[q];
            if (tq == CELL_WALL || o[k] != -1) { stop = true; break; }
            if (qx != px && qy != py &&
                (s.type[py * Wp + qx] == CELL_WALL || s.type[qy * Wp + px] == CELL_WALL)) {
                stop = true;
                break;
            }
            if (tq == CELL_EXIT) { gone = true; break; }
            at = q; px = qx; py = qy;
        }
        if (gone) {
            st_agent(&s.occ[c], -1);
            atomicAdd(&s.ctr[C_EXITED], 1);
            atomicSub(&s.ctr[C_NACTIVE], 1);
        } else if (at != c) {
            st_agent(&s.occ[c], -1);
            st_agent(&s.occ[at], id);
        }
    }
    __syncthreads();
    return sh_cnt;
}

template <int V>
__device__ void move_group(const SlotDev &s, int g, int G, int step)
{
    __shared__ int sh_scan[MOVE_THREADS];
    const int tid = threadIdx.x;
    const int T = s.ntx * s.nty, TC = s.tx * s.ty;
    // workgroup g takes tiles g, g + G, g + 2G, ...: every region of the grid
    // (the congested exit above all) is spread over the whole group, so the
    // rounds stay balanced; its mover lists own tiles' worth of room
    const int q = T / G, rm = T % G;
    const int nt_g = q + (g < rm ? 1 : 0);
    const long base_g = ((long)g * q + min(g, rm)) * TC;
    Mover *cur = s.mv_a + base_g, *nxt = s.mv_b + base_g;
    unsigned long long seen0 = 0, seen1 = 0;
    uint32_t tag = (uint32_t)s.ctr[C_TAG];
    if (g == 0 && tid == 0)   // agents planned this step, for the throughput counters
        atomicAdd(&s.stat[S_PLANNED], (unsigned long long)s.ctr[C_NACTIVE]);

    // gather this workgroup's movers (the records of its tiles) with their
    // priority words [~x0:32][~id:20] (larger = earlier)
    int n = 0;
    for (int j0 = 0; j0 < nt_g; j0 += MOVE_THREADS) {
        const int nt = min(MOVE_THREADS, nt_g - j0);
        sh_scan[tid] = tid < nt ? s.seg_cnt[g + (long)(j0 + tid) * G] : 0;
        __syncthreads();
        for (int off = 1; off < MOVE_THREADS; off <<= 1) {
            const int add = tid >= off ? sh_scan[tid - off] : 0;
            __syncthreads();
            sh_scan[tid] += add;
            __syncthreads();
        }
        const int chunk = sh_scan[MOVE_THREADS - 1];
        for (int i = tid; i < chunk; i += blockDim.x) {
            int a = 0, b = nt - 1;                   // first tile whose inclusive count exceeds i
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (sh_scan[mid] > i) b = mid; else a = mid + 1;
            }
            const int k = i - (a ? sh_scan[a - 1] : 0);
            const MoveRec rec = s.seg[(g + (long)(j0 + a) * G) * TC + k];
            const uint32_t x0 = philox_word0(rec.id, (uint32_t)step, s.scn, STREAM_ORDER,
                                             s.seed_lo, s.seed_hi);
            Mover mv;
            mv.key = ((unsigned long long)(~x0) << ID_BITS) | (unsigned long long)(~rec.id & ID_MASK);
            mv.cxy = rec.cxy;
            mv.dxy = rec.dxy;
            cur[n + i] = mv;
        }
        n += chunk;
        __syncthreads();
    }

    int total = 1, rounds = 0, bar_r = 0;          // round 0's total comes from its barrier
    for (int r = 0; total > 0; ++r) {
        unsigned long long *res = (r & 1) ? s.res1 : s.res0;
        if (r > 0) {
            // round r's movers are the losers of round r - 1 (this workgroup's share)
            n = commit_list<V>(s, (r & 1) ? s.res0 : s.res1, cur, nxt, n,
                               (unsigned long long)tag << TAG_SHIFT);
            Mover *t = cur; cur = nxt; nxt = t;
        }
        if (tag >= TAG_LIMIT) {
            // tags are exhausted: once every check of the last round is done,
            // wipe both reservation arrays and restart the tags at 1
            if (group_sync_count(s, G, bar_r++, 0, seen0, seen1) < 0) return;
            const long cells = (long)s.Wp * s.Hp;
            for (long i = cells * g / G + tid; i < cells * (g + 1) / G; i += blockDim.x) {
                __hip_atomic_store(&s.res0[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&s.res1[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            tag = 0;
            if (group_sync_count(s, G, bar_r++, 0, seen0, seen1) < 0) return;
        }
        ++tag;
        reserve_list<V>(s, res, cur, n, (unsigned long long)tag << TAG_SHIFT);
        total = group_sync_count(s, G, bar_r++, n, seen0, seen1);
        if (total < 0) return;
        rounds += total > 0 ? 1 : 0;
    }
    if (g == 0 && tid == 0) {
        s.ctr[C_TAG] = (int)tag;
        s.ctr[C_ROUNDS] = rounds;
        s.ctr[C_STEP] = step + 1;
    }
}

// mitems[i] = slot | g << 12 | (G - 1) << 22: workgroup g of the G that move
// the slot's agents.
__global__ __launch_bounds__(MOVE_THREADS) void move_kernel(const SlotDev *__restrict__ table,
                                                            const uint32_t *__restrict__ mitems)
{
    const uint32_t it = mitems[blockIdx.x];
    const SlotDev &s = table[it & 0xFFFu];
    const int g = (int)((it >> 12) & 0x3FFu);
    const int G = (int)(it >> 22) + 1;
    const int step = s.ctr[C_STEP];
    if (step >= s.ctr[C_LIMIT]) return;
    switch (s.v) {
        case 1: move_group<1>(s, g, G, step); break;
        case 2: move_group<2>(s, g, G, step); break;
        case 3: move_group<3>(s, g, G, step); break;
        case 4: move_group<4>(s, g, G, step); break;
        case 5: move_group<5>(s, g, G, step); break;
        default: break;
    }
}

}  // namespace fk

// ---------------------------------------------------------------------------
// Launchers used by the host runtime.
// ---------------------------------------------------------------------------
extern "C" hipError_t fk_launch_plan_one(const fk::SlotDev *slot, int n_tiles, int debug,
                                         hipStream_t stream)
{
    if (n_tiles <= 0) return hipSuccess;
    if (debug)
        hipLaunchKernelGGL(fk::plan_kernel_one<true>, dim3(n_tiles), dim3(fk::PLAN_THREADS), 0, stream,
                           *slot);
    else
        hipLaunchKernelGGL(fk::plan_kernel_one<false>, dim3(n_tiles), dim3(fk::PLAN_THREADS), 0,
                           stream, *slot);
    return hipGetLastError();
}

extern "C" hipError_t fk_launch_plan(const fk::SlotDev *table, const uint32_t *items, int n_items,
                                     int debug, hipStream_t stream)
{
    if (n_items <= 0) return hipSuccess;
    if (debug)
        hipLaunchKernelGGL(fk::plan_kernel<true>, dim3(n_items), dim3(fk::PLAN_THREADS), 0, stream,
                           table, items);
    else
        hipLaunchKernelGGL(fk::plan_kernel<false>, dim3(n_items), dim3(fk::PLAN_THREADS), 0, stream,
                           table, items);
    return hipGetLastError();
}

extern "C" hipError_t fk_launch_move(const fk::SlotDev *table, const uint32_t *mitems, int n_items,
                                     hipStream_t stream)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk::move_kernel, dim3(n_items), dim3(fk::MOVE_THREADS), 0, stream, table,
                       mitems);
    return hipGetLastError();
}

// Workgroups of move_kernel that one device holds at once.
extern "C" hipError_t fk_move_capacity(int *blocks)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fk::move_kernel,
                                                                fk::MOVE_THREADS, 0);
    if (e != hipSuccess) return e;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

