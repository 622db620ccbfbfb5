// kernels.hip -- gfx950 kernels of the F.A.S.T. time step.
//
//   plan_kernel   the planning phase, choose_desired_cell for every agent
//                 (paper Sec. 1 and Sec. 2): one workgroup per grid tile; the
//                 tile's (tx+2v) x (ty+2v) window of the exp table, masked by
//                 the occupancy snapshot, is staged in LDS; agents are found
//                 by scanning the tile's occupancy; one lane per agent forms
//                 the weights, the CDF over the reach disc, and the Philox
//                 draw in FP32; draws inside the guard band are re-resolved
//                 in FP64 by a whole wavefront.
//   move_kernel   the motion phase with the model's sequential semantics
//                 (Sec. 1), run as deterministic reservations: one workgroup
//                 per scenario; every round each pending agent reserves its
//                 path cells with atomicMax of its priority word, and the
//                 agents holding all their cells move.  Agents that commit in
//                 one round have disjoint paths and commute, and an agent
//                 only moves once every earlier agent sharing a cell with it
//                 has moved, so the result equals moving them one by one in
//                 priority order.
//   reset_kernel  clears the per-step mover count (used when a plan is
//                 issued again without a motion phase in between).
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

// Row r (dy = r - V) of the disc around the agent's LDS cell l: sum of the
// masked exp values, the agent's own cell taking e_c.
template <int V, int R>
__device__ __forceinline__ float row_sum(const float *Em, int l, int LX, float ec)
{
    constexpr int dy = R - V;
    constexpr int a = half_width(V, dy);
    float x[2 * a + 1];
#pragma unroll
    for (int k = 0; k <= 2 * a; ++k) {
        if (dy == 0 && k == a) x[k] = ec;
        else x[k] = Em[l + dy * LX + (k - a)];
    }
    return Tree<2 * a + 1, 0>::sum(x);
}

template <int V, int... R>
__device__ __forceinline__ void all_rows(std::integer_sequence<int, R...>, float *Rs,
                                         const float *Em, int l, int LX, float ec)
{
    ((Rs[R] = row_sum<V, R>(Em, l, LX, ec)), ...);
}

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

template <int V, bool DEBUG>
__device__ int resolve64_lane(const SlotDev &s, int gc, int id, float u32)
{
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    double C = 0.0;
    for (int dy = -V; dy <= V; ++dy)
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
    for (int dy = -V; dy <= V; ++dy)
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
// j + 64; the prefix sum is still taken sequentially, slot by slot, in raster
// order, so the result is bit-identical to resolve64_lane.
template <int V>
__device__ int resolve64_wave(const SlotDev &s, int gc, float u32, int lane)
{
    constexpr int SIDE = 2 * V + 1;
    constexpr int NS = SIDE * SIDE;           // <= 121
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    double w[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = lane + 64 * h;
        if (j < NS) {
            const int dy = j / SIDE - V, dx = j % SIDE - V;
            const int t = gc + dy * s.Wp + dx;
            if (reach_ok<V>(s, gc, t, dx, dy)) w[h] = exp(ks * (Sc - s.S[t]));
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
    else j = V * SIDE + V;                       // not reached
    return gc + (j / SIDE - V) * s.Wp + (j % SIDE - V);
}

// ---------------------------------------------------------------------------
// Planning kernel.
// ---------------------------------------------------------------------------
struct PlanShared {
    float Em[MAX_STAGE];                // masked exp table window
    int32_t a_id[MAX_TILE_CELLS];       // agents found on the tile
    int32_t a_g[MAX_TILE_CELLS];        // their padded cell
    int16_t a_l[MAX_TILE_CELLS];        // their LDS cell
    float a_ec[MAX_TILE_CELLS];         // e_c of their own cell
    int16_t f_k[MAX_TILE_CELLS];        // flagged agents (index into a_*)
    float f_u[MAX_TILE_CELLS];
    int32_t m_nb[9];
    int n_agents, n_flag;
};

// Appends movers (target != own cell) to the slot's pending list with one
// atomic per wavefront.
__device__ __forceinline__ void append_movers(const SlotDev &s, bool mover, int id)
{
    const unsigned long long mask = __ballot(mover);
    if (mask == 0) return;
    const int lane = __lane_id();
    const int leader = __builtin_ctzll(mask);
    int base = 0;
    if (lane == leader) base = atomicAdd(&s.ctr[C_PEND], __popcll(mask));
    base = __shfl(base, leader);
    if (mover) {
        const unsigned long long below = mask & ((1ull << lane) - 1ull);
        s.pend[base + __popcll(below)] = id;
    }
}

template <int V, bool DEBUG>
__device__ void plan_tile(const SlotDev &s, int tile_x, int tile_y, int step, PlanShared &sh)
{
    constexpr int SIDE = 2 * V + 1;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int LX = s.tx + 2 * V, LY = s.ty + 2 * V;
    const int ns = LX * LY;
    const int gx0 = tile_x * s.tx, gy0 = tile_y * s.ty;     // padded origin of the window
    const int tstride = s.ntx + 2;
    const bool fallback = s.tile_fb[tile_y * s.ntx + tile_x] != 0;

    if (tid < 9) sh.m_nb[tid] = s.tile_m[(tile_y + tid / 3) * tstride + tile_x + tid % 3];
    if (tid == 0) { sh.n_agents = 0; sh.n_flag = 0; }
    __syncthreads();
    const int mT = sh.m_nb[4];

    // --- stage the window: Em = 2^(m_T - m_T') G where free, 0 where occupied
    const float invLX = 1.0f / (float)LX;
    for (int i = tid; i < ns; i += nthr) {
        const int ly = (int)(((float)i + 0.5f) * invLX);
        const int lx = i - ly * LX;
        const int g = (gy0 + ly) * s.Wp + gx0 + lx;
        const int o = s.occ[g];
        const float G = s.G[g];
        const int nbx = (lx >= V) + (lx >= V + s.tx);
        const int nby = (ly >= V) + (ly >= V + s.ty);
        const float e = ldexpf(G, mT - sh.m_nb[nby * 3 + nbx]);
        sh.Em[i] = o < 0 ? e : 0.0f;
        if (nbx == 1 && nby == 1 && o >= 0) {
            const int k = atomicAdd(&sh.n_agents, 1);
            sh.a_id[k] = o;
            sh.a_g[k] = g;
            sh.a_l[k] = (int16_t)i;
            sh.a_ec[k] = e;
        }
    }
    __syncthreads();
    const int na = sh.n_agents;
    const uint32_t kseed0 = s.seed_lo, kseed1 = s.seed_hi;
    if (tid == 0 && na > 0) atomicAdd(&s.stat[S_PLANNED], (unsigned long long)na);

    if (fallback) {
        // every draw of this tile in FP64, one lane per agent
        for (int k = tid; k < na; k += nthr) {
            const int id = sh.a_id[k], gc = sh.a_g[k];
            const uint32_t x0 = philox_word0((uint32_t)id, (uint32_t)step, s.scn, STREAM_PLAN,
                                             kseed0, kseed1);
            const float u = (float)(x0 >> 8) * 0x1p-24f;
            const int t = resolve64_lane<V, DEBUG>(s, gc, id, u);
            s.desired[id] = t;
            if (DEBUG && s.dbg_flag) s.dbg_flag[id] = 2;
            if (DEBUG && s.dbg_margin) s.dbg_margin[id] = -1.0f;
        }
        for (int base = 0; base < na; base += nthr) {
            const int k = base + tid;
            bool mover = false;
            int id = 0;
            if (k < na) { id = sh.a_id[k]; mover = s.desired[id] != sh.a_g[k]; }
            append_movers(s, mover, id);
        }
        if (tid == 0 && na > 0) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)na);
        return;
    }

    // --- one lane per agent, FP32 from the LDS table
    for (int base = 0; base < na; base += nthr) {
        const int k = base + tid;
        bool mover = false;
        int id = 0;
        if (k < na) {
            id = sh.a_id[k];
            const int gc = sh.a_g[k];
            const int l = sh.a_l[k];
            const float ec = sh.a_ec[k];

            float Rs[SIDE];
            all_rows<V>(std::make_integer_sequence<int, SIDE>{}, Rs, sh.Em, l, LX, ec);
            float P[SIDE + 1];
            P[0] = 0.0f;
#pragma unroll
            for (int r = 0; r < SIDE; ++r) P[r + 1] = P[r] + Rs[r];
            const float Wsum = P[SIDE];

            const uint32_t x0 = philox_word0((uint32_t)id, (uint32_t)step, s.scn, STREAM_PLAN,
                                             kseed0, kseed1);
            const float u = (float)(x0 >> 8) * 0x1p-24f;
            const float tau = u * Wsum;

            // row: the last r with P_r <= tau
            int rs = 0, as = half_width(V, -V);
            float Ps = 0.0f;
#pragma unroll
            for (int r = 1; r < SIDE; ++r) {
                const bool le = P[r] <= tau;
                rs = le ? r : rs;
                Ps = le ? P[r] : Ps;
                as = le ? half_width(V, r - V) : as;
            }
            // slot within the row: count of in-row boundaries <= tau
            const int rowbase = l + (rs - V) * LX - as;
            float Q = 0.0f;
            float margin = fabsf(tau - Ps);
            int ks = 0;
#pragma unroll
            for (int d = 0; d < SIDE; ++d) {
                if (d <= 2 * as) {
                    const float val = (rs == V && d == as) ? ec : sh.Em[rowbase + d];
                    Q = Q + val;
                    const float C = Ps + Q;
                    const float diff = tau - C;
                    ks += diff >= 0.0f ? 1 : 0;
                    margin = fminf(margin, fabsf(diff));
                }
            }
            const bool flag = (margin <= s.eps * Wsum) || (ks > 2 * as);
            const int tgt = gc + (rs - V) * s.Wp + (ks - as);

            if (DEBUG) {
                if (s.dbg_w) {
                    float *wd = s.dbg_w + (size_t)id * SIDE * SIDE;
                    for (int dy = -V; dy <= V; ++dy)
                        for (int dx = -V; dx <= V; ++dx) {
                            float wv = 0.0f;
                            if (dx * dx + dy * dy <= V * V)
                                wv = (dx == 0 && dy == 0) ? 1.0f : sh.Em[l + dy * LX + dx] / ec;
                            wd[(dy + V) * SIDE + dx + V] = wv;
                        }
                }
                if (s.dbg_flag) s.dbg_flag[id] = flag ? 1 : 0;
                if (s.dbg_margin) s.dbg_margin[id] = margin / Wsum;
            }
            if (flag) {
                const int f = atomicAdd(&sh.n_flag, 1);
                sh.f_k[f] = (int16_t)k;
                sh.f_u[f] = u;
            } else {
                s.desired[id] = tgt;
                mover = tgt != gc;
            }
        }
        append_movers(s, mover, id);
    }
    __syncthreads();

    // --- FP64 re-resolve of the flagged draws, one wavefront per draw
    const int nf = sh.n_flag;
    if (nf == 0) return;
    const int lane = __lane_id();
    const int wave = tid >> 6, nwaves = nthr >> 6;
    for (int f = wave; f < nf; f += nwaves) {
        const int k = sh.f_k[f];
        const int id = sh.a_id[k], gc = sh.a_g[k];
        const int t = resolve64_wave<V>(s, gc, sh.f_u[f], lane);
        if (lane == 0) {
            s.desired[id] = t;
            if (t != gc) {
                const int p = atomicAdd(&s.ctr[C_PEND], 1);
                s.pend[p] = id;
            }
        }
    }
    if (tid == 0) atomicAdd(&s.stat[S_FLAGGED], (unsigned long long)nf);
}

// items[i] = (slot << 20) | tile index (row-major over the slot's tiles)
template <bool DEBUG>
__global__ __launch_bounds__(PLAN_THREADS) void plan_kernel(const SlotDev *__restrict__ table,
                                                            const uint32_t *__restrict__ items)
{
    __shared__ PlanShared sh;
    const uint32_t it = items[blockIdx.x];
    const SlotDev &s = table[it >> 20];
    const int tile = (int)(it & 0xFFFFFu);
    const int step = s.ctr[C_STEP];
    if (step >= s.ctr[C_LIMIT]) return;
    const int tile_y = tile / s.ntx, tile_x = tile - tile_y * s.ntx;
    if (tile == 0 && threadIdx.x < 4) s.ctr[C_BAR + threadIdx.x] = 0;   // fresh motion barriers
    switch (s.v) {
        case 1: plan_tile<1, DEBUG>(s, tile_x, tile_y, step, sh); break;
        case 2: plan_tile<2, DEBUG>(s, tile_x, tile_y, step, sh); break;
        case 3: plan_tile<3, DEBUG>(s, tile_x, tile_y, step, sh); break;
        case 4: plan_tile<4, DEBUG>(s, tile_x, tile_y, step, sh); break;
        case 5: plan_tile<5, DEBUG>(s, tile_x, tile_y, step, sh); break;
        default: break;
    }
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
            s.pos[id] = -1;
            s.desired[id] = -1;
            atomicAdd(&s.ctr[C_EXITED], 1);
            atomicSub(&s.ctr[C_NACTIVE], 1);
        } else if (at != c) {
            st_agent(&s.occ[c], -1);
            st_agent(&s.occ[at], id);
            s.pos[id] = at;
        }
    }
    __syncthreads();
    return sh_cnt;
}

template <int V>
__device__ void move_group(const SlotDev &s, int g, int G, int step)
{
    const int tid = threadIdx.x;
    const int Wp = s.Wp;
    const int n0 = s.ctr[C_PEND];
    const int lo = (int)((long)n0 * g / G), hi = (int)((long)n0 * (g + 1) / G);
    Mover *cur = s.mv_a + lo, *nxt = s.mv_b + lo;
    unsigned long long seen0 = 0, seen1 = 0;
    uint32_t tag = (uint32_t)s.ctr[C_TAG];

    // this workgroup's movers with priority words [~x0:32][~id:20] (larger = earlier)
    int n = hi - lo;
    for (int i = tid; i < n; i += blockDim.x) {
        const int id = s.pend[lo + i];
        const uint32_t x0 = philox_word0((uint32_t)id, (uint32_t)step, s.scn, STREAM_ORDER,
                                         s.seed_lo, s.seed_hi);
        const int c = s.pos[id], d = s.desired[id];
        const int cy = c / Wp, dy = d / Wp;
        Mover mv;
        mv.key = ((unsigned long long)(~x0) << ID_BITS) | (unsigned long long)(~(uint32_t)id & ID_MASK);
        mv.cxy = (uint32_t)(c - cy * Wp) | ((uint32_t)cy << 16);
        mv.dxy = (uint32_t)(d - dy * Wp) | ((uint32_t)dy << 16);
        cur[i] = mv;
    }
    __syncthreads();

    int total = n0, rounds = 0, bar_r = 0;
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
        s.ctr[C_PEND] = 0;
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

__global__ void reset_kernel(const SlotDev *__restrict__ table, const int32_t *__restrict__ slots,
                             int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) table[slots[i]].ctr[C_PEND] = 0;
}

}  // namespace fk

// ---------------------------------------------------------------------------
// Launchers used by the host runtime.
// ---------------------------------------------------------------------------
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

extern "C" hipError_t fk_launch_reset(const fk::SlotDev *table, const int32_t *slots, int n_slots,
                                      hipStream_t stream)
{
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk::reset_kernel, dim3((n_slots + 255) / 256), dim3(256), 0, stream, table,
                       slots, n_slots);
    return hipGetLastError();
}
