// plan_het.hip -- planning with a maximum speed per agent.
//
// Sec. 3 of the paper expects richer situations than one speed for everybody
// to cost more planning work.  Here agent i reaches only the cells of its own
// disc dx^2 + dy^2 <= v_i^2 (v_i <= the scenario's v_max, which sets the
// staged window).  Every draw is made in FP64, one lane per agent, in the
// paper's order: weights exp(k_S (S(c) - S(t))) over the window in raster
// order (zero outside the reach set), the sequential sum W, tau = u W with
// the agent's Philox u, and the first cell whose prefix exceeds tau.  The
// tile's agents are listed by the same staging as the uniform kernels.
#include <hip/hip_ext.h>

#include "plan_tile.h"

namespace fk {

// Agent at padded cell gc with reach vr: the chosen padded cell.  The first
// pass sums the weights sequentially in raster order and keeps the prefix at
// the end of every window row; the second starts from the prefix before the
// first row whose end exceeds tau and sums that row again, cell by cell.  Its
// prefixes are the very values of the full sequential sum, so the choice is
// the same, at one row of exps instead of the whole window.
template <int V>
__device__ __forceinline__ bool reach_het(const SlotDev &s, int gc, int t, int dx, int dy, int vr)
{
    return dx * dx + dy * dy <= vr * vr && (s.cell[t] & CELL_TYPE_MASK) != CELL_WALL &&
           (s.occ[t] < 0 || t == gc);
}

template <int V>
__device__ int draw_het(const SlotDev &s, int gc, float u32, int vr)
{
    constexpr int SIDE = 2 * V + 1;
    const double Sc = s.S[gc];
    const double ks = s.k_s;
    double rowC[SIDE];
    double C = 0.0;
#pragma unroll
    for (int r = 0; r < SIDE; ++r) {
        const int dy = r - V;
#pragma unroll
        for (int dx = -V; dx <= V; ++dx) {
            const int t = gc + dy * s.Wp + dx;
            if (reach_het<V>(s, gc, t, dx, dy, vr)) C = C + exp(ks * (Sc - s.S[t]));
        }
        rowC[r] = C;
    }
    const double tau = (double)u32 * C;
    int row = SIDE - 1;
    double Cprev = SIDE > 1 ? rowC[SIDE - 2] : 0.0;
    bool found = false;
#pragma unroll
    for (int r = 0; r < SIDE; ++r) {
        const bool hit = !found && tau < rowC[r];
        row = hit ? r : row;
        Cprev = hit ? (r > 0 ? rowC[r - 1] : 0.0) : Cprev;
        found = found || hit;
    }
    const int dy = row - V;
    double C2 = Cprev;
#pragma unroll 1
    for (int dx = -V; dx <= V; ++dx) {
        const int t = gc + dy * s.Wp + dx;
        if (reach_het<V>(s, gc, t, dx, dy, vr)) {
            C2 = C2 + exp(ks * (Sc - s.S[t]));
            if (tau < C2) return t;
        }
    }
    return gc;   // not reached: the own cell has weight 1 and tau < W
}

// Workgroup i plans tile i; vi[id] is agent id's speed (1..v_max).
template <int V, int TX>
__global__ __launch_bounds__(PLAN_THREADS) void plan_kernel_het(const SlotDev s,
                                                                const uint8_t *__restrict__ vi)
{
    __shared__ PlanShared<false> sh;
    using T = TileGeom<V, TX>;
    constexpr int P = T::P;
    const int tile = (int)blockIdx.x;
    const int step = s.ctr[C_STEP];
    const int limit = s.ctr[C_LIMIT];
    const T tg(s, tile);
    StageRegs<false> r;
    stage_issue<V, TX, false>(s, tg, r);
    if (step >= limit) return;                                // scenario finished
    if (tile == 0 && threadIdx.x < 4) s.ctr[C_BAR + threadIdx.x] = 0;   // fresh motion barriers
    stage_commit<V, TX, false>(s, tg, sh, r);                 // lists the tile's agents
    MoveRec *seg = s.seg + (long)tile * (TX * s.ty);
    const int na = sh.n_agents;
    for (int base = 0; base < na; base += (int)blockDim.x) {
        const int k = base + (int)threadIdx.x;
        if (k < na) {
            const int id = (int)(sh.a_pk[k] >> 12);
            const int l = (int)(sh.a_pk[k] & 0xFFFu);
            const int ly = l / P;
            const int cx = tg.gx0 + (l - ly * P), cy = tg.gy0 + ly;
            const int gc = cy * s.Wp + cx;
            const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, s.scn, s.seed_lo,
                                               s.seed_hi);
            const float u = (float)(x0 >> 8) * 0x1p-24f;
            const int t = draw_het<V>(s, gc, u, (int)vi[id]);
            const int d = t - gc;                               // |dx|, |dy| <= V < Wp / 2
            const int ddy = (d + V * s.Wp + V) / s.Wp - V, ddx = d - ddy * s.Wp;
            gstore_rec(seg + k, (uint32_t)id, pack_xy(cx, cy), pack_xy(cx + ddx, cy + ddy));
        }
    }
    if (threadIdx.x == 0) {
        s.seg_cnt[tile] = na;
        if (na > 0) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)na);
    }
}

template <int V>
hipError_t launch_het_v(const SlotDev &s, const uint8_t *vi, dim3 grid, hipStream_t stream,
                        hipEvent_t start, hipEvent_t stop)
{
    const dim3 block(PLAN_THREADS);
    switch (s.tx) {
        case 8: hipExtLaunchKernelGGL((plan_kernel_het<V, 8>), grid, block, 0, stream, start, stop, 0, s, vi); break;
        case 16: hipExtLaunchKernelGGL((plan_kernel_het<V, 16>), grid, block, 0, stream, start, stop, 0, s, vi); break;
        case 32: hipExtLaunchKernelGGL((plan_kernel_het<V, 32>), grid, block, 0, stream, start, stop, 0, s, vi); break;
        case 64: hipExtLaunchKernelGGL((plan_kernel_het<V, 64>), grid, block, 0, stream, start, stop, 0, s, vi); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fk

// Planning launch of one scenario with per-agent speeds vi (device, n_agents).
extern "C" hipError_t fk_launch_plan_het(const fk::SlotDev *slot, const uint8_t *vi, int n_tiles,
                                         hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    const dim3 grid(n_tiles);
    switch (slot->v) {
        case 1: return fk::launch_het_v<1>(*slot, vi, grid, stream, start, stop);
        case 2: return fk::launch_het_v<2>(*slot, vi, grid, stream, start, stop);
        case 3: return fk::launch_het_v<3>(*slot, vi, grid, stream, start, stop);
        case 4: return fk::launch_het_v<4>(*slot, vi, grid, stream, start, stop);
        case 5: return fk::launch_het_v<5>(*slot, vi, grid, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
}
