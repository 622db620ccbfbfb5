// plan_het.hip -- planning with a maximum speed per agent.
//
// Sec. 3 of the paper expects richer situations than one speed for everybody
// to cost more planning work.  Here agent i reaches only the cells of its own
// disc dx^2 + dy^2 <= v_i^2 (v_i <= the scenario's v_max, which sets the
// staged window).  The same kernel plans scenarios with several floor fields
// (one per exit group): agent i then weighs its window with field fi[i].
// Every draw is made in FP64, one wavefront per agent, and
// chooses what the paper's order gives: weights exp(k_S (S(c) - S(t))) over
// the window in raster order (zero outside the reach set), the sequential sum
// W, tau = u W with the agent's Philox u, and the first cell whose prefix
// exceeds tau.  The tile's agents are listed by the same staging as the
// uniform kernels.
#include <hip/hip_ext.h>

#include "plan_tile.h"

namespace fk {

// The draw of the agent at padded cell gc with reach vr, by a whole
// wavefront: lane j takes raster slot j of the (2V+1)^2 window (and slot
// j + 64 when the window has more than 64 slots) and evaluates its weight;
// an FP64 wavefront scan gives the prefixes.  As in the uniform kernels' FP64
// path, a scanned prefix of at most 128 non-negative terms lies within
// 1.5e-14 W of the sequential one, so when no prefix is within s.near64 W
// (1e-12 W) of tau every comparison tau < C_j, and with it the choice, is the
// sequential sum's; otherwise the prefix is rebuilt strictly sequentially,
// slot by slot (slots outside the reach set add exactly nothing).  Every lane
// returns the chosen raster slot of the window.
template <int V>
__device__ int draw_het_wave(const SlotDev &s, const double *__restrict__ S, int gc, float u32,
                             int lane, int vr)
{
    constexpr int SIDE = 2 * V + 1, NS = SIDE * SIDE, NH = (NS + 63) / 64;
    const double NEAR = s.near64;
    const double Sc = S[gc];
    const double ks = s.k_s;
    const double u = (double)u32;
    double w[NH], C[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int j = lane + 64 * h;
        w[h] = 0.0;
        if (j < NS) {
            // the three reads of the slot are independent (every slot lies in
            // the padded grid), so they are issued together
            const int dy = j / SIDE - V, dx = j % SIDE - V;
            const int t = gc + dy * s.Wp + dx;
            const uint8_t ct = s.cell[t];
            const int o = s.occ[t];
            const double St = S[t];
            const bool reach = dx * dx + dy * dy <= vr * vr && (ct & CELL_TYPE_MASK) != CELL_WALL &&
                               (o < 0 || t == gc);
            if (reach) w[h] = exp(ks * (Sc - St));
        }
    }
    C[0] = wave_scan64(w[0]);
    if constexpr (NH == 2) C[1] = wave_scan64(w[1]) + lane_value(C[0], 63);
    const double Wt = lane_value(C[NH - 1], (NS - 1) % 64);
    const double tp = u * Wt;
    bool near = false;
#pragma unroll
    for (int h = 0; h < NH; ++h) near = near || (lane + 64 * h < NS && fabs(tp - C[h]) <= NEAR * Wt);
    unsigned long long m[NH];
    if (__ballot(near) == 0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) m[h] = __ballot(lane + 64 * h < NS && tp < C[h]);
    } else {
        double acc = 0.0, my[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) my[h] = 0.0;
#pragma unroll 1
        for (int j = 0; j < NS; ++j) {
            const double wj = NH == 2 && j >= 64 ? lane_value(w[NH - 1], j - 64) : lane_value(w[0], j & 63);
            acc = acc + wj;
            if (j < 64) { if (lane == j) my[0] = acc; }
            else if (lane == j - 64) my[NH - 1] = acc;
        }
        const double tau = u * acc;
#pragma unroll
        for (int h = 0; h < NH; ++h) m[h] = __ballot(lane + 64 * h < NS && tau < my[h]);
    }
    int jw = (NS - 1) / 2;                                    // own cell if unreached
    if (m[0]) jw = __builtin_ctzll(m[0]);
    else if (NH == 2 && m[NH - 1]) jw = 64 + __builtin_ctzll(m[NH - 1]);
    return jw;
}

// Workgroup i plans tile i with HET_THREADS threads; wavefront q draws the
// tile's agents q, q + HET_THREADS / 64, ...; vi[id] is agent id's speed.
// FIELDS: agent id follows the floor field at Sf + fi[id] * field_cells and
// vi may be NULL (every agent has V); otherwise the scenario's one field
// s.S, with vi set.  Each form is its own kernel, so the single-field form
// does no per-agent field lookup.
constexpr int HET_THREADS = 1024;

template <int V, int TX, bool FIELDS>
__global__ __launch_bounds__(HET_THREADS) void plan_kernel_het(const SlotDev s,
                                                               const uint8_t *__restrict__ vi,
                                                               const uint8_t *__restrict__ fi,
                                                               const double *__restrict__ Sf,
                                                               long field_cells)
{
    __shared__ PlanShared sh;
    using T = TileGeom<V, TX>;
    constexpr int P = T::P;
    const int tile = (int)blockIdx.x;
    const T tg(s, tile);
    int step = 0;
    if (!stage_tile<V, TX>(s, tg, tile, sh.Em, sh.L, step)) return;   // lists the tile's agents
    if (tile == 0 && threadIdx.x < 4) s.ctr[C_BAR + threadIdx.x] = 0;   // fresh motion barriers
    uint32_t *seg = s.seg + (long)tile * (TX * tg.ty);
    const int na = sh.L.n_agents;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int nw = (int)(blockDim.x >> 6);
    for (int k = wave; k < na; k += nw) {
        const int id = (int)(sh.L.a_pk[k] >> 12);
        const int l = (int)(sh.L.a_pk[k] & 0xFFFu);
        const int ly = l / P, lx = l - ly * P;
        const int gc = (tg.gy0 + ly) * s.Wp + tg.gx0 + lx;
        const uint32_t x0 = plan_draw_word((uint32_t)id, (uint32_t)step, s.scn, s.seed_lo, s.seed_hi);
        const float u = (float)(x0 >> 8) * 0x1p-24f;
        int slot;
        if constexpr (FIELDS) {
            // the whole wavefront draws agent k, so its field is uniform
            const int f = __builtin_amdgcn_readfirstlane((int)fi[id]);
            const int vr = vi ? (int)vi[id] : V;
            slot = draw_het_wave<V>(s, Sf + (long)f * field_cells, gc, u, lane, vr);
        } else {
            slot = draw_het_wave<V>(s, s.S, gc, u, lane, (int)vi[id]);
        }
        if (lane == 0) seg[k] = plan_rec((ly - V) * TX + (lx - T::Hc), slot);
    }
    if (threadIdx.x == 0) {
        s.seg_cnt[tile] = na;
        if (na > 0) atomicAdd(&s.stat[S_FALLBACK], (unsigned long long)na);
    }
}

template <int V>
hipError_t launch_het_v(const SlotDev &s, const uint8_t *vi, const uint8_t *fi, const double *Sf,
                        long fc, dim3 grid, hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    const dim3 block(HET_THREADS);
    if (fi) {
        switch (s.tx) {
            case 8: hipExtLaunchKernelGGL((plan_kernel_het<V, 8, true>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
            case 16: hipExtLaunchKernelGGL((plan_kernel_het<V, 16, true>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
            case 32: hipExtLaunchKernelGGL((plan_kernel_het<V, 32, true>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
            case 64: hipExtLaunchKernelGGL((plan_kernel_het<V, 64, true>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (!vi) return hipErrorInvalidValue;
    switch (s.tx) {
        case 8: hipExtLaunchKernelGGL((plan_kernel_het<V, 8, false>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
        case 16: hipExtLaunchKernelGGL((plan_kernel_het<V, 16, false>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
        case 32: hipExtLaunchKernelGGL((plan_kernel_het<V, 32, false>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
        case 64: hipExtLaunchKernelGGL((plan_kernel_het<V, 64, false>), grid, block, 0, stream, start, stop, 0, s, vi, fi, Sf, fc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fk

// Planning launch of one scenario with per-agent speeds vi and per-agent floor
// fields fi (device, n_agents each, or NULL), the fields at Sf, field_cells
// padded cells apart (Sf NULL: the scenario's one field).
extern "C" hipError_t fk_launch_plan_het(const fk::SlotDev *slot, const uint8_t *vi,
                                         const uint8_t *fi, const double *Sf, long field_cells,
                                         int n_tiles, hipStream_t stream, hipEvent_t start,
                                         hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    const dim3 grid(n_tiles);
    if (!Sf) { Sf = slot->S; fi = nullptr; }
    switch (slot->v) {
        case 1: return fk::launch_het_v<1>(*slot, vi, fi, Sf, field_cells, grid, stream, start, stop);
        case 2: return fk::launch_het_v<2>(*slot, vi, fi, Sf, field_cells, grid, stream, start, stop);
        case 3: return fk::launch_het_v<3>(*slot, vi, fi, Sf, field_cells, grid, stream, start, stop);
        case 4: return fk::launch_het_v<4>(*slot, vi, fi, Sf, field_cells, grid, stream, start, stop);
        case 5: return fk::launch_het_v<5>(*slot, vi, fi, Sf, field_cells, grid, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
}
