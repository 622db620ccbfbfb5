// plan_het.hip -- planning with a maximum speed per agent and with several
// floor fields (one per exit group), the richer situations that Sec. 3 of the
// paper expects to cost more planning work.
//
// Agent i reaches only its own disc dx^2 + dy^2 <= v_i^2 (v_i <= the
// scenario's v_max, which sets the staged window), and weighs its window with
// the floor field of its group.  The draw is the uniform model's -- weights
// exp(k_S (S(c) - S(t))) over the window in raster order, zero outside the
// reach set, the sequential sum W, tau = u W, the first cell whose prefix
// exceeds tau -- made on the same FP32 table path: each field has its own
// exp table (per-tile scales, range-fallback flags), the tile stages one
// window per field, and an agent's slots outside its own disc take an exact
// 0, which leaves the rounding structure of the sums, and so the guard band,
// unchanged.  Draws inside the band are re-resolved in FP64 by the wavefront
// with the agent's own field and reach; agents of a field for which the tile
// is a range-fallback tile draw in FP64.
//
// This file is compiled once per v_max (PLAN_V), like plan_fixed.hip.
#include <hip/hip_ext.h>

#include "plan_tile.h"

#ifndef PLAN_V
#error "PLAN_V (the v_max this object is compiled for) must be defined"
#endif

#define FK_CAT2(a, b) a##b
#define FK_CAT(a, b) FK_CAT2(a, b)

namespace fk {

// LDS of the kernel besides the staged windows (dynamic: one per field and,
// with several fields, the window of D for the occupancy bits).
struct HetShared {
    TileLists L;
    uint8_t a_gv[MAX_TILE_CELLS];      // per listed agent: field << 4 | maximum speed
    int32_t m_nbf[MAX_FIELDS * 9];     // per field: exponents of the 3 x 3 tiles around
    int fbf[MAX_FIELDS];               // per field: the tile is a range-fallback tile
};

// One tile of a scenario with per-agent speeds and / or several fields:
// workgroup i plans tile row_tile(i).
template <int V, int TX, bool DEBUG>
__global__ __launch_bounds__(ONE_MAX_THREADS) void plan_kernel_het(const SlotDev s, const HetDev h)
{
    using T = TileGeom<V, TX>;
    constexpr int cpr = T::cpr;
    extern __shared__ float4 het_dyn[];
    __shared__ HetShared sh;
    float *Ew = (float *)het_dyn;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = __lane_id();
    const int tile = row_tile((int)blockIdx.x, s.ntx, s.nty);
    if (tile < 0) return;
    const T tg(s, tile);
    const int win = 4 * tg.n_win;                             // floats per window
    const bool fields = h.nf > 1;
    const int nw = fields ? h.nf : 1;                         // windows of tables
    float *Dw = Ew + (fields ? h.nf * win : 0);               // the window of D
    int step = 0;
    const bool live = scenario_live(s, step);

    // every load: the window of D (with one field it is the table itself),
    // each field's table window, the tile's own occupancy (ids), exponents
    StageRegs r;
    stage_issue<V, TX>(s, tg, tile, Dw, r);
    int mf = 0, ff = 0;
    if (fields) {
        for (int g = 0; g < h.nf; ++g)
            issue_window<V, TX>(h.Gf + g * h.field_cells, s.Wp, s.Hp, tg, Ew + g * win);
        const int tstride = s.ntx + 2, tm_size = tstride * (s.nty + 2);
        if (tid < 9 * h.nf) {
            const int g = tid / 9, i = tid - 9 * g;
            mf = gload(&h.tile_mf[g * tm_size + (tg.tile_y + i / 3) * tstride + tg.tile_x + i % 3]);
        } else if (tid < 10 * h.nf) {
            ff = gload(&h.tile_fbf[(tid - 9 * h.nf) * (s.ntx * s.nty) + tile]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (!live) return;                                        // scenario finished
    if (tile == 0 && tid < 4) s.ctr[C_BAR + tid] = 0;         // fresh motion barriers
    if (fields) {
        if (tid < 9 * h.nf) sh.m_nbf[tid] = mf;
        else if (tid < 10 * h.nf) sh.fbf[tid - 9 * h.nf] = ff;
    } else {
        if (tid < 9) sh.m_nbf[tid] = r.mnb;
        if (tid == 9) sh.fbf[0] = r.fb;
    }
    if (tid == 0) { sh.L.n_agents = 0; sh.L.n_flag = 0; sh.L.fb = 0; }
    __syncthreads();

    // list the tile's agents from the occupancy bits of D (lane-major order,
    // as in the uniform kernels)
    {
        const bool lv = tid < tg.n_in;
        const int j = T::in_chunk(lv ? tid : 0);
        uint4 d = make_uint4(0, 0, 0, 0);
        if (lv) d = *(const uint4 *)&Dw[4 * j];
        const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
        const int ov[4] = {r.oc.x, r.oc.y, r.oc.z, r.oc.w};
        unsigned long long m[4];
        int tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) { m[k] = __ballot(lv && (dv[k] & D_OCC)); tot += __popcll(m[k]); }
        if (tot) {
            int idx0 = 0;
            if (lane == 0) idx0 = atomicAdd(&sh.L.n_agents, tot);
            int idx = __shfl(idx0, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) idx += lanes_below(m[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (lv && (dv[k] & D_OCC)) sh.L.a_pk[idx++] = ((uint32_t)ov[k] << 12) | (uint32_t)(4 * j + k);
        }
    }
    __syncthreads();
    // each agent's field, speed and own-cell value (its field's table entry,
    // read before the windows are masked)
    const int na = sh.L.n_agents;
    for (int k = tid; k < na; k += nthr) {
        const uint32_t pk = sh.L.a_pk[k];
        const int id = (int)(pk >> 12), l = (int)(pk & 0xFFFu);
        const int g = fields ? (int)h.fi[id] : 0;
        const int vr = h.vi ? (int)h.vi[id] : V;
        sh.a_gv[k] = (uint8_t)((g << 4) | vr);
        const uint32_t raw = fields ? __float_as_uint(Ew[g * win + l]) : __float_as_uint(Dw[l]);
        sh.L.a_ec[k] = __uint_as_float(raw & ~D_OCC);
    }
    __syncthreads();
    // every window: occupied cells 0, halo chunks rescaled to this tile's
    // exponent of the window's field
    for (int c = tid; c < nw * tg.n_win; c += nthr) {
        const int g = c / tg.n_win, j = c - g * tg.n_win;
        const int row = (int)((unsigned)j / cpr), cc = j - row * cpr;
        const int nby = (row >= V) + (row >= V + tg.ty);
        const int nbx = (cc >= T::hc4) + (cc >= T::hc4 + T::cw);
        const int dm = sh.m_nbf[g * 9 + 4] - sh.m_nbf[g * 9 + nby * 3 + nbx];
        // (with one field, the table window is the window of D itself)
        const uint4 o = *(const uint4 *)&Dw[4 * j];
        const uint4 d = *(const uint4 *)&Ew[g * win + 4 * j];
        auto val = [&](uint32_t occ, uint32_t x) {
            return (occ & D_OCC) ? 0.0f : ldexpf(__uint_as_float(x & ~D_OCC), dm);
        };
        *(float4 *)&Ew[g * win + 4 * j] = make_float4(val(o.x, d.x), val(o.y, d.y), val(o.z, d.z),
                                                       val(o.w, d.w));
    }
    __syncthreads();
    HetView hv;
    hv.a_gv = sh.a_gv;
    hv.fbf = sh.fbf;
    hv.Sf = fields ? h.Sf : nullptr;
    hv.field_cells = h.field_cells;
    hv.win = win;
    plan_agents<V, TX, DEBUG, true>(s, tg, tile, Ew, sh.L, step, hv);
}

}  // namespace fk

namespace {

// (Internal linkage: this file is compiled once per v_max, and each object
// must launch its own kernels.)
template <int V, bool DEBUG, int TX>
hipError_t launch_het_tx(const fk::SlotDev &s, const fk::HetDev &h, int n_tiles, hipStream_t stream,
                         hipEvent_t start, hipEvent_t stop)
{
    using T = fk::TileGeom<V, TX>;
    const int cells = s.tx * s.ty;
    const int threads = cells < fk::PLAN_THREADS ? fk::PLAN_THREADS
                        : cells > fk::ONE_MAX_THREADS ? fk::ONE_MAX_THREADS : cells;
    const size_t n_win = (size_t)T::cpr * (s.ty + 2 * V);
    const size_t lds = (size_t)(h.nf > 1 ? h.nf + 1 : 1) * n_win * 16;
    hipExtLaunchKernelGGL((fk::plan_kernel_het<V, TX, DEBUG>), dim3(fk::row_grid(s.ntx, s.nty)), dim3(threads), lds,
                          stream, start, stop, 0, s, h);
    return hipGetLastError();
}

}  // namespace

// Planning launch of one scenario with per-agent speeds and / or several
// fields (h), one workgroup per tile; debug: also the weights, flags,
// margins and CDF of every draw (the descriptor's debug outputs).
extern "C" hipError_t FK_CAT(fk_launch_plan_het_v, PLAN_V)(const fk::SlotDev *slot,
                                                            const fk::HetDev *h, int n_tiles,
                                                            int debug, hipStream_t stream,
                                                            hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    if (slot->v != PLAN_V) return hipErrorInvalidValue;
    // (fi may be null when the scenario has no agents)
    if (h->nf < 1 || h->nf > fk::MAX_FIELDS || (h->nf > 1 && (!h->Gf || !h->Sf)))
        return hipErrorInvalidValue;
    if (debug) {
        switch (slot->tx) {
            case 8: return launch_het_tx<PLAN_V, true, 8>(*slot, *h, n_tiles, stream, start, stop);
            case 16: return launch_het_tx<PLAN_V, true, 16>(*slot, *h, n_tiles, stream, start, stop);
            case 32: return launch_het_tx<PLAN_V, true, 32>(*slot, *h, n_tiles, stream, start, stop);
            case 64: return launch_het_tx<PLAN_V, true, 64>(*slot, *h, n_tiles, stream, start, stop);
            default: return hipErrorInvalidValue;
        }
    }
    switch (slot->tx) {
        case 8: return launch_het_tx<PLAN_V, false, 8>(*slot, *h, n_tiles, stream, start, stop);
        case 16: return launch_het_tx<PLAN_V, false, 16>(*slot, *h, n_tiles, stream, start, stop);
        case 32: return launch_het_tx<PLAN_V, false, 32>(*slot, *h, n_tiles, stream, start, stop);
        case 64: return launch_het_tx<PLAN_V, false, 64>(*slot, *h, n_tiles, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
}
