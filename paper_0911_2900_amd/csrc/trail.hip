// trail.hip -- the dynamic floor field: one of the couplings k_other that the
// paper sets to 0 (Sec. 2) and cites without restating.  This library's
// reading: every cell holds a trail value T (FP64), zero at the start; an
// agent that leaves the cell it started the step on deposits 1 there (the
// motion kernel counts the deposits); after each motion phase every non-wall
// cell takes
//     T' = (1 - delta) ((1 - alpha) T + (alpha / 8) N) + deposits,
// N the sum of its 8 neighbours in raster order (walls hold 0); and the
// planning weight of a window cell t becomes exp(k_S (S(c) - S(t)) +
// k_D (T(t) - T(c))).
//
// One launch follows each motion phase of a scenario with a trail field:
// workgroup i takes tile i, forms the trail of its own cells for the new step
// and their exp table entries with the trail term (G(t) = fl32(exp(m_T ln 2 -
// k_S S(t) + k_D T(t)))), and takes the tile's range-fallback flag afresh
// from its whole window, whose trail values it forms again itself (the same
// operations in the same order, so the same values the neighbouring tiles
// store).  The trail of step s lives in buffer s & 1, so the launch only
// reads the counters and can run again with the same result (a served
// scenario past its last step skips its motion phase but not this launch).
#include <hip/hip_runtime.h>

#include "fast_dev.h"

namespace fk {

constexpr int TRAIL_THREADS = 1024;
constexpr double LN2_64 = 0x1.62e42fefa39efp-1;   // nearest double to ln 2
constexpr double RANGE = 80.0;                    // |exponent| bound of a table entry

// The trail of non-wall cell t for the new step, from the old trail To and
// the deposits.  The padded border is wall, so every non-wall cell has its 8
// neighbours inside the padded grid; wall neighbours hold 0, and adding 0
// leaves the sum unchanged bit for bit.  All loads are issued before any
// arithmetic.
__device__ __forceinline__ double trail_at(const SlotDev &s, const double *__restrict__ To, long t,
                                           double keep, double stay, double share)
{
    const int Wp = s.Wp;
    double n[8];
    int q = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
            if (dx || dy) n[q++] = To[t + dy * Wp + dx];
    const double own = To[t];
    const double dep = (double)s.dep[t];
    double nb = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) nb = nb + n[k];
    return keep * (stay * own + share * nb) + dep;
}

__global__ __launch_bounds__(TRAIL_THREADS) void trail_kernel(const SlotDev s)
{
    __shared__ int out_of_range;
    const int tile = (int)blockIdx.x;
    const int stp = s.ctr[C_STEP];
    if (stp <= 0) return;                                     // no motion phase yet
    const long cells = (long)s.Wp * s.Hp;
    const double *__restrict__ To = s.Tr + (long)((stp - 1) & 1) * cells;
    double *__restrict__ Tn = s.Tr + (long)(stp & 1) * cells;
    const double keep = 1.0 - s.t_decay, stay = 1.0 - s.t_diff, share = s.t_diff / 8.0;
    const int ty0 = tile / s.ntx, tx0 = tile - ty0 * s.ntx;
    const int ts = s.ntx + 2;
    const int mT = s.tile_m[(ty0 + 1) * ts + tx0 + 1];
    const double ks = s.k_s, kd = s.k_d;
    if (threadIdx.x == 0) out_of_range = 0;
    // the tile's own cells: the new trail and the exp table entry (the
    // occupancy bit of D kept)
    for (int k = threadIdx.x; k < s.tx * s.ty; k += blockDim.x) {
        const int ly = k / s.tx, lx = k - ly * s.tx;
        const long t = (long)(ty0 * s.ty + s.pad + ly) * s.Wp + tx0 * s.tx + s.pad + lx;
        const double St = s.S[t];
        if (!(St < INFINITY)) {                               // wall: no trail, the entry stays 0
            Tn[t] = 0.0;
            continue;
        }
        const double T = trail_at(s, To, t, keep, stay, share);
        Tn[t] = T;
        const double e = (double)mT * LN2_64 - ks * St + kd * T;
        const float g = fabs(e) > RANGE ? 0.0f : (float)exp(e);
        s.D[t] = __float_as_uint(g) | (s.D[t] & D_OCC);
    }
    __syncthreads();
    // the window, this tile grown by v on every side: is any exponent, in
    // this tile's scale or in the scale of the tile holding the cell, out of
    // [-80, 80]?  (The rule the scenario's setup applies with T = 0.)
    const int wx0 = tx0 * s.tx + s.pad - s.v, wy0 = ty0 * s.ty + s.pad - s.v;
    const int ww = s.tx + 2 * s.v, wh = s.ty + 2 * s.v;
    int bad = 0;
    for (int k = threadIdx.x; k < ww * wh; k += blockDim.x) {
        const int wy = k / ww, wx = k - wy * ww;
        const int y = wy0 + wy, x = wx0 + wx;
        const long t = (long)y * s.Wp + x;
        const double St = s.S[t];
        if (!(St < INFINITY)) continue;
        // the tile holding t (t has a finite floor field, so it lies on the grid)
        const int oy = (y - s.pad) / s.ty, ox = (x - s.pad) / s.tx;
        const int mo = s.tile_m[(oy + 1) * ts + ox + 1];
        const double rest = -ks * St + kd * trail_at(s, To, t, keep, stay, share);
        const double eT = (double)mT * LN2_64 + rest, eO = (double)mo * LN2_64 + rest;
        bad |= (fabs(eT) > RANGE || fabs(eO) > RANGE) ? 1 : 0;
    }
    if (bad) out_of_range = 1;
    __syncthreads();
    if (threadIdx.x == 0) s.tile_fb[tile] = out_of_range ? 1 : 0;
}

}  // namespace fk

// The launch that closes a motion phase of a scenario with a trail field.
extern "C" hipError_t fk_launch_trail(const fk::SlotDev *slot, int n_tiles, hipStream_t stream)
{
    if (!slot->Tr || n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk::trail_kernel, dim3(n_tiles), dim3(fk::TRAIL_THREADS), 0, stream, *slot);
    return hipGetLastError();
}
