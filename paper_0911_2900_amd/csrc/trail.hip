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
// workgroup i takes tile i.  It stages the old trail of the tile's window
// (this tile grown by v on every side) and of a ring of one cell around it
// in LDS, with one round of loads, then forms the new trail of every window
// cell from there (the same operations in the same order for every cell, so
// each tile forms the values its neighbours store): for the tile's own cells
// it stores that trail and the exp table entry with the trail term
// (G(t) = fl32(exp(m_T ln 2 - k_S S(t) + k_D T(t)))); over the whole window it
// takes the tile's range-fallback flag afresh.  The trail of step s lives in
// buffer s & 1, so the launch only reads the counters and can run again with
// the same result (a served scenario past its last step skips its motion
// phase but not this launch).
#include <hip/hip_runtime.h>

#include "fast_dev.h"

namespace fk {

constexpr int TRAIL_THREADS = 1024;
constexpr int TRAIL_CELLS = 2;                    // window cells per thread at most
constexpr int TRAIL_RING_MAX = 2128;              // (tx + 2v + 2)(ty + 2v + 2), allowed tiles, v <= 5
constexpr double LN2_64 = 0x1.62e42fefa39efp-1;   // nearest double to ln 2
constexpr double RANGE = 80.0;                    // |exponent| bound of a table entry

__global__ __launch_bounds__(TRAIL_THREADS) void trail_kernel(const SlotDev s)
{
    __shared__ double ring[TRAIL_RING_MAX];       // old trail of the window and a ring around it
    __shared__ int m_nb[9];                       // exponents of the 3 x 3 tiles around this one
    __shared__ int out_of_range;
    const int tile = (int)blockIdx.x, tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int stp = s.ctr[C_STEP];
    if (stp <= 0) return;                                     // no motion phase yet
    const long cells = (long)s.Wp * s.Hp;
    const double *__restrict__ To = s.Tr + (long)((stp - 1) & 1) * cells;
    double *__restrict__ Tn = s.Tr + (long)(stp & 1) * cells;
    const double keep = 1.0 - s.t_decay, stay = 1.0 - s.t_diff, share = s.t_diff / 8.0;
    const int ty0 = tile / s.ntx, tx0 = tile - ty0 * s.ntx;
    const int ts = s.ntx + 2;
    const double ks = s.k_s, kd = s.k_d;
    const int v = s.v, Wp = s.Wp;
    const int wx0 = tx0 * s.tx + s.pad - v, wy0 = ty0 * s.ty + s.pad - v;   // window cell (0, 0)
    const int ww = s.tx + 2 * v, wh = s.ty + 2 * v, rw = ww + 2, rh = wh + 2;

    // every load at once: the ring (padded cells only; none of the cells
    // outside the grid is read below), the exponents, and each thread's
    // window cells' floor field, deposits and table words
    for (int k = tid; k < rw * rh; k += nthr) {
        const int ry = k / rw, rx = k - ry * rw;
        const int y = wy0 - 1 + ry, x = wx0 - 1 + rx;
        ring[k] = (x >= 0 && x < Wp && y >= 0 && y < s.Hp) ? To[(long)y * Wp + x] : 0.0;
    }
    if (tid < 9) m_nb[tid] = s.tile_m[(ty0 + tid / 3) * ts + tx0 + tid % 3];
    if (tid == 0) out_of_range = 0;
    double St[TRAIL_CELLS];
    int dep[TRAIL_CELLS];
    uint32_t dw[TRAIL_CELLS];
#pragma unroll
    for (int c = 0; c < TRAIL_CELLS; ++c) {
        const int k = tid + c * nthr;
        St[c] = INFINITY;
        dep[c] = 0;
        dw[c] = 0;
        if (k < ww * wh) {
            const int wy = k / ww, wx = k - wy * ww;
            const long t = (long)(wy0 + wy) * Wp + wx0 + wx;
            St[c] = s.S[t];
            dep[c] = s.dep[t];
            if (wy >= v && wy < v + s.ty && wx >= v && wx < v + s.tx) dw[c] = s.D[t];
        }
    }
    __syncthreads();

    const int mT = m_nb[4];
    int bad = 0;
#pragma unroll
    for (int c = 0; c < TRAIL_CELLS; ++c) {
        const int k = tid + c * nthr;
        if (k >= ww * wh) continue;
        const int wy = k / ww, wx = k - wy * ww;
        const int y = wy0 + wy, x = wx0 + wx;
        const long t = (long)y * Wp + x;
        const bool own = wy >= v && wy < v + s.ty && wx >= v && wx < v + s.tx;
        if (!(St[c] < INFINITY)) {                            // wall: no trail, the entry stays 0
            if (own) Tn[t] = 0.0;
            continue;
        }
        // the new trail: the 8 neighbours in (dy, dx) order, summed in that
        // order, then (1 - delta) ((1 - alpha) T + (alpha / 8) N) + deposits;
        // the padded border is wall, so every neighbour lies in the ring
        const int r0 = (wy + 1) * rw + wx + 1;
        double n[8];
        int q = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                if (dx || dy) n[q++] = ring[r0 + dy * rw + dx];
        double nb = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) nb = nb + n[j];
        const double T = keep * (stay * ring[r0] + share * nb) + (double)dep[c];
        if (own) {
            Tn[t] = T;
            const double e = (double)mT * LN2_64 - ks * St[c] + kd * T;
            const float g = fabs(e) > RANGE ? 0.0f : (float)exp(e);
            s.D[t] = __float_as_uint(g) | (dw[c] & D_OCC);
        }
        // is the exponent, in this tile's scale or in the scale of the tile
        // holding t (one of the 3 x 3 around: v is below the tile size),
        // out of [-80, 80]?  (The rule the scenario's setup applies with T = 0.)
        const int oy = (y - s.pad) / s.ty, ox = (x - s.pad) / s.tx;
        const int mo = m_nb[(oy - ty0 + 1) * 3 + ox - tx0 + 1];
        const double rest = -ks * St[c] + kd * T;
        const double eT = (double)mT * LN2_64 + rest, eO = (double)mo * LN2_64 + rest;
        bad |= (fabs(eT) > RANGE || fabs(eO) > RANGE) ? 1 : 0;
    }
    if (bad) out_of_range = 1;
    __syncthreads();
    if (tid == 0) s.tile_fb[tile] = out_of_range ? 1 : 0;
}

}  // namespace fk

// The launch that closes a motion phase of a scenario with a trail field.
extern "C" hipError_t fk_launch_trail(const fk::SlotDev *slot, int n_tiles, hipStream_t stream)
{
    if (!slot->Tr || n_tiles <= 0) return hipSuccess;
    const int ww = slot->tx + 2 * slot->v, wh = slot->ty + 2 * slot->v;
    if (ww * wh > fk::TRAIL_CELLS * fk::TRAIL_THREADS || (ww + 2) * (wh + 2) > fk::TRAIL_RING_MAX)
        return hipErrorInvalidValue;                          // a tile shape the kernel does not hold
    hipLaunchKernelGGL(fk::trail_kernel, dim3(n_tiles), dim3(fk::TRAIL_THREADS), 0, stream, *slot);
    return hipGetLastError();
}
