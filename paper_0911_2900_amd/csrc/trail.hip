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
// Two launches follow each motion phase of a scenario with a trail field:
// the update of T, then the exp table the next planning phase reads, rebuilt
// with the trail term (G(t) = fl32(exp(m_T ln 2 - k_S S(t) + k_D T(t)))),
// with every tile's range-fallback flag taken afresh.  The trail of step s
// lives in buffer s & 1, so both launches only read the counters and can run
// again with the same result (a served scenario past its last step skips its
// motion phase but not these launches).
#include <hip/hip_runtime.h>

#include "fast_dev.h"

namespace fk {

constexpr int TRAIL_THREADS = 256;
constexpr double LN2_64 = 0x1.62e42fefa39efp-1;   // nearest double to ln 2
constexpr double RANGE = 80.0;                    // |exponent| bound of a table entry

// T of step C_STEP from T of step C_STEP - 1 and the deposits of the motion
// phase in between.  The padded border is wall, so every non-wall cell has
// its 8 neighbours inside the padded grid; off-grid and wall neighbours hold
// 0, and adding 0 leaves the sum unchanged bit for bit.
__global__ __launch_bounds__(TRAIL_THREADS) void trail_update_kernel(const SlotDev s)
{
    const int stp = s.ctr[C_STEP];
    if (stp <= 0) return;                                     // no motion phase yet
    const long cells = (long)s.Wp * s.Hp;
    const double *__restrict__ To = s.Tr + (long)((stp - 1) & 1) * cells;
    double *__restrict__ Tn = s.Tr + (long)(stp & 1) * cells;
    const double keep = 1.0 - s.t_decay, stay = 1.0 - s.t_diff, share = s.t_diff / 8.0;
    const int Wp = s.Wp;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
         i += (long)gridDim.x * blockDim.x) {
        if ((s.cell[i] & CELL_TYPE_MASK) == CELL_WALL) {
            Tn[i] = 0.0;
            continue;
        }
        double nb = 0.0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                if (dx || dy) nb = nb + To[i + dy * Wp + dx];
        Tn[i] = keep * (stay * To[i] + share * nb) + (double)s.dep[i];
    }
}

// The exp table of one tile with the trail term, in the tile's own scale
// (the occupancy bit of D kept), and the tile's fallback flag: set when a
// window cell's exponent, in this tile's scale or in its own tile's, lies
// outside [-80, 80] (the rule the scenario's setup applies with T = 0).
__global__ __launch_bounds__(TRAIL_THREADS) void trail_table_kernel(const SlotDev s)
{
    __shared__ int out_of_range;
    const int tile = (int)blockIdx.x;
    const int stp = s.ctr[C_STEP];
    const long cells = (long)s.Wp * s.Hp;
    const double *__restrict__ T = s.Tr + (long)(stp & 1) * cells;
    const int ty0 = tile / s.ntx, tx0 = tile - ty0 * s.ntx;
    const int ts = s.ntx + 2;
    const int mT = s.tile_m[(ty0 + 1) * ts + tx0 + 1];
    const double ks = s.k_s, kd = s.k_d;
    if (threadIdx.x == 0) out_of_range = 0;
    __syncthreads();
    // the tile's own cells
    for (int k = threadIdx.x; k < s.tx * s.ty; k += blockDim.x) {
        const int ly = k / s.tx, lx = k - ly * s.tx;
        const long t = (long)(ty0 * s.ty + s.pad + ly) * s.Wp + tx0 * s.tx + s.pad + lx;
        const double St = s.S[t];
        if (!(St < INFINITY)) continue;                        // wall: the entry stays 0
        const double e = (double)mT * LN2_64 - ks * St + kd * T[t];
        const float g = fabs(e) > RANGE ? 0.0f : (float)exp(e);
        s.D[t] = __float_as_uint(g) | (s.D[t] & D_OCC);
    }
    // the window: this tile grown by v on every side
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
        const double rest = -ks * St + kd * T[t];
        const double eT = (double)mT * LN2_64 + rest, eO = (double)mo * LN2_64 + rest;
        bad |= (fabs(eT) > RANGE || fabs(eO) > RANGE) ? 1 : 0;
    }
    if (bad) out_of_range = 1;
    __syncthreads();
    if (threadIdx.x == 0) s.tile_fb[tile] = out_of_range ? 1 : 0;
}

}  // namespace fk

// The two launches that close a motion phase of a scenario with a trail field.
extern "C" hipError_t fk_launch_trail(const fk::SlotDev *slot, int n_tiles, hipStream_t stream)
{
    if (!slot->Tr || n_tiles <= 0) return hipSuccess;
    const long cells = (long)slot->Wp * slot->Hp;
    long blocks = (cells + fk::TRAIL_THREADS - 1) / fk::TRAIL_THREADS;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fk::trail_update_kernel, dim3((unsigned)blocks), dim3(fk::TRAIL_THREADS), 0,
                       stream, *slot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fk::trail_table_kernel, dim3(n_tiles), dim3(fk::TRAIL_THREADS), 0, stream,
                       *slot);
    return hipGetLastError();
}
