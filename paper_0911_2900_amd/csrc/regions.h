// regions.h -- region counts: the measurements behind a fundamental diagram.
//
// The paper picks v_m = 4 because the model then reproduces Weidmann's
// fundamental diagram (Sec. 2).  Such a diagram is measured from counts of
// agents: the number inside a measurement area gives the density, and the
// drop in the number upstream of a line gives the net flow across it (agents
// only move, so a closed upstream end loses agents only over the line).
// After every motion phase the count kernel stores, for each rectangle of a
// scenario, the number of agents on its cells as row `step` of a series,
// `step` being the scenario's completed steps.
#pragma once
#include <stdint.h>

namespace fk {

constexpr int MAX_REGIONS = 8;
constexpr int COUNT_THREADS = 256;

struct RegionDev {
    const int32_t *occ;              // the scenario's padded occupancy grid (agent id or -1)
    const int32_t *ctr;              // its counters (steps completed at C_STEP)
    int32_t *series;                 // rows * n: agents per rectangle when the step counter was k
    int32_t Wp, pad, n, rows;        // padded width, border, rectangles, rows of `series`
    int32_t rect[MAX_REGIONS * 4];   // x0, y0, x1, y1 in grid cells, half-open
};

}  // namespace fk
