// fast_host.h -- host-side pieces of libfast shared by builder.cpp and
// runtime.cpp: the built scenario and the kernel launchers (plan_batch.hip,
// plan_one.hip, motion.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fast.h"
#include "fast_dev.h"
#include "regions.h"

namespace fh {

// A scenario laid out for the device (see fast_dev.h for the layout).
struct Built {
    int W = 0, H = 0, v = 0, pad = 0, tx = 0, ty = 0, ntx = 0, nty = 0, Wp = 0, Hp = 0;
    std::vector<uint8_t> type;     // padded
    std::vector<float> G;          // padded exp table
    std::vector<double> S;         // padded floor field
    std::vector<int32_t> tile_m;   // (ntx+2)*(nty+2)
    std::vector<uint8_t> tile_fb;  // ntx*nty
    std::vector<int32_t> occ;      // padded
    std::vector<int32_t> pos;      // padded cell per agent
    std::vector<uint8_t> vi;       // per-agent speeds (empty: every agent has v)
    std::vector<uint8_t> fi;       // per-agent floor field (empty: one field for all)
    std::vector<double> Sf;        // padded floor fields of the exit groups, one after another
    std::vector<float> Gf;         // their exp tables, one after another (several fields only)
    std::vector<int32_t> tile_mf;  // their tile scales, (ntx+2)*(nty+2) each
    std::vector<uint8_t> tile_fbf; // their fallback flags, ntx*nty each
    int n = 0;
    int n_fb = 0;
    int n_fbf = 0;                 // fallback (tile, field) pairs
    float eps = 0.0f;
};

void floor_field(int W, int H, std::vector<uint8_t> &type, std::vector<double> &S,
                 const uint8_t *exit_field = nullptr, int g = 0);
bool place(int W, int H, const std::vector<uint8_t> &type, int n, uint64_t seed, uint32_t scn,
           std::vector<int32_t> &xy);
float guard_band(int v);
// The device cell bytes of a built scenario (fk::cut_bit).
std::vector<uint8_t> cell_bytes(const Built &b);
int build_scenario(const fast_scenario_desc &d, int tx, int ty, Built &b, std::string &err);

}  // namespace fh

namespace fk {
// Bytes of the static work-item scratch (scratch.hip) of the allocation-free
// batched run: 1 MiB per GPU.
constexpr size_t SCRATCH_BYTES = (size_t)1 << 20;
}  // namespace fk

// Batched planning: v, tx = the v_max and tile width shared by every item's
// scenario (the specialised kernels), or 0, 0 for a mixed batch.
extern "C" hipError_t fk_launch_plan(const fk::SlotDev *table, const uint32_t *items, int n_items,
                                     int v, int tx, hipStream_t stream, hipEvent_t start,
                                     hipEvent_t stop);
// plan_fixed.hip, one object per v_max.
#define FK_FIXED_LAUNCHERS(V)                                                                     \
    extern "C" hipError_t fk_launch_plan_fixed_v##V(int tx, const fk::SlotDev *table,              \
                                                    const uint32_t *items, int n_items,            \
                                                    hipStream_t stream, hipEvent_t start,          \
                                                    hipEvent_t stop);                              \
    extern "C" hipError_t fk_launch_plan_one_fixed_v##V(const fk::SlotDev *slot, int n_tiles,      \
                                                        hipStream_t stream, hipEvent_t start,      \
                                                        hipEvent_t stop);                          \
    extern "C" hipError_t fk_launch_plan_het_v##V(const fk::SlotDev *slot, const fk::HetDev *h,    \
                                                  int n_tiles, int debug, hipStream_t stream,      \
                                                  hipEvent_t start, hipEvent_t stop);
FK_FIXED_LAUNCHERS(1)
FK_FIXED_LAUNCHERS(2)
FK_FIXED_LAUNCHERS(3)
FK_FIXED_LAUNCHERS(4)
FK_FIXED_LAUNCHERS(5)
#undef FK_FIXED_LAUNCHERS
extern "C" hipError_t fk_launch_plan_one(const fk::SlotDev *slot, int n_tiles, int debug,
                                         hipStream_t stream, hipEvent_t start, hipEvent_t stop);
extern "C" hipError_t fk_launch_move(const fk::SlotDev *table, const uint32_t *mitems, int n_items,
                                     hipStream_t stream);
extern "C" hipError_t fk_move_per_cu(int *per_cu);
extern "C" hipError_t fk_cu_probe(hipStream_t stream, int n_wg, uint32_t *ids_host);
extern "C" hipError_t fk_launch_plan_het(const fk::SlotDev *slot, const fk::HetDev *h, int n_tiles,
                                         int debug, hipStream_t stream, hipEvent_t start,
                                         hipEvent_t stop);
extern "C" hipError_t fk_launch_count(const fk::RegionDev *jobs, int n_jobs, int max_regions,
                                      hipStream_t stream);
extern "C" hipError_t fk_scratch_ptr(int device, void **out);
extern "C" hipError_t fk_launch_trail(const fk::SlotDev *slot, int n_tiles, hipStream_t stream);
extern "C" hipError_t fk_launch_stream(float4 *base, size_t n4, hipStream_t stream,
                                       hipEvent_t start, hipEvent_t stop);
