// runtime.cpp -- libfast's host runtime and C-ABI (include/fast.h): contexts,
// scenario slots in HBM, single-scenario plan / move launches, batched runs
// replayed from captured HIP graphs, and the continuous-batching server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fast_dev.h"
#include "fast_host.h"

namespace {

thread_local std::string g_err = "no error";

fast_status fail(fast_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FAST_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Slot {
    bool live = false;
    fk::SlotDev dev{};           // host copy of the device descriptor
    void *block = nullptr;       // one allocation holding all of the slot's buffers
    size_t bytes = 0;
    uint32_t *items = nullptr;   // device: plan work items of this slot alone
    int32_t *self = nullptr;     // device: [slot index]
    uint32_t *mitems = nullptr;  // device: motion work items of this slot alone
    int n_items = 0;
    int group = 1;               // motion workgroups when stepped alone
    int n_fb_tiles = 0;
    int host_steps = 0;          // steps launched (== device step once the stream drains)
    bool planned = false;        // a plan was launched after the last motion phase
    int n_agents = 0;
    fk::HetDev hd{};             // device: per-agent speeds and several fields (plan_het.hip)
    bool het = false;            // planned by the per-agent kernel (speeds or fields)
    // region counts (fast_set_regions)
    fk::RegionDev rhost{};       // host copy of the job
    fk::RegionDev *rdev = nullptr;  // device: the job, then its series
    size_t rbytes = 0;
    int n_regions = 0;
};

// Time steps a batch's long graph captures: a graph launch costs about 8 us
// between one step's motion launch and the next step's planning launch, so
// runs of many steps replay GRAPH_STEPS steps per launch.
constexpr int GRAPH_STEPS = 8;

struct Batch {
    hipGraphExec_t exec = nullptr;       // one step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec_k = nullptr;     // GRAPH_STEPS steps
    hipGraph_t graph_k = nullptr;
    uint32_t *items = nullptr;
    uint32_t *mitems = nullptr;
    int32_t *slots = nullptr;
    int n_items = 0, n_mitems = 0, n_slots = 0;
    int v = 0, tx = 0;           // v_max and tile width shared by all members, else 0
    fk::RegionDev *rjobs = nullptr;  // device: region-count jobs of the members that have them
    int n_rjobs = 0, max_regions = 0;
    std::vector<int32_t> het;        // members with per-agent speeds: a planning launch each
    std::vector<int32_t> trails;     // members with a trail field: its update after motion
    void *block = nullptr;
    size_t bytes = 0;
    std::vector<int32_t> members;
};

// The work items of a batch, built on the host: the planning launch's tile
// items (the larger scenarios first, so their tiles start early on the
// hardware queue; members with per-agent speeds are planned by launches of
// their own), the motion launch's workgroup items, and the region-count jobs.
struct BatchItems {
    std::vector<int32_t> order;
    std::vector<uint32_t> items, mitems;
    std::vector<int32_t> het;
    std::vector<int32_t> trails;     // members with a trail field: its launches after motion
    std::vector<fk::RegionDev> rj;
    int v = 0, tx = 0, max_regions = 0;
};

struct Request {
    uint64_t ticket = 0;
    fast_scenario_desc desc{};
    std::vector<uint8_t> cells;
    std::vector<int32_t> xy;
    std::vector<uint8_t> vi;         // per-agent speeds (desc.agent_v points here)
    std::vector<uint8_t> ef, fi;     // exit groups and per-agent fields (desc points here)
    int steps = 0;
    double t_submit = 0, t_done = 0;
    int state = 0;               // 0 queued, 1 running, 2 done, -1 rejected
    int built_state = 0;         // host build: 0 pending, 1 ready, -1 failed
    std::unique_ptr<fh::Built> built;
    int32_t handle = -1;
    std::vector<int32_t> out_xy;
    std::vector<uint8_t> out_alive;
    int32_t out_step = 0, out_active = 0;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct fast_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0, used = 0;
    fast_alloc_fn alloc = nullptr;
    fast_free_fn free_fn = nullptr;
    void *user = nullptr;
    fk::SlotDev *table = nullptr;    // device, FAST_MAX_SLOTS entries
    int n_cus = 0;                   // CUs the stream's launches reach
    int move_capacity = 0;           // motion workgroups those CUs hold at once
    std::vector<Slot> slots;
    std::map<std::vector<int32_t>, Batch> batches;
    std::vector<hipEvent_t> timing;  // kernel timing: start / stop pairs of plan launches
    int timing_used = 0;
    // allocation-free batched runs (fast_run_noalloc): the device address of
    // the library's static scratch on this context's device, a pinned host
    // staging buffer of the same size (set up here, at creation), the event
    // after which the staging buffer may be rewritten, and the item lists
    void *scratch = nullptr;
    void *stage = nullptr;
    hipEvent_t staged = nullptr;
    BatchItems nb;
    std::recursive_mutex mu;         // guards everything above

    // serving
    std::thread server;
    std::vector<std::thread> builders;
    std::mutex smu;
    std::condition_variable scv;     // server: a request is built, or stop
    std::condition_variable bcv;     // builders: a request is queued, or stop
    bool serving = false, stopping = false;
    size_t serve_budget = 0;
    int serve_max_active = 0;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> queue;       // admission order
    std::deque<uint64_t> build_queue; // awaiting their host build
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
};

namespace {

// The next start / stop event pair of kernel timing (none when it is off or full).
void next_timing_pair(fast_ctx *c, hipEvent_t *e0, hipEvent_t *e1)
{
    if (c->timing_used * 2 + 1 < (int)c->timing.size()) {
        *e0 = c->timing[c->timing_used * 2];
        *e1 = c->timing[c->timing_used * 2 + 1];
        ++c->timing_used;
    }
}

fast_status dev_alloc(fast_ctx *c, size_t bytes, void **out)
{
    bytes = align_up(std::max<size_t>(bytes, 256), 256);
    if (c->budget && c->used + bytes > c->budget)
        return fail(FAST_E_BUDGET, "device budget exceeded: %zu + %zu > %zu bytes", c->used, bytes,
                    c->budget);
    void *p = nullptr;
    if (c->alloc) {
        p = c->alloc(bytes, c->user);
        if (!p) return fail(FAST_E_NOMEM, "allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return fail(FAST_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    c->used += bytes;
    *out = p;
    return FAST_OK;
}

void dev_free(fast_ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    bytes = align_up(std::max<size_t>(bytes, 256), 256);
    if (c->free_fn) c->free_fn(p, c->user);
    else (void)hipFree(p);
    c->used -= std::min(c->used, bytes);
}

// Planning tile when the descriptor leaves it open: the largest tile that
// still gives the launch at least ~2 workgroups per compute unit on the grid,
// so that small scenarios fill the chip while large ones keep the halo
// (re-staged cells) small.
void choose_tile(int W, int H, int v, int *tx, int *ty)
{
    static const int cand[][2] = {{32, 32}, {32, 16}, {16, 16}, {16, 8}, {8, 8}};
    for (auto &c : cand) {
        const long tiles = (long)((W + c[0] - 1) / c[0]) * ((H + c[1] - 1) / c[1]);
        if (tiles >= 512) { *tx = c[0]; *ty = c[1]; return; }
    }
    (void)v;
    *tx = 8;
    *ty = 8;
}

bool valid_tile_dim(int t) { return t == 8 || t == 16 || t == 32 || t == 64; }

// Motion workgroups for a scenario of n agents: one per MOVE_AGENTS_PER_WG
// agents, at most MOVE_GROUP_MAX.
int motion_group(int n)
{
    const int g = (n + fk::MOVE_AGENTS_PER_WG - 1) / fk::MOVE_AGENTS_PER_WG;
    return std::max(1, std::min(g, fk::MOVE_GROUP_MAX));
}

// alone: the launch moves this scenario only (see move_kernel).
uint32_t motion_item(int32_t slot, int g, int G, bool alone = false)
{
    return (uint32_t)slot | ((uint32_t)g << 12) | ((uint32_t)(G - 1) << 22) | (alone ? 1u << 31 : 0u);
}

// Group sizes for a batch.  Every workgroup of the motion launch must be
// resident at once (group barriers), so the sizes share the device's
// capacity: every scenario gets one workgroup, and the rest go one at a time
// to the scenario whose motion phase is expected to take longest -- agents
// per workgroup times v_max, since a longer reach makes longer chains of
// reservation rounds -- up to its own size alone.  A batch with more
// scenarios than the capacity runs one workgroup each (those need no group
// barrier).
std::vector<int> batch_groups(const fast_ctx *c, const std::vector<int32_t> &hs)
{
    std::vector<int> G(hs.size(), 1);
    long total = (long)hs.size();
    const long cap = std::max(1, c->move_capacity);
    using Item = std::pair<double, size_t>;          // (expected cost per workgroup, index)
    std::priority_queue<Item> q;
    auto cost = [&](size_t i, int g) {
        const Slot &s = c->slots[hs[i]];
        return (double)s.n_agents * s.dev.v / g;
    };
    for (size_t i = 0; i < hs.size(); ++i)
        if (motion_group(c->slots[hs[i]].n_agents) > 1) q.push({cost(i, 1), i});
    while (total < cap && !q.empty()) {
        const size_t i = q.top().second;
        q.pop();
        ++G[i];
        ++total;
        if (G[i] < motion_group(c->slots[hs[i]].n_agents)) q.push({cost(i, G[i]), i});
    }
    return G;
}

// Distinct CUs one probe launch of n_wg workgroups occupies on `s`, and how
// many of them lie on each of the XCDs 0..7 (per_xcd may be NULL).
hipError_t probe_cus(hipStream_t s, int n_wg, int *seen, int32_t *per_xcd)
{
    n_wg = std::max(1, std::min(n_wg, 4096));
    std::vector<uint32_t> ids((size_t)n_wg);
    const hipError_t e = fk_cu_probe(s, n_wg, ids.data());
    if (e != hipSuccess) return e;
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    *seen = (int)ids.size();
    if (per_xcd) {
        std::fill(per_xcd, per_xcd + 8, 0);
        for (uint32_t id : ids)
            if ((id >> 8) < 8) ++per_xcd[id >> 8];
    }
    return hipSuccess;
}

// CUs that launches on `s` can fill with co-resident workgroups: the whole
// device unless the stream carries a CU mask with fewer bits (or its mask
// cannot be read).  Then a probe launch counts the CUs it reaches on each XCD;
// a dispatch hands its workgroups to the eight XCDs in turn, so the count is
// eight times the fewest on any XCD (at most the mask's bits, at least 1),
// and the motion phase never plans on more resident workgroups than that.
hipError_t stream_cus(hipStream_t s, int device, int *n_cus)
{
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    int bits = 0;
    if (hipExtStreamGetCUMask(s, (uint32_t)mask.size(), mask.data()) == hipSuccess)
        for (uint32_t w : mask) bits += __builtin_popcount(w);
    else
        (void)hipGetLastError();
    const bool known = bits > 0;
    if (known && bits >= cus) {
        *n_cus = cus;
        return hipSuccess;
    }
    int seen = 0;
    int32_t per_xcd[8];
    e = probe_cus(s, 4 * (known ? bits : cus), &seen, per_xcd);
    if (e != hipSuccess) return e;
    const int fewest = *std::min_element(per_xcd, per_xcd + 8);
    *n_cus = std::max(1, std::min(known ? bits : cus, 8 * fewest));
    return hipSuccess;
}

// The scenario keeps a trail field (the dynamic floor field of fast.h).
bool has_trail(const fast_scenario_desc *d)
{
    return d->k_d != 0.0 || d->trail_decay != 0.0 || d->trail_diffusion != 0.0;
}

fast_status check_desc(const fast_scenario_desc *d)
{
    if (!d) return fail(FAST_E_INVALID, "descriptor is NULL");
    if (d->width < 3 || d->height < 3 || d->width > 16384 || d->height > 16384)
        return fail(FAST_E_INVALID, "grid %dx%d outside 3..16384", d->width, d->height);
    if (!d->cell_type) return fail(FAST_E_INVALID, "cell_type is NULL");
    if (d->v_max < 1 || d->v_max > fk::MAX_V)
        return fail(FAST_E_INVALID, "v_max %d outside 1..5", d->v_max);
    if (!(d->k_s >= 0.0) || !std::isfinite(d->k_s))
        return fail(FAST_E_INVALID, "k_s must be finite and >= 0");
    if (!(d->k_d >= 0.0) || !std::isfinite(d->k_d))
        return fail(FAST_E_INVALID, "k_d must be finite and >= 0");
    if (!(d->trail_decay >= 0.0 && d->trail_decay <= 1.0) ||
        !(d->trail_diffusion >= 0.0 && d->trail_diffusion <= 1.0))
        return fail(FAST_E_INVALID, "trail_decay and trail_diffusion must lie in 0..1");
    if (has_trail(d) && d->n_fields >= 2)
        return fail(FAST_E_INVALID, "a trail field (k_d, trail_decay, trail_diffusion) does not "
                    "combine with several floor fields");
    if (d->n_agents < 0 || d->n_agents > FAST_MAX_AGENTS)
        return fail(FAST_E_INVALID, "n_agents %d outside 0..%d", d->n_agents, FAST_MAX_AGENTS);
    if (d->tile_w || d->tile_h) {
        if (!valid_tile_dim(d->tile_w) || !valid_tile_dim(d->tile_h) || d->tile_w * d->tile_h > 1024)
            return fail(FAST_E_INVALID, "tile %dx%d: powers of two in 8..64, at most 1024 cells",
                        d->tile_w, d->tile_h);
    }
    return FAST_OK;
}

Slot *get_slot(fast_ctx *c, int32_t h)
{
    if (h < 0 || h >= (int32_t)c->slots.size() || !c->slots[h].live) return nullptr;
    return &c->slots[h];
}

void drop_batches_with(fast_ctx *c, int32_t h)
{
    for (auto it = c->batches.begin(); it != c->batches.end();) {
        if (std::find(it->first.begin(), it->first.end(), h) != it->first.end()) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
            if (it->second.exec_k) (void)hipGraphExecDestroy(it->second.exec_k);
            if (it->second.graph_k) (void)hipGraphDestroy(it->second.graph_k);
            dev_free(c, it->second.block, it->second.bytes);
            it = c->batches.erase(it);
        } else {
            ++it;
        }
    }
}

// Builds a scenario into a free slot; `limit` is the step at which its kernels
// stop acting (INT_MAX for scenarios stepped by the caller).
// Host half of scenario setup: floor field, placement, exp table and tile
// metadata.  Touches no device state, so the server runs it on builder threads.
fast_status build_host(const fast_scenario_desc *d, fh::Built &b)
{
    fast_status st = check_desc(d);
    if (st) return st;
    int tx = d->tile_w, ty = d->tile_h;
    if (!tx) choose_tile(d->width, d->height, d->v_max, &tx, &ty);
    std::string err;
    st = fh::build_scenario(*d, tx, ty, b, err);
    if (st) return fail(st, "%s", err.c_str());
    return FAST_OK;
}

// Device half: one allocation for the slot, upload, descriptor table entry.
fast_status upload_slot(fast_ctx *c, const fast_scenario_desc *d, const fh::Built &b, int limit,
                        int32_t *handle)
{
    fast_status st = FAST_OK;
    int32_t h = -1;
    for (int32_t i = 0; i < (int32_t)c->slots.size(); ++i)
        if (!c->slots[i].live) { h = i; break; }
    if (h < 0) {
        if ((int)c->slots.size() >= FAST_MAX_SLOTS)
            return fail(FAST_E_STATE, "all %d scenario slots are in use", FAST_MAX_SLOTS);
        c->slots.emplace_back();
        h = (int32_t)c->slots.size() - 1;
    }

    const size_t cells = (size_t)b.Wp * b.Hp;
    const size_t ntiles = (size_t)b.ntx * b.nty;
    const size_t tcells = ntiles * (size_t)b.tx * b.ty;   // record capacity
    // mover lists: the G motion workgroups' lists take at most
    // tiles + 2 MOVE_GROUP_MAX tiles' worth
    const size_t lcells = (ntiles + 2 * fk::MOVE_GROUP_MAX) * (size_t)b.tx * b.ty;
    const size_t tm = (size_t)(b.ntx + 2) * (b.nty + 2);
    // carve one block: 256-byte aligned sub-buffers
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_S = take(cells * 8), o_res = take(cells * 16), o_D = take(cells * 4),
                 o_occ = take(cells * 4), o_type = take(cells), o_tm = take(tm * 4),
                 o_fb = take(ntiles), o_scnt = take(ntiles * 4),
                 o_seg = take(tcells * 4), o_ka = take(lcells * sizeof(fk::Mover)),
                 o_kb = take(lcells * sizeof(fk::Mover)), o_ctr = take(fk::C_NCTR * 4),
                 o_stat = take(fk::S_NSTAT * 8), o_items = take(ntiles * 4), o_self = take(4),
                 o_mitems = take(fk::MOVE_GROUP_MAX * 4),
                 // every motion group of this scenario has at most motion_group(n)
                 // workgroups, each handing over at most MOVE_SOLO_MAX movers
                 o_hand = take((size_t)motion_group(b.n) * fk::MOVE_SOLO_MAX * sizeof(fk::Mover)),
                 o_vi = take(b.vi.size()), o_fi = take(b.fi.size()),
                 o_Sf = take(b.Sf.size() * 8), o_Gf = take(b.Gf.size() * 4),
                 o_tmf = take(b.tile_mf.size() * 4), o_fbf = take(b.tile_fbf.size());
    const bool trail = has_trail(d);
    const size_t o_Tr = take(trail ? cells * 16 : 0), o_dep = take(trail ? cells * 4 : 0);
    void *block = nullptr;
    st = dev_alloc(c, off, &block);
    if (st) return st;
    char *base = (char *)block;

    fk::SlotDev sd{};
    sd.W = b.W; sd.H = b.H; sd.Wp = b.Wp; sd.Hp = b.Hp; sd.v = b.v; sd.pad = b.pad;
    sd.tx = b.tx; sd.ty = b.ty; sd.ntx = b.ntx; sd.nty = b.nty; sd.n_agents = b.n;
    sd.seed_lo = (uint32_t)d->seed; sd.seed_hi = (uint32_t)(d->seed >> 32);
    sd.scn = d->scenario_id; sd.eps = b.eps; sd.k_s = d->k_s;
    // FAST_FP64_SEQUENTIAL=1 (read when the scenario is set up) sends every
    // FP64 re-resolve through the sequential sum, so tests can cover it
    const char *seq = std::getenv("FAST_FP64_SEQUENTIAL");
    sd.near64 = (seq && seq[0] == '1') ? 1e300 : 1e-12;
    sd.S = (const double *)(base + o_S);
    sd.res0 = (unsigned long long *)(base + o_res);
    sd.res1 = (unsigned long long *)(base + o_res + cells * 8);

    sd.D = (uint32_t *)(base + o_D);
    sd.occ = (int32_t *)(base + o_occ);
    sd.cell = (const uint8_t *)(base + o_type);
    sd.tile_m = (const int32_t *)(base + o_tm);
    sd.tile_fb = (uint8_t *)(base + o_fb);
    if (trail) {
        sd.Tr = (double *)(base + o_Tr);
        sd.dep = (int32_t *)(base + o_dep);
        sd.k_d = d->k_d;
        sd.t_decay = d->trail_decay;
        sd.t_diff = d->trail_diffusion;
    }
    sd.seg_cnt = (int32_t *)(base + o_scnt);
    sd.seg = (uint32_t *)(base + o_seg);
    sd.mv_a = (fk::Mover *)(base + o_ka);
    sd.mv_b = (fk::Mover *)(base + o_kb);
    sd.hand = (fk::Mover *)(base + o_hand);
    sd.ctr = (int32_t *)(base + o_ctr);
    sd.stat = (unsigned long long *)(base + o_stat);

    std::vector<int32_t> ctr(fk::C_NCTR, 0);
    ctr[fk::C_NACTIVE] = b.n;
    ctr[fk::C_LIMIT] = limit;
    std::vector<uint32_t> items(ntiles);
    for (size_t i = 0; i < ntiles; ++i) items[i] = ((uint32_t)h << 20) | (uint32_t)i;
    const int32_t self = h;
    int group = motion_group(b.n);
    const int half = std::max(1, c->move_capacity / 2);
    if (group > half) group = half;
    std::vector<uint32_t> mitems((size_t)group);
    for (int g = 0; g < group; ++g) mitems[g] = motion_item(h, g, group, true);

    hipError_t e = hipSuccess;
    auto cp = [&](size_t o, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
    };
    cp(o_S, b.S.data(), cells * 8);
    if (e == hipSuccess) e = hipMemset(base + o_res, 0, cells * 16);
    // D: each cell's table entry, bit 31 set under an agent
    std::vector<uint32_t> dtab(cells);
    for (size_t g = 0; g < cells; ++g) {
        uint32_t bits;
        std::memcpy(&bits, &b.G[g], 4);
        dtab[g] = bits | (b.occ[g] >= 0 ? fk::D_OCC : 0u);
    }
    cp(o_D, dtab.data(), cells * 4);
    cp(o_occ, b.occ.data(), cells * 4);
    const std::vector<uint8_t> cellb = fh::cell_bytes(b);
    cp(o_type, cellb.data(), cells);
    cp(o_tm, b.tile_m.data(), tm * 4);
    cp(o_fb, b.tile_fb.data(), ntiles);
    if (e == hipSuccess) e = hipMemset(base + o_scnt, 0, ntiles * 4);   // nothing planned yet
    cp(o_ctr, ctr.data(), fk::C_NCTR * 4);
    if (e == hipSuccess) e = hipMemset(base + o_stat, 0, fk::S_NSTAT * 8);
    cp(o_items, items.data(), ntiles * 4);
    cp(o_self, &self, 4);
    cp(o_mitems, mitems.data(), mitems.size() * 4);
    cp(o_vi, b.vi.data(), b.vi.size());
    cp(o_fi, b.fi.data(), b.fi.size());
    cp(o_Sf, b.Sf.data(), b.Sf.size() * 8);
    cp(o_Gf, b.Gf.data(), b.Gf.size() * 4);
    cp(o_tmf, b.tile_mf.data(), b.tile_mf.size() * 4);
    cp(o_fbf, b.tile_fbf.data(), b.tile_fbf.size());
    if (trail && e == hipSuccess) e = hipMemset(base + o_Tr, 0, cells * 16);   // T of steps 0 and 1
    if (trail && e == hipSuccess) e = hipMemset(base + o_dep, 0, cells * 4);
    if (e == hipSuccess) e = hipMemcpy(c->table + h, &sd, sizeof sd, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(c, block, off);
        return fail(FAST_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }

    Slot &s = c->slots[h];
    s = Slot();
    s.live = true;
    s.dev = sd;
    s.block = block;
    s.bytes = off;
    s.items = (uint32_t *)(base + o_items);
    s.self = (int32_t *)(base + o_self);
    s.mitems = (uint32_t *)(base + o_mitems);
    s.group = group;
    s.n_items = (int)ntiles;
    s.n_fb_tiles = b.Gf.empty() ? b.n_fb : b.n_fbf;   // several fields: (tile, field) pairs
    s.n_agents = b.n;
    s.hd.vi = b.vi.empty() ? nullptr : (const uint8_t *)(base + o_vi);
    s.hd.fi = b.fi.empty() ? nullptr : (const uint8_t *)(base + o_fi);
    s.hd.Sf = b.Sf.empty() ? nullptr : (const double *)(base + o_Sf);
    s.hd.Gf = b.Gf.empty() ? nullptr : (const uint32_t *)(base + o_Gf);
    s.hd.tile_mf = b.tile_mf.empty() ? nullptr : (const int32_t *)(base + o_tmf);
    s.hd.tile_fbf = b.tile_fbf.empty() ? nullptr : (const uint8_t *)(base + o_fbf);
    s.hd.field_cells = (long)cells;
    s.hd.nf = s.hd.Gf ? (int)(b.Sf.size() / cells) : 1;
    s.het = s.hd.vi || s.hd.Gf;
    *handle = h;
    return FAST_OK;
}

fast_status init_slot(fast_ctx *c, const fast_scenario_desc *d, int limit, int32_t *handle)
{
    fh::Built b;
    fast_status st = build_host(d, b);
    if (st) return st;
    return upload_slot(c, d, b, limit, handle);
}

fast_status destroy_slot(fast_ctx *c, int32_t h)
{
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    HIP_TRY(hipStreamSynchronize(c->stream));
    drop_batches_with(c, h);
    dev_free(c, s->rdev, s->rbytes);
    dev_free(c, s->block, s->bytes);
    *s = Slot();
    return FAST_OK;
}

// Per-agent state rebuilt from the occupancy grid (positions) and the tiles'
// records of the last plan (chosen cells).
fast_status read_state(fast_ctx *c, Slot *s, int32_t *xy, uint8_t *alive, int32_t *desired,
                       int32_t *step, int32_t *n_active)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    const fk::SlotDev &d = s->dev;
    const int n = s->n_agents;
    std::vector<int32_t> ctr(fk::C_NCTR);
    HIP_TRY(hipMemcpy(ctr.data(), d.ctr, fk::C_NCTR * 4, hipMemcpyDeviceToHost));
    if (ctr[fk::C_ERR])
        return fail(FAST_E_DEVICE, "a motion-phase group barrier timed out: the scenario state is invalid");
    if (step) *step = ctr[fk::C_STEP];
    if (n_active) *n_active = ctr[fk::C_NACTIVE];
    if (!xy && !alive && !desired) return FAST_OK;
    const size_t cells = (size_t)d.Wp * d.Hp;
    std::vector<int32_t> occ(cells), pos((size_t)std::max(n, 1), -1);
    HIP_TRY(hipMemcpy(occ.data(), d.occ, cells * 4, hipMemcpyDeviceToHost));
    for (size_t g = 0; g < cells; ++g)
        if (occ[g] >= 0 && occ[g] < n) pos[occ[g]] = (int32_t)g;
    const int Wp = d.Wp, pad = d.pad, W = d.W;
    // desired cells: the records of the last plan, while its motion phase has
    // not run (the record's agent is the occupant of its start cell until then)
    std::vector<int32_t> tgt;
    if (desired) {
        tgt.assign((size_t)std::max(n, 1), -1);
        if (s->planned) {
            const size_t ntiles = (size_t)d.ntx * d.nty, tc = (size_t)d.tx * d.ty;
            const int side = 2 * d.v + 1;
            std::vector<int32_t> cnt(ntiles);
            std::vector<uint32_t> rec(ntiles * tc);
            HIP_TRY(hipMemcpy(cnt.data(), d.seg_cnt, ntiles * 4, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(rec.data(), d.seg, rec.size() * 4, hipMemcpyDeviceToHost));
            for (size_t t = 0; t < ntiles; ++t) {
                const int tyy = (int)(t / d.ntx), txx = (int)(t % d.ntx);
                for (int k = 0; k < cnt[t]; ++k) {
                    const uint32_t r = rec[t * tc + k];
                    const int lc = (int)(r & ((1u << fk::REC_SLOT_SHIFT) - 1u));
                    const int slot = (int)(r >> fk::REC_SLOT_SHIFT);
                    const int cx = txx * d.tx + d.pad + lc % d.tx, cy = tyy * d.ty + d.pad + lc / d.tx;
                    const int g = cy * Wp + cx;
                    const int id = occ[(size_t)g];
                    if (id < 0 || id >= n) continue;
                    tgt[id] = g + (slot / side - d.v) * Wp + (slot % side - d.v);
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        const int p = pos[i];
        if (xy) {
            xy[2 * i] = p < 0 ? -1 : p % Wp - pad;
            xy[2 * i + 1] = p < 0 ? -1 : p / Wp - pad;
        }
        if (alive) alive[i] = p >= 0 ? 1 : 0;
        if (desired) {
            const int q = tgt[i];
            desired[i] = (p < 0 || q < 0) ? -1 : (q / Wp - pad) * W + (q % Wp - pad);
        }
    }
    return FAST_OK;
}

fast_status batch_items(fast_ctx *c, const std::vector<int32_t> &hs, BatchItems &p)
{
    for (int32_t h : hs)                              // items carry a 20-bit tile index
        if (c->slots[h].n_items > (1 << 20))
            return fail(FAST_E_INVALID, "scenario %d has %d tiles; batched launches take at most 2^20 "
                        "per scenario (choose a larger tile)", h, c->slots[h].n_items);
    p.order.assign(hs.begin(), hs.end());
    std::stable_sort(p.order.begin(), p.order.end(), [&](int32_t a, int32_t b) {
        return c->slots[a].n_agents > c->slots[b].n_agents;
    });
    p.het.clear();
    p.trails.clear();
    for (int32_t h : p.order)
        if (c->slots[h].dev.Tr) p.trails.push_back(h);
    p.v = p.tx = 0;
    bool first = true;
    for (int32_t h : p.order) {
        const Slot &s = c->slots[h];
        if (s.het) { p.het.push_back(h); continue; }
        if (first) { p.v = s.dev.v; p.tx = s.dev.tx; first = false; }
        else if (s.dev.v != p.v || s.dev.tx != p.tx) p.v = p.tx = 0;
    }
    // Planning items in an order that keeps neighbouring tiles on one XCD.
    // A dispatch hands its workgroups to the XCDs in turn (workgroup i to
    // XCD i mod 8), and each XCD has an L2 of its own.  Each scenario's
    // tiles, in raster order, are cut into 8 runs of (nearly) equal length;
    // run r goes to XCD (r + q) mod 8, q the scenario's place in the batch
    // (which spreads small scenarios over the XCDs).  So every XCD plans
    // bands of neighbouring tiles one after another, and the window rows
    // they share come from its L2.  Lists of unequal length are padded with
    // empty items.  Scenarios with the larger v_max come first (a tile's
    // draws cost more the larger the reach), so the launch ends on cheap
    // tiles; in the 256-scenario ensemble this took about 1 us off a
    // planning launch against the order by agent count, and the reverse
    // order added as much.
    std::vector<uint32_t> per[fk::DIES];
    int q = 0;
    std::vector<int32_t> porder(p.order);
    std::stable_sort(porder.begin(), porder.end(), [&](int32_t a, int32_t b) {
        return c->slots[a].dev.v > c->slots[b].dev.v;
    });
    for (int32_t h : porder) {
        const Slot &s = c->slots[h];
        if (s.het) continue;
        const int T = s.n_items;
        for (int r = 0; r < fk::DIES; ++r) {
            auto &l = per[(r + q) % fk::DIES];
            for (int i = (int)((long)T * r / fk::DIES); i < (int)((long)T * (r + 1) / fk::DIES); ++i)
                l.push_back(((uint32_t)h << 20) | (uint32_t)i);
        }
        ++q;
    }
    size_t longest = 0;
    for (const auto &l : per) longest = std::max(longest, l.size());
    p.items.clear();
    for (size_t j = 0; j < longest; ++j)
        for (int x = 0; x < fk::DIES; ++x)
            p.items.push_back(j < per[x].size() ? per[x][j] : fk::PLAN_ITEM_NONE);
    while (!p.items.empty() && p.items.back() == fk::PLAN_ITEM_NONE) p.items.pop_back();
    const std::vector<int> G = batch_groups(c, p.order);
    p.mitems.clear();
    for (size_t i = 0; i < p.order.size(); ++i)
        for (int g = 0; g < G[i]; ++g)
            p.mitems.push_back(motion_item(p.order[i], g, G[i], p.order.size() == 1));
    p.rj.clear();
    p.max_regions = 0;
    for (int32_t h : p.order)
        if (c->slots[h].n_regions) {
            p.rj.push_back(c->slots[h].rhost);
            p.max_regions = std::max(p.max_regions, c->slots[h].n_regions);
        }
    return FAST_OK;
}

fast_status get_batch(fast_ctx *c, const std::vector<int32_t> &hs, Batch **out)
{
    auto it = c->batches.find(hs);
    if (it != c->batches.end()) { *out = &it->second; return FAST_OK; }
    BatchItems p;
    fast_status st = batch_items(c, hs, p);
    if (st) return st;
    const std::vector<int32_t> &order = p.order;
    const std::vector<uint32_t> &items = p.items, &mitems = p.mitems;
    const std::vector<fk::RegionDev> &rj = p.rj;
    Batch b;
    b.members = hs;
    b.het = p.het;
    b.trails = p.trails;
    b.v = p.v;
    b.tx = p.tx;
    b.max_regions = p.max_regions;
    const size_t ib = align_up(items.size() * 4, 256), mb = align_up(mitems.size() * 4, 256);
    const size_t ob = align_up(order.size() * 4, 256);
    b.bytes = ib + mb + ob + rj.size() * sizeof(fk::RegionDev);
    st = dev_alloc(c, b.bytes, &b.block);
    if (st) return st;
    b.items = (uint32_t *)b.block;
    b.mitems = (uint32_t *)((char *)b.block + ib);
    b.slots = (int32_t *)((char *)b.block + ib + mb);
    b.n_items = (int)items.size();
    b.n_mitems = (int)mitems.size();
    b.n_slots = (int)order.size();
    b.rjobs = rj.empty() ? nullptr : (fk::RegionDev *)((char *)b.block + ib + mb + ob);
    b.n_rjobs = (int)rj.size();
    hipError_t e = hipSuccess;
    if (!rj.empty())
        e = hipMemcpy(b.rjobs, rj.data(), rj.size() * sizeof(fk::RegionDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b.items, items.data(), items.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b.mitems, mitems.data(), mitems.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b.slots, order.data(), order.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(c, b.block, b.bytes);
        return fail(FAST_E_DEVICE, "batch setup: %s", hipGetErrorString(e));
    }
    auto res = c->batches.emplace(hs, b);
    *out = &res.first->second;
    return FAST_OK;
}

// The shared planning launch of a batch.  A batch of one scenario (without
// per-agent speeds or several fields) runs the single-scenario kernel: up to
// one thread per tile cell and tile rows dealt to the dies, the faster launch
// for a scenario too small to fill the device by itself.  (Its descriptor is
// passed by value, which a captured graph keeps; a slot's descriptor never
// changes after setup.)
hipError_t launch_batch_plan(fast_ctx *c, const Batch *b, hipEvent_t e0, hipEvent_t e1)
{
    if (b->members.size() == 1 && b->het.empty()) {
        const Slot &s = c->slots[b->members[0]];
        return fk_launch_plan_one(&s.dev, s.n_items, 0, c->stream, e0, e1);
    }
    return fk_launch_plan(c->table, b->items, b->n_items, b->v, b->tx, c->stream, e0, e1);
}

// The planning launches of a batch's members with per-agent speeds.
hipError_t launch_het_members(fast_ctx *c, const std::vector<int32_t> &het)
{
    for (int32_t h : het) {
        const Slot &s = c->slots[h];
        const hipError_t e = fk_launch_plan_het(&s.dev, &s.hd, s.n_items, 0, c->stream, nullptr,
                                                nullptr);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The trail-field launches that close the motion phase of each listed member.
hipError_t launch_trails(fast_ctx *c, const std::vector<int32_t> &trails)
{
    for (int32_t h : trails) {
        const Slot &s = c->slots[h];
        const hipError_t e = fk_launch_trail(&s.dev, s.n_items, c->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Time steps of a batch captured as a HIP graph (k = 1: exec, k =
// GRAPH_STEPS: exec_k): per step one planning launch over every tile of
// every member, one motion launch over their workgroup groups.
fast_status batch_graph(fast_ctx *c, Batch *b, int k)
{
    hipGraphExec_t &exec = k == 1 ? b->exec : b->exec_k;
    hipGraph_t &graph = k == 1 ? b->graph : b->graph_k;
    if (exec) return FAST_OK;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    for (int j = 0; j < k && e1 == hipSuccess && e2 == hipSuccess; ++j) {
        e1 = launch_batch_plan(c, b, nullptr, nullptr);
        if (e1 == hipSuccess) e1 = launch_het_members(c, b->het);
        if (e1 == hipSuccess) e2 = fk_launch_move(c->table, b->mitems, b->n_mitems, c->stream);
        if (e2 == hipSuccess) e2 = launch_trails(c, b->trails);
        if (e2 == hipSuccess) e2 = fk_launch_count(b->rjobs, b->n_rjobs, b->max_regions, c->stream);
    }
    hipError_t e3 = hipStreamEndCapture(c->stream, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        graph = nullptr;
        return fail(FAST_E_DEVICE, "graph capture failed: %s / %s / %s", hipGetErrorString(e1),
                    hipGetErrorString(e2), hipGetErrorString(e3));
    }
    hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e4 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
        exec = nullptr;
        return fail(FAST_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e4));
    }
    return FAST_OK;
}

fast_status check_handles(fast_ctx *c, const int32_t *hs, int32_t n, std::vector<int32_t> &out)
{
    if (!hs || n < 1) return fail(FAST_E_INVALID, "empty handle list");
    out.assign(hs, hs + n);
    std::sort(out.begin(), out.end());
    if (std::adjacent_find(out.begin(), out.end()) != out.end())
        return fail(FAST_E_INVALID, "a handle appears twice");
    for (int32_t h : out)
        if (!get_slot(c, h)) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    return FAST_OK;
}

// Steps of a batch as plain launches (one planning and one motion launch per
// step), for member sets that change too often to be worth a graph.
fast_status launch_batch(fast_ctx *c, const std::vector<int32_t> &hs, int steps)
{
    Batch *b = nullptr;
    fast_status st = get_batch(c, hs, &b);
    if (st) return st;
    for (int k = 0; k < steps; ++k) {
        HIP_TRY(launch_batch_plan(c, b, nullptr, nullptr));
        HIP_TRY(launch_het_members(c, b->het));
        HIP_TRY(fk_launch_move(c->table, b->mitems, b->n_mitems, c->stream));
        HIP_TRY(launch_trails(c, b->trails));
        HIP_TRY(fk_launch_count(b->rjobs, b->n_rjobs, b->max_regions, c->stream));
    }
    for (int32_t h : hs) c->slots[h].host_steps += steps;
    return FAST_OK;
}

fast_status run_batch(fast_ctx *c, const std::vector<int32_t> &hs, int steps)
{
    for (int32_t h : hs) {
        Slot *s = get_slot(c, h);
        if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
        if (s->planned) return fail(FAST_E_STATE, "scenario %d has a plan without its motion phase", h);
    }
    if (steps == 0) return FAST_OK;
    Batch *b = nullptr;
    fast_status st = get_batch(c, hs, &b);
    if (st) return st;
    int left = steps;
    if (left >= GRAPH_STEPS) {
        st = batch_graph(c, b, GRAPH_STEPS);
        if (st) return st;
        for (; left >= GRAPH_STEPS; left -= GRAPH_STEPS) HIP_TRY(hipGraphLaunch(b->exec_k, c->stream));
    }
    if (left > 0) {
        st = batch_graph(c, b, 1);
        if (st) return st;
        for (; left > 0; --left) HIP_TRY(hipGraphLaunch(b->exec, c->stream));
    }
    for (int32_t h : hs) c->slots[h].host_steps += steps;
    return FAST_OK;
}

// ---------------------------------------------------------------------------
// Serving.  Builder threads do each request's host setup (floor field,
// placement, exp table) as soon as it is submitted; the server thread admits
// built requests in arrival order while the budget and the active cap allow
// (upload only), advances every active scenario with batched launches of up to
// 8 steps, retires finished ones, and records completion times.
// ---------------------------------------------------------------------------
void build_loop(fast_ctx *c)
{
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(c->smu);
            c->bcv.wait(lk, [&] { return c->stopping || !c->build_queue.empty(); });
            if (c->build_queue.empty()) return;                 // stopping, nothing left
            r = c->reqs[c->build_queue.front()].get();
            c->build_queue.pop_front();
        }
        std::unique_ptr<fh::Built> b(new fh::Built());
        const fast_status st = build_host(&r->desc, *b);
        {
            std::lock_guard<std::mutex> lk(c->smu);
            if (st) {
                r->built_state = -1;
            } else {
                r->built = std::move(b);
                r->built_state = 1;
            }
        }
        c->scv.notify_all();
    }
}

void serve_loop(fast_ctx *c)
{
    std::vector<uint64_t> active;
    auto head_ready = [&] {
        return !c->queue.empty() && c->reqs[c->queue.front()]->built_state != 0;
    };
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(c->smu);
            if (active.empty()) {
                c->scv.wait(lk, [&] { return (c->stopping && c->queue.empty()) || head_ready(); });
                if (c->stopping && c->queue.empty()) break;
            }
        }
        // admit, in arrival order
        for (;;) {
            uint64_t t = 0;
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(c->smu);
                if (!head_ready()) break;
                if (c->serve_max_active && (int)active.size() >= c->serve_max_active) break;
                t = c->queue.front();
                r = c->reqs[t].get();
                if (r->built_state < 0) {
                    c->queue.pop_front();
                    r->state = -1;
                    r->t_done = now_s();
                    continue;
                }
            }
            std::lock_guard<std::recursive_mutex> g(c->mu);
            const size_t saved = c->budget;
            if (c->serve_budget) c->budget = c->serve_budget;
            int32_t h = -1;
            fast_status st = upload_slot(c, &r->desc, *r->built, r->steps, &h);
            c->budget = saved;
            if (st == FAST_E_BUDGET && !active.empty()) break;      // wait for memory
            std::lock_guard<std::mutex> lk(c->smu);
            c->queue.pop_front();
            r->built.reset();
            if (st) { r->state = -1; r->t_done = now_s(); continue; }
            r->handle = h;
            r->state = 1;
            active.push_back(t);
        }
        if (active.empty()) continue;
        // one batched step over the active scenarios
        std::vector<int32_t> hs;
        {
            std::lock_guard<std::mutex> lk(c->smu);
            for (uint64_t t : active) hs.push_back(c->reqs[t]->handle);
        }
        std::sort(hs.begin(), hs.end());
        int chunk = INT_MAX;
        {
            std::lock_guard<std::mutex> lk(c->smu);
            for (uint64_t t : active) {
                Request *r = c->reqs[t].get();
                chunk = std::min(chunk, r->steps - c->slots[r->handle].host_steps);
            }
        }
        chunk = std::max(1, std::min(chunk, 8));
        {
            std::lock_guard<std::recursive_mutex> g(c->mu);
            if (launch_batch(c, hs, chunk)) {
                std::lock_guard<std::mutex> lk(c->smu);
                for (uint64_t t : active) { c->reqs[t]->state = -1; c->reqs[t]->t_done = now_s(); }
                active.clear();
                continue;
            }
            (void)hipStreamSynchronize(c->stream);
        }
        // retire
        std::vector<uint64_t> still;
        for (uint64_t t : active) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(c->smu);
                r = c->reqs[t].get();
            }
            std::lock_guard<std::recursive_mutex> g(c->mu);
            Slot &s = c->slots[r->handle];
            if (s.host_steps < r->steps) { still.push_back(t); continue; }
            const int n = s.n_agents;
            r->out_xy.assign((size_t)2 * std::max(n, 1), -1);
            r->out_alive.assign((size_t)std::max(n, 1), 0);
            read_state(c, &s, r->out_xy.data(), r->out_alive.data(), nullptr, &r->out_step,
                       &r->out_active);
            destroy_slot(c, r->handle);
            std::lock_guard<std::mutex> lk(c->smu);
            r->state = 2;
            r->t_done = now_s();
        }
        active.swap(still);
    }
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char *fast_last_error(void) { return g_err.c_str(); }

static fast_status check_grid(int32_t width, int32_t height, const uint8_t *cell_type)
{
    if (width < 3 || height < 3 || width > 16384 || height > 16384 || !cell_type)
        return fail(FAST_E_INVALID, "grid %dx%d outside 3..16384 or NULL", width, height);
    for (int64_t i = 0; i < (int64_t)width * height; ++i)
        if (cell_type[i] > fk::CELL_EXIT) return fail(FAST_E_INVALID, "cell_type values must be 0, 1 or 2");
    return FAST_OK;
}

fast_status fast_floor_field(int32_t width, int32_t height, const uint8_t *cell_type,
                             uint8_t *type_out, double *S_out)
{
    fast_status st = check_grid(width, height, cell_type);
    if (st) return st;
    std::vector<uint8_t> t(cell_type, cell_type + (size_t)width * height);
    std::vector<double> S;
    fh::floor_field(width, height, t, S);
    if (type_out) std::memcpy(type_out, t.data(), t.size());
    if (S_out) std::memcpy(S_out, S.data(), S.size() * sizeof(double));
    return FAST_OK;
}

fast_status fast_place(int32_t width, int32_t height, const uint8_t *cell_type, int32_t n_agents,
                       uint64_t seed, uint32_t scenario_id, int32_t *xy_out)
{
    fast_status st = check_grid(width, height, cell_type);
    if (st) return st;
    if (n_agents < 0 || !xy_out) return fail(FAST_E_INVALID, "bad n_agents or xy_out");
    std::vector<uint8_t> t(cell_type, cell_type + (size_t)width * height);
    std::vector<double> S;
    fh::floor_field(width, height, t, S);
    std::vector<int32_t> xy;
    if (!fh::place(width, height, t, n_agents, seed, scenario_id, xy))
        return fail(FAST_E_INVALID, "more agents than eligible cells");
    if (n_agents) std::memcpy(xy_out, xy.data(), xy.size() * sizeof(int32_t));
    return FAST_OK;
}

double fast_guard_band(int32_t v_max)
{
    if (v_max < 1 || v_max > fk::MAX_V) return -1.0;
    return (double)fh::guard_band(v_max);
}

fast_status fast_ctx_create(int device, void *hip_stream, size_t hbm_budget, fast_alloc_fn alloc,
                            fast_free_fn free_fn, void *user, fast_ctx **out)
{
    if (!out) return fail(FAST_E_INVALID, "out is NULL");
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(FAST_E_INVALID, "alloc and free_fn must both be set or both be NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(FAST_E_INVALID, "device %d of %d", device, ndev);
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<fast_ctx> c(new fast_ctx());
    c->device = device;
    c->budget = hbm_budget;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    c->slots.reserve(FAST_MAX_SLOTS);     // handles index a vector that never moves
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    int per_cu = 0;
    hipError_t e = stream_cus(c->stream, device, &c->n_cus);
    if (e == hipSuccess) e = fk_move_per_cu(&per_cu);
    if (e != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        return fail(FAST_E_DEVICE, "CU count of the stream: %s", hipGetErrorString(e));
    }
    c->move_capacity = per_cu * c->n_cus;
    e = fk_scratch_ptr(device, &c->scratch);         // device current (hipSetDevice above)
    if (e != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        return fail(FAST_E_DEVICE, "address of the static scratch: %s", hipGetErrorString(e));
    }
    e = hipMalloc(&c->table, sizeof(fk::SlotDev) * FAST_MAX_SLOTS);
    if (e != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        return fail(FAST_E_NOMEM, "slot table: %s", hipGetErrorString(e));
    }
    e = hipHostMalloc(&c->stage, fk::SCRATCH_BYTES, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->stage) (void)hipHostFree(c->stage);
        (void)hipFree(c->table);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        return fail(FAST_E_NOMEM, "staging buffer of the allocation-free run: %s", hipGetErrorString(e));
    }
    *out = c.release();
    return FAST_OK;
}

fast_status fast_ctx_destroy(fast_ctx *c)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    fast_serve_stop(c);
    {
        std::lock_guard<std::recursive_mutex> g(c->mu);
        (void)hipStreamSynchronize(c->stream);
        for (int32_t h = 0; h < (int32_t)c->slots.size(); ++h)
            if (c->slots[h].live) destroy_slot(c, h);
        for (auto &kv : c->batches) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
            if (kv.second.exec_k) (void)hipGraphExecDestroy(kv.second.exec_k);
            if (kv.second.graph_k) (void)hipGraphDestroy(kv.second.graph_k);
            dev_free(c, kv.second.block, kv.second.bytes);
        }
        c->batches.clear();
        for (hipEvent_t e : c->timing) (void)hipEventDestroy(e);
        c->timing.clear();
        (void)hipFree(c->table);
        (void)hipEventDestroy(c->staged);
        (void)hipHostFree(c->stage);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    }
    delete c;
    return FAST_OK;
}

fast_status fast_ctx_cus(fast_ctx *c, int32_t *n_cus)
{
    if (!c || !n_cus) return fail(FAST_E_INVALID, "ctx or n_cus is NULL");
    *n_cus = c->n_cus;
    return FAST_OK;
}

fast_status fast_cu_mask(int32_t n_cus, int32_t device_cus, uint32_t *mask, int32_t n_words)
{
    if (!mask || device_cus < 64 || device_cus % 64 || n_words < device_cus / 32)
        return fail(FAST_E_INVALID, "device_cus %d must be a positive multiple of 64 and n_words "
                    ">= device_cus / 32", device_cus);
    if (n_cus < 8 || n_cus > device_cus || n_cus % 8)
        return fail(FAST_E_INVALID, "n_cus %d: a multiple of 8 in 8..%d", n_cus, device_cus);
    const int per = device_cus / 8, m = n_cus / 8;
    std::fill(mask, mask + n_words, 0u);
    // XCD j owns bits j*per .. j*per + per - 1 when the driver hands out the
    // mask in blocks, and the bits b with b mod 8 == j when it interleaves.
    // Block j takes whole residue classes mod 8 starting at j (class j, then
    // j + 1, ...), so each XCD gets m bits under either rule.
    for (int j = 0; j < 8; ++j) {
        int taken = 0;
        for (int i = 0; i < 8 && taken < m; ++i)
            for (int k = (j + i) % 8; k < per && taken < m; k += 8, ++taken) {
                const int b = j * per + k;
                mask[b / 32] |= 1u << (b % 32);
            }
    }
    return FAST_OK;
}

fast_status fast_cu_stream_create(int32_t device, int32_t n_cus, void **stream, int32_t *n_cus_run,
                                  int32_t *per_xcd)
{
    if (!stream) return fail(FAST_E_INVALID, "stream is NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(FAST_E_INVALID, "device %d of %d", device, ndev);
    HIP_TRY(hipSetDevice(device));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    const fast_status st = fast_cu_mask(n_cus, cus, mask.data(), (int32_t)mask.size());
    if (st != FAST_OK) return st;
    hipStream_t s = nullptr;
    HIP_TRY(hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data()));
    int seen = 0;
    int32_t xcd[8];
    const hipError_t e = probe_cus(s, 4 * n_cus, &seen, xcd);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return fail(FAST_E_DEVICE, "CU probe: %s", hipGetErrorString(e));
    }
    if (n_cus_run) *n_cus_run = seen;
    if (per_xcd) std::copy(xcd, xcd + 8, per_xcd);
    *stream = (void *)s;
    return FAST_OK;
}

fast_status fast_cu_stream_destroy(void *stream)
{
    if (!stream) return fail(FAST_E_INVALID, "stream is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipStreamDestroy((hipStream_t)stream));
    return FAST_OK;
}

fast_status fast_init_scenario(fast_ctx *c, const fast_scenario_desc *d, int32_t *handle)
{
    if (!c || !handle) return fail(FAST_E_INVALID, "ctx or handle is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    return init_slot(c, d, INT_MAX, handle);
}

fast_status fast_destroy_scenario(fast_ctx *c, int32_t h)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    return destroy_slot(c, h);
}

fast_status fast_plan_step(fast_ctx *c, int32_t h)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    next_timing_pair(c, &e0, &e1);
    if (s->het)
        HIP_TRY(fk_launch_plan_het(&s->dev, &s->hd, s->n_items, 0, c->stream, e0, e1));
    else
        HIP_TRY(fk_launch_plan_one(&s->dev, s->n_items, 0, c->stream, e0, e1));
    s->planned = true;
    return FAST_OK;
}

fast_status fast_move_step(fast_ctx *c, int32_t h)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    if (!s->planned) return fail(FAST_E_STATE, "scenario %d: motion without a plan of this step", h);
    HIP_TRY(fk_launch_move(c->table, s->mitems, s->group, c->stream));
    HIP_TRY(fk_launch_trail(&s->dev, s->n_items, c->stream));
    if (s->n_regions) HIP_TRY(fk_launch_count(s->rdev, 1, s->n_regions, c->stream));
    s->planned = false;
    s->host_steps += 1;
    return FAST_OK;
}

fast_status fast_run(fast_ctx *c, const int32_t *hs, int32_t n, int32_t steps)
{
    if (!c || steps < 0) return fail(FAST_E_INVALID, "bad arguments to fast_run");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    std::vector<int32_t> v;
    fast_status st = check_handles(c, hs, n, v);
    if (st) return st;
    return run_batch(c, v, steps);
}

fast_status fast_run_noalloc(fast_ctx *c, const int32_t *hs, int32_t n, int32_t steps)
{
    if (!c || steps < 0) return fail(FAST_E_INVALID, "bad arguments to fast_run_noalloc");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    std::vector<int32_t> v;
    fast_status st = check_handles(c, hs, n, v);
    if (st) return st;
    for (int32_t h : v)
        if (c->slots[h].planned)
            return fail(FAST_E_STATE, "scenario %d has a plan without its motion phase", h);
    if (steps == 0) return FAST_OK;
    BatchItems &p = c->nb;
    st = batch_items(c, v, p);
    if (st) return st;
    // scratch layout: planning items | motion items | region-count jobs
    const size_t ib = align_up(p.items.size() * 4, 256), mb = align_up(p.mitems.size() * 4, 256);
    const size_t rb = p.rj.size() * sizeof(fk::RegionDev);
    if (ib + mb + rb > fk::SCRATCH_BYTES)
        return fail(FAST_E_INVALID, "the batch's work items take %zu bytes (%zu tiles, %zu motion "
                    "workgroups, %zu region jobs); the allocation-free run holds at most %zu",
                    ib + mb + rb, p.items.size(), p.mitems.size(), p.rj.size(),
                    (size_t)fk::SCRATCH_BYTES);
    // the previous call's copy out of the staging buffer has finished
    HIP_TRY(hipEventSynchronize(c->staged));
    char *stage = (char *)c->stage, *dev = (char *)c->scratch;
    std::memcpy(stage, p.items.data(), p.items.size() * 4);
    std::memcpy(stage + ib, p.mitems.data(), p.mitems.size() * 4);
    if (rb) std::memcpy(stage + ib + mb, p.rj.data(), rb);
    HIP_TRY(hipMemcpyAsync(dev, stage, ib + mb + rb, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(c->staged, c->stream));
    const uint32_t *items = (const uint32_t *)dev, *mitems = (const uint32_t *)(dev + ib);
    const fk::RegionDev *rjobs = rb ? (const fk::RegionDev *)(dev + ib + mb) : nullptr;
    for (int k = 0; k < steps; ++k) {
        HIP_TRY(fk_launch_plan(c->table, items, (int)p.items.size(), p.v, p.tx, c->stream, nullptr,
                               nullptr));
        HIP_TRY(launch_het_members(c, p.het));
        HIP_TRY(fk_launch_move(c->table, mitems, (int)p.mitems.size(), c->stream));
        HIP_TRY(launch_trails(c, p.trails));
        HIP_TRY(fk_launch_count(rjobs, (int)p.rj.size(), p.max_regions, c->stream));
    }
    for (int32_t h : v) c->slots[h].host_steps += steps;
    return FAST_OK;
}

fast_status fast_plan_batch(fast_ctx *c, const int32_t *hs, int32_t n)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    std::vector<int32_t> v;
    fast_status st = check_handles(c, hs, n, v);
    if (st) return st;
    Batch *b = nullptr;
    st = get_batch(c, v, &b);
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->n_items > 0) next_timing_pair(c, &e0, &e1);   // times the shared planning launch
    HIP_TRY(launch_batch_plan(c, b, e0, e1));
    HIP_TRY(launch_het_members(c, b->het));
    for (int32_t h : v) c->slots[h].planned = true;
    return FAST_OK;
}

fast_status fast_timing_start(fast_ctx *c, int32_t max_launches)
{
    if (!c || max_launches < 1 || max_launches > (1 << 20))
        return fail(FAST_E_INVALID, "bad arguments to fast_timing_start");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    for (hipEvent_t e : c->timing) (void)hipEventDestroy(e);
    c->timing.assign((size_t)2 * max_launches, nullptr);
    // Timing only: no system-scope fence when the event completes (its cache
    // writeback and invalidation would slow the launches that follow).  The
    // readers synchronise with the stream, not with these events.
    for (auto &e : c->timing) {
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            for (hipEvent_t x : c->timing) if (x) (void)hipEventDestroy(x);
            c->timing.clear();
            return fail(FAST_E_DEVICE, "hipEventCreate failed");
        }
    }
    c->timing_used = 0;
    return FAST_OK;
}

fast_status fast_timing_read(fast_ctx *c, float *ms, int32_t cap, int32_t *n)
{
    if (!c || !n || cap < 0 || (cap > 0 && !ms)) return fail(FAST_E_INVALID, "bad arguments to fast_timing_read");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int used = c->timing_used;
    for (int i = 0; i < used && i < cap; ++i)
        HIP_TRY(hipEventElapsedTime(&ms[i], c->timing[2 * i], c->timing[2 * i + 1]));
    *n = used;
    for (hipEvent_t e : c->timing) (void)hipEventDestroy(e);
    c->timing.clear();
    c->timing_used = 0;
    return FAST_OK;
}

fast_status fast_move_batch(fast_ctx *c, const int32_t *hs, int32_t n)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    std::vector<int32_t> v;
    fast_status st = check_handles(c, hs, n, v);
    if (st) return st;
    for (int32_t h : v)
        if (!c->slots[h].planned)
            return fail(FAST_E_STATE, "scenario %d: motion without a plan of this step", h);
    Batch *b = nullptr;
    st = get_batch(c, v, &b);
    if (st) return st;
    HIP_TRY(fk_launch_move(c->table, b->mitems, b->n_mitems, c->stream));
    HIP_TRY(launch_trails(c, b->trails));
    HIP_TRY(fk_launch_count(b->rjobs, b->n_rjobs, b->max_regions, c->stream));
    for (int32_t h : v) {
        c->slots[h].planned = false;
        c->slots[h].host_steps += 1;
    }
    return FAST_OK;
}

fast_status fast_set_regions(fast_ctx *c, int32_t h, const int32_t *rects, int32_t n_regions,
                             int32_t max_step)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    if (n_regions < 0 || n_regions > fk::MAX_REGIONS || (n_regions && !rects))
        return fail(FAST_E_INVALID, "n_regions %d outside 0..%d (or rects NULL)", n_regions,
                    fk::MAX_REGIONS);
    if (n_regions && (max_step < 0 || max_step >= (1 << 24)))
        return fail(FAST_E_INVALID, "max_step %d outside 0..2^24-1", max_step);
    const fk::SlotDev &d = s->dev;
    for (int r = 0; r < n_regions; ++r) {
        const int32_t *q = rects + 4 * r;
        if (q[0] < 0 || q[1] < 0 || q[0] >= q[2] || q[1] >= q[3] || q[2] > d.W || q[3] > d.H)
            return fail(FAST_E_INVALID, "rectangle %d (%d,%d)-(%d,%d) is empty or outside the %dx%d grid",
                        r, q[0], q[1], q[2], q[3], d.W, d.H);
    }
    fk::RegionDev j{};
    const size_t rows = (size_t)max_step + 1;
    const size_t bytes = n_regions ? align_up(sizeof j, 256) + rows * n_regions * 4 : 0;
    void *block = nullptr;
    if (n_regions) {
        fast_status st = dev_alloc(c, bytes, &block);
        if (st) return st;
    }
    const hipError_t es = hipStreamSynchronize(c->stream);
    if (es != hipSuccess) {
        dev_free(c, block, bytes);
        return fail(FAST_E_DEVICE, "region setup: %s", hipGetErrorString(es));
    }
    drop_batches_with(c, h);                          // their graphs count the old regions
    dev_free(c, s->rdev, s->rbytes);
    s->rdev = nullptr;
    s->rbytes = 0;
    s->n_regions = 0;
    s->rhost = fk::RegionDev{};
    if (!n_regions) return FAST_OK;
    j.occ = d.occ;
    j.ctr = d.ctr;
    j.series = (int32_t *)((char *)block + align_up(sizeof j, 256));
    j.Wp = d.Wp;
    j.pad = d.pad;
    j.n = n_regions;
    j.rows = (int32_t)rows;
    std::copy(rects, rects + 4 * n_regions, j.rect);
    // all on the context stream, in order: -1 for steps not reached, the job,
    // then the count of the current step
    hipError_t e = hipMemsetAsync(j.series, 0xFF, rows * n_regions * 4, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(block, &j, sizeof j, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = fk_launch_count((fk::RegionDev *)block, 1, n_regions, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        dev_free(c, block, bytes);
        return fail(FAST_E_DEVICE, "region setup: %s", hipGetErrorString(e));
    }
    s->rhost = j;
    s->rdev = (fk::RegionDev *)block;
    s->rbytes = bytes;
    s->n_regions = n_regions;
    return FAST_OK;
}

fast_status fast_get_regions(fast_ctx *c, int32_t h, int32_t *counts, int64_t capacity,
                             int32_t *n_regions, int32_t *rows)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    if (n_regions) *n_regions = s->n_regions;
    if (rows) *rows = s->n_regions ? s->rhost.rows : 0;
    if (!s->n_regions || !counts) return FAST_OK;
    const int64_t total = (int64_t)s->rhost.rows * s->n_regions;
    if (capacity < total)
        return fail(FAST_E_INVALID, "counts holds %lld ints; the series has %lld", (long long)capacity,
                    (long long)total);
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(counts, s->rhost.series, (size_t)total * 4, hipMemcpyDeviceToHost));
    return FAST_OK;
}

fast_status fast_get_state(fast_ctx *c, int32_t h, int32_t *xy, uint8_t *alive, int32_t *desired,
                           int32_t *step, int32_t *n_active)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    return read_state(c, s, xy, alive, desired, step, n_active);
}

fast_status fast_get_trail(fast_ctx *c, int32_t h, double *out, int64_t capacity)
{
    if (!c || !out) return fail(FAST_E_INVALID, "ctx or out is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    const fk::SlotDev &d = s->dev;
    if (!d.Tr) return fail(FAST_E_INVALID, "scenario %d keeps no trail field (k_d, trail_decay and trail_diffusion are 0)", h);
    if (capacity < (int64_t)d.W * d.H)
        return fail(FAST_E_INVALID, "out holds %lld doubles; the grid has %lld", (long long)capacity,
                    (long long)d.W * d.H);
    HIP_TRY(hipStreamSynchronize(c->stream));
    int32_t step = 0;
    HIP_TRY(hipMemcpy(&step, d.ctr + fk::C_STEP, 4, hipMemcpyDeviceToHost));
    const size_t cells = (size_t)d.Wp * d.Hp;
    std::vector<double> t(cells);
    HIP_TRY(hipMemcpy(t.data(), d.Tr + (size_t)(step & 1) * cells, cells * 8, hipMemcpyDeviceToHost));
    for (int y = 0; y < d.H; ++y)
        for (int x = 0; x < d.W; ++x)
            out[(size_t)y * d.W + x] = t[(size_t)(y + d.pad) * d.Wp + x + d.pad];
    return FAST_OK;
}

fast_status fast_get_stats(fast_ctx *c, int32_t h, fast_stats *out)
{
    if (!c || !out) return fail(FAST_E_INVALID, "ctx or out is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    HIP_TRY(hipStreamSynchronize(c->stream));
    int32_t ctr[fk::C_NCTR];
    unsigned long long stat[fk::S_NSTAT];
    HIP_TRY(hipMemcpy(ctr, s->dev.ctr, sizeof ctr, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(stat, s->dev.stat, sizeof stat, hipMemcpyDeviceToHost));
    if (ctr[fk::C_ERR])
        return fail(FAST_E_DEVICE, "a motion-phase group barrier timed out: the scenario state is invalid");
    std::memset(out, 0, sizeof *out);
    out->step = ctr[fk::C_STEP];
    out->n_agents = s->n_agents;
    out->n_active = ctr[fk::C_NACTIVE];
    out->exited = ctr[fk::C_EXITED];
    out->flagged = (int64_t)stat[fk::S_FLAGGED];
    out->fallback = (int64_t)stat[fk::S_FALLBACK];
    out->last_rounds = ctr[fk::C_ROUNDS];
    out->tile_w = s->dev.tx;
    out->tile_h = s->dev.ty;
    out->n_tiles = s->n_items;
    out->n_fallback_tiles = s->n_fb_tiles;
    out->guard_band = s->dev.eps;
    out->device_bytes = (int64_t)s->bytes;
    out->planned = (int64_t)stat[fk::S_PLANNED];
    return FAST_OK;
}

fast_status fast_debug_plan(fast_ctx *c, int32_t h, float *w32, uint8_t *flag, float *margin,
                            float *cdf32)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    Slot *s = get_slot(c, h);
    if (!s) return fail(FAST_E_NOTFOUND, "unknown scenario handle %d", h);
    const int n = std::max(s->n_agents, 1);
    const int side = 2 * s->dev.v + 1;
    const size_t bw = align_up((size_t)n * side * side * 4, 256), bf = align_up((size_t)n, 256),
                 bm = align_up((size_t)n * 4, 256), bc = (size_t)n * side * side * 4;
    const size_t total = bw + bf + bm + bc;
    void *block = nullptr;
    fast_status st = dev_alloc(c, total, &block);
    if (st) return st;
    fk::SlotDev sd = s->dev;
    sd.dbg_w = (float *)block;
    sd.dbg_flag = (uint8_t *)((char *)block + bw);
    sd.dbg_margin = (float *)((char *)block + bw + bf);
    sd.dbg_cdf = (float *)((char *)block + bw + bf + bm);
    hipError_t e = hipMemsetAsync(block, 0, total, c->stream);
    if (e == hipSuccess)
        e = s->het ? fk_launch_plan_het(&sd, &s->hd, s->n_items, 1, c->stream, nullptr, nullptr)
                   : fk_launch_plan_one(&sd, s->n_items, 1, c->stream, nullptr, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
        s->planned = true;
        const int na = s->n_agents;
        const size_t wb = (size_t)na * side * side * 4;
        if (w32 && na) e = hipMemcpy(w32, sd.dbg_w, wb, hipMemcpyDeviceToHost);
        if (e == hipSuccess && flag && na) e = hipMemcpy(flag, sd.dbg_flag, (size_t)na, hipMemcpyDeviceToHost);
        if (e == hipSuccess && margin && na) e = hipMemcpy(margin, sd.dbg_margin, (size_t)na * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && cdf32 && na) e = hipMemcpy(cdf32, sd.dbg_cdf, wb, hipMemcpyDeviceToHost);
    }
    dev_free(c, block, total);
    if (e != hipSuccess) return fail(FAST_E_DEVICE, "debug plan: %s", hipGetErrorString(e));
    return FAST_OK;
}

fast_status fast_stream_bandwidth(fast_ctx *c, size_t footprint, int32_t reps, double *gb_per_s,
                                  double *us_per_launch)
{
    if (!c || !gb_per_s || reps < 1 || reps > 10000 || footprint < 96 || footprint > ((size_t)64 << 30))
        return fail(FAST_E_INVALID, "bad arguments to fast_stream_bandwidth");
    std::lock_guard<std::recursive_mutex> g(c->mu);
    const size_t n4 = footprint / 96;                          // six arrays of n4 float4
    const size_t bytes = n4 * 96;
    void *block = nullptr;
    fast_status st = dev_alloc(c, bytes, &block);
    if (st) return st;
    std::vector<hipEvent_t> ev((size_t)2 * (reps + 2), nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)                                        // timing only, as fast_timing_start's
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipMemsetAsync(block, 0, bytes, c->stream);
    for (int i = 0; i < reps + 2 && e == hipSuccess; ++i)       // two untimed launches first
        e = fk_launch_stream((float4 *)block, n4, c->stream, ev[2 * i], ev[2 * i + 1]);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double total_ms = 0.0;
    for (int i = 2; i < reps + 2 && e == hipSuccess; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        total_ms += ms;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    dev_free(c, block, bytes);
    if (e != hipSuccess) return fail(FAST_E_DEVICE, "stream bandwidth: %s", hipGetErrorString(e));
    const double avg_s = total_ms / reps / 1e3;
    *gb_per_s = (double)bytes / avg_s / 1e9;
    if (us_per_launch) *us_per_launch = avg_s * 1e6;
    return FAST_OK;
}

fast_status fast_serve_start(fast_ctx *c, size_t budget, int32_t max_active)
{
    if (!c || max_active < 0) return fail(FAST_E_INVALID, "bad arguments to fast_serve_start");
    std::lock_guard<std::mutex> lk(c->smu);
    if (c->serving) return fail(FAST_E_STATE, "already serving");
    c->serve_budget = budget;
    c->serve_max_active = max_active;
    c->stopping = false;
    c->serving = true;
    c->server = std::thread(serve_loop, c);
    const unsigned hw = std::thread::hardware_concurrency();
    const int nb = (int)std::max(1u, std::min(8u, hw / 2));
    for (int i = 0; i < nb; ++i) c->builders.emplace_back(build_loop, c);
    return FAST_OK;
}

fast_status fast_serve_submit(fast_ctx *c, const fast_scenario_desc *d, int32_t steps,
                              uint64_t *ticket)
{
    if (!c || !ticket || steps < 0) return fail(FAST_E_INVALID, "bad arguments to fast_serve_submit");
    fast_status st = check_desc(d);
    if (st) return st;
    std::unique_ptr<Request> r(new Request());
    r->desc = *d;
    r->cells.assign(d->cell_type, d->cell_type + (size_t)d->width * d->height);
    r->desc.cell_type = r->cells.data();
    if (d->agent_xy) {
        r->xy.assign(d->agent_xy, d->agent_xy + (size_t)2 * d->n_agents);
        r->desc.agent_xy = r->xy.data();
    }
    if (d->agent_v) {
        r->vi.assign(d->agent_v, d->agent_v + d->n_agents);
        r->desc.agent_v = r->vi.data();
    }
    if (d->exit_field) {
        r->ef.assign(d->exit_field, d->exit_field + (size_t)d->width * d->height);
        r->desc.exit_field = r->ef.data();
    }
    if (d->agent_field && d->n_agents > 0) {
        r->fi.assign(d->agent_field, d->agent_field + d->n_agents);
        r->desc.agent_field = r->fi.data();
    }
    r->steps = steps;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(c->smu);
    if (!c->serving) return fail(FAST_E_STATE, "serving is not started");
    r->ticket = c->next_ticket++;
    *ticket = r->ticket;
    c->queue.push_back(r->ticket);
    c->build_queue.push_back(r->ticket);
    c->reqs[r->ticket] = std::move(r);
    c->bcv.notify_one();
    return FAST_OK;
}

fast_status fast_serve_poll(fast_ctx *c, uint64_t ticket, int32_t *done, double *latency_s)
{
    if (!c || !done) return fail(FAST_E_INVALID, "bad arguments to fast_serve_poll");
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->reqs.find(ticket);
    if (it == c->reqs.end()) return fail(FAST_E_NOTFOUND, "unknown ticket");
    Request *r = it->second.get();
    if (r->state == -1) return fail(FAST_E_INVALID, "request was rejected");
    *done = r->state == 2 ? 1 : 0;
    if (latency_s) *latency_s = r->state == 2 ? r->t_done - r->t_submit : now_s() - r->t_submit;
    return FAST_OK;
}

fast_status fast_serve_result(fast_ctx *c, uint64_t ticket, int32_t *xy, uint8_t *alive,
                              int32_t *step, int32_t *n_active)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->reqs.find(ticket);
    if (it == c->reqs.end()) return fail(FAST_E_NOTFOUND, "unknown ticket");
    Request *r = it->second.get();
    if (r->state != 2) return fail(FAST_E_STATE, "request not finished");
    const int n = r->desc.n_agents;
    if (xy && n) std::memcpy(xy, r->out_xy.data(), (size_t)2 * n * 4);
    if (alive && n) std::memcpy(alive, r->out_alive.data(), (size_t)n);
    if (step) *step = r->out_step;
    if (n_active) *n_active = r->out_active;
    return FAST_OK;
}

fast_status fast_serve_stop(fast_ctx *c)
{
    if (!c) return fail(FAST_E_INVALID, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(c->smu);
        if (!c->serving) return FAST_OK;
        c->stopping = true;
        c->scv.notify_all();
        c->bcv.notify_all();
    }
    for (auto &b : c->builders) b.join();
    c->builders.clear();
    c->scv.notify_all();
    if (c->server.joinable()) c->server.join();
    std::lock_guard<std::mutex> lk(c->smu);
    c->serving = false;
    return FAST_OK;
}

}  // extern "C"
