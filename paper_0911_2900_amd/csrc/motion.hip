// motion.hip -- the motion phase with the model's sequential semantics
// (paper Sec. 1): agents walk their lines one by one in priority order.  It
// runs as deterministic reservations on a group of workgroups per scenario.
//
// What an agent A can meet on its line is decided once per phase, when the
// movers are gathered and nothing has moved yet: a wall or a cut wall corner
// ends the line; so does a cell held by an agent of lower priority in this
// step's order (a mover of lower priority is still there when A's turn comes;
// an agent that does not move stays anyway); a cell held by an agent of
// higher priority stays open (if it is a mover it may leave first; if not,
// A finds the cell occupied when it walks).  The line up to that point, cells
// 0..m_eff, is A's reach.  Cells other than movers' start cells only ever
// gain occupants, committed movers that stay.
//
// Every round each pending mover reserves its reach with atomicMax of its
// priority word.  A mover commits once it holds every reach cell it can still
// enter: cells 1..j, where cell j + 1 is the first cell (other than a
// higher-priority mover's start) that has become occupied, necessarily by a
// committed mover that stays there.  Its own start cell need not be held:
// a higher-priority mover whose line crosses it stops short of it anyway.
// A committed mover walks cells 1..j and stops before the first occupied one
// (a higher-priority mover that stayed) or leaves at an exit.  Two movers
// commit in the same round only if neither can affect the other's walk, and
// each mover commits only after every higher-priority mover that can, so the
// result equals moving them one by one in priority order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fast_dev.h"

namespace fk {

// ---------------------------------------------------------------------------
// Motion kernel: deterministic reservations.  The movers of a scenario are
// split over a group of G workgroups; each keeps its share in a private list.
// Round r reserves into res[r & 1] with tag r (tags grow, so stale words of
// earlier rounds always lose), so the checks of round r and the reservations
// of round r + 1 never touch the same array and one group barrier per round
// suffices:
//     reserve r+1 (own losers) | count | barrier | check r+1, commit, ...
// Most movers commit in the first rounds; the long tail of rounds has few
// movers and its cost is the latency of the group barrier.  Once at most
// MOVE_SOLO_MAX movers are left, workgroup 0 gathers every workgroup's list
// and runs the remaining rounds alone, with workgroup barriers only.
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
// (The quotients have numerators <= 2 v^2 + v = 55 and denominators 2m <= 10:
// n / 2m is an integer or at least 0.1 below the next one, so the FP32
// product with 1 / 2m plus 0.05, truncated, is the exact floor.)
struct Line {
    int cx, cy, sx, sy, adx, ady, m;
    float inv2m;
    __device__ __forceinline__ void at(int k, int &x, int &y) const
    {
        x = cx + sx * (int)((float)(2 * k * adx + m) * inv2m + 0.05f);
        y = cy + sy * (int)((float)(2 * k * ady + m) * inv2m + 0.05f);
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
    L.inv2m = 0.5f / (float)max(L.m, 1);
    return L;
}

// Barrier of the G workgroups of one scenario that also sums their mover
// counts.  Round r uses the 64-bit word bar[r & 1] = [arrivals:32][count:32]
// (both zeroed by the planning kernel): each workgroup adds (1 << 32) | n and
// waits until the arrivals reach (r / 2 + 1) * G.  A word is touched again only
// two barriers later, after every workgroup has read it, so the count part
// minus its value at the previous barrier of the same parity is this round's
// total.
//
// Everything one workgroup writes for the others (reservations, occupancy,
// movers handed over, counts) is written with agent-scope atomics or atomic
// stores and read with agent-scope loads: each location is coherent across
// the device's dies by itself.  So the barrier needs no cache write-back or
// invalidation (a fence at agent scope does both, on the L2 of each die):
// every thread waits until its own memory operations have completed, then
// thread 0 arrives.  `acquire`: thread 0 then also invalidates its caches
// (an agent-scope acquire fence), after which plain loads of the workgroup
// see what the others wrote.  A wait longer than SPIN_LIMIT polls marks the
// scenario as failed (C_ERR) instead of hanging; the function then returns -1.
__device__ int group_sync_count(const SlotDev &s, int G, int r, int n, unsigned long long &seen0,
                                unsigned long long &seen1, bool acquire = false)
{
    __shared__ int sh_total;
    if (G == 1) {
        __syncthreads();
        return n;
    }
    __builtin_amdgcn_s_waitcnt(0);                 // this thread's stores and atomics are done
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *bar = (unsigned long long *)&s.ctr[C_BAR] + (r & 1);
        unsigned long long &seen = (r & 1) ? seen1 : seen0;
        atomicAdd(bar, (1ull << 32) | (unsigned long long)(uint32_t)n);
        const unsigned long long target = (unsigned long long)(r / 2 + 1) * (unsigned long long)G;
        uint32_t spins = 0;
        unsigned long long w;
        int total = -1;
        for (;;) {
            w = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((w >> 32) >= target) { total = (int)((uint32_t)w - (uint32_t)seen); seen = w; break; }
            if (++spins > SPIN_LIMIT) { atomicOr(&s.ctr[C_ERR], 1); break; }
            __builtin_amdgcn_s_sleep(1);           // back off: fewer polls of the shared word
        }
        if (acquire) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sh_total = total;
    }
    __syncthreads();
    return sh_total;
}

__device__ __forceinline__ int mover_reach(unsigned long long key)
{
    return (int)((key >> MEFF_SHIFT) & 7ull);
}

// Reserves a mover's reach, cells 0..m_eff of its line, for a round: the
// largest word on a cell is the round's earliest mover there.
template <int V>
__device__ __forceinline__ void reserve_reach(const SlotDev &s, unsigned long long *res,
                                              const Mover &mv, unsigned long long tagw)
{
    const Line L = make_line(mv.cxy, mv.dxy);
    const int me = mover_reach(mv.key);
    const unsigned long long word = (mv.key & KEY_MASK) | tagw;
#pragma unroll
    for (int k = 0; k <= V; ++k) {
        if (k <= me) {
            int x, y;
            L.at(k, x, y);
            atomicMax(&res[y * s.Wp + x], word);
        }
    }
}

template <int V>
__device__ __forceinline__ void reserve_list(const SlotDev &s, unsigned long long *res,
                                             const Mover *list, int n, unsigned long long tagw)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) reserve_reach<V>(s, res, list[i], tagw);
}

// Priority word [~x0:32][~id:20] of agent id in this step's motion order.
__device__ __forceinline__ unsigned long long order_key(const SlotDev &s, uint32_t id, int step)
{
    const uint32_t x0 = philox_word0(id, (uint32_t)step, s.scn, STREAM_ORDER, s.seed_lo, s.seed_hi);
    return ((unsigned long long)(~x0) << ID_BITS) | (unsigned long long)(~id & ID_MASK);
}

// The reach of a mover (see the protocol above), from the cell types and the
// occupancy at the start of the phase: returns the m_eff, higher-priority-cell
// and exit bits of its key.  Runs while the movers are gathered, before any
// mover of the scenario moves.
template <int V>
__device__ unsigned long long line_reach(const SlotDev &s, const Mover &mv, int step)
{
    const Line L = make_line(mv.cxy, mv.dxy);
    const int Wp = s.Wp;
    const unsigned long long self = mv.key & KEY_MASK;
    // every load of the line first (one memory round trip), then the walk
    uint32_t wallm = 0, exitm = 0;                      // bit k: wall or cut corner / exit
    int o[V + 1];
    int px = L.cx, py = L.cy;
#pragma unroll
    for (int k = 1; k <= V; ++k) {
        int qx = px, qy = py;
        if (k <= L.m) L.at(k, qx, qy);
        const int q = qy * Wp + qx;
        const bool in = k <= L.m;
        // one byte holds the cell's type and, per diagonal direction,
        // whether stepping in that way cuts a wall corner; walls are never
        // occupied, so the occupancy load need not wait for the type
        const uint32_t cb = in ? s.cell[q] : (uint32_t)CELL_WALL;
        const bool diag = qx != px && qy != py;
        const bool cut = diag && ((cb >> cut_bit(qx - px, qy - py)) & 1u);
        const uint32_t t = cb & CELL_TYPE_MASK;
        wallm |= (t == CELL_WALL || cut) ? 1u << k : 0u;
        exitm |= t == CELL_EXIT ? 1u << k : 0u;
        o[k] = in ? s.occ[q] : -1;
        px = qx;
        py = qy;
    }
    const int first_wall = __builtin_ctz(wallm | (1u << (V + 1)));   // V + 1: none
    const int ms = min(first_wall - 1, L.m);
    int me = ms;
    uint32_t hp = 0;
    bool ex = false;
#pragma unroll
    for (int k = 1; k <= V; ++k) {
        if (k > ms) break;
        if (o[k] >= 0) {
            if (order_key(s, (uint32_t)o[k], step) > self) {
                hp |= 1u << (k - 1);                // higher priority: may have left by then
                continue;
            }
            me = k - 1;                             // there when this mover's turn comes
            break;
        }
        if ((exitm >> k) & 1u) {
            me = k;
            ex = true;
            break;
        }
    }
    return ((unsigned long long)me << MEFF_SHIFT) | ((unsigned long long)hp << HP_SHIFT) |
           (ex ? (1ull << EXIT_BIT) : 0ull);
}

__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Appends the kept movers of one pass of the workgroup to list + n (the
// count comes from sh_kept after the caller's barrier).
__device__ __forceinline__ void append_kept(Mover *list, int n, bool keep, const Mover &mv, int *sh_kept)
{
    const unsigned long long m = __ballot(keep);
    if (m) {
        const int lane = __lane_id();
        int base = 0;
        if (lane == 0) base = atomicAdd(sh_kept, __popcll(m));
        base = __shfl(base, 0);
        if (keep) list[n + base + lanes_below(m)] = mv;
    }
}

// Check-and-commit of one mover (see the protocol above).  Returns true if
// it cannot commit yet; then, when res_next is given, it reserves its reach
// for the next round there with tagw_next (the other array: this round's
// checks never read it).  Reservations and occupancy are read with
// agent-scope loads, or with plain (cacheable) ones when the last barrier
// ended with an acquire fence (`acquired`): either way they see every
// reservation of the round and at least the occupancy at its start (commits
// of this round may or may not be seen, which the protocol allows).
template <int V>
__device__ __forceinline__ bool commit_one(const SlotDev &s, const unsigned long long *res,
                                           const Mover &mv, unsigned long long tagw, bool acquired,
                                           unsigned long long *res_next,
                                           unsigned long long tagw_next)
{
    const int Wp = s.Wp;
    const Line L = make_line(mv.cxy, mv.dxy);
    const int me = mover_reach(mv.key);
    const uint32_t hp = (uint32_t)(mv.key >> HP_SHIFT) & 0x1Fu;
    const unsigned long long word = (mv.key & KEY_MASK) | tagw;
    int cell[V + 1];
    unsigned long long w[V + 1];
    int o[V + 1];
#pragma unroll
    for (int k = 0; k <= V; ++k) {
        int x = L.cx, y = L.cy;
        if (k <= me) L.at(k, x, y);
        cell[k] = y * Wp + x;
        const bool in = k >= 1 && k <= me;
        if (acquired) {
            w[k] = in ? res[cell[k]] : word;
            o[k] = in ? s.occ[cell[k]] : -1;
        } else {
            w[k] = in ? ld_res(&res[cell[k]]) : word;
            o[k] = in ? ld_agent(&s.occ[cell[k]]) : -1;
        }
    }
    // j: the reach cells still enterable; the mover must hold all of them
    int j = me;
#pragma unroll
    for (int k = V; k >= 1; --k)
        if (k <= me && o[k] >= 0 && !((hp >> (k - 1)) & 1u)) j = k - 1;
    bool holds = true;
#pragma unroll
    for (int k = 1; k <= V; ++k) holds &= (k > j) || (w[k] == word);
    if (!holds) {
        if (res_next) {
            const unsigned long long wn = (mv.key & KEY_MASK) | tagw_next;
#pragma unroll
            for (int k = 0; k <= V; ++k)
                if (k <= me) atomicMax(&res_next[cell[k]], wn);
        }
        return true;
    }
    const int id = (int)(~(uint32_t)mv.key & ID_MASK);
    const int c = cell[0];
    int at = c, reached = 0;
#pragma unroll
    for (int k = 1; k <= V; ++k) {
        if (k > j || o[k] >= 0) break;
        at = cell[k];
        reached = k;
    }
    const bool gone = reached == me && me > 0 && ((mv.key >> EXIT_BIT) & 1ull);
    if (gone) {
        st_agent(&s.occ[c], -1);
        atomicAnd(&s.D[c], ~D_OCC);
        atomicAdd(&s.ctr[C_EXITED], 1);
        atomicSub(&s.ctr[C_NACTIVE], 1);
    } else if (at != c) {
        st_agent(&s.occ[c], -1);
        atomicAnd(&s.D[c], ~D_OCC);
        st_agent(&s.occ[at], id);
        atomicOr(&s.D[at], D_OCC);
    }
    if (s.dep && (gone || at != c)) atomicAdd(&s.dep[c], 1);   // it left its cell: a trail deposit
    return false;
}

// Check-and-commit for the workgroup's list; movers that cannot commit yet
// are appended to `nxt` (the workgroup's own list, one LDS atomic per
// wavefront) and reserve the next round (commit_one).  Returns the number
// appended.
template <int V>
__device__ int commit_list(const SlotDev &s, const unsigned long long *res, const Mover *cur,
                           Mover *nxt, int n, unsigned long long tagw, bool acquired,
                           unsigned long long *res_next, unsigned long long tagw_next)
{
    __shared__ int sh_cnt;
    if (threadIdx.x == 0) sh_cnt = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + (int)threadIdx.x;
        Mover mv{};
        bool lose = false;
        if (i < n) {
            mv = cur[i];
            lose = commit_one<V>(s, res, mv, tagw, acquired, res_next, tagw_next);
        }
        append_kept(nxt, 0, lose, mv, &sh_cnt);
    }
    __syncthreads();
    return sh_cnt;
}

// Room of each workgroup's mover lists (mv_a, mv_b), in tiles' worth: enough
// for every split of the records below (ceil(tiles / G), or with G a multiple
// of DIES ceil(ceil(tiles / DIES) / (G / DIES)) if larger); G times it is at
// most tiles + 2 MOVE_GROUP_MAX, the room of the arrays.
__device__ __forceinline__ long list_capacity(const SlotDev &s, int G)
{
    const int T = s.ntx * s.nty;
    int tiles = (T + G - 1) / G;
    if (G % DIES == 0) {                                   // the split by dies
        const int m = G / DIES;
        tiles = max(tiles, ((T + DIES - 1) / DIES + m - 1) / m);
    }
    return (long)tiles * (s.tx * s.ty);
}

// Workgroup 0 gathers the movers left in every workgroup's list (copies in
// the handoff area, MOVE_SOLO_MAX per workgroup, counts in ctr[C_SOLO + g])
// into `to`, starting at 0.  Other workgroups wrote them with agent-scope
// stores before the last group barrier, so they are read with agent-scope
// loads.  Returns the count.
__device__ int gather_lists(const SlotDev &s, int G, Mover *to, int *sh_scan)
{
    const int tid = threadIdx.x;
    if (tid < G) sh_scan[tid] = ld_agent(&s.ctr[C_SOLO + tid]);
    __syncthreads();
    if (tid == 0)
        for (int k = 1; k < G; ++k) sh_scan[k] += sh_scan[k - 1];
    __syncthreads();
    const int total = sh_scan[G - 1];
    for (int i = tid; i < total; i += blockDim.x) {
        int a = 0, b = G - 1;                       // first list whose inclusive count exceeds i
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (sh_scan[mid] > i) b = mid; else a = mid + 1;
        }
        const int k = i - (a ? sh_scan[a - 1] : 0);
        const Mover *src = s.hand + (long)a * MOVE_SOLO_MAX + k;
        Mover mv;
        mv.key = __hip_atomic_load(&src->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        mv.cxy = __hip_atomic_load(&src->cxy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        mv.dxy = __hip_atomic_load(&src->dxy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        to[i] = mv;
    }
    __syncthreads();
    return total;
}


// Inclusive prefix sum of sh[0 .. MOVE_THREADS) in place (all threads call;
// each thread's own element must be in place): a shuffle scan within each
// wavefront, then one over the wavefront totals, three workgroup barriers in
// all.
__device__ __forceinline__ void block_scan(int *sh)
{
    constexpr int NW = MOVE_THREADS / 64;
    __shared__ int wsum[NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int x = sh[tid];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {
        int t = lane < NW ? wsum[lane] : 0;
#pragma unroll
        for (int off = 1; off < NW; off <<= 1) {
            const int y = __shfl_up(t, off);
            if (lane >= off) t += y;
        }
        if (lane < NW) wsum[lane] = t;
    }
    __syncthreads();
    if (wv > 0) x += wsum[wv - 1];
    sh[tid] = x;
    __syncthreads();
}

// The mover of record rec of tile `tile` (an agent's plan: its cell in the
// tile and the window slot it chose) with its priority word [~x0:32][~id:20]
// (larger = earlier) and reach bits; the id is the occupant of the start cell
// (nothing has moved yet).  False if it never moves: an agent that stays, or
// a mover blocked at its first cell, is at every other mover's turn still
// where it started, which is what they see without it taking part.
template <int V>
__device__ __forceinline__ bool gather_one(const SlotDev &s, uint32_t rec, int tile, int step, Mover &mv)
{
    constexpr int SIDE = 2 * V + 1;
    const int slot = (int)(rec >> REC_SLOT_SHIFT);
    if (slot == V * SIDE + V) return false;
    const int lc = (int)(rec & ((1u << REC_SLOT_SHIFT) - 1u));
    const int tlog = __builtin_ctz((unsigned)s.tx);
    const int tile_y = tile / s.ntx, tile_x = tile - tile_y * s.ntx;
    const int cx = tile_x * s.tx + s.pad + (lc & (s.tx - 1));
    const int cy = tile_y * s.ty + s.pad + (lc >> tlog);
    const int dy = slot / SIDE - V, dx = slot - (dy + V) * SIDE - V;
    const int id = s.occ[cy * s.Wp + cx];
    mv.key = order_key(s, (uint32_t)id, step);
    mv.cxy = (uint32_t)cx | ((uint32_t)cy << 16);
    mv.dxy = (uint32_t)(cx + dx) | ((uint32_t)(cy + dy) << 16);
    mv.key |= line_reach<V>(s, mv, step);
    return mover_reach(mv.key) > 0;
}

// sh_scan[MOVE_THREADS], sh_tp[GATHER_TILES_MAX], sh_kept: LDS of the kernel
// (declared there once, not per v_max).
template <int V>
__device__ __forceinline__ void move_group(const SlotDev &s, int g, int G, int step, bool alone,
                                           int *sh_scan, int *sh_tp, int &sh_kept)
{
    const int tid = threadIdx.x;
    const int T = s.ntx * s.nty, TC = s.tx * s.ty;
    const long cap = list_capacity(s, G);
    Mover *cur = s.mv_a + (long)g * cap, *nxt = s.mv_b + (long)g * cap;
    unsigned long long seen0 = 0, seen1 = 0;
    uint32_t tag = (uint32_t)s.ctr[C_TAG];
    // movers reserve round 0 as they are gathered unless the tags run out
    // first (then the arrays are wiped before the first reservation)
    const bool early0 = tag < TAG_LIMIT;
    const unsigned long long tagw0 = (unsigned long long)(tag + 1) << TAG_SHIFT;
    if (g == 0 && tid == 0)   // agents planned this step, for the throughput counters
        atomicAdd(&s.stat[S_PLANNED], (unsigned long long)s.ctr[C_NACTIVE]);
    // a trail field: this phase's deposits start from 0 (agent-scope stores,
    // complete before the first group barrier, after which movers commit)
    if (s.dep) {
        const long cells = (long)s.Wp * s.Hp;
        for (long i = cells * g / G + tid; i < cells * (g + 1) / G; i += blockDim.x)
            st_agent(&s.dep[i], 0);
        __builtin_amdgcn_s_waitcnt(0);   // (a one-workgroup barrier waits for none)
    }

    // gather this workgroup's movers from the planned records
    int n = 0;
    if (T <= GATHER_TILES_MAX) {
        // The records, numbered tile by tile, are split into equal runs: every
        // workgroup gets the same count, from neighbouring tiles (dealing
        // records out in turn instead balances regions, but scatters every
        // workgroup's memory accesses over the whole grid: slower).
        // Workgroups go to the device's DIES dies in turn; with G a multiple
        // of DIES, workgroup g takes only tiles t = g (mod DIES), so that
        // each die's workgroups share the records of one tile in DIES.
        const bool by_die = G % DIES == 0;
        const int c = by_die ? g % DIES : 0, stride = by_die ? DIES : 1;
        const int m = by_die ? G / DIES : G, w = by_die ? g / DIES : g;
        const int Tc = c < T ? (T - c + stride - 1) / stride : 0;   // tiles c, c + stride, ...
        int carry = 0;
        for (int j0 = 0; j0 < Tc; j0 += MOVE_THREADS) {
            const int nt = min(MOVE_THREADS, Tc - j0);
            sh_scan[tid] = tid < nt ? s.seg_cnt[c + (j0 + tid) * stride] : 0;
            block_scan(sh_scan);
            if (tid < nt) sh_tp[j0 + tid] = sh_scan[tid] + carry;
            carry += sh_scan[MOVE_THREADS - 1];
            __syncthreads();
        }
        const int r0 = (int)((long)carry * w / m), mine = (int)((long)carry * (w + 1) / m) - r0;
        if (tid == 0) sh_kept = 0;
        __syncthreads();
        for (int j0 = 0; j0 < mine; j0 += blockDim.x) {
            const int i = r0 + j0 + tid;
            Mover mv;
            bool keep = false;
            if (j0 + tid < mine) {
                int a = 0, b = Tc - 1;               // first tile whose inclusive count exceeds i
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (sh_tp[mid] > i) b = mid; else a = mid + 1;
                }
                const int k = i - (a ? sh_tp[a - 1] : 0);
                const int tile = c + a * stride;
                keep = gather_one<V>(s, s.seg[(long)tile * TC + k], tile, step, mv);
                if (keep && early0) reserve_reach<V>(s, s.res0, mv, tagw0);
            }
            append_kept(cur, n, keep, mv, &sh_kept);
        }
        __syncthreads();
        n = sh_kept;
        __syncthreads();
    } else {
        // very many tiles: workgroup g takes the records of a run of tiles,
        // t0 .. t1 - 1
        const int t0 = (int)((long)T * g / G), nt_g = (int)((long)T * (g + 1) / G) - t0;
        for (int j0 = 0; j0 < nt_g; j0 += MOVE_THREADS) {
            const int nt = min(MOVE_THREADS, nt_g - j0);
            sh_scan[tid] = tid < nt ? s.seg_cnt[t0 + j0 + tid] : 0;
            block_scan(sh_scan);
            const int chunk = sh_scan[MOVE_THREADS - 1];
            if (tid == 0) sh_kept = 0;
            __syncthreads();
            for (int i0 = 0; i0 < chunk; i0 += blockDim.x) {
                const int i = i0 + tid;
                Mover mv;
                bool keep = false;
                if (i < chunk) {
                    int a = 0, b = nt - 1;           // first tile whose inclusive count exceeds i
                    while (a < b) {
                        const int mid = (a + b) >> 1;
                        if (sh_scan[mid] > i) b = mid; else a = mid + 1;
                    }
                    const int k = i - (a ? sh_scan[a - 1] : 0);
                    const int tile = t0 + j0 + a;
                    keep = gather_one<V>(s, s.seg[(long)tile * TC + k], tile, step, mv);
                    if (keep && early0) reserve_reach<V>(s, s.res0, mv, tagw0);
                }
                append_kept(cur, n, keep, mv, &sh_kept);
            }
            __syncthreads();
            n += sh_kept;
            __syncthreads();
        }
    }

    int total = 1, rounds = 0, bar_r = 0;          // round 0's total comes from its barrier
    int Gr = G;                                    // workgroups still in the phase
    // A launch that moves one scenario invalidates the caches of its dies at
    // each group barrier and reads with cacheable loads; in a batch those
    // invalidations would evict every other scenario's lines from the dies'
    // L2s, so batches read with agent-scope loads instead.
    bool acq = false;                              // the last barrier ended with an acquire
    for (int r = 0; total > 0; ++r) {
        unsigned long long *res = (r & 1) ? s.res1 : s.res0;
        // this round's reservations made already: by the gather (round 0) or
        // by the losers as they failed their checks (later rounds); not when
        // the tags must be restarted first
        bool reserved = r == 0 && early0;
        if (r > 0) {
            // round r's movers are the losers of round r - 1 (this workgroup's share)
            const bool merge = tag < TAG_LIMIT;
            n = commit_list<V>(s, (r & 1) ? s.res0 : s.res1, cur, nxt, n,
                               (unsigned long long)tag << TAG_SHIFT, acq, merge ? res : nullptr,
                               (unsigned long long)(tag + 1) << TAG_SHIFT);
            Mover *t = cur; cur = nxt; nxt = t;
            reserved = merge;
        }
        if (tag >= TAG_LIMIT) {
            // tags are exhausted: once every check of the last round is done,
            // wipe both reservation arrays and restart the tags at 1
            if (group_sync_count(s, Gr, bar_r++, 0, seen0, seen1) < 0) return;
            const long cells = (long)s.Wp * s.Hp;
            for (long i = cells * g / Gr + tid; i < cells * (g + 1) / Gr; i += blockDim.x) {
                __hip_atomic_store(&s.res0[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&s.res1[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            tag = 0;
            if (group_sync_count(s, Gr, bar_r++, 0, seen0, seen1) < 0) return;
        }
        ++tag;
        if (!reserved) reserve_list<V>(s, res, cur, n, (unsigned long long)tag << TAG_SHIFT);
        if (Gr > 1 && n <= MOVE_SOLO_MAX) {         // workgroup 0 may take these over
            Mover *h = s.hand + (long)g * MOVE_SOLO_MAX;
            for (int i = tid; i < n; i += blockDim.x) {
                const Mover mv = cur[i];
                __hip_atomic_store(&h[i].key, mv.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&h[i].cxy, mv.cxy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&h[i].dxy, mv.dxy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (Gr > 1 && tid == 0) st_agent(&s.ctr[C_SOLO + g], n);
        total = group_sync_count(s, Gr, bar_r++, n, seen0, seen1, alone);
        acq = alone && Gr > 1;
        if (total < 0) return;
        rounds += total > 0 ? 1 : 0;
        if (Gr > 1 && total > 0 && total <= MOVE_SOLO_MAX) {
            // the same decision in every workgroup (total is the group's sum)
            if (g != 0) return;
            n = gather_lists(s, G, s.mv_a, sh_scan);    // workgroup 0's lists start at 0
            cur = s.mv_a;
            nxt = s.mv_b;
            Gr = 1;
        }
    }
    if (g == 0 && tid == 0) {
        s.ctr[C_TAG] = (int)tag;
        s.ctr[C_ROUNDS] = rounds;
        s.ctr[C_STEP] = step + 1;
    }
}

// mitems[i] = slot | g << 12 | (G - 1) << 22 | alone << 31: workgroup g of
// the G that move the slot's agents; alone: the launch moves this scenario
// only.
__global__ __launch_bounds__(MOVE_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void move_kernel(const SlotDev *__restrict__ table,
                                                            const uint32_t *__restrict__ mitems)
{
    const uint32_t it = mitems[blockIdx.x];
    const SlotDev &s = table[it & 0xFFFu];
    const int g = (int)((it >> 12) & 0x3FFu);
    const int G = (int)((it >> 22) & 0x1FFu) + 1;
    const bool alone = (it >> 31) != 0;
    const int step = s.ctr[C_STEP];
    if (step >= s.ctr[C_LIMIT]) return;
    __shared__ int sh_scan[MOVE_THREADS];
    __shared__ int sh_tp[GATHER_TILES_MAX];
    __shared__ int sh_kept;
    switch (s.v) {
        case 1: move_group<1>(s, g, G, step, alone, sh_scan, sh_tp, sh_kept); break;
        case 2: move_group<2>(s, g, G, step, alone, sh_scan, sh_tp, sh_kept); break;
        case 3: move_group<3>(s, g, G, step, alone, sh_scan, sh_tp, sh_kept); break;
        case 4: move_group<4>(s, g, G, step, alone, sh_scan, sh_tp, sh_kept); break;
        case 5: move_group<5>(s, g, G, step, alone, sh_scan, sh_tp, sh_kept); break;
        default: break;
    }
}

}  // namespace fk

extern "C" hipError_t fk_launch_move(const fk::SlotDev *table, const uint32_t *mitems, int n_items,
                                     hipStream_t stream)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk::move_kernel, dim3(n_items), dim3(fk::MOVE_THREADS), 0, stream, table,
                       mitems);
    return hipGetLastError();
}

// Motion workgroups one CU holds at once.
extern "C" hipError_t fk_move_per_cu(int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fk::move_kernel, fk::MOVE_THREADS,
                                                        0);
}

