// builder.cpp -- host-side scenario setup for libfast: validation, the exact
// static floor field, seeded placement, the padded grid, and the per-tile
// FP32 exp table with its fallback flags.
//
// Floor field (paper Sec. 2 fixes k_S and the exp coupling; the field itself
// is the model's static distance-to-exit potential): shortest walking length
// from the nearest exit cell over the 8-neighbour stencil, orthogonal step 1,
// diagonal step sqrt 2, a diagonal allowed only when both orthogonal
// neighbours are not walls.  Lengths are kept exactly as a + b sqrt 2 with
// integers a, b -- sqrt 2 is irrational, so the shortest pair of a cell is
// unique -- and S = fl(fl(b * sqrt2) + a), a value that does not depend on the
// order in which the search visits cells.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include "fast_dev.h"
#include "fast_host.h"

namespace fh {

namespace {

constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;   // nearest double to sqrt 2
constexpr double kLn2 = 0x1.62e42fefa39efp-1;     // nearest double to ln 2
constexpr double kRange = 80.0;                   // |exponent| bound of a table entry

// Sign of p + q sqrt 2 for integers p, q.
int sign_z2(int64_t p, int64_t q)
{
    if (q == 0) return (p > 0) - (p < 0);
    if (p == 0) return (q > 0) - (q < 0);
    if ((p > 0) == (q > 0)) return p > 0 ? 1 : -1;
    const int64_t pp = p * p, qq = 2 * q * q;     // opposite signs: compare magnitudes
    if (p > 0) return pp > qq ? 1 : -1;
    return pp > qq ? -1 : 1;
}

struct Len {
    int64_t a = -1, b = -1;                       // a + b sqrt 2; a < 0 = unreached
    bool reached() const { return a >= 0; }
};

bool shorter(const Len &x, const Len &y) { return sign_z2(x.a - y.a, x.b - y.b) < 0; }

struct QItem {
    Len len;
    int32_t cell;
};
struct QAfter {
    bool operator()(const QItem &x, const QItem &y) const
    {
        if (shorter(y.len, x.len)) return true;
        if (shorter(x.len, y.len)) return false;
        return x.cell > y.cell;
    }
};

}  // namespace

// Exact floor field on the unpadded grid; unreachable free cells become walls.
// With exit_field given, the field of exit group g alone: only the exits
// tagged g are sources, type is left as it is, and cells those exits do not
// reach get +inf.
void floor_field(int W, int H, std::vector<uint8_t> &type, std::vector<double> &S,
                 const uint8_t *exit_field, int g)
{
    const int64_t n = (int64_t)W * H;
    std::vector<Len> L((size_t)n);
    std::vector<char> settled((size_t)n, 0);
    std::priority_queue<QItem, std::vector<QItem>, QAfter> q;
    for (int64_t i = 0; i < n; ++i)
        if (type[i] == fk::CELL_EXIT && (!exit_field || exit_field[i] == g)) {
            L[i].a = 0;
            L[i].b = 0;
            q.push({L[i], (int32_t)i});
        }
    static const int ddx[8] = {1, -1, 0, 0, 1, 1, -1, -1};
    static const int ddy[8] = {0, 0, 1, -1, 1, -1, 1, -1};
    while (!q.empty()) {
        const QItem it = q.top();
        q.pop();
        const int32_t c = it.cell;
        if (settled[c] || it.len.a != L[c].a || it.len.b != L[c].b) continue;
        settled[c] = 1;
        const int cx = c % W, cy = c / W;
        for (int k = 0; k < 8; ++k) {
            const int nx = cx + ddx[k], ny = cy + ddy[k];
            if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
            const int64_t t = (int64_t)ny * W + nx;
            if (type[t] == fk::CELL_WALL || settled[t]) continue;
            Len cand = L[c];
            if (k >= 4) {
                if (type[(int64_t)cy * W + nx] == fk::CELL_WALL ||
                    type[(int64_t)ny * W + cx] == fk::CELL_WALL)
                    continue;
                cand.b += 1;
            } else {
                cand.a += 1;
            }
            if (!L[t].reached() || shorter(cand, L[t])) {
                L[t] = cand;
                q.push({cand, (int32_t)t});
            }
        }
    }
    S.assign((size_t)n, INFINITY);
    for (int64_t i = 0; i < n; ++i) {
        if (!exit_field && type[i] == fk::CELL_FREE && !L[i].reached()) type[i] = fk::CELL_WALL;
        if (type[i] != fk::CELL_WALL && L[i].reached()) {
            const double bs = (double)L[i].b * kSqrt2;
            S[i] = bs + (double)L[i].a;
        }
    }
}

// Seeded placement: partial Fisher-Yates over the eligible cells (free and
// reachable) in raster order, index k + ((x0 * (M - k)) >> 32) with x0 word 0
// of Philox at counter (k, 0, scenario, 2).
bool place(int W, int H, const std::vector<uint8_t> &type, int n, uint64_t seed, uint32_t scn,
           std::vector<int32_t> &xy)
{
    std::vector<int32_t> cells;
    cells.reserve((size_t)W * H);
    for (int64_t i = 0; i < (int64_t)W * H; ++i)
        if (type[i] == fk::CELL_FREE) cells.push_back((int32_t)i);
    const int64_t M = (int64_t)cells.size();
    if (n > M) return false;
    xy.resize((size_t)2 * n);
    for (int k = 0; k < n; ++k) {
        const uint32_t r = fk::philox_word0((uint32_t)k, 0u, scn, fk::STREAM_PLACE, (uint32_t)seed,
                                            (uint32_t)(seed >> 32));
        const int64_t j = k + (int64_t)(((uint64_t)r * (uint64_t)(M - k)) >> 32);
        std::swap(cells[k], cells[j]);
        xy[2 * k] = cells[k] % W;
        xy[2 * k + 1] = cells[k] / W;
    }
    return true;
}

// Rounding-depth bound of the FP32 CDF: rows are pairwise sums (depth
// ceil(log2(2v+1))), row prefixes and in-row prefixes sequential; a CDF value
// and W each carry at most d + 1 roundings (d additions plus the table entry),
// tau one more.  A draw whose |tau - C| exceeds (d_W + d_C + 3) u W decides
// the same way in exact arithmetic; the band adds 25 % and is never below the
// 1e-6 W the method asks for (1.01e-6, so that the float band and its product
// with W stay above 1e-6 W after rounding).
float guard_band(int v)
{
    int dR = 0;
    while ((1 << dR) < 2 * v + 1) ++dR;
    const int d = dR + 2 * v;
    const double band = 1.25 * (2.0 * d + 3.0) * 0x1p-24;
    return (float)std::max(1.01e-6, band);
}

std::vector<uint8_t> cell_bytes(const Built &b)
{
    const int Wp = b.Wp, Hp = b.Hp;
    auto wall = [&](int x, int y) {
        return x < 0 || y < 0 || x >= Wp || y >= Hp || b.type[(size_t)y * Wp + x] == fk::CELL_WALL;
    };
    std::vector<uint8_t> out(b.type.size());
    for (int y = 0; y < Hp; ++y)
        for (int x = 0; x < Wp; ++x) {
            uint32_t c = b.type[(size_t)y * Wp + x];
            // a diagonal step (sx, sy) into (x, y) comes from (x - sx, y - sy);
            // it cuts a corner if (x, y - sy) or (x - sx, y) is a wall
            for (int sx = -1; sx <= 1; sx += 2)
                for (int sy = -1; sy <= 1; sy += 2)
                    if (wall(x, y - sy) || wall(x - sx, y)) c |= 1u << fk::cut_bit(sx, sy);
            out[(size_t)y * Wp + x] = (uint8_t)c;
        }
    return out;
}

// The FP32 exp table of one floor field S (padded layout of b): per tile T
// the scale m_T = round(k_S * mid(S over T's window) / ln 2), every cell's
// entry G = fl32(exp(m_T ln 2 - k_S S)) in the scale of its own tile (0 for
// walls, unreachable cells and entries beyond e^+-80), and the fallback flag
// of every tile whose window holds a reachable cell outside [e^-80, e^80] in
// the tile's scale.
void exp_table(const Built &b, const double *S, double ks, std::vector<float> &G,
               std::vector<int32_t> &tile_m, std::vector<uint8_t> &tile_fb, int &n_fb)
{
    const int v = b.v, tx = b.tx, ty = b.ty, pad = b.pad;
    const int64_t np = (int64_t)b.Wp * b.Hp;
    const int ts = b.ntx + 2;
    G.assign((size_t)np, 0.0f);
    tile_m.assign((size_t)ts * (b.nty + 2), 0);
    std::vector<int32_t> mcell((size_t)np, 0);
    for (int j = 0; j < b.nty; ++j)
        for (int i = 0; i < b.ntx; ++i) {
            double lo = INFINITY, hi = -INFINITY;
            for (int y = j * ty + pad - v; y < j * ty + pad + ty + v; ++y)
                for (int x = i * tx + pad - v; x < i * tx + pad + tx + v; ++x) {
                    const double s = S[(int64_t)y * b.Wp + x];
                    if (std::isfinite(s)) { lo = std::min(lo, s); hi = std::max(hi, s); }
                }
            int32_t m = 0;
            if (lo <= hi) m = (int32_t)std::llround(ks * 0.5 * (lo + hi) / kLn2);
            tile_m[(size_t)(j + 1) * ts + i + 1] = m;
            for (int y = j * ty + pad; y < j * ty + ty + pad; ++y)
                for (int x = i * tx + pad; x < i * tx + tx + pad; ++x) mcell[(int64_t)y * b.Wp + x] = m;
        }
    // table entries in the scale of their own tile
    std::vector<char> cell_ok((size_t)np, 1);
    for (int64_t g = 0; g < np; ++g) {
        const double s = S[g];
        if (!std::isfinite(s)) continue;
        const double ex = (double)mcell[g] * kLn2 - ks * s;
        if (std::fabs(ex) > kRange) { cell_ok[g] = 0; continue; }
        G[g] = (float)std::exp(ex);
    }
    // fallback tiles: some window cell outside [e^-80, e^80] in the tile's scale
    tile_fb.assign((size_t)b.ntx * b.nty, 0);
    n_fb = 0;
    for (int j = 0; j < b.nty; ++j)
        for (int i = 0; i < b.ntx; ++i) {
            const int32_t m = tile_m[(size_t)(j + 1) * ts + i + 1];
            bool ok = true;
            for (int y = j * ty + pad - v; ok && y < j * ty + pad + ty + v; ++y)
                for (int x = i * tx + pad - v; x < i * tx + pad + tx + v; ++x) {
                    const int64_t g = (int64_t)y * b.Wp + x;
                    const double s = S[g];
                    if (!std::isfinite(s)) continue;
                    if (!cell_ok[g] || std::fabs((double)m * kLn2 - ks * s) > kRange) { ok = false; break; }
                }
            if (!ok) { tile_fb[(size_t)j * b.ntx + i] = 1; ++n_fb; }
        }
}

int build_scenario(const fast_scenario_desc &d, int tx, int ty, Built &b, std::string &err)
{
    const int W = d.width, H = d.height, v = d.v_max;
    b = Built();
    b.W = W; b.H = H; b.v = v; b.tx = tx; b.ty = ty;
    std::vector<uint8_t> type(d.cell_type, d.cell_type + (size_t)W * H);
    bool any_exit = false;
    for (uint8_t t : type) {
        if (t > fk::CELL_EXIT) { err = "cell_type values must be 0, 1 or 2"; return FAST_E_INVALID; }
        any_exit = any_exit || t == fk::CELL_EXIT;
    }
    if (!any_exit) { err = "the grid has no exit cell"; return FAST_E_INVALID; }

    std::vector<double> S;
    floor_field(W, H, type, S);

    std::vector<int32_t> xy;
    if (d.agent_xy) {
        xy.assign(d.agent_xy, d.agent_xy + (size_t)2 * d.n_agents);
        std::vector<char> used((size_t)W * H, 0);
        for (int i = 0; i < d.n_agents; ++i) {
            const int x = xy[2 * i], y = xy[2 * i + 1];
            if (x < 0 || y < 0 || x >= W || y >= H) { err = "an agent lies off the grid"; return FAST_E_INVALID; }
            const int64_t c = (int64_t)y * W + x;
            if (type[c] != fk::CELL_FREE) { err = "an agent stands on a wall, an exit or an unreachable cell"; return FAST_E_INVALID; }
            if (used[c]) { err = "two agents share a cell"; return FAST_E_INVALID; }
            used[c] = 1;
        }
    } else if (!place(W, H, type, d.n_agents, d.seed, d.scenario_id, xy)) {
        err = "more agents than eligible cells";
        return FAST_E_INVALID;
    }
    if (d.agent_v) {
        b.vi.assign(d.agent_v, d.agent_v + d.n_agents);
        for (uint8_t s : b.vi)
            if (s < 1 || s > v) { err = "agent_v values must lie in 1..v_max"; return FAST_E_INVALID; }
    }
    // several floor fields: one per exit group, agent i follows agent_field[i]
    const int nf = d.n_fields;
    std::vector<std::vector<double>> fields;
    if (nf < 0 || nf > 8) { err = "n_fields must lie in 0..8"; return FAST_E_INVALID; }
    if (nf >= 2) {
        if (!d.exit_field || (!d.agent_field && d.n_agents > 0)) {
            err = "n_fields >= 2 needs exit_field and (with agents) agent_field";
            return FAST_E_INVALID;
        }
        std::vector<int> exits((size_t)nf, 0);
        for (int64_t i = 0; i < (int64_t)W * H; ++i)
            if (type[i] == fk::CELL_EXIT) {
                if (d.exit_field[i] >= nf) { err = "exit_field values must lie in 0..n_fields-1"; return FAST_E_INVALID; }
                ++exits[d.exit_field[i]];
            }
        for (int g = 0; g < nf; ++g)
            if (!exits[g]) { err = "every floor field needs an exit cell"; return FAST_E_INVALID; }
        fields.resize((size_t)nf);
        for (int g = 0; g < nf; ++g) floor_field(W, H, type, fields[g], d.exit_field, g);
        if (d.n_agents > 0) b.fi.assign(d.agent_field, d.agent_field + d.n_agents);
        for (int i = 0; i < d.n_agents; ++i) {
            if (b.fi[i] >= nf) { err = "agent_field values must lie in 0..n_fields-1"; return FAST_E_INVALID; }
            const int64_t c = (int64_t)xy[2 * i + 1] * W + xy[2 * i];
            if (!std::isfinite(fields[b.fi[i]][c])) { err = "an agent stands where its floor field does not reach"; return FAST_E_INVALID; }
        }
    }

    // padded layout
    b.ntx = (W + tx - 1) / tx;
    b.nty = (H + ty - 1) / ty;
    // a wall border of pad = round4(v) cells (the planning kernel stages whole
    // 4-cell chunks, each inside one tile column), rows padded to 32 cells
    const int pad = (v + 3) / 4 * 4;
    b.pad = pad;
    b.Wp = (b.ntx * tx + 2 * pad + 31) / 32 * 32;
    b.Hp = b.nty * ty + 2 * pad;
    const int64_t np = (int64_t)b.Wp * b.Hp;
    b.type.assign((size_t)np, fk::CELL_WALL);
    b.S.assign((size_t)np, INFINITY);
    b.occ.assign((size_t)np, -1);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int64_t g = (int64_t)(y + pad) * b.Wp + (x + pad);
            b.type[g] = type[(int64_t)y * W + x];
            b.S[g] = S[(int64_t)y * W + x];
        }
    if (nf >= 2) {
        b.Sf.assign((size_t)nf * np, INFINITY);
        for (int g = 0; g < nf; ++g)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x)
                    b.Sf[(size_t)g * np + (size_t)(y + pad) * b.Wp + (x + pad)] = fields[g][(int64_t)y * W + x];
    }
    b.n = d.n_agents;
    b.pos.resize((size_t)b.n);
    for (int i = 0; i < b.n; ++i) {
        const int64_t g = (int64_t)(xy[2 * i + 1] + pad) * b.Wp + (xy[2 * i] + pad);
        b.pos[i] = (int32_t)g;
        b.occ[g] = i;
    }

    exp_table(b, b.S.data(), d.k_s, b.G, b.tile_m, b.tile_fb, b.n_fb);
    // several fields: one table per field, each with its own tile scales and
    // fallback flags
    if (nf >= 2) {
        b.Gf.resize((size_t)nf * np);
        b.tile_mf.resize((size_t)nf * (b.ntx + 2) * (b.nty + 2));
        b.tile_fbf.resize((size_t)nf * b.ntx * b.nty);
        b.n_fbf = 0;
        for (int g = 0; g < nf; ++g) {
            std::vector<float> G;
            std::vector<int32_t> tm;
            std::vector<uint8_t> fb;
            int nfb = 0;
            exp_table(b, b.Sf.data() + (size_t)g * np, d.k_s, G, tm, fb, nfb);
            std::copy(G.begin(), G.end(), b.Gf.begin() + (size_t)g * np);
            std::copy(tm.begin(), tm.end(), b.tile_mf.begin() + (size_t)g * tm.size());
            std::copy(fb.begin(), fb.end(), b.tile_fbf.begin() + (size_t)g * fb.size());
            b.n_fbf += nfb;
        }
    }
    b.eps = guard_band(v);
    return FAST_OK;
}

}  // namespace fh
