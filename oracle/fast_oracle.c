/*
 * fast_oracle.c -- plain CPU oracle of one F.A.S.T. time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product library
 * (libfast) neither links nor includes it, and this file includes nothing of
 * the product: the two share no code, table or constant generator.
 *
 * Paper: T. Kretz, "Computation Speed of the F.A.S.T. Model", arXiv:0911.2900.
 *  - Sec. 1: a time step is a planning phase, in which every agent picks a
 *    desired cell while shared data is only read (this phase holds the costly
 *    exp evaluations and is the parallel part), followed by a motion phase in
 *    which the agents move one after another with simple operations that
 *    write the shared structures.  At most one agent per cell.
 *  - Sec. 2: k_S = 1.2, k_other = 0, the same maximum speed v_m for all
 *    agents (v_m = 1..5), 396 steps of one simulated second; the only parallel
 *    loop calls choose_desired_cell(i) for every agent i.
 *
 * Everything below is double precision, single threaded (apart from a
 * threaded copy of the planning loop for the CPU baseline, which gives the
 * same draws), and written to be read against the model rather than to be
 * fast.
 *
 * The paper does not restate the model's formulas; where it is silent this
 * file takes these readings (each function names the one it implements):
 *  R1  reach set: cells t = c + (dx, dy) with dx^2 + dy^2 <= v_m^2 inside the
 *      grid, not a wall, and free in the step's start snapshot -- the agent's
 *      own cell is always a candidate.
 *  R2  weight w(t) = exp(k_S * (S(c) - S(t))), S in cell units, so cells
 *      closer to an exit are preferred; k_other = 0 makes every other factor 1.
 *  R3  draw: candidates in raster order (dy outer, dx inner, both from -v_m),
 *      sequential prefix sum C, W = last C, u = (x0 >> 8) * 2^-24 from
 *      Philox4x32-10 word 0 at counter (agent, step, scenario, 0) and key
 *      (seed low, seed high); the choice is the first t with u*W < C_t.
 *  R4  motion order: ascending (x0 of Philox at counter (agent, step,
 *      scenario, 1), agent id), drawn afresh each step.
 *  R5  motion path: DDA line p_k = c + (sgn dx * floor((2k|dx| + m)/(2m)),
 *      sgn dy * floor((2k|dy| + m)/(2m))), k = 1..m, m = max(|dx|,|dy|); the
 *      agent stops before a wall, before an occupied cell, and before a
 *      diagonal step whose two orthogonal neighbours are not both non-wall.
 *  R6  exits sit in the border; entering one removes the agent at once.
 *  R7  floor field: Dijkstra from every exit cell over 8 neighbours,
 *      orthogonal step 1, diagonal step sqrt 2 (only if both orthogonal
 *      neighbours are non-wall); lengths are kept exactly as a + b*sqrt 2 and
 *      S = fl(fl(b * sqrt2) + a); free cells that no exit reaches become walls.
 *  R8  seeded placement: partial Fisher-Yates over the eligible cells (free,
 *      reachable) in raster order with j = k + ((x0 * (M - k)) >> 32), x0 from
 *      Philox at counter (k, 0, scenario, 2).
 *  R13 several floor fields (route choice, counterflow; Sec. 3 names richer
 *      situations as the next cost driver): field g is R7's exact field from
 *      the exit cells tagged g alone, +inf where those exits do not reach;
 *      agent i weighs its window with its own field in R2; walls stay those
 *      of R7 (all exits), and R6 removes an agent at any exit cell.
 *  R14 dynamic floor field (one of the couplings k_other that Sec. 2 sets to
 *      0; the paper cites its definition without restating it): every cell
 *      holds a trail value T >= 0, zero at the start.  An agent that leaves
 *      the cell it started the step on (it moves, or it exits) adds 1 to that
 *      cell's deposit count during the motion phase.  After the motion phase
 *      every non-wall cell takes T' = (1 - delta) * ((1 - alpha) * T +
 *      (alpha / 8) * N) + deposits, N the sum of T over its 8 neighbours in
 *      raster order (walls and cells off the grid count 0); walls keep 0; the
 *      deposits restart at 0.  R2's weight becomes w(t) = exp(k_S * (S(c) -
 *      S(t)) + k_D * (T(t) - T(c))): agents lean towards cells others have
 *      just left.  k_D = 0 leaves R2's weights unchanged bit for bit.
 *
 * Philox4x32-10 follows its published definition: J. K. Salmon, M. A. Moraes,
 * R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11 (the Philox S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and the
 * Weyl key schedule 0x9E3779B9 / 0xBB67AE85).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <pthread.h>
#include <stdatomic.h>
#include <unistd.h>

enum { CELL_FREE = 0, CELL_WALL = 1, CELL_EXIT = 2 };

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11).                                      */
/* ------------------------------------------------------------------------- */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {           /* key schedule: add the Weyl constants */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word 0 of Philox4x32-10 at counter (a, b, c, d) with a 64-bit seed key. */
static uint32_t philox_x0(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint64_t seed)
{
    uint32_t ctr[4] = { a, b, c, d };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[0];
}

/* ------------------------------------------------------------------------- */
/* Floor field (reading R7).                                                 */
/* ------------------------------------------------------------------------- */

/* Is a1 + b1*sqrt2 < a2 + b2*sqrt2 ?  Exact: sqrt 2 is irrational, so the
 * sign of p + q*sqrt2 (p = a1 - a2, q = b1 - b2) follows from the signs of p
 * and q, or, when they differ, from comparing p^2 with 2 q^2. */
static int zlen_less(int64_t a1, int64_t b1, int64_t a2, int64_t b2)
{
    int64_t p = a1 - a2, q = b1 - b2;
    if (p <= 0 && q <= 0) return (p < 0 || q < 0);
    if (p >= 0 && q >= 0) return 0;
    if (p < 0) return p * p > 2 * q * q;      /* q > 0: negative iff |p| > q*sqrt2 */
    return 2 * q * q > p * p;                 /* p > 0, q < 0                     */
}

typedef struct { int64_t a, b; int32_t cell; } heap_item;

static int item_less(const heap_item *x, const heap_item *y)
{
    if (zlen_less(x->a, x->b, y->a, y->b)) return 1;
    if (zlen_less(y->a, y->b, x->a, x->b)) return 0;
    return x->cell < y->cell;
}

static void heap_push(heap_item *h, int64_t *n, heap_item it)
{
    int64_t i = (*n)++;
    h[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!item_less(&h[i], &h[p])) break;
        heap_item t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, int64_t *n)
{
    heap_item top = h[0];
    h[0] = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && item_less(&h[l], &h[m])) m = l;
        if (r < *n && item_less(&h[r], &h[m])) m = r;
        if (m == i) break;
        heap_item t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

/*
 * Static floor field by Dijkstra from all exit cells (reading R7).
 * type  : W*H cell types (0 free, 1 wall, 2 exit), row-major y*W + x; free
 *         cells that no exit reaches are turned into walls in place.
 * S     : out, W*H doubles; +inf on walls.
 * a_out, b_out : out (may be NULL), exact length a + b*sqrt2; -1 on walls.
 * Returns 0, or -1 on bad input / allocation failure.
 */
/* Shortest exact lengths A + B*sqrt2 from the source exits (all exit cells
 * when ef is NULL, else those with ef[cell] == g) to every cell; -1 where no
 * source reaches. */
static int exit_lengths(int32_t W, int32_t H, const uint8_t *type, const uint8_t *ef,
                        int32_t g, int64_t *A, int64_t *B)
{
    int64_t n = (int64_t)W * H;
    uint8_t *done = calloc((size_t)n, 1);
    /* each cell is pushed at most once per improvement; 8 improvements bound it */
    heap_item *heap = malloc(sizeof(heap_item) * (size_t)(9 * n + 1));
    if (!done || !heap) { free(done); free(heap); return -1; }
    int64_t hn = 0;
    for (int64_t i = 0; i < n; ++i) {
        A[i] = -1; B[i] = -1;
        if (type[i] == CELL_EXIT && (!ef || ef[i] == g)) {
            A[i] = 0; B[i] = 0;
            heap_item it = { 0, 0, (int32_t)i };
            heap_push(heap, &hn, it);
        }
    }
    while (hn > 0) {
        heap_item it = heap_pop(heap, &hn);
        int32_t c = it.cell;
        if (done[c]) continue;
        if (it.a != A[c] || it.b != B[c]) continue;   /* stale entry */
        done[c] = 1;
        int32_t cx = c % W, cy = c / W;
        for (int dy = -1; dy <= 1; ++dy) {
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                int32_t nx = cx + dx, ny = cy + dy;
                if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
                int64_t t = (int64_t)ny * W + nx;
                if (type[t] == CELL_WALL) continue;
                int64_t na = A[c], nb = B[c];
                if (dx != 0 && dy != 0) {
                    /* diagonal: both orthogonal neighbours must be non-wall */
                    if (type[(int64_t)cy * W + nx] == CELL_WALL) continue;
                    if (type[(int64_t)ny * W + cx] == CELL_WALL) continue;
                    nb += 1;
                } else {
                    na += 1;
                }
                if (done[t]) continue;
                if (A[t] < 0 || zlen_less(na, nb, A[t], B[t])) {
                    A[t] = na; B[t] = nb;
                    heap_item nt = { na, nb, (int32_t)t };
                    heap_push(heap, &hn, nt);
                }
            }
        }
    }
    free(done); free(heap);
    return 0;
}

int oracle_floor_field(int32_t W, int32_t H, uint8_t *type, double *S,
                       int64_t *a_out, int64_t *b_out)
{
    if (W <= 0 || H <= 0) return -1;
    int64_t n = (int64_t)W * H;
    int64_t *A = malloc(sizeof(int64_t) * n), *B = malloc(sizeof(int64_t) * n);
    if (!A || !B || exit_lengths(W, H, type, NULL, 0, A, B) != 0) { free(A); free(B); return -1; }
    const double sqrt2 = sqrt(2.0);   /* correctly rounded: nearest double to sqrt 2 */
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] == CELL_FREE && A[i] < 0) type[i] = CELL_WALL;   /* unreachable */
        if (type[i] == CELL_WALL) {
            S[i] = INFINITY;
            if (a_out) a_out[i] = -1;
            if (b_out) b_out[i] = -1;
        } else {
            double bs = (double)B[i] * sqrt2;
            S[i] = bs + (double)A[i];
            if (a_out) a_out[i] = A[i];
            if (b_out) b_out[i] = B[i];
        }
    }
    free(A); free(B);
    return 0;
}

/*
 * Floor field g of a scenario with several fields (route choice, counterflow:
 * each group of agents heads for its own exits).  The same exact Dijkstra
 * lengths as R7, from the exit cells with exit_field[cell] == g only; type is
 * the grid after oracle_floor_field (read, not changed).  Cells that field g
 * does not reach get +inf, like walls.  Returns 0, or -1 on bad input.
 */
int oracle_floor_field_of(int32_t W, int32_t H, const uint8_t *type, const uint8_t *exit_field,
                          int32_t g, double *S)
{
    if (W <= 0 || H <= 0 || !exit_field) return -1;
    int64_t n = (int64_t)W * H;
    int64_t *A = malloc(sizeof(int64_t) * n), *B = malloc(sizeof(int64_t) * n);
    if (!A || !B || exit_lengths(W, H, type, exit_field, g, A, B) != 0) { free(A); free(B); return -1; }
    const double sqrt2 = sqrt(2.0);
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] == CELL_WALL || A[i] < 0) S[i] = INFINITY;
        else S[i] = (double)B[i] * sqrt2 + (double)A[i];
    }
    free(A); free(B);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Seeded placement (reading R8).                                            */
/* ------------------------------------------------------------------------- */

/* Places agents 0..n-1; x, y out.  Returns 0, or -1 if n exceeds the number
 * of eligible cells. */
int oracle_place(int32_t W, int32_t H, const uint8_t *type, const double *S,
                 int32_t n, uint64_t seed, uint32_t scn, int32_t *x, int32_t *y)
{
    int64_t cells = (int64_t)W * H, M = 0;
    int32_t *L = malloc(sizeof(int32_t) * (size_t)(cells > 0 ? cells : 1));
    if (!L) return -1;
    for (int64_t i = 0; i < cells; ++i)
        if (type[i] == CELL_FREE && isfinite(S[i])) L[M++] = (int32_t)i;
    if (n < 0 || n > M) { free(L); return -1; }
    for (int32_t k = 0; k < n; ++k) {
        uint32_t r = philox_x0((uint32_t)k, 0u, scn, 2u, seed);
        int64_t j = k + (int64_t)(((uint64_t)r * (uint64_t)(M - k)) >> 32);
        int32_t t = L[k]; L[k] = L[j]; L[j] = t;
        x[k] = L[k] % W;
        y[k] = L[k] / W;
    }
    free(L);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Model state.                                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t W, H;
    const uint8_t *type;    /* W*H, after oracle_floor_field                       */
    const double *S;        /* W*H floor field                                     */
    int32_t v;              /* v_m, 1..5                                           */
    double k_s;             /* k_S                                                 */
    uint64_t seed;
    uint32_t scn;           /* scenario id (Philox counter word 2)                 */
    int32_t step;           /* next step number, starts at 0                       */
    int32_t n;              /* agents, ids 0..n-1                                  */
    int32_t *x, *y;         /* positions; -1 once the agent has left               */
    uint8_t *alive;
    int32_t *desired;       /* y*W + x of the planned cell; -1 when not alive      */
    int32_t *occ;           /* W*H: -1 free, else the id of the agent on the cell  */
    int64_t exited;
    const uint8_t *vi;      /* optional, n: agent i's own maximum speed (1..v); NULL:
                               every agent has v.  The window stays (2v+1)^2; agent i
                               reaches the cells of its own disc dx^2 + dy^2 <= vi^2 */
    const double *Sf;       /* optional: several floor fields, W*H each, one after
                               another (oracle_floor_field_of)                      */
    const uint8_t *fi;      /* optional, n: the field agent i follows; NULL: every
                               agent follows S                                      */
    double *Tr;             /* optional, W*H: the trail field of R14; NULL: none  */
    int32_t *dep;           /* W*H deposit counts of the running motion phase (with Tr) */
    double k_d, decay, diffusion;  /* R14's k_D, delta, alpha                      */
} oracle_state;

/* Rebuilds occupancy from positions; returns -1 if an agent is off-grid, on
 * a wall or exit, or shares a cell. */
int oracle_reset_occ(oracle_state *st)
{
    int64_t cells = (int64_t)st->W * st->H;
    for (int64_t i = 0; i < cells; ++i) st->occ[i] = -1;
    for (int32_t i = 0; i < st->n; ++i) {
        if (!st->alive[i]) { st->desired[i] = -1; continue; }
        int32_t px = st->x[i], py = st->y[i];
        if (px < 0 || py < 0 || px >= st->W || py >= st->H) return -1;
        int64_t c = (int64_t)py * st->W + px;
        if (st->type[c] != CELL_FREE) return -1;
        if (st->occ[c] != -1) return -1;
        st->occ[c] = i;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Planning phase: choose_desired_cell (readings R1-R3).                     */
/* ------------------------------------------------------------------------- */

/*
 * Plans agent i against the current state (the step's start snapshot).
 * w_out    : optional, (2v+1)^2 weights in raster order (0 outside the reach set).
 * c_out    : optional, (2v+1)^2 prefix sums C in the same order.
 * u_out    : optional, the uniform u.
 * slot_out : optional, chosen raster slot (dy+v)*(2v+1) + (dx+v).
 * Returns the linear cell y*W + x of the desired cell, or -1 if i is not alive.
 */
int32_t oracle_plan_agent(const oracle_state *st, int32_t i, double *w_out,
                          double *c_out, double *u_out, int32_t *slot_out)
{
    if (!st->alive[i]) return -1;
    const int32_t v = st->v, side = 2 * v + 1, W = st->W, H = st->H;
    const int32_t vr = st->vi ? st->vi[i] : v;    /* the agent's own reach */
    const int32_t cx = st->x[i], cy = st->y[i];
    const int64_t c = (int64_t)cy * W + cx;
    /* the floor field agent i follows */
    const double *S = st->fi ? st->Sf + (int64_t)st->fi[i] * W * H : st->S;
    double *w = malloc(sizeof(double) * (size_t)(side * side));
    if (!w) return -2;

    /* R1 + R2: weights over the window in raster order */
    for (int32_t dy = -v; dy <= v; ++dy) {
        for (int32_t dx = -v; dx <= v; ++dx) {
            int32_t slot = (dy + v) * side + (dx + v);
            int32_t tx = cx + dx, ty = cy + dy;
            int in_reach = dx * dx + dy * dy <= vr * vr;
            int in_grid = tx >= 0 && ty >= 0 && tx < W && ty < H;
            double wt = 0.0;
            if (in_reach && in_grid) {
                int64_t t = (int64_t)ty * W + tx;
                int free_or_own = st->occ[t] == -1 || t == c;
                if (st->type[t] != CELL_WALL && free_or_own) {
                    if (st->Tr)     /* R14 */
                        wt = exp(st->k_s * (S[c] - S[t]) + st->k_d * (st->Tr[t] - st->Tr[c]));
                    else
                        wt = exp(st->k_s * (S[c] - S[t]));
                }
            }
            w[slot] = wt;
        }
    }

    /* R3: sequential prefix sum, then the first slot with u*W < C */
    uint32_t x0 = philox_x0((uint32_t)i, (uint32_t)st->step, st->scn, 0u, st->seed);
    double u = (double)(x0 >> 8) * 0x1p-24;
    double C = 0.0, Wsum;
    for (int32_t s = 0; s < side * side; ++s) {
        C = C + w[s];
        if (c_out) c_out[s] = C;
    }
    Wsum = C;
    double tau = u * Wsum;
    int32_t chosen = -1;
    C = 0.0;
    for (int32_t s = 0; s < side * side; ++s) {
        C = C + w[s];
        if (tau < C) { chosen = s; break; }
    }
    if (w_out) memcpy(w_out, w, sizeof(double) * (size_t)(side * side));
    free(w);
    if (u_out) *u_out = u;
    if (slot_out) *slot_out = chosen;
    if (chosen < 0) return -2;       /* cannot happen: own cell has weight 1 */
    int32_t dy = chosen / side - v, dx = chosen % side - v;
    return (cy + dy) * W + (cx + dx);
}

/* One planning phase over all agents (Sec. 2: the parallel loop body). */
int oracle_plan_step(oracle_state *st)
{
    for (int32_t i = 0; i < st->n; ++i) {
        int32_t d = oracle_plan_agent(st, i, NULL, NULL, NULL, NULL);
        if (d == -2) return -1;
        st->desired[i] = d;
    }
    return 0;
}

/*
 * The same planning phase on `threads` host threads, used only to time a CPU
 * baseline that parallelises the way Sec. 2 describes: the agents are cut into
 * consecutive chunks, and a thread that runs out of work claims the next
 * unclaimed chunk.  A chunk holds N / threads agents, capped at 32767 and at
 * least one (the chunk size Sec. 2 uses).  Every draw depends on its agent
 * and the shared snapshot only, so the result equals oracle_plan_step's.
 */
typedef struct {
    oracle_state *st;
    int32_t chunk;
    atomic_int next;      /* first agent of the next unclaimed chunk */
    atomic_int failed;
} claim_pool;

static void *claim_and_plan(void *arg)
{
    claim_pool *p = arg;
    const int32_t n = p->st->n;
    for (;;) {
        const int32_t lo = atomic_fetch_add(&p->next, p->chunk);
        if (lo >= n) break;
        const int32_t hi = n - lo > p->chunk ? lo + p->chunk : n;
        for (int32_t i = lo; i < hi; ++i) {
            const int32_t d = oracle_plan_agent(p->st, i, NULL, NULL, NULL, NULL);
            if (d == -2) atomic_store(&p->failed, 1);
            p->st->desired[i] = d;
        }
    }
    return NULL;
}

enum { MAX_PLAN_THREADS = 256 };

int oracle_plan_step_threads(oracle_state *st, int32_t threads)
{
    if (threads < 1) threads = 1;
    if (threads > MAX_PLAN_THREADS) threads = MAX_PLAN_THREADS;
    claim_pool p;
    p.st = st;
    p.chunk = st->n / threads;
    if (p.chunk > 32767) p.chunk = 32767;
    if (p.chunk < 1) p.chunk = 1;
    atomic_init(&p.next, 0);
    atomic_init(&p.failed, 0);
    pthread_t helper[MAX_PLAN_THREADS];
    int32_t started = 0;
    for (int32_t k = 1; k < threads; ++k) {     /* the calling thread is the first worker */
        if (pthread_create(&helper[started], NULL, claim_and_plan, &p) != 0) break;
        ++started;
    }
    claim_and_plan(&p);
    for (int32_t k = 0; k < started; ++k) pthread_join(helper[k], NULL);
    return atomic_load(&p.failed) ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Motion phase (readings R4-R6).                                            */
/* ------------------------------------------------------------------------- */

int oracle_trail_update(oracle_state *st);

typedef struct { uint32_t key; int32_t id; } order_item;

static int order_cmp(const void *pa, const void *pb)
{
    const order_item *a = pa, *b = pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static int isgn(int32_t a) { return (a > 0) - (a < 0); }

/* Moves agent i from its cell towards desired[i] along the DDA line (R5),
 * updating occupancy in place; removes it on entering an exit (R6). */
static void move_agent(oracle_state *st, int32_t i)
{
    const int32_t W = st->W;
    int32_t cx = st->x[i], cy = st->y[i];
    int32_t d = st->desired[i];
    int32_t tx = d % W, ty = d / W;
    int32_t dx = tx - cx, dy = ty - cy;
    int32_t adx = abs(dx), ady = abs(dy);
    int32_t m = adx > ady ? adx : ady;
    int32_t px = cx, py = cy;
    for (int32_t k = 1; k <= m; ++k) {
        int32_t nx = cx + isgn(dx) * ((2 * k * adx + m) / (2 * m));
        int32_t ny = cy + isgn(dy) * ((2 * k * ady + m) / (2 * m));
        int64_t nc = (int64_t)ny * W + nx;
        if (st->type[nc] == CELL_WALL) break;
        if (st->occ[nc] != -1) break;
        if (nx != px && ny != py) {
            if (st->type[(int64_t)py * W + nx] == CELL_WALL) break;
            if (st->type[(int64_t)ny * W + px] == CELL_WALL) break;
        }
        st->occ[(int64_t)py * W + px] = -1;
        if (k == 1 && st->Tr) st->dep[(int64_t)cy * W + cx] += 1;   /* R14: it leaves */
        if (st->type[nc] == CELL_EXIT) {
            st->alive[i] = 0;
            st->x[i] = -1; st->y[i] = -1;
            st->desired[i] = -1;
            st->exited += 1;
            return;
        }
        st->occ[nc] = i;
        px = nx; py = ny;
    }
    st->x[i] = px; st->y[i] = py;
}

/* The trail update of reading R14 that closes a motion phase: every non-wall
 * cell from the values before the update, then the deposits restart. */
int oracle_trail_update(oracle_state *st)
{
    const int32_t W = st->W, H = st->H;
    const double keep = 1.0 - st->decay, stay = 1.0 - st->diffusion, share = st->diffusion / 8.0;
    double *nt = malloc(sizeof(double) * (size_t)W * (size_t)H);
    if (!nt) return -1;
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            const int64_t c = (int64_t)y * W + x;
            if (st->type[c] == CELL_WALL) { nt[c] = 0.0; continue; }
            double nb = 0.0;
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int32_t qx = x + dx, qy = y + dy;
                    if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
                    nb = nb + st->Tr[(int64_t)qy * W + qx];    /* walls hold 0 */
                }
            nt[c] = keep * (stay * st->Tr[c] + share * nb) + (double)st->dep[c];
        }
    memcpy(st->Tr, nt, sizeof(double) * (size_t)W * (size_t)H);
    for (int64_t c = 0; c < (int64_t)W * H; ++c) st->dep[c] = 0;
    free(nt);
    return 0;
}

/* One motion phase: agents one after another in the order of reading R4,
 * then (with a trail field) R14's update. */
int oracle_move_step(oracle_state *st)
{
    int32_t n = st->n, k = 0;
    order_item *ord = malloc(sizeof(order_item) * (size_t)(n > 0 ? n : 1));
    if (!ord) return -1;
    for (int32_t i = 0; i < n; ++i) {
        if (!st->alive[i]) continue;
        ord[k].key = philox_x0((uint32_t)i, (uint32_t)st->step, st->scn, 1u, st->seed);
        ord[k].id = i;
        ++k;
    }
    qsort(ord, (size_t)k, sizeof(order_item), order_cmp);
    for (int32_t j = 0; j < k; ++j) {
        int32_t i = ord[j].id;
        if (st->desired[i] < 0) continue;
        move_agent(st, i);
    }
    free(ord);
    if (st->Tr) return oracle_trail_update(st);
    return 0;
}

/* Full time steps: plan, then move, then advance the step number (Sec. 1). */
int oracle_run(oracle_state *st, int32_t steps)
{
    for (int32_t s = 0; s < steps; ++s) {
        if (oracle_plan_step(st)) return -1;
        if (oracle_move_step(st)) return -1;
        st->step += 1;
    }
    return 0;
}

/* Number of agents still in the simulation. */
int32_t oracle_count_alive(const oracle_state *st)
{
    int32_t c = 0;
    for (int32_t i = 0; i < st->n; ++i) c += st->alive[i] ? 1 : 0;
    return c;
}

/* Host threads online (the CPU baseline may be told to use fewer). */
int32_t oracle_num_threads(void)
{
    const long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int32_t)n : 1;
}
