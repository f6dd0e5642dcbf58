/*
 * sg_oracle.c -- plain, slow, sequential CPU reference for the aging
 * Metropolis dynamics of the Viana-Bray and Sherrington-Kirkpatrick spin
 * glasses.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP library: the Philox
 * generator, the graph generator, the colouring, the threshold table and the
 * dynamics are all written out again here, directly from their definitions.
 *
 * What is computed, and where the paper states it:
 *  - Hamiltonians: SK, Eq. (1), H = -sum_{i<j} J_ij s_i s_j; VB, Eq. (3),
 *    H = -sum_{(ij) in E} J_ij s_i s_j with J = +-1 (main text, after Eq. 3).
 *    SK couplings are binary, +-1/sqrt(N) (SI, "The Sherrington-Kirkpatrick
 *    model"); here the integer part +-1 is kept and 1/sqrt(N) goes into the
 *    energy change.
 *  - Dynamics: single-spin-flip Metropolis at fixed T from a random start, one
 *    unit of time = one update of every spin (Methods; SI, "Spin glass on a
 *    bipartite random regular graph").  A spin with local field h_i is flipped
 *    with probability min(1, exp(-beta * dE)), dE = 2 s_i h_i.
 *  - Parallel update by a proper colouring of the graph (the paper's
 *    bipartition, SI "Simulations of the Bethe Lattice on GPUs", generalised):
 *    the sweep visits colour class 0, then class 1, ...; inside a class the
 *    order is irrelevant because no two spins of a class interact.  The oracle
 *    runs it strictly sequentially (mode 0) or class-synchronously (mode 1);
 *    the two agree exactly iff the colouring is proper.
 *  - SK order: i = 0..N-1, a fixed order (SI, SK section).
 *  - Observables: two-time correlation C(t, t') = (1/N) sum_i s_i(t) s_i(t')
 *    (introduction, definition of C and R; SI Eq. formula1), energy, and the
 *    two-clone overlap.  All are kept as exact integers: bond sum B = -H
 *    (times sqrt(N) for SK), overlap Q = sum_i s^a_i s^b_i, and the Gram
 *    matrix G[k][l] = sum_i s_i(t_k) s_i(t_l), so that C = G / N.
 *
 * The paper names no random number generator.  The counter layout below is
 * this library's own definition, implemented independently on both sides.
 * Philox4x32-10 and Philox4x64-10 are from J. K. Salmon, M. A. Moraes,
 * R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11 (multipliers, Weyl key increments, 10 rounds).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox                                                                     */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* The 64-bit-word member of the same family; only used to check the round
 * structure against an independent implementation (numpy's Philox). */
void orc_philox4x64_10(const uint64_t in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ull, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ull, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream domains (third counter word, bits 24..31). */
enum { DOM_SWEEP_HI = 0, DOM_SWEEP_LO = 1, DOM_INIT = 2, DOM_GRAPH = 3, DOM_COUPLING = 4 };

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                          uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 16-bit half-word h (0..7) of a 128-bit Philox output. */
static uint32_t half_word(const uint32_t out[4], unsigned h)
{
    return (out[h >> 1] >> (16u * (h & 1u))) & 0xffffu;
}

/* The uniform 32-bit number that decides the update of sweep position p in
 * sweep t of chain (inst, rep).  High and low halves come from two streams;
 * each Philox block serves eight consecutive positions. */
uint32_t orc_accept_uniform(uint64_t seed, uint32_t inst, uint32_t rep, uint32_t t, uint64_t p)
{
    uint32_t a[4], b[4];
    philox_seeded(seed, (uint32_t)(p >> 3), t, ((uint32_t)DOM_SWEEP_HI << 24) | rep, inst, a);
    philox_seeded(seed, (uint32_t)(p >> 3), t, ((uint32_t)DOM_SWEEP_LO << 24) | rep, inst, b);
    unsigned h = (unsigned)(p & 7u);
    return (half_word(a, h) << 16) | half_word(b, h);
}

/* Random start: +1 or -1 for sweep position p of chain (inst, rep). */
int orc_init_spin(uint64_t seed, uint32_t inst, uint32_t rep, uint64_t p)
{
    uint32_t o[4];
    philox_seeded(seed, (uint32_t)(p >> 7), 0u, ((uint32_t)DOM_INIT << 24) | rep, inst, o);
    uint32_t bit = (o[(p >> 5) & 3u] >> (p & 31u)) & 1u;
    return bit ? -1 : +1;
}

/* ------------------------------------------------------------------------ */
/* Instances                                                                  */
/* ------------------------------------------------------------------------ */

/* Erdos-Renyi G(N, M): attempt a = 0, 1, 2, ... draws an ordered pair
 * (u, v) = (floor(w0 N / 2^32), floor(w1 N / 2^32)); the attempt is rejected
 * if u == v or the pair {u, v} is already an edge, else edge number
 * "accepted" is (u, v) with coupling +1 if w2 is even and -1 if odd.
 * Stops after m accepted edges.  A plain open-addressing set keeps the edges
 * seen so far.  Returns the number of attempts, or -1 on bad arguments. */
int64_t orc_er_graph(int64_t n, int64_t m, uint64_t seed, uint32_t graph_id,
                     int32_t* eu, int32_t* ev, int8_t* J)
{
    if (n < 2 || m < 0 || n > 0x7fffffffLL || m > n * (n - 1) / 2) return -1;
    uint64_t cap = 16;
    while (cap < (uint64_t)(4 * m + 16)) cap <<= 1;
    uint64_t* set = (uint64_t*)malloc(cap * sizeof(uint64_t));
    if (!set) return -1;
    for (uint64_t i = 0; i < cap; ++i) set[i] = UINT64_MAX;
    int64_t accepted = 0;
    uint64_t a = 0;
    while (accepted < m) {
        uint32_t w[4];
        philox_seeded(seed, (uint32_t)(a & 0xffffffffu), (uint32_t)(a >> 32),
                      (uint32_t)DOM_GRAPH << 24, graph_id, w);
        ++a;
        int64_t u = (int64_t)(((uint64_t)w[0] * (uint64_t)n) >> 32);
        int64_t v = (int64_t)(((uint64_t)w[1] * (uint64_t)n) >> 32);
        if (u == v) continue;
        uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
        uint64_t key = lo * (uint64_t)n + hi;
        uint64_t slot = (key * 0x9E3779B97F4A7C15ull) & (cap - 1);
        int present = 0;
        while (set[slot] != UINT64_MAX) {
            if (set[slot] == key) { present = 1; break; }
            slot = (slot + 1) & (cap - 1);
        }
        if (present) continue;
        set[slot] = key;
        eu[accepted] = (int32_t)u;
        ev[accepted] = (int32_t)v;
        J[accepted] = (w[2] & 1u) ? (int8_t)-1 : (int8_t)1;
        ++accepted;
    }
    free(set);
    return (int64_t)a;
}

/* Binary SK couplings: for i < j, bit idx = i*N + j of the COUPLING stream
 * decides J_ij = J_ji (bit 1 -> -1).  Diagonal is 0.  J is N x N row-major. */
void orc_sk_couplings(int64_t n, uint64_t seed, uint32_t graph_id, int8_t* J)
{
    for (int64_t i = 0; i < n; ++i) J[i * n + i] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            uint64_t idx = (uint64_t)i * (uint64_t)n + (uint64_t)j;
            uint32_t w[4];
            philox_seeded(seed, (uint32_t)((idx >> 7) & 0xffffffffu), (uint32_t)(idx >> 39),
                          (uint32_t)DOM_COUPLING << 24, graph_id, w);
            uint32_t bit = (w[(idx >> 5) & 3u] >> (idx & 31u)) & 1u;
            int8_t v = bit ? (int8_t)-1 : (int8_t)1;
            J[i * n + j] = v;
            J[j * n + i] = v;
        }
    }
}

/* Adjacency lists in vertex order (plain CSR, built by counting). */
typedef struct {
    int64_t n;
    int64_t* start;   /* [n+1] */
    int32_t* nbr;     /* [2m]  */
    int8_t* cpl;      /* [2m]  */
} adj_t;

static int adj_build(adj_t* g, int64_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                     const int8_t* J)
{
    g->n = n;
    g->start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    g->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->cpl = (int8_t*)malloc((size_t)(2 * m + 1));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!g->start || !g->nbr || !g->cpl || !fill) { free(fill); return -1; }
    for (int64_t e = 0; e < m; ++e) { g->start[eu[e] + 1]++; g->start[ev[e] + 1]++; }
    for (int64_t v = 0; v < n; ++v) g->start[v + 1] += g->start[v];
    for (int64_t e = 0; e < m; ++e) {
        int64_t u = eu[e], v = ev[e];
        int64_t a = g->start[u] + fill[u]++;
        g->nbr[a] = (int32_t)v; g->cpl[a] = J[e];
        int64_t b = g->start[v] + fill[v]++;
        g->nbr[b] = (int32_t)u; g->cpl[b] = J[e];
    }
    free(fill);
    return 0;
}

static void adj_free(adj_t* g)
{
    free(g->start); free(g->nbr); free(g->cpl);
}

/* Greedy colouring in vertex order: colour(v) is the smallest colour not
 * used by any neighbour u < v.  Returns the number of colours. */
int32_t orc_greedy_colour(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                          int32_t* colour)
{
    int8_t* J = (int8_t*)calloc((size_t)m + 1, 1);
    adj_t g;
    if (!J || adj_build(&g, n, m, eu, ev, J) != 0) { free(J); return -1; }
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (g.start[v + 1] - g.start[v] > maxdeg) maxdeg = g.start[v + 1] - g.start[v];
    char* used = (char*)calloc((size_t)maxdeg + 2, 1);
    int32_t ncol = 0;
    for (int64_t v = 0; v < n; ++v) {
        memset(used, 0, (size_t)maxdeg + 2);
        for (int64_t a = g.start[v]; a < g.start[v + 1]; ++a) {
            int64_t u = g.nbr[a];
            if (u < v && colour[u] <= maxdeg) used[colour[u]] = 1;
        }
        int32_t c = 0;
        while (used[c]) ++c;
        colour[v] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(used);
    adj_free(&g);
    free(J);
    return ncol;
}

/* Sweep order: class 0, then class 1, ...; inside a class by decreasing
 * degree, ties by increasing vertex id.  order[p] is the vertex visited at
 * position p. */
void orc_sweep_order(int64_t n, const int32_t* colour, int32_t ncol, const int32_t* deg,
                     int32_t* order)
{
    int32_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (deg[v] > maxdeg) maxdeg = deg[v];
    int64_t p = 0;
    for (int32_t c = 0; c < ncol; ++c)
        for (int32_t d = maxdeg; d >= 0; --d)
            for (int64_t v = 0; v < n; ++v)
                if (colour[v] == c && deg[v] == d) order[p++] = (int32_t)v;
}

/* Metropolis acceptance thresholds, thr[x] = floor(2^32 exp(-beta dE)) for
 * x = s_i h_i >= 1 with dE = 2 x * de_scale (de_scale = 1 for VB, 1/sqrt(N)
 * for SK).  A move with x <= 0 is always accepted; a move with x >= 1 is
 * accepted iff the 32-bit uniform r satisfies r < thr[x].  thr[0] = 2^32. */
void orc_thresholds(double T, double de_scale, int32_t xmax, uint64_t* thr)
{
    double beta = 1.0 / T;
    thr[0] = (uint64_t)1 << 32;
    for (int32_t x = 1; x <= xmax; ++x) {
        double dE = 2.0 * (double)x * de_scale;
        double p = exp(-beta * dE);
        thr[x] = (uint64_t)floor(ldexp(p, 32));
    }
}

/* Measurement grid {0} U {2^k <= t_max}; returns its size. */
int32_t orc_grid(int64_t t_max, int64_t* times)
{
    int32_t k = 0;
    times[k++] = 0;
    for (int64_t t = 1; t <= t_max; t <<= 1) times[k++] = t;
    return k;
}

static int is_grid_time(int64_t t)
{
    return t == 0 || (t > 0 && (t & (t - 1)) == 0);
}

/* Windowed correlation (the paper's estimator: the measured C(t_w + t, t_w)
 * averaged over geometric "minor third" time intervals, ratio 2^(1/4) from
 * one to the next; Results and discussion, and the SI section on the
 * extrapolation to large sizes and times).  Here the intervals are taken in
 * the absolute time tau = t_w + t: interval m holds the integer times with
 * 2^(m/4) <= tau < 2^((m+1)/4), so m = floor(4 log2 tau) = floor(log2 tau^4),
 * computed from the exact fourth power (tau < 2^32, so tau^4 < 2^128). */
int32_t orc_window_bin(uint64_t tau)
{
    unsigned __int128 p = (unsigned __int128)tau * (unsigned __int128)tau;
    p = p * p;
    int32_t m = -1;
    while (p != 0) {
        p >>= 1;
        ++m;
    }
    return m;
}

/* Number of waiting times of the windowed estimator: the grid times <= tw_max. */
int32_t orc_window_tw_count(int64_t t_max, int64_t tw_max)
{
    int64_t grid[70];
    int32_t K = orc_grid(t_max, grid), kw = 0;
    for (int32_t k = 0; k < K; ++k)
        if (grid[k] <= tw_max) ++kw;
    return kw;
}

/* ------------------------------------------------------------------------ */
/* Viana-Bray                                                                 */
/* ------------------------------------------------------------------------ */

/* Runs n_rep replicas of one VB instance for n_sweeps sweeps.
 *  graph: m edges (eu, ev, J), vertex ids 0..n-1.
 *  start: 0 random (INIT stream), 1 all +1, 2 given s0[n_rep][n] (vertex order).
 *  mode: 0 sequential in sweep order, 1 class-synchronous.
 * Outputs (caller-allocated; K = grid size for t_max):
 *  times[K], bond[n_rep][K], overlap[n_pairs][K] (pairs a<b in lexicographic
 *  order), gram[n_rep][K][K], accepted[n_rep], spins[n_rep][n] (vertex order,
 *  after the last sweep), k_done = number of grid times reached.
 * Windowed correlation, when window != NULL (t_max >= 1): waiting times are
 * the kw = orc_window_tw_count(t_max, tw_max) first grid times, intervals
 * m = 0 .. M-1 with M = orc_window_bin(t_max) + 1; after every sweep that
 * ends at a time tau <= t_max, for every waiting time t_w < tau,
 *   window[r][k][m(tau)] += sum_i s_i(tau) s_i(t_w)   (replica r),
 *   window_count[k][m(tau)] += 1,
 * so that window / (window_count n) is C(tau, t_w) averaged over interval m.
 * Returns 0, or -1 on bad input. */
int orc_vb_run(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const int8_t* J,
               double T, uint64_t seed, uint32_t inst, int32_t n_rep, int32_t start,
               const int8_t* s0, int64_t n_sweeps, int64_t t_max, int32_t mode,
               int64_t* times, int64_t* bond, int64_t* overlap, int64_t* gram,
               int64_t* accepted, int8_t* spins, int32_t* k_done,
               int64_t tw_max, int64_t* window, int64_t* window_count)
{
    if (n < 1 || n_rep < 1 || n_sweeps < 0 || t_max < 0) return -1;
    if (window && (t_max < 1 || tw_max < 0 || !window_count)) return -1;
    const int32_t kw = window ? orc_window_tw_count(t_max, tw_max) : 0;
    const int32_t n_bins = window ? orc_window_bin((uint64_t)t_max) + 1 : 0;
    if (window) {
        memset(window, 0, sizeof(int64_t) * (size_t)n_rep * (size_t)kw * (size_t)n_bins);
        memset(window_count, 0, sizeof(int64_t) * (size_t)kw * (size_t)n_bins);
    }
    adj_t g;
    if (adj_build(&g, n, m, eu, ev, J) != 0) return -1;
    int32_t* colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t ncol = orc_greedy_colour(n, m, eu, ev, colour);
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) deg[v] = (int32_t)(g.start[v + 1] - g.start[v]);
    orc_sweep_order(n, colour, ncol, deg, order);
    free(deg);
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (g.start[v + 1] - g.start[v] > maxdeg) maxdeg = g.start[v + 1] - g.start[v];
    uint64_t* thr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(maxdeg + 1));
    orc_thresholds(T, 1.0, (int32_t)maxdeg, thr);

    int64_t grid[70];
    int32_t K = orc_grid(t_max, grid);
    for (int32_t k = 0; k < K; ++k) times[k] = grid[k];

    int8_t* snaps = (int8_t*)malloc((size_t)n_rep * (size_t)K * (size_t)n);
    int8_t* s = (int8_t*)malloc((size_t)n);
    int8_t* nxt = (int8_t*)malloc((size_t)n);
    int32_t kd = 0;

    for (int32_t r = 0; r < n_rep; ++r) {
        /* initial configuration, in vertex order */
        for (int64_t p = 0; p < n; ++p) {
            int64_t v = order[p];
            if (start == 0) s[v] = (int8_t)orc_init_spin(seed, inst, (uint32_t)r, (uint64_t)p);
            else if (start == 1) s[v] = 1;
            else s[v] = s0[(int64_t)r * n + v];
        }
        accepted[r] = 0;
        int32_t k = 0;
        for (int64_t t = 0;; ++t) {
            if (t <= t_max && is_grid_time(t)) {
                memcpy(snaps + ((int64_t)r * K + k) * n, s, (size_t)n);
                int64_t B = 0;
                for (int64_t e = 0; e < m; ++e) B += (int64_t)J[e] * s[eu[e]] * s[ev[e]];
                bond[(int64_t)r * K + k] = B;
                ++k;
            }
            if (t == n_sweeps) break;
            if (mode == 0) {
                for (int64_t p = 0; p < n; ++p) {
                    int64_t v = order[p];
                    int64_t h = 0;
                    for (int64_t a = g.start[v]; a < g.start[v + 1]; ++a) h += g.cpl[a] * s[g.nbr[a]];
                    int64_t x = s[v] * h;
                    int flip;
                    if (x <= 0) flip = 1;
                    else flip = (uint64_t)orc_accept_uniform(seed, inst, (uint32_t)r, (uint32_t)t,
                                                             (uint64_t)p) < thr[x];
                    if (flip) { s[v] = (int8_t)-s[v]; accepted[r]++; }
                }
            } else {
                /* class-synchronous: every spin of a class decides from the
                 * configuration at the start of that class. */
                int64_t p = 0;
                while (p < n) {
                    int32_t c = colour[order[p]];
                    int64_t q = p;
                    memcpy(nxt, s, (size_t)n);
                    while (q < n && colour[order[q]] == c) {
                        int64_t v = order[q];
                        int64_t h = 0;
                        for (int64_t a = g.start[v]; a < g.start[v + 1]; ++a) h += g.cpl[a] * s[g.nbr[a]];
                        int64_t x = s[v] * h;
                        int flip;
                        if (x <= 0) flip = 1;
                        else flip = (uint64_t)orc_accept_uniform(seed, inst, (uint32_t)r, (uint32_t)t,
                                                                 (uint64_t)q) < thr[x];
                        if (flip) { nxt[v] = (int8_t)-s[v]; accepted[r]++; }
                        ++q;
                    }
                    memcpy(s, nxt, (size_t)n);
                    p = q;
                }
            }
            /* windowed correlation at the time this sweep ends */
            const int64_t tau = t + 1;
            if (window && tau <= t_max) {
                const int32_t bin = orc_window_bin((uint64_t)tau);
                for (int32_t kk = 0; kk < kw; ++kk) {
                    if (times[kk] >= tau) continue;
                    const int8_t* sw = snaps + ((int64_t)r * K + kk) * n;
                    int64_t O = 0;
                    for (int64_t i = 0; i < n; ++i) O += s[i] * sw[i];
                    window[((int64_t)r * kw + kk) * n_bins + bin] += O;
                    if (r == 0) window_count[(int64_t)kk * n_bins + bin] += 1;
                }
            }
        }
        kd = k;
        memcpy(spins + (int64_t)r * n, s, (size_t)n);
    }

    /* overlaps between replicas a < b, and Gram matrices, at every grid time */
    int64_t pair = 0;
    for (int32_t a = 0; a < n_rep; ++a)
        for (int32_t b = a + 1; b < n_rep; ++b, ++pair)
            for (int32_t k = 0; k < kd; ++k) {
                const int8_t* sa = snaps + ((int64_t)a * K + k) * n;
                const int8_t* sb = snaps + ((int64_t)b * K + k) * n;
                int64_t Q = 0;
                for (int64_t i = 0; i < n; ++i) Q += sa[i] * sb[i];
                overlap[pair * K + k] = Q;
            }
    for (int32_t r = 0; r < n_rep; ++r)
        for (int32_t k = 0; k < K; ++k)
            for (int32_t l = 0; l < K; ++l) {
                int64_t G = 0;
                if (k < kd && l < kd) {
                    const int8_t* sk = snaps + ((int64_t)r * K + k) * n;
                    const int8_t* sl = snaps + ((int64_t)r * K + l) * n;
                    for (int64_t i = 0; i < n; ++i) G += sk[i] * sl[i];
                }
                gram[((int64_t)r * K + k) * K + l] = G;
            }
    *k_done = kd;
    free(snaps); free(s); free(nxt); free(thr); free(order); free(colour);
    adj_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sherrington-Kirkpatrick                                                    */
/* ------------------------------------------------------------------------ */

/* Runs n_rep replicas of one SK instance (J: n x n int8 +-1, symmetric, zero
 * diagonal) for n_sweeps sweeps in the fixed order i = 0..n-1.  The local
 * field H_i = sum_j J_ij s_j is recomputed from scratch for every update when
 * direct != 0; otherwise it is kept up to date after every flip by adding
 * 2 s_i(new) J_ij to every H_j.  Outputs as for orc_vb_run; the bond sum is
 * B = sum_{i<j} J_ij s_i s_j (energy = -B / sqrt(N)). */
int orc_sk_run(int64_t n, const int8_t* J, double T, uint64_t seed, uint32_t inst,
               int32_t n_rep, int32_t start, const int8_t* s0, int64_t n_sweeps,
               int64_t t_max, int32_t direct, int64_t* times, int64_t* bond,
               int64_t* overlap, int64_t* gram, int64_t* accepted, int8_t* spins,
               int32_t* k_done)
{
    if (n < 1 || n_rep < 1 || n_sweeps < 0 || t_max < 0) return -1;
    uint64_t* thr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    orc_thresholds(T, 1.0 / sqrt((double)n), (int32_t)(n - 1), thr);
    int64_t grid[70];
    int32_t K = orc_grid(t_max, grid);
    for (int32_t k = 0; k < K; ++k) times[k] = grid[k];
    int8_t* snaps = (int8_t*)malloc((size_t)n_rep * (size_t)K * (size_t)n);
    int8_t* s = (int8_t*)malloc((size_t)n);
    int64_t* H = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t kd = 0;

    for (int32_t r = 0; r < n_rep; ++r) {
        for (int64_t i = 0; i < n; ++i) {
            if (start == 0) s[i] = (int8_t)orc_init_spin(seed, inst, (uint32_t)r, (uint64_t)i);
            else if (start == 1) s[i] = 1;
            else s[i] = s0[(int64_t)r * n + i];
        }
        for (int64_t i = 0; i < n; ++i) {
            int64_t h = 0;
            for (int64_t j = 0; j < n; ++j) h += (int64_t)J[i * n + j] * s[j];
            H[i] = h;
        }
        accepted[r] = 0;
        int32_t k = 0;
        for (int64_t t = 0;; ++t) {
            if (t <= t_max && is_grid_time(t)) {
                memcpy(snaps + ((int64_t)r * K + k) * n, s, (size_t)n);
                int64_t B = 0;
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t j = i + 1; j < n; ++j) B += (int64_t)J[i * n + j] * s[i] * s[j];
                bond[(int64_t)r * K + k] = B;
                ++k;
            }
            if (t == n_sweeps) break;
            for (int64_t i = 0; i < n; ++i) {
                int64_t h;
                if (direct) {
                    h = 0;
                    for (int64_t j = 0; j < n; ++j) h += (int64_t)J[i * n + j] * s[j];
                } else {
                    h = H[i];
                }
                int64_t x = s[i] * h;
                int flip;
                if (x <= 0) flip = 1;
                else flip = (uint64_t)orc_accept_uniform(seed, inst, (uint32_t)r, (uint32_t)t,
                                                         (uint64_t)i) < thr[x];
                if (flip) {
                    s[i] = (int8_t)-s[i];
                    accepted[r]++;
                    if (!direct)
                        for (int64_t j = 0; j < n; ++j) H[j] += 2 * (int64_t)s[i] * J[i * n + j];
                }
            }
        }
        kd = k;
        memcpy(spins + (int64_t)r * n, s, (size_t)n);
    }

    int64_t pair = 0;
    for (int32_t a = 0; a < n_rep; ++a)
        for (int32_t b = a + 1; b < n_rep; ++b, ++pair)
            for (int32_t k = 0; k < kd; ++k) {
                const int8_t* sa = snaps + ((int64_t)a * K + k) * n;
                const int8_t* sb = snaps + ((int64_t)b * K + k) * n;
                int64_t Q = 0;
                for (int64_t i = 0; i < n; ++i) Q += sa[i] * sb[i];
                overlap[pair * K + k] = Q;
            }
    for (int32_t r = 0; r < n_rep; ++r)
        for (int32_t k = 0; k < K; ++k)
            for (int32_t l = 0; l < K; ++l) {
                int64_t G = 0;
                if (k < kd && l < kd) {
                    const int8_t* sk = snaps + ((int64_t)r * K + k) * n;
                    const int8_t* sl = snaps + ((int64_t)r * K + l) * n;
                    for (int64_t i = 0; i < n; ++i) G += sk[i] * sl[i];
                }
                gram[((int64_t)r * K + k) * K + l] = G;
            }
    *k_done = kd;
    free(snaps); free(s); free(H); free(thr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sherrington-Kirkpatrick with real (Gaussian) couplings                    */
/* ------------------------------------------------------------------------ */

/* SK with real couplings J_ij (Eq. 1: Gaussian, variance 1/N; given here as
 * float32, symmetric, zero diagonal, the 1/sqrt(N) already included), so the
 * energy is H = -sum_{i<j} J_ij s_i s_j and flipping s_i changes it by
 * dE = 2 x with x = s_i h_i, h_i = sum_j J_ij s_j.  Fields are kept in IEEE
 * double: initially the direct sums (j ascending); after a flip of s_i,
 * h_j += 2 s_i J_ij (new s_i) for every j, in flip order; every `period`
 * sweeps (period > 0) they are recomputed directly (j ascending), as the
 * paper's periodic recomputation of the fields prescribes for real
 * couplings.  With direct != 0 every field is computed directly when it is
 * used instead.  Acceptance as for the binary model with x real: flip if
 * x <= 0, else iff r < floor(ldexp(exp(-(1/T) (2 x)), 32)) in double, r the
 * same 32-bit uniform.  Outputs as orc_sk_run, except bond[n_rep][K] is the
 * real B = sum_{i<j} J_ij s_i s_j (i ascending, then j), and h_out[n_rep][n]
 * (may be NULL) receives the final fields.  Returns 0, or -1 on bad input. */
int orc_skg_run(int64_t n, const float* J, double T, uint64_t seed, uint32_t inst,
                int32_t n_rep, int32_t start, const int8_t* s0, int64_t n_sweeps,
                int64_t t_max, int32_t period, int32_t direct, int64_t* times, double* bond,
                int64_t* overlap, int64_t* gram, int64_t* accepted, int8_t* spins,
                double* h_out, int32_t* k_done)
{
    if (n < 1 || n_rep < 1 || n_sweeps < 0 || t_max < 0 || period < 0) return -1;
    const double beta = 1.0 / T;
    int64_t grid[70];
    int32_t K = orc_grid(t_max, grid);
    for (int32_t k = 0; k < K; ++k) times[k] = grid[k];
    int8_t* snaps = (int8_t*)malloc((size_t)n_rep * (size_t)K * (size_t)n);
    int8_t* s = (int8_t*)malloc((size_t)n);
    double* H = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t kd = 0;

    for (int32_t r = 0; r < n_rep; ++r) {
        for (int64_t i = 0; i < n; ++i) {
            if (start == 0) s[i] = (int8_t)orc_init_spin(seed, inst, (uint32_t)r, (uint64_t)i);
            else if (start == 1) s[i] = 1;
            else s[i] = s0[(int64_t)r * n + i];
        }
        for (int64_t i = 0; i < n; ++i) {
            double h = 0.0;
            for (int64_t j = 0; j < n; ++j) h += (double)J[i * n + j] * (double)s[j];
            H[i] = h;
        }
        accepted[r] = 0;
        int32_t k = 0;
        for (int64_t t = 0;; ++t) {
            if (t <= t_max && is_grid_time(t)) {
                memcpy(snaps + ((int64_t)r * K + k) * n, s, (size_t)n);
                double B = 0.0;
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t j = i + 1; j < n; ++j) B += (double)J[i * n + j] * (double)(s[i] * s[j]);
                bond[(int64_t)r * K + k] = B;
                ++k;
            }
            if (t == n_sweeps) break;
            for (int64_t i = 0; i < n; ++i) {
                double h;
                if (direct) {
                    h = 0.0;
                    for (int64_t j = 0; j < n; ++j) h += (double)J[i * n + j] * (double)s[j];
                } else {
                    h = H[i];
                }
                const double x = (double)s[i] * h;
                int flip;
                if (x <= 0.0) {
                    flip = 1;
                } else {
                    const double p = exp(-beta * (2.0 * x));
                    const uint64_t thr = (uint64_t)floor(ldexp(p, 32));
                    flip = (uint64_t)orc_accept_uniform(seed, inst, (uint32_t)r, (uint32_t)t, (uint64_t)i) < thr;
                }
                if (flip) {
                    s[i] = (int8_t)-s[i];
                    accepted[r]++;
                    if (!direct) {
                        const double a = 2.0 * (double)s[i];
                        for (int64_t j = 0; j < n; ++j) H[j] += a * (double)J[i * n + j];
                    }
                }
            }
            if (period > 0 && (t + 1) % period == 0 && !direct)
                for (int64_t i = 0; i < n; ++i) {
                    double h = 0.0;
                    for (int64_t j = 0; j < n; ++j) h += (double)J[i * n + j] * (double)s[j];
                    H[i] = h;
                }
        }
        kd = k;
        memcpy(spins + (int64_t)r * n, s, (size_t)n);
        if (h_out)
            for (int64_t i = 0; i < n; ++i) {
                double h = H[i];
                if (direct) {
                    h = 0.0;
                    for (int64_t j = 0; j < n; ++j) h += (double)J[i * n + j] * (double)s[j];
                }
                h_out[(int64_t)r * n + i] = h;
            }
    }

    int64_t pair = 0;
    for (int32_t a = 0; a < n_rep; ++a)
        for (int32_t b = a + 1; b < n_rep; ++b, ++pair)
            for (int32_t k = 0; k < kd; ++k) {
                const int8_t* sa = snaps + ((int64_t)a * K + k) * n;
                const int8_t* sb = snaps + ((int64_t)b * K + k) * n;
                int64_t Q = 0;
                for (int64_t i = 0; i < n; ++i) Q += sa[i] * sb[i];
                overlap[pair * K + k] = Q;
            }
    for (int32_t r = 0; r < n_rep; ++r)
        for (int32_t k = 0; k < K; ++k)
            for (int32_t l = 0; l < K; ++l) {
                int64_t G = 0;
                if (k < kd && l < kd) {
                    const int8_t* sk = snaps + ((int64_t)r * K + k) * n;
                    const int8_t* sl = snaps + ((int64_t)r * K + l) * n;
                    for (int64_t i = 0; i < n; ++i) G += sk[i] * sl[i];
                }
                gram[((int64_t)r * K + k) * K + l] = G;
            }
    *k_done = kd;
    free(snaps); free(s); free(H);
    return 0;
}
