/*
 * sg.h -- C ABI of the MI355X (gfx950) aging Metropolis library for the
 * Viana-Bray and Sherrington-Kirkpatrick spin glasses.
 *
 * The operation (arXiv:1906.11195): quench a configuration of N Ising spins
 * from a random start to temperature T and run single-spin-flip Metropolis
 * dynamics (Methods; SI section on the bipartite random regular graph, where
 * one unit of time is one update of every spin), measuring the energy, the
 * overlap of two clones and the two-time correlation
 *     C(t, t') = (1/N) sum_i s_i(t) s_i(t')
 * (introduction, definition of C and R; SI Eq. formula1) on the grid of times
 * t in {0} U {2^k}.
 *
 *   VB (Eq. 3):  H = - sum_{(ij) in E} J_ij s_i s_j,   J_ij = +-1,
 *                on an Erdos-Renyi graph with M = floor(c N / 2) edges or on
 *                a caller-given edge list.
 *   SK (Eq. 1):  H = - sum_{i<j} J_ij s_i s_j,  J_ij = +-1/sqrt(N) (the binary
 *                couplings of the SI section on the SK model), stored as int8
 *                +-1; the factor 1/sqrt(N) enters the energy change.
 *
 * Acceptance (Metropolis): with x = s_i h_i (h_i the integer local field), a
 * flip is accepted if x <= 0, else iff r < thr[x], where r is a 32-bit
 * uniform and, in IEEE double with the C library's exp,
 *     beta = 1.0 / T;  dE = 2.0 * (double)x * s;
 *     thr[x] = (uint64_t) floor(ldexp(exp(-beta * dE), 32)),
 * with s = 1.0 (VB) or s = 1.0 / sqrt((double)N) (SK).
 * T = +inf accepts every move; T = 0 accepts only moves with x <= 0.
 *
 * Update order (the paper's bipartite parallel update, SI "Simulations of the
 * Bethe Lattice on GPUs", generalised to any graph): the vertices are coloured
 * greedily in vertex order (colour(v) = smallest colour not used by a
 * neighbour u < v); the sweep visits colour class 0, then class 1, ...; inside
 * a class by decreasing degree, ties by increasing vertex id (the order inside
 * a class does not change the dynamics' law; it fixes which random number each
 * spin uses).  "Position" p is the index of a vertex in that visiting order.  SK visits i = 0..N-1 (fixed order, SI SK section),
 * so p = i.
 *
 * Random numbers.  The paper names no generator.  This library uses
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 * (seed mod 2^32, seed >> 32) and counter (c0, c1, c2, c3):
 *   acceptance, sweep t (0-based, sweeps already done), position p, chain
 *   (instance_id, replica): r = (A << 16) | B where A is half-word (p & 7) of
 *   Philox(p >> 3, t, (0 << 24) | replica, instance_id) and B is half-word
 *   (p & 7) of Philox(p >> 3, t, (1 << 24) | replica, instance_id); half-word
 *   h of (w0, w1, w2, w3) is (w[h >> 1] >> (16 (h & 1))) & 0xffff.
 *   random start: s_p = -1 iff bit (p & 31) of word ((p >> 5) & 3) of
 *   Philox(p >> 7, 0, (2 << 24) | replica, instance_id) is 1.
 *   ER graph: attempt a = 0, 1, ... uses w = Philox(a mod 2^32, a >> 32,
 *   3 << 24, graph_id); u = (w0 N) >> 32, v = (w1 N) >> 32 (64-bit
 *   products); rejected if u == v or {u, v} is already an edge; else the
 *   next edge is (u, v) with J = -1 iff w2 is odd.  Stops at M edges.
 *   SK couplings: for i < j, idx = i N + j; J_ij = J_ji = -1 iff bit
 *   (idx & 31) of word ((idx >> 5) & 3) of Philox(idx >> 7 (low 32 bits),
 *   idx >> 39, 4 << 24, graph_id) is 1; J_ii = 0.
 *
 * Determinism: every output is a pure function of the descriptors and the
 * number of sweeps done; it does not depend on how instances are batched into
 * one context, on streams, or on launch shapes.
 *
 * Conventions: every call except sg_free returns an sg_status; on failure a
 * create call sets *out to NULL and leaks nothing.  Host arrays passed in are
 * copied during the call; the caller keeps ownership.  Output arrays are
 * caller-owned.  The context owns all device memory it allocated.  A context
 * must not be used from two host threads at once.  No C++ exception crosses
 * this interface.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
#define SG_OK 0
#define SG_EINVAL (-1)   /* bad argument or descriptor */
#define SG_ENOMEM (-2)   /* device or host allocation failed */
#define SG_EDEVICE (-3)  /* HIP runtime error or no usable gfx950 device */
#define SG_ESTATE (-4)   /* call not valid in the context's state */
#define SG_EPARITY (-5)  /* SK incremental fields disagreed with the exact recompute */
#define SG_ENOTSUP (-6)  /* valid request outside the library's limits */

#define SG_START_RANDOM 0   /* Philox random start (the paper's quench) */
#define SG_START_ALIGNED 1  /* all spins +1 (the SI's SK protocol) */
#define SG_START_GIVEN 2    /* s0 given by the caller */

typedef struct sg_ctx sg_ctx;

/* One Viana-Bray instance: a graph with couplings, a temperature and
 * n_replicas independent chains ("clones") on it.
 *  n          number of spins, 2 <= n <= 2^20 (a chain stays in one
 *             workgroup's LDS during a sweep).
 *  c          mean degree used when edges == NULL: M = floor(c n / 2).
 *  n_edges    number of edges when edges != NULL.
 *  edges      host int32[2 n_edges] = (u0, v0, u1, v1, ...), 0 <= u, v < n,
 *             u != v, no repeated pair; NULL to generate G(n, M) from
 *             (seed, graph_id).  Maximum degree <= 63.
 *  J          host int8[n_edges] of +-1 when edges != NULL (else ignored).
 *  T          temperature, T >= 0, +inf allowed.
 *  seed       Philox key.  instance_id keys the dynamics; graph_id keys the
 *             generated graph.  Instances with equal (n, c, seed, graph_id)
 *             and no explicit edges share one graph and its couplings, and
 *             so do instances that pass the same edges and J arrays (equal
 *             pointers, n, n_edges and seed); instances with other seeds get
 *             units of their own.
 *  n_replicas 1 <= n_replicas <= 8, equal for all instances of a context.
 *  start      SG_START_*; s0 is host int8[n_replicas][n] of +-1 in vertex
 *             order when start == SG_START_GIVEN. */
typedef struct sg_vb_desc {
    int64_t n;
    double c;
    int64_t n_edges;
    const int32_t* edges;
    const int8_t* J;
    double T;
    uint64_t seed;
    uint32_t instance_id;
    uint32_t graph_id;
    int32_t n_replicas;
    int32_t start;
    const int8_t* s0;
} sg_vb_desc;

/* One Sherrington-Kirkpatrick instance.
 *  n          number of spins, 2 <= n <= 32768 (the paper's largest SK size;
 *             n <= 16384 with real couplings).
 *  J          host int8[n][n] row-major, +-1, symmetric, zero diagonal; NULL
 *             to generate from (seed, graph_id).  Binary couplings +-1/sqrt(N)
 *             (SI, SK section).
 *  Jf         host float32[n][n] row-major, symmetric, zero diagonal, finite:
 *             real couplings (Eq. 1 with Gaussian J_ij of variance 1/N, the
 *             1/sqrt(N) included in the values); J must then be NULL.  The
 *             energy is -sum_{i<j} Jf_ij s_i s_j; the local fields are kept in
 *             IEEE double and a move with x = s_i h_i > 0 is accepted iff
 *             r < floor(ldexp(exp(-beta (2 x)), 32)) (the binary rule with x
 *             real).  A flip's change 2 s_i Jf_ij is added to every field in
 *             flip order, as in the sequential sweep, so the fields are those
 *             of the sequential definition until the first recomputation,
 *             and equal to them within rounding (< 1e-12) after it.
 *             Instances passing the same Jf pointer share one device copy.
 *             All instances of a context have real couplings or none has.
 *  recompute_period  sweeps between exact recomputations of the local fields
 *             (0 selects 64); binary couplings: a mismatch with the
 *             incremental fields makes the next sg_measure return
 *             SG_EPARITY; real couplings: the recomputed fields replace the
 *             incremental ones, and a difference above 1e-9 (1 + |h|)
 *             returns SG_EPARITY.
 *  other fields as for sg_vb_desc. */
typedef struct sg_sk_desc {
    int64_t n;
    const int8_t* J;
    double T;
    uint64_t seed;
    uint32_t instance_id;
    uint32_t graph_id;
    int32_t n_replicas;
    int32_t start;
    const int8_t* s0;
    int32_t recompute_period;
    int32_t reserved;
    const float* Jf;
} sg_sk_desc;

/* Device memory callbacks (for instance a framework's caching allocator).
 * alloc returns a device pointer on the context's device or NULL; free
 * releases one.  With alloc == NULL the library uses hipMalloc/hipFree. */
typedef void* (*sg_alloc_fn)(size_t bytes, void* user);
typedef void (*sg_free_fn)(void* ptr, size_t bytes, void* user);

/* Options shared by both create calls; NULL selects all defaults.
 *  t_max            last measurement time; the grid is {0} U {2^k <= t_max}
 *                   (K = its size).  Snapshots are kept for every grid time.
 *  chains_per_unit  VB: chains updated together by one workgroup (they share
 *                   the graph stream); 0 = automatic.  Has no effect on any
 *                   result.
 *  threads_per_unit VB/SK: workgroup size (64..1024, multiple of 64); 0 =
 *                   automatic.  Has no effect on any result.
 *  split_members    VB: a large graph's unit can be spread over several
 *                   workgroups that exchange each colour class's spins through
 *                   HBM at a device-scope barrier.  0 = automatic (the
 *                   units above twice one CU's share of the batch's work,
 *                   when no unit left whole would outlast them), 1 = never,
 *                   k >= 2 =
 *                   k workgroups for every unit with at least 2 k chunks of
 *                   64 positions per wavefront in its largest colour class.
 *                   Has no effect on any result; a barrier that times out
 *                   (20 s) makes sg_measure return SG_EDEVICE.
 *  t_start          resume (0 = a new run): the time, 0 <= t_start < 2^32,
 *                   of the start configurations the descriptors pass
 *                   (SG_START_GIVEN, typically the spins sg_measure exported
 *                   from a run at that time).  The sweep counter starts at
 *                   t_start, so every random stream (counter-based, keyed by
 *                   the sweep index; Methods) continues where that run
 *                   stopped and the sweeps from t_start on are those of one
 *                   uninterrupted run, bit for bit.  Snapshot slot 0 then
 *                   holds the start configuration (times[0] = t_start); the
 *                   slots of grid times <= t_start are not taken (times[k] =
 *                   -1, their entries 0); accepted counts the flips since
 *                   t_start.  Not with SG_OPT_WINDOW (SG_ENOTSUP; the
 *                   waiting-time configurations before t_start are not
 *                   kept).  Real SK couplings: t_start must be a multiple of
 *                   the recompute period (the fields are then the exact
 *                   direct sums the uninterrupted run also has), else
 *                   SG_EINVAL. */
typedef struct sg_opts {
    int64_t t_max;
    sg_alloc_fn alloc;
    sg_free_fn free;
    void* user;
    int32_t chains_per_unit;
    int32_t threads_per_unit;
    uint32_t flags;
    int32_t split_members;
    int64_t window_tw_max;
    int64_t t_start;
} sg_opts;

/* sg_opts.flags (VB contexts; AUTOTUNE and GRAPH have no effect on any result) */
#define SG_OPT_AUTOTUNE 1u   /* time candidate workgroup sizes per launch group at create
                                (on a saved copy of the state, restored afterwards) */
#define SG_OPT_GRAPH 2u      /* replay each sweep chunk as a captured hipGraph */
/* SG_OPT_WINDOW: also measure the windowed correlation, the paper's estimator
 * of C (Results and discussion: each measurement averages the time interval
 * [t / 2^(1/4), t]; SI, extrapolation to large sizes and times: C(t_w + t,
 * t_w) is averaged over "minor third" intervals of t_w + t whose bounds grow
 * by 2^(1/4)).  Reading used here: interval m holds the times tau = t_w + t
 * with 2^(m/4) <= tau < 2^((m+1)/4), i.e. m = floor(log2 tau^4) (exact
 * integer arithmetic), for m = 0 .. n_bins - 1, n_bins = m(t_max) + 1.  The
 * waiting times are the first kw grid times, those <= window_tw_max
 * (>= 0).  After every sweep ending at a time tau <= t_max, every chain adds,
 * for each waiting time t_w < tau, the overlap sum_i s_i(tau) s_i(t_w) to
 * its sum for (t_w, m(tau)); window_count[k][m] counts the terms, so that
 * window / (window_count n) is C(tau, t_w) averaged over interval m.  Needs
 * t_max >= 1; VB contexts only (SG_ENOTSUP for SK). */
#define SG_OPT_WINDOW 4u
/* SG_OPT_MULTISPIN: the paper's multispin coding (Methods; SI bipartite-graph
 * section): instances that share a graph -- generated from one (n, c, seed,
 * graph_id), or passing one edges array with one seed, whatever J arrays they
 * pass -- are packed 64 chains per work unit, one bit per chain in a 64-bit
 * word per vertex, each chain with its own couplings, temperature and random
 * streams, when they bring at least 16 chains and n <= 16384 (the words stay
 * in LDS); other instances get the per-chain layout.  No effect on any
 * result.  Not combined with SG_OPT_WINDOW (SG_ENOTSUP). */
#define SG_OPT_MULTISPIN 8u
/* SG_OPT_PLAIN_LDS: keep no complemented copy of the spin words in LDS.  By
 * default a per-chain unit that is neither LDS-resident nor split keeps one
 * when it fits, and its adjacency entries then address the neighbour's word
 * or its complement by the sign of the coupling.  A layout choice: no effect
 * on any result. */
#define SG_OPT_PLAIN_LDS 16u

#define SG_MEASURE_OBS 1u    /* times, bond, overlap, gram, accepted */
#define SG_MEASURE_SPINS 2u  /* current spins, vertex order */

/* Observables.  The library fills the four scalars; each array pointer is
 * caller-owned host memory, or NULL to skip it.  For instance i, replica r,
 * grid index k (time times[k]):
 *   bond[i][r][k]      B = sum_{(uv) in E} J_uv s_u s_v (VB; energy -B) or
 *                      sum_{u<v} J_uv s_u s_v with integer J (SK; energy
 *                      -B / sqrt(N));
 *   overlap[i][p][k]   sum_u s^a_u s^b_u for the p-th replica pair a < b
 *                      (lexicographic);
 *   gram[i][r][k][l]   sum_u s_u(t_k) s_u(t_l), so C(t_k, t_l) = gram / N;
 *   accepted[i][r]     accepted flips so far.
 * Entries for grid times not reached yet, and for slots not taken after a
 * resume (times[k] = -1, see sg_opts.t_start), are 0.  spins holds, for each
 * instance in order, n_replicas rows of n int8 +-1 in vertex order. */
typedef struct sg_obs {
    int32_t count;
    int32_t n_replicas;
    int32_t k_cap;
    int32_t k_done;
    int64_t t_done;
    int64_t* times;     /* [k_cap] */
    int64_t* bond;      /* [count][n_replicas][k_cap] */
    int64_t* overlap;   /* [count][n_replicas (n_replicas - 1) / 2][k_cap] */
    int64_t* gram;      /* [count][n_replicas][k_cap][k_cap] */
    int64_t* accepted;  /* [count][n_replicas] */
    int8_t* spins;      /* [sum_i n_replicas n_i] */
    int32_t kw;         /* waiting times of the windowed correlation (0: not measured) */
    int32_t n_bins;     /* its intervals */
    int64_t* window;    /* [count][n_replicas][kw][n_bins] overlap sums (SG_OPT_WINDOW) */
    int64_t* window_count;   /* [kw][n_bins] number of terms of each sum */
    double* bond_real;  /* [count][n_replicas][k_cap] SK with real couplings: B = sum_{u<v}
                           Jf_uv s_u s_v (energy -B; bond is then 0) */
} sg_obs;

/* Creates a context holding `count` VB instances on the current HIP device,
 * builds their graphs (SG_START_RANDOM chains are initialised on the device)
 * and records the t = 0 snapshot.  Synchronous: returns once its own set-up
 * work (on the null stream) is done; work of other contexts keeps running.
 * Different contexts may be created from different host threads at once. */
sg_status sg_create_vb(const sg_vb_desc* d, int32_t count, const sg_opts* o, sg_ctx** out);

/* Same for `count` SK instances. */
sg_status sg_create_sk(const sg_sk_desc* d, int32_t count, const sg_opts* o, sg_ctx** out);

/* Enqueues n_sweeps >= 0 Metropolis sweeps of every chain of the context on
 * `stream` (a hipStream_t; NULL = the null stream) and returns without
 * waiting.  Snapshots are taken on the device whenever the number of sweeps
 * done reaches a grid time <= t_max.  The total number of sweeps must stay
 * below 2^32. */
sg_status sg_sweep(sg_ctx* c, int64_t n_sweeps, void* stream);

/* Computes the observables of every grid time reached so far on `stream`,
 * waits for the stream, and fills `out` (see sg_obs).  Returns SG_EPARITY
 * if an SK field check has failed since the context was created. */
sg_status sg_measure(sg_ctx* c, uint32_t flags, sg_obs* out, void* stream);

/* Variant of sg_measure for callers that cannot allocate memory (code that
 * must not call hipMalloc, such as tight serving loops or hosts that forbid
 * allocation after set-up).  Same observables, same values and the same
 * statuses as sg_measure with flags = SG_MEASURE_OBS, for the arrays of `out`
 * that are not NULL; out->spins must be NULL (SG_EINVAL otherwise).  The
 * measurement kernels stage their results in a fixed device array of
 * 2^20 int64 (8 MiB) that the library holds on each device until the process
 * ends, and the results are copied straight into the caller's arrays: no
 * device or host memory is allocated.  A context needs
 * count R K (1 + K) + count R (R - 1) / 2 K of those entries (K = grid size);
 * larger contexts get SG_ENOTSUP.  Waits for `stream` before returning.
 * Calls that overlap on one device (from several host threads, with any
 * contexts) race on the shared array and must be serialised by the caller. */
sg_status sg_measure_noalloc(sg_ctx* c, sg_obs* out, void* stream);

/* Waits for every stream the context's calls have used (and for its set-up
 * work), never for other contexts, and releases everything it owns.
 * sg_free(NULL) does nothing. */
void sg_free(sg_ctx* c);

/* Fault injection for tests of the SK integrity check (the exact
 * recomputation of the local fields every recompute_period sweeps, SI SK
 * section: the force computation is the path's critical part).  Adds `delta`
 * to the incremental local field H_i of chain (instance, replica) between
 * sweeps, after waiting for the context's streams.  The next recomputation
 * finds the mismatch and overwrites the field with the exact value, and
 * sg_measure returns SG_EPARITY from then on; the trajectory after the
 * corruption is not the method's.  SG_EINVAL for a VB context or indices out
 * of range. */
sg_status sg_sk_corrupt_field(sg_ctx* c, int32_t instance, int32_t replica, int64_t i, int32_t delta);

/* Static description of a status code. */
const char* sg_strerror(sg_status s);

/* Host-side tables of one VB instance, as the library builds them, for
 * tests of the host builder.  Touches no GPU.  Call once with all array
 * pointers NULL to obtain the sizes, then with arrays of at least those
 * sizes.
 *  n_edges, n_colours, max_degree   sizes (out).
 *  edges[2 m], J[m]                 the edge list used (generated or copied).
 *  colour[n]                        greedy colour of each vertex.
 *  order[n]                         vertex at each sweep position.
 *  row_start[n+1], entries[2 m]     adjacency in sweep order: the neighbours
 *                                   of position p are entries[row_start[p] ..
 *                                   row_start[p+1]), each the neighbour's
 *                                   position in bits 0..30 and bit 31 set
 *                                   when the coupling is -1.
 *  thr[64]                          acceptance thresholds thr[x], x < 64. */
typedef struct sg_vb_tables {
    int64_t n_edges;
    int32_t n_colours;
    int32_t max_degree;
    int32_t* edges;
    int8_t* J;
    int32_t* colour;
    int32_t* order;
    int32_t* row_start;
    uint32_t* entries;
    uint64_t* thr;
} sg_vb_tables;

sg_status sg_vb_inspect(const sg_vb_desc* d, sg_vb_tables* out);

/* Host-side SK tables: J[n][n] as used (generated or copied) and the
 * threshold table thr[x] for 0 <= x < n.  Touches no GPU; NULL skips. */
sg_status sg_sk_inspect(const sg_sk_desc* d, int8_t* J, uint64_t* thr);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
