// Sherrington-Kirkpatrick sweeps with real couplings (Eq. 1: Gaussian J_ij
// of variance 1/N, given as float32) on gfx950.
//
// The local fields h_i = sum_j J_ij s_j are real and are kept in IEEE double.
// A flip of s_i changes every field by 2 s_i J_ij (new s_i): the product is
// exact in double, so a field's value depends only on the order in which the
// flips reach it, and this kernel applies them to every field in flip order,
// as the sequential definition does.  Every `period` sweeps the fields are
// recomputed directly (sk_recompute for real couplings below), which bounds
// the rounding drift of the incremental sums (SI, SK section: the force is
// the costly part and is recomputed periodically).
//
// Acceptance of a move with x = s_i h_i: x <= 0 accepts, else the move is
// accepted iff r < floor(ldexp(exp(-beta (2 x)), 32)) in double, r the same
// 32-bit uniform as for binary couplings.
//
// One workgroup runs one chain, visiting i = 0..N-1 in blocks of 64 spins:
//  1. the block's 64 x 64 coupling tile is staged in LDS (loaded during the
//     block before it);
//  2. one wavefront decides the block in rounds: every undecided lane tests
//     its move with its current field; the first lane that accepts flips,
//     the lanes before it keep their spins, and the lanes after it add the
//     flip's change to their fields (from the tile) and are tested again;
//  3. all wavefronts apply the block's flips, in order, to every field not
//     already updated in step 2 (the fields before a flip's lane in the
//     block and all fields outside it), streaming the flipped spins' rows.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

// Threads per chain: in step 3 a thread takes 4 fields at a time, so with
// 1024 threads the fields of N <= 4096 take one pass and a block's row loads
// cost one memory latency (with 256 threads, four passes one after another).
#ifndef SG_SKG_THREADS
#define SG_SKG_THREADS 1024
#endif
constexpr int kSkgThreads = SG_SKG_THREADS;
typedef float v4f __attribute__((ext_vector_type(4)));

struct SkgLds {
    double* H;          // [n]
    uint32_t* bits;     // [wn + 2]
    float* tile;        // [64][64]: rows of the block's spins, its columns
    int32_t* flips;     // [64]: lane | (new spin -1) << 31, in flip order
    int32_t* nflip;     // [2]
    uint32_t* rnd;      // [2][64]: a block's acceptance uniforms (two blocks in turn)
    double* xlo;        // [2][64]: their acceptance bounds (SkgBound)
    double* xhi;        // [2][64]
};

__device__ __forceinline__ SkgLds skg_carve(uint8_t* base, int32_t n, int32_t wn)
{
    SkgLds L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t* p = base + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    L.H = (double*)take((size_t)n * 8);
    L.bits = (uint32_t*)take((size_t)(wn + 2) * 4);
    L.tile = (float*)take(64 * 64 * 4);
    L.flips = (int32_t*)take(64 * 4);
    L.nflip = (int32_t*)take(16);
    L.rnd = (uint32_t*)take(2 * 64 * 4);
    L.xlo = (double*)take(2 * 64 * 8);
    L.xhi = (double*)take(2 * 64 * 8);
    return L;
}

// 32-bit acceptance uniform of position p in sweep t (the two half-word
// streams of the binary model, both drawn).
__device__ __forceinline__ uint32_t skg_uniform(const SkChain* ch, uint32_t t, uint32_t p)
{
    const U4 A = philox_stream(ch->seed, p >> 3, t, kDomSweepHi, ch->rep, ch->inst);
    const U4 B = philox_stream(ch->seed, p >> 3, t, kDomSweepLo, ch->rep, ch->inst);
    return (half_word(A, p & 7u) << 16) | half_word(B, p & 7u);
}

__device__ __forceinline__ bool skg_accept(double x, double beta, uint32_t r)
{
    if (x <= 0.0) return true;
    const double p = exp(-beta * (2.0 * x));
    const uint64_t thr = (uint64_t)floor(ldexp(p, 32));
    return (uint64_t)r < thr;
}

// The same decision through a per-lane bound on x, fixed by r before the
// rounds: r < floor(2^32 exp(-2 beta x)) holds iff 2^32 exp(-2 beta x) >=
// r + 1, i.e. x <= xc = -ln((r + 1) 2^-32) / (2 beta).  Outside a band of
// relative width 1e-9 around xc (far wider than the rounding of exp, ln and
// the division) the bound decides; inside it, and for beta = 0 or infinite,
// the rule itself does, so every decision is that of skg_accept.
struct SkgBound {
    double lo, hi;   // accept below lo, reject above hi, else evaluate
};

__device__ __forceinline__ SkgBound skg_bound(double beta, uint32_t r)
{
    if (!(beta > 0.0) || !(beta < 1e300)) return SkgBound{0.0, 1e308};
    const double xc = -log(((double)r + 1.0) * 0x1p-32) / (2.0 * beta);
    const double band = 1e-9 * (xc + 1.0);
    return SkgBound{xc - band, xc + band};
}

__device__ __forceinline__ bool skg_accept_b(double x, double beta, uint32_t r, const SkgBound& bd)
{
    if (x <= 0.0 || x < bd.lo) return true;
    if (x > bd.hi) return false;
    return skg_accept(x, beta, r);
}

__global__ void __launch_bounds__(kSkgThreads) skg_sweep_kernel(const SkChain* __restrict__ chains, int64_t t0,
                                                                int32_t nsw, int64_t t_max)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t skg_smem[];
    const SkChain* ch = chains + blockIdx.x;
    const int32_t n = ch->n, wn = ch->words_n;
    const SkgLds L = skg_carve(skg_smem, n, wn);
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const SG_G float* __restrict__ J = gl(ch->Jf);
    const double beta = ch->beta;
    for (int32_t i = tid; i < n; i += nthr) L.H[i] = gl(ch->Hd)[i];
    for (int32_t w = tid; w < wn + 2; w += nthr) L.bits[w] = w < wn ? gl(ch->state)[w] : 0u;
    __syncthreads();
    const int32_t NB = (n + 63) >> 6;
    const bool vec4 = (n & 3) == 0;   // rows start 16-byte aligned
    unsigned long long acc = 0;   // accepted flips (wave 0, lane 0)

    // 1. the coupling tile of a block, T[i][j] = J[p0 + i][p0 + j], is loaded
    //    into registers (4096 / threads floats per thread, 16-byte loads when the rows
    //    are 16-byte aligned) while the block before it is decided and
    //    applied, and stored to LDS at the end of that block
    constexpr int TS = 64 * 64 / kSkgThreads, T4 = TS / 4;   // tile floats, 16-byte loads per thread
    static_assert(TS * kSkgThreads == 64 * 64 && T4 * 4 == TS, "the tile splits evenly into 16-byte parts");
    v4f tv[T4];
    float ts[TS];
    auto tile_load = [&](int32_t bb) {
        const int32_t q0 = bb << 6;
        const int32_t mm = min(64, n - q0);
        if (vec4) {
#pragma unroll
            for (int k = 0; k < T4; ++k) {
                const int32_t idx = tid + k * kSkgThreads;
                const int32_t i = idx >> 4, j = (idx & 15) << 2;
                const v4f z = {0.f, 0.f, 0.f, 0.f};
                tv[k] = (i < mm && j < mm) ? *(const SG_G v4f*)(J + (int64_t)(q0 + i) * n + q0 + j) : z;
            }
        } else {
#pragma unroll
            for (int k = 0; k < TS; ++k) {
                const int32_t idx = tid + k * kSkgThreads;
                const int32_t i = idx >> 6, j = idx & 63;
                ts[k] = (i < mm && j < mm) ? J[(int64_t)(q0 + i) * n + q0 + j] : 0.0f;
            }
        }
    };
    auto tile_store = [&]() {
        if (vec4) {
#pragma unroll
            for (int k = 0; k < T4; ++k) {
                const int32_t idx = tid + k * kSkgThreads;
                *(v4f*)(L.tile + ((idx >> 4) << 6) + ((idx & 15) << 2)) = tv[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < TS; ++k) L.tile[tid + k * kSkgThreads] = ts[k];
        }
    };
    if (nsw > 0) tile_load(0);

    // The acceptance uniforms of a block's lanes and their bounds on x are
    // drawn by wavefront 1 while wavefront 0 decides the block before it
    // (they depend on the sweep and the position only), into the half of
    // the double buffer that block will read.
    static_assert(kSkgThreads >= 128, "wavefront 1 draws the next block's uniforms");
    auto draw = [&](int32_t bb, uint32_t tt, int32_t half) {
        const int32_t p = (bb << 6) + lane;
        const uint32_t r = p < n ? skg_uniform(ch, tt, (uint32_t)p) : 0u;
        const SkgBound bd = skg_bound(beta, r);
        L.rnd[half * 64 + lane] = r;
        L.xlo[half * 64 + lane] = bd.lo;
        L.xhi[half * 64 + lane] = bd.hi;
    };
    if (nsw > 0) {
        tile_store();
        if (wave == 1) draw(0, (uint32_t)t0, 0);
    }
    __syncthreads();
    int32_t half = 0;   // the buffer half of the current block

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        for (int32_t b = 0; b < NB; ++b, half ^= 1) {
            const int32_t p0 = b << 6;
            const int32_t m = min(64, n - p0);
            // the next block's tile (the first block of the next sweep after
            // the last one), stored to LDS once this block's decisions no
            // longer read the tile (after its flips are applied)
            const bool next_tile = b + 1 < NB || s + 1 < nsw;
            if (b + 1 < NB)
                tile_load(b + 1);
            else if (s + 1 < nsw)
                tile_load(0);
            // 2. decisions (wavefront 0)
            if (wave == 0) {
                const bool act = lane < m;
                const int32_t p = p0 + lane;
                double h = act ? L.H[p] : 0.0;
                double sp = act && ((L.bits[p >> 5] >> (p & 31)) & 1u) ? -1.0 : 1.0;
                const uint32_t r = L.rnd[half * 64 + lane];
                const SkgBound bd{L.xlo[half * 64 + lane], L.xhi[half * 64 + lane]};
                // a lane flips at most once in its block, so the new spin
                // of a flipping lane is the opposite of its spin here
                const unsigned long long was_neg = __builtin_amdgcn_ballot_w64(act && sp < 0.0);
                int32_t first = 0;   // lanes below `first` are decided
                int32_t nf = 0;
                for (;;) {
                    const bool cand = act && lane >= first && skg_accept_b(sp * h, beta, r, bd);
                    const unsigned long long mk = __builtin_amdgcn_ballot_w64(cand);
                    if (mk == 0ull) break;
                    const int32_t i = __builtin_ctzll(mk);
                    if (lane == i) sp = -sp;
                    const double si = ((was_neg >> i) & 1ull) ? 1.0 : -1.0;   // the new spin of lane i
                    if (lane > i) h = h + (2.0 * si) * (double)L.tile[i * 64 + lane];
                    if (lane == 0) L.flips[nf] = i | (si < 0.0 ? (int32_t)0x80000000 : 0);
                    ++nf;
                    first = i + 1;
                }
                if (act) L.H[p] = h;
                const unsigned long long neg = __builtin_amdgcn_ballot_w64(act && sp < 0.0);
                if (lane == 0) {
                    L.bits[p0 >> 5] = (uint32_t)neg;
                    if (m > 32) L.bits[(p0 >> 5) + 1] = (uint32_t)(neg >> 32);
                    L.nflip[0] = nf;
                    acc += (unsigned long long)nf;
                }
            } else if (wave == 1) {
                if (b + 1 < NB)
                    draw(b + 1, t, half ^ 1);
                else if (s + 1 < nsw)
                    draw(0, t + 1u, half ^ 1);
            }
            __syncthreads();
            // 3. the block's flips reach every other field, in flip order
            //    (fields after a flip's lane in the block already have it);
            //    each thread takes 4 consecutive fields and loads the rows of
            //    up to 8 flips at once
            const int32_t nf = L.nflip[0];
            if (nf > 0) {
                if (vec4) {
                    for (int32_t k4 = tid; k4 < (n >> 2); k4 += nthr) {
                        const int32_t k0 = k4 << 2;
                        double h[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) h[c] = L.H[k0 + c];
                        for (int32_t f0 = 0; f0 < nf; f0 += 8) {
                            v4f v[8];
                            int32_t fi[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int32_t f = f0 + u;
                                fi[u] = f < nf ? L.flips[f] : 0;
                                const v4f z = {0.f, 0.f, 0.f, 0.f};
                                v[u] = z;
                                if (f < nf) v[u] = *(const SG_G v4f*)(J + (int64_t)(p0 + (fi[u] & 63)) * n + k0);
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                if (f0 + u >= nf) break;
                                const int32_t i = p0 + (fi[u] & 63);
                                const double a = fi[u] < 0 ? -2.0 : 2.0;
                                const float vv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                                for (int c = 0; c < 4; ++c) {
                                    const int32_t k = k0 + c;
                                    if (!(k > i && k < p0 + m)) h[c] = h[c] + a * (double)vv[c];
                                }
                            }
                        }
#pragma unroll
                        for (int c = 0; c < 4; ++c) L.H[k0 + c] = h[c];
                    }
                } else {
                    for (int32_t k = tid; k < n; k += nthr) {
                        double h = L.H[k];
                        for (int32_t f0 = 0; f0 < nf; f0 += 8) {
                            float v[8];
                            int32_t fi[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int32_t f = f0 + u;
                                fi[u] = f < nf ? L.flips[f] : 0;
                                v[u] = f < nf ? J[(int64_t)(p0 + (fi[u] & 63)) * n + k] : 0.0f;
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                if (f0 + u >= nf) break;
                                const int32_t i = p0 + (fi[u] & 63);
                                if (!(k > i && k < p0 + m)) h = h + (fi[u] < 0 ? -2.0 : 2.0) * (double)v[u];
                            }
                        }
                        L.H[k] = h;
                    }
                }
            }
            if (next_tile) tile_store();
            __syncthreads();
        }
        const int64_t tn = t0 + s + 1;
        if (tn <= t_max && (tn & (tn - 1)) == 0) {
            const int k = 1 + (63 - __clzll((unsigned long long)tn));
            for (int32_t w = tid; w < wn; w += nthr) gl(ch->snap)[(int64_t)k * wn + w] = L.bits[w];
        }
    }
    for (int32_t i = tid; i < n; i += nthr) gl(ch->Hd)[i] = L.H[i];
    for (int32_t w = tid; w < wn; w += nthr) gl(ch->state)[w] = L.bits[w];
    if (tid == 0 && acc) atomicAdd(ch->accepted, acc);
}

// Direct fields h = J s of every chain of one sample, in a fixed order (rows
// by wavefronts, columns strided over lanes, then a fixed butterfly), in
// double; with `check`, a field that differs from the incremental one by more
// than 1e-9 (1 + |h|) raises bit 0 of the error word (the rounding drift of a
// period is many orders of magnitude below that).  grid = (row blocks of 16,
// samples), one wavefront per block.
__global__ void __launch_bounds__(64) skg_recompute_kernel(const SkSample* __restrict__ samples,
                                                           const SkChain* __restrict__ chains, int check,
                                                           int* err)
{
    const SkSample* sm = samples + blockIdx.y;
    const int32_t n = sm->n;
    const int lane = threadIdx.x;
    const int32_t i0 = blockIdx.x * 16;
    if (i0 >= n) return;
    const SG_G float* __restrict__ J = gl(sm->Jf);
    for (int32_t c = 0; c < sm->nch; ++c) {
        const SkChain* ch = chains + sm->chain0 + c;
        const SG_G uint32_t* st = gl(ch->state);
        for (int32_t i = i0; i < min(n, i0 + 16); ++i) {
            const SG_G float* row = J + (int64_t)i * n;
            double part = 0.0;
            for (int32_t j = lane; j < n; j += 64) {
                const double v = (double)row[j];
                part += ((st[j >> 5] >> (j & 31)) & 1u) ? -v : v;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
            if (lane == 0) {
                const double old = ch->Hd[i];
                if (check && fabs(old - part) > 1e-9 * (1.0 + fabs(part))) atomicOr(err, 1);
                ch->Hd[i] = part;
            }
        }
    }
}

// Bond sums B = (1/2) sum_i s_i (J s)_i of every snapshot (chain c, grid time
// k) of one sample, in double and in a fixed order: each wavefront forms
// partial sums over 16 rows, written to part[sample][row block][column], then
// skg_bond_reduce adds the row blocks in order.  The columns (snapshots) go in
// tiles of 8, so a row of J is read once per tile: lane l adds, for its
// entries j = l, l + 64, ..., the signed couplings s_j J_ij of each column,
// multiplies by the row's spin s_i (the same on every lane) and keeps the
// sum; the wavefront sum is formed once per tile.  grid = (row blocks of 16,
// samples).
__global__ void __launch_bounds__(64) skg_bond_kernel(const SkSample* __restrict__ samples,
                                                      const SkChain* __restrict__ chains, int kd, int nrb,
                                                      int ncol_cap, double* __restrict__ part)
{
    constexpr int CT = 8;   // columns per tile
    const SkSample* sm = samples + blockIdx.y;
    const int32_t n = sm->n;
    const int lane = threadIdx.x;
    const int32_t i0 = blockIdx.x * 16;
    if (i0 >= n) return;
    const SG_G float* __restrict__ J = gl(sm->Jf);
    const int32_t ncol = sm->nch * kd;
    const int32_t i1 = min(n, i0 + 16);
    for (int32_t c0 = 0; c0 < ncol; c0 += CT) {
        const SG_G uint32_t* sn[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int32_t col = min(c0 + c, ncol - 1);
            const SkChain* ch = chains + sm->chain0 + col / kd;
            sn[c] = gl(ch->snap) + (int64_t)(col % kd) * ch->words_n;
        }
        double acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = 0.0;
        for (int32_t i = i0; i < i1; ++i) {
            const SG_G float* row = J + (int64_t)i * n;
            double d[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) d[c] = 0.0;
            for (int32_t j = lane; j < n; j += 64) {
                const double v = (double)row[j];
#pragma unroll
                for (int c = 0; c < CT; ++c) d[c] += ((sn[c][j >> 5] >> (j & 31)) & 1u) ? -v : v;
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] += ((sn[c][i >> 5] >> (i & 31)) & 1u) ? -d[c] : d[c];
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            double a = acc[c];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
            if (lane == 0 && c0 + c < ncol) part[((int64_t)blockIdx.y * nrb + blockIdx.x) * ncol_cap + c0 + c] = a;
        }
    }
}

// out[chain][k] = (1/2) sum over row blocks (in order) of the partial sums.
__global__ void skg_bond_reduce(const SkSample* __restrict__ samples, int n_samples, int kd, int nrb,
                                int ncol_cap, int k_cap, const double* __restrict__ part,
                                double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_samples * ncol_cap) return;
    const int32_t smp = (int32_t)(idx / ncol_cap), col = (int32_t)(idx % ncol_cap);
    const SkSample* sm = samples + smp;
    if (col >= sm->nch * kd) return;
    const int32_t rbs = (sm->n + 15) / 16;
    double s = 0.0;
    for (int32_t rb = 0; rb < rbs; ++rb) s += part[((int64_t)smp * nrb + rb) * ncol_cap + col];
    out[(int64_t)(sm->chain0 + col / kd) * k_cap + col % kd] = 0.5 * s;
}

}  // namespace

size_t skg_lds_bytes(int32_t n)
{
    const size_t wn = (size_t)(n + 31) / 32;
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return r16((size_t)n * 8) + r16((wn + 2) * 4) + 64 * 64 * 4 + 64 * 4 + 16 + 2 * 64 * 4 + 2 * 2 * 64 * 8;
}

hipError_t skg_sweep(const SkChain* chains, int n_chains, size_t lds_bytes, int64_t t0, int32_t n_sweeps,
                     int64_t t_max, hipStream_t s)
{
    if (n_chains <= 0 || n_sweeps <= 0) return hipSuccess;
    static const hipError_t attr = hipFuncSetAttribute((const void*)skg_sweep_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(skg_sweep_kernel, dim3(n_chains), dim3(kSkgThreads), lds_bytes, s, chains, t0, n_sweeps,
                       t_max);
    return hipGetLastError();
}

hipError_t skg_recompute(const SkSample* samples, int n_samples, const SkChain* chains, int max_n, int check,
                         int* err_flag, hipStream_t s)
{
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(skg_recompute_kernel, dim3((max_n + 15) / 16, n_samples), dim3(64), 0, s, samples, chains,
                       check, err_flag);
    return hipGetLastError();
}

hipError_t skg_bond(const SkSample* samples, int n_samples, const SkChain* chains, int max_n, int max_nch,
                    int k_done, int k_cap, double* part, double* out, hipStream_t s)
{
    if (n_samples <= 0 || k_done <= 0) return hipSuccess;
    const int nrb = (max_n + 15) / 16, ncol_cap = max_nch * k_cap;
    hipLaunchKernelGGL(skg_bond_kernel, dim3(nrb, n_samples), dim3(64), 0, s, samples, chains, k_done, nrb,
                       ncol_cap, part);
    const int64_t tot = (int64_t)n_samples * ncol_cap;
    hipLaunchKernelGGL(skg_bond_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, samples, n_samples,
                       k_done, nrb, ncol_cap, k_cap, part, out);
    return hipGetLastError();
}

}  // namespace sg
