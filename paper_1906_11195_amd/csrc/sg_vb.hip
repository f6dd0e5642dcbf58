// Viana-Bray Metropolis sweeps on gfx950.
//
// One workgroup owns one work unit: a graph stored in sweep order (the
// colour classes of a proper colouring, the paper's bipartite parallel update
// generalised; SI "Simulations of the Bethe Lattice on GPUs") and up to eight
// chains that share it.  The chains' spins stay in LDS for the whole launch,
// packed vertex-major (rpad bits per position, bit c = chain c), so that one
// LDS read of a neighbour returns its spin in every chain.
//
// A sweep visits colour class 0, 1, ...; inside a class all positions are
// independent (no two are adjacent).  A class is cut into aligned chunks of 64
// positions; wavefront w of the workgroup updates chunks w, w + W, ... of the
// class (lane i takes position 64 b + i of block b), for every chain of the
// unit.  Workgroup barriers separate classes only.  Each wavefront streams
// the adjacency of its chunks straight from HBM through a two-stage register
// pipeline: the row starts of the chunk after next and the entries of the
// next chunk are in flight while the current chunk is updated.
//
// Metropolis rule (Methods; SI bipartite-graph section): with x = s_p h_p the
// move is accepted if x <= 0, else iff r < thr[x], thr[x] = floor(2^32
// exp(-2x/T)).  r = (A << 16) | B with A, B half-words of two Philox streams.
// The eight lanes of an aligned group of 8 positions share one Philox block
// per chain: lane j computes the block of chain j and the group exchanges the
// half-words through LDS.  B is computed only when A ties with the high half
// of the threshold (probability 2^-16).
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

constexpr int kDMax = 8;   // adjacency entries prefetched per position

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct VbLds {
    uint32_t* sp;                 // spins, vertex-major
    uint32_t* thi;                // [8][64]
    uint32_t* tlo;                // [8][64]
    unsigned long long* accs;     // [8]
    uint4* xch;                   // [threads] Philox blocks
    int32_t* area;                // resident adjacency: row starts, then entries
};

__device__ __forceinline__ VbLds vb_carve(uint32_t* smem, int32_t sw, int nthr)
{
    VbLds L;
    L.sp = smem;
    L.thi = smem + ((sw + 3) & ~3);
    L.tlo = L.thi + kVbMaxChains * kVbXMax;
    L.accs = (unsigned long long*)(L.tlo + kVbMaxChains * kVbXMax);
    L.xch = (uint4*)(L.accs + kVbMaxChains);
    L.area = (int32_t*)(L.xch + nthr);
    return L;
}

// Chunk cursor of one wavefront: sweep s, colour class k, chunk j of the class
// (the aligned block (cls[k] >> 6) + j of 64 positions).
struct Cursor {
    int32_t s, k, j;
};

template <class PC>
__device__ __forceinline__ int32_t n_chunks(PC cls, int32_t k)
{
    const int32_t lo = cls[k], hi = cls[k + 1];
    return hi > lo ? ((hi - 1) >> 6) - (lo >> 6) + 1 : 0;
}

// Moves to the next chunk owned by wavefront `wave`; false past the launch.
template <class PC>
__device__ __forceinline__ bool cursor_next(Cursor& c, int W, int wave, int32_t ncls, PC cls, int32_t nsw)
{
    c.j += W;
    for (;;) {
        if (c.j < n_chunks(cls, c.k)) return true;
        c.j = wave;
        if (++c.k == ncls) {
            c.k = 0;
            if (++c.s >= nsw) return false;
        }
    }
}

struct Stage {
    int32_t q, r0, r1;
    uint32_t e[kDMax];
};

// `row` and `ent` point to HBM, or to LDS when the adjacency is resident.
template <class PR, class PC>
__device__ __forceinline__ void load_rows(PR row, PC cls, const Cursor& c, int lane, Stage& st)
{
    const int32_t lo = cls[c.k], hi = cls[c.k + 1];
    st.q = (((lo >> 6) + c.j) << 6) + lane;
    const bool act = st.q >= lo && st.q < hi;
    st.r0 = act ? row[st.q] : 0;
    st.r1 = act ? row[st.q + 1] : 0;
}

template <class PE>
__device__ __forceinline__ void load_ents(PE ent, Stage& st)
{
    const int32_t deg = st.r1 - st.r0;
#pragma unroll
    for (int d = 0; d < kDMax; ++d) st.e[d] = d < deg ? ent[st.r0 + d] : 0u;
}

// Updates the positions of one chunk for every chain of the unit.
template <int RPAD, class PE>
__device__ __forceinline__ void vb_chunk(const VbUnit* __restrict__ up, const VbLds& L, PE ent, const Stage& st,
                                         int32_t lo, int32_t hi, uint32_t t, int32_t nch,
                                         uint64_t key, uint32_t my_rep, uint32_t my_inst,
                                         uint32_t* acc)
{
    const int tid = threadIdx.x;
    const int32_t q = st.q;
    const int cc = tid & 7;

    // Philox block of chain cc for the group of q (shared by the 8 lanes).
    U4 A = U4{0, 0, 0, 0};
    if (cc < nch) A = philox_stream(key, (uint32_t)q >> 3, t, kDomSweepHi, my_rep, my_inst);
    L.xch[tid] = make_uint4(A.x, A.y, A.z, A.w);
    wave_sync();
    if (q < lo || q >= hi) return;

    const uint32_t ob = (uint32_t)q * RPAD;
    const uint32_t own = L.sp[ob >> 5] >> (ob & 31u);
    const int32_t deg = st.r1 - st.r0;
    uint32_t c0 = 0, c1 = 0;
    auto bond = [&](uint32_t en) {
        const uint32_t qb = (en & 0x7fffffffu) * RPAD;
        // bit c of f is 1 iff the bond (q, neighbour) is unsatisfied in chain c
        const uint32_t f = (L.sp[qb >> 5] >> (qb & 31u)) ^ own ^ (uint32_t)((int32_t)en >> 31);
        if (RPAD == 1) {
            c0 += f & 1u;
        } else {
            // one byte counter per chain (degree <= 63)
            c0 += ((f & 0xFu) * 0x00204081u) & 0x01010101u;
            if (RPAD == 8) c1 += (((f >> 4) & 0xFu) * 0x00204081u) & 0x01010101u;
        }
    };
#pragma unroll
    for (int d = 0; d < kDMax; ++d) {
        if (!__any(d < deg)) break;
        if (d < deg) bond(st.e[d]);
    }
    for (int32_t d = kDMax; d < deg; ++d) bond(ent[st.r0 + d]);

    const uint32_t* gx = (const uint32_t*)(L.xch + (tid & ~7));
    const uint32_t hsel = (uint32_t)tid & 7u;
    uint32_t fl = 0;
#pragma unroll
    for (int c = 0; c < RPAD; ++c) {
        if (c >= nch) break;
        const uint32_t cnt = RPAD == 1 ? c0 : (((c < 4) ? (c0 >> (8 * c)) : (c1 >> (8 * (c - 4)))) & 0xFFu);
        const int32_t x = deg - 2 * (int32_t)cnt;   // x = s_q h_q
        bool flip = x <= 0;
        if (!flip) {
            const uint32_t th = L.thi[c * kVbXMax + x];
            const uint32_t rh = (gx[4 * c + (hsel >> 1)] >> (16u * (hsel & 1u))) & 0xffffu;
            flip = rh < th;
            if (rh == th) {
                const U4 B = philox_stream(key, (uint32_t)q >> 3, t, kDomSweepLo, up->rep[c], up->inst[c]);
                flip = half_word(B, hsel) < L.tlo[c * kVbXMax + x];
            }
        }
        if (flip) {
            fl |= 1u << c;
            acc[c] += 1;
        }
    }
    if (fl) atomicXor(&L.sp[ob >> 5], fl << (ob & 31u));
}

template <int RPAD>
__device__ void vb_snapshot(const VbUnit* __restrict__ up, const uint32_t* __restrict__ sp, int k)
{
    const int32_t n = up->n, wn = up->words_n, nch = up->nch;
    for (int32_t idx = threadIdx.x; idx < nch * wn; idx += blockDim.x) {
        const int32_t c = idx / wn;
        const int32_t w = idx - c * wn;
        uint32_t bits = 0;
        const int32_t pe = min(32, n - 32 * w);
        for (int32_t i = 0; i < pe; ++i) {
            const uint32_t b = (uint32_t)(32 * w + i) * RPAD + (uint32_t)c;
            bits |= ((sp[b >> 5] >> (b & 31u)) & 1u) << i;
        }
        gl(up->snap[c])[(int64_t)k * wn + w] = bits;
    }
}

template <int RPAD, class PR, class PE, class PC>
__device__ void vb_loop(const VbUnit* __restrict__ up, const VbLds& L, PR row, PE ent, PC cls, int64_t t0,
                        int32_t nsw, int64_t t_max, int lane, int wave, int W);

template <int RPAD, bool RES>
__device__ void vb_run(const VbUnit* __restrict__ up, uint32_t* smem, int64_t t0, int32_t nsw,
                       int64_t t_max)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    // wave index made explicitly wave-uniform: the chunk cursor then lives in
    // scalar registers and class bounds come from scalar loads
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), W = nthr >> 6;
    const int32_t sw = up->state_words, nch = up->nch, ncls = up->ncls;
    const SG_G int32_t* __restrict__ cls = gl(up->cls);
    const VbLds L = vb_carve(smem, sw, nthr);

    const SG_G uint32_t* gstate = gl(up->state);
    for (int32_t w = tid; w < sw; w += nthr) L.sp[w] = gstate[w];
    for (int i = tid; i < kVbMaxChains * kVbXMax; i += nthr) {
        L.thi[i] = (&up->thr_hi[0][0])[i];
        L.tlo[i] = (&up->thr_lo[0][0])[i];
    }
    if (tid < kVbMaxChains) L.accs[tid] = 0;
    if (RES) {
        const int32_t n = up->n;
        const SG_G int32_t* grow = gl(up->row);
        const SG_G uint32_t* gent = gl(up->ent);
        for (int32_t i = tid; i <= n; i += nthr) L.area[i] = grow[i];
        uint32_t* re = (uint32_t*)(L.area + n + 1);
        for (int32_t i = tid; i < up->m2; i += nthr) re[i] = gent[i];
        __syncthreads();
        vb_loop<RPAD>(up, L, (const int32_t*)L.area, (const uint32_t*)(L.area + n + 1), cls, t0, nsw,
                      t_max, lane, wave, W);
    } else {
        vb_loop<RPAD>(up, L, gl(up->row), gl(up->ent), cls, t0, nsw, t_max, lane, wave, W);
    }
    for (int32_t w = tid; w < sw; w += nthr) gl(up->state)[w] = L.sp[w];
    __syncthreads();
    if (tid < nch) atomicAdd(up->accepted[tid], L.accs[tid]);
}

// The sweep loop of one unit, for adjacency pointers in HBM or in LDS.
template <int RPAD, class PR, class PE, class PC>
__device__ void vb_loop(const VbUnit* __restrict__ up, const VbLds& L, PR row, PE ent, PC cls, int64_t t0,
                        int32_t nsw, int64_t t_max, int lane, int wave, int W)
{
    const int tid = threadIdx.x;
    const int32_t nch = up->nch, ncls = up->ncls;
    // chain whose Philox block this lane computes
    const uint64_t key = up->key;
    const int cc = tid & 7;
    const uint32_t my_rep = cc < nch ? up->rep[cc] : 0u;
    const uint32_t my_inst = cc < nch ? up->inst[cc] : 0u;

    // pipeline: E = chunk to update next (rows + entries), R = the one after
    // (rows only)
    Stage E, R;
    Cursor cR{0, 0, wave - W};
    bool haveR = nsw > 0 && cursor_next(cR, W, wave, ncls, cls, nsw);
    if (haveR) {
        load_rows(row, cls, cR, lane, E);
        load_ents(ent, E);
        haveR = cursor_next(cR, W, wave, ncls, cls, nsw);
        if (haveR) load_rows(row, cls, cR, lane, R);
    }
    __syncthreads();

    uint32_t acc[RPAD];
#pragma unroll
    for (int c = 0; c < RPAD; ++c) acc[c] = 0;

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        for (int32_t k = 0; k < ncls; ++k) {
            const int32_t lo = cls[k], hi = cls[k + 1];
            const int32_t nck = n_chunks(cls, k);
            for (int32_t j = wave; j < nck; j += W) {
                const Stage cur = E;
                if (haveR) {
                    E.q = R.q;
                    E.r0 = R.r0;
                    E.r1 = R.r1;
                    load_ents(ent, E);
                    haveR = cursor_next(cR, W, wave, ncls, cls, nsw);
                    if (haveR) load_rows(row, cls, cR, lane, R);
                }
                vb_chunk<RPAD>(up, L, ent, cur, lo, hi, t, nch, key, my_rep, my_inst, acc);
            }
            __syncthreads();
        }
        const int64_t tn = t0 + s + 1;
        if (tn <= t_max && (tn & (tn - 1)) == 0) {
            vb_snapshot<RPAD>(up, L.sp, 1 + (63 - __clzll((unsigned long long)tn)));
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < RPAD; ++c)
        if (c < nch && acc[c]) atomicAdd(&L.accs[c], (unsigned long long)acc[c]);
}

// t0p: device-resident number of sweeps done before this launch (read once;
// the counter is advanced by vb_advance_kernel after every launch group), so
// a captured graph of the sweep loop can be replayed unchanged.
__global__ void __launch_bounds__(1024) vb_sweep_kernel(const VbUnit* __restrict__ units,
                                                        const int64_t* __restrict__ t0p,
                                                        int32_t nsw, int64_t t_max)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
    const VbUnit* up = (const VbUnit*)(gl(units) + blockIdx.x);
    const int64_t t0 = *gl(t0p);
    if (up->resident) {
        switch (up->rpad) {
            case 1: vb_run<1, true>(up, smem, t0, nsw, t_max); break;
            case 2: vb_run<2, true>(up, smem, t0, nsw, t_max); break;
            case 4: vb_run<4, true>(up, smem, t0, nsw, t_max); break;
            default: vb_run<8, true>(up, smem, t0, nsw, t_max); break;
        }
    } else {
        switch (up->rpad) {
            case 1: vb_run<1, false>(up, smem, t0, nsw, t_max); break;
            case 2: vb_run<2, false>(up, smem, t0, nsw, t_max); break;
            case 4: vb_run<4, false>(up, smem, t0, nsw, t_max); break;
            default: vb_run<8, false>(up, smem, t0, nsw, t_max); break;
        }
    }
}

__global__ void vb_advance_kernel(int64_t* t, int32_t nsw)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += nsw;
}

// Initial configurations and the t = 0 snapshot.
__global__ void __launch_bounds__(1024) vb_init_kernel(const VbUnit* __restrict__ units)
{
    const VbUnit* up = units + blockIdx.x;
    const int32_t n = up->n, wn = up->words_n, nch = up->nch, rpad = up->rpad;
    for (int32_t idx = threadIdx.x; idx < nch * wn; idx += blockDim.x) {
        const int32_t c = idx / wn;
        const int32_t w = idx - c * wn;
        uint32_t bits;
        if (up->init_mode[c] == 0) {
            const U4 o = philox_stream(up->seed[c], (uint32_t)(w >> 2), 0u, kDomInit, up->rep[c],
                                       up->inst[c]);
            bits = word_of(o, (uint32_t)(w & 3));
        } else if (up->init_mode[c] == 1) {
            bits = 0;
        } else {
            bits = up->given[c][w];
        }
        const int32_t pe = n - 32 * w;
        if (pe < 32) bits &= (1u << pe) - 1u;
        up->snap[c][w] = bits;
    }
    __syncthreads();
    const int32_t per = 32 / rpad;
    for (int32_t w = threadIdx.x; w < up->state_words; w += blockDim.x) {
        uint32_t word = 0;
        for (int32_t i = 0; i < per; ++i) {
            const int32_t p = w * per + i;
            if (p >= n) break;
            for (int32_t c = 0; c < nch; ++c) {
                const uint32_t b = (up->snap[c][p >> 5] >> (p & 31)) & 1u;
                word |= b << (i * rpad + c);
            }
        }
        up->state[w] = word;
    }
}

}  // namespace

size_t vb_resident_bytes(int32_t n, int32_t m2)
{
    return ((size_t)(n + 1 + m2) * 4 + 15) & ~(size_t)15;
}

size_t vb_lds_bytes(int32_t n, int32_t rpad, int threads)
{
    const size_t sw = ((size_t)n * (size_t)rpad + 31) / 32;
    return ((sw + 3) & ~(size_t)3) * 4 + 2 * kVbMaxChains * kVbXMax * 4 + kVbMaxChains * 8 +
           (size_t)threads * 16;
}

hipError_t vb_init(const VbUnit* units, int n_units, int threads, size_t, hipStream_t s)
{
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(vb_init_kernel, dim3(n_units), dim3(threads), 0, s, units);
    return hipGetLastError();
}

hipError_t vb_prepare()
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)vb_sweep_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    return hipSuccess;
}

hipError_t vb_sweep(const VbUnit* units, int n_units, int threads, size_t lds_bytes, const int64_t* t0p,
                    int32_t n_sweeps, int64_t t_max, hipStream_t s)
{
    if (n_units <= 0 || n_sweeps <= 0) return hipSuccess;
    hipLaunchKernelGGL(vb_sweep_kernel, dim3(n_units), dim3(threads), lds_bytes, s, units, t0p,
                       n_sweeps, t_max);
    return hipGetLastError();
}

hipError_t vb_advance(int64_t* t, int32_t n_sweeps, hipStream_t s)
{
    hipLaunchKernelGGL(vb_advance_kernel, dim3(1), dim3(64), 0, s, t, n_sweeps);
    return hipGetLastError();
}

}  // namespace sg
