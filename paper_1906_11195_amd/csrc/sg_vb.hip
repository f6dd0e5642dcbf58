// Viana-Bray Metropolis sweeps on gfx950.
//
// One workgroup owns one work unit: a graph stored in sweep order (the
// colour classes of a proper colouring, the paper's bipartite parallel update
// generalised; SI "Simulations of the Bethe Lattice on GPUs") and up to eight
// chains that share it.  The chains' spins stay in LDS for the whole launch,
// packed vertex-major (rpad bits per position, bit c = chain c), so that one
// LDS read of a neighbour returns its spin in every chain.  The adjacency
// (row starts + packed entries) is streamed from HBM once per sweep for all
// chains of the unit.
//
// A sweep visits colour class 0, 1, ...; inside a class every position is
// independent (no two positions of a class are adjacent), so the class is
// split over the lanes: one lane takes an aligned group of 8 positions, which
// shares one Philox block per chain for the acceptance draws.  A workgroup
// barrier separates classes.  Flips are XORed into LDS.
//
// Metropolis rule (Methods; SI bipartite-graph section): with x = s_p h_p the
// move is accepted if x <= 0, else iff r < thr[x], thr[x] = floor(2^32
// exp(-2x/T)).  r = (A << 16) | B with A, B half-words of two Philox streams;
// B is evaluated only when A ties with the threshold's high half.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

template <int RPAD>
__device__ __forceinline__ void vb_group(const VbUnit* __restrict__ up, uint32_t* __restrict__ sp,
                                         const uint32_t* __restrict__ thi,
                                         const uint32_t* __restrict__ tlo, int32_t g, int32_t lo,
                                         int32_t hi, uint32_t t, int32_t nch, uint32_t* acc)
{
    const int32_t* __restrict__ row = up->row;
    const uint32_t* __restrict__ ent = up->ent;
    const int32_t pb = g << 3;

    U4 A[RPAD];
#pragma unroll
    for (int c = 0; c < RPAD; ++c) {
        if (c < nch)
            A[c] = philox_stream(up->seed[c], (uint32_t)g, t, kDomSweepHi, up->rep[c], up->inst[c]);
        else
            A[c] = U4{0, 0, 0, 0};
    }

    uint64_t fl = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int32_t p = pb + j;
        if (p < lo || p >= hi) continue;
        const int32_t e0 = row[p];
        const int32_t e1 = row[p + 1];
        const uint32_t ob = (uint32_t)p * RPAD;
        const uint32_t own = sp[ob >> 5] >> (ob & 31u);
        uint32_t cnt[RPAD];
#pragma unroll
        for (int c = 0; c < RPAD; ++c) cnt[c] = 0;
        for (int32_t e = e0; e < e1; ++e) {
            const uint32_t en = ent[e];
            const uint32_t qb = (en & 0x7fffffffu) * RPAD;
            // bit c of f is 1 iff the bond (p, q) is unsatisfied in chain c
            const uint32_t f = (sp[qb >> 5] >> (qb & 31u)) ^ own ^ (uint32_t)((int32_t)en >> 31);
#pragma unroll
            for (int c = 0; c < RPAD; ++c) cnt[c] += (f >> c) & 1u;
        }
        const int32_t deg = e1 - e0;
#pragma unroll
        for (int c = 0; c < RPAD; ++c) {
            if (c >= nch) break;
            const int32_t x = deg - 2 * (int32_t)cnt[c];   // x = s_p h_p
            bool flip = x <= 0;
            if (!flip) {
                const uint32_t th = thi[c * kVbXMax + x];
                const uint32_t rh = half_word(A[c], (uint32_t)j);
                flip = rh < th;
                if (rh == th) {
                    const U4 B = philox_stream(up->seed[c], (uint32_t)g, t, kDomSweepLo, up->rep[c],
                                               up->inst[c]);
                    flip = half_word(B, (uint32_t)j) < tlo[c * kVbXMax + x];
                }
            }
            if (flip) {
                fl |= 1ull << (j * RPAD + c);
                acc[c] += 1;
            }
        }
    }
    if (fl) {
        const uint32_t gb = (uint32_t)pb * RPAD;
        if (RPAD == 8) {
            if ((uint32_t)fl) atomicXor(&sp[gb >> 5], (uint32_t)fl);
            if ((uint32_t)(fl >> 32)) atomicXor(&sp[(gb >> 5) + 1], (uint32_t)(fl >> 32));
        } else {
            atomicXor(&sp[gb >> 5], (uint32_t)fl << (gb & 31u));
        }
    }
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
        up->snap[c][(int64_t)k * wn + w] = bits;
    }
}

template <int RPAD>
__device__ void vb_run(const VbUnit* __restrict__ up, uint32_t* smem, int64_t t0, int32_t nsw,
                       int64_t t_max)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int32_t sw = up->state_words;
    uint32_t* sp = smem;
    uint32_t* thi = smem + ((sw + 3) & ~3);
    uint32_t* tlo = thi + kVbMaxChains * kVbXMax;
    unsigned long long* accs = (unsigned long long*)(tlo + kVbMaxChains * kVbXMax);

    for (int32_t w = tid; w < sw; w += nthr) sp[w] = up->state[w];
    for (int i = tid; i < kVbMaxChains * kVbXMax; i += nthr) {
        thi[i] = (&up->thr_hi[0][0])[i];
        tlo[i] = (&up->thr_lo[0][0])[i];
    }
    if (tid < kVbMaxChains) accs[tid] = 0;
    __syncthreads();

    const int32_t ncls = up->ncls, nch = up->nch;
    const int32_t* __restrict__ cls = up->cls;
    uint32_t acc[RPAD];
#pragma unroll
    for (int c = 0; c < RPAD; ++c) acc[c] = 0;

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        for (int32_t c = 0; c < ncls; ++c) {
            const int32_t lo = cls[c], hi = cls[c + 1];
            const int32_t g1 = (hi + 7) >> 3;
            for (int32_t g = (lo >> 3) + tid; g < g1; g += nthr)
                vb_group<RPAD>(up, sp, thi, tlo, g, lo, hi, t, nch, acc);
            __syncthreads();
        }
        const int64_t tn = t0 + s + 1;
        if (tn <= t_max && (tn & (tn - 1)) == 0) {
            vb_snapshot<RPAD>(up, sp, 1 + (63 - __clzll((unsigned long long)tn)));
            __syncthreads();
        }
    }

    for (int32_t w = tid; w < sw; w += nthr) up->state[w] = sp[w];
#pragma unroll
    for (int c = 0; c < RPAD; ++c)
        if (c < nch && acc[c]) atomicAdd(&accs[c], (unsigned long long)acc[c]);
    __syncthreads();
    if (tid < nch) atomicAdd(up->accepted[tid], accs[tid]);
}

__global__ void __launch_bounds__(1024) vb_sweep_kernel(const VbUnit* __restrict__ units,
                                                        int64_t t0, int32_t nsw, int64_t t_max)
{
    extern __shared__ uint32_t smem[];
    const VbUnit* up = units + blockIdx.x;
    switch (up->rpad) {
        case 1: vb_run<1>(up, smem, t0, nsw, t_max); break;
        case 2: vb_run<2>(up, smem, t0, nsw, t_max); break;
        case 4: vb_run<4>(up, smem, t0, nsw, t_max); break;
        default: vb_run<8>(up, smem, t0, nsw, t_max); break;
    }
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

size_t vb_lds_bytes(int32_t n, int32_t rpad)
{
    const size_t sw = ((size_t)n * (size_t)rpad + 31) / 32;
    return ((sw + 3) & ~(size_t)3) * 4 + 2 * kVbMaxChains * kVbXMax * 4 + kVbMaxChains * 8;
}

hipError_t vb_init(const VbUnit* units, int n_units, int threads, size_t, hipStream_t s)
{
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(vb_init_kernel, dim3(n_units), dim3(threads), 0, s, units);
    return hipGetLastError();
}

hipError_t vb_sweep(const VbUnit* units, int n_units, int threads, size_t lds_bytes, int64_t t0,
                    int32_t n_sweeps, int64_t t_max, hipStream_t s)
{
    if (n_units <= 0 || n_sweeps <= 0) return hipSuccess;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)vb_sweep_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(vb_sweep_kernel, dim3(n_units), dim3(threads), lds_bytes, s, units, t0,
                       n_sweeps, t_max);
    return hipGetLastError();
}

}  // namespace sg
