// Observables at the grid times, from the device-resident snapshots.
//
//  * Gram matrices G[k][l] = sum_i s_i(t_k) s_i(t_l) per chain (the two-time
//    correlation C = G / N of the introduction and SI Eq. formula1).  The
//    snapshots of a chain form an N x K matrix S of +-1 with K <= 32, and
//    G = S^T S is an int8 contraction over N: it runs on the matrix cores as
//    v_mfma_i32_32x32x32_i8 with int32 accumulation.  Each lane expands 16
//    packed spins of one snapshot into 16 int8; the same register serves as
//    the A operand (S^T) and the B operand (S).
//  * Two-clone overlaps Q = sum_i s^a_i s^b_i = N - 2 popcount(a xor b).
//  * VB bond sums B = sum_{(uv) in E} J_uv s_u s_v (energy -B, Eq. 3), one
//    pass over the unit's adjacency per snapshot time.
#include "sg_internal.h"

#include <mutex>

// Staging of sg_measure_noalloc (bond sums, overlaps, Gram matrices before
// they are copied to the caller's host arrays): a fixed device array instead
// of memory allocated by the library.  Each device holds its own copy until
// the process ends.  In host code the name stands for a host-side shadow, so
// the kernels get the device address from measure_scratch() instead.
static __device__ __align__(256) long long scratch[sg::kMeasureScratchElems];

namespace sg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t spread4(uint32_t nib)
{
    return (nib * 0x00204081u) & 0x01010101u;
}

// 16 spins (1 = -1) -> 16 int8 +-1, zero where keep bit is 0.
__device__ __forceinline__ v4i pm1_bytes(uint32_t bits, uint32_t keep)
{
    v4i r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t v = (spread4((bits >> (4 * q)) & 0xFu) * 0xFEu) ^ 0x01010101u;
        const uint32_t kb = spread4((keep >> (4 * q)) & 0xFu) * 0xFFu;
        r[q] = (int)(v & kb);
    }
    return r;
}

// grid = (chains, splits); one wavefront per block.
__global__ void __launch_bounds__(64) gram_kernel(const MeasureChain* __restrict__ chains, int k_done,
                                                  int k_cap, int words_per_split,
                                                  long long* __restrict__ out)
{
    const MeasureChain mc = chains[blockIdx.x];
    const int32_t wn = mc.words_n, n = mc.n;
    const int32_t w0 = blockIdx.y * words_per_split;
    const int32_t w1 = min(wn, w0 + words_per_split);
    if (w0 >= w1) return;
    const int lane = threadIdx.x;
    const int snap = lane & 31;      // row/column of G held by this lane
    const int half = lane >> 5;      // which 16 positions of a 32-position word
    const bool live = snap < k_done;
    const uint32_t* __restrict__ src = mc.snap + (int64_t)snap * wn;
    v16i acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0;
    for (int32_t w = w0; w < w1; ++w) {
        const uint32_t word = live ? src[w] : 0u;
        const int32_t first = 32 * w + 16 * half;
        const int32_t valid = live ? max(0, min(16, n - first)) : 0;
        const uint32_t keep = valid >= 16 ? 0xffffu : ((1u << valid) - 1u);
        const v4i a = pm1_bytes((word >> (16 * half)) & 0xffffu, keep);
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, acc, 0, 0, 0);
    }
    long long* G = out + (int64_t)blockIdx.x * k_cap * k_cap;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
        const int col = snap;
        if (row < k_done && col < k_done)
            atomicAdd((unsigned long long*)&G[row * k_cap + col], (unsigned long long)(long long)acc[r]);
    }
}

// grid = (pairs, k_done)
__global__ void __launch_bounds__(256) overlap_kernel(const MeasureChain* __restrict__ chains,
                                                      const int32_t* __restrict__ pairs, int k_cap,
                                                      long long* __restrict__ out)
{
    __shared__ unsigned int red;
    const int k = blockIdx.y;
    const MeasureChain a = chains[pairs[2 * blockIdx.x]];
    const MeasureChain b = chains[pairs[2 * blockIdx.x + 1]];
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    unsigned int cnt = 0;
    const uint32_t* pa = a.snap + (int64_t)k * a.words_n;
    const uint32_t* pb = b.snap + (int64_t)k * b.words_n;
    for (int32_t w = threadIdx.x; w < a.words_n; w += blockDim.x) cnt += __popc(pa[w] ^ pb[w]);
    atomicAdd(&red, cnt);
    __syncthreads();
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * k_cap + k] = (long long)a.n - 2LL * (long long)red;
}

// grid = (units, k_done).  Snapshot bits of the unit's chains are staged in
// LDS chain-major; every directed adjacency entry is visited once, so the sum
// counts each edge twice.
__global__ void __launch_bounds__(1024) vb_bond_kernel(const VbUnit* __restrict__ units,
                                                       const int32_t* __restrict__ chain_ids,
                                                       int k_first, int k_cap, long long* __restrict__ out)
{
    extern __shared__ uint32_t bsm[];
    const VbUnit* up = units + blockIdx.x;
    if (up->member != 0) return;   // a split unit is measured once
    const int k = k_first + (int)blockIdx.y;
    const int32_t n = up->n, wn = up->words_n, nch = up->nch;
    long long* red = (long long*)(bsm + ((nch * wn + 1) & ~1));
    for (int32_t idx = threadIdx.x; idx < nch * wn; idx += blockDim.x) {
        const int32_t c = idx / wn;
        const int32_t w = idx - c * wn;
        bsm[idx] = up->snap[c][(int64_t)k * wn + w];
    }
    if (threadIdx.x < kVbMaxChains) red[threadIdx.x] = 0;
    __syncthreads();
    int32_t sum[kVbMaxChains];
#pragma unroll
    for (int c = 0; c < kVbMaxChains; ++c) sum[c] = 0;
    const int32_t* __restrict__ row = up->row;
    const uint32_t* __restrict__ ent = up->ent;
    for (int32_t p = threadIdx.x; p < n; p += blockDim.x) {
        const int32_t e0 = row[p], e1 = row[p + 1];
        for (int32_t e = e0; e < e1; ++e) {
            const uint32_t en = ent[e];
            const int32_t q = (int32_t)(en & 0x7fffffffu);
            const uint32_t neg = en >> 31;
#pragma unroll
            for (int c = 0; c < kVbMaxChains; ++c) {
                if (c >= nch) break;
                const uint32_t bp = (bsm[c * wn + (p >> 5)] >> (p & 31)) & 1u;
                const uint32_t bq = (bsm[c * wn + (q >> 5)] >> (q & 31)) & 1u;
                sum[c] += 1 - 2 * (int32_t)(bp ^ bq ^ neg);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kVbMaxChains; ++c)
        if (c < nch && sum[c] != 0)
            atomicAdd((unsigned long long*)&red[c], (unsigned long long)(long long)sum[c]);
    __syncthreads();
    if (threadIdx.x < nch)
        out[(int64_t)chain_ids[blockIdx.x * kVbMaxChains + threadIdx.x] * k_cap + k] =
            red[threadIdx.x] / 2;
}

__global__ void zero_kernel(long long* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

hipError_t zero_i64(long long* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t measure_scratch(long long** ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static long long* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        // once per device, with that device current: its copy's address
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<long long*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t measure_gram(const MeasureChain* chains, int n_chains, int k_done, int k_cap,
                        int max_words, long long* out, hipStream_t s)
{
    if (n_chains <= 0 || k_done <= 0) return hipSuccess;
    const int wps = 256;
    const int splits = (max_words + wps - 1) / wps;
    hipLaunchKernelGGL(gram_kernel, dim3(n_chains, splits), dim3(64), 0, s, chains, k_done, k_cap, wps,
                       out);
    return hipGetLastError();
}

hipError_t measure_overlap(const MeasureChain* chains, const int32_t* pairs, int n_pairs, int k_done,
                           int k_cap, long long* out, hipStream_t s)
{
    if (n_pairs <= 0 || k_done <= 0) return hipSuccess;
    hipLaunchKernelGGL(overlap_kernel, dim3(n_pairs, k_done), dim3(256), 0, s, chains, pairs, k_cap,
                       out);
    return hipGetLastError();
}

hipError_t vb_bond(const VbUnit* units, int n_units, int k_first, int k_done, long long* bond_out,
                   const int32_t* unit_chain_ids, int k_cap, int threads, size_t lds_bytes,
                   hipStream_t s)
{
    if (n_units <= 0 || k_done <= k_first) return hipSuccess;
    // set once (thread-safe initialisation of a local static)
    static const hipError_t attr = hipFuncSetAttribute((const void*)vb_bond_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(vb_bond_kernel, dim3(n_units, k_done - k_first), dim3(threads), lds_bytes, s, units,
                       unit_chain_ids, k_first, k_cap, bond_out);
    return hipGetLastError();
}

}  // namespace sg
