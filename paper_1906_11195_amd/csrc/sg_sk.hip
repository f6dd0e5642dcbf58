// Sherrington-Kirkpatrick Metropolis sweeps on gfx950.
//
// The SK sweep visits i = 0..N-1 in a fixed order (SI, SK section), so a chain
// is inherently sequential.  One workgroup runs one chain with its integer
// local fields H_i = sum_j J_ij s_j resident in LDS.  The sweep is cut into
// blocks of 64 consecutive spins, one per wavefront lane:
//   * every lane decides its spin speculatively, as if no earlier spin of the
//     block flipped (the Philox draw of a position does not depend on the
//     attempt, so a decision made with the exact field is final);
//   * a ballot finds the first accepting lane j; lanes before j are final
//     rejections, lane j flips, the fields of lanes after j are patched with
//     row j of the 64 x 64 coupling tile held in LDS, and the scan resumes
//     at j + 1;
//   * after the block every thread applies the rank-f update
//     H_k += 2 s_j J_jk of the f flipped rows to all N fields.
// The result equals the plain sequential sweep exactly (integer fields).
//
// Every `period` sweeps the fields are recomputed exactly as H = J S with
// int8 MFMA (v_mfma_i32_16x16x64_i8, int32 accumulation) and compared with
// the incremental ones; a mismatch raises the context's error flag.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

struct SkLds {
    int32_t* H;
    uint32_t* bits;
    unsigned long long* thr;
    int8_t* tile;
    int32_t* flips;
    int32_t* misc;        // [0] = number of flips in the block
    long long* red;       // reduction slot
};

__device__ __forceinline__ SkLds sk_carve(uint8_t* base, int32_t n, int32_t wn)
{
    SkLds L;
    size_t off = 0;
    L.H = (int32_t*)(base + off);
    off += ((size_t)n * 4 + 15) & ~(size_t)15;
    L.bits = (uint32_t*)(base + off);
    off += ((size_t)(wn + 2) * 4 + 15) & ~(size_t)15;
    L.thr = (unsigned long long*)(base + off);
    off += (size_t)kSkThrLds * 8;
    L.tile = (int8_t*)(base + off);
    off += (size_t)kSkTile * kSkTile;
    L.flips = (int32_t*)(base + off);
    off += kSkTile * 4;
    L.red = (long long*)(base + off);
    off += 16;
    L.misc = (int32_t*)(base + off);
    return L;
}

__global__ void __launch_bounds__(256) sk_sweep_kernel(const SkChain* __restrict__ chains,
                                                       int64_t t0, int32_t nsw, int64_t t_max)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t sk_smem[];
    const SkChain* ch = chains + blockIdx.x;
    const int32_t n = ch->n, wn = ch->words_n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    SkLds L = sk_carve(sk_smem, n, wn);
    const int8_t* __restrict__ J = ch->J;
    const int32_t thr_len = ch->thr_len;
    const int32_t thr_cached = min(thr_len, kSkThrLds);

    for (int32_t i = tid; i < n; i += nthr) L.H[i] = ch->H[i];
    for (int32_t w = tid; w < wn + 2; w += nthr) L.bits[w] = w < wn ? ch->state[w] : 0u;
    for (int32_t x = tid; x < thr_cached; x += nthr) L.thr[x] = ch->thr[x];
    __syncthreads();

    const int32_t nb = (n + kSkTile - 1) / kSkTile;
    const int lane = tid & 63;
    uint32_t acc = 0;

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t base = b * kSkTile;
            for (int32_t idx = tid; idx < kSkTile * kSkTile; idx += nthr) {
                const int32_t r = idx >> 6, c = idx & 63;
                const int32_t pr = base + r, pc = base + c;
                L.tile[idx] = (pr < n && pc < n) ? J[(int64_t)pr * n + pc] : (int8_t)0;
            }
            __syncthreads();
            if (tid < 64) {
                const int32_t p = base + lane;
                const bool act = p < n;
                int32_t Hp = act ? L.H[p] : 0;
                uint32_t sb = act ? (L.bits[p >> 5] >> (p & 31)) & 1u : 0u;
                const U4 A = philox_stream(ch->seed, (uint32_t)(p >> 3), t, kDomSweepHi, ch->rep,
                                           ch->inst);
                const uint32_t rh = half_word(A, (uint32_t)(p & 7));
                uint32_t rl = 0;
                bool have_lo = false;
                int32_t start = 0, nf = 0;
                while (true) {
                    const int32_t x = sb ? -Hp : Hp;
                    const bool cand = act && lane >= start;
                    bool accept = false, tie = false;
                    uint32_t tlo = 0;
                    if (cand) {
                        if (x <= 0) {
                            accept = true;
                        } else {
                            unsigned long long th = 0;
                            if (x < thr_cached) th = L.thr[x];
                            else if (x < thr_len) th = ch->thr[x];
                            const uint32_t thi = (uint32_t)(th >> 16);
                            tlo = (uint32_t)(th & 0xffffu);
                            accept = rh < thi;
                            tie = rh == thi;
                        }
                    }
                    if (__ballot(tie) != 0ull && !have_lo) {
                        const U4 B = philox_stream(ch->seed, (uint32_t)(p >> 3), t, kDomSweepLo,
                                                   ch->rep, ch->inst);
                        rl = half_word(B, (uint32_t)(p & 7));
                        have_lo = true;
                    }
                    if (tie) accept = rl < tlo;
                    const unsigned long long m = __ballot(accept);
                    if (m == 0ull) break;
                    const int j = __ffsll((long long)m) - 1;
                    const uint32_t sbj = (uint32_t)__shfl((int)sb, j) ^ 1u;   // new bit of j
                    if (lane == j) sb = sbj;
                    if (lane == 0) L.flips[nf] = (base + j) | (int32_t)(sbj << 31);
                    ++nf;
                    const int32_t sj = sbj ? -1 : 1;
                    if (lane > j) Hp += 2 * sj * (int32_t)L.tile[j * kSkTile + lane];
                    start = j + 1;
                }
                const unsigned long long mask = __ballot(sb != 0u);
                if (lane == 0) {
                    // base is a multiple of 64: two whole words
                    L.bits[base >> 5] = (uint32_t)mask;
                    if ((base >> 5) + 1 < wn) L.bits[(base >> 5) + 1] = (uint32_t)(mask >> 32);
                    L.misc[0] = nf;
                }
                acc += (lane == 0) ? (uint32_t)nf : 0u;
            }
            __syncthreads();
            const int32_t nf = L.misc[0];
            for (int32_t f = 0; f < nf; ++f) {
                const int32_t fv = L.flips[f];
                const int32_t pf = fv & 0x7fffffff;
                const int32_t two_s = fv < 0 ? -2 : 2;
                const int8_t* __restrict__ row = J + (int64_t)pf * n;
                for (int32_t k = tid; k < n; k += nthr) L.H[k] += two_s * (int32_t)row[k];
            }
            __syncthreads();
        }
        const int64_t tn = t0 + s + 1;
        if (tn <= t_max && (tn & (tn - 1)) == 0) {
            const int k = 1 + (63 - __clzll((unsigned long long)tn));
            for (int32_t w = tid; w < wn; w += nthr) ch->snap[(int64_t)k * wn + w] = L.bits[w];
            if (tid == 0) L.red[0] = 0;
            __syncthreads();
            long long part = 0;
            for (int32_t i = tid; i < n; i += nthr) {
                const int32_t si = ((L.bits[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
                part += (long long)si * L.H[i];
            }
            atomicAdd((unsigned long long*)&L.red[0], (unsigned long long)part);
            __syncthreads();
            if (tid == 0) ch->bond[k] = L.red[0] / 2;
            __syncthreads();
        }
    }

    for (int32_t i = tid; i < n; i += nthr) ch->H[i] = L.H[i];
    for (int32_t w = tid; w < wn; w += nthr) ch->state[w] = L.bits[w];
    if (tid == 0 && acc) atomicAdd(ch->accepted, (unsigned long long)acc);
}

// Initial configuration and the t = 0 snapshot of every chain.
__global__ void sk_init_kernel(const SkChain* __restrict__ chains)
{
    const SkChain* ch = chains + blockIdx.x;
    const int32_t n = ch->n, wn = ch->words_n;
    for (int32_t w = threadIdx.x; w < wn; w += blockDim.x) {
        uint32_t bits;
        if (ch->init_mode == 0) {
            const U4 o = philox_stream(ch->seed, (uint32_t)(w >> 2), 0u, kDomInit, ch->rep, ch->inst);
            bits = word_of(o, (uint32_t)(w & 3));
        } else if (ch->init_mode == 1) {
            bits = 0;
        } else {
            bits = ch->given[w];
        }
        const int32_t pe = n - 32 * w;
        if (pe < 32) bits &= (1u << pe) - 1u;
        ch->state[w] = bits;
        ch->snap[w] = bits;
    }
}

// B(t = 0) = (1/2) sum_i s_i H_i from the freshly computed exact fields.
__global__ void sk_bond0_kernel(const SkChain* __restrict__ chains)
{
    __shared__ long long red;
    const SkChain* ch = chains + blockIdx.x;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    long long part = 0;
    for (int32_t i = threadIdx.x; i < ch->n; i += blockDim.x) {
        const int32_t si = ((ch->state[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
        part += (long long)si * ch->H[i];
    }
    atomicAdd((unsigned long long*)&red, (unsigned long long)part);
    __syncthreads();
    if (threadIdx.x == 0) ch->bond[0] = red / 2;
}

// 16 spins (bits, 1 = -1) -> 16 int8 of +-1, zeroed where keep_mask bit is 0.
__device__ __forceinline__ v4i expand16(uint32_t bits, uint32_t keep_mask)
{
    v4i r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t nib = (bits >> (4 * q)) & 0xFu;
        const uint32_t spread = (nib * 0x00204081u) & 0x01010101u;
        uint32_t v = (spread * 0xFEu) ^ 0x01010101u;
        const uint32_t km = (keep_mask >> (4 * q)) & 0xFu;
        const uint32_t kb = ((km * 0x00204081u) & 0x01010101u) * 0xFFu;
        r[q] = (int)(v & kb);
    }
    return r;
}

// Exact fields H = J S for all chains of one sample, by int8 MFMA.
// Block = 4 wavefronts = 64 rows; grid = (row blocks, samples).
__global__ void __launch_bounds__(256) sk_recompute_kernel(const SkSample* __restrict__ samples,
                                                           const SkChain* __restrict__ chains,
                                                           int check, int* err)
{
    const SkSample* sm = samples + blockIdx.y;
    const int32_t n = sm->n, nch = sm->nch;
    const int32_t i0 = blockIdx.x * 64 + (threadIdx.x >> 6) * 16;
    if (i0 >= n) return;
    const int lane = threadIdx.x & 63;
    const int32_t row = i0 + (lane & 15);
    const int kg = lane >> 4;
    const int jc = lane & 15;               // chain column of operand B
    const SkChain* cj = jc < nch ? &chains[sm->chain0 + jc] : nullptr;
    const int8_t* __restrict__ J = sm->J;
    v4i acc = {0, 0, 0, 0};
    const bool vec_ok = (n & 15) == 0;
    for (int32_t kc = 0; kc < n; kc += 64) {
        const int32_t k0 = kc + 16 * kg;
        v4i a = {0, 0, 0, 0};
        if (row < n) {
            const int8_t* src = J + (int64_t)row * n + k0;
            if (vec_ok && k0 + 16 <= n) {
                const int4 v = *(const int4*)src;
                a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
            } else {
                uint32_t w4[4] = {0, 0, 0, 0};
                for (int b = 0; b < 16; ++b)
                    if (k0 + b < n) w4[b >> 2] |= (uint32_t)(uint8_t)src[b] << (8 * (b & 3));
                a[0] = (int)w4[0]; a[1] = (int)w4[1]; a[2] = (int)w4[2]; a[3] = (int)w4[3];
            }
        }
        v4i bv = {0, 0, 0, 0};
        if (cj != nullptr && k0 < n) {
            const uint32_t bits = (cj->state[k0 >> 5] >> (k0 & 31)) & 0xffffu;
            const int32_t valid = min(16, n - k0);
            const uint32_t keep = valid >= 16 ? 0xffffu : ((1u << valid) - 1u);
            bv = expand16(bits, keep);
        }
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bv, acc, 0, 0, 0);
    }
    if (cj == nullptr) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int32_t i = i0 + 4 * kg + r;
        if (i < n) {
            if (check && cj->H[i] != acc[r]) atomicOr(err, 1);
            cj->H[i] = acc[r];
        }
    }
}

}  // namespace

size_t sk_lds_bytes(int32_t n)
{
    const int32_t wn = (n + 31) / 32;
    return (((size_t)n * 4 + 15) & ~(size_t)15) + (((size_t)(wn + 2) * 4 + 15) & ~(size_t)15) +
           (size_t)kSkThrLds * 8 + (size_t)kSkTile * kSkTile + kSkTile * 4 + 16 + 16;
}

hipError_t sk_init(const SkChain* chains, int n_chains, int threads, hipStream_t s)
{
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(sk_init_kernel, dim3(n_chains), dim3(threads), 0, s, chains);
    return hipGetLastError();
}

hipError_t sk_bond_t0(const SkChain* chains, int n_chains, hipStream_t s)
{
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(sk_bond0_kernel, dim3(n_chains), dim3(256), 0, s, chains);
    return hipGetLastError();
}

hipError_t sk_recompute(const SkSample* samples, int n_samples, const SkChain* chains, int max_n,
                        int check, int* err_flag, hipStream_t s)
{
    if (n_samples <= 0) return hipSuccess;
    dim3 grid((max_n + 63) / 64, n_samples);
    hipLaunchKernelGGL(sk_recompute_kernel, grid, dim3(256), 0, s, samples, chains, check, err_flag);
    return hipGetLastError();
}

hipError_t sk_sweep(const SkChain* chains, int n_chains, int threads, size_t lds_bytes, int64_t t0,
                    int32_t n_sweeps, int64_t t_max, hipStream_t s)
{
    if (n_chains <= 0 || n_sweeps <= 0) return hipSuccess;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)sk_sweep_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(sk_sweep_kernel, dim3(n_chains), dim3(threads), lds_bytes, s, chains, t0,
                       n_sweeps, t_max);
    return hipGetLastError();
}

}  // namespace sg
