// Viana-Bray sweeps in the paper's multispin coding (Methods; SI section on
// the bipartite random regular graph): up to 64 chains that share one graph,
// each with its own couplings, temperature and random numbers, are the 64
// bits of one word per vertex.  The chains are those of the per-chain layout
// (sg_vb.hip), with the same colour-class sweep and the same random streams,
// so every trajectory is identical; only the data layout differs.
//
// One workgroup owns one unit and keeps its n spin words in LDS for the whole
// launch.  A colour class is cut into aligned chunks of 64 positions;
// wavefront w takes chunks w, w + W, ..., lane i position 64 b + i.  For
// every neighbour the lane XORs the neighbour's word, its own word and the
// edge's coupling word: bit c is set where chain c's bond is unsatisfied, and
// a bit-sliced counter (4 bit planes, 6 when a degree in the chunk exceeds
// 15) counts them for all 64 chains at once.  The decisions are then taken
// chain by chain: the bit planes of 8 chains' counts are spread to bytes and
// combined into the byte offsets of the chains' entries x = deg - 2 count in
// their threshold tables (high 16 bits, 65536 for x <= 0), and the high
// half-word A of the chain's uniform is compared with it by the sign of the
// difference; a tie (probability 2^-16) is settled on the low halves as in
// the per-chain layout.  The adjacency is prefetched along the wavefront's
// chunk sequence (rows two chunks ahead, the first entries one ahead).  The Philox blocks of 8 chains are drawn per pass,
// one per lane, and exchanged through LDS.  Each lane owns its position's
// word, so the flips are written back with a plain XOR.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

constexpr int kMaxClsM = 64;   // colour classes (degree <= 63)
constexpr int kThrSpan = 32;   // LDS threshold entries per chain: x = 15 .. -16 (index 15 - x)

__device__ __forceinline__ void wave_sync_m()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct VbmLds {
    uint64_t* sp;                 // [n] spin words
    uint32_t* thr;                // [64][kThrSpan]: chain c, 15 - x -> thr[x] >> 16; 65536 for x <= 0
    uint32_t* ri;                 // [64][2]: replica, instance
    int32_t* cls;                 // [kMaxClsM + 4]
    unsigned long long* acc;      // [64] accepted flips of the launch
    uint4* xch;                   // [waves][64] Philox blocks of 8 chains
    unsigned long long* spr8;     // [256]: bit j of the index -> byte j
};

__device__ __forceinline__ VbmLds vbm_carve(uint8_t* base, int32_t n, int waves)
{
    VbmLds L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t* p = base + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    L.sp = (uint64_t*)take((size_t)n * 8);
    L.thr = (uint32_t*)take((size_t)kVbmChains * kThrSpan * 4);
    L.ri = (uint32_t*)take((size_t)kVbmChains * 8);
    L.cls = (int32_t*)take((size_t)(kMaxClsM + 4) * 4);
    L.acc = (unsigned long long*)take((size_t)kVbmChains * 8);
    L.xch = (uint4*)take((size_t)waves * 64 * 16);
    L.spr8 = (unsigned long long*)take(256 * 8);
    return L;
}

// Count of chain c from np bit planes.
__device__ __forceinline__ int32_t count_of(const uint64_t* pl, int np, int c)
{
    int32_t u = 0;
    for (int k = 0; k < np; ++k) u |= (int32_t)((pl[k] >> c) & 1ull) << k;
    return u;
}

__global__ void __launch_bounds__(1024) vbm_sweep_kernel(const VbmUnit* __restrict__ units,
                                                         const int64_t* __restrict__ t0p, int32_t nsw,
                                                         int64_t t_max)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t vbm_smem[];
    const VbmUnit* up = (const VbmUnit*)(gl(units) + blockIdx.x);
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    const int W = nthr >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int32_t n = up->n, nch = up->nch, ncls = up->ncls, wn = up->words_n;
    const VbmLds L = vbm_carve(vbm_smem, n, W);
    const SG_G uint64_t* gstate = gl(up->state);
    for (int32_t i = tid; i < n; i += nthr) L.sp[i] = gstate[i];
    const SG_G uint32_t* gthr = gl(up->thr);
    for (int i = tid; i < kVbmChains * kThrSpan; i += nthr) {
        const int c = i / kThrSpan, x = 15 - (i - c * kThrSpan);
        L.thr[i] = x <= 0 ? 0x10000u : (c < nch ? gthr[c * kVbXMax + x] : 0u);
    }
    for (int i = tid; i < 256; i += nthr) {
        unsigned long long v = 0ull;
        for (int j = 0; j < 8; ++j) v |= (unsigned long long)((i >> j) & 1) << (8 * j);
        L.spr8[i] = v;
    }
    if (tid < kVbmChains) {
        L.ri[2 * tid] = up->rep[tid];
        L.ri[2 * tid + 1] = up->inst[tid];
        L.acc[tid] = 0ull;
    }
    for (int32_t k = tid; k <= ncls; k += nthr) L.cls[k] = gl(up->cls)[k];
    __syncthreads();
    const int64_t t0 = *gl(t0p);
    const uint64_t key = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(up->key >> 32)) << 32) |
                         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)up->key);
    const SG_G int32_t* __restrict__ row = gl(up->row);
    const SG_G uint32_t* __restrict__ ent = gl(up->ent);
    const SG_G uint64_t* __restrict__ jw = gl(up->jw);

    // Adjacency prefetch over the wavefront's chunk sequence (class by class,
    // sweep after sweep): the rows of the chunk after next and the first four
    // entries and coupling words of the next chunk are loaded while a chunk is
    // updated (the adjacency does not depend on the spins, so the loads run
    // across class barriers; every entry read stays inside the padded arrays).
    struct Cur {
        int32_t s, k, j;
    };
    struct Stg {
        int32_t qb, lo, hi;
        int32_t r0, d;
        uint32_t e[4];
        uint64_t jv[4];
    };
    auto cnk = [&](int32_t k) {
        const int32_t lo = __builtin_amdgcn_readfirstlane(L.cls[k]);
        const int32_t hi = __builtin_amdgcn_readfirstlane(L.cls[k + 1]);
        return hi > lo ? ((hi - 1) >> 6) - (lo >> 6) + 1 : 0;
    };
    // the next chunk of this wavefront after c; false past the launch
    auto advance = [&](Cur& c) -> bool {
        c.j += W;
        for (;;) {
            if (c.j < cnk(c.k)) return true;
            c.j = wave;
            if (++c.k == ncls) {
                c.k = 0;
                if (++c.s == nsw) return false;
            }
        }
    };
    auto rows = [&](const Cur& c, Stg& g) {
        g.lo = __builtin_amdgcn_readfirstlane(L.cls[c.k]);
        g.hi = __builtin_amdgcn_readfirstlane(L.cls[c.k + 1]);
        g.qb = ((g.lo >> 6) + c.j) << 6;
        const int32_t q = g.qb + lane;
        const bool act = q >= g.lo && q < g.hi;
        g.r0 = act ? row[q] : 0;
        g.d = act ? row[q + 1] - g.r0 : 0;
    };
    auto ents = [&](Stg& g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            g.e[i] = ent[g.r0 + i];
            g.jv[i] = jw[g.r0 + i];
        }
    };
    Stg S0, S1, SR;
    S1.qb = S1.lo = S1.hi = S1.r0 = S1.d = 0;
    SR.qb = SR.lo = SR.hi = SR.r0 = SR.d = 0;
    Cur cR = {0, 0, wave - W};
    bool haveR = nsw > 0 && advance(cR);
    if (haveR) {
        rows(cR, S0);
        ents(S0);
        haveR = advance(cR);
        if (haveR) rows(cR, SR);
    }

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        // accepted flips of this sweep, per chain, in 8 bit planes (a lane
        // takes at most 255 chunks per sweep: threads >= 128, n <= 16384)
        uint64_t ap[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) ap[k] = 0ull;
        for (int32_t k = 0; k < ncls; ++k) {
            const int32_t nck = cnk(k);
            for (int32_t j = wave; j < nck; j += W) {
                // the next chunk's entries, the rows of the one after it
                S1.qb = SR.qb;
                S1.lo = SR.lo;
                S1.hi = SR.hi;
                S1.r0 = SR.r0;
                S1.d = SR.d;
                ents(S1);
                if (haveR) {
                    haveR = advance(cR);
                    if (haveR) rows(cR, SR);
                }
                const int32_t qb = S0.qb;
                const int32_t q = qb + lane;
                const bool act = q >= S0.lo && q < S0.hi;
                const int32_t r0 = S0.r0;
                const int32_t d = S0.d;
                const uint64_t own = act ? L.sp[q] : 0ull;
                const bool wide = __any(d > 15);
                // Decisions, 8 chains per Philox pass.  Below degree 16 the
                // counts' bit planes are spread to bytes (spr8) and turned into
                // byte offsets 4 (15 - d) + 8 count = 4 (15 - x) of the chains'
                // entries in their tables, one bit-field extract per chain; the
                // sign of e = A - thr decides (shifted into fv, chain 8 i + j at
                // bit j) and a zero e (a tie) shows in the running minimum.
                uint64_t A = 0ull, tie = 0ull;
                typedef const __attribute__((address_space(3))) uint32_t lds_u32;
                typedef const __attribute__((address_space(3))) uint16_t lds_u16;
                const uint32_t thr_off = (uint32_t)(size_t)(const __attribute__((address_space(3))) uint32_t*)L.thr;
                const uint32_t rh_off = (uint32_t)(size_t)(const __attribute__((address_space(3))) uint4*)(L.xch + wave * 64) +
                                        (uint32_t)(lane >> 3) * 16u + (uint32_t)(lane & 7) * 2u;
                // pass i's Philox blocks: lane l draws chain 8 i + l / 8 for the
                // 8 positions of group l mod 8
                auto draw = [&](int i) {
                    const int cc = 8 * i + (lane >> 3);
                    const int ce = cc < nch ? cc : 0;
                    const U4 B = philox_stream(key, ((uint32_t)qb >> 3) + (uint32_t)(lane & 7), t, kDomSweepHi,
                                               L.ri[2 * ce], L.ri[2 * ce + 1]);
                    L.xch[wave * 64 + lane] = make_uint4(B.x, B.y, B.z, B.w);
                    wave_sync_m();
                };
                // ties: A equals the high half of the threshold; decided on
                // the low halves (second stream), rare
                auto resolve = [&](const uint64_t* planes, int np) {
                    if (!act) {
                        A = 0ull;
                        tie = 0ull;
                    }
                    if (__any(tie != 0ull)) {
                        uint64_t tm = tie;
                        while (tm) {
                            const int c = __builtin_ctzll(tm);
                            tm &= tm - 1ull;
                            const int32_t x = d - 2 * count_of(planes, np, c);
                            const U4 Bl = philox_stream(key, (uint32_t)q >> 3, t, kDomSweepLo, L.ri[2 * c], L.ri[2 * c + 1]);
                            if (half_word(Bl, (uint32_t)q & 7u) < gthr[kVbmChains * kVbXMax + c * kVbXMax + x]) A |= 1ull << c;
                        }
                    }
                };
                if (!wide) {
                    // counts below 16: four planes.  The first four neighbours are
                    // added one by one into only the planes their running count can
                    // reach, further ones four entries at a time
                    uint64_t pl[4];
                    {
                        uint64_t nb[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) nb[i] = L.sp[S0.e[i] & 0x7fffffffu];
                        const uint64_t u0 = d > 0 ? nb[0] ^ own ^ S0.jv[0] : 0ull;
                        const uint64_t u1 = d > 1 ? nb[1] ^ own ^ S0.jv[1] : 0ull;
                        pl[0] = u0 ^ u1;
                        pl[1] = u0 & u1;
                        const uint64_t u2 = d > 2 ? nb[2] ^ own ^ S0.jv[2] : 0ull;
                        uint64_t c0 = pl[0] & u2;
                        pl[0] ^= u2;
                        pl[2] = pl[1] & c0;
                        pl[1] ^= c0;
                        const uint64_t u3 = d > 3 ? nb[3] ^ own ^ S0.jv[3] : 0ull;
                        c0 = pl[0] & u3;
                        pl[0] ^= u3;
                        pl[2] |= pl[1] & c0;
                        pl[1] ^= c0;
                        pl[3] = 0ull;
                    }
                    for (int32_t e0 = 4; __any(e0 < d); e0 += 4) {
                        uint32_t en[4];
                        uint64_t jv[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            // (a lane past its degree reads entry 0)
                            const int32_t ix = e0 + i < d ? r0 + e0 + i : 0;
                            en[i] = ent[ix] & 0x7fffffffu;
                            jv[i] = jw[ix];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            uint64_t cy = e0 + i < d ? L.sp[en[i]] ^ own ^ jv[i] : 0ull;
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const uint64_t nc = pl[b] & cy;
                                pl[b] ^= cy;
                                cy = nc;
                            }
                        }
                    }
                    const uint32_t bias = __builtin_amdgcn_perm(0u, (uint32_t)(60 - 4 * d), 0u);
                    // (passes unrolled: constant shifts; the chains of a pass are
                    // decided without branches, those past nch masked off)
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        if (8 * i >= nch) break;
                        draw(i);
                        const uint32_t live = nch - 8 * i >= 8 ? 0xffu : (1u << (nch - 8 * i)) - 1u;
                        // (the four spread words are read before any is used,
                        // so that their LDS round trips overlap)
                        unsigned long long sp[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            sp[k] = L.spr8[__builtin_amdgcn_ubfe((uint32_t)(pl[k] >> (32 * (i >> 2))),
                                                                 8u * (uint32_t)(i & 3), 8u)];
                        uint32_t olo = bias, ohi = bias;   // chains 8 i .. 8 i + 3, 8 i + 4 .. 8 i + 7
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            olo += (uint32_t)sp[k] << (3 + k);
                            ohi += (uint32_t)(sp[k] >> 32) << (3 + k);
                        }
                        // chain c's table at the constant offset c kThrSpan 4 (a chain
                        // past the unit's count reads zeros, masked off below)
                        uint32_t th[8], rh[8];
#pragma unroll
                        for (int c8 = 0; c8 < 8; ++c8) {
                            const uint32_t off = __builtin_amdgcn_ubfe(c8 < 4 ? olo : ohi, 8u * (uint32_t)(c8 & 3), 8u);
                            th[c8] = *(lds_u32*)(size_t)(thr_off + (uint32_t)((8 * i + c8) * kThrSpan * 4) + off);
                            rh[c8] = *(lds_u16*)(size_t)(rh_off + (uint32_t)(c8 * 128));
                        }
                        uint32_t fv = 0u, emin = 0xFFFFFFFFu;
#pragma unroll
                        for (int c8 = 7; c8 >= 0; --c8) {
                            const uint32_t e = rh[c8] - th[c8];
                            fv = __builtin_amdgcn_alignbit(fv, e, 31u);
                            emin = min(emin, e);
                        }
                        A |= (uint64_t)(fv & live) << (8 * i);
                        if (__builtin_amdgcn_ballot_w64(act && emin == 0u) != 0ull) {
                            // a half-word equals a threshold (rare): mark those chains
                            uint32_t tm = 0u;
#pragma unroll
                            for (int c8 = 0; c8 < 8; ++c8) tm |= (uint32_t)(rh[c8] == th[c8]) << c8;
                            tie |= (uint64_t)(tm & live) << (8 * i);
                        }
                        wave_sync_m();
                    }
                    resolve(pl, 4);
                } else {
                    // a degree above 15 in the chunk: six planes, thresholds from HBM
                    uint64_t pl[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
                    for (int32_t e0 = 0; __any(e0 < d); e0 += 4) {
                        uint32_t en[4];
                        uint64_t jv[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int32_t ix = e0 + i < d ? r0 + e0 + i : 0;
                            en[i] = ent[ix] & 0x7fffffffu;
                            jv[i] = jw[ix];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            uint64_t cy = e0 + i < d ? L.sp[en[i]] ^ own ^ jv[i] : 0ull;
#pragma unroll
                            for (int b = 0; b < 6; ++b) {
                                const uint64_t nc = pl[b] & cy;
                                pl[b] ^= cy;
                                cy = nc;
                            }
                        }
                    }
                    for (int i = 0; i < 8; ++i) {
                        if (8 * i >= nch) break;
                        draw(i);
                        for (int c8 = 0; c8 < 8; ++c8) {
                            const int c = 8 * i + c8;
                            if (c >= nch) break;
                            const uint32_t rh1 = *(lds_u16*)(size_t)(rh_off + (uint32_t)(c8 * 128));
                            const int32_t x = d - 2 * count_of(pl, 6, c);
                            const uint32_t th1 = x <= 0 ? 0x10000u : gthr[c * kVbXMax + x];
                            A |= (uint64_t)(rh1 < th1) << c;
                            tie |= (uint64_t)(rh1 == th1) << c;
                        }
                        wave_sync_m();
                    }
                    resolve(pl, 6);
                }
                if (act) L.sp[q] = own ^ A;
                // count the accepted flips in the bit-sliced counter
                uint64_t cy = A;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const uint64_t nc = ap[b] & cy;
                    ap[b] ^= cy;
                    cy = nc;
                }
                S0 = S1;
            }
            __syncthreads();
        }
        // flush the sweep's accepted counts: per chain, the wavefront's sum
#pragma unroll 1
        for (int c = 0; c < nch; ++c) {
            unsigned long long tot = 0ull;
#pragma unroll
            for (int b = 0; b < 8; ++b)
                tot += (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(((ap[b] >> c) & 1ull) != 0ull)) << b;
            if (lane == 0 && tot) atomicAdd(&L.acc[c], tot);
        }
        const int64_t tn = t0 + s + 1;
        if (tn <= t_max && (tn & (tn - 1)) == 0) {
            const int kk = 1 + (63 - __clzll((unsigned long long)tn));
            for (int32_t idx = tid; idx < nch * wn; idx += nthr) {
                const int32_t c = idx / wn, w = idx - c * wn;
                uint32_t bits = 0u;
                for (int b = 0; b < 32; ++b) {
                    const int32_t p = 32 * w + b;
                    if (p < n) bits |= (uint32_t)((L.sp[p] >> c) & 1ull) << b;
                }
                gl(up->snap[c])[(int64_t)kk * wn + w] = bits;
            }
            __syncthreads();
        }
    }
    for (int32_t i = tid; i < n; i += nthr) gl(up->state)[i] = L.sp[i];
    __syncthreads();
    if (tid < nch && L.acc[tid]) atomicAdd(up->accepted[tid], L.acc[tid]);
}

// Initial configurations (the per-chain definition: chain c's start bits in
// position order) and the t = 0 snapshots.
__global__ void __launch_bounds__(256) vbm_init_kernel(const VbmUnit* __restrict__ units)
{
    const VbmUnit* up = units + blockIdx.x;
    const int32_t n = up->n, wn = up->words_n, nch = up->nch;
    for (int32_t idx = threadIdx.x; idx < nch * wn; idx += blockDim.x) {
        const int32_t c = idx / wn, w = idx - c * wn;
        uint32_t bits;
        if (up->init_mode[c] == 0) {
            const U4 o = philox_stream(up->seed, (uint32_t)(w >> 2), 0u, kDomInit, up->rep[c], up->inst[c]);
            bits = word_of(o, (uint32_t)(w & 3));
        } else if (up->init_mode[c] == 1) {
            bits = 0u;
        } else {
            bits = up->given[c][w];
        }
        const int32_t pe = n - 32 * w;
        if (pe < 32) bits &= (1u << pe) - 1u;
        up->snap[c][w] = bits;
    }
    __syncthreads();
    for (int32_t p = threadIdx.x; p < n; p += blockDim.x) {
        uint64_t word = 0ull;
        for (int32_t c = 0; c < nch; ++c) word |= (uint64_t)((up->snap[c][p >> 5] >> (p & 31)) & 1u) << c;
        up->state[p] = word;
    }
}

// Bond sums of every chain's snapshot k.  The chains' position-order
// snapshot words are transposed into one 64-bit word per position by wave
// ballots (lane c holds chain c's word of 32 positions), then every directed
// adjacency entry gives the unsatisfied bonds of all chains as one XOR,
// counted in a bit-sliced counter per thread.  Each edge is two directed
// entries, so per chain B = (entries - 2 unsatisfied entries) / 2.
// grid = (units, k_done - k_first), 256 threads, n 64-bit words of dynamic LDS.
__global__ void __launch_bounds__(256) vbm_bond_kernel(const VbmUnit* __restrict__ units,
                                                       const int32_t* __restrict__ chain_ids, int k_first,
                                                       int k_cap, long long* __restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) uint64_t bw[];
    __shared__ unsigned long long uns[kVbmChains];
    __shared__ unsigned long long ents;
    const VbmUnit* up = units + blockIdx.x;
    const int k = k_first + (int)blockIdx.y;
    const int32_t n = up->n, wn = up->words_n, nch = up->nch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, W = blockDim.x >> 6;
    if (tid < kVbmChains) uns[tid] = 0ull;
    if (tid == 0) ents = 0ull;
    for (int32_t w = wave; w < wn; w += W) {
        const uint32_t word = lane < nch ? up->snap[lane][(int64_t)k * wn + w] : 0u;
        for (int b = 0; b < 32; ++b) {
            const unsigned long long m = __builtin_amdgcn_ballot_w64(((word >> b) & 1u) != 0u);
            if (lane == b && 32 * w + b < n) bw[32 * w + b] = m;
        }
    }
    __syncthreads();
    uint64_t pl[12];
#pragma unroll
    for (int b = 0; b < 12; ++b) pl[b] = 0ull;
    uint32_t e_cnt = 0;
    for (int32_t p = tid; p < n; p += blockDim.x) {
        const uint64_t wp = bw[p];
        const int32_t e1 = up->row[p + 1];
        for (int32_t e = up->row[p]; e < e1; ++e) {
            const int32_t q = (int32_t)(up->ent[e] & 0x7fffffffu);
            uint64_t cy = wp ^ bw[q] ^ up->jw[e];
#pragma unroll
            for (int b = 0; b < 12; ++b) {
                const uint64_t nc = pl[b] & cy;
                pl[b] ^= cy;
                cy = nc;
            }
            ++e_cnt;
        }
    }
    // per chain: the workgroup's unsatisfied directed entries
    for (int c = 0; c < nch; ++c) {
        unsigned long long tot = 0ull;
#pragma unroll
        for (int b = 0; b < 12; ++b)
            tot += (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(((pl[b] >> c) & 1ull) != 0ull)) << b;
        if (lane == 0 && tot) atomicAdd(&uns[c], tot);
    }
    unsigned long long et = e_cnt;
    for (int o = 32; o >= 1; o >>= 1) et += __shfl_xor(et, o);
    if (lane == 0 && et) atomicAdd(&ents, et);
    __syncthreads();
    if (tid < nch)
        out[(int64_t)chain_ids[blockIdx.x * kVbmChains + tid] * k_cap + k] =
            ((long long)ents - 2ll * (long long)uns[tid]) / 2;
}

}  // namespace

size_t vbm_lds_bytes(int32_t n, int threads)
{
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return r16((size_t)n * 8) + r16((size_t)kVbmChains * kThrSpan * 4) + r16((size_t)kVbmChains * 8) +
           r16((size_t)(kMaxClsM + 4) * 4) + r16((size_t)kVbmChains * 8) + (size_t)(threads / 64) * 64 * 16 +
           256 * 8;
}

hipError_t vbm_init(const VbmUnit* units, int n_units, hipStream_t s)
{
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(vbm_init_kernel, dim3(n_units), dim3(256), 0, s, units);
    return hipGetLastError();
}

hipError_t vbm_prepare()
{
    static const hipError_t a1 = hipFuncSetAttribute((const void*)vbm_sweep_kernel,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (a1 != hipSuccess) return a1;
    // the bond kernel also has static LDS: ask for the dynamic part it uses
    static const hipError_t a2 = hipFuncSetAttribute((const void*)vbm_bond_kernel,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kVbmMaxN * 8);
    return a2;
}

hipError_t vbm_sweep(const VbmUnit* units, int n_units, int threads, size_t lds_bytes, const int64_t* t0p,
                     int32_t n_sweeps, int64_t t_max, hipStream_t s)
{
    if (n_units <= 0 || n_sweeps <= 0) return hipSuccess;
    hipLaunchKernelGGL(vbm_sweep_kernel, dim3(n_units), dim3(threads), lds_bytes, s, units, t0p, n_sweeps,
                       t_max);
    return hipGetLastError();
}

hipError_t vbm_bond(const VbmUnit* units, int n_units, int k_first, int k_done, long long* out,
                    const int32_t* chain_ids, int k_cap, hipStream_t s)
{
    if (n_units <= 0 || k_done <= k_first) return hipSuccess;
    // one 64-bit word per position of the largest unit (n <= kVbmMaxN)
    hipLaunchKernelGGL(vbm_bond_kernel, dim3(n_units, k_done - k_first), dim3(256), (size_t)kVbmMaxN * 8, s,
                       units, chain_ids, k_first, k_cap, out);
    return hipGetLastError();
}

}  // namespace sg
