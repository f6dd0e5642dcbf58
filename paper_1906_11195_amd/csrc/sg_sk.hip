// Sherrington-Kirkpatrick Metropolis sweeps on gfx950.
//
// The SK sweep visits i = 0..N-1 in a fixed order (SI, SK section), so a chain
// is sequential.  One workgroup runs one chain with its integer local fields
// H_i = sum_j J_ij s_j resident in LDS, split into three roles that form a
// pipeline over blocks of 64 consecutive spins (block g of the launch is block
// b = g mod NB of sweep t0 + g / NB):
//
//  * prep wavefront (ahead of the decider by up to kRing blocks): draws the
//    acceptance uniform r of every position of the block (two Philox streams)
//    and turns it into xmax = max{x : r < thr[x]}, so that a spin with
//    x = s_i H_i flips iff x <= xmax; it also fetches, from the bit-packed
//    couplings, the 64 x 64 tile of the block's own rows and the tile of the
//    previous block's rows restricted to this block's columns.
//  * decider wavefront: lane i owns spin 64 b + i.  It corrects the block's
//    fields for the flips of the previous block (previous-block tile), then
//    decides the block in rounds: a lane whose decision cannot change
//    whichever way the undecided lanes before it go (each moves its field by
//    at most 2) is decided now, the first undecided lane always is, and the
//    flips decided in a round patch the fields of the later lanes from row j
//    of the block tile.  The result is exactly the plain sequential sweep.
//    The block's flips are published to a ring buffer.
//  * updater wavefronts: apply each published block's flips to all other fields
//    (H_k += 2 s_j J_jk, rows read bit-packed, a few fields per lane), lagging one
//    block behind; they skip the flipped block (patched in the decider) and the
//    next block (corrected by the decider from its tile), except for the last
//    block of a launch.
//
// Every `period` sweeps the fields are recomputed exactly as H = J S with int8
// MFMA (v_mfma_i32_16x16x64_i8, int32 accumulation) and compared with the
// incremental ones; a mismatch raises the context's error flag.  Bond sums
// B = (1/2) s^T J s of the snapshots are computed the same way at measurement
// time.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Pipeline depth (compile-time tuning parameters).
#ifndef SG_SK_RING
#define SG_SK_RING 4
#endif
constexpr int kRing = SG_SK_RING;   // blocks in flight between the roles
constexpr int kWin = 1;             // previous blocks the decider corrects for itself
constexpr int kTileWords = 2 + 2 * kWin;   // per lane: own-block row, kWin previous rows
constexpr int kThrCache = 512;      // threshold entries cached in LDS
#ifndef SG_SK_UPD
#define SG_SK_UPD 8
#endif
#ifndef SG_SK_COLS
#define SG_SK_COLS 8
#endif
constexpr int kUpdWaves = SG_SK_UPD;   // updater wavefronts
constexpr int kUpdCols = SG_SK_COLS;   // fields one updater lane owns (4, 8 or 16)
static_assert(kUpdCols == 4 || kUpdCols == 8 || kUpdCols == 16, "updater item width");
constexpr int kSkThreads = 64 * (2 + kUpdWaves);
constexpr int kSpinLimit = 1 << 22; // bounded waits: a stuck pipeline aborts
static_assert(kRing >= kWin + 1, "flip batches must outlive the correction window");

struct SkLds {
    int32_t* H;                 // [n]
    uint32_t* bits;             // [wn + 2]
    unsigned long long* thr;    // [kThrCache]
    int32_t* xm;                // [kRing][64]
    uint32_t* tile;             // [kRing][64][kTileWords]
    int32_t* flips;             // [kRing][64]: local row | (new spin -1) << 31
    int32_t* nflip;             // [kRing]
    int32_t* sync;              // decided, applied, prepared, abort, done[kRing]
    uint4* pr;                  // [64] Philox blocks of the prep's current 4 spin blocks
};

__device__ __forceinline__ SkLds sk_carve(uint8_t* base, int32_t n, int32_t wn)
{
    SkLds L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t* p = base + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    L.H = (int32_t*)take((size_t)n * 4);
    L.bits = (uint32_t*)take((size_t)(wn + 2) * 4);
    L.thr = (unsigned long long*)take((size_t)kThrCache * 8);
    L.xm = (int32_t*)take((size_t)kRing * 64 * 4);
    L.tile = (uint32_t*)take((size_t)kRing * 64 * kTileWords * 4);
    L.flips = (int32_t*)take((size_t)kRing * 64 * 4);
    L.nflip = (int32_t*)take((size_t)kRing * 4);
    L.sync = (int32_t*)take((size_t)(4 + kRing) * 4);
    L.pr = (uint4*)take(64 * 16);
    return L;
}

enum { kDecided = 0, kApplied = 1, kPrepared = 2, kAbort = 3, kDone = 4 };

__device__ __forceinline__ int ld_acq(int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void st_rel(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits (whole wavefront) until *p >= target.  After kSpinLimit polls the
// pipeline is declared stuck: the abort flag releases every other wait and
// the context's error flag reports it.
__device__ __forceinline__ void wait_ge(const SkLds& L, int32_t idx, int32_t target, int* err)
{
    int spins = 0;
    while (ld_acq(&L.sync[idx]) < target) {
        if (ld_acq(&L.sync[kAbort])) return;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
            st_rel(&L.sync[kAbort], 1);
            atomicOr(err, 2);
            return;
        }
    }
}

__device__ __forceinline__ void wave_sync_sk()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_release()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ unsigned long long thr_at(const SkLds& L, const SkChain* ch,
                                                      int32_t cached, int32_t x)
{
    if (x >= ch->thr_len) return 0ull;
    return x < cached ? L.thr[x] : gl(ch->thr)[x];
}

__global__ void __launch_bounds__(kSkThreads) sk_sweep_kernel(const SkChain* __restrict__ chains,
                                                              int64_t t0, int32_t nsw,
                                                              int64_t t_max, int* err)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t sk_smem[];
    const SkChain* ch = (const SkChain*)(gl(chains) + blockIdx.x);
    const int32_t n = ch->n, wn = ch->words_n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const SkLds L = sk_carve(sk_smem, n, wn);
    const int32_t cached = min(ch->thr_len, kThrCache);

    for (int32_t i = tid; i < n; i += nthr) L.H[i] = gl(ch->H)[i];
    for (int32_t w = tid; w < wn + 2; w += nthr) L.bits[w] = w < wn ? gl(ch->state)[w] : 0u;
    for (int32_t x = tid; x < cached; x += nthr) L.thr[x] = gl(ch->thr)[x];
    if (tid < 4 + kRing) L.sync[tid] = 0;
    __syncthreads();

    const int32_t NB = (n + 63) >> 6;
    // correction window: the decider adds the flips of the previous DW blocks
    // itself; the updaters skip those blocks' columns (DW < NB keeps a block
    // from correcting for its own earlier visit)
    const int32_t DW = min(kWin, NB - 1);
    const int64_t total = (int64_t)nsw * NB;
    const SG_G uint32_t* __restrict__ Jb = gl(ch->Jb);

    if (wave == 1) {
        // ---------------- prep ----------------
        // coupling tiles (bit-packed, bit 1 = J -1) of lane i's own row
        // 64 b + i: its columns in block b, then in blocks b - d, d = 1..DW
        // (J is symmetric, so bit j is the coupling of spin j of that block to
        // spin i); the tiles of the next block are loaded while this block's
        // uniforms are drawn
        uint32_t tw[2 * (kWin + 1)];
        auto load_tiles = [&](int32_t bq) {
            const int32_t rr = (bq << 6) + lane;
#pragma unroll
            for (int d = 0; d <= kWin; ++d) {
                const int32_t bb = bq - d < 0 ? bq - d + NB : bq - d;
                const int32_t w0 = 2 * bb, w1 = 2 * bb + 1;
                const bool live = d <= DW && rr < n;
                tw[2 * d] = live ? Jb[(int64_t)rr * wn + w0] : 0u;
                tw[2 * d + 1] = (live && w1 < wn) ? Jb[(int64_t)rr * wn + w1] : 0u;
            }
        };
        if (total > 0) load_tiles(0);
        int32_t b = 0, s = 0, slot = 0;
        for (int64_t g = 0; g < total; ++g) {
            if (g >= kRing) wait_ge(L, kDecided, (int32_t)(g - kRing + 1), err);
            uint32_t* tl = L.tile + ((size_t)slot * 64 + lane) * kTileWords;
#pragma unroll
            for (int d = 0; d < 2 * (kWin + 1); ++d) tl[d] = tw[d];
            if (g + 1 < total) load_tiles(b + 1 == NB ? 0 : b + 1);
            if ((g & 3) == 0) {
                // one pass of the 64 lanes draws both streams' blocks of the
                // next four spin blocks: lane 16 j + 8 h + q holds stream h
                // (high / low half-words) of 8-position group q of block g + j
                const int32_t j = lane >> 4;
                int32_t bq = b + j, sq = s;
                while (bq >= NB) {
                    bq -= NB;
                    ++sq;
                }
                const uint32_t dom = (lane >> 3) & 1 ? kDomSweepLo : kDomSweepHi;
                const U4 A = philox_stream(ch->seed, (uint32_t)(bq * 8 + (lane & 7)), (uint32_t)(t0 + sq), dom,
                                           ch->rep, ch->inst);
                L.pr[lane] = make_uint4(A.x, A.y, A.z, A.w);
                wave_sync_sk();
            }
            const uint32_t* pw = (const uint32_t*)(L.pr + (int)(g & 3) * 16 + (lane >> 3));
            const uint32_t hsel = (uint32_t)lane & 7u;
            const uint32_t r = (__builtin_amdgcn_ubfe(pw[hsel >> 1], 16u * (hsel & 1u), 16u) << 16) |
                               __builtin_amdgcn_ubfe(pw[32 + (hsel >> 1)], 16u * (hsel & 1u), 16u);
            // starting guess from the logarithm, then exact fix-up on the table
            int32_t x0;
            const float slope = ch->xslope;
            if (slope <= 0.0f) {
                x0 = ch->thr_len - 1;
            } else {
                const float lv = 22.18070977791825f - __logf((float)r + 1.0f);
                const float xf = lv / slope;
                x0 = xf >= (float)(ch->thr_len - 1) ? ch->thr_len - 1 : (xf <= 0.0f ? 0 : (int32_t)xf);
            }
            while (x0 > 0 && !((unsigned long long)r < thr_at(L, ch, cached, x0))) --x0;
            while (x0 + 1 < ch->thr_len && (unsigned long long)r < thr_at(L, ch, cached, x0 + 1)) ++x0;
            L.xm[slot * 64 + lane] = x0;
            wave_release();
            if (lane == 0) st_rel(&L.sync[kPrepared], (int32_t)(g + 1));
            if (++slot == kRing) slot = 0;
            if (++b == NB) {
                b = 0;
                ++s;
            }
        }
    } else if (wave == 0) {
        // ---------------- decider ----------------
        // the sequential critical path: issue ahead of the wavefronts that
        // share its SIMD
        __builtin_amdgcn_s_setprio(3);
        uint32_t acc = 0;
        int32_t b = 0, s = 0, slot = 0;
        // flips of the previous block: to spin +1 (bit 1 -> 0) and to -1
        unsigned long long pFp = 0ull, pFn = 0ull;
        const unsigned long long lt = (1ull << lane) - 1ull;   // lanes before this one
        const unsigned long long gt = ~lt & ~(1ull << lane);   // lanes after it
        // field change of this lane from flips F+ (to +1) and F- (to -1) with
        // coupling bits row (bit j = 1: J = -1): sum over j of 2 s_j' J_jk
        auto delta = [](unsigned long long fp, unsigned long long fn, unsigned long long row) -> int32_t {
            return 2 * (__popcll(fp) - __popcll(fn)) - 4 * (__popcll(fp & row) - __popcll(fn & row));
        };
        for (int64_t g = 0; g < total; ++g) {
            wait_ge(L, kPrepared, (int32_t)(g + 1), err);
            if (g > DW) wait_ge(L, kApplied, (int32_t)(g - DW), err);
            const int32_t p = (b << 6) + lane;
            const bool act = p < n;
            const int32_t xm = L.xm[slot * 64 + lane];
            const uint32_t* tl = L.tile + ((size_t)slot * 64 + lane) * kTileWords;
            const unsigned long long D = ((unsigned long long)tl[1] << 32) | tl[0];   // own row, this block
            int32_t Hp = act ? L.H[p] : 0;
            uint32_t sb = act ? (L.bits[p >> 5] >> (p & 31)) & 1u : 0u;
            // this block's fields still miss the flips of the previous block
            if (DW >= 1 && g >= 1) {
                const unsigned long long C = ((unsigned long long)tl[3] << 32) | tl[2];   // own row, previous block
                Hp += delta(pFp, pFn, C);
            }
            // Decisions in rounds.  A lane's decision is certain once it
            // cannot change whichever way the undecided lanes before it go:
            // each of them moves its field by at most 2.  The first undecided
            // lane is always certain, so every round decides at least one lane
            // (the exact sequential result, usually in one or two rounds).  The
            // flips decided in a round change the fields of the lanes after
            // them at once; after the last round every lane adds the flips
            // after it.
            unsigned long long SB = __builtin_amdgcn_ballot_w64(sb != 0u);
            unsigned long long und = __builtin_amdgcn_ballot_w64(act);
            unsigned long long Fp = 0ull, Fn = 0ull;
            int32_t nf = 0;
            while (und != 0ull) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(und >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)und, 0u));
                const bool mine = (und >> lane) & 1ull;
                const int32_t x = sb ? -Hp : Hp;
                const int32_t slack = 2 * (int32_t)below;
                const unsigned long long F = __builtin_amdgcn_ballot_w64(mine && x + slack <= xm);
                const unsigned long long K = __builtin_amdgcn_ballot_w64(mine && x - slack > xm);
                und &= ~(F | K);
                const unsigned long long fp = F & SB, fn = F & ~SB;
                Hp += delta(fp & lt, fn & lt, D);
                if ((F >> lane) & 1ull) {
                    // flip entry: local row | (new spin -1) << 31, in lane order
                    L.flips[slot * 64 + nf + __popcll(F & lt)] = lane | (int32_t)((sb ^ 1u) << 31);
                    sb ^= 1u;
                }
                nf += __popcll(F);
                SB ^= F;
                Fp |= fp;
                Fn |= fn;
            }
            Hp += delta(Fp & gt, Fn & gt, D);
            pFp = Fp;
            pFn = Fn;
            if (act) L.H[p] = Hp;
            const unsigned long long mask = __ballot(sb != 0u);
            if (lane == 0) {
                L.bits[2 * b] = (uint32_t)mask;
                if (2 * b + 1 < wn) L.bits[2 * b + 1] = (uint32_t)(mask >> 32);
                L.nflip[slot] = nf;
                acc += (uint32_t)nf;
            }
            wave_release();
            if (lane == 0) st_rel(&L.sync[kDecided], (int32_t)(g + 1));
            if (++slot == kRing) slot = 0;
            if (++b == NB) {
                b = 0;
                ++s;
                const int64_t tn = t0 + s;
                if (tn <= t_max && (tn & (tn - 1)) == 0) {
                    const int k = 1 + (63 - __clzll((unsigned long long)tn));
                    for (int32_t w = lane; w < wn; w += 64) gl(ch->snap)[(int64_t)k * wn + w] = L.bits[w];
                }
            }
        }
        if (lane == 0 && acc) atomicAdd(ch->accepted, (unsigned long long)acc);
    } else {
        // ---------------- updaters ----------------
        // updater lane items: kUpdCols consecutive fields (one slice of a
        // coupling-row word)
        const int ut = tid - 128;
        const int32_t nitem = (n + kUpdCols - 1) / kUpdCols;
        int32_t bk = 0, slot = 0;
        for (int64_t k = 0; k < total; ++k) {
            wait_ge(L, kDecided, (int32_t)(k + 1), err);
            const int32_t nf = L.nflip[slot];
            // blocks bk + d (1 <= d <= DW) decided later in this launch get
            // this batch from the decider's correction
            const int32_t dskip = (int32_t)min((int64_t)DW, total - 1 - k);
            if (nf > 0) {
                for (int32_t h = ut; h < nitem; h += 64 * kUpdWaves) {
                    const int32_t col0 = h * kUpdCols;
                    int32_t dist = (col0 >> 6) - bk;
                    if (dist < 0) dist += NB;
                    if (dist <= dskip) continue;   // dist 0: the flipped block itself
                    const int32_t wi = col0 >> 5;
                    const uint32_t shift = (uint32_t)col0 & 31u;
                    int32_t accb[kUpdCols];
#pragma unroll
                    for (int c = 0; c < kUpdCols; ++c) accb[c] = 0;
                    int32_t sum2 = 0;
                    for (int32_t f0 = 0; f0 < nf; f0 += 8) {
                        // eight independent row loads in flight: every load
                        // is issued (entries past the last flip re-read the
                        // last flip's row and are weighted 0), so no load
                        // sits behind a branch that waits for the one before
                        uint32_t wv[8];
                        int32_t s2v[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const bool live = f0 + i < nf;
                            const int32_t fv = L.flips[slot * 64 + min(f0 + i, nf - 1)];
                            s2v[i] = live ? (fv < 0 ? -2 : 2) : 0;
                            wv[i] = Jb[(int64_t)((bk << 6) + (fv & 63)) * wn + wi];
                        }
#pragma unroll
                        for (int i = 0; i < 8; ++i) wv[i] >>= shift;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            sum2 += s2v[i];
#pragma unroll
                            for (int c = 0; c < kUpdCols; ++c) accb[c] += (int32_t)((wv[i] >> c) & 1u) * s2v[i];
                        }
                    }
                    // H_c += sum_f 2 s_f J_fc with J = 1 - 2 bit
#pragma unroll
                    for (int c = 0; c < kUpdCols; ++c) {
                        const int32_t col = col0 + c;
                        if (col < n) L.H[col] += sum2 - 2 * accb[c];
                    }
                }
            }
            wave_release();
            if (lane == 0) {
                const int old = __hip_atomic_fetch_add(&L.sync[kDone + slot], 1, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if (old == kUpdWaves - 1) {
                    L.sync[kDone + slot] = 0;
                    st_rel(&L.sync[kApplied], (int32_t)(k + 1));
                }
            }
            if (++slot == kRing) slot = 0;
            bk = bk + 1 == NB ? 0 : bk + 1;
        }
    }
    __syncthreads();

    for (int32_t i = tid; i < n; i += nthr) gl(ch->H)[i] = L.H[i];
    for (int32_t w = tid; w < wn; w += nthr) gl(ch->state)[w] = L.bits[w];
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

// A operand of v_mfma_i32_16x16x64_i8: 16 bytes of row `row` of J from column k0.
__device__ __forceinline__ v4i j_bytes(const int8_t* __restrict__ J, int32_t n, int32_t row, int32_t k0)
{
    v4i a = {0, 0, 0, 0};
    if (row >= n) return a;
    const int8_t* src = J + (int64_t)row * n + k0;
    if ((n & 15) == 0 && k0 + 16 <= n) {
        const int4 v = *(const int4*)src;
        a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
    } else {
        uint32_t w4[4] = {0, 0, 0, 0};
        for (int b = 0; b < 16; ++b)
            if (k0 + b < n) w4[b >> 2] |= (uint32_t)(uint8_t)src[b] << (8 * (b & 3));
        a[0] = (int)w4[0]; a[1] = (int)w4[1]; a[2] = (int)w4[2]; a[3] = (int)w4[3];
    }
    return a;
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
    const int kg = lane >> 4;
    const int jc = lane & 15;               // chain column of operand B
    const SkChain* cj = jc < nch ? &chains[sm->chain0 + jc] : nullptr;
    v4i acc = {0, 0, 0, 0};
    for (int32_t kc = 0; kc < n; kc += 64) {
        const int32_t k0 = kc + 16 * kg;
        const v4i a = j_bytes(sm->J, n, i0 + (lane & 15), k0);
        v4i bv = {0, 0, 0, 0};
        if (cj != nullptr && k0 < n) {
            const uint32_t bits = (cj->state[k0 >> 5] >> (k0 & 31)) & 0xffffu;
            const int32_t valid = min(16, n - k0);
            bv = expand16(bits, valid >= 16 ? 0xffffu : ((1u << valid) - 1u));
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

// Bond sums of the snapshots: D = J S for the columns (chain r, snapshot k) of
// one sample by int8 MFMA, then sum_i S_ic D_ic.  Accumulates 2 B into
// out[chain][k]; grid = (row blocks, column tiles of 16, samples).
__global__ void __launch_bounds__(256) sk_bond_kernel(const SkSample* __restrict__ samples,
                                                      const SkChain* __restrict__ chains, int kd,
                                                      int k_cap, long long* __restrict__ out)
{
    const SkSample* sm = samples + blockIdx.z;
    const int32_t n = sm->n, nch = sm->nch;
    const int32_t i0 = blockIdx.x * 64 + (threadIdx.x >> 6) * 16;
    const int32_t ncol = nch * kd;
    if (i0 >= n || (int32_t)blockIdx.y * 16 >= ncol) return;
    const int lane = threadIdx.x & 63;
    const int kg = lane >> 4;
    const int32_t col = blockIdx.y * 16 + (lane & 15);
    const bool live = col < ncol;
    const int32_t cr = live ? col / kd : 0, ck = live ? col - (col / kd) * kd : 0;
    const SkChain* cj = &chains[sm->chain0 + cr];
    const uint32_t* snap = cj->snap + (int64_t)ck * cj->words_n;
    v4i acc = {0, 0, 0, 0};
    for (int32_t kc = 0; kc < n; kc += 64) {
        const int32_t k0 = kc + 16 * kg;
        const v4i a = j_bytes(sm->J, n, i0 + (lane & 15), k0);
        v4i bv = {0, 0, 0, 0};
        if (live && k0 < n) {
            const uint32_t bits = (snap[k0 >> 5] >> (k0 & 31)) & 0xffffu;
            const int32_t valid = min(16, n - k0);
            bv = expand16(bits, valid >= 16 ? 0xffffu : ((1u << valid) - 1u));
        }
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bv, acc, 0, 0, 0);
    }
    long long part = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int32_t i = i0 + 4 * kg + r;
        if (live && i < n) {
            const int32_t si = ((snap[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
            part += (long long)si * acc[r];
        }
    }
    // lanes l, l+16, l+32, l+48 hold the same column
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (live && kg == 0)
        atomicAdd((unsigned long long*)&out[(int64_t)(sm->chain0 + cr) * k_cap + ck],
                  (unsigned long long)part);
}

}  // namespace

size_t sk_lds_bytes(int32_t n)
{
    const size_t wn = (size_t)(n + 31) / 32;
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return r16((size_t)n * 4) + r16((wn + 2) * 4) + r16((size_t)kThrCache * 8) + r16(kRing * 64 * 4) +
           r16((size_t)kRing * 64 * kTileWords * 4) + r16(kRing * 64 * 4) + r16(kRing * 4) +
           r16((4 + kRing) * 4) + 64 * 16;
}

int sk_threads() { return kSkThreads; }

hipError_t sk_init(const SkChain* chains, int n_chains, int threads, hipStream_t s)
{
    if (n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(sk_init_kernel, dim3(n_chains), dim3(threads), 0, s, chains);
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

hipError_t sk_bond(const SkSample* samples, int n_samples, const SkChain* chains, int max_n, int max_nch,
                   int k_done, int k_cap, long long* out, hipStream_t s)
{
    if (n_samples <= 0 || k_done <= 0) return hipSuccess;
    dim3 grid((max_n + 63) / 64, (max_nch * k_done + 15) / 16, n_samples);
    hipLaunchKernelGGL(sk_bond_kernel, grid, dim3(256), 0, s, samples, chains, k_done, k_cap, out);
    return hipGetLastError();
}

hipError_t sk_sweep(const SkChain* chains, int n_chains, int, size_t lds_bytes, int64_t t0,
                    int32_t n_sweeps, int64_t t_max, int* err_flag, hipStream_t s)
{
    if (n_chains <= 0 || n_sweeps <= 0) return hipSuccess;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)sk_sweep_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(sk_sweep_kernel, dim3(n_chains), dim3(kSkThreads), lds_bytes, s, chains, t0,
                       n_sweeps, t_max, err_flag);
    return hipGetLastError();
}

}  // namespace sg
