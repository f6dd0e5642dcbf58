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
//    couplings, lane i's own row 64 b + i restricted to the columns of block b
//    and of the kWin blocks before it (J is symmetric: these are the
//    couplings of those blocks' spins to spin i).
//  * decider wavefront: lane i owns spin 64 b + i.  It corrects the block's
//    fields for the flips of the previous kWin blocks (masked popcounts of
//    their flip masks against its own row), then decides the block in rounds:
//    a lane whose decision cannot change whichever way the undecided lanes
//    before it go (each moves its field by at most 2) is decided now, the
//    first undecided lane always is, and the flips decided in a round change
//    the fields of the later lanes by masked popcounts against the own-block
//    row.  The result is exactly the plain sequential sweep.  The block's
//    flips are published to a ring buffer.
//  * updater wavefronts: apply each published block's flips to all other fields
//    (H_k += 2 s_j J_jk, rows read bit-packed, a few fields per lane), up to
//    kWin blocks behind the decider; they skip the flipped block (patched in
//    the decider) and the next kWin blocks (corrected by the decider), except
//    for blocks decided after the end of the launch.
//
// Every `period` sweeps the fields are recomputed exactly as H = J S with int8
// MFMA (v_mfma_i32_16x16x64_i8, int32 accumulation) and compared with the
// incremental ones; a mismatch raises the context's error flag.  Bond sums
// B = (1/2) s^T J s of the snapshots are computed the same way at measurement
// time.
#include <type_traits>

#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// Pipeline depth (compile-time tuning parameters).
#ifndef SG_SK_RING
#define SG_SK_RING 4
#endif
#ifndef SG_SK_WIN
#define SG_SK_WIN 1
#endif
constexpr int kRing = SG_SK_RING;   // blocks in flight between the roles
constexpr int kWin = SG_SK_WIN;     // previous blocks the decider corrects for itself
constexpr int kTileWords = (2 + 2 * kWin + 3) & ~3;   // per lane: own-block row, kWin previous rows (16-byte multiple)
constexpr int kThrCache = 512;      // threshold entries cached in LDS
// Updater wavefronts: a lane owns 8 fields per pass, so 14 wavefronts (a
// workgroup of 1024 threads) apply a block to up to 7168 fields in one pass.
// Measured, us per sweep with 8 / 12 / 14: N = 4096 100.6 / 100.8 / 100.9
// (one pass each), N = 5944 203 / 169 / 169, N = 8192 364 / 326 / 314.
#ifndef SG_SK_UPD
#define SG_SK_UPD 14
#endif
#ifndef SG_SK_SLEEP
#define SG_SK_SLEEP 1   // s_sleep units (64 clocks) between polls of a wait
#endif
#ifndef SG_SK_UPB
#define SG_SK_UPB 1
#endif
#ifndef SG_SK_PROF
#define SG_SK_PROF 0    // 1: per-role cycle counters, printed by workgroups 0..2 after a launch
#endif
#if SG_SK_PROF
#define SK_CLK(v) const unsigned long long v = clock64()
#define SK_ACC(acc, a, b) (acc) += (b) - (a)
#else
#define SK_CLK(v)
#define SK_ACC(acc, a, b)
#endif
constexpr int kUpdWaves = SG_SK_UPD;   // updater wavefronts
constexpr int kUpdBlocks = SG_SK_UPB;  // decided blocks an updater pass takes at most
static_assert(kUpdBlocks >= 1 && kUpdBlocks <= kRing, "updater pass width");
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
    int32_t* nflip;             // [kRing]: flips | flips to +1 << 8
    int32_t* sync;              // decided, prepared, abort, progress[kUpdWaves]
    uint4* pr;                  // [64] Philox blocks of the prep's current 4 spin blocks
    unsigned long long* spr;    // [512] byte-spread table of the updaters
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
    L.sync = (int32_t*)take((size_t)(3 + kUpdWaves) * 4);
    L.pr = (uint4*)take(64 * 16);
    L.spr = (unsigned long long*)take(512 * 8);
    return L;
}

enum { kDecided = 0, kPrepared = 1, kAbort = 2, kProg = 3 };

__device__ __forceinline__ int ld_acq(int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void st_rel(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One poll of a wait that has not been met yet: true when the wait must end
// without its condition (abort raised, or this wait was the one that ran out
// of polls: after kSpinLimit polls the pipeline is declared stuck, the abort
// flag releases every other wait and the context's error flag reports it).
__device__ __forceinline__ bool wait_giveup(const SkLds& L, int& spins, int* err)
{
    if (ld_acq(&L.sync[kAbort])) return true;
    if (SG_SK_SLEEP > 0) __builtin_amdgcn_s_sleep(SG_SK_SLEEP);
    if (++spins > kSpinLimit) {
        st_rel(&L.sync[kAbort], 1);
        atomicOr(err, 2);
        return true;
    }
    return false;
}

// Waits (whole wavefront) until *p >= target.
__device__ __forceinline__ void wait_ge(const SkLds& L, int32_t idx, int32_t target, int* err)
{
    int spins = 0;
    while (ld_acq(&L.sync[idx]) < target) {
        if (wait_giveup(L, spins, err)) return;
    }
}

// Waits (whole wavefront) until every updater wavefront has applied the
// first `target` blocks of the launch (lane w reads wavefront w's progress).
__device__ __forceinline__ void wait_applied(const SkLds& L, int32_t target, int* err)
{
    const int lane = threadIdx.x & 63;
    int spins = 0;
    while (__builtin_amdgcn_ballot_w64(lane < kUpdWaves && ld_acq(&L.sync[kProg + lane]) < target) != 0ull) {
        if (wait_giveup(L, spins, err)) return;
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
    if (tid < 3 + kUpdWaves) L.sync[tid] = 0;
    for (int e = tid; e < 512; e += nthr) {
        // byte c of entry b + 256 m: bit c of b, in the low nibble (m = 0) or
        // the high nibble (m = 1)
        unsigned long long v = 0ull;
        for (int c = 0; c < 8; ++c) v |= (unsigned long long)((e >> c) & 1) << (8 * c + 4 * (e >> 8));
        L.spr[e] = v;
    }
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
        // spin i), stored contiguously per block by the host (zero past the
        // last row or column and beyond DW); the tiles of the next block are
        // loaded while this block's uniforms are drawn
        static_assert(kTileWords % 4 == 0, "tiles are read as 16-byte vectors");
        uint32_t tw[kTileWords];
        const SG_G v4u* __restrict__ Jt = (const SG_G v4u*)gl(ch->Jt);
        auto load_tiles = [&](int32_t bq) {
            const SG_G v4u* src = Jt + ((size_t)((bq << 6) + lane) * kTileWords) / 4;
#pragma unroll
            for (int v = 0; v < kTileWords / 4; ++v) {
                const v4u q = src[v];
                tw[4 * v] = q.x;
                tw[4 * v + 1] = q.y;
                tw[4 * v + 2] = q.z;
                tw[4 * v + 3] = q.w;
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
            // (entries cached in LDS first; a long table's tail is read from
            // HBM on a path of its own, so that the common path holds no
            // wait for this wavefront's outstanding loads)
            if (x0 < cached) {
                while (x0 > 0 && !((unsigned long long)r < L.thr[x0])) --x0;
                while (x0 + 1 < cached && (unsigned long long)r < L.thr[x0 + 1]) ++x0;
            }
            if (x0 + 1 >= cached && cached < ch->thr_len) {
                while (x0 > 0 && !((unsigned long long)r < thr_at(L, ch, cached, x0))) --x0;
                while (x0 + 1 < ch->thr_len && (unsigned long long)r < thr_at(L, ch, cached, x0 + 1)) ++x0;
            }
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
        // flips of the previous kWin blocks (d = 0: the block before this
        // one): to spin +1 (bit 1 -> 0) and to -1
        unsigned long long pFp[kWin], pFn[kWin];
#pragma unroll
        for (int d = 0; d < kWin; ++d) pFp[d] = pFn[d] = 0ull;
        const unsigned long long lt = (1ull << lane) - 1ull;   // lanes before this one
        const unsigned long long gt = ~lt & ~(1ull << lane);   // lanes after it
        // field change of this lane from flips F+ (to +1) and F- (to -1) with
        // coupling bits row (bit j = 1: J = -1): sum over j of 2 s_j' J_jk
        auto delta = [](unsigned long long fp, unsigned long long fn, unsigned long long row) -> int32_t {
            return 2 * (__popcll(fp) - __popcll(fn)) - 4 * (__popcll(fp & row) - __popcll(fn & row));
        };
#if SG_SK_PROF
        // cycles waiting for the prep, reading its outputs, waiting for the
        // updaters, correcting the fields, deciding, publishing; rounds
        unsigned long long tp[7] = {0, 0, 0, 0, 0, 0, 0};
#endif
        for (int64_t g = 0; g < total; ++g) {
            SK_CLK(c0);
            wait_ge(L, kPrepared, (int32_t)(g + 1), err);
            SK_CLK(c1);
            SK_ACC(tp[0], c0, c1);
            // the prep's outputs and the spins (written by this wavefront
            // only) are read before waiting for the updaters
            const int32_t p = (b << 6) + lane;
            const bool act = p < n;
            const int32_t xm = L.xm[slot * 64 + lane];
            const uint32_t* tl = L.tile + ((size_t)slot * 64 + lane) * kTileWords;
            const unsigned long long D = ((unsigned long long)tl[1] << 32) | tl[0];   // own row, this block
            uint32_t sb = act ? (L.bits[p >> 5] >> (p & 31)) & 1u : 0u;
            SK_CLK(c2);
            SK_ACC(tp[1], c1, c2);
            if (g > DW) wait_applied(L, (int32_t)(g - DW), err);
            SK_CLK(c3);
            SK_ACC(tp[2], c2, c3);
            int32_t Hp = act ? L.H[p] : 0;
            // this block's fields still miss the flips of the previous DW
            // blocks (own row restricted to block b - d, d = 1..DW)
#pragma unroll
            for (int d = 1; d <= kWin; ++d) {
                if (d <= DW && g >= d) {
                    const unsigned long long C = ((unsigned long long)tl[2 * d + 1] << 32) | tl[2 * d];
                    Hp += delta(pFp[d - 1], pFn[d - 1], C);
                }
            }
            // Decisions in rounds.  A lane's decision is certain once it
            // cannot change whichever way the undecided lanes before it go:
            // each of them would move its x by 2, in a direction known from
            // the spins and the coupling.  The first undecided lane is always
            // certain, so every round decides at least one lane (the exact
            // sequential result, in about three rounds).  The flips decided in
            // a round change the fields of the lanes after them at once; after
            // the last round every lane adds the flips after it.
            SK_CLK(c4);
            SK_ACC(tp[3], c3, c4);
            unsigned long long SB = __builtin_amdgcn_ballot_w64(sb != 0u);
            unsigned long long und = __builtin_amdgcn_ballot_w64(act);
            unsigned long long Fp = 0ull, Fn = 0ull;
            int32_t nf = 0;
            while (und != 0ull) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(und >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)und, 0u));
                const bool mine = (und >> lane) & 1ull;
                const int32_t x = sb ? -Hp : Hp;
                // a flip of an undecided lane j before this one changes x by
                // -2 s s_j J_j: down where s s_j J_j > 0 (spin and coupling
                // bits XOR to 0), up elsewhere
                const unsigned long long own = sb ? ~0ull : 0ull;
                const int32_t dn = __popcll(~(SB ^ D ^ own) & und & lt);
                const int32_t upc = (int32_t)below - dn;
                const unsigned long long F = __builtin_amdgcn_ballot_w64(mine && x + 2 * upc <= xm);
                const unsigned long long K = __builtin_amdgcn_ballot_w64(mine && x - 2 * dn > xm);
                und &= ~(F | K);
                const unsigned long long fp = F & SB, fn = F & ~SB;
                Hp += delta(fp & lt, fn & lt, D);
                if ((F >> lane) & 1ull) {
                    // flip entry: local row | (new spin -1) << 31, in lane order
                    L.flips[slot * 64 + nf + __popcll(F & lt)] = lane | (int32_t)((sb ^ 1u) << 31);
                    sb ^= 1u;
                }
                nf += __popcll(F);
#if SG_SK_PROF
                ++tp[6];
#endif
                SB ^= F;
                Fp |= fp;
                Fn |= fn;
            }
            SK_CLK(c5);
            SK_ACC(tp[4], c4, c5);
            Hp += delta(Fp & gt, Fn & gt, D);
#pragma unroll
            for (int d = kWin - 1; d > 0; --d) {
                pFp[d] = pFp[d - 1];
                pFn[d] = pFn[d - 1];
            }
            pFp[0] = Fp;
            pFn[0] = Fn;
            if (act) L.H[p] = Hp;
            const unsigned long long mask = __ballot(sb != 0u);
            if (lane == 0) {
                L.bits[2 * b] = (uint32_t)mask;
                if (2 * b + 1 < wn) L.bits[2 * b + 1] = (uint32_t)(mask >> 32);
                L.nflip[slot] = nf | (__popcll(Fp) << 8);
                acc += (uint32_t)nf;
            }
            wave_release();
            if (lane == 0) st_rel(&L.sync[kDecided], (int32_t)(g + 1));
            SK_CLK(c6);
            SK_ACC(tp[5], c5, c6);
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
#if SG_SK_PROF
        if (lane == 0 && blockIdx.x < 3)
            printf("[sk-prof] wg %d decider blocks %lld cycles: wait-prep %llu reads %llu wait-updaters %llu "
                   "correct %llu rounds %llu publish %llu; rounds %llu\n",
                   (int)blockIdx.x, (long long)total, tp[0], tp[1], tp[2], tp[3], tp[4], tp[5], tp[6]);
#endif
    } else {
        // ---------------- updaters ----------------
        // An updater lane owns items of 8 consecutive fields (one byte of a
        // coupling-row word).  L.spr spreads the row byte of a flip over the
        // bytes of a 64-bit word: bit c goes to byte c, in its low nibble for a
        // flip to +1 and its high nibble for a flip to -1, so one 64-bit add
        // per flip counts the couplings of all 8 fields (8 flips per batch:
        // no nibble overflows).  A wavefront takes every decided block it
        // finds, up to kUpdBlocks, in one pass: their row loads share one
        // memory latency.  Its progress word tells the decider how many blocks
        // of the launch it has applied.
        const int uw = wave - 2;   // updater index
        const int ut = uw * 64 + lane;
        const int32_t nitem = (n + 7) >> 3;
        const char* sprb = (const char*)L.spr;
        int32_t bk = 0, slot = 0;
#if SG_SK_PROF
        unsigned long long tu[2] = {0, 0};   // cycles waiting for decided blocks, applying them
#endif
        for (int64_t k = 0; k < total;) {
            SK_CLK(u0);
            wait_ge(L, kDecided, (int32_t)(k + 1), err);
            SK_CLK(u1);
            SK_ACC(tu[0], u0, u1);
            int32_t np = 1;
            if (kUpdBlocks > 1) {
                const int32_t dec = __builtin_amdgcn_readfirstlane(ld_acq(&L.sync[kDecided]));
                np = (int32_t)max((int64_t)1, min((int64_t)kUpdBlocks, min((int64_t)dec, total) - k));
            }
            // per block j of the pass: ring slot, block index, first flip in
            // the concatenated list, sum of 2 s' over its flips, and the
            // blocks after it whose columns the decider corrects itself
            int32_t sl[kUpdBlocks], bq[kUpdBlocks], cum[kUpdBlocks + 1], s2[kUpdBlocks], dsk[kUpdBlocks];
            cum[0] = 0;
#pragma unroll
            for (int j = 0; j < kUpdBlocks; ++j) {
                sl[j] = j == 0 ? slot : (sl[j - 1] + 1 == kRing ? 0 : sl[j - 1] + 1);
                bq[j] = j == 0 ? bk : (bq[j - 1] + 1 == NB ? 0 : bq[j - 1] + 1);
                const int32_t w = j < np ? __builtin_amdgcn_readfirstlane(L.nflip[sl[j]]) : 0;
                const int32_t nfj = w & 0xff;
                cum[j + 1] = cum[j] + nfj;
                s2[j] = 2 * (2 * (w >> 8) - nfj);
                dsk[j] = (int32_t)min((int64_t)DW, total - 1 - (k + j));
            }
            const int32_t ntot = cum[kUpdBlocks];
            if (ntot > 0) {
                for (int32_t h = ut; h < nitem; h += 64 * kUpdWaves) {
                    const int32_t col0 = h << 3;
                    // the item takes a block's flips unless it lies in the
                    // flipped block (patched in the decider) or in one of the
                    // next dsk blocks (corrected by the decider)
                    bool use[kUpdBlocks];
                    bool any = false;
                    int32_t sum2 = 0;
#pragma unroll
                    for (int j = 0; j < kUpdBlocks; ++j) {
                        int32_t dist = (col0 >> 6) - bq[j];
                        if (dist < 0) dist += NB;
                        use[j] = j < np && dist > dsk[j];
                        any = any || use[j];
                        sum2 += use[j] ? s2[j] : 0;
                    }
                    if (!any) continue;
                    const int32_t wi = col0 >> 5;
                    const uint32_t shift = (uint32_t)col0 & 31u;
                    int32_t dlt[8];   // per field: flips to +1 minus flips to -1 with coupling bit 1
#pragma unroll
                    for (int c = 0; c < 8; ++c) dlt[c] = 0;
                    // One batch: NL row loads in flight, all issued before any
                    // is used (the NL flip entries are read from LDS first, so
                    // their latencies overlap too); entries past the last flip
                    // re-read its row with a zero-width byte.  Batches of 16
                    // when more than 8 flips are left, so that a block with up
                    // to 16 flips costs one memory latency.
                    auto batch = [&](int32_t f0, auto nlc) {
                        constexpr int NL = decltype(nlc)::value;
                        uint32_t wv[NL], wd[NL], tb[NL];
                        int32_t fe[NL], rb[NL];
#pragma unroll
                        for (int i = 0; i < NL; ++i) {
                            const int32_t fi = min(f0 + i, ntot - 1);
                            int32_t slj = sl[0], bqj = bq[0], cj = 0;
                            bool uj = use[0];
#pragma unroll
                            for (int j = 1; j < kUpdBlocks; ++j) {
                                if (fi >= cum[j]) {
                                    slj = sl[j];
                                    bqj = bq[j];
                                    cj = cum[j];
                                    uj = use[j];
                                }
                            }
                            fe[i] = L.flips[slj * 64 + fi - cj];
                            rb[i] = bqj << 6;
                            wd[i] = (f0 + i < ntot && uj) ? 8u : 0u;
                        }
#pragma unroll
                        for (int i = 0; i < NL; ++i) {
                            const int32_t fv = __builtin_amdgcn_readfirstlane(fe[i]);
                            tb[i] = fv < 0 ? 2048u : 0u;
                            wv[i] = Jb[(int64_t)(rb[i] + (fv & 63)) * wn + wi];
                        }
                        // nibble counts of 8 flips at a time (at most 8: no carry)
#pragma unroll
                        for (int i0 = 0; i0 < NL; i0 += 8) {
                            unsigned long long acc = 0ull;
#pragma unroll
                            for (int i = i0; i < i0 + 8; ++i) {
                                const uint32_t byte = __builtin_amdgcn_ubfe(wv[i], shift, wd[i]);
                                acc += *(const unsigned long long*)(sprb + tb[i] + (byte << 3));
                            }
                            const uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                dlt[c] += (int32_t)__builtin_amdgcn_ubfe(lo, 8u * c, 4u) -
                                          (int32_t)__builtin_amdgcn_ubfe(lo, 8u * c + 4u, 4u);
                                dlt[c + 4] += (int32_t)__builtin_amdgcn_ubfe(hi, 8u * c, 4u) -
                                              (int32_t)__builtin_amdgcn_ubfe(hi, 8u * c + 4u, 4u);
                            }
                        }
                    };
                    for (int32_t f0 = 0; f0 < ntot;) {
                        if (ntot - f0 > 8) {
                            batch(f0, std::integral_constant<int, 16>{});
                            f0 += 16;
                        } else {
                            batch(f0, std::integral_constant<int, 8>{});
                            f0 += 8;
                        }
                    }
                    // H_c += sum over flips of 2 s' J_fc, J = 1 - 2 bit
                    if (col0 + 8 <= n) {
                        int4* hp = (int4*)(L.H + col0);
                        int4 u0 = hp[0], u1 = hp[1];
                        u0.x += sum2 - 4 * dlt[0];
                        u0.y += sum2 - 4 * dlt[1];
                        u0.z += sum2 - 4 * dlt[2];
                        u0.w += sum2 - 4 * dlt[3];
                        u1.x += sum2 - 4 * dlt[4];
                        u1.y += sum2 - 4 * dlt[5];
                        u1.z += sum2 - 4 * dlt[6];
                        u1.w += sum2 - 4 * dlt[7];
                        hp[0] = u0;
                        hp[1] = u1;
                    } else {
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            if (col0 + c < n) L.H[col0 + c] += sum2 - 4 * dlt[c];
                    }
                }
            }
            wave_release();
            k += np;
            if (lane == 0) st_rel(&L.sync[kProg + uw], (int32_t)k);
            SK_CLK(u2);
            SK_ACC(tu[1], u1, u2);
            slot += np;
            if (slot >= kRing) slot -= kRing;
            bk += np;
            while (bk >= NB) bk -= NB;
        }
#if SG_SK_PROF
        if (lane == 0 && blockIdx.x < 3)
            printf("[sk-prof] wg %d updater %d cycles: wait %llu apply %llu\n", (int)blockIdx.x, uw, tu[0], tu[1]);
#endif
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
           r16((3 + kUpdWaves) * 4) + 64 * 16 + 512 * 8;
}

int sk_threads() { return kSkThreads; }
int sk_tile_words() { return kTileWords; }
int sk_window() { return kWin; }

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
    // set once (thread-safe initialisation of a local static)
    static const hipError_t attr = hipFuncSetAttribute((const void*)sk_sweep_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(sk_sweep_kernel, dim3(n_chains), dim3(kSkThreads), lds_bytes, s, chains, t0,
                       n_sweeps, t_max, err_flag);
    return hipGetLastError();
}

}  // namespace sg
