// Viana-Bray Metropolis sweeps on gfx950.
//
// One workgroup owns one work unit: a graph stored in sweep order (the
// colour classes of a proper colouring, the paper's bipartite parallel update
// generalised; SI "Simulations of the Bethe Lattice on GPUs") and up to eight
// chains that share it.  The chains' spins stay in LDS for the whole launch in
// the sliced packing of VbLayout (one 32-bit word = P = 32 / rpad consecutive
// positions of every chain, chain c in its own P-bit field), so that one LDS
// read of a neighbour's word returns its spin in every chain and the
// unsatisfied-bond counts of all chains advance with one shift, XOR, mask and
// add (4-bit fields while every degree of the chunk is below 16, else two
// sets of 8-bit fields).
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
// One Philox block serves the eight positions of an aligned group for one
// chain.  A wavefront draws 64 blocks per pass (one per lane) into LDS: the
// blocks of its next B = max(1, 8 / nch) chunks, so with 1, 2 or 4 chains no
// lane draws a block nobody uses.  A is compared with the high half of the threshold,
// read from a per-chain table indexed by 64 + x (entries for x <= 0 exceed
// every A); B is computed only when A ties with it (probability 2^-16).  The
// flips of a chunk are collected as one ballot per chain and written back by
// one lane per spin word.
#include "sg_internal.h"
#include "sg_philox.h"

namespace sg {
namespace {

constexpr int kDMax = 8;   // adjacency entries prefetched per position
constexpr int kTab = 128;  // threshold table per chain: index 64 + x, -63 <= x <= 63
constexpr int kThc = 32;   // compact threshold table per chain: index 15 - x, -16 <= x <= 15
constexpr int kMaxCls = 64; // colour classes (greedy colouring, degree <= 63)
// LDS byte offsets of the flip-spreading table (256 words) and of the spin
// words: the compact tables come first, so that all three are addressed
// with the instructions' constant offsets
constexpr uint32_t kSprOff = kVbMaxChains * kThc * 4;
constexpr uint32_t kSpOff = kSprOff + 256 * 4;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Compile-time form of VbLayout for a unit with RPAD chain slots.
template <int RPAD>
struct Sl {
    static constexpr int P = 32 / RPAD;             // positions per word (= field width)
    static constexpr int LP = RPAD == 1 ? 5 : RPAD == 2 ? 4 : RPAD == 4 ? 3 : 2;   // log2 P
    // field bottoms; for RPAD 8 the 4-bit fields
    static constexpr uint32_t M = RPAD == 1 ? 1u : RPAD == 2 ? 0x00010001u : RPAD == 4 ? 0x01010101u : 0x11111111u;
    // byte offset in LDS of the word holding position (en & 0x7fffffff); the
    // sign bit of an adjacency entry is masked off
    static __device__ __forceinline__ uint32_t boff(uint32_t en)
    {
        return (en & (0x7fffffffu & ~(uint32_t)(P - 1))) >> (LP - 2);
    }
};

struct VbLds {
    uint32_t* thc;                // [8][kThc] at LDS offset 0: 15 - x -> thr[x] >> 16; 0x10000 for x <= 0
    uint32_t* spr;                // [256] at kSprOff: bit c of v -> bit 4 c of spr[v]
    uint32_t* sp;                 // spins, VbLayout words, at LDS offset kSpOff
    uint32_t sp_lds;              // the same array as a byte offset in LDS
    uint32_t* cp;                 // (units with cpl) the complemented words
    uint32_t cp_lds;
    uint32_t* thr;                // [8][kTab]: 64 - x -> thr[x] >> 16; 0x10000 for x <= 0
    unsigned long long* accs;     // [8]
    int32_t* flag;                // [4]: split units' abort flag
    int32_t* cls;                 // [kMaxCls + 1] first position of each colour class
    uint32_t* ri;                 // [8][2]: replica, instance of each chain
    uint32_t* wacc;               // [kMaxGrid][8]: window overlap counts of a sweep
    uint4* xch;                   // [waves][64] Philox blocks of a batch of chunks
    int32_t* area;                // resident adjacency: row starts, then entries
};

// Chunks whose Philox blocks one pass of 64 lanes draws.
__host__ __device__ __forceinline__ int32_t vb_batch_chunks(int32_t nch)
{
    return nch <= 8 ? (8 / nch > 0 ? 8 / nch : 1) : 1;
}

__device__ __forceinline__ VbLds vb_carve(uint32_t* smem, uint32_t smem_lds, int32_t sw, int nthr, int32_t nch,
                                          bool cpl)
{
    VbLds L;
    const int32_t swp = (sw + 3) & ~3;
    L.thc = smem;
    L.spr = smem + kSprOff / 4;
    L.sp = smem + kSpOff / 4;
    L.sp_lds = smem_lds + kSpOff;
    L.cp = L.sp + swp;
    L.cp_lds = L.sp_lds + 4u * (uint32_t)swp;
    L.thr = L.sp + (cpl ? 2 * swp : swp);
    L.accs = (unsigned long long*)(L.thr + kVbMaxChains * kTab);
    L.flag = (int32_t*)(L.accs + kVbMaxChains);
    L.cls = L.flag + 4;
    L.ri = (uint32_t*)(L.cls + kMaxCls + 4);
    L.wacc = L.ri + 2 * kVbMaxChains;
    L.xch = (uint4*)(L.wacc + kMaxGrid * kVbMaxChains);
    L.area = (int32_t*)(L.xch + (nthr >> 6) * 64);
    return L;
}

// Class bounds live in LDS and are read wave-uniformly: the cursor stays in
// scalar registers and its reads never wait on the vector-memory counter that
// the prefetched adjacency loads use.
__device__ __forceinline__ int32_t cls_at(const int32_t* cls, int32_t k)
{
    return __builtin_amdgcn_readfirstlane(cls[k]);
}

// Chunk cursor of one wavefront: sweep s, colour class k, chunk j of the class
// (the aligned block (cls[k] >> 6) + j of 64 positions).  The class's bounds
// and chunk count are kept with it, so that a step inside a class reads
// nothing from LDS.
struct Cursor {
    int32_t s, k, j;
    int32_t lo, hi, nck;
};

template <class PC>
__device__ __forceinline__ int32_t n_chunks(PC cls, int32_t k)
{
    const int32_t lo = cls_at(cls, k), hi = cls_at(cls, k + 1);
    return hi > lo ? ((hi - 1) >> 6) - (lo >> 6) + 1 : 0;
}

template <class PC>
__device__ __forceinline__ void cursor_class(Cursor& c, PC cls)
{
    c.lo = cls_at(cls, c.k);
    c.hi = cls_at(cls, c.k + 1);
    c.nck = c.hi > c.lo ? ((c.hi - 1) >> 6) - (c.lo >> 6) + 1 : 0;
}

// A cursor before the first chunk of wavefront `wave` (cursor_next moves it
// there).
template <class PC>
__device__ __forceinline__ Cursor cursor_start(int W, int wave, PC cls)
{
    Cursor c{0, 0, wave - W, 0, 0, 0};
    cursor_class(c, cls);
    return c;
}

// Moves to the next chunk owned by wavefront `wave`; false past the launch.
template <class PC>
__device__ __forceinline__ bool cursor_next(Cursor& c, int W, int wave, int32_t ncls, PC cls, int32_t nsw)
{
    c.j += W;
    for (;;) {
        if (c.j < c.nck) return true;
        c.j = wave;
        if (++c.k == ncls) {
            c.k = 0;
            if (++c.s >= nsw) return false;
        }
        cursor_class(c, cls);
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
    st.q = (((c.lo >> 6) + c.j) << 6) + lane;
    const bool act = st.q >= c.lo && st.q < c.hi;
    st.r0 = act ? row[st.q] : 0;
    st.r1 = act ? row[st.q + 1] : 0;
}

// Loads kDMax entries from the row start whatever the degree (the adjacency
// is followed by kVbEntPad zero entries): no load waits behind a branch.
template <class PE>
__device__ __forceinline__ void load_ents(PE ent, Stage& st)
{
    static_assert(kDMax <= kVbEntPad, "entry prefetch must stay inside the padded adjacency");
#pragma unroll
    for (int d = 0; d < kDMax; ++d) st.e[d] = ent[st.r0 + d];
}

// Metropolis decisions of one chunk for every chain, from the unsatisfied-bond
// counts: chain c's count is the `width`-bit field of cA (c even or RPAD < 8)
// or cB (c odd, RPAD 8, 8-bit fields) at bit fsh(c).  Returns this lane's
// flips in spin-word form (chain c's flip at bit c P).  The counts index the
// full tables (x = deg - 2 cnt at word c kTab + 64 - x).
template <int RPAD>
__device__ __forceinline__ uint32_t vb_decide_full(const VbUnit* __restrict__ up, const VbLds& L,
                                                   const uint32_t* gx, uint32_t cA, uint32_t cB, int32_t deg,
                                                   bool act, int32_t q, uint32_t t, int32_t nch, uint64_t key)
{
    using S = Sl<RPAD>;
    const int lane = threadIdx.x & 63;
    const uint32_t hsel = (uint32_t)lane & 7u;
    constexpr uint32_t width = RPAD == 8 ? 8u : (uint32_t)S::P;
    // (the counts are selected as values: a selected reference would put
    // cA and cB in private memory when c is not a constant)
    auto count = [&](int c) -> uint32_t {
        const uint32_t a = cA, b = cB;
        if (RPAD == 1) return a;
        const uint32_t fsh = RPAD == 8 ? 8u * (uint32_t)(c >> 1) : (uint32_t)(c * S::P);
        return __builtin_amdgcn_ubfe(RPAD == 8 && (c & 1) ? b : a, fsh, width);
    };
    // `tb` includes the lane's 4 (64 - deg), so each address is a single
    // shift-add
    const char* tb = (const char*)L.thr + (uint32_t)(64 - deg) * 4u;
    auto thr_of = [&](int c, uint32_t cnt) -> uint32_t { return *(const uint32_t*)(tb + c * kTab * 4 + (cnt << 3)); };
    const uint32_t hs = 16u * (hsel & 1u);
    uint32_t fl = 0;
    bool tie = false;
#pragma unroll
    for (int c = 0; c < RPAD; ++c) {
        if (c < nch) {
            const uint32_t th = thr_of(c, count(c));
            const uint32_t rh = __builtin_amdgcn_ubfe(gx[4 * c], hs, 16u);
            tie = tie || rh == th;
            fl |= rh < th ? 1u << (c * S::P) : 0u;
        }
    }
    fl = act ? fl : 0u;
    if (__builtin_amdgcn_ballot_w64(act && tie) != 0ull) {
        // A equals the high half of the threshold (those lanes did not flip
        // above): decide on the low half (rare: a loop, not unrolled)
#pragma unroll 1
        for (int c = 0; c < nch; ++c) {
            const uint32_t cnt = count(c);
            const uint32_t th = thr_of(c, cnt);
            const uint32_t rh = __builtin_amdgcn_ubfe(gx[4 * c], hs, 16u);
            const bool ti = act && rh == th;
            if (__builtin_amdgcn_ballot_w64(ti) != 0ull) {
                bool f2 = false;
                if (ti) {
                    const int32_t x = deg - 2 * (int32_t)cnt;
                    const U4 Bk = philox_stream(key, (uint32_t)q >> 3, t, kDomSweepLo, up->rep[c], up->inst[c]);
                    f2 = half_word(Bk, hsel) < gl(&up->thr_lo[c][0])[x];
                }
                fl |= f2 ? 1u << (c * S::P) : 0u;
            }
        }
    }
    return fl;
}

// The same with 8 chain slots and every degree of the chunk below 16 (the
// usual case), in fewer instructions.  The 4-bit counts are spread to bytes
// (even chains in oE, odd chains in oO, chain c at byte c / 2) and each byte
// is turned, for all chains at once, into the byte offset 4 (15 - x) = 60 -
// 4 deg + 8 cnt of the chain's entry in its compact table at LDS offset 0,
// so that one bit-field extract per chain addresses its threshold; the
// lane's random half-word is read as such, and e = A - thr (|e| < 2^17)
// decides: a flip iff e < 0, a tie iff e = 0.  The sign bits are shifted into a flip vector (bit c: chain c, from
// the highest chain down), which the spreading table turns into spin-word
// form; ties are detected by the running unsigned minimum of e.
__device__ __forceinline__ uint32_t vb_decide_compact(const VbUnit* __restrict__ up, const VbLds& L,
                                                      const uint32_t* gx, uint32_t cA, int32_t deg, bool act,
                                                      int32_t q, uint32_t t, int32_t nch, uint64_t key)
{
    typedef const __attribute__((address_space(3))) uint32_t lds_u32;
    const int lane = threadIdx.x & 63;
    // (60 - 4 deg) in every byte
    const uint32_t bias = __builtin_amdgcn_perm(0u, (uint32_t)(60 - 4 * deg), 0u);
    const uint32_t oE = ((cA & 0x0F0F0F0Fu) << 3) + bias;          // chain 2k at byte k
    const uint32_t oO = (((cA >> 4) & 0x0F0F0F0Fu) << 3) + bias;   // chain 2k + 1 at byte k
    const uint16_t* rp = (const uint16_t*)gx + (lane & 1);        // chain c's A at rp[8 c]
    uint32_t fv = 0u, emin = 0xFFFFFFFFu;
    auto chain = [&](int c) {
        const uint32_t off = __builtin_amdgcn_ubfe((c & 1) ? oO : oE, 8u * (uint32_t)(c >> 1), 8u);
        const uint32_t e = (uint32_t)rp[8 * c] - *(lds_u32*)(size_t)(off + (uint32_t)(c * kThc * 4));
        fv = __builtin_amdgcn_alignbit(fv, e, 31u);
        emin = min(emin, e);
    };
    // a unit with 8 slots has 5 to 8 chains: chains 0..4 are decided without
    // a test (in one block, so that their LDS reads are issued together)
#pragma unroll
    for (int c = kVbMaxChains - 1; c >= 5; --c)
        if (c < nch) chain(c);
#pragma unroll
    for (int c = 4; c >= 0; --c) chain(c);
    fv = act ? fv : 0u;
    uint32_t fl = *(lds_u32*)(size_t)(kSprOff + fv * 4u);
    if (__builtin_amdgcn_ballot_w64(act && emin == 0u) != 0ull) {
        // A equals the high half of the threshold (those lanes did not flip
        // above): decide on the low half (rare: a loop, not unrolled)
        const uint32_t hsel = (uint32_t)lane & 7u;
#pragma unroll 1
        for (int c = 0; c < nch; ++c) {
            const uint32_t src = (c & 1) ? oO : oE;
            const uint32_t off = __builtin_amdgcn_ubfe(src, 8u * (uint32_t)(c >> 1), 8u);
            const bool ti = act && (uint32_t)rp[8 * c] == *(lds_u32*)(size_t)(off + (uint32_t)(c * kThc * 4));
            if (__builtin_amdgcn_ballot_w64(ti) != 0ull) {
                bool f2 = false;
                if (ti) {
                    const int32_t x = 15 - (int32_t)(off >> 2);
                    const U4 Bk = philox_stream(key, (uint32_t)q >> 3, t, kDomSweepLo, up->rep[c], up->inst[c]);
                    f2 = half_word(Bk, hsel) < gl(&up->thr_lo[c][0])[x];
                }
                fl |= f2 ? 1u << (4 * c) : 0u;
            }
        }
    }
    return fl;
}

template <int RPAD>
__device__ __forceinline__ uint32_t vb_decide(const VbUnit* __restrict__ up, const VbLds& L, const uint32_t* gx,
                                              uint32_t cA, uint32_t cB, bool wide, int32_t deg, bool act,
                                              int32_t q, uint32_t t, int32_t nch, uint64_t key)
{
    if (RPAD == 8 && !wide) return vb_decide_compact(up, L, gx, cA, deg, act, q, t, nch, key);
    return vb_decide_full<RPAD>(up, L, gx, cA, cB, deg, act, q, t, nch, key);
}

// Updates the positions of one chunk for every chain of the unit and returns
// this lane's flips in spin-word form.  gx: this lane's group's Philox blocks
// of the chunk (chain c at gx + 4 c).
template <int RPAD, bool SPLIT, bool CPL, class PE>
__device__ __forceinline__ uint32_t vb_chunk(const VbUnit* __restrict__ up, const VbLds& L, PE ent, const Stage& st,
                                             int32_t lo, int32_t hi, uint32_t t, int32_t nch,
                                             uint64_t key, const uint32_t* gx)
{
    using S = Sl<RPAD>;
    // adjacency resident in LDS: such units are small and bound by the
    // latency of a chunk, not by instruction issue
    constexpr bool LAT = !__is_same(PE, const SG_G uint32_t*);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int32_t q = st.q;

    const bool act = q >= lo && q < hi;
    const int32_t deg = st.r1 - st.r0;   // 0 on inactive lanes
    // spin words read through a local-address-space pointer made from the
    // array's LDS offset (the constant kSpOff), so that the base is neither
    // kept in a register nor re-read for every neighbour
    const uint32_t spo = L.sp_lds;
    auto spw = [&](uint32_t off) -> uint32_t {
        return *(const __attribute__((address_space(3))) uint32_t*)(size_t)(spo + off);
    };
    const uint32_t qsh = (uint32_t)q & (uint32_t)(S::P - 1);
    // own word, position q at the field bottoms
    const uint32_t o0 = act ? spw(S::boff((uint32_t)q)) >> qsh : 0u;
    // bit c P of f: the bond to the neighbour is unsatisfied in chain c.
    // With a complemented copy of the words the entry holds the LDS byte
    // address of the neighbour's word (of its complement when J < 0) above
    // the in-word shift, which the shift takes from its low 5 bits
    auto unsat = [&](uint32_t en) {
        if (CPL) return (*(const __attribute__((address_space(3))) uint32_t*)(size_t)(en >> 5) >> (en & 31u)) ^ o0;
        const uint32_t sh = en & (uint32_t)(S::P - 1);
        return (spw(S::boff(en)) >> sh) ^ o0 ^ (uint32_t)((int32_t)en >> 31);
    };
    // per-chain counts of unsatisfied bonds: cA holds P-bit fields (for RPAD 8
    // while every degree of the chunk is below 16), else for RPAD 8 cA / cB
    // hold the even / odd chains in 8-bit fields
    uint32_t cA = 0, cB = 0;
    const bool wide = RPAD == 8 && __any(deg > 15);
    if (!wide) {
        if (LAT) {
            // every prefetched neighbour word is read before any is counted,
            // so that the LDS round trips overlap; a lane past its degree
            // reads its own word, whose contribution is zero (an inactive
            // lane reads word 0: its counts stay below 9 and are not used)
            const uint32_t qa = act ? (uint32_t)q : 0u;
            uint32_t wv[kDMax];
#pragma unroll
            for (int d = 0; d < kDMax; ++d) {
                const uint32_t en = d < deg ? st.e[d] : qa;
                wv[d] = (spw(S::boff(en)) >> (en & (uint32_t)(S::P - 1))) ^ (uint32_t)((int32_t)en >> 31);
            }
#pragma unroll
            for (int d = 0; d < kDMax; ++d) cA += (wv[d] ^ o0) & S::M;
        } else {
#pragma unroll
            for (int d = 0; d < kDMax; ++d) {
                if (!__any(d < deg)) break;
                if (d < deg) cA += unsat(st.e[d]) & S::M;
            }
        }
        for (int32_t d = kDMax; d < deg; ++d) cA += unsat(ent[st.r0 + d]) & S::M;
    } else {
        // rare (a degree above 15 in the chunk): entries re-read from the adjacency
        for (int32_t d = 0; d < deg; ++d) {
            const uint32_t f = unsat(ent[st.r0 + d]);
            cA += f & 0x01010101u;
            cB += (f >> 4) & 0x01010101u;
        }
    }

    const uint32_t fl = vb_decide<RPAD>(up, L, gx, cA, cB, wide, deg, act, q, t, nch, key);
    // write the flips back: every lane XORs its flips into its spin word (the
    // P lanes of a word are in this wavefront's chunk, nothing else writes it)
    if (fl) {
        const uint32_t wo = ((uint32_t)q >> S::LP) * 4u;
        __atomic_fetch_xor((__attribute__((address_space(3))) uint32_t*)(size_t)(spo + wo), fl << qsh,
                           __ATOMIC_RELAXED);
        if (CPL)
            __atomic_fetch_xor((__attribute__((address_space(3))) uint32_t*)(size_t)(L.cp_lds + wo), fl << qsh,
                               __ATOMIC_RELAXED);
    }
    if (SPLIT) {
        // a member of a split unit also writes the chunk's words through to HBM
        wave_sync();
        if (lane < 64 / S::P) {
            const uint32_t wi = ((uint32_t)(q - lane) >> S::LP) + (uint32_t)lane;
            if (wi < (uint32_t)up->state_words) gl(up->state)[wi] = spw(wi * 4u);
        }
    }
    return fl;
}

// Split units: after a colour class, the members publish the words they
// changed (already written through), meet at a device-scope barrier and read
// the class's words back, so that every member's LDS copy is complete before
// the next class.  The wait is bounded: a member that does not see all
// arrivals within kBarrierTicks of the 100 MHz real-time clock raises the
// unit's abort flag and the context's error bit, and every member stops.
constexpr uint64_t kBarrierTicks = 2000000000ull;

template <int RPAD>
__device__ bool vb_exchange(const VbUnit* __restrict__ up, const VbLds& L, int32_t lo, int32_t hi,
                            uint32_t target)
{
    using S = Sl<RPAD>;
    // One thread fences for the workgroup (as a grid barrier does): the
    // workgroup barrier orders every wavefront's write-through stores before
    // its device-scope release, and its device-scope acquire before the
    // read-back below.  (A fence in every wavefront wrote back and invalidated
    // the shared caches once per wavefront, slowing every workgroup on them.)
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* bar = up->bar;
        int32_t ab = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t start = wall_clock64();
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                ab = 1;
                break;
            }
            if (wall_clock64() - start > kBarrierTicks) {
                __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicOr(up->err, 4);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        L.flag[0] = ab;
    }
    __syncthreads();
    if (L.flag[0] != 0) return false;
    const SG_G uint32_t* gs = gl(up->state);
    const int32_t w0 = lo >> S::LP, w1 = hi > lo ? ((hi - 1) >> S::LP) : w0 - 1;
    for (int32_t w = w0 + (int32_t)threadIdx.x; w <= w1; w += (int32_t)blockDim.x) L.sp[w] = gs[w];
    __syncthreads();
    return true;
}

// Draws the Philox blocks of this wavefront's next chunks (up to B =
// max(1, 8 / nch) of them, following cursor pc) into its LDS batch: block
// m = i 8 nch + g nch + c is group g of chunk i for chain c (lanes past the
// last such block draw nothing that is used).
template <int B, class PC>
__device__ __forceinline__ void vb_fill(const VbLds& L, Cursor& pc, bool& pc_ok, PC cls, int32_t ncls,
                                        int32_t nsw, int W, int wave, int wl, int lane, int64_t t0,
                                        int32_t nch, uint64_t key)
{
    // the batch's chunk positions and sweeps stay in scalar registers; each
    // lane picks its chunk's pair by selection (no table in LDS)
    uint32_t base[B], tt[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        base[i] = 0u;
        tt[i] = 0u;
        if (pc_ok) {
            base[i] = (uint32_t)((((pc.lo >> 6) + pc.j) << 6));
            tt[i] = (uint32_t)(t0 + pc.s);
            pc_ok = cursor_next(pc, W, wave, ncls, cls, nsw);
        }
    }
    const uint32_t mul = (65536u + (uint32_t)nch - 1u) / (uint32_t)nch;
    {
        const uint32_t m = (uint32_t)lane;
        const uint32_t dq = (m * mul) >> 16;           // m / nch = 8 i + g
        const uint32_t c = m - dq * (uint32_t)nch;
        const uint32_t i = min(dq >> 3, (uint32_t)(B - 1)), g = dq & 7u;
        uint32_t bq = base[0], tq = tt[0];
#pragma unroll
        for (int k = 1; k < B; ++k) {
            bq = i == (uint32_t)k ? base[k] : bq;
            tq = i == (uint32_t)k ? tt[k] : tq;
        }
        const U4 A = philox_stream(key, (bq >> 3) + g, tq, kDomSweepHi, L.ri[2 * c], L.ri[2 * c + 1]);
        L.xch[wl * 64 + lane] = make_uint4(A.x, A.y, A.z, A.w);
    }
    wave_sync();
}

// One pass for the chunk at positions base.. of sweep t (the only chunk of a
// batch when 8 / nch < 2, i.e. for 5 to 8 chains): no cursor, no table.
// Lane m draws group g of chain c, m = g nch + c (lanes past 8 nch draw
// blocks nobody reads); `fr` holds (g, replica, instance), fixed per lane.
struct FillLane {
    uint32_t g, rep, inst;
};

__device__ __forceinline__ FillLane fill_lane(const VbLds& L, int lane, int32_t nch)
{
    const uint32_t mul = (65536u + (uint32_t)nch - 1u) / (uint32_t)nch;
    const uint32_t m = (uint32_t)lane;
    const uint32_t dq = (m * mul) >> 16;           // m / nch
    const uint32_t c = m - dq * (uint32_t)nch;
    return FillLane{dq & 7u, L.ri[2 * c], L.ri[2 * c + 1]};
}

__device__ __forceinline__ void vb_fill_one(const VbLds& L, const FillLane& fr, uint32_t base, uint32_t t, int wl,
                                            int lane, uint64_t key)
{
    const U4 A = philox_stream(key, (base >> 3) + fr.g, t, kDomSweepHi, fr.rep, fr.inst);
    L.xch[wl * 64 + lane] = make_uint4(A.x, A.y, A.z, A.w);
    wave_sync();
}

template <int RPAD>
__device__ void vb_snapshot(const VbUnit* __restrict__ up, const uint32_t* __restrict__ sp, int k)
{
    using S = Sl<RPAD>;
    const int32_t wn = up->words_n, nch = up->nch, sw = up->state_words;
    for (int32_t idx = threadIdx.x; idx < nch * wn; idx += blockDim.x) {
        const int32_t c = idx / wn;
        const int32_t w = idx - c * wn;
        uint32_t bits = 0;
#pragma unroll
        for (int b = 0; b < 32 / S::P; ++b) {
            const int32_t wi = w * (32 / S::P) + b;
            const uint32_t v = wi < sw ? sp[wi] : 0u;
            const uint32_t f = S::P == 32 ? v : (v >> (c * S::P)) & ((1u << (S::P & 31)) - 1u);
            bits |= f << (b * S::P);
        }
        gl(up->snap[c])[(int64_t)k * wn + w] = bits;
    }
}

// cnt[c] += the set bits of d in chain c's field (chains c < nch)
template <int RPAD>
__device__ __forceinline__ void win_count(uint32_t* cnt, uint32_t d, int32_t nch)
{
    using S = Sl<RPAD>;
#pragma unroll
    for (int c = 0; c < RPAD; ++c)
        if (c < nch)
            cnt[c] += (uint32_t)__popc(d & (S::P == 32 ? 0xffffffffu : (((1u << (S::P & 31)) - 1u) << (c * S::P))));
}

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Adds the four words of d ^ e, bit by bit, to the bit-sliced counters
// (ones, twos) of a thread, and the carries of weight 4 to the per-chain
// counts cnt4 (carry-save adders: sum = a ^ b ^ c, carry = majority): one
// masked popcount per chain for four words instead of four.
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) { return (a & b) | (c & (a | b)); }

template <int RPAD>
__device__ __forceinline__ void win_add4(uint32_t& ones, uint32_t& twos, uint32_t* cnt4, v4u a, v4u b, int32_t nch)
{
    const v4u d = a ^ b;
    const uint32_t h1 = maj3(ones, d.x, d.y);
    ones ^= d.x ^ d.y;
    const uint32_t h2 = maj3(ones, d.z, d.w);
    ones ^= d.z ^ d.w;
    const uint32_t f = maj3(twos, h1, h2);
    twos ^= h1 ^ h2;
    win_count<RPAD>(cnt4, f, nch);
}

// cnt = 4 cnt4 + the counts of the planes (ones, twos), per chain
template <int RPAD>
__device__ __forceinline__ void win_fold(uint32_t* cnt, uint32_t ones, uint32_t twos, int32_t nch)
{
    uint32_t c1[RPAD], c2[RPAD];
#pragma unroll
    for (int c = 0; c < RPAD; ++c) {
        c1[c] = 0u;
        c2[c] = 0u;
    }
    win_count<RPAD>(c1, ones, nch);
    win_count<RPAD>(c2, twos, nch);
#pragma unroll
    for (int c = 0; c < RPAD; ++c) cnt[c] = 4u * cnt[c] + c1[c] + 2u * c2[c];
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v);

// Windowed correlation (the paper's estimator: C(t_w + t, t_w) averaged over
// minor-third intervals of t_w + t, ratio 2^(1/4); Results and discussion,
// and the SI section on the extrapolation to large sizes and times), at the
// end of the sweep that ends at time tau <= t_max: for every stored waiting
// time t_w < tau and every chain, the overlap sum_i s_i(tau) s_i(t_w) =
// n - 2 popcount(s(tau) xor s(t_w)) over the chain's fields, added to the
// chain's sum for the interval of tau.  The spin words at the waiting times
// are stored in the same sliced packing as the LDS words (rows of `ws4`
// 16-byte groups; the words past state_words are zero on both sides), so the
// XOR of two words holds every chain's disagreements; a thread adds them up
// bit-sliced (carry-save adders) and counts the chains' fields of the carry
// planes.  The work is cut into blocks of 64 groups of one waiting time's
// row, taken in (waiting time, block) order as contiguous ranges by the
// wavefronts of all members (lane l counts group 64 b + l of block b): a
// lane keeps adding into the same carry-save planes until its wavefront
// reaches the next waiting time, so the planes are folded and the wavefront
// sums formed once or twice per sweep instead of once per waiting time.  The
// stored words are streamed from HBM with 16-byte loads, four blocks in
// flight per lane.  At the waiting times each thread stores the groups
// i = tid + member * threads (mod members * threads); no thread reads another's
// stores.
template <int RPAD>
__device__ __attribute__((noinline)) void vb_window(const VbUnit* __restrict__ up, uint32_t sp_off,
                                                   uint32_t acc_off, int64_t tau, int32_t k_store)
{
    constexpr int U = 4;
    typedef __attribute__((address_space(3))) v4u lds_u4;
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    const lds_u4* sp4 = (const lds_u4*)(size_t)sp_off;
    lds_u32* wacc = (lds_u32*)(size_t)acc_off;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    const int32_t nch = up->nch;
    const int32_t sw4 = (up->state_words + 3) >> 2;
    // waiting times before tau: t_w = 0, and t_w = 2^(k-1) < tau for k >= 1
    const int32_t kv = min(up->kw, tau >= 2 ? 2 + (63 - __clzll((unsigned long long)(tau - 1))) : 1);
    const int32_t stride = nthr * up->members;
    const int32_t w0 = tid + up->member * nthr;
    SG_G v4u* ws4 = (SG_G v4u*)gl(up->wsnap);
    for (int i = tid; i < kv * RPAD; i += nthr) wacc[i] = 0u;
    __syncthreads();
    const int32_t nbr = (sw4 + 63) >> 6;   // blocks per row
    const int32_t nb = kv * nbr;
    const int32_t W = nthr >> 6;
    const int32_t gw = __builtin_amdgcn_readfirstlane(up->member * W + (tid >> 6));
    const int32_t GW = up->members * W;
    const int32_t per = (nb + GW - 1) / GW;
    const int32_t b0 = min(gw * per, nb), b1 = min(b0 + per, nb);
    const v4u zero = {0u, 0u, 0u, 0u};
    uint32_t cnt[RPAD];
#pragma unroll
    for (int c = 0; c < RPAD; ++c) cnt[c] = 0u;
    uint32_t ones = 0u, twos = 0u;   // bit-sliced counters
    int32_t kc = b0 / nbr;           // the waiting time being counted
    auto flush = [&](int32_t k) {
        win_fold<RPAD>(cnt, ones, twos, nch);
#pragma unroll
        for (int c = 0; c < RPAD; ++c) {
            if (c < nch) {
                const uint32_t v = wave_sum(cnt[c]);
                if (lane == 0 && v) atomicAdd((uint32_t*)&wacc[k * RPAD + c], v);
            }
            cnt[c] = 0u;
        }
        ones = twos = 0u;
    };
    for (int32_t b = b0; b < b1; b += U) {
        v4u a[U], w[U];
        int32_t kb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t bb = b + u;
            const int32_t k = bb < b1 ? bb / nbr : kc;
            const int32_t g = (bb - k * nbr) * 64 + lane;
            const bool ok = bb < b1 && g < sw4;
            kb[u] = k;
            w[u] = ok ? ws4[(int64_t)k * sw4 + g] : zero;
            a[u] = ok ? sp4[g] : zero;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b + u < b1) {
                if (kb[u] != kc) {
                    flush(kc);
                    kc = kb[u];
                }
                win_add4<RPAD>(ones, twos, cnt, a[u], w[u], nch);
            }
        }
    }
    if (b1 > b0) flush(kc);
    if (k_store >= 0) {
        SG_G v4u* dst = ws4 + (int64_t)k_store * sw4;
        for (int32_t i = w0; i < sw4; i += stride) dst[i] = sp4[i];
    }
    __syncthreads();
    const int32_t bin = vb_window_bin((uint64_t)tau);
    for (int i = tid; i < kv * nch; i += nthr) {
        const int32_t k = i / nch, c = i - k * nch;
        const long long o = (up->member == 0 ? (long long)up->n : 0ll) - 2ll * (long long)wacc[k * RPAD + c];
        atomicAdd((unsigned long long*)(up->win[c] + (int64_t)k * up->n_bins + bin), (unsigned long long)o);
    }
}

template <int RPAD, bool SPLIT, bool CPL, class PR, class PE, class PC>
__device__ bool vb_loop(const VbUnit* __restrict__ up, const VbLds& L, PR row, PE ent, PC cls, int64_t t0,
                        int32_t nsw, int64_t t_max, int lane, int wave, int W);

// (each variant is a function of its own so that its registers are
// allocated for it alone)
template <int RPAD, bool RES, bool SPLIT, bool CPL>
__device__ __attribute__((noinline)) void vb_run(const VbUnit* __restrict__ up, uint32_t* smem_arr, uint32_t lds0,
                                                int64_t t0, int32_t nsw, int64_t t_max)
{
    // With fewer than 8 chain slots the dynamic LDS base is taken as a plain
    // offset: from the array itself this (called) function re-reads the base
    // from a per-kernel table at each use, and each re-read waits for all
    // outstanding LDS operations.  (With 8 slots the register the offset
    // would hold costs more than the re-reads: measured.)
    uint32_t* smem = RPAD == 8 ? smem_arr : (uint32_t*)(__attribute__((address_space(3))) uint32_t*)(size_t)lds0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // wave index made explicitly wave-uniform: the chunk cursor then lives in
    // scalar registers and class bounds come from scalar loads; a member of a
    // split unit numbers its wavefronts after those of the members before it
    const int Wl = nthr >> 6;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane((tid >> 6) + (SPLIT ? up->member * Wl : 0));
    const int W = SPLIT ? up->members * Wl : Wl;
    const int32_t sw = up->state_words, nch = up->nch, ncls = up->ncls;
    const VbLds L = vb_carve(smem, 0u, sw, nthr, nch, CPL);

    const SG_G uint32_t* gstate = gl(up->state);
    for (int32_t w = tid; w < sw; w += nthr) {
        const uint32_t v = gstate[w];
        L.sp[w] = v;
        if (CPL) L.cp[w] = ~v;
    }
    if (tid < ((sw + 3) & ~3) - sw) L.sp[sw + tid] = 0u;   // pad to 16 bytes (read by vb_window)
    // chain c's threshold high halves: word c kTab + j holds the entry for
    // x = 64 - j (0x10000 for x <= 0: always accepted)
    for (int i = tid; i < kVbMaxChains * kTab; i += nthr) {
        const int c = i / kTab, x = 64 - (i - c * kTab);
        L.thr[i] = x <= 0 ? 0x10000u : x < kVbXMax ? gl(&up->thr_hi[c][0])[x] : 0u;
    }
    // the same for |x| <= 15 in the compact tables: word c kThc + j holds the
    // entry for x = 15 - j
    for (int i = tid; i < kVbMaxChains * kThc; i += nthr) {
        const int c = i / kThc, x = 15 - (i - c * kThc);
        L.thc[i] = x <= 0 ? 0x10000u : gl(&up->thr_hi[c][0])[x];
    }
    for (int i = tid; i < 256; i += nthr) {
        uint32_t v = 0;
        for (int c = 0; c < 8; ++c) v |= (uint32_t)((i >> c) & 1) << (4 * c);
        L.spr[i] = v;
    }
    if (tid < kVbMaxChains) {
        L.accs[tid] = 0;
        L.ri[2 * tid] = up->rep[tid];
        L.ri[2 * tid + 1] = up->inst[tid];
    }
    for (int32_t k = tid; k <= ncls; k += nthr) L.cls[k] = gl(up->cls)[k];
    const int32_t* cls = L.cls;
    __syncthreads();
    if (RES) {
        const int32_t n = up->n;
        const SG_G int32_t* grow = gl(up->row);
        const SG_G uint32_t* gent = gl(up->ent);
        for (int32_t i = tid; i <= n; i += nthr) L.area[i] = grow[i];
        uint32_t* re = (uint32_t*)(L.area + n + 1);
        for (int32_t i = tid; i < up->m2 + kVbEntPad; i += nthr) re[i] = i < up->m2 ? gent[i] : 0u;
        __syncthreads();
        vb_loop<RPAD, false, CPL>(up, L, (const int32_t*)L.area, (const uint32_t*)(L.area + n + 1), cls, t0, nsw,
                                  t_max, lane, wave, W);
    } else {
        vb_loop<RPAD, SPLIT, CPL>(up, L, gl(up->row), gl(CPL ? up->entc : up->ent), cls, t0, nsw, t_max, lane,
                                  wave, W);
    }
    // (split units keep `state` current by writing through)
    if (!SPLIT)
        for (int32_t w = tid; w < sw; w += nthr) gl(up->state)[w] = L.sp[w];
    __syncthreads();
    if (tid < nch) atomicAdd(up->accepted[tid], L.accs[tid]);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    return v;
}

// Accepted flips of one wavefront, counted per lane in the flips' own
// spin-word fields (n += flips of each chunk).  A P-bit field holds the flips
// of at most 2^P - 1 chunks: with 8 chain slots (4-bit fields) the counts move
// to byte fields (e: even chains, o: odd chains, chain c at byte c / 2) every
// 15 chunks; byte and 16-bit fields are summed over the wavefront into the
// unit's LDS totals every 255 (65535) chunks, and every field at the end of
// each sweep.
template <int RPAD>
struct VbAcc {
    uint32_t n = 0, e = 0, o = 0;   // per lane
    int32_t cn = 0, cb = 0;         // wave-uniform chunk counts since the last fold / flush
};

template <int RPAD>
__device__ __forceinline__ void acc_fold(VbAcc<RPAD>& a)
{
    if (RPAD == 8) {
        a.e += a.n & 0x0F0F0F0Fu;
        a.o += (a.n >> 4) & 0x0F0F0F0Fu;
        a.n = 0u;
    }
    a.cn = 0;
}

template <int RPAD>
__device__ __forceinline__ void acc_flush(VbAcc<RPAD>& a, const VbLds& L, int32_t nch)
{
    const int lane = threadIdx.x & 63;
    // chain sums in 16-bit halves (at most 64 x 255 each) or whole words
    auto put = [&](int c, uint32_t v) {
        if (lane == 0 && c < nch && v != 0u) atomicAdd(&L.accs[c], (unsigned long long)v);
    };
    if (RPAD == 8) {
        const uint32_t e0 = wave_sum(a.e & 0x00FF00FFu), e1 = wave_sum((a.e >> 8) & 0x00FF00FFu);
        const uint32_t o0 = wave_sum(a.o & 0x00FF00FFu), o1 = wave_sum((a.o >> 8) & 0x00FF00FFu);
        put(0, e0 & 0xFFFFu);
        put(4, e0 >> 16);
        put(2, e1 & 0xFFFFu);
        put(6, e1 >> 16);
        put(1, o0 & 0xFFFFu);
        put(5, o0 >> 16);
        put(3, o1 & 0xFFFFu);
        put(7, o1 >> 16);
        a.e = 0u;
        a.o = 0u;
    } else if (RPAD == 4) {
        const uint32_t s0 = wave_sum(a.n & 0x00FF00FFu), s1 = wave_sum((a.n >> 8) & 0x00FF00FFu);
        put(0, s0 & 0xFFFFu);
        put(2, s0 >> 16);
        put(1, s1 & 0xFFFFu);
        put(3, s1 >> 16);
        a.n = 0u;
    } else if (RPAD == 2) {
        put(0, wave_sum(a.n & 0xFFFFu));
        put(1, wave_sum(a.n >> 16));
        a.n = 0u;
    } else {
        put(0, wave_sum(a.n));
        a.n = 0u;
    }
    a.cn = 0;
    a.cb = 0;
}

template <int RPAD>
__device__ __forceinline__ void acc_add(VbAcc<RPAD>& a, uint32_t fl, const VbLds& L, int32_t nch)
{
    a.n += fl;
    ++a.cn;
    if (RPAD == 8) {
        if (a.cn == 15) {
            acc_fold(a);
            if (++a.cb == 17) acc_flush(a, L, nch);
        }
    } else if (RPAD == 4) {
        if (a.cn == 255) acc_flush(a, L, nch);
    } else if (RPAD == 2) {
        if (a.cn == 65535) acc_flush(a, L, nch);
    }
}

// The sweep loop of one unit (or of one member of a split unit: `wave` and
// `W` then count the wavefronts of all members), for adjacency pointers in
// HBM or in LDS.  False if a split unit's barrier aborted.
template <int RPAD, bool SPLIT, bool CPL, class PR, class PE, class PC>
__device__ bool vb_loop(const VbUnit* __restrict__ up, const VbLds& L, PR row, PE ent, PC cls, int64_t t0,
                        int32_t nsw, int64_t t_max, int lane, int wave, int W)
{
    const int tid = threadIdx.x;
    // The unit's scalars arrive through a pointer argument, which the
    // compiler cannot take as uniform: made explicitly wave-uniform, the
    // per-chain tests and the sweep loop branch on scalar registers instead
    // of masking lanes
    const int32_t nch = __builtin_amdgcn_readfirstlane(up->nch), ncls = __builtin_amdgcn_readfirstlane(up->ncls);
    nsw = __builtin_amdgcn_readfirstlane(nsw);
    W = __builtin_amdgcn_readfirstlane(W);
    t0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)((uint64_t)t0 >> 32)) << 32) |
                   (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)t0));
    // the Philox key is the same for every lane: kept in scalar registers,
    // so that the per-round keys cost no vector registers
    const uint64_t key = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(up->key >> 32)) << 32) |
                         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)up->key);
    const int wl = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront inside the workgroup
    // Philox batches: cursor of the next chunk to draw for, chunks left in
    // the current batch and the batch position of the next chunk
    const int32_t B = vb_batch_chunks(nch);
    // (with 8 chain slots a batch is one chunk: its blocks are drawn for the
    // chunk itself, and the cursor is not needed)
    Cursor pc = cursor_start(W, wave, cls);
    bool pc_ok = RPAD != 8 && nsw > 0 && cursor_next(pc, W, wave, ncls, cls, nsw);
    int32_t left = 0, bi = 0;
    const uint32_t* xg = (const uint32_t*)(L.xch + wl * 64);
    const uint32_t lane_off = (uint32_t)(lane >> 3) * (uint32_t)nch * 4u + (((uint32_t)lane & 7u) >> 1);

    // pipeline: the chunk being updated and the next one (rows + entries)
    // take turns in E0 and E1, so that no stage is copied; R holds the rows
    // of the chunk after next
    Stage E0, E1, R;
    E1.q = 0;
    E1.r0 = 0;
    E1.r1 = 0;
    R.q = 0;
    R.r0 = 0;
    R.r1 = 0;
    Cursor cR = cursor_start(W, wave, cls);
    bool haveR = nsw > 0 && cursor_next(cR, W, wave, ncls, cls, nsw);
    if (haveR) {
        load_rows(row, cls, cR, lane, E0);
        load_ents(ent, E0);
        haveR = cursor_next(cR, W, wave, ncls, cls, nsw);
        if (haveR) load_rows(row, cls, cR, lane, R);
    }
    __syncthreads();
    if (nsw <= 0) return true;

    const FillLane fr = fill_lane(L, lane, nch);
    VbAcc<RPAD> acc;

    // one chunk (j of colour class [lo, hi) in sweep t): C holds it, N
    // receives the next one.  The stage moves on unconditionally (past the
    // last chunk of the launch it re-reads valid entries that are not used),
    // so that the loads issue without branches
    auto step = [&](const Stage& C, Stage& N, int32_t lo, int32_t hi, int32_t j, uint32_t t)
                    __attribute__((always_inline)) {
        N.q = R.q;
        N.r0 = R.r0;
        N.r1 = R.r1;
        load_ents(ent, N);
        if (haveR) {
            haveR = cursor_next(cR, W, wave, ncls, cls, nsw);
            if (haveR) load_rows(row, cls, cR, lane, R);
        }
        if (RPAD == 8) {
            vb_fill_one(L, fr, (uint32_t)(((lo >> 6) + j) << 6), t, wl, lane, key);
            left = 1;
            bi = 0;
        } else if (left == 0) {
            vb_fill<(RPAD < 8 ? 8 / RPAD : 1)>(L, pc, pc_ok, cls, ncls, nsw, W, wave, wl, lane, t0, nch, key);
            left = B;
            bi = 0;
        }
        const uint32_t fl = vb_chunk<RPAD, SPLIT, CPL>(up, L, ent, C, lo, hi, t, nch, key,
                                                  xg + (uint32_t)bi * 32u * (uint32_t)nch + lane_off);
        acc_add(acc, fl, L, nch);
        --left;
        ++bi;
    };

    for (int32_t s = 0; s < nsw; ++s) {
        const uint32_t t = (uint32_t)(t0 + s);
        for (int32_t k = 0; k < ncls; ++k) {
            const int32_t lo = cls_at(cls, k), hi = cls_at(cls, k + 1);
            const int32_t nck = n_chunks(cls, k);
            // chunks in pairs: E0 and E1 take turns; after an odd count the
            // next chunk is moved back to E0 (once per class)
            for (int32_t j = wave; j < nck; j += W) {
                step(E0, E1, lo, hi, j, t);
                E0 = E1;
            }
            if (SPLIT) {
                if (!vb_exchange<RPAD>(up, L, lo, hi, (uint32_t)up->members * (uint32_t)(s * ncls + k + 1)))
                    return false;
            } else {
                __syncthreads();
            }
        }
        acc_fold(acc);
        acc_flush(acc, L, nch);
        const int64_t tn = t0 + s + 1;
        const bool grid = tn <= t_max && (tn & (tn - 1)) == 0;
        const int32_t kn = grid ? 1 + (63 - __clzll((unsigned long long)tn)) : -1;
        if (grid) {
            if (!SPLIT || up->member == 0) vb_snapshot<RPAD>(up, L.sp, kn);
            __syncthreads();
        }
        if (up->kw > 0 && tn <= t_max) {
            vb_window<RPAD>(up, L.sp_lds, L.sp_lds + (uint32_t)((const char*)L.wacc - (const char*)L.sp), tn,
                            kn < up->kw ? kn : -1);
            __syncthreads();
        }
    }
    return true;
}

// t0p: device-resident number of sweeps done before this launch (read once;
// the counter is advanced by vb_advance_kernel after every launch group), so
// a captured graph of the sweep loop can be replayed unchanged.
__global__ void __launch_bounds__(1024) vb_sweep_kernel(const VbUnit* __restrict__ units,
                                                        const int64_t* __restrict__ t0p,
                                                        int32_t nsw, int64_t t_max)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
    uint32_t lds0 = (uint32_t)(size_t)(__attribute__((address_space(3))) uint32_t*)smem;
    const VbUnit* up = (const VbUnit*)(gl(units) + blockIdx.x);
    // The sweep functions read the spin words at LDS offset 0, where the
    // dynamic array starts in a kernel that declares no static LDS (a
    // constant test: a build where that does not hold reports an error)
    if (lds0 != 0u) {
        if (threadIdx.x == 0) atomicOr(up->err, 8);
        return;
    }
    asm volatile("" : "+s"(lds0));   // an opaque value: the callee cannot re-derive it from the array
    const int64_t t0 = *gl(t0p);
    if (up->resident) {
        switch (up->rpad) {
            case 1: vb_run<1, true, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 2: vb_run<2, true, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 4: vb_run<4, true, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            default: vb_run<8, true, false, false>(up, smem, lds0, t0, nsw, t_max); break;
        }
    } else if (up->members > 1) {
        switch (up->rpad) {
            case 1: vb_run<1, false, true, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 2: vb_run<2, false, true, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 4: vb_run<4, false, true, false>(up, smem, lds0, t0, nsw, t_max); break;
            default: vb_run<8, false, true, false>(up, smem, lds0, t0, nsw, t_max); break;
        }
    } else if (up->cpl) {
        switch (up->rpad) {
            case 1: vb_run<1, false, false, true>(up, smem, lds0, t0, nsw, t_max); break;
            case 2: vb_run<2, false, false, true>(up, smem, lds0, t0, nsw, t_max); break;
            case 4: vb_run<4, false, false, true>(up, smem, lds0, t0, nsw, t_max); break;
            default: vb_run<8, false, false, true>(up, smem, lds0, t0, nsw, t_max); break;
        }
    } else {
        switch (up->rpad) {
            case 1: vb_run<1, false, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 2: vb_run<2, false, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            case 4: vb_run<4, false, false, false>(up, smem, lds0, t0, nsw, t_max); break;
            default: vb_run<8, false, false, false>(up, smem, lds0, t0, nsw, t_max); break;
        }
    }
}

__global__ void vb_advance_kernel(int64_t* t, int32_t nsw, uint32_t* bars, int n_bar)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += nsw;
    for (int i = threadIdx.x; i < n_bar; i += blockDim.x) bars[i] = 0u;
}

// Initial configurations and the t = 0 snapshot.
__global__ void __launch_bounds__(1024) vb_init_kernel(const VbUnit* __restrict__ units)
{
    const VbUnit* up = units + blockIdx.x;
    if (up->member != 0) return;   // members of a split unit share its state
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
    const VbLayout lay(rpad);
    for (int32_t w = threadIdx.x; w < up->state_words; w += blockDim.x) {
        const int32_t p0 = w * lay.P;   // first position of the word
        uint32_t word = 0;
        for (int32_t c = 0; c < nch; ++c) {
            const uint32_t v = up->snap[c][p0 >> 5];
            const uint32_t f = lay.P == 32 ? v : (v >> (p0 & 31)) & ((1u << lay.P) - 1u);
            word |= f << (c * lay.P);
        }
        up->state[w] = word;
        if (up->kw > 0) up->wsnap[w] = word;   // the waiting time t_w = 0
    }
}

}  // namespace

size_t vb_resident_bytes(int32_t n, int32_t m2)
{
    return ((size_t)(n + 1 + m2 + kVbEntPad) * 4 + 15) & ~(size_t)15;
}

size_t vb_lds_bytes(int32_t n, int32_t rpad, int32_t nch, int threads, bool cpl)
{
    const size_t sw = (size_t)VbLayout(rpad).words(n);
    const size_t waves = (size_t)threads / 64;
    return kSpOff + ((sw + 3) & ~(size_t)3) * 4 * (cpl ? 2 : 1) + (size_t)kVbMaxChains * kTab * 4 + kVbMaxChains * 8 + 16 +
           (kMaxCls + 4) * 4 + kVbMaxChains * 8 + (size_t)kMaxGrid * kVbMaxChains * 4 + waves * 64 * 16;
}

void vb_cpl_entries(const uint32_t* ent, size_t m, size_t pad, int32_t rpad, int32_t n, uint32_t* out)
{
    const VbLayout lay(rpad);
    const uint32_t swp = ((uint32_t)lay.words(n) + 3u) & ~3u;
    for (size_t e = 0; e < m + pad; ++e) {
        const uint32_t en = e < m ? ent[e] : 0u;
        const uint32_t pos = en & 0x7fffffffu;
        const uint32_t addr = kSpOff + 4u * (pos / (uint32_t)lay.P) + ((en >> 31) != 0u ? 4u * swp : 0u);
        out[e] = (addr << 5) | (pos % (uint32_t)lay.P);
    }
}

hipError_t vb_init(const VbUnit* units, int n_units, int threads, size_t, hipStream_t s)
{
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(vb_init_kernel, dim3(n_units), dim3(threads), 0, s, units);
    return hipGetLastError();
}

hipError_t vb_prepare()
{
    // set once (thread-safe initialisation of a local static)
    static const hipError_t attr = hipFuncSetAttribute((const void*)vb_sweep_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
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

hipError_t vb_advance(int64_t* t, int32_t n_sweeps, uint32_t* bars, int n_bar, hipStream_t s)
{
    hipLaunchKernelGGL(vb_advance_kernel, dim3(1), dim3(256), 0, s, t, n_sweeps, bars, n_bar);
    return hipGetLastError();
}

}  // namespace sg
