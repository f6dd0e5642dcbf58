// Per-chain VB work units: the device-side descriptor and spin layout of the
// VB sweep kernel (sg_vb.hip), with the helpers and constants it depends on.
// Included by sg_internal.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

// Device pointers stored in descriptors are generic; re-qualifying them as
// global memory lets the compiler emit global/scalar loads, which wait only on
// their own counters, instead of flat loads, which wait on every outstanding
// load and LDS access.
#define SG_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ SG_G T* gl(T* p)
{
    return (SG_G T*)p;
}

constexpr int kVbMaxChains = 8;    // chains per VB work unit
constexpr int kVbEntPad = 8;       // zero entries after the adjacency (loads past a row stay in bounds)
constexpr int kVbXMax = 64;        // threshold table length (max degree 63)
constexpr int kMaxGrid = 32;       // grid times {0} U {2^k <= t_max}, t_max < 2^31

// Packed spins of a VB work unit with `rpad` (1, 2, 4 or 8) chain slots,
// "sliced" so that one 32-bit word holds P = 32 / rpad consecutive positions
// of all rpad chains, chain c in bits [c P, c P + P) and position p at bit
// c P + (p mod P): a word shifted right by (p mod P) has the bit of position p
// of every chain at the bottom of that chain's field, so counting a bond for
// all chains is a shift, an XOR and a mask.  Position p is in word p / P.
// Bit value 1 = spin -1.
struct VbLayout {
    int32_t P;
    __host__ __device__ explicit VbLayout(int32_t rpad) : P(32 / rpad) {}
    __host__ __device__ int64_t words(int64_t n) const { return (n + P - 1) / P; }
    __host__ __device__ int64_t word(int64_t p, int32_t) const { return p / P; }
    __host__ __device__ int32_t bit(int64_t p, int32_t c) const { return c * P + (int32_t)(p % P); }
};

// One VB work unit = one workgroup: a graph in sweep (colour) order and up to
// eight chains that share it.  The chains' spins live in LDS during a launch,
// in the VbLayout packing (the same words as `state` between launches).
struct VbUnit {
    const int32_t* row;        // [n+1] adjacency row starts, sweep order
    const uint32_t* ent;       // [2m + kVbEntPad] neighbour position | (J < 0) << 31, then zeros
    const uint32_t* entc;      // (cpl) the same entries in the form of vb_cpl_entries, read by the sweep
    const int32_t* cls;        // [ncls+1] first position of each colour class
    int32_t resident;          // 1: whole adjacency kept in LDS for the launch
    int32_t cpl;               // 1: a complemented copy of the spin words is kept in LDS
    int32_t m2;                // 2m entries
    uint64_t key;              // Philox key (seed) shared by every chain of the unit
    uint32_t* state;           // [state_words] packed spins between launches
    uint32_t* snap[kVbMaxChains];       // per chain: [K][words_n] position-order bits
    unsigned long long* accepted[kVbMaxChains];
    uint64_t seed[kVbMaxChains];
    uint32_t inst[kVbMaxChains];
    uint32_t rep[kVbMaxChains];
    uint32_t thr_hi[kVbMaxChains][kVbXMax];   // threshold >> 16 (0..65536)
    uint32_t thr_lo[kVbMaxChains][kVbXMax];   // threshold & 0xffff
    int32_t n;
    int32_t ncls;
    int32_t nch;
    int32_t rpad;              // bits per position: 1, 2, 4 or 8 (>= nch)
    int32_t state_words;       // VbLayout(rpad).words(n)
    int32_t words_n;           // ceil(n / 32)
    int32_t init_mode[kVbMaxChains];   // SG_START_* for the init kernel
    const uint32_t* given[kVbMaxChains];   // position-order bits when GIVEN
    // A unit split over `members` workgroups (one descriptor each, member =
    // 0 .. members - 1): every member keeps all spins in LDS, updates its
    // share of each colour class's chunks, writes the spin words it changed
    // through to `state`, meets the others at a device-scope barrier (bar[0]
    // counts arrivals within the launch, bar[1] is an abort flag; both are
    // zeroed before every launch) and reads the class's words back.
    int32_t members;
    int32_t member;
    uint32_t* bar;
    int* err;                  // bit 2: a barrier wait timed out; bit 3: dynamic LDS not at offset 0
    // Windowed correlation (kw > 0): the spin words at the first kw grid
    // times (the waiting times) in the VbLayout packing, and per chain the
    // sums of the overlap with each of them over the minor-third interval of
    // the time each sweep ends at (see vb_window_bin).
    uint32_t* wsnap;           // [kw][state_words]
    long long* win[kVbMaxChains];   // per chain: [kw][n_bins]
    int32_t kw;
    int32_t n_bins;
};

// Minor-third interval of time tau >= 1: m = floor(4 log2 tau) =
// floor(log2 tau^4), from the exact 128-bit fourth power (tau < 2^32).
__host__ __device__ __forceinline__ int32_t vb_window_bin(uint64_t tau)
{
    const uint64_t a = tau * tau;   // < 2^64
#if defined(__HIP_DEVICE_COMPILE__)
    const uint64_t hi = __umul64hi(a, a);
#else
    const uint64_t hi = (uint64_t)(((unsigned __int128)a * a) >> 64);
#endif
    const uint64_t lo = a * a;
    return hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
}

}  // namespace sg
