// Internal device-side descriptors and kernel launchers shared by the host
// runtime (sg_host.cpp) and the HIP kernels (sg_vb.hip, sg_vbm.hip,
// sg_sk.hip, sg_skg.hip, sg_measure.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_vb_unit.h"

namespace sg {

constexpr int kSkTile = 64;        // SK decision block (one wavefront)
constexpr int kSkThrLds = 1024;    // SK threshold entries cached in LDS
constexpr int kWindowBinsMax = 128;  // minor-third intervals of times below 2^32
constexpr size_t kMeasureScratchElems = (size_t)1 << 20;   // int64 staging of sg_measure_noalloc (8 MiB)

// A multispin VB work unit (sg_vbm.hip): one graph and up to 64 chains on it,
// each with its own couplings, temperature and random numbers, packed as the
// bits of one 64-bit word per vertex (the paper's multispin coding: Methods;
// SI bipartite-graph section).  The spins stay in LDS during a launch.
constexpr int kVbmChains = 64;
constexpr int kVbmMaxN = 16384;    // n 64-bit words must fit in LDS
struct VbmUnit {
    const int32_t* row;        // [n+1] adjacency row starts, sweep order
    const uint32_t* ent;       // [2m + kVbEntPad] neighbour position in bits 0..30 (bit 31 ignored)
    const uint64_t* jw;        // [2m + kVbEntPad] bit c: chain c's coupling on the entry is -1
    const int32_t* cls;        // [ncls+1] first position of each colour class
    uint64_t* state;           // [n] spin words between launches (bit c: chain c's spin is -1)
    const uint32_t* thr;       // [2][64][kVbXMax]: chain c's thr[x] >> 16 (0..65536), then thr[x] & 0xffff
                               // (entry x = 0 unused)
    uint64_t key;              // Philox key (seed) shared by every chain of the unit
    uint32_t* snap[kVbmChains];
    unsigned long long* accepted[kVbmChains];
    uint32_t inst[kVbmChains];
    uint32_t rep[kVbmChains];
    int32_t n;
    int32_t ncls;
    int32_t nch;
    int32_t words_n;           // ceil(n / 32)
    int32_t init_mode[kVbmChains];
    const uint32_t* given[kVbmChains];
    uint64_t seed;
};

// One SK chain (a replica of an instance).
struct SkChain {
    const int8_t* J;           // [n][n]
    const uint32_t* Jb;        // [n][words_n] bit-packed rows, bit 1 = coupling -1
    const uint32_t* Jt;        // [n_blocks][64][sk_tile_words()] the decider's tiles, contiguous
    uint32_t* state;           // [words_n] position-order bits (1 = spin -1)
    int32_t* H;                // [n] local fields between launches
    uint32_t* snap;            // [K][words_n]
    unsigned long long* accepted;
    const uint64_t* thr;       // [thr_len] thresholds (uint64), x < thr_len
    uint64_t seed;
    uint32_t inst;
    uint32_t rep;
    int32_t n;
    int32_t words_n;
    int32_t thr_len;           // thr[x] == 0 for x >= thr_len
    int32_t init_mode;
    const uint32_t* given;     // position-order bits when GIVEN
    int32_t sample;            // index of the instance in the context
    float xslope;              // 2 beta / sqrt(N): thr[x] ~ 2^32 exp(-xslope x)
    // real couplings (sg_skg.hip): J, J_b, J_t, H, thr unused
    const float* Jf;           // [n][n]
    double* Hd;                // [n] local fields between launches
    double beta;               // 1 / T
};

// SK instance (sample) for the exact field recompute: all its chains.
struct SkSample {
    const int8_t* J;
    int32_t n;
    int32_t nch;
    int32_t chain0;            // index of its first chain in the chain array
    int32_t pad_;
    const float* Jf;           // real couplings, or null
};

struct MeasureChain {
    const uint32_t* snap;      // [K][words_n]
    int32_t words_n;
    int32_t n;
};

// ---- launchers (return hipError_t) ----
hipError_t vb_init(const VbUnit* units, int n_units, int threads, size_t lds_bytes, hipStream_t s);
// One-time kernel attributes (large dynamic LDS); call before launching or
// capturing VB sweeps.
hipError_t vb_prepare();
// t0p: device counter of sweeps done, read by the kernel; vb_advance adds
// n_sweeps to it on the stream (after every launch group of a chunk).
hipError_t vb_sweep(const VbUnit* units, int n_units, int threads, size_t lds_bytes, const int64_t* t0p,
                    int32_t n_sweeps, int64_t t_max, hipStream_t s);
// also zeroes the n_bar barrier words of split units for the next launch
hipError_t vb_advance(int64_t* t, int32_t n_sweeps, uint32_t* bars, int n_bar, hipStream_t s);
// LDS a unit needs for a launch with `threads` lanes per workgroup, and the
// extra LDS that keeps its whole adjacency resident.
size_t vb_lds_bytes(int32_t n, int32_t rpad, int32_t nch, int threads, bool cpl = false);
// Adjacency entries (position | (J < 0) << 31) in the form a unit with a
// complemented copy of its spin words reads: the LDS byte address of the
// neighbour's word, of its complement when J < 0, above 5 bits of in-word
// shift; `pad` entries of position 0 follow the m entries.
void vb_cpl_entries(const uint32_t* ent, size_t m, size_t pad, int32_t rpad, int32_t n, uint32_t* out);
size_t vb_resident_bytes(int32_t n, int32_t m2);

// Multispin units (sg_vbm.hip).
size_t vbm_lds_bytes(int32_t n, int threads);
hipError_t vbm_init(const VbmUnit* units, int n_units, hipStream_t s);
hipError_t vbm_prepare();
hipError_t vbm_sweep(const VbmUnit* units, int n_units, int threads, size_t lds_bytes, const int64_t* t0p,
                     int32_t n_sweeps, int64_t t_max, hipStream_t s);
// bond sums of the snapshots k_first .. k_done - 1 of every chain of every
// unit: out[chain][k], chain ids [unit][64]
hipError_t vbm_bond(const VbmUnit* units, int n_units, int k_first, int k_done, long long* out,
                    const int32_t* chain_ids, int k_cap, hipStream_t s);

// err_flag bit 0: recompute mismatch; bit 1: the sweep pipeline stalled.
hipError_t sk_init(const SkChain* chains, int n_chains, int threads, hipStream_t s);
hipError_t sk_recompute(const SkSample* samples, int n_samples, const SkChain* chains,
                        int max_n, int check, int* err_flag, hipStream_t s);
hipError_t sk_bond(const SkSample* samples, int n_samples, const SkChain* chains, int max_n,
                   int max_nch, int k_done, int k_cap, long long* out, hipStream_t s);
hipError_t sk_sweep(const SkChain* chains, int n_chains, int threads, size_t lds_bytes, int64_t t0,
                    int32_t n_sweeps, int64_t t_max, int* err_flag, hipStream_t s);
size_t sk_lds_bytes(int32_t n);
int sk_threads();
// Decider tiles: words per row of a 64-spin block (its own columns, then those
// of the sk_window() blocks before it, two words each).
int sk_tile_words();
int sk_window();

// SK with real couplings (sg_skg.hip): sweeps, direct field recomputation
// (with `check`, error bit 0 when a field drifted by more than 1e-9 (1 + |h|))
// and bond sums of the snapshots (partials `part` of max_samples x
// ceil(max_n / 16) x max_nch x k_cap doubles; out[chain][k]).
size_t skg_lds_bytes(int32_t n);
hipError_t skg_sweep(const SkChain* chains, int n_chains, size_t lds_bytes, int64_t t0, int32_t n_sweeps,
                     int64_t t_max, hipStream_t s);
hipError_t skg_recompute(const SkSample* samples, int n_samples, const SkChain* chains, int max_n, int check,
                         int* err_flag, hipStream_t s);
hipError_t skg_bond(const SkSample* samples, int n_samples, const SkChain* chains, int max_n, int max_nch,
                    int k_done, int k_cap, double* part, double* out, hipStream_t s);

// bond sums of the snapshots k_first .. k_done - 1 of every chain:
// bond_out[chain][k] (the other entries are left as they are)
hipError_t vb_bond(const VbUnit* units, int n_units, int k_first, int k_done, long long* bond_out,
                   const int32_t* unit_chain_ids, int k_cap, int threads, size_t lds_bytes,
                   hipStream_t s);
hipError_t measure_overlap(const MeasureChain* chains, const int32_t* pairs, int n_pairs,
                           int k_done, int k_cap, long long* out, hipStream_t s);
hipError_t measure_gram(const MeasureChain* chains, int n_chains, int k_done, int k_cap,
                        int max_words, long long* out, hipStream_t s);
hipError_t zero_i64(long long* p, size_t n, hipStream_t s);
// Device address of the fixed staging array (kMeasureScratchElems int64) on
// the current device; looked up once per device.
hipError_t measure_scratch(long long** ptr);

}  // namespace sg
