// eis_internal.h -- declarations shared by the host runtime (eis_api.cpp) and
// the kernel launchers (eis_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eis {

typedef uint32_t u32;
typedef uint64_t u64;

// Candidates handled by one pass of the pipeline.  A multiple of 32, so that
// every pass starts on a bitmap word, and small enough that every index fits
// 31 bits.
constexpr u64 kPassCandidates = u64(1) << 24;

// Candidates per sieve workgroup (one LDS bitmap of kSegWords words).
constexpr u32 kSegCandidates = 32768;
constexpr u32 kSegWords = kSegCandidates / 32;

// Device-side prime table entry for the squarefree sieve: an odd prime p,
// its square m = p^2, and 8^{-1} mod m.
struct PrimeEntry {
    u64 m;
    u64 inv8;
};

// Per-pass device counters (one cache line each to avoid false sharing).
struct PassCounters {
    u32 list_len;      // number of squarefree candidates written by the sieve
    u32 pad0[15];
    u32 work_next;     // walk queue head
    u32 pad1[15];
    u32 err_count;     // walks that exceeded the step budget
    u32 pad2[15];
    unsigned long long baby_steps;
    unsigned long long refills;
    unsigned long long giant_steps;
    u64 pad3[5];
};

struct WalkParams {
    u64 d0;                       // first candidate of the pass
    const u32 *list;              // compacted squarefree candidate indices
    PassCounters *ctr;            // list_len, queue head, error and step counters
    u32 *eis_words;               // output bitmap, bit i <-> d0 + 8 i
    u32 max_steps;                // per-d step budget
};

// ---- infrastructure method ------------------------------------------------
// Per-d record written by the window walk for the giant-step walk.
struct WindowState {
    u32 q_bits;   // fp32 bit pattern of Q of mu_1 (the giant step)
    u32 p_bits;   // fp32 bit pattern of P of mu_1, OR its residue (2 bits)
    u32 count;    // dictionary entries written
    u32 idx;      // candidate index of d in the pass
};

struct InfraParams {
    u64 d0;                     // first candidate of the pass
    const u32 *list;            // compacted squarefree candidate indices of the pass
    u32 k0, k1;                 // batch: list positions [k0, k1)
    PassCounters *ctr;          // pass counters: err_count and step statistics
    u32 *win_next;              // window-walk queue head (per batch)
    u32 *giant_list;            // batch-relative positions that need giant steps
    u32 *giant_len;             // their number
    u32 *giant_next;            // giant-walk queue head
    u32 *fb_list;               // candidate indices handed to the plain walk
    PassCounters *fb_ctr;       // fb_ctr->list_len counts fb_list
    WindowState *state;         // per batch position
    unsigned long long *lists;  // window lists, tile-interleaved: entry e of batch
                                // position k at ((k / 64) * emax + e) * 64 + k % 64
    unsigned long long *tables; // hash tables, tsize slots per batch position
    u32 emax;                   // list capacity per d
    u32 tsize;                  // table slots per d (power of two)
    float window_scale;         // mu_1 is the distinguished ideal number
                                // round(window_scale * d^(1/4) / 16)
    u32 max_steps;              // per-d budget of reduction steps (window)
    u32 max_giants;             // per-d budget of giant steps
    u32 *eis_words;             // output bitmap of the pass
};

// Launchers (all enqueue on `stream`, never synchronise).
hipError_t launch_zero_u32(u32 *p, u64 nwords, hipStream_t stream);
hipError_t launch_prime_offsets(const PrimeEntry *primes, u32 nprimes, u64 d0, u64 *roff,
                                hipStream_t stream);
hipError_t launch_sieve(const PrimeEntry *primes, const u64 *roff, u32 nprimes, u32 nsmall,
                        u32 n, u32 *sq_words, u32 *list, PassCounters *ctr, hipStream_t stream);
hipError_t launch_walk_baby(const WalkParams &p, u32 grid, hipStream_t stream);
hipError_t launch_popcount_add(const u32 *words, u64 nwords, unsigned long long *out,
                               hipStream_t stream);

hipError_t launch_walk_window(const InfraParams &p, u32 grid, hipStream_t stream);
hipError_t launch_build_tables(const InfraParams &p, u32 nmax, hipStream_t stream);
hipError_t launch_walk_giant(const InfraParams &p, u32 grid, hipStream_t stream);
int walk_window_blocks_per_cu();
int walk_giant_blocks_per_cu();

// Occupancy helper: resident 256-thread blocks per CU of the baby walk.
int walk_baby_blocks_per_cu();

}  // namespace eis
