// eis_internal.h -- declarations shared by the host runtime (eis_api.cpp) and
// the kernel launchers (eis_kernels.hip, eis_infra.hip).  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eis {

typedef uint16_t u16;
typedef uint32_t u32;
typedef uint64_t u64;

// Candidates of one pass of the pipeline (all segments together).  A
// multiple of 32, so that segments can start on bitmap words.
constexpr u64 kPassCandidates = u64(1) << 24;

// A pass covers up to kMaxSegments segments (ranges or pieces of ranges).
// A work item is (segment << kItemShift) | index, index < 2^kItemShift.
constexpr u32 kMaxSegments = 256;
constexpr u32 kItemShift = 24;
constexpr u32 kItemMask = (1u << kItemShift) - 1;

// Candidates per sieve workgroup (one LDS bitmap of kSegWords words).
constexpr u32 kSegCandidates = 32768;
constexpr u32 kSegWords = kSegCandidates / 32;

// Device-side prime table entry for the sieves: an odd prime p, its square
// m = p^2 and 8^{-1} mod m (squarefree sieve), and 8^{-1} mod p (prime sieve).
struct PrimeEntry {
    u64 m;
    u64 inv8;
    u32 p;
    u32 inv8p;
};

// The candidate set a segment counts and walks: D (squarefree d = 5 mod 8)
// or its primes.
constexpr u32 kSetSquarefree = 0;
constexpr u32 kSetPrime = 1;

// One segment of a pass: candidates d0 + 8 i, i < n.
struct SegInfo {
    u64 d0;
    u32 n;
    u32 word_off;    // first bitmap word of the segment in the pass bitmaps
    u32 block_off;   // first sieve workgroup of the segment
    u32 np;          // odd primes p with p^2 <= the segment's largest d
    u32 roff_off;    // the segment's prime offsets start here
    u32 method;      // 0 = plain walk, 1 = giant steps
    u32 count_slot;  // counts go to counts[2 slot] (D) and counts[2 slot + 1] (E)
    float wscale;    // giant steps: mu_1 is the distinguished ideal number
                     // round(wscale * d^(1/4) / 16)
    u32 set;         // kSetSquarefree or kSetPrime
};

// Per-pass device counters (one cache line each to avoid false sharing).
struct PassCounters {
    u32 list_len;      // number of items in the list this counter belongs to
    u32 pad0[15];
    u32 work_next;     // walk queue head
    u32 pad1[15];
    u32 err_count;     // walks that exceeded the step budget
    u32 pad2[15];
    unsigned long long baby_steps;   // rho steps of the window or plain walk
    unsigned long long refills;
    unsigned long long giant_steps;
    unsigned long long chunk_steps;  // rho steps inside the giant-step walk
    // work of the giant walk's compositions (see GiantWork)
    unsigned long long giant_comps, giant_euclid, giant_reduce, giant_lookups, giant_gcd_branch;
    unsigned long long giant_xgcd;  // of giant_euclid, the extended Euclid's steps
    unsigned long long window_entries;  // list appends of the window walk
    // phases of the giant walk (compose, walk) and the lanes they kept busy
    unsigned long long giant_phases[2], giant_lanes[2];
};

// The fields of a segment that the walk kernels need, kept in LDS.
struct SegLds {
    u64 d0;
    u32 word_off;
    float wscale;
};

template <typename Seg>
__device__ __forceinline__ u64 item_d(const Seg *segs, u32 item)
{
    return segs[item >> kItemShift].d0 + 8ull * (item & kItemMask);
}

// bit of the pass bitmaps that belongs to an item
template <typename Seg>
__device__ __forceinline__ u32 item_bit(const Seg *segs, u32 item)
{
    return segs[item >> kItemShift].word_off * 32u + (item & kItemMask);
}

struct WalkParams {
    const SegInfo *segs;          // segment table of the pass
    u32 nseg;                     // its number of segments
    const u32 *list;              // items to walk
    PassCounters *ctr;            // list_len, queue head, error and step counters
    u32 *eis_words;               // output bitmaps of the pass
    u32 max_steps;                // per-d step budget
    u32 exact_quot;               // 1: every d of the pass is at most kExactQuotMaxD
};

// ---- infrastructure method ------------------------------------------------
// Per-d record written by the window walk for the giant-step walk.
struct WindowState {
    u32 emain;    // mu_1 (the giant step) is list entry emain - 1
    u32 count;    // dictionary entries written; 0 = the d takes no giant steps
    u32 item;     // the d's work item
    u32 pad;
};

// Per-d task of the giant walk, written by the squaring kernel: the d's
// batch position and work item, the giant step g = reduce(mu_1^2) and the
// second giant ideal g2 = reduce(g^2), each as a reduced ideal (Q/4, P/4 in
// fp32, Qp/4 its rho predecessor) and its residue S in Z/3 (g.S = kSquareBad
// when a check of the squarings failed: the d is handed off), and
// s = isqrt(d) (as s/4) and L = isqrt(s), which the squaring kernel has
// computed already (exact in fp32 for d < 2^48).
struct GiantIdeal {
    float Q4, P4, Qp4;
    u32 S;
};
struct GiantTask {
    u32 pos, item;
    GiantIdeal g, g2;
    float s4, L;
};
constexpr u32 kSquareBad = ~0u;

// The squaring kernel sorts the tasks into kCostBuckets buckets by estimated
// walk length (bucket 0 longest), each bucket an array of task_cap tasks; the
// giant walk takes bucket 0 first.  Bucket b's task count is gbuckets[16 b].
constexpr u32 kCostBuckets = 8;

struct InfraParams {
    const SegInfo *segs;        // segment table of the pass
    u32 nseg;                   // its number of segments
    const u32 *list;            // items that take giant steps
    const PassCounters *list_ctr;  // list_ctr->list_len: number of such items
    u32 k0, batch;              // this launch handles list positions [k0, k0 + batch)
    PassCounters *ctr;          // step statistics
    u32 *win_next;              // window-walk queue head (per batch)
    u32 *giant_next;            // giant-walk queue head (per batch)
    u32 *fb_list;               // items handed to the plain walk
    PassCounters *fb_ctr;       // fb_ctr->list_len counts fb_list
    WindowState *state;         // per batch position
    GiantTask *tasks;           // kCostBuckets buckets of task_cap tasks
    u32 task_cap;               // tasks per bucket (>= batch)
    u32 *gbuckets;              // task counts of the buckets (one cache line each)
    unsigned long long *lists;  // window lists: entry e of batch position k at
                                // k * emax + e; an entry is the ideal's
                                // (Q/4, P/4) as fp32 bits
    u32 *lres;                  // 2 S (twice the residue sum) of each entry, same layout
    u16 *tables;                // hash tables, tsize 16-bit slots per batch position
    u32 emax;                   // list capacity per d (a multiple of 8)
    u32 tsize;                  // table slots per d (whole groups of 8, at most kTableSlotsMax)
    u32 max_steps;              // per-d budget of reduction steps (window)
    u32 max_giants;             // per-d budget of giant steps
    u32 emain_shift;            // mu_1 this many entries later (the retry round)
    u32 *eis_words;             // output bitmaps of the pass
    u32 variant;                // kVariant* bits (0: the default method)
    u32 walk_chunk;             // giant walk: reduction steps per walk phase
    u32 exact_quot;             // 1: every d of the pass is at most kExactQuotMaxD
};

// Heights up to which the biased fp32 quotient of a reduction step is never
// one too large (the step's overshoot test can be left out; the bound is
// derived beside rho_step_q and holds with margin: 4.1 10^11).
constexpr u64 kExactQuotMaxD = 145000000000ull;

// Largest dictionary table per d (16-bit slots).
constexpr u32 kTableSlotsMax = 1024;

// Default reduction steps per walk phase of the giant walk (the tuner's
// usual choice above 10^10).
constexpr u32 kDefaultWalkChunk = 16;

// Method variants (all give the same bits).  kVariantNoConjugate: the giant
// step is mu_1 itself (the paper's stride) and only direct lookups are made;
// the window then runs to 1.5 times mu_1's step count, so that a step cannot
// jump over the stored stretch past a period.  kVariantNoSmallNorm: NUCOMP /
// NUDUPL with their partial reduction for every norm, instead of the plain
// ideal product when a norm u is <= 50.
constexpr u32 kVariantNoConjugate = 1;
constexpr u32 kVariantNoSmallNorm = 2;

// Launchers (all enqueue on `stream`, never synchronise).
hipError_t launch_zero_u32(u32 *p, u64 nwords, hipStream_t stream);
hipError_t launch_prime_offsets(const PrimeEntry *primes, const SegInfo *segs, u32 nseg,
                                u32 np_max, u64 *roff, hipStream_t stream);
hipError_t launch_sieve(const PrimeEntry *primes, const u64 *roff, const SegInfo *segs,
                        u32 nseg, u32 nblocks, u32 nsmall, u32 nsmall_p, u32 *sq_words,
                        u32 *list_plain,
                        PassCounters *ctr_plain, u32 *list_giant, PassCounters *ctr_giant,
                        hipStream_t stream);
hipError_t launch_walk_baby(const WalkParams &p, u32 grid, hipStream_t stream);
hipError_t launch_popcount_segs(const u32 *sq_words, const u32 *eis_words, const SegInfo *segs,
                                u32 nseg, u32 words_max, unsigned long long *counts,
                                hipStream_t stream);

// `retry`: the same kernels under their own names (k_retry_*), for the round
// that runs the first round's hand-offs again with another mu_1.
hipError_t launch_walk_window(const InfraParams &p, u32 grid, bool retry, hipStream_t stream);
hipError_t launch_build_tables(const InfraParams &p, u32 grid, bool retry, hipStream_t stream);
hipError_t launch_giant_square(const InfraParams &p, bool retry, hipStream_t stream);
hipError_t launch_walk_giant(const InfraParams &p, u32 grid, bool retry, hipStream_t stream);
int walk_window_blocks_per_cu();
int walk_giant_blocks_per_cu();

// Occupancy helper: resident 256-thread blocks per CU of the baby walk.
int walk_baby_blocks_per_cu();

// ---- no-allocation entry point (eis_noalloc.hip) ---------------------------
// Size of the file-scope device scratch, and the largest range (in
// candidates) one call may cover.
constexpr u64 kNoAllocScratchBytes = u64(256) << 20;
constexpr u64 kNoAllocMaxCandidates = u64(1) << 20;
// Look up the scratch's device address on `device` (current) once.
hipError_t noalloc_scratch_init(int device);
// That address, or null when the lookup failed or has not run.
void *noalloc_scratch(int device);
// Store one segment-table entry on the device from a kernel argument.
hipError_t launch_store_seg(const SegInfo &s, SegInfo *dst, hipStream_t stream);

}  // namespace eis
