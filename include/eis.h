/*
 * eis.h -- C ABI of libeis, an MI355X (gfx950) implementation of the search
 * for Eisenstein discriminants of Breuer & Punch, "Quadratic units and cubic
 * fields".
 *
 * Problem (Section 1 of the paper): for every candidate d in a half-open
 * range [a, b) decide whether d lies in
 *     D = { d > 0 : d = 5 (mod 8), d squarefree }   and in
 *     E = { d in D : eps_d = 1 (mod 2 O_K) },
 * where eps_d is the fundamental unit of Q(sqrt d) and O_K = Z[(1+sqrt d)/2],
 * and count both sets (pi_D, pi_E).  pi_E(x) is the n_eis of [5, x+1).
 *
 * Method (Appendix A): the cycle of reduced principal ideals of O_K is
 * walked with the reduction map rho (baby steps), optionally combined with
 * the infrastructure giant steps of Algorithm "Infrastructure" using NUCOMP,
 * NUDUPL and NUCOMPchoose, while the relative generators are carried as
 * elements of (O_K/2O_K)^* ~ F_4^* ~ Z/3.  The result per d is exact:
 * no heuristic, no tolerance.
 *
 * Conventions shared by every call:
 *  - Candidate lattice.  d_i = d0 + 8 i, i = 0 .. n-1, where d0 is the least
 *    d >= a with d = 5 (mod 8) and n = eis_num_candidates(a, b).
 *  - Bitmaps.  Bit i of a bitmap is bit (i % 8) of byte i / 8 (LSB first);
 *    a bitmap for [a, b) is ceil(n / 8) bytes; the unused high bits of the
 *    last byte are written as 0.
 *  - Ranges.  a >= b is an empty range: OK, zero counts, nothing written.
 *    b > EIS_MAX_D gives EIS_ERANGE.
 *  - Errors.  Every call returns an eis_status (0 = OK, < 0 = error).  On
 *    error, caller-owned outputs are left untouched.  No C++ exception
 *    crosses this boundary.
 *  - Ownership.  The library owns everything inside an eis_ctx (device
 *    memory, streams, queues); pointers passed in are borrowed for the
 *    duration of the call (or, for the _async call, until the stream has
 *    passed the work).
 *  - Threads.  One eis_ctx may be used by one host thread at a time, except
 *    eis_submit, eis_wait, eis_cancel and eis_get_stats, which are safe to
 *    call from any thread.
 *  - There is no CPU fallback: an eis_ctx needs a gfx950 device, and
 *    eis_create fails with EIS_EDEVICE without one.
 */
#ifndef EIS_H
#define EIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EIS_ABI_VERSION 8

/* Largest supported exclusive upper bound b.  The baby-step walk keeps every
 * quantity below 2^24 and exact in fp32 up to this height, and the giant-step
 * composition checks every 64-bit product against overflow. */
#define EIS_MAX_D 1000000000000ULL /* 10^12 */

typedef struct eis_ctx eis_ctx;

typedef enum {
    EIS_OK = 0,
    EIS_EINVAL = -1,     /* bad argument (NULL pointer, short buffer, bad config) */
    EIS_ERANGE = -2,     /* b > EIS_MAX_D */
    EIS_ENOMEM = -3,     /* device memory or the memory budget exhausted */
    EIS_EDEVICE = -4,    /* no usable gfx950 device, or a HIP runtime error */
    EIS_EBUSY = -5,      /* serving queue full (eis_submit) */
    EIS_ECANCELED = -6,  /* request was cancelled (eis_wait) */
    EIS_ETIMEDOUT = -7,  /* eis_wait timed out; the request is still pending */
    EIS_EINTERNAL = -8   /* a walk exceeded max_steps_per_d or an internal check
                            failed; no result bit was produced for it */
} eis_status;

typedef enum {
    EIS_METHOD_BABY = 0,  /* rho steps only, to the half-period symmetry point */
    EIS_METHOD_INFRA = 1, /* baby window + infrastructure giant steps */
    EIS_METHOD_AUTO = 2   /* per-range choice by height (autotuned) */
} eis_method;

/* Candidate sets (the *_set calls): D itself, or the primes in D (the
 * prime subsequence of Section 3.2; a prime d = 5 mod 8 is squarefree). */
#define EIS_SET_SQUAREFREE 0
#define EIS_SET_PRIME 1

/* eis_config.flags bits */
#define EIS_FLAG_NO_GRAPHS 1u    /* run batched passes as plain launches, not hipGraph replays */
#define EIS_FLAG_KERNEL_TIMES 2u /* time every kernel launch of plain (non-graph) passes with
                                    events on the launch stream; totals in eis_stats */
/* Method variants of the giant-step method (Appendix A); every setting gives
 * the same bits, only the work differs. */
#define EIS_FLAG_NO_CONJUGATE_LOOKUPS 4u /* the paper's stride: giant step mu_1 with direct
                                            lookups only (default: step mu_1^2, each giant
                                            ideal looked up with its conjugate too, by the
                                            symmetry of the cycle under conjugation) */
#define EIS_FLAG_NO_SMALL_NORM_PRODUCT 8u /* NUCOMP/NUDUPL with partial reduction for every
                                             norm (default: the plain ideal product when a
                                             norm u <= 50, as NUCOMPchoose prescribes) */

/* Kernels of a pass, for the per-kernel entries of eis_stats. */
typedef enum {
    EIS_K_PRIME_OFFSETS = 0, /* first multiple of every p^2 in each segment */
    EIS_K_SIEVE = 1,         /* squarefree sieve and work-list compaction */
    EIS_K_WALK_PLAIN = 2,    /* rho walk (Appendix A) to the half-period exit of Algorithm
                                Infrastructure; the exit rule is derived here from the
                                symmetry of the cycle under conjugation */
    EIS_K_WALK_WINDOW = 3,   /* giant-step method: baby window and dictionary */
    EIS_K_BUILD_TABLES = 4,  /* giant-step method: dictionary hash tables */
    EIS_K_WALK_GIANT = 5,    /* giant-step method: giant steps with lookups */
    EIS_K_WALK_HANDOFF = 6,  /* plain walk of the d's the giant-step method handed off */
    EIS_K_POPCOUNT = 7,      /* per-segment counts */
    EIS_K_GIANT_SQUARE = 8,  /* giant-step method: g = mu_1^2 and g^2 (NUDUPL) */
    EIS_K_GIANT_RETRY = 9,   /* giant-step method again, with a later mu_1, for the d's
                                the first round handed off (its four kernels together) */
    EIS_K_COUNT = 10
} eis_kernel;

typedef struct {
    int device;                /* HIP device ordinal */
    int method;                /* an eis_method */
    uint64_t mem_budget_bytes; /* device bytes the context may hold; 0 = 1/4 of free memory */
    uint64_t max_steps_per_d;  /* per-d step budget; 0 = default (2^28) */
    double window_scale;       /* giant-step method: baby window = window_scale * d^(1/4)
                                  reduction steps; 0 = autotuned */
    uint32_t serve_slots;      /* serving: max requests in flight; 0 = default (64) */
    uint32_t flags;            /* EIS_FLAG_* bits; other bits must be 0 */
    const char *tune_cache_path; /* autotuner JSON cache; NULL = no persistence */
} eis_config;

typedef struct {
    uint64_t launches;         /* kernel launches issued */
    uint64_t discriminants;    /* members of D classified */
    uint64_t baby_steps;       /* rho steps executed on the device */
    uint64_t giant_steps;      /* giant steps (NUCOMP / NUDUPL) executed */
    uint64_t refills;          /* lane refills in the walk kernels */
    uint64_t fallbacks;        /* d's the giant-step method handed to the plain walk */
    uint64_t requests_done;    /* serving requests completed */
    double last_walk_ms;       /* device time of the last walk launch(es) */
    double last_total_ms;      /* device time of the last whole classify */
    /* per eis_kernel: rho steps executed by that kernel (walk kernels only) */
    uint64_t kernel_steps[EIS_K_COUNT];
    /* per eis_kernel, only with EIS_FLAG_KERNEL_TIMES: timed launches and
     * their summed device time */
    uint64_t kernel_launches[EIS_K_COUNT];
    double kernel_ms[EIS_K_COUNT];
    /* work of the giant-step walk (the operation counts of its instruction
     * model): NUCOMP compositions, the Euclid steps inside them (extended and
     * partial Euclid), the reduction steps after them, the compositions that
     * took NUCOMP's gcd branch, and the dictionary lookups (pairs of keys) */
    uint64_t giant_compositions;
    uint64_t giant_euclid_steps;
    uint64_t giant_reduce_steps;
    uint64_t giant_gcd_branches;
    uint64_t giant_lookups;
    /* distinguished ideals the window walk appended to the dictionary lists
     * (the operation count of its list-append path) */
    uint64_t window_entries;
    /* d's the giant-step method handed off and ran again with mu_1 four
     * distinguished ideals later; `fallbacks` counts those it handed off
     * again, which the plain walk classifies */
    uint64_t giant_retries;
    /* how full the giant-step walk's phases ran: the phases that looked up
     * and composed, the phases that walked to distinguished ideals, and the
     * lanes each kind kept busy (64 per phase at most) */
    uint64_t giant_compose_phases;
    uint64_t giant_compose_lanes;
    uint64_t giant_walk_phases;
    uint64_t giant_walk_lanes;
    /* serving admission by device memory: the bytes the admitted requests
     * hold for their giant-step scratch, and the budget they share (the
     * context's mem_budget_bytes less its fixed buffers; 0 before the first
     * eis_submit) */
    uint64_t serve_bytes_reserved;
    uint64_t serve_bytes_budget;
    /* of giant_euclid_steps, the steps of the extended Euclid loops (the two
     * loops have different instruction counts) */
    uint64_t giant_xgcd_steps;
} eis_stats;

/* Fill *cfg with defaults (device 0, EIS_METHOD_AUTO). */
void eis_config_default(eis_config *cfg);

/* Create a context on cfg->device.  *out receives the context.
 * EIS_EDEVICE without a gfx950 device, EIS_EINVAL on a bad config. */
int eis_create(const eis_config *cfg, eis_ctx **out);

/* Destroy a context (waits for its outstanding work).  NULL is a no-op. */
void eis_destroy(eis_ctx *ctx);

/* Number of candidates d = 5 (mod 8) with a <= d < b (Section 1: D is a
 * subset of this lattice).  Pure host arithmetic, no context needed. */
uint64_t eis_num_candidates(uint64_t a, uint64_t b);

/* d0: least d >= a with d = 5 (mod 8). */
uint64_t eis_first_candidate(uint64_t a);

/* Counts only: *n_sqfree = #(D n [a,b)) and *n_eis = #(E n [a,b))
 * (Section 1, pi_D and pi_E).  Either output pointer may be NULL. */
int eis_count(eis_ctx *ctx, uint64_t a, uint64_t b, uint64_t *n_sqfree, uint64_t *n_eis);

/* Flags and counts into caller-owned HOST buffers (Section 1, the sets D, E):
 * sqfree_bits bit i = [d_i in D], eis_bits bit i = [d_i in E] (eis is a
 * subset of sqfree).  Either bitmap may be NULL; a non-NULL bitmap needs
 * len_bytes >= ceil(n / 8), else EIS_EINVAL.  Synchronous. */
int eis_classify(eis_ctx *ctx, uint64_t a, uint64_t b, uint8_t *sqfree_bits,
                 uint8_t *eis_bits, size_t len_bytes, uint64_t *n_sqfree, uint64_t *n_eis);

/* Same as eis_classify, with DEVICE outputs, enqueued on the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the context's own stream).
 * d_sqfree_bits / d_eis_bits: device buffers of ceil(n/8) bytes or NULL.
 * d_counts2: device uint64_t[2] receiving {n_sqfree, n_eis}, or NULL.
 * Returns after enqueueing; results are valid once the stream reaches them.
 * Ranges of more than 2^24 candidates wait on the host between passes (the
 * pass buffers are reused); the last pass is left running.  The next call on
 * the context that runs a pass waits for it first.  Step-budget overruns
 * (EIS_EINTERNAL) are reported by eis_last_error. */
int eis_classify_async(eis_ctx *ctx, uint64_t a, uint64_t b, void *d_sqfree_bits,
                       void *d_eis_bits, uint64_t *d_counts2, void *hip_stream);

/* Largest range, in candidates, of one eis_classify_async_noalloc call, and
 * the size of the device scratch that call works in. */
#define EIS_NOALLOC_MAX_CANDIDATES (1ULL << 20)
#define EIS_NOALLOC_SCRATCH_BYTES (256ULL << 20)

/* eis_classify_async for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and error behaviour as
 * eis_classify_async, but the call allocates nothing: every buffer its
 * kernels use beyond the caller's outputs (segment table, prime offsets, work
 * lists, counters, pass bitmaps and the giant-step lists, tables and tasks)
 * lives in one file-scope device array of EIS_NOALLOC_SCRATCH_BYTES per
 * device, which the loaded library holds until the process ends; its address
 * is looked up once per device by eis_create.  The range is one pass of at
 * most EIS_NOALLOC_MAX_CANDIDATES candidates: a larger one gives EIS_ENOMEM
 * and nothing is enqueued.  Giant-step batches are sized to the scratch
 * (about 8*10^4 d's near 10^12), so a range at that height takes several.
 * Every call on one device shares that device's scratch, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one device -- on different streams, contexts or threads --
 * race, while calls on one stream are ordered.  Results are valid once the
 * stream reaches them; step-budget overruns are reported by eis_last_error. */
int eis_classify_async_noalloc(eis_ctx *ctx, uint64_t a, uint64_t b, void *d_sqfree_bits,
                               void *d_eis_bits, uint64_t *d_counts2, void *hip_stream);

/* Status of the asynchronous calls since the last eis_last_error (EIS_OK,
 * or EIS_EINTERNAL if a walk of theirs overran its step budget).  Waits for
 * the last pass they left running, on the stream it was enqueued on (which
 * must still exist). */
int eis_last_error(eis_ctx *ctx);

/* n ranges [a[k], b[k]) counted together (Section 1 counts, per range).
 * The ranges are cut into pieces, ordered by height (the costliest walks
 * first) and packed into passes; a pass is one sieve launch over all its
 * pieces, ONE persistent walk launch over all their members of D (plus the
 * giant-step launches of the pieces above the method-switch height), and
 * the counts, replayed from a captured hipGraph.
 * n_sqfree / n_eis: caller-owned host arrays of n entries (either NULL).
 * Overlapping ranges are allowed and are counted independently. */
int eis_count_batch(eis_ctx *ctx, const uint64_t *a, const uint64_t *b, size_t n,
                    uint64_t *n_sqfree, uint64_t *n_eis);

/* Counts over a candidate set: *n_set = #(S n [a,b)) and *n_eis =
 * #(E n S n [a,b)) for S = D (EIS_SET_SQUAREFREE, same as eis_count) or
 * S = D n P, the primes p = 5 (mod 8) (EIS_SET_PRIME; Section 3.2, the prime
 * subsequence pi_{E n P}).  The prime set is sieved by every odd prime up
 * to sqrt(b) and only its members are walked.  EIS_EINVAL for another set. */
int eis_count_set(eis_ctx *ctx, int set, uint64_t a, uint64_t b, uint64_t *n_set,
                  uint64_t *n_eis);

/* eis_count_batch over a candidate set (see eis_count_set). */
int eis_count_batch_set(eis_ctx *ctx, int set, const uint64_t *a, const uint64_t *b, size_t n,
                        uint64_t *n_set, uint64_t *n_eis);

/* ----- Serving (continuous batching of range-count queries) ----------- */

/* Queue the count of [a, b).  *ticket receives a handle for eis_wait.
 * A server thread (started by the first call) runs passes back to back, two
 * in flight at a time; each pass takes the next chunk (at most 2^20
 * candidates) of every admitted request, so requests that arrive while
 * others run join the next pass and a large request does not hold up small
 * ones (continuous batching).  Admission is by slots and by device memory:
 * a request reserves the giant-step scratch (dictionary lists, tables,
 * window records, tasks) of its first chunk -- nothing at heights the plain
 * walk takes -- against the serving budget (mem_budget_bytes less the
 * context's fixed buffers; see eis_stats.serve_bytes_*), until it finishes
 * or is cancelled.  EIS_EBUSY when serve_slots requests are already queued
 * or running, or when the admitted requests hold so much of the budget that
 * this one does not fit now (retry later); EIS_ENOMEM when it could not fit
 * even alone.  Nothing is queued on error. */
int eis_submit(eis_ctx *ctx, uint64_t a, uint64_t b, uint64_t *ticket);

/* Wait up to timeout_us microseconds (< 0 = forever) for a ticket.  On
 * EIS_OK the counts are written and the ticket is retired.  EIS_ETIMEDOUT
 * leaves it pending; EIS_ECANCELED / EIS_EINTERNAL retire it.  An unknown
 * or retired ticket gives EIS_EINVAL, also when another thread's eis_wait
 * retires it during the wait. */
int eis_wait(eis_ctx *ctx, uint64_t ticket, int64_t timeout_us, uint64_t *n_sqfree,
             uint64_t *n_eis);

/* Cancel a pending ticket (its eis_wait returns EIS_ECANCELED).  A request
 * whose work is already on the device finishes there and is discarded. */
int eis_cancel(eis_ctx *ctx, uint64_t ticket);

/* ----- Autotuner ----------------------------------------------------- */

/* Autotuner.  Per half-decade height bin 10^(b/2) <= d < 10^((b+1)/2) from
 * 10^6 to 10^12: time the plain walk and the giant-step method at eight
 * window scales from 1 to 5, each on 2^22 candidates at the bin's lower and
 * upper quarter points, and keep the faster method and its best scale by the
 * summed times (below 10^6: the plain walk); at the bin's geometric middle,
 * for the giant-step method, time the giant walk's walk chunk (8, 16, 32
 * reduction steps per phase) at that scale on 2^24 candidates; then time a
 * full pass's worth of candidates cut into passes of 2^22, 2^23 and 2^24
 * candidates.  The AUTO
 * method then follows these choices (an explicit method or window scale in
 * the config still wins).  With cfg.tune_cache_path set at eis_create, the
 * choices are loaded from that file when it exists and holds every bin, and
 * eis_tune writes them there with every timing (EIS_EINVAL if the file
 * cannot be written; the choices are in force anyway).  Every choice gives
 * the same bits; only the time differs.  Takes a few seconds.  Thread-safe
 * against the other calls. */
int eis_tune(eis_ctx *ctx);

/* The choice in force for height d: *method (an eis_method, BABY or INFRA)
 * and *window_scale. */
int eis_tuned_choice(eis_ctx *ctx, uint64_t d, int *method, double *window_scale);

/* The tuned shape parameters in force for height d: *walk_chunk, the giant
 * walk's reduction steps per walk phase (default 16), and *pass_candidates,
 * the candidates per pass a range starting at d is cut into (default 2^24).
 * Either pointer may be NULL. */
int eis_tuned_shape(eis_ctx *ctx, uint64_t d, uint32_t *walk_chunk, uint64_t *pass_candidates);

/* Counters since eis_create. */
int eis_get_stats(eis_ctx *ctx, eis_stats *out);

/* Static text for a status code. */
const char *eis_strerror(int status);

/* Library ABI version (EIS_ABI_VERSION). */
int eis_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIS_H */
