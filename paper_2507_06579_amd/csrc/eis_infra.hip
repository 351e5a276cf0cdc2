// eis_infra.hip -- the infrastructure method of Appendix A on gfx950.
//
// Algorithm "Infrastructure" with the generators carried in
// (O_K/2O_K)^* ~ Z/3, split into four kernels so that every lane of a wave
// runs the same phase:
//
//   k_walk_window  one d per lane: reduction steps from (1), with the
//                  half-period symmetry exit; the "distinguished" ideals of
//                  the walk (Q = 2 mod 64, about one in 16) are appended to
//                  the d's dictionary list (the ideal's (Q/4, P/4) as fp32
//                  bits, and twice its residue sum beside it).  mu_1 is the
//                  n-th distinguished ideal (n = wscale * d^(1/4) / 16, at
//                  least 16); the window ends at the first distinguished
//                  ideal at least six steps after mu_1 (the two extra ideals
//                  of the algorithm, with margin), and that extension must
//                  stay within mu_1's own step count.
//   k_build_tables one wave per d: the list is indexed by an open-addressed
//                  hash table of 16-bit slots (9-bit list index + 7-bit
//                  fingerprint; a fingerprint match is confirmed against the
//                  list entry), built in LDS and written out whole.
//   k_giant_square four d's per lane: the giant step g = reduce(mu_1^2) and
//                  the second giant ideal reduce(g^2), by NUDUPL; each d's
//                  task goes into a bucket by its estimated walk length.
//   k_walk_giant   one d per lane, lanes refilled from a queue over the
//                  buckets, longest estimated walks first: starting
//                  from g and g^2, the giant ideals g_k = reduce(g * g_{k-1})
//                  (NUCOMP), the residue updated with log g + log g_{k-1} -
//                  log gamma + the residues of the reduction steps; after
//                  each, reduction steps forward to the first distinguished
//                  ideal, which is looked up twice: itself (a hit means one
//                  period past a window ideal: log eps = log(ideal) -
//                  log(window ideal)) and its conjugate (one period short of
//                  a window ideal: log eps = log(ideal) + log(window ideal)).
//                  The dictionary thus covers distances on both sides of
//                  (1), and the giant step can be twice mu_1.
//
// Why the distinguished ideals: a dictionary with every window ideal would
// cost one scattered 8-byte store per reduction step.  With only every 16th
// ideal stored, the stores are rare and the tables small, at the price of a
// short walk after every giant step.  A distinguished ideal's conjugate is
// distinguished too (Q_{l-m} = Q_m), so the conjugate lookups see the same
// set.  Coverage: the dictionary holds the distinguished ideals at
// distances [0, D] and, through the conjugate lookups, [-D, 0] (mod the
// regulator), where D is the window's end; the giant step g = mu_1^2
// advances by about twice mu_1's distance, and the window runs at least six
// ideals past mu_1, so consecutive giant ideals cannot jump over the covered
// stretch around a period.  A direct hit at the first lookup (g itself) is
// skipped: when the window is short, g can land inside the window, which
// reads as a "unit" of distance 0.  Later giant ideals lie beyond the
// window, so a direct hit is at one regulator (or two after a skipped true
// hit); a conjugate hit can never be at distance 0, since giant ideals move
// forward.  "Beyond the window": the second giant ideal lies about four
// times mu_1's distance from (1), while the window ends within twice it
// (its extension past mu_1 is at most mu_1's own step count; a d whose
// extension is longer goes to the plain walk), a margin of a factor two over
// the fluctuation of distance per step.  log eps^2 = 2 log eps is 0 in Z/3
// exactly when log eps is, so a hit at two regulators gives the same flag.
//
// Any arithmetic check that fails (fp64 exactness, exact divisions, step or
// walk budgets, table overflow) hands the d off.  The four kernels have a
// second set of entry points (k_retry_*) for a round that runs the hand-offs
// again with mu_1 emain_shift distinguished ideals later, so that the giant
// ideals differ; what that round hands off goes to the plain walk, which is
// exact for every d below 10^12.
#include "eis_giant.h"
#include "eis_internal.h"
#include "eis_walk.h"

namespace eis {

// Q = 2 (mod 64), tested on the quarter-unit value Q/4: fract(Q/64) = 1/32
// exactly for integer-valued Q < 2^24.
constexpr float kDpScale = 1.0f / 16.0f;
constexpr float kDpHit = 2.0f / 64.0f;
__device__ __forceinline__ bool is_dp(float Q4) { return __builtin_amdgcn_fractf(Q4 * kDpScale) == kDpHit; }

constexpr u32 kTableMax = kTableSlotsMax;  // largest table (slots) per d
constexpr u32 kWalkLimit = 4096;    // reduction steps from a giant ideal to a distinguished one
constexpr u32 kExtraSteps = 6;      // window runs at least this far past mu_1
constexpr u32 kMinMain = 16;        // mu_1 is at least the 16th distinguished ideal

// dictionary key of a reduced ideal: its quarter-unit (Q, P) as fp32 bits
__device__ __forceinline__ unsigned long long entry_of(float Q4, float P4)
{
    return ((unsigned long long)__float_as_uint(Q4) << 32) | (unsigned long long)__float_as_uint(P4);
}

// ---------------------------------------------------------------------------
// k_walk_window: persistent, one d per lane.  A lane whose window ends (or
// whose walk reaches the half period) idles until kBatch lanes of the wave
// are idle; then all of them take their next batch position from a queue
// (claimed 64 at a time per wave; the list entry of a lane's next d is
// loaded one refill ahead).  The per-position outcome goes to p.state:
// count > 0 = the d takes giant steps; count = 0 = its flag is out (half
// period) or it was handed to the plain walk.
//
// List entries are staged in LDS, kRing per lane, and written out as one
// contiguous chunk per kRing entries (32 bytes of keys, 16 of residue sums),
// instead of one scattered 8-byte write each.  Four entries per lane keep
// the rings at 12 KB per block and the kernel at 66 VGPRs, seven waves per
// SIMD (with eight entries, 24 KB and 80 VGPRs: six waves, and the walk took
// 9.8 instead of 8.5 ms per 10^8 window at 10^11; two entries: 9.8 ms).
// ---------------------------------------------------------------------------
constexpr u32 kRing = 4;
static_assert(kRing % 4 == 0, "the residue sums are written four at a time");

struct WindowRing {
    unsigned long long key[kRing][64];
    u32 res[kRing][64];
};

// Write the lane's staged chunk (entries [base, base + kRing) of its list).
__device__ __forceinline__ void ring_flush(const WindowRing &rg, u32 lane, unsigned long long *lb,
                                           u32 *rb, u32 base)
{
    unsigned long long k[kRing];
    u32 r[kRing];
#pragma unroll
    for (u32 e = 0; e < kRing; e++) {
        k[e] = rg.key[e][lane];
        r[e] = rg.res[e][lane];
    }
#pragma unroll
    for (u32 e = 0; e < kRing; e += 2)
        *reinterpret_cast<ulonglong2 *>(lb + base + e) = make_ulonglong2(k[e], k[e + 1]);
#pragma unroll
    for (u32 e = 0; e < kRing; e += 4)
        *reinterpret_cast<uint4 *>(rb + base + e) = make_uint4(r[e], r[e + 1], r[e + 2], r[e + 3]);
}

// `hit` is the distinguished-ideal test value (see is_dp); idle lanes get
// one that never matches.
__device__ __forceinline__ bool window_hit(float Q, float hit)
{
    return __builtin_amdgcn_fractf(Q * kDpScale) == hit;
}

// Stage a distinguished ideal (Q, P) (quarter units) with twice its residue
// sum res2 as entry cnt of the lane's list, and write out a full chunk.
__device__ __forceinline__ void window_append(WindowRing &rg, u32 lane, unsigned long long *lb,
                                              u32 *rb, float Q, float P, u32 res2, u32 &cnt)
{
    const u32 slot = cnt % kRing;
    rg.key[slot][lane] = entry_of(Q, P);
    rg.res[slot][lane] = res2;
    cnt++;
    if (slot == kRing - 1) ring_flush(rg, lane, lb, rb, cnt - kRing);
}

// How a lane's window ended, kept until the wave's next pause (the lane
// appends nothing meanwhile, so its list, count and steps stay as they were):
// half period (the flag in bit 0), window end (residue sums within range or
// not).
constexpr u32 kFinNone = 0, kFinWindow = 1, kFinRange = 2, kFinHalf = 4;

template <bool kCheck>
__device__ __forceinline__ void walk_window_body(const InfraParams &p, const SegLds *segs,
                                                 WindowRing *rings)
{
    const u32 lane = __lane_id();
    WindowRing &rg = rings[threadIdx.x >> 6];
    const u32 total = p.list_ctr->list_len;
    const u32 nb = (p.k0 < total) ? min(p.batch, total - p.k0) : 0u;
    const u32 K = __builtin_amdgcn_readfirstlane(min(kInnerChunk, max(p.max_steps, 1u)));
    const u32 cnt_end = p.emax - 1;  // a full list ends the window (then the d goes plain)
    // Exit batch: the refill (queue, decode, first step, window set-up) costs
    // about as much as 30 reduction steps of the wave; a window is about
    // 16 emain steps.
    const u32 batch = (u32)fminf(fmaxf(rintf(sqrtf(16000.f / (float)(p.emax - 16))), 1.f), 32.f);
    // lane state: the d at batch position pos, its list (entry e at lb[e],
    // rb[e]), the walk in quarter units (see rho_step_q), S2 = twice the
    // residue sum at the start of the current chunk of steps, and the window
    // bookkeeping: jlast = the step of the last entry; e1 = emain until mu_1
    // (entry emain - 1) is staged, then ~0; an entry at step >= j1e ends the
    // window, which is kept if that entry's step is at most jok.
    unsigned long long *lb = p.lists;
    u32 *rb = p.lres;
    float sq = 0.f, sqc = 0.f, P = 0.25f, Q = 0.5f, Qp = 0.5f, hit = -1.f;
    u32 S2 = 0, j = 0, idx = 0, pos = 0, item = 0, cnt = 0, emain = kMinMain, e1 = ~0u;
    u32 j1e = ~0u, jok = 0, jlast = 0;
    u32 fin = kFinNone, jend = 0;  // how and after how many steps the window ended
    const bool long_ext = (p.variant & kVariantNoConjugate) != 0;
    u32 cbase = 0, cend = 0;  // the wave's claimed chunk of the queue
    bool live = false;
    u64 my_steps = 0, my_refills = 0, my_entries = 0;
    // the lane's next batch position and its work item, loaded one refill ahead
    u32 npos = nb;
    wave_take(p.win_next, nb, true, npos, cbase, cend);
    u32 nitem = (npos < nb) ? p.list[p.k0 + npos] : 0u;
    if (npos >= nb) npos = kNoItem;

    for (;;) {
        // ---- refill every idle lane that has a prefetched d -------------
        for (;;) {
            const bool want = !live && npos != kNoItem;
            if (!__any(want)) break;
            u32 k = nb;
            wave_take(p.win_next, nb, want, k, cbase, cend);
            if (want) {
                pos = npos;
                item = nitem;
                npos = (k < nb) ? k : kNoItem;
                nitem = (k < nb) ? p.list[p.k0 + k] : 0u;
                idx = item_bit(segs, item);
                my_refills++;
                lb = p.lists + (u64)pos * p.emax;
                rb = p.lres + (u64)pos * p.emax;
                const u64 d = item_d(segs, item);
                double sd, P1, Q1;
                u32 S1;
                first_step(d, sd, P1, Q1, S1);
                j = 1;
                my_steps += 1;
                if (Q1 == 2.0) {
                    emit_flag(p.eis_words, idx, S1 % 3u == 0u);
                    WindowState st = {0u, 0u, item, 0u};
                    p.state[pos] = st;
                } else {
                    sq = (float)sd * 0.25f;
                    sqc = sq * kQuotBias;
                    P = (float)P1 * 0.25f;
                    Q = (float)Q1 * 0.25f;
                    Qp = 0.5f;
                    S2 = 2u * S1;
                    hit = kDpHit;
                    // the ideal (1) = [1, (P_1 + sqrt d)/2], residue 0
                    rg.key[0][lane] = entry_of(0.5f, P);
                    rg.res[0][lane] = 0u;
                    cnt = 1;
                    jlast = 0;
                    const float n = segs[item >> kItemShift].wscale * sqrtf(sqrtf((float)d)) * (1.f / 16.f);
                    emain = min((u32)fminf(fmaxf(rintf(n), (float)kMinMain), (float)(p.emax - 8)) + p.emain_shift,
                                p.emax - 8);
                    e1 = emain;
                    if (window_hit(Q, hit)) {
                        window_append(rg, lane, lb, rb, Q, P, S2, cnt);
                        jlast = 1;
                    }
                    live = true;
                }
            }
        }
        u64 lm = __builtin_amdgcn_ballot_w64(live);
        if (lm == 0) break;

        // Two steps per iteration.  A lane that reaches the half period or
        // the end of its window is finished at once and idles (its steps go
        // on, but it appends nothing); its outcome is written at the next
        // pause of the loop, which comes when `batch` lanes idle (when all
        // idle once the queue is drained).  The window ends once an entry at
        // least kExtraSteps past mu_1 is staged, or when the list is full;
        // the test runs after every pair, so no lane starts a pair with fewer
        // than two free entries.  With the short extension the list cannot
        // fill: at most seven entries follow mu_1 (entries at the five steps
        // after it, the one that ends the window and its pair's second), and
        // mu_1 is at most entry emax - 9.
        const u32 keep = __any(npos != kNoItem) ? 64u - batch : 0u;
        const u32 iters = (K + 1) / 2;
        u32 it = 0;
        bool stop = false;
        float P1 = 0.f, Q1 = 0.f, acc = 0.f;
        for (;;) {
            float P2, Q2;
            rho_step_q<kCheck>(sq, sqc, P, Q, Qp, P1, Q1, acc);
            const u64 mA = __builtin_amdgcn_ballot_w64(Q1 == Q) | __builtin_amdgcn_ballot_w64(P1 == P);
            const float accA = acc;
            rho_step_q<kCheck>(sq, sqc, P1, Q1, Q, P2, Q2, acc);
            const u64 mB = __builtin_amdgcn_ballot_w64(Q2 == Q1) | __builtin_amdgcn_ballot_w64(P2 == P1);
            // The pair's distinguished ideals, in walk order: one append for
            // the first, which the wave runs at almost every pair, and a
            // second for a lane whose two ideals are both distinguished (one
            // lane-pair in 256), instead of an append per step.
            const bool dA = window_hit(Q1, hit), dB = window_hit(Q2, hit);
            if (dA || dB) {
                const u32 k = 2 * it + (dA ? 1u : 2u);
                window_append(rg, lane, lb, rb, dA ? Q1 : Q2, dA ? P1 : P2,
                              S2 + k + (u32)(dA ? accA : acc), cnt);
                jlast = j + k;
            }
            if (dA && dB) {
                window_append(rg, lane, lb, rb, Q2, P2, S2 + 2 * it + 2 + (u32)acc, cnt);
                jlast = j + 2 * it + 2;
            }
            // mu_1 staged (once per window): it is the last entry, or the
            // pair's first when the pair staged two and went past it
            if (__builtin_amdgcn_ballot_w64(cnt >= e1)) {
                if (cnt >= e1) {
                    const u32 j1 = (cnt == emain) ? jlast : jlast - 1;
                    // the window runs kExtraSteps past mu_1, or (the variant
                    // with the paper's stride) half mu_1's step count; its
                    // extension must stay short next to mu_1's own distance:
                    // at most mu_1's step count, or three quarters of it with
                    // the paper's stride (whose second giant ideal lies only
                    // twice as far as mu_1)
                    j1e = j1 + (long_ext ? max(kExtraSteps, j1 / 2) : kExtraSteps);
                    jok = j1 + (long_ext ? (3 * j1) / 4 : j1);
                    e1 = ~0u;
                }
            }
            u64 ms = __builtin_amdgcn_ballot_w64(jlast >= j1e);
            if (long_ext) ms |= __builtin_amdgcn_ballot_w64(cnt >= cnt_end);
            const u64 ev = (mA | mB | ms) & lm;
            if (ev) {
                if ((ev >> lane) & 1ull) {
                    const bool exA = (mA >> lane) & 1ull;
                    const bool exB = !exA && ((mB >> lane) & 1ull);
                    if (exA || exB) {
                        // half-period symmetry: the unit is found without giant steps
                        const u32 kx = 2 * it + (exA ? 1u : 2u);
                        const float accx = exA ? accA : acc;
                        const float Pj = exA ? P1 : P2;
                        const bool qrule = exA ? (Q1 == Q) : (Q2 == Q1);
                        const u32 S = (S2 + kx + (u32)accx) >> 1;
                        const u32 rj = __builtin_amdgcn_fractf(Pj) > 0.5f ? 2u : 1u;
                        const u32 v = qrule ? (2u * S - rj) : (2u * (S - rj));
                        fin = kFinHalf | (v % 3u == 0u ? 1u : 0u);
                        jend = j + kx - 1;
                    } else {
                        const u32 S2e = S2 + 2 * it + 2 + (u32)acc;
                        fin = S2e < (1u << 24) ? kFinWindow : kFinRange;
                        jend = j + 2 * it + 1;
                    }
                    hit = -1.f;
                }
                lm &= ~ev;
                stop = (u32)__builtin_popcountll(lm) <= keep;
            }
            Qp = Q1;
            Q = Q2;
            P = P2;
            if (++it >= iters || stop) break;
        }
        // ---- outcomes of the windows that ended -------------------------
        if (fin != kFinNone) {
            WindowState st = {0u, 0u, item, 0u};
            if (fin & kFinHalf) {
                emit_flag(p.eis_words, idx, (fin & 1u) != 0u);
            } else {
                const bool ok = fin == kFinWindow && e1 == ~0u && jlast <= jok && cnt < p.emax;
                if (ok) {
                    if (cnt % kRing) ring_flush(rg, lane, lb, rb, cnt / kRing * kRing);
                    st.emain = emain;
                    st.count = cnt;
                } else {
                    const u32 f = atomicAdd(&p.fb_ctr->list_len, 1u);
                    p.fb_list[f] = item;
                }
            }
            p.state[pos] = st;
            my_steps += jend;
            my_entries += cnt - 1;  // appends after the entry of (1)
            j1e = ~0u;
            e1 = ~0u;
            cnt = 0;
            fin = kFinNone;
        }
        live = (lm >> lane) & 1ull;
        if (live) {
            const u32 k = 2 * it;
            j += k;
            S2 += k + (u32)acc;
            if (j > p.max_steps) {
                WindowState st = {0u, 0u, item, 0u};
                p.state[pos] = st;
                const u32 f = atomicAdd(&p.fb_ctr->list_len, 1u);
                p.fb_list[f] = item;
                my_steps += j - 1;
                my_entries += cnt - 1;
                hit = -1.f;
                j1e = ~0u;
                e1 = ~0u;
                cnt = 0;
                live = false;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        my_steps += __shfl_down(my_steps, off, 64);
        my_refills += __shfl_down(my_refills, off, 64);
        my_entries += __shfl_down(my_entries, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&p.ctr->baby_steps, (unsigned long long)my_steps);
        atomicAdd(&p.ctr->refills, (unsigned long long)my_refills);
        atomicAdd(&p.ctr->window_entries, (unsigned long long)my_entries);
    }
}

__device__ __forceinline__ void walk_window_entry(const InfraParams &p)
{
    if (p.k0 >= p.list_ctr->list_len) return;  // nothing in this batch (an empty retry)
    // The segment table is sized at launch (p.nseg entries), so that LDS
    // (the rings, 12 KB per block) stays below the register limit on the
    // workgroups per CU.
    extern __shared__ SegLds segs[];
    __shared__ WindowRing rings[4];
    load_segs(segs, p.segs, p.nseg);
    if (p.exact_quot)
        walk_window_body<false>(p, segs, rings);
    else
        walk_window_body<true>(p, segs, rings);
}

__global__ __launch_bounds__(256) void k_walk_window(InfraParams p) { walk_window_entry(p); }
__global__ __launch_bounds__(256) void k_retry_window(InfraParams p) { walk_window_entry(p); }

hipError_t launch_walk_window(const InfraParams &p, u32 grid, bool retry, hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(retry ? k_retry_window : k_walk_window, dim3(grid), dim3(256),
                       p.nseg * sizeof(SegLds), stream, p);
    return hipGetLastError();
}

int walk_window_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_window, 256, 0) != hipSuccess)
        return 4;
    return nb > 0 ? nb : 1;
}

// ---------------------------------------------------------------------------
// k_build_tables: one wave per d that needs giant steps.  Workgroups are
// numbered so that consecutive ones (d's of the same list tile) run on the
// same XCD and share its L2: hardware block b goes to XCD b % 8.
//
// A slot holds (fingerprint << 9) | (e + 1) for list entry e (emax <= 496,
// so e + 1 < 2^9), the fingerprint being the top 7 bits of the key's hash
// (1 in place of 0, so that no fingerprint matches an empty slot); 0 is
// empty.  An entry goes to its key's home group (kGroup aligned slots, one
// 16-byte load), or, when that group is full, to the first group after it
// that is not, so that a lookup reads the home group whole: the key is in
// it, or the group is full and the key may lie further on.
// ---------------------------------------------------------------------------
constexpr u32 kSlotIndexBits = 9;
constexpr u32 kSlotIndexMask = (1u << kSlotIndexBits) - 1;
constexpr u32 kGroup = 8;
__device__ __forceinline__ u32 slot_fp(u32 h) { return max(h >> (32 - (16 - kSlotIndexBits)), 1u); }
// The home group of hash h among `groups` groups: the low 24 bits of h
// scaled to [0, groups) (the fingerprint takes the top bits, independent of
// these).
__device__ __forceinline__ u32 home_group(u32 h, u32 groups) { return __umul24(h, groups) >> 24; }

// Insert val (hash h) into a wave's LDS table of `groups` groups: at the next
// position of its home group, or, when that group is full, of the first
// group after it (cyclically) that is not (so a key lies in its home group,
// or that group is full and the key lies further on).  fill counts the
// insertions per group; a group's entries fill its first slots.
__device__ __forceinline__ void table_insert(u32 *tab, u32 *fill, u32 h, u32 groups, u32 val)
{
    u32 g = home_group(h, groups);
    for (u32 probe = 0; probe < groups; probe++) {
        const u32 k = atomicAdd(&fill[g], 1u);
        if (k < kGroup) {
            tab[g * kGroup + k] = val;
            return;
        }
        g = (g + 1 == groups) ? 0u : g + 1;
    }
}

// The lane's list entries (entry lane + 64 k, k < kLoads) of the d at batch
// position pos, which has cnt of them.
template <u32 kLoads>
__device__ __forceinline__ void load_entries(const InfraParams &p, u32 pos, u32 cnt,
                                             unsigned long long (&ent)[kLoads])
{
    const unsigned long long *lst = p.lists + (u64)pos * p.emax;
    const u32 lane = threadIdx.x & 63;
#pragma unroll
    for (u32 k = 0; k < kLoads; k++) {
        const u32 e = lane + 64 * k;
        ent[k] = (e < cnt) ? lst[e] : 0ull;
    }
}

// Each wave builds its d's table in its own LDS region, so the phases of a
// table (clear, insert, write out) need only the wave's own LDS operations
// to be complete and visible to its lanes, not a workgroup barrier.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Short lists: kLoads list entries per lane (64 kLoads >= emax).
// Persistent: the block takes groups of four positions (one per wave); each
// wave works on its own table, so its phases are ordered by wave_lds_sync
// alone.  A position's entries are loaded kAhead groups ahead and its entry
// count one group earlier still, so that the loads overlap the insertions
// of the groups in between.  With short lists (64 kLoads = 128 entries at
// most) a wave issues two loads per lane instead of eight mostly idle ones
// (3.37 -> 3.02 ms per 10^8 window at 10^11; 2 to 5 groups ahead measured
// alike, 7 slower).  A position takes giant steps iff its window left
// entries (count > 0).
template <u32 kLoads, u32 kAhead>
__device__ __forceinline__ void build_tables_body(const InfraParams &p, u32 (&tab)[4][kTableMax],
                                                  u32 (&fill)[4][kTableMax / kGroup])
{
    const u32 nblk = gridDim.x, b = blockIdx.x;
    const u32 xcd = b % 8, q = nblk / 8, r = nblk % 8;
    const u32 lb = xcd * q + min(xcd, r) + b / 8;  // logical block
    const u32 wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const u32 total = p.list_ctr->list_len;
    const u32 n = (p.k0 < total) ? min(p.batch, total - p.k0) : 0u;
    const u32 tgroups = p.tsize / kGroup;  // table groups per d
    auto count_of = [&](u32 g) -> u32 {
        const u32 pos = 4 * g + wv;
        return (pos < n) ? p.state[pos].count : 0u;
    };
    u32 cnt[kAhead + 2];
    unsigned long long ent[kAhead + 1][kLoads];
#pragma unroll
    for (u32 i = 0; i < kAhead + 2; i++) cnt[i] = count_of(lb + i * nblk);
#pragma unroll
    for (u32 i = 0; i <= kAhead; i++) load_entries<kLoads>(p, 4 * (lb + i * nblk) + wv, cnt[i], ent[i]);
    for (u32 g = lb; 4 * g < n; g += nblk) {
        const u32 pos = 4 * g + wv;
        for (u32 t = lane; t < p.tsize; t += 64) tab[wv][t] = 0u;
        for (u32 t = lane; t < tgroups; t += 64) fill[wv][t] = 0u;
        wave_lds_sync();
#pragma unroll
        for (u32 k = 0; k < kLoads; k++) {
            const u32 e = lane + 64 * k;
            if (e < cnt[0]) {
                const u32 qb = (u32)(ent[0][k] >> 32), pb = (u32)ent[0][k];
                const u32 h = dict_hash(qb, pb);
                const u32 val = (e + 1) | (slot_fp(h) << kSlotIndexBits);
                table_insert(tab[wv], fill[wv], h, tgroups, val);
            }
        }
        wave_lds_sync();
        if (cnt[0] != 0u) {
            // two slots per 32-bit store
            u32 *tbl = reinterpret_cast<u32 *>(p.tables + (u64)pos * p.tsize);
            for (u32 t = lane; t < p.tsize / 2; t += 64) tbl[t] = tab[wv][2 * t] | (tab[wv][2 * t + 1] << 16);
        }
        wave_lds_sync();
        // advance the pipeline by one group
#pragma unroll
        for (u32 i = 0; i < kAhead; i++) {
            cnt[i] = cnt[i + 1];
#pragma unroll
            for (u32 k = 0; k < kLoads; k++) ent[i][k] = ent[i + 1][k];
        }
        cnt[kAhead] = cnt[kAhead + 1];
        cnt[kAhead + 1] = count_of(g + (kAhead + 2) * nblk);
        load_entries<kLoads>(p, 4 * (g + (kAhead + 1) * nblk) + wv, cnt[kAhead], ent[kAhead]);
    }
}

// Long lists (64 kLoadsLong >= emax): entries one group ahead, counts two.
constexpr u32 kLoadsLong = 8;

__device__ __forceinline__ void build_tables_long(const InfraParams &p, u32 (&tab)[4][kTableMax],
                                                  u32 (&fill)[4][kTableMax / kGroup])
{
    const u32 nblk = gridDim.x, b = blockIdx.x;
    const u32 xcd = b % 8, q = nblk / 8, r = nblk % 8;
    const u32 lb = xcd * q + min(xcd, r) + b / 8;  // logical block
    const u32 wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const u32 total = p.list_ctr->list_len;
    const u32 n = (p.k0 < total) ? min(p.batch, total - p.k0) : 0u;
    const u32 tgroups = p.tsize / kGroup;  // table groups per d
    auto count_of = [&](u32 g) -> u32 {
        const u32 pos = 4 * g + wv;
        return (pos < n) ? p.state[pos].count : 0u;
    };
    u32 cnt0 = count_of(lb), cnt1 = count_of(lb + nblk);
    unsigned long long ent0[kLoadsLong], ent1[kLoadsLong];
    load_entries<kLoadsLong>(p, 4 * lb + wv, cnt0, ent0);
    for (u32 g = lb; 4 * g < n; g += nblk) {
        const u32 pos = 4 * g + wv;
        const u32 cnt2 = count_of(g + 2 * nblk);
        load_entries<kLoadsLong>(p, pos + 4 * nblk, cnt1, ent1);
        for (u32 t = lane; t < p.tsize; t += 64) tab[wv][t] = 0u;
        for (u32 t = lane; t < tgroups; t += 64) fill[wv][t] = 0u;
        wave_lds_sync();
#pragma unroll
        for (u32 k = 0; k < kLoadsLong; k++) {
            const u32 e = lane + 64 * k;
            if (e < cnt0) {
                const u32 qb = (u32)(ent0[k] >> 32), pb = (u32)ent0[k];
                const u32 h = dict_hash(qb, pb);
                const u32 val = (e + 1) | (slot_fp(h) << kSlotIndexBits);
                table_insert(tab[wv], fill[wv], h, tgroups, val);
            }
        }
        wave_lds_sync();
        if (cnt0 != 0u) {
            // two slots per 32-bit store
            u32 *tbl = reinterpret_cast<u32 *>(p.tables + (u64)pos * p.tsize);
            for (u32 t = lane; t < p.tsize / 2; t += 64) tbl[t] = tab[wv][2 * t] | (tab[wv][2 * t + 1] << 16);
        }
        wave_lds_sync();
        cnt0 = cnt1;
        cnt1 = cnt2;
#pragma unroll
        for (u32 k = 0; k < kLoadsLong; k++) ent0[k] = ent1[k];
    }
}

__device__ __forceinline__ void build_tables_entry(InfraParams p)
{
    __shared__ u32 tab[4][kTableMax];
    __shared__ u32 fill[4][kTableMax / kGroup];
    if (p.emax <= 128)
        build_tables_body<2, 3>(p, tab, fill);
    else
        build_tables_long(p, tab, fill);
}

__global__ __launch_bounds__(256) void k_build_tables(InfraParams p) { build_tables_entry(p); }
__global__ __launch_bounds__(256) void k_retry_tables(InfraParams p) { build_tables_entry(p); }

hipError_t launch_build_tables(const InfraParams &p, u32 grid, bool retry, hipStream_t stream)
{
    if (p.batch == 0 || grid == 0) return hipSuccess;
    if (p.tsize > kTableMax || p.tsize < kGroup || p.tsize % kGroup != 0) return hipErrorInvalidValue;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(retry ? k_retry_tables : k_build_tables, dim3(grid), dim3(256), 0, stream, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_giant_square: for each batch position whose window left entries, the
// giant step g = reduce(mu_1^2) and the second giant ideal g2 = reduce(g^2),
// both by NUDUPL, with their residues.  Every lane runs the same squarings
// (only the Euclid loops' lengths differ).  This keeps squarings out of the
// giant walk, whose lanes are at different giant steps: composed by NUCOMP,
// the square g g would take NUCOMP's gcd branch with the full norm as gcd,
// whose long extended Euclid the whole wave would wait for.  The d's task
// (position, item, g, g2) goes into its cost bucket (below).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double isqrt_f64(double x)
{
    // floor(sqrt(x)) for integer-valued 0 <= x < 2^52, corrected exactly
    double r = floor(sqrt(x));
    if ((r + 1.0) * (r + 1.0) <= x)
        r += 1.0;
    else if (r * r > x)
        r -= 1.0;
    return r;
}

// Cost order.  A d's giant walk is about R / log g giant steps long, R its
// regulator, and by the analytic class number formula h R = sqrt(d)
// L(1, chi_d) / 2.  In a persistent walk that takes the d's in list order,
// the long walks that start late leave most lanes idle at the end.  The
// estimate below orders the d's by L(1, chi_d) / h instead: the Euler
// factors p / (p - chi(p)) of L at the odd primes up to 97 (chi(p) the
// Legendre symbol (d/p)) and a factor 1/2 for each of these primes that
// divides d (each prime factor of d beyond the first adds one to the 2-rank
// of the narrow class group, by genus theory).  Its distribution over D
// depends only on d modulo these primes, so it is the same at every height;
// the bucket edges are its eighths over D (log scale).  The estimate only
// orders the work: every order gives the same results.
constexpr u32 kCostPrimes[24] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                 43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};
struct QrMasks {
    u64 m[24][2];  // bit r set iff r is a nonzero square mod the prime
};
constexpr QrMasks make_qr_masks()
{
    QrMasks t{};
    for (int i = 0; i < 24; i++) {
        const u32 pr = kCostPrimes[i];
        for (u32 x = 1; x < pr; x++) {
            const u32 r = x * x % pr;
            t.m[i][r >> 6] |= 1ull << (r & 63);
        }
    }
    return t;
}
constexpr QrMasks kQrMasks = make_qr_masks();
constexpr float kCostEdges[kCostBuckets - 1] = {0.236f, -0.124f, -0.400f, -0.660f,
                                                 -0.930f, -1.237f, -1.674f};

__device__ __forceinline__ u32 cost_bucket(u64 d)
{
    const double dd = (double)d;  // d < 2^53: exact
    float f = 1.f;
#pragma unroll
    for (int i = 0; i < 24; i++) {
        const double pr = (double)kCostPrimes[i];
        const double q = floor(dd * (1.0 / pr));
        double r = fma(-q, pr, dd);  // exact; within one p of d mod p
        r = (r < 0.0) ? r + pr : r;
        r = (r >= pr) ? r - pr : r;
        const u32 ri = (u32)r;
        const u64 lo = kQrMasks.m[i][0], hi = kQrMasks.m[i][1];  // immediates
        const u64 mw = (ri < 64) ? lo : hi;
        const bool sq = (mw >> (ri & 63)) & 1ull;
        const float up = (float)(pr / (pr - 1.0)), down = (float)(pr / (pr + 1.0));
        f *= (ri == 0) ? 0.5f : (sq ? up : down);
    }
    const float e = __logf(f);
    u32 b = 0;
#pragma unroll
    for (u32 k = 0; k < kCostBuckets - 1; k++) b += (e < kCostEdges[k]) ? 1u : 0u;
    return b;
}

// Positions per thread.  A workgroup handles 256 kSquarePerThread positions
// and reserves its tasks' slots with one atomic per bucket: device-wide
// atomics on the same counter are serialised, so one reservation per 256
// positions would cost more than the squarings.
constexpr u32 kSquarePerThread = 4;

__device__ __forceinline__ void giant_square_body(InfraParams p)
{
    {
        const u32 total = p.list_ctr->list_len;  // workgroups past the batch's end leave
        if (p.k0 >= total || blockIdx.x * (256u * kSquarePerThread) >= total - p.k0) return;
    }
    __shared__ SegLds segs[kMaxSegments];
    __shared__ u32 bcount[kCostBuckets], bbase[kCostBuckets];
    if (threadIdx.x < kCostBuckets) bcount[threadIdx.x] = 0u;
    load_segs(segs, p.segs, p.nseg);  // ends with a barrier
    const u32 total = p.list_ctr->list_len;
    const u32 n = (p.k0 < total) ? min(p.batch, total - p.k0) : 0u;
    const u32 pos0 = blockIdx.x * (256u * kSquarePerThread) + threadIdx.x;
    // Phase 1: the bucket of each position that takes giant steps and its
    // rank there within the workgroup (packed: rank << 8 | bucket; 0xff =
    // no task); then one reservation per bucket.
    u32 slot[kSquarePerThread];
#pragma unroll
    for (u32 j = 0; j < kSquarePerThread; j++) {
        const u32 pos = pos0 + 256u * j;
        slot[j] = 0xffu;
        if (pos < n) {
            const WindowState st = p.state[pos];
            if (st.count != 0u) {
                const u32 b = cost_bucket(item_d(segs, st.item));
                slot[j] = (atomicAdd(&bcount[b], 1u) << 8) | b;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kCostBuckets)
        bbase[threadIdx.x] = bcount[threadIdx.x] ? atomicAdd(&p.gbuckets[16 * threadIdx.x], bcount[threadIdx.x]) : 0u;
    __syncthreads();
    // Phase 2: the squarings, each task written to its slot.  A failed check
    // leaves the task in its bucket; the walk hands it to the plain walk.
#pragma unroll 1
    for (u32 j = 0; j < kSquarePerThread; j++) {
        if (slot[j] == 0xffu) continue;
        const u32 pos = pos0 + 256u * j;
        const WindowState st = p.state[pos];
        const u32 e1 = st.emain - 1;
        const unsigned long long m1 = p.lists[(u64)pos * p.emax + e1];
        const u32 m1S = (p.lres[(u64)pos * p.emax + e1] >> 1) % 3u;
        const u64 d = item_d(segs, st.item);
        double s, P1, Q1;
        u32 S1;
        first_step(d, s, P1, Q1, S1);
        const double dd = (double)d;
        const double L = isqrt_f64(s);
        GiantTask out;
        Chk ck;
        GiantWork wk;
        // g = reduce(mu_1^2), then g2 = reduce(g^2): log g = 2 log mu_1 - log
        // gamma + the residues of the reduction steps, and likewise for g2.
        // With the paper's stride the step is mu_1 itself (its predecessor
        // Q' = (d - P^2)/Q exact in fp64) and g2 = reduce(mu_1^2).
        double uQ = 4.0 * (double)__uint_as_float((u32)(m1 >> 32)), uP = 4.0 * (double)__uint_as_float((u32)m1);
        u32 uS = m1S;
        const bool stride1 = (p.variant & kVariantNoConjugate) != 0;
        const bool snp = (p.variant & kVariantNoSmallNorm) == 0;
        if (stride1) {
            const double Qp = ex_div(fma(-uP, uP, dd), uQ, ck);
            out.g.Q4 = (float)uQ * 0.25f;
            out.g.P4 = (float)uP * 0.25f;
            out.g.Qp4 = (float)Qp * 0.25f;
            out.g.S = uS;
        }
#pragma unroll 1
        for (int k = stride1 ? 1 : 0; k < 2; k++) {
            Form f3;
            Gamma gm;
            square_ideal(uQ, uP, dd, L, f3, gm, ck, wk, snp);
            const u32 lg = gamma_log(gm, ck);
            double Qk, Pk, Qpk;
            const u32 Sr = reduce_form(f3, dd, s, Qk, Pk, Qpk, ck, wk);
            GiantIdeal &gi = (k == 0) ? out.g : out.g2;
            gi.Q4 = (float)Qk * 0.25f;
            gi.P4 = (float)Pk * 0.25f;
            gi.Qp4 = (float)Qpk * 0.25f;
            gi.S = (2u * uS + 3u - lg + Sr) % 3u;
            uQ = Qk;
            uP = Pk;
            uS = gi.S;
        }
        out.pos = pos;
        out.item = st.item;
        out.s4 = (float)s * 0.25f;
        out.L = (float)L;
        if (ck.bad()) out.g.S = kSquareBad;
        const u32 b = slot[j] & 0xffu;
        p.tasks[(u64)b * p.task_cap + bbase[b] + (slot[j] >> 8)] = out;
    }
}

__global__ __launch_bounds__(256) void k_giant_square(InfraParams p) { giant_square_body(p); }
__global__ __launch_bounds__(256) void k_retry_square(InfraParams p) { giant_square_body(p); }

hipError_t launch_giant_square(const InfraParams &p, bool retry, hipStream_t stream)
{
    if (p.batch == 0) return hipSuccess;
    const u32 per_block = 256u * kSquarePerThread;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(retry ? k_retry_square : k_giant_square, dim3((p.batch + per_block - 1) / per_block),
                       dim3(256), 0, stream, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_walk_giant
// ---------------------------------------------------------------------------
constexpr u32 kNoEntry = ~0u;

// Lookup of the window entries with keys (qb, pa) and (qb, pc) in a d's
// table of `groups` groups: their indices and residue sums, or kNoEntry.  Split in
// two so that the loads of the two home groups are issued well before their
// values are needed (their latency then hides behind the composition).  A
// group's first slot with the key's fingerprint is confirmed against the
// full key in the list, whose residue sum is loaded with it; the rest (a
// false first candidate with another after it, or a full group without the
// key) goes on group by group, in a branch the wave takes only when one of
// its lanes needs it.
struct DictProbe {
    unsigned long long ka, kc;  // the two keys
    u32 fa, fc;                 // their fingerprints, shifted to the slot's field
    u32 ga, gc;                 // the first slots of their home groups
    uint4 va, vc;               // the home groups (loads in flight)
};

__device__ __forceinline__ DictProbe dict_start2(const u16 *tbl, u32 groups, u32 qb, u32 pa, u32 pc)
{
    DictProbe d;
    d.ka = ((unsigned long long)qb << 32) | pa;
    d.kc = ((unsigned long long)qb << 32) | pc;
    const u32 ha = dict_hash(qb, pa), hc = dict_hash(qb, pc);
    d.fa = slot_fp(ha) << kSlotIndexBits;
    d.fc = slot_fp(hc) << kSlotIndexBits;
    d.ga = home_group(ha, groups) * kGroup;
    d.gc = home_group(hc, groups) * kGroup;
    d.va = *reinterpret_cast<const uint4 *>(tbl + d.ga);
    d.vc = *reinterpret_cast<const uint4 *>(tbl + d.gc);
    return d;
}

// Slots of group g whose fingerprint field is f: bit 8 i + 7 is set for
// slot i (empty slots never match, fingerprints being nonzero).  In each
// 32-bit word, x = word ^ f in both fields, bit 15 of a field of
// ((x & 0x7e00) + 0x7e00) | x is set iff the field's fingerprint bits 9-15
// differ from f's (the sum carries into bit 15 iff one of bits 9-14 of x is
// set, and never out of the field); a byte permute gathers the high byte of
// every field, slot order kept.
__device__ __forceinline__ unsigned long long group_match(uint4 g, u32 f)
{
    const u32 pat = f | (f << 16);
    auto differs = [pat](u32 w) {
        const u32 x = w ^ pat;
        return ((x & 0x7e007e00u) + 0x7e007e00u) | x;
    };
    // result bytes: byte 1 and byte 3 of the low word, then of the high word
    const u32 lo = __builtin_amdgcn_perm(differs(g.y), differs(g.x), 0x07050301u);
    const u32 hi = __builtin_amdgcn_perm(differs(g.w), differs(g.z), 0x07050301u);
    return ~(((unsigned long long)hi << 32) | lo) & 0x8080808080808080ull;
}

// the lowest set bit of m (m != 0)
__device__ __forceinline__ u32 low_bit(unsigned long long m) { return (u32)__builtin_ctzll(m); }

// Whether group g has an empty slot.  A group's entries fill its first
// slots (insertion takes the group's next position), so its last slot tells.
__device__ __forceinline__ bool group_open(uint4 g) { return g.w < 0x10000u; }

// list entry of the slot whose match bit is b (= 8 i + 7 for slot i)
__device__ __forceinline__ u32 group_entry(uint4 g, u32 b)
{
    const unsigned long long h = (b >= 32u) ? (((unsigned long long)g.w << 32) | g.z)
                                            : (((unsigned long long)g.y << 32) | g.x);
    return ((u32)(h >> ((b << 1) & 0x30u)) & kSlotIndexMask) - 1u;
}

// Group by group from slot s (a home group's first): the entry with key k
// and fingerprint field f and its residue sum r, or kNoEntry.
__device__ __forceinline__ u32 dict_scan(const u16 *tbl, const unsigned long long *lst,
                                         const u32 *lres, u32 tsize, u32 s, u32 f,
                                         unsigned long long k, u32 &r)
{
    for (u32 t = 0; t < tsize / kGroup; t++) {
        const uint4 g = *reinterpret_cast<const uint4 *>(tbl + s);
        for (unsigned long long m = group_match(g, f); m != 0ull; m &= m - 1ull) {
            const u32 e = group_entry(g, low_bit(m));
            if (lst[e] == k) {
                r = lres[e];
                return e;
            }
        }
        if (group_open(g)) break;
        s += kGroup;
        if (s == tsize) s = 0;
    }
    return kNoEntry;
}

__device__ __forceinline__ void dict_finish2(const u16 *tbl, const unsigned long long *lst,
                                             const u32 *lres, u32 tsize, const DictProbe &d,
                                             u32 &ea, u32 &ec, u32 &ra, u32 &rc)
{
    const unsigned long long ma = group_match(d.va, d.fa), mc = group_match(d.vc, d.fc);
    const bool ha = ma != 0ull, hc = mc != 0ull;
    // the first candidates, their list keys and residue sums loaded together
    const u32 ca = ha ? group_entry(d.va, low_bit(ma)) : 0u;
    const u32 cc = hc ? group_entry(d.vc, low_bit(mc)) : 0u;
    unsigned long long la = 0, lc = 0;
    ra = rc = 0u;
    if (ha) {
        la = lst[ca];
        ra = lres[ca];
    }
    if (hc) {
        lc = lst[cc];
        rc = lres[cc];
    }
    ea = (ha && la == d.ka) ? ca : kNoEntry;
    ec = (hc && lc == d.kc) ? cc : kNoEntry;
    const bool slowa = ea == kNoEntry && ((ma & (ma - 1ull)) != 0ull || !group_open(d.va));
    const bool slowc = ec == kNoEntry && ((mc & (mc - 1ull)) != 0ull || !group_open(d.vc));
    if (__builtin_amdgcn_ballot_w64(slowa || slowc)) {
        if (slowa) ea = dict_scan(tbl, lst, lres, tsize, d.ga, d.fa, d.ka, ra);
        if (slowc) ec = dict_scan(tbl, lst, lres, tsize, d.gc, d.fc, d.kc, rc);
    }
}

// The giant walk keeps a pool of kPoolSlots d's per wave in LDS and runs
// them in phases that every lane of the wave takes part in, instead of one d
// per lane with the lanes at different stages:
//   compose phase  up to 64 d's whose walk stands at a distinguished ideal:
//                  each lane looks that ideal up (itself and its
//                  conjugate), and on a miss composes the d's next giant
//                  ideal c_{k+1} = reduce(g c_k) by NUCOMP (or, after the
//                  first lookup, takes the precomputed second giant ideal);
//   walk phase     up to 64 walking d's: each lane takes at most walk_chunk
//                  reduction steps towards the next distinguished ideal.
// A phase runs once 64 d's are ready for it (else the fuller queue runs), so
// that NUCOMP, the costliest part, runs with every lane busy, and a long
// walk holds up only its own lane for one chunk.  The d's move between
// three rings of slot numbers (free, compose, walk) whose heads and tails
// only this wave touches: no barrier, no LDS atomic.  Free slots are filled
// from the queue over the squaring kernel's tasks, bucket 0 (longest
// estimated walks) first.
constexpr u32 kPoolSlots = 128;  // d's per wave (a power of two)
constexpr u32 kPoolMask = kPoolSlots - 1;

// Structure of arrays, indexed by slot: a walk phase touches only the walk
// fields.  pk packs the residues (bits 0-1 of g, 2-3 of c_k, 4-5 of the walk,
// 6-7 of g2) and the walk's step count (bits 8-20).
struct GiantPool {
    u32 pos[kPoolSlots], item[kPoolSlots], ng[kPoolSlots], pk[kPoolSlots];
    float sq[kPoolSlots], L[kPoolSlots];
    float m1Q[kPoolSlots], m1P[kPoolSlots];           // the giant step g
    float cQ[kPoolSlots], cP[kPoolSlots];             // the current giant ideal c_k
    float Qw[kPoolSlots], Pw[kPoolSlots], Qpw[kPoolSlots];  // the walk from it
    float g2Q[kPoolSlots], g2P[kPoolSlots], g2Qp[kPoolSlots];  // the second giant ideal
    unsigned char ring[3][kPoolSlots];               // free, compose, walk
};
constexpr u32 kRingFree = 0, kRingCompose = 1, kRingWalk = 2;

__device__ __forceinline__ u32 pk_make(u32 m1S, u32 cS, u32 Sw, u32 g2S, u32 w)
{
    return m1S | (cS << 2) | (Sw << 4) | (g2S << 6) | (w << 8);
}

// number of lanes below this one in mask m
__device__ __forceinline__ u32 lanes_below(u64 m)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}

template <bool kCheck>
__device__ __forceinline__ void walk_giant_body(const InfraParams &p, const SegLds *segs,
                                                const u32 *bstart, GiantPool *pools)
{
    const u32 n = bstart[kCostBuckets];
    auto task_of = [&](u32 q) -> const GiantTask * {
        u32 b = 0;
#pragma unroll
        for (u32 k = 1; k < kCostBuckets; k++) b += (q >= bstart[k]) ? 1u : 0u;
        return p.tasks + (u64)b * p.task_cap + (q - bstart[b]);
    };
    GiantPool &pl = pools[threadIdx.x >> 6];
    const u32 lane = __lane_id();
    // reduction steps per walk phase (a tuned shape parameter), even
    const u32 chunk = __builtin_amdgcn_readfirstlane((min(max(p.walk_chunk, 2u), 64u) + 1u) & ~1u);
    const u32 tgroups = p.tsize / kGroup;  // table groups per d
    // ring heads and tails (wave-uniform); every slot starts free
    u32 head[3] = {0u, 0u, 0u}, tail[3] = {kPoolSlots, 0u, 0u};
    for (u32 s = lane; s < kPoolSlots; s += 64) pl.ring[kRingFree][s] = (unsigned char)s;
    auto push = [&](u32 r, bool f, u32 slot) {
        const u64 m = __builtin_amdgcn_ballot_w64(f);
        if (f) pl.ring[r][(tail[r] + lanes_below(m)) & kPoolMask] = (unsigned char)slot;
        tail[r] += (u32)__builtin_popcountll(m);
    };
    auto handoff = [&](u32 item) {
        const u32 f = atomicAdd(&p.fb_ctr->list_len, 1u);
        p.fb_list[f] = item;
    };
    bool drained = false;
    u32 cbase = 0, cend = 0;  // the wave's claimed chunk of the task queue
    u32 my_giants = 0, my_comps = 0, my_eu = 0, my_xg = 0, my_red = 0, my_gcdb = 0, my_looks = 0;
    u64 my_steps = 0;
    // phases run (compose, walk) and the lanes they kept busy (wave-uniform)
    u32 phases[2] = {0u, 0u}, lanes_on[2] = {0u, 0u};

    for (;;) {
        u32 nfree = tail[kRingFree] - head[kRingFree];
        u32 nc = tail[kRingCompose] - head[kRingCompose];
        u32 nw = tail[kRingWalk] - head[kRingWalk];
        // ---- refill: new d's into free slots, each starting its walk at g
        if (!drained && (nfree >= 64 || (nfree > 0 && nc < 64 && nw < 64))) {
            const bool want = lane < nfree;
            u32 q = n;
            wave_take(p.giant_next, n, want, q, cbase, cend);
            drained = __any(want && q >= n);
            bool take = false;
            GiantTask t;
            if (q < n) {
                t = *task_of(q);
                if (t.g.S == kSquareBad) {
                    handoff(t.item);
                    my_giants += 1;
                } else {
                    take = true;
                }
            }
            const u64 mt = __builtin_amdgcn_ballot_w64(take);
            if (take) {
                const u32 s = pl.ring[kRingFree][(head[kRingFree] + lanes_below(mt)) & kPoolMask];
                pl.pos[s] = t.pos;
                pl.item[s] = t.item;
                pl.ng[s] = 1u;
                pl.pk[s] = pk_make(t.g.S, t.g.S, t.g.S, t.g2.S, 0u);
                pl.sq[s] = t.s4;
                pl.L[s] = t.L;
                pl.m1Q[s] = t.g.Q4;
                pl.m1P[s] = t.g.P4;
                pl.cQ[s] = t.g.Q4;
                pl.cP[s] = t.g.P4;
                pl.Qw[s] = t.g.Q4;
                pl.Pw[s] = t.g.P4;
                pl.Qpw[s] = t.g.Qp4;
                pl.g2Q[s] = t.g2.Q4;
                pl.g2P[s] = t.g2.P4;
                pl.g2Qp[s] = t.g2.Qp4;
                pl.ring[kRingWalk][(tail[kRingWalk] + lanes_below(mt)) & kPoolMask] = (unsigned char)s;
            }
            const u32 nt = (u32)__builtin_popcountll(mt);
            head[kRingFree] += nt;
            tail[kRingWalk] += nt;
            nw += nt;
        }
        if (nc == 0 && nw == 0) {
            if (drained) break;
            continue;
        }
        const bool compose = nc >= 64 || (nw < 64 && nc >= nw);
        if (compose) {
            // ---- lookup + compose phase -------------------------------------
            // Two lookups at once: the ideal (Q_m, P_m) itself -- a hit means
            // one period past a window ideal -- and its conjugate (Q_m,
            // P_{m+1}) -- a hit means as many ideals short of a period as the
            // window ideal lies past (1) (conjugation reverses the cycle and
            // acts as log -> -log, so log eps = S_m + S_i).  A direct hit at
            // the first lookup (g itself) is skipped: g may lie inside the
            // window (a "unit" of distance 0); if it was a true hit, a later
            // one is at eps or eps^2, whose residues are both 0 or both not.
            // The first probe's loads are issued before the composition,
            // which is computed for every lane that may need it (a lane whose
            // lookup then hits drops it), so that NUCOMP hides their latency.
            const bool on = lane < nc;
            u32 s = 0;
            if (on) s = pl.ring[kRingCompose][(head[kRingCompose] + lane) & kPoolMask];
            head[kRingCompose] += min(nc, 64u);
            phases[0]++;
            lanes_on[0] += min(nc, 64u);
            u32 ng = 0, pk = 0, item = 0, pos = 0;
            DictProbe dp;
            if (on) {
                ng = pl.ng[s];
                pk = pl.pk[s];
                item = pl.item[s];
                pos = pl.pos[s];
                const float sq = pl.sq[s], sqc = sq * kQuotBias;
                const float Qw = pl.Qw[s], Pw = pl.Pw[s], Qpw = pl.Qpw[s];
                float Pn, Qn, acc1 = 0.f;
                rho_step_q<kCheck>(sq, sqc, Pw, Qw, Qpw, Pn, Qn, acc1);
                dp = dict_start2(p.tables + (u64)pos * p.tsize, tgroups, __float_as_uint(Qw),
                                 __float_as_uint(Pw), __float_as_uint(Pn));
            }
            const bool comp = on && ng > 1 && ng < p.max_giants;
            bool cbad = false;
            GiantWork cwk;  // the composition's work, counted when it is used
            float cQ4 = 0.f, cP4 = 0.f, cQp4 = 0.f;
            u32 Sk = 0;
            if (comp) {
                Form f3;
                Gamma gm;
                Chk ck;
                GiantWork wk;
                const double dd = (double)item_d(segs, item);
                const float sq = pl.sq[s];
                compose_ideals(4.0 * (double)pl.m1Q[s], 4.0 * (double)pl.m1P[s], 4.0 * (double)pl.cQ[s],
                               4.0 * (double)pl.cP[s], dd, (double)pl.L[s], f3, gm, ck, wk,
                               (p.variant & kVariantNoSmallNorm) == 0);
                const u32 lg = gamma_log(gm, ck);
                double Qk, Pk, Qpk;
                const u32 Sr = reduce_form(f3, dd, 4.0 * (double)sq, Qk, Pk, Qpk, ck, wk);
                cwk = wk;
                Sk = ((pk & 3u) + ((pk >> 2) & 3u) + 3u - lg + Sr) % 3u;
                cbad = ck.bad();
                cQ4 = (float)Qk * 0.25f;
                cP4 = (float)Pk * 0.25f;
                cQp4 = (float)Qpk * 0.25f;
            }
            bool gone = false, next_walk = false;
            if (on) {
                u32 ed, ec, rd, rc;
                dict_finish2(p.tables + (u64)pos * p.tsize, p.lists + (u64)pos * p.emax,
                             p.lres + (u64)pos * p.emax, p.tsize, dp, ed, ec, rd, rc);
                my_looks++;
                const u32 Sw = (pk >> 4) & 3u;
                bool done = false, flag = false;
                if (ed != kNoEntry && ng > 1) {
                    const u32 St = (rd >> 1) % 3u;
                    flag = ((Sw + 3u - St) % 3u) == 0u;
                    done = true;
                } else if (ec != kNoEntry && !(p.variant & kVariantNoConjugate)) {
                    const u32 St = (rc >> 1) % 3u;
                    flag = ((Sw + St) % 3u) == 0u;
                    done = true;
                }
                if (done) {
                    emit_flag(p.eis_words, item_bit(segs, item), flag);
                    my_giants += ng;
                    gone = true;
                } else if (ng == 1) {
                    // the second giant ideal, squared beforehand
                    const float gQ = pl.g2Q[s], gP = pl.g2P[s];
                    const u32 gS = (pk >> 6) & 3u;
                    pl.cQ[s] = gQ;
                    pl.cP[s] = gP;
                    pl.Qw[s] = gQ;
                    pl.Pw[s] = gP;
                    pl.Qpw[s] = pl.g2Qp[s];
                    pl.pk[s] = pk_make(pk & 3u, gS, gS, gS, 0u);
                    pl.ng[s] = 2u;
                    next_walk = true;
                } else if (!comp || cbad) {
                    // the giant-step budget is spent, or a check failed
                    handoff(item);
                    my_giants += ng;
                    gone = true;
                } else {
                    my_comps++;
                    my_eu += cwk.euclid;
                    my_xg += cwk.xgcd;
                    my_red += cwk.reduce;
                    my_gcdb += cwk.gcd_branch;
                    pl.cQ[s] = cQ4;
                    pl.cP[s] = cP4;
                    pl.Qw[s] = cQ4;
                    pl.Pw[s] = cP4;
                    pl.Qpw[s] = cQp4;
                    pl.pk[s] = pk_make(pk & 3u, Sk, Sk, (pk >> 6) & 3u, 0u);
                    pl.ng[s] = ng + 1u;
                    next_walk = true;
                }
            }
            push(kRingWalk, next_walk, s);
            push(kRingFree, gone, s);
        } else {
            // ---- walk phase -------------------------------------------------
            const bool on = lane < nw;
            u32 s = 0;
            if (on) s = pl.ring[kRingWalk][(head[kRingWalk] + lane) & kPoolMask];
            head[kRingWalk] += min(nw, 64u);
            phases[1]++;
            lanes_on[1] += min(nw, 64u);
            bool at_dp = false, gone = false, more = false;
            if (on) {
                const float sq = pl.sq[s], sqc = sq * kQuotBias;
                // Two steps per iteration on fixed registers: the next Q
                // overwrites the previous one (Q_{j+1} = Q_{j-1} + q (P_j -
                // P_{j+1})), so Qa and Qb swap roles every step, and so do Pa
                // and Pb; nothing is copied.  After an odd number of steps the
                // current ideal is (Pb, Qb).
                float Pa = pl.Pw[s], Pb = 0.f, Qa = pl.Qw[s], Qb = pl.Qpw[s];
                const u32 pk = pl.pk[s];
                u32 u = 0;
                float acc = 0.f;
                bool run = !is_dp(Qa);
                for (u32 k = 0; k < chunk; k += 2) {
                    if (run) {
                        rho_step_q<kCheck>(sq, sqc, Pa, Qa, Qb, Pb, Qb, acc);
                        u++;
                        run = !is_dp(Qb);
                    }
                    if (run) {
                        rho_step_q<kCheck>(sq, sqc, Pb, Qb, Qa, Pa, Qa, acc);
                        u++;
                        run = !is_dp(Qa);
                    }
                    if (!__any(run)) break;
                }
                const bool odd = (u & 1u) != 0u;
                const float Qw = odd ? Qb : Qa, Qpw = odd ? Qa : Qb, Pw = odd ? Pb : Pa;
                const u32 Sw = (((pk >> 4) & 3u) + ((u + (u32)acc) >> 1)) % 3u;
                const u32 w = (pk >> 8) + u;
                my_steps += u;
                at_dp = !run;
                if (!at_dp && w >= kWalkLimit) {
                    handoff(pl.item[s]);
                    my_giants += pl.ng[s];
                    gone = true;
                } else {
                    pl.Qw[s] = Qw;
                    pl.Pw[s] = Pw;
                    pl.Qpw[s] = Qpw;
                    pl.pk[s] = (pk & 0xcfu) | (Sw << 4) | (w << 8);
                    more = !at_dp;
                }
            }
            push(kRingCompose, at_dp, s);
            push(kRingWalk, more, s);
            push(kRingFree, gone, s);
        }
    }
    u64 sums[7] = {my_giants, my_comps, my_eu, my_red, my_gcdb, my_looks, my_xg};
    for (int off = 32; off > 0; off >>= 1) {
        my_steps += __shfl_down(my_steps, off, 64);
#pragma unroll
        for (int k = 0; k < 7; k++) sums[k] += __shfl_down(sums[k], off, 64);
    }
    if (lane == 0) {
        atomicAdd(&p.ctr->chunk_steps, (unsigned long long)my_steps);
        atomicAdd(&p.ctr->giant_steps, (unsigned long long)sums[0]);
        atomicAdd(&p.ctr->giant_comps, (unsigned long long)sums[1]);
        atomicAdd(&p.ctr->giant_euclid, (unsigned long long)sums[2]);
        atomicAdd(&p.ctr->giant_reduce, (unsigned long long)sums[3]);
        atomicAdd(&p.ctr->giant_gcd_branch, (unsigned long long)sums[4]);
        atomicAdd(&p.ctr->giant_lookups, (unsigned long long)sums[5]);
        atomicAdd(&p.ctr->giant_xgcd, (unsigned long long)sums[6]);
        for (int k = 0; k < 2; k++) {
            atomicAdd(&p.ctr->giant_phases[k], (unsigned long long)phases[k]);
            atomicAdd(&p.ctr->giant_lanes[k], (unsigned long long)lanes_on[k]);
        }
    }
}

__device__ __forceinline__ void walk_giant_entry(const InfraParams &p)
{
    if (p.k0 >= p.list_ctr->list_len) return;  // nothing in this batch (an empty retry)
    __shared__ SegLds segs[kMaxSegments];
    __shared__ u32 bstart[kCostBuckets + 1];  // queue index of each bucket's first task
    __shared__ GiantPool pools[4];
    if (threadIdx.x == 0) {
        u32 acc = 0;
        for (u32 b = 0; b < kCostBuckets; b++) {
            bstart[b] = acc;
            acc += p.gbuckets[16 * b];
        }
        bstart[kCostBuckets] = acc;
    }
    load_segs(segs, p.segs, p.nseg);  // ends with a barrier
    if (p.exact_quot)
        walk_giant_body<false>(p, segs, bstart, pools);
    else
        walk_giant_body<true>(p, segs, bstart, pools);
}

__global__ __launch_bounds__(256) void k_walk_giant(InfraParams p) { walk_giant_entry(p); }
__global__ __launch_bounds__(256) void k_retry_giant(InfraParams p) { walk_giant_entry(p); }

hipError_t launch_walk_giant(const InfraParams &p, u32 grid, bool retry, hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    // lookups read whole 16-byte groups of the tables
    if (p.tsize > kTableMax || p.tsize < kGroup || p.tsize % kGroup != 0) return hipErrorInvalidValue;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(retry ? k_retry_giant : k_walk_giant, dim3(grid), dim3(256), 0, stream, p);
    return hipGetLastError();
}

int walk_giant_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_giant, 256, 0) != hipSuccess)
        return 2;
    return nb > 0 ? nb : 1;
}

}  // namespace eis
