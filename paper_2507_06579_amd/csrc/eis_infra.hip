// eis_infra.hip -- the infrastructure method of Appendix A on gfx950.
//
// Algorithm "Infrastructure" with the generators carried in
// (O_K/2O_K)^* ~ Z/3, split into three kernels so that every lane of a wave
// runs the same phase:
//
//   k_walk_window  one d per lane: reduction steps from (1), with the
//                  half-period symmetry exit; the "distinguished" ideals of
//                  the walk (Q = 2 mod 64, about one in 16) are appended to
//                  the d's dictionary list (the ideal's (Q/4, P/4) as fp32
//                  bits, and twice its residue sum beside it).  mu_1 is the n-th distinguished
//                  ideal (n = wscale * d^(1/4) / 16, at least 16); the
//                  window ends at the first distinguished ideal at least six
//                  steps after mu_1 (the two extra ideals of the algorithm,
//                  with margin), and that extension must stay within a
//                  quarter of mu_1's step count.
//   k_build_tables one wave per d: the list is indexed by an open-addressed
//                  hash table of 32-bit slots (list index + 16-bit
//                  fingerprint; a fingerprint match is confirmed against the
//                  list entry), built in LDS and written out whole.
//   k_walk_giant   one d per lane, lanes refilled from a queue: mu_k =
//                  reduce(mu_1 * mu_{k-1}) (NUDUPL for k = 2, then NUCOMP),
//                  the residue updated with log mu_1 + log mu_{k-1} - log gamma
//                  + the residues of the reduction steps; then reduction steps
//                  forward to the first distinguished ideal, which is looked
//                  up.  A hit gives log eps = log(ideal) - log(stored ideal).
//
// Why the distinguished ideals: a dictionary with every window ideal would
// cost one scattered 8-byte store per reduction step.  With only every 16th
// ideal stored, the stores are rare and the tables small, at the price of a
// short walk after every giant step.  Correctness is unchanged: giant steps
// advance by at most the distance of mu_1 plus the few reduction steps of
// the composition, so the first giant ideal past a full period lies at most
// (position of mu_1 + 6) ideals past (1), and the first distinguished ideal
// at or after it is in the dictionary.  A hit at k = 2 is skipped: when the
// window is short, mu_2 can land inside the window itself, which reads as a
// "unit" of distance 0.  From k = 3 on, the giant ideals lie beyond the
// window's short extension, so a hit is at one regulator, or at two when the
// skipped k = 2 hit was a true one; log eps^2 = 2 log eps is 0 in Z/3 exactly
// when log eps is, so the flag is the same.
//
// Any arithmetic check that fails (fp64 exactness, exact divisions, step or
// walk budgets, table overflow) sends the d to the plain walk, which is exact
// for every d below 10^12.
#include "eis_giant.h"
#include "eis_internal.h"
#include "eis_walk.h"

namespace eis {

// Q = 2 (mod 64), tested on the quarter-unit value Q/4: fract(Q/64) = 1/32
// exactly for integer-valued Q < 2^24.
constexpr float kDpScale = 1.0f / 16.0f;
constexpr float kDpHit = 2.0f / 64.0f;
__device__ __forceinline__ bool is_dp(float Q4) { return __builtin_amdgcn_fractf(Q4 * kDpScale) == kDpHit; }

constexpr u32 kTableMax = 1024;     // largest table (slots) per d
constexpr u32 kWalkLimit = 4096;    // reduction steps from a giant ideal to a distinguished one
constexpr u32 kWalkChunk = 24;      // of which one iteration of the giant walk takes at most this many
constexpr u32 kExtraSteps = 6;      // window runs at least this far past mu_1
constexpr u32 kMinMain = 16;        // mu_1 is at least the 16th distinguished ideal

// dictionary key of a reduced ideal: its quarter-unit (Q, P) as fp32 bits
__device__ __forceinline__ unsigned long long entry_of(float Q4, float P4)
{
    return ((unsigned long long)__float_as_uint(Q4) << 32) | (unsigned long long)__float_as_uint(P4);
}

// ---------------------------------------------------------------------------
// k_walk_window: a wave takes a tile of 64 consecutive batch positions, one d
// per lane, and keeps it until every lane's window has ended, so that the
// 64 lanes append to one tile of the list array (tile-interleaved layout:
// the writes of a wave stay within one small region of memory).
// ---------------------------------------------------------------------------
// Window bookkeeping of one reduction step that landed on (Q, P) (quarter
// units): append a distinguished ideal to the list -- entry cnt of this lane
// of the tile at lt[64 cnt + lane], twice its residue sum at rt[...] -- and
// note the step jc = jb + k of the last entry and, for mu_1 (the emain-th
// entry), the step from which an entry ends the window (jc + kExtraSteps).
// S2k + acc is twice the residue sum up to this step.
__device__ __forceinline__ void window_insert(unsigned long long *lt, u32 *rt, u32 lane, float Q,
                                              float P, u32 S2k, float acc, u32 jb, u32 k,
                                              u32 emain, u32 &cnt, u32 &j1e, u32 &jlast)
{
    if (is_dp(Q)) {
        const u32 o = cnt * 64u + lane;
        lt[o] = entry_of(Q, P);
        rt[o] = S2k + (u32)acc;
        cnt++;
        jlast = jb + k;
        j1e = (cnt == emain) ? jlast + kExtraSteps : j1e;
    }
}

__global__ __launch_bounds__(256) void k_walk_window(InfraParams p)
{
    const u32 lane = __lane_id();
    const u32 total = p.list_ctr->list_len;
    const u32 nb = (p.k0 < total) ? min(p.batch, total - p.k0) : 0u;
    const u32 ntiles = (nb + 63) / 64;
    const u32 K = __builtin_amdgcn_readfirstlane(min(kInnerChunk, max(p.max_steps, 1u)));
    const u32 cnt_end = p.emax - 1;  // a full list ends the window (then the d goes plain)
    u64 my_steps = 0, my_refills = 0;

    for (;;) {
        u32 t = 0;
        if (lane == 0) t = atomicAdd(p.win_next, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const u32 pos = t * 64 + lane;
        // the tile's list and residue entries (wave-uniform bases)
        unsigned long long *lt = p.lists + (u64)t * p.emax * 64;
        u32 *rt = p.lres + (u64)t * p.emax * 64;
        // walk state in quarter units (see rho_step_q); S2 = twice the
        // residue sum at the start of the current chunk of steps; an entry
        // at step >= j1e ends the window (j1e = step of mu_1 + kExtraSteps)
        float sq = 0.f, sqc = 0.f, P = 0.25f, Q = 0.5f, Qp = 0.5f;
        u32 S2 = 0, j = 0, idx = 0, cnt = 0, emain = kMinMain, j1e = ~0u, jlast = 0;
        bool active = false, to_giant = false, to_plain = false;
        u32 item = 0;
        if (pos < nb) {
            item = p.list[p.k0 + pos];
            idx = item_bit(p.segs, item);
            my_refills++;
            const u64 d = item_d(p.segs, item);
            const u64 si = isqrt_u64(d);
            const u64 P1 = ((si + 1) >> 1) * 2 - 1;
            const u64 Q1 = (d - P1 * P1) >> 1;
            const u32 S1 = 1u + (u32)((P1 >> 1) & 1);
            j = 1;
            if (Q1 == 2) {
                emit_flag(p.eis_words, idx, S1 % 3u == 0u);
            } else {
                sq = (float)si * 0.25f;
                sqc = sq * kQuotBias;
                P = (float)P1 * 0.25f;
                Q = (float)Q1 * 0.25f;
                S2 = 2u * S1;
                // the ideal (1) = [1, (P_1 + sqrt d)/2], residue 0
                lt[lane] = entry_of(0.5f, P);
                rt[lane] = 0u;
                cnt = 1;
                const float n = p.segs[item >> kItemShift].wscale * sqrtf(sqrtf((float)d)) * (1.f / 16.f);
                emain = (u32)fminf(fmaxf(rintf(n), (float)kMinMain), (float)(p.emax - 8));
                window_insert(lt, rt, lane, Q, P, S2, 0.f, 1, 0, emain, cnt, j1e, jlast);
                active = true;
            }
        }
        while (__any(active)) {
            if (active) {
                // Two steps per iteration; the loop leaves as soon as any lane
                // reaches the half-period or the end of its window.  The
                // window ends once an entry at least kExtraSteps past mu_1 is
                // stored (or the list is full).
                u32 k = 0;
                u64 mh = 0, ms = 0;
                bool first_half = false;
                float P1 = 0.f, Q1 = 0.f, acc = 0.f;
                for (;;) {
                    float P2, Q2;
                    rho_step_q(sq, sqc, P, Q, Qp, P1, Q1, acc);
                    mh = __builtin_amdgcn_ballot_w64(Q1 == Q) | __builtin_amdgcn_ballot_w64(P1 == P);
                    window_insert(lt, rt, lane, Q1, P1, S2 + k + 1, acc, j + 1, k, emain, cnt, j1e,
                                  jlast);
                    if (mh) {
                        // the window-end test runs on every exit from the
                        // loop, so that no lane starts a pair with fewer than
                        // two free list entries
                        ms = __builtin_amdgcn_ballot_w64(jlast >= j1e) |
                             __builtin_amdgcn_ballot_w64(cnt >= cnt_end);
                        first_half = true;
                        break;
                    }
                    rho_step_q(sq, sqc, P1, Q1, Q, P2, Q2, acc);
                    mh = __builtin_amdgcn_ballot_w64(Q2 == Q1) | __builtin_amdgcn_ballot_w64(P2 == P1);
                    window_insert(lt, rt, lane, Q2, P2, S2 + k + 2, acc, j + 2, k, emain, cnt, j1e,
                                  jlast);
                    ms = __builtin_amdgcn_ballot_w64(jlast >= j1e) |
                         __builtin_amdgcn_ballot_w64(cnt >= cnt_end);
                    Qp = Q1;
                    Q = Q2;
                    P = P2;
                    k += 2;
                    if ((mh | ms) || k >= K) break;
                }
                if (first_half) {
                    Qp = Q;
                    Q = Q1;
                    P = P1;
                    k += 1;
                }
                j += k;
                S2 += k + (u32)acc;
                if ((mh >> lane) & 1ull) {
                    // half-period symmetry: the unit is found without giant steps
                    const u32 S = S2 >> 1;
                    const u32 rj = __builtin_amdgcn_fractf(P) > 0.5f ? 2u : 1u;
                    const u32 v = (Q == Qp) ? (2u * S - rj) : (2u * (S - rj));
                    emit_flag(p.eis_words, idx, v % 3u == 0u);
                    active = false;
                } else if ((ms >> lane) & 1ull) {
                    // end of the window; its extension past mu_1 must be short
                    // next to mu_1's own distance (see above)
                    const u32 j1 = j1e - kExtraSteps;
                    if (j1e != ~0u && jlast - j1 <= j1 / 4 && cnt < p.emax && S2 < (1u << 24)) {
                        WindowState st;
                        st.emain = emain;
                        st.count = cnt;
                        st.item = item;
                        st.pad = 0;
                        p.state[pos] = st;
                        to_giant = true;
                    } else {
                        to_plain = true;
                    }
                    active = false;
                } else if (j > p.max_steps) {
                    to_plain = true;
                    active = false;
                }
            }
        }
        // hand the tile's d's on, one atomic per wave and list
        if (to_giant) {
            const u32 gslot = atomicAdd(p.giant_len, 1u);
            p.giant_list[gslot] = pos;
        }
        if (to_plain) {
            const u32 f = atomicAdd(&p.fb_ctr->list_len, 1u);
            p.fb_list[f] = item;
        }
        my_steps += j;
    }
    for (int off = 32; off > 0; off >>= 1) {
        my_steps += __shfl_down(my_steps, off, 64);
        my_refills += __shfl_down(my_refills, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&p.ctr->baby_steps, (unsigned long long)my_steps);
        atomicAdd(&p.ctr->refills, (unsigned long long)my_refills);
    }
}

hipError_t launch_walk_window(const InfraParams &p, u32 grid, hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk_window, dim3(grid), dim3(256), 0, stream, p);
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
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_build_tables(InfraParams p)
{
    __shared__ u32 tab[4][kTableMax];
    const u32 nblk = gridDim.x, b = blockIdx.x;
    const u32 xcd = b % 8, q = nblk / 8, r = nblk % 8;
    const u32 lb = xcd * q + min(xcd, r) + b / 8;  // logical block
    const u32 wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const u32 w = lb * 4 + wv;
    const u32 n = *p.giant_len;
    const bool valid = w < n;
    const u32 mask = p.tsize - 1;
    for (u32 t = lane; t < p.tsize; t += 64) tab[wv][t] = 0u;
    __syncthreads();
    u32 pos = 0;
    if (valid) {
        pos = p.giant_list[w];
        const unsigned long long *lst = p.lists + (u64)(pos / 64) * p.emax * 64 + (pos % 64);
        const u32 cnt = p.state[pos].count;
        for (u32 e = lane; e < cnt; e += 64) {
            const unsigned long long ent = lst[(u64)e * 64];
            const u32 qb = (u32)(ent >> 32), pb = (u32)ent;
            const u32 h = dict_hash(qb, pb);
            const u32 val = (e + 1) | (h & 0xffff0000u);
            u32 slot = h & mask;
            for (u32 probe = 0; probe < p.tsize; probe++) {
                const u32 prev = atomicCAS(&tab[wv][slot], 0u, val);
                if (prev == 0u) break;
                slot = (slot + 1) & mask;
            }
        }
    }
    __syncthreads();
    if (valid) {
        u32 *tbl = p.tables + (u64)pos * p.tsize;
        for (u32 t = lane; t < p.tsize; t += 64) tbl[t] = tab[wv][t];
    }
}

hipError_t launch_build_tables(const InfraParams &p, hipStream_t stream)
{
    if (p.batch == 0) return hipSuccess;
    if (p.tsize > kTableMax || (p.tsize & (p.tsize - 1)) != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_tables, dim3((p.batch + 3) / 4), dim3(256), 0, stream, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_walk_giant
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_walk_giant(InfraParams p)
{
    const u32 n = *p.giant_len;
    const u32 mask = p.tsize - 1;
    // per-lane state
    u32 idx = 0, item = 0, ng = 0;
    double dd = 0.0, sd = 0.0, L = 0.0;
    double m1Q = 0.0, m1P = 0.0, cQ = 0.0, cP = 0.0;
    u32 m1S = 0, cS = 0;
    const u32 *tbl = nullptr;
    const unsigned long long *lst = nullptr;
    const u32 *lrs = nullptr;
    float sq = 0.f, sqc = 0.f;
    float Qw = 0.f, Pw = 0.f, Qpw = 0.f;  // walk state, quarter units
    u32 Sw = 0, w = 0;
    bool walking = false;
    u32 cbase = 0, cend = 0;  // the wave's claimed chunk of the queue
    bool active = false, exhausted = false;
    u64 my_giants = 0, my_steps = 0;

    for (;;) {
        for (;;) {
            bool want = !active && !exhausted;
            if (!__any(want)) break;
            u32 g = n;
            wave_take(p.giant_next, n, want, g, cbase, cend);
            if (want) {
                if (g >= n) {
                    exhausted = true;
                } else {
                    const u32 pos = p.giant_list[g];
                    const WindowState st = p.state[pos];
                    lst = p.lists + (u64)(pos / 64) * p.emax * 64 + (pos % 64);
                    lrs = p.lres + (u64)(pos / 64) * p.emax * 64 + (pos % 64);
                    const unsigned long long m1 = lst[(u64)(st.emain - 1) * 64];
                    item = st.item;
                    idx = item_bit(p.segs, item);
                    const u64 d = item_d(p.segs, item);
                    const u64 s64 = isqrt_u64(d);
                    dd = (double)d;
                    sd = (double)s64;
                    sq = (float)s64 * 0.25f;
                    sqc = sq * kQuotBias;
                    L = (double)isqrt_u64(s64);
                    m1Q = 4.0 * (double)__uint_as_float((u32)(m1 >> 32));
                    m1P = 4.0 * (double)__uint_as_float((u32)m1);
                    m1S = (lrs[(u64)(st.emain - 1) * 64] >> 1) % 3u;
                    cQ = m1Q;
                    cP = m1P;
                    cS = m1S;
                    tbl = p.tables + (u64)pos * p.tsize;
                    ng = 0;
                    active = true;
                }
            }
        }
        if (!__any(active)) break;

        if (active) {
            // Two phases per iteration: a lane that is not walking composes
            // (and reduces) its next giant ideal; then every walking lane
            // takes up to kWalkChunk reduction steps towards the next
            // distinguished ideal.  A lane with a long walk continues it in
            // the next iteration instead of holding up the other lanes.
            bool bad = false;
            if (!walking) {
                Form f3;
                Gamma gm;
                nucomp_choose(m1Q, m1P, cQ, cP, dd, L, f3, gm, bad);
                const u32 lg = gamma_log(gm, bad);
                double Qk, Pk, Qpk;
                const u32 Sr = reduce_form(f3, dd, sd, Qk, Pk, Qpk, bad);
                const u32 Sk = (m1S + cS + 3u - lg + Sr) % 3u;
                ng++;
                if (!bad) {
                    cQ = Qk;
                    cP = Pk;
                    cS = Sk;
                    Qw = (float)Qk * 0.25f;
                    Pw = (float)Pk * 0.25f;
                    Qpw = (float)Qpk * 0.25f;
                    Sw = Sk;
                    w = 0;
                    walking = true;
                }
            }
            bool done = false, flag = false;
            if (walking) {
                u32 u = 0;
                float acc = 0.f;
                for (; u < kWalkChunk && !is_dp(Qw); u++) {
                    float Pn, Qn;
                    rho_step_q(sq, sqc, Pw, Qw, Qpw, Pn, Qn, acc);
                    Qpw = Qw;
                    Qw = Qn;
                    Pw = Pn;
                }
                Sw += (u + (u32)acc) >> 1;
                w += u;
                my_steps += u;
                if (is_dp(Qw)) {
                    walking = false;
                    const u32 qb = __float_as_uint(Qw), pb = __float_as_uint(Pw);
                    const unsigned long long key = ((unsigned long long)qb << 32) | pb;
                    const u32 h = dict_hash(qb, pb);
                    u32 slot = h & mask;
                    for (u32 probe = 0; probe < p.tsize; probe++) {
                        const u32 v = tbl[slot];
                        if (v == 0u) break;
                        if ((v & 0xffff0000u) == (h & 0xffff0000u)) {
                            // fingerprint matches: compare the full key
                            const u32 e = (v & 0xffffu) - 1;
                            if (lst[(u64)e * 64] == key) {
                                // a hit at k = 2 is skipped: mu_2 may lie inside
                                // the window (a "unit" of distance 0); if it was a
                                // true hit, the next one is at eps or eps^2, whose
                                // residues are both 0 or both not
                                if (ng > 1) {
                                    const u32 St = (lrs[(u64)e * 64] >> 1) % 3u;
                                    flag = ((Sw + 3u - St) % 3u) == 0u;
                                    done = true;
                                }
                                break;
                            }
                        }
                        slot = (slot + 1) & mask;
                    }
                } else if (w >= kWalkLimit) {
                    bad = true;
                }
            }
            if (done) {
                emit_flag(p.eis_words, idx, flag);
                my_giants += ng;
                active = false;
            } else if (bad || ng >= p.max_giants) {
                const u32 f = atomicAdd(&p.fb_ctr->list_len, 1u);
                p.fb_list[f] = item;
                my_giants += ng;
                active = false;
                walking = false;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        my_steps += __shfl_down(my_steps, off, 64);
        my_giants += __shfl_down(my_giants, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&p.ctr->chunk_steps, (unsigned long long)my_steps);
        atomicAdd(&p.ctr->giant_steps, (unsigned long long)my_giants);
    }
}

hipError_t launch_walk_giant(const InfraParams &p, u32 grid, hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk_giant, dim3(grid), dim3(256), 0, stream, p);
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
