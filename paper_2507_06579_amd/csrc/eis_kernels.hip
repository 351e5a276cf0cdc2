// eis_kernels.hip -- gfx950 kernels of the Eisenstein-discriminant search.
//
// Pipeline of one pass (at most kPassCandidates candidates d_i = d0 + 8 i):
//   k_prime_offsets : for every odd prime p <= sqrt(b-1), the first candidate
//                     index i with p^2 | d0 + 8 i
//   k_sieve         : squarefree sieve over d = 5 (mod 8) (Section 1, the set
//                     D), one LDS bitmap per 32768-candidate segment, then
//                     compaction of the survivors into a work list
//   k_walk_baby     : one d per lane, reduction steps rho (Appendix A) with the
//                     generator carried in (O_K/2O_K)^* ~ Z/3 and the
//                     half-period symmetry exit; persistent, lanes refilled
//                     from a global queue as their walks end
//   k_popcount_add  : pi_D and pi_E of the pass
//
// Everything on the result path is integer-exact.  The walk keeps its
// quantities (all integers below 2^22 for d < 10^12) in fp32 registers, where
// adds, subtracts and fused multiply-adds of such integers are exact, and
// takes the partial quotient from a reciprocal estimate that is corrected to
// the exact floor.
#include "eis_internal.h"
#include "eis_walk.h"

namespace eis {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ void k_zero_u32(u32 *p, u64 n)
{
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 stride = (u64)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_zero_u32(u32 *p, u64 nwords, hipStream_t stream)
{
    if (nwords == 0) return hipSuccess;
    u64 blocks = (nwords + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_zero_u32, dim3((u32)blocks), dim3(256), 0, stream, p, nwords);
    return hipGetLastError();
}

// a * b mod m for a, b < m < 2^42: the quotient estimate from fp64 is off by
// at most one, and the wrapped 64-bit difference a*b - q*m is then exact.
__device__ __forceinline__ u64 mulmod_small(u64 a, u64 b, u64 m)
{
    double q = ((double)a * (double)b) / (double)m;
    u64 qi = (u64)q;
    long long r = (long long)(a * b - qi * m);
    while (r < 0) r += (long long)m;
    while (r >= (long long)m) r -= (long long)m;
    return (u64)r;
}

// ---------------------------------------------------------------------------
// k_prime_offsets: for segment s (blockIdx.y) and prime k < np_s,
// roff[roff_off_s + k] = the least i >= 0 with m_k | d0_s + 8 i, that is
// i = (-d0_s) * 8^{-1} (mod m_k), where m_k = p_k^2 for the squarefree set
// and m_k = p_k for the primes.
// ---------------------------------------------------------------------------
__global__ void k_prime_offsets(const PrimeEntry *__restrict__ primes,
                                const SegInfo *__restrict__ segs, u64 *__restrict__ roff)
{
    const SegInfo sg = segs[blockIdx.y];
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= sg.np) return;
    const PrimeEntry pe = primes[k];
    const bool prime_set = sg.set == kSetPrime;
    const u64 m = prime_set ? (u64)pe.p : pe.m;
    const u64 r = sg.d0 % m;
    const u64 neg = r ? m - r : 0;
    roff[sg.roff_off + k] = mulmod_small(neg, prime_set ? (u64)pe.inv8p : pe.inv8, m);
}

hipError_t launch_prime_offsets(const PrimeEntry *primes, const SegInfo *segs, u32 nseg,
                                u32 np_max, u64 *roff, hipStream_t stream)
{
    if (np_max == 0 || nseg == 0) return hipSuccess;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_prime_offsets, dim3((np_max + 255) / 256, nseg), dim3(256), 0, stream,
                       primes, segs, roff);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_sieve: one workgroup per block of kSegCandidates candidates of one
// segment (the segment is found from the workgroup index).
//   1. LDS bitmap <- all candidates of the block that lie below the
//      segment's n
//   2. strike i = roff (mod m) for every prime square m (squarefree set)
//      or every prime m (prime set).  The first primes (m < 4096, many
//      strikes per block: `nsmall` squares or `nsmall_p` primes) are spread
//      over all threads; each larger prime belongs to one thread.  In the
//      prime set a sieving prime that is itself a candidate of the block
//      struck itself; its bit is set again.
//   3. write the bitmap words, and append the surviving items to the work
//      list of the segment's method (block-wide prefix sum, one global atomic
//      per block).  Workgroups beyond the pass's blocks exit at once, so that
//      a fixed grid can serve every pass.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sieve(const PrimeEntry *__restrict__ primes,
                                               const u64 *__restrict__ roff,
                                               const SegInfo *__restrict__ segs, u32 nseg,
                                               u32 nblocks, u32 nsmall, u32 nsmall_p,
                                               u32 *__restrict__ sq_words,
                                               u32 *__restrict__ list_plain,
                                               PassCounters *__restrict__ ctr_plain,
                                               u32 *__restrict__ list_giant,
                                               PassCounters *__restrict__ ctr_giant)
{
    __shared__ u32 bits[kSegWords];
    __shared__ u32 scan[256];
    __shared__ u32 base_sh;
    const u32 b = blockIdx.x;
    if (b >= nblocks) return;
    // segment of this block: the last s with block_off <= b
    u32 lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (segs[mid].block_off <= b) lo = mid;
        else hi = mid;
    }
    const SegInfo sg = segs[lo];
    const u32 tid = threadIdx.x;
    const u32 seg0 = (b - sg.block_off) * kSegCandidates;  // first index of the block
    const u32 n = sg.n;
    const u32 segn = min(kSegCandidates, n - seg0);
    const u64 *ro = roff + sg.roff_off;
    const u32 np = sg.np;
    const bool prime_set = sg.set == kSetPrime;
    const u32 ns = min(prime_set ? nsmall_p : nsmall, np);

    for (u32 w = tid; w < kSegWords; w += 256) {
        const u32 l0 = w * 32;
        u32 v;
        if (l0 + 32 <= segn) v = 0xffffffffu;
        else if (l0 >= segn) v = 0u;
        else v = (1u << (segn - l0)) - 1u;
        bits[w] = v;
    }
    __syncthreads();

    // small prime squares: all threads share each prime's strikes
    for (u32 k = 0; k < ns; k++) {
        const u32 m = prime_set ? primes[k].p : (u32)primes[k].m;
        const u32 r = (u32)ro[k];
        const u32 off = seg0 % m;
        const u32 first = (r >= off) ? r - off : r + m - off;  // (r - seg0) mod m
        for (u32 i = first + tid * m; i < segn; i += 256 * m)
            atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
    }
    // larger prime squares: one prime per thread
    for (u32 k = ns + tid; k < np; k += 256) {
        const u64 m = prime_set ? (u64)primes[k].p : primes[k].m;
        const u64 r = ro[k];
        if (m >= (u64)n) {
            // at most one strike in the whole segment: index r itself
            if (r >= seg0 && r < (u64)seg0 + segn) {
                const u32 i = (u32)r - seg0;
                atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
            }
            continue;
        }
        // here m < n <= 2^24, so 32-bit arithmetic is exact
        const u32 m32 = (u32)m, r32 = (u32)r;
        const u32 off = seg0 % m32;
        const u32 first = (r32 >= off) ? r32 - off : r32 + m32 - off;  // (r - seg0) mod m
        for (u32 i = first; i < segn; i += m32)
            atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
    }
    __syncthreads();
    if (prime_set) {
        const u64 lo_d = sg.d0 + 8ull * seg0, hi_d = lo_d + 8ull * segn;
        if (np > 0 && lo_d <= (u64)primes[np - 1].p) {
            for (u32 k = tid; k < np; k += 256) {
                const u64 pk = primes[k].p;
                if (pk >= lo_d && pk < hi_d && (pk - lo_d) % 8 == 0) {
                    const u32 i = (u32)((pk - lo_d) >> 3);
                    atomicOr(&bits[i >> 5], 1u << (i & 31));
                }
            }
        }
        __syncthreads();
    }

    // write bitmap words and compact the survivors
    const u32 wbase = sg.word_off + seg0 / 32;
    u32 cnt = 0;
    u32 wv[kSegWords / 256];
#pragma unroll
    for (u32 t = 0; t < kSegWords / 256; t++) {
        const u32 w = tid * (kSegWords / 256) + t;
        wv[t] = bits[w];
        cnt += __popc(wv[t]);
    }
    for (u32 w = tid; w < kSegWords; w += 256) {
        if (w * 32 < segn) sq_words[wbase + w] = bits[w];
    }
    scan[tid] = cnt;
    __syncthreads();
    for (u32 off = 1; off < 256; off <<= 1) {
        const u32 v = (tid >= off) ? scan[tid - off] : 0u;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    u32 *list = sg.method ? list_giant : list_plain;
    PassCounters *ctr = sg.method ? ctr_giant : ctr_plain;
    if (tid == 255) base_sh = atomicAdd(&ctr->list_len, scan[255]);
    __syncthreads();
    u32 pos = base_sh + scan[tid] - cnt;
    const u32 tag = (u32)lo << kItemShift;
#pragma unroll
    for (u32 t = 0; t < kSegWords / 256; t++) {
        u32 v = wv[t];
        const u32 ibase = seg0 + (tid * (kSegWords / 256) + t) * 32;
        while (v) {
            const u32 bb = __ffs(v) - 1;
            v &= v - 1;
            list[pos++] = tag | (ibase + bb);
        }
    }
}

hipError_t launch_sieve(const PrimeEntry *primes, const u64 *roff, const SegInfo *segs,
                        u32 nseg, u32 nblocks, u32 nsmall, u32 nsmall_p, u32 *sq_words,
                        u32 *list_plain, PassCounters *ctr_plain, u32 *list_giant,
                        PassCounters *ctr_giant, hipStream_t stream)
{
    if (nblocks == 0 || nseg == 0) return hipSuccess;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_sieve, dim3(nblocks), dim3(256), 0, stream, primes, roff, segs, nseg,
                       nblocks, nsmall, nsmall_p, sq_words, list_plain, ctr_plain, list_giant,
                       ctr_giant);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Baby-step walk.
//
// Ideal (theta_{j+1}) = [Q_j/2, (P_j + sqrt d)/2], (P_0, Q_0) = (1, 2), and rho:
//   q = floor((P + sqrt d)/Q) = floor((P + s)/Q),  s = floor(sqrt d)
//   P' = q Q - P,   Q' = Q_prev + q (P - P')        (= (d - P'^2)/Q)
// The relative generator (P' + sqrt d)/Q has residue log 1 in F_4^* ~ Z/3
// when P' = 1 (mod 4) and log 2 when P' = 3 (mod 4) (Q/2 is odd and 2 is
// inert), so S_j = sum_{i<=j} (1 + bit1(P_i)) is log theta_{j+1} (mod 3).
// Half-period exit (the symmetry of the cycle under conjugation, which acts
// on F_4 as the Frobenius, log -> -log):
//   Q_j = Q_{j-1}          -> log eps = S_j + S_{j-1}
//   P_j = P_{j-1}, j >= 2  -> log eps = 2 S_{j-1}
// and d is Eisenstein iff log eps = 0 (mod 3).
// ---------------------------------------------------------------------------

// Exit batching: a lane whose walk ends idles (its steps are wasted) until
// kBatch lanes of the wave are idle; then they are all refilled at once, so
// that the wave-wide refill (queue, decode, first step) is paid once per
// kBatch walks.  The best batch balances the refill cost against the idle
// lanes: about sqrt(5.2e6 / sqrt(d)) for mean walks of 0.075 sqrt(d) steps,
// i.e. 32 at 10^6, 13 at 10^9, 4 at 10^11.
__device__ __forceinline__ u32 exit_batch(float s)
{
    return (u32)fminf(fmaxf(rintf(sqrtf(5.2e6f / s)), 1.f), 32.f);
}

template <bool kCheck>
__device__ __forceinline__ void walk_baby_body(const WalkParams &p, const SegLds *segs)
{
    const u32 n = p.ctr->list_len;
    // inner-loop length between budget checks; a walk that has not ended
    // after max_steps (rounded up to a multiple of K) is abandoned and counted
    const u32 K = __builtin_amdgcn_readfirstlane(min(kInnerChunk, max(p.max_steps, 1u)));
    const u32 lane = __lane_id();
    // walk state in quarter units (see rho_step_q)
    float sq = 0.f, sqc = 0.f, P = 0.25f, Q = 0.5f, Qp = 0.5f;
    u32 S = 0, j = 0, idx = 0;
    u32 cbase = 0, cend = 0;  // the wave's claimed chunk of the queue
    bool live = false;        // the lane walks a d
    bool drained = false;     // wave-uniform: the queue has no more items
    u32 batch = 1;            // wave-uniform exit batch
    u64 my_steps = 0, my_refills = 0;

    for (;;) {
        // ---- refill every idle lane -------------------------------------
        while (!drained) {
            const bool want = !live;
            if (!__any(want)) break;
            u32 k = n;
            wave_take(&p.ctr->work_next, n, want, k, cbase, cend);
            if (__any(want && k >= n)) drained = true;
            if (want && k < n) {
                const u32 item = p.list[k];
                idx = item_bit(segs, item);
                my_refills++;
                double sd, P1, Q1;
                u32 S1;
                first_step(item_d(segs, item), sd, P1, Q1, S1);
                my_steps += 1;
                if (Q1 == 2.0) {
                    // Q_1 = Q_0: log eps = S_1 + S_0 = S_1
                    emit_flag(p.eis_words, idx, S1 % 3u == 0u);
                } else {
                    sq = (float)sd * 0.25f;
                    sqc = sq * kQuotBias;
                    P = (float)P1 * 0.25f;
                    Q = (float)Q1 * 0.25f;
                    Qp = 0.5f;
                    S = S1;
                    j = 1;
                    live = true;
                }
            }
        }
        if (!__any(live)) break;
        {
            // the batch follows the walk lengths of the wave's current d's
            // (those of its first walking lane)
            const u32 first = (u32)__builtin_ctzll(__builtin_amdgcn_ballot_w64(live));
            const float s0 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(sq), first)) * 4.f;
            batch = exit_batch(s0);
        }
        // Up to K steps, two per iteration (so that the state never needs
        // moves); a lane whose walk ends emits its flag at once and idles.
        // The loop control is wave-uniform and kept to a few scalar
        // instructions per iteration (the scalar unit is shared by the four
        // SIMDs of a CU): lm is the mask of walking lanes, and the exits of
        // both steps are tested once per iteration.
        u64 lm = __builtin_amdgcn_ballot_w64(live);
        // leave for a refill once `batch` lanes idle (once all idle when the
        // queue is drained): at most `keep` walking lanes
        const u32 keep = drained ? 0u : 64u - batch;
        const u32 iters = (K + 1) / 2;
        u32 it = 0;
        bool stop = false;
        float P1 = 0.f, Q1 = 0.f, acc = 0.f;
        for (;;) {
            float P2, Q2;
            rho_step_q<kCheck>(sq, sqc, P, Q, Qp, P1, Q1, acc);
            const u64 mA = __builtin_amdgcn_ballot_w64(Q1 == Q) | __builtin_amdgcn_ballot_w64(P1 == P);
            rho_step_q<kCheck>(sq, sqc, P1, Q1, Q, P2, Q2, acc);
            const u64 mB = __builtin_amdgcn_ballot_w64(Q2 == Q1) | __builtin_amdgcn_ballot_w64(P2 == P1);
            const u64 em = (mA | mB) & lm;
            if (em) {
                // some walk ended at the first (A) or second (B) step
                const bool exA = (mA & lm) >> lane & 1ull;
                const bool exB = !exA && ((mB & lm) >> lane & 1ull);
                if (exA || exB) {
                    const u32 kx = 2 * it + (exA ? 1u : 2u);
                    // acc up to the exit step (exact: small integers)
                    const float accx = exA ? fmaf(__builtin_amdgcn_fractf(P2), -4.f, acc) : acc;
                    const float Pj = exA ? P1 : P2;
                    const bool qrule = exA ? (Q1 == Q) : (Q2 == Q1);
                    const u32 Sj = S + ((kx + (u32)accx) >> 1);
                    const u32 rj = __builtin_amdgcn_fractf(Pj) > 0.5f ? 2u : 1u;
                    // Q-rule first (it also covers the tie at the period's end)
                    const u32 v = qrule ? (2u * Sj - rj) : (2u * (Sj - rj));
                    emit_flag(p.eis_words, idx, v % 3u == 0u);
                    my_steps += j + kx - 1;
                }
                lm &= ~em;
                stop = (u32)__builtin_popcountll(lm) <= keep;
            }
            Qp = Q1;
            Q = Q2;
            P = P2;
            if (++it >= iters || stop) break;
        }
        const u32 k = 2 * it;
        live = (lm >> lane) & 1ull;
        if (live) {
            j += k;
            S += (k + (u32)acc) >> 1;
            if (j > p.max_steps) {
                atomicAdd(&p.ctr->err_count, 1u);
                my_steps += j - 1;
                live = false;
            }
        }
    }
    // wave-level reduction of the counters, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        my_steps += __shfl_down(my_steps, off, 64);
        my_refills += __shfl_down(my_refills, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&p.ctr->baby_steps, (unsigned long long)my_steps);
        atomicAdd(&p.ctr->refills, (unsigned long long)my_refills);
    }
}

__global__ __launch_bounds__(256) void k_walk_baby(WalkParams p)
{
    __shared__ SegLds segs[kMaxSegments];
    load_segs(segs, p.segs, p.nseg);
    if (p.exact_quot)
        walk_baby_body<false>(p, segs);
    else
        walk_baby_body<true>(p, segs);
}

hipError_t launch_walk_baby(const WalkParams &p, u32 grid, hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_walk_baby, dim3(grid), dim3(256), 0, stream, p);
    return hipGetLastError();
}

int walk_baby_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_baby, 256, 0) != hipSuccess)
        return 4;
    return nb > 0 ? nb : 1;
}

// ---------------------------------------------------------------------------
// k_popcount_segs: for segment s (blockIdx.y), add the set bits of its
// squarefree and Eisenstein bitmap words to counts[2 slot_s] and
// counts[2 slot_s + 1].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_popcount_segs(const u32 *__restrict__ sq_words,
                                                       const u32 *__restrict__ eis_words,
                                                       const SegInfo *__restrict__ segs,
                                                       unsigned long long *counts)
{
    __shared__ unsigned long long red[2][4];
    const SegInfo sg = segs[blockIdx.y];
    const u32 nw = (sg.n + 31) / 32;
    unsigned long long cs = 0, ce = 0;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += gridDim.x * blockDim.x) {
        cs += __popc(sq_words[sg.word_off + i]);
        ce += __popc(eis_words[sg.word_off + i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        cs += __shfl_down(cs, off, 64);
        ce += __shfl_down(ce, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = cs;
        red[1][threadIdx.x >> 6] = ce;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long ts = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const unsigned long long te = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        if (ts) atomicAdd(&counts[2 * sg.count_slot], ts);
        if (te) atomicAdd(&counts[2 * sg.count_slot + 1], te);
    }
}

hipError_t launch_popcount_segs(const u32 *sq_words, const u32 *eis_words, const SegInfo *segs,
                                u32 nseg, u32 words_max, unsigned long long *counts,
                                hipStream_t stream)
{
    if (nseg == 0 || words_max == 0) return hipSuccess;
    u32 bx = (words_max + 255) / 256;
    if (bx > 256) bx = 256;
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_popcount_segs, dim3(bx, nseg), dim3(256), 0, stream, sq_words,
                       eis_words, segs, counts);
    return hipGetLastError();
}

}  // namespace eis
