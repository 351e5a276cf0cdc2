// eis_walk.h -- the reduction step rho in fp32 registers, shared by the
// plain walk and the two walks of the infrastructure method.
#pragma once

#include "eis_internal.h"

namespace eis {

// The first reduction step of a walk, from (P_0, Q_0) = (1, 2):
// s = isqrt(d), P_1 = the largest odd number <= s, Q_1 = (d - P_1^2)/2, and
// the residue r(P_1).  In fp64: for d < 10^12 every value is an integer below
// 2^41, so products and differences are exact, and the square root estimate
// (off by at most one near squares) is corrected exactly.
__device__ __forceinline__ void first_step(u64 d, double &s, double &P1, double &Q1, u32 &S1)
{
    const double dd = (double)d;
    s = floor(sqrt(dd));
    if (s * s > dd)
        s -= 1.0;
    else if ((s + 1.0) * (s + 1.0) <= dd)
        s += 1.0;
    P1 = 2.0 * floor((s + 1.0) * 0.5) - 1.0;
    Q1 = (dd - P1 * P1) * 0.5;
    S1 = 1u + (((u32)P1 >> 1) & 1u);
}

__device__ __forceinline__ void emit_flag(u32 *eis_words, u32 idx, bool eis)
{
    if (eis) atomicOr(&eis_words[idx >> 5], 1u << (idx & 31));
}

// One reduction step rho (Appendix A) from (P, Q) with predecessor Qp:
//   q = floor((P + sqrt d)/Q) = floor((P + s)/Q),  P' = qQ - P,
//   Q' = (d - P'^2)/Q = Qp + q (P - P')   (division-free form),
// and the residue r(P') of the relative generator (P' + sqrt d)/Q in Z/3.
// For d < 10^12 every quantity is an integer below 2^21, so fp32 adds and
// fmas are exact.  The state is kept in quarter units (P/4, Q/4, Qp/4, s/4:
// exact power-of-two scalings), and the quotient is
//   q = floor(fl(fl(P c + s c) rcp(Q)))  with c = 1 + 2^-21.
// The relative errors of the roundings (the product s c, the fma, the
// reciprocal's 1 ulp, the product) add up to less than 2^-21, so the bias c
// keeps the estimate at or above t/Q = (P + s)/Q, and q is never below the
// true floor k (k is representable, so rounding a value >= k cannot fall
// below it).  q exceeds k by at most one, and only when t/Q is within about
// 2^-20 (t/Q) of k + 1; then P' = qQ - P = (s - r) + Q > s, where r < Q is
// the true remainder, while the true P' = s - r is at most s.  So P' > s
// detects the overshoot exactly, and q - 1, P' - Q undo it.  For d < 10^12
// that happens about once per 10^6 steps, and only above 10^11.
// The residue: P' is odd, so fract(P'/4) is 1/4 when P' = 1 (mod 4) and 3/4
// when P' = 3 (mod 4); acc sums 4 fract(P'/4), i.e. 1 or 3 per step (an exact
// integer while acc < 2^24), and the caller folds it into S: over k steps,
// the residues r = 1 + bit1(P') add up to (k + acc) / 2.
// kCheck = false leaves the overshoot test out, for walks whose every d is at
// most kExactQuotMaxD: an overshoot needs (k + 1) Q - t <= t (2^-21 + 5 2^-24)
// with (k + 1) Q - t >= 1 for the integers t = P + s and Q, i.e. t >= 2^24 / 13,
// and t <= 2 s, so it cannot happen below d = 4.1 10^11.
constexpr float kQuotBias = 1.f + 0x1p-21f;

template <bool kCheck = true>
__device__ __forceinline__ void rho_step_q(float sq, float sqc, float P, float Q, float Qp,
                                           float &Pn, float &Qn, float &acc)
{
    const float rq = __builtin_amdgcn_rcpf(Q);
    float q = floorf(fmaf(P, kQuotBias, sqc) * rq);
    Pn = fmaf(q, Q, -P);
    if (kCheck && __builtin_amdgcn_ballot_w64(Pn > sq)) {
        // rare: keep it a branch (an empty volatile asm is not speculated)
        __asm__ volatile("");
        if (Pn > sq) {
            q -= 1.f;
            Pn -= Q;
        }
    }
    Qn = fmaf(q, P - Pn, Qp);
    acc = fmaf(__builtin_amdgcn_fractf(Pn), 4.f, acc);
}

// Wave-level work queue.  A wave claims kQueueChunk consecutive items of a
// global queue with ONE atomic and hands them to its lanes as they ask for
// work, so that a queue head is touched once per kQueueChunk items instead of
// once per item (same-address atomics serialise in L2).  `cbase` and `cend`
// are wave-uniform: every lane computes them identically.
constexpr u32 kQueueChunk = 64;

// Lanes with `want` set receive an item index in `item` (< n); lanes that
// get nothing because the queue is drained get `item` = n.  Must be called
// by the whole wave (lane 0 claims the chunks).
__device__ __forceinline__ void wave_take(u32 *head, u32 n, bool want, u32 &item, u32 &cbase,
                                          u32 &cend)
{
    const u64 m = __builtin_amdgcn_ballot_w64(want);
    if (m == 0) return;
    const u32 lane = __lane_id();
    const u64 below = (lane == 0) ? 0ull : (m & (~0ull >> (64 - lane)));
    const u32 rank = (u32)__builtin_popcountll(below);
    u32 need = (u32)__builtin_popcountll(m);
    item = n;
    u32 given = 0;  // wanting lanes served so far (ranks below `given` are done)
    while (need > 0) {
        if (cbase >= cend) {
            u32 c = 0;
            if (lane == 0) c = atomicAdd(head, kQueueChunk);
            c = __builtin_amdgcn_readfirstlane(c);
            if (c >= n) {
                cbase = cend = n;
                return;  // drained: the remaining wanting lanes keep item = n
            }
            cbase = c;
            cend = min(c + kQueueChunk, n);
        }
        const u32 avail = cend - cbase;
        const u32 take = min(avail, need);
        if (want && rank >= given && rank < given + take) item = cbase + (rank - given);
        cbase += take;
        given += take;
        need -= take;
    }
}

// The pass's segment table, copied into LDS by every block of a walk kernel
// (decoding a work item then costs an LDS read, not a dependent global one).
__device__ __forceinline__ void load_segs(SegLds *dst, const SegInfo *src, u32 nseg)
{
    for (u32 i = threadIdx.x; i < nseg; i += blockDim.x) {
        dst[i].d0 = src[i].d0;
        dst[i].word_off = src[i].word_off;
        dst[i].wscale = src[i].wscale;
    }
    __syncthreads();
}

// Empty prefetch slot.  The walk kernels load the list entry of a lane's next
// work item one refill ahead, so that the load's latency overlaps the walk.
constexpr u32 kNoItem = ~0u;

// Iterations of the inner loop between two checks of the step budget.
constexpr u32 kInnerChunk = 1u << 14;


}  // namespace eis
