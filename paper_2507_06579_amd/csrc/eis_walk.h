// eis_walk.h -- the reduction step rho in fp32 registers, shared by the
// plain walk and the two walks of the infrastructure method.
#pragma once

#include "eis_internal.h"

namespace eis {

__device__ __forceinline__ u64 isqrt_u64(u64 d)
{
    u64 s = (u64)sqrt((double)d);
    while (s * s > d) s--;
    while ((s + 1) * (s + 1) <= d) s++;
    return s;
}

__device__ __forceinline__ void emit_flag(u32 *eis_words, u32 idx, bool eis)
{
    if (eis) atomicOr(&eis_words[idx >> 5], 1u << (idx & 31));
}

// One reduction step from (P, Q) with predecessor Qp to (Pn, Qn); S gains the
// residue of the relative generator (Pn + sqrt d)/Q.
__device__ __forceinline__ void baby_step(float s, float P, float Q, float Qp, float &Pn,
                                          float &Qn, u32 &S)
{
    const float t = P + s;
    const float rq = __builtin_amdgcn_rcpf(Q);
    // floor(t/Q) - 1 <= q0 <= floor(t/Q): the estimate t*rq is within 0.16
    // of t/Q for t/Q < 2^20, and the bias -0.5 keeps it on the low side
    const float q0 = floorf(fmaf(t, rq, -0.5f));
    const float r = fmaf(-q0, Q, t);
    const float q = (r >= Q) ? q0 + 1.f : q0;
    Pn = fmaf(q, Q, -P);
    Qn = fmaf(q, P - Pn, Qp);
    S += 1u + (((u32)Pn >> 1) & 1u);
}

// Wave-level work queue.  A wave claims kQueueChunk consecutive items of a
// global queue with ONE atomic and hands them to its lanes as they ask for
// work, so that a queue head is touched once per kQueueChunk items instead of
// once per item (same-address atomics serialise in L2).  `cbase` and `cend`
// are wave-uniform: every lane computes them identically.
constexpr u32 kQueueChunk = 64;

// Lanes with `want` set receive an item index in `item` (< n); lanes that
// get nothing because the queue is drained get `item` = n.  Returns false
// when the queue is drained for the whole wave.
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

// Iterations of the inner loop between two checks of the step budget.
constexpr u32 kInnerChunk = 1u << 14;


}  // namespace eis
