// md_sweep.h -- the in-LDS neighbour sweep for the pairwise downwash of
// Eq. 6, shared by the semi-implicit Euler and the Runge-Kutta step kernels.
// Positions of a bin's drones are published to LDS; each drone sums the
// terms of the other drones of its environment in ascending slot order.
#pragma once

#include "md_physics.h"

namespace md {
namespace phys {

// The constants of the pair term with C3s pinned in a vector register: the
// term's fused multiply-add C2s dz + C3s may read only one scalar operand, and
// without this the compiler re-copies C3s into a vector register on every
// iteration of the neighbour loops.
__device__ __forceinline__ KConst pair_consts(const KConst &c) {
    KConst cc = c;
    float c3 = c.C3s;
    asm volatile("" : "+v"(c3));
    cc.C3s = c3;
    return cc;
}

// This lane's share of the downwash sum over its environment's slots
// [lo, lo + mmax), in ascending order (every LPD-th slot from `sub`).  In a
// uniform bin every environment has mmax drones and the bound check is
// dropped.
template <bool DZMIN, int LPD, int UNROLL>
__device__ __forceinline__ float dw_sweep(const KConst &c0, const float4 *buf, int lo, int sub, int mmax,
                                          int menv, bool uniform, const Drone &d) {
    const KConst c = pair_consts(c0);
    float acc = 0.f;
    if (uniform) {
#pragma unroll UNROLL
        for (int j = sub; j < mmax; j += LPD) {
            const float4 pj = buf[lo + j];
            acc += dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
        }
    } else {
#pragma unroll UNROLL
        for (int j = sub; j < mmax; j += LPD) {
            const float4 pj = buf[lo + j];
            const float term = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
            acc += (j < menv) ? term : 0.f;
        }
    }
    return acc;
}

// Pair-symmetric downwash sweep: each unordered pair of an environment is
// evaluated once, by lane i for partners (i + d) mod M, d = 1..(M-1)/2, plus
// d = M/2 from the lower half when M is even.  The term goes to the lower
// drone's row of the LDS matrix T (the other entry gets 0); after a barrier
// each drone sums its row in ascending order (the diagonal and the padding
// to a multiple of 4 hold 0, and x + 0 = x).  The term depends only on
// dxy^2 and |dz|, and fl(a - b) = -fl(b - a), so every entry and the sum are
// bitwise those of the all-pairs sweep.
template <bool DZMIN, int UNROLL>
__device__ __forceinline__ void dw_pairs(const KConst &c, const float4 *buf, float *T, int ts, int slot,
                                         int lo, int m, const Drone &d) {
    const int li = slot - lo;
    const int h = (m - 1) >> 1;
#pragma unroll UNROLL
    for (int k = 1; k <= h; ++k) {
        int lj = li + k;
        lj -= (lj >= m) ? m : 0;
        const float4 pj = buf[lo + lj];
        const float dz = pj.z - d.pz;
        const float d2 = dw_d2(pj.x - d.px, pj.y - d.py);
        const float t = dw_raw<DZMIN>(c, d2, fabsf(dz));
        const bool near = dw_near(d2);
        T[slot * ts + lj] = (near && dz > 0.f) ? t : 0.f;
        T[(lo + lj) * ts + li] = (near && dz < 0.f) ? t : 0.f;
    }
    if ((m & 1) == 0 && li < (m >> 1) && m > 0) {
        const int lj = li + (m >> 1);
        const float4 pj = buf[lo + lj];
        const float dz = pj.z - d.pz;
        const float d2 = dw_d2(pj.x - d.px, pj.y - d.py);
        const float t = dw_raw<DZMIN>(c, d2, fabsf(dz));
        const bool near = dw_near(d2);
        T[slot * ts + lj] = (near && dz > 0.f) ? t : 0.f;
        T[(lo + lj) * ts + li] = (near && dz < 0.f) ? t : 0.f;
    }
}

// Pair-symmetric sweep through wave shuffles, for bins whose environments
// each lie inside one wavefront (one lane per drone).  As in dw_pairs, lane i
// evaluates the pairs (i, (i + k) mod M) for k = 1..(M-1)/2; the term stays
// with lane i when its partner is above, and otherwise travels to the
// partner's lane through a cross-lane permute (ds_bpermute): at shift k lane
// j receives from lane (j - k) mod M.  The loop runs to the bin's largest
// environment so that every permute executes with the whole wave.  For even
// M the pair at distance M/2 is evaluated by both members, each keeping it
// when its partner is above.  The summation order (per shift: own term, then
// the received one) is fixed by the drone's place in its environment.
template <bool DZMIN, bool UNIFORM, int UNROLL>
__device__ __forceinline__ float dw_pairs_shfl(const KConst &c0, const float4 *buf, int slot, int lo, int m,
                                               int mmax, const Drone &d) {
    const KConst c = pair_consts(c0);
    // an idle slot (m = 0) runs the loop as a one-drone environment of itself
    const int mm = m > 0 ? m : 1;
    const int li = m > 0 ? slot - lo : 0;
    const int base = (slot & 63) - li;  // the environment's first lane in this wave
    // every lane runs to the bin's largest environment, so that each permute
    // executes with the whole wave; in a uniform bin every environment has
    // that size and no shift needs masking
    const int h = (m - 1) >> 1, hmax = (mmax - 1) >> 1;
    // advanced cyclically: the partner's position (li + k) mod M in `buf`, and
    // the byte address of lane (li - k) mod M, whose term this lane receives
    const float4 *q_beg = buf + lo, *q_end = buf + lo + mm;
    const float4 *qj = buf + lo + li;
    const int p_beg = base * 4, p_last = (base + mm - 1) * 4;
    int ps = (base + li) * 4;
    float acc = 0.f;
#pragma unroll UNROLL
    for (int k = 1; k <= hmax; ++k) {
        qj = (qj + 1 == q_end) ? q_beg : qj + 1;
        ps = (ps == p_beg) ? p_last : ps - 4;
        const float4 q = *qj;
        const float dz = q.z - d.pz;
        const float d2 = dw_d2(q.x - d.px, q.y - d.py);
        const float t = dw_raw<DZMIN>(c, d2, fabsf(dz));
        const bool near = dw_near(d2) && (UNIFORM || k <= h);
        // the term stays with the lower drone: each of the two lane masks
        // selects it or 0 (at dz = 0 neither does, and t is not used)
        float mine = (near && dz > 0.f) ? t : 0.f;
        asm volatile("" : "+v"(mine));
        const float theirs = (near && dz < 0.f) ? t : 0.f;
        const float recv = __int_as_float(__builtin_amdgcn_ds_bpermute(ps, __float_as_int(theirs)));
        acc += mine;
        acc += recv;
    }
    if ((m & 1) == 0 && m > 0) {
        const int half = m >> 1;
        const int lj = li < half ? li + half : li - half;
        const float4 q = buf[lo + lj];
        acc += dw_term<DZMIN>(c, q.x - d.px, q.y - d.py, q.z - d.pz);
    }
    return acc;
}

// The same pairs, shifts, routing and summation order as dw_pairs_shfl, for
// bins whose environments all have one power-of-two size M = 64 / E and sit
// interleaved in their wave: drone li of the wave's environment e in lane
// E li + e.  Then the partner (li + k) mod M of every lane is lane
// (lane + E k) mod 64 and the drone whose term arrives is lane
// (lane - E k) mod 64, for all lanes at once: a rotation of the whole wave.
// The positions are stored twice per wave (entries lane and 64 + lane of the
// wave's 128), so the partner's entry is a fixed offset from the lane's own,
// and the permute address wraps in hardware (lane bits of the byte address);
// with k unrolled neither costs an instruction.
// `seg.at<H>(s)` runs after each of the H + 1 segments (shifts 1..H, then
// the half pair), s = 0..H, and `seg.all()` after a sweep that takes no hook:
// the caller's work to interleave with the sweep (the step kernel's
// observation stores).
struct NoSeg {
    template <int H>
    __device__ __forceinline__ void at(int) const {}
    __device__ __forceinline__ void all() const {}
};

template <bool DZMIN, int E, class Seg = NoSeg>
__device__ __forceinline__ float dw_pairs_rot(const KConst &c0, const float4 *own, int lane, const Drone &d,
                                              const Seg &seg = Seg()) {
    constexpr int M = 64 / E;
    constexpr int H = (M - 1) / 2;
    const KConst c = pair_consts(c0);
    // the permute addresses pa + 256 - 4 E k fold into the instructions'
    // offset field when pa is formed inside the step: hoisted out of the
    // step loop instead, they would hold one register per shift
    int pa = 4 * lane;
    asm volatile("" : "+v"(pa));
    float acc = 0.f;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        const float4 q = own[E * k];
        const float dz = q.z - d.pz;
        const float d2 = dw_d2(q.x - d.px, q.y - d.py);
        const float t = dw_raw<DZMIN>(c, d2, fabsf(dz));
        const bool near = dw_near(d2);
        float mine = (near && dz > 0.f) ? t : 0.f;
        // formed here, not where the serial sum reaches it: otherwise its
        // lane mask stays live across shifts and the masks spill
        asm volatile("" : "+v"(mine));
        const float theirs = (near && dz < 0.f) ? t : 0.f;
        const float recv = __int_as_float(__builtin_amdgcn_ds_bpermute(pa + (256 - 4 * E * k), __float_as_int(theirs)));
        acc += mine;
        acc += recv;
        seg.template at<H>(k - 1);
    }
    {
        // M is even: the pair at distance M / 2 (lane + 32), kept by the lower drone
        const float4 q = own[32];
        acc += dw_term<DZMIN>(c, q.x - d.px, q.y - d.py, q.z - d.pz);
    }
    seg.template at<H>(H);
    return acc;
}

template <bool DZMIN, class Seg = NoSeg>
__device__ __forceinline__ float dw_rot(const KConst &c, const float4 *own, int lane, int m, const Drone &d,
                                        const Seg &seg = Seg()) {
    switch (m) {
        case 64: {
            // 31 shifts unrolled leave no registers for interleaved stores
            const float r = dw_pairs_rot<DZMIN, 1>(c, own, lane, d);
            seg.all();
            return r;
        }
        case 32: return dw_pairs_rot<DZMIN, 2>(c, own, lane, d, seg);
        case 16: return dw_pairs_rot<DZMIN, 4>(c, own, lane, d, seg);
        case 8: return dw_pairs_rot<DZMIN, 8>(c, own, lane, d, seg);
        case 4: return dw_pairs_rot<DZMIN, 16>(c, own, lane, d, seg);
        default: return dw_pairs_rot<DZMIN, 32>(c, own, lane, d, seg);
    }
}

// Downwash sum (without K1) of this slot's drone against the positions in
// `buf`.  SYM 0: the all-pairs sweep over LPD lanes (their partial sums
// combined in a fixed order); SYM 1: the pair-symmetric sweep through the LDS
// term matrix (it contains the barrier between the term writes and the row
// sums; bitwise equal to SYM 0 with one lane); SYM 2: the pair-symmetric
// sweep through wave shuffles (environments inside one wave); SYM 3: the same
// sweep as a whole-wave rotation on interleaved uniform bins (bitwise equal
// to SYM 2).
template <int LPD, int UNROLL, int SYM>
__device__ __forceinline__ float dw_sum(const KConst &c, const float4 *buf, float *tmat, int ts, int slot,
                                        int sub, int lo, int mmax, int menv, bool uniform, const Drone &d) {
    float acc = 0.f;
    if (SYM == 3) {
        // interleaved uniform bins (see dw_pairs_rot): `buf` holds each wave's
        // positions twice, 128 entries per wave
        const int lane = slot & 63;
        const float4 *own = buf + 2 * (slot - lane) + lane;
        acc = c.dz_min > 0.f ? dw_rot<true>(c, own, lane, mmax, d) : dw_rot<false>(c, own, lane, mmax, d);
    } else if (SYM == 2) {
        // `uniform` and dz_min are the same for the whole workgroup: the
        // permutes inside run with every lane of the wave
        if (uniform)
            acc = c.dz_min > 0.f ? dw_pairs_shfl<true, true, UNROLL>(c, buf, slot, lo, menv, mmax, d)
                                 : dw_pairs_shfl<false, true, UNROLL>(c, buf, slot, lo, menv, mmax, d);
        else
            acc = c.dz_min > 0.f ? dw_pairs_shfl<true, false, UNROLL>(c, buf, slot, lo, menv, mmax, d)
                                 : dw_pairs_shfl<false, false, UNROLL>(c, buf, slot, lo, menv, mmax, d);
    } else if (SYM == 1) {
        if (c.dz_min > 0.f)
            dw_pairs<true, UNROLL>(c, buf, tmat, ts, slot, lo, menv, d);
        else
            dw_pairs<false, UNROLL>(c, buf, tmat, ts, slot, lo, menv, d);
        __syncthreads();
        // ascending row sum, four entries per 16-byte read (zero padded)
        const float4 *row = (const float4 *)(tmat + slot * ts);
        for (int j = 0; j < ((menv + 3) >> 2); ++j) {
            const float4 t = row[j];
            acc += t.x;
            acc += t.y;
            acc += t.z;
            acc += t.w;
        }
    } else if (c.dz_min > 0.f) {
        acc = dw_sweep<true, LPD, UNROLL>(c, buf, lo, sub, mmax, menv, uniform, d);
    } else {
        acc = dw_sweep<false, LPD, UNROLL>(c, buf, lo, sub, mmax, menv, uniform, d);
    }
    // the partial sums of a drone's lanes, combined across the lanes of a
    // quad by DPP quad permutes (lane ^ 1, then lane ^ 2; every lane of the
    // wave is active here); a + b = b + a exactly, so all lanes of a drone
    // hold the same sum
    if (LPD >= 2) {
        const float o = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0xB1, 0xF, 0xF, true));
        acc = acc + o;
    }
    if (LPD >= 4) {
        const float o = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0x4E, 0xF, 0xF, true));
        acc = acc + o;
    }
    return acc;
}

}  // namespace phys
}  // namespace md
