// md_sweep.h -- the in-LDS neighbour sweep for the pairwise downwash of
// Eq. 6, shared by the semi-implicit Euler and the Runge-Kutta step kernels.
// Positions of a bin's drones are published to LDS; each drone sums the
// terms of the other drones of its environment in ascending slot order.
#pragma once

#include "md_physics.h"

namespace md {
namespace phys {

// This lane's share of the downwash sum over its environment's slots
// [lo, lo + mmax), in ascending order (every LPD-th slot from `sub`).  In a
// uniform bin every environment has mmax drones and the bound check is
// dropped.
template <bool DZMIN, int LPD, int UNROLL>
__device__ __forceinline__ float dw_sweep(const KConst &c, const float4 *buf, int lo, int sub, int mmax,
                                          int menv, bool uniform, const Drone &d) {
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
        const float t = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, fabsf(dz));
        T[slot * ts + lj] = dz > 0.f ? t : 0.f;
        T[(lo + lj) * ts + li] = dz < 0.f ? t : 0.f;
    }
    if ((m & 1) == 0 && li < (m >> 1) && m > 0) {
        const int lj = li + (m >> 1);
        const float4 pj = buf[lo + lj];
        const float dz = pj.z - d.pz;
        const float t = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, fabsf(dz));
        T[slot * ts + lj] = dz > 0.f ? t : 0.f;
        T[(lo + lj) * ts + li] = dz < 0.f ? t : 0.f;
    }
}

// Downwash sum (without K1) of this slot's drone against the positions in
// `buf`: the all-pairs sweep over LPD lanes (their partial sums combined in a
// fixed order) or the pair-symmetric sweep through the LDS term matrix (it
// contains the barrier between the term writes and the row sums).
template <int LPD, int UNROLL, bool SYM>
__device__ __forceinline__ float dw_sum(const KConst &c, const float4 *buf, float *tmat, int ts, int slot,
                                        int sub, int lo, int mmax, int menv, bool uniform, const Drone &d) {
    float acc = 0.f;
    if (SYM) {
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
    if (LPD >= 2) {
        const float o = __shfl_xor(acc, 1, 64);
        acc = (sub & 1) ? (o + acc) : (acc + o);
    }
    if (LPD >= 4) {
        const float o = __shfl_xor(acc, 2, 64);
        acc = (sub & 2) ? (o + acc) : (acc + o);
    }
    return acc;
}

}  // namespace phys
}  // namespace md
