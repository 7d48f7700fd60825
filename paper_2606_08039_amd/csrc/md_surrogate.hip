// md_surrogate.hip -- the learned aerodynamic residual inside the step.
//
// Three pieces share one feature builder:
//   datagen_kernel   features + the plain residual (Eq. 4-6 in the body frame)
//                    at the current state: the surrogate's training samples;
//   sur_step_kernel  the persistent step with Eq. 4-6 replaced by the network:
//                    per drone, 8 laterally nearest same-environment neighbours, 60 features,
//                    fp32 standardisation, bfloat16 rounding, then the 64-128-128-128-6
//                    network on MFMA (v_mfma_f32_16x16x32_bf16) for the wave's 64
//                    drones at once; a drone whose neighbour sits just above it
//                    (0 < dz < dz_ood, the downwash singularity) takes the plain terms
//                    instead (fallback); every judge_stride-th drone-step also
//                    evaluates the plain terms and accumulates the force error (judge).
//
// MFMA data flow per wave (64 drones = 4 column tiles of 16 drones):
//   Z^T[out][drone] = W[out][in] X^T[in][drone].  A operand = weight rows read
//   from global memory (L2-resident, 84 KB bf16 for all layers, stored
//   fragment-major so that each wave-wide fragment load is 1 KB in order, and
//   requested one output tile ahead of its use), B operand = activations.  The 16x16 C tile leaves lane l holding rows 4*(l/16)+t of
//   drone l%16, which is exactly half of the next layer's B fragment for a
//   32-wide K chunk; the host permutes the K columns of layers 2-4 to match,
//   so activations never leave registers between layers.
#include <cmath>
#include <cstring>
#include <vector>

#include "md_ctx.h"
#include "md_mlp.h"
#include "md_physics.h"

namespace md {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KNN = 8;
// Candidate lists: environments of at least LIST + 2 drones keep per drone its
// LIST laterally nearest (in ascending slot order) and rank only those while
// every drone of the bin stays within the list's margin (see knn_list).
constexpr int LIST = 12;
constexpr int LIST_MIN_ENV = LIST + 2;
static_assert(LIST % 2 == 0 && LIST <= 12, "a list is at most six words of 16-bit slot offsets");
constexpr int MAX_SLOTS = 512;  // environments of up to 512 drones
constexpr int MAX_BIN_WAVES = MAX_SLOTS / 64;
constexpr int FEAT_STRIDE = MLP_IN + 8;  // bf16 per staged feature row (144 B, 16 B aligned)
// floats between the output rows, which overwrite the start of each drone's
// input row once the network has read it (inputs and outputs of a pass
// belong to the same 32 drones, whose inputs are loaded at the pass's start)
constexpr int OUT_ROW = FEAT_STRIDE / 2;
constexpr int W4_ROWS = 16;
// offsets (in bf16 elements) of the permuted device weights
constexpr int WOFF1 = 0, WOFF2 = WOFF1 + MLP_H * MLP_IN, WOFF3 = WOFF2 + MLP_H * MLP_H,
              WOFF4 = WOFF3 + MLP_H * MLP_H, WTOTAL = WOFF4 + W4_ROWS * MLP_H;
constexpr int BOFF1 = 0, BOFF2 = 128, BOFF3 = 256, BOFF4 = 384, BTOTAL = 400;

enum { J_ERR2 = 0, J_REF2, J_TERR2, J_N, J_FALLBACK, J_STEPS, J_NONFINITE, J_FULLKNN, J_COUNT };

struct SurrogateState {
    bf16 *W = nullptr;      // permuted bf16 weights [WTOTAL], fragment-major per layer
    float *b = nullptr;     // biases [BTOTAL]
    float *norm = nullptr;  // x_mean[64], x_inv_std[64], y_mean[6], y_std[6]
    double *judge = nullptr;
    float dz_ood = 1e-3f;
    float ood_speed = 0.f, ood_rel = 0.f, ood_tilt_s = 0.f;  // 0: check off
    float near_dz = 0.f, near_r2 = 0.f, far_dz = 0.f;         // region fallback, 0: off
    int judge_stride = 64;
    bool knn_reuse = true;
    bool loaded = false;
};

struct SurArgs {
    StepArgs s;
    const bf16 *W;
    const float *b;
    const float *norm;
    double *judge;
    float dz_ood;
    float ood_speed, ood_rel;  // world speed / relative speed component bounds (0: off)
    float near_dz, near_r2, far_dz;  // region fallback (near_dz 0: cylinder off; far_dz 0: off)
    float ood_tilt_s;          // sin^2(max tilt / 2) (0: off)
    int judge_mask;  // judge_stride - 1 (power of two), or -1 for no judging
    int knn_reuse;   // candidate lists (1) or every drone ranked every step (0)
};

struct GenArgs {
    KConst c;
    StatePtr s;
    int N;
    BinTables bins;
    uint32_t mask;
    float *X;
    float *Y;
    int *nbr;
};

namespace {

using namespace phys;

__device__ __forceinline__ void load_drone(const StatePtr &s, int N, int di, Drone &d) {
    d.px = s.p[di];
    d.py = s.p[N + di];
    d.pz = s.p[2 * N + di];
    d.qw = s.q[di];
    d.qx = s.q[N + di];
    d.qy = s.q[2 * N + di];
    d.qz = s.q[3 * N + di];
    d.vx = s.v[di];
    d.vy = s.v[N + di];
    d.vz = s.v[2 * N + di];
    d.wx = s.w[di];
    d.wy = s.w[N + di];
    d.wz = s.w[2 * N + di];
}

// Squared horizontal distance of a candidate, formed as dx*dx + dy*dy with
// every operation rounded (no fused multiply-add), as the oracle forms it, so
// both sides take the same integer decisions.  The empty asm keeps the
// arithmetic from being moved under the caller's branch on the candidate.
__device__ __forceinline__ float knn_d2(float4 pj, float px, float py) {
#pragma clang fp contract(off)
    const float dx = pj.x - px, dy = pj.y - py;
    const float a = dx * dx, b = dy * dy;
    float d2 = a + b;
    asm volatile("" : "+v"(d2));
    return d2;
}

// One candidate into the ascending list (bd, bj) of the K nearest seen so
// far.  Candidates arrive in ascending slot order and a candidate enters
// only below a strictly larger distance, so ties go to the lower slot (=
// the lower drone index).  bd is sorted, so the kept, shifted or inserted
// distance of slot t is the median of bd[t - 1], bd[t] and d2.
template <int K>
__device__ __forceinline__ void knn_insert(float d2, int j, float (&bd)[K], int (&bj)[K]) {
    // slots from the last down: the comparison of slot t - 1 is taken before
    // that slot changes, and only two comparisons are live at a time
    bool cn = d2 < bd[K - 1];
#pragma unroll
    for (int t = K - 1; t >= 1; --t) {
        const bool cp = d2 < bd[t - 1];
        bd[t] = __builtin_amdgcn_fmed3f(bd[t - 1], bd[t], d2);
        bj[t] = cn ? (cp ? bj[t - 1] : j) : bj[t];
        cn = cp;
    }
    bd[0] = cn ? d2 : bd[0];
    bj[0] = cn ? j : bj[0];
}

// The K nearest neighbours by horizontal distance among the environment's
// slots [lo, lo + m) other than self, ascending, ties to the lower slot.
// Lateral metric: the downwash (Eq. 6) varies with the lateral offset on the
// centimetre scale of beta and with the height difference on the metre
// scale, so the laterally closest drones are the ones that matter, and a
// drone's column partner always lands in the first input slot.  Masked and
// non-finite candidates become +inf, which never enters.
template <int K>
__device__ __forceinline__ void knn_sweep(const float4 *pos, int lo, int m, int mmax, int self, float px, float py,
                                          float (&bd)[K], int (&bj)[K]) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
        bd[t] = __builtin_inff();
        bj[t] = -1;
    }
    for (int jj = 0; jj < mmax; ++jj) {
        const int j = lo + jj;
        // read and formed by every lane (the position buffer holds 2 entries
        // per slot, so lo + jj stays inside it)
        float d2 = knn_d2(pos[j], px, py);
        d2 = (jj < m && j != self && d2 < __builtin_inff()) ? d2 : __builtin_inff();
        knn_insert<K>(d2, j, bd, bj);
    }
}

// The 8 nearest from a drone's candidate list: LIST (at most 12) 16-bit slot
// offsets from lo in ascending order, 2 per word; unused entries hold the
// drone's own offset (never a member).  Ranking the list in slot order gives
// exactly knn_sweep's result whenever every drone the sweep would pick is on
// the list (the caller's margin test).
__device__ __forceinline__ void knn_list(const float4 *pos, int lo, int self, const uint32_t (&L)[6], float px,
                                         float py, int (&bj)[KNN]) {
    float bd[KNN];
#pragma unroll
    for (int t = 0; t < KNN; ++t) {
        bd[t] = __builtin_inff();
        bj[t] = -1;
    }
#pragma unroll
    for (int t = 0; t < LIST; ++t) {
        const int j = lo + (int)((L[t >> 1] >> (16 * (t & 1))) & 0xffffu);
        const bool on = j != self;
        float d2 = knn_d2(pos[j], px, py);
        d2 = (on && d2 < __builtin_inff()) ? d2 : __builtin_inff();
        knn_insert<KNN>(d2, j, bd, bj);
    }
}

// Fixed-order reductions over the 64 lanes of a wave (all lanes active):
// pairs, quads, half rows and rows through DPP, then rows 1 and 3 take row
// 0's and row 2's total (row_bcast:15) and row 3 takes rows 0-1's
// (row_bcast:31); the result is lane 63's, returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

template <class Op>
__device__ __forceinline__ float wave_reduce(float x, Op op) {
    x = op(x, dpp_mov<0xb1, 0xf>(x));   // quad_perm [1, 0, 3, 2]
    x = op(x, dpp_mov<0x4e, 0xf>(x));   // quad_perm [2, 3, 0, 1]
    x = op(x, dpp_mov<0x141, 0xf>(x));  // row_half_mirror
    x = op(x, dpp_mov<0x140, 0xf>(x));  // row_mirror
    const float b15 = dpp_mov<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x = (threadIdx.x & 16) ? op(x, b15) : x;
    const float b31 = dpp_mov<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    x = (threadIdx.x & 32) ? op(x, b31) : x;
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Raw surrogate inputs (see md.h): v_body, world up in the body frame, n/HOVER,
// 8 x (dp, dv) of the nearest neighbours (world frame, zero if missing), z,
// ground proximity (h_clip / max(z, h_clip))^2, 0-pad.
// Returns whether a neighbour sits above within (0, dz_ood), inside the
// cylinder |dz| < near_dz, dxy^2 < near_r2 (near_dz > 0), beyond |dz| >
// far_dz (far_dz > 0), or (ood_rel > 0) moves relative to the drone faster
// than ood_rel along an axis.  dz is the exact difference of the stored
// heights and dxy^2 is formed as the neighbour ranking forms it, so the oracle
// takes the same decisions.
__device__ __forceinline__ bool features(const KConst &c, const Drone &d, const Rot &R, const float n[4],
                                         const float4 *pos, const float4 *vel, const int bj[KNN],
                                         float dz_ood, float ood_rel, float near_dz, float near_r2,
                                         float far_dz, float f[MLP_IN]) {
    f[0] = R.r00 * d.vx + R.r10 * d.vy + R.r20 * d.vz;
    f[1] = R.r01 * d.vx + R.r11 * d.vy + R.r21 * d.vz;
    f[2] = R.r02 * d.vx + R.r12 * d.vy + R.r22 * d.vz;
    f[3] = R.r20;
    f[4] = R.r21;
    f[5] = R.r22;
#pragma unroll
    for (int k = 0; k < 4; ++k) f[6 + k] = n[k] * c.hover_inv;
    bool ood = false;
#pragma unroll
    for (int t = 0; t < KNN; ++t) {
        const int j = bj[t];
        float4 pj = make_float4(0.f, 0.f, 0.f, 0.f), vj = pj;
        if (j >= 0) {
            pj = pos[j];
            vj = vel[j];
        }
        const bool h = j >= 0;
        const float dz = pj.z - d.pz;
        f[10 + 6 * t + 0] = h ? pj.x - d.px : 0.f;
        f[10 + 6 * t + 1] = h ? pj.y - d.py : 0.f;
        f[10 + 6 * t + 2] = h ? dz : 0.f;
        f[10 + 6 * t + 3] = h ? vj.x - d.vx : 0.f;
        f[10 + 6 * t + 4] = h ? vj.y - d.vy : 0.f;
        f[10 + 6 * t + 5] = h ? vj.z - d.vz : 0.f;
        ood |= h && dz > 0.f && dz < dz_ood;
        const float d2 = knn_d2(pj, d.px, d.py);
        ood |= h && near_dz > 0.f && fabsf(dz) < near_dz && d2 < near_r2;
        ood |= h && far_dz > 0.f && fabsf(dz) > far_dz;
        ood |= h && ood_rel > 0.f &&
               (fabsf(f[10 + 6 * t + 3]) > ood_rel || fabsf(f[10 + 6 * t + 4]) > ood_rel ||
                fabsf(f[10 + 6 * t + 5]) > ood_rel);
    }
    f[58] = d.pz;
    const float gp = c.h_clip / fmaxf(d.pz, c.h_clip);
    f[59] = gp * gp;
#pragma unroll
    for (int k = 60; k < MLP_IN; ++k) f[k] = 0.f;
    return ood;
}

// Plain aerodynamic residual of the selected effects (world frame): ground
// effect, drag, and the downwash sweep over the environment in ascending order.
__device__ __forceinline__ void plain_aero(const KConst &c, uint32_t mask, const Drone &d, const Rot &R,
                                           const float n[4], float T, const float4 *pos, int lo, int m,
                                           int mmax, float &Fx, float &Fy, float &Fz) {
    Fx = Fy = Fz = 0.f;
    if (mask & 1u) Fz += ground_effect(c, d, R, T);
    if (mask & 2u) {
        float dx, dy, dz;
        drag(c, d, R, n, dx, dy, dz);
        Fx += dx;
        Fy += dy;
        Fz += dz;
    }
    if (mask & 4u) {
        float acc = 0.f;
        for (int j = 0; j < mmax; ++j) {
            const float4 pj = pos[lo + j];
            const float term = c.dz_min > 0.f ? dw_term<true>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz)
                                              : dw_term<false>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
            acc += (j < m) ? term : 0.f;
        }
        Fz -= c.K1 * acc;
    }
}

// The plain downwash sum (Eq. 6, without K1) of every lane with `need`, the
// whole wave evaluating one such drone at a time: lane l takes environment
// slots l, l + 64, ... of that drone's environment, and the 64 partial sums
// are added in wave_reduce's fixed tree, so a drone's sum depends only on its
// place in its environment, not on the packing.  Costs one pass per drone
// that needs it instead of a sweep by every lane of the wave whenever one
// lane does.  All lanes must be active.
__device__ __forceinline__ float dw_coop(const KConst &c, const float4 *pos, bool need, int lo, int m,
                                         const Drone &d) {
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(need);
    float mine = 0.f;
    while (todo) {
        const int f = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int flo = __builtin_amdgcn_readlane(lo, f), fm = __builtin_amdgcn_readlane(m, f);
        const float fx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d.px), f));
        const float fy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d.py), f));
        const float fz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d.pz), f));
        float acc = 0.f;
        for (int base = 0; base < fm; base += 64) {
            const int j = base + lane;
            const float4 pj = pos[flo + min(j, fm - 1)];
            const float t = c.dz_min > 0.f ? dw_term<true>(c, pj.x - fx, pj.y - fy, pj.z - fz)
                                           : dw_term<false>(c, pj.x - fx, pj.y - fy, pj.z - fz);
            acc += (j < fm) ? t : 0.f;  // the drone's own slot has dz = 0: no term
        }
        const float sum = wave_reduce(acc, [](float a, float b) { return a + b; });
        mine = (lane == f) ? sum : mine;
    }
    return mine;
}

// qx^2 + qy^2 = sin^2(tilt / 2) with every operation rounded (no fused
// multiply-add), the value the tilt fallback compares.
__device__ __forceinline__ float tilt_sq(const Drone &d) {
#pragma clang fp contract(off)
    const float a = d.qx * d.qx, b = d.qy * d.qy;
    return a + b;
}

// Weight fragments are read through a global (address space 1) pointer, so
// that their loads count on the vector-memory counter alone and the wait for
// one fragment does not also wait for the LDS traffic in flight.
typedef const __attribute__((address_space(1))) bf16x8 gbf16x8;
typedef const __attribute__((address_space(1))) f32x4 gf32x4;

__device__ __forceinline__ bf16x8 ldw(const bf16 *p) { return *(gbf16x8 *)p; }

__device__ __forceinline__ f32x4 ldb(const float *p) { return *(gf32x4 *)p; }

// Drone tiles (16 drones each) evaluated together by one pass of the network.
constexpr int DT = 2;

// The network as a stream of output-tile jobs: 8 tiles of 16 rows per hidden
// layer (layers 1-3) and one for the output layer, 25 per pass.  A job needs
// its weight fragments (A operands, one per 32-wide K chunk: 2 for layer 1,
// 4 otherwise) and its 16 biases.
constexpr int N_JOBS = 3 * 8 + 1;

struct WFrag {
    bf16x8 a[4];
    f32x4 b;
};

__device__ __forceinline__ void load_job(WFrag &w, const bf16 *W, const float *b, int j, int r, int g) {
    const int layer = j / 8, ot = j % 8;
    const int kcs = layer == 0 ? 2 : 4;
    const int woff = layer == 0 ? WOFF1 : layer == 1 ? WOFF2 : layer == 2 ? WOFF3 : WOFF4;
    const int boff = layer == 0 ? BOFF1 : layer == 1 ? BOFF2 : layer == 2 ? BOFF3 : BOFF4;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
        if (kc < kcs) w.a[kc] = ldw(W + woff + ((ot * kcs + kc) * 64 + 16 * g + r) * 8);
    w.b = ldb(b + boff + 16 * ot + 4 * g);
}

// The network on the 64 drones of one wave, DT tiles of 16 drones per pass:
// standardised bfloat16 inputs in feat (row per drone), standardised outputs
// to out (row per drone, 6 used).  Passes reuse the activation registers;
// the weights (L2-resident) are read once per pass.  The weight stream is
// software pipelined: the fragments of job j + 1 are requested before the
// MFMAs of job j, and scheduling fences keep them there, so every L2 round
// trip overlaps a job's work instead of stalling it.
__device__ __forceinline__ void mlp_wave(const bf16 *feat, float *out, const bf16 *W, const float *b, int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll 1
    for (int pass = 0; pass < 4 / DT; ++pass) {
        const int t0 = pass * DT;
        // an empty asm operand makes the weight pointers opaque per pass, so the
        // (loop-invariant) weight loads are not hoisted out of the pass loop,
        // which would hold all 84 KB of weights in registers
        const bf16 *Wv = W;
        const float *bv_ = b;
        asm volatile("" : "+s"(Wv), "+s"(bv_));
        WFrag cur, nxt;
        load_job(cur, Wv, bv_, 0, r, g);
        // layer 1 B fragments straight from the staged rows (K = 64)
        bf16x8 x[2][DT];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
#pragma unroll
            for (int dt = 0; dt < DT; ++dt)
                x[kc][dt] = *(const bf16x8 *)(feat + (16 * (t0 + dt) + r) * FEAT_STRIDE + 32 * kc + 8 * g);
        bf16x4 h1[8][DT], h2[8][DT];
        // SiLU epilogue of a hidden-layer job: layers 1 and 3 write h1, layer 2 h2
        // four SiLUs at a time, each stage fenced, so that the four chains
        // interleave (the exponential and the reciprocal of one SiLU hide the
        // others' latency instead of a no-op per transcendental)
        auto epilogue = [&](int jj, const f32x4 (&ac)[DT]) {
            const int layer = jj / 8, ot = jj % 8;
            bf16x4(&hout)[8][DT] = layer == 1 ? h2 : h1;
#pragma unroll
            for (int dt = 0; dt < DT; ++dt) {
                float e[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) e[t] = __expf(-ac[dt][t]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 4; ++t) e[t] = __builtin_amdgcn_rcpf(1.f + e[t]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 4; ++t) hout[ot][dt][t] = (bf16)(ac[dt][t] * e[t]);
            }
        };
        f32x4 prev[DT];
#pragma unroll
        for (int j = 0; j < N_JOBS; ++j) {
            const int layer = j / 8, ot = j % 8;
            if (j + 1 < N_JOBS) load_job(nxt, Wv, bv_, j + 1, r, g);
            // the first job of a layer reads every tile of the previous one
            if (j > 0 && ot == 0) epilogue(j - 1, prev);
            __builtin_amdgcn_sched_barrier(0);
            f32x4 acc[DT];
            if (layer == 0) {
#pragma unroll
                for (int kc = 0; kc < 2; ++kc)
#pragma unroll
                    for (int dt = 0; dt < DT; ++dt)
                        acc[dt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.a[kc], x[kc][dt], kc == 0 ? cur.b : acc[dt],
                                                                          0, 0, 0);
            } else {
                // layers 2 and 4 read h1, layer 3 reads h2
                const bf16x4(&hin)[8][DT] = layer == 2 ? h2 : h1;
#pragma unroll
                for (int kc = 0; kc < 4; ++kc)
#pragma unroll
                    for (int dt = 0; dt < DT; ++dt) {
                        const bf16x8 bv =
                            __builtin_shufflevector(hin[2 * kc][dt], hin[2 * kc + 1][dt], 0, 1, 2, 3, 4, 5, 6, 7);
                        acc[dt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.a[kc], bv, kc == 0 ? cur.b : acc[dt], 0,
                                                                          0, 0);
                    }
            }
            // within a layer the previous job's epilogue runs while this
            // job's MFMAs occupy the matrix pipe
            if (ot > 0) epilogue(j - 1, prev);
            if (j == N_JOBS - 1) {
                // output layer: rows 0..5 used; bias rows 6..15 are 0
#pragma unroll
                for (int dt = 0; dt < DT; ++dt)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int o = 4 * g + t;
                        if (o < MLP_OUT) out[(16 * (t0 + dt) + r) * OUT_ROW + o] = acc[dt][t];
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int dt = 0; dt < DT; ++dt) prev[dt] = acc[dt];
            if (j + 1 < N_JOBS) cur = nxt;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int ACT>
__global__ void __launch_bounds__(MAX_SLOTS) sur_step_kernel(SurArgs sa) {
    const StepArgs &a = sa.s;
    const KConst &c0 = a.c;
    const int S = blockDim.x;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // LDS (248 bytes per slot: eight one-wave workgroups fit a CU's 160 KB,
    // a 512-slot bin 124 KB)
    float4 *posb = (float4 *)smem;              // [2][2S] positions, double buffered
    float4 *vel = posb + 4 * S;                 // [S] velocities (read before the step's second barrier)
    bf16 *feat = (bf16 *)(vel + S);             // [S][FEAT_STRIDE] network inputs; a row's first
                                                // 24 bytes then take its outputs (OUT_ROW floats apart)
    uint2 *lst = (uint2 *)(feat + S * FEAT_STRIDE);   // [3][S] candidate lists, 12 16-bit slot offsets
    float *wred = (float *)(lst + 3 * S);             // [2][2][MAX_BIN_WAVES] per-wave max / min
    const int slot = threadIdx.x, lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
    const int wave = threadIdx.x >> 6, n_waves = S >> 6;
    const int2 tab = a.bins.slot[blockIdx.x * S + slot];
    const int di = tab.x;
    const bool valid = di >= 0;
    const int lo = tab.y >> 16, menv = tab.y & 0xffff;
    const int mmax = a.bins.bin_mmax[blockIdx.x] & 0xffff;
    const int N = a.N;
    // device normalisation layout: x_inv_std[64], -x_mean * x_inv_std[64], y_mean[6], y_std[6]

    Drone d{};
    d.qw = 1.f;
    float I[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float n[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
        load_drone(a.s, N, di, d);
        for (int k = 0; k < 4; ++k) n[k] = a.s.rpm[k * N + di];
        if (ACT >= 1)
            for (int k = 0; k < 6; ++k) I[k] = a.s.pid_int[k * N + di];
    }
    const bool held = a.act_step_stride == 0;
    constexpr int ROWS = action_rows(ACT);
    float tgt_held[ROWS];
    float sp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ROWS; ++k) tgt_held[k] = 0.f;
    if (ACT >= 1 && held && valid)
        for (int k = 0; k < ROWS; ++k) tgt_held[k] = a.action[(long long)k * N + di];
    if (ACT == 4 && valid)
        for (int k = 0; k < 4; ++k) sp[k] = a.s.ctl[k * N + di];
    // per-lane judge sums (a lane judges at most one step in judge_stride)
    // and counts, combined in double at the end
    float jerr = 0.f, jref = 0.f, jterr = 0.f;
    int jn = 0, jfb = 0, jnf = 0;
    int nfull = 0;  // drone-steps that ranked the whole environment
    int phase = (ACT >= 1) ? (int)(a.step0 % (long long)c0.decim) : 0;
    int oslot = 0;
    // Candidate lists (bins whose largest environment has at least
    // LIST_MIN_ENV drones).  At a rebuild every drone ranks its whole
    // environment, keeps its LIST nearest (lateral distances, in slot order)
    // and records where it stood (bx, by) and its margin
    //   slack = (r_LIST - r_8) / 4
    // (r_k its k-th nearest distance).  While the bin's largest lateral
    // displacement since the rebuild, D, stays below the bin's smallest
    // slack, ranking the list gives exactly the sweep's 8 nearest: each of
    // the 8 nearest at the rebuild is now within r_8 + 2D, so the current
    // 8th distance is at most that, while a drone off the list is at least
    // r_LIST - 2D > r_8 + 2D away.  Margins are shrunk by 2^-18 against the
    // float32 rounding of the distances.  Rebuilds are bin-wide, so that every
    // displacement counts from the same step.
    const bool use_list = sa.knn_reuse && mmax >= LIST_MIN_ENV;
    float bx = d.px, by = d.py;
    float S2 = -1.f;     // the bin's smallest slack squared (< 0: rebuild)
    bool fresh = false;  // a rebuild in the previous step left its wave minima in wred
    for (int step = 0; step < a.n_steps; ++step) {
        const KConst &c = c0;
        const int par = step & 1;
        float4 *pos = posb + par * 2 * S;
        pos[slot] = make_float4(d.px, d.py, d.pz, 0.f);
        vel[slot] = make_float4(d.vx, d.vy, d.vz, 0.f);
        if (use_list) {
            // lateral displacement since the rebuild (non-finite: +inf, a rebuild)
            const float ex = d.px - bx, ey = d.py - by;
            float e2 = valid ? ex * ex + ey * ey : 0.f;
            e2 = e2 < __builtin_inff() ? e2 : __builtin_inff();
            const float wmax = wave_reduce(e2, [](float u, float v) { return fmaxf(u, v); });
            if (lane == 0) wred[(par * 2 + 0) * MAX_BIN_WAVES + wave] = wmax;
        }
        __syncthreads();
        const float *act = a.action + a.act_step_stride * step;
        if (ACT == 0) {
            if (valid)
                for (int k = 0; k < 4; ++k) n[k] = clampf(act[(long long)k * N + di], 0.f, c.max_rpm);
        } else {
            if (phase == 0 && valid) {
                float cmd[ROWS];
                for (int k = 0; k < ROWS; ++k) cmd[k] = held ? tgt_held[k] : act[(long long)k * N + di];
                control<ACT>(c, d, cmd, I, sp, n);
            }
            phase = (phase + 1 == c.decim) ? 0 : phase + 1;
        }
        // ---- neighbours: the candidate list, or the whole environment
        int bj[KNN];
        bool rebuild = true;
        if (use_list) {
            float D2 = 0.f;
            for (int w = 0; w < n_waves; ++w) D2 = fmaxf(D2, wred[(par * 2 + 0) * MAX_BIN_WAVES + w]);
            if (fresh) {
                // the rebuild's wave minima, written before this step's barrier
                float sm = __builtin_inff();
                for (int w = 0; w < n_waves; ++w) sm = fminf(sm, wred[((par ^ 1) * 2 + 1) * MAX_BIN_WAVES + w]);
                S2 = sm > 0.f ? sm * sm : -1.f;
                fresh = false;
            }
            rebuild = !(D2 < S2);
        }
        if (!use_list) {
            float bd[KNN];
            knn_sweep<KNN>(pos, lo, menv, mmax, slot, d.px, d.py, bd, bj);
        } else if (rebuild) {
            float bd[LIST];
            int bl[LIST];
            knn_sweep<LIST>(pos, lo, menv, mmax, slot, d.px, d.py, bd, bl);
#pragma unroll
            for (int t = 0; t < KNN; ++t) bj[t] = bl[t];
            // the list in slot order: every candidate at or before the LIST-th
            // in (distance, slot) order, found by a second pass
            const float r2 = bd[LIST - 1];
            const int rj = bl[LIST - 1];
            const uint32_t own = (uint32_t)(slot - lo) * 0x00010001u;  // unused entries: self
            uint32_t L[6] = {own, own, own, own, own, own};
            int cnt = 0;
            for (int jj = 0; jj < mmax; ++jj) {
                const int j = lo + jj;
                const float d2 = knn_d2(pos[j], d.px, d.py);
                const bool in = jj < menv && j != slot && d2 < __builtin_inff() &&
                                (rj < 0 || d2 < r2 || (d2 == r2 && j <= rj));
                if (in) {
                    // entry cnt of the list (at most LIST candidates pass)
                    const int w = cnt >> 1, sh = 16 * (cnt & 1);
                    const uint32_t v = (uint32_t)jj << sh, keep = ~(0xffffu << sh);
#pragma unroll
                    for (int q = 0; q < 6; ++q) L[q] = w == q ? ((L[q] & keep) | v) : L[q];
                    ++cnt;
                }
            }
            lst[slot] = make_uint2(L[0], L[1]);
            lst[S + slot] = make_uint2(L[2], L[3]);
            lst[2 * S + slot] = make_uint2(L[4], L[5]);
            // margin of this drone (+inf when the list holds its whole environment)
            float slack = __builtin_inff();
            if (valid && r2 < __builtin_inff())
                slack = 0.25f * (fsqrt(r2) * (1.f - 0x1p-18f) - fsqrt(bd[KNN - 1]) * (1.f + 0x1p-18f));
            slack = slack == slack ? slack : -1.f;
            const float wmin = wave_reduce(slack, [](float u, float v) { return fminf(u, v); });
            if (lane == 0) wred[(par * 2 + 1) * MAX_BIN_WAVES + wave] = wmin;
            fresh = true;
            S2 = -1.f;
            bx = d.px;
            by = d.py;
        } else {
            const uint2 l0 = lst[slot], l1 = lst[S + slot], l2 = lst[2 * S + slot];
            const uint32_t L[6] = {l0.x, l0.y, l1.x, l1.y, l2.x, l2.y};
            knn_list(pos, lo, slot, L, d.px, d.py, bj);
        }
        nfull += (valid && rebuild) ? 1 : 0;
        // ---- features -> standardised bfloat16 row
        bool ood;
        float f[MLP_IN];
        {
            const Rot R = rot_of(d);
            ood = features(c, d, R, n, pos, vel, bj, sa.dz_ood, sa.ood_rel, sa.near_dz, sa.near_r2, sa.far_dz, f);
        }
        // outside the trained region: fast or tilted drones take the plain terms
        ood |= sa.ood_speed > 0.f &&
               (fabsf(d.vx) > sa.ood_speed || fabsf(d.vy) > sa.ood_speed || fabsf(d.vz) > sa.ood_speed);
        ood |= sa.ood_tilt_s > 0.f && tilt_sq(d) > sa.ood_tilt_s;
        ood = ood && valid;
        bf16 *row = feat + slot * FEAT_STRIDE;
        // the normalisation is read here each step rather than held in
        // scalar registers for the launch (the empty asm keeps the loads in
        // the loop), which leaves the scalar registers to the step's constants
        const float *nrm = sa.norm;
        asm volatile("" : "+s"(nrm));
#pragma unroll
        for (int k = 0; k < MLP_IN; k += 8) {
            bf16x8 v;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                v[t] = valid ? (bf16)fmaf(f[k + t], nrm[k + t], nrm[MLP_IN + k + t]) : (bf16)0.f;
            *(bf16x8 *)(row + k) = v;
        }
        __syncthreads();
        mlp_wave(feat + wbase * FEAT_STRIDE, (float *)(feat + wbase * FEAT_STRIDE), sa.W, sa.b, lane);
        __syncthreads();
        // the rotation and the rotor terms are formed from the (unchanged)
        // attitude and rotor speeds after the network instead of being held in
        // registers across it; the empty asm keeps them from being reused
        asm volatile("" : "+v"(d.qw), "+v"(d.qx), "+v"(d.qy), "+v"(d.qz), "+v"(n[0]), "+v"(n[1]), "+v"(n[2]),
                     "+v"(n[3]));
        float T, tx, ty, tz;
        motor(c, n, T, tx, ty, tz);
        const Rot R = rot_of(d);
        float y[MLP_OUT];
#pragma unroll
        for (int o = 0; o < MLP_OUT; ++o)
            y[o] = ((const float *)feat)[slot * OUT_ROW + o] * nrm[2 * MLP_IN + MLP_OUT + o] + nrm[2 * MLP_IN + o];
        float Fx = R.r02 * T, Fy = R.r12 * T, Fz = R.r22 * T - c.mg;
        float ax, ay, az;
        // surrogate force, body -> world
        const float sx = R.r00 * y[0] + R.r01 * y[1] + R.r02 * y[2];
        const float sy = R.r10 * y[0] + R.r11 * y[1] + R.r12 * y[2];
        const float sz = R.r20 * y[0] + R.r21 * y[1] + R.r22 * y[2];
        const bool judge = valid && !ood && sa.judge_mask >= 0 &&
                           (((unsigned)di + (unsigned)(a.step0 + step)) & (unsigned)sa.judge_mask) == 0u;
        // plain terms for the drones that fall back or are judged: ground
        // effect and drag per lane, the downwash sweep by the whole wave per drone
        float px_ = 0.f, py_ = 0.f, pz_ = 0.f;
        const float dws = dw_coop(c, pos, ood || judge, lo, menv, d);
        if (ood || judge) {
            plain_aero(c, 3u, d, R, n, T, pos, lo, menv, mmax, px_, py_, pz_);
            pz_ -= c.K1 * dws;
        }
        if (ood) {
            ax = px_;
            ay = py_;
            az = pz_;
            jfb += 1;
        } else {
            ax = sx;
            ay = sy;
            az = sz;
            tx += y[3];
            ty += y[4];
            tz += y[5];
        }
        if (judge) {
            const float ex = sx - px_, ey = sy - py_, ez = sz - pz_;
            const float e2 = ex * ex + ey * ey + ez * ez, r2 = px_ * px_ + py_ * py_ + pz_ * pz_;
            const float t2 = y[3] * y[3] + y[4] * y[4] + y[5] * y[5];
            // a non-finite sample (a state that has left every sensible range)
            // is counted apart so that it cannot poison the sums
            const bool fin = __builtin_isfinite(e2) && __builtin_isfinite(r2) && __builtin_isfinite(t2);
            jerr += fin ? e2 : 0.f;
            jref += fin ? r2 : 0.f;
            jterr += fin ? t2 : 0.f;
            jn += fin ? 1 : 0;
            jnf += fin ? 0 : 1;
        }
        Fx += ax;
        Fy += ay;
        Fz += az;
        integrate(c, d, Fx, Fy, Fz, tx, ty, tz);
        if (a.obs != nullptr && valid) {
            float roll, pitch, yaw;
            euler_zyx(d, roll, pitch, yaw);
            const float rowo[20] = {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, roll, pitch, yaw,
                                    d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, n[0], n[1], n[2], n[3]};
            store_obs(a.obs, oslot, N, di, rowo);
        }
        oslot = (oslot + 1 == a.n_obs_slots) ? 0 : oslot + 1;
    }
    if (valid) {
        a.s.p[di] = d.px;
        a.s.p[N + di] = d.py;
        a.s.p[2 * N + di] = d.pz;
        a.s.q[di] = d.qw;
        a.s.q[N + di] = d.qx;
        a.s.q[2 * N + di] = d.qy;
        a.s.q[3 * N + di] = d.qz;
        a.s.v[di] = d.vx;
        a.s.v[N + di] = d.vy;
        a.s.v[2 * N + di] = d.vz;
        a.s.w[di] = d.wx;
        a.s.w[N + di] = d.wy;
        a.s.w[2 * N + di] = d.wz;
        for (int k = 0; k < 4; ++k) a.s.rpm[k * N + di] = n[k];
        if (ACT >= 1)
            for (int k = 0; k < 6; ++k) a.s.pid_int[k * N + di] = I[k];
        if (ACT == 4)
            for (int k = 0; k < 4; ++k) a.s.ctl[k * N + di] = sp[k];
    }
    if (sa.judge != nullptr) {
        const double s0 = wave_sum((double)jerr), s1 = wave_sum((double)jref), s2 = wave_sum((double)jterr),
                     s3 = wave_sum((double)jn), s4 = wave_sum((double)jfb), s5 = wave_sum((double)jnf);
        const double steps = wave_sum(valid ? (double)a.n_steps : 0.0);
        const double s6 = wave_sum((double)nfull);
        if (lane == 0) {
            atomicAdd(sa.judge + J_FULLKNN, s6);
            atomicAdd(sa.judge + J_ERR2, s0);
            atomicAdd(sa.judge + J_REF2, s1);
            atomicAdd(sa.judge + J_TERR2, s2);
            atomicAdd(sa.judge + J_N, s3);
            atomicAdd(sa.judge + J_FALLBACK, s4);
            atomicAdd(sa.judge + J_STEPS, steps);
            atomicAdd(sa.judge + J_NONFINITE, s5);
        }
    }
}

__global__ void __launch_bounds__(MAX_SLOTS) datagen_kernel(GenArgs g) {
    const KConst &c = g.c;
    const int S = blockDim.x;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float4 *pos = (float4 *)smem;  // [2S]
    float4 *vel = pos + 2 * S;     // [2S]
    const int slot = threadIdx.x;
    const int2 tab = g.bins.slot[blockIdx.x * S + slot];
    const int di = tab.x;
    const bool valid = di >= 0;
    const int lo = tab.y >> 16, menv = tab.y & 0xffff;
    const int mmax = g.bins.bin_mmax[blockIdx.x] & 0xffff;
    Drone d{};
    d.qw = 1.f;
    float n[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
        load_drone(g.s, g.N, di, d);
        for (int k = 0; k < 4; ++k) n[k] = g.s.rpm[k * g.N + di];
    }
    pos[slot] = make_float4(d.px, d.py, d.pz, 0.f);
    vel[slot] = make_float4(d.vx, d.vy, d.vz, 0.f);
    pos[S + slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    vel[S + slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    if (!valid) return;
    float T, tx, ty, tz;
    motor(c, n, T, tx, ty, tz);
    const Rot R = rot_of(d);
    int bj[KNN];
    {
        float bd[KNN];
        knn_sweep<KNN>(pos, lo, menv, mmax, slot, d.px, d.py, bd, bj);
    }
    float f[MLP_IN];
    (void)features(c, d, R, n, pos, vel, bj, 0.f, 0.f, 0.f, 0.f, 0.f, f);
    float *x = g.X + (long long)di * MLP_IN;
#pragma unroll
    for (int k = 0; k < MLP_IN; k += 4) *(float4 *)(x + k) = make_float4(f[k], f[k + 1], f[k + 2], f[k + 3]);
    float Fx, Fy, Fz;
    plain_aero(c, g.mask, d, R, n, T, pos, lo, menv, mmax, Fx, Fy, Fz);
    float *y = g.Y + (long long)di * MLP_OUT;
    y[0] = R.r00 * Fx + R.r10 * Fy + R.r20 * Fz;
    y[1] = R.r01 * Fx + R.r11 * Fy + R.r21 * Fz;
    y[2] = R.r02 * Fx + R.r12 * Fy + R.r22 * Fz;
    y[3] = 0.f;
    y[4] = 0.f;
    y[5] = 0.f;
    if (g.nbr) {
        // neighbour slots back to drone indices: same environment, same offset
        const int base = di - (slot - lo);
        for (int t = 0; t < KNN; ++t) g.nbr[(long long)di * KNN + t] = bj[t] >= 0 ? base + (bj[t] - lo) : -1;
    }
}

}  // namespace

size_t sur_lds_bytes(int S) {
    return sizeof(float4) * 5 * (size_t)S + sizeof(bf16) * (size_t)S * FEAT_STRIDE + sizeof(uint2) * 3 * (size_t)S +
           sizeof(float) * 4 * MAX_BIN_WAVES;
}

template <int ACT>
hipError_t launch_sur_act(const SurArgs &sa, int n_bins, int S, size_t lds, hipStream_t st) {
    if (lds > 65536) {
        // bins of more than 256 slots take more than 64 KB of LDS
        const hipError_t e = hipFuncSetAttribute((const void *)sur_step_kernel<ACT>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sur_step_kernel<ACT>, dim3(n_bins), dim3(S), lds, st, sa);
    return hipGetLastError();
}

hipError_t launch_sur_step(const SurArgs &sa, int act, int n_bins, int S, hipStream_t st) {
    const size_t lds = sur_lds_bytes(S);
    switch (act) {
        case 0: return launch_sur_act<0>(sa, n_bins, S, lds, st);
        case 1: return launch_sur_act<1>(sa, n_bins, S, lds, st);
        case 2: return launch_sur_act<2>(sa, n_bins, S, lds, st);
        case 3: return launch_sur_act<3>(sa, n_bins, S, lds, st);
        default: return launch_sur_act<4>(sa, n_bins, S, lds, st);
    }
}

hipError_t launch_datagen(const GenArgs &g, int n_bins, int S, hipStream_t st) {
    hipLaunchKernelGGL(datagen_kernel, dim3(n_bins), dim3(S), sizeof(float4) * 4 * (size_t)S, st, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host side

// Hidden unit that feeds slot s (0..31) of a 32-wide K chunk when the
// previous layer's C tiles are used as B fragments in place (see top).
static int permuted_unit(int s) {
    const int g = s / 8, t = s % 8;
    return t < 4 ? 4 * g + t : 16 + 4 * g + (t - 4);
}

static md_status sur_alloc(md_ctx *ctx) {
    if (!ctx->sur) ctx->sur = new (std::nothrow) SurrogateState();
    if (!ctx->sur) return MD_E_OOM;
    SurrogateState *S = ctx->sur;
    if (S->W) return MD_OK;
    hipError_t e = hipMalloc(&S->W, sizeof(bf16) * WTOTAL);
    if (e == hipSuccess) e = hipMalloc(&S->b, sizeof(float) * BTOTAL);
    if (e == hipSuccess) e = hipMalloc(&S->norm, sizeof(float) * MLP_NORM);
    if (e == hipSuccess) e = hipMalloc(&S->judge, sizeof(double) * J_COUNT);
    if (e == hipSuccess) e = hipMemset(S->judge, 0, sizeof(double) * J_COUNT);
    if (e != hipSuccess) {
        ctx->err = hip_msg("surrogate buffers", e);
        return MD_E_OOM;
    }
    return MD_OK;
}

md_status load_surrogate(md_ctx *ctx, const float *params, const float *norm, float dz_ood, int judge_stride) {
    if (!(dz_ood >= 0.f) || judge_stride < 0 || (judge_stride > 0 && (judge_stride & (judge_stride - 1)))) {
        ctx->err = "md_load_surrogate: dz_ood must be >= 0 and judge_stride 0 or a power of two";
        return MD_E_INVALID_ARG;
    }
    for (int i = 0; i < MLP_IN; ++i)
        if (!(norm[MLP_IN + i] > 0.f)) {
            ctx->err = "md_load_surrogate: input scales must be > 0";
            return MD_E_INVALID_ARG;
        }
    md_status rc = sur_alloc(ctx);
    if (rc != MD_OK) return rc;
    std::vector<bf16> W(WTOTAL, (bf16)0.f);
    std::vector<float> b(BTOTAL, 0.f);
    const float *W1 = params + kParamOff[0], *W2 = params + kParamOff[2], *W3 = params + kParamOff[4],
                *W4 = params + kParamOff[6];
    for (int o = 0; o < MLP_H; ++o)
        for (int k = 0; k < MLP_IN; ++k) W[WOFF1 + o * MLP_IN + k] = (bf16)W1[o * MLP_IN + k];
    const float *Ws[2] = {W2, W3};
    const int offs[2] = {WOFF2, WOFF3};
    for (int l = 0; l < 2; ++l)
        for (int o = 0; o < MLP_H; ++o)
            for (int kc = 0; kc < 4; ++kc)
                for (int s = 0; s < 32; ++s)
                    W[offs[l] + o * MLP_H + 32 * kc + s] = (bf16)Ws[l][o * MLP_H + 32 * kc + permuted_unit(s)];
    for (int o = 0; o < MLP_OUT; ++o)
        for (int kc = 0; kc < 4; ++kc)
            for (int s = 0; s < 32; ++s)
                W[WOFF4 + o * MLP_H + 32 * kc + s] = (bf16)W4[o * MLP_H + 32 * kc + permuted_unit(s)];
    // fragment-major order: the A fragment of (output tile, K chunk) for all 64
    // lanes stored contiguously, lane l = r + 16 g holding row 16 ot + r,
    // columns 32 kc + 8 g .. + 7, so each wave-wide load reads 1 KB in order
    std::vector<bf16> F(WTOTAL, (bf16)0.f);
    const int loff[4] = {WOFF1, WOFF2, WOFF3, WOFF4}, lk[4] = {MLP_IN, MLP_H, MLP_H, MLP_H},
              lrows[4] = {MLP_H, MLP_H, MLP_H, W4_ROWS};
    for (int l = 0; l < 4; ++l) {
        const int kcs = lk[l] / 32;
        for (int ot = 0; ot < lrows[l] / 16; ++ot)
            for (int kc = 0; kc < kcs; ++kc)
                for (int lane = 0; lane < 64; ++lane)
                    for (int t = 0; t < 8; ++t)
                        F[loff[l] + ((ot * kcs + kc) * 64 + lane) * 8 + t] =
                            W[loff[l] + (16 * ot + lane % 16) * lk[l] + 32 * kc + 8 * (lane / 16) + t];
    }
    W.swap(F);
    for (int i = 0; i < MLP_H; ++i) {
        b[BOFF1 + i] = params[kParamOff[1] + i];
        b[BOFF2 + i] = params[kParamOff[3] + i];
        b[BOFF3 + i] = params[kParamOff[5] + i];
    }
    for (int o = 0; o < MLP_OUT; ++o) b[BOFF4 + o] = params[kParamOff[7] + o];
    SurrogateState *S = ctx->sur;
    // captured rollouts go stale before any buffer changes (also when a copy fails)
    invalidate_graphs(ctx);
    hipError_t e = hipMemcpy(S->W, W.data(), sizeof(bf16) * WTOTAL, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->b, b.data(), sizeof(float) * BTOTAL, hipMemcpyHostToDevice);
    // standardisation as one fused multiply-add per input: x' = x s + (-m s)
    std::vector<float> dn(MLP_NORM);
    for (int i = 0; i < MLP_IN; ++i) {
        dn[i] = norm[MLP_IN + i];
        dn[MLP_IN + i] = (float)(-(double)norm[i] * (double)norm[MLP_IN + i]);
    }
    for (int o = 0; o < 2 * MLP_OUT; ++o) dn[2 * MLP_IN + o] = norm[2 * MLP_IN + o];
    if (e == hipSuccess) e = hipMemcpy(S->norm, dn.data(), sizeof(float) * MLP_NORM, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx->err = hip_msg("md_load_surrogate", e);
        return MD_E_HIP;
    }
    S->dz_ood = dz_ood;
    S->ood_speed = S->ood_rel = S->ood_tilt_s = 0.f;
    S->near_dz = S->near_r2 = S->far_dz = 0.f;
    S->judge_stride = judge_stride;
    S->loaded = true;
    return MD_OK;
}

md_status surrogate_step(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step, float *d_obs,
                         int n_obs_slots, int n_steps, int64_t step0, hipStream_t st) {
    if (!ctx->sur || !ctx->sur->loaded) {
        ctx->err = "md_step: surrogate weights not loaded (md_load_surrogate)";
        return MD_E_INVALID_ARG;
    }
    if (ctx->max_m > MAX_SLOTS) {
        ctx->err = "md_step: the surrogate path supports environments of up to 512 drones";
        return MD_E_UNSUPPORTED;
    }
    int waves = 1;
    while (64 * waves < ctx->max_m) waves *= 2;
    BinSet *bs = nullptr;
    md_status rc = build_bins(ctx, 64 * waves, BIN_PACKED, &bs);
    if (rc != MD_OK) return rc;
    SurArgs sa;
    sa.s.c = ctx->kc;
    sa.s.s = StatePtr{s->p, s->q, s->v, s->w, s->pid_int, s->rpm, s->ctl};
    sa.s.action = d_action;
    sa.s.act_step_stride = action_per_step ? (long long)action_rows(ctx->act) * ctx->n_drones : 0;
    sa.s.obs = (n_obs_slots > 0) ? d_obs : nullptr;
    sa.s.n_obs_slots = n_obs_slots > 0 ? n_obs_slots : 1;
    sa.s.n_steps = n_steps;
    sa.s.step0 = step0;
    sa.s.N = ctx->n_drones;
    sa.s.bins = BinTables{bs->d_slot, bs->d_mmax};
    sa.W = ctx->sur->W;
    sa.b = ctx->sur->b;
    sa.norm = ctx->sur->norm;
    sa.judge = ctx->sur->judge;
    sa.dz_ood = ctx->sur->dz_ood;
    sa.ood_speed = ctx->sur->ood_speed;
    sa.ood_rel = ctx->sur->ood_rel;
    sa.near_dz = ctx->sur->near_dz;
    sa.near_r2 = ctx->sur->near_r2;
    sa.far_dz = ctx->sur->far_dz;
    sa.ood_tilt_s = ctx->sur->ood_tilt_s;
    sa.judge_mask = ctx->sur->judge_stride > 0 ? ctx->sur->judge_stride - 1 : -1;
    sa.knn_reuse = ctx->sur->knn_reuse ? 1 : 0;
    hipError_t e = launch_sur_step(sa, ctx->act, bs->n_bins, bs->slots, st);
    if (e != hipSuccess) {
        ctx->err = hip_msg("surrogate step launch", e);
        return MD_E_HIP;
    }
    return MD_OK;
}

md_status datagen(md_ctx *ctx, const md_state *s, uint32_t mask, float *d_X, float *d_Y, int32_t *d_nbr,
                  hipStream_t st) {
    if (ctx->max_m > MAX_SLOTS) {
        ctx->err = "md_datagen: environments of up to 512 drones";
        return MD_E_UNSUPPORTED;
    }
    int waves = 1;
    while (64 * waves < ctx->max_m) waves *= 2;
    BinSet *bs = nullptr;
    md_status rc = build_bins(ctx, 64 * waves, BIN_PACKED, &bs);
    if (rc != MD_OK) return rc;
    GenArgs g;
    g.c = ctx->kc;
    g.s = StatePtr{s->p, s->q, s->v, s->w, s->pid_int, s->rpm, s->ctl};
    g.N = ctx->n_drones;
    g.bins = BinTables{bs->d_slot, bs->d_mmax};
    g.mask = mask;
    g.X = d_X;
    g.Y = d_Y;
    g.nbr = d_nbr;
    hipError_t e = launch_datagen(g, bs->n_bins, bs->slots, st);
    if (e != hipSuccess) {
        ctx->err = hip_msg("datagen launch", e);
        return MD_E_HIP;
    }
    return MD_OK;
}

md_status judge_stats(md_ctx *ctx, md_judge *out) {
    std::memset(out, 0, sizeof *out);
    if (!ctx->sur || !ctx->sur->judge) return MD_OK;
    double h[J_COUNT];
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, ctx->sur->judge, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        ctx->err = hip_msg("md_judge_stats", e);
        return MD_E_HIP;
    }
    out->n_judged = h[J_N];
    out->force_err2 = h[J_ERR2];
    out->force_ref2 = h[J_REF2];
    out->torque_err2 = h[J_TERR2];
    out->n_fallback = h[J_FALLBACK];
    out->n_drone_steps = h[J_STEPS];
    out->n_nonfinite = h[J_NONFINITE];
    out->force_rel_err = std::sqrt(h[J_ERR2] / h[J_REF2]);  // NaN when nothing was judged
    out->n_knn_full = h[J_FULLKNN];
    return MD_OK;
}

md_status judge_reset(md_ctx *ctx) {
    if (!ctx->sur || !ctx->sur->judge) return MD_OK;
    if (hipMemset(ctx->sur->judge, 0, sizeof(double) * J_COUNT) != hipSuccess) return MD_E_HIP;
    return MD_OK;
}

void free_surrogate(md_ctx *ctx) {
    if (!ctx->sur) return;
    (void)hipFree(ctx->sur->W);
    (void)hipFree(ctx->sur->b);
    (void)hipFree(ctx->sur->norm);
    (void)hipFree(ctx->sur->judge);
    delete ctx->sur;
    ctx->sur = nullptr;
}

}  // namespace md

extern "C" {

md_status md_load_surrogate(md_ctx *ctx, const float *h_params, const float *h_norm, float dz_ood,
                            int judge_stride) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!h_params || !h_norm) {
        ctx->err = "md_load_surrogate: null parameters";
        return MD_E_INVALID_ARG;
    }
    (void)hipSetDevice(ctx->device);
    return md::load_surrogate(ctx, h_params, h_norm, dz_ood, judge_stride);
}

md_status md_set_surrogate_ood(md_ctx *ctx, float max_speed, float max_rel_speed, float max_tilt) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->sur || !ctx->sur->loaded) {
        ctx->err = "md_set_surrogate_ood: no surrogate loaded";
        return MD_E_INVALID_ARG;
    }
    if (!(max_speed >= 0.f) || !(max_rel_speed >= 0.f) || !(max_tilt >= 0.f)) {
        ctx->err = "md_set_surrogate_ood: bounds must be >= 0 (0 turns a check off)";
        return MD_E_INVALID_ARG;
    }
    md::invalidate_graphs(ctx);
    const double sh = std::sin(0.5 * (double)max_tilt);
    ctx->sur->ood_speed = max_speed;
    ctx->sur->ood_rel = max_rel_speed;
    ctx->sur->ood_tilt_s = max_tilt > 0.f ? (float)(sh * sh) : 0.f;
    return MD_OK;
}

md_status md_set_surrogate_region(md_ctx *ctx, float near_dz, float near_r, float far_dz) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->sur || !ctx->sur->loaded) {
        ctx->err = "md_set_surrogate_region: no surrogate loaded";
        return MD_E_INVALID_ARG;
    }
    if (!(near_dz >= 0.f) || !(near_r >= 0.f) || !(far_dz >= 0.f)) {
        ctx->err = "md_set_surrogate_region: bounds must be >= 0 (0 turns a check off)";
        return MD_E_INVALID_ARG;
    }
    md::invalidate_graphs(ctx);
    const bool on = near_dz > 0.f && near_r > 0.f;
    ctx->sur->near_dz = on ? near_dz : 0.f;
    ctx->sur->near_r2 = on ? (float)((double)near_r * (double)near_r) : 0.f;
    ctx->sur->far_dz = far_dz;
    return MD_OK;
}

md_status md_set_surrogate_knn_reuse(md_ctx *ctx, int reuse) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->sur || !ctx->sur->loaded) {
        ctx->err = "md_set_surrogate_knn_reuse: no surrogate loaded";
        return MD_E_INVALID_ARG;
    }
    md::invalidate_graphs(ctx);
    ctx->sur->knn_reuse = reuse != 0;
    return MD_OK;
}

md_status md_load_surrogate_mlp(md_ctx *ctx, const md_mlp *m, float dz_ood, int judge_stride) {
    if (!ctx || !m) return MD_E_INVALID_ARG;
    std::vector<float> p(md::MLP_NPARAMS), nrm(md::MLP_NORM);
    if (md_mlp_get_params(m, p.data()) != MD_OK || md_mlp_get_norm(m, nrm.data()) != MD_OK) {
        ctx->err = "md_load_surrogate_mlp: could not read the network";
        return MD_E_HIP;
    }
    return md_load_surrogate(ctx, p.data(), nrm.data(), dz_ood, judge_stride);
}

md_status md_datagen(md_ctx *ctx, const md_state *s, uint32_t aero_mask, float *d_X, float *d_Y,
                     int32_t *d_nbr, void *stream) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->has_layout) {
        ctx->err = "md_datagen: no layout bound";
        return MD_E_LAYOUT;
    }
    if (ctx->n_drones == 0) return MD_OK;
    if (!s || !s->p || !s->q || !s->v || !s->w || !s->rpm || !d_X || !d_Y || (aero_mask & ~7u)) {
        ctx->err = "md_datagen: null pointer or aero_mask outside GND|DRAG|DW";
        return MD_E_INVALID_ARG;
    }
    return md::datagen(ctx, s, aero_mask, d_X, d_Y, d_nbr, (hipStream_t)stream);
}

md_status md_judge_stats(md_ctx *ctx, md_judge *out) {
    if (!ctx || !out) return MD_E_INVALID_ARG;
    return md::judge_stats(ctx, out);
}

md_status md_judge_reset(md_ctx *ctx) {
    if (!ctx) return MD_E_INVALID_ARG;
    return md::judge_reset(ctx);
}

}  // extern "C"
