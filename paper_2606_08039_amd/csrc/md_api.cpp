// md_api.cpp -- host implementation of the libmd C ABI (include/md.h).
//
// Validates arguments, owns the per-context device tables (environment bins),
// turns md_params into the kernels' float32 constants and launches the step
// kernel on the caller's stream.  No C++ exception crosses the ABI.
#include "md.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "md_ctx.h"

using md::KConst;

static thread_local std::string g_create_err;

namespace md {

std::string hip_msg(const char *what, hipError_t e) {
    return std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}

void derive(const md_params &p, md_derived &d) {
    d.hover_rpm = std::sqrt(p.m * p.g / (4.0 * p.kf));
    d.max_rpm = std::sqrt(p.thrust2weight * p.m * p.g / (4.0 * p.kf));
    d.max_thrust = 4.0 * p.kf * d.max_rpm * d.max_rpm;
    // height at which one rotor at MAX_RPM gains MAX_THRUST / 15 from Eq. 4
    d.h_clip = 0.25 * p.r_p * std::sqrt(15.0 * p.C_gnd * p.kf * d.max_rpm * d.max_rpm / d.max_thrust);
}

KConst make_kconst(const md_params &p, const md_derived &d, double dt, int decim) {
    KConst c;
    std::memset(&c, 0, sizeof c);
    c.dt = (float)dt;
    c.m = (float)p.m;
    c.m_inv = (float)(1.0 / p.m);
    c.g = (float)p.g;
    c.mg = (float)(p.m * p.g);
    c.kf = (float)p.kf;
    c.km = (float)p.km;
    c.l_arm = (float)(p.L / std::sqrt(2.0));
    c.Jx = (float)p.Ixx;
    c.Jy = (float)p.Iyy;
    c.Jz = (float)p.Izz;
    c.Jx_inv = (float)(1.0 / p.Ixx);
    c.Jy_inv = (float)(1.0 / p.Iyy);
    c.Jz_inv = (float)(1.0 / p.Izz);
    c.max_rpm = (float)d.max_rpm;
    c.h_clip = (float)d.h_clip;
    c.K_gnd = (float)(p.C_gnd * p.r_p * p.r_p / 16.0);
    c.drag_s = (float)(2.0 * M_PI / 60.0);
    c.c_xy = (float)p.c_xy;
    c.c_z = (float)p.c_z;
    c.K1 = (float)(p.C1 * p.r_p * p.r_p / 16.0);
    c.C2 = (float)p.C2;
    c.C3 = (float)p.C3;
    c.dz_min = (float)std::max(0.0, p.dw_dz_min);
    c.C2s = (float)(std::sqrt(2.0 * std::log(2.0)) * p.C2);
    c.C3s = (float)(std::sqrt(2.0 * std::log(2.0)) * p.C3);
    for (int k = 0; k < 3; ++k) {
        c.pkp[k] = (float)p.pos_kp[k];
        c.pki[k] = (float)p.pos_ki[k];
        c.pkd[k] = (float)p.pos_kd[k];
        c.akp[k] = (float)p.att_kp[k];
        c.aki[k] = (float)p.att_ki[k];
        c.akd[k] = (float)p.att_kd[k];
    }
    c.p_clamp = (float)p.pos_i_clamp;
    c.a_clamp = (float)p.att_i_clamp;
    for (int k = 0; k < 3; ++k) {
        c.dsl_pkp[k] = (float)p.dsl_pos_kp[k];
        c.dsl_pki[k] = (float)p.dsl_pos_ki[k];
        c.dsl_pkd[k] = (float)p.dsl_pos_kd[k];
        c.dsl_akp[k] = (float)p.dsl_att_kp[k];
        c.dsl_aki[k] = (float)p.dsl_att_ki[k];
        c.dsl_akd[k] = (float)p.dsl_att_kd[k];
    }
    c.dsl_p_clamp = (float)p.dsl_pos_i_clamp;
    c.dsl_a_clamp = (float)p.dsl_att_i_clamp;
    c.dsl_step = (float)(p.dsl_max_speed * dt * decim);
    c.dsl_ystep = (float)(p.dsl_max_yaw_rate * dt * decim);
    c.dt_c = (float)(dt * decim);
    c.g_inv = (float)(1.0 / p.g);
    c.l_inv = (float)(std::sqrt(2.0) / p.L);
    c.kappa_inv = (float)(p.kf / p.km);
    c.fmax = (float)(p.kf * d.max_rpm * d.max_rpm);
    c.kf_inv = (float)(1.0 / p.kf);
    c.hover_inv = (float)(1.0 / d.hover_rpm);
    c.decim = decim;
    return c;
}

// Best-fit-decreasing packing of environments into bins of `slots` drone
// slots; environments larger than a bin are rejected by the caller.  Each
// environment occupies a contiguous run of slots.  Bins are ordered by their
// largest environment, heaviest first, so the longest neighbour sweeps start
// first.
static void pack_bins(const std::vector<int32_t> &off, int slots, std::vector<int2> &tab,
                      std::vector<int> &mmax, int &n_bins) {
    const int E = (int)off.size() - 1;
    std::vector<int> order;
    order.reserve(E);
    for (int e = 0; e < E; ++e)
        if (off[e + 1] > off[e]) order.push_back(e);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (off[a + 1] - off[a]) > (off[b + 1] - off[b]);
    });
    struct Bin {
        int used = 0, mmax = 0;
        std::vector<int> envs;
    };
    std::vector<Bin> bins;
    std::vector<std::vector<int>> by_free(slots + 1);  // bins indexed by free slots
    for (int e : order) {
        const int m = off[e + 1] - off[e];
        int pick = -1;
        for (int f = m; f <= slots && pick < 0; ++f) {
            while (!by_free[f].empty()) {
                const int b = by_free[f].back();
                by_free[f].pop_back();
                if (slots - bins[b].used == f) {
                    pick = b;
                    break;
                }
            }
        }
        if (pick < 0) {
            pick = (int)bins.size();
            bins.emplace_back();
        }
        Bin &B = bins[pick];
        B.envs.push_back(e);
        B.used += m;
        B.mmax = std::max(B.mmax, m);
        by_free[slots - B.used].push_back(pick);
    }
    std::vector<int> border(bins.size());
    for (size_t b = 0; b < bins.size(); ++b) border[b] = (int)b;
    std::stable_sort(border.begin(), border.end(),
                     [&](int a, int b) { return bins[a].mmax > bins[b].mmax; });
    n_bins = (int)bins.size();
    tab.assign((size_t)n_bins * slots, make_int2(-1, 0));
    mmax.assign(n_bins, 0);
    for (int ob = 0; ob < n_bins; ++ob) {
        const Bin &B = bins[border[ob]];
        bool uniform = true;
        for (int e : B.envs) uniform = uniform && (off[e + 1] - off[e] == B.mmax);
        mmax[ob] = B.mmax | (uniform ? 0x10000 : 0);
        int lo = 0;
        for (int e : B.envs) {
            const int m = off[e + 1] - off[e];
            for (int t = 0; t < m; ++t)
                tab[(size_t)ob * slots + lo + t] = make_int2(off[e] + t, (lo << 16) | m);
            lo += m;
        }
    }
}

// Bins for the wave-shuffle sweep: environments packed into 64-slot wave
// bins (best fit decreasing, as above), then consecutive wave bins grouped
// into workgroups of slots / 64 waves, so that no environment crosses a
// wavefront.
static void pack_bins_wave_aligned(const std::vector<int32_t> &off, int slots, std::vector<int2> &tab,
                                   std::vector<int> &mmax, int &n_bins) {
    std::vector<int2> t64;
    std::vector<int> m64;
    int n64 = 0;
    pack_bins(off, 64, t64, m64, n64);
    const int W = slots / 64;
    n_bins = (n64 + W - 1) / W;
    tab.assign((size_t)n_bins * slots, make_int2(-1, 0));
    mmax.assign(n_bins, 0);
    for (int b = 0; b < n_bins; ++b) {
        int mm = 0;
        bool uniform = true;
        int first = -1;
        for (int w = 0; w < W && b * W + w < n64; ++w) {
            const int src = b * W + w;
            for (int s = 0; s < 64; ++s) {
                int2 e = t64[(size_t)src * 64 + s];
                if (e.x >= 0) e.y = (((e.y >> 16) + 64 * w) << 16) | (e.y & 0xffff);
                tab[(size_t)b * slots + 64 * w + s] = e;
            }
            const int mw = m64[src] & 0xffff;
            uniform = uniform && (m64[src] >> 16) != 0 && (first < 0 || mw == first);
            if (first < 0) first = mw;
            mm = std::max(mm, mw);
        }
        // a trailing group may hold fewer waves; their idle slots hold no drone
        mmax[b] = mm | ((uniform && b * W + W <= n64) ? 0x10000 : 0);
    }
}

// Bins for the rotation sweep: every non-empty environment has the same
// power-of-two size M <= 64; E = 64 / M consecutive environments share a
// wave, drone li of the wave's e-th environment in lane E li + e; waves are
// grouped in order into workgroups of slots / 64.  A wave that receives
// fewer than E environments (the last one) keeps idle lanes in the missing
// residues, and each bin reports M with the uniform flag.
static void pack_bins_interleaved(const std::vector<int32_t> &off, int M, int slots, std::vector<int2> &tab,
                                  std::vector<int> &mmax, int &n_bins) {
    const int E = 64 / M, W = slots / 64;
    std::vector<int> envs;
    for (int e = 0; e + 1 < (int)off.size(); ++e)
        if (off[e + 1] > off[e]) envs.push_back(e);
    const int n_waves = ((int)envs.size() + E - 1) / E;
    n_bins = (n_waves + W - 1) / W;
    tab.assign((size_t)n_bins * slots, make_int2(-1, 0));
    mmax.assign(n_bins, M | 0x10000);
    for (size_t k = 0; k < envs.size(); ++k) {
        const int wave = (int)k / E, e = (int)k % E;
        const int b = wave / W, w = wave % W;
        for (int li = 0; li < M; ++li) {
            const int lane = E * li + e;
            tab[(size_t)b * slots + 64 * w + lane] = make_int2(off[envs[k]] + li, ((64 * w + e) << 16) | M);
        }
    }
}

md_status build_bins(md_ctx *ctx, int slots, int mode, BinSet **out) {
    const int key = slots * 4 + mode;
    auto it = ctx->binsets.find(key);
    if (it != ctx->binsets.end()) {
        *out = &it->second;
        return MD_OK;
    }
    if (ctx->max_m > slots) {
        ctx->err = "environment of " + std::to_string(ctx->max_m) + " drones exceeds a bin of " +
                   std::to_string(slots) + " slots";
        return MD_E_UNSUPPORTED;
    }
    std::vector<int2> tab;
    std::vector<int> mm;
    BinSet bs;
    if (mode == BIN_INTERLEAVED) {
        const int M = ctx->uniform_m;
        if (M < 2 || M > 64 || (M & (M - 1)) || slots % 64) {
            ctx->err = "interleaved bins need environments of one power-of-two size 2..64";
            return MD_E_UNSUPPORTED;
        }
        pack_bins_interleaved(ctx->off, M, slots, tab, mm, bs.n_bins);
    } else if (mode == BIN_WAVE_ALIGNED) {
        pack_bins_wave_aligned(ctx->off, slots, tab, mm, bs.n_bins);
    } else {
        pack_bins(ctx->off, slots, tab, mm, bs.n_bins);
    }
    bs.slots = slots;
    if (bs.n_bins > 0) {
        hipError_t e = hipMalloc(&bs.d_slot, sizeof(int2) * tab.size());
        if (e == hipSuccess) e = hipMalloc(&bs.d_mmax, sizeof(int) * mm.size());
        if (e != hipSuccess) {
            (void)hipFree(bs.d_slot);
            ctx->err = hip_msg("hipMalloc(bin tables)", e);
            return MD_E_OOM;
        }
        e = hipMemcpy(bs.d_slot, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(bs.d_mmax, mm.data(), sizeof(int) * mm.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(bs.d_slot);
            (void)hipFree(bs.d_mmax);
            ctx->err = hip_msg("hipMemcpy(bin tables)", e);
            return MD_E_HIP;
        }
        bs.h_mmax = mm;
    }
    auto ins = ctx->binsets.emplace(key, std::move(bs));
    *out = &ins.first->second;
    return MD_OK;
}

void free_bins(md_ctx *ctx) {
    for (auto &kv : ctx->binsets) {
        (void)hipFree(kv.second.d_slot);
        (void)hipFree(kv.second.d_mmax);
    }
    ctx->binsets.clear();
}

int slots_for(const md_ctx *ctx, const LaunchCfg &cfg) {
    const int lpd = (ctx->mask & MD_AERO_DW) ? cfg.lpd : 1;
    return 64 * cfg.waves / lpd;
}

int bin_mode_for(const md_ctx *ctx, const LaunchCfg &cfg) {
    if (!(ctx->mask & MD_AERO_DW)) return BIN_PACKED;
    return cfg.sym == 3 ? BIN_INTERLEAVED : cfg.sym == 2 ? BIN_WAVE_ALIGNED : BIN_PACKED;
}

LaunchCfg default_cfg(const md_ctx *ctx) {
    LaunchCfg c{1, 4, 1, 0};
    const int max_waves = ctx->dr_on ? MAX_THREADS_DR / 64 : 16;
    while (64 * c.waves < ctx->max_m && c.waves < max_waves) c.waves *= 2;
    return c;
}

md_status prepare_launch(md_ctx *ctx) {
    if (!ctx->has_layout) {
        ctx->err = "no layout bound";
        return MD_E_LAYOUT;
    }
    BinSet *bs = nullptr;
    if (ctx->mask & MD_AERO_SURROGATE) {
        int waves = 1;
        while (64 * waves < ctx->max_m) waves *= 2;
        return build_bins(ctx, 64 * waves, BIN_PACKED, &bs);
    }
    return build_bins(ctx, slots_for(ctx, ctx->cfg), bin_mode_for(ctx, ctx->cfg), &bs);
}

md_status launch(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                 float *d_obs, int n_obs_slots, int n_steps, int64_t step0, hipStream_t st,
                 const LaunchCfg &cfg) {
    BinSet *bs = nullptr;
    md_status rc = build_bins(ctx, slots_for(ctx, cfg), bin_mode_for(ctx, cfg), &bs);
    if (rc != MD_OK) return rc;
    StepArgs a;
    a.c = ctx->kc;
    a.s = StatePtr{s->p, s->q, s->v, s->w, s->pid_int, s->rpm, s->ctl, s->rpm_cmd, s->act_hist, s->act_count,
                   s->wind, s->obs_hist, s->obs_count};
    a.dr = ctx->dr;
    a.wind = ctx->wind;
    a.action = d_action;
    a.act_step_stride = action_per_step ? (long long)action_rows(ctx->act) * ctx->n_drones : 0;
    a.obs = (n_obs_slots > 0) ? d_obs : nullptr;
    a.n_obs_slots = n_obs_slots > 0 ? n_obs_slots : 1;
    a.n_steps = n_steps;
    a.step0 = step0;
    a.N = ctx->n_drones;
    a.bins = BinTables{bs->d_slot, bs->d_mmax};
    a.tstride = pair_stride(ctx->max_m);
    hipError_t e = (ctx->integ == MD_INTEG_RK4) ? launch_step_rk4(a, ctx->mask, ctx->act, cfg, bs->n_bins, bs->slots, st)
                   : ctx->dr_on ? launch_step_dr(a, ctx->mask, ctx->act, cfg, bs->n_bins, bs->slots, st)
                   : ctx->wind.models ? launch_step_wind(a, ctx->mask, ctx->act, cfg, bs->n_bins, bs->slots, st)
                                      : launch_step(a, ctx->mask, ctx->act, cfg, bs->n_bins, bs->slots, st);
    if (e != hipSuccess) {
        ctx->err = hip_msg("step kernel launch", e);
        return MD_E_HIP;
    }
    return MD_OK;
}

}  // namespace md

extern "C" {

const char *md_version(void) { return "libmd 0.1 (gfx950)"; }

md_status md_default_params_cf2x(md_params *out) {
    if (!out) return MD_E_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    // Table "Drone model parameters", CF2X
    out->m = 0.027;
    out->L = 0.0397;
    out->thrust2weight = 2.25;
    out->Ixx = 1.4e-5;
    out->Iyy = 1.4e-5;
    out->Izz = 2.17e-5;
    out->kf = 3.16e-10;
    out->km = 7.94e-12;
    out->r_p = 0.02325;
    out->g = 9.81;
    // ground effect and drag coefficients (not printed; the predecessor's CF2X values)
    out->C_gnd = 11.36359;
    out->c_xy = 9.1785e-7;
    out->c_z = 10.311e-7;
    // Eq. 6
    out->C1 = 2267.18;
    out->C2 = 0.16;
    out->C3 = -0.11;
    out->dw_dz_min = 0.0;
    // Table "Default PIDControl gains"
    const double pkp[3] = {0.4, 0.4, 1.0}, pki[3] = {0.01, 0.01, 0.01}, pkd[3] = {0.9, 0.9, 2.0};
    const double akp[3] = {2e-3, 2e-3, 1e-3}, aki[3] = {0.0, 0.0, 1e-4}, akd[3] = {5e-4, 5e-4, 2e-4};
    for (int k = 0; k < 3; ++k) {
        out->pos_kp[k] = pkp[k];
        out->pos_ki[k] = pki[k];
        out->pos_kd[k] = pkd[k];
        out->att_kp[k] = akp[k];
        out->att_ki[k] = aki[k];
        out->att_kd[k] = akd[k];
    }
    out->pos_i_clamp = 2.0;
    out->att_i_clamp = 0.5;
    // DSL-style PID: the PIDControl gains (its retuned values are not printed),
    // halved integral clamps, setpoint limits 2 m/s and pi rad/s
    for (int k = 0; k < 3; ++k) {
        out->dsl_pos_kp[k] = pkp[k];
        out->dsl_pos_ki[k] = pki[k];
        out->dsl_pos_kd[k] = pkd[k];
        out->dsl_att_kp[k] = akp[k];
        out->dsl_att_ki[k] = aki[k];
        out->dsl_att_kd[k] = akd[k];
    }
    out->dsl_pos_i_clamp = 1.0;
    out->dsl_att_i_clamp = 0.25;
    out->dsl_max_speed = 2.0;
    out->dsl_max_yaw_rate = M_PI;
    return MD_OK;
}

md_status md_derive(const md_params *p, md_derived *out) {
    if (!p || !out) return MD_E_INVALID_ARG;
    md::derive(*p, *out);
    return MD_OK;
}

md_status md_create(const md_params *p, float dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                    md_ctx **out) {
    if (out) *out = nullptr;
    if (!p || !out) {
        g_create_err = "md_create: null params or output pointer";
        return MD_E_INVALID_ARG;
    }
    if (!(dt > 0.f) || ctrl_decim < 1 || act_type < MD_ACT_RPM || act_type > MD_ACT_DSL ||
        (aero_mask & ~15u) != 0) {
        g_create_err = "md_create: invalid dt, ctrl_decim, act_type or aero_mask";
        return MD_E_INVALID_ARG;
    }
    if ((aero_mask & MD_AERO_SURROGATE) && (aero_mask & 7u)) {
        g_create_err = "md_create: MD_AERO_SURROGATE replaces GND|DRAG|DW and cannot be combined with them";
        return MD_E_INVALID_ARG;
    }
    if (!(p->m > 0 && p->kf > 0 && p->km > 0 && p->Ixx > 0 && p->Iyy > 0 && p->Izz > 0 &&
          p->L > 0 && p->g > 0 && p->thrust2weight > 0 && p->r_p > 0)) {
        g_create_err = "md_create: non-positive mass, inertia, arm, rotor or gravity constant";
        return MD_E_INVALID_ARG;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        g_create_err = md::hip_msg("md_create: no usable HIP device", e);
        return MD_E_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_err = std::string("md_create: libmd is built for gfx950 only; device is ") + prop.gcnArchName;
        return MD_E_UNSUPPORTED;
    }
    md_ctx *ctx = new (std::nothrow) md_ctx();
    if (!ctx) {
        g_create_err = "md_create: out of host memory";
        return MD_E_OOM;
    }
    ctx->P = *p;
    md::derive(*p, ctx->D);
    ctx->dt = dt;
    ctx->mask = aero_mask;
    ctx->act = act_type;
    ctx->decim = ctrl_decim;
    ctx->device = dev;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->kc = md::make_kconst(*p, ctx->D, dt, ctrl_decim);
    *out = ctx;
    return MD_OK;
}

void md_destroy(md_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    // captured rollouts outlive their context only as handles md_graph_launch refuses
    for (md_graph *g : ctx->graphs) g->ctx = nullptr;
    ctx->graphs.clear();
    md::free_surrogate(ctx);
    md::free_bins(ctx);
    delete ctx;
}

const char *md_last_error(const md_ctx *ctx) {
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

md_status md_bind_layout(md_ctx *ctx, const int32_t *h_env_offsets, int n_envs, int n_drones) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!h_env_offsets || n_envs < 0 || n_drones < 0) {
        ctx->err = "md_bind_layout: null offsets or negative sizes";
        return MD_E_INVALID_ARG;
    }
    if (h_env_offsets[0] != 0 || h_env_offsets[n_envs] != n_drones) {
        ctx->err = "md_bind_layout: offsets must start at 0 and end at n_drones";
        return MD_E_LAYOUT;
    }
    int maxm = 0;
    for (int e = 0; e < n_envs; ++e) {
        const int m = h_env_offsets[e + 1] - h_env_offsets[e];
        if (m < 0) {
            ctx->err = "md_bind_layout: offsets must be non-decreasing";
            return MD_E_LAYOUT;
        }
        maxm = std::max(maxm, m);
    }
    if (maxm > 1024) {
        ctx->err = "md_bind_layout: environments of more than 1024 drones are not supported";
        return MD_E_UNSUPPORTED;
    }
    if (n_drones > (1 << 25)) {
        ctx->err = "md_bind_layout: more than 2^25 drones per context are not supported";
        return MD_E_UNSUPPORTED;
    }
    (void)hipSetDevice(ctx->device);
    md::invalidate_graphs(ctx);  // they point at the bin tables freed here
    md::free_bins(ctx);
    ctx->off.assign(h_env_offsets, h_env_offsets + n_envs + 1);
    ctx->n_envs = n_envs;
    ctx->n_drones = n_drones;
    ctx->max_m = maxm;
    ctx->uniform_m = maxm;
    for (int e = 0; e < n_envs; ++e) {
        const int m = h_env_offsets[e + 1] - h_env_offsets[e];
        if (m != 0 && m != maxm) ctx->uniform_m = 0;
    }
    ctx->has_layout = true;
    ctx->cfg = md::default_cfg(ctx);
    md::BinSet *bs = nullptr;
    return md::build_bins(ctx, md::slots_for(ctx, ctx->cfg), md::bin_mode_for(ctx, ctx->cfg), &bs);
}

md_status md_set_integrator(md_ctx *ctx, int integrator) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (integrator != MD_INTEG_EULER && integrator != MD_INTEG_RK4) {
        ctx->err = "md_set_integrator: unknown integrator";
        return MD_E_INVALID_ARG;
    }
    if (integrator == MD_INTEG_RK4 && ((ctx->mask & MD_AERO_SURROGATE) || ctx->dr_on || ctx->wind.models)) {
        ctx->err = "md_set_integrator: the learned residual and domain randomisation run with the "
                   "semi-implicit Euler step only";
        return MD_E_UNSUPPORTED;
    }
    if (integrator != ctx->integ) md::invalidate_graphs(ctx);
    ctx->integ = integrator;
    if (ctx->has_layout && !md::cfg_valid(ctx, ctx->cfg)) {
        // the Runge-Kutta kernel sweeps neighbours with one lane per drone
        ctx->cfg = md::default_cfg(ctx);
        ctx->tuned = false;
    }
    return MD_OK;
}

md_status md_set_domain_randomization(md_ctx *ctx, const md_dr *dr) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!dr) {
        if (ctx->dr_on) md::invalidate_graphs(ctx);
        ctx->dr_on = false;
        ctx->dr = md::DrPtr{};
        return MD_OK;
    }
    if (!dr->scale) {
        ctx->err = "md_set_domain_randomization: null scale array";
        return MD_E_INVALID_ARG;
    }
    const float sig[4] = {dr->noise_p, dr->noise_v, dr->noise_rpy, dr->noise_w};
    for (float x : sig)
        if (!(x >= 0.f) || !std::isfinite(x)) {
            ctx->err = "md_set_domain_randomization: negative or non-finite sensor noise level";
            return MD_E_INVALID_ARG;
        }
    if ((ctx->mask & MD_AERO_SURROGATE) || ctx->integ == MD_INTEG_RK4) {
        ctx->err = "md_set_domain_randomization: supported with the plain semi-implicit Euler step only";
        return MD_E_UNSUPPORTED;
    }
    md::DrPtr d{};
    d.scale = dr->scale;
    d.tau_mot = dr->tau_mot;
    d.delay = dr->delay;
    for (int k = 0; k < 4; ++k) d.sig[k] = sig[k];
    d.noisy = sig[0] > 0.f || sig[1] > 0.f || sig[2] > 0.f || sig[3] > 0.f;
    d.key0 = (uint32_t)(dr->seed & 0xffffffffull);
    d.key1 = (uint32_t)(dr->seed >> 32);
    d.obs_delay = dr->obs_delay;
    d.obs_bias = dr->obs_bias;
    if (ctx->has_layout && ctx->max_m > md::MAX_THREADS_DR) {
        ctx->err = "md_set_domain_randomization: supported for environments of up to 512 drones";
        return MD_E_UNSUPPORTED;
    }
    ctx->dr = d;
    ctx->dr_on = true;
    md::invalidate_graphs(ctx);
    if (ctx->has_layout && !md::cfg_valid(ctx, ctx->cfg)) {
        // workgroups of the randomised step hold at most MAX_THREADS_DR threads
        ctx->cfg = md::default_cfg(ctx);
        ctx->tuned = false;
    }
    return MD_OK;
}

md_status md_set_wind(md_ctx *ctx, const md_wind *w) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!w || w->models == 0) {
        if (ctx->wind.models) md::invalidate_graphs(ctx);
        ctx->wind = md::WindArgs{};
        return MD_OK;
    }
    if ((w->models & ~MD_WIND_COMBINED) || !(w->rho >= 0.f) || !(w->cd_area >= 0.f) || !(w->gust_prob >= 0.f) ||
        !(w->gust_prob <= 1.f) || !(w->gust_amp >= 0.f) || !(w->dryden_sigma >= 0.f) ||
        !(w->dryden_airspeed >= 0.f) || ((w->models & MD_WIND_GUST) && !(w->gust_duration > 0.f))) {
        ctx->err = "md_set_wind: unknown model bits or a negative / non-finite parameter";
        return MD_E_INVALID_ARG;
    }
    if ((ctx->mask & MD_AERO_SURROGATE) || ctx->integ == MD_INTEG_RK4) {
        ctx->err = "md_set_wind: supported with the plain semi-implicit Euler step only";
        return MD_E_UNSUPPORTED;
    }
    md::WindArgs a{};
    a.models = w->models;
    for (int k = 0; k < 3; ++k) a.vm[k] = w->v_mean[k];
    a.kd = (float)(0.5 * (double)w->rho * (double)w->cd_area);
    a.gust_prob = w->gust_prob;
    a.gust_amp = w->gust_amp;
    a.gust_steps = std::max(1L, std::lround((double)w->gust_duration / (double)ctx->dt));
    a.sigma = w->dryden_sigma;
    a.airspeed = w->dryden_airspeed;
    a.sin_amp = w->sin_amp;
    a.sin_wdt = (double)w->sin_omega * (double)ctx->dt;
    a.key0 = (uint32_t)(w->seed & 0xffffffffull);
    a.key1 = (uint32_t)(w->seed >> 32);
    a.vm_drone = w->v_mean_drone;
    ctx->wind = a;
    md::invalidate_graphs(ctx);
    return MD_OK;
}

md_status md_get_integrator(const md_ctx *ctx, int *out) {
    if (!ctx || !out) return MD_E_INVALID_ARG;
    *out = ctx->integ;
    return MD_OK;
}

md_status md_step(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                  float *d_obs, int n_obs_slots, int n_steps, int64_t step0, void *stream) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->has_layout) {
        ctx->err = "md_step: no layout bound (call md_bind_layout first)";
        return MD_E_LAYOUT;
    }
    if (!s || n_steps < 0 || step0 < 0 || n_obs_slots < 0) {
        ctx->err = "md_step: null state, or negative n_steps, step0 or n_obs_slots";
        return MD_E_INVALID_ARG;
    }
    if (n_steps == 0 || ctx->n_drones == 0) return MD_OK;
    if (!s->p || !s->q || !s->v || !s->w || !s->rpm || (ctx->act != MD_ACT_RPM && !s->pid_int) ||
        (ctx->act == MD_ACT_DSL && !s->ctl) || !d_action || (n_obs_slots > 0 && !d_obs)) {
        ctx->err = "md_step: null state block, action or observation pointer";
        return MD_E_INVALID_ARG;
    }
    if (ctx->dr_on && ((ctx->act != MD_ACT_RPM && !s->rpm_cmd) ||
                       (ctx->dr.delay && (!s->act_hist || !s->act_count)) ||
                       (ctx->dr.obs_delay && (!s->obs_hist || !s->obs_count)))) {
        ctx->err = "md_step: domain randomisation needs rpm_cmd (controller actions), with action delays "
                   "act_hist and act_count, with sensor delays obs_hist and obs_count";
        return MD_E_INVALID_ARG;
    }
    if ((ctx->wind.models & (MD_WIND_GUST | MD_WIND_DRYDEN)) && !s->wind) {
        ctx->err = "md_step: wind gusts and turbulence need the wind state block";
        return MD_E_INVALID_ARG;
    }
    if (ctx->dr_on && ctx->max_m > md::MAX_THREADS_DR) {
        ctx->err = "md_step: domain randomisation is supported for environments of up to 512 drones";
        return MD_E_UNSUPPORTED;
    }
    if (ctx->mask & MD_AERO_SURROGATE) return md::surrogate_step(ctx, s, d_action, action_per_step, d_obs,
                                                                 n_obs_slots, n_steps, step0,
                                                                 (hipStream_t)stream);
    return md::launch(ctx, s, d_action, action_per_step, d_obs, n_obs_slots, n_steps, step0,
                      (hipStream_t)stream, ctx->cfg);
}

}  // extern "C"
