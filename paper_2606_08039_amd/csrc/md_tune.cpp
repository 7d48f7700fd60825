// md_tune.cpp -- launch-configuration autotuner and captured rollouts.
//
// Autotuner: for the bound layout and the context's mask, time every valid
// launch configuration (lanes per drone for the neighbour sweep, bin size in
// waves, neighbour-loop unroll, all-pairs or pair-symmetric sweep) on scratch
// copies of the caller's state (round robin, the median of three timed
// repetitions after a warm-up round; the three best again as runs of
// consecutive launches), keep the fastest, and remember it in a small
// JSON cache keyed by the layout signature.  Every configuration computes the
// same physics; the pair-symmetric and the one-lane all-pairs sweeps are
// bitwise identical, the multi-lane sweeps differ only in summation order.
//
// Graphs: n_launches consecutive md_step launches of steps_per_launch steps
// each, captured once on a stream and replayed with hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "md_ctx.h"

namespace md {

static std::string signature(const md_ctx *ctx) {
    // layout shape: drones, environments, largest environment and a hash of
    // the environment-size sequence; plus mask and action type
    uint64_t h = 1469598103934665603ull;
    for (size_t e = 0; e + 1 < ctx->off.size(); ++e) {
        h ^= (uint64_t)(ctx->off[e + 1] - ctx->off[e]);
        h *= 1099511628211ull;
    }
    char buf[176];
    std::snprintf(buf, sizeof buf, "n%d_e%d_m%d_h%016llx_mask%u_act%d_int%d", ctx->n_drones, ctx->n_envs,
                  ctx->max_m, (unsigned long long)h, ctx->mask, ctx->act, ctx->integ);
    return buf;
}

bool cfg_valid(const md_ctx *ctx, const LaunchCfg &c) {
    const int slots = 64 * c.waves / c.lpd;
    if (slots < ctx->max_m || slots < 1) return false;
    if (c.sym < 0 || c.sym > 3) return false;
    if (c.sym && c.lpd != 1) return false;
    if (c.sym == 2 && ctx->max_m > 64) return false;  // environments inside one wave
    // the permute loop's trip count is the bin's largest environment, and a
    // loop of cross-lane permutes cannot be unrolled with a remainder (each
    // permute must run with the whole wave): its unroll variants would be
    // the same code, so only unroll 1 exists
    if (c.sym == 2 && c.unroll != 1) return false;
    if (c.sym == 3) {
        // one power-of-two environment size 2..64
        const int m = ctx->uniform_m;
        if (m < 2 || m > 64 || (m & (m - 1))) return false;
        if (c.unroll != 1) return false;  // fully unrolled
    }
    if (ctx->integ == MD_INTEG_RK4 && (ctx->mask & MD_AERO_DW) && c.lpd != 1) return false;
    if (c.sym == 1) {
        const size_t lds = 16 * 4 * (size_t)slots + 4 * (size_t)slots * (size_t)pair_stride(ctx->max_m);
        if (lds > 64 * 1024) return false;
    }
    if (64 * c.waves > 1024) return false;
    if (ctx->dr_on && 64 * c.waves > MAX_THREADS_DR) return false;
    return true;
}

static std::vector<LaunchCfg> candidates(const md_ctx *ctx) {
    std::vector<LaunchCfg> out;
    if (!(ctx->mask & MD_AERO_DW)) {
        for (int w : {1, 2, 4})
            if (64 * w >= ctx->max_m) out.push_back(LaunchCfg{1, 1, w, 0});
        if (out.empty()) out.push_back(default_cfg(ctx));
        return out;
    }
    for (int sym : {0, 1, 2, 3})
        for (int lpd : {1, 2, 4})
            for (int w : {1, 2, 4, 8, 16})
                for (int u : {1, 2, 4}) {
                    LaunchCfg c{lpd, u, w, sym};
                    if (cfg_valid(ctx, c)) out.push_back(c);
                }
    return out;
}

static std::string cache_path(const char *path) {
    if (path && *path) return path;
    const char *env = std::getenv("MD_AUTOTUNE_CACHE");
    if (env && *env) return env;
    return "";
}

// Cache format: one JSON object per line inside a JSON array:
// [{"sig": "...", "lpd": 1, "unroll": 4, "waves": 1, "sym": 1, "us": 123.4}, ...]
static bool cache_lookup(const std::string &path, const std::string &sig, LaunchCfg &out) {
    if (path.empty()) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    while (std::getline(f, line)) {
        const std::string key = "\"sig\": \"" + sig + "\"";
        if (line.find(key) == std::string::npos) continue;
        int lpd = 0, unroll = 0, waves = 0, sym = 0;
        auto grab = [&](const char *name, int &v) {
            const std::string k = std::string("\"") + name + "\": ";
            const size_t p = line.find(k);
            if (p == std::string::npos) return false;
            v = std::atoi(line.c_str() + p + k.size());
            return true;
        };
        if (grab("lpd", lpd) && grab("unroll", unroll) && grab("waves", waves) && grab("sym", sym)) {
            out = LaunchCfg{lpd, unroll, waves, sym};
            return true;
        }
    }
    return false;
}

static void cache_store(const std::string &path, const std::string &sig, const LaunchCfg &c, double us) {
    if (path.empty()) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            if (line.find("\"sig\"") == std::string::npos) continue;
            if (line.find("\"sig\": \"" + sig + "\"") != std::string::npos) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            keep.push_back(line);
        }
    }
    char buf[400];
    std::snprintf(buf, sizeof buf, "{\"sig\": \"%s\", \"lpd\": %d, \"unroll\": %d, \"waves\": %d, \"sym\": %d, \"us\": %.3f}",
                  sig.c_str(), c.lpd, c.unroll, c.waves, c.sym, us);
    keep.push_back(buf);
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        f << "[\n";
        for (size_t i = 0; i < keep.size(); ++i) f << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        f << "]\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

// A new launch configuration makes the captured rollouts stale.
static void set_cfg(md_ctx *ctx, const LaunchCfg &c) {
    const LaunchCfg &o = ctx->cfg;
    if (o.lpd != c.lpd || o.unroll != c.unroll || o.waves != c.waves || o.sym != c.sym) invalidate_graphs(ctx);
    ctx->cfg = c;
    ctx->tuned = true;
}

md_status autotune(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step, float *d_obs,
                   int n_obs_slots, int n_steps, int64_t step0, hipStream_t st, const char *path, int force) {
    // a choice timed with the observation stream is kept apart from one timed without
    const std::string sig = signature(ctx) + (d_obs ? "_obs" : "");
    const std::string cp = cache_path(path);
    LaunchCfg cached;
    if (!force && cache_lookup(cp, sig, cached) && cfg_valid(ctx, cached)) {
        set_cfg(ctx, cached);
        return MD_OK;
    }
    const size_t N = (size_t)ctx->n_drones;
    if (N == 0 || n_steps <= 0) {
        ctx->tuned = true;
        return MD_OK;
    }
    // scratch copies of the state: the caller's state is never advanced
    const bool dr = ctx->dr_on, ring = dr && ctx->dr.delay != nullptr;
    const bool oring = dr && ctx->dr.obs_delay != nullptr;
    const size_t nr[13] = {3, 4, 3, 3, 6, 4, 4, dr ? 4u : 0u,
                           ring ? (size_t)MD_DR_HIST * action_rows(ctx->act) : 0u, ring ? 1u : 0u,
                           (ctx->wind.models && s->wind) ? 5u : 0u,
                           oring ? (size_t)MD_DR_OBS_HIST * 20u : 0u, oring ? 1u : 0u};
    size_t rows = 0;
    for (size_t r : nr) rows += r;
    float *scratch = nullptr, *work = nullptr;
    hipError_t e = hipMalloc(&scratch, sizeof(float) * rows * N);
    if (e == hipSuccess) e = hipMalloc(&work, sizeof(float) * rows * N);
    if (e != hipSuccess) {
        (void)hipFree(scratch);
        ctx->err = hip_msg("autotune scratch", e);
        return MD_E_OOM;
    }
    // act_count and obs_count are int32: copied bit for bit through float-sized slots
    const float *src[13] = {s->p, s->q, s->v, s->w, s->pid_int, s->rpm, s->ctl, s->rpm_cmd, s->act_hist,
                            (const float *)s->act_count, s->wind, s->obs_hist, (const float *)s->obs_count};
    size_t o = 0;
    md_state ws{};
    float *blk[13] = {};
    for (int k = 0; k < 13 && e == hipSuccess; ++k) {
        if (nr[k] == 0) continue;
        if (src[k])
            e = hipMemcpyAsync(scratch + o, src[k], sizeof(float) * nr[k] * N, hipMemcpyDeviceToDevice, st);
        else
            e = hipMemsetAsync(scratch + o, 0, sizeof(float) * nr[k] * N, st);
        blk[k] = work + o;
        o += nr[k] * N;
    }
    ws.p = blk[0];
    ws.q = blk[1];
    ws.v = blk[2];
    ws.w = blk[3];
    ws.pid_int = blk[4];
    ws.rpm = blk[5];
    ws.ctl = blk[6];
    ws.rpm_cmd = blk[7];
    ws.act_hist = blk[8];
    ws.act_count = (int32_t *)blk[9];
    ws.wind = blk[10];
    ws.obs_hist = blk[11];
    ws.obs_count = (int32_t *)blk[12];
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best_us = 1e300;
    LaunchCfg best = ctx->cfg;
    const char *venv = std::getenv("MD_AUTOTUNE_VERBOSE");
    const bool verbose = venv && *venv && *venv != '0';
    md_status rc = MD_OK;
    // Stage 1, round robin: every repetition times each candidate once, so
    // all of them see the same drift of the clock under load; the first
    // round warms up, the score is the median of the other three.
    const std::vector<LaunchCfg> cands = candidates(ctx);
    constexpr int REPS = 4;
    std::vector<float> ms_of(cands.size() * (REPS - 1), 0.f);
    auto timed = [&](const LaunchCfg &c, float &ms) {
        e = hipEventRecord(a, st);
        if (e != hipSuccess) return;
        rc = launch(ctx, &ws, d_action, action_per_step, d_obs, d_obs ? n_obs_slots : 0, n_steps, step0, st, c);
        if (rc != MD_OK) return;
        e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    };
    for (int rep = 0; rep < REPS && e == hipSuccess && rc == MD_OK; ++rep) {
        for (size_t i = 0; i < cands.size() && e == hipSuccess && rc == MD_OK; ++i) {
            e = hipMemcpyAsync(work, scratch, sizeof(float) * rows * N, hipMemcpyDeviceToDevice, st);
            float ms = 0.f;
            if (e == hipSuccess) timed(cands[i], ms);
            if (rep > 0) ms_of[i * (REPS - 1) + (rep - 1)] = ms;
        }
    }
    std::vector<double> score(cands.size(), 1e300);
    for (size_t i = 0; i < cands.size() && e == hipSuccess && rc == MD_OK; ++i) {
        float *t = &ms_of[i * (REPS - 1)];
        std::sort(t, t + (REPS - 1));
        score[i] = t[(REPS - 1) / 2] * 1000.0;
        const LaunchCfg &c = cands[i];
        if (verbose)
            std::fprintf(stderr, "md_autotune %s: lpd %d unroll %d waves %d sym %d: %.1f us\n", sig.c_str(), c.lpd,
                         c.unroll, c.waves, c.sym, score[i]);
    }
    // Stage 2: the three best, each as a run of consecutive launches (the
    // load a rollout puts on the chip, under which the clock settles lower
    // than after the pauses of stage 1), two rounds round robin; the score
    // is the median launch time after each run's first launch.
    std::vector<size_t> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return score[x] < score[y]; });
    const size_t top = std::min<size_t>(3, order.size());
    constexpr int RUN = 6, ROUNDS = 2;
    std::vector<float> run_ms(top * ROUNDS * (RUN - 1), 0.f);
    for (int r = 0; r < ROUNDS && top > 1 && e == hipSuccess && rc == MD_OK; ++r) {
        for (size_t k = 0; k < top && e == hipSuccess && rc == MD_OK; ++k) {
            e = hipMemcpyAsync(work, scratch, sizeof(float) * rows * N, hipMemcpyDeviceToDevice, st);
            for (int l = 0; l < RUN && e == hipSuccess && rc == MD_OK; ++l) {
                float ms = 0.f;
                timed(cands[order[k]], ms);
                if (l > 0) run_ms[(k * ROUNDS + r) * (RUN - 1) + (l - 1)] = ms;
            }
        }
    }
    for (size_t k = 0; k < top && e == hipSuccess && rc == MD_OK; ++k) {
        const size_t i = order[k];
        double us = score[i];
        if (top > 1) {
            float *t = &run_ms[k * ROUNDS * (RUN - 1)];
            std::sort(t, t + ROUNDS * (RUN - 1));
            us = t[ROUNDS * (RUN - 1) / 2] * 1000.0;
        }
        const LaunchCfg &c = cands[i];
        if (verbose)
            std::fprintf(stderr, "md_autotune %s: sustained: lpd %d unroll %d waves %d sym %d: %.1f us\n",
                         sig.c_str(), c.lpd, c.unroll, c.waves, c.sym, us);
        if (us < best_us) {
            best_us = us;
            best = c;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(scratch);
    (void)hipFree(work);
    if (rc != MD_OK) return rc;
    if (e != hipSuccess) {
        ctx->err = hip_msg("autotune", e);
        return MD_E_HIP;
    }
    set_cfg(ctx, best);
    cache_store(cp, sig, best, best_us);
    return MD_OK;
}

}  // namespace md

extern "C" {

md_status md_autotune(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step, int n_steps,
                      int64_t step0, void *stream, const char *cache_path, int force) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->has_layout) {
        ctx->err = "md_autotune: no layout bound";
        return MD_E_LAYOUT;
    }
    if (!s || !d_action || n_steps < 0 || step0 < 0) {
        ctx->err = "md_autotune: null state or action, or negative n_steps / step0";
        return MD_E_INVALID_ARG;
    }
    if (ctx->mask & MD_AERO_SURROGATE) {
        ctx->tuned = true;  // the surrogate kernel has one configuration
        return MD_OK;
    }
    return md::autotune(ctx, s, d_action, action_per_step, nullptr, 0, n_steps, step0, (hipStream_t)stream,
                        cache_path, force);
}

md_status md_autotune_obs(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step, float *d_obs,
                          int n_obs_slots, int n_steps, int64_t step0, void *stream, const char *cache_path,
                          int force) {
    if (!ctx) return MD_E_INVALID_ARG;
    if (!ctx->has_layout) {
        ctx->err = "md_autotune_obs: no layout bound";
        return MD_E_LAYOUT;
    }
    if (!s || !d_action || !d_obs || n_obs_slots < 1 || n_steps < 0 || step0 < 0) {
        ctx->err = "md_autotune_obs: null state, action or observation buffer, n_obs_slots < 1, or negative "
                   "n_steps / step0";
        return MD_E_INVALID_ARG;
    }
    if (ctx->mask & MD_AERO_SURROGATE) {
        ctx->tuned = true;  // the surrogate kernel has one configuration
        return MD_OK;
    }
    return md::autotune(ctx, s, d_action, action_per_step, d_obs, n_obs_slots, n_steps, step0, (hipStream_t)stream,
                        cache_path, force);
}

md_status md_get_launch_config(const md_ctx *ctx, md_launch_config *out) {
    if (!ctx || !out) return MD_E_INVALID_ARG;
    out->lanes_per_drone = ctx->cfg.lpd;
    out->unroll = ctx->cfg.unroll;
    out->waves_per_group = ctx->cfg.waves;
    out->pair_symmetric = ctx->cfg.sym;
    return MD_OK;
}

md_status md_set_launch_config(md_ctx *ctx, md_launch_config *cfg) {
    if (!ctx || !cfg) return MD_E_INVALID_ARG;
    if (!ctx->has_layout) {
        ctx->err = "md_set_launch_config: bind a layout first";
        return MD_E_LAYOUT;
    }
    md::LaunchCfg c{cfg->lanes_per_drone, cfg->unroll, cfg->waves_per_group, cfg->pair_symmetric};
    const bool lpd_ok = c.lpd == 1 || c.lpd == 2 || c.lpd == 4;
    const bool u_ok = c.unroll == 1 || c.unroll == 2 || c.unroll == 4;
    const bool w_ok = c.waves == 1 || c.waves == 2 || c.waves == 4 || c.waves == 8 || c.waves == 16;
    if (!lpd_ok || !u_ok || !w_ok || !md::cfg_valid(ctx, c)) {
        ctx->err = "md_set_launch_config: invalid configuration for this layout";
        return MD_E_INVALID_ARG;
    }
    md::set_cfg(ctx, c);
    return MD_OK;
}

md_status md_rollout_graph_create(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                                  float *d_obs, int n_obs_slots, int steps_per_launch, int n_launches,
                                  int64_t step0, void *stream, md_graph **out) {
    if (!ctx || !out) return MD_E_INVALID_ARG;
    *out = nullptr;
    if (steps_per_launch < 1 || n_launches < 1 || step0 < 0) {
        ctx->err = "md_rollout_graph_create: steps_per_launch and n_launches must be >= 1";
        return MD_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    // bin tables are uploaded synchronously on first use: do it before capture
    md_status prc = md::prepare_launch(ctx);
    if (prc != MD_OK) return prc;
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ctx->err = md::hip_msg("graph capture stream", e);
        return MD_E_HIP;
    }
    md_graph *g = new (std::nothrow) md_graph();
    if (!g) {
        (void)hipStreamDestroy(cap);
        return MD_E_OOM;
    }
    g->ctx = ctx;
    g->gen = ctx->gen;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    md_status rc = MD_OK;
    if (e == hipSuccess) {
        const long long N = ctx->n_drones;
        for (int l = 0; l < n_launches && rc == MD_OK; ++l) {
            const float *act =
                d_action + (action_per_step ? (long long)l * steps_per_launch * md::action_rows(ctx->act) * N : 0);
            float *obs = d_obs;
            int slots = n_obs_slots;
            if (d_obs && n_obs_slots >= steps_per_launch * n_launches) {
                obs = d_obs + (long long)l * steps_per_launch * 20 * N;
                slots = steps_per_launch;
            }
            rc = md_step(ctx, s, act, action_per_step, obs, slots, steps_per_launch,
                         step0 + (int64_t)l * steps_per_launch, cap);
        }
        hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
        if (e == hipSuccess) e = e2;
    }
    if (rc == MD_OK && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    (void)st;
    if (rc != MD_OK || e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        if (rc == MD_OK) {
            ctx->err = md::hip_msg("rollout graph capture", e);
            rc = MD_E_HIP;
        }
        return rc;
    }
    ctx->graphs.insert(g);
    *out = g;
    return MD_OK;
}

md_status md_graph_launch(md_graph *g, void *stream) {
    if (!g || !g->exec) return MD_E_INVALID_ARG;
    // the captured kernels point at the bin tables, surrogate buffers and
    // settings of the context as it was at capture: refuse a graph whose
    // context has since changed them or been destroyed (nothing is launched)
    if (!g->ctx) return MD_E_LAYOUT;
    if (g->gen != g->ctx->gen) {
        g->ctx->err = "md_graph_launch: the context's layout or settings changed since capture; capture again";
        return MD_E_LAYOUT;
    }
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        g->ctx->err = md::hip_msg("hipGraphLaunch", e);
        return MD_E_HIP;
    }
    return MD_OK;
}

void md_graph_destroy(md_graph *g) {
    if (!g) return;
    if (g->ctx) g->ctx->graphs.erase(g);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
