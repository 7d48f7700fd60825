// md_ctx.h -- the context object behind the opaque md_ctx* of the C ABI.
#pragma once

#include <map>
#include <set>
#include <string>
#include <vector>

#include "md.h"
#include "md_internal.h"

namespace md {

// Environment bins for one bin size (slots per workgroup).
struct BinSet {
    int slots = 0;
    int n_bins = 0;
    int2 *d_slot = nullptr;
    int *d_mmax = nullptr;
    std::vector<int> h_mmax;
};

struct SurrogateState;  // md_surrogate.hip

std::string hip_msg(const char *what, hipError_t e);
void derive(const md_params &p, md_derived &d);

}  // namespace md

struct md_ctx {
    // Bumped by every call that frees or replaces what captured kernels point
    // at, or changes which kernel md_step launches (layout, launch
    // configuration, integrator, randomisation, wind, surrogate); a captured
    // rollout remembers the value it was captured under.
    uint64_t gen = 1;
    std::set<md_graph *> graphs;  // live captured rollouts of this context
    md_params P{};
    md_derived D{};
    float dt = 0.f;
    uint32_t mask = 0;
    int act = 0;
    int decim = 1;
    int integ = MD_INTEG_EULER;
    bool dr_on = false;
    md::DrPtr dr{nullptr, nullptr, nullptr};
    md::WindArgs wind{};  // models == 0: off
    int device = 0;
    int n_cu = 0;
    md::KConst kc{};
    // layout
    bool has_layout = false;
    int n_envs = 0, n_drones = 0, max_m = 0;
    std::vector<int32_t> off;
    int uniform_m = 0;  // the common size of all non-empty environments, or 0
    std::map<int, md::BinSet> binsets;  // keyed by 4 x slots per bin + packing mode (BinMode)
    md::LaunchCfg cfg{1, 4, 1, 0};
    bool tuned = false;
    // optional subsystems
    md::SurrogateState *sur = nullptr;
    std::string err;
};

// A captured rollout (md_rollout_graph_create).  ctx is null once the context
// is destroyed; gen is the context's generation at capture.
struct md_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    md_ctx *ctx = nullptr;
    uint64_t gen = 0;
};

namespace md {

// Packing of environments into bins: contiguous runs (best fit decreasing),
// contiguous runs that never cross a wavefront, or interleaved inside each
// wave (uniform power-of-two environments, the rotation sweep).
enum BinMode { BIN_PACKED = 0, BIN_WAVE_ALIGNED = 1, BIN_INTERLEAVED = 2 };
md_status build_bins(md_ctx *ctx, int slots, int mode, BinSet **out);
void free_bins(md_ctx *ctx);
int slots_for(const md_ctx *ctx, const LaunchCfg &cfg);
int bin_mode_for(const md_ctx *ctx, const LaunchCfg &cfg);
LaunchCfg default_cfg(const md_ctx *ctx);
md_status launch(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                 float *d_obs, int n_obs_slots, int n_steps, int64_t step0, hipStream_t st,
                 const LaunchCfg &cfg);

// Build the bin tables the next md_step will use (synchronous uploads).
md_status prepare_launch(md_ctx *ctx);
bool cfg_valid(const md_ctx *ctx, const LaunchCfg &c);
md_status autotune(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step, float *d_obs,
                   int n_obs_slots, int n_steps, int64_t step0, hipStream_t st, const char *path, int force);

// Captured rollouts of ctx become stale (md_graph_launch refuses them).
inline void invalidate_graphs(md_ctx *ctx) { ++ctx->gen; }
// Subsystems with per-context resources.
md_status surrogate_step(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                         float *d_obs, int n_obs_slots, int n_steps, int64_t step0, hipStream_t st);
void free_surrogate(md_ctx *ctx);
md_status load_surrogate(md_ctx *ctx, const float *params, const float *norm, float dz_ood, int judge_stride);
md_status datagen(md_ctx *ctx, const md_state *s, uint32_t mask, float *d_X, float *d_Y, int32_t *d_nbr,
                  hipStream_t st);
md_status judge_stats(md_ctx *ctx, md_judge *out);
md_status judge_reset(md_ctx *ctx);

}  // namespace md
