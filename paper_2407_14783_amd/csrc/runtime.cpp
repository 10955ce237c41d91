// Host runtime of the C ABI declared in include/visfly.h: contexts, the HBM
// budget ledger, the device scene table, argument validation and launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "vf_internal.h"

namespace vf {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

vf_status fail(vf_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

vf_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VF_ENOMEM : VF_EHIP;
}

vf_status ctx_alloc(vf_ctx* ctx, void** p, int64_t bytes) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->budget > 0 && ctx->used + bytes > ctx->budget)
            return fail(VF_ENOMEM, "HBM budget exceeded: need " + std::to_string(bytes) + " bytes, " +
                                       std::to_string(ctx->budget - ctx->used) + " left");
        ctx->used += bytes;
    }
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->used -= bytes;
        return hip_fail(e, "hipMalloc");
    }
    return VF_OK;
}

void ctx_free(vf_ctx* ctx, void* p, int64_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= bytes;
}

bool check_dyn_params(const vf_dyn_params& p, std::string* why) {
    auto pos = [](float x) { return isfinite(x) && x > 0.f; };
    auto fin = [](float x) { return isfinite(x); };
    if (!pos(p.dt)) return *why = "dt must be > 0", false;
    if (p.n_sub < 1 || p.n_sub > 1024) return *why = "n_sub must be in [1, 1024]", false;
    if (p.integrator != VF_RK4 && p.integrator != VF_EULER) return *why = "integrator must be VF_RK4 or VF_EULER", false;
    if (p.ctrl != VF_CTBR && p.ctrl != VF_SRT) return *why = "ctrl must be VF_CTBR or VF_SRT", false;
    if (!pos(p.mass) || !pos(p.arm) || !pos(p.tau_motor) || !pos(p.kappa_yaw) || !pos(p.f_max))
        return *why = "mass, arm, tau_motor, kappa_yaw and f_max must be > 0", false;
    for (int i = 0; i < 3; ++i) {
        if (!pos(p.J[i])) return *why = "J must be > 0", false;
        if (!fin(p.k_lin[i]) || !fin(p.c_quad[i]) || !fin(p.k_rate[i]))
            return *why = "drag and rate gains must be finite", false;
    }
    if (!fin(p.g)) return *why = "g must be finite", false;
    return true;
}

DynConst make_dyn_const(const vf_dyn_params& p) {
    DynConst c;
    c.h = (float)((double)p.dt / (double)p.n_sub);
    c.n_sub = p.n_sub;
    c.integrator = p.integrator;
    c.ctrl = p.ctrl;
    c.mass = p.mass;
    c.inv_mass = (float)(1.0 / (double)p.mass);
    c.g = p.g;
    for (int i = 0; i < 3; ++i) {
        c.J[i] = p.J[i];
        c.inv_J[i] = (float)(1.0 / (double)p.J[i]);
        c.kJ[i] = (float)((double)p.J[i] * (double)p.k_rate[i]);
        c.k_lin[i] = p.k_lin[i];
        c.c_quad[i] = p.c_quad[i];
    }
    c.arm_a = (float)((double)p.arm / sqrt(2.0));
    c.inv_a = (float)(sqrt(2.0) / (double)p.arm);
    c.kappa = p.kappa_yaw;
    c.inv_kappa = (float)(1.0 / (double)p.kappa_yaw);
    c.f_max = p.f_max;
    double h = (double)p.dt / (double)p.n_sub;
    c.e_half = (float)exp(-0.5 * h / (double)p.tau_motor);
    c.e_full = (float)exp(-h / (double)p.tau_motor);
    return c;
}

static vf_status sync_scene_table(vf_ctx* ctx) {
    std::vector<SceneDesc> tab(kMaxScenes);
    memset(tab.data(), 0, sizeof(SceneDesc) * kMaxScenes);
    for (size_t i = 0; i < ctx->scenes.size(); ++i)
        if (ctx->scenes[i].used) tab[i] = ctx->scenes[i].desc;
    VF_HIP(hipMemcpy(ctx->d_scenes, tab.data(), sizeof(SceneDesc) * kMaxScenes, hipMemcpyHostToDevice));
    return VF_OK;
}

static int32_t* counters_for(vf_ctx* ctx, const float* state, int64_t n_slots, vf_status* st) {
    for (auto& c : ctx->counters) {
        if (c.state == state && c.capacity >= n_slots) return c.counters;
    }
    for (auto it = ctx->counters.begin(); it != ctx->counters.end(); ++it) {
        if (it->state == state) {  // grow: free the old array (no work may be in flight on it)
            (void)hipDeviceSynchronize();
            ctx_free(ctx, it->counters, it->capacity * 4);
            ctx->counters.erase(it);
            break;
        }
    }
    Counters c;
    c.state = state;
    c.capacity = std::max<int64_t>(n_slots, 1024);
    void* p = nullptr;
    *st = ctx_alloc(ctx, &p, c.capacity * 4);
    if (*st != VF_OK) return nullptr;
    if (hipMemset(p, 0, c.capacity * 4) != hipSuccess) {
        *st = fail(VF_EHIP, "hipMemset of arrival counters");
        return nullptr;
    }
    c.counters = (int32_t*)p;
    ctx->counters.push_back(c);
    *st = VF_OK;
    return c.counters;
}

}  // namespace vf

using namespace vf;

extern "C" {

vf_status vf_create(int device, size_t hbm_budget_bytes, vf_ctx** out) {
    if (!out) return fail(VF_EINVAL, "vf_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    VF_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(VF_EINVAL, "vf_create: no such device");
    VF_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    VF_HIP(hipGetDeviceProperties(&prop, device));
    vf_ctx* ctx = new vf_ctx();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->budget = (int64_t)hbm_budget_bytes;
    void* p = nullptr;
    vf_status s = ctx_alloc(ctx, &p, sizeof(SceneDesc) * kMaxScenes);
    if (s != VF_OK) { delete ctx; return s; }
    ctx->d_scenes = (SceneDesc*)p;
    s = ctx_alloc(ctx, &p, 256);
    if (s != VF_OK) { ctx_free(ctx, ctx->d_scenes, sizeof(SceneDesc) * kMaxScenes); delete ctx; return s; }
    ctx->d_err = (uint32_t*)p;
    ctx->d_stats = (unsigned long long*)((char*)p + 64);
    if (hipMemset(p, 0, 256) != hipSuccess || sync_scene_table(ctx) != VF_OK) {
        vf_destroy(ctx);
        return fail(VF_EHIP, "vf_create: device initialisation failed");
    }
    *out = ctx;
    return VF_OK;
}

vf_status vf_destroy(vf_ctx* ctx) {
    if (!ctx) return fail(VF_EINVAL, "vf_destroy: NULL context");
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& s : ctx->scenes)
        if (s.used) ctx_free(ctx, s.block, s.bytes);
    for (auto& c : ctx->counters) ctx_free(ctx, c.counters, c.capacity * 4);
    ctx_free(ctx, ctx->d_scenes, sizeof(SceneDesc) * kMaxScenes);
    ctx_free(ctx, ctx->d_err, 256);
    delete ctx;
    return VF_OK;
}

vf_status vf_scene_build(vf_ctx* ctx, const float* verts, int64_t V, const int32_t* tris, int64_t T,
                         const uint8_t* tri_rgb, void* stream, int32_t* scene_id) {
    if (!ctx || !verts || !tris || !scene_id) return fail(VF_EINVAL, "vf_scene_build: NULL argument");
    if (V < 1 || T < 1 || T >= (1LL << 27)) return fail(VF_EINVAL, "vf_scene_build: need V >= 1 and 1 <= T < 2^27");
    VF_HIP(hipSetDevice(ctx->device));
    int32_t id = -1;
    for (size_t i = 0; i < ctx->scenes.size(); ++i)
        if (!ctx->scenes[i].used) { id = (int32_t)i; break; }
    if (id < 0) {
        if ((int)ctx->scenes.size() >= kMaxScenes) return fail(VF_ENOMEM, "vf_scene_build: scene table full");
        ctx->scenes.emplace_back();
        id = (int32_t)ctx->scenes.size() - 1;
    }
    hipStream_t st = (hipStream_t)stream;
    uint32_t zero = 0;
    VF_HIP(hipMemcpyAsync(ctx->d_err, &zero, 4, hipMemcpyHostToDevice, st));
    SceneHost sh;
    vf_status s = build_scene(ctx, verts, V, tris, (int32_t)T, tri_rgb, st, &sh);
    if (s != VF_OK) return s;
    uint32_t err = 0;
    VF_HIP(hipMemcpy(&err, ctx->d_err, 4, hipMemcpyDeviceToHost));
    if (err & kErrTriIndex) {
        ctx_free(ctx, sh.block, sh.bytes);
        VF_HIP(hipMemcpy(ctx->d_err, &zero, 4, hipMemcpyHostToDevice));
        return fail(VF_EINVAL, "vf_scene_build: triangle vertex index out of range");
    }
    sh.used = true;
    ctx->scenes[id] = sh;
    s = sync_scene_table(ctx);
    if (s != VF_OK) return s;
    *scene_id = id;
    return VF_OK;
}

vf_status vf_scene_free(vf_ctx* ctx, int32_t scene_id) {
    if (!ctx) return fail(VF_EINVAL, "vf_scene_free: NULL context");
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
        return fail(VF_ENOSCENE, "vf_scene_free: no such scene");
    VF_HIP(hipSetDevice(ctx->device));
    SceneHost& s = ctx->scenes[scene_id];
    s.used = false;
    vf_status st = sync_scene_table(ctx);
    ctx_free(ctx, s.block, s.bytes);
    s = SceneHost();
    return st;
}

vf_status vf_scene_info_get(vf_ctx* ctx, int32_t scene_id, vf_scene_info* out) {
    if (!ctx || !out) return fail(VF_EINVAL, "vf_scene_info_get: NULL argument");
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
        return fail(VF_ENOSCENE, "vf_scene_info_get: no such scene");
    *out = ctx->scenes[scene_id].info;
    return VF_OK;
}

vf_status vf_scene_export(vf_ctx* ctx, int32_t scene_id, void* nodes_host, int64_t nodes_cap, void* tris_host,
                          int64_t tris_cap) {
    if (!ctx) return fail(VF_EINVAL, "vf_scene_export: NULL context");
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
        return fail(VF_ENOSCENE, "vf_scene_export: no such scene");
    VF_HIP(hipSetDevice(ctx->device));
    const SceneHost& s = ctx->scenes[scene_id];
    int64_t nb = s.info.n_nodes * (int64_t)sizeof(Node4), tb = s.info.n_tris * (int64_t)sizeof(Tri);
    if (nodes_host) {
        if (nodes_cap < nb) return fail(VF_EINVAL, "vf_scene_export: node buffer too small");
        VF_HIP(hipMemcpy(nodes_host, s.desc.nodes, nb, hipMemcpyDeviceToHost));
    }
    if (tris_host) {
        if (tris_cap < tb) return fail(VF_EINVAL, "vf_scene_export: triangle buffer too small");
        VF_HIP(hipMemcpy(tris_host, s.desc.tris, tb, hipMemcpyDeviceToHost));
    }
    return VF_OK;
}

static vf_status check_render_common(vf_ctx* ctx, int64_t n, const float* state, int64_t n_slots,
                                     const vf_view* views, int32_t max_h, int32_t max_w, float* depth,
                                     int32_t* tri_id, uint8_t* rgb, int64_t out_pixels, const char* who) {
    std::string w(who);
    if (!ctx) return fail(VF_EINVAL, w + ": NULL context");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, w + ": n must be in [0, 2^24]");
    if (n > 0 && !state) return fail(VF_EINVAL, w + ": state is NULL");
    if (n_slots < 0 || (n > 0 && n_slots < 1)) return fail(VF_EINVAL, w + ": n_slots must be >= 1");
    if (views) {
        if (max_h < 1 || max_w < 1 || max_h > kMaxImage || max_w > kMaxImage)
            return fail(VF_EINVAL, w + ": max_h/max_w must be in [1, 1024]");
        if (out_pixels < 0) return fail(VF_EINVAL, w + ": out_pixels must be >= 0");
        if (!depth && !tri_id && !rgb) return fail(VF_EINVAL, w + ": no output requested");
    }
    return VF_OK;
}

static RenderArgs make_render_args(vf_ctx* ctx, int64_t n, const int32_t* env_idx, float* state, int64_t n_slots,
                                   const vf_view* views, int32_t max_h, int32_t max_w, float* depth, int32_t* tri_id,
                                   uint8_t* rgb, int64_t out_pixels) {
    RenderArgs a;
    memset(&a, 0, sizeof(a));
    a.scenes = ctx->d_scenes;
    a.n_scenes = (int32_t)ctx->scenes.size();
    a.n = (int32_t)n;
    a.env_idx = env_idx;
    a.state = state;
    a.n_slots = n_slots;
    a.views = views;
    a.max_h = max_h;
    a.max_w = max_w;
    a.depth = depth;
    a.tri_id = tri_id;
    a.rgb = rgb;
    a.out_pixels = out_pixels;
    a.err = ctx->d_err;
    a.stats = ctx->d_stats;
    return a;
}

vf_status vf_step(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx, float* state,
                  int64_t n_slots, const float* action, const vf_view* views, int32_t max_h, int32_t max_w,
                  float* depth, int32_t* tri_id, uint8_t* rgb, int64_t out_pixels, void* stream) {
    vf_status s = check_render_common(ctx, n, state, n_slots, views, max_h, max_w, depth, tri_id, rgb, out_pixels,
                                      "vf_step");
    if (s != VF_OK) return s;
    if (!params) return fail(VF_EINVAL, "vf_step: params is NULL");
    if (n > 0 && !action) return fail(VF_EINVAL, "vf_step: action is NULL");
    std::string why;
    if (!check_dyn_params(*params, &why)) return fail(VF_EINVAL, "vf_step: " + why);
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    DynConst dc = make_dyn_const(*params);
    if (!views) {
        StepArgs a{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        VF_HIP(launch_step(a, st));
        return VF_OK;
    }
    RenderArgs a = make_render_args(ctx, n, env_idx, state, n_slots, views, max_h, max_w, depth, tri_id, rgb,
                                    out_pixels);
    bool split = ctx->launch_mode == VF_LAUNCH_SPLIT;
    if (ctx->launch_mode == VF_LAUNCH_AUTO) {
        int64_t tiles = (int64_t)((max_h + kTile - 1) / kTile) * ((max_w + kTile - 1) / kTile);
        int64_t groups = n * ((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
        split = groups > 1024;
    }
    if (split) {
        StepArgs sa{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        VF_HIP(launch_step(sa, st));
        VF_HIP(launch_render(a, false, ctx->stats, st));
        return VF_OK;
    }
    int32_t* counters = counters_for(ctx, state, n_slots, &s);
    if (!counters) return s;
    a.action = action;
    a.counters = counters;
    a.dyn = dc;
    VF_HIP(launch_render(a, true, ctx->stats, st));
    return VF_OK;
}

vf_status vf_render(vf_ctx* ctx, int64_t n, const int32_t* env_idx, const float* state, int64_t n_slots,
                    const vf_view* views, int32_t max_h, int32_t max_w, float* depth, int32_t* tri_id, uint8_t* rgb,
                    int64_t out_pixels, void* stream) {
    vf_status s = check_render_common(ctx, n, state, n_slots, views, max_h, max_w, depth, tri_id, rgb, out_pixels,
                                      "vf_render");
    if (s != VF_OK) return s;
    if (n > 0 && !views) return fail(VF_EINVAL, "vf_render: views is NULL");
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    RenderArgs a = make_render_args(ctx, n, env_idx, (float*)state, n_slots, views, max_h, max_w, depth, tri_id, rgb,
                                    out_pixels);
    VF_HIP(launch_render(a, false, ctx->stats, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_step_backward(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const float* state_in,
                           const float* action, const float* grad_state_out, float* grad_state_in,
                           float* grad_action, void* stream) {
    if (!ctx || !params) return fail(VF_EINVAL, "vf_step_backward: NULL argument");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, "vf_step_backward: n must be in [0, 2^24]");
    if (n > 0 && (!state_in || !action || !grad_state_out || !grad_state_in || !grad_action))
        return fail(VF_EINVAL, "vf_step_backward: NULL array");
    std::string why;
    if (!check_dyn_params(*params, &why)) return fail(VF_EINVAL, "vf_step_backward: " + why);
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    StepBackArgs a{(int32_t)n, state_in, action, grad_state_out, grad_state_in, grad_action, make_dyn_const(*params)};
    VF_HIP(launch_step_backward(a, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_render_backward(vf_ctx* ctx, int64_t n, const float* state, const vf_view* views, int32_t max_h,
                             int32_t max_w, const int32_t* tri_id, const float* grad_depth, int64_t out_pixels,
                             float* grad_state, void* stream) {
    if (!ctx) return fail(VF_EINVAL, "vf_render_backward: NULL context");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, "vf_render_backward: n must be in [0, 2^24]");
    if (n > 0 && (!state || !views || !tri_id || !grad_depth || !grad_state))
        return fail(VF_EINVAL, "vf_render_backward: NULL array");
    if (max_h < 1 || max_w < 1 || max_h > kMaxImage || max_w > kMaxImage)
        return fail(VF_EINVAL, "vf_render_backward: max_h/max_w must be in [1, 1024]");
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    RenderBackArgs a{ctx->d_scenes, (int32_t)ctx->scenes.size(), (int32_t)n, state, views, max_h, max_w,
                     tri_id, grad_depth, out_pixels, grad_state, ctx->d_err};
    VF_HIP(launch_render_backward(a, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_closest_point(vf_ctx* ctx, int64_t n, const float* points, const int32_t* scene_ids, int32_t scene_id0,
                           float max_dist, float* dist, float* closest, int32_t* tri_id, void* stream) {
    if (!ctx) return fail(VF_EINVAL, "vf_closest_point: NULL context");
    if (n < 0 || n > (1 << 26)) return fail(VF_EINVAL, "vf_closest_point: n must be in [0, 2^26]");
    if (n > 0 && (!points || !dist)) return fail(VF_EINVAL, "vf_closest_point: NULL array");
    if (!(max_dist > 0.0f)) return fail(VF_EINVAL, "vf_closest_point: max_dist must be > 0");
    if (!scene_ids && (scene_id0 < 0 || scene_id0 >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id0].used))
        return fail(VF_ENOSCENE, "vf_closest_point: no such scene");
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    QueryArgs q{ctx->d_scenes, (int32_t)ctx->scenes.size(), (int32_t)n, points, scene_ids, scene_id0, max_dist, dist,
                closest, tri_id, ctx->d_err};
    VF_HIP(launch_closest_point(q, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_set_launch_mode(vf_ctx* ctx, int32_t mode) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_launch_mode: NULL context");
    if (mode != VF_LAUNCH_SPLIT && mode != VF_LAUNCH_FUSED && mode != VF_LAUNCH_AUTO)
        return fail(VF_EINVAL, "vf_set_launch_mode: bad mode");
    ctx->launch_mode = mode;
    return VF_OK;
}

vf_status vf_set_stats(vf_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_stats: NULL context");
    ctx->stats = enable != 0;
    return VF_OK;
}

vf_status vf_stats_read(vf_ctx* ctx, uint64_t out[8], int32_t reset) {
    if (!ctx || !out) return fail(VF_EINVAL, "vf_stats_read: NULL argument");
    VF_HIP(hipSetDevice(ctx->device));
    VF_HIP(hipDeviceSynchronize());
    VF_HIP(hipMemcpy(out, ctx->d_stats, 64, hipMemcpyDeviceToHost));
    if (reset) VF_HIP(hipMemset(ctx->d_stats, 0, 64));
    return VF_OK;
}

vf_status vf_sync_check(vf_ctx* ctx, void* stream) {
    if (!ctx) return fail(VF_EINVAL, "vf_sync_check: NULL context");
    VF_HIP(hipSetDevice(ctx->device));
    VF_HIP(hipStreamSynchronize((hipStream_t)stream));
    uint32_t err = 0, zero = 0;
    VF_HIP(hipMemcpy(&err, ctx->d_err, 4, hipMemcpyDeviceToHost));
    if (!err) return VF_OK;
    VF_HIP(hipMemcpy(ctx->d_err, &zero, 4, hipMemcpyHostToDevice));
    std::string m = "device reported:";
    if (err & kErrScene) m += " bad scene id;";
    if (err & kErrSlot) m += " env slot out of range;";
    if (err & kErrPixels) m += " output pixels out of range;";
    if (err & kErrView) m += " bad view (size or hfov);";
    if (err & kErrStack) m += " traversal stack overflow;";
    if (err & kErrTriIndex) m += " triangle vertex index out of range;";
    if (err & kErrTriId) m += " triangle id out of range;";
    return fail(VF_EDEVICE, m);
}

vf_status vf_mem_usage(vf_ctx* ctx, int64_t* used_bytes, int64_t* budget_bytes) {
    if (!ctx) return fail(VF_EINVAL, "vf_mem_usage: NULL context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (used_bytes) *used_bytes = ctx->used;
    if (budget_bytes) *budget_bytes = ctx->budget;
    return VF_OK;
}

const char* vf_last_error(vf_ctx*) { return g_last_error.c_str(); }

}  // extern "C"
