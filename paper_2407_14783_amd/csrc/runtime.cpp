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
    if (p.ctrl != VF_CTBR && p.ctrl != VF_SRT && p.ctrl != VF_PS && p.ctrl != VF_LV)
        return *why = "ctrl must be VF_CTBR, VF_SRT, VF_PS or VF_LV", false;
    if (!pos(p.mass) || !pos(p.arm) || !pos(p.tau_motor) || !pos(p.kappa_yaw) || !pos(p.f_max))
        return *why = "mass, arm, tau_motor, kappa_yaw and f_max must be > 0", false;
    for (int i = 0; i < 3; ++i) {
        if (!pos(p.J[i])) return *why = "J must be > 0", false;
        if (!fin(p.k_lin[i]) || !fin(p.c_quad[i]) || !fin(p.k_rate[i]))
            return *why = "drag and rate gains must be finite", false;
    }
    if (!fin(p.g)) return *why = "g must be finite", false;
    if (p.ctrl == VF_PS || p.ctrl == VF_LV) {
        if (!(p.g > 0.f)) return *why = "PS / LV need g > 0", false;
        for (int i = 0; i < 3; ++i)
            if (!fin(p.k_pos[i]) || !fin(p.k_vel[i]) || !fin(p.k_att[i]))
                return *why = "PS / LV gains must be finite", false;
        if (!(p.max_tilt > 0.f && p.max_tilt < 1.5707f)) return *why = "max_tilt must be in (0, pi/2)", false;
    }
    return true;
}

template <typename T>
static DynConstT<T> dyn_const(const vf_dyn_params& p) {
    DynConstT<T> c;
    const double h = (double)p.dt / (double)p.n_sub;
    c.h = (T)h;
    c.n_sub = p.n_sub;
    c.integrator = p.integrator;
    c.ctrl = p.ctrl;
    c.mass = (T)p.mass;
    c.inv_mass = (T)(1.0 / (double)p.mass);
    c.g = (T)p.g;
    for (int i = 0; i < 3; ++i) {
        c.J[i] = (T)p.J[i];
        c.inv_J[i] = (T)(1.0 / (double)p.J[i]);
        c.kJ[i] = (T)((double)p.J[i] * (double)p.k_rate[i]);
        c.k_lin[i] = (T)p.k_lin[i];
        c.c_quad[i] = (T)p.c_quad[i];
    }
    c.arm_a = (T)((double)p.arm / sqrt(2.0));
    c.inv_a = (T)(sqrt(2.0) / (double)p.arm);
    c.kappa = (T)p.kappa_yaw;
    c.inv_kappa = (T)(1.0 / (double)p.kappa_yaw);
    c.f_max = (T)p.f_max;
    c.e_half = (T)exp(-0.5 * h / (double)p.tau_motor);
    c.e_full = (T)exp(-h / (double)p.tau_motor);
    for (int i = 0; i < 3; ++i) {
        c.k_pos[i] = (T)p.k_pos[i];
        c.k_vel[i] = (T)p.k_vel[i];
        c.k_att[i] = (T)p.k_att[i];
    }
    c.tan_tilt = (T)tan((double)p.max_tilt);
    c.min_lift = (T)(0.25 * (double)p.g);
    return c;
}

DynConst make_dyn_const(const vf_dyn_params& p) { return dyn_const<float>(p); }
DynConstD make_dyn_const_d(const vf_dyn_params& p) { return dyn_const<double>(p); }

bool check_noise(const vf_noise& c, std::string* why) {
    auto model_ok = [](int32_t m) { return m >= VF_NOISE_NONE && m <= VF_NOISE_POISSON; };
    if (!model_ok(c.depth_model) || !model_ok(c.rgb_model) || !model_ok(c.seg_model))
        return *why = "noise model must be one of VF_NOISE_NONE .. VF_NOISE_POISSON", false;
    auto sig = [](float x) { return isfinite(x) && x >= 0.f; };
    auto prob = [](float x) { return x >= 0.f && x <= 1.f; };
    if (!sig(c.depth_sigma) || !sig(c.rgb_sigma) || !sig(c.seg_sigma))
        return *why = "noise sigma must be finite and >= 0", false;
    if (!prob(c.depth_p) || !prob(c.rgb_p) || !prob(c.seg_p)) return *why = "noise p must be in [0, 1]", false;
    auto scale_ok = [](int32_t m, float c) { return m != VF_NOISE_POISSON || (isfinite(c) && c > 0.f); };
    if (!scale_ok(c.depth_model, c.depth_scale) || !scale_ok(c.rgb_model, c.rgb_scale) ||
        !scale_ok(c.seg_model, c.seg_scale))
        return *why = "a Poisson model needs a finite scale > 0", false;
    if (c.reserved != 0) return *why = "reserved must be 0", false;
    return true;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free step (vf_step_noalloc): a file-scope device array, one copy per GPU,
// held until the process ends.  Layout: the fused launch's arrival counters (one per state slot), then
// the cost order's per-workgroup work and its workgroup order.  The host reaches it only through the
// address hipGetSymbolAddress returns on each device (the array's name is not a device address in host
// code).
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocSlots = 1 << 18;
constexpr int64_t kNoAllocCost = (int64_t)kGroupOrderMax * kWavesPerBlock;
constexpr int64_t kNoAllocWords = kNoAllocSlots + kNoAllocCost + kGroupOrderMax;
static __device__ __align__(256) int32_t scratch[kNoAllocWords];

struct NoAllocDevice {
    int32_t* ptr = nullptr;              // this device's copy of scratch
    int32_t cost_n = -1, cost_groups = -1;   // launch shape the work in the cost section belongs to
};
constexpr int kNoAllocDevices = 64;
static std::mutex g_noalloc_mu;
static NoAllocDevice g_noalloc[kNoAllocDevices];

// Once per device, with that device current: the device address of its scratch.
static vf_status noalloc_setup(int device) {
    if (device >= kNoAllocDevices) return fail(VF_EINVAL, "vf_create: device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc[device].ptr) return VF_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_noalloc[device].ptr = (int32_t*)p;
    return VF_OK;
}

static vf_status sync_scene_table(vf_ctx* ctx) {
    std::vector<SceneDesc> tab(kMaxScenes);
    std::vector<const int32_t*> lab(kMaxScenes, nullptr);
    memset(tab.data(), 0, sizeof(SceneDesc) * kMaxScenes);
    int32_t deepest = 0;
    for (size_t i = 0; i < ctx->scenes.size(); ++i)
        if (ctx->scenes[i].used) {
            deepest = std::max(deepest, (int32_t)ctx->scenes[i].info.depth);
            tab[i] = ctx->scenes[i].desc;
            lab[i] = ctx->scenes[i].labels;
        }
    // a deeper scene is announced before the device table holds it, a shallower maximum only after
    if (deepest > ctx->max_bvh_depth.load()) ctx->max_bvh_depth.store(deepest);
    VF_HIP(hipMemcpy(ctx->d_scenes, tab.data(), sizeof(SceneDesc) * kMaxScenes, hipMemcpyHostToDevice));
    VF_HIP(hipMemcpy(ctx->d_labels, lab.data(), sizeof(void*) * kMaxScenes, hipMemcpyHostToDevice));
    ctx->max_bvh_depth.store(deepest);
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
    s = ctx_alloc(ctx, &p, sizeof(void*) * kMaxScenes);
    if (s != VF_OK) { ctx_free(ctx, ctx->d_scenes, sizeof(SceneDesc) * kMaxScenes); delete ctx; return s; }
    ctx->d_labels = (const int32_t**)p;
    s = ctx_alloc(ctx, &p, 256);
    if (s != VF_OK) { ctx_free(ctx, ctx->d_scenes, sizeof(SceneDesc) * kMaxScenes); delete ctx; return s; }
    ctx->d_err = (uint32_t*)p;
    ctx->d_stats = (unsigned long long*)((char*)p + 64);        // VF_STAT_COUNT counters
    ctx->d_build_err = (uint32_t*)((char*)p + 192);
    if (hipMemset(p, 0, 256) != hipSuccess || sync_scene_table(ctx) != VF_OK) {
        vf_destroy(ctx);
        return fail(VF_EHIP, "vf_create: device initialisation failed");
    }
    s = noalloc_setup(device);
    if (s != VF_OK) {
        const std::string why = vf_last_error(nullptr);
        vf_destroy(ctx);
        return fail(s, why);
    }
    *out = ctx;
    return VF_OK;
}

vf_status vf_destroy(vf_ctx* ctx) {
    if (!ctx) return fail(VF_EINVAL, "vf_destroy: NULL context");
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& s : ctx->scenes)
        if (s.used) {
            ctx_free(ctx, s.block, s.bytes);
            if (s.labels) ctx_free(ctx, s.labels, s.label_bytes);
        }
    for (auto& c : ctx->counters) ctx_free(ctx, c.counters, c.capacity * 4);
    ctx_free(ctx, ctx->d_scenes, sizeof(SceneDesc) * kMaxScenes);
    ctx_free(ctx, (void*)ctx->d_labels, sizeof(void*) * kMaxScenes);
    if (ctx->swarm_bytes) ctx_free(ctx, (void*)ctx->swarm.off, ctx->swarm_bytes);
    for (auto& tr : ctx->swarm_trees) ctx_free(ctx, tr.block, tr.bytes);
    for (auto& o : ctx->orders) ctx_free(ctx, o.order, kStreamScratchBytes);
    for (auto* list : {&ctx->timing_events, &ctx->timing_free})
        for (auto& ev : *list) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
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
    // the build's input check reports into a word of its own; the shared sticky word is left alone
    const uint32_t zero = 0;
    VF_HIP(hipMemcpyAsync(ctx->d_build_err, &zero, 4, hipMemcpyHostToDevice, st));
    SceneHost sh;
    vf_status s = build_scene(ctx, verts, V, tris, (int32_t)T, tri_rgb, st, &sh);
    if (s != VF_OK) return s;
    uint32_t err = 0;
    VF_HIP(hipMemcpy(&err, ctx->d_build_err, 4, hipMemcpyDeviceToHost));
    if (err & kErrTriIndex) {
        ctx_free(ctx, sh.block, sh.bytes);
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
    if (s.labels) ctx_free(ctx, s.labels, s.label_bytes);
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
    int64_t nb = s.info.n_nodes * (int64_t)sizeof(Node), tb = s.info.n_tris * (int64_t)sizeof(Tri);
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

// Render launch, bracketed by a pair of events on the stream while timing is enabled.
static hipError_t timed_render(vf_ctx* ctx, const RenderArgs& a, bool fused, hipStream_t st) {
    const bool noise = ctx->render_noise_on;
    if (!ctx->timing) return launch_render(a, fused, ctx->stats, noise, st);
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->timing_free.empty()) {
            ev = ctx->timing_free.back();
            ctx->timing_free.pop_back();
        }
    }
    hipError_t e = hipSuccess;
    if (!ev.first) {
        // timing only: no system-scope fence (cache write-back and invalidation) at each record
        e = hipEventCreateWithFlags(&ev.first, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev.second, hipEventDisableSystemFence);
        if (e != hipSuccess) return e;
    }
    e = hipEventRecord(ev.first, st);
    if (e == hipSuccess) e = launch_render(a, fused, ctx->stats, noise, st);
    if (e == hipSuccess) e = hipEventRecord(ev.second, st);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->timing_events.push_back(ev);
    return e;
}

// Launch-order scratch of a stream (one per stream, so concurrent streams never share it).
static StreamScratch* scratch_for(vf_ctx* ctx, hipStream_t st) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto& o : ctx->orders)
            if (o.stream == (void*)st) return &o;
    }
    void* p = nullptr;
    if (ctx_alloc(ctx, &p, kStreamScratchBytes) != VF_OK) return nullptr;
    StreamScratch sc;
    sc.stream = (void*)st;
    sc.order = (int32_t*)p;
    sc.cost = sc.order + kOrderMax;
    sc.perm = sc.cost + (int64_t)kGroupOrderMax * kWavesPerBlock;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->orders.push_back(sc);
    return &ctx->orders.back();
}

// Launch order of a render: each XCD's workgroups longest first by the work the previous launch of the
// same shape on this stream reported (launches of kGroupOrderMin .. kGroupOrderMax workgroups; the first
// launch of a shape keeps the plain workgroup order and records the work).  Other batches of 64 ..
// kOrderAutoMax agents are put in spatial order (at 1,024 agents the rank-counting kernel takes 25 us and
// the render gains nothing measurable); the two are not combined: a cost-ordered launch gains nothing
// from the spatial order, and its work estimates are kept per logical group, which the spatial order
// would move between agents from one step to the next.
// The cost order of a split render: when the launch is eligible, a.cost gets the stream's work record (the
// render writes its work there), and when the previous launch of this shape on the stream left work
// estimates, *g holds the k_group_order arguments for a.group_order and the result is true.
static bool plan_cost_order(vf_ctx* ctx, RenderArgs& a, hipStream_t st, GroupOrderArgs* g) {
    const int32_t gpa = render_groups_per_agent(a.max_h, a.max_w);
    const int64_t total = (int64_t)a.n * gpa;
    if (!(ctx->cost_order && total >= kGroupOrderMin && total <= kGroupOrderMax)) return false;
    StreamScratch* sc = scratch_for(ctx, st);
    if (!sc) return false;   // no memory for the scratch: plain order
    bool have_cost;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        have_cost = sc->cost_n == a.n && sc->cost_groups == gpa;
        sc->cost_n = a.n;
        sc->cost_groups = gpa;
    }
    a.cost = sc->cost;
    if (!have_cost) return false;
    *g = GroupOrderArgs{(int32_t)total, sc->cost, sc->perm};
    return true;
}

// Spatial order (agents of a launch by position) for launches that are not cost-ordered.
static void maybe_spatial_order(vf_ctx* ctx, RenderArgs& a, hipStream_t st) {
    if (a.cost || !(ctx->spatial_order && a.n >= 64 && a.n <= kOrderAutoMax)) return;
    StreamScratch* sc = scratch_for(ctx, st);
    if (!sc) return;
    OrderArgs o{a.n, a.env_idx, a.state, a.n_slots, a.views, sc->order};
    if (launch_order(o, st) == hipSuccess) a.order = sc->order;
}

static void maybe_order(vf_ctx* ctx, RenderArgs& a, hipStream_t st) {
    a.order = nullptr;
    a.group_order = nullptr;
    a.cost = nullptr;
    GroupOrderArgs g{};
    if (plan_cost_order(ctx, a, st, &g) && launch_group_order(g, st) == hipSuccess) a.group_order = g.perm;
    maybe_spatial_order(ctx, a, st);
}

// While swarms are set: the member trees of this stream (allocated once per vf_set_swarms generation),
// rebuilt from the states the render reads, on the render's stream before it.
static vf_status prepare_swarm(vf_ctx* ctx, RenderArgs& a, hipStream_t st) {
    if (ctx->swarm.n <= 0) return VF_OK;
    SwarmTree* tree = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto& tr : ctx->swarm_trees)
            if (tr.stream == (void*)st && tr.gen == ctx->swarm_gen) tree = &tr;
    }
    const int64_t node_bytes = ((int64_t)ctx->swarm_nodes * (int64_t)sizeof(Node4) + 255) / 256 * 256;
    if (!tree) {
        SwarmTree tr;
        tr.stream = (void*)st;
        tr.gen = ctx->swarm_gen;
        tr.bytes = node_bytes + std::max<int64_t>(ctx->swarm_members, 1) * (int64_t)sizeof(SwarmMember);
        vf_status s = ctx_alloc(ctx, &tr.block, tr.bytes);
        if (s != VF_OK) return s;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->swarm_trees.push_back(tr);
        tree = &ctx->swarm_trees.back();
    }
    a.swarm.nodes = (Node4*)tree->block;
    a.swarm.members = (SwarmMember*)((char*)tree->block + node_bytes);
    VF_HIP(launch_swarm_tree(a.swarm, a.state, a.n_slots, ctx->d_err, st));
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
    a.swarm = ctx->swarm;
    a.noise = ctx->render_noise;
    a.max_depth = ctx->max_bvh_depth.load();
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
    DynConstD dc = make_dyn_const_d(*params);
    if (!views) {
        StepArgs a{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        VF_HIP(launch_step(a, st));
        return VF_OK;
    }
    RenderArgs a = make_render_args(ctx, n, env_idx, state, n_slots, views, max_h, max_w, depth, tri_id, rgb,
                                    out_pixels);
    bool split = ctx->launch_mode == VF_LAUNCH_SPLIT;
    if (ctx->launch_mode == VF_LAUNCH_AUTO) {
        const int th = kTileH * kPacketRows, tw = kTileW * kPacketCols;
        int64_t tiles = (int64_t)((max_h + th - 1) / th) * ((max_w + tw - 1) / tw);
        int64_t groups = n * ((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
        split = groups > 1024;
    }
    if (ctx->swarm.n > 0) split = true;   // members must be read after every agent has stepped
    if (split) {
        StepArgs sa{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        // the cost order does not read the states: it runs in the dynamics' launch
        a.order = nullptr;
        a.group_order = nullptr;
        a.cost = nullptr;
        GroupOrderArgs g{};
        if (plan_cost_order(ctx, a, st, &g)) {
            VF_HIP(launch_step_order(sa, g, st));
            a.group_order = g.perm;
        } else {
            VF_HIP(launch_step(sa, st));
        }
        s = prepare_swarm(ctx, a, st);
        if (s != VF_OK) return s;
        maybe_spatial_order(ctx, a, st);
        VF_HIP(timed_render(ctx, a, false, st));
        return VF_OK;
    }
    int32_t* counters = counters_for(ctx, state, n_slots, &s);
    if (!counters) return s;
    a.action = action;
    a.counters = counters;
    a.dyn = dc;
    VF_HIP(timed_render(ctx, a, true, st));
    return VF_OK;
}

vf_status vf_step_noalloc(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx, float* state,
                          int64_t n_slots, const float* action, const vf_view* views, int32_t max_h, int32_t max_w,
                          float* depth, int32_t* tri_id, uint8_t* rgb, int64_t out_pixels, void* stream) {
    vf_status s = check_render_common(ctx, n, state, n_slots, views, max_h, max_w, depth, tri_id, rgb, out_pixels,
                                      "vf_step_noalloc");
    if (s != VF_OK) return s;
    if (!params) return fail(VF_EINVAL, "vf_step_noalloc: params is NULL");
    if (n > 0 && !action) return fail(VF_EINVAL, "vf_step_noalloc: action is NULL");
    std::string why;
    if (!check_dyn_params(*params, &why)) return fail(VF_EINVAL, "vf_step_noalloc: " + why);
    if (n == 0) return VF_OK;
    NoAllocDevice& nd = g_noalloc[ctx->device];
    if (!nd.ptr) return fail(VF_EHIP, "vf_step_noalloc: the device's scratch address is not known");
    if (views && ctx->swarm.n > 0)
        return fail(VF_EINVAL, "vf_step_noalloc: swarm mode needs the per-stream member trees vf_step allocates");
    VF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    DynConstD dc = make_dyn_const_d(*params);
    if (!views) {
        StepArgs a{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        VF_HIP(launch_step(a, st));
        return VF_OK;
    }
    RenderArgs a = make_render_args(ctx, n, env_idx, state, n_slots, views, max_h, max_w, depth, tri_id, rgb,
                                    out_pixels);
    const int32_t gpa = render_groups_per_agent(max_h, max_w);
    const int64_t total = n * (int64_t)gpa;
    const bool split = ctx->launch_mode == VF_LAUNCH_SPLIT || (ctx->launch_mode == VF_LAUNCH_AUTO && total > 1024);
    if (split) {
        StepArgs sa{(int32_t)n, env_idx, state, n_slots, action, ctx->d_err, dc};
        VF_HIP(launch_step(sa, st));
        // the cost order on the scratch's work and order sections (launches of kGroupOrderMin ..
        // kGroupOrderMax workgroups; the first launch of a shape on the device records the work)
        if (ctx->cost_order && total >= kGroupOrderMin && total <= kGroupOrderMax) {
            bool have_cost;
            {
                std::lock_guard<std::mutex> lk(g_noalloc_mu);
                have_cost = nd.cost_n == (int32_t)n && nd.cost_groups == gpa;
                nd.cost_n = (int32_t)n;
                nd.cost_groups = gpa;
            }
            a.cost = nd.ptr + kNoAllocSlots;
            if (have_cost) {
                int32_t* perm = a.cost + kNoAllocCost;
                GroupOrderArgs g{(int32_t)total, a.cost, perm};
                VF_HIP(launch_group_order(g, st));
                a.group_order = perm;
            }
        }
        VF_HIP(launch_render(a, false, ctx->stats, ctx->render_noise_on, st));
        return VF_OK;
    }
    if (n_slots > kNoAllocSlots)
        return fail(VF_EINVAL, "vf_step_noalloc: a fused launch takes at most 262,144 state slots (the scratch's "
                               "arrival counters); use a split launch or vf_step");
    VF_HIP(launch_fill_i32(nd.ptr, n_slots, 0, st));     // the arrival counters start at zero
    a.action = action;
    a.counters = nd.ptr;
    a.dyn = dc;
    VF_HIP(launch_render(a, true, ctx->stats, ctx->render_noise_on, st));
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
    s = prepare_swarm(ctx, a, (hipStream_t)stream);
    if (s != VF_OK) return s;
    maybe_order(ctx, a, (hipStream_t)stream);
    VF_HIP(timed_render(ctx, a, false, (hipStream_t)stream));
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
    StepBackArgs a{(int32_t)n, state_in, action, grad_state_out, grad_state_in, grad_action,
                   make_dyn_const_d(*params)};
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

vf_status vf_sensor_noise(vf_ctx* ctx, int64_t n, const vf_view* views, int32_t max_h, int32_t max_w,
                          const vf_noise* noise, const int32_t* tri_id, float* depth, uint8_t* rgb, int32_t* seg,
                          int64_t out_pixels, void* stream) {
    if (!ctx || !noise) return fail(VF_EINVAL, "vf_sensor_noise: NULL argument");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, "vf_sensor_noise: n must be in [0, 2^24]");
    if (n > 0 && !views) return fail(VF_EINVAL, "vf_sensor_noise: views is NULL");
    if (max_h < 1 || max_w < 1 || max_h > kMaxImage || max_w > kMaxImage)
        return fail(VF_EINVAL, "vf_sensor_noise: max_h/max_w must be in [1, 1024]");
    if (out_pixels < 0) return fail(VF_EINVAL, "vf_sensor_noise: out_pixels must be >= 0");
    std::string why;
    if (!check_noise(*noise, &why)) return fail(VF_EINVAL, "vf_sensor_noise: " + why);
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    NoiseArgs a{(int32_t)n, views, max_h, max_w, 0, *noise, tri_id, depth, rgb, seg, out_pixels, ctx->d_err};
    VF_HIP(launch_noise(a, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_set_render_noise(vf_ctx* ctx, const vf_noise* noise) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_render_noise: NULL context");
    if (!noise) {
        ctx->render_noise_on = false;
        ctx->render_noise = vf_noise{};
        return VF_OK;
    }
    std::string why;
    if (!check_noise(*noise, &why)) return fail(VF_EINVAL, "vf_set_render_noise: " + why);
    ctx->render_noise = *noise;
    ctx->render_noise_on = noise->depth_model != VF_NOISE_NONE || noise->rgb_model != VF_NOISE_NONE;
    return VF_OK;
}

vf_status vf_scene_set_labels(vf_ctx* ctx, int32_t scene_id, const int32_t* labels) {
    if (!ctx) return fail(VF_EINVAL, "vf_scene_set_labels: NULL context");
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].used)
        return fail(VF_ENOSCENE, "vf_scene_set_labels: no such scene");
    VF_HIP(hipSetDevice(ctx->device));
    SceneHost& s = ctx->scenes[scene_id];
    VF_HIP(hipDeviceSynchronize());
    if (s.labels) {
        ctx_free(ctx, s.labels, s.label_bytes);
        s.labels = nullptr;
        s.label_bytes = 0;
    }
    if (labels) {
        void* p = nullptr;
        int64_t bytes = s.info.n_tris * 4;
        vf_status st = ctx_alloc(ctx, &p, bytes);
        if (st != VF_OK) return st;
        VF_HIP(hipMemcpy(p, labels, bytes, hipMemcpyDeviceToDevice));
        s.labels = (int32_t*)p;
        s.label_bytes = bytes;
    }
    return sync_scene_table(ctx);
}

vf_status vf_segmentation(vf_ctx* ctx, int64_t n, const vf_view* views, int32_t max_h, int32_t max_w,
                          const int32_t* tri_id, int32_t* seg, int64_t out_pixels, void* stream) {
    if (!ctx) return fail(VF_EINVAL, "vf_segmentation: NULL context");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, "vf_segmentation: n must be in [0, 2^24]");
    if (n > 0 && (!views || !tri_id || !seg)) return fail(VF_EINVAL, "vf_segmentation: NULL array");
    if (max_h < 1 || max_w < 1 || max_h > kMaxImage || max_w > kMaxImage)
        return fail(VF_EINVAL, "vf_segmentation: max_h/max_w must be in [1, 1024]");
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    SegArgs a{ctx->d_scenes, ctx->d_labels, (int32_t)ctx->scenes.size(), (int32_t)n, views, max_h, max_w, 0,
              tri_id, seg, out_pixels, ctx->d_err};
    VF_HIP(launch_segment(a, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_imu(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx, const float* state,
                 int64_t n_slots, float sigma_acc, float sigma_gyro, uint64_t seed, const int32_t* keys, float* out,
                 void* stream) {
    if (!ctx || !params) return fail(VF_EINVAL, "vf_imu: NULL argument");
    if (n < 0 || n > (1 << 24)) return fail(VF_EINVAL, "vf_imu: n must be in [0, 2^24]");
    if (n > 0 && (!state || !out || n_slots < 1)) return fail(VF_EINVAL, "vf_imu: NULL array or empty table");
    if (!(sigma_acc >= 0.f) || !(sigma_gyro >= 0.f)) return fail(VF_EINVAL, "vf_imu: sigma must be >= 0");
    std::string why;
    if (!check_dyn_params(*params, &why)) return fail(VF_EINVAL, "vf_imu: " + why);
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    ImuArgs a{(int32_t)n, env_idx, state, n_slots, sigma_acc, sigma_gyro, seed, keys, out, ctx->d_err,
              make_dyn_const(*params)};
    VF_HIP(launch_imu(a, (hipStream_t)stream));
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
                closest, tri_id, ctx->d_err, nullptr, nullptr, 0, nullptr, 0.0f, nullptr, nullptr, SwarmTable{}};
    VF_HIP(launch_closest_point(q, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_collision(vf_ctx* ctx, int64_t n, const int32_t* env_idx, const float* state, int64_t n_slots,
                       const vf_view* views, float radius, float max_dist, float* dist, float* rel, uint8_t* collided,
                       void* stream) {
    if (!ctx) return fail(VF_EINVAL, "vf_collision: NULL context");
    if (n < 0 || n > (1 << 26)) return fail(VF_EINVAL, "vf_collision: n must be in [0, 2^26]");
    if (n > 0 && (!state || !views || !dist || n_slots < 1)) return fail(VF_EINVAL, "vf_collision: NULL array");
    if (!(max_dist > 0.0f) || !(radius >= 0.0f)) return fail(VF_EINVAL, "vf_collision: need max_dist > 0, radius >= 0");
    if (n == 0) return VF_OK;
    VF_HIP(hipSetDevice(ctx->device));
    QueryArgs q{ctx->d_scenes, (int32_t)ctx->scenes.size(), (int32_t)n, nullptr, nullptr, 0, max_dist, dist,
                nullptr, nullptr, ctx->d_err, state, env_idx, n_slots, views, radius, rel, collided, ctx->swarm};
    VF_HIP(launch_closest_point(q, (hipStream_t)stream));
    return VF_OK;
}

vf_status vf_set_swarms(vf_ctx* ctx, int32_t n_swarms, const int32_t* offsets, const int32_t* slots,
                        const float half_extent[3], const uint8_t rgb[3]) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_swarms: NULL context");
    if (n_swarms < 0 || n_swarms > (1 << 20)) return fail(VF_EINVAL, "vf_set_swarms: n_swarms must be in [0, 2^20]");
    if (n_swarms > 0 && (!offsets || !half_extent || !rgb)) return fail(VF_EINVAL, "vf_set_swarms: NULL argument");
    int64_t total = 0;
    if (n_swarms > 0) {
        if (offsets[0] != 0) return fail(VF_EINVAL, "vf_set_swarms: offsets[0] must be 0");
        for (int32_t s = 0; s < n_swarms; ++s)
            if (offsets[s + 1] < offsets[s]) return fail(VF_EINVAL, "vf_set_swarms: offsets must not decrease");
        total = offsets[n_swarms];
        if (total > 0 && !slots) return fail(VF_EINVAL, "vf_set_swarms: slots is NULL");
        for (int64_t j = 0; j < total; ++j)
            if (slots[j] < 0) return fail(VF_EINVAL, "vf_set_swarms: negative slot");
        for (int32_t s = 0; s < n_swarms; ++s)
            if (offsets[s + 1] - offsets[s] > kSwarmMaxMembers)
                return fail(VF_EINVAL, "vf_set_swarms: a swarm holds at most 4,096 members");
        for (int k = 0; k < 3; ++k)
            if (!(half_extent[k] > 0.f) || !isfinite(half_extent[k]))
                return fail(VF_EINVAL, "vf_set_swarms: half extents must be > 0");
    }
    VF_HIP(hipSetDevice(ctx->device));
    VF_HIP(hipDeviceSynchronize());
    if (ctx->swarm_bytes) {
        ctx_free(ctx, (void*)ctx->swarm.off, ctx->swarm_bytes);
        ctx->swarm = SwarmTable{};
        ctx->swarm_bytes = 0;
    }
    for (auto& tr : ctx->swarm_trees) ctx_free(ctx, tr.block, tr.bytes);
    ctx->swarm_trees.clear();
    ctx->swarm_members = 0;
    ctx->swarm_nodes = 0;
    ++ctx->swarm_gen;
    if (n_swarms == 0) return VF_OK;
    // first node of each swarm's tree
    std::vector<int32_t> node_off((size_t)n_swarms + 1, 0);
    for (int32_t s = 0; s < n_swarms; ++s) node_off[s + 1] = node_off[s] + swarm_tree_nodes(offsets[s + 1] - offsets[s]);
    const int64_t off_bytes = ((int64_t)(n_swarms + 1) * 4 + 255) / 256 * 256;
    const int64_t slot_bytes = (std::max<int64_t>(total, 1) * 4 + 255) / 256 * 256;
    const int64_t bytes = 2 * off_bytes + slot_bytes;
    void* p = nullptr;
    vf_status st = ctx_alloc(ctx, &p, bytes);
    if (st != VF_OK) return st;
    char* base = (char*)p;
    int32_t* d_off = (int32_t*)base;
    int32_t* d_node_off = (int32_t*)(base + off_bytes);
    int32_t* d_slots = (int32_t*)(base + 2 * off_bytes);
    VF_HIP(hipMemcpy(d_off, offsets, (size_t)(n_swarms + 1) * 4, hipMemcpyHostToDevice));
    VF_HIP(hipMemcpy(d_node_off, node_off.data(), (size_t)(n_swarms + 1) * 4, hipMemcpyHostToDevice));
    if (total > 0) VF_HIP(hipMemcpy(d_slots, slots, total * 4, hipMemcpyHostToDevice));
    SwarmTable t{};
    t.off = d_off;
    t.slots = d_slots;
    t.node_off = d_node_off;
    t.n = n_swarms;
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        t.half[k] = half_extent[k];
        r2 += (double)half_extent[k] * half_extent[k];
    }
    t.radius = (float)sqrt(r2);
    for (int k = 0; k < 3; ++k) t.rgb[k] = rgb[k];
    ctx->swarm = t;
    ctx->swarm_bytes = bytes;
    ctx->swarm_members = total;
    ctx->swarm_nodes = node_off[n_swarms];
    return VF_OK;
}

vf_status vf_set_cost_order(vf_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_cost_order: NULL context");
    ctx->cost_order = enable != 0;
    return VF_OK;
}

vf_status vf_set_spatial_order(vf_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_spatial_order: NULL context");
    ctx->spatial_order = enable != 0;
    return VF_OK;
}

vf_status vf_set_launch_mode(vf_ctx* ctx, int32_t mode) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_launch_mode: NULL context");
    if (mode != VF_LAUNCH_SPLIT && mode != VF_LAUNCH_FUSED && mode != VF_LAUNCH_AUTO)
        return fail(VF_EINVAL, "vf_set_launch_mode: bad mode");
    ctx->launch_mode = mode;
    return VF_OK;
}

vf_status vf_set_bvh_builder(vf_ctx* ctx, int32_t builder) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_bvh_builder: NULL context");
    if (builder != VF_BVH_CLUSTER && builder != VF_BVH_RADIX) return fail(VF_EINVAL, "vf_set_bvh_builder: bad builder");
    ctx->bvh_builder = builder;
    return VF_OK;
}

vf_status vf_set_bvh_leaf_size(vf_ctx* ctx, int32_t max_tris) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_bvh_leaf_size: NULL context");
    if (max_tris < 1 || max_tris > kLeafMax) return fail(VF_EINVAL, "vf_set_bvh_leaf_size: size out of range");
    ctx->bvh_leaf = max_tris;
    return VF_OK;
}

vf_status vf_set_stats(vf_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_stats: NULL context");
    ctx->stats = enable != 0;
    return VF_OK;
}

vf_status vf_stats_read(vf_ctx* ctx, uint64_t out[VF_STAT_COUNT], int32_t reset) {
    if (!ctx || !out) return fail(VF_EINVAL, "vf_stats_read: NULL argument");
    VF_HIP(hipSetDevice(ctx->device));
    VF_HIP(hipDeviceSynchronize());
    VF_HIP(hipMemcpy(out, ctx->d_stats, 8 * VF_STAT_COUNT, hipMemcpyDeviceToHost));
    if (reset) VF_HIP(hipMemset(ctx->d_stats, 0, 8 * VF_STAT_COUNT));
    return VF_OK;
}

vf_status vf_set_timing(vf_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(VF_EINVAL, "vf_set_timing: NULL context");
    VF_HIP(hipSetDevice(ctx->device));
    if (!enable) {
        VF_HIP(hipDeviceSynchronize());
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto& ev : ctx->timing_events) ctx->timing_free.push_back(ev);
        ctx->timing_events.clear();
    }
    ctx->timing = enable != 0;
    return VF_OK;
}

vf_status vf_timing_read(vf_ctx* ctx, double* total_ms, int64_t* launches, int32_t reset) {
    if (!ctx || !total_ms || !launches) return fail(VF_EINVAL, "vf_timing_read: NULL argument");
    VF_HIP(hipSetDevice(ctx->device));
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        evs = ctx->timing_events;
    }
    double total = 0.0;
    for (auto& ev : evs) {
        VF_HIP(hipEventSynchronize(ev.second));
        float ms = 0.f;
        VF_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
        total += ms;
    }
    *total_ms = total;
    *launches = (int64_t)evs.size();
    if (reset) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto& ev : evs) ctx->timing_free.push_back(ev);
        ctx->timing_events.erase(ctx->timing_events.begin(), ctx->timing_events.begin() + evs.size());
    }
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
    if (err & kErrView) m += " bad view (size, hfov or clip range);";
    if (err & kErrStack) m += " traversal stack overflow;";
    if (err & kErrTriIndex) m += " triangle vertex index out of range;";
    if (err & kErrVertex) m += " vertex coordinate not finite;";
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
