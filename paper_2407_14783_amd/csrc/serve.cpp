// Continuous-batching server for step + render requests (the serving form of the
// batched per-environment step: parallel agents in several scenes, Sec. III-B/D).
//
// Requests (a scene, an image size, a set of resident env slots and one action
// per env) are queued on submit with their host inputs copied.  A worker thread
// runs the admission logic of batcher.h (arrival order, arena bytes, no env slot in
// two batches at once, max_batch_agents) over the server's stream slots.  The
// batch's work list (views with output offsets, env slots, actions) goes to the
// device in one copy; the step kernel saves the env slots' states before it steps
// them, the render kernel follows on the slot's stream and the outputs come back to pinned
// host memory on the same stream.  Several slots are in flight at once, so batches
// overlap on the device while new requests are admitted.  A batch that fails to
// launch, or that the host reports failed (vf_server_inject_faults), has its env
// slots restored from the snapshot and its requests queued again.  Agents are
// independent, so a request's result is bitwise the same alone or in any mix.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_set>

#include "batcher.h"
#include "vf_internal.h"

namespace vf {

using Clock = std::chrono::steady_clock;

struct Request : sched::Item {
    int64_t ticket = 0;
    vf_request_desc desc{};
    vf_request_out out{};
    bool host = true;
    std::vector<float> actions;
    Clock::time_point arrival;
    Clock::time_point done_at;
    // results (host)
    std::vector<float> depth;
    std::vector<int32_t> tri_id;
    std::vector<uint8_t> rgb;
    std::vector<float> state;
};

struct SlotArena {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    void* dev = nullptr;        // device arena
    void* host = nullptr;       // pinned host arena (work list upload + results)
    int64_t bytes = 0;
    std::vector<int64_t> px_off;   // per request: first pixel in the batch
    int64_t n_agents = 0, n_px = 0;
    bool snapshot = false;      // the batch's env slots were saved before its step
    // arena sections: error word | views | depth targets | env idx | actions | slot snapshot | depth | ids |
    // rgb | state echo
    int64_t off_views = 0, off_targets = 0, off_idx = 0, off_act = 0, off_before = 0, off_depth = 0, off_ids = 0,
            off_rgb = 0, off_state = 0, end = 0;
};

struct HipBackend;

}  // namespace vf

struct vf_server {
    vf_ctx* ctx = nullptr;
    vf_server_config cfg{};
    float* state = nullptr;
    int64_t n_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int64_t, vf::Request*> all;
    std::vector<vf::SlotArena> arenas;
    vf::HipBackend* backend = nullptr;
    vf::sched::Scheduler<vf::HipBackend>* sched = nullptr;
    std::thread worker;
    std::atomic<bool> stop{false};
    int64_t next_ticket = 1;
    vf::DynConstD dyn{};
    std::string worker_error;
};

namespace vf {

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Bytes a request needs in an arena (work list + slot snapshot + outputs + state echo).
static int64_t request_bytes(const vf_server_config& cfg, const vf_request_desc& d) {
    int64_t px = (int64_t)d.H * d.W * d.n_env;
    // view, depth target, slot, action, snapshot, state
    int64_t b = (int64_t)d.n_env * ((int64_t)sizeof(vf_view) + 8 + 4 + 16 + 17 * 4 + 17 * 4);
    b += px * 4;                                  // depth
    if (cfg.want_tri_id) b += px * 4;
    if (cfg.want_rgb) b += px * 3;
    return b + 10 * 256;                          // the error word's section and the alignment of the nine others
}

// A depth-only server renders a request's depth straight into the device buffer it named, when it keeps no
// host results and the buffer is 4-byte aligned.
static bool renders_in_place(const vf_server* s, const Request* r) {
    return !s->cfg.want_tri_id && !s->cfg.want_rgb && r->out.depth && !r->host &&
           (uintptr_t)r->out.depth % 4 == 0;
}

// Device error bits as text.
static std::string device_error_text(uint32_t err) {
    std::string m = "device reported:";
    if (err & kErrScene) m += " bad scene id;";
    if (err & kErrSlot) m += " env slot out of range;";
    if (err & kErrPixels) m += " output pixels out of range;";
    if (err & kErrView) m += " bad view;";
    if (err & kErrStack) m += " traversal stack overflow;";
    return m;
}

// The scheduler's backend on the device: one arena (device + pinned host memory, a stream, an event) per
// batch in flight.
struct HipBackend {
    vf_server* s;

    // Lay out the arena, upload the work list, save the env slots' states, then step, render, gather the new
    // states and return the outputs, all on the arena's stream.  False when a call failed (the scheduler then
    // restores the slots from the snapshot if it was taken).
    bool launch(int i, std::vector<sched::Item*>& items) {
        SlotArena& a = s->arenas[i];
        a.snapshot = false;
        int64_t n = 0, px = 0;
        for (sched::Item* it : items) {
            const Request* r = static_cast<const Request*>(it);
            n += r->desc.n_env;
            px += (int64_t)r->desc.H * r->desc.W * r->desc.n_env;
        }
        a.n_agents = n;
        a.n_px = px;
        a.off_views = 256;
        a.off_targets = align_up(a.off_views + n * (int64_t)sizeof(vf_view), 256);
        a.off_idx = align_up(a.off_targets + n * 8, 256);
        a.off_act = align_up(a.off_idx + n * 4, 256);
        a.off_before = align_up(a.off_act + n * 16, 256);
        a.off_depth = align_up(a.off_before + n * 17 * 4, 256);
        a.off_ids = align_up(a.off_depth + px * 4, 256);
        a.off_rgb = align_up(a.off_ids + (s->cfg.want_tri_id ? px * 4 : 0), 256);
        a.off_state = align_up(a.off_rgb + (s->cfg.want_rgb ? px * 3 : 0), 256);
        a.end = align_up(a.off_state + n * 17 * 4, 256);
        if (a.end > a.bytes) {   // admission sizes requests so this cannot happen; never launch past the arena
            s->worker_error = "batch larger than its arena";
            return false;
        }
        char* h = (char*)a.host;
        char* d = (char*)a.dev;
        *(uint32_t*)h = 0;          // the batch's own error word, uploaded with the work list
        vf_view* hv = (vf_view*)(h + a.off_views);
        float** ht = (float**)(h + a.off_targets);
        int32_t* hi = (int32_t*)(h + a.off_idx);
        float* ha = (float*)(h + a.off_act);
        // A depth-only batch renders a request that asked for a device depth buffer (and no host results)
        // straight into that buffer: the render writes each view's depth to the entry of a per-view target
        // table (the view's own H x W block of the request's buffer, or of the arena's depth section for the
        // other requests), built here from each request's own buffer and size.  Ids and colours keep the
        // arena offsets and the arena-sized bound check.
        const bool direct = !s->cfg.want_tri_id && !s->cfg.want_rgb;
        int64_t agent = 0, pix = 0;
        a.px_off.clear();
        for (sched::Item* it : items) {
            Request* r = static_cast<Request*>(it);
            a.px_off.push_back(pix);
            const int64_t req_off = pix;
            const bool in_place = renders_in_place(s, r);
            for (int32_t e = 0; e < r->desc.n_env; ++e) {
                const int64_t view_px = (int64_t)r->desc.H * r->desc.W;
                ht[agent] = in_place ? r->out.depth + (int64_t)e * view_px : (float*)(d + a.off_depth) + pix;
                vf_view& v = hv[agent];
                memset(&v, 0, sizeof(v));
                v.scene_id = r->desc.scene_id;
                v.H = r->desc.H;
                v.W = r->desc.W;
                v.flags = 0;
                v.hfov = r->desc.hfov;
                v.near_clip = r->desc.near_clip;
                v.far_clip = r->desc.far_clip;
                v.miss_depth = r->desc.miss_depth;
                v.out_offset = req_off + (int64_t)e * r->desc.H * r->desc.W;
                hi[agent] = r->slots[e];
                memcpy(ha + 4 * agent, r->actions.data() + 4 * e, 16);
                pix += view_px;
                ++agent;
            }
        }
        const int32_t* d_idx = (const int32_t*)(d + a.off_idx);
        hipError_t e = hipMemcpyAsync(d, h, a.off_before, hipMemcpyHostToDevice, a.stream);
        if (e != hipSuccess) {
            s->worker_error = std::string("batch launch: ") + hipGetErrorString(e);
            return false;
        }
        uint32_t* d_err = (uint32_t*)d;
        // the step also keeps the slots' states before it, for a batch that has to run again
        StepArgs sa{(int32_t)n, d_idx, s->state, s->n_slots, (const float*)(d + a.off_act), d_err, s->dyn,
                    (float*)(d + a.off_before)};
        e = launch_step(sa, a.stream);
        if (e != hipSuccess) {
            s->worker_error = std::string("batch launch: ") + hipGetErrorString(e);
            return false;
        }
        a.snapshot = true;
        RenderArgs ra;
        memset(&ra, 0, sizeof(ra));
        ra.scenes = s->ctx->d_scenes;
        ra.n_scenes = (int32_t)s->ctx->scenes.size();
        ra.n = (int32_t)n;
        ra.env_idx = d_idx;
        ra.state = s->state;
        ra.n_slots = s->n_slots;
        ra.views = (const vf_view*)(d + a.off_views);
        ra.max_h = s->cfg.max_h;
        ra.max_w = s->cfg.max_w;
        ra.depth = (float*)(d + a.off_depth);
        ra.depth_views = direct ? (float* const*)(d + a.off_targets) : nullptr;
        ra.tri_id = s->cfg.want_tri_id ? (int32_t*)(d + a.off_ids) : nullptr;
        ra.rgb = s->cfg.want_rgb ? (uint8_t*)(d + a.off_rgb) : nullptr;
        ra.out_pixels = px;
        ra.err = d_err;
        ra.stats = s->ctx->d_stats;
        ra.max_depth = s->ctx->max_bvh_depth.load();
        // no swarms (server views show none) and no spatial order: for the server's batches (mostly one or two
        // requests) the ordering kernel cost more than the cache locality it bought
        if (e == hipSuccess) e = launch_render(ra, false, false, false, a.stream);
        // gather the new states of the batch's env slots with the render's view of them, when a request of
        // the batch takes states back (host results or a device state buffer)
        bool want_state = false;
        for (sched::Item* it : items) {
            const Request* r = static_cast<const Request*>(it);
            want_state = want_state || r->host || r->out.state;
        }
        if (e == hipSuccess && want_state)
            e = launch_gather_rows(s->state, d_idx, (int32_t)n, (float*)(d + a.off_state), a.stream);
        // device outputs: one copy per requested buffer
        bool any_host = false;
        int64_t ag = 0;
        for (size_t k = 0; k < items.size() && e == hipSuccess; ++k) {
            Request* r = static_cast<Request*>(items[k]);
            any_host |= r->host;
            const int64_t rpx = (int64_t)r->desc.H * r->desc.W * r->desc.n_env, p0 = a.px_off[k];
            if (r->out.depth && !renders_in_place(s, r) && e == hipSuccess)
                e = hipMemcpyAsync(r->out.depth, d + a.off_depth + 4 * p0, rpx * 4, hipMemcpyDeviceToDevice,
                                   a.stream);
            if (r->out.tri_id && s->cfg.want_tri_id && e == hipSuccess)
                e = hipMemcpyAsync(r->out.tri_id, d + a.off_ids + 4 * p0, rpx * 4, hipMemcpyDeviceToDevice, a.stream);
            if (r->out.rgb && s->cfg.want_rgb && e == hipSuccess)
                e = hipMemcpyAsync(r->out.rgb, d + a.off_rgb + 3 * p0, rpx * 3, hipMemcpyDeviceToDevice, a.stream);
            if (r->out.state && e == hipSuccess)
                e = hipMemcpyAsync(r->out.state, d + a.off_state + 4 * 17 * ag, (int64_t)r->desc.n_env * 17 * 4,
                                   hipMemcpyDeviceToDevice, a.stream);
            ag += r->desc.n_env;
        }
        if (e == hipSuccess && any_host)
            e = hipMemcpyAsync(h + a.off_depth, d + a.off_depth, a.end - a.off_depth, hipMemcpyDeviceToHost, a.stream);
        // the batch's error word comes back with it (the upload has read the host word before, in stream order)
        if (e == hipSuccess) e = hipMemcpyAsync(h, d, 4, hipMemcpyDeviceToHost, a.stream);
        if (e == hipSuccess) e = hipEventRecord(a.event, a.stream);
        if (e != hipSuccess) {
            s->worker_error = std::string("batch launch: ") + hipGetErrorString(e);
            return false;
        }
        return true;
    }

    int poll(int i) {
        const hipError_t q = hipEventQuery(s->arenas[i].event);
        if (q == hipSuccess) return 1;
        if (q == hipErrorNotReady) return 0;
        s->worker_error = std::string("batch failed: ") + hipGetErrorString(q);
        return -1;
    }

    uint32_t finish(int i, std::vector<sched::Item*>& items) {
        SlotArena& a = s->arenas[i];
        const char* h = (const char*)a.host;
        // a fault a kernel of this batch flagged (data it skipped) fails every request of the batch
        const uint32_t err = *(const uint32_t*)h;
        const float* depth = (const float*)(h + a.off_depth);
        const int32_t* ids = (const int32_t*)(h + a.off_ids);
        const uint8_t* rgb = (const uint8_t*)(h + a.off_rgb);
        const float* st = (const float*)(h + a.off_state);
        int64_t agent = 0;
        for (size_t k = 0; k < items.size(); ++k) {
            Request* r = static_cast<Request*>(items[k]);
            const int64_t px = (int64_t)r->desc.H * r->desc.W * r->desc.n_env, p0 = a.px_off[k];
            if (r->host) {
                r->depth.assign(depth + p0, depth + p0 + px);
                if (s->cfg.want_tri_id) r->tri_id.assign(ids + p0, ids + p0 + px);
                if (s->cfg.want_rgb) r->rgb.assign(rgb + 3 * p0, rgb + 3 * p0 + 3 * px);   // planar per agent
                r->state.assign(st + 17 * agent, st + 17 * (agent + r->desc.n_env));
            }
            agent += r->desc.n_env;
            if (err) r->why = device_error_text(err);
        }
        return err;
    }

    // Put the batch's env slots back to their states before the batch and wait for it.
    bool restore(int i, std::vector<sched::Item*>& items) {
        SlotArena& a = s->arenas[i];
        if (!a.snapshot) return items.empty();
        char* d = (char*)a.dev;
        hipError_t e = hipStreamSynchronize(a.stream);
        if (e == hipSuccess)
            e = launch_scatter_rows(s->state, (const int32_t*)(d + a.off_idx), (int32_t)a.n_agents,
                                    (const float*)(d + a.off_before), a.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
        a.snapshot = false;
        return e == hipSuccess;
    }

    void on_done(sched::Item* it) { static_cast<Request*>(it)->done_at = Clock::now(); }
};

static void worker_loop(vf_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        const bool progressed = s->sched->step();
        if (progressed) s->cv_done.notify_all();
        if (s->sched->any_busy()) {
            // batches in flight: check their events again at once (a timed wait of a few microseconds
            // sleeps for the kernel's timer slack, tens of microseconds, on every batch's latency);
            // the lock is released meanwhile so submitters and waiters get in
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (!progressed) {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace vf

using namespace vf;

extern "C" {

vf_status vf_server_create(vf_ctx* ctx, const vf_server_config* cfg, float* state_table, int64_t n_slots,
                           vf_server** out) {
    if (!ctx || !cfg || !state_table || !out) return fail(VF_EINVAL, "vf_server_create: NULL argument");
    std::string why;
    if (!check_dyn_params(cfg->params, &why)) return fail(VF_EINVAL, "vf_server_create: " + why);
    if (cfg->n_streams < 1 || cfg->n_streams > 16) return fail(VF_EINVAL, "vf_server_create: n_streams in [1, 16]");
    if (cfg->max_h < 1 || cfg->max_w < 1 || cfg->max_h > kMaxImage || cfg->max_w > kMaxImage)
        return fail(VF_EINVAL, "vf_server_create: max_h/max_w in [1, 1024]");
    if (cfg->max_batch_agents < 1 || n_slots < 1) return fail(VF_EINVAL, "vf_server_create: empty batch or table");
    if (cfg->hbm_budget_bytes < 1) return fail(VF_EINVAL, "vf_server_create: hbm_budget_bytes must be > 0");
    VF_HIP(hipSetDevice(ctx->device));
    vf_server* s = new vf_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    s->state = state_table;
    s->n_slots = n_slots;
    s->dyn = make_dyn_const_d(cfg->params);
    int64_t per = cfg->hbm_budget_bytes / cfg->n_streams / 256 * 256;
    s->arenas.resize(cfg->n_streams);
    vf_status st = VF_OK;
    for (auto& a : s->arenas) {
        a.bytes = per;
        st = ctx_alloc(ctx, &a.dev, per);
        if (st != VF_OK) break;
        if (hipHostMalloc(&a.host, per, hipHostMallocDefault) != hipSuccess) {
            a.host = nullptr;
            st = fail(VF_ENOMEM, "vf_server_create: pinned host arena");
            break;
        }
        if (hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&a.event, hipEventDisableTiming) != hipSuccess) {
            st = fail(VF_EHIP, "vf_server_create: stream/event");
            break;
        }
    }
    if (st != VF_OK) {
        for (auto& a : s->arenas) {
            if (a.dev) ctx_free(ctx, a.dev, a.bytes);
            if (a.host) (void)hipHostFree(a.host);
            if (a.event) (void)hipEventDestroy(a.event);
            if (a.stream) (void)hipStreamDestroy(a.stream);
        }
        delete s;
        return st;
    }
    s->backend = new HipBackend{s};
    s->sched = new sched::Scheduler<HipBackend>(*s->backend, cfg->n_streams, per, cfg->max_batch_agents,
                                                kServerMaxAttempts);
    // a host-forced backend error for failure-path runs: the first VF_FAULT_INJECT batches that finish fail
    if (const char* inj = getenv("VF_FAULT_INJECT")) {
        const long long k = atoll(inj);
        if (k > 0) s->sched->inject_faults(k);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return VF_OK;
}

vf_status vf_server_submit(vf_server* s, const vf_request_desc* d, const int32_t* env_slots, const float* actions,
                           const vf_request_out* out, int64_t* ticket) {
    if (!s || !d || !env_slots || !actions || !ticket) return fail(VF_EINVAL, "vf_server_submit: NULL argument");
    if (d->n_env < 1) return fail(VF_EINVAL, "vf_server_submit: n_env must be >= 1");
    if (d->H < 1 || d->W < 1 || d->H > s->cfg.max_h || d->W > s->cfg.max_w)
        return fail(VF_EINVAL, "vf_server_submit: image size outside the server's limits");
    if (!(d->hfov > 0.f && d->hfov < 3.1415926f)) return fail(VF_EINVAL, "vf_server_submit: bad hfov");
    if (!(d->near_clip > 0.f && d->far_clip > d->near_clip))
        return fail(VF_EINVAL, "vf_server_submit: need 0 < near_clip < far_clip");
    if (d->scene_id < 0 || d->scene_id >= (int32_t)s->ctx->scenes.size() || !s->ctx->scenes[d->scene_id].used)
        return fail(VF_ENOSCENE, "vf_server_submit: no such scene");
    const int64_t bytes = request_bytes(s->cfg, *d);
    if (bytes > s->arenas[0].bytes)
        return fail(VF_ENOMEM, "vf_server_submit: request larger than one in-flight batch's share of the budget");
    if (d->n_env > s->cfg.max_batch_agents) return fail(VF_EINVAL, "vf_server_submit: n_env > max_batch_agents");
    std::unordered_set<int32_t> seen;
    for (int32_t e = 0; e < d->n_env; ++e) {
        if (env_slots[e] < 0 || env_slots[e] >= s->n_slots) return fail(VF_EINVAL, "vf_server_submit: env slot out of range");
        if (!seen.insert(env_slots[e]).second) return fail(VF_EINVAL, "vf_server_submit: duplicate env slot");
    }
    Request* r = new Request();
    r->desc = *d;
    if (out) {
        r->out = *out;
        r->host = out->host_results != 0;
    }
    r->slots.assign(env_slots, env_slots + d->n_env);
    r->n_env = d->n_env;
    r->bytes = bytes;
    r->actions.assign(actions, actions + 4 * (int64_t)d->n_env);
    r->arrival = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->sched->submit(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return VF_OK;
}

vf_status vf_server_poll(vf_server* s, int64_t ticket, int32_t* done) {
    if (!s || !done) return fail(VF_EINVAL, "vf_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VF_EINVAL, "vf_server_poll: unknown ticket");
    *done = it->second->done ? 1 : 0;
    return VF_OK;
}

vf_status vf_server_wait(vf_server* s, int64_t ticket, float* depth, int32_t* tri_id, uint8_t* rgb, float* state,
                         double* latency_s) {
    if (!s) return fail(VF_EINVAL, "vf_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VF_EINVAL, "vf_server_wait: unknown ticket");
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(it);
    lk.unlock();
    const vf_status st = (vf_status)r->status;
    if (st == VF_OK && r->host) {
        if (depth) memcpy(depth, r->depth.data(), r->depth.size() * 4);
        if (tri_id && !r->tri_id.empty()) memcpy(tri_id, r->tri_id.data(), r->tri_id.size() * 4);
        if (rgb && !r->rgb.empty()) memcpy(rgb, r->rgb.data(), r->rgb.size());
        if (state) memcpy(state, r->state.data(), r->state.size() * 4);
    }
    if (latency_s) *latency_s = std::chrono::duration<double>(r->done_at - r->arrival).count();
    const std::string why = r->why;
    delete r;
    if (st != VF_OK) return fail(st, "vf_server_wait: batch failed" + (why.empty() ? std::string() : ": " + why));
    return VF_OK;
}

vf_status vf_server_inject_faults(vf_server* s, int64_t n) {
    if (!s || n < 0) return fail(VF_EINVAL, "vf_server_inject_faults: NULL server or negative count");
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched->inject_faults(n);
    return VF_OK;
}

vf_status vf_server_stats_get(vf_server* s, vf_server_stats* out) {
    if (!s || !out) return fail(VF_EINVAL, "vf_server_stats_get: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const sched::Stats& st = s->sched->stats();
    out->batches = st.batches;
    out->agents = st.agents;
    out->requests = st.requests;
    out->max_batch_agents = st.max_batch;
    out->pending = (int64_t)s->sched->pending();
    out->in_flight_batches = s->sched->in_flight();
    out->requeued = st.requeued;
    out->failed_batches = st.failed_batches;
    return VF_OK;
}

vf_status vf_server_destroy(vf_server* s) {
    if (!s) return fail(VF_EINVAL, "vf_server_destroy: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->sched->pending() > 0) return fail(VF_EBUSY, "vf_server_destroy: requests still pending");
    }
    s->stop.store(true);
    s->cv_work.notify_all();
    s->worker.join();
    for (auto& a : s->arenas)
        if (a.stream) (void)hipStreamSynchronize(a.stream);
    for (auto& a : s->sched->arenas())
        for (sched::Item* it : a.items) delete static_cast<Request*>(it);
    for (auto& a : s->arenas) {
        ctx_free(s->ctx, a.dev, a.bytes);
        (void)hipHostFree(a.host);
        (void)hipEventDestroy(a.event);
        (void)hipStreamDestroy(a.stream);
    }
    for (auto& kv : s->all) {
        bool in_arena = false;
        for (auto& a : s->sched->arenas())
            for (sched::Item* it : a.items) in_arena |= it == kv.second;
        if (!in_arena) delete kv.second;
    }
    delete s->sched;
    delete s->backend;
    delete s;
    return VF_OK;
}

}  // extern "C"
