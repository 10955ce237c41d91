/*
 * visfly.h -- C ABI of the MI355X (gfx950) batched quadrotor step + ray-cast renderer.
 *
 * The library advances N quadrotors by one control step (Sec. III-A: Eq. (1)
 * rigid body, Eq. (2) drag, Eq. (3) thrust and moment, Eq. (4) rotor lag, the
 * CTBR / SRT controllers, RK4 or Euler with sub-steps) and renders each agent's
 * onboard depth / triangle-id / flat-colour view (Sec. III-B) of a triangle
 * mesh by ray casting through a BVH that is built on the device.  Agents are
 * independent (Sec. III-B: parallel agents ignore each other) and may sit in
 * different scenes and use different resolutions in one call (Sec. III-D:
 * several scenes at once; Fig. 4: 64x64 up to 256x256).
 *
 * Conventions shared by every call
 *  - Pointers marked [dev] are device pointers on the context's GPU, owned by
 *    the caller; the library never frees them.  Pointers marked [host] are read
 *    before the call returns.  Scenes, BVHs and internal scratch are owned by
 *    the context and charged against its HBM budget.
 *  - Every call that takes a `stream` (a hipStream_t, NULL = default stream)
 *    only enqueues work and returns after argument validation; results are
 *    ready when the stream reaches that point.  Data-dependent faults found by
 *    the kernels (bad scene id, out-of-range slot or pixel offset, traversal
 *    stack overflow) never write out of bounds: the affected agent is skipped
 *    and a sticky device error word is set; vf_sync_check() reports it.
 *  - Status codes only, never abort; vf_last_error() gives a text message for
 *    the last failing call on the calling thread.
 *  - State row (17 float32): p[3] world position (m), q[4] unit quaternion
 *    (w,x,y,z) body->world (Hamilton), v[3] world velocity (m/s), Omega[3] body
 *    rates (rad/s), w[4] normalised rotor speeds (rotor i thrust = w_i^2, N).
 *    World z is up; body x forward, y left, z up.
 *  - Action row (4 float32): CTBR = (collective acceleration m/s^2, body-rate
 *    command x,y,z rad/s); SRT = four rotor thrusts (N).
 *  - Camera: at the body origin looking along +x_B, image right = -y_B, image up
 *    = +z_B.  Pixel (r, c) casts d = R(q) (1, -u_c, v_r) with
 *    u_c = (2(c+1/2)/W - 1) tan(hfov/2), v_r = (1 - 2(r+1/2)/H) tan(hfov/2) H/W,
 *    so the hit distance t is the planar depth.  Closest hit in [near, far],
 *    double-sided triangles, ties to the lower original triangle index; a miss
 *    gives depth = miss_depth, tri_id = -1, rgb = 0.
 *  - Outputs of agent i start at views[i].out_offset: depth and tri_id are
 *    [H][W] row-major there; rgb is planar [3][H][W] starting at
 *    3 * out_offset.  Every written pixel must lie below out_pixels.
 */
#ifndef VISFLY_H
#define VISFLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vf_status {
    VF_OK = 0,
    VF_EINVAL = -1,    /* malformed argument (null pointer, negative size, bad enum) */
    VF_ENOMEM = -2,    /* HBM budget of the context or device memory exhausted */
    VF_ENOSCENE = -3,  /* scene id not built or already freed */
    VF_EHIP = -4,      /* HIP runtime error or a kernel fault reported by the runtime */
    VF_EBUSY = -5,     /* the object is in use (e.g. a server still holds requests) */
    VF_EDEVICE = -6    /* a kernel flagged bad data (see vf_sync_check) */
} vf_status;

enum { VF_RK4 = 0, VF_EULER = 1 };
enum { VF_CTBR = 0, VF_SRT = 1 };

typedef struct vf_ctx vf_ctx; /* opaque; owned by the library */

/* Airframe, controller and integrator parameters (Sec. III-A). 88 bytes. */
typedef struct vf_dyn_params {
    float dt;            /* control step (s) */
    int32_t n_sub;       /* sub-steps per control step, >= 1; the controller runs every sub-step */
    int32_t integrator;  /* VF_RK4 or VF_EULER */
    int32_t ctrl;        /* VF_CTBR or VF_SRT */
    float mass;          /* kg */
    float arm;           /* rotor distance from the centre (m); X frame at +-45 deg */
    float J[3];          /* diagonal inertia (kg m^2) */
    float tau_motor;     /* rotor time constant (s) of Eq. (4) */
    float kappa_yaw;     /* rotor reaction torque per newton of thrust (m) */
    float f_max;         /* per-rotor thrust limit (N) */
    float k_lin[3];      /* linear body-frame drag (N s/m) of Eq. (2) */
    float c_quad[3];     /* quadratic body-frame drag (N s^2/m^2) of Eq. (2) */
    float g;             /* gravity (m/s^2), along -z */
    float k_rate[3];     /* CTBR body-rate gains (1/s) */
} vf_dyn_params;

/* Per-agent camera/output descriptor. 40 bytes, 8-byte aligned. */
typedef struct vf_view {
    int32_t scene_id;    /* scene the agent flies in */
    int32_t H, W;        /* image size, 1..1024 each */
    int32_t flags;       /* reserved, must be 0 */
    float hfov;          /* horizontal field of view (rad), (0, pi) */
    float near_clip;     /* hits closer than this are ignored (m) */
    float far_clip;      /* hits farther than this are ignored (m) */
    float miss_depth;    /* depth written where nothing is hit */
    int64_t out_offset;  /* first output pixel of this agent */
} vf_view;

/* Summary of a built scene. */
typedef struct vf_scene_info {
    int64_t n_tris;       /* triangles */
    int64_t n_nodes;      /* 4-wide BVH nodes */
    int64_t n_leaves;     /* leaf slots */
    int64_t bytes;        /* device bytes held (nodes + triangles + colours + index map) */
    int32_t depth;        /* BVH depth in 4-wide nodes (root = 1) */
    int32_t leaf_max;     /* maximum triangles per leaf */
    float bounds_lo[3];   /* scene bounds */
    float bounds_hi[3];
    float build_ms;       /* device time of the build (ms) */
    int32_t pad;
} vf_scene_info;

/* 4-wide BVH node as stored in HBM (128 bytes; for vf_scene_export).
 * child[k] >= 0: index of an inner node; child[k] < 0: leaf holding count[k]
 * triangles starting at sorted position first = -child[k] - 1; count[k] == 0
 * with child[k] < 0 marks an empty slot.  order_lo/order_hi hold, for each of
 * the 8 ray-direction octants o (bit 0: x<0, bit 1: y<0, bit 2: z<0), a byte of
 * four 2-bit child slots in near-to-far order (octant o at bits 8*o..8*o+7 of
 * the 64-bit value order_hi:order_lo). */
typedef struct vf_bvh4_node {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    int32_t child[4];
    uint8_t count[4];
    uint32_t order_lo, order_hi;
    uint32_t pad;
} vf_bvh4_node;

/* Leaf triangle as stored in HBM (48 bytes): v0 and the two edges in float32,
 * and the caller's triangle index (bit pattern in v0w). */
typedef struct vf_tri {
    float v0x, v0y, v0z; int32_t id;
    float e1x, e1y, e1z, pad1;
    float e2x, e2y, e2z, pad2;
} vf_tri;

/* Create a context on HIP device `device`; hbm_budget_bytes caps what the
 * library itself allocates (scenes + scratch); 0 = no cap. */
vf_status vf_create(int device, size_t hbm_budget_bytes, vf_ctx** out);

/* Destroy a context: frees its scenes and scratch; waits for its work. */
vf_status vf_destroy(vf_ctx* ctx);

/* Build a scene (Sec. III-B: triangle-mesh scenes) on the device: per-triangle
 * bounds and centroids, 30-bit Morton codes, a stable LSD radix sort, the
 * binary radix tree of Karras (HPG 2012), collapse to a 4-wide BVH, bottom-up
 * bounds and per-octant child orders.  verts [V][3] float32 [dev], tris [T][3]
 * int32 [dev] (indices must be in [0, V); checked on the device, VF_EINVAL if
 * violated), tri_rgb [T][3] uint8 [dev] or NULL (grey).  The inputs are copied;
 * the caller may free them after the call returns.  Synchronous: returns when
 * the scene is ready.  1 <= T < 2^27. */
vf_status vf_scene_build(vf_ctx* ctx, const float* verts, int64_t V, const int32_t* tris, int64_t T,
                         const uint8_t* tri_rgb, void* stream, int32_t* scene_id);

/* Release a scene; its id may be reused by a later build.  The caller must not
 * have work in flight that uses it. */
vf_status vf_scene_free(vf_ctx* ctx, int32_t scene_id);

/* Counts, bytes and bounds of a scene. */
vf_status vf_scene_info_get(vf_ctx* ctx, int32_t scene_id, vf_scene_info* out);

/* Copy a scene's BVH nodes (vf_bvh4_node[n_nodes]) and leaf triangles
 * (vf_tri[n_tris], sorted leaf order) to host buffers (either may be NULL);
 * capacities in bytes.  Synchronous.  For inspection and tests. */
vf_status vf_scene_export(vf_ctx* ctx, int32_t scene_id, void* nodes_host, int64_t nodes_cap,
                          void* tris_host, int64_t tris_cap);

/* One control step for n agents, then (if views != NULL) render each agent at
 * its new state -- the Gym step order of Sec. III-C (act, then observe).
 * env_idx [n] int32 [dev] or NULL (identity): agent i updates state row
 * env_idx[i] of state [n_slots][17] float32 [dev, in/out, updated in place].
 * action [n][4] float32 [dev].  views [n] [dev] or NULL (dynamics only).
 * max_h/max_w bound every views[i].H/W (agents beyond them are rejected on the
 * device).  depth [dev] float32, tri_id [dev] int32, rgb [dev] uint8: each may
 * be NULL to skip that output; out_pixels = pixel capacity of depth/tri_id.
 * With views the render follows the step on the same stream (see
 * vf_set_launch_mode for the single-launch fused form). */
vf_status vf_step(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx,
                  float* state, int64_t n_slots, const float* action,
                  const vf_view* views, int32_t max_h, int32_t max_w,
                  float* depth, int32_t* tri_id, uint8_t* rgb, int64_t out_pixels, void* stream);

/* Render only (the second half of vf_step) at the given states. */
vf_status vf_render(vf_ctx* ctx, int64_t n, const int32_t* env_idx, const float* state, int64_t n_slots,
                    const vf_view* views, int32_t max_h, int32_t max_w,
                    float* depth, int32_t* tri_id, uint8_t* rgb, int64_t out_pixels, void* stream);

/* Vector-Jacobian product of one vf_step (dynamics part) for n agents
 * (differentiable dynamics, Sec. III-A): given the saved state_in s_k [n][17],
 * action a_k [n][4] and grad_state_out = dL/ds_{k+1} [n][17], writes
 * grad_state_in = (ds_{k+1}/ds_k)^T grad_state_out [n][17] and grad_action =
 * (ds_{k+1}/da_k)^T grad_state_out [n][4] (both overwritten).  The forward
 * sub-steps are recomputed from state_in.  Clamped rotor commands pass no
 * gradient; the square root of a zero rotor command passes none either. */
vf_status vf_step_backward(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const float* state_in,
                           const float* action, const float* grad_state_out, float* grad_state_in,
                           float* grad_action, void* stream);

/* Vector-Jacobian product of the depth image with respect to camera pose: for
 * every pixel that hit triangle tri_id (the saved forward ids, caller's
 * indices), depth t = n.(V0 - o) / n.d on that triangle's plane, so
 * dt/do = -n / n.d and dt/dd = -t n / n.d, chained through d = R(q/|q|) d_B.
 * Adds sum_pixels grad_depth * dt/d(p, q) to grad_state[i][0:7] (rows of the
 * agents, compact [n][17]); misses contribute nothing.  Deterministic (fixed
 * reduction order). */
vf_status vf_render_backward(vf_ctx* ctx, int64_t n, const float* state, const vf_view* views,
                             int32_t max_h, int32_t max_w, const int32_t* tri_id, const float* grad_depth,
                             int64_t out_pixels, float* grad_state, void* stream);

/* Nearest obstacle point (Sec. III-B: the spatial distance module that reports the
 * relative position of the nearest obstacle point without a collision having to
 * happen).  For each query point p_i [n][3] float32 [dev] in scene scene_ids[i]
 * (int32 [dev]) or, if scene_ids is NULL, in scene_id0: the Euclidean distance
 * to the closest point of any triangle, dist [n] float32 [dev, out], that point
 * closest [n][3] float32 [dev, out, nullable] and its caller triangle index
 * tri_id [n] int32 [dev, out, nullable].  Points farther than max_dist from every
 * triangle give dist = +inf, tri_id = -1.  Equal distances go to the lower index. */
vf_status vf_closest_point(vf_ctx* ctx, int64_t n, const float* points, const int32_t* scene_ids, int32_t scene_id0,
                           float max_dist, float* dist, float* closest, int32_t* tri_id, void* stream);

/* How vf_step with views launches its work.  VF_LAUNCH_SPLIT: a dynamics
 * kernel (one thread per agent) then the render kernel, two launches on the
 * stream.  VF_LAUNCH_FUSED: one kernel in which every render workgroup advances
 * its agent's dynamics in one lane and the last workgroup of the agent to finish
 * writes the new state.  Both give bitwise identical states and images.  The
 * split form keeps the render kernel at its lower register count and is faster
 * for batches that fill the GPU; the fused form saves a launch and wins for
 * small, latency-bound batches.  VF_LAUNCH_AUTO (the default) picks fused when
 * the render grid has at most 1,024 workgroups (16 agents at 64x64), else split. */
enum { VF_LAUNCH_SPLIT = 0, VF_LAUNCH_FUSED = 1, VF_LAUNCH_AUTO = 2 };
vf_status vf_set_launch_mode(vf_ctx* ctx, int32_t mode);

/* Enable (1) / disable (0) traversal statistics: while enabled, vf_step and
 * vf_render use a counting variant of the render kernel that accumulates node
 * visits, box tests, triangle tests and rays into the context's counters. */
vf_status vf_set_stats(vf_ctx* ctx, int32_t enable);

/* Read (and optionally reset) the counters: out[0] rays, out[1] inner-node
 * visits per lane, out[2] ray-box tests, out[3] ray-triangle tests,
 * out[4] wave-level node visits, out[5] wave-level triangle loads,
 * out[6] active-lane box tests, out[7] hits.  Synchronises the device. */
vf_status vf_stats_read(vf_ctx* ctx, uint64_t out[8], int32_t reset);

/* Wait for `stream`, then report (and clear) the sticky device error word:
 * VF_OK, or VF_EDEVICE with the reason in vf_last_error(). */
vf_status vf_sync_check(vf_ctx* ctx, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching request loop over resident env slots.
 * A request is one step + render of n_env envs of one scene at one image size.
 * The server keeps drone states resident in the caller's state table, copies a
 * request's host inputs on submit, and a worker thread admits pending requests
 * in arrival order into batches as stream slots and arena memory free up:
 * n_streams batches may be in flight at once (they overlap on the GPU), each in
 * a device arena of hbm_budget_bytes / n_streams (charged to the context).  A
 * request that does not fit the arena blocks those behind it (no starvation);
 * a request touching an env slot that an in-flight or earlier queued request
 * touches waits for it, so each env sees its requests in submission order.
 * Results (depth, optional ids / colours, new states) come back to host memory;
 * latency is measured from submit to the completion of the batch.  Agents are
 * independent, so a request's result does not depend on the batch it joins.
 * ------------------------------------------------------------------------- */
typedef struct vf_server vf_server; /* opaque */

typedef struct vf_server_config {
    vf_dyn_params params;      /* dynamics of every request */
    int32_t n_streams;         /* batches in flight at once, 1..16 */
    int32_t max_batch_agents;  /* agents per batch */
    int32_t max_h, max_w;      /* largest image a request may ask for */
    int32_t want_tri_id;       /* 1: return hit triangle ids */
    int32_t want_rgb;          /* 1: return planar colour */
    int64_t hbm_budget_bytes;  /* device memory for in-flight batches (work lists + outputs) */
} vf_server_config;

typedef struct vf_request_desc {
    int32_t scene_id, H, W, n_env;
    float hfov, near_clip, far_clip, miss_depth;
} vf_request_desc;

/* Where a request's results go.  Device buffers (any may be NULL) receive them by
 * device-to-device copies on the batch's stream before the request completes:
 * depth [n_env][H][W] float32, tri_id [n_env][H][W] int32 (needs want_tri_id),
 * rgb [n_env][3][H][W] uint8 (needs want_rgb), state [n_env][17] float32.
 * host_results = 1 also keeps host copies for vf_server_wait. */
typedef struct vf_request_out {
    float* depth;
    int32_t* tri_id;
    uint8_t* rgb;
    float* state;
    int32_t host_results;
    int32_t pad;
} vf_request_out;

typedef struct vf_server_stats {
    int64_t batches, agents, requests, max_batch_agents, pending, in_flight_batches;
} vf_server_stats;

/* state_table [n_slots][17] float32 [dev]: resident env states, updated in place. */
vf_status vf_server_create(vf_ctx* ctx, const vf_server_config* cfg, float* state_table, int64_t n_slots,
                           vf_server** out);
/* env_slots [n_env] int32 [host], distinct, in [0, n_slots); actions [n_env][4] float32 [host];
 * out [host] or NULL (= host results only).  Returns at once with a ticket; VF_ENOSCENE /
 * VF_EINVAL / VF_ENOMEM (larger than one arena).  Device output buffers must stay valid until
 * the request completes. */
vf_status vf_server_submit(vf_server* s, const vf_request_desc* d, const int32_t* env_slots, const float* actions,
                           const vf_request_out* out, int64_t* ticket);
/* done = 1 once the ticket's batch has completed. */
vf_status vf_server_poll(vf_server* s, int64_t ticket, int32_t* done);
/* Block until done, copy the host results (if the request kept them) to host buffers (depth
 * [n_env][H][W]; tri_id likewise; rgb per env planar [3][H][W]; state [n_env][17]; any may be NULL)
 * and release the ticket; latency_s = completion - submission (s). */
vf_status vf_server_wait(vf_server* s, int64_t ticket, float* depth, int32_t* tri_id, uint8_t* rgb, float* state,
                         double* latency_s);
vf_status vf_server_stats_get(vf_server* s, vf_server_stats* out);
/* VF_EBUSY while requests are pending; in-flight batches are drained. */
vf_status vf_server_destroy(vf_server* s);

/* Bytes the context currently holds, and its budget (0 = none). */
vf_status vf_mem_usage(vf_ctx* ctx, int64_t* used_bytes, int64_t* budget_bytes);

/* Text of the last error on the calling thread ("" if none). */
const char* vf_last_error(vf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* VISFLY_H */
