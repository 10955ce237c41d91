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
enum { VF_CTBR = 0, VF_SRT = 1, VF_PS = 2, VF_LV = 3 };

typedef struct vf_ctx vf_ctx; /* opaque; owned by the library */

/* Airframe, controller and integrator parameters (Sec. III-A). 128 bytes.
 * Controllers (controller paragraph of Sec. III-A):
 *   VF_CTBR  action (c m/s^2, Omega_des rad/s): tau = J k_rate (Omega_des - Omega) + Omega x J Omega, F = m c
 *   VF_SRT   action = four rotor thrusts (N)
 *   VF_PS    action (x_d, y_d, z_d m, yaw_d rad): a = -k_pos (p - p_d) - k_vel v
 *   VF_LV    action (vx_d, vy_d, vz_d m/s, yaw_d rad): a = -k_vel (v - v_d)
 * PS and LV are geometric (SE(3)) outer loops cascaded onto the CTBR rate loop: F = a + g e_z with its
 * vertical part at least g/4 and its tilt at most max_tilt; R_d from F/|F| and the yaw heading;
 * c = F . R e_z; Omega_des = -k_att e_R with e_R = 1/2 (R_d^T R - R^T R_d)^vee.
 * Every controller's rotor thrusts are clamped to [0, f_max]. */
typedef struct vf_dyn_params {
    float dt;            /* control step (s) */
    int32_t n_sub;       /* sub-steps per control step, >= 1; the controller runs every sub-step */
    int32_t integrator;  /* VF_RK4 or VF_EULER */
    int32_t ctrl;        /* VF_CTBR, VF_SRT, VF_PS or VF_LV */
    float mass;          /* kg */
    float arm;           /* rotor distance from the centre (m); X frame at +-45 deg */
    float J[3];          /* diagonal inertia (kg m^2) */
    float tau_motor;     /* rotor time constant (s) of Eq. (4) */
    float kappa_yaw;     /* rotor reaction torque per newton of thrust (m) */
    float f_max;         /* per-rotor thrust limit (N) */
    float k_lin[3];      /* linear body-frame drag (N s/m) of Eq. (2) */
    float c_quad[3];     /* quadratic body-frame drag (N s^2/m^2) of Eq. (2) */
    float g;             /* gravity (m/s^2), along -z */
    float k_rate[3];     /* body-rate gains (1/s) of the rate loop */
    float k_pos[3];      /* PS position gains (1/s^2) */
    float k_vel[3];      /* PS / LV velocity gains (1/s) */
    float k_att[3];      /* PS / LV attitude gains (1/s) */
    float max_tilt;      /* PS / LV tilt limit of the commanded thrust (rad), in (0, pi/2) */
} vf_dyn_params;

/* Per-view camera/output descriptor. 72 bytes, 8-byte aligned.
 * The camera frame has its optical axis along +x, image right along -y and image up along +z (the
 * body frame's convention); mount_q rotates it into the body frame and mount_t places its centre, so a
 * ray leaves p + R(q) mount_t along R(q) R(mount_q) (1, -u, v).  A quaternion with x = y = z = 0 (the
 * all-zero default included) means no rotation.  Several views of one agent (a camera rig) are views
 * whose env_idx entries name the same state slot (vf_render). */
typedef struct vf_view {
    int32_t scene_id;    /* scene the agent flies in */
    int32_t H, W;        /* image size, 1..1024 each */
    int32_t flags;       /* the agent's sensor-noise key (vf_sensor_noise); ignored by the renderer */
    float hfov;          /* horizontal field of view (rad), (0, pi) */
    float near_clip;     /* hits closer than this are ignored (m); must be > 0 */
    float far_clip;      /* hits farther than this are ignored (m); must be > near_clip */
    float miss_depth;    /* depth written where nothing is hit */
    int64_t out_offset;  /* first output pixel of this view */
    float mount_q[4];    /* camera orientation in the body frame (w, x, y, z) */
    float mount_t[3];    /* camera position in the body frame (m) */
    int32_t swarm;       /* 0: none; k > 0: the agent flies in swarm k - 1 (vf_set_swarms) and sees its members */
} vf_view;

/* Summary of a built scene. */
typedef struct vf_scene_info {
    int64_t n_tris;       /* triangles */
    int64_t n_nodes;      /* BVH nodes */
    int64_t n_leaves;     /* leaf slots */
    int64_t bytes;        /* device bytes held (nodes + triangles + colours + index map) */
    int32_t depth;        /* BVH depth in nodes (root = 1) */
    int32_t leaf_max;     /* maximum triangles per leaf */
    float bounds_lo[3];   /* scene bounds */
    float bounds_hi[3];
    float build_ms;       /* device time of the build (ms) */
    int32_t width;        /* children per node: 4 (vf_bvh4_node) or 8 (vf_bvh8_node) */
    int32_t builder;      /* binary tree the BVH was collapsed from: VF_BVH_CLUSTER or VF_BVH_RADIX */
    int32_t reserved;
} vf_scene_info;

/* BVH node as stored in HBM (for vf_scene_export); vf_scene_info.width says which
 * layout the library uses.  child[k] >= 0: index of an inner node; child[k] ==
 * INT32_MIN: empty slot, whose box is [FLT_MAX, FLT_MAX]^3; otherwise a leaf of
 * ((-child[k] - 1) & 7) + 1 triangles starting at sorted position
 * (-child[k] - 1) >> 3 (the traversal's stack entry itself).  The orders give,
 * for each of the 8 ray-direction octants o (bit 0: x<0, bit 1: y<0, bit 2:
 * z<0), the child slots in near-to-far order.
 * 4-wide (128 bytes): count[k] is the leaf's triangle count (0 otherwise);
 * octant o's four 2-bit slots are byte o of the 64-bit order[1]:order[0]. */
typedef struct vf_bvh4_node {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    int32_t child[4];
    uint8_t count[4];
    uint32_t order[3];   /* order[2] = 0 */
} vf_bvh4_node;

/* 8-wide (256 bytes): octant o's eight 3-bit slots are the low 24 bits of order[o]. */
typedef struct vf_bvh8_node {
    float lo_x[8], hi_x[8], lo_y[8], hi_y[8], lo_z[8], hi_z[8];
    int32_t child[8];
    uint32_t order[8];
} vf_bvh8_node;

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
 * bounds and centroids, 30-bit Morton codes (one scale for the three axes), a
 * stable LSD radix sort, a binary tree by locally-ordered clustering of the
 * sorted triangles (or the Morton radix tree; see vf_set_bvh_builder), collapse
 * to a 4-wide BVH with leaves of at most vf_set_bvh_leaf_size triangles,
 * bottom-up bounds and per-octant child orders.  verts [V][3] float32 [dev], tris [T][3]
 * int32 [dev] (indices must be in [0, V) and the vertices they use finite;
 * checked on the device, VF_EINVAL if violated), tri_rgb [T][3] uint8 [dev] or NULL (grey).  The inputs are copied;
 * the caller may free them after the call returns.  Synchronous: returns when
 * the scene is ready.  1 <= T < 2^27. */
vf_status vf_scene_build(vf_ctx* ctx, const float* verts, int64_t V, const int32_t* tris, int64_t T,
                         const uint8_t* tri_rgb, void* stream, int32_t* scene_id);

/* Release a scene; its id may be reused by a later build.  The caller must not
 * have work in flight that uses it. */
vf_status vf_scene_free(vf_ctx* ctx, int32_t scene_id);

/* Counts, bytes and bounds of a scene. */
vf_status vf_scene_info_get(vf_ctx* ctx, int32_t scene_id, vf_scene_info* out);

/* Copy a scene's BVH nodes (vf_bvh4_node or vf_bvh8_node [n_nodes]) and leaf triangles
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

/* Allocation-free form of vf_step, for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, semantics and results
 * as vf_step (bit for bit: the same kernels).  It allocates nothing and calls no allocating routine: its
 * scratch -- the fused launch's arrival counters (one per state slot) and the cost order's per-workgroup
 * work and workgroup order -- lives in a file-scope device array of 3 MiB, one copy per GPU, held until
 * the process ends; vf_create looks up its address once per device.  Limits: a fused launch (small
 * batches, or VF_LAUNCH_FUSED) takes at most 262,144 state slots (n_slots), else VF_EINVAL; the cost
 * order covers split launches of 1,024 .. 262,144 workgroups, larger ones keep the plain order; no
 * spatial order and no timing events; swarm mode is refused (VF_EINVAL: its member trees are allocated
 * per stream).  Every call on a GPU shares that GPU's array and leaves its contents for the next call
 * (the arrival counters are cleared by a fill kernel at each fused call; work estimates from another
 * call only change the workgroup order, never a result): calls that overlap on one GPU race. */
vf_status vf_step_noalloc(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx, float* state,
                          int64_t n_slots, const float* action, const vf_view* views, int32_t max_h, int32_t max_w,
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
 * gradient; the square root of a zero rotor command passes none either.
 * Every controller: VF_CTBR and VF_SRT by a hand-written reverse mode, VF_PS
 * and VF_LV by forward mode (one dual-number pass per input coordinate, 21
 * per agent), where the outer loop's lift and tilt limits pass the gradient
 * of the side the forward took. */
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

/* Collision check of agents (the same distance module, used to end an episode on
 * contact): for agent i at state slot env_idx[i] (identity if NULL) of state
 * [n_slots][17] float32 [dev], in scene views[i].scene_id: dist [n] float32 [dev,
 * out] to the nearest triangle (+inf beyond max_dist), rel [n][3] float32 [dev,
 * out, nullable] = nearest point - position (0 when none within max_dist), and
 * collided [n] uint8 [dev, out, nullable] = dist <= radius.  Bad slots or scenes
 * give +inf / 0 and raise VF_EDEVICE at the next vf_sync_check. */
vf_status vf_collision(vf_ctx* ctx, int64_t n, const int32_t* env_idx, const float* state, int64_t n_slots,
                       const vf_view* views, float radius, float max_dist, float* dist, float* rel,
                       uint8_t* collided, void* stream);

/* ---------------------------------------------------------------------------
 * Sensor extensions (Table I sensors; Sec. III-D Table II noise models).
 * Noise draws come from Philox4x32-10 keyed by (seed, views[i].flags, pixel,
 * stream): deterministic and independent of batch composition.
 * ------------------------------------------------------------------------- */
enum { VF_NOISE_NONE = 0, VF_NOISE_NORMAL = 1, VF_NOISE_SPECKLE = 2, VF_NOISE_SALT_PEPPER = 3, VF_NOISE_POISSON = 4 };

/* Noise of the three image sensors (Table II names Normal, speckle, Poisson and salt & pepper noise;
 * its parameters are not in the paper, so every model takes its own).  Misses keep their depth;
 * colour noise acts on every pixel; label noise acts on labelled pixels (label >= 0). 64 bytes. */
typedef struct vf_noise {
    int32_t depth_model;  /* NORMAL D + s n; SPECKLE D (1 + s n); SALT_PEPPER p/2 -> far, p/2 -> near;
                             POISSON P(D c) / c, drawn in FP64 and rounded to float32 once */
    float depth_sigma;    /* s (m for NORMAL, relative for SPECKLE), >= 0 */
    float depth_p;        /* salt & pepper probability in [0, 1] */
    float depth_scale;    /* c, Poisson counts per metre, > 0 when POISSON */
    int32_t rgb_model;    /* per channel, rounded half up and clamped to [0, 255]: NORMAL v + s n,
                             SPECKLE v (1 + s n), POISSON P(v c) / c; SALT_PEPPER sets the pixel to 255 / 0 */
    float rgb_sigma;      /* in 0..255 units for NORMAL */
    float rgb_p;
    float rgb_scale;      /* c, Poisson counts per colour level */
    int32_t seg_model;    /* labels: NORMAL l + floor(s n + 1/2); SPECKLE floor(l (1 + s n) + 1/2);
                             POISSON floor(P(l c) / c + 1/2); SALT_PEPPER p/2 -> seg_salt_label, p/2 -> -1 */
    float seg_sigma;
    float seg_p;
    float seg_scale;      /* c, Poisson counts per label unit */
    int32_t seg_salt_label;
    int32_t reserved;     /* must be 0 */
    uint64_t seed;
} vf_noise;

/* Apply noise in place to rendered depth, planar rgb and segmentation labels [dev, each nullable] of
 * n agents laid out by views [n] [dev] (Sec. III-D, Table II).  tri_id [dev, nullable]: misses (id -1)
 * keep their depth; without ids every depth pixel is perturbed.  Draws are keyed by (seed,
 * views[i].flags, pixel, stream), so an agent's noise does not depend on the batch.  Bad models or
 * parameters -> VF_EINVAL; bad views raise VF_EDEVICE at the next vf_sync_check. */
vf_status vf_sensor_noise(vf_ctx* ctx, int64_t n, const vf_view* views, int32_t max_h, int32_t max_w,
                          const vf_noise* noise, const int32_t* tri_id, float* depth, uint8_t* rgb, int32_t* seg,
                          int64_t out_pixels, void* stream);

/* The same depth and colour noise applied by the render kernel itself, before its writes, in every
 * later vf_step / vf_render of this context (a fused epilogue: no second pass over the images).  The
 * result equals vf_render followed by vf_sensor_noise with the same configuration, bit for bit.
 * noise is copied; NULL (or models NONE) turns it off.  The label fields are ignored (labels are not
 * a render output).  The server's batches are not affected. */
vf_status vf_set_render_noise(vf_ctx* ctx, const vf_noise* noise);

/* Per-triangle semantic labels of a scene ([T] int32 [dev], copied; NULL removes them). */
vf_status vf_scene_set_labels(vf_ctx* ctx, int32_t scene_id, const int32_t* labels);

/* Segmentation view: seg[p] = label of the hit triangle tri_id[p] (the triangle index itself if the
 * scene has no labels), -1 on a miss, -2 - j on swarm member j; same layout as depth. */
vf_status vf_segmentation(vf_ctx* ctx, int64_t n, const vf_view* views, int32_t max_h, int32_t max_w,
                          const int32_t* tri_id, int32_t* seg, int64_t out_pixels, void* stream);

/* IMU at the given states: out [n][6] = specific force (F_b + d) / m in the body frame (m/s^2) and
 * body rates (rad/s), plus Normal noise of the given sigmas keyed by keys[i] (int32 [dev], NULL =
 * agent index) and seed. */
vf_status vf_imu(vf_ctx* ctx, const vf_dyn_params* params, int64_t n, const int32_t* env_idx, const float* state,
                 int64_t n_slots, float sigma_acc, float sigma_gyro, uint64_t seed, const int32_t* keys, float* out,
                 void* stream);

/* ---------------------------------------------------------------------------
 * Swarm mode (the swarm example of Sec. IV: agents see and avoid each other).
 * Renders find the members through a top-level tree per swarm, rebuilt from the states before every
 * vf_step / vf_render that shows swarms (members in Morton order, four to a leaf, an implicit 4-wide
 * tree of their world-axis boxes; one tree buffer per stream).  At most 4,096 members per swarm.
 * Swarm s has the state slots slots[offsets[s] .. offsets[s + 1]) (host arrays, copied; the slots index
 * the state array of the later calls).  A view with swarm = s + 1 renders the other members of swarm s
 * as boxes of half sizes half_extent centred on their positions and turned with their attitude, in the
 * flat colour rgb: member j (its position in the list) has id n_tris + j of the view's scene, and a
 * member at the same depth as a triangle leaves the triangle.  Members are read at the state the render
 * sees, so vf_step launches split (dynamics first) while swarms are set.  vf_collision reports for swarm
 * views the smaller of the mesh distance and the distance to the nearest other member's bounding sphere
 * (radius |half_extent|).  Member pixels pass no gradient in vf_render_backward.  n_swarms = 0 clears.
 * ------------------------------------------------------------------------- */
vf_status vf_set_swarms(vf_ctx* ctx, int32_t n_swarms, const int32_t* offsets, const int32_t* slots,
                        const float half_extent[3], const uint8_t rgb[3]);

/* Render order of split launches (vf_step split form, vf_render): with enable != 0 (the default) a
 * batch of 64 .. 512 agents is first sorted by (scene id, 2-D Morton code of position) in one small
 * kernel, so that the agents one XCD renders share a scene region and its L2 holds the part of the BVH
 * they touch (larger batches, and the server's batches, are not ordered: there the ordering kernel
 * costs more than it saves; nor are launches put in cost order, see vf_set_cost_order).  The order
 * changes which workgroup renders an agent, never the results. */
vf_status vf_set_spatial_order(vf_ctx* ctx, int32_t enable);

/* Workgroup order of split launches of 1,024 .. 262,144 packets (vf_step split form, vf_render): with
 * enable != 0 (the default) each render records the traversal work of every packet in per-stream scratch,
 * and the next launch on that stream with the same number of views and packets per view first runs one
 * small kernel that puts each XCD's workgroups in decreasing order of that work (in chunks of 16,384), so
 * the longest packets start first instead of running alone at the end of the launch.  The first launch
 * of a shape keeps the plain order.  The scratch (about 2 MB per stream, charged to the context's budget)
 * is allocated on a stream's first ordered launch and freed by vf_destroy; without memory for it the
 * launch keeps the plain order.  The order changes which workgroup renders a packet, never the results.
 * Returns VF_EINVAL for a NULL context. */
vf_status vf_set_cost_order(vf_ctx* ctx, int32_t enable);

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

/* Binary tree that later scene builds collapse into the wide BVH.
 * VF_BVH_CLUSTER (the default): locally-ordered clustering (PLOC, Meister and
 * Bittner 2018) of the triangles in Morton order, radius 6.  VF_BVH_RADIX: the
 * Morton radix tree (Karras 2012), about half the build time.  A clustered tree
 * too deep for the traversal stack is replaced by the radix tree;
 * vf_scene_info.builder reports which one a scene got.  Both give identical
 * images (up to exact depth ties, broken by the lower triangle id either way). */
enum { VF_BVH_CLUSTER = 0, VF_BVH_RADIX = 1 };
vf_status vf_set_bvh_builder(vf_ctx* ctx, int32_t builder);

/* Largest number of triangles in a BVH leaf for later scene builds, 1..4 (the
 * default 4; vf_scene_info.leaf_max reports a scene's).  Subtrees of at most this
 * many triangles become leaves, and free child slots are filled by splitting
 * leaf-sized subtrees further.  Scenes of large flat faces (rooms) traverse
 * faster with 3, scenes of long thin triangles (the forest's trunks) with 4.
 * VF_EINVAL outside 1..4. */
vf_status vf_set_bvh_leaf_size(vf_ctx* ctx, int32_t max_tris);

/* Enable (1) / disable (0) traversal statistics: while enabled, vf_step and
 * vf_render use a counting variant of the render kernel that accumulates node
 * visits, box tests, triangle tests and rays into the context's counters. */
vf_status vf_set_stats(vf_ctx* ctx, int32_t enable);

/* Read (and optionally reset) the counters: out[0] rays, out[1] inner-node
 * visits per lane, out[2] ray-box tests, out[3] ray-triangle tests (1-3: issued, every
 * valid lane at every node or leaf its packet visits), out[4] wave-level node visits,
 * out[5] wave-level triangle loads, out[6] VALU operations of the box tests (11 per test
 * in a packet whose rays share one direction octant, 14 where they differ in the sign of
 * one axis, 18 otherwise), out[7] hits, out[8] node visits, out[9] ray-box tests and
 * out[10] ray-triangle tests a lane's own ray asked for (visits of nodes and leaves whose
 * box that ray entered), out[11] swarm member tests (oriented member boxes tested per
 * lane; the member trees' box tests are in out[2]).  Synchronises the device. */
#define VF_STAT_COUNT 12
vf_status vf_stats_read(vf_ctx* ctx, uint64_t out[VF_STAT_COUNT], int32_t reset);

/* Render-kernel timing: while enabled (1), vf_step and vf_render record a pair of
 * HIP events on the caller's stream around every render-kernel launch.
 * vf_timing_read waits for the recorded events and returns the summed kernel
 * time (ms) and the number of launches since the last reset.  Disabling clears
 * the record. */
vf_status vf_set_timing(vf_ctx* ctx, int32_t enable);
vf_status vf_timing_read(vf_ctx* ctx, double* total_ms, int64_t* launches, int32_t reset);

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
 * Results (depth, optional ids / colours, new states) go to device buffers the
 * request names and/or back to host memory; latency is measured from submit to the
 * completion of the batch.  While batches are in flight the server's worker thread
 * polls their completion without sleeping (one host core).  Agents are
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

/* Where a request's results go.  Device buffers (any may be NULL) receive them on
 * the batch's stream before the request completes: depth [n_env][H][W] float32,
 * tri_id [n_env][H][W] int32 (needs want_tri_id), rgb [n_env][3][H][W] uint8 (needs
 * want_rgb), state [n_env][17] float32.  A server without ids and colours renders a
 * request's depth straight into its depth buffer when the request keeps no host
 * results (the buffer must be 4-byte aligned; otherwise, and for the other outputs,
 * a device-to-device copy).  host_results = 1 also keeps host copies for
 * vf_server_wait. */
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
    int64_t requeued;          /* requests queued again after their batch failed */
    int64_t failed_batches;    /* batches that failed to launch or were reported failed */
} vf_server_stats;

/* state_table [n_slots][17] float32 [dev]: resident env states, updated in place. */
vf_status vf_server_create(vf_ctx* ctx, const vf_server_config* cfg, float* state_table, int64_t n_slots,
                           vf_server** out);
/* env_slots [n_env] int32 [host], distinct, in [0, n_slots); actions [n_env][4] float32 [host];
 * out [host] or NULL (= host results only).  Returns at once with a ticket; VF_ENOSCENE /
 * VF_EINVAL (image size, hfov in (0, pi), 0 < near_clip < far_clip, slots) / VF_ENOMEM (larger
 * than one arena).  Device output buffers must stay valid until the request completes.  Each
 * batch has a device error word of its own: data a kernel of the batch had to skip fails that
 * batch's requests with VF_EDEVICE (vf_server_wait), and never touches the context's word. */
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
/* A host-forced backend error, for failure-path runs: the next n batches that finish are treated as
 * failed.  Each such batch's env slots are restored to their states before it (the batch saves them
 * before its step) and its requests go back to the front of the queue, in order; a request that has
 * been in 8 failed batches fails with VF_EHIP.  Results are unchanged by the retries.  The environment
 * variable VF_FAULT_INJECT=n at vf_server_create does the same for the server's first n batches.
 * A batch that fails to launch is handled the same way. */
vf_status vf_server_inject_faults(vf_server* s, int64_t n);
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
