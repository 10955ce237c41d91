// Internal definitions shared by the HIP sources of the library (device structs,
// launch constants, the context).  Not part of the public ABI (include/visfly.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <list>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/visfly.h"

namespace vf {

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
constexpr int kWave = 64;             // CDNA wavefront
#ifndef VF_TILE_W
#define VF_TILE_W 4
#endif
// a wavefront's packet: kTileH x kTileW pixels, one ray per lane.  Tall packets (16 x 4) keep the rays of a
// vertical edge -- trunks, walls, pillars seen by a level camera -- in fewer packets than 8 x 8 squares
constexpr int kTileW = VF_TILE_W;
constexpr int kTileH = 64 / kTileW;
static_assert(kTileW * kTileH == 64 && kTileW >= 1, "a packet has one ray per lane of a wavefront");
#ifndef VF_OCTANT_PACKETS
#define VF_OCTANT_PACKETS 1   // packets of one ray octant take the traversal with fixed slab planes
#endif
#ifndef VF_PARTIAL_OCTANT
#define VF_PARTIAL_OCTANT 1   // packets mixed in one axis fix the slab planes of the other two
#endif
#ifndef VF_RENDER_WAVES
#define VF_RENDER_WAVES 1
#endif
constexpr int kWavesPerBlock = VF_RENDER_WAVES;  // render workgroup = this many wavefronts, one packet each
constexpr int kOrderMax = 1024;      // capacity of the spatial-order kernel (agents per batch)
constexpr int kOrderAutoMax = 512;   // split launches of 64 .. this many agents are put in spatial order
constexpr int kGroupOrderMax = 1 << 18;  // capacity of the cost-order kernel (workgroups per launch)
constexpr int kGroupOrderChunk = 16384; // groups one workgroup of that kernel sorts
constexpr int kGroupOrderMin = 1024;    // smaller launches keep the plain order
constexpr int kCostBuckets = 32;
#ifndef VF_PACKET_ROWS
#define VF_PACKET_ROWS 1
#endif
#ifndef VF_PACKET_COLS
#define VF_PACKET_COLS 1
#endif
constexpr int kPacketRows = VF_PACKET_ROWS;  // a wavefront's packet: rows x cols of such tiles,
constexpr int kPacketCols = VF_PACKET_COLS;  // one ray of each per lane
#ifndef VF_LEAF_MAX
#define VF_LEAF_MAX 4
#endif
constexpr int kLeafMax = VF_LEAF_MAX;  // triangles per BVH leaf (at most 8: the stack entry keeps 3 bits)
#ifndef VF_BVH_WIDTH
#define VF_BVH_WIDTH 4
#endif
constexpr int kWidth = VF_BVH_WIDTH;                 // children per BVH node
static_assert(kWidth == 4 || kWidth == 8, "4- or 8-wide BVH");
constexpr int kWidthBits = kWidth == 4 ? 2 : 3;      // bits of a child slot index
// waves per SIMD the render kernel is compiled for: the 8-wide node needs 64 scalar registers
// for one node, which 8 waves per SIMD cannot hold besides the rest
constexpr int kRenderWavesPerEu = kWidth == 4 ? 8 : 6;
constexpr int kFusedWavesPerEu = 2;   // the fused step + render (small batches: at most 1,024 workgroups)
constexpr int kStackCap = 128;        // traversal stack entries per wavefront (lanes of 2 VGPRs at most)
// builds deeper than this are rejected: a packet keeps at most kWidth - 1 pending siblings per level
constexpr int kMaxBvhDepth = kWidth == 4 ? 40 : 18;
// a packet keeps at most kWidth - 1 pending siblings per level of its path plus the children just pushed
static_assert((kWidth - 1) * (kMaxBvhDepth - 1) + kWidth <= kStackCap, "traversal stack cannot overflow");
// BVHs up to this depth keep a packet's pending entries within one VGPR's 64 lanes: launches over such
// scenes only take the render with a one-register stack
constexpr int kShallowDepth = (kWave - kWidth) / (kWidth - 1) + 1;
static_assert((kWidth - 1) * (kShallowDepth - 1) + kWidth <= kWave, "one stack register holds a shallow BVH's walk");
constexpr int kMaxScenes = 1024;
constexpr int kServerMaxAttempts = 8;   // batches a server request may be launched in before it fails
constexpr int kMaxImage = 1024;

// sticky device error bits
enum : uint32_t {
    kErrScene = 1u << 0,      // scene id out of range or freed
    kErrSlot = 1u << 1,       // env_idx out of [0, n_slots)
    kErrPixels = 1u << 2,     // out_offset + H*W beyond out_pixels (or negative)
    kErrView = 1u << 3,       // H, W outside [1, max], bad hfov, near <= 0 or far <= near
    kErrStack = 1u << 4,      // traversal stack overflow
    kErrTriIndex = 1u << 5,   // scene build: vertex index out of range
    kErrTriId = 1u << 6,      // render_backward: tri id out of range
    kErrVertex = 1u << 7,     // scene build: a triangle's vertex coordinate is not finite
};

// ---------------------------------------------------------------------------
// device scene layout
// ---------------------------------------------------------------------------
// A BVH node: SoA child boxes, one stack entry per child (node index, or a leaf's encoded range, or
// kEmptyChild), and the near-to-far child order of each of the 8 ray-direction octants.
//   4-wide (128 B): + leaf counts (byte per child) and the orders as one 64-bit value (a byte per octant)
//   8-wide (256 B): the orders as 8 words (octant o: 3-bit slots in word o)
constexpr int32_t kEmptyChild = INT32_MIN;
struct alignas(16) Node4 {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    int32_t child[4];
    uint8_t count[4];
    uint32_t order[3];   // order[0] | order[1] << 32: byte o = octant o's slots; order[2] = 0
};
struct alignas(16) Node8 {
    float lo_x[8], hi_x[8], lo_y[8], hi_y[8], lo_z[8], hi_z[8];
    int32_t child[8];
    uint32_t order[8];   // word o: octant o's eight 3-bit slots
};
static_assert(sizeof(Node4) == 128 && sizeof(Node4) == sizeof(vf_bvh4_node), "4-wide node layout");
static_assert(sizeof(Node8) == 256 && sizeof(Node8) == sizeof(vf_bvh8_node), "8-wide node layout");
using Node = typename std::conditional<kWidth == 4, Node4, Node8>::type;
constexpr int kNodeWords = (int)sizeof(Node) / 4;
constexpr int kChildWord = 6 * kWidth;                     // first child word
constexpr int kOrderWord = kWidth == 4 ? 29 : 56;          // first order word
// leaf count of a child entry (0 for an inner node or an empty slot)
__host__ __device__ inline int leaf_count(int32_t c) { return (c < 0 && c != kEmptyChild) ? ((-c - 1) & 7) + 1 : 0; }
__host__ __device__ inline int leaf_first(int32_t c) { return (-c - 1) >> 3; }
__host__ __device__ inline void set_leaf_count(Node4& n, int k, int c) { n.count[k] = (uint8_t)c; }
__host__ __device__ inline void set_leaf_count(Node8&, int, int) {}

struct alignas(16) Tri {
    float v0x, v0y, v0z; int32_t id;
    float e1x, e1y, e1z, pad1;
    float e2x, e2y, e2z, pad2;
};
static_assert(sizeof(Tri) == 48, "triangle record is 48 bytes");
static_assert(sizeof(Tri) == sizeof(vf_tri), "triangle matches the exported layout");

// One entry of the device scene table (64 bytes).
struct alignas(16) SceneDesc {
    const Node* nodes;
    const Tri* tris;          // sorted leaf order
    const uint8_t* rgb;       // [T][3] caller order, or null
    const int32_t* sorted_of; // caller triangle index -> sorted position
    int32_t n_tris;
    int32_t root_leaf;        // 1: the whole scene is one leaf (T <= kLeafMax), no nodes
    int32_t valid;
    int32_t n_nodes;
    int32_t pad[4];
};
static_assert(sizeof(SceneDesc) == 64, "scene table entry is 64 bytes");
static_assert(sizeof(vf_scene_info) == 80, "vf_scene_info layout");
static_assert(sizeof(vf_view) == 72, "view descriptor is 72 bytes");
static_assert(sizeof(vf_dyn_params) == 128, "parameter block is 128 bytes");
static_assert(sizeof(vf_noise) == 64, "noise block is 64 bytes");

// ---------------------------------------------------------------------------
// dynamics constants, derived once per call on the host
// ---------------------------------------------------------------------------
// Dynamics constants derived on the host from vf_dyn_params (in double, then held in T): the forward step
// runs on the double set, the adjoint's float32 linearisation and the IMU on the float set.
template <typename T>
struct DynConstT {
    T h;                  // sub-step length dt / n_sub
    int32_t n_sub, integrator, ctrl;
    T mass, inv_mass, g;
    T J[3], inv_J[3];
    T kJ[3];              // J * k_rate
    T arm_a, inv_a;       // arm / sqrt(2) and its reciprocal
    T kappa, inv_kappa, f_max;
    T k_lin[3], c_quad[3];
    T e_half, e_full;     // exp(-h / (2 tau)), exp(-h / tau)
    T k_pos[3], k_vel[3], k_att[3];
    T tan_tilt, min_lift; // tan(max_tilt), g / 4
};
using DynConst = DynConstT<float>;
using DynConstD = DynConstT<double>;

DynConst make_dyn_const(const vf_dyn_params& p);
DynConstD make_dyn_const_d(const vf_dyn_params& p);
bool check_dyn_params(const vf_dyn_params& p, std::string* why);
bool check_noise(const vf_noise& c, std::string* why);

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// One swarm member in its swarm's tree order (64 bytes: one 16-dword scalar load).
struct alignas(16) SwarmMember {
    float r[9];       // R(q / |q|) of the member's state, row major (float32, as the render tests it)
    float c[3];       // the member's position (box centre)
    int32_t j;        // index in the swarm's slot list: the member's id is n_tris + j
    int32_t slot;     // its state slot (a view does not see its own agent)
    int32_t pad[2];
};
static_assert(sizeof(SwarmMember) == 64, "swarm member record is 64 bytes");
constexpr int kSwarmMaxMembers = 4096;   // members per swarm (the tree build sorts them in LDS)

// Swarm table: CSR lists of member state slots, the members' body box, and the members' trees of the
// launch (per stream; rebuilt from the states before every render that shows swarms).
struct SwarmTable {
    const int32_t* off;       // [n + 1]
    const int32_t* slots;     // [off[n]]
    const int32_t* node_off;  // [n + 1] first node of each swarm's tree
    int32_t n;
    float half[3];
    float radius;             // |half|, the bounding-sphere radius used by the collision check
    uint8_t rgb[4];
    Node4* nodes;             // trees, node_off[n] nodes
    SwarmMember* members;     // members in tree order, swarm s at off[s]
};
// Nodes of the implicit tree over m members (four per leaf, four children per node).
__host__ __device__ inline int32_t swarm_tree_levels(int32_t m) {
    const int32_t groups = (m + 3) / 4;
    int32_t levels = 1;
    for (int64_t span = 4; span < groups; span *= 4) ++levels;
    return levels;
}
__host__ __device__ inline int32_t swarm_level_nodes(int32_t m, int32_t levels, int32_t d) {
    // level d (0 = root) of a tree of `levels` levels: each node of the lowest level holds four leaves
    const int64_t groups = (m + 3) / 4;
    int64_t span = 1;
    for (int32_t k = d; k < levels; ++k) span *= 4;
    return (int32_t)((groups + span - 1) / span);
}
__host__ __device__ inline int32_t swarm_tree_nodes(int32_t m) {
    if (m <= 0) return 0;
    const int32_t levels = swarm_tree_levels(m);
    int32_t total = 0;
    for (int32_t d = 0; d < levels; ++d) total += swarm_level_nodes(m, levels, d);
    return total;
}

// Member trees of one stream's launches (nodes, then member records), for one vf_set_swarms generation.
struct SwarmTree {
    void* stream = nullptr;
    void* block = nullptr;
    int64_t bytes = 0;
    int64_t gen = -1;
};

struct SceneHost {
    bool used = false;
    void* block = nullptr;      // one device allocation holding everything below
    int64_t bytes = 0;
    int32_t* labels = nullptr;  // optional per-triangle semantic labels
    int64_t label_bytes = 0;
    vf_scene_info info{};
    SceneDesc desc{};
};

struct Counters {               // per state buffer arrival counters of the fused kernel
    const float* state = nullptr;
    int32_t* counters = nullptr;
    int64_t capacity = 0;
};

}  // namespace vf

namespace vf {
// Launch-order scratch of one stream: the agent order, the per-packet work its last render reported and
// the workgroup order computed from it.  Only launches on that stream touch it.
struct StreamScratch {
    void* stream = nullptr;
    int32_t* order = nullptr;     // [kOrderMax]
    int32_t* cost = nullptr;      // [kGroupOrderMax * waves per workgroup]
    int32_t* perm = nullptr;      // [kGroupOrderMax]
    int32_t cost_n = -1;          // launch shape the cost array holds (views, groups per view)
    int32_t cost_groups = -1;
};
constexpr int64_t kStreamScratchBytes = 4 * (kOrderMax + (int64_t)kGroupOrderMax * (kWavesPerBlock + 1));
}  // namespace vf

struct vf_ctx {
    int device = 0;
    int n_cu = 0;
    int64_t budget = 0;
    int64_t used = 0;
    std::mutex mu;
    std::vector<vf::SceneHost> scenes;
    std::atomic<int32_t> max_bvh_depth{0};  // deepest BVH of the resident scenes
    vf::SceneDesc* d_scenes = nullptr;     // device scene table [kMaxScenes]
    const int32_t** d_labels = nullptr;    // device table of per-scene label arrays [kMaxScenes]
    uint32_t* d_err = nullptr;             // sticky error word of the calls that take a stream
    uint32_t* d_build_err = nullptr;       // error word of vf_scene_build's input check (its own, so a build
                                           // never clears a fault another stream has reported)
    unsigned long long* d_stats = nullptr; // 8 counters
    bool stats = false;
    int32_t launch_mode = VF_LAUNCH_AUTO;
    int32_t bvh_builder = VF_BVH_CLUSTER;
    int32_t bvh_leaf = vf::kLeafMax;    // leaf size of later builds (1..kLeafMax)
    std::vector<vf::Counters> counters;
    vf::SwarmTable swarm{};                // device copy of the swarm lists (n = 0: none)
    int64_t swarm_bytes = 0;
    int64_t swarm_members = 0;             // members over all swarms
    int64_t swarm_nodes = 0;               // tree nodes over all swarms
    int64_t swarm_gen = 0;                 // bumped by every vf_set_swarms
    std::list<vf::SwarmTree> swarm_trees;  // per stream: the member trees of its launches
    bool timing = false;                   // events around every render launch
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_events;   // recorded pairs
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_free;     // reusable pairs
    bool spatial_order = true;             // render agents in (scene, position) order
    bool cost_order = true;                // start each XCD's longest packets first
    std::list<vf::StreamScratch> orders;   // per stream: order scratch (stable addresses)
    vf_noise render_noise{};               // depth / colour noise of the render epilogue
    bool render_noise_on = false;
};

namespace vf {
// ---------------------------------------------------------------------------
// kernel launch arguments (passed by value)
// ---------------------------------------------------------------------------
struct RenderArgs {
    const SceneDesc* scenes;
    int32_t n_scenes;
    int32_t n;
    const int32_t* env_idx;
    float* state;
    int64_t n_slots;
    const float* action;
    const vf_view* views;
    int32_t max_h, max_w;
    int32_t groups_per_agent;
    int32_t total_groups;
    float* depth;
    float* const* depth_views;    // per view: the view's own H x W depth target (replaces depth), or NULL
    int32_t* tri_id;
    uint8_t* rgb;
    int64_t out_pixels;
    uint32_t* err;
    unsigned long long* stats;
    int32_t* counters;
    const int32_t* order;    // logical agent -> view index (spatial order), or NULL for identity
    const int32_t* group_order;   // dispatch position -> logical group (cost order), or NULL for identity
    int32_t* cost;                // per (logical group, wavefront) traversal work written by the launch, or NULL
    SwarmTable swarm;
    DynConstD dyn;
    vf_noise noise;               // depth / colour noise of the epilogue (read by the noise variant only)
    int32_t max_depth;            // deepest BVH of the resident scenes (picks the stack form, host only)
};
struct OrderArgs {
    int32_t n;
    const int32_t* env_idx;
    const float* state;
    int64_t n_slots;
    const vf_view* views;
    int32_t* order;
};
hipError_t launch_order(const OrderArgs& a, hipStream_t st);
struct GroupOrderArgs {
    int32_t total;               // workgroups of the launch
    const int32_t* cost;         // [logical group][waves per workgroup] from the previous launch
    int32_t* perm;               // out: [total], dispatch position -> logical group
};
hipError_t launch_group_order(const GroupOrderArgs& a, hipStream_t st);
int32_t render_groups_per_agent(int32_t max_h, int32_t max_w);
struct StepArgs {
    int32_t n;
    const int32_t* env_idx;
    float* state;
    int64_t n_slots;
    const float* action;
    uint32_t* err;
    DynConstD dyn;
    float* before;       // [n][17] the rows before the step (a batch that may run again), or NULL
};
struct StepBackArgs {
    int32_t n;
    const float* state_in;
    const float* action;
    const float* grad_out;
    float* grad_in;
    float* grad_action;
    DynConstD dyn;       // the step's FP64 constants (the adjoint recomputes and linearises its sub-steps)
};
struct RenderBackArgs {
    const SceneDesc* scenes;
    int32_t n_scenes;
    int32_t n;
    const float* state;
    const vf_view* views;
    int32_t max_h, max_w;
    const int32_t* tri_id;
    const float* grad_depth;
    int64_t out_pixels;
    float* grad_state;
    uint32_t* err;
};
struct NoiseArgs {
    int32_t n;
    const vf_view* views;
    int32_t max_h, max_w;
    int32_t blocks_per_agent;
    vf_noise cfg;
    const int32_t* tri_id;
    float* depth;
    uint8_t* rgb;
    int32_t* seg;
    int64_t out_pixels;
    uint32_t* err;
};
struct SegArgs {
    const SceneDesc* scenes;
    const int32_t* const* labels;
    int32_t n_scenes;
    int32_t n;
    const vf_view* views;
    int32_t max_h, max_w;
    int32_t blocks_per_agent;
    const int32_t* tri_id;
    int32_t* seg;
    int64_t out_pixels;
    uint32_t* err;
};
struct ImuArgs {
    int32_t n;
    const int32_t* env_idx;
    const float* state;
    int64_t n_slots;
    float sigma_acc, sigma_gyro;
    uint64_t seed;
    const int32_t* keys;
    float* out;
    uint32_t* err;
    DynConst dyn;
};
hipError_t launch_noise(NoiseArgs a, hipStream_t st);
hipError_t launch_segment(SegArgs a, hipStream_t st);
hipError_t launch_imu(const ImuArgs& a, hipStream_t st);

struct QueryArgs {
    const SceneDesc* scenes;
    int32_t n_scenes;
    int32_t n;
    const float* points;
    const int32_t* scene_ids;
    int32_t scene_id0;
    float max_dist;
    float* dist;
    float* closest;
    int32_t* tri_id;
    uint32_t* err;
    // agent mode (collision check): points are state rows, scenes come from the views
    const float* state;
    const int32_t* env_idx;
    int64_t n_slots;
    const vf_view* views;
    float radius;
    float* rel;
    uint8_t* collided;
    SwarmTable swarm;
};
hipError_t launch_closest_point(const QueryArgs& q, hipStream_t st);
hipError_t launch_step(const StepArgs& a, hipStream_t st);
// a split step's dynamics and the cost order of the render after it, in one launch
hipError_t launch_step_order(const StepArgs& s, const GroupOrderArgs& g, hipStream_t st);
hipError_t launch_render(RenderArgs a, bool fused, bool stats, bool noise, hipStream_t st);
hipError_t launch_step_backward(const StepBackArgs& a, hipStream_t st);
hipError_t launch_swarm_tree(const SwarmTable& sw, const float* state, int64_t n_slots, uint32_t* err,
                             hipStream_t st);
hipError_t launch_render_backward(const RenderBackArgs& a, hipStream_t st);
hipError_t launch_gather_rows(const float* state, const int32_t* idx, int32_t n, float* out, hipStream_t st);
hipError_t launch_scatter_rows(float* state, const int32_t* idx, int32_t n, const float* rows, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t st);
vf_status build_scene(vf_ctx* ctx, const float* verts, int64_t nv, const int32_t* tris, int32_t nt,
                      const uint8_t* rgb, hipStream_t st, SceneHost* out);

void set_error(const std::string& msg);
vf_status fail(vf_status st, const std::string& msg);
vf_status hip_fail(hipError_t e, const char* what);
vf_status ctx_alloc(vf_ctx* ctx, void** p, int64_t bytes);
void ctx_free(vf_ctx* ctx, void* p, int64_t bytes);
}  // namespace vf

#define VF_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return vf::hip_fail(e_, #call); \
    } while (0)
