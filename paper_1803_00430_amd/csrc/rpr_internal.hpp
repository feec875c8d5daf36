// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/rpr.h"

namespace rpr {

// Thread-local error message; set_error returns the code for `return set_error(...)`.
int set_error(int code, const char* fmt, ...);

#define RPR_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            return ::rpr::set_error(e_ == hipErrorOutOfMemory ? RPR_ENOMEM : RPR_EDEVICE,  \
                                    "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),        \
                                    __FILE__, __LINE__);                                   \
        }                                                                                  \
    } while (0)

constexpr int kWave = 64;
constexpr int kMaxStack = 64;       // traversal stack entries per lane
constexpr int kNode4 = 8;           // float4 per 4-wide node
constexpr int kMatStride = 32;      // floats per material record
// A reflected segment starts this far (metres) off the surface along the
// normal facing the incoming ray.  FP32 hit points lie a few units in the last
// place off their plane; with the origin on the plane, a ray reflected near
// the shared edge of two coplanar triangles can meet the neighbour at t ~ 0 and
// alternate between the two.  1 mm is >= 30 ulps for coordinates up to 500 m.
constexpr float kSurfaceOffset = 1e-3f;
constexpr double kSurfaceOffset64 = 1e-3;
// Material record: [1 + b] alpha_b, [9 + b] scattering s_b, [17 + b] 1 - alpha_b.
constexpr int kMatAlpha = 1, kMatS = 9, kMatKeep = 17;

// Node links: >= 0 internal node index, < 0 leaf = ~sorted triangle index.
__host__ __device__ inline bool is_leaf(int32_t link) { return link < 0; }
__host__ __device__ inline int32_t leaf_index(int32_t link) { return ~link; }
__host__ __device__ inline int32_t leaf_link(int32_t i) { return ~i; }

// One scene's BVH as consumed by the traversal kernels.
//   nodes: 4-wide nodes of 128 bytes (one cache line): four 32-byte child
//     slots, slot j = float4 (lo.x, lo.y, lo.z, link bits), float4 (hi.x,
//     hi.y, hi.z, 0).  An empty slot has the box lo = hi = +inf, whose entry
//     distance is never finite, and a leaf link.
//   tris: 3 float4 per triangle in Morton (leaf) order, the input vertices
//     unchanged: (v0.xyz, original index bits), (v1.xyz, material bits),
//     (v2.xyz, 0)
struct SceneView {
    const float4* nodes;
    const float4* tris;
    const float* mats;
    int32_t root;  // link of the root (leaf link when n_tris == 1; 0 when empty and n_tris == 0)
    int32_t n_tris;
    int32_t n_bands;
    int32_t pad;
};

// Per source-listener pair, as read by the trace kernel.
struct PairDesc {
    SceneView scene;
    float src[3];
    float lst[3];
    float radius;
    float inv_vs;       // 1 / sphere volume
    float c;            // speed of sound
    float dt;           // bin width
    float l_window;     // path length at which the histogram window ends: c * T * dt
    float e0;           // 1 / n_rays_total
    int32_t n_bins;
    int32_t max_bounces;
    int32_t sh_order;
    int32_t n_coeffs;
    uint32_t key0, key1;
    uint32_t pair_id;   // RNG counter word 1
    int32_t flags;      // RPR_TRACE_* bits
    int64_t ray_begin;  // absolute id of the pair's first ray
    int64_t n_rays;     // rays of this pair in the launch
    int64_t queue_begin;// first global queue slot of this pair
    float* hist;        // [T][B][NC]
    float* hist_late;   // [T][B] or null
    RprIrStats* stats;
    uint32_t* ray_hash; // [n_rays] or null
    // deterministic accumulation (RPR_TRACE_DETERMINISTIC): deposits are
    // added as round(value x fx_scale) to 64-bit integer cells, whose sums do
    // not depend on the order of the atomics, then converted to hist/hist_late
    long long* hist_fx; // [T][B][NC] or null (float accumulation)
    long long* late_fx; // [T][B] or null
    double fx_scale;
};

// Device memory for a build's temporaries (grow-only).
struct BuildMem {
    char* base = nullptr;
    size_t cap = 0;
};

struct Workspace {
    void* dev = nullptr;      // queue counter (+ padding) followed by the pair table
    size_t bytes = 0;
    void* host_pin = nullptr; // pinned staging for the pair table
    size_t host_bytes = 0;
};

}  // namespace rpr

struct RprScene {
    std::mutex mu;  // guards the pending-rebuild state below
    int device = 0;
    int64_t n_tris = 0;
    int32_t n_bands = 0;
    int32_t n_materials = 0;
    int32_t max_depth = 0;     // binary tree depth
    int32_t stack_need = 0;    // traversal stack entries the 4-wide tree can need
    int64_t n_nodes4 = 0;
    int32_t n_degenerate = 0;
    int64_t cap_tris = 0;        // triangles and materials the arrays below hold
    int32_t cap_materials = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float4* nodes = nullptr;
    float4* tris = nullptr;
    float* mats = nullptr;
    rpr::SceneView view{};
    rpr::Workspace ws;
    // scene_rebuild: its own build temporaries (grow-only), the pinned host
    // copy of the build's flags and the event after that copy; `pending` until
    // the result is applied (rpr::scene_settle)
    rpr::BuildMem build_mem;
    void* flags_host = nullptr;
    hipEvent_t built = nullptr;
    bool pending = false;
    int64_t pending_tris = 0;
};

namespace rpr {
// Wait for the scene's pending rebuild, if any, and apply its result: the
// scene's sizes on success; an empty scene and the build's error otherwise
// (reported once).  Every call that reads a scene calls this first.
int scene_settle(const RprScene* scene);
// Ensure the workspace holds `pairs` pair descriptors, and fx_bytes more from
// workspace_fx_offset(pairs) on (fixed-point histogram cells, then the slot
// order of the trace); returns RPR_OK or an error.
int workspace_reserve(Workspace& ws, size_t pairs, size_t fx_bytes = 0);
size_t workspace_fx_offset(size_t pairs);
void workspace_free(Workspace& ws);
// Launch the persistent trace over `n_pairs` descriptors already in device memory.
int launch_trace(const PairDesc* d_pairs, int n_pairs, unsigned long long* d_queue, int64_t total_rays,
                 int nb, int stack_need, bool count_visits, int waves_per_cu, int grid_override, hipStream_t stream,
                 float* rec = nullptr, unsigned* rec_count = nullptr, int rec_cap = 0,
                 const long long* total_dev = nullptr, const uint32_t* order = nullptr);

// Early-reflection path records (trace_ir_paths, path_cache_*): 32 words each,
// words 0-1 the key (source << 48 | order << 46 | tri1 << 23 | tri2, 23-bit
// triangle fields, kRecNoTri for none), 2-9 band intensity, 10 arrival time,
// 11-26 SH directivity.
constexpr int kRecWords = 32;
constexpr uint32_t kRecNoTri = 0x7FFFFFu;
// Launch the listener-origin trace (next-event queries toward each pair's
// source ball) over `n_chunks` chunk descriptors already in device memory
// (the queue counts chunks; each is traced by one wave).
int launch_trace_listener_pairs(const PairDesc* d_chunks, int n_chunks, unsigned long long* d_queue, int64_t total_rays,
                                int nb, int stack_need, int waves_per_cu, hipStream_t stream);
int trace_listener_max_waves_per_cu(int nb, int stack_need);
int device_cu_count();
// Largest resident waves per CU of the trace variant for (nb, stack_need).
int trace_max_waves_per_cu(int nb, int stack_need);
// Zero n floats (a kernel, so that it can be captured into a graph).
int enqueue_fill_zero(float* p, size_t n, hipStream_t stream);
// Fixed-point histogram cells to FP32: out[i] = fx[i] / scale of its pair
// (scales[j] for pair j = i / per_pair, or `scale` when scales is null).
int enqueue_fx_convert(const long long* fx, float* out, long long per_pair, int n_pairs, const double* scales,
                       double scale, hipStream_t stream);
// Initialise n statistics records and zero the ray queue counter.
int enqueue_stats_reset(RprIrStats* stats, int n, unsigned long long* queue, hipStream_t stream);
}  // namespace rpr
