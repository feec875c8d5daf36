/*
 * rpr.h -- C ABI of librpr.so: ray-parameterized reverberation propagation on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Schissler & Manocha, "Interactive Sound Rendering on Mobile Devices
 * using Ray-Parameterized Reverberation Filters" (arXiv 1803.00430).  Rays
 * leave each sound source carrying energy in N frequency bands, reflect
 * specularly or diffusely off a triangle scene under per-band absorption and
 * scattering (Section 5, "Sound Propagation"), and are scored at a listener
 * sphere into a low-rate impulse response: an intensity histogram per band
 * together with the real spherical-harmonic (SH) coefficients of the arrival
 * direction per time sample (Section 4.2, first paragraph).  Reverb
 * parameters -- RT60 per band, direct/early/late energies, reverb gain
 * (Eq. 5-8), predelay, mean free path and the energy-weighted directivity of
 * Eq. 1 -- are then estimated from that histogram (Section 4.2).  The
 * spherical-harmonic reverberator that those parameters drive (Section 4.1)
 * is built and rendered at audio rate by the reverb_setup / reverb_render
 * group.
 *
 * Conventions for every entry point
 *  - Return value: RPR_OK (0) or a negative RPR_E* code; last_error() then
 *    holds a message for the calling thread.  Argument errors are detected
 *    before anything is launched or written.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are read before the call returns.  The library never frees a
 *    caller buffer.  Objects created by the library (RprScene, RprBatch,
 *    RprModel) are owned by the library until the matching destroy call.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the legacy
 *    default stream) and is complete when that stream is synchronised,
 *    unless the entry point says it synchronises.
 *  - Calls that use the same RprScene, RprBatch or RprModel must be ordered
 *    on one stream: each object owns a workspace (queue counter, pair table,
 *    activations) that concurrent calls would share.
 *  - A device fault is reported as RPR_EDEVICE by the call that observes it.
 */
#ifndef RPR_H
#define RPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RPR_OK 0
#define RPR_EINVAL (-1)       /* invalid argument */
#define RPR_ENOMEM (-2)       /* device allocation failed */
#define RPR_EDEVICE (-3)      /* HIP runtime error or device fault */
#define RPR_EUNSUPPORTED (-4) /* valid but outside what this build supports */

#define RPR_MAX_BANDS 8
#define RPR_MAX_SH_ORDER 3
#define RPR_MAX_COEFFS 16

/* Per-band estimation status bits (RprReverbParams.status). */
#define RPR_ST_OK 0
#define RPR_ST_NO_ENERGY 1            /* the band's histogram is all zero */
#define RPR_ST_BAD_FIT 2              /* least-squares slope >= 0 */
#define RPR_ST_NO_RANGE 4             /* no decay range (T30/T20/T10/EDT) reachable */
#define RPR_ST_TRUNCATED_BY_BOUNCES 8 /* > 1e-3 of the emitted energy was alive at the bounce limit */
#define RPR_ST_TAIL_COMPENSATED 16    /* the window cut the decay; the missing tail was added */

typedef struct RprScene RprScene;

typedef struct {
    float pos[3]; /* metres */
} RprSource;

typedef struct {
    float pos[3];
    float radius; /* metres, > 0 */
} RprListener;

/* Parameters of one trace.  Every source traces the absolute ray ids
 * [ray_begin, ray_end); each ray starts with energy 1/n_rays_total in every
 * band, so disjoint ray ranges of the same n_rays_total add up.  The random
 * numbers of ray i of pair j at reflection order k are Philox4x32-10 of the
 * counter (i, j, k, 0) under the key (seed mod 2^32, seed >> 32), with
 * j = pair_base + source index. */
typedef struct {
    int64_t n_rays_total;
    int64_t ray_begin;
    int64_t ray_end;
    int32_t max_bounces;  /* K >= 0: segments of reflection order 0..K are traced */
    int32_t sh_order;     /* 0..3: (sh_order+1)^2 SH coefficients */
    int32_t n_bins;       /* T >= 1 histogram bins */
    int32_t pair_base;
    float bin_width_s;    /* > 0 */
    float speed_of_sound; /* > 0, m/s */
    uint64_t seed;
    int32_t flags;        /* RPR_TRACE_* bits */
    int32_t waves_per_cu; /* launch width of the persistent trace: resident waves per compute unit
                             (0 = the library's default); results do not depend on it */
    int64_t segment_budget; /* > 0: trace_ir chooses each source's ray count in the call (below) */
    int64_t max_rays;       /* with segment_budget: most rays per source, >= ray_end */
} RprTraceParams;

/* Segment budget (Section 5: every frame traces the same number of ray path
 * segments; rays that escape early leave budget for more primary rays).  With
 * segment_budget = B > 0 (ray_begin = 0, n_rays_total = ray_end = N0), trace_ir
 * traces rays [0, N0) of every source, then per source, from its own segment
 * count S0 of those rays,
 *     N' = clamp(N0 + floor((B - S0) * N0 / S0), N0, max_rays),
 * traces rays [N0, N') as well (one more launch on the stream, no host
 * round trip), and weights every ray of the source by 1/N' (the outputs are
 * rescaled by N0 / N').  stats.n_rays = N'.  ray_hash, when given, holds
 * max_rays entries per source (the first N' written).  B * max_rays must stay
 * below 2^63.  Only trace_ir takes a budget. */

/* RprTraceParams.flags: count BVH nodes visited and triangles tested into
 * RprIrStats.n_node_visits / n_tri_tests (a separate, slower kernel variant;
 * the counts size the traversal's memory traffic). */
#define RPR_TRACE_COUNT_VISITS 1
/* RprTraceParams.flags: accumulate the histograms in 64-bit fixed point
 * (every deposit rounded to a multiple of 2^-61 x the largest sum a cell can
 * reach, 4 x n_bands x bin_width / sphere volume), so that the histograms do
 * not depend on the order in which the deposits land: repeated calls, any
 * launch width and graph replays give bit-identical histograms and RT60.
 * Source-origin trace only (trace_ir without paths); the library holds the
 * 8-byte cells in the scene's workspace. */
#define RPR_TRACE_DETERMINISTIC 2

/* Per-IR trace statistics (device, written by trace_ir). */
typedef struct {
    int64_t n_segments;        /* closest-hit queries (ray-bounces), escaping ones included */
    int64_t n_finite_segments; /* segments that ended on a surface */
    int64_t n_escaped;
    int64_t n_rays;
    double seg_len_sum;        /* metres, over finite segments */
    double e_emitted;          /* n_rays / n_rays_total */
    int32_t first_arrival_bin; /* first bin with any deposit, INT32_MAX if none */
    int32_t first_late_bin;    /* first bin reached by an order >= 3 segment, INT32_MAX if none */
    double e_class[3][RPR_MAX_BANDS]; /* deposited intensity of orders 0 / 1-2 / >=3 */
    double e_escaped[RPR_MAX_BANDS];
    double e_alive_at_stop[RPR_MAX_BANDS];       /* energy of rays stopped by K or the window */
    double e_alive_at_bounce_cap[RPR_MAX_BANDS]; /* ... of those, stopped by K alone */
    double e_absorbed[RPR_MAX_BANDS];            /* sum over bounces of alpha_b * E_b */
    int64_t n_node_visits; /* internal BVH nodes fetched (with RPR_TRACE_COUNT_VISITS, else 0) */
    int64_t n_tri_tests;   /* triangle records fetched (with RPR_TRACE_COUNT_VISITS, else 0) */
    int64_t n_next_event;  /* trace_listener: next-event (occlusion) queries of the ray set; else 0 */
    int64_t n_deposit_rows;/* listener-origin traces: histogram bin rows (n_bands x coefficients floats)
                              added by deposits; else 0 */
} RprIrStats;

typedef struct {
    int64_t n_tris;
    int64_t n_nodes;      /* 4-wide BVH nodes */
    int32_t max_depth;    /* deepest leaf of the binary tree, in edges from the root */
    int32_t n_bands;
    int32_t n_materials;
    int32_t n_degenerate; /* zero-area triangles (kept; never hit) */
    float bounds_lo[3];
    float bounds_hi[3];
    int32_t stack_need;   /* traversal stack entries the deepest path can need (< 64) */
    int32_t reserved;
} RprSceneInfo;

/* Build a scene and its BVH (linear BVH: Morton codes of triangle centroids,
 * 30-bit, or 63-bit from 2^19 triangles on, radix sort, hierarchy from
 * longest common key prefixes, node boxes over each node's range of leaves,
 * collapsed into 4-wide nodes for traversal).
 *   verts        device [n_verts][3] f32, metres
 *   tris         device [n_tris][3] i32 vertex indices
 *   tri_material device [n_tris] i32 in [0, n_materials), or NULL = material 0
 *   absorption   device [n_materials][n_bands] f32 in [0, 1]
 *   scattering   device [n_materials][n_bands] f32 in [0, 1]
 *   n_bands      1..8 (Section 5 uses 4 bands)
 * The scene copies what it needs; the inputs may be freed afterwards.
 * Synchronises hip_stream (the build reads back validation flags and the tree
 * depth).  Errors: RPR_EINVAL for out-of-range indices or materials,
 * non-finite vertices, coefficients outside [0, 1]; RPR_EUNSUPPORTED if a
 * path of the tree could need 64 or more stack entries (the traversal takes 63). */
int scene_create(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                 const int32_t* tri_material, const float* absorption, const float* scattering,
                 int32_t n_materials, int32_t n_bands, void* hip_stream, RprScene** out);
/* Rebuild a scene in place from new geometry and materials (the same
 * arguments and build as scene_create), for scenes that change from frame to
 * frame (Section 5: the propagation update runs every frame).  Asynchronous:
 * the build is enqueued on hip_stream into the scene's own arrays and its own
 * temporaries, and the call returns without waiting (the inputs must stay
 * valid until the build has run on hip_stream).  The first call that reads
 * the scene afterwards (trace_ir, trace_ir_noalloc, trace_ir_paths,
 * trace_listener, scene_closest_hit, scene_info, batch_create, scene_wait)
 * waits for the build and reports what the device found (scene_create's
 * errors: out-of-range indices or materials, non-finite vertices,
 * coefficients outside [0, 1], a tree too deep); after such an error the
 * scene holds no triangles (every ray escapes) until a rebuild succeeds.
 * Work that reads the scene on other streams must be complete before the
 * call.  No allocation when the new triangles and materials fit what the
 * scene holds and its temporaries were sized by an earlier rebuild; otherwise
 * the arrays grow first (hipFree and hipMalloc, which wait for the device's
 * pending work).  A batch holds its scenes' state at batch_create: create it
 * again after rebuilding one of them.
 * Errors at the call: RPR_EINVAL for bad sizes or null arrays, or when the
 * current device is not the scene's; RPR_ENOMEM. */
int scene_rebuild(RprScene* scene, const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                  const int32_t* tri_material, const float* absorption, const float* scattering,
                  int32_t n_materials, int32_t n_bands, void* hip_stream);
/* Wait for the scene's last scene_rebuild and return its result (RPR_OK, or
 * the error the build found, reported once; the scene is then empty). */
int scene_wait(RprScene* scene);
int scene_destroy(RprScene* scene);
int scene_info(const RprScene* scene, RprSceneInfo* out /* host */);

/* Stochastic ray tracing from each source to the listener sphere (Section 5,
 * "Sound Propagation", traced forward from the sources; Section 4.2, the
 * low-rate IR).  The sphere is transparent; every segment of reflection
 * order k deposits, into each bin m it overlaps in propagation time, the
 * track-length estimate E_b * Y_c(-d) * overlap_s / V_sphere (d = propagation
 * direction, so -d points back along the path as in the notation table).
 *   srcs      host [n_src]
 *   lst       host, one listener
 *   p         host
 *   hist      device [n_src][n_bins][n_bands][(sh_order+1)^2] f32, overwritten
 *   hist_late device [n_src][n_bins][n_bands] f32 (orders >= 3 only), or NULL
 *   stats     device [n_src], overwritten
 *   ray_hash  device [n_src][ray_end - ray_begin] u32, or NULL: FNV-1a of the
 *             ray's sequence of hit triangle ids and bounce kinds.
 * Rays are traced by persistent workgroups that refill lanes from a global
 * queue; the scene's workspace makes calls on one scene stream-ordered.
 * Without a segment budget, and for up to 1,024 sources of at least 64 rays
 * and at most 2^26 rays in all, each source's queue slots take its rays in
 * the order of their first directions (a counting sort in the workspace,
 * 16 KB per source + 4 bytes per ray), which changes no ray's path or
 * deposits. */
int trace_ir(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
             const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
             uint32_t* ray_hash, void* hip_stream);

/* trace_ir for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as trace_ir (except that a segment budget and
 * RPR_TRACE_DETERMINISTIC, which need more scratch, are refused with
 * RPR_EINVAL), but the queue counter and the
 * pair table live in a static device array of the library (256 + 1,024 x 200
 * bytes, one per GPU, held until the process ends) instead of the scene's
 * workspace, so the call allocates nothing on the host or the device.  Its
 * queue slots take the rays in ray order (no direction sort: per-ray results
 * are those of trace_ir) at the full launch width unless p->waves_per_cu
 * says otherwise.
 * Limit: n_src <= 1024 (RPR_EINVAL above).  Every call on one GPU shares that
 * array and leaves its contents behind (each call rewrites what it reads):
 * calls that overlap on one GPU -- on different streams or from different
 * threads -- race and must be ordered by the caller. */
int trace_ir_noalloc(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                     const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                     uint32_t* ray_hash, void* hip_stream);

/* Path tracing from the listener with next-event estimation toward every
 * source (Section 5: backward path tracing from the listener, augmented
 * with diffuse rain; one set of rays serves all sources).  Each source is a
 * ball of radius lst->radius around its position; the listener is the point
 * lst->pos.  Ray i leaves the listener uniformly on the sphere (counter
 * (i, pair_base, 0, 0)) and reflects as in trace_ir.  Contributions, scored
 * with the track-length estimator of trace_ir into the histogram of source s:
 *   - at the listener and at each reflection k (1 <= k <= max_bounces, before
 *     the window end), one query per source: a direction drawn uniformly in
 *     the cone the ball subtends (counter (i, pair_base, k, 1 + s)), followed
 *     to its nearest hit; weight Omega / (4 pi) at the listener, and
 *     (1 - alpha_b) s_b cos Omega / pi times the band energy at a reflection
 *     (Omega the cone's solid angle);
 *   - every segment after a specular reflection, at every ball.
 * SH are those of the ray's first direction (its arrival direction at the
 * listener), or of the query direction for the direct sound.
 *   srcs      host [n_src], 1 <= n_src <= 256 (0 returns at once)
 *   lst       host: listener point, source ball radius (> 0)
 *   p         host; flags must be 0
 *   hist, hist_late, stats: as in trace_ir.  The path statistics (segments,
 *             escapes, energies, n_next_event) belong to the one ray set and
 *             are repeated in every record; e_class and the first bins are
 *             per source.
 *   ray_hash  device [ray_end - ray_begin] u32 (one per ray), or NULL: hit
 *             triangles, bounce kinds and each query's outcome.
 * Errors: RPR_EINVAL as trace_ir, or for more than 256 sources;
 * RPR_EUNSUPPORTED if the per-wave LDS of the sources does not fit. */
int trace_listener(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                   const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                   uint32_t* ray_hash, void* hip_stream);

typedef struct {
    int32_t rt60_source; /* 1: orders >= 3 only (hist_late), the IR Section 4.2 estimates the
                            parameters from; 0: all orders */
    int32_t tail_iters;  /* refits with the missing tail added when the window cut the decay (3) */
} RprEstimateParams;

typedef struct {
    float rt60[RPR_MAX_BANDS];       /* seconds; 0 if status has NO_ENERGY/BAD_FIT/NO_RANGE */
    int32_t rt60_range[RPR_MAX_BANDS]; /* 0 T30, 1 T20, 2 T10, 3 EDT, -1 none */
    int32_t status[RPR_MAX_BANDS];   /* RPR_ST_* bits */
    float e_direct[RPR_MAX_BANDS];
    float e_early[RPR_MAX_BANDS];
    float e_late[RPR_MAX_BANDS];
    float g_reverb[RPR_MAX_BANDS];   /* Eq. 5 with Eq. 8: sqrt(e_late * 6 ln 10 / rt60) */
    float predelay_s;                /* first late (order >= 3) bin * bin width; -1 if none */
    float first_arrival_s;           /* first bin with any energy * bin width; -1 if none */
    float mean_free_path_m;          /* seg_len_sum / n_finite_segments */
    float reserved;
    float dir_loudness[RPR_MAX_BANDS][RPR_MAX_COEFFS]; /* Eq. 1 */
} RprReverbParams;

/* Reverb parameters of n_ir histograms (Section 4.2): per band, the intensity
 * I[m] = sqrt(4 pi) hist[m][b][0] (or hist_late) is integrated backwards
 * (Schroeder), converted to dB and fitted by least squares on the first
 * reachable range of T30, T20, T10, EDT; RT60 = -60 / slope.  FP64
 * internally.
 *   hist      device [n_ir][n_bins][n_bands][(sh_order+1)^2] f32
 *   hist_late device [n_ir][n_bins][n_bands] f32, or NULL (then rt60_source must be 0)
 *   stats     device [n_ir]
 *   ep        host, or NULL for {1, 3} ({0, 3} when hist_late is NULL)
 *   out       device [n_ir] */
int estimate_reverb(const float* hist, const float* hist_late, const RprIrStats* stats, int32_t n_ir,
                    int32_t n_bins, int32_t n_bands, int32_t sh_order, float bin_width_s,
                    const RprEstimateParams* ep, RprReverbParams* out, void* hip_stream);

/* ---------------------------------------------------------- temporal coherence
 * Smoothing across frames (Section 4.2, Eq. 4: the RT60 of each frame is
 * blended into a cached value; Section 5: early- and late-reflection caches
 * with time constants tau_ER = 1 s and tau_LR = 3 s).  With frame length dt,
 * alpha = 1 - exp(-dt / tau), so a step is covered to 1 - exp(-t / tau)
 * after time t. */

/* alpha = 1 - exp(-frame_dt_s / tau_s); 1 when tau_s <= 0 (no smoothing). */
float temporal_alpha(float frame_dt_s, float tau_s);

/* Rays of the next frame under a segment budget (Section 5: every frame
 * traces the same number of ray segments; rays that escape early leave budget
 * for more primary rays).  A parallel trace cannot stop at the ray where the
 * budget runs out, so the frame traces N' rays with 1/N' of the energy each,
 * N' = clamp(floor(budget_segments * prev_rays / prev_segments), min_rays,
 * max_rays) from the previous frame's measured segments and rays (summed over
 * the sources traced together), or clamp(nominal) when there is no previous
 * frame (prev_segments or prev_rays <= 0).  Host arithmetic; no device call. */
int64_t budget_ray_count(int64_t budget_segments, int64_t prev_segments, int64_t prev_rays, int64_t min_rays,
                         int64_t max_rays, int64_t nominal);

/* IR cache: cache[i] = alpha * fresh[i] + (1 - alpha) * cache[i] for
 * i < n, or cache[i] = fresh[i] when first != 0 (the first frame or a reset).
 * Use it on the all-orders histogram with the early factor and on hist_late
 * with the late factor, then estimate from the caches.
 *   cache, fresh  device f32, 16-byte aligned, n floats each (the caller owns both)
 * Errors: RPR_EINVAL for a null or misaligned buffer or alpha outside [0, 1]. */
int ir_cache_update(float* cache, const float* fresh, int64_t n, float alpha, int32_t first, void* hip_stream);

/* Parameter smoothing of n_ir IRs, in place in `cache` (the output of the
 * frame and the cache of the next, as in Eq. 4):
 *   rt60[b]      Eq. 4 with alpha_late; a frame whose fit is invalid (status
 *                NO_ENERGY, BAD_FIT or NO_RANGE) keeps the cached value, and
 *                a valid frame after an invalid cache takes its own value;
 *                status and rt60_range follow the frame whose RT60 was used
 *   e_direct, e_early  smoothed with alpha_early; e_late with alpha_late
 *   g_reverb     sqrt(e_late * 6 ln 10 / rt60) of the smoothed values (Eq. 5, Eq. 8)
 *   all other fields: the fresh frame's
 * first != 0 copies fresh into cache.
 *   cache, fresh  device [n_ir]
 * Errors: RPR_EINVAL for bad sizes, null buffers or alphas outside [0, 1]. */
int reverb_params_smooth(RprReverbParams* cache, const RprReverbParams* fresh, int32_t n_ir, int32_t n_bands,
                         float alpha_early, float alpha_late, int32_t first, void* hip_stream);

/* ------------------------------------------------------------------ batches
 * Many source-listener pairs over several scenes traced by one persistent
 * launch (the paper traces every source of a frame; Section 5 "Sound
 * Propagation").  A batch is planned once and then run any number of times;
 * each run resets the outputs, traces every ray of every pair and estimates
 * the reverb parameters of every pair, with results that do not depend on the
 * launch shape. */
typedef struct RprBatch RprBatch;

typedef struct {
    int32_t scene;        /* index into the scenes passed to batch_create */
    int32_t pair_id;      /* RNG counter word 1 of this pair's rays */
    float src[3];
    float lst[3];
    float radius;         /* listener sphere radius, > 0 */
    int32_t max_bounces;  /* K >= 0 */
    int64_t n_rays;       /* rays of this pair (>= 1); each starts with energy 1/n_rays */
    uint64_t seed;        /* Philox key of this pair */
} RprPair;

typedef struct {
    int32_t n_bins;       /* T, shared by all pairs */
    int32_t sh_order;     /* 0..3 */
    float bin_width_s;
    float speed_of_sound;
    int32_t rt60_source;  /* as RprEstimateParams */
    int32_t tail_iters;
    int32_t autotune;     /* 1: time the candidate launch shapes at creation and keep the fastest */
    int32_t use_graph;    /* 1: capture the run (reset, trace, estimate) into a HIP graph */
    int32_t waves_per_cu; /* launch width when autotune = 0 (0 = library default) */
    int32_t order;        /* queue order when autotune = 0: 0 as given, 1 most rays x bounces first,
                             2 interleaved (pairs split into chunks of chunk_rays rays dealt
                             round-robin) */
    int32_t method;       /* 0: each pair traced from its source to the listener sphere (trace_ir);
                             1: from its listener point with next-event queries toward its source,
                             a ball of the pair's radius (trace_listener, one source per pair) */
    int32_t chunk_rays;   /* rays per chunk of the interleaved order and of the listener method's
                             chunk table when autotune = 0: 256, 1024 or 4096 (0 = 1024) */
    int32_t deterministic; /* 1: histograms accumulated as RPR_TRACE_DETERMINISTIC (method 0 only;
                              the batch holds the fixed-point cells) */
} RprBatchParams;

typedef struct {
    int64_t total_rays;
    int32_t n_pairs;
    int32_t waves_per_cu;  /* chosen launch width */
    int32_t order;         /* chosen queue order */
    int32_t stack_need;
    int32_t graph;         /* 1 if runs replay a captured graph */
    int32_t n_candidates;  /* launch shapes timed by the autotuner (0 without autotune or when the
                              shape came from the tuning cache) */
    float best_ms;         /* autotuner's best trace time */
    float worst_ms;        /* autotuner's worst trace time */
    int32_t chunk_rays;    /* chosen chunk size (interleaved order, listener method) */
    int32_t from_cache;    /* 1 if the shape came from the tuning cache (in memory or file) */
    int32_t stack_entries; /* traversal stack depth of the chosen kernel variant: 32, 48 or 64 (the
                              autotuner may pick one deeper than stack_need asks for) */
    int32_t fixed_point;   /* 1 if the histograms are accumulated in 64-bit fixed point: asked for
                              (deterministic), or picked by the autotuner as the faster deposit */
} RprBatchInfo;

/* Plan a batch.
 *   scenes     host [n_scenes] pointers; all scenes must have the same band count
 *   pairs      host [n_pairs], copied
 *   hist       device [n_pairs][n_bins][n_bands][(sh_order+1)^2] f32 (outputs of each run)
 *   hist_late  device [n_pairs][n_bins][n_bands] f32, or NULL
 *   stats      device [n_pairs]
 *   params     device [n_pairs]
 * The caller keeps the scenes and output buffers alive until batch_destroy.
 * Synchronises hip_stream (uploads the pair table; the autotuner runs the
 * batch a few times per candidate shape).
 * Autotuning times resident waves per CU (4 widths) x queue order (as given,
 * longest first, interleaved) x chunk size (256, 1,024, 4,096 rays; for the
 * interleaved order and the listener method) and keeps the fastest.  The
 * choice is cached per (GPU architecture, CU count, method, bands, bins, SH
 * coefficients, stack variant, and the log2 buckets of pairs, total rays,
 * mean bounces and largest scene); when the environment variable
 * RPR_AUTOTUNE_CACHE names a file, the cache is read from it at the first
 * batch_create and every new choice is written back (one line per key). */
int batch_create(const RprScene* const* scenes, int32_t n_scenes, const RprPair* pairs, int32_t n_pairs,
                 const RprBatchParams* bp, float* hist, float* hist_late, RprIrStats* stats,
                 RprReverbParams* params, void* hip_stream, RprBatch** out);
/* Enqueue one run on hip_stream (a graph launch when use_graph = 1). */
int batch_run(RprBatch* batch, void* hip_stream);
int batch_info(const RprBatch* batch, RprBatchInfo* out /* host */);
int batch_destroy(RprBatch* batch);

/* --------------------------------------------------------- learned estimator
 * The paper denoises the parameters of a low-ray-count trace by temporal
 * smoothing across frames (Section 4.2, Eq. 4).  The learned estimator maps
 * the SH x band histogram of a cheap trace (e.g. 1k rays, 200 bins of 10 ms)
 * directly to the parameters that the estimator above returns on a converged
 * trace, with an uncertainty per output; where the uncertainty is high the
 * caller re-traces the pair with more rays.
 *
 * Network: an MLP with layers dims[0] -> dims[1] -> ... -> dims[n_layers]
 * (ReLU between layers, the last layer linear).  For B bands the output has
 * 8B entries: mu = [log RT60_b | log(E_direct_b / e_in + 1e-4) | same for
 * early | late] and s = log sigma^2 of each, where e_in is the cheap trace's
 * mean per-band time-integrated intensity.  Training minimises the Gaussian
 * negative log-likelihood mean_i sum_j w_ij/2 ((mu_ij - t_ij)^2 exp(-s_ij) +
 * s_ij) by Adam.  Products run on BF16 matrix cores with FP32 accumulation;
 * master weights, gradients and Adam moments are FP32.
 *
 * Parameter vector (FP32, n_params floats): for each layer l, W_l
 * [dims[l+1]][dims[l]] row-major then b_l [dims[l+1]].
 * Features are BF16 (raw 16-bit patterns, uint16_t), [n][dims[0]]. */
typedef struct RprModel RprModel;

#define RPR_MODEL_MAX_LAYERS 8
#define RPR_ST_LEARNED 32       /* RprReverbParams.status: the values come from the learned estimator */
#define RPR_ST_UNCERTAIN 64     /* ... whose uncertainty exceeded the threshold */

typedef struct {
    int64_t n_params;
    int32_t n_layers;
    int32_t dims[RPR_MODEL_MAX_LAYERS + 1];
    int32_t max_batch;
    int64_t step;         /* Adam steps taken */
} RprModelInfo;

typedef struct {
    float lr;
    float beta1;          /* 0.9 */
    float beta2;          /* 0.999 */
    float eps;            /* 1e-8 */
    float weight_decay;   /* decoupled, matrices only: W -= lr * weight_decay * W */
    float reserved;
} RprAdamParams;

/* Create a model.  dims host [n_layers + 1], every entry a multiple of 32 and
 * <= 65536, n_layers in 1..8; max_batch in 1..8192 bounds the rows of one
 * training step and of one forward chunk.  Weights are initialised from
 * Philox4x32-10 under `seed`: W_l uniform in +-sqrt(6 / dims[l]) (scaled by
 * 0.1 for the last layer), biases 0.  Synchronises hip_stream. */
int reverb_model_create(const int32_t* dims, int32_t n_layers, int32_t max_batch, uint64_t seed,
                        void* hip_stream, RprModel** out);
int reverb_model_destroy(RprModel* model);
int reverb_model_info(const RprModel* model, RprModelInfo* out /* host */);
/* Replace / copy out the FP32 parameter vector (device [n], n = n_params).
 * load also refreshes the BF16 copies and resets the Adam moments and step. */
int reverb_model_load(RprModel* model, const float* params, int64_t n, void* hip_stream);
int reverb_model_save(const RprModel* model, float* params, int64_t n, void* hip_stream);

/* Input features of n_ir traces, rounded to BF16; one row of
 * n_bins * n_bands * n_coeffs + 64 values per trace.
 *
 * Histogram part (hist device [n_ir][n_bins][n_bands][n_coeffs] f32, the
 * layout trace_ir writes), in the histogram's own order; e_in = (1/B)
 * sum_{m,b} sqrt(4 pi) H[m][b][0]:
 *   coefficient 0 of band b: its Schroeder decay curve, the backward integral
 *     S_b[m] = sum_{j>=m} sqrt(4 pi) H[j][b][0] (Section 4.2): bin 0 holds
 *     ln(S_b[0] / e_in), bins m >= 1 hold 10 log10(S_b[m] / S_b[0]) / 60
 *     clipped below at -1; zero for a band without energy;
 *   coefficients k >= 1: sign(u) log1p(1e6 |u|) / 8 with u = H / e_in;
 *   all zero when e_in = 0.
 * Statistics part (stats device [n_ir], or NULL for zeros), 64 values, with
 * r(x) = ln(max(x / e_emitted, floor)): for each band b, [4b]
 * ln(max(-r(e_alive_at_stop), 1e-3)) / 5 (floor 1e-300; the log of the ray
 * population's decay exponent over the window), [4b+1] r(e_absorbed) / 10,
 * [4b+2] r(e_escaped) / 10 (floor 1e-12), [4b+3] r(e_alive_at_bounce_cap) / 60
 * (other floors 1e-30); [32] ln(mean free
 * path / 1 m) / 3, [33] ln(segments per ray) / 5, [34] escaped rays / rays,
 * [35] first arrival bin / n_bins, [36] min(first late bin, n_bins) / n_bins;
 * the rest 0.  The ray population's decay over the window uses every ray,
 * not only those that cross the listener sphere.
 * n_bins * n_bands <= 7936 (RPR_EUNSUPPORTED above).
 *   features device [n_ir][n_bins * n_bands * n_coeffs + 64] u16 (BF16)
 *   e_in     device [n_ir] f32 */
int reverb_model_featurize(const float* hist, const RprIrStats* stats, int32_t n_ir, int32_t n_bins,
                           int32_t n_bands, int32_t n_coeffs, uint16_t* features, float* e_in, void* hip_stream);
/* Training targets from the parameters of converged traces (device
 * [n_ir]) and the cheap traces' e_in (device [n_ir]):
 *   t device [n_ir][4B] f32 = [log rt60 | log(e_direct/e_in + 1e-4) | early | late]
 *   w device [n_ir][4B] f32 = 1 where defined (RT60: status without
 *     NO_ENERGY / BAD_FIT / NO_RANGE and rt60 > 0; energies: e_in > 0), else 0 */
int reverb_model_targets(const RprReverbParams* ref, const float* e_in, int32_t n_ir, int32_t n_bands, float* t,
                         float* w, void* hip_stream);
/* Network output for n feature rows (device [n][dims[0]] BF16) into out
 * (device [n][dims[n_layers]] f32); any n >= 0 (chunks of max_batch). */
int reverb_model_forward(RprModel* model, const uint16_t* features, int64_t n, float* out, void* hip_stream);
/* Loss and gradients of one minibatch: rows i = 0..m-1 are dataset rows
 * rows[i] (device [m] i32, or NULL for 0..m-1) of a dataset of n_rows rows:
 * features (device [n_rows][dims[0]] BF16), t and w (device
 * [n_rows][dims[n_layers]/2] f32).  m in 1..max_batch.  A row index outside
 * [0, n_rows) contributes a zero feature row with zero weights.  Gradients
 * stay in the model (reverb_model_grads copies them out, in the layout of the
 * parameter vector); loss (device, 1 f64) receives the mean NLL over the m
 * rows. */
int reverb_model_backward(RprModel* model, const uint16_t* features, int64_t n_rows, const int32_t* rows,
                          int32_t m, const float* t, const float* w, double* loss, void* hip_stream);
int reverb_model_grads(const RprModel* model, float* grads, int64_t n, void* hip_stream);
/* Two-tower layer 0: the first n_hist inputs (the histogram features) feed
 * a tower of tower_width units, and the remaining S = dims[0] - n_hist inputs
 * (the trace statistics) pass through unchanged as +s and -s, so that after
 * the ReLU layer 1 sees [tower(histogram) | max(s, 0) | max(-s, 0)]; requires
 * dims[1] = tower_width + 2 S and at least two layers.  The fixed entries of
 * W_0 and b_0 (zeros, +-1) are written now, after every Adam step and after
 * reverb_model_load.  n_hist = tower_width = 0 restores a dense layer 0 (the
 * weights keep their current values).  A narrow tower keeps the network from
 * fitting the 1k-ray histogram's noise, which swamps the statistics when all
 * inputs share one wide layer.  Errors: RPR_EINVAL for shapes that do not fit. */
int reverb_model_set_tower(RprModel* model, int32_t n_hist, int32_t tower_width, void* hip_stream);
/* One Adam step with the gradients of the last backward (host `ap`). */
int reverb_model_adam(RprModel* model, const RprAdamParams* ap, void* hip_stream);
/* backward followed by adam. */
int reverb_model_train_step(RprModel* model, const uint16_t* features, int64_t n_rows, const int32_t* rows,
                            int32_t m, const float* t, const float* w, const RprAdamParams* ap, double* loss,
                            void* hip_stream);
/* Reverb parameters from network outputs (device [n][8B]) and e_in (device
 * [n]): rt60 = exp(mu), energies = max(exp(mu) - 1e-4, 0) e_in, g_reverb by
 * Eq. 5 with Eq. 8, status RPR_ST_LEARNED, plus RPR_ST_UNCERTAIN (and
 * uncertain[i] = 1) where e_in = 0 or any band's sigma = exp(s/2) of its log
 * RT60 exceeds kappa.  Fields the network does not predict are zero.
 *   params device [n], sigma device [n][B] f32 or NULL, uncertain device [n] i32 or NULL */
int reverb_model_decode(const float* out, const float* e_in, int64_t n, int32_t n_bands, float kappa,
                        RprReverbParams* params, float* sigma, int32_t* uncertain, void* hip_stream);
/* Input normalisation of the network, fitted on a training set of n rows of
 * BF16 features [n][F] (device): mean[f] (FP64 accumulation) and
 * scale[f] = gain / max(std[f], 1e-3) with the population std; gain =
 * sqrt((F - F_hist) / F_hist) for the first F_hist features (the histogram)
 * and 1 for the rest (the statistics), so that both groups enter with the
 * same total variance.  mean, scale device [F] f32.  0 <= F_hist < F. */
int reverb_model_feature_stats(const uint16_t* features, int64_t n, int32_t F, int32_t F_hist, float* mean,
                               float* scale, void* hip_stream);
/* In place on n rows of BF16 features [n][F] (device): x = (x - shift[f]) *
 * scale[f], rounded to BF16 (shift, scale device [F] f32). */
int reverb_model_normalize(uint16_t* features, int64_t n, int32_t F, const float* shift, const float* scale,
                           void* hip_stream);
/* Input-support gate, applied after reverb_model_decode: a network's
 * uncertainty is only meaningful for inputs like those it was trained on, so
 * row i (features device [n][F] BF16, already normalised by
 * reverb_model_normalize) is also marked uncertain -- uncertain[i] = 1 and
 * RPR_ST_UNCERTAIN in params[i].status -- when any feature in columns
 * [c0, c1) lies beyond +-zmax training standard deviations.  params device
 * [n] or NULL, uncertain device [n] i32 or NULL (not both NULL). */
int reverb_model_ood_gate(const uint16_t* features, int64_t n, int32_t F, int32_t c0, int32_t c1, float zmax,
                          int32_t n_bands, RprReverbParams* params, int32_t* uncertain, void* hip_stream);
/* dst[idx[i]] = src[i] for i < n (device arrays): merges the parameters of
 * re-traced pairs into a learned result. */
int reverb_params_scatter(const RprReverbParams* src, const int32_t* idx, int64_t n, RprReverbParams* dst,
                          void* hip_stream);

/* ------------------------------------------------------- early-reflection paths
 * The early reflections as individual paths (Section 5): the first two
 * reflection orders, kept across frames in a diffuse path cache with SH
 * directivity per path, and prioritised for rendering -- paths below the
 * threshold of hearing discarded, the N_ER = 100 strongest among all sources
 * rendered, the others added to the late IR before it is analysed. */
#define RPR_PATH_RECORD_WORDS 32

/* trace_ir, plus one record per deposit of an order-1 or order-2 segment at
 * the listener sphere, in records (device [max_records][32] f32, in no
 * particular order): words 0-1 the 64-bit path key (little-endian words:
 * source << 48 | order << 46 | tri1 << 23 | tri2, triangles as original
 * indices, 0x7FFFFF for none), 2-9 the band intensity the histogram received
 * within the window (zero past n_bands), 10 the midpoint of the chord's
 * arrival-time interval clipped to the window (s), 11-26 the SH directivity
 * e_total Y_k(arrival direction) (zero past (sh_order+1)^2).  n_records
 * (device, 1 u32) is zeroed, then counts every record; those past
 * max_records are dropped (n_records > max_records tells).  Up to 65535
 * sources and 2^23 - 2 triangles (else RPR_EUNSUPPORTED); no
 * RPR_TRACE_COUNT_VISITS. */
int trace_ir_paths(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                   const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats, float* records,
                   uint32_t* n_records, int32_t max_records, void* hip_stream);

typedef struct RprPathCache RprPathCache;

/* A path for rendering (device). */
typedef struct {
    int32_t source;
    int32_t order;                /* 1 or 2 */
    int32_t tri[2];               /* triangles of the reflections (original indices), -1 for none */
    float e[RPR_MAX_BANDS];       /* band intensity */
    float t;                      /* intensity-weighted mean arrival time, s */
    float d[RPR_MAX_COEFFS];      /* SH directivity: sum of e_total Y_k(arrival direction) */
    float reserved[3];
} RprEarlyPath;

typedef struct {
    int32_t max_paths;
    int32_t n_paths;     /* paths in the cache now */
    int32_t overflow;    /* 1 once a frame's paths exceeded the capacity (sticky) */
    int32_t table_size;  /* hash-table slots (a power of two >= 4 max_paths) */
} RprPathCacheInfo;

/* A cache of up to max_paths (1..2^20) paths on the current device.
 * Allocates; synchronises the device. */
int path_cache_create(int32_t max_paths, RprPathCache** out);
int path_cache_destroy(RprPathCache* cache);
/* One frame of the cache (the diffuse path cache, Section 5, with the
 * early-reflection time constant): per path key, P <- (1 - alpha) P +
 * alpha F, F the sum of the frame's records of that key (0 if none), with P
 * the band intensities, the intensity-weighted arrival time (as a sum of
 * e_total t) and the SH directivity; first != 0 takes F alone.  Paths whose
 * total intensity falls below min_energy leave the cache.  records and
 * n_records as written by trace_ir_paths (the first min(*n_records,
 * max_records) are read).  Calls on one cache must be ordered on one
 * stream. */
int path_cache_update(RprPathCache* cache, const float* records, const uint32_t* n_records, int32_t max_records,
                      float alpha, int32_t first, float min_energy, void* hip_stream);
/* Prioritization of the cache's paths (Section 5): paths with total
 * intensity below threshold are discarded; the others are ranked by
 * decreasing total intensity over all sources (ties by key), the first n_er
 * written to out (device [n_er], strongest first) and their number to n_out
 * (device, 1 i32); every other path joins the late class of its source:
 * its band intensity is added to hist_late (device [n_src][n_bins][n_bands]
 * f32, or NULL) at the bin of its mean arrival time and moved from
 * stats[source].e_class[1] to e_class[2] (device [n_src], or NULL).  The
 * cache is not changed.  The ranking compares every pair of paths. */
int path_cache_select(RprPathCache* cache, float threshold, int32_t n_er, RprEarlyPath* out, int32_t* n_out,
                      float* hist_late, RprIrStats* stats, int32_t n_src, int32_t n_bins, int32_t n_bands,
                      float bin_width_s, void* hip_stream);
/* Counts and flags of the cache (host out); synchronises the device. */
int path_cache_info(const RprPathCache* cache, RprPathCacheInfo* out);

/* ------------------------------------------------------------ SH reverberator
 * The reverberator that renders the late reverberation from the estimated
 * parameters (Section 4.1 "Sound Rendering"; Section 4.2 for the comb gains
 * of Eq. 7, the comb delays and the predelay; Section 5 "Auralization" for 8
 * combs and 4 all-passes).  Per source and band, 8 feedback combs in parallel
 * take the band audio x_b, each comb i with delay M_i, input gains a_i (the
 * real SH of its input direction over 8) and feedback matrix g_b,i J_i (an SH
 * rotation times the Eq. 7 gain):  y_i[n] = a_i x_b[n - M_i] + g_b,i J_i
 * y_i[n - M_i].  Their sum passes 4 Schroeder all-passes per SH channel
 * (delays 4.9, 4.1, 3.4, 2.9 ms, gain 0.7), then the directional-loudness
 * matrix D_b and the gain g_reverb,b; the bands are summed into
 * (sh_order+1)^2 output channels.  The input is the band audio read at the
 * predelay tap of the caller's delay line. */
#define RPR_REVERB_COMBS 8
#define RPR_REVERB_ALLPASS 4

typedef struct {
    int32_t n_bands;        /* 1..RPR_MAX_BANDS */
    int32_t sh_order;       /* 0..RPR_MAX_SH_ORDER */
    float sample_rate;      /* Hz, 8000..192000 */
    float speed_of_sound;   /* m/s, > 0 */
    float max_comb_delay_s; /* comb delay capacity of the state, 0.005..2 s; longer delays are clamped */
    int32_t reserved;
} RprReverbDesc;

/* Parameters of one source's reverberator (device, written by reverb_setup). */
typedef struct {
    float t_comb[RPR_REVERB_COMBS];  /* seconds: mean free path / c (1 + z / 3), z clamped to [-2.7, 3],
                                        then clamped to [1 ms, max_comb_delay_s] */
    int32_t m_comb[RPR_REVERB_COMBS];/* samples: floor(t fs + 1/2) >= 1 */
    float mfp_drawn;                 /* mean free path of the last draw (m); 0 = none yet */
    int32_t predelay_samples;        /* floor(t_first fs + 1/2): the caller's input tap */
    int32_t n_bands;
    int32_t sh_order;
    float g_comb[RPR_MAX_BANDS][RPR_REVERB_COMBS]; /* Eq. 7: 10^(-3 t / RT60); 0 if RT60 <= 0 */
    float g_reverb[RPR_MAX_BANDS];                 /* Eq. 5 with Eq. 8 */
    float dir[RPR_REVERB_COMBS][4];                /* input direction (x, y, z, 1), or (0, 0, 0, 0) */
    float a[RPR_REVERB_COMBS][RPR_MAX_COEFFS];     /* comb input gains */
    float J[RPR_REVERB_COMBS][RPR_MAX_COEFFS][RPR_MAX_COEFFS]; /* SH rotation of each comb's feedback */
    float D[RPR_MAX_BANDS][RPR_MAX_COEFFS][RPR_MAX_COEFFS];   /* directional loudness */
} RprReverbSetup;

/* Bytes of rendering state one source needs (comb and all-pass delay lines
 * plus a 64-byte header), for the given description.  Returns RPR_EINVAL for
 * a description out of range. */
int reverb_state_bytes(const RprReverbDesc* desc /* host */, int64_t* bytes_per_source /* host */);

/* Zero the state of n_src sources (device, n_src * bytes_per_source bytes,
 * 16-byte aligned), e.g. before the first render or to silence them. */
int reverb_state_reset(void* state, int32_t n_src, const RprReverbDesc* desc, void* hip_stream);

/* Reverberator parameters of n_ir sources from their reverb estimates
 * (Section 4.1, Section 4.2):
 *   - comb delays drawn from the caller's standard normals z (device
 *     [n_ir][8] f32) around mean_free_path_m / c with sigma a third of that;
 *     with first = 0 the delays in setup[i] are kept while mean_free_path_m /
 *     c stays within 2 sigma of the mean of their draw, and also when
 *     mean_free_path_m <= 0;
 *   - Eq. 7 gains per band from rt60; g_reverb copied;
 *   - input direction of comb i from hist (device [n_ir][n_bins][n_bands]
 *     [(sh_order+1)^2] f32, the all-orders histogram) at t_first + t_comb,i,
 *     t_first = predelay_s (first_arrival_s if that is < 0, else 0): the
 *     band-summed first-order coefficients, linear between bin starts, zero
 *     past the last bin; direction (-X_11, -X_1-1, X_10) normalised; a zero
 *     vector (or sh_order 0) gives an omnidirectional input a_i = Y_00 e_0 / 8;
 *   - J_i, the SH rotation of R_i = Rz(c) Ry(b) Rx(a) with angles (a, b, c)
 *     from the caller (device [n_ir][8][3] f32, radians), built by exact
 *     quadrature of Y_k(R v) Y_k'(v) over the sphere;
 *   - D_b = sum_q w_q g_b(v_q) Y(v_q) Y(v_q)^T, g_b = sqrt(max(0, 4 pi
 *     dir_loudness_b . Y)), over 8 Gauss-Legendre nodes in cos(theta) x 16
 *     azimuths; the identity where dir_loudness_b,00 <= 0.
 *   params device [n_ir]; setup device [n_ir], read (first = 0) and written.
 *   The histogram's SH order and band count are desc's. */
int reverb_setup(const RprReverbParams* params, const float* hist, int32_t n_ir, int32_t n_bins, float bin_width_s,
                 const float* z, const float* angles, int32_t first, const RprReverbDesc* desc,
                 RprReverbSetup* setup, void* hip_stream);

/* Render n samples of n_src reverberators.
 *   setup device [n_src] (from reverb_setup with the same desc)
 *   x     device [n_src][n_bands][n] f32: band audio at each source's predelay tap
 *   state device [n_src] x bytes_per_source, 16-byte aligned: delay lines and
 *         their positions, carried from call to call (zeroed by
 *         reverb_state_reset); one source's state must not be rendered by two
 *         calls at once
 *   out   device [n_src][(sh_order+1)^2][n] f32, overwritten
 * Consecutive calls continue the same output stream.  A comb whose delay
 * changes between calls keeps the contents of its delay line.  n >= 0; n = 0
 * (or n_src = 0) does nothing. */
int reverb_render(const RprReverbSetup* setup, int32_t n_src, const float* x, int32_t n, void* state, float* out,
                  const RprReverbDesc* desc, void* hip_stream);

/* Closest hit of arbitrary rays against the scene's BVH, with the same
 * traversal and triangle test as trace_ir (no triangle excluded).
 *   orig, dir device [n][3] f32;  t_out device [n] f32 (INFINITY on a miss);
 *   tri_out device [n] i32 (original triangle index, -1 on a miss). */
int scene_closest_hit(const RprScene* scene, const float* orig, const float* dir, int64_t n,
                      float* t_out, int32_t* tri_out, void* hip_stream);

/* Memory-hierarchy probe: one launch that reads a working set the way the
 * BVH traversal does, to measure the roof the traversal runs under (Table 1:
 * ray tracing is nearly all of the propagation update, and its bytes are
 * node lines and triangle records read from the cache hierarchy).
 *   buf      device, `bytes` bytes (a multiple of 128, 16-byte aligned): the
 *            working set; its contents are only summed
 *   pattern  0 streaming: coalesced 16-byte reads, grid-stride, `iters` passes
 *            over the buffer (bytes read: iters x bytes);
 *            1 gather: each thread reads `iters` whole 128-byte lines at
 *            pseudo-random line indices, independent of the data (bytes read:
 *            grid x block x iters x 128);
 *            2 chase: as 1, each index depending on the previous line's data
 *            (one line in flight per thread: latency)
 *   grid, block  launch shape; block a multiple of 64, at most 1024
 *   sink     device [grid x block] f32, overwritten (keeps the reads alive)
 * Enqueues one kernel on the stream; the caller times it (events on that
 * stream).  Errors: RPR_EINVAL for a bad size, pattern or shape. */
int memory_probe(const void* buf, int64_t bytes, int32_t pattern, int32_t iters, int32_t grid, int32_t block,
                 float* sink, void* hip_stream);

/* Device implementations of the shared primitives, exposed for unit checks.
 * debug_philox: in device [n][6] u32 = ctr0..3, key0..1; out device [n][4].
 * debug_sh_eval: dirs device [n][3] f32 (unit), out device [n][16] f32 (the
 * first (order+1)^2 entries written, real SH with the Condon-Shortley phase,
 * index l(l+1)+m). */
int debug_philox(const uint32_t* in, int64_t n, uint32_t* out, void* hip_stream);
int debug_sh_eval(const float* dirs, int64_t n, int32_t order, float* out, void* hip_stream);

/* Thread-local message describing the last non-zero status. */
const char* last_error(void);
/* Library version string. */
const char* rpr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPR_H */
