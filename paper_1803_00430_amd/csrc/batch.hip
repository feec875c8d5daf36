// Batches: many source-listener pairs over several scenes in one persistent
// trace launch.
//
// The pair table (one PairDesc per pair, each pointing at its scene's BVH and
// at its slices of the caller's output buffers) is uploaded once.  A run is
// four launches on one stream -- reset the statistics and the ray queue, zero
// the histograms, trace every ray of every pair through the shared queue,
// estimate every pair -- which can be captured into a HIP graph and replayed.
//
// Launch shape: the resident waves per compute unit, the order in which
// pairs enter the queue (as given; most rays x bounces first, so that the
// longest pairs start early and the tail is shorter; or interleaved chunks)
// and the chunk size of the interleaved order and of the listener method's
// chunk table.  The autotuner times every candidate shape on the batch
// itself and keeps the fastest; the choice is cached per key (see tune_key),
// in memory and, when RPR_AUTOTUNE_CACHE names a file, on disk.  Results do
// not depend on the shape: every ray is a function of (pair, ray id).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "rpr_internal.hpp"

struct RprBatch {
    int device = 0;
    int n_pairs = 0, nb = 0, nc = 0, T = 0, sh_order = 0;
    float dt = 0.f;
    int64_t total = 0;
    int stack_need = 0;
    int stack_launch = 0;  // stack bound the launches take (at least stack_need: a deeper variant)
    int waves_per_cu = 0, order = 0;
    int64_t chunk = 1024;  // rays per chunk (interleaved order, listener chunk table)
    int method = 0;        // 0 source-origin, 1 listener-origin
    RprEstimateParams ep{0, 3};
    std::vector<rpr::PairDesc> pairs;  // caller order
    rpr::PairDesc* d_pairs = nullptr;  // queue order (pairs, or chunks of pairs when interleaved)
    int n_table = 0;                   // descriptors in d_pairs
    int64_t table_cap = 0;
    unsigned long long* d_queue = nullptr;
    float* hist = nullptr;
    float* hist_late = nullptr;
    RprIrStats* stats = nullptr;
    RprReverbParams* params = nullptr;
    long long* fx = nullptr;       // the fixed-point cells while deposits are in fixed point, else null
    long long* fx_mem = nullptr;   // fixed-point cells [n_pairs][T][B][NC] then [n_pairs][T][B], once allocated
    double* fx_scales = nullptr;   // device [n_pairs]
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    RprBatchInfo info{};
};

namespace rpr {
namespace {

// The tuning cache: key -> (waves per CU, queue order, chunk rays, stack
// bound the launches take, fixed-point deposits).
struct TuneChoice {
    int waves_per_cu, order, chunk, stack, fixed;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;
bool g_tune_file_read = false;

constexpr int kChunkChoices[3] = {256, 1024, 4096};

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

// What a launch shape's speed depends on: the device (architecture, CUs), the
// kernel variant (method, bands, stack variant), the per-ray work (bins, SH
// coefficients, mean bounces, scene size) and the amount of work (pairs,
// total rays), the continuous ones as log2 buckets.
std::string tune_key(int device, const RprBatch& b, int64_t max_tris)
{
    hipDeviceProp_t prop;
    const char* arch = hipGetDeviceProperties(&prop, device) == hipSuccess ? prop.gcnArchName : "unknown";
    double bounces = 0.0;
    for (const auto& d : b.pairs) bounces += (double)d.n_rays * (d.max_bounces + 1);
    bounces /= (double)std::max<int64_t>(1, b.total);
    char buf[256];
    const int stack = b.stack_need < 32 ? 32 : (b.stack_need < 48 ? 48 : 64);
    std::snprintf(buf, sizeof(buf), "%s/cu%d/m%d/nb%d/T%d/nc%d/st%d/p%d/r%d/k%d/t%d", arch, device_cu_count(),
                  b.method, b.nb, b.T, b.nc, stack, ilog2(b.n_pairs), ilog2((double)b.total), ilog2(bounces),
                  ilog2((double)max_tris));
    std::string k(buf);
    for (char& c : k)
        if (c == ' ') c = '_';
    return k;
}

// Read the file cache once (lines: key waves order chunk stack fixed); called
// with g_tune_mu held.
void tune_file_read()
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = std::getenv("RPR_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    int w, o, c, s, x;
    while (std::fscanf(f, "%255s %d %d %d %d %d", key, &w, &o, &c, &s, &x) == 6)
        if (w >= 1 && o >= 0 && o <= 2 && (c == 256 || c == 1024 || c == 4096) && s >= 0 && s < kMaxStack &&
            (x == 0 || x == 1))
            g_tune_cache[key] = TuneChoice{w, o, c, s, x};
    std::fclose(f);
}

// Rewrite the file cache with every known choice; called with g_tune_mu held.
void tune_file_write()
{
    const char* path = std::getenv("RPR_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto& kv : g_tune_cache)
        std::fprintf(f, "%s %d %d %d %d %d\n", kv.first.c_str(), kv.second.waves_per_cu, kv.second.order,
                     kv.second.chunk, kv.second.stack, kv.second.fixed);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
}

// Upload the pair table in queue order `ord` (indices into b.pairs): 0 as
// given, 1 most rays x bounces first, 2 interleaved -- every pair split into
// chunks of b.chunk rays, dealt round-robin across the pairs, so that the
// resident waves work on many pairs' histograms at once instead of
// contending for the atomics of a few.  A chunk is a copy of its pair's
// descriptor with its own ray range; the energy normalisation, outputs and
// statistics stay the pair's.  The listener-origin kernel always takes a
// table of chunks (one wave per chunk), in pair order for orders 0 and 1.
int upload_order(RprBatch& b, int ord, hipStream_t st)
{
    std::vector<int> idx(b.n_pairs);
    std::iota(idx.begin(), idx.end(), 0);
    if (ord == 1) {
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
            const double cx = (double)b.pairs[x].n_rays * (b.pairs[x].max_bounces + 1);
            const double cy = (double)b.pairs[y].n_rays * (b.pairs[y].max_bounces + 1);
            return cx > cy;
        });
    }
    std::vector<PairDesc> q;
    if (ord != 2 && b.method == 1) {
        for (int i = 0; i < b.n_pairs; ++i) {
            const PairDesc& P = b.pairs[idx[i]];
            for (int64_t o = 0; o < P.n_rays; o += b.chunk) {
                PairDesc c = P;
                c.ray_begin = P.ray_begin + o;
                c.n_rays = std::min(b.chunk, P.n_rays - o);
                q.push_back(c);
            }
        }
    } else if (ord == 2) {
        std::vector<int64_t> next(b.n_pairs, 0);
        for (bool more = true; more;) {
            more = false;
            for (int i = 0; i < b.n_pairs; ++i) {
                const PairDesc& P = b.pairs[i];
                if (next[i] >= P.n_rays) continue;
                PairDesc c = P;
                c.ray_begin = P.ray_begin + next[i];
                c.n_rays = std::min(b.chunk, P.n_rays - next[i]);
                next[i] += c.n_rays;
                q.push_back(c);
                more = more || next[i] < P.n_rays;
            }
        }
    } else {
        for (int i = 0; i < b.n_pairs; ++i) q.push_back(b.pairs[idx[i]]);
    }
    int64_t off = 0;
    for (auto& d : q) {
        d.queue_begin = off;
        off += d.n_rays;
    }
    if ((int64_t)q.size() > b.table_cap) {
        if (b.d_pairs) (void)hipFree(b.d_pairs);
        b.d_pairs = nullptr;
        b.table_cap = 0;
        RPR_HIP_TRY(hipMalloc(&b.d_pairs, sizeof(PairDesc) * q.size()));
        b.table_cap = (int64_t)q.size();
    }
    RPR_HIP_TRY(hipMemcpyAsync(b.d_pairs, q.data(), sizeof(PairDesc) * q.size(), hipMemcpyHostToDevice, st));
    RPR_HIP_TRY(hipStreamSynchronize(st));
    b.n_table = (int)q.size();
    b.order = ord;
    return RPR_OK;
}

// Deposits in 64-bit fixed point (RPR_TRACE_DETERMINISTIC's cells, allocated
// on first use, released when FP32 deposits are chosen again) or in FP32
// atomics: points the pair descriptors at the cells or not; upload_order then
// carries the change to the device table.
int set_deposit(RprBatch& b, bool fixed)
{
    const size_t hstride = (size_t)b.T * b.nb * b.nc, lstride = (size_t)b.T * b.nb;
    if (!fixed && b.fx_mem) {
        RPR_HIP_TRY(hipFree(b.fx_mem));
        RPR_HIP_TRY(hipFree(b.fx_scales));
        b.fx_mem = nullptr;
        b.fx_scales = nullptr;
    }
    if (fixed && !b.fx_mem) {
        const size_t cells = (size_t)b.n_pairs * hstride + (b.hist_late ? (size_t)b.n_pairs * lstride : 0);
        RPR_HIP_TRY(hipMalloc(&b.fx_mem, sizeof(long long) * cells));
        RPR_HIP_TRY(hipMalloc(&b.fx_scales, sizeof(double) * b.n_pairs));
    }
    std::vector<double> scales(b.n_pairs);
    for (int i = 0; i < b.n_pairs; ++i) {
        // 2^61 x sphere volume / (4 x bands x bin width)
        const double r = b.pairs[i].radius;
        scales[i] = 0x1p61 * (4.0 / 3.0 * M_PI * r * r * r) / (4.0 * b.nb * (double)b.dt);
        PairDesc& d = b.pairs[i];
        d.hist_fx = fixed ? b.fx_mem + (size_t)i * hstride : nullptr;
        d.late_fx = fixed && b.hist_late ? b.fx_mem + (size_t)b.n_pairs * hstride + (size_t)i * lstride : nullptr;
        d.fx_scale = fixed ? scales[i] : 0.0;
    }
    if (fixed) RPR_HIP_TRY(hipMemcpy(b.fx_scales, scales.data(), sizeof(double) * b.n_pairs, hipMemcpyHostToDevice));
    b.fx = fixed ? b.fx_mem : nullptr;
    return RPR_OK;
}

int enqueue_run(RprBatch& b, hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr)
{
    int rc = enqueue_stats_reset(b.stats, b.n_pairs, b.d_queue, st);
    if (rc != RPR_OK) return rc;
    rc = enqueue_fill_zero(b.hist, (size_t)b.n_pairs * b.T * b.nb * b.nc, st);
    if (rc != RPR_OK) return rc;
    const size_t hn = (size_t)b.n_pairs * b.T * b.nb * b.nc, ln = b.hist_late ? (size_t)b.n_pairs * b.T * b.nb : 0;
    if (b.fx) {
        rc = enqueue_fill_zero((float*)b.fx, 2 * (hn + ln), st);  // zero bits, as floats
        if (rc != RPR_OK) return rc;
    }
    if (b.hist_late) {
        rc = enqueue_fill_zero(b.hist_late, (size_t)b.n_pairs * b.T * b.nb, st);
        if (rc != RPR_OK) return rc;
    }
    if (t0) RPR_HIP_TRY(hipEventRecord(t0, st));
    rc = b.method == 1
             ? launch_trace_listener_pairs(b.d_pairs, b.n_table, b.d_queue, b.total, b.nb, b.stack_launch,
                                           b.waves_per_cu, st)
             : launch_trace(b.d_pairs, b.n_table, b.d_queue, b.total, b.nb, b.stack_launch, false, b.waves_per_cu,
                            0, st);
    if (rc != RPR_OK) return rc;
    if (b.fx) {
        rc = enqueue_fx_convert(b.fx, b.hist, (long long)b.T * b.nb * b.nc, b.n_pairs, b.fx_scales, 0.0, st);
        if (rc == RPR_OK && b.hist_late)
            rc = enqueue_fx_convert(b.fx + hn, b.hist_late, (long long)b.T * b.nb, b.n_pairs, b.fx_scales, 0.0, st);
        if (rc != RPR_OK) return rc;
    }
    if (t1) RPR_HIP_TRY(hipEventRecord(t1, st));
    return estimate_reverb(b.hist, b.hist_late, b.stats, b.n_pairs, b.T, b.nb, b.sh_order, b.dt, &b.ep, b.params,
                           st);
}

// Time the trace of one run with the current shape (best of `reps`).
int time_shape(RprBatch& b, hipStream_t st, int reps, float& best_ms)
{
    hipEvent_t e0, e1;
    RPR_HIP_TRY(hipEventCreate(&e0));
    RPR_HIP_TRY(hipEventCreate(&e1));
    best_ms = 1e30f;
    int rc = RPR_OK;
    for (int r = 0; r < reps && rc == RPR_OK; ++r) {
        rc = enqueue_run(b, st, e0, e1);
        if (rc != RPR_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = set_error(RPR_EDEVICE, "batch autotune: event wait failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 || reps == 1) best_ms = std::min(best_ms, ms);  // the first run warms the caches
    }
    if (rc == RPR_OK && hipStreamSynchronize(st) != hipSuccess) rc = set_error(RPR_EDEVICE, "batch autotune sync");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

void batch_free(RprBatch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_pairs) (void)hipFree(b->d_pairs);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->fx_mem) (void)hipFree(b->fx_mem);
    if (b->fx_scales) (void)hipFree(b->fx_scales);
    delete b;
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int batch_create(const RprScene* const* scenes, int32_t n_scenes, const RprPair* pairs, int32_t n_pairs,
                            const RprBatchParams* bp, float* hist, float* hist_late, RprIrStats* stats,
                            RprReverbParams* params, void* hip_stream, RprBatch** out)
{
    if (!out) return set_error(RPR_EINVAL, "batch_create: out is null");
    *out = nullptr;
    if (!scenes || n_scenes < 1 || !pairs || n_pairs < 1 || !bp || !hist || !stats || !params)
        return set_error(RPR_EINVAL, "batch_create: null or empty argument");
    if (bp->n_bins < 1 || bp->sh_order < 0 || bp->sh_order > RPR_MAX_SH_ORDER || !(bp->bin_width_s > 0.f) ||
        !(bp->speed_of_sound > 0.f) || bp->waves_per_cu < 0 || bp->order < 0 || bp->order > 2 ||
        bp->tail_iters < 0 || bp->tail_iters > 100 || (bp->rt60_source != 0 && bp->rt60_source != 1) ||
        (bp->rt60_source == 1 && !hist_late) || (bp->method != 0 && bp->method != 1) ||
        (bp->chunk_rays != 0 && bp->chunk_rays != 256 && bp->chunk_rays != 1024 && bp->chunk_rays != 4096) ||
        (bp->deterministic != 0 && bp->deterministic != 1) || (bp->deterministic && bp->method != 0))
        return set_error(RPR_EINVAL, "batch_create: bad batch parameters");
    for (int i = 0; i < n_scenes; ++i)
        if (scenes[i])
            if (const int rc = scene_settle(scenes[i]); rc != RPR_OK) return rc;
    const int nb = scenes[0] ? scenes[0]->n_bands : 0;
    int stack_need = 1;
    int64_t max_tris = 0;
    for (int i = 0; i < n_scenes; ++i) {
        if (!scenes[i]) return set_error(RPR_EINVAL, "batch_create: scene %d is null", i);
        if (scenes[i]->n_bands != nb) return set_error(RPR_EINVAL, "batch_create: scenes differ in band count");
        stack_need = std::max(stack_need, scenes[i]->stack_need);
        max_tris = std::max(max_tris, scenes[i]->n_tris);
    }
    const int nc = (bp->sh_order + 1) * (bp->sh_order + 1);
    int64_t total = 0;
    for (int i = 0; i < n_pairs; ++i) {
        const RprPair& p = pairs[i];
        if (p.scene < 0 || p.scene >= n_scenes) return set_error(RPR_EINVAL, "batch_create: pair %d scene index", i);
        if (p.n_rays < 1 || p.n_rays > ((int64_t)1 << 32) || p.max_bounces < 0 || p.max_bounces > 10000000 ||
            !(p.radius > 0.f) || !std::isfinite(p.radius))
            return set_error(RPR_EINVAL, "batch_create: pair %d parameters", i);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(p.src[a]) || !std::isfinite(p.lst[a]))
                return set_error(RPR_EINVAL, "batch_create: pair %d position", i);
        total += p.n_rays;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    RprBatch* b = new RprBatch();
    RPR_HIP_TRY(hipGetDevice(&b->device));
    b->n_pairs = n_pairs;
    b->nb = nb;
    b->nc = nc;
    b->T = bp->n_bins;
    b->sh_order = bp->sh_order;
    b->dt = bp->bin_width_s;
    b->total = total;
    b->stack_need = stack_need;
    b->method = bp->method;
    b->ep = RprEstimateParams{bp->rt60_source, bp->tail_iters};
    b->hist = hist;
    b->hist_late = hist_late;
    b->stats = stats;
    b->params = params;
    b->pairs.resize(n_pairs);
    const size_t hstride = (size_t)bp->n_bins * nb * nc, lstride = (size_t)bp->n_bins * nb;
    for (int i = 0; i < n_pairs; ++i) {
        const RprPair& p = pairs[i];
        PairDesc d;
        std::memset(&d, 0, sizeof(d));
        d.scene = scenes[p.scene]->view;
        for (int a = 0; a < 3; ++a) {
            d.src[a] = p.src[a];
            d.lst[a] = p.lst[a];
        }
        d.radius = p.radius;
        d.inv_vs = (float)(1.0 / (4.0 / 3.0 * M_PI * (double)p.radius * p.radius * p.radius));
        d.c = bp->speed_of_sound;
        d.dt = bp->bin_width_s;
        d.l_window = (float)((double)bp->speed_of_sound * (double)bp->n_bins * (double)bp->bin_width_s);
        d.e0 = (float)(1.0 / (double)p.n_rays);
        d.n_bins = bp->n_bins;
        d.max_bounces = p.max_bounces;
        d.sh_order = bp->sh_order;
        d.n_coeffs = nc;
        d.key0 = (uint32_t)(p.seed & 0xFFFFFFFFull);
        d.key1 = (uint32_t)(p.seed >> 32);
        d.pair_id = (uint32_t)p.pair_id;
        d.ray_begin = 0;
        d.n_rays = p.n_rays;
        d.hist = hist + (size_t)i * hstride;
        d.hist_late = hist_late ? hist_late + (size_t)i * lstride : nullptr;
        d.stats = stats + i;
        d.ray_hash = nullptr;
        b->pairs[i] = d;
    }
    auto fail = [&](int code) {
        batch_free(b);
        return code;
    };
    if (bp->deterministic) {
        const int rc0 = set_deposit(*b, true);
        if (rc0 != RPR_OK) return fail(rc0);
    }
    if (hipMalloc(&b->d_queue, 256) != hipSuccess)
        return fail(set_error(RPR_ENOMEM, "batch_create: device allocation failed"));
    if (device_cu_count() <= 0) return fail(set_error(RPR_EDEVICE, "batch_create: no device"));
    // stack bounds the launches may take: the scene's own, or one that selects a
    // deeper stack variant (more LDS per wave, fewer waves per CU)
    auto max_wpc_for = [&](int stack) {
        return bp->method == 1 ? trace_listener_max_waves_per_cu(nb, stack) : trace_max_waves_per_cu(nb, stack);
    };
    std::vector<int> stacks = {stack_need};
    if (stack_need < 32) stacks.push_back(47);
    if (stack_need < 48) stacks.push_back(63);
    b->stack_launch = stack_need;
    const int max_wpc = max_wpc_for(stack_need);

    // launch shape: cached, autotuned or as requested
    int rc = RPR_OK;
    b->info.n_candidates = 0;
    b->info.from_cache = 0;
    if (bp->autotune) {
        const std::string key = tune_key(b->device, *b, max_tris);
        bool cached = false;
        TuneChoice pick{max_wpc, 0, 1024, stack_need, bp->deterministic ? 1 : 0};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_file_read();
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                pick = it->second;
                cached = true;
            }
        }
        if (cached) {
            b->info.from_cache = 1;
            if (std::find(stacks.begin(), stacks.end(), pick.stack) == stacks.end()) pick.stack = stack_need;
            pick.fixed = bp->deterministic || (pick.fixed && bp->method == 0) ? 1 : 0;
        } else {
            auto widths_for = [](int mw) {
                std::vector<int> widths;
                for (int w : {mw / 4, mw / 2, (3 * mw) / 4, mw})
                    if (w >= 1 && std::find(widths.begin(), widths.end(), w) == widths.end()) widths.push_back(w);
                return widths;
            };
            float best = 1e30f, worst = 0.f;
            auto time_width = [&](int w, float& ms) {
                b->waves_per_cu = w;
                const int rc1 = time_shape(*b, st, 3, ms);
                if (rc1 != RPR_OK) return rc1;
                ++b->info.n_candidates;
                worst = std::max(worst, ms);
                return RPR_OK;
            };
            // stage 1: widths x queue orders x chunk sizes, on the scene's own stack bound
            for (int o = 0; o < 3; ++o) {
                // the chunk size matters to the interleaved order and to the listener method's chunk table
                const bool chunked = o == 2 || b->method == 1;
                for (int ci = 0; ci < (chunked ? 3 : 1); ++ci) {
                    b->chunk = chunked ? kChunkChoices[ci] : 1024;
                    rc = upload_order(*b, o, st);
                    if (rc != RPR_OK) return fail(rc);
                    for (int w : widths_for(max_wpc)) {
                        float ms = 0.f;
                        rc = time_width(w, ms);
                        if (rc != RPR_OK) return fail(rc);
                        if (ms < best) {
                            best = ms;
                            pick = TuneChoice{w, o, (int)b->chunk, stack_need, pick.fixed};
                        }
                    }
                }
            }
            // stage 2: the deeper stack variants, at the best order and chunk size
            b->chunk = pick.chunk;
            rc = upload_order(*b, pick.order, st);
            if (rc != RPR_OK) return fail(rc);
            for (size_t si = 1; si < stacks.size(); ++si) {
                b->stack_launch = stacks[si];
                for (int w : widths_for(max_wpc_for(stacks[si]))) {
                    float ms = 0.f;
                    rc = time_width(w, ms);
                    if (rc != RPR_OK) return fail(rc);
                    if (ms < best) {
                        best = ms;
                        pick.waves_per_cu = w;
                        pick.stack = stacks[si];
                    }
                }
            }
            // stage 3: 64-bit fixed-point deposits at the best shape (unless already asked
            // for); skipped when the cells do not fit in device memory
            if (bp->method == 0 && !bp->deterministic) {
                b->stack_launch = pick.stack;
                if (set_deposit(*b, true) == RPR_OK) {
                    rc = upload_order(*b, pick.order, st);
                    float ms = 0.f;
                    if (rc == RPR_OK) rc = time_width(pick.waves_per_cu, ms);
                    if (rc != RPR_OK) return fail(rc);
                    if (ms < best) {
                        best = ms;
                        pick.fixed = 1;
                    }
                } else {
                    (void)hipGetLastError();
                    rc = RPR_OK;
                }
            }
            b->info.best_ms = best;
            b->info.worst_ms = worst;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = pick;
            tune_file_write();
        }
        b->stack_launch = pick.stack;
        b->waves_per_cu = std::min(pick.waves_per_cu, max_wpc_for(pick.stack));
        b->chunk = pick.chunk;
        rc = set_deposit(*b, pick.fixed != 0);
        if (rc == RPR_OK) rc = upload_order(*b, pick.order, st);
        if (rc != RPR_OK) return fail(rc);
    } else {
        b->waves_per_cu = bp->waves_per_cu > 0 ? std::min(bp->waves_per_cu, max_wpc) : max_wpc;
        b->chunk = bp->chunk_rays > 0 ? bp->chunk_rays : 1024;
        rc = upload_order(*b, bp->order, st);
        if (rc != RPR_OK) return fail(rc);
    }

    if (bp->use_graph) {
        hipStream_t cap;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
            return fail(set_error(RPR_EDEVICE, "batch_create: stream creation failed"));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = enqueue_run(*b, cap);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cap, &g);
            if (rc == RPR_OK && e2 != hipSuccess) rc = set_error(RPR_EDEVICE, "batch_create: capture failed");
            b->graph = g;
            if (rc == RPR_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
                rc = set_error(RPR_EDEVICE, "batch_create: graph instantiation failed");
        } else {
            rc = set_error(RPR_EDEVICE, "batch_create: capture could not start");
        }
        (void)hipStreamDestroy(cap);
        if (rc != RPR_OK) return fail(rc);
    }
    b->info.total_rays = total;
    b->info.n_pairs = n_pairs;
    b->info.waves_per_cu = b->waves_per_cu;
    b->info.order = b->order;
    b->info.stack_need = stack_need;
    b->info.graph = b->exec ? 1 : 0;
    b->info.chunk_rays = (int32_t)b->chunk;
    b->info.stack_entries = b->stack_launch < 32 ? 32 : (b->stack_launch < 48 ? 48 : 64);
    b->info.fixed_point = b->fx ? 1 : 0;
    *out = b;
    return RPR_OK;
}

extern "C" int batch_run(RprBatch* batch, void* hip_stream)
{
    if (!batch) return set_error(RPR_EINVAL, "batch_run: null batch");
    hipStream_t st = (hipStream_t)hip_stream;
    if (batch->exec) {
        RPR_HIP_TRY(hipGraphLaunch(batch->exec, st));
        return RPR_OK;
    }
    return enqueue_run(*batch, st);
}

extern "C" int batch_info(const RprBatch* batch, RprBatchInfo* out)
{
    if (!batch || !out) return set_error(RPR_EINVAL, "batch_info: null argument");
    *out = batch->info;
    return RPR_OK;
}

extern "C" int batch_destroy(RprBatch* batch)
{
    if (!batch) return RPR_OK;
    (void)hipDeviceSynchronize();
    batch_free(batch);
    return RPR_OK;
}
