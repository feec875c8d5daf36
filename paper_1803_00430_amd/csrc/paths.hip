// Early-reflection paths across frames: the diffuse path cache and the
// prioritization for rendering (Section 5: the first two reflection orders
// with the diffuse path cache, augmented with SH directivity per path; paths
// below the threshold of hearing are discarded, the N_ER strongest among all
// sources are rendered, the others are added to the late IR before it is
// analysed).
//
// A path is identified by the 64-bit key of its records (source, order and
// the triangles of its reflections; trace_ir_paths).  The cache is a list of
// (key, payload) with payload = band intensity, intensity x arrival time and
// SH directivity.  A frame's update rebuilds it through a hash table (linear
// probing, keys claimed with 64-bit compare-and-swap, payloads accumulated
// with atomic adds): the cached paths enter scaled by 1 - alpha, the frame's
// records by alpha, and the paths at or above min_energy are compacted into
// the new list.  The selection ranks the paths exactly (each against all
// others, in LDS tiles; ties by key) and writes the first N_ER in rank order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rpr_internal.hpp"

static_assert(sizeof(RprEarlyPath) == 128, "RprEarlyPath layout");

namespace rpr {
namespace {

constexpr int kPay = 28;          // payload words: e[8], e*t, d[16], 3 spare
constexpr int kPayE = 0, kPayET = 8, kPayD = 9;
constexpr uint64_t kEmpty = 0ull; // no valid key is 0 (the order field is 1 or 2)

__device__ __forceinline__ uint32_t mix64(uint64_t x)
{
    x ^= x >> 31;
    x *= 0x9E3779B97F4A7C15ull;
    x ^= x >> 29;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 32;
    return (uint32_t)x;
}

// Slot of `key` in the table (claimed if absent), or -1 when the table is full.
__device__ int table_slot(unsigned long long* __restrict__ tkeys, uint32_t mask, uint64_t key,
                          int* __restrict__ overflow)
{
    uint32_t h = mix64(key) & mask;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long prev = atomicCAS(tkeys + h, (unsigned long long)kEmpty, (unsigned long long)key);
        if (prev == kEmpty || prev == key) return (int)h;
        h = (h + 1) & mask;
    }
    atomicOr(overflow, 1);
    return -1;
}

__global__ void k_pc_clear(unsigned long long* __restrict__ tkeys, float* __restrict__ tvals, uint32_t n,
                           int* __restrict__ count)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        tkeys[i] = kEmpty;
        for (int w = 0; w < kPay; ++w) tvals[(size_t)i * kPay + w] = 0.f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

__global__ void k_pc_insert_list(const unsigned long long* __restrict__ keys, const float* __restrict__ vals,
                                 const int* __restrict__ count, int cap, float scale,
                                 unsigned long long* __restrict__ tkeys, float* __restrict__ tvals, uint32_t mask,
                                 int* __restrict__ overflow)
{
    const int n = std::min(*count, cap);  // the compaction counts past the capacity when it overflows
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int h = table_slot(tkeys, mask, keys[i], overflow);
        if (h < 0) continue;
        for (int w = 0; w < kPay; ++w) atomicAdd(tvals + (size_t)h * kPay + w, scale * vals[(size_t)i * kPay + w]);
    }
}

__global__ void k_pc_insert_records(const float* __restrict__ rec, const uint32_t* __restrict__ n_rec, int max_rec,
                                    float scale, unsigned long long* __restrict__ tkeys, float* __restrict__ tvals,
                                    uint32_t mask, int* __restrict__ overflow)
{
    const int n = (int)std::min<uint32_t>(*n_rec, (uint32_t)max_rec);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float* r = rec + (size_t)i * kRecWords;
        const uint64_t key = (uint64_t)__float_as_uint(r[0]) | ((uint64_t)__float_as_uint(r[1]) << 32);
        if (key == kEmpty) continue;
        const int h = table_slot(tkeys, mask, key, overflow);
        if (h < 0) continue;
        float* v = tvals + (size_t)h * kPay;
        float et = 0.f;
        for (int b = 0; b < RPR_MAX_BANDS; ++b) {
            atomicAdd(v + kPayE + b, scale * r[2 + b]);
            et += r[2 + b];
        }
        atomicAdd(v + kPayET, scale * et * r[10]);
        for (int k = 0; k < RPR_MAX_COEFFS; ++k) atomicAdd(v + kPayD + k, scale * r[11 + k]);
    }
}

__global__ void k_pc_compact(const unsigned long long* __restrict__ tkeys, const float* __restrict__ tvals,
                             uint32_t n, float min_energy, unsigned long long* __restrict__ keys,
                             float* __restrict__ vals, int* __restrict__ count, int cap, int* __restrict__ overflow)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t key = tkeys[i];
        if (key == kEmpty) continue;
        const float* v = tvals + (size_t)i * kPay;
        float e = 0.f;
        for (int b = 0; b < RPR_MAX_BANDS; ++b) e += v[kPayE + b];
        if (!(e >= min_energy)) continue;
        const int j = atomicAdd(count, 1);
        if (j >= cap) {
            atomicOr(overflow, 1);
            continue;
        }
        keys[j] = key;
        for (int w = 0; w < kPay; ++w) vals[(size_t)j * kPay + w] = v[w];
    }
}

constexpr int kRankTile = 256;

// Rank of every path among the eligible ones (total intensity >= threshold):
// the number with a larger intensity, or an equal one and a smaller key.
__global__ __launch_bounds__(kRankTile) void k_pc_select(
    const unsigned long long* __restrict__ keys, const float* __restrict__ vals, const int* __restrict__ count,
    int cap, float threshold, int n_er, RprEarlyPath* __restrict__ out, int* __restrict__ n_eligible,
    float* __restrict__ hist_late, RprIrStats* __restrict__ stats, int n_src, int n_bins, int nb, float dt)
{
    __shared__ float s_I[kRankTile];
    __shared__ unsigned long long s_k[kRankTile];
    const int n = std::min(*count, cap);
    const int i = blockIdx.x * kRankTile + threadIdx.x;
    float Ii = -1.f;
    uint64_t ki = 0;
    if (i < n) {
        ki = keys[i];
        float e = 0.f;
        for (int b = 0; b < RPR_MAX_BANDS; ++b) e += vals[(size_t)i * kPay + kPayE + b];
        Ii = e;
    }
    const bool elig = i < n && Ii >= threshold;
    int rank = 0;
    for (int t0 = 0; t0 < n; t0 += kRankTile) {
        const int j = t0 + threadIdx.x;
        float Ij = -1.f;
        unsigned long long kj = 0;
        if (j < n) {
            float e = 0.f;
            for (int b = 0; b < RPR_MAX_BANDS; ++b) e += vals[(size_t)j * kPay + kPayE + b];
            Ij = e;
            kj = keys[j];
        }
        __syncthreads();
        s_I[threadIdx.x] = Ij >= threshold ? Ij : -1.f;
        s_k[threadIdx.x] = kj;
        __syncthreads();
        if (elig) {
            const int m = std::min(kRankTile, n - t0);
            for (int q = 0; q < m; ++q) {
                const float Iq = s_I[q];
                rank += (Iq > Ii || (Iq == Ii && Iq >= 0.f && s_k[q] < ki)) ? 1 : 0;
            }
        }
    }
    if (!elig) return;
    atomicAdd(n_eligible, 1);
    const float* v = vals + (size_t)i * kPay;
    const int src = (int)(ki >> 48);
    if (rank < n_er) {
        RprEarlyPath p;
        p.source = src;
        p.order = (int)((ki >> 46) & 3u);
        const uint32_t t1 = (uint32_t)((ki >> 23) & kRecNoTri), t2 = (uint32_t)(ki & kRecNoTri);
        p.tri[0] = t1 == kRecNoTri ? -1 : (int)t1;
        p.tri[1] = t2 == kRecNoTri ? -1 : (int)t2;
        for (int b = 0; b < RPR_MAX_BANDS; ++b) p.e[b] = v[kPayE + b];
        p.t = Ii > 0.f ? v[kPayET] / Ii : 0.f;
        for (int k = 0; k < RPR_MAX_COEFFS; ++k) p.d[k] = v[kPayD + k];
        p.reserved[0] = p.reserved[1] = p.reserved[2] = 0.f;
        out[rank] = p;
        return;
    }
    // culled: the path joins the late class of its source
    if (src >= n_src) return;
    const float tm = Ii > 0.f ? v[kPayET] / Ii : 0.f;
    int m = (int)floorf(tm / dt);
    m = std::min(std::max(m, 0), n_bins - 1);
    for (int b = 0; b < nb; ++b) {
        const float e = v[kPayE + b];
        if (hist_late) atomicAdd(hist_late + ((size_t)src * n_bins + m) * nb + b, e);
        if (stats) {
            atomicAdd(&stats[src].e_class[1][b], -(double)e);
            atomicAdd(&stats[src].e_class[2][b], (double)e);
        }
    }
}

__global__ void k_pc_nout(const int* __restrict__ n_eligible, int n_er, int32_t* __restrict__ n_out)
{
    *n_out = std::min(*n_eligible, n_er);
}

__global__ void k_pc_zero(int* __restrict__ p, int n)
{
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

int grid_for(long long n) { return (int)std::max(1ll, std::min((n + 255) / 256, 8192ll)); }

}  // namespace
}  // namespace rpr

using namespace rpr;

struct RprPathCache {
    int device = 0;
    int32_t max_paths = 0;
    uint32_t table_size = 0;  // power of two >= 4 max_paths
    unsigned long long* keys[2] = {nullptr, nullptr};
    float* vals[2] = {nullptr, nullptr};
    unsigned long long* tkeys = nullptr;
    float* tvals = nullptr;
    int* ints = nullptr;      // [0..1] list counts, [2] overflow, [3] eligible count
    int cur = 0;              // the list holding the cache
};

extern "C" int path_cache_create(int32_t max_paths, RprPathCache** out)
{
    if (!out || max_paths < 1 || max_paths > (1 << 20)) return set_error(RPR_EINVAL, "path_cache_create: bad argument");
    *out = nullptr;
    int dev = 0;
    RPR_HIP_TRY(hipGetDevice(&dev));
    RprPathCache* c = new RprPathCache();
    c->device = dev;
    c->max_paths = max_paths;
    uint32_t t = 1;
    while (t < 4u * (uint32_t)max_paths) t <<= 1;
    c->table_size = t;
    int rc = RPR_OK;
    auto alloc = [&](void** p, size_t bytes) {
        if (rc != RPR_OK) return;
        if (hipMalloc(p, bytes) != hipSuccess) rc = set_error(RPR_ENOMEM, "path_cache_create: out of device memory");
    };
    for (int l = 0; l < 2; ++l) {
        alloc((void**)&c->keys[l], sizeof(unsigned long long) * max_paths);
        alloc((void**)&c->vals[l], sizeof(float) * kPay * (size_t)max_paths);
    }
    alloc((void**)&c->tkeys, sizeof(unsigned long long) * t);
    alloc((void**)&c->tvals, sizeof(float) * kPay * (size_t)t);
    alloc((void**)&c->ints, sizeof(int) * 4);
    if (rc == RPR_OK) {
        hipLaunchKernelGGL(k_pc_zero, dim3(1), dim3(64), 0, nullptr, c->ints, 4);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            rc = set_error(RPR_EDEVICE, "path_cache_create: initialisation failed");
    }
    if (rc != RPR_OK) {
        path_cache_destroy(c);
        return rc;
    }
    *out = c;
    return RPR_OK;
}

extern "C" int path_cache_destroy(RprPathCache* c)
{
    if (!c) return RPR_OK;
    (void)hipDeviceSynchronize();
    for (int l = 0; l < 2; ++l) {
        if (c->keys[l]) (void)hipFree(c->keys[l]);
        if (c->vals[l]) (void)hipFree(c->vals[l]);
    }
    if (c->tkeys) (void)hipFree(c->tkeys);
    if (c->tvals) (void)hipFree(c->tvals);
    if (c->ints) (void)hipFree(c->ints);
    delete c;
    return RPR_OK;
}

extern "C" int path_cache_update(RprPathCache* c, const float* records, const uint32_t* n_records,
                                 int32_t max_records, float alpha, int32_t first, float min_energy, void* hip_stream)
{
    if (!c || max_records < 0 || (max_records > 0 && (!records || !n_records)))
        return set_error(RPR_EINVAL, "path_cache_update: bad argument");
    if (!(alpha >= 0.f && alpha <= 1.f)) return set_error(RPR_EINVAL, "path_cache_update: alpha not in [0, 1]");
    if (!(min_energy >= 0.f)) return set_error(RPR_EINVAL, "path_cache_update: min_energy < 0");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nxt = 1 - c->cur;
    const uint32_t T = c->table_size, mask = T - 1;
    hipLaunchKernelGGL(k_pc_clear, dim3(grid_for(T)), dim3(256), 0, s, c->tkeys, c->tvals, T, c->ints + nxt);
    if (!first)
        hipLaunchKernelGGL(k_pc_insert_list, dim3(grid_for(c->max_paths)), dim3(256), 0, s, c->keys[c->cur],
                           c->vals[c->cur], c->ints + c->cur, c->max_paths, 1.f - alpha, c->tkeys, c->tvals, mask,
                           c->ints + 2);
    if (max_records > 0)
        hipLaunchKernelGGL(k_pc_insert_records, dim3(grid_for(max_records)), dim3(256), 0, s, records, n_records,
                           max_records, first ? 1.f : alpha, c->tkeys, c->tvals, mask, c->ints + 2);
    hipLaunchKernelGGL(k_pc_compact, dim3(grid_for(T)), dim3(256), 0, s, c->tkeys, c->tvals, T, min_energy,
                       c->keys[nxt], c->vals[nxt], c->ints + nxt, c->max_paths, c->ints + 2);
    RPR_HIP_TRY(hipGetLastError());
    c->cur = nxt;
    return RPR_OK;
}

extern "C" int path_cache_select(RprPathCache* c, float threshold, int32_t n_er, RprEarlyPath* out, int32_t* n_out,
                                 float* hist_late, RprIrStats* stats, int32_t n_src, int32_t n_bins,
                                 int32_t n_bands, float bin_width_s, void* hip_stream)
{
    if (!c || n_er < 0 || (n_er > 0 && !out) || !n_out || n_src < 0 || n_bins < 1 || n_bands < 1 ||
        n_bands > RPR_MAX_BANDS || !(bin_width_s > 0.f) || !(threshold >= 0.f))
        return set_error(RPR_EINVAL, "path_cache_select: bad argument");
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_pc_zero, dim3(1), dim3(64), 0, s, c->ints + 3, 1);
    const int blocks = (c->max_paths + kRankTile - 1) / kRankTile;
    hipLaunchKernelGGL(k_pc_select, dim3(blocks), dim3(kRankTile), 0, s, c->keys[c->cur], c->vals[c->cur],
                       c->ints + c->cur, c->max_paths, threshold, n_er, out, c->ints + 3, hist_late, stats, n_src,
                       n_bins, n_bands, bin_width_s);
    hipLaunchKernelGGL(k_pc_nout, dim3(1), dim3(1), 0, s, c->ints + 3, n_er, n_out);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int path_cache_info(const RprPathCache* c, RprPathCacheInfo* out)
{
    if (!c || !out) return set_error(RPR_EINVAL, "path_cache_info: bad argument");
    int v[4];
    RPR_HIP_TRY(hipDeviceSynchronize());
    RPR_HIP_TRY(hipMemcpy(v, c->ints, sizeof(v), hipMemcpyDeviceToHost));
    out->max_paths = c->max_paths;
    out->n_paths = std::min(v[c->cur], c->max_paths);
    out->overflow = v[2];
    out->table_size = (int32_t)c->table_size;
    return RPR_OK;
}
