// Temporal coherence across frames (Section 4.2, Eq. 4; Section 5, the
// early- and late-reflection caches with their own time constants), and the
// frame's ray count under a segment budget (Section 5).
//
// ir_cache_update: every histogram cell of the cache becomes
// alpha * fresh + (1 - alpha) * cache (the fresh value on the first frame).
// reverb_params_smooth: Eq. 4 on each band's RT60 with the late factor
// (an invalid frame keeps the cached value), the direct and early energies
// with the early factor, the late energy with the late factor, and g_reverb
// recomputed from the smoothed late energy and RT60 (Eq. 5 with Eq. 8).
// Both are elementwise and bound by HBM traffic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rpr_internal.hpp"

namespace rpr {
namespace {

constexpr int kInvalidFit = RPR_ST_NO_ENERGY | RPR_ST_BAD_FIT | RPR_ST_NO_RANGE;

__global__ void k_ema(float* __restrict__ cache, const float* __restrict__ fresh, long long n, float alpha,
                      int first)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long n4 = n >> 2;
    float4* c4 = reinterpret_cast<float4*>(cache);
    const float4* f4 = reinterpret_cast<const float4*>(fresh);
    const float keep = 1.0f - alpha;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 f = f4[i];
        if (first) {
            c4[i] = f;
        } else {
            const float4 c = c4[i];
            c4[i] = make_float4(fmaf(alpha, f.x, keep * c.x), fmaf(alpha, f.y, keep * c.y),
                                fmaf(alpha, f.z, keep * c.z), fmaf(alpha, f.w, keep * c.w));
        }
    }
    for (long long i = (n4 << 2) + (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        cache[i] = first ? fresh[i] : fmaf(alpha, fresh[i], keep * cache[i]);
}

__global__ void k_params_smooth(RprReverbParams* __restrict__ cache, const RprReverbParams* __restrict__ fresh,
                                int n_ir, int nb, float a_early, float a_late, int first)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ir) return;
    RprReverbParams& C = cache[i];
    const RprReverbParams& F = fresh[i];
    if (first) {
        C = F;
        return;
    }
    RprReverbParams out = F;
    for (int b = 0; b < nb; ++b) {
        const bool valid = (F.status[b] & kInvalidFit) == 0;
        const bool prev = C.rt60[b] > 0.f;
        float rt = C.rt60[b];
        if (valid) rt = prev ? fmaf(a_late, F.rt60[b], (1.0f - a_late) * C.rt60[b]) : F.rt60[b];
        out.rt60[b] = rt;
        out.status[b] = valid ? F.status[b] : C.status[b];
        out.rt60_range[b] = valid ? F.rt60_range[b] : C.rt60_range[b];
        out.e_direct[b] = fmaf(a_early, F.e_direct[b], (1.0f - a_early) * C.e_direct[b]);
        out.e_early[b] = fmaf(a_early, F.e_early[b], (1.0f - a_early) * C.e_early[b]);
        out.e_late[b] = fmaf(a_late, F.e_late[b], (1.0f - a_late) * C.e_late[b]);
        out.g_reverb[b] = rt > 0.f ? sqrtf(out.e_late[b] * (float)(6.0 * M_LN10) / rt) : 0.f;
    }
    C = out;
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int64_t budget_ray_count(int64_t budget_segments, int64_t prev_segments, int64_t prev_rays,
                                    int64_t min_rays, int64_t max_rays, int64_t nominal)
{
    int64_t n = nominal;
    if (prev_segments > 0 && prev_rays > 0) {
        // floor(budget * prev_rays / prev_segments) without overflowing 64 bits
        const __int128 q = (__int128)budget_segments * (__int128)prev_rays / (__int128)prev_segments;
        n = q > (__int128)INT64_MAX ? INT64_MAX : (int64_t)q;
    }
    return std::max(min_rays, std::min(n, max_rays));
}

extern "C" float temporal_alpha(float frame_dt_s, float tau_s)
{
    if (!(tau_s > 0.f)) return 1.0f;
    return (float)(1.0 - std::exp(-(double)frame_dt_s / (double)tau_s));
}

extern "C" int ir_cache_update(float* cache, const float* fresh, int64_t n, float alpha, int32_t first,
                               void* hip_stream)
{
    if (n < 0 || (n > 0 && (!cache || !fresh))) return set_error(RPR_EINVAL, "ir_cache_update: bad argument");
    if (!(alpha >= 0.f && alpha <= 1.f)) return set_error(RPR_EINVAL, "ir_cache_update: alpha not in [0, 1]");
    if ((reinterpret_cast<uintptr_t>(cache) | reinterpret_cast<uintptr_t>(fresh)) & 15u)
        return set_error(RPR_EINVAL, "ir_cache_update: buffers must be 16-byte aligned");
    if (n == 0) return RPR_OK;
    const long long blocks = std::min<long long>((n / 4 + 255) / 256 + 1, 16384);
    hipLaunchKernelGGL(k_ema, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, cache, fresh,
                       (long long)n, alpha, first ? 1 : 0);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_params_smooth(RprReverbParams* cache, const RprReverbParams* fresh, int32_t n_ir,
                                    int32_t n_bands, float alpha_early, float alpha_late, int32_t first,
                                    void* hip_stream)
{
    if (n_ir < 0 || (n_ir > 0 && (!cache || !fresh)) || n_bands < 1 || n_bands > RPR_MAX_BANDS)
        return set_error(RPR_EINVAL, "reverb_params_smooth: bad argument");
    if (!(alpha_early >= 0.f && alpha_early <= 1.f && alpha_late >= 0.f && alpha_late <= 1.f))
        return set_error(RPR_EINVAL, "reverb_params_smooth: alpha not in [0, 1]");
    if (n_ir == 0) return RPR_OK;
    hipLaunchKernelGGL(k_params_smooth, dim3((unsigned)((n_ir + 127) / 128)), dim3(128), 0, (hipStream_t)hip_stream,
                       cache, fresh, n_ir, n_bands, alpha_early, alpha_late, first ? 1 : 0);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
