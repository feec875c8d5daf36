// Reverb-parameter estimation (Section 4.2) on the device: one wave per
// (IR, band), FP64 throughout.
//
// RT60: the band's intensity I[m] is integrated backwards from its last
// nonzero bin (Schroeder), S[m] = C + sum_{j=m..m_last} I[j]; the decay curve
// y[m] = 10 log10(S[m] / S[0]) at the bins' left edges is fitted by ordinary
// least squares over the first of T30 [-5,-35], T20 [-5,-25], T10 [-5,-15],
// EDT [0,-10] dB whose bottom is reached by bin m_last - W (W = max(1, T/20))
// with at least three points; RT60 = -60 / slope.  When the energy reaches
// the last W bins of the window, the missing tail C is estimated from the
// mean of those bins extrapolated to the window end with the current decay
// constant, and the fit is repeated.  Reverb gain from Eq. 5 and Eq. 8,
// directivity from Eq. 1.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

namespace rpr {
namespace {

struct EstArgs {
    const float* hist;
    const float* hist_late;
    const RprIrStats* stats;
    int n_ir, T, nb, nc;
    double dt;
    int rt60_source, tail_iters;
    int vec4;  // nc == 16 and 16-byte aligned rows
    RprReverbParams* out;
};

struct Fit {
    double rt;
    int range;
    int status;
};

__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }

__device__ __forceinline__ int wmax(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Intensity used for the fit.
__device__ __forceinline__ double I_fit(const EstArgs& a, const float* H, const float* HL, int m, int b)
{
    if (a.rt60_source == 1) return (double)HL[(size_t)m * a.nb + b];
    return 3.5449077018110318 * (double)H[((size_t)m * a.nb + b) * a.nc];  // sqrt(4 pi) * H_00
}

// Backward integral without the tail constant, Sb[m] = sum_{j=m..m_last} I[j],
// accumulated in FP64 strictly from the last bin down (Sb[m] = Sb[m+1] +
// I[m]), one chunk of 64 bins at a time with each lane's value broadcast in
// turn; S[m] = C + Sb[m].  That order makes S exactly non-increasing: bins
// without energy (before the first arrival, or gaps in a sparse decay) keep
// S exactly constant, so their decay-curve value is exactly 0 dB, or exactly
// that of the next bin, and a range whose top is 0 dB (EDT) takes them all.
// A tree-shaped suffix sum would round such plateaus up or down by an ulp
// and drop some of them from the fit.  Every use of S -- its value at 0 and
// at the range-test bin, and the decay curve -- is formed from the same Sb.
// With LDS, Sb is computed once and kept (T <= kLdsBins), from the
// intensities that the kernel's first pass staged there (so the serial scan
// waits on no memory load); otherwise it is recomputed by every pass.
constexpr int kLdsBins = 8192;

template <bool LDS>
struct SbSource {
    const EstArgs& a;
    const float* H;
    const float* HL;
    int b, m_last, lane;
    double* sS;  // LDS copy when LDS

    template <class F>
    __device__ __forceinline__ double scan(F&& visit) const
    {
        double carry = 0.0;
        const int last = __builtin_amdgcn_readfirstlane(m_last);  // uniform: keeps the loops scalar
        const int n_chunks = (last + kWave) / kWave;
        for (int ch = n_chunks - 1; ch >= 0; --ch) {
            const int m = ch * kWave + lane;
            // with LDS, the first pass has left I[m] in sS (overwritten here by Sb[m])
            const double v = m <= last ? (LDS ? sS[m] : I_fit(a, H, HL, m, b)) : 0.0;
            const int top = min(kWave - 1, last - ch * kWave);
            // each lane's value in turn, read as a scalar (no LDS round trip per step)
            const uint64_t vb = (uint64_t)__double_as_longlong(v);
            const uint32_t lo = (uint32_t)vb, hi = (uint32_t)(vb >> 32);
            double mine = 0.0;
            auto step = [&](int j) {
                const uint32_t l = __builtin_amdgcn_readlane(lo, j), h = __builtin_amdgcn_readlane(hi, j);
                carry += __longlong_as_double((long long)(((uint64_t)h << 32) | l));
                mine = lane == j ? carry : mine;
            };
            if (top == kWave - 1) {
                // a full chunk: constant lane indices, no loop control between the adds
#pragma unroll
                for (int j = kWave - 1; j >= 0; --j) step(j);
            } else {
                for (int j = top; j >= 0; --j) step(j);
            }
            if (m <= last) visit(m, mine);
        }
        return carry;
    }

    __device__ __forceinline__ void prepare()
    {
        if (LDS) scan([&](int m, double Sb) { sS[m] = Sb; });
        __syncthreads();
    }

    // visit(m, Sb[m]) for m in [0, m_last]; returns Sb[0]
    template <class F>
    __device__ __forceinline__ double each(F&& visit) const
    {
        if (LDS) {
            for (int m = lane; m <= m_last; m += kWave) visit(m, sS[m]);
            return sS[0];
        }
        return scan(visit);
    }
};

template <bool LDS>
__device__ Fit fit_once(const SbSource<LDS>& src, double dt, int m_last, int W, double C, int lane)
{
    Fit f{0.0, -1, RPR_ST_NO_RANGE};
    const int top = m_last - W;
    if (top < 0) return f;
    double sb_top_lane = 0.0;
    const double Sb0 = src.each([&](int m, double Sb) {
        if (m == top) sb_top_lane = Sb;
    });
    const double S0 = C + Sb0;
    const double S_top = C + wsum(sb_top_lane);  // exactly one lane holds Sb[top]
    const double y_top = 10.0 * log10(S_top / S0);
    const double his[4] = {-5.0, -5.0, -5.0, 0.0};
    const double los[4] = {-35.0, -25.0, -15.0, -10.0};
    // One pass over the decay curve gathers the sums of every range that the
    // curve reaches (each lane adds its bins in the same order as a pass per
    // range would, so the sums are the same); the ranges are then tried in turn.
    bool want[4];
    bool any = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) any |= (want[r] = y_top <= los[r]);
    if (!any) return f;
    double acc[4][5];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[r][q] = 0.0;
    src.each([&](int m, double Sb) {
        const double y = 10.0 * log10((C + Sb) / S0);
        const double t = (double)m * dt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (want[r] && y <= his[r] && y >= los[r]) {
                acc[r][0] += 1.0;
                acc[r][1] += t;
                acc[r][2] += y;
                acc[r][3] += t * t;
                acc[r][4] += t * y;
            }
        }
    });
    for (int r = 0; r < 4; ++r) {
        if (!want[r]) continue;
        const double n = wsum(acc[r][0]), s_t = wsum(acc[r][1]), s_y = wsum(acc[r][2]);
        const double s_tt = wsum(acc[r][3]), s_ty = wsum(acc[r][4]);
        if (n < 3.0) continue;
        const double den = n * s_tt - s_t * s_t;
        if (!(den > 0.0)) continue;
        const double slope = (n * s_ty - s_t * s_y) / den;
        if (slope >= 0.0) return Fit{0.0, r, RPR_ST_BAD_FIT};
        return Fit{-60.0 / slope, r, RPR_ST_OK};
    }
    return f;
}

template <bool LDS>
__global__ void __launch_bounds__(kWave) k_estimate(EstArgs a)
{
    extern __shared__ double sS[];
    const int ir = blockIdx.x / a.nb, b = blockIdx.x % a.nb;
    const int lane = threadIdx.x;
    const int T = a.T, nb = a.nb, nc = a.nc;
    const float* H = a.hist + (size_t)ir * T * nb * nc;
    const float* HL = a.hist_late ? a.hist_late + (size_t)ir * T * nb : nullptr;
    const RprIrStats& S = a.stats[ir];
    RprReverbParams* out = a.out + ir;

    // pass 1: last nonzero bin of the fitted intensity, its total, and the
    // per-coefficient sums of Eq. 1
    int m_last = -1;
    double tot_all = 0.0;
    double dsum[RPR_MAX_COEFFS];
#pragma unroll
    for (int c = 0; c < RPR_MAX_COEFFS; ++c) dsum[c] = 0.0;
    if (a.vec4) {
        // 16 coefficients per (bin, band): four 16-byte loads per row
#pragma unroll 4
        for (int m = lane; m < T; m += kWave) {
            const float4* row = reinterpret_cast<const float4*>(H + ((size_t)m * nb + b) * 16);
            const float4 q[4] = {row[0], row[1], row[2], row[3]};
            const double v = a.rt60_source == 1 ? (double)HL[(size_t)m * nb + b] : 3.5449077018110318 * (double)q[0].x;
            if (LDS) sS[m] = v;
            if (v > 0.0) m_last = m;
            tot_all += 3.5449077018110318 * (double)q[0].x;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                dsum[4 * c] += (double)q[c].x;
                dsum[4 * c + 1] += (double)q[c].y;
                dsum[4 * c + 2] += (double)q[c].z;
                dsum[4 * c + 3] += (double)q[c].w;
            }
        }
    } else {
        for (int m = lane; m < T; m += kWave) {
            const double v = I_fit(a, H, HL, m, b);
            if (LDS) sS[m] = v;
            if (v > 0.0) m_last = m;
            const float* row = H + ((size_t)m * nb + b) * nc;
            tot_all += 3.5449077018110318 * (double)row[0];
#pragma unroll
            for (int c = 0; c < RPR_MAX_COEFFS; ++c)
                if (c < nc) dsum[c] += (double)row[c];
        }
    }
    if (LDS) __syncthreads();
    m_last = wmax(m_last);
    tot_all = wsum(tot_all);
#pragma unroll
    for (int c = 0; c < RPR_MAX_COEFFS; ++c) dsum[c] = wsum(dsum[c]);

    const int W = T / 20 > 1 ? T / 20 : 1;
    Fit f{0.0, -1, RPR_ST_NO_ENERGY};
    SbSource<LDS> src{a, H, HL, b, m_last, lane, sS};
    if (m_last >= 0) src.prepare();
    if (m_last >= 0) {
        f = fit_once(src, a.dt, m_last, W, 0.0, lane);
        if (f.status == RPR_ST_OK && m_last >= T - W) {
            double ts = 0.0;
            for (int m = m_last - W + 1 + lane; m <= m_last; m += kWave) ts += I_fit(a, H, HL, m, b);
            const double tail = wsum(ts) / (double)W;
            for (int it = 0; it < a.tail_iters; ++it) {
                const double tau = f.rt / (6.0 * 2.302585092994046);
                const double C = tail * exp(-(double)(W + 1) * a.dt / (2.0 * tau)) * tau / a.dt;
                const Fit g = fit_once(src, a.dt, m_last, W, C, lane);
                if (g.status != RPR_ST_OK) break;
                f = Fit{g.rt, g.range, RPR_ST_OK | RPR_ST_TAIL_COMPENSATED};
            }
        }
    }
    int status = f.status;
    if (S.e_alive_at_bounce_cap[b] > 1e-3 * S.e_emitted) status |= RPR_ST_TRUNCATED_BY_BOUNCES;
    const double e_late = S.e_class[2][b];
    if (lane == 0) {
        out->rt60[b] = (float)f.rt;
        out->rt60_range[b] = f.range;
        out->status[b] = status;
        out->e_direct[b] = (float)S.e_class[0][b];
        out->e_early[b] = (float)S.e_class[1][b];
        out->e_late[b] = (float)e_late;
        out->g_reverb[b] = f.rt > 0.0 ? (float)sqrt(e_late * 6.0 * 2.302585092994046 / f.rt) : 0.0f;
    }
    if (lane < RPR_MAX_COEFFS) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < RPR_MAX_COEFFS; ++c)
            if (c == lane) v = dsum[c];
        out->dir_loudness[b][lane] = (lane < nc && tot_all > 0.0) ? (float)(v / tot_all) : 0.0f;
    }
    if (b == 0 && lane == 0) {
        const double dt = a.dt;
        out->predelay_s = S.first_late_bin != INT32_MAX ? (float)(S.first_late_bin * dt) : -1.0f;
        out->first_arrival_s = S.first_arrival_bin != INT32_MAX ? (float)(S.first_arrival_bin * dt) : -1.0f;
        out->mean_free_path_m =
            S.n_finite_segments > 0 ? (float)(S.seg_len_sum / (double)S.n_finite_segments) : 0.0f;
        out->reserved = 0.0f;
        for (int bb = nb; bb < RPR_MAX_BANDS; ++bb) {
            out->rt60[bb] = 0.0f;
            out->rt60_range[bb] = -1;
            out->status[bb] = 0;
            out->e_direct[bb] = out->e_early[bb] = out->e_late[bb] = out->g_reverb[bb] = 0.0f;
            for (int c = 0; c < RPR_MAX_COEFFS; ++c) out->dir_loudness[bb][c] = 0.0f;
        }
    }
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int estimate_reverb(const float* hist, const float* hist_late, const RprIrStats* stats, int32_t n_ir,
                               int32_t n_bins, int32_t n_bands, int32_t sh_order, float bin_width_s,
                               const RprEstimateParams* ep, RprReverbParams* out, void* hip_stream)
{
    const RprEstimateParams def{hist_late ? 1 : 0, 3};
    const RprEstimateParams e = ep ? *ep : def;
    if (n_ir < 0) return set_error(RPR_EINVAL, "estimate_reverb: n_ir < 0");
    if (n_ir == 0) return RPR_OK;
    if (!hist || !stats || !out) return set_error(RPR_EINVAL, "estimate_reverb: null argument");
    if (n_bins < 1) return set_error(RPR_EINVAL, "estimate_reverb: n_bins < 1");
    if (n_bands < 1 || n_bands > RPR_MAX_BANDS) return set_error(RPR_EINVAL, "estimate_reverb: n_bands out of range");
    if (sh_order < 0 || sh_order > RPR_MAX_SH_ORDER) return set_error(RPR_EINVAL, "estimate_reverb: bad sh_order");
    if (!(bin_width_s > 0.f)) return set_error(RPR_EINVAL, "estimate_reverb: bin_width_s must be > 0");
    if (e.rt60_source != 0 && e.rt60_source != 1) return set_error(RPR_EINVAL, "estimate_reverb: bad rt60_source");
    if (e.rt60_source == 1 && !hist_late)
        return set_error(RPR_EINVAL, "estimate_reverb: rt60_source=1 needs hist_late");
    if (e.tail_iters < 0 || e.tail_iters > 100) return set_error(RPR_EINVAL, "estimate_reverb: bad tail_iters");
    const int nc = (sh_order + 1) * (sh_order + 1);
    const int vec4 = nc == 16 && ((uintptr_t)hist % 16) == 0;
    EstArgs a{hist, hist_late, stats, n_ir, n_bins, n_bands, nc, (double)bin_width_s, e.rt60_source, e.tail_iters,
              vec4, out};
    const long long grid = (long long)n_ir * n_bands;
    if (grid > 0x7FFFFFFF) return set_error(RPR_EUNSUPPORTED, "estimate_reverb: too many IRs");
    if (n_bins <= kLdsBins)
        hipLaunchKernelGGL(k_estimate<true>, dim3((unsigned)grid), dim3(kWave), sizeof(double) * n_bins,
                           (hipStream_t)hip_stream, a);
    else
        hipLaunchKernelGGL(k_estimate<false>, dim3((unsigned)grid), dim3(kWave), 0, (hipStream_t)hip_stream, a);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
