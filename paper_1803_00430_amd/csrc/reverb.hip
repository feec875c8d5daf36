// SH-domain Schroeder reverberator (Section 4.1 "Sound Rendering": input
// spatialization, SH rotations in the comb feedback paths, directional
// loudness; Section 4.2: Eq. 7 comb gains, comb delays drawn around the mean
// free path, the predelay; Section 5 "Auralization": 8 combs, 4 all-passes).
//
// reverb_setup: one workgroup per source builds every parameter: the comb
// delays (FP64 scalar work), the Eq. 7 gains, the input directions read from
// the histogram, and the SH rotation and loudness matrices by quadrature
// over the sphere (8 Gauss-Legendre nodes in cos(theta) x 16 azimuths; exact
// for the rotation, whose integrand is a polynomial of degree <= 6).
//
// reverb_render: one workgroup per source renders all its bands and SH
// channels.  Every delay line is a ring of exactly its delay: the slot of
// sample n holds the line's value from n - M, so a sample reads its slot and
// writes it back, and a run of up to min(M) consecutive samples touches
// distinct slots.  The block is walked in such sub-steps, the samples of a
// sub-step in parallel (one wave per band and run of 64 samples), with a
// barrier between sub-steps.  Comb lines hold w[n] = a x[n] + G y[n] (so
// that y[n] = w[n - M]), all-pass lines w[n] = u[n] + g w[n - M] with output
// v[n] = -g w[n] + w[n - M].  The comb lines are read and written once per
// sample and dominate the traffic, so the render is bound by HBM; the short
// all-pass lines stay in LDS for the launch where they fit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

static_assert(sizeof(RprReverbSetup) == 17392, "RprReverbSetup layout");

namespace rpr {
namespace {

constexpr int kCombs = RPR_REVERB_COMBS;
constexpr int kAllpass = RPR_REVERB_ALLPASS;
constexpr double kApDelayS[kAllpass] = {4.9e-3, 4.1e-3, 3.4e-3, 2.9e-3};
constexpr float kApGain = 0.7f;
constexpr double kMinCombS = 1e-3;
constexpr int kHeaderBytes = 64;
constexpr int kRenderThreads = 512;
constexpr int kRenderWaves = kRenderThreads / 64;
constexpr int kOutStage = 2048;  // floats of LDS for the per-band outputs of one sub-step
constexpr int kLdsLimit = 65536; // bytes of LDS a render workgroup may use
constexpr int kQuadZ = 8, kQuadPhi = 16, kQuad = kQuadZ * kQuadPhi;

struct Geometry {
    int nb, nc, m_cap, a_cap, ap_m[kAllpass];
    int64_t bytes;  // per source, a multiple of 256
};

int samples_of(double t, double fs) { return (int)std::floor(t * fs + 0.5); }

int geometry(const RprReverbDesc* d, Geometry* g)
{
    if (!d) return set_error(RPR_EINVAL, "reverb: desc is NULL");
    if (d->n_bands < 1 || d->n_bands > RPR_MAX_BANDS || d->sh_order < 0 || d->sh_order > RPR_MAX_SH_ORDER ||
        !(d->sample_rate >= 8000.f && d->sample_rate <= 192000.f) || !(d->speed_of_sound > 0.f) ||
        !(d->max_comb_delay_s >= 0.005f && d->max_comb_delay_s <= 2.f))
        return set_error(RPR_EINVAL, "reverb: description out of range");
    g->nb = d->n_bands;
    g->nc = (d->sh_order + 1) * (d->sh_order + 1);
    g->m_cap = samples_of((double)d->max_comb_delay_s, (double)d->sample_rate);
    g->a_cap = 0;
    for (int j = 0; j < kAllpass; ++j) {
        g->ap_m[j] = std::max(1, samples_of(kApDelayS[j], (double)d->sample_rate));
        g->a_cap = std::max(g->a_cap, g->ap_m[j]);
    }
    const int64_t pad = g->nc == 1 ? 1 : (g->nc + 3) / 4 * 4;  // channels of a comb-line slot
    const int64_t floats = (int64_t)g->nb * ((int64_t)kCombs * g->m_cap * pad + (int64_t)kAllpass * g->nc * g->a_cap);
    g->bytes = (kHeaderBytes + floats * 4 + 255) / 256 * 256;
    return RPR_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on the
// Legendre polynomial (three-term recurrence), from the asymptotic guess
// cos(pi (i - 1/4) / (n + 1/2)).
struct Quad {
    float z[kQuadZ];
    float w[kQuadZ];
};

Quad gauss_legendre()
{
    Quad q;
    const int n = kQuadZ;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        q.z[i] = (float)x;
        q.w[i] = (float)(2.0 / ((1.0 - x * x) * dp * dp));
    }
    return q;
}

// ------------------------------------------------------------------ setup
__global__ __launch_bounds__(256) void k_reverb_setup(const RprReverbParams* __restrict__ params,
                                                       const float* __restrict__ hist, int n_bins, double dt,
                                                       const float* __restrict__ zn, const float* __restrict__ ang,
                                                       int first, int nb, int order, double fs, double c,
                                                       double t_max, Quad quad, RprReverbSetup* __restrict__ setup)
{
    const int ir = blockIdx.x, tid = threadIdx.x;
    const int nc = (order + 1) * (order + 1);
    const RprReverbParams& P = params[ir];
    RprReverbSetup& S = setup[ir];

    __shared__ float s_v[kQuad][3], s_w[kQuad];
    __shared__ float s_Y[kQuad][RPR_MAX_COEFFS], s_YR[kQuad][RPR_MAX_COEFFS];
    __shared__ float s_g[kQuad];
    __shared__ double s_t[kCombs];
    __shared__ double s_tfirst;
    __shared__ float s_R[kCombs][3][3];

    // comb delays (Section 4.2): kept while the mean free path stays within
    // 2 sigma of the last draw's mean, else drawn from the caller's normals
    if (tid == 0) {
        const double mfp = (double)P.mean_free_path_m;
        const double drawn = first ? 0.0 : (double)S.mfp_drawn;
        bool keep = false;
        if (drawn > 0.0) {
            const double m_prev = drawn / c;
            keep = mfp <= 0.0 || std::fabs(mfp / c - m_prev) <= 2.0 * (m_prev / 3.0);
        }
        if (keep) {
            for (int i = 0; i < kCombs; ++i) s_t[i] = (double)S.t_comb[i];
        } else {
            const double m = std::max(mfp, 0.0) / c;
            for (int i = 0; i < kCombs; ++i) {
                const double z = std::min(std::max((double)zn[ir * kCombs + i], -2.7), 3.0);
                s_t[i] = std::min(std::max(m * (1.0 + z / 3.0), kMinCombS), t_max);
            }
            S.mfp_drawn = mfp > 0.0 ? (float)mfp : 0.f;
        }
        const double tf = P.predelay_s >= 0.f ? (double)P.predelay_s
                          : (P.first_arrival_s >= 0.f ? (double)P.first_arrival_s : 0.0);
        s_tfirst = tf;
        S.predelay_samples = (int)floor(tf * fs + 0.5);
        S.n_bands = nb;
        S.sh_order = order;
    }
    // quadrature nodes and the SH basis at them
    for (int q = tid; q < kQuad; q += blockDim.x) {
        const int iz = q / kQuadPhi, ip = q % kQuadPhi;
        const float z = quad.z[iz], r = sqrtf(fmaxf(0.f, 1.f - z * z));
        float sp, cp;
        sincospif((2.f * ip + 1.f) / (float)kQuadPhi, &sp, &cp);
        s_v[q][0] = r * cp;
        s_v[q][1] = r * sp;
        s_v[q][2] = z;
        s_w[q] = quad.w[iz] * (2.f * (float)M_PI / kQuadPhi);
        for (int k = 0; k < nc; ++k) s_Y[q][k] = sh_coeff(k, r * cp, r * sp, z);
    }
    if (tid < kCombs) {  // R = Rz(c) Ry(b) Rx(a)
        const float* a3 = ang + ((size_t)ir * kCombs + tid) * 3;
        float sa, ca, sb, cb, sc, cc;
        sincosf(a3[0], &sa, &ca);
        sincosf(a3[1], &sb, &cb);
        sincosf(a3[2], &sc, &cc);
        const float Rx[3][3] = {{1, 0, 0}, {0, ca, -sa}, {0, sa, ca}};
        const float Ry[3][3] = {{cb, 0, sb}, {0, 1, 0}, {-sb, 0, cb}};
        const float Rz[3][3] = {{cc, -sc, 0}, {sc, cc, 0}, {0, 0, 1}};
        float T[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) T[i][j] = Ry[i][0] * Rx[0][j] + Ry[i][1] * Rx[1][j] + Ry[i][2] * Rx[2][j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                s_R[tid][i][j] = Rz[i][0] * T[0][j] + Rz[i][1] * T[1][j] + Rz[i][2] * T[2][j];
    }
    __syncthreads();

    if (tid < kCombs) {
        const int i = tid;
        const double t = s_t[i];
        S.t_comb[i] = (float)t;
        S.m_comb[i] = std::max(1, (int)floor(t * fs + 0.5));
        for (int b = 0; b < RPR_MAX_BANDS; ++b) {
            const double rt = b < nb ? (double)P.rt60[b] : 0.0;
            S.g_comb[b][i] = rt > 0.0 ? (float)pow(10.0, -3.0 * t / rt) : 0.f;  // Eq. 7
        }
        // input direction: band-summed first-order coefficients at t_first + t
        float v[3] = {0.f, 0.f, 0.f};
        if (nc >= 4) {
            const double p = (s_tfirst + t) / dt;
            const double fl = floor(p);
            const float f = (float)(p - fl);
            float acc[3] = {0.f, 0.f, 0.f};
            for (int e = 0; e < 2; ++e) {
                const double jd = fl + e;
                if (jd < 0.0 || jd >= (double)n_bins) continue;
                const float wgt = e ? f : 1.f - f;
                const float* h = hist + ((size_t)ir * n_bins + (size_t)jd) * nb * nc;
                for (int b = 0; b < nb; ++b)
                    for (int k = 0; k < 3; ++k) acc[k] += wgt * h[b * nc + 1 + k];
            }
            v[0] = -acc[2];
            v[1] = -acc[0];
            v[2] = acc[1];
        }
        const float n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (n2 > 0.f) {
            const float inv = 1.f / sqrtf(n2);
            for (int k = 0; k < 3; ++k) v[k] *= inv;
        }
        S.dir[i][0] = v[0];
        S.dir[i][1] = v[1];
        S.dir[i][2] = v[2];
        S.dir[i][3] = n2 > 0.f ? 1.f : 0.f;
        for (int k = 0; k < RPR_MAX_COEFFS; ++k) {
            float a = 0.f;
            if (n2 > 0.f && k < nc) a = sh_coeff(k, v[0], v[1], v[2]) / kCombs;
            else if (k == 0) a = sh_coeff(0, 0.f, 0.f, 1.f) / kCombs;
            S.a[i][k] = a;
        }
    }
    if (tid < RPR_MAX_BANDS) S.g_reverb[tid] = tid < nb ? P.g_reverb[tid] : 0.f;

    // J_i[k][k'] = sum_q w_q Y_k(R_i v_q) Y_k'(v_q)
    for (int i = 0; i < kCombs; ++i) {
        for (int q = tid; q < kQuad; q += blockDim.x) {
            const float* R = &s_R[i][0][0];
            const float x = R[0] * s_v[q][0] + R[1] * s_v[q][1] + R[2] * s_v[q][2];
            const float y = R[3] * s_v[q][0] + R[4] * s_v[q][1] + R[5] * s_v[q][2];
            const float z = R[6] * s_v[q][0] + R[7] * s_v[q][1] + R[8] * s_v[q][2];
            for (int k = 0; k < nc; ++k) s_YR[q][k] = sh_coeff(k, x, y, z);
        }
        __syncthreads();
        for (int e = tid; e < RPR_MAX_COEFFS * RPR_MAX_COEFFS; e += blockDim.x) {
            const int k = e / RPR_MAX_COEFFS, kk = e % RPR_MAX_COEFFS;
            float s = 0.f;
            if (k < nc && kk < nc)
                for (int q = 0; q < kQuad; ++q) s = fmaf(s_w[q] * s_YR[q][k], s_Y[q][kk], s);
            S.J[i][k][kk] = s;
        }
        __syncthreads();
    }
    // D_b[k][k'] = sum_q w_q g_b(v_q) Y_k(v_q) Y_k'(v_q)
    for (int b = 0; b < RPR_MAX_BANDS; ++b) {
        const bool iso = b >= nb || !(P.dir_loudness[b][0] > 0.f);
        if (!iso) {
            for (int q = tid; q < kQuad; q += blockDim.x) {
                float f = 0.f;
                for (int k = 0; k < nc; ++k) f = fmaf(P.dir_loudness[b][k], s_Y[q][k], f);
                s_g[q] = s_w[q] * sqrtf(fmaxf(4.f * (float)M_PI * f, 0.f));
            }
        }
        __syncthreads();
        for (int e = tid; e < RPR_MAX_COEFFS * RPR_MAX_COEFFS; e += blockDim.x) {
            const int k = e / RPR_MAX_COEFFS, kk = e % RPR_MAX_COEFFS;
            float s = 0.f;
            if (k < nc && kk < nc) {
                if (iso) s = k == kk ? 1.f : 0.f;
                else
                    for (int q = 0; q < kQuad; ++q) s = fmaf(s_g[q] * s_Y[q][k], s_Y[q][kk], s);
            }
            S.D[b][k][kk] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ render
struct ApArgs {
    int m[kAllpass];
    int pref[kAllpass];  // offset of each all-pass line in the LDS copy (prefix sums of m)
    int sum;
};

// Static LDS of the render kernel, an upper bound for the budget of the
// all-pass lines (which take the rest when they fit).
constexpr int render_static_lds(int nc)
{
    return 4 * (kOutStage + kCombs * nc * nc + RPR_MAX_BANDS * nc * nc + kCombs * nc + RPR_MAX_BANDS * kCombs +
                RPR_MAX_BANDS + 2 * (kCombs + kAllpass)) + 256;
}

// Comb line layout [band][comb][slot][channel]: the channels of a sample are
// contiguous, padded to a multiple of 4 from order 1 on, and move as float4.
// kGroup combs have their loads in flight together.
template <int NC>
struct CombLine {
    static constexpr int kPad = NC == 1 ? 1 : (NC + 3) / 4 * 4;
    static constexpr int kGroup = NC == 1 ? kCombs : std::max(1, 32 / kPad);
    __device__ static void load(const float* p, float (&y)[kPad])
    {
        if constexpr (NC == 1) {
            y[0] = *p;
        } else {
#pragma unroll
            for (int v = 0; v < kPad / 4; ++v) {
                const float4 t = reinterpret_cast<const float4*>(p)[v];
                y[4 * v] = t.x;
                y[4 * v + 1] = t.y;
                y[4 * v + 2] = t.z;
                y[4 * v + 3] = t.w;
            }
        }
    }
    __device__ static void store(float* p, const float (&w)[kPad])
    {
        if constexpr (NC == 1) {
            *p = w[0];
        } else {
#pragma unroll
            for (int v = 0; v < kPad / 4; ++v)
                reinterpret_cast<float4*>(p)[v] = make_float4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
        }
    }
};

// AP_LDS: the all-pass lines are copied into LDS for the launch (loaded at
// the start, stored at the end).  They are short (a few ms) and touched
// every few sub-steps; in global memory the streaming comb lines evict them
// from L2 between touches.
template <int NC, bool AP_LDS>
__global__ __launch_bounds__(kRenderThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_reverb_render(const RprReverbSetup* __restrict__ setup,
                                                                   const float* __restrict__ x, int n,
                                                                   char* __restrict__ state, int64_t stride,
                                                                   float* __restrict__ out, int nb, int m_cap,
                                                                   int a_cap, ApArgs ap)
{
    extern __shared__ float s_apl[];
    const int src = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const RprReverbSetup& S = setup[src];
    char* st = state + (size_t)src * stride;
    int* header = reinterpret_cast<int*>(st);
    float* comb = reinterpret_cast<float*>(st + kHeaderBytes);
    float* apl = comb + (size_t)nb * kCombs * CombLine<NC>::kPad * m_cap;

    __shared__ float s_J[kCombs][NC][NC];
    __shared__ float s_a[kCombs][NC];
    __shared__ float s_g[RPR_MAX_BANDS][kCombs];
    __shared__ float s_D[RPR_MAX_BANDS][NC][NC];
    __shared__ float s_gr[RPR_MAX_BANDS];
    __shared__ int s_M[kCombs], s_ph[kCombs + kAllpass];
    __shared__ float s_out[kOutStage];

    for (int e = tid; e < kCombs * NC * NC; e += kRenderThreads) {
        const int i = e / (NC * NC), k = (e / NC) % NC, kk = e % NC;
        s_J[i][k][kk] = S.J[i][k][kk];
    }
    for (int e = tid; e < nb * NC * NC; e += kRenderThreads) {
        const int b = e / (NC * NC), k = (e / NC) % NC, kk = e % NC;
        s_D[b][k][kk] = S.D[b][k][kk];
    }
    for (int e = tid; e < kCombs * NC; e += kRenderThreads) s_a[e / NC][e % NC] = S.a[e / NC][e % NC];
    for (int e = tid; e < nb * kCombs; e += kRenderThreads) s_g[e / kCombs][e % kCombs] = S.g_comb[e / kCombs][e % kCombs];
    if (tid < nb) s_gr[tid] = S.g_reverb[tid];
    if (tid < kCombs) {
        const int M = std::min(std::max(S.m_comb[tid], 1), m_cap);  // bounds the line even for a bad setup
        s_M[tid] = M;
        s_ph[tid] = (int)((unsigned)header[tid] % (unsigned)M);
    } else if (tid < kCombs + kAllpass) {
        s_ph[tid] = (int)((unsigned)header[tid] % (unsigned)ap.m[tid - kCombs]);
    }
    if constexpr (AP_LDS) {  // [b][k][all-pass lines one after another]
        for (int e = tid; e < nb * NC * ap.sum; e += kRenderThreads) {
            const int bk = e / ap.sum, q = e - bk * ap.sum, b = bk / NC, k = bk - b * NC;
            const int s = (q >= ap.pref[1]) + (q >= ap.pref[2]) + (q >= ap.pref[3]);
            s_apl[e] = apl[((size_t)(b * kAllpass + s) * NC + k) * a_cap + (q - ap.pref[s])];
        }
    }
    __syncthreads();

    int M[kCombs], base[kCombs + kAllpass];
    int step = std::min(kOutStage / (nb * NC), 256);
    // uniform across the workgroup: kept in scalar registers
    for (int i = 0; i < kCombs; ++i) {
        M[i] = __builtin_amdgcn_readfirstlane(s_M[i]);
        base[i] = __builtin_amdgcn_readfirstlane(s_ph[i]);
        step = std::min(step, M[i]);
    }
    for (int j = 0; j < kAllpass; ++j) {
        base[kCombs + j] = __builtin_amdgcn_readfirstlane(s_ph[kCombs + j]);
        step = std::min(step, ap.m[j]);
    }

    for (int n1 = 0; n1 < n; n1 += step) {
        const int sc = std::min(step, n - n1);
        // one wave per band and run of 64 samples: the band, and with it every line base, is uniform
        const int nj = (sc + 63) >> 6;
        for (int grp = wave; grp < nb * nj; grp += kRenderWaves) {
            const int b = grp / nj, j = ((grp - b * nj) << 6) + lane;
            if (j >= sc) continue;
            // keeps the LDS reads of J and D inside the loop: hoisted, they would hold
            // 8 NC^2 + NC^2 registers for the whole loop and spill
            __asm__ volatile("" ::: "memory");
            const int nn = n1 + j;
            const float xv = x[((size_t)src * nb + b) * n + nn];
            float u[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) u[k] = 0.f;
            // all loads of a group of combs are issued before its stores (a comb's line
            // may alias another's as far as the compiler knows)
#pragma unroll
            for (int i0 = 0; i0 < kCombs; i0 += CombLine<NC>::kGroup) {
                constexpr int G = CombLine<NC>::kGroup, NP = CombLine<NC>::kPad;
                float y[G][NP];
                float* line[G];
#pragma unroll
                for (int gi = 0; gi < G; ++gi) {
                    const int i = i0 + gi;
                    int pos = base[i] + j;
                    if (pos >= M[i]) pos -= M[i];
                    line[gi] = comb + ((size_t)(b * kCombs + i) * m_cap + pos) * NP;
                    CombLine<NC>::load(line[gi], y[gi]);
                }
#pragma unroll
                for (int gi = 0; gi < G; ++gi) {
                    const int i = i0 + gi;
                    const float g = s_g[b][i];
                    float w[NP];
#pragma unroll
                    for (int k = 0; k < NP; ++k) w[k] = 0.f;
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        float r = 0.f;
#pragma unroll
                        for (int kk = 0; kk < NC; ++kk) r = fmaf(s_J[i][k][kk], y[gi][kk], r);
                        w[k] = fmaf(s_a[i][k], xv, g * r);
                        u[k] += y[gi][k];
                    }
                    CombLine<NC>::store(line[gi], w);
                }
            }
#pragma unroll
            for (int s = 0; s < kAllpass; ++s) {
                int pos = base[kCombs + s] + j;
                if (pos >= ap.m[s]) pos -= ap.m[s];
                float* line;
                int ks;
                if constexpr (AP_LDS) {
                    line = s_apl + (size_t)b * NC * ap.sum + ap.pref[s] + pos;
                    ks = ap.sum;
                } else {
                    line = apl + ((size_t)(b * kAllpass + s) * NC) * a_cap + pos;
                    ks = a_cap;
                }
                float wh[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) wh[k] = line[(size_t)k * ks];  // all loads before the stores
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const float w = fmaf(kApGain, wh[k], u[k]);
                    line[(size_t)k * ks] = w;
                    u[k] = fmaf(-kApGain, w, wh[k]);
                }
            }
            const float gr = s_gr[b];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                float r = 0.f;
#pragma unroll
                for (int kk = 0; kk < NC; ++kk) r = fmaf(s_D[b][k][kk], u[kk], r);
                s_out[(b * NC + k) * step + j] = gr * r;
            }
        }
        __syncthreads();
        for (int it = tid; it < NC * sc; it += kRenderThreads) {
            const int k = it / sc, j = it - k * sc;
            float s = 0.f;
            for (int b = 0; b < nb; ++b) s += s_out[(b * NC + k) * step + j];
            out[((size_t)src * NC + k) * n + n1 + j] = s;
        }
        for (int i = 0; i < kCombs; ++i) {
            base[i] += sc;
            if (base[i] >= M[i]) base[i] -= M[i];
        }
        for (int s = 0; s < kAllpass; ++s) {
            base[kCombs + s] += sc;
            if (base[kCombs + s] >= ap.m[s]) base[kCombs + s] -= ap.m[s];
        }
        __syncthreads();
    }
    __syncthreads();
    if constexpr (AP_LDS) {
        for (int e = tid; e < nb * NC * ap.sum; e += kRenderThreads) {
            const int bk = e / ap.sum, q = e - bk * ap.sum, b = bk / NC, k = bk - b * NC;
            const int s = (q >= ap.pref[1]) + (q >= ap.pref[2]) + (q >= ap.pref[3]);
            apl[((size_t)(b * kAllpass + s) * NC + k) * a_cap + (q - ap.pref[s])] = s_apl[e];
        }
    }
    if (tid < kCombs + kAllpass) header[tid] = base[tid];
}

__global__ void k_reverb_zero(float4* __restrict__ p, long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int reverb_state_bytes(const RprReverbDesc* desc, int64_t* bytes_per_source)
{
    Geometry g;
    if (int rc = geometry(desc, &g)) return rc;
    if (!bytes_per_source) return set_error(RPR_EINVAL, "reverb_state_bytes: output is NULL");
    *bytes_per_source = g.bytes;
    return RPR_OK;
}

extern "C" int reverb_state_reset(void* state, int32_t n_src, const RprReverbDesc* desc, void* hip_stream)
{
    Geometry g;
    if (int rc = geometry(desc, &g)) return rc;
    if (n_src < 0 || (n_src > 0 && !state)) return set_error(RPR_EINVAL, "reverb_state_reset: bad argument");
    if (reinterpret_cast<uintptr_t>(state) & 15u) return set_error(RPR_EINVAL, "reverb_state_reset: state must be 16-byte aligned");
    if (n_src == 0) return RPR_OK;
    const long long n4 = (long long)n_src * g.bytes / 16;
    const long long blocks = std::min<long long>((n4 + 255) / 256, 16384);
    hipLaunchKernelGGL(k_reverb_zero, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       reinterpret_cast<float4*>(state), n4);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_setup(const RprReverbParams* params, const float* hist, int32_t n_ir, int32_t n_bins,
                            float bin_width_s, const float* z, const float* angles, int32_t first,
                            const RprReverbDesc* desc, RprReverbSetup* setup, void* hip_stream)
{
    Geometry g;
    if (int rc = geometry(desc, &g)) return rc;
    if (n_ir < 0 || n_bins < 1 || !(bin_width_s > 0.f) ||
        (n_ir > 0 && (!params || !hist || !z || !angles || !setup)))
        return set_error(RPR_EINVAL, "reverb_setup: bad argument");
    if (n_ir == 0) return RPR_OK;
    static const Quad quad = gauss_legendre();
    const double fs = (double)desc->sample_rate;
    hipLaunchKernelGGL(k_reverb_setup, dim3((unsigned)n_ir), dim3(256), 0, (hipStream_t)hip_stream, params, hist,
                       (int)n_bins, (double)bin_width_s, z, angles, first ? 1 : 0, g.nb, desc->sh_order, fs,
                       (double)desc->speed_of_sound, (double)desc->max_comb_delay_s, quad, setup);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_render(const RprReverbSetup* setup, int32_t n_src, const float* x, int32_t n, void* state,
                             float* out, const RprReverbDesc* desc, void* hip_stream)
{
    Geometry g;
    if (int rc = geometry(desc, &g)) return rc;
    if (n_src < 0 || n < 0 || (n_src > 0 && n > 0 && (!setup || !x || !state || !out)))
        return set_error(RPR_EINVAL, "reverb_render: bad argument");
    if (reinterpret_cast<uintptr_t>(state) & 15u) return set_error(RPR_EINVAL, "reverb_render: state must be 16-byte aligned");
    if (n_src == 0 || n == 0) return RPR_OK;  // nothing to render: the state is left as it is
    ApArgs ap;
    ap.sum = 0;
    for (int j = 0; j < kAllpass; ++j) {
        ap.m[j] = g.ap_m[j];
        ap.pref[j] = ap.sum;
        ap.sum += g.ap_m[j];
    }
    const size_t ap_lds = (size_t)g.nb * g.nc * ap.sum * sizeof(float);
    const bool in_lds = ap_lds + (size_t)render_static_lds(g.nc) <= (size_t)kLdsLimit;
    const dim3 grid((unsigned)n_src), block(kRenderThreads);
    hipStream_t s = (hipStream_t)hip_stream;
    char* st = reinterpret_cast<char*>(state);
    const size_t dyn = in_lds ? ap_lds : 0;
#define RPR_RENDER(NCV)                                                                                    \
    do {                                                                                                   \
        if (in_lds)                                                                                        \
            hipLaunchKernelGGL((k_reverb_render<NCV, true>), grid, block, dyn, s, setup, x, n, st, g.bytes, out, \
                               g.nb, g.m_cap, g.a_cap, ap);                                                \
        else                                                                                               \
            hipLaunchKernelGGL((k_reverb_render<NCV, false>), grid, block, 0, s, setup, x, n, st, g.bytes, out,  \
                               g.nb, g.m_cap, g.a_cap, ap);                                                \
    } while (0)
    switch (g.nc) {
    case 1: RPR_RENDER(1); break;
    case 4: RPR_RENDER(4); break;
    case 9: RPR_RENDER(9); break;
    default: RPR_RENDER(16); break;
    }
#undef RPR_RENDER
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
