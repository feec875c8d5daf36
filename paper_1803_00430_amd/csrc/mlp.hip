// Learned reverb-parameter estimator: featurisation of a cheap trace's
// histogram, a BF16 MLP trained and evaluated with hand-written matrix-core
// kernels, Gaussian negative log-likelihood, Adam, and decoding of the
// network output into reverb parameters.
//
// The paper denoises low-ray-count parameters by temporal smoothing
// (Section 4.2, Eq. 4); this estimator is the build's replacement for that
// step and has no counterpart in the paper's text.
//
// Products.  Every product is C[M][N] = A[M][K] * B[N][K]^T with both operands
// BF16 and contiguous along K ("NT"), accumulated in FP32 by
// v_mfma_f32_32x32x16_bf16:
//   forward  Z_l  = H_l   * W_l^T        A = H_l  [M][d_l],      B = W_l  [d_l+1][d_l]
//   dgrad    dH_l = G_l   * W_l          A = G_l  [M][d_l+1],    B = W_l^T [d_l][d_l+1]
//   wgrad    dW_l = G_l^T * H_l          A = G_l^T [d_l+1][M],   B = H_l^T [d_l][M]
// so the forward pass also writes each activation transposed, the loss and
// dgrad epilogues write the gradient transposed, and every Adam step refreshes
// a transposed BF16 copy of each weight matrix used by dgrad.  A workgroup of
// four waves computes a 64 x 64 tile (each wave one 32 x 32 MFMA tile);
// K is split across workgroups when the tile grid alone cannot fill the chip,
// and an epilogue kernel sums the split partials in a fixed order
// (deterministic), adds the bias, applies ReLU or the ReLU derivative mask and
// writes FP32 / BF16 / transposed-BF16 outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;

constexpr int kTile = 64;          // output tile of one workgroup (M and N)
constexpr int kKStep = 32;         // K consumed per iteration of the product loop (two MFMAs)
constexpr int kMaxBatch = 8192;
constexpr int kMaxDim = 65536;
constexpr float kFeatGain = 1.0e6f;
constexpr float kFeatScale = 0.125f;
constexpr float kEnergyFloor = 1.0e-4f;
constexpr int kStatFeatures = 64;        // trace statistics appended to every feature row
constexpr int kFeatMaxBinsBands = 7936;  // decay curves in LDS: 8 bytes each, with the 2 KB reduction buffer <= 64 KB
constexpr size_t kPartialFloats = size_t(32) << 20;  // split-K partial sums (128 MB)

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ products
// C (partial) = A[M][kb:ke] * B[N][kb:ke]^T for one 64 x 64 tile per
// workgroup; each wave owns a 32 x 32 sub-tile held in one accumulator of
// v_mfma_f32_32x32x16_bf16.  Per K-step of 32 the workgroup stages the tile's
// 64 rows of A and of B in LDS once (four threads per row, 64 contiguous
// bytes each), so no operand row is fetched twice and every fetch is a whole
// 64-byte segment; the next step's rows are loaded into registers while the
// current step's products run, and LDS is double-buffered (one barrier per
// step).  Rows are padded to 80 bytes in LDS, which puts the eight rows read
// together by a 128-bit fragment load on distinct banks.  Lane l supplies row
// (l & 31) of the A and B fragments with the 8 consecutive K entries starting
// at 8 (l >> 5); entry e of the accumulator is row 8 (e >> 2) + 4 (l >> 5) +
// (e & 3), column (l & 31) of the sub-tile.  A row past M (B row past N) is
// read from the last valid row instead: it only feeds outputs that are never
// stored.  Requires K % 32 == 0, kchunk % 32 == 0 and 16-byte aligned rows
// (lda, ldb multiples of 8).
constexpr int kLdsRow = kKStep + 8;  // BF16 per staged row (80 bytes)

__global__ void __launch_bounds__(256) k_gemm_nt(const uint16_t* __restrict__ A, int lda,
                                                 const uint16_t* __restrict__ B, int ldb, float* __restrict__ P,
                                                 int ldp, size_t split_stride, int M, int N, int K, int kchunk)
{
    __shared__ __attribute__((aligned(16))) uint16_t sa[2][kTile * kLdsRow];
    __shared__ __attribute__((aligned(16))) uint16_t sb[2][kTile * kLdsRow];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int r = lane & 31, q = lane >> 5;
    const int M0 = blockIdx.y * kTile, N0 = blockIdx.x * kTile;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int nsteps = (ke - kb) / kKStep;
    // staging: thread t copies row t / 4, K entries 8 (t % 4) .. +8 of the step
    const int srow = tid >> 2, sseg = (tid & 3) * 8;
    const uint16_t* ga = A + (size_t)min(M0 + srow, M - 1) * lda + kb + sseg;
    const uint16_t* gb = B + (size_t)min(N0 + srow, N - 1) * ldb + kb + sseg;
    const int soff = srow * kLdsRow + sseg;
    // fragments: this wave's rows of the staged tiles
    const int fa = ((wave >> 1) * 32 + r) * kLdsRow + q * 8;
    const int fb = ((wave & 1) * 32 + r) * kLdsRow + q * 8;
    f32x16_t c = {};
    uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
    if (nsteps > 0) {
        ra = *reinterpret_cast<const uint4*>(ga);
        rb = *reinterpret_cast<const uint4*>(gb);
        *reinterpret_cast<uint4*>(&sa[0][soff]) = ra;
        *reinterpret_cast<uint4*>(&sb[0][soff]) = rb;
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        const bool more = s + 1 < nsteps;
        if (more) {
            ra = *reinterpret_cast<const uint4*>(ga + (size_t)(s + 1) * kKStep);
            rb = *reinterpret_cast<const uint4*>(gb + (size_t)(s + 1) * kKStep);
        }
        const uint4 a0 = *reinterpret_cast<const uint4*>(&sa[cur][fa]);
        const uint4 a1 = *reinterpret_cast<const uint4*>(&sa[cur][fa + 16]);
        const uint4 b0 = *reinterpret_cast<const uint4*>(&sb[cur][fb]);
        const uint4 b1 = *reinterpret_cast<const uint4*>(&sb[cur][fb + 16]);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a0), __builtin_bit_cast(bf16x8_t, b0),
                                                    c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a1), __builtin_bit_cast(bf16x8_t, b1),
                                                    c, 0, 0, 0);
        if (more) {
            // the other buffer was last read in step s - 1, before that step's barrier
            *reinterpret_cast<uint4*>(&sa[cur ^ 1][soff]) = ra;
            *reinterpret_cast<uint4*>(&sb[cur ^ 1][soff]) = rb;
        }
        __syncthreads();
    }
    const int m0 = M0 + (wave >> 1) * 32;
    const int n0 = N0 + (wave & 1) * 32;
    float* out = P + blockIdx.z * split_stride;
    const int col = n0 + r;
    if (col >= N) return;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int row = m0 + 8 * (e >> 2) + 4 * q + (e & 3);
        if (row < M) out[(size_t)row * ldp + col] = c[e];
    }
}

struct Epi {
    const float* P;        // [splits][M][ldp]
    size_t split_stride;
    int splits, ldp;
    int M, N;
    const float* bias;     // [N] or null
    int relu;              // max(0, .)
    const uint16_t* mask;  // [M][ldmask] BF16 activations: zero where mask <= 0 (ReLU derivative), or null
    int ldmask;
    float* out32;          // [M][ld32] or null
    int ld32;
    uint16_t* outbf;       // [M][ldbf] or null
    int ldbf;
    uint16_t* outT;        // [N][ldT] BF16 transposed, or null; columns M..ldT-1 are written as zero
    int ldT;
};

// One 32 x 32 tile per workgroup of 256 threads (32 columns x 8 rows, 4 rows each).
__global__ void __launch_bounds__(256) k_epilogue(Epi e)
{
    __shared__ uint16_t tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + tx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = blockIdx.y * 32 + ty + 8 * i;
        float v = 0.f;
        const bool ok = m < e.M && n < e.N;
        if (ok) {
            const float* p = e.P + (size_t)m * e.ldp + n;
            for (int s = 0; s < e.splits; ++s) v += p[s * e.split_stride];
            if (e.bias) v += e.bias[n];
            if (e.relu) v = fmaxf(v, 0.f);
            if (e.mask && !(bf2f(e.mask[(size_t)m * e.ldmask + n]) > 0.f)) v = 0.f;
            if (e.out32) e.out32[(size_t)m * e.ld32 + n] = v;
            if (e.outbf) e.outbf[(size_t)m * e.ldbf + n] = f2bf(v);
        }
        tile[ty + 8 * i][tx] = ok ? f2bf(v) : (uint16_t)0;
    }
    if (!e.outT) return;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = blockIdx.x * 32 + ty + 8 * i;
        const int mm = blockIdx.y * 32 + tx;
        if (nn < e.N && mm < e.ldT) e.outT[(size_t)nn * e.ldT + mm] = tile[tx][ty + 8 * i];
    }
}

// dst[c][r] = src[row(r)][c] for r < R (row(r) = rows[r] if given, rows outside
// [0, n_rows) read as zero), zero for R <= r < Rpad.  32 x 32 tiles via LDS.
__global__ void __launch_bounds__(256) k_transpose_bf16(const uint16_t* __restrict__ src, int lds,
                                                        const int32_t* __restrict__ rows, long long n_rows, int R,
                                                        int Cn, uint16_t* __restrict__ dst, int ldd, int Rpad)
{
    __shared__ uint16_t tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = blockIdx.y * 32 + ty + 8 * i;
        const int c = blockIdx.x * 32 + tx;
        uint16_t v = 0;
        if (r < R && c < Cn) {
            const long long sr = rows ? (long long)rows[r] : (long long)r;
            if (sr >= 0 && sr < n_rows) v = src[(size_t)sr * lds + c];
        }
        tile[ty + 8 * i][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = blockIdx.x * 32 + ty + 8 * i;
        const int r = blockIdx.y * 32 + tx;
        if (c < Cn && r < Rpad) dst[(size_t)c * ldd + r] = tile[tx][ty + 8 * i];
    }
}

// X[i][:] = features[rows[i]][:] (zero row when out of range); 8 BF16 per thread.
__global__ void k_gather_rows(const uint16_t* __restrict__ src, long long n_rows, const int32_t* __restrict__ rows,
                              int M, int F, uint16_t* __restrict__ dst)
{
    const int per_row = F / 8;
    const long long total = (long long)M * per_row;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / per_row), c = (int)(idx % per_row);
        const long long sr = rows ? (long long)rows[i] : (long long)i;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (sr >= 0 && sr < n_rows) v = reinterpret_cast<const uint4*>(src + (size_t)sr * F)[c];
        reinterpret_cast<uint4*>(dst + (size_t)i * F)[c] = v;
    }
}

// ------------------------------------------------------------------ loss
// Gaussian NLL of M rows (one workgroup, fixed reduction order):
// loss = (1/M) sum_i sum_j w/2 ((mu - t)^2 exp(-s) + s); its gradient w.r.t.
// [mu | s] into g32 [M][2n], gbf [M][2n] and gT [2n][Mpad] (BF16, zero padded).
__global__ void __launch_bounds__(256) k_nll(const float* __restrict__ out, int n, const float* __restrict__ T,
                                             const float* __restrict__ W, const int32_t* __restrict__ rows,
                                             long long n_rows, int M, int Mpad, double* __restrict__ loss,
                                             float* __restrict__ g32, uint16_t* __restrict__ gbf,
                                             uint16_t* __restrict__ gT)
{
    __shared__ double red[256];
    const int n2 = 2 * n;
    const float invM = 1.0f / (float)M;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < M * n; idx += 256) {
        const int i = idx / n, j = idx % n;
        const long long row = rows ? (long long)rows[i] : (long long)i;
        const bool inr = row >= 0 && row < n_rows;
        const float w = inr ? W[(size_t)row * n + j] : 0.f;
        float gm = 0.f, gs = 0.f;
        if (w != 0.f) {
            const float mu = out[(size_t)i * n2 + j], s = out[(size_t)i * n2 + n + j];
            const float r = mu - T[(size_t)row * n + j];
            const float e = expf(-s);
            acc += 0.5 * (double)w * ((double)r * r * e + s);
            gm = w * r * e * invM;
            gs = 0.5f * w * (1.f - r * r * e) * invM;
        }
        g32[(size_t)i * n2 + j] = gm;
        g32[(size_t)i * n2 + n + j] = gs;
        gbf[(size_t)i * n2 + j] = f2bf(gm);
        gbf[(size_t)i * n2 + n + j] = f2bf(gs);
        gT[(size_t)j * Mpad + i] = f2bf(gm);
        gT[(size_t)(n + j) * Mpad + i] = f2bf(gs);
    }
    const int pad = Mpad - M;
    for (int idx = threadIdx.x; idx < pad * n2; idx += 256) gT[(size_t)(idx / pad) * Mpad + M + idx % pad] = 0;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)M;
}

// db[j] = sum_i g[i][j] (fixed order per column).
__global__ void k_colsum(const float* __restrict__ g, int M, int N, float* __restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += g[(size_t)i * N + j];
    db[j] = s;
}

// ------------------------------------------------------------------ optimiser
// Adam with bias correction (ic1 = 1/(1-beta1^t), ic2 = 1/(1-beta2^t)) and
// decoupled weight decay; writes the BF16 copy of the updated values if asked.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float wd,
                       float ic1, float ic2, uint16_t* __restrict__ pbf)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float pi = p[i];
        if (wd != 0.f) pi -= lr * wd * pi;
        pi -= lr * (mi * ic1) / (sqrtf(vi * ic2) + eps);
        p[i] = pi;
        if (pbf) pbf[i] = f2bf(pi);
    }
}

// Two-tower structure of layer 0 (reverb_model_set_tower).  Rows r < tw
// read the first n_hist inputs only; with S = d0 - n_hist statistics inputs,
// row tw + j (j < S) passes input n_hist + j through with weight +1 and row
// tw + S + j with weight -1, bias 0, so that after the ReLU layer 1 sees
// [tower(histogram) | max(s, 0) | max(-s, 0)].  The fixed entries are
// written into the FP32 weights, their BF16 copy and the bias.
__global__ void k_tower_structure(float* __restrict__ W, float* __restrict__ b, uint16_t* __restrict__ wbf, int d0,
                                  int d1, int n_hist, int tw)
{
    const int S = d0 - n_hist;
    const long long n = (long long)d1 * d0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i / d0), c = (int)(i % d0);
        if (r < tw) {
            if (c >= n_hist) {
                W[i] = 0.f;
                wbf[i] = 0;
            }
        } else {
            const int j = r - tw;
            const float v = c == n_hist + (j % S) ? (j < S ? 1.f : -1.f) : 0.f;
            W[i] = v;
            wbf[i] = f2bf(v);
        }
    }
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x + tw; r < d1;
         r += (long long)gridDim.x * blockDim.x)
        b[r] = 0.f;
}

__global__ void k_to_bf16(const float* __restrict__ src, long long n, uint16_t* __restrict__ dst)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = f2bf(src[i]);
}

// Per-feature mean (FP64, fixed order) and scale = gain / max(std, 1e-3)
// over n rows of BF16 features [n][F]; gain = sqrt((F - F_hist) / F_hist) for
// the first F_hist (histogram) features and 1 for the rest.  One thread per
// feature, two passes over the rows (mean, then squared deviations).
__global__ void k_feature_stats(const uint16_t* __restrict__ x, long long n, int F, int F_hist,
                                float* __restrict__ mean, float* __restrict__ scale)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double s = 0.0;
    for (long long i = 0; i < n; ++i) s += (double)bf2f(x[(size_t)i * F + f]);
    const double mu = s / (double)n;
    double v = 0.0;
    for (long long i = 0; i < n; ++i) {
        const double d = (double)bf2f(x[(size_t)i * F + f]) - mu;
        v += d * d;
    }
    const double sd = sqrt(v / (double)n);
    const double gain = (f < F_hist && F_hist > 0) ? sqrt((double)(F - F_hist) / (double)F_hist) : 1.0;
    mean[f] = (float)mu;
    scale[f] = (float)(gain / fmax(sd, 1e-3));
}

// x = (x - shift[f]) * scale[f], rounded to BF16, in place.
__global__ void k_normalize(uint16_t* __restrict__ x, long long n, int F, const float* __restrict__ shift,
                            const float* __restrict__ scale)
{
    const long long total = n * (long long)F;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int f = (int)(i % F);
        x[i] = f2bf((bf2f(x[i]) - shift[f]) * scale[f]);
    }
}

// Input-support gate: row i is flagged uncertain (uncertain[i] = 1 and
// RPR_ST_UNCERTAIN in every band's status) when any of its normalised features
// in columns [c0, c1) lies beyond +-zmax.  One wave per row.
__global__ void __launch_bounds__(64) k_ood_gate(const uint16_t* __restrict__ x, int F, int c0, int c1, float zmax,
                                                 int n_bands, RprReverbParams* __restrict__ params,
                                                 int32_t* __restrict__ uncertain)
{
    const uint16_t* r = x + (size_t)blockIdx.x * F;
    bool out = false;
    for (int c = c0 + threadIdx.x; c < c1; c += 64) out |= !(fabsf(bf2f(r[c])) <= zmax);
    if (__builtin_amdgcn_ballot_w64(out) == 0) return;
    if (threadIdx.x == 0) {
        if (uncertain) uncertain[blockIdx.x] = 1;
        if (params)
            for (int b = 0; b < n_bands; ++b) params[blockIdx.x].status[b] |= RPR_ST_UNCERTAIN;
    }
}

__global__ void k_zero_f32(float* __restrict__ p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// Uniform initialisation in [-bound, bound] from Philox4x32-10 with the
// counter (element, layer, 0x4d4c5000, 0) under the key (seed lo, seed hi).
__global__ void k_init_uniform(float* __restrict__ p, long long n, int layer, float bound, uint32_t k0, uint32_t k1)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const uint4 x = rpr::philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)layer, 0x4d4c5000u),
                                           k0, k1);
        p[i] = (2.f * rpr::u01(x.x) - 1.f) * bound;
    }
}

// ------------------------------------------------------------------ features, targets, decoding
// One workgroup per IR.  e_in = sqrt(4 pi) / B * sum_{m,b} H[m][b][0] (FP64,
// fixed order).  Channel 0 of every band becomes its Schroeder decay curve:
// one thread per band sums S_b[m] = sum_{j>=m} sqrt(4 pi) H[j][b][0] from the
// last bin down in FP64 (kept in LDS), bin 0 then holds ln(S_b[0] / e_in) and
// bins m >= 1 hold 10 log10(S_b[m] / S_b[0]) / 60 clipped at -1.  The other
// channels hold sign(u) log1p(gain |u|) scale with u = H / e_in.
__global__ void __launch_bounds__(256) k_featurize(const float* __restrict__ hist,
                                                   const RprIrStats* __restrict__ stats, int T, int B, int NC,
                                                   uint16_t* __restrict__ feat, float* __restrict__ e_in)
{
    __shared__ double red[256];
    extern __shared__ double sS[];  // [B][T]
    const size_t F = (size_t)T * B * NC;
    const float* h = hist + blockIdx.x * F;
    uint16_t* f = feat + blockIdx.x * (F + kStatFeatures);
    // statistics block: the ray population's energies relative to the emitted
    // energy (log, floored), mean free path, segments per ray, escapes, first bins
    if (threadIdx.x < kStatFeatures) {
        const int j = threadIdx.x;
        float v = 0.f;
        if (stats) {
            const RprIrStats& S = stats[blockIdx.x];
            if (S.n_rays > 0 && S.e_emitted > 0.0) {
                const double em = S.e_emitted;
                if (j < 4 * B) {
                    const int b = j / 4, q = j % 4;
                    const double x = q == 0 ? S.e_alive_at_stop[b] : q == 1 ? S.e_absorbed[b]
                                     : q == 2 ? S.e_escaped[b] : S.e_alive_at_bounce_cap[b];
                    const double fl = q == 0 ? 1e-300 : q == 2 ? 1e-12 : 1e-30;
                    const double r = log(fmax(x / em, fl));
                    // [4b]: log of the population's decay exponent; others: log fractions
                    v = q == 0 ? (float)(log(fmax(-r, 1e-3)) / 5.0) : (float)(r / (q == 3 ? 60.0 : 10.0));
                } else if (j == 32) {
                    v = (S.n_finite_segments > 0 && S.seg_len_sum > 0.0)
                            ? (float)(log(S.seg_len_sum / (double)S.n_finite_segments) / 3.0) : 0.f;
                } else if (j == 33) {
                    v = (float)(log((double)S.n_segments / (double)S.n_rays) / 5.0);
                } else if (j == 34) {
                    v = (float)((double)S.n_escaped / (double)S.n_rays);
                } else if (j == 35) {
                    v = (float)((double)min(S.first_arrival_bin, T) / (double)T);
                } else if (j == 36) {
                    v = (float)((double)min(S.first_late_bin, T) / (double)T);
                }
            }
        }
        f[F + j] = f2bf(v);
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < T * B; i += 256) s += (double)h[(size_t)i * NC];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double e = red[0] * 3.5449077018110318 / (double)B;  // sqrt(4 pi)
    if (threadIdx.x == 0) e_in[blockIdx.x] = (float)e;
    if (!(e > 0.0)) {
        for (size_t i = threadIdx.x; i < F; i += 256) f[i] = 0;
        return;
    }
    if ((int)threadIdx.x < B) {
        const int b = threadIdx.x;
        double acc = 0.0;
        for (int m = T - 1; m >= 0; --m) {
            acc += 3.5449077018110318 * (double)h[((size_t)m * B + b) * NC];
            sS[b * T + m] = acc;
        }
    }
    __syncthreads();
    const float inv = (float)(1.0 / e);
    for (size_t i = threadIdx.x; i < F; i += 256) {
        const int k = (int)(i % NC);
        if (k == 0) {
            const int b = (int)((i / NC) % B), m = (int)(i / ((size_t)NC * B));
            const double S0 = sS[b * T];
            float v = 0.f;
            if (S0 > 0.0) {
                if (m == 0) {
                    v = (float)log(S0 / e);
                } else {
                    const double db = 10.0 * log10(sS[b * T + m] / S0);
                    v = (float)(fmax(db, -60.0) / 60.0);
                }
            }
            f[i] = f2bf(v);
        } else {
            const float u = h[i] * inv;
            f[i] = f2bf(copysignf(log1pf(kFeatGain * fabsf(u)), u) * kFeatScale);
        }
    }
}

__global__ void k_targets(const RprReverbParams* __restrict__ ref, const float* __restrict__ e_in, int n, int B,
                          float* __restrict__ t, float* __restrict__ w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RprReverbParams& p = ref[i];
    const float e = e_in[i];
    float* ti = t + (size_t)i * 4 * B;
    float* wi = w + (size_t)i * 4 * B;
    for (int b = 0; b < B; ++b) {
        const bool ok = p.rt60[b] > 0.f &&
                        !(p.status[b] & (RPR_ST_NO_ENERGY | RPR_ST_BAD_FIT | RPR_ST_NO_RANGE));
        ti[b] = ok ? logf(p.rt60[b]) : 0.f;
        wi[b] = ok ? 1.f : 0.f;
        const float cls[3] = {p.e_direct[b], p.e_early[b], p.e_late[b]};
        for (int c = 0; c < 3; ++c) {
            const bool ek = e > 0.f;
            ti[(c + 1) * B + b] = ek ? logf(cls[c] / e + kEnergyFloor) : 0.f;
            wi[(c + 1) * B + b] = ek ? 1.f : 0.f;
        }
    }
}

__global__ void k_decode(const float* __restrict__ out, const float* __restrict__ e_in, long long n, int B,
                         float kappa, RprReverbParams* __restrict__ params, float* __restrict__ sigma,
                         int32_t* __restrict__ uncertain)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* o = out + i * 8 * B;
    const float e = e_in[i];
    RprReverbParams p = {};
    bool unc = !(e > 0.f);
    for (int b = 0; b < B; ++b) {
        const float sg = expf(0.5f * o[4 * B + b]);
        if (!(sg <= kappa)) unc = true;
        if (sigma) sigma[i * B + b] = sg;
        p.rt60[b] = expf(o[b]);
        p.rt60_range[b] = -1;
        p.e_direct[b] = fmaxf(expf(o[B + b]) - kEnergyFloor, 0.f) * e;
        p.e_early[b] = fmaxf(expf(o[2 * B + b]) - kEnergyFloor, 0.f) * e;
        p.e_late[b] = fmaxf(expf(o[3 * B + b]) - kEnergyFloor, 0.f) * e;
        p.g_reverb[b] = sqrtf(p.e_late[b] * 13.815510557964274f / p.rt60[b]);  // 6 ln 10
    }
    for (int b = 0; b < B; ++b) p.status[b] = RPR_ST_LEARNED | (unc ? RPR_ST_UNCERTAIN : 0);
    params[i] = p;
    if (uncertain) uncertain[i] = unc ? 1 : 0;
}

__global__ void k_scatter_params(const RprReverbParams* __restrict__ src, const int32_t* __restrict__ idx,
                                 long long n, RprReverbParams* __restrict__ dst)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}

unsigned grid_for(long long n, int threads = 256)
{
    return (unsigned)std::max<long long>(1, std::min<long long>((n + threads - 1) / threads, 65536));
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

struct RprModel {
    int device = 0;
    int L = 0;
    int dims[RPR_MODEL_MAX_LAYERS + 1] = {};
    int max_batch = 0;
    int mpad = 0;               // max_batch rounded up to 32
    int maxd = 0;               // widest layer
    int64_t n_params = 0;
    int64_t woff[RPR_MODEL_MAX_LAYERS] = {}, boff[RPR_MODEL_MAX_LAYERS] = {};
    int64_t step = 0;
    void* block = nullptr;      // one allocation for everything below
    float* params = nullptr;    // FP32 master weights
    float* grads = nullptr;
    float* m1 = nullptr;        // Adam moments
    float* m2 = nullptr;
    uint16_t* wbf[RPR_MODEL_MAX_LAYERS] = {};  // W_l [d_l+1][d_l] BF16
    uint16_t* wt[RPR_MODEL_MAX_LAYERS] = {};   // W_l^T [d_l][d_l+1] BF16 (l >= 1)
    uint16_t* x = nullptr;      // gathered features [max_batch][d_0]
    uint16_t* xt = nullptr;     // [d_0][mpad]
    uint16_t* hbf[RPR_MODEL_MAX_LAYERS] = {};  // activations h_l [max_batch][d_l], l = 1..L-1
    uint16_t* ht[RPR_MODEL_MAX_LAYERS] = {};   // [d_l][mpad]
    float* out = nullptr;       // [max_batch][d_L]
    float* g32 = nullptr;       // [max_batch][maxd]
    uint16_t* gbf[2] = {};      // [max_batch][maxd]
    uint16_t* gt[2] = {};       // [maxd][mpad]
    float* partial = nullptr;   // split-K partial sums
    int tower_hist = 0;         // two-tower layer 0 (reverb_model_set_tower): histogram inputs, or 0
    int tower_w = 0;            // tower width
};

namespace {

using rpr::set_error;

// Z = A * B^T through split-K partials and the epilogue `e` (whose P, splits,
// ldp, split_stride, M, N are filled in here).  When no epilogue work is
// asked beyond an FP32 store and one split suffices, the product is stored
// straight into e.out32.
int gemm(RprModel& md, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K, Epi e,
         hipStream_t st)
{
    if (M <= 0 || N <= 0) return RPR_OK;
    const int tiles = ((N + kTile - 1) / kTile) * ((M + kTile - 1) / kTile);
    const int ksteps = K / kKStep;
    const int want = std::max(1, (2 * rpr::device_cu_count() + tiles - 1) / tiles);
    int splits = std::max(1, std::min(want, ksteps / 8));
    while (splits > 1 && (size_t)splits * M * N > kPartialFloats) --splits;
    const int kchunk = ((ksteps + splits - 1) / splits) * kKStep;
    splits = (K + kchunk - 1) / kchunk;
    const bool direct = splits == 1 && e.out32 && !e.bias && !e.relu && !e.mask && !e.outbf && !e.outT;
    if (!direct && (size_t)splits * M * N > kPartialFloats)
        return set_error(RPR_EUNSUPPORTED, "product of %d x %d exceeds the workspace", M, N);
    float* P = direct ? e.out32 : md.partial;
    const int ldp = direct ? e.ld32 : N;
    const size_t stride = (size_t)M * N;
    hipLaunchKernelGGL(k_gemm_nt, dim3((N + kTile - 1) / kTile, (M + kTile - 1) / kTile, splits), dim3(256), 0, st,
                       A, lda, B, ldb, P, ldp, stride, M, N, K, kchunk);
    RPR_HIP_TRY(hipGetLastError());
    if (direct) return RPR_OK;
    e.P = md.partial;
    e.split_stride = stride;
    e.splits = splits;
    e.ldp = N;
    e.M = M;
    e.N = N;
    hipLaunchKernelGGL(k_epilogue, dim3((N + 31) / 32, (M + 31) / 32), dim3(256), 0, st, e);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

Epi epi0()
{
    Epi e{};
    return e;
}

// Forward of M rows of X ([M][d_0] BF16).  Hidden activations go to hbf (and,
// when training, transposed to ht); the output to `out` ([M][d_L] FP32).
int forward(RprModel& md, const uint16_t* X, int M, bool training, float* out, hipStream_t st)
{
    const int Mp = round_up(M, 32);
    for (int l = 0; l < md.L; ++l) {
        const uint16_t* A = l == 0 ? X : md.hbf[l];
        Epi e = epi0();
        e.bias = md.params + md.boff[l];
        if (l < md.L - 1) {
            e.relu = 1;
            e.outbf = md.hbf[l + 1];
            e.ldbf = md.dims[l + 1];
            if (training) {
                e.outT = md.ht[l + 1];
                e.ldT = Mp;
            }
        } else {
            e.out32 = out;
            e.ld32 = md.dims[md.L];
        }
        const int rc = gemm(md, A, md.dims[l], md.wbf[l], md.dims[l], M, md.dims[l + 1], md.dims[l], e, st);
        if (rc != RPR_OK) return rc;
    }
    return RPR_OK;
}

int refresh_bf16(RprModel& md, hipStream_t st)
{
    for (int l = 0; l < md.L; ++l) {
        const long long n = (long long)md.dims[l + 1] * md.dims[l];
        hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, st, md.params + md.woff[l], n, md.wbf[l]);
        if (l > 0) {
            hipLaunchKernelGGL(k_transpose_bf16, dim3((md.dims[l] + 31) / 32, (md.dims[l + 1] + 31) / 32),
                               dim3(256), 0, st, md.wbf[l], md.dims[l], nullptr, (long long)md.dims[l + 1],
                               md.dims[l + 1], md.dims[l], md.wt[l], md.dims[l + 1], md.dims[l + 1]);
        }
    }
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

int zero_moments(RprModel& md, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(md.n_params)), dim3(256), 0, st, md.m1, (long long)md.n_params);
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(md.n_params)), dim3(256), 0, st, md.m2, (long long)md.n_params);
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(md.n_params)), dim3(256), 0, st, md.grads, (long long)md.n_params);
    RPR_HIP_TRY(hipGetLastError());
    md.step = 0;
    return RPR_OK;
}

int check_model(const RprModel* md)
{
    if (!md) return set_error(RPR_EINVAL, "model is NULL");
    int dev = -1;
    RPR_HIP_TRY(hipGetDevice(&dev));
    if (dev != md->device) return set_error(RPR_EINVAL, "model lives on device %d, current device is %d", md->device, dev);
    return RPR_OK;
}

int backward_impl(RprModel& md, const uint16_t* features, int64_t n_rows, const int32_t* rows, int32_t m,
                  const float* t, const float* w, double* loss, hipStream_t st)
{
    const int L = md.L;
    const int Mp = round_up(m, 32);
    const int d0 = md.dims[0];
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((long long)m * d0 / 8)), dim3(256), 0, st, features,
                       (long long)n_rows, rows, m, d0, md.x);
    hipLaunchKernelGGL(k_transpose_bf16, dim3((d0 + 31) / 32, Mp / 32), dim3(256), 0, st, features, d0, rows,
                       (long long)n_rows, m, d0, md.xt, Mp, Mp);
    RPR_HIP_TRY(hipGetLastError());
    int rc = forward(md, md.x, m, true, md.out, st);
    if (rc != RPR_OK) return rc;
    int cur = 0;
    hipLaunchKernelGGL(k_nll, dim3(1), dim3(256), 0, st, md.out, md.dims[L] / 2, t, w, rows, (long long)n_rows, m, Mp,
                       loss, md.g32, md.gbf[cur], md.gt[cur]);
    RPR_HIP_TRY(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        const int dout = md.dims[l + 1], din = md.dims[l];
        // dW_l = G^T H_l
        Epi ew = epi0();
        ew.out32 = md.grads + md.woff[l];
        ew.ld32 = din;
        rc = gemm(md, md.gt[cur], Mp, l == 0 ? md.xt : md.ht[l], Mp, dout, din, Mp, ew, st);
        if (rc != RPR_OK) return rc;
        hipLaunchKernelGGL(k_colsum, dim3((dout + 255) / 256), dim3(256), 0, st, md.g32, m, dout,
                           md.grads + md.boff[l]);
        RPR_HIP_TRY(hipGetLastError());
        if (l == 0) break;
        // dH_l = G W_l, masked by the ReLU derivative of layer l-1's output
        const int nxt = cur ^ 1;
        Epi ed = epi0();
        ed.mask = md.hbf[l];
        ed.ldmask = din;
        ed.out32 = md.g32;
        ed.ld32 = din;
        ed.outbf = md.gbf[nxt];
        ed.ldbf = din;
        ed.outT = md.gt[nxt];
        ed.ldT = Mp;
        rc = gemm(md, md.gbf[cur], dout, md.wt[l], dout, m, din, dout, ed, st);
        if (rc != RPR_OK) return rc;
        cur = nxt;
    }
    return RPR_OK;
}

void apply_tower(RprModel& md, hipStream_t st)
{
    const long long n = (long long)md.dims[1] * md.dims[0];
    hipLaunchKernelGGL(k_tower_structure, dim3(grid_for(n)), dim3(256), 0, st, md.params + md.woff[0],
                       md.params + md.boff[0], md.wbf[0], md.dims[0], md.dims[1], md.tower_hist, md.tower_w);
}

int adam_impl(RprModel& md, const RprAdamParams* ap, hipStream_t st)
{
    if (!ap) return set_error(RPR_EINVAL, "adam parameters are NULL");
    if (!(ap->lr >= 0.f) || !(ap->beta1 >= 0.f && ap->beta1 < 1.f) || !(ap->beta2 >= 0.f && ap->beta2 < 1.f) ||
        !(ap->eps >= 0.f) || !(ap->weight_decay >= 0.f))
        return set_error(RPR_EINVAL, "invalid Adam parameters");
    md.step += 1;
    const double ic1 = 1.0 / (1.0 - std::pow((double)ap->beta1, (double)md.step));
    const double ic2 = 1.0 / (1.0 - std::pow((double)ap->beta2, (double)md.step));
    for (int l = 0; l < md.L; ++l) {
        const long long nw = (long long)md.dims[l + 1] * md.dims[l];
        hipLaunchKernelGGL(k_adam, dim3(grid_for(nw)), dim3(256), 0, st, md.params + md.woff[l],
                           md.grads + md.woff[l], md.m1 + md.woff[l], md.m2 + md.woff[l], nw, ap->lr, ap->beta1,
                           ap->beta2, ap->eps, ap->weight_decay, (float)ic1, (float)ic2, md.wbf[l]);
        const long long nb = md.dims[l + 1];
        hipLaunchKernelGGL(k_adam, dim3(grid_for(nb)), dim3(256), 0, st, md.params + md.boff[l],
                           md.grads + md.boff[l], md.m1 + md.boff[l], md.m2 + md.boff[l], nb, ap->lr, ap->beta1,
                           ap->beta2, ap->eps, 0.f, (float)ic1, (float)ic2, (uint16_t*)nullptr);
        if (l == 0 && md.tower_w > 0) apply_tower(md, st);
        if (l > 0) {
            hipLaunchKernelGGL(k_transpose_bf16, dim3((md.dims[l] + 31) / 32, (md.dims[l + 1] + 31) / 32),
                               dim3(256), 0, st, md.wbf[l], md.dims[l], nullptr, (long long)md.dims[l + 1],
                               md.dims[l + 1], md.dims[l], md.wt[l], md.dims[l + 1], md.dims[l + 1]);
        }
    }
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

}  // namespace

extern "C" int reverb_model_create(const int32_t* dims, int32_t n_layers, int32_t max_batch, uint64_t seed,
                                   void* hip_stream, RprModel** out)
{
    if (!out) return set_error(RPR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dims) return set_error(RPR_EINVAL, "dims is NULL");
    if (n_layers < 1 || n_layers > RPR_MODEL_MAX_LAYERS)
        return set_error(RPR_EINVAL, "n_layers must be in 1..%d", RPR_MODEL_MAX_LAYERS);
    for (int l = 0; l <= n_layers; ++l)
        if (dims[l] < 32 || dims[l] > kMaxDim || dims[l] % 32)
            return set_error(RPR_EINVAL, "dims[%d] = %d: must be a positive multiple of 32 <= %d", l, dims[l], kMaxDim);
    if (max_batch < 1 || max_batch > kMaxBatch)
        return set_error(RPR_EINVAL, "max_batch must be in 1..%d", kMaxBatch);
    for (int l = 0; l <= n_layers; ++l)
        if ((size_t)max_batch * dims[l] > kPartialFloats)
            return set_error(RPR_EINVAL, "max_batch x dims[%d] exceeds the product workspace (%zu floats)", l,
                             kPartialFloats);
    auto* md = new RprModel();
    RPR_HIP_TRY(hipGetDevice(&md->device));
    md->L = n_layers;
    for (int l = 0; l <= n_layers; ++l) {
        md->dims[l] = dims[l];
        md->maxd = std::max(md->maxd, (int)dims[l]);
    }
    md->max_batch = max_batch;
    md->mpad = round_up(max_batch, 32);
    int64_t np = 0;
    for (int l = 0; l < n_layers; ++l) {
        md->woff[l] = np;
        np += (int64_t)dims[l + 1] * dims[l];
        md->boff[l] = np;
        np += dims[l + 1];
    }
    md->n_params = np;
    // carve one allocation (256-byte aligned pieces)
    std::vector<std::pair<void**, size_t>> parts;
    parts.push_back({(void**)&md->params, sizeof(float) * np});
    parts.push_back({(void**)&md->grads, sizeof(float) * np});
    parts.push_back({(void**)&md->m1, sizeof(float) * np});
    parts.push_back({(void**)&md->m2, sizeof(float) * np});
    for (int l = 0; l < n_layers; ++l) {
        parts.push_back({(void**)&md->wbf[l], 2ull * dims[l + 1] * dims[l]});
        if (l > 0) parts.push_back({(void**)&md->wt[l], 2ull * dims[l + 1] * dims[l]});
        if (l > 0) {
            parts.push_back({(void**)&md->hbf[l], 2ull * max_batch * dims[l]});
            parts.push_back({(void**)&md->ht[l], 2ull * dims[l] * md->mpad});
        }
    }
    parts.push_back({(void**)&md->x, 2ull * max_batch * dims[0]});
    parts.push_back({(void**)&md->xt, 2ull * dims[0] * md->mpad});
    parts.push_back({(void**)&md->out, sizeof(float) * max_batch * dims[n_layers]});
    parts.push_back({(void**)&md->g32, sizeof(float) * max_batch * md->maxd});
    for (int i = 0; i < 2; ++i) {
        parts.push_back({(void**)&md->gbf[i], 2ull * max_batch * md->maxd});
        parts.push_back({(void**)&md->gt[i], 2ull * md->maxd * md->mpad});
    }
    parts.push_back({(void**)&md->partial, sizeof(float) * kPartialFloats});
    size_t total = 0;
    for (auto& p : parts) total += (p.second + 255) / 256 * 256;
    hipError_t e = hipMalloc(&md->block, total);
    if (e != hipSuccess) {
        delete md;
        return set_error(e == hipErrorOutOfMemory ? RPR_ENOMEM : RPR_EDEVICE, "model allocation of %zu bytes: %s",
                         total, hipGetErrorString(e));
    }
    size_t off = 0;
    for (auto& p : parts) {
        *p.first = (char*)md->block + off;
        off += (p.second + 255) / 256 * 256;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    int rc = RPR_OK;
    for (int l = 0; l < n_layers; ++l) {
        const long long nw = (long long)dims[l + 1] * dims[l];
        float bound = std::sqrt(6.0f / (float)dims[l]);
        if (l == n_layers - 1) bound *= 0.1f;
        hipLaunchKernelGGL(k_init_uniform, dim3(grid_for(nw)), dim3(256), 0, st, md->params + md->woff[l], nw, l,
                           bound, k0, k1);
        hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(dims[l + 1])), dim3(256), 0, st, md->params + md->boff[l],
                           (long long)dims[l + 1]);
    }
    if (hipGetLastError() != hipSuccess) rc = set_error(RPR_EDEVICE, "model initialisation launch failed");
    if (rc == RPR_OK) rc = refresh_bf16(*md, st);
    if (rc == RPR_OK) rc = zero_moments(*md, st);
    if (rc == RPR_OK && hipStreamSynchronize(st) != hipSuccess) rc = set_error(RPR_EDEVICE, "model initialisation");
    if (rc != RPR_OK) {
        (void)hipFree(md->block);
        delete md;
        return rc;
    }
    *out = md;
    return RPR_OK;
}

extern "C" int reverb_model_set_tower(RprModel* model, int32_t n_hist, int32_t tower_width, void* hip_stream)
{
    if (!model) return set_error(RPR_EINVAL, "model is NULL");
    RprModel& md = *model;
    if (n_hist == 0 && tower_width == 0) {
        md.tower_hist = md.tower_w = 0;
        return RPR_OK;
    }
    if (md.L < 2) return set_error(RPR_EINVAL, "a two-tower layer 0 needs at least two layers");
    if (n_hist < 1 || n_hist >= md.dims[0])
        return set_error(RPR_EINVAL, "n_hist = %d must be in 1..%d", n_hist, md.dims[0] - 1);
    const int S = md.dims[0] - n_hist;
    if (tower_width < 1 || md.dims[1] != tower_width + 2 * S)
        return set_error(RPR_EINVAL, "dims[1] = %d must equal tower_width + 2 x %d statistics inputs", md.dims[1], S);
    md.tower_hist = n_hist;
    md.tower_w = tower_width;
    apply_tower(md, (hipStream_t)hip_stream);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_destroy(RprModel* model)
{
    if (!model) return RPR_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(model->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(model->block);
    (void)hipSetDevice(prev);
    delete model;
    return RPR_OK;
}

extern "C" int reverb_model_info(const RprModel* model, RprModelInfo* out)
{
    if (!model || !out) return set_error(RPR_EINVAL, "model or out is NULL");
    *out = RprModelInfo{};
    out->n_params = model->n_params;
    out->n_layers = model->L;
    for (int l = 0; l <= model->L; ++l) out->dims[l] = model->dims[l];
    out->max_batch = model->max_batch;
    out->step = model->step;
    return RPR_OK;
}

extern "C" int reverb_model_load(RprModel* model, const float* params, int64_t n, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    if (!params || n != model->n_params)
        return set_error(RPR_EINVAL, "load: expected %lld parameters", (long long)model->n_params);
    hipStream_t st = (hipStream_t)hip_stream;
    RPR_HIP_TRY(hipMemcpyAsync(model->params, params, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    rc = refresh_bf16(*model, st);
    if (rc != RPR_OK) return rc;
    if (model->tower_w > 0) apply_tower(*model, st);
    return zero_moments(*model, st);
}

extern "C" int reverb_model_save(const RprModel* model, float* params, int64_t n, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    if (!params || n != model->n_params)
        return set_error(RPR_EINVAL, "save: expected %lld parameters", (long long)model->n_params);
    RPR_HIP_TRY(hipMemcpyAsync(params, model->params, sizeof(float) * n, hipMemcpyDeviceToDevice,
                               (hipStream_t)hip_stream));
    return RPR_OK;
}

extern "C" int reverb_model_grads(const RprModel* model, float* grads, int64_t n, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    if (!grads || n != model->n_params)
        return set_error(RPR_EINVAL, "grads: expected %lld values", (long long)model->n_params);
    RPR_HIP_TRY(hipMemcpyAsync(grads, model->grads, sizeof(float) * n, hipMemcpyDeviceToDevice,
                               (hipStream_t)hip_stream));
    return RPR_OK;
}

extern "C" int reverb_model_featurize(const float* hist, const RprIrStats* stats, int32_t n_ir, int32_t n_bins,
                                      int32_t n_bands, int32_t n_coeffs, uint16_t* features, float* e_in,
                                      void* hip_stream)
{
    if (n_ir < 0 || n_bins < 1 || n_bands < 1 || n_bands > RPR_MAX_BANDS || n_coeffs < 1 ||
        n_coeffs > RPR_MAX_COEFFS)
        return set_error(RPR_EINVAL, "featurize: invalid sizes");
    if (n_ir == 0) return RPR_OK;
    if (!hist || !features || !e_in) return set_error(RPR_EINVAL, "featurize: NULL buffer");
    if ((int64_t)n_bins * n_bands > kFeatMaxBinsBands)
        return set_error(RPR_EUNSUPPORTED, "featurize: n_bins x n_bands must be <= %d", kFeatMaxBinsBands);
    hipLaunchKernelGGL(k_featurize, dim3(n_ir), dim3(256), sizeof(double) * n_bins * n_bands,
                       (hipStream_t)hip_stream, hist, stats, n_bins, n_bands, n_coeffs, features, e_in);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_targets(const RprReverbParams* ref, const float* e_in, int32_t n_ir, int32_t n_bands,
                                    float* t, float* w, void* hip_stream)
{
    if (n_ir < 0 || n_bands < 1 || n_bands > RPR_MAX_BANDS) return set_error(RPR_EINVAL, "targets: invalid sizes");
    if (n_ir == 0) return RPR_OK;
    if (!ref || !e_in || !t || !w) return set_error(RPR_EINVAL, "targets: NULL buffer");
    hipLaunchKernelGGL(k_targets, dim3((n_ir + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, ref, e_in, n_ir,
                       n_bands, t, w);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_forward(RprModel* model, const uint16_t* features, int64_t n, float* out,
                                    void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    if (n < 0) return set_error(RPR_EINVAL, "forward: n < 0");
    if (n == 0) return RPR_OK;
    if (!features || !out) return set_error(RPR_EINVAL, "forward: NULL buffer");
    hipStream_t st = (hipStream_t)hip_stream;
    for (int64_t c = 0; c < n; c += model->max_batch) {
        const int m = (int)std::min<int64_t>(model->max_batch, n - c);
        rc = forward(*model, features + c * model->dims[0], m, false, out + c * model->dims[model->L], st);
        if (rc != RPR_OK) return rc;
    }
    return RPR_OK;
}

static int check_batch_args(const RprModel* model, const uint16_t* features, int64_t n_rows, int32_t m,
                            const float* t, const float* w, const double* loss)
{
    if (m < 1 || m > model->max_batch) return set_error(RPR_EINVAL, "m must be in 1..max_batch (%d)", model->max_batch);
    if (n_rows < 1) return set_error(RPR_EINVAL, "n_rows must be >= 1");
    if (!features || !t || !w || !loss) return set_error(RPR_EINVAL, "NULL buffer");
    return RPR_OK;
}

extern "C" int reverb_model_backward(RprModel* model, const uint16_t* features, int64_t n_rows, const int32_t* rows,
                                     int32_t m, const float* t, const float* w, double* loss, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    rc = check_batch_args(model, features, n_rows, m, t, w, loss);
    if (rc != RPR_OK) return rc;
    return backward_impl(*model, features, n_rows, rows, m, t, w, loss, (hipStream_t)hip_stream);
}

extern "C" int reverb_model_adam(RprModel* model, const RprAdamParams* ap, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    return adam_impl(*model, ap, (hipStream_t)hip_stream);
}

extern "C" int reverb_model_train_step(RprModel* model, const uint16_t* features, int64_t n_rows,
                                       const int32_t* rows, int32_t m, const float* t, const float* w,
                                       const RprAdamParams* ap, double* loss, void* hip_stream)
{
    int rc = check_model(model);
    if (rc != RPR_OK) return rc;
    rc = check_batch_args(model, features, n_rows, m, t, w, loss);
    if (rc != RPR_OK) return rc;
    if (!ap) return set_error(RPR_EINVAL, "adam parameters are NULL");
    rc = backward_impl(*model, features, n_rows, rows, m, t, w, loss, (hipStream_t)hip_stream);
    if (rc != RPR_OK) return rc;
    return adam_impl(*model, ap, (hipStream_t)hip_stream);
}

extern "C" int reverb_model_decode(const float* out, const float* e_in, int64_t n, int32_t n_bands, float kappa,
                                   RprReverbParams* params, float* sigma, int32_t* uncertain, void* hip_stream)
{
    if (n < 0 || n_bands < 1 || n_bands > RPR_MAX_BANDS) return set_error(RPR_EINVAL, "decode: invalid sizes");
    if (n == 0) return RPR_OK;
    if (!out || !e_in || !params) return set_error(RPR_EINVAL, "decode: NULL buffer");
    hipLaunchKernelGGL(k_decode, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)hip_stream, out, e_in,
                       (long long)n, n_bands, kappa, params, sigma, uncertain);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_feature_stats(const uint16_t* features, int64_t n, int32_t F, int32_t F_hist,
                                          float* mean, float* scale, void* hip_stream)
{
    if (n < 1 || F < 1 || F_hist < 0 || F_hist >= F) return set_error(RPR_EINVAL, "feature_stats: invalid sizes");
    if (!features || !mean || !scale) return set_error(RPR_EINVAL, "feature_stats: NULL buffer");
    hipLaunchKernelGGL(k_feature_stats, dim3((F + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, features,
                       (long long)n, F, F_hist, mean, scale);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_normalize(uint16_t* features, int64_t n, int32_t F, const float* shift, const float* scale,
                                      void* hip_stream)
{
    if (n < 0 || F < 1) return set_error(RPR_EINVAL, "normalize: invalid sizes");
    if (n == 0) return RPR_OK;
    if (!features || !shift || !scale) return set_error(RPR_EINVAL, "normalize: NULL buffer");
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n * (long long)F)), dim3(256), 0, (hipStream_t)hip_stream, features,
                       (long long)n, F, shift, scale);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_model_ood_gate(const uint16_t* features, int64_t n, int32_t F, int32_t c0, int32_t c1,
                                     float zmax, int32_t n_bands, RprReverbParams* params, int32_t* uncertain,
                                     void* hip_stream)
{
    if (n < 0 || F < 1 || c0 < 0 || c1 > F || c0 >= c1 || !(zmax > 0.f) || n_bands < 1 || n_bands > RPR_MAX_BANDS)
        return set_error(RPR_EINVAL, "ood_gate: invalid arguments");
    if (n == 0) return RPR_OK;
    if (n > 0x7FFFFFFF) return set_error(RPR_EUNSUPPORTED, "ood_gate: too many rows");
    if (!features || (!params && !uncertain)) return set_error(RPR_EINVAL, "ood_gate: NULL buffer");
    hipLaunchKernelGGL(k_ood_gate, dim3((unsigned)n), dim3(64), 0, (hipStream_t)hip_stream, features, F, c0, c1, zmax,
                       n_bands, params, uncertain);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int reverb_params_scatter(const RprReverbParams* src, const int32_t* idx, int64_t n, RprReverbParams* dst,
                                     void* hip_stream)
{
    if (n < 0) return set_error(RPR_EINVAL, "scatter: n < 0");
    if (n == 0) return RPR_OK;
    if (!src || !idx || !dst) return set_error(RPR_EINVAL, "scatter: NULL buffer");
    hipLaunchKernelGGL(k_scatter_params, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)hip_stream,
                       src, idx, (long long)n, dst);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
