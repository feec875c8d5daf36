// Scene creation: material table, triangle records and a linear BVH.
//
// Linear BVH (Karras, HPG 2012): Morton codes (30-bit; 63-bit for large scenes) of the triangle
// centroids in the scene's centroid bounds, a stable least-significant-digit
// radix sort of (code, triangle) pairs, internal nodes from the longest common
// prefixes of neighbouring codes (ties broken by the sorted index), and
// bottom-up bounds where the second child to finish builds its parent.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

namespace rpr {
namespace {

constexpr int kBuildBlock = 256;
constexpr int kPrepBlocks = 128;  // k_prep's grid cap (it strides over the triangles)
constexpr int kSortItems = 8;
constexpr int kSortTile = kBuildBlock * kSortItems;
// Scenes of at least this many triangles get 64-bit Morton keys (21 bits per axis).
constexpr int64_t kWideKeyTris = (int64_t)1 << 19;

// Validation flags, set by the prep kernel and read back by scene_create.
enum : uint32_t {
    kBadIndex = 1u,
    kBadVertex = 2u,
    kBadMaterial = 4u,
    kBadCoeff = 8u,
    kBadTree = 16u,  // internal consistency check of the build failed
};

struct BuildFlags {
    uint32_t flags;
    int32_t max_depth;
    int32_t max_stack;  // most stack entries any root-to-leaf path of the 4-wide tree can push
    uint32_t n_nodes4;  // 4-wide nodes
    uint32_t n_degenerate;
    uint32_t pad;
    // centroid bounds as order-preserving integer keys of the floats
    int32_t clo[3], chi[3];
    int32_t blo[3], bhi[3];  // triangle bounds (all vertices)
};

__device__ __forceinline__ int32_t ordered(float f)
{
    const int32_t i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__host__ __device__ inline float unordered(int32_t i)
{
    const int32_t j = i >= 0 ? i : i ^ 0x7FFFFFFF;
    float f;
    std::memcpy(&f, &j, 4);
    return f;
}

__global__ void k_init_flags(BuildFlags* f)
{
    if (threadIdx.x == 0) {
        f->flags = 0;
        f->max_depth = 0;
        f->max_stack = 0;
        f->n_nodes4 = 0;
        f->n_degenerate = 0;
        for (int a = 0; a < 3; ++a) {
            f->clo[a] = ordered(__builtin_inff());
            f->chi[a] = ordered(-__builtin_inff());
            f->blo[a] = ordered(__builtin_inff());
            f->bhi[a] = ordered(-__builtin_inff());
        }
    }
}

// Material record per material (see kMat* offsets): per band the absorption
// alpha_b, the scattering coefficient s_b (the hero band's s_b is the diffuse
// probability of a bounce; every band's s_b or 1 - s_b enters the band
// weights) and 1 - alpha_b, formed in FP64 and rounded to FP32.
__global__ void k_materials(const float* __restrict__ absorption, const float* __restrict__ scattering, int nm,
                            int nb, float* __restrict__ mats, BuildFlags* f)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    bool bad = false;
    for (int b = 0; b < nb; ++b) {
        const float a = absorption[m * nb + b], s = scattering[m * nb + b];
        if (!(a >= 0.0f && a <= 1.0f) || !(s >= 0.0f && s <= 1.0f)) bad = true;
    }
    if (bad) atomicOr(&f->flags, (uint32_t)kBadCoeff);
    float* r = mats + (int64_t)m * kMatStride;
    for (int i = 0; i < kMatStride; ++i) r[i] = 0.0f;
    for (int b = 0; b < nb; ++b) {
        const float a = absorption[m * nb + b];
        r[kMatAlpha + b] = a;
        r[kMatS + b] = scattering[m * nb + b];
        r[kMatKeep + b] = (float)(1.0 - (double)a);
    }
}

// Triangle bounds, centroids and validation; reduces the centroid bounds.
__global__ void k_prep(const float* __restrict__ verts, int64_t nv, const int32_t* __restrict__ tris, int64_t nt,
                       const int32_t* __restrict__ tri_mat, int nm, float4* __restrict__ cent,
                       uint32_t* __restrict__ seen, uint32_t* __restrict__ refs, BuildFlags* f)
{
    __shared__ int32_t s_lo[3][kBuildBlock / kWave], s_hi[3][kBuildBlock / kWave];
    __shared__ int32_t s_blo[3][kBuildBlock / kWave], s_bhi[3][kBuildBlock / kWave];
    float c[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float cm[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    // grid-stride over the triangles: fewer blocks, so fewer of the atomics
    // below, which all land on the same flag words
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
        // clear the counters of later kernels: seen [nt], refs [2 nt - 1]
        seen[t] = 0u;
        refs[t] = 0u;
        if (t > 0) refs[nt - 1 + t] = 0u;
        uint32_t flags = 0;
        int32_t idx[3];
        for (int k = 0; k < 3; ++k) {
            idx[k] = tris[3 * t + k];
            if (idx[k] < 0 || idx[k] >= nv) {
                flags |= kBadIndex;
                idx[k] = 0;
            }
        }
        if (tri_mat) {
            const int32_t m = tri_mat[t];
            if (m < 0 || m >= nm) flags |= kBadMaterial;
        }
        float v[3][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                v[k][a] = nv > 0 ? verts[3 * (int64_t)idx[k] + a] : 0.0f;
                if (!isfinite(v[k][a])) flags |= kBadVertex;
            }
        const float e1x = v[1][0] - v[0][0], e1y = v[1][1] - v[0][1], e1z = v[1][2] - v[0][2];
        const float e2x = v[2][0] - v[0][0], e2y = v[2][1] - v[0][1], e2z = v[2][2] - v[0][2];
        const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        if (nx == 0.0f && ny == 0.0f && nz == 0.0f) atomicAdd(&f->n_degenerate, 1u);
        if (flags) atomicOr(&f->flags, flags);
        float cen[3];
        for (int a = 0; a < 3; ++a) {
            const float l = fminf(fminf(v[0][a], v[1][a]), v[2][a]);
            const float h = fmaxf(fmaxf(v[0][a], v[1][a]), v[2][a]);
            cen[a] = 0.5f * (l + h);
            lo[a] = fminf(lo[a], l);
            hi[a] = fmaxf(hi[a], h);
            c[a] = fminf(c[a], cen[a]);
            cm[a] = fmaxf(cm[a], cen[a]);
        }
        cent[t] = make_float4(cen[0], cen[1], cen[2], 0.0f);
    }
    // wave then block reduction of the bounds
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o > 0; o >>= 1) {
            c[a] = fminf(c[a], __shfl_xor(c[a], o));
            cm[a] = fmaxf(cm[a], __shfl_xor(cm[a], o));
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
        }
        if (lane == 0) {
            s_lo[a][w] = ordered(c[a]);
            s_hi[a][w] = ordered(cm[a]);
            s_blo[a][w] = ordered(lo[a]);
            s_bhi[a][w] = ordered(hi[a]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        int32_t l = s_lo[a][0], h = s_hi[a][0], bl = s_blo[a][0], bh = s_bhi[a][0];
        for (int i = 1; i < kBuildBlock / kWave; ++i) {
            l = min(l, s_lo[a][i]);
            h = max(h, s_hi[a][i]);
            bl = min(bl, s_blo[a][i]);
            bh = max(bh, s_bhi[a][i]);
        }
        atomicMin(&f->clo[a], l);
        atomicMax(&f->chi[a], h);
        atomicMin(&f->blo[a], bl);
        atomicMax(&f->bhi[a], bh);
    }
}

// Spread the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Spread the low 21 bits of v to every third bit.
__device__ __forceinline__ uint64_t spread3_64(uint64_t v)
{
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Morton key of each centroid in the centroid bounds: 10 bits per axis in a
// 32-bit key, or 21 bits per axis in a 64-bit key (large scenes, where 10
// bits per axis leave triangles sharing a key).
template <class K>
__global__ void k_morton(const float4* __restrict__ cent, int64_t nt, const BuildFlags* f, K* __restrict__ keys,
                         uint32_t* __restrict__ vals)
{
    constexpr int kBits = sizeof(K) == 4 ? 10 : 21;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const float4 c = cent[t];
    const float cc[3] = {c.x, c.y, c.z};
    K code = 0;
    for (int a = 0; a < 3; ++a) {
        const float lo = unordered(f->clo[a]), hi = unordered(f->chi[a]);
        const float ext = hi - lo;
        float u = ext > 0.0f ? (cc[a] - lo) / ext : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const uint32_t q = min((uint32_t)(u * (float)(1u << kBits)), (1u << kBits) - 1u);
        if constexpr (sizeof(K) == 4) code |= spread3(q) << (2 - a);
        else code |= spread3_64(q) << (2 - a);
    }
    keys[t] = code;
    vals[t] = (uint32_t)t;
}

// ---------------------------------------------------------------- radix sort
// Per-tile digit counts, stored digit-major: counts[d * n_tiles + tile].
template <class K>
__global__ void __launch_bounds__(kBuildBlock) k_radix_count(const K* __restrict__ keys, int64_t n, int shift,
                                                             uint32_t* __restrict__ counts, int n_tiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBuildBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major counts in one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_radix_scan(uint32_t* __restrict__ counts, int64_t len)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (len + 1023) / 1024;
    const int64_t b = t * per, e = min(len, b + per);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        const uint32_t c = counts[i];
        counts[i] = run;
        run += c;
    }
}

// Device-wide exclusive scan of u32 in tiles of kSortTile elements (thread t
// of a tile owns elements 8t..8t+7): per-tile sums, an exclusive scan of the
// tile sums by k_radix_scan, then each tile scans itself and adds its
// offset.  Replaces a single-workgroup scan whose serial per-thread chunks
// made it latency bound for long arrays.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* s_wave)
{
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) s_wave[w] = inc;
    __syncthreads();
    uint32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += s_wave[i];
    return wbase + inc - v;
}

__global__ void __launch_bounds__(kBuildBlock) k_scan_sums(const uint32_t* __restrict__ in, int64_t len,
                                                           uint32_t* __restrict__ sums)
{
    __shared__ uint32_t s_wave[kBuildBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (base + i < len) v += in[base + i];
    const uint32_t ex = block_exclusive(v, s_wave);
    if (threadIdx.x == kBuildBlock - 1) sums[blockIdx.x] = ex + v;
}

__global__ void __launch_bounds__(kBuildBlock) k_scan_apply(uint32_t* __restrict__ data, int64_t len,
                                                            const uint32_t* __restrict__ offsets)
{
    __shared__ uint32_t s_wave[kBuildBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t x[kSortItems];
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        x[i] = base + i < len ? data[base + i] : 0u;
        v += x[i];
    }
    uint32_t run = block_exclusive(v, s_wave) + (offsets ? offsets[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (base + i < len) data[base + i] = run;
        run += x[i];
    }
}

// Stable scatter: each tile is processed in rounds of 256 keys; within a
// round, lanes of a wave with equal digits are matched by eight ballots and
// ranked by position, and waves are ordered through per-digit counters.
template <class K>
__global__ void __launch_bounds__(kBuildBlock) k_radix_scatter(const K* __restrict__ keys_in,
                                                               const uint32_t* __restrict__ vals_in, int64_t n,
                                                               int shift, const uint32_t* __restrict__ offsets,
                                                               int n_tiles, K* __restrict__ keys_out,
                                                               uint32_t* __restrict__ vals_out, BuildFlags* bad)
{
    constexpr int W = kBuildBlock / kWave;
    __shared__ uint32_t g_off[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t woff[W][256];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    g_off[tid] = offsets[(int64_t)tid * n_tiles + blockIdx.x];
    run[tid] = 0;
    for (int i = 0; i < W; ++i) wcnt[i][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBuildBlock + tid;
        const bool valid = i < n;
        const K key = valid ? keys_in[i] : (K)0;
        const uint32_t val = valid ? vals_in[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        const uint32_t rank = __popcll(peers & lanemask_lt(lane));
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t s = run[tid];
            for (int k = 0; k < W; ++k) {
                woff[k][tid] = s;
                s += wcnt[k][tid];
                wcnt[k][tid] = 0;
            }
            run[tid] = s;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = g_off[d] + woff[w][d] + rank;
            if (pos < (uint64_t)n) {
                keys_out[pos] = key;
                vals_out[pos] = val;
            } else {
                atomicOr(&bad->flags, (uint32_t)kBadTree);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hierarchy
// Length of the common prefix of keys i and j, extended by the indices' own
// common prefix when the keys are equal (so every key is distinct); -1 out of range.
template <class K>
__device__ __forceinline__ int delta(const K* __restrict__ k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const K a = k[i], b = k[j];
    constexpr int kKeyBits = 8 * (int)sizeof(K);
    if (a != b) {
        if constexpr (sizeof(K) == 4) return __clz(a ^ b);
        else return __clzll((long long)(a ^ b));
    }
    return kKeyBits + __clz((uint32_t)(i ^ j));
}

// Internal node i covers a key range [min(i,j), max(i,j)] grown from i in the
// direction of the neighbour with the longer common prefix; it splits where
// the common prefix of the range ends.  parent[] indexes internal nodes
// 0..n-2 then leaves n-1..2n-2.
template <class K>
__global__ void k_karras(const K* __restrict__ keys, int n, int2* __restrict__ child,
                         int32_t* __restrict__ parent, int2* __restrict__ range, BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    if (g < 0 || g + 1 > n - 1 || lo < 0 || hi > n - 1) {
        // cannot happen for a correct split search; keep every index in range
        atomicOr(&f->flags, (uint32_t)kBadTree);
        child[i] = make_int2(leaf_link(0), leaf_link(0));
        range[i] = make_int2(0, 0);
        return;
    }
    range[i] = make_int2(lo, hi);
    const int c0 = (lo == g) ? leaf_link(g) : g;
    const int c1 = (hi == g + 1) ? leaf_link(g + 1) : g + 1;
    child[i] = make_int2(c0, c1);
    parent[is_leaf(c0) ? (n - 1) + leaf_index(c0) : c0] = i;
    parent[is_leaf(c1) ? (n - 1) + leaf_index(c1) : c1] = i;
}

// Sorted triangle records and leaf bounds (box[n-1+i]).
__global__ void k_tri_records(const float* __restrict__ verts, int64_t nv, const int32_t* __restrict__ tris,
                              const int32_t* __restrict__ tri_mat, const uint32_t* __restrict__ order, int n,
                              float4* __restrict__ recs, float4* __restrict__ box, uint32_t* __restrict__ seen,
                              BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t t = order[i];
    if (t >= (uint32_t)n) {
        atomicOr(&f->flags, (uint32_t)kBadTree);
        t = 0;
    } else if (atomicAdd(&seen[t], 1u) != 0u) {
        atomicOr(&f->flags, (uint32_t)kBadTree);  // not a permutation
    }
    float v[3][3];
    for (int k = 0; k < 3; ++k) {
        int32_t vi = tris[3 * (int64_t)t + k];
        if (vi < 0 || vi >= nv) vi = 0;  // flagged by k_prep; the scene is rejected after the build
        for (int a = 0; a < 3; ++a) v[k][a] = verts[3 * (int64_t)vi + a];
    }
    const int32_t m = tri_mat ? tri_mat[t] : 0;
    recs[3 * (int64_t)i + 0] = make_float4(v[0][0], v[0][1], v[0][2], __uint_as_float(t));
    recs[3 * (int64_t)i + 1] = make_float4(v[1][0], v[1][1], v[1][2], __int_as_float(m));
    recs[3 * (int64_t)i + 2] = make_float4(v[2][0], v[2][1], v[2][2], 0.0f);
    // The traversal tests boxes in FP32 against the ray rounded to FP32, which
    // moves it by a few units in the last place of the coordinates and of the
    // distance travelled (about 2^-24 x (|origin| + t) each).  Padding each leaf
    // box by 2^-22 x (largest |coordinate| + diagonal) of the scene keeps every
    // box that the exact ray enters within reach of the rounded one, for
    // origins inside the scene's bounds (grazing rays excepted), so the FP64
    // triangle tests see every candidate.  The pad stays well below the 1 mm
    // by which a reflected segment starts off its surface (0.3 mm for a
    // 500 m scene), so a new origin is not inside the boxes of the coplanar
    // neighbours of the triangle it leaves.
    float m_abs = 0.0f, diag2 = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float bl = unordered(f->blo[a]), bh = unordered(f->bhi[a]);
        m_abs = fmaxf(m_abs, fmaxf(fabsf(bl), fabsf(bh)));
        diag2 += (bh - bl) * (bh - bl);
    }
    const float pad = 0x1p-22f * (m_abs + sqrtf(diag2));
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(fminf(v[0][a], v[1][a]), v[2][a]) - pad;
        hi[a] = fmaxf(fmaxf(v[0][a], v[1][a]), v[2][a]) + pad;
    }
    const int64_t b = (int64_t)(n - 1) + i;
    box[2 * b + 0] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    box[2 * b + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
}

// Internal boxes from leaf ranges.  Every internal node of the LBVH covers a
// contiguous range [lo, hi] of the Morton-sorted leaves (known to k_karras),
// so its box is the union of the leaf boxes over that range.  A pyramid of
// unions over aligned blocks (level L, entry m covers leaves
// [m 2^L, (m + 1) 2^L)) answers each range with at most two blocks per level,
// as a segment tree does; no atomics and no ordering between nodes.
constexpr int kPyrMaxLevels = 32;
struct PyrLevels {
    int64_t off[kPyrMaxLevels + 1];  // first entry of level L >= 1 in pyr (off[0] unused)
    int64_t len[kPyrMaxLevels + 1];  // entries of level L, ceil(n / 2^L)
    int top;                         // highest level (1 entry)
};

__device__ __forceinline__ void box_union(float4& lo, float4& hi, const float4 l, const float4 h)
{
    lo = make_float4(fminf(lo.x, l.x), fminf(lo.y, l.y), fminf(lo.z, l.z), 0.0f);
    hi = make_float4(fmaxf(hi.x, h.x), fmaxf(hi.y, h.y), fmaxf(hi.z, h.z), 0.0f);
}

// Levels 1..8 of the pyramid: each workgroup reduces its 256 leaves in LDS.
__global__ void __launch_bounds__(kBuildBlock) k_pyr_low(int n, const float4* __restrict__ box, PyrLevels pl,
                                                         float4* __restrict__ pyr)
{
    __shared__ float4 s_lo[kBuildBlock], s_hi[kBuildBlock];
    const int t = threadIdx.x;
    const int64_t leaf = (int64_t)blockIdx.x * kBuildBlock + t;
    const float inf = __builtin_inff();
    float4 lo = make_float4(inf, inf, inf, 0.0f), hi = make_float4(-inf, -inf, -inf, 0.0f);
    if (leaf < n) {
        lo = box[2 * ((int64_t)(n - 1) + leaf)];
        hi = box[2 * ((int64_t)(n - 1) + leaf) + 1];
    }
    s_lo[t] = lo;
    s_hi[t] = hi;
    __syncthreads();
    for (int L = 1, w = kBuildBlock / 2; w >= 1 && L <= pl.top; ++L, w >>= 1) {
        if (t < w) {
            float4 a = s_lo[2 * t], b = s_hi[2 * t];
            box_union(a, b, s_lo[2 * t + 1], s_hi[2 * t + 1]);
            const int64_t m = (int64_t)blockIdx.x * w + t;
            if (m < pl.len[L]) {
                pyr[2 * (pl.off[L] + m)] = a;
                pyr[2 * (pl.off[L] + m) + 1] = b;
            }
            lo = a;
            hi = b;
        }
        __syncthreads();
        if (t < w) {
            s_lo[t] = lo;
            s_hi[t] = hi;
        }
        __syncthreads();
    }
}

// Levels 9 and up, by one workgroup (their entries number n / 256 and fewer).
__global__ void __launch_bounds__(1024) k_pyr_high(PyrLevels pl, float4* __restrict__ pyr)
{
    for (int L = 9; L <= pl.top; ++L) {
        for (int64_t m = threadIdx.x; m < pl.len[L]; m += blockDim.x) {
            const int64_t a = 2 * m, b = 2 * m + 1;
            float4 lo = pyr[2 * (pl.off[L - 1] + a)], hi = pyr[2 * (pl.off[L - 1] + a) + 1];
            if (b < pl.len[L - 1]) box_union(lo, hi, pyr[2 * (pl.off[L - 1] + b)], pyr[2 * (pl.off[L - 1] + b) + 1]);
            pyr[2 * (pl.off[L] + m)] = lo;
            pyr[2 * (pl.off[L] + m) + 1] = hi;
        }
        __syncthreads();
    }
}

__global__ void k_refit(int n, const int2* __restrict__ range, const float4* __restrict__ box,
                        const float4* __restrict__ pyr, PyrLevels pl, int32_t* __restrict__ ibox)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int2 r = range[i];
    const float inf = __builtin_inff();
    float4 lo = make_float4(inf, inf, inf, 0.0f), hi = make_float4(-inf, -inf, -inf, 0.0f);
    int64_t a = r.x, b = r.y;
    for (int L = 0; a <= b && L <= pl.top; ++L) {
        if (a & 1) {
            const int64_t e = L == 0 ? 2 * ((int64_t)(n - 1) + a) : 2 * (pl.off[L] + a);
            box_union(lo, hi, L == 0 ? box[e] : pyr[e], L == 0 ? box[e + 1] : pyr[e + 1]);
            ++a;
        }
        if (!(b & 1) && a <= b) {
            const int64_t e = L == 0 ? 2 * ((int64_t)(n - 1) + b) : 2 * (pl.off[L] + b);
            box_union(lo, hi, L == 0 ? box[e] : pyr[e], L == 0 ? box[e + 1] : pyr[e + 1]);
            --b;
        }
        a >>= 1;
        b >>= 1;
    }
    int32_t* q = ibox + 6 * (int64_t)i;
    q[0] = ordered(lo.x);
    q[1] = ordered(lo.y);
    q[2] = ordered(lo.z);
    q[3] = ordered(hi.x);
    q[4] = ordered(hi.y);
    q[5] = ordered(hi.z);
}

// Structure check: every link in range, and every node except the root
// referenced by exactly one parent (refs indexes internal nodes then leaves).
__global__ void k_check_links(int n, const int2* __restrict__ child, uint32_t* __restrict__ refs, BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int2 c = child[i];
    const int32_t l[2] = {c.x, c.y};
    for (int k = 0; k < 2; ++k) {
        const int64_t idx = is_leaf(l[k]) ? (int64_t)(n - 1) + leaf_index(l[k]) : l[k];
        const bool ok = is_leaf(l[k]) ? (leaf_index(l[k]) < n) : (l[k] > 0 && l[k] < n - 1);
        if (!ok) atomicOr(&f->flags, (uint32_t)kBadTree);
        else atomicAdd(&refs[idx], 1u);
    }
}

__global__ void k_check_refs(int n, const uint32_t* __restrict__ refs, BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * n - 1) return;
    const uint32_t want = i == 0 ? 0u : 1u;
    if (refs[i] != want) atomicOr(&f->flags, (uint32_t)kBadTree);
}

__device__ __forceinline__ void node_box(int n, int32_t link, const float4* __restrict__ box,
                                         const int32_t* __restrict__ ibox, float4& lo, float4& hi)
{
    if (is_leaf(link)) {
        const int64_t b = (int64_t)(n - 1) + leaf_index(link);
        lo = box[2 * b];
        hi = box[2 * b + 1];
    } else {
        const int32_t* q = ibox + 6 * (int64_t)link;
        lo = make_float4(unordered(q[0]), unordered(q[1]), unordered(q[2]), 0.0f);
        hi = make_float4(unordered(q[3]), unordered(q[4]), unordered(q[5]), 0.0f);
    }
}

// Push count of binary node i in the 4-wide traversal: its slot count
// (a leaf child fills one slot, an internal child two) minus the one taken.
__device__ __forceinline__ int push_weight(int2 c) { return (is_leaf(c.x) ? 1 : 2) + (is_leaf(c.y) ? 1 : 2) - 1; }

// One record per internal node for the upward walk of k_node_depth: parent,
// grandparent (-1 past the root, which is node 0), and the push counts of the
// node and of its parent, so that the walk climbs two levels per load.
__global__ void k_node_up(int n, const int32_t* __restrict__ parent, const int2* __restrict__ child,
                          int4* __restrict__ up)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int p = i == 0 ? -1 : parent[i];
    int gp = -1, wp = 0;
    if (p >= 0) {
        gp = p == 0 ? -1 : parent[p];
        wp = push_weight(child[p]);
    }
    up[i] = make_int4(p, gp, push_weight(child[i]), wp);
}

// Depth of every internal node of the binary tree (the root has depth 0), its
// parity for the 4-wide collapse (written to even and idx4, the scan's input),
// and the sizes of the 4-wide traversal.  On the path from the root to a
// leaf, every binary node at even depth becomes a 4-wide node that pushes at
// most its slot count minus one entries.  Walking up from node i, the push
// counts of the ancestors at even and at odd distance from i are summed
// apart; once the walk gives i's depth d, the ancestors at even depth are
// those whose distance has the parity of d.  A node with a leaf child ends
// that leaf's path: its depth + 1 and its sum give the tree depth and the
// stack bound (maxima over such nodes, reduced over the wave first).  The
// walk reads one k_node_up record per two levels; it stops past 4 kMaxStack
// levels (such a tree is rejected by its stack bound).
__global__ void k_node_depth(int n, const int4* __restrict__ up, const int2* __restrict__ child,
                             uint32_t* __restrict__ even, uint32_t* __restrict__ idx4, BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int depth_leaf = 0, need = 0;
    uint32_t is_even = 0;
    if (i < n - 1) {
        int d = 0, sum[2] = {0, 0};
        int node = i;
        for (;;) {
            const int4 u = up[node];
            sum[d & 1] += u.z;
            if (u.x < 0 || d > 4 * kMaxStack) break;
            sum[(d + 1) & 1] += u.w;
            ++d;
            if (u.y < 0 || d > 4 * kMaxStack) break;
            node = u.y;
            ++d;
        }
        is_even = (d % 2 == 0) ? 1u : 0u;
        even[i] = is_even;
        idx4[i] = is_even;
        const int2 c = child[i];
        if (is_leaf(c.x) || is_leaf(c.y)) {
            depth_leaf = d + 1;
            need = sum[d & 1];
        }
    }
    // maxima and count over the wave, then over the block: one set of
    // atomics per block (every block updates the same three words)
    uint32_t cnt = is_even;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        depth_leaf = max(depth_leaf, __shfl_xor(depth_leaf, o, kWave));
        need = max(need, __shfl_xor(need, o, kWave));
        cnt += __shfl_xor(cnt, o, kWave);
    }
    __shared__ int s_depth[kBuildBlock / kWave], s_need[kBuildBlock / kWave];
    __shared__ uint32_t s_cnt[kBuildBlock / kWave];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_depth[w] = depth_leaf;
        s_need[w] = need;
        s_cnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < kBuildBlock / kWave; ++j) {
            depth_leaf = max(depth_leaf, s_depth[j]);
            need = max(need, s_need[j]);
            cnt += s_cnt[j];
        }
        if (depth_leaf > 0) atomicMax(&f->max_depth, depth_leaf);
        if (need > 0) atomicMax(&f->max_stack, need);
        if (cnt) atomicAdd(&f->n_nodes4, cnt);
    }
}

// Collapse of the binary tree into 4-wide nodes: every internal node at an
// even depth becomes a 4-wide node whose slots are its children, with each
// internal child replaced by that child's own two children (which sit at the
// next even depth).  idx4 = exclusive prefix sum of the even-depth flags, so
// the root becomes node 0 and nodes keep the Morton order of the binary tree.
__global__ void k_collapse4(int n, const int2* __restrict__ child, const float4* __restrict__ box,
                            const int32_t* __restrict__ ibox, const uint32_t* __restrict__ even,
                            const uint32_t* __restrict__ idx4, float4* __restrict__ nodes)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1 || !even[i]) return;
    int32_t links[4];
    float4 lo[4], hi[4];
    int k = 0;
    const int2 c = child[i];
    const int32_t cs[2] = {c.x, c.y};
    for (int a = 0; a < 2; ++a) {
        if (is_leaf(cs[a])) {
            node_box(n, cs[a], box, ibox, lo[k], hi[k]);
            links[k++] = cs[a];
        } else {
            const int2 g = child[cs[a]];
            const int32_t gs[2] = {g.x, g.y};
            for (int b = 0; b < 2; ++b) {
                node_box(n, gs[b], box, ibox, lo[k], hi[k]);
                links[k++] = is_leaf(gs[b]) ? gs[b] : (int32_t)idx4[gs[b]];
            }
        }
    }
    // Empty slots: a box at +inf, which the slab test reports either as a miss
    // or as an entry at t = +inf -- both ignored by the traversal.  Its link is
    // a leaf, never an internal node, so a visit could not loop.
    for (; k < 4; ++k) {
        lo[k] = make_float4(__builtin_inff(), __builtin_inff(), __builtin_inff(), 0.0f);
        hi[k] = lo[k];
        links[k] = leaf_link(0);
    }
    float4* o = nodes + (int64_t)kNode4 * idx4[i];
    for (int j = 0; j < 4; ++j) {
        o[2 * j] = make_float4(lo[j].x, lo[j].y, lo[j].z, __int_as_float(links[j]));
        o[2 * j + 1] = make_float4(hi[j].x, hi[j].y, hi[j].z, 0.0f);
    }
}

// Build temporaries come from one grow-only device arena per device, reused
// by every scene_create (which holds the arena's lock and synchronises its
// stream before returning), so a rebuild does not allocate.
struct Arena {
    std::mutex mu;
    char* base = nullptr;
    size_t cap = 0, used = 0;
    BuildFlags* host = nullptr;   // pinned host copy of the build's flags
    hipEvent_t done = nullptr;    // marks the copy's completion on the build's stream
};
Arena g_arena[16];

// Read the build's flags back: the copy lands in pinned host memory (one
// direct DMA instead of a staged pageable copy) and the host polls the copy's
// event rather than blocking on the stream, returning as soon as it is done.
// Called with the arena's lock held, which also guards `host` and `done`.
hipError_t read_flags(Arena& a, const BuildFlags* dev_flags, hipStream_t st, BuildFlags* out)
{
    if (!a.host) {
        hipError_t e = hipHostMalloc((void**)&a.host, sizeof(BuildFlags), hipHostMallocDefault);
        if (e != hipSuccess) return e;
    }
    if (!a.done) {
        hipError_t e = hipEventCreateWithFlags(&a.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(a.host, dev_flags, sizeof(BuildFlags), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a.done, st);
    if (e != hipSuccess) return e;
    while ((e = hipEventQuery(a.done)) == hipErrorNotReady) __builtin_ia32_pause();
    if (e != hipSuccess) return e;
    *out = *a.host;
    return hipSuccess;
}

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t bytes = 0;
    hipError_t alloc(size_t n)
    {
        bytes = (sizeof(T) * (n ? n : 1) + 255) & ~(size_t)255;
        return hipSuccess;
    }
};

// Lay out `bufs` in the arena (growing it when needed).
template <class... B>
hipError_t arena_place(Arena& a, B&... bufs)
{
    size_t need = 0;
    ((need += bufs.bytes), ...);
    if (need > a.cap) {
        if (a.base) {
            hipError_t e = hipFree(a.base);
            if (e != hipSuccess) return e;
            a.base = nullptr;
            a.cap = 0;
        }
        hipError_t e = hipMalloc(&a.base, need + need / 4);
        if (e != hipSuccess) return e;
        a.cap = need + need / 4;
    }
    size_t off = 0;
    auto put = [&](auto& b) {
        b.p = reinterpret_cast<std::remove_reference_t<decltype(b.p)>>(a.base + off);
        off += b.bytes;
    };
    (put(bufs), ...);
    a.used = off;
    return hipSuccess;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// In-place exclusive scan of len u32; `sums` holds blocks(len, kSortTile) entries.
void scan_exclusive(uint32_t* data, int64_t len, uint32_t* sums, hipStream_t st)
{
    const unsigned nb = blocks(len, kSortTile);
    if (nb > 1) {
        hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kBuildBlock), 0, st, data, len, sums);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, sums, (int64_t)nb);
    }
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBuildBlock), 0, st, data, len, nb > 1 ? sums : nullptr);
}

// Morton keys of the centroids and a stable LSD radix sort of (key, triangle)
// pairs, eight bits per pass; the sorted pairs end in (k0, v0).
template <class K>
void morton_sort(const float4* cent, int64_t n, BuildFlags* flags, K* k0, K* k1, uint32_t* v0, uint32_t* v1,
                 uint32_t* counts, uint32_t* sums, int n_tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_morton<K>, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st, cent, n, flags, k0, v0);
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = 0; shift < 8 * (int)sizeof(K); shift += 8) {
        hipLaunchKernelGGL(k_radix_count<K>, dim3(n_tiles), dim3(kBuildBlock), 0, st, ki, n, shift, counts, n_tiles);
        scan_exclusive(counts, (int64_t)256 * n_tiles, sums, st);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(n_tiles), dim3(kBuildBlock), 0, st, ki, vi, n, shift, counts,
                           n_tiles, ko, vo, flags);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int scene_create(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                            const int32_t* tri_material, const float* absorption, const float* scattering,
                            int32_t n_materials, int32_t n_bands, void* hip_stream, RprScene** out)
{
    if (!out) return set_error(RPR_EINVAL, "scene_create: out is null");
    *out = nullptr;
    if (n_bands < 1 || n_bands > RPR_MAX_BANDS)
        return set_error(RPR_EINVAL, "scene_create: n_bands=%d not in 1..%d", n_bands, RPR_MAX_BANDS);
    if (n_materials < 1) return set_error(RPR_EINVAL, "scene_create: n_materials=%d < 1", n_materials);
    if (n_tris < 0 || n_verts < 0) return set_error(RPR_EINVAL, "scene_create: negative size");
    if (n_tris > (int64_t)1 << 30) return set_error(RPR_EUNSUPPORTED, "scene_create: n_tris=%lld too large", (long long)n_tris);
    if (n_tris > 0 && (!verts || !tris || n_verts < 1))
        return set_error(RPR_EINVAL, "scene_create: null geometry with n_tris=%lld", (long long)n_tris);
    if (!absorption || !scattering) return set_error(RPR_EINVAL, "scene_create: null material arrays");
    hipStream_t st = (hipStream_t)hip_stream;
    const int n = (int)n_tris;

    RprScene* sc = new RprScene();
    auto fail = [&](int code) {
        if (sc->nodes) (void)hipFree(sc->nodes);
        if (sc->tris) (void)hipFree(sc->tris);
        if (sc->mats) (void)hipFree(sc->mats);
        workspace_free(sc->ws);
        delete sc;
        return code;
    };
    {
        hipError_t e = hipGetDevice(&sc->device);
        if (e != hipSuccess) return fail(set_error(RPR_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
    }
    sc->n_tris = n_tris;
    sc->n_bands = n_bands;
    sc->n_materials = n_materials;

#define TRY(expr)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(set_error(e_ == hipErrorOutOfMemory ? RPR_ENOMEM : RPR_EDEVICE,           \
                                  "scene_create: %s: %s", #expr, hipGetErrorString(e_)));         \
    } while (0)

    int dev = sc->device;
    if (dev < 0 || dev >= 16) return fail(set_error(RPR_EUNSUPPORTED, "scene_create: device %d", dev));
    Arena& arena = g_arena[dev];
    std::lock_guard<std::mutex> arena_lock(arena.mu);
    DevBuf<BuildFlags> flags;
    TRY(flags.alloc(1));
    TRY(hipMalloc(&sc->mats, sizeof(float) * kMatStride * n_materials));
    TRY(hipMalloc(&sc->tris, sizeof(float4) * 3 * (size_t)(n > 0 ? n : 1)));
    TRY(hipMalloc(&sc->nodes, sizeof(float4) * kNode4 * (size_t)(n > 1 ? n - 1 : 1)));
    DevBuf<float4> cent, box;
    DevBuf<uint64_t> k0, k1;  // Morton keys: 32 or 64 bits each
    DevBuf<uint32_t> v0, v1, counts, seen, refs, even, idx4, scan_sums;
    DevBuf<int32_t> ibox, parent;
    DevBuf<int2> child, range;
    DevBuf<float4> pyr;
    const int n_tiles = (int)blocks(n > 0 ? n : 1, kSortTile);
    if (n > 0) {
        TRY(cent.alloc(n));
        TRY(k0.alloc(n));
        TRY(v0.alloc(n));
        TRY(k1.alloc(n));
        TRY(v1.alloc(n));
        TRY(counts.alloc((size_t)256 * n_tiles));
        TRY(box.alloc(2 * (size_t)(2 * n - 1)));
        TRY(child.alloc(n > 1 ? n - 1 : 1));
        TRY(range.alloc(n > 1 ? n - 1 : 1));
        // sum over levels of ceil(n / 2^L) <= n - 1 + levels
        TRY(pyr.alloc(2 * ((size_t)n + kPyrMaxLevels + 1)));
        TRY(parent.alloc(2 * (size_t)n - 1));
        TRY(ibox.alloc(6 * (size_t)(n > 1 ? n - 1 : 1)));
        TRY(seen.alloc(n));
        TRY(even.alloc(n > 1 ? n - 1 : 1));
        TRY(idx4.alloc(n > 1 ? n - 1 : 1));
        TRY(refs.alloc(2 * (size_t)n - 1));
        TRY(scan_sums.alloc(std::max<size_t>(blocks((int64_t)256 * n_tiles, kSortTile), blocks(n, kSortTile))));
    }
    TRY(arena_place(arena, flags, cent, box, k0, v0, k1, v1, counts, seen, refs, even, idx4, ibox, parent, child,
                    range, pyr, scan_sums));
    hipLaunchKernelGGL(k_init_flags, dim3(1), dim3(64), 0, st, flags.p);
    hipLaunchKernelGGL(k_materials, dim3(blocks(n_materials, 64)), dim3(64), 0, st, absorption, scattering,
                       n_materials, n_bands, sc->mats, flags.p);
    TRY(hipGetLastError());

    if (n > 0) {
        hipLaunchKernelGGL(k_prep, dim3(std::min(blocks(n, kBuildBlock), (unsigned)kPrepBlocks)), dim3(kBuildBlock), 0, st,
                           verts, n_verts, tris,
                           n_tris, tri_material, n_materials, cent.p, seen.p, refs.p, flags.p);
        const bool wide = n >= kWideKeyTris;
        if (wide) morton_sort<uint64_t>(cent.p, n_tris, flags.p, (uint64_t*)k0.p, (uint64_t*)k1.p, v0.p, v1.p, counts.p,
                                        scan_sums.p, n_tiles, st);
        else morton_sort<uint32_t>(cent.p, n_tris, flags.p, (uint32_t*)k0.p, (uint32_t*)k1.p, v0.p, v1.p, counts.p,
                                   scan_sums.p, n_tiles, st);
        uint32_t* vi = v0.p;
        // after an even number of passes the sorted keys/ids are back in (k0, v0)
        TRY(hipMemsetAsync(parent.p, 0xFF, sizeof(int32_t) * (2 * (size_t)n - 1), st));

        hipLaunchKernelGGL(k_tri_records, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st, verts,
                           n_verts, tris, tri_material, vi, n, sc->tris, box.p, seen.p, flags.p);
        if (n > 1) {
            if (wide)
                hipLaunchKernelGGL(k_karras<uint64_t>, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st,
                                   (const uint64_t*)k0.p, n, child.p, parent.p, range.p, flags.p);
            else
                hipLaunchKernelGGL(k_karras<uint32_t>, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st,
                                   (const uint32_t*)k0.p, n, child.p, parent.p, range.p, flags.p);
            hipLaunchKernelGGL(k_check_links, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st, n,
                               child.p, refs.p, flags.p);
            hipLaunchKernelGGL(k_check_refs, dim3(blocks(2 * (int64_t)n - 1, kBuildBlock)), dim3(kBuildBlock), 0,
                               st, n, refs.p, flags.p);
            PyrLevels pl;
            std::memset(&pl, 0, sizeof(pl));
            int64_t off = 0, len = n;
            pl.top = 0;
            while (len > 1 && pl.top < kPyrMaxLevels) {
                len = (len + 1) / 2;
                ++pl.top;
                pl.off[pl.top] = off;
                pl.len[pl.top] = len;
                off += len;
            }
            hipLaunchKernelGGL(k_pyr_low, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st, n, box.p, pl, pyr.p);
            if (pl.top > 8) hipLaunchKernelGGL(k_pyr_high, dim3(1), dim3(1024), 0, st, pl, pyr.p);
            hipLaunchKernelGGL(k_refit, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st, n, range.p, box.p,
                               pyr.p, pl, ibox.p);
            // the centroids are dead after the Morton codes: their n float4 hold the n - 1 walk records
            int4* up = reinterpret_cast<int4*>(cent.p);
            hipLaunchKernelGGL(k_node_up, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st, n, parent.p,
                               child.p, up);
            hipLaunchKernelGGL(k_node_depth, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st, n, up,
                               child.p, even.p, idx4.p, flags.p);
            scan_exclusive(idx4.p, (int64_t)(n - 1), scan_sums.p, st);
            hipLaunchKernelGGL(k_collapse4, dim3(blocks(n - 1, kBuildBlock)), dim3(kBuildBlock), 0, st, n, child.p,
                               box.p, ibox.p, even.p, idx4.p, sc->nodes);
        }
        TRY(hipGetLastError());
        BuildFlags hf;
        TRY(read_flags(arena, flags.p, st, &hf));
        if (hf.flags & kBadIndex) return fail(set_error(RPR_EINVAL, "scene_create: vertex index out of range"));
        if (hf.flags & kBadVertex) return fail(set_error(RPR_EINVAL, "scene_create: non-finite vertex"));
        if (hf.flags & kBadMaterial) return fail(set_error(RPR_EINVAL, "scene_create: material index out of range"));
        if (hf.flags & kBadCoeff)
            return fail(set_error(RPR_EINVAL, "scene_create: absorption/scattering outside [0, 1]"));
        if (hf.flags & kBadTree) return fail(set_error(RPR_EDEVICE, "scene_create: BVH consistency check failed"));
        sc->max_depth = hf.max_depth;
        sc->stack_need = hf.max_stack;
        sc->n_nodes4 = hf.n_nodes4;
        sc->n_degenerate = (int32_t)hf.n_degenerate;
        for (int a = 0; a < 3; ++a) {
            sc->lo[a] = unordered(hf.blo[a]);
            sc->hi[a] = unordered(hf.bhi[a]);
        }
        // the traversal writes one slot past the deepest entry (a push without a branch)
        if (sc->stack_need >= kMaxStack)
            return fail(set_error(RPR_EUNSUPPORTED,
                                  "scene_create: BVH depth %d needs %d stack entries, the traversal takes at most %d",
                                  sc->max_depth, sc->stack_need, kMaxStack - 1));
    } else {
        BuildFlags hf;
        TRY(read_flags(arena, flags.p, st, &hf));
        if (hf.flags & kBadCoeff)
            return fail(set_error(RPR_EINVAL, "scene_create: absorption/scattering outside [0, 1]"));
    }
#undef TRY
    sc->view.nodes = sc->nodes;
    sc->view.tris = sc->tris;
    sc->view.mats = sc->mats;
    sc->view.root = n == 1 ? leaf_link(0) : 0;
    sc->view.n_tris = n;
    sc->view.n_bands = n_bands;
    *out = sc;
    return RPR_OK;
}

extern "C" int scene_destroy(RprScene* scene)
{
    if (!scene) return RPR_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != scene->device) (void)hipSetDevice(scene->device);
    (void)hipFree(scene->nodes);
    (void)hipFree(scene->tris);
    (void)hipFree(scene->mats);
    workspace_free(scene->ws);
    if (dev >= 0 && dev != scene->device) (void)hipSetDevice(dev);
    delete scene;
    return RPR_OK;
}

extern "C" int scene_info(const RprScene* scene, RprSceneInfo* out)
{
    if (!scene || !out) return set_error(RPR_EINVAL, "scene_info: null argument");
    std::memset(out, 0, sizeof(*out));
    out->n_tris = scene->n_tris;
    out->n_nodes = scene->n_nodes4;
    out->max_depth = scene->max_depth;
    out->stack_need = scene->stack_need;
    out->n_bands = scene->n_bands;
    out->n_materials = scene->n_materials;
    out->n_degenerate = scene->n_degenerate;
    for (int a = 0; a < 3; ++a) {
        out->bounds_lo[a] = scene->lo[a];
        out->bounds_hi[a] = scene->hi[a];
    }
    return RPR_OK;
}
