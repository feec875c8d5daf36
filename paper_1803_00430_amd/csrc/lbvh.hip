// Scene creation: material table, triangle records and a linear BVH.
//
// Linear BVH (Karras, HPG 2012): Morton codes (30-bit; 63-bit for large scenes) of the triangle
// centroids in the scene's centroid bounds (cells of bounded aspect), a stable least-significant-digit
// radix sort of (code, triangle) pairs, internal nodes from the longest common
// prefixes of neighbouring codes (ties broken by the sorted index), node
// boxes as unions over each node's range of sorted leaves, and a collapse of
// the binary tree into 4-wide nodes.
//
// A rebuild is a chain of dependent launches on one stream, and each launch
// costs a few microseconds before its first wave runs (more while another
// stream's trace holds the compute units), so the chain is kept short: the
// material table and the validation share the first kernel, the Morton keys
// share the first digit count, the scatter scans the digit counts itself, and
// the leaf records, the hierarchy and its structure checks share launches.
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
constexpr int kPrepBlock = 64;     // k_prep's workgroup: one wave, so it can start in any free wave slot
constexpr int kPrepBlocks = 512;   // k_prep's grid cap (it strides over the triangles)
constexpr int kSortItems = 8;
constexpr int kSortTile = kBuildBlock * kSortItems;
// Scenes of at least this many triangles get 64-bit Morton keys (21 bits per axis).
constexpr int64_t kWideKeyTris = (int64_t)1 << 19;
// Largest ratio of the Morton cells' sides (see k_morton_count).
constexpr float kMaxCellAspect = 8.0f;
// Up to this many sort tiles the scatter forms its digit offsets from the
// per-tile counts itself (two launches per pass instead of five); beyond it a
// device-wide scan runs between count and scatter.
constexpr int kFusedScanTiles = 128;
// Up to this many blocks of internal nodes the collapse forms the 4-wide node
// indices itself (from the even-depth bit masks and per-block counts, scanned
// in LDS); beyond it a device-wide scan runs before the collapse.
constexpr int kFusedIndexBlocks = 1024;

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

// What each k_prep block found: validation flags, degenerate triangles, and
// the bounds of its centroids and of its triangles (as order-preserving keys).
// The next kernel reduces them, so that no launch has to clear shared counters
// before k_prep's blocks could update them.
struct PrepPartial {
    uint32_t flags;
    uint32_t n_degenerate;
    int32_t clo[3], chi[3];
    int32_t blo[3], bhi[3];
};

// Reduce k_prep's per-block results within one wave; every lane returns the total.
__device__ PrepPartial reduce_prep(const PrepPartial* __restrict__ part, int n_part)
{
    const int lane = threadIdx.x % kWave;
    PrepPartial r;
    r.flags = 0;
    r.n_degenerate = 0;
    for (int a = 0; a < 3; ++a) {
        r.clo[a] = r.blo[a] = ordered(__builtin_inff());
        r.chi[a] = r.bhi[a] = ordered(-__builtin_inff());
    }
    for (int j = lane; j < n_part; j += kWave) {
        const PrepPartial q = part[j];
        r.flags |= q.flags;
        r.n_degenerate += q.n_degenerate;
        for (int a = 0; a < 3; ++a) {
            r.clo[a] = min(r.clo[a], q.clo[a]);
            r.chi[a] = max(r.chi[a], q.chi[a]);
            r.blo[a] = min(r.blo[a], q.blo[a]);
            r.bhi[a] = max(r.bhi[a], q.bhi[a]);
        }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        r.flags |= __shfl_xor(r.flags, o, kWave);
        r.n_degenerate += __shfl_xor(r.n_degenerate, o, kWave);
        for (int a = 0; a < 3; ++a) {
            r.clo[a] = min(r.clo[a], __shfl_xor(r.clo[a], o, kWave));
            r.chi[a] = max(r.chi[a], __shfl_xor(r.chi[a], o, kWave));
            r.blo[a] = min(r.blo[a], __shfl_xor(r.blo[a], o, kWave));
            r.bhi[a] = max(r.bhi[a], __shfl_xor(r.bhi[a], o, kWave));
        }
    }
    return r;
}

// The build's flag record, started from k_prep's totals (written by one lane,
// before any kernel that updates it).
__device__ void write_flags(const PrepPartial& r, BuildFlags* f)
{
    f->flags = r.flags;
    f->max_depth = 0;
    f->max_stack = 0;
    f->n_nodes4 = 0;
    f->n_degenerate = r.n_degenerate;
    f->pad = 0;
    for (int a = 0; a < 3; ++a) {
        f->clo[a] = r.clo[a];
        f->chi[a] = r.chi[a];
        f->blo[a] = r.blo[a];
        f->bhi[a] = r.bhi[a];
    }
}

// A scene without triangles: the flag record from the material check alone.
__global__ void k_flags_only(const PrepPartial* __restrict__ part, int n_part, BuildFlags* f)
{
    const PrepPartial r = reduce_prep(part, n_part);
    if (threadIdx.x == 0) write_flags(r, f);
}

// Material records, then triangle bounds, centroids and validation, with the
// per-block results in part[blockIdx.x].  Material record per material (see
// kMat* offsets): per band the absorption alpha_b, the scattering coefficient
// s_b (the hero band's s_b is the diffuse probability of a bounce; every
// band's s_b or 1 - s_b enters the band weights) and 1 - alpha_b, formed in
// FP64 and rounded to FP32.  Also clears the counters of later kernels (seen
// [nt], refs [2 nt - 1]) and sets every parent link to -1.
__global__ void __launch_bounds__(kPrepBlock)
k_prep(const float* __restrict__ verts, int64_t nv, const int32_t* __restrict__ tris, int64_t nt,
       const int32_t* __restrict__ tri_mat, const float* __restrict__ absorption,
       const float* __restrict__ scattering, int nm, int nb, float* __restrict__ mats, float4* __restrict__ cent,
       uint32_t* __restrict__ seen, uint32_t* __restrict__ refs, int32_t* __restrict__ parent,
       PrepPartial* __restrict__ part)
{
    float c[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float cm[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    uint32_t flags = 0, ndeg = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t m = g; m < nm; m += stride) {
        for (int b = 0; b < nb; ++b) {
            const float a = absorption[m * nb + b], s = scattering[m * nb + b];
            if (!(a >= 0.0f && a <= 1.0f) || !(s >= 0.0f && s <= 1.0f)) flags |= kBadCoeff;
        }
        float* r = mats + m * kMatStride;
        for (int i = 0; i < kMatStride; ++i) r[i] = 0.0f;
        for (int b = 0; b < nb; ++b) {
            const float a = absorption[m * nb + b];
            r[kMatAlpha + b] = a;
            r[kMatS + b] = scattering[m * nb + b];
            r[kMatKeep + b] = (float)(1.0 - (double)a);
        }
    }
    // grid-stride over the triangles
    for (int64_t t = g; t < nt; t += stride) {
        seen[t] = 0u;
        refs[t] = 0u;
        if (t > 0) refs[nt - 1 + t] = 0u;
        parent[t] = -1;
        if (t + 1 < nt) parent[nt + t] = -1;
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
        if (nx == 0.0f && ny == 0.0f && nz == 0.0f) ++ndeg;
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
    // reduction over the block (one wave)
    for (int o = kWave / 2; o > 0; o >>= 1) {
        flags |= __shfl_xor(flags, o, kWave);
        ndeg += __shfl_xor(ndeg, o, kWave);
        for (int a = 0; a < 3; ++a) {
            c[a] = fminf(c[a], __shfl_xor(c[a], o, kWave));
            cm[a] = fmaxf(cm[a], __shfl_xor(cm[a], o, kWave));
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, kWave));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, kWave));
        }
    }
    if (threadIdx.x == 0) {
        PrepPartial r;
        r.flags = flags;
        r.n_degenerate = ndeg;
        for (int a = 0; a < 3; ++a) {
            r.clo[a] = ordered(c[a]);
            r.chi[a] = ordered(cm[a]);
            r.blo[a] = ordered(lo[a]);
            r.bhi[a] = ordered(hi[a]);
        }
        part[blockIdx.x] = r;
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

// Morton key of a centroid in the box [lo, lo + ext] on the centroid bounds:
// 10 bits per axis in a 32-bit key, or 21 bits per axis in a 64-bit key
// (large scenes, where 10 bits per axis leave triangles sharing a key).
template <class K>
__device__ __forceinline__ K morton_key(const float4 c, const float lo[3], const float ext[3])
{
    constexpr int kBits = sizeof(K) == 4 ? 10 : 21;
    const float cc[3] = {c.x, c.y, c.z};
    K code = 0;
    for (int a = 0; a < 3; ++a) {
        float u = ext[a] > 0.0f ? (cc[a] - lo[a]) / ext[a] : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const uint32_t q = min((uint32_t)(u * (float)(1u << kBits)), (1u << kBits) - 1u);
        if constexpr (sizeof(K) == 4) code |= spread3(q) << (2 - a);
        else code |= spread3_64(q) << (2 - a);
    }
    return code;
}

// ---------------------------------------------------------------- radix sort
// Per-tile digit counts, stored digit-major: counts[d * n_tiles + tile].
__device__ __forceinline__ void store_tile_counts(uint32_t* h, uint32_t* __restrict__ counts, int n_tiles)
{
    __syncthreads();
    counts[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// The first pass's count with the keys made on the way: k_prep's results are
// reduced (block 0 writes them to the flag record), each centroid's Morton key
// and its triangle index are stored, and the low digit is counted.
template <class K>
__global__ void __launch_bounds__(kBuildBlock)
k_morton_count(const float4* __restrict__ cent, int64_t n, const PrepPartial* __restrict__ part, int n_part,
               BuildFlags* f, K* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ counts,
               int n_tiles)
{
    __shared__ uint32_t h[256];
    __shared__ float s_lo[3], s_hi[3];
    h[threadIdx.x] = 0;
    if (threadIdx.x < kWave) {
        const PrepPartial r = reduce_prep(part, n_part);
        if (threadIdx.x == 0) {
            for (int a = 0; a < 3; ++a) {
                s_lo[a] = unordered(r.clo[a]);
                s_hi[a] = unordered(r.chi[a]);
            }
            if (blockIdx.x == 0) write_flags(r, f);
        }
    }
    __syncthreads();
    // Each axis spans its centroid extent, raised to at least 1/kMaxCellAspect
    // of the longest: the key's cells are then at most that many times longer
    // on one axis than on another, so a flat scene (a storey 3 m high and
    // 90 m wide) is not cut along its short axis as often as along the long
    // ones, while a scene of moderate aspect keeps its own extents.
    const float lo[3] = {s_lo[0], s_lo[1], s_lo[2]};
    const float emax = fmaxf(fmaxf(s_hi[0] - s_lo[0], s_hi[1] - s_lo[1]), s_hi[2] - s_lo[2]);
    const float ext[3] = {fmaxf(s_hi[0] - s_lo[0], emax / kMaxCellAspect),
                          fmaxf(s_hi[1] - s_lo[1], emax / kMaxCellAspect),
                          fmaxf(s_hi[2] - s_lo[2], emax / kMaxCellAspect)};
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBuildBlock + threadIdx.x;
        if (i < n) {
            const K key = morton_key<K>(cent[i], lo, ext);
            keys[i] = key;
            vals[i] = (uint32_t)i;
            atomicAdd(&h[(uint32_t)key & 255u], 1u);
        }
    }
    store_tile_counts(h, counts, n_tiles);
}

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
    store_tile_counts(h, counts, n_tiles);
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
// `counts` holds the digit-major per-tile counts (fused: the tile forms its
// offsets from them, the keys of all smaller digits plus those of its digit
// in earlier tiles) or their exclusive scan (the offsets themselves).
template <class K>
__global__ void __launch_bounds__(kBuildBlock) k_radix_scatter(const K* __restrict__ keys_in,
                                                               const uint32_t* __restrict__ vals_in, int64_t n,
                                                               int shift, const uint32_t* __restrict__ counts,
                                                               int n_tiles, bool fused, K* __restrict__ keys_out,
                                                               uint32_t* __restrict__ vals_out, BuildFlags* bad)
{
    constexpr int W = kBuildBlock / kWave;
    __shared__ uint32_t g_off[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t woff[W][256];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    if (fused) {
        const uint32_t* row = counts + (int64_t)tid * n_tiles;
        uint32_t before = 0, total = 0;
#pragma unroll 8
        for (int t = 0; t < n_tiles; ++t) {
            const uint32_t c = row[t];
            total += c;
            before += t < (int)blockIdx.x ? c : 0u;
        }
        __shared__ uint32_t s_wave[W];
        g_off[tid] = block_exclusive(total, s_wave) + before;
    } else {
        g_off[tid] = counts[(int64_t)tid * n_tiles + blockIdx.x];
    }
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
// 0..n-2 then leaves n-1..2n-2.  Structure check, first half: each child link
// is counted in refs (same indexing), and a link out of range is flagged.
template <class K>
__device__ __forceinline__ void karras_node(int i, const K* __restrict__ keys, int n, int2* __restrict__ child,
                                            int32_t* __restrict__ parent, int2* __restrict__ range,
                                            uint32_t* __restrict__ refs, BuildFlags* f)
{
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
    const int32_t links[2] = {c0, c1};
    for (int k = 0; k < 2; ++k) {
        const int32_t c = links[k];
        const int64_t idx = is_leaf(c) ? (int64_t)(n - 1) + leaf_index(c) : c;
        const bool ok = is_leaf(c) ? (leaf_index(c) < n) : (c > 0 && c < n - 1);
        if (!ok) {
            atomicOr(&f->flags, (uint32_t)kBadTree);
        } else {
            parent[idx] = i;
            atomicAdd(&refs[idx], 1u);
        }
    }
}

// Sorted triangle records and leaf bounds (box[n-1+i]).
__device__ __forceinline__ void tri_record(int i, const float* __restrict__ verts, int64_t nv,
                                           const int32_t* __restrict__ tris, const int32_t* __restrict__ tri_mat,
                                           const uint32_t* __restrict__ order, int n, float4* __restrict__ recs,
                                           float4* __restrict__ box, uint32_t* __restrict__ seen, BuildFlags* f)
{
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

// After the sort: thread i writes leaf i's record and box (i < n) and internal
// node i's split, children and parent links (i < n - 1).
template <class K>
__global__ void __launch_bounds__(kBuildBlock)
k_leaves_nodes(const float* __restrict__ verts, int64_t nv, const int32_t* __restrict__ tris,
               const int32_t* __restrict__ tri_mat, const K* __restrict__ keys, const uint32_t* __restrict__ order,
               int n, float4* __restrict__ recs, float4* __restrict__ box, uint32_t* __restrict__ seen,
               int2* __restrict__ child, int32_t* __restrict__ parent, int2* __restrict__ range,
               uint32_t* __restrict__ refs, BuildFlags* f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) karras_node<K>(i, keys, n, child, parent, range, refs, f);
    if (i < n) tri_record(i, verts, nv, tris, tri_mat, order, n, recs, box, seen, f);
}

// Internal boxes from leaf ranges.  Every internal node of the LBVH covers a
// contiguous range [lo, hi] of the Morton-sorted leaves (known from its split),
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
// Structure check, second half: every node but the root (internal node 0)
// has exactly one parent link (thread j checks internal node j and leaf j).
__global__ void __launch_bounds__(kBuildBlock) k_pyr_low(int n, const float4* __restrict__ box, PyrLevels pl,
                                                         float4* __restrict__ pyr, const uint32_t* __restrict__ refs,
                                                         BuildFlags* f)
{
    __shared__ float4 s_lo[kBuildBlock], s_hi[kBuildBlock];
    const int t = threadIdx.x;
    const int64_t leaf = (int64_t)blockIdx.x * kBuildBlock + t;
    if (leaf < n) {
        bool bad = refs[(n - 1) + leaf] != 1u;
        if (leaf < n - 1) bad = bad || refs[leaf] != (leaf == 0 ? 0u : 1u);
        if (bad) atomicOr(&f->flags, (uint32_t)kBadTree);
    }
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

// Push count of binary node i in the 4-wide traversal: its slot count
// (a leaf child fills one slot, an internal child two) minus the one taken.
__device__ __forceinline__ int push_weight(int2 c) { return (is_leaf(c.x) ? 1 : 2) + (is_leaf(c.y) ? 1 : 2) - 1; }

// One record per internal node for the upward walk of k_node_depth: parent,
// grandparent (-1 past the root, which is node 0), and the push counts of the
// node and of its parent, so that the walk climbs two levels per load.
__device__ __forceinline__ void node_up(int i, const int32_t* __restrict__ parent, const int2* __restrict__ child,
                                        int4* __restrict__ up)
{
    const int p = i == 0 ? -1 : parent[i];
    int gp = -1, wp = 0;
    if (p >= 0) {
        gp = p == 0 ? -1 : parent[p];
        wp = push_weight(child[p]);
    }
    up[i] = make_int4(p, gp, push_weight(child[i]), wp);
}

// Internal node i's box (as order-preserving keys in ibox) from the pyramid,
// and its record for the upward walk of k_node_depth.
__global__ void k_refit_up(int n, const int2* __restrict__ range, const float4* __restrict__ box,
                           const float4* __restrict__ pyr, PyrLevels pl, int32_t* __restrict__ ibox,
                           const int32_t* __restrict__ parent, const int2* __restrict__ child, int4* __restrict__ up)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    node_up(i, parent, child, up);
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

// Depth of every internal node of the binary tree (the root has depth 0), its
// parity for the 4-wide collapse (as bits, 64 nodes to a mask word, and the
// count per block of kBuildBlock nodes; or as flags in even and idx4, the
// input of a device-wide scan), and the sizes of the 4-wide traversal.  On the path from the root to a
// leaf, every binary node at even depth becomes a 4-wide node that pushes at
// most its slot count minus one entries.  Walking up from node i, the push
// counts of the ancestors at even and at odd distance from i are summed
// apart; once the walk gives i's depth d, the ancestors at even depth are
// those whose distance has the parity of d.  A node with a leaf child ends
// that leaf's path: its depth + 1 and its sum give the tree depth and the
// stack bound (maxima over such nodes, reduced over the wave first).  The
// walk reads one node_up record per two levels; it stops past 4 kMaxStack
// levels (such a tree is rejected by its stack bound).
__global__ void __launch_bounds__(kBuildBlock)
k_node_depth(int n, const int4* __restrict__ up, const int2* __restrict__ child, uint64_t* __restrict__ mask,
             uint32_t* __restrict__ blk_cnt, uint32_t* __restrict__ even, uint32_t* __restrict__ idx4, BuildFlags* f)
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
        if (even) {
            even[i] = is_even;
            idx4[i] = is_even;
        }
        const int2 c = child[i];
        if (is_leaf(c.x) || is_leaf(c.y)) {
            depth_leaf = d + 1;
            need = sum[d & 1];
        }
    }
    // maxima and count over the wave, then over the block: one set of
    // atomics per block (every block updates the same three words)
    const uint64_t bits = __ballot(is_even);
    if (mask && (threadIdx.x & (kWave - 1)) == 0 && i < n - 1) mask[i / kWave] = bits;
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
        if (blk_cnt) blk_cnt[blockIdx.x] = cnt;
        if (depth_leaf > 0) atomicMax(&f->max_depth, depth_leaf);
        if (need > 0) atomicMax(&f->max_stack, need);
        if (cnt) atomicAdd(&f->n_nodes4, cnt);
    }
}

// 4-wide index of an even-depth internal node j: the number of even-depth
// nodes before it.  Either read from the device-wide scan (idx4), or formed
// from the per-block prefix (pref, in LDS) and the bit masks of j's block.
struct Index4 {
    const uint32_t* idx4;
    const uint64_t* mask;
    const uint32_t* pref;
    __device__ __forceinline__ bool even(int j) const { return ((mask[j / kWave] >> (j % kWave)) & 1u) != 0; }
    __device__ __forceinline__ uint32_t operator()(int j) const
    {
        if (idx4) return idx4[j];
        uint32_t r = pref[j / kBuildBlock];
        for (int w = (j / kBuildBlock) * (kBuildBlock / kWave); w < j / kWave; ++w) r += __popcll(mask[w]);
        return r + (uint32_t)__popcll(mask[j / kWave] & lanemask_lt(j % kWave));
    }
};

// Collapse of the binary tree into 4-wide nodes: every internal node at an
// even depth becomes a 4-wide node whose slots are its children, with each
// internal child replaced by that child's own two children (which sit at the
// next even depth).  Node indices are the exclusive prefix sum of the
// even-depth flags, so the root becomes node 0 and nodes keep the Morton order
// of the binary tree.  With the bit masks (mask non-null), the block first
// scans the n_blk per-block counts into the dynamic LDS array pref.
__global__ void __launch_bounds__(kBuildBlock)
k_collapse4(int n, const int2* __restrict__ child, const float4* __restrict__ box, const int32_t* __restrict__ ibox,
            const uint32_t* __restrict__ even, const uint32_t* __restrict__ idx4, const uint64_t* __restrict__ mask,
            const uint32_t* __restrict__ blk_cnt, int n_blk, float4* __restrict__ nodes)
{
    extern __shared__ uint32_t pref[];
    if (mask) {
        __shared__ uint32_t s_wave[kBuildBlock / kWave];
        const int per = (n_blk + kBuildBlock - 1) / kBuildBlock;
        const int b0 = threadIdx.x * per;
        uint32_t v = 0;
        for (int k = 0; k < per; ++k)
            if (b0 + k < n_blk) v += blk_cnt[b0 + k];
        uint32_t run = block_exclusive(v, s_wave);
        for (int k = 0; k < per; ++k)
            if (b0 + k < n_blk) {
                pref[b0 + k] = run;
                run += blk_cnt[b0 + k];
            }
        __syncthreads();
    }
    const Index4 ix{mask ? nullptr : idx4, mask, pref};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1 || !(mask ? ix.even(i) : even[i] != 0u)) return;
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
                links[k++] = is_leaf(gs[b]) ? gs[b] : (int32_t)ix(gs[b]);
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
    float4* o = nodes + (int64_t)kNode4 * ix(i);
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
    BuildMem mem;
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

// Lay out `bufs` in the build memory (growing it when needed; hipFree waits
// for the device's pending work).
template <class... B>
hipError_t mem_place(BuildMem& m, B&... bufs)
{
    size_t need = 0;
    ((need += bufs.bytes), ...);
    if (need > m.cap) {
        if (m.base) {
            hipError_t e = hipFree(m.base);
            if (e != hipSuccess) return e;
            m.base = nullptr;
            m.cap = 0;
        }
        hipError_t e = hipMalloc(&m.base, need + need / 4);
        if (e != hipSuccess) return e;
        m.cap = need + need / 4;
    }
    size_t off = 0;
    auto put = [&](auto& b) {
        b.p = reinterpret_cast<std::remove_reference_t<decltype(b.p)>>(m.base + off);
        off += b.bytes;
    };
    (put(bufs), ...);
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
// pairs, eight bits per pass (an even number of passes, so the sorted pairs
// end in (k0, v0)).  The first count also reduces k_prep's per-block results
// into the flag record.
template <class K>
void morton_sort(const float4* cent, int64_t n, const PrepPartial* part, int n_part, BuildFlags* flags, K* k0,
                 K* k1, uint32_t* v0, uint32_t* v1, uint32_t* counts, uint32_t* sums, int n_tiles, hipStream_t st)
{
    const bool fused = n_tiles <= kFusedScanTiles;
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = 0; shift < 8 * (int)sizeof(K); shift += 8) {
        if (shift == 0)
            hipLaunchKernelGGL(k_morton_count<K>, dim3(n_tiles), dim3(kBuildBlock), 0, st, cent, n, part, n_part,
                               flags, k0, v0, counts, n_tiles);
        else
            hipLaunchKernelGGL(k_radix_count<K>, dim3(n_tiles), dim3(kBuildBlock), 0, st, ki, n, shift, counts,
                               n_tiles);
        if (!fused) scan_exclusive(counts, (int64_t)256 * n_tiles, sums, st);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(n_tiles), dim3(kBuildBlock), 0, st, ki, vi, n, shift, counts,
                           n_tiles, fused, ko, vo, flags);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
}

}  // namespace
}  // namespace rpr

using namespace rpr;

namespace {

// Arguments shared by scene_create and scene_rebuild; `who` names the call in errors.
int check_args(const char* who, const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
               const float* absorption, const float* scattering, int32_t n_materials, int32_t n_bands)
{
    if (n_bands < 1 || n_bands > RPR_MAX_BANDS)
        return set_error(RPR_EINVAL, "%s: n_bands=%d not in 1..%d", who, n_bands, RPR_MAX_BANDS);
    if (n_materials < 1) return set_error(RPR_EINVAL, "%s: n_materials=%d < 1", who, n_materials);
    if (n_tris < 0 || n_verts < 0) return set_error(RPR_EINVAL, "%s: negative size", who);
    if (n_tris > (int64_t)1 << 30)
        return set_error(RPR_EUNSUPPORTED, "%s: n_tris=%lld too large", who, (long long)n_tris);
    if (n_tris > 0 && (!verts || !tris || n_verts < 1))
        return set_error(RPR_EINVAL, "%s: null geometry with n_tris=%lld", who, (long long)n_tris);
    if (!absorption || !scattering) return set_error(RPR_EINVAL, "%s: null material arrays", who);
    return RPR_OK;
}

void free_scene_memory(RprScene* sc)
{
    if (sc->nodes) (void)hipFree(sc->nodes);
    if (sc->tris) (void)hipFree(sc->tris);
    if (sc->mats) (void)hipFree(sc->mats);
    sc->nodes = sc->tris = nullptr;
    sc->mats = nullptr;
    sc->cap_tris = 0;
    sc->cap_materials = 0;
}

// The scene's own arrays: material records, triangle records and 4-wide nodes
// for up to cap_tris triangles and cap_materials materials.
int alloc_scene(RprScene* sc, const char* who, int64_t cap_tris, int32_t cap_materials)
{
    const size_t nt = (size_t)(cap_tris > 0 ? cap_tris : 1);
    const size_t nn = (size_t)(cap_tris > 1 ? cap_tris - 1 : 1);
    hipError_t e = hipMalloc(&sc->mats, sizeof(float) * kMatStride * cap_materials);
    if (e == hipSuccess) e = hipMalloc(&sc->tris, sizeof(float4) * 3 * nt);
    if (e == hipSuccess) e = hipMalloc(&sc->nodes, sizeof(float4) * kNode4 * nn);
    if (e != hipSuccess) {
        free_scene_memory(sc);
        return set_error(e == hipErrorOutOfMemory ? RPR_ENOMEM : RPR_EDEVICE, "%s: hipMalloc: %s", who,
                         hipGetErrorString(e));
    }
    sc->cap_tris = cap_tris;
    sc->cap_materials = cap_materials;
    return RPR_OK;
}

// An empty scene: every ray escapes.  A failed build leaves the scene so.
void set_empty(RprScene* sc)
{
    sc->n_tris = 0;
    sc->max_depth = 0;
    sc->stack_need = 0;
    sc->n_nodes4 = 0;
    sc->n_degenerate = 0;
    for (int a = 0; a < 3; ++a) sc->lo[a] = sc->hi[a] = 0.0f;
    sc->view.nodes = sc->nodes;
    sc->view.tris = sc->tris;
    sc->view.mats = sc->mats;
    sc->view.root = 0;
    sc->view.n_tris = 0;
    sc->view.n_bands = sc->n_bands;
}

// Enqueue the build of the material table, triangle records and BVH into the
// scene's arrays (which hold at least n_tris triangles and n_materials
// materials) on hip_stream, with its temporaries in `mem`; *flags_dev is the
// device record of the build's flags, which finish_build checks once the
// build has run.  The scene is empty until then.
int enqueue_build(RprScene* sc, const char* who, BuildMem& mem, const float* verts, int64_t n_verts,
                  const int32_t* tris, int64_t n_tris, const int32_t* tri_material, const float* absorption,
                  const float* scattering, int32_t n_materials, int32_t n_bands, hipStream_t st,
                  BuildFlags** flags_dev)
{
    const int n = (int)n_tris;
    sc->n_bands = n_bands;
    sc->n_materials = n_materials;
    set_empty(sc);
    auto fail = [&](int code) {
        set_empty(sc);
        return code;
    };

#define TRY(expr)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(set_error(e_ == hipErrorOutOfMemory ? RPR_ENOMEM : RPR_EDEVICE,           \
                                  "%s: %s: %s", who, #expr, hipGetErrorString(e_)));              \
    } while (0)

    DevBuf<BuildFlags> flags;
    TRY(flags.alloc(1));
    DevBuf<PrepPartial> part;
    DevBuf<float4> cent, box;
    DevBuf<uint64_t> k0, k1;  // Morton keys: 32 or 64 bits each
    DevBuf<uint32_t> v0, v1, counts, seen, refs, even, idx4, blk_cnt, scan_sums;
    DevBuf<uint64_t> mask;
    DevBuf<int32_t> ibox, parent;
    DevBuf<int2> child, range;
    DevBuf<float4> pyr;
    const int n_tiles = (int)blocks(n > 0 ? n : 1, kSortTile);
    const int n_blk = (int)blocks(n > 1 ? n - 1 : 1, kBuildBlock);
    const bool fused_index = n_blk <= kFusedIndexBlocks;
    const int n_part = (int)std::min<unsigned>(
        std::max({blocks(n, kPrepBlock), blocks(n_materials, kPrepBlock), 1u}), (unsigned)kPrepBlocks);
    TRY(part.alloc(n_part));
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
        if (fused_index) {
            TRY(mask.alloc(blocks(n > 1 ? n - 1 : 1, kWave)));
            TRY(blk_cnt.alloc(n_blk));
        } else {
            TRY(even.alloc(n - 1));
            TRY(idx4.alloc(n - 1));
        }
        TRY(refs.alloc(2 * (size_t)n - 1));
        TRY(scan_sums.alloc(std::max<size_t>(blocks((int64_t)256 * n_tiles, kSortTile), blocks(n, kSortTile))));
    }
    TRY(mem_place(mem, flags, part, cent, box, k0, v0, k1, v1, counts, seen, refs, even, idx4, blk_cnt, mask,
                    ibox, parent, child, range, pyr, scan_sums));
    hipLaunchKernelGGL(k_prep, dim3(n_part), dim3(kPrepBlock), 0, st, verts, n_verts, tris, n_tris, tri_material,
                       absorption, scattering, n_materials, n_bands, sc->mats, cent.p, seen.p, refs.p, parent.p,
                       part.p);
    TRY(hipGetLastError());

    if (n > 0) {
        const bool wide = n >= kWideKeyTris;
        if (wide) {
            morton_sort<uint64_t>(cent.p, n_tris, part.p, n_part, flags.p, (uint64_t*)k0.p, (uint64_t*)k1.p, v0.p,
                                  v1.p, counts.p, scan_sums.p, n_tiles, st);
            hipLaunchKernelGGL(k_leaves_nodes<uint64_t>, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st,
                               verts, n_verts, tris, tri_material, (const uint64_t*)k0.p, v0.p, n, sc->tris, box.p,
                               seen.p, child.p, parent.p, range.p, refs.p, flags.p);
        } else {
            morton_sort<uint32_t>(cent.p, n_tris, part.p, n_part, flags.p, (uint32_t*)k0.p, (uint32_t*)k1.p, v0.p,
                                  v1.p, counts.p, scan_sums.p, n_tiles, st);
            hipLaunchKernelGGL(k_leaves_nodes<uint32_t>, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st,
                               verts, n_verts, tris, tri_material, (const uint32_t*)k0.p, v0.p, n, sc->tris, box.p,
                               seen.p, child.p, parent.p, range.p, refs.p, flags.p);
        }
        if (n > 1) {
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
            hipLaunchKernelGGL(k_pyr_low, dim3(blocks(n, kBuildBlock)), dim3(kBuildBlock), 0, st, n, box.p, pl, pyr.p,
                               refs.p, flags.p);
            if (pl.top > 8) hipLaunchKernelGGL(k_pyr_high, dim3(1), dim3(1024), 0, st, pl, pyr.p);
            // the centroids are dead after the Morton codes: their n float4 hold the n - 1 walk records
            int4* up = reinterpret_cast<int4*>(cent.p);
            hipLaunchKernelGGL(k_refit_up, dim3(n_blk), dim3(kBuildBlock), 0, st, n, range.p, box.p, pyr.p, pl,
                               ibox.p, parent.p, child.p, up);
            hipLaunchKernelGGL(k_node_depth, dim3(n_blk), dim3(kBuildBlock), 0, st, n, up, child.p,
                               fused_index ? mask.p : nullptr, fused_index ? blk_cnt.p : nullptr,
                               fused_index ? nullptr : even.p, fused_index ? nullptr : idx4.p, flags.p);
            if (!fused_index) scan_exclusive(idx4.p, (int64_t)(n - 1), scan_sums.p, st);
            hipLaunchKernelGGL(k_collapse4, dim3(n_blk), dim3(kBuildBlock),
                               fused_index ? sizeof(uint32_t) * n_blk : 0, st, n, child.p, box.p, ibox.p,
                               fused_index ? nullptr : even.p, fused_index ? nullptr : idx4.p,
                               fused_index ? mask.p : nullptr, fused_index ? blk_cnt.p : nullptr, n_blk, sc->nodes);
        }
        TRY(hipGetLastError());
    } else {
        hipLaunchKernelGGL(k_flags_only, dim3(1), dim3(kWave), 0, st, part.p, n_part, flags.p);
        TRY(hipGetLastError());
    }
    *flags_dev = flags.p;
    return RPR_OK;
#undef TRY
}

// Check a finished build's flags and apply its sizes; on failure the scene
// stays empty.
int finish_build(RprScene* sc, const char* who, int64_t n_tris, const BuildFlags& hf)
{
    const int n = (int)n_tris;
    if (hf.flags & kBadIndex) return set_error(RPR_EINVAL, "%s: vertex index out of range", who);
    if (hf.flags & kBadVertex) return set_error(RPR_EINVAL, "%s: non-finite vertex", who);
    if (hf.flags & kBadMaterial) return set_error(RPR_EINVAL, "%s: material index out of range", who);
    if (hf.flags & kBadCoeff) return set_error(RPR_EINVAL, "%s: absorption/scattering outside [0, 1]", who);
    if (hf.flags & kBadTree) return set_error(RPR_EDEVICE, "%s: BVH consistency check failed", who);
    if (n == 0) return RPR_OK;
    // the traversal writes one slot past the deepest entry (a push without a branch)
    if (hf.max_stack >= kMaxStack)
        return set_error(RPR_EUNSUPPORTED, "%s: BVH depth %d needs %d stack entries, the traversal takes at most %d",
                         who, hf.max_depth, hf.max_stack, kMaxStack - 1);
    sc->max_depth = hf.max_depth;
    sc->stack_need = hf.max_stack;
    sc->n_nodes4 = hf.n_nodes4;
    sc->n_degenerate = (int32_t)hf.n_degenerate;
    for (int a = 0; a < 3; ++a) {
        sc->lo[a] = unordered(hf.blo[a]);
        sc->hi[a] = unordered(hf.bhi[a]);
    }
    sc->n_tris = n_tris;
    sc->view.root = n == 1 ? leaf_link(0) : 0;
    sc->view.n_tris = n;
    return RPR_OK;
}

// Wait (polling, as read_flags) for the event after a rebuild's flag copy.
hipError_t wait_event(hipEvent_t ev)
{
    hipError_t e;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) __builtin_ia32_pause();
    return e;
}

}  // namespace

extern "C" int scene_create(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                            const int32_t* tri_material, const float* absorption, const float* scattering,
                            int32_t n_materials, int32_t n_bands, void* hip_stream, RprScene** out)
{
    if (!out) return set_error(RPR_EINVAL, "scene_create: out is null");
    *out = nullptr;
    int rc = check_args("scene_create", verts, n_verts, tris, n_tris, absorption, scattering, n_materials, n_bands);
    if (rc != RPR_OK) return rc;
    RprScene* sc = new RprScene();
    hipError_t e = hipGetDevice(&sc->device);
    rc = e != hipSuccess ? set_error(RPR_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)) : RPR_OK;
    if (rc == RPR_OK && (sc->device < 0 || sc->device >= 16))
        rc = set_error(RPR_EUNSUPPORTED, "scene_create: device %d", sc->device);
    if (rc == RPR_OK) rc = alloc_scene(sc, "scene_create", n_tris, n_materials);
    if (rc == RPR_OK) {
        // temporaries from the device's shared arena, held until the flags are back
        Arena& arena = g_arena[sc->device];
        std::lock_guard<std::mutex> arena_lock(arena.mu);
        BuildFlags* fd = nullptr;
        rc = enqueue_build(sc, "scene_create", arena.mem, verts, n_verts, tris, n_tris, tri_material, absorption,
                           scattering, n_materials, n_bands, (hipStream_t)hip_stream, &fd);
        BuildFlags hf;
        if (rc == RPR_OK) {
            hipError_t e2 = read_flags(arena, fd, (hipStream_t)hip_stream, &hf);
            if (e2 != hipSuccess) rc = set_error(RPR_EDEVICE, "scene_create: reading the build's flags: %s",
                                                 hipGetErrorString(e2));
        }
        if (rc == RPR_OK) rc = finish_build(sc, "scene_create", n_tris, hf);
    }
    if (rc != RPR_OK) {
        free_scene_memory(sc);
        workspace_free(sc->ws);
        delete sc;
        return rc;
    }
    *out = sc;
    return RPR_OK;
}

extern "C" int scene_rebuild(RprScene* scene, const float* verts, int64_t n_verts, const int32_t* tris,
                             int64_t n_tris, const int32_t* tri_material, const float* absorption,
                             const float* scattering, int32_t n_materials, int32_t n_bands, void* hip_stream)
{
    if (!scene) return set_error(RPR_EINVAL, "scene_rebuild: scene is null");
    int rc = check_args("scene_rebuild", verts, n_verts, tris, n_tris, absorption, scattering, n_materials, n_bands);
    if (rc != RPR_OK) return rc;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(RPR_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != scene->device)
        return set_error(RPR_EINVAL, "scene_rebuild: the scene is on device %d, the current device is %d",
                         scene->device, dev);
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lk(scene->mu);
    if (scene->pending) {
        // an earlier rebuild not yet applied: this one replaces it
        (void)wait_event(scene->built);
        scene->pending = false;
    }
    if (n_tris > scene->cap_tris || n_materials > scene->cap_materials) {
        // grow (never shrink) the arrays; hipFree waits for the device's pending work
        const int64_t cap_tris = std::max(n_tris, scene->cap_tris);
        const int32_t cap_materials = std::max(n_materials, scene->cap_materials);
        free_scene_memory(scene);
        set_empty(scene);
        rc = alloc_scene(scene, "scene_rebuild", cap_tris, cap_materials);
        if (rc != RPR_OK) {
            set_empty(scene);
            return rc;
        }
    }
    if (!scene->flags_host) {
        e = hipHostMalloc(&scene->flags_host, sizeof(BuildFlags), hipHostMallocDefault);
        if (e != hipSuccess) return set_error(RPR_ENOMEM, "scene_rebuild: hipHostMalloc: %s", hipGetErrorString(e));
    }
    if (!scene->built) {
        e = hipEventCreateWithFlags(&scene->built, hipEventDisableTiming);
        if (e != hipSuccess) return set_error(RPR_EDEVICE, "scene_rebuild: hipEventCreate: %s", hipGetErrorString(e));
    }
    BuildFlags* fd = nullptr;
    rc = enqueue_build(scene, "scene_rebuild", scene->build_mem, verts, n_verts, tris, n_tris, tri_material,
                       absorption, scattering, n_materials, n_bands, st, &fd);
    if (rc != RPR_OK) return rc;
    e = hipMemcpyAsync(scene->flags_host, fd, sizeof(BuildFlags), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(scene->built, st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        set_empty(scene);
        return set_error(RPR_EDEVICE, "scene_rebuild: flag copy: %s", hipGetErrorString(e));
    }
    scene->pending = true;
    scene->pending_tris = n_tris;
    return RPR_OK;
}

extern "C" int scene_wait(RprScene* scene)
{
    if (!scene) return set_error(RPR_EINVAL, "scene_wait: scene is null");
    return scene_settle(scene);
}

int rpr::scene_settle(const RprScene* scene_c)
{
    RprScene* sc = const_cast<RprScene*>(scene_c);
    std::lock_guard<std::mutex> lk(sc->mu);
    if (!sc->pending) return RPR_OK;
    sc->pending = false;
    const hipError_t e = wait_event(sc->built);
    if (e != hipSuccess) return set_error(RPR_EDEVICE, "scene_rebuild: %s", hipGetErrorString(e));
    BuildFlags hf;
    std::memcpy(&hf, sc->flags_host, sizeof(hf));
    return finish_build(sc, "scene_rebuild", sc->pending_tris, hf);
}

extern "C" int scene_destroy(RprScene* scene)
{
    if (!scene) return RPR_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != scene->device) (void)hipSetDevice(scene->device);
    if (scene->pending) (void)wait_event(scene->built);
    free_scene_memory(scene);
    if (scene->build_mem.base) (void)hipFree(scene->build_mem.base);
    if (scene->flags_host) (void)hipHostFree(scene->flags_host);
    if (scene->built) (void)hipEventDestroy(scene->built);
    workspace_free(scene->ws);
    if (dev >= 0 && dev != scene->device) (void)hipSetDevice(dev);
    delete scene;
    return RPR_OK;
}

extern "C" int scene_info(const RprScene* scene, RprSceneInfo* out)
{
    if (!scene || !out) return set_error(RPR_EINVAL, "scene_info: null argument");
    std::memset(out, 0, sizeof(*out));
    const int rc = scene_settle(scene);
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
    return rc;
}
