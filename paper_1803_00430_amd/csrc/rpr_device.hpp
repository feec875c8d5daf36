// Device-side primitives of the trace: the counter-based random stream, real
// spherical harmonics, the orthonormal basis of a normal, and the ray/box and
// ray/triangle tests of the BVH traversal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rpr_internal.hpp"

namespace rpr {

// ---------------------------------------------------------------- random stream
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// multiplies whose halves are xored with the other two words and the key;
// the key advances by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = c.x, b = c.z;
        const uint32_t hi_a = __umulhi(0xD2511F53u, a), lo_a = 0xD2511F53u * a;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, b), lo_b = 0xCD9E8D57u * b;
        c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Odd multiple of 2^-24 in (0, 1) from the top 23 bits: exact in FP32.
__device__ __forceinline__ float u01(uint32_t x)
{
    return (float)((x >> 9) * 2u + 1u) * 0x1p-24f;
}

// ---------------------------------------------------------------- real SH
// Real orthonormal spherical harmonics with the Condon-Shortley phase as
// polynomials in the unit vector (x, y, z), coefficient index l(l+1)+m, l <= 3.
__device__ __forceinline__ float sh_coeff(int k, float x, float y, float z)
{
    switch (k) {
    case 0: return 0.28209479177387814f;
    case 1: return -0.4886025119029199f * y;
    case 2: return 0.4886025119029199f * z;
    case 3: return -0.4886025119029199f * x;
    case 4: return 1.0925484305920792f * x * y;
    case 5: return -1.0925484305920792f * y * z;
    case 6: return 0.31539156525252005f * (3.0f * z * z - 1.0f);
    case 7: return -1.0925484305920792f * x * z;
    case 8: return 0.5462742152960396f * (x * x - y * y);
    case 9: return -0.5900435899266435f * y * (3.0f * x * x - y * y);
    case 10: return 2.890611442640554f * x * y * z;
    case 11: return -0.4570457994644658f * y * (5.0f * z * z - 1.0f);
    case 12: return 0.3731763325901154f * z * (5.0f * z * z - 3.0f);
    case 13: return -0.4570457994644658f * x * (5.0f * z * z - 1.0f);
    case 14: return 1.445305721320277f * z * (x * x - y * y);
    case 15: return -0.5900435899266435f * x * (x * x - 3.0f * y * y);
    default: return 0.0f;
    }
}

// ---------------------------------------------------------------- directions
// Uniform direction on the sphere from two uniforms.
__device__ __forceinline__ void sphere_dir(float u0, float u1, float& x, float& y, float& z)
{
    z = 1.0f - 2.0f * u0;                       // exact
    const float rxy = 2.0f * sqrtf(u0 * (1.0f - u0)); // sqrt(1 - z^2) without cancellation
    float s, c;
    sincospif(2.0f * u1, &s, &c);
    x = rxy * c;
    y = rxy * s;
}

// Cosine-weighted direction about the unit normal n, through the branchless
// orthonormal basis of Duff et al. (JCGT 2017).
__device__ __forceinline__ void lambert_dir(float nx, float ny, float nz, float u1, float u2, float& dx,
                                            float& dy, float& dz)
{
    const float sg = nz >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (sg + nz);
    const float b = nx * ny * a;
    const float b1x = 1.0f + sg * nx * nx * a, b1y = sg * b, b1z = -sg * nx;
    const float b2x = b, b2y = sg + ny * ny * a, b2z = -ny;
    const float rr = sqrtf(u2);
    float s, c;
    sincospif(2.0f * u1, &s, &c);
    const float lx = rr * c, ly = rr * s, lz = sqrtf(1.0f - u2);
    dx = lx * b1x + ly * b2x + lz * nx;
    dy = lx * b1y + ly * b2y + lz * ny;
    dz = lx * b1z + ly * b2z + lz * nz;
}

// sin(pi x) and cos(pi x) in FP64 for x in [0, 2]: x = k/2 + r with k = rint(2x)
// and |r| <= 1/4 (exact for the multiples of 2^-23 used here), the Taylor
// series of sin y and cos y at y = pi r (terms through y^17 and y^18, whose
// truncation is below 1e-17), then the quarter turn k.  A dedicated short
// routine: the general one reduces arguments of any size and holds many more
// registers in the trace loop.  The coefficients (-1)^n / (2n+1)! and
// (-1)^n / (2n)!, highest order first, are read from constant memory one at a
// time in a rolled loop: as immediates, or loaded together, the compiler
// hoists them out of the trace loop and holds all of them in registers
// throughout it.
__constant__ double kSinPoly[8] = {-1.0 / 355687428096000.0, 1.0 / 1307674368000.0, -1.0 / 6227020800.0,
                                   1.0 / 39916800.0,         -1.0 / 362880.0,       1.0 / 5040.0,
                                   -1.0 / 120.0,             1.0 / 6.0};
__constant__ double kCosPoly[9] = {1.0 / 6402373705728000.0, -1.0 / 20922789888000.0, 1.0 / 87178291200.0,
                                   -1.0 / 479001600.0,       1.0 / 3628800.0,         -1.0 / 40320.0,
                                   1.0 / 720.0,              -1.0 / 24.0,             0.5};
__device__ __forceinline__ void sincospi_f64(double x, double& s, double& c)
{
    const double k = rint(2.0 * x);
    const double r = x - 0.5 * k;
    const double y = r * 3.141592653589793;
    const double z = y * y;
    double ps = kSinPoly[0], pc = kCosPoly[0];
#pragma unroll 1
    for (int i = 1; i < 8; ++i) ps = fma(ps, z, kSinPoly[i]);
#pragma unroll 1
    for (int i = 1; i < 9; ++i) pc = fma(pc, z, kCosPoly[i]);
    const double sy = fma(-y * z, ps, y);  // y - y^3/3! + ...
    const double cy = fma(-z, pc, 1.0);    // 1 - y^2/2! + ...
    const int q = (int)k & 3;
    const double ss = (q & 1) ? cy : sy, cc = (q & 1) ? sy : cy;
    s = (q & 2) ? -ss : ss;
    c = (q == 1 || q == 2) ? -cc : cc;
}

// The same two samplers in FP64, for the ray state of the forward trace:
// z = 1 - 2 u0, phi = 2 pi u1, radius sqrt(1 - z^2) (uniform sphere), and the
// Lambert lobe (sqrt(u2) cos 2 pi u1, sqrt(u2) sin 2 pi u1, sqrt(1 - u2)) in
// the Duff et al. basis of n.
__device__ __forceinline__ void sphere_dir_f64(double u0, double u1, double& x, double& y, double& z)
{
    z = 1.0 - 2.0 * u0;
    const double rxy = sqrt(fmax(0.0, 1.0 - z * z));
    double s, c;
    sincospi_f64(2.0 * u1, s, c);
    x = rxy * c;
    y = rxy * s;
}

__device__ __forceinline__ void lambert_dir_f64(double nx, double ny, double nz, double u1, double u2, double& dx,
                                                double& dy, double& dz)
{
    const double sg = nz >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (sg + nz);
    const double b = nx * ny * a;
    const double b1x = 1.0 + sg * nx * nx * a, b1y = sg * b, b1z = -sg * nx;
    const double b2x = b, b2y = sg + ny * ny * a, b2z = -ny;
    const double rr = sqrt(u2);
    double s, c;
    sincospi_f64(2.0 * u1, s, c);
    const double lx = rr * c, ly = rr * s, lz = sqrt(fmax(0.0, 1.0 - u2));
    dx = lx * b1x + ly * b2x + lz * nx;
    dy = lx * b1y + ly * b2y + lz * ny;
    dz = lx * b1z + ly * b2z + lz * nz;
}

// ---------------------------------------------------------------- memory
// Loads through the global address space (plain pointers in structs would
// otherwise become flat accesses, which wait on both memory counters).
__device__ __forceinline__ float4 gld(const float4* p)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(1))) v4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------- intersection
// Slab test of one box against [0, tmax], with the plane distances formed as
// lo * (1/d) - o * (1/d) (one fused multiply-add per plane; oi = o * (1/d)).
// No box is flat: every leaf box is padded on all sides (see the build), so
// a ray through an axis-aligned wall's box has tn < tf by the pad's width.
__device__ __forceinline__ bool slab(float lox, float loy, float loz, float hix, float hiy, float hiz,
                                     float oix, float oiy, float oiz, float ix, float iy, float iz, float tmax,
                                     float& tnear)
{
    const float t0x = fmaf(lox, ix, -oix), t1x = fmaf(hix, ix, -oix);
    const float t0y = fmaf(loy, iy, -oiy), t1y = fmaf(hiy, iy, -oiy);
    const float t0z = fmaf(loz, iz, -oiz), t1z = fmaf(hiz, iz, -oiz);
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tnear = tn;
    return tn <= tf;
}

// Moller-Trumbore in FP32 against a triangle record (v0, v1, v2), with the
// barycentric and distance tests done on the numerators scaled by |det| so
// that only the accepted distance needs the reciprocal of det.  The
// barycentric bounds are widened by 1e-6 so that rays through a shared edge
// hit one of its two triangles.  Returns t > 0 or +inf.  Used by the
// occlusion queries, which only need to know whether a hit lies before a
// distance.
__device__ __forceinline__ float tri_test(const float4 a, const float4 b, const float4 c, float ox, float oy,
                                          float oz, float dx, float dy, float dz)
{
    const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const float det = e1x * px + e1y * py + e1z * pz;
    const float sx = ox - a.x, sy = oy - a.y, sz = oz - a.z;
    const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const float sg = det < 0.0f ? -1.0f : 1.0f;
    const float ad = fabsf(det);
    const float u = sg * (sx * px + sy * py + sz * pz);
    const float v = sg * (dx * qx + dy * qy + dz * qz);
    const float t = sg * (e2x * qx + e2y * qy + e2z * qz);
    const float eps = 1e-6f * ad;
    const bool ok = ad != 0.0f && u >= -eps && v >= -eps && u + v <= ad + eps && t > 0.0f;
    return ok ? t / ad : __builtin_inff();
}

// Moller-Trumbore in FP64 against the triangle's exact vertices (the record
// holds the input FP32 coordinates, which FP64 represents exactly): edges
// e1 = v1 - v0, e2 = v2 - v0, p = d x e2, det = e1 . p, s = o - v0,
// u = s . p / det, q = s x e1, v = d . q / det, t = e2 . q / det, accepted when
// 0 <= u, 0 <= v, u + v <= 1 and t > 0.  The bounds are tested on the
// numerators scaled by the sign of det, so only an accepted hit divides.
// Returns t or +inf.  This is the test that decides the closest hit of a path
// segment.
__device__ __forceinline__ double tri_test_f64(const float4 a, const float4 b, const float4 c, double ox,
                                               double oy, double oz, double dx, double dy, double dz)
{
    const double v0x = a.x, v0y = a.y, v0z = a.z;
    const double e1x = (double)b.x - v0x, e1y = (double)b.y - v0y, e1z = (double)b.z - v0z;
    const double e2x = (double)c.x - v0x, e2y = (double)c.y - v0y, e2z = (double)c.z - v0z;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    const double sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const double sg = det < 0.0 ? -1.0 : 1.0;
    const double ad = fabs(det);
    const double u = sg * (sx * px + sy * py + sz * pz);
    const double v = sg * (dx * qx + dy * qy + dz * qz);
    const double t = sg * (e2x * qx + e2y * qy + e2z * qz);
    const bool ok = ad != 0.0 && u >= 0.0 && u <= ad && v >= 0.0 && u + v <= ad && t > 0.0;
    return ok ? t / ad : __builtin_inf();
}

__device__ __forceinline__ float safe_inv(float d)
{
    const float m = 1e-30f;
    return 1.0f / (fabsf(d) > m ? d : (d >= 0.0f ? m : -m));
}

// Closest hit with a per-lane stack in LDS (stack[slot * 64 + lane]) over the
// 4-wide BVH, for the ray o + t d given in FP64.  Boxes are tested in FP32
// against the ray rounded to FP32; the build pads every leaf box by more than
// that rounding moves the ray within the scene, so a box that the FP64 ray
// enters is not culled.  Triangles are tested in FP64 (tri_test_f64), so the
// closest hit is the one the FP64 ray meets.  At an internal node all four
// child boxes are tested; the hit children are ordered by entry distance, the
// nearest is visited next and the others are pushed farthest first.  The
// leaf `exclude` (sorted index) is skipped: the triangle the ray just left.
// Ties in t go to the lower original triangle index.  Only hits closer than
// `tmax` count.  Returns the sorted leaf index of the hit or -1, with t in
// `t_hit` (tmax when there is none).
__device__ __forceinline__ void cswap(float& ta, int32_t& la, float& tb, int32_t& lb)
{
    const bool s = tb < ta;
    const float t0 = s ? tb : ta, t1 = s ? ta : tb;
    const int32_t l0 = s ? lb : la, l1 = s ? la : lb;
    ta = t0;
    tb = t1;
    la = l0;
    lb = l1;
}

template <int STACK, bool COUNT = false>
__device__ __forceinline__ int closest_hit(const SceneView& sc, double ox, double oy, double oz, double dx,
                                           double dy, double dz, int exclude, int32_t* __restrict__ stack, int lane,
                                           double& t_hit, uint32_t& hit_id, uint32_t* n_nodes = nullptr,
                                           uint32_t* n_tris = nullptr, double tmax = __builtin_inf())
{
    const float inf = __builtin_inff();
    double tb = tmax;
    float tbf = (float)tmax;
    int best = -1;
    uint32_t best_id = 0xFFFFFFFFu;
    if (sc.n_tris <= 0) {
        t_hit = tb;
        hit_id = best_id;
        return -1;
    }
    const float ix = safe_inv((float)dx), iy = safe_inv((float)dy), iz = safe_inv((float)dz);
    const float oix = (float)ox * ix, oiy = (float)oy * iy, oiz = (float)oz * iz;
    int sp = 0;
    int32_t node = sc.root;
    // Internal nodes and leaves are handled in separate loops: every lane
    // descends through internal nodes until it holds a leaf (or has nothing
    // left), then the wave tests its leaves together.  A single loop that
    // takes one node of either kind per iteration would run both code paths
    // on every iteration of a wave whose lanes disagree on the kind.
    for (;;) {
        bool done = false;
        while (!is_leaf(node)) {
            const float4* nd = sc.nodes + (int64_t)kNode4 * node;
            float t[4];
            int32_t l[4];
            float4 na[4], nb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                na[j] = gld(nd + 2 * j);
                nb[j] = gld(nd + 2 * j + 1);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 a = na[j], b = nb[j];
                float tn;
                const bool h = slab(a.x, a.y, a.z, b.x, b.y, b.z, oix, oiy, oiz, ix, iy, iz, tbf, tn);
                t[j] = h ? tn : inf;
                l[j] = __float_as_int(a.w);
            }
            if (COUNT) ++*n_nodes;
            // sorting network for four (t, link) pairs
            cswap(t[0], l[0], t[1], l[1]);
            cswap(t[2], l[2], t[3], l[3]);
            cswap(t[0], l[0], t[2], l[2]);
            cswap(t[1], l[1], t[3], l[3]);
            cswap(t[1], l[1], t[2], l[2]);
            if (t[0] < inf) {
                // Every slot is written and the pointer advances over the hit
                // ones only (no branch per child): a write lands at most at
                // the deepest entry a path can reach, which the build checks
                // is below STACK (stack_need < STACK).
#pragma unroll
                for (int j = 3; j >= 1; --j) {
                    stack[sp * kWave + lane] = l[j];
                    sp += t[j] < inf ? 1 : 0;
                }
                node = l[0];
            } else if (sp > 0) {
                node = stack[--sp * kWave + lane];
            } else {
                done = true;
                break;
            }
        }
        if (done) break;
        const int li = leaf_index(node);
        if (li != exclude) {
            const float4* tr = sc.tris + 3 * (int64_t)li;
            const float4 a = gld(tr), b = gld(tr + 1), c = gld(tr + 2);
            if (COUNT) ++*n_tris;
            const double th = tri_test_f64(a, b, c, ox, oy, oz, dx, dy, dz);
            const uint32_t id = __float_as_uint(a.w);
            // a miss is +inf and must never win the tie-break against "no hit yet"
            if (th < tb || (th == tb && th < (double)inf && id < best_id)) {
                tb = th;
                tbf = (float)th;
                best = li;
                best_id = id;
            }
        }
        if (sp == 0) break;
        node = stack[--sp * kWave + lane];
    }
    t_hit = tb;
    hit_id = best_id;
    return best;
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (lane == 0) ? 0ull : (~0ull >> (64 - lane)); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Value of lane `l` (wave-uniform) as a scalar: every lane gets lane l's value.
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdlane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ uint32_t fnv1a(uint32_t h, uint32_t w) { return (h ^ w) * 16777619u; }

}  // namespace rpr
