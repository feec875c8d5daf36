// Listener-origin stochastic ray tracing with next-event estimation toward
// every source (Section 5: backward path tracing from the listener,
// augmented with diffuse rain; one set of rays serves all sources).
//
// One wave per workgroup, one ray per lane, dead lanes refilled from a global
// ray queue as in the source-origin trace.  Each source is a ball of radius r.
// A ray leaves the listener point, reflects like a source-origin ray
// (hero-band kind, balance-heuristic band weights), and contributes:
//   * at the listener (order 0) and at every reflection, one occlusion query
//     per source in a direction uniform in the cone that the source's ball
//     subtends, scored with the track-length estimator and weighted by the
//     lobe density over the cone's density: cos * Omega / pi times the diffuse
//     share E_b (1 - alpha_b) s_b at a reflection, Omega / (4 pi) times E_b at
//     the listener;
//   * every segment that follows a specular choice is scored at each ball
//     with the track-length estimator (the mirror share no query can reach).
// The queries of one source run across the wave together: lanes with a
// pending vertex draw their direction, find the nearest hit up to the far
// side of the ball (the traversal's distance bound culls most of the tree),
// and the wave then issues the deposits of source s as coalesced atomics, one
// 64-lane row (bands x SH coefficients) per depositing lane.  Class energies
// and first bins are summed per source in LDS and flushed once per wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"
#include "trace_acc.hpp"

namespace rpr {
namespace {

constexpr int kSrcChunk = 64;
constexpr int kMaxListenerSources = 256;

struct LstDesc {
    SceneView scene;
    float lst[3];
    float radius, r2, inv_vs;
    float c, dt, l_window, t_window, e0;
    int32_t n_bins, max_bounces, n_coeffs, n_src;
    uint32_t key0, key1, pair_id;
    int32_t pad;
    int64_t ray_begin, n_rays;
    const float4* src;   // [n_src] (x, y, z, 0)
    float* hist;         // [n_src][T][B][NC]
    float* hist_late;    // [n_src][T][B] or null
    RprIrStats* stats;   // [n_src]; the ray-set statistics are summed into stats[0]
    uint32_t* ray_hash;  // [n_rays] or null
    int64_t hist_stride, late_stride;
};

// The 16 real SH of order <= 3 of a unit direction into row[0..15].
__device__ __forceinline__ void sh_row(float x, float y, float z, float* __restrict__ row)
{
#pragma unroll
    for (int c = 0; c < RPR_MAX_COEFFS; ++c) row[c] = sh_coeff(c, x, y, z);
}

// Value of lane l (wave-uniform) of a float.
__device__ __forceinline__ float lane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Each lane's (band, coefficient) in the two 64-float blocks of a bin row
// (B x (n+1)^2 <= 128 floats), fixed for a launch, and 1 / bin width.
struct RowMap {
    int b0, c0, b1, c1;
    float inv_dt;
};

__device__ __forceinline__ RowMap row_map(int lane, int nc, float dt)
{
    RowMap r;
    r.b0 = lane / nc;
    r.c0 = lane % nc;
    r.b1 = (lane + kWave) / nc;
    r.c1 = (lane + kWave) % nc;
    r.inv_dt = 1.0f / dt;
    return r;
}

// Deposit, for every lane with `has` set, the chord [ta, tb] (in seconds of
// propagation time) of source s with band energies e[] and the SH row that
// the lane keeps in shrow (LDS, 16 per lane), as the wave-cooperative row
// update of the source-origin trace.
// Class energies (double) and first bins go to this wave's LDS accumulators.
template <int NB>
__device__ __forceinline__ void wave_deposit(const LstDesc& D, int s, bool has, float ta, float tb, const float* e,
                                             const float* __restrict__ shrow, int order, int lane, const RowMap& rm,
                                             double* __restrict__ cls_acc, int* __restrict__ first_acc,
                                             uint32_t& rows)
{
    uint64_t dm = __ballot(has);
    if (!dm) return;
    const int T = D.n_bins, nc = D.n_coeffs, nb = D.scene.n_bands;
    const float dt = D.dt, inv_vs = D.inv_vs;
    float* __restrict__ hist = D.hist + (size_t)s * D.hist_stride;
    float* __restrict__ hlate = D.hist_late ? D.hist_late + (size_t)s * D.late_stride : nullptr;
    const int nbc = nb * nc;
    while (dm) {
        const int l = __ffsll((unsigned long long)dm) - 1;
        dm &= dm - 1;
        const float a = lane_f(ta, l), b_ = lane_f(tb, l);
        const int kk = __builtin_amdgcn_readlane(order, l);
        float Eb[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) Eb[b] = lane_f(e[b], l);
        int m0 = (int)floorf(a * rm.inv_dt);
        if ((float)m0 * dt > a) --m0;  // never start past the chord
        m0 = m0 < 0 ? 0 : m0;
        float sum_dtau = 0.f;
        int first_m = INT_MAX, n_rows = 0;
        for (int base = 0; base < nbc; base += kWave) {
            const int j = base + lane;
            const bool act = j < nbc;
            const int b = act ? (base ? rm.b1 : rm.b0) : 0, ci = act ? (base ? rm.c1 : rm.c0) : 0;
            float eb = 0.f;
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) eb = (bb == b) ? Eb[bb] : eb;
            const float val = eb * shrow[l * RPR_MAX_COEFFS + ci] * inv_vs;
            const bool late = act && kk >= 3 && ci == 0 && hlate != nullptr;
            for (int m = m0; m < T; ++m) {
                const float lo = fmaxf(a, (float)m * dt);
                const float hi = fminf(b_, (float)(m + 1) * dt);
                if (lo >= b_) break;
                const float dtau = hi - lo;
                if (dtau > 0.f) {
                    if (act) unsafeAtomicAdd(hist + ((size_t)m * nb + b) * nc + ci, val * dtau);
                    if (late) unsafeAtomicAdd(hlate + (size_t)m * nb + b, eb * dtau * inv_vs);
                    if (base == 0) {
                        sum_dtau += dtau;
                        first_m = min(first_m, m);
                        ++n_rows;
                    }
                }
            }
        }
        rows += (uint32_t)n_rows;
        const int cls = kk == 0 ? 0 : (kk <= 2 ? 1 : 2);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (lane == b && b < nb) cls_acc[(s * 3 + cls) * NB + b] += (double)(Eb[b] * sum_dtau * inv_vs);
        if (lane == 0 && first_m != INT_MAX) {
            first_acc[2 * s] = min(first_acc[2 * s], first_m);
            if (kk >= 3) first_acc[2 * s + 1] = min(first_acc[2 * s + 1], first_m);
        }
    }
}

// Chord of o + t d, 0 <= t <= tmax, through the ball (p, r2 = r^2).
__device__ __forceinline__ bool ball_chord(float ox, float oy, float oz, float dx, float dy, float dz, float tmax,
                                           float4 p, float r2, float& ta, float& tb)
{
    const float cx = ox - p.x, cy = oy - p.y, cz = oz - p.z;
    const float bq = dx * cx + dy * cy + dz * cz;
    const float wx = cx - bq * dx, wy = cy - bq * dy, wz = cz - bq * dz;
    const float disc = r2 - (wx * wx + wy * wy + wz * wz);
    if (!(disc > 0.f)) return false;
    const float sq = sqrtf(disc);
    ta = fmaxf(-bq - sq, 0.f);
    tb = fminf(-bq + sq, tmax);
    return tb > ta;
}

// Occlusion query of a next-event segment: the nearest hit in (0, tb) of
// o + t d, except that any hit at t <= ta (before the ball's chord begins)
// ends the search at once, since the segment is then occluded whatever lies
// nearer.  The excluded leaf is the vertex's own triangle.  Returns that
// first blocking t (<= ta), else the nearest hit in (ta, tb), else tb: the
// same three outcomes as the nearest-hit definition.  Traversal as
// closest_hit (4-wide nodes, per-lane LDS stack, internal and leaf loops).
template <int STACK>
__device__ __forceinline__ float occlusion_query(const SceneView& sc, float ox, float oy, float oz, float dx,
                                                 float dy, float dz, float ta, float tb, int exclude,
                                                 int32_t* __restrict__ stack, int lane)
{
    const float inf = __builtin_inff();
    if (sc.n_tris <= 0) return tb;
    const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
    const float oix = ox * ix, oiy = oy * iy, oiz = oz * iz;
    int sp = 0;
    int32_t node = sc.root;
    float tcur = tb;
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
                const bool h = slab(a.x, a.y, a.z, b.x, b.y, b.z, oix, oiy, oiz, ix, iy, iz, tcur, tn);
                t[j] = h ? tn : inf;
                l[j] = __float_as_int(a.w);
            }
            cswap(t[0], l[0], t[1], l[1]);
            cswap(t[2], l[2], t[3], l[3]);
            cswap(t[0], l[0], t[2], l[2]);
            cswap(t[1], l[1], t[3], l[3]);
            cswap(t[1], l[1], t[2], l[2]);
            if (t[0] < inf) {
#pragma unroll
                for (int j = 3; j >= 1; --j)
                    if (t[j] < inf && sp < STACK) stack[sp++ * kWave + lane] = l[j];
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
            const float th = tri_test(gld(tr), gld(tr + 1), gld(tr + 2), ox, oy, oz, dx, dy, dz);
            if (th <= ta) return th;
            if (th < tcur) tcur = th;
        }
        if (sp == 0) break;
        node = stack[--sp * kWave + lane];
    }
    return tcur;
}

template <int NB, int STACK>
// With four bands and up to 48 stack entries the kernel is held to 168 VGPRs
// (a few bytes of spills) so that 3 waves fit per SIMD instead of 2.
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(NB <= 4 && STACK <= 48 ? 3 : 1)))
k_trace_lst(const LstDesc D, unsigned long long* __restrict__ queue)
{
    __shared__ int32_t stk[STACK * kWave];
    __shared__ float shrow[kWave * RPR_MAX_COEFFS];  // SH of each lane's arrival direction
    extern __shared__ double dyn[];
    double* cls_acc = dyn;                                     // [n_src][3][NB]
    int* first_acc = (int*)(dyn + (size_t)D.n_src * 3 * NB);   // [n_src][2]
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt(lane);
    for (int i = lane; i < D.n_src * 3 * NB; i += kWave) cls_acc[i] = 0.0;
    for (int i = lane; i < 2 * D.n_src; i += kWave) first_acc[i] = INT_MAX;
    __syncthreads();

    const SceneView& sc = D.scene;
    const int nbr = sc.n_bands;
    const long long total = D.n_rays;
    const RowMap rm = row_map(lane, D.n_coeffs, D.dt);
    bool alive = false, spec = false, nee = false, nee_lst = false;
    uint32_t ray = 0;
    long long rl = 0;
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 1.f, L = 0.f;
    float ax = 0.f, ay = 0.f, az = 1.f;  // arrival direction at the listener
    int k = 0, last = -1;
    uint32_t h = 0;
    float E[NB], Q[NB];
    // pending next-event vertex: origin, facing normal, path length, order,
    // excluded leaf, per-band share, and the bounce kind still to be hashed
    float vx = 0.f, vy = 0.f, vz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f, vL = 0.f;
    int vk = 0, vexcl = -1;
    uint32_t vkind = 0;
    float F[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) E[b] = Q[b] = F[b] = 0.f;
    uint32_t a_seg = 0, a_fin = 0, a_esc = 0, a_rays = 0, a_nq = 0, a_rows = 0;  // a_rows: wave-uniform
    double a_len = 0.0;
    float a_esc_e[NB], a_alive[NB], a_cap[NB], a_absb[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) a_esc_e[b] = a_alive[b] = a_cap[b] = a_absb[b] = 0.f;
    bool exhausted = false;
    // each wave's first 64 slots are fixed by its index; the counter hands
    // out the slots after gridDim.x * 64 (no burst of atomics at the start)
    const unsigned long long n_static = (unsigned long long)gridDim.x * kWave;
    bool first = true;

    for (;;) {
        // ------------------------------------------------ refill dead lanes
        if (!exhausted) {
            const uint64_t dead = __ballot(!alive);
            if (dead) {
                const int nd = __popcll(dead);
                const int leader = __ffsll((unsigned long long)dead) - 1;
                unsigned long long base = 0;
                if (first) {
                    // every lane is dead before the first fill: nd = 64
                    base = (unsigned long long)blockIdx.x * kWave;
                    first = false;
                    if (n_static >= (unsigned long long)total) exhausted = true;
                } else {
                    if (lane == leader) base = atomicAdd(queue, (unsigned long long)nd);
                    base = n_static + __shfl(base, leader);
                    if (base + (unsigned long long)nd >= (unsigned long long)total) exhausted = true;
                }
                if (!alive) {
                    const long long r = (long long)(base + (unsigned long long)__popcll(dead & lt));
                    if (r < total) {
                        rl = r;
                        ray = (uint32_t)(D.ray_begin + rl);
                        const uint4 x = philox4x32_10(make_uint4(ray, D.pair_id, 0u, 0u), D.key0, D.key1);
                        sphere_dir(u01(x.x), u01(x.y), dx, dy, dz);
                        ax = dx;
                        ay = dy;
                        az = dz;
                        sh_row(ax, ay, az, shrow + lane * RPR_MAX_COEFFS);
                        ox = vx = D.lst[0];
                        oy = vy = D.lst[1];
                        oz = vz = D.lst[2];
                        L = vL = 0.f;
                        k = vk = 0;
                        last = vexcl = -1;
                        h = 2166136261u;
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            E[b] = b < nbr ? D.e0 : 0.f;
                            Q[b] = b < nbr ? 1.f : 0.f;
                            F[b] = E[b];
                        }
                        spec = false;
                        nee = true;
                        nee_lst = true;
                        alive = true;
                    }
                }
            }
        }
        if (__ballot(alive) == 0) break;

        // ------------------------------------------------ next-event queries
        if (__ballot(nee)) {
            for (int s = 0; s < D.n_src; ++s) {
                const float4 ps = gld(D.src + s);
                bool has = false;
                float ta = 0.f, tb = 0.f, wx = 0.f, wy = 0.f, wz = 1.f;
                float e[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) e[b] = 0.f;
                if (nee) {
                    const uint4 x =
                        philox4x32_10(make_uint4(ray, D.pair_id, (uint32_t)vk, 1u + (uint32_t)s), D.key0, D.key1);
                    const float px = ps.x - vx, py = ps.y - vy, pz = ps.z - vz;
                    const float rc2 = px * px + py * py + pz * pz;
                    float g = 0.f;
                    if (rc2 <= D.r2) {
                        // inside the ball: the whole lobe
                        if (nee_lst) sphere_dir(u01(x.x), u01(x.y), wx, wy, wz);
                        else lambert_dir(nx, ny, nz, u01(x.y), u01(x.z), wx, wy, wz);
                        g = 1.f;
                    } else {
                        // uniform in the cone of the ball: 1 - cos = u0 (1 - cos g),
                        // with 1 - cos g = h / (1 + sqrt(1 - h)), h = r^2 / d^2
                        const float irc = 1.0f / sqrtf(rc2);
                        const float qx = px * irc, qy = py * irc, qz = pz * irc;
                        const float hq = D.r2 / rc2;
                        const float omc = hq / (1.0f + sqrtf(1.0f - hq));
                        const float w1 = u01(x.x) * omc;  // 1 - cos
                        const float ct = 1.0f - w1;
                        const float st = sqrtf(w1 * (2.0f - w1));
                        const float sg = qz >= 0.0f ? 1.0f : -1.0f;
                        const float aa = -1.0f / (sg + qz);
                        const float bb = qx * qy * aa;
                        const float b1x = 1.0f + sg * qx * qx * aa, b1y = sg * bb, b1z = -sg * qx;
                        const float b2x = bb, b2y = sg + qy * qy * aa, b2z = -qy;
                        float sn, cs;
                        sincospif(2.0f * u01(x.y), &sn, &cs);
                        wx = st * cs * b1x + st * sn * b2x + ct * qx;
                        wy = st * cs * b1y + st * sn * b2y + ct * qy;
                        wz = st * cs * b1z + st * sn * b2z + ct * qz;
                        const float omega = 2.0f * (float)M_PI * omc;
                        if (nee_lst) {
                            g = omega * (float)(0.25 / M_PI);
                        } else {
                            const float cw = nx * wx + ny * wy + nz * wz;
                            g = cw > 0.f ? cw * omega * (float)(1.0 / M_PI) : 0.f;
                        }
                    }
                    if (g > 0.f && ball_chord(vx, vy, vz, wx, wy, wz, __builtin_inff(), ps, D.r2, ta, tb) &&
                        vL + ta < D.l_window) {
                        ++a_nq;
                        const float t_occ = occlusion_query<STACK>(sc, vx, vy, vz, wx, wy, wz, ta, tb, vexcl, stk, lane);
                        if (t_occ <= ta) {
                            h = fnv1a(h, 3u);
                        } else {
                            if (t_occ < tb) {
                                tb = t_occ;
                                h = fnv1a(h, 4u);
                            } else {
                                h = fnv1a(h, 2u);
                            }
                            has = true;
#pragma unroll
                            for (int b = 0; b < NB; ++b) e[b] = F[b] * g;
                            ta = (vL + ta) / D.c;
                            tb = (vL + tb) / D.c;
                        }
                    }
                }
                // the direct sound arrives from the query direction itself
                const bool own = has && nee_lst;
                if (own) sh_row(wx, wy, wz, shrow + lane * RPR_MAX_COEFFS);
                __syncthreads();
                wave_deposit<NB>(D, s, has, ta, tb, e, shrow, vk, lane, rm, cls_acc, first_acc, a_rows);
                __syncthreads();
                if (own) sh_row(ax, ay, az, shrow + lane * RPR_MAX_COEFFS);
            }
            if (nee && !nee_lst) h = fnv1a(h, vkind);
            nee = false;
        }

        // ------------------------------------------------ closest hit
        float t_hit = __builtin_inff();
        uint32_t hit_id = 0xFFFFFFFFu;
        int hit = -1;
        if (alive) {
            double th;
            hit = closest_hit<STACK>(sc, ox, oy, oz, dx, dy, dz, last, stk, lane, th, hit_id);
            t_hit = (float)th;
        }

        // ------------------------------------------------ mirror share at the source balls
        if (__ballot(alive && spec)) {
            for (int s = 0; s < D.n_src; ++s) {
                const float4 ps = gld(D.src + s);
                float ta = 0.f, tb = 0.f;
                bool has = false;
                if (alive && spec && ball_chord(ox, oy, oz, dx, dy, dz, t_hit, ps, D.r2, ta, tb)) {
                    ta = (L + ta) / D.c;
                    tb = (L + tb) / D.c;
                    has = ta < D.t_window;
                }
                wave_deposit<NB>(D, s, has, ta, tb, E, shrow, k, lane, rm, cls_acc, first_acc, a_rows);
            }
        }

        // ------------------------------------------------ bounce or terminate
        if (alive) {
            ++a_seg;
            bool term = false;
            if (hit < 0) {
                ++a_esc;
                h = fnv1a(h, 0xFFFFFFFFu);
#pragma unroll
                for (int b = 0; b < NB; ++b) a_esc_e[b] += E[b];
                term = true;
            } else {
                L += t_hit;
                ++a_fin;
                a_len += (double)t_hit;
                h = fnv1a(h, hit_id);
                const bool win = L >= D.l_window;
                if (win || k == D.max_bounces) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        a_alive[b] += E[b];
                        if (!win) a_cap[b] += E[b];
                    }
                    term = true;
                } else {
                    ++k;
                    ox += t_hit * dx;
                    oy += t_hit * dy;
                    oz += t_hit * dz;
                    const float4* tr = sc.tris + 3 * (int64_t)hit;
                    const float4 v0 = tr[0], v1 = tr[1], v2 = tr[2];
                    const float4 e1 = make_float4(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z, v1.w);
                    const float4 e2 = make_float4(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z, 0.0f);
                    float mx = e1.y * e2.z - e1.z * e2.y, my = e1.z * e2.x - e1.x * e2.z,
                          mz = e1.x * e2.y - e1.y * e2.x;
                    const float inl = 1.0f / sqrtf(mx * mx + my * my + mz * mz);
                    mx *= inl;
                    my *= inl;
                    mz *= inl;
                    if (dx * mx + dy * my + dz * mz > 0.f) {
                        mx = -mx;
                        my = -my;
                        mz = -mz;
                    }
                    const float* __restrict__ mr = sc.mats + (int64_t)__float_as_int(e1.w) * kMatStride;
                    // the next-event vertex: the offset hit point with the
                    // reflection's diffuse share, queried at the next iteration
                    ox = fmaf(kSurfaceOffset, mx, ox);
                    oy = fmaf(kSurfaceOffset, my, oy);
                    oz = fmaf(kSurfaceOffset, mz, oz);
                    vx = ox;
                    vy = oy;
                    vz = oz;
                    nx = mx;
                    ny = my;
                    nz = mz;
                    vL = L;
                    vk = k;
                    vexcl = hit;
#pragma unroll
                    for (int b = 0; b < NB; ++b) F[b] = E[b] * mr[kMatKeep + b] * mr[kMatS + b];
                    nee = true;
                    nee_lst = false;
                    const uint4 x = philox4x32_10(make_uint4(ray, D.pair_id, (uint32_t)k, 0u), D.key0, D.key1);
#pragma unroll
                    for (int b = 0; b < NB; ++b) a_absb[b] += mr[kMatAlpha + b] * E[b];
                    const bool diffuse = u01(x.x) < mr[kMatS + (int)(ray % (uint32_t)nbr)];
                    float q[NB], mean_q = 0.f;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        q[b] = diffuse ? mr[kMatS + b] : 1.f - mr[kMatS + b];
                        mean_q += Q[b] * q[b];
                    }
                    const float inv_mean = (float)nbr / fmaxf(mean_q, 1e-30f);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float r = q[b] * inv_mean;
                        Q[b] *= r;
                        E[b] *= mr[kMatKeep + b] * r;
                    }
                    if (diffuse) {
                        lambert_dir(mx, my, mz, u01(x.y), u01(x.z), dx, dy, dz);
                    } else {
                        const float dn = 2.0f * (dx * mx + dy * my + dz * mz);
                        dx -= dn * mx;
                        dy -= dn * my;
                        dz -= dn * mz;
                        const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                        dx *= il;
                        dy *= il;
                        dz *= il;
                    }
                    vkind = diffuse ? 1u : 0u;
                    spec = !diffuse;
                    last = hit;
                }
            }
            if (term) {
                ++a_rays;
                if (D.ray_hash) D.ray_hash[rl] = h;
                alive = false;
            }
        }
    }

    // ------------------------------------------------ flush
    RprIrStats* S = D.stats;
    const uint32_t seg = wave_sum_u32(a_seg), fin = wave_sum_u32(a_fin), esc = wave_sum_u32(a_esc);
    const uint32_t rays = wave_sum_u32(a_rays), nq = wave_sum_u32(a_nq);
    const double len = wave_sum(a_len);
    if (lane == 0 && rays + seg > 0) {
        atomicAdd((unsigned long long*)&S->n_segments, (unsigned long long)seg);
        atomicAdd((unsigned long long*)&S->n_finite_segments, (unsigned long long)fin);
        atomicAdd((unsigned long long*)&S->n_escaped, (unsigned long long)esc);
        atomicAdd((unsigned long long*)&S->n_rays, (unsigned long long)rays);
        atomicAdd((unsigned long long*)&S->n_next_event, (unsigned long long)nq);
        atomicAdd((unsigned long long*)&S->n_deposit_rows, (unsigned long long)a_rows);
        unsafeAtomicAdd(&S->seg_len_sum, len);
        unsafeAtomicAdd(&S->e_emitted, (double)rays * (double)D.e0);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nbr) break;
        const double ve = wave_sum((double)a_esc_e[b]);
        const double va = wave_sum((double)a_alive[b]);
        const double vc = wave_sum((double)a_cap[b]);
        const double vb = wave_sum((double)a_absb[b]);
        if (lane == 0 && rays + seg > 0) {
            unsafeAtomicAdd(&S->e_escaped[b], ve);
            unsafeAtomicAdd(&S->e_alive_at_stop[b], va);
            unsafeAtomicAdd(&S->e_alive_at_bounce_cap[b], vc);
            unsafeAtomicAdd(&S->e_absorbed[b], vb);
        }
    }
    __syncthreads();
    for (int i = lane; i < D.n_src * 3 * NB; i += kWave) {
        const int s = i / (3 * NB), c = (i / NB) % 3, b = i % NB;
        if (b < nbr && cls_acc[i] != 0.0) unsafeAtomicAdd(&D.stats[s].e_class[c][b], cls_acc[i]);
    }
    for (int i = lane; i < 2 * D.n_src; i += kWave) {
        const int v = first_acc[i];
        if (v != INT_MAX) {
            if (i & 1) atomicMin(&D.stats[i >> 1].first_late_bin, v);
            else atomicMin(&D.stats[i >> 1].first_arrival_bin, v);
        }
    }
}

// ---------------------------------------------------------------- batched pairs
// Wave-cooperative deposit of every lane with `has` set into the histogram of
// its own pair (as the source-origin trace's deposit), with the lane's SH row
// in shrow and the class of `order`; class energies and first bins
// go to the per-pair accumulator `dep`.
template <int NB>
__device__ __forceinline__ void pair_deposit(const PairDesc* __restrict__ pairs, bool has, int p, float ta, float tb,
                                             const float* e, const float* __restrict__ shrow, int order, int lane,
                                             const RowMap& rm, DepAcc& dep)
{
    uint64_t dm = __ballot(has);
    while (dm) {
        const int l = __ffsll((unsigned long long)dm) - 1;
        dm &= dm - 1;
        const int q = __builtin_amdgcn_readlane(p, l);
        const float a = lane_f(ta, l), b_ = lane_f(tb, l);
        const int kk = __builtin_amdgcn_readlane(order, l);
        float Eb[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) Eb[b] = lane_f(e[b], l);
        const PairDesc& P = pairs[q];
        const int T = P.n_bins, nc = P.n_coeffs, nb = P.scene.n_bands;
        const float dt = P.dt, inv_vs = P.inv_vs;
        float* __restrict__ hist = P.hist;
        float* __restrict__ hlate = P.hist_late;
        const int nbc = nb * nc;
        int m0 = (int)floorf(a * rm.inv_dt);
        if ((float)m0 * dt > a) --m0;  // never start past the chord
        m0 = m0 < 0 ? 0 : m0;
        float sum_dtau = 0.f;
        int first_m = INT_MAX, n_rows = 0;
        for (int base = 0; base < nbc; base += kWave) {
            const int j = base + lane;
            const bool act = j < nbc;
            const int b = act ? (base ? rm.b1 : rm.b0) : 0, ci = act ? (base ? rm.c1 : rm.c0) : 0;
            float eb = 0.f;
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) eb = (bb == b) ? Eb[bb] : eb;
            const float val = eb * shrow[l * RPR_MAX_COEFFS + ci] * inv_vs;
            const bool late = act && kk >= 3 && ci == 0 && hlate != nullptr;
            for (int m = m0; m < T; ++m) {
                const float lo = fmaxf(a, (float)m * dt);
                const float hi = fminf(b_, (float)(m + 1) * dt);
                if (lo >= b_) break;
                const float dtau = hi - lo;
                if (dtau > 0.f) {
                    if (act) unsafeAtomicAdd(hist + ((size_t)m * nb + b) * nc + ci, val * dtau);
                    if (late) unsafeAtomicAdd(hlate + (size_t)m * nb + b, eb * dtau * inv_vs);
                    if (base == 0) {
                        sum_dtau += dtau;
                        first_m = min(first_m, m);
                        ++n_rows;
                    }
                }
            }
        }
        if (q != dep.p) {
            dep_acc_flush<NB>(dep, pairs, lane);
            dep.p = q;
        }
        dep.rows += (uint32_t)n_rows;
        const int cls = kk == 0 ? 0 : (kk <= 2 ? 1 : 2);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (lane == cls * NB + b) dep.e += (double)(Eb[b] * sum_dtau * inv_vs);
        if (first_m != INT_MAX) {
            dep.fa = min(dep.fa, first_m);
            if (kk >= 3) dep.fl = min(dep.fl, first_m);
        }
    }
}

// The listener-origin trace over a table of chunks of pairs (one source
// each; a chunk is a pair's descriptor with a ray range of its own).  A wave
// takes a whole chunk from the queue with one atomic and fills its lanes from
// that chunk alone, so its lanes hold rays of one or two chunks at a time and
// the per-pair statistics are flushed about once per chunk, while the chunks
// of different pairs, dealt to different waves, spread the histogram atomics
// over many pairs.  Each pair's rays leave its listener point and query its
// source's ball.
template <int NB, int STACK>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(NB <= 4 && STACK <= 48 ? 3 : 1)))
k_trace_lstp(const PairDesc* __restrict__ pairs, int n_table, unsigned long long* __restrict__ queue)
{
    __shared__ int32_t stk[STACK * kWave];
    __shared__ float shrow[kWave * RPR_MAX_COEFFS];  // SH of each lane's arrival direction
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt(lane);
    bool alive = false, spec = false, nee = false, nee_lst = false;
    int p = -1;
    uint32_t ray = 0;
    long long rl = 0;
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 1.f, L = 0.f;
    float ax = 0.f, ay = 0.f, az = 1.f;
    int k = 0, last = -1;
    uint32_t h = 0;
    float E[NB], Q[NB], F[NB];
    float vx = 0.f, vy = 0.f, vz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f, vL = 0.f;
    int vk = 0, vexcl = -1;
    uint32_t vkind = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) E[b] = Q[b] = F[b] = 0.f;
    SceneView sc{};
    LaneAcc<NB> acc;
    lane_acc_zero(acc);
    DepAcc dep{-1, 0.0, INT_MAX, INT_MAX, 0u};
    bool exhausted = false;
    int ch = -1;                      // the wave's current chunk (wave-uniform)
    long long ch_off = 0, ch_len = 0; // next ray of the chunk, its ray count
    // bands, coefficients and bin width are the same for every pair of a batch
    const RowMap rm = row_map(lane, pairs[0].n_coeffs, pairs[0].dt);

    for (;;) {
        if (!exhausted) {
            uint64_t dead = __ballot(!alive);
            int np = -1;
            long long rr = 0;
            while (dead) {
                if (ch_off >= ch_len) {
                    // the first chunk of each wave is fixed by its index (the
                    // grid has at most one wave per chunk); the counter hands
                    // out the chunks after gridDim.x
                    unsigned long long c = 0;
                    if (ch < 0) {
                        c = blockIdx.x;
                    } else {
                        if (lane == 0) c = atomicAdd(queue, 1ull);
                        c = (unsigned long long)gridDim.x + __shfl(c, 0);
                    }
                    if (c >= (unsigned long long)n_table) {
                        exhausted = true;
                        break;
                    }
                    ch = (int)c;
                    ch_off = 0;
                    ch_len = pairs[ch].n_rays;
                }
                const long long avail = ch_len - ch_off;
                const int nd = __popcll(dead);
                const int take = (int)(avail < (long long)nd ? avail : (long long)nd);
                const int rank = __popcll(dead & lt);
                const bool mine = ((dead >> lane) & 1ull) && rank < take;
                if (mine) {
                    np = ch;
                    rr = ch_off + rank;
                }
                dead &= ~__ballot(mine);
                ch_off += take;
            }
            if (__ballot(np >= 0 && acc.p >= 0 && acc.p != np)) lane_acc_flush<NB, false, true>(acc, pairs, lane);
            if (np >= 0) {
                const PairDesc& P = pairs[np];
                p = np;
                rl = rr;
                ray = (uint32_t)(P.ray_begin + rl);
                const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, 0u, 0u), P.key0, P.key1);
                sphere_dir(u01(x.x), u01(x.y), dx, dy, dz);
                ax = dx;
                ay = dy;
                az = dz;
                sh_row(ax, ay, az, shrow + lane * RPR_MAX_COEFFS);
                ox = vx = P.lst[0];
                oy = vy = P.lst[1];
                oz = vz = P.lst[2];
                L = vL = 0.f;
                k = vk = 0;
                last = vexcl = -1;
                h = 2166136261u;
                sc = P.scene;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    E[b] = b < sc.n_bands ? P.e0 : 0.f;
                    Q[b] = b < sc.n_bands ? 1.f : 0.f;
                    F[b] = E[b];
                }
                spec = false;
                nee = true;
                nee_lst = true;
                alive = true;
            }
        }
        if (__ballot(alive) == 0) break;

        // ------------------------------------------------ next-event query toward the pair's source
        if (__ballot(nee)) {
            bool has = false;
            float ta = 0.f, tb = 0.f, wx = 0.f, wy = 0.f, wz = 1.f;
            float e[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) e[b] = 0.f;
            if (nee) {
                const PairDesc& P = pairs[p];
                const float4 ps = make_float4(P.src[0], P.src[1], P.src[2], 0.f);
                const float r2 = P.radius * P.radius;
                const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, (uint32_t)vk, 1u), P.key0, P.key1);
                const float px = ps.x - vx, py = ps.y - vy, pz = ps.z - vz;
                const float rc2 = px * px + py * py + pz * pz;
                float g = 0.f;
                if (rc2 <= r2) {
                    if (nee_lst) sphere_dir(u01(x.x), u01(x.y), wx, wy, wz);
                    else lambert_dir(nx, ny, nz, u01(x.y), u01(x.z), wx, wy, wz);
                    g = 1.f;
                } else {
                    const float irc = 1.0f / sqrtf(rc2);
                    const float qx = px * irc, qy = py * irc, qz = pz * irc;
                    const float hq = r2 / rc2;
                    const float omc = hq / (1.0f + sqrtf(1.0f - hq));
                    const float w1 = u01(x.x) * omc;
                    const float ct = 1.0f - w1;
                    const float st = sqrtf(w1 * (2.0f - w1));
                    const float sg = qz >= 0.0f ? 1.0f : -1.0f;
                    const float aa = -1.0f / (sg + qz);
                    const float bb = qx * qy * aa;
                    const float b1x = 1.0f + sg * qx * qx * aa, b1y = sg * bb, b1z = -sg * qx;
                    const float b2x = bb, b2y = sg + qy * qy * aa, b2z = -qy;
                    float sn, cs;
                    sincospif(2.0f * u01(x.y), &sn, &cs);
                    wx = st * cs * b1x + st * sn * b2x + ct * qx;
                    wy = st * cs * b1y + st * sn * b2y + ct * qy;
                    wz = st * cs * b1z + st * sn * b2z + ct * qz;
                    const float omega = 2.0f * (float)M_PI * omc;
                    if (nee_lst) {
                        g = omega * (float)(0.25 / M_PI);
                    } else {
                        const float cw = nx * wx + ny * wy + nz * wz;
                        g = cw > 0.f ? cw * omega * (float)(1.0 / M_PI) : 0.f;
                    }
                }
                if (g > 0.f && ball_chord(vx, vy, vz, wx, wy, wz, __builtin_inff(), ps, r2, ta, tb) &&
                    vL + ta < P.l_window) {
                    ++acc.nq;
                    const float t_occ = occlusion_query<STACK>(sc, vx, vy, vz, wx, wy, wz, ta, tb, vexcl, stk, lane);
                    if (t_occ <= ta) {
                        h = fnv1a(h, 3u);
                    } else {
                        if (t_occ < tb) {
                            tb = t_occ;
                            h = fnv1a(h, 4u);
                        } else {
                            h = fnv1a(h, 2u);
                        }
                        has = true;
#pragma unroll
                        for (int b = 0; b < NB; ++b) e[b] = F[b] * g;
                        ta = (vL + ta) / P.c;
                        tb = (vL + tb) / P.c;
                    }
                }
                if (!nee_lst) h = fnv1a(h, vkind);
            }
            // the direct sound arrives from the query direction itself
            const bool own = has && nee_lst;
            if (own) sh_row(wx, wy, wz, shrow + lane * RPR_MAX_COEFFS);
            __syncthreads();
            pair_deposit<NB>(pairs, has, p, ta, tb, e, shrow, vk, lane, rm, dep);
            __syncthreads();
            if (own) sh_row(ax, ay, az, shrow + lane * RPR_MAX_COEFFS);
            nee = false;
        }

        // ------------------------------------------------ closest hit
        float t_hit = __builtin_inff();
        uint32_t hit_id = 0xFFFFFFFFu;
        int hit = -1;
        if (alive) {
            double th;
            hit = closest_hit<STACK>(sc, ox, oy, oz, dx, dy, dz, last, stk, lane, th, hit_id);
            t_hit = (float)th;
        }

        // ------------------------------------------------ mirror share at the source ball
        if (__ballot(alive && spec)) {
            float ta = 0.f, tb = 0.f;
            bool has = false;
            if (alive && spec) {
                const PairDesc& P = pairs[p];
                const float4 ps = make_float4(P.src[0], P.src[1], P.src[2], 0.f);
                if (ball_chord(ox, oy, oz, dx, dy, dz, t_hit, ps, P.radius * P.radius, ta, tb)) {
                    ta = (L + ta) / P.c;
                    tb = (L + tb) / P.c;
                    has = ta < (float)P.n_bins * P.dt;
                }
            }
            pair_deposit<NB>(pairs, has, p, ta, tb, E, shrow, k, lane, rm, dep);
        }

        // ------------------------------------------------ bounce or terminate
        if (alive) {
            const PairDesc& P = pairs[p];
            if (acc.p < 0) acc.p = p;
            bool term = false;
            if (hit < 0) {
                ++acc.esc;
                h = fnv1a(h, 0xFFFFFFFFu);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc.esc_e[b] += E[b];
                term = true;
            } else {
                L += t_hit;
                ++acc.fin;
                acc.len += (double)t_hit;
                h = fnv1a(h, hit_id);
                const bool win = L >= P.l_window;
                if (win || k == P.max_bounces) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        acc.alive[b] += E[b];
                        if (!win) acc.cap[b] += E[b];
                    }
                    term = true;
                } else {
                    ++k;
                    ox += t_hit * dx;
                    oy += t_hit * dy;
                    oz += t_hit * dz;
                    const float4* tr = sc.tris + 3 * (int64_t)hit;
                    const float4 v0 = tr[0], v1 = tr[1], v2 = tr[2];
                    const float4 e1 = make_float4(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z, v1.w);
                    const float4 e2 = make_float4(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z, 0.0f);
                    float mx = e1.y * e2.z - e1.z * e2.y, my = e1.z * e2.x - e1.x * e2.z,
                          mz = e1.x * e2.y - e1.y * e2.x;
                    const float inl = 1.0f / sqrtf(mx * mx + my * my + mz * mz);
                    mx *= inl;
                    my *= inl;
                    mz *= inl;
                    if (dx * mx + dy * my + dz * mz > 0.f) {
                        mx = -mx;
                        my = -my;
                        mz = -mz;
                    }
                    const float* __restrict__ mr = sc.mats + (int64_t)__float_as_int(e1.w) * kMatStride;
                    ox = fmaf(kSurfaceOffset, mx, ox);
                    oy = fmaf(kSurfaceOffset, my, oy);
                    oz = fmaf(kSurfaceOffset, mz, oz);
                    vx = ox;
                    vy = oy;
                    vz = oz;
                    nx = mx;
                    ny = my;
                    nz = mz;
                    vL = L;
                    vk = k;
                    vexcl = hit;
#pragma unroll
                    for (int b = 0; b < NB; ++b) F[b] = E[b] * mr[kMatKeep + b] * mr[kMatS + b];
                    nee = true;
                    nee_lst = false;
                    const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, (uint32_t)k, 0u), P.key0, P.key1);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc.absb[b] += mr[kMatAlpha + b] * E[b];
                    const int nbr = sc.n_bands;
                    const bool diffuse = u01(x.x) < mr[kMatS + (int)(ray % (uint32_t)nbr)];
                    float q[NB], mean_q = 0.f;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        q[b] = diffuse ? mr[kMatS + b] : 1.f - mr[kMatS + b];
                        mean_q += Q[b] * q[b];
                    }
                    const float inv_mean = (float)nbr / fmaxf(mean_q, 1e-30f);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float r = q[b] * inv_mean;
                        Q[b] *= r;
                        E[b] *= mr[kMatKeep + b] * r;
                    }
                    if (diffuse) {
                        lambert_dir(mx, my, mz, u01(x.y), u01(x.z), dx, dy, dz);
                    } else {
                        const float dn = 2.0f * (dx * mx + dy * my + dz * mz);
                        dx -= dn * mx;
                        dy -= dn * my;
                        dz -= dn * mz;
                        const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                        dx *= il;
                        dy *= il;
                        dz *= il;
                    }
                    vkind = diffuse ? 1u : 0u;
                    spec = !diffuse;
                    last = hit;
                }
            }
            if (term) {
                ++acc.rays;
                if (P.ray_hash) P.ray_hash[rl] = h;
                alive = false;
            }
        }
    }
    lane_acc_flush<NB, false, true>(acc, pairs, lane);
    dep_acc_flush<NB>(dep, pairs, lane);
}

// ---------------------------------------------------------------- setup / finalize
struct LstSetupArgs {
    int s0, ns;
    float src[kSrcChunk][3];
};

__global__ void k_lst_setup(LstSetupArgs a, float4* __restrict__ src, RprIrStats* __restrict__ stats,
                            unsigned long long* __restrict__ queue)
{
    const int i = threadIdx.x;
    if (i == 0 && a.s0 == 0) *queue = 0ull;
    if (i >= a.ns) return;
    const int s = a.s0 + i;
    src[s] = make_float4(a.src[i][0], a.src[i][1], a.src[i][2], 0.f);
    RprIrStats* S = stats + s;
    S->n_segments = S->n_finite_segments = S->n_escaped = S->n_rays = 0;
    S->seg_len_sum = 0.0;
    S->e_emitted = 0.0;
    S->first_arrival_bin = INT_MAX;
    S->first_late_bin = INT_MAX;
    S->n_node_visits = S->n_tri_tests = S->n_next_event = S->n_deposit_rows = 0;
    for (int b = 0; b < RPR_MAX_BANDS; ++b) {
        S->e_class[0][b] = S->e_class[1][b] = S->e_class[2][b] = 0.0;
        S->e_escaped[b] = S->e_alive_at_stop[b] = S->e_alive_at_bounce_cap[b] = S->e_absorbed[b] = 0.0;
    }
}

// Copy the ray-set statistics of stats[0] into the other records.
__global__ void k_lst_finalize(RprIrStats* __restrict__ stats, int n_src)
{
    const int s = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    const RprIrStats& A = stats[0];
    RprIrStats& S = stats[s];
    S.n_segments = A.n_segments;
    S.n_finite_segments = A.n_finite_segments;
    S.n_escaped = A.n_escaped;
    S.n_rays = A.n_rays;
    S.seg_len_sum = A.seg_len_sum;
    S.e_emitted = A.e_emitted;
    S.n_next_event = A.n_next_event;
    S.n_deposit_rows = A.n_deposit_rows;
    for (int b = 0; b < RPR_MAX_BANDS; ++b) {
        S.e_escaped[b] = A.e_escaped[b];
        S.e_alive_at_stop[b] = A.e_alive_at_stop[b];
        S.e_alive_at_bounce_cap[b] = A.e_alive_at_bounce_cap[b];
        S.e_absorbed[b] = A.e_absorbed[b];
    }
}

__global__ void k_lst_fill(float* __restrict__ p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

using LstFn = void (*)(const LstDesc, unsigned long long*);

struct LstVariant {
    LstFn fn;
};

std::mutex g_lmu;
// Stack depths of the variants, 32, 48 and 64 entries: a scene takes the
// smallest that exceeds its stack bound.
inline int lst_stack_bucket(int stack_need) { return stack_need < 32 ? 0 : (stack_need < 48 ? 1 : 2); }
LstVariant g_lvar[2][3];  // [bands 4/8][stack 32/48/64]
bool g_lvar_init = false;
int g_lcus = 0;

int ensure_lst_variants()
{
    std::lock_guard<std::mutex> lk(g_lmu);
    if (g_lvar_init) return RPR_OK;
    int dev = 0;
    RPR_HIP_TRY(hipGetDevice(&dev));
    RPR_HIP_TRY(hipDeviceGetAttribute(&g_lcus, hipDeviceAttributeMultiprocessorCount, dev));
    g_lvar[0][0].fn = k_trace_lst<4, 32>;
    g_lvar[0][1].fn = k_trace_lst<4, 48>;
    g_lvar[0][2].fn = k_trace_lst<4, 64>;
    g_lvar[1][0].fn = k_trace_lst<8, 32>;
    g_lvar[1][1].fn = k_trace_lst<8, 48>;
    g_lvar[1][2].fn = k_trace_lst<8, 64>;
    g_lvar_init = true;
    return RPR_OK;
}

using LstpFn = void (*)(const PairDesc*, int, unsigned long long*);

std::mutex g_pmu;
LstpFn g_pfn[2][3];
int g_pper[2][3];
bool g_p_init = false;

int ensure_lstp_variants()
{
    std::lock_guard<std::mutex> lk(g_pmu);
    if (g_p_init) return RPR_OK;
    g_pfn[0][0] = k_trace_lstp<4, 32>;
    g_pfn[0][1] = k_trace_lstp<4, 48>;
    g_pfn[0][2] = k_trace_lstp<4, 64>;
    g_pfn[1][0] = k_trace_lstp<8, 32>;
    g_pfn[1][1] = k_trace_lstp<8, 48>;
    g_pfn[1][2] = k_trace_lstp<8, 64>;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            int nb = 0;
            RPR_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)g_pfn[a][b], kWave, 0));
            g_pper[a][b] = nb > 0 ? nb : 1;
        }
    g_p_init = true;
    return RPR_OK;
}

}  // namespace

int launch_trace_listener_pairs(const PairDesc* d_chunks, int n_chunks, unsigned long long* d_queue, int64_t total_rays,
                                int nb, int stack_need, int waves_per_cu, hipStream_t stream)
{
    if (total_rays <= 0 || n_chunks <= 0) return RPR_OK;
    int rc = ensure_lstp_variants();
    if (rc != RPR_OK) return rc;
    const int bi = nb <= 4 ? 0 : 1, si = lst_stack_bucket(stack_need);
    const int per_cu = waves_per_cu > 0 ? std::min(waves_per_cu, g_pper[bi][si]) : g_pper[bi][si];
    long long grid = (long long)device_cu_count() * per_cu;
    grid = std::max(1ll, std::min(grid, (long long)n_chunks));
    hipLaunchKernelGGL(g_pfn[bi][si], dim3((unsigned)grid), dim3(kWave), 0, stream, d_chunks, n_chunks, d_queue);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

int trace_listener_max_waves_per_cu(int nb, int stack_need)
{
    if (ensure_lstp_variants() != RPR_OK) return 1;
    return g_pper[nb <= 4 ? 0 : 1][lst_stack_bucket(stack_need)];
}

}  // namespace rpr

using namespace rpr;

extern "C" int trace_listener(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                              const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                              uint32_t* ray_hash, void* hip_stream)
{
    if (!scene || !p || !lst || (n_src > 0 && (!srcs || !hist || !stats)))
        return set_error(RPR_EINVAL, "trace_listener: null argument");
    if (const int rc = scene_settle(scene); rc != RPR_OK) return rc;
    if (n_src < 0 || n_src > kMaxListenerSources)
        return set_error(RPR_EINVAL, "trace_listener: n_src=%d not in 0..%d", n_src, kMaxListenerSources);
    if (p->sh_order < 0 || p->sh_order > RPR_MAX_SH_ORDER)
        return set_error(RPR_EINVAL, "trace_listener: sh_order=%d not in 0..3", p->sh_order);
    if (p->n_bins < 1) return set_error(RPR_EINVAL, "trace_listener: n_bins=%d < 1", p->n_bins);
    if (!(p->bin_width_s > 0.f) || !std::isfinite(p->bin_width_s))
        return set_error(RPR_EINVAL, "trace_listener: bin_width_s must be > 0");
    if (!(p->speed_of_sound > 0.f) || !std::isfinite(p->speed_of_sound))
        return set_error(RPR_EINVAL, "trace_listener: speed_of_sound must be > 0");
    if (p->max_bounces < 0 || p->max_bounces > 10000000)
        return set_error(RPR_EINVAL, "trace_listener: max_bounces=%d not in 0..1e7", p->max_bounces);
    if (p->waves_per_cu < 0) return set_error(RPR_EINVAL, "trace_listener: waves_per_cu < 0");
    if (p->n_rays_total < 1) return set_error(RPR_EINVAL, "trace_listener: n_rays_total < 1");
    if (p->ray_begin < 0 || p->ray_end < p->ray_begin || p->ray_end > ((int64_t)1 << 32))
        return set_error(RPR_EINVAL, "trace_listener: bad ray range [%lld, %lld)", (long long)p->ray_begin,
                         (long long)p->ray_end);
    if (!(lst->radius > 0.f) || !std::isfinite(lst->radius))
        return set_error(RPR_EINVAL, "trace_listener: source radius must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(lst->pos[a])) return set_error(RPR_EINVAL, "trace_listener: non-finite listener position");
    for (int s = 0; s < n_src; ++s)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(srcs[s].pos[a]))
                return set_error(RPR_EINVAL, "trace_listener: non-finite source %d", s);
    if (p->flags != 0) return set_error(RPR_EINVAL, "trace_listener: flags must be 0");
    if (n_src == 0) return RPR_OK;
    int rc = ensure_lst_variants();
    if (rc != RPR_OK) return rc;

    hipStream_t st = (hipStream_t)hip_stream;
    RprScene* sc = const_cast<RprScene*>(scene);
    // queue counter, then the source positions
    const size_t need = 256 + sizeof(float4) * (size_t)n_src;
    rc = workspace_reserve(sc->ws, (need + sizeof(PairDesc) - 1) / sizeof(PairDesc));
    if (rc != RPR_OK) return rc;
    unsigned long long* d_queue = (unsigned long long*)sc->ws.dev;
    float4* d_src = (float4*)((char*)sc->ws.dev + 256);

    const int nb = scene->n_bands;
    const int nc = (p->sh_order + 1) * (p->sh_order + 1);
    const long long R = p->ray_end - p->ray_begin;
    LstDesc d;
    std::memset(&d, 0, sizeof(d));
    d.scene = scene->view;
    for (int a = 0; a < 3; ++a) d.lst[a] = lst->pos[a];
    d.radius = lst->radius;
    d.r2 = lst->radius * lst->radius;
    d.inv_vs = (float)(1.0 / (4.0 / 3.0 * M_PI * (double)lst->radius * lst->radius * lst->radius));
    d.c = p->speed_of_sound;
    d.dt = p->bin_width_s;
    d.l_window = (float)((double)p->speed_of_sound * (double)p->n_bins * (double)p->bin_width_s);
    d.t_window = (float)((double)p->n_bins * (double)p->bin_width_s);
    d.e0 = (float)(1.0 / (double)p->n_rays_total);
    d.n_bins = p->n_bins;
    d.max_bounces = p->max_bounces;
    d.n_coeffs = nc;
    d.n_src = n_src;
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.pair_id = (uint32_t)p->pair_base;
    d.ray_begin = p->ray_begin;
    d.n_rays = R;
    d.src = d_src;
    d.hist = hist;
    d.hist_late = hist_late;
    d.stats = stats;
    d.ray_hash = ray_hash;
    d.hist_stride = (int64_t)p->n_bins * nb * nc;
    d.late_stride = (int64_t)p->n_bins * nb;

    LstSetupArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int s0 = 0; s0 < n_src; s0 += kSrcChunk) {
        a.s0 = s0;
        a.ns = std::min(kSrcChunk, n_src - s0);
        for (int i = 0; i < a.ns; ++i)
            for (int c = 0; c < 3; ++c) a.src[i][c] = srcs[s0 + i].pos[c];
        hipLaunchKernelGGL(k_lst_setup, dim3(1), dim3(kSrcChunk), 0, st, a, d_src, stats, d_queue);
    }
    const size_t nh = (size_t)d.hist_stride * n_src;
    hipLaunchKernelGGL(k_lst_fill, dim3((unsigned)std::min<size_t>((nh + 255) / 256, 16384)), dim3(256), 0, st, hist,
                       nh);
    if (hist_late) {
        const size_t nl = (size_t)d.late_stride * n_src;
        hipLaunchKernelGGL(k_lst_fill, dim3((unsigned)std::min<size_t>((nl + 255) / 256, 16384)), dim3(256), 0, st,
                           hist_late, nl);
    }
    RPR_HIP_TRY(hipGetLastError());
    if (R > 0) {
        const int bi = nb <= 4 ? 0 : 1, si = lst_stack_bucket(scene->stack_need);
        const LstFn fn = g_lvar[bi][si].fn;
        const int NBv = bi == 0 ? 4 : 8;
        const size_t dyn = sizeof(double) * (size_t)n_src * 3 * NBv + sizeof(int) * 2 * (size_t)n_src;
        int per_cu = 0;
        RPR_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kWave, dyn));
        if (per_cu < 1) return set_error(RPR_EUNSUPPORTED, "trace_listener: kernel does not fit (%d sources)", n_src);
        if (p->waves_per_cu > 0) per_cu = std::min(per_cu, p->waves_per_cu);
        long long grid = (long long)g_lcus * per_cu;
        grid = std::max(1ll, std::min(grid, (R + kWave - 1) / kWave));
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kWave), dyn, st, d, d_queue);
        RPR_HIP_TRY(hipGetLastError());
    }
    if (n_src > 1) {
        hipLaunchKernelGGL(k_lst_finalize, dim3((unsigned)((n_src + 254) / 255)), dim3(255), 0, st, stats, n_src);
        RPR_HIP_TRY(hipGetLastError());
    }
    return RPR_OK;
}
