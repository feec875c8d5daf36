// Persistent stochastic ray tracing from sources to a listener sphere.
//
// One wave per workgroup.  Each lane owns one ray at a time; lanes whose ray
// has terminated are refilled from a global queue of (pair, ray) slots with
// one atomic per wave (each wave's first 64 slots are fixed by its index), so
// waves stay full while ray lifetimes differ (an
// escape after one segment vs. a hundred bounces).  Closest hits use the
// scene's 4-wide BVH with a per-lane node stack in LDS.  Listener-sphere
// deposits are gathered over the wave and issued as coalesced atomics: for
// each depositing lane, the 64 lanes cover the band x SH-coefficient row of a
// histogram bin (4 bands x 16 coefficients at SH order 3).
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

constexpr int kSetupChunk = 64;

// REC: every deposit of an order-1 or order-2 segment also writes one early-reflection
// path record of kRecWords words (see trace_ir_paths) at rec[slot], slot from *rec_count.
// total_dev: when not null, the number of queue slots is read from it (a
// count that an earlier kernel on the stream computed), else it is `total`.
template <int NB, int STACK, bool COUNT, bool REC>
__global__ void __launch_bounds__(kWave) k_trace(const PairDesc* __restrict__ pairs, int n_pairs,
                                                 unsigned long long* __restrict__ queue, long long total,
                                                 float* __restrict__ rec, unsigned* __restrict__ rec_count,
                                                 int rec_cap, const long long* __restrict__ total_dev,
                                                 const uint32_t* __restrict__ order)
{
    if (total_dev) total = *total_dev;
    __shared__ int32_t stk[STACK * kWave];
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt(lane);

    bool alive = false;
    int p = -1;
    uint32_t ray = 0;
    // The ray's origin, direction and path length are FP64: every hit point,
    // reflection and listener chord is formed from them in FP64, so the path
    // does not drift from the one the definition traces; only the box tests
    // of the traversal round the ray to FP32 (see closest_hit).
    double ox = 0.0, oy = 0.0, oz = 0.0, dx = 0.0, dy = 0.0, dz = 1.0, L = 0.0;
    int k = 0, last = -1;
    uint32_t tri1 = kRecNoTri, tri2 = kRecNoTri;  // triangles of the first two reflections (REC)
    uint32_t h = 0;
    // E(b): band energy; Q(b): the path's probability under band b's choice
    // rule relative to the mean over the bands (see the bounce below).  They
    // live in registers (with four bands the kernel still fits 4 waves per
    // SIMD): in LDS they would take 2 KB per wave, and with 16 waves per CU
    // the stacks and they would fill the CU's LDS, so that the next scene's
    // build kernels could start on a CU only as this launch's waves leave it.
    BandState<NB> eq;
#pragma unroll
    for (int b = 0; b < NB; ++b) eq.E(b) = eq.Q(b) = 0.f;
    LaneAcc<NB> acc;
    lane_acc_zero(acc);
    DepAcc dep{-1, 0.0, INT_MAX, INT_MAX};
    bool exhausted = false;
    // Each wave's first 64 slots are fixed (slot blockIdx.x * 64 + lane); the
    // queue counter hands out the slots after the first gridDim.x * 64, so the
    // launch does not start with every wave's atomic on the same counter.
    const unsigned long long n_static = (unsigned long long)gridDim.x * kWave;
    bool first = true;

    for (;;) {
        // A lane that takes a ray of another pair than the one its statistics
        // hold needs them flushed; they change only at a bounce, so the flush
        // waits until the refill is done (one call site keeps the kernel's
        // register count down).
        bool flush_req = false;
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
                int np = -1;
                long long r = -1;
                if (!alive) {
                    r = (long long)(base + (unsigned long long)__popcll(dead & lt));
                    if (r < total) {
                        if (order) r = (long long)order[r];  // the slot's ray (see k_dir_scatter)
                        np = find_pair(pairs, n_pairs, r);
                    }
                }
                flush_req = np >= 0 && acc.p >= 0 && acc.p != np;
                if (np >= 0) {
                    const PairDesc& P = pairs[np];
                    p = np;
                    ray = (uint32_t)(P.ray_begin + (r - P.queue_begin));
                    const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, 0u, 0u), P.key0, P.key1);
                    sphere_dir_f64((double)u01(x.x), (double)u01(x.y), dx, dy, dz);
                    ox = P.src[0];
                    oy = P.src[1];
                    oz = P.src[2];
                    L = 0.0;
                    k = 0;
                    last = -1;
                    h = 2166136261u;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        eq.E(b) = P.e0;
                        eq.Q(b) = b < P.scene.n_bands ? 1.f : 0.f;
                    }
                    alive = true;
                }
            }
        }
        if (__ballot(flush_req)) lane_acc_flush<NB, COUNT>(acc, pairs, lane);
        if (__ballot(alive) == 0) break;

        // ------------------------------------------------ closest hit
        double t_hit = __builtin_inf();
        uint32_t hit_id = 0xFFFFFFFFu;
        int hit = -1;
        if (alive) {
            const SceneView sc = pairs[p].scene;
            hit = closest_hit<STACK, COUNT>(sc, ox, oy, oz, dx, dy, dz, last, stk, lane, t_hit, hit_id, &acc.nodes,
                                            &acc.tris);
        }

        // ------------------------------------------------ listener sphere
        bool has_dep = false;
        double tau_a = 0.0, tau_b = 0.0;
        if (alive) {
            const PairDesc& P = pairs[p];
            const double r = P.radius, c = P.c;
            const double cx = ox - (double)P.lst[0], cy = oy - (double)P.lst[1], cz = oz - (double)P.lst[2];
            const double bq = dx * cx + dy * cy + dz * cz;
            const double wx = cx - bq * dx, wy = cy - bq * dy, wz = cz - bq * dz;
            const double disc = r * r - (wx * wx + wy * wy + wz * wz);
            if (disc > 0.0) {
                const double sq = sqrt(disc);
                const double ta = fmax(-bq - sq, 0.0);
                const double tb = fmin(-bq + sq, t_hit);
                if (tb > ta) {
                    tau_a = (L + ta) / c;
                    tau_b = (L + tb) / c;
                    has_dep = tau_a < (double)P.n_bins * (double)P.dt;
                }
            }
        }

        // ------------------------------------------------ wave-aggregated deposits
        uint64_t dm = __ballot(has_dep);
        while (dm) {
            const int src = __ffsll((unsigned long long)dm) - 1;
            dm &= dm - 1;
            // the depositing lane's values, as wave-uniform scalars
            const int q = rdlane(p, src);
            const double ta = rdlane(tau_a, src), tb = rdlane(tau_b, src);
            const float ax = -rdlane((float)dx, src), ay = -rdlane((float)dy, src), az = -rdlane((float)dz, src);
            const int kk = rdlane(k, src);
            float Eb[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) Eb[b] = rdlane(eq.E(b), src);
            const PairDesc& P = pairs[q];
            const int T = P.n_bins, nc = P.n_coeffs, nb = P.scene.n_bands;
            const double dt = P.dt;
            const float inv_vs = P.inv_vs;
            float* __restrict__ hist = P.hist;
            float* __restrict__ hlate = P.hist_late;
            const int nbc = nb * nc;
            int m0 = (int)floor(ta / dt);
            m0 = m0 < 0 ? 0 : m0;
            double sum_dtau = 0.0;
            int first_m = INT_MAX;
            for (int base = 0; base < nbc; base += kWave) {
                const int j = base + lane;
                const bool act = j < nbc;
                const int b = act ? j / nc : 0, ci = act ? j % nc : 0;
                float eb = 0.f;
#pragma unroll
                for (int bb = 0; bb < NB; ++bb) eb = (bb == b) ? Eb[bb] : eb;
                const float val = eb * sh_coeff(ci, ax, ay, az) * inv_vs;
                const bool late = act && kk >= 3 && ci == 0 && hlate != nullptr;
                for (int m = m0; m < T; ++m) {
                    const double lo = fmax(ta, (double)m * dt);
                    const double hi = fmin(tb, (double)(m + 1) * dt);
                    if (lo >= tb) break;
                    const double dtau = hi - lo;
                    if (dtau > 0.0) {
                        const float fd = (float)dtau;
                        if (P.hist_fx) {  // fixed point: the sum does not depend on the order of the adds
                            const double fx = P.fx_scale;
                            if (act)
                                atomicAdd((unsigned long long*)(P.hist_fx + ((size_t)m * nb + b) * nc + ci),
                                          (unsigned long long)__double2ll_rn((double)(val * fd) * fx));
                            if (late)
                                atomicAdd((unsigned long long*)(P.late_fx + (size_t)m * nb + b),
                                          (unsigned long long)__double2ll_rn((double)(eb * fd * inv_vs) * fx));
                        } else {
                            if (act) unsafeAtomicAdd(hist + ((size_t)m * nb + b) * nc + ci, val * fd);
                            if (late) unsafeAtomicAdd(hlate + (size_t)m * nb + b, eb * fd * inv_vs);
                        }
                        if (base == 0) {
                            sum_dtau += dtau;
                            first_m = min(first_m, m);
                        }
                    }
                }
            }
            if (q != dep.p) {
                dep_acc_flush<NB>(dep, pairs, lane);
                dep.p = q;
            }
            const int cls = kk == 0 ? 0 : (kk <= 2 ? 1 : 2);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (lane == cls * NB + b) dep.e += (double)(Eb[b] * (float)sum_dtau * inv_vs);
            if (first_m != INT_MAX) {
                dep.fa = min(dep.fa, first_m);
                if (kk >= 3) dep.fl = min(dep.fl, first_m);
            }
            if constexpr (REC) {
                // one record per early deposit: lane w writes word w (a 128-byte store)
                if ((kk == 1 || kk == 2) && sum_dtau > 0.0) {
                    unsigned slot = 0;
                    if (lane == 0) slot = atomicAdd(rec_count, 1u);
                    slot = __shfl(slot, 0);
                    if (slot < (unsigned)rec_cap) {
                        const uint32_t t1 = __shfl(tri1, src), t2 = kk == 2 ? __shfl(tri2, src) : kRecNoTri;
                        const uint64_t key = ((uint64_t)q << 48) | ((uint64_t)kk << 46) |
                                             ((uint64_t)(t1 & kRecNoTri) << 23) | (uint64_t)(t2 & kRecNoTri);
                        float et = 0.f;
#pragma unroll
                        for (int b = 0; b < NB; ++b) et += b < nb ? Eb[b] * (float)sum_dtau * inv_vs : 0.f;
                        float v = 0.f;
                        if (lane == 0) v = __uint_as_float((uint32_t)key);
                        else if (lane == 1) v = __uint_as_float((uint32_t)(key >> 32));
                        else if (lane < 2 + RPR_MAX_BANDS) {
                            const int b = lane - 2;
#pragma unroll
                            for (int bb = 0; bb < NB; ++bb)
                                if (bb == b && bb < nb) v = Eb[bb] * (float)sum_dtau * inv_vs;
                        } else if (lane == 10) {
                            v = (float)(0.5 * (ta + fmin(tb, (double)T * dt)));
                        } else if (lane >= 11 && lane < 11 + RPR_MAX_COEFFS) {
                            const int ci = lane - 11;
                            v = ci < nc ? et * sh_coeff(ci, ax, ay, az) : 0.f;
                        }
                        if (lane < kRecWords) rec[(size_t)slot * kRecWords + lane] = v;
                    }
                }
            }
        }

        // ------------------------------------------------ bounce or terminate
        if (alive) {
            const PairDesc& P = pairs[p];
            const SceneView sc = P.scene;
            if (acc.p < 0) acc.p = p;
            bool term = false;
            if (hit < 0) {
                ++acc.esc;
                h = fnv1a(h, 0xFFFFFFFFu);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc.esc_e[b] += eq.E(b);
                term = true;
            } else {
                L += t_hit;
                ++acc.fin;
                acc.len += t_hit;
                h = fnv1a(h, hit_id);
                const bool win = L / (double)P.c >= (double)P.n_bins * (double)P.dt;
                if (win || k == P.max_bounces) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float e = eq.E(b);
                        acc.alive[b] += e;
                        if (!win) acc.cap[b] += e;
                    }
                    term = true;
                } else {
                    ++k;
                    if constexpr (REC) {
                        if (k == 1) tri1 = hit_id;
                        else if (k == 2) tri2 = hit_id;
                    }
                    const double hx = ox + t_hit * dx, hy = oy + t_hit * dy, hz = oz + t_hit * dz;
                    // unit normal of the exact triangle, turned to face the incoming ray
                    const float4* tr = sc.tris + 3 * (int64_t)hit;
                    const float4 v0 = tr[0], v1 = tr[1], v2 = tr[2];
                    const double e1x = (double)v1.x - v0.x, e1y = (double)v1.y - v0.y, e1z = (double)v1.z - v0.z;
                    const double e2x = (double)v2.x - v0.x, e2y = (double)v2.y - v0.y, e2z = (double)v2.z - v0.z;
                    double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
                    const double inl = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
                    nx *= inl;
                    ny *= inl;
                    nz *= inl;
                    if (dx * nx + dy * ny + dz * nz > 0.0) {
                        nx = -nx;
                        ny = -ny;
                        nz = -nz;
                    }
                    const float* __restrict__ mr = sc.mats + (int64_t)__float_as_int(v1.w) * kMatStride;
                    const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, (uint32_t)k, 0u), P.key0, P.key1);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc.absb[b] += mr[kMatAlpha + b] * eq.E(b);
                    // The ray's hero band (ray id mod bands) picks the kind of
                    // reflection with its own scattering coefficient; each band
                    // is weighted by its rule's path probability over the mean
                    // of all bands' (balance heuristic, one-sample multiple
                    // importance sampling over the bands).  Q is renormalised
                    // to mean 1 at every bounce.
                    const int nbr = sc.n_bands;
                    const bool diffuse = u01(x.x) < mr[kMatS + (int)(ray % (uint32_t)nbr)];
                    float q[NB], mean_q = 0.f;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        q[b] = diffuse ? mr[kMatS + b] : 1.f - mr[kMatS + b];
                        mean_q += eq.Q(b) * q[b];
                    }
                    // mean_q >= Q_hero q_hero / bands > 0 in exact arithmetic; the
                    // floor only guards an FP32 underflow of every term
                    const float inv_mean = (float)nbr / fmaxf(mean_q, 1e-30f);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float r = q[b] * inv_mean;
                        eq.Q(b) *= r;
                        eq.E(b) *= mr[kMatKeep + b] * r;
                    }
                    if (diffuse) {
                        lambert_dir_f64(nx, ny, nz, (double)u01(x.y), (double)u01(x.z), dx, dy, dz);
                        h = fnv1a(h, 1u);
                    } else {
                        const double dn = 2.0 * (dx * nx + dy * ny + dz * nz);
                        dx -= dn * nx;
                        dy -= dn * ny;
                        dz -= dn * nz;
                        h = fnv1a(h, 0u);
                    }
                    // the reflected segment starts just off the surface, on its facing side
                    ox = hx + kSurfaceOffset64 * nx;
                    oy = hy + kSurfaceOffset64 * ny;
                    oz = hz + kSurfaceOffset64 * nz;
                    last = hit;
                }
            }
            if (term) {
                ++acc.rays;
                if (P.ray_hash) P.ray_hash[(int64_t)ray - P.ray_begin] = h;
                alive = false;
            }
        }
    }
    lane_acc_flush<NB, COUNT>(acc, pairs, lane);
    dep_acc_flush<NB>(dep, pairs, lane);
}

__device__ __forceinline__ void stats_init(RprIrStats* S)
{
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

// ---------------------------------------------------------------- setup kernels
struct SetupArgs {
    PairDesc base;
    int s0, ns;
    long long rays_per_src;
    long long hash_stride;  // ray_hash entries per source
    long long hist_stride, late_stride;
    float src[kSetupChunk][3];
    unsigned long long* queue;
};

__device__ __forceinline__ void setup_pair(const SetupArgs& a, PairDesc* __restrict__ out, int i)
{
    if (i == 0 && a.s0 == 0) *a.queue = 0ull;
    if (i >= a.ns) return;
    const int s = a.s0 + i;
    PairDesc d = a.base;
    d.src[0] = a.src[i][0];
    d.src[1] = a.src[i][1];
    d.src[2] = a.src[i][2];
    d.pair_id = a.base.pair_id + (uint32_t)s;
    d.queue_begin = (long long)s * a.rays_per_src;
    d.hist = a.base.hist + (size_t)s * a.hist_stride;
    d.hist_late = a.base.hist_late ? a.base.hist_late + (size_t)s * a.late_stride : nullptr;
    d.stats = a.base.stats + s;
    d.ray_hash = a.base.ray_hash ? a.base.ray_hash + (size_t)s * a.hash_stride : nullptr;
    d.hist_fx = a.base.hist_fx ? a.base.hist_fx + (size_t)s * a.hist_stride : nullptr;
    d.late_fx = a.base.late_fx ? a.base.late_fx + (size_t)s * a.late_stride : nullptr;
    out[s] = d;
    stats_init(d.stats);
}

__global__ void k_setup(SetupArgs a, PairDesc* __restrict__ out) { setup_pair(a, out, threadIdx.x); }

// The last (usually the only) chunk of pair descriptors, in the same launch
// as the clearing of the outputs the trace accumulates into: block 0 writes
// the descriptors, and every block clears its grid-stride share of up to
// three ranges (null when absent).
__global__ void __launch_bounds__(256) k_setup_fill(SetupArgs a, PairDesc* __restrict__ out, float* __restrict__ z0,
                                                    size_t n0, float* __restrict__ z1, size_t n1,
                                                    float* __restrict__ z2, size_t n2, uint32_t* __restrict__ z3,
                                                    size_t n3)
{
    if (blockIdx.x == 0 && threadIdx.x < kSetupChunk) setup_pair(a, out, threadIdx.x);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = i0; i < n0; i += stride) z0[i] = 0.0f;
    if (z1)
        for (size_t i = i0; i < n1; i += stride) z1[i] = 0.0f;
    if (z2)
        for (size_t i = i0; i < n2; i += stride) z2[i] = 0.0f;
    if (z3)
        for (size_t i = i0; i < n3; i += stride) z3[i] = 0u;
}

// Lanes of a wave that trace rays of similar first direction visit the same
// nodes for that segment, and wait less for each other: which queue slot
// traces which ray does not change any ray's path (every random number is
// drawn from the ray id), so the slots of each source are given its rays
// sorted into 64 x 64 cells of the two uniforms that set the first direction
// (height and azimuth on the sphere, an equal-area map), in Morton order of the
// cells.  A counting sort: cell counts, an exclusive scan over each source's
// cells, then each ray takes the next position of its cell.  The order inside
// a cell is that of the atomics.
constexpr int kDirCellBits = 6;
constexpr int kDirCells = 1 << (2 * kDirCellBits);
constexpr int kDirMaxSources = 1024;  // 16 KB of cell counts each

__device__ __forceinline__ uint32_t dir_cell(const PairDesc& P, uint32_t ray)
{
    const uint4 x = philox4x32_10(make_uint4(ray, P.pair_id, 0u, 0u), P.key0, P.key1);
    uint32_t a = x.x >> (32 - kDirCellBits), b = x.y >> (32 - kDirCellBits), c = 0;
#pragma unroll
    for (int k = 0; k < kDirCellBits; ++k) c |= (((a >> k) & 1u) << (2 * k + 1)) | (((b >> k) & 1u) << (2 * k));
    return c;
}

// Blocks of kDirChunk rays of one source (grid: chunks x sources) count in
// LDS first; each block then adds its nonzero cells to the source's counts
// with atomics over consecutive words, a few cache lines per wave.
constexpr int kDirThreads = 256;
constexpr int kDirChunk = 4 * kDirThreads;

__global__ void __launch_bounds__(kDirThreads) k_dir_count(const PairDesc* __restrict__ pairs, long long R,
                                                           uint32_t* __restrict__ counts)
{
    __shared__ uint32_t h[kDirCells];
    const int s = blockIdx.y;
    const PairDesc& P = pairs[s];
    for (int i = threadIdx.x; i < kDirCells; i += kDirThreads) h[i] = 0u;
    __syncthreads();
    const long long j0 = (long long)blockIdx.x * kDirChunk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kDirChunk / kDirThreads; ++k) {
        const long long j = j0 + k * kDirThreads;
        if (j < R) atomicAdd(&h[dir_cell(P, (uint32_t)(P.ray_begin + j))], 1u);
    }
    __syncthreads();
    uint32_t* row = counts + (size_t)s * kDirCells;
    for (int i = threadIdx.x; i < kDirCells; i += kDirThreads)
        if (const uint32_t c = h[i]) atomicAdd(&row[i], c);
}

// Each source's cell counts become the first queue slot of each cell: an
// exclusive scan of its kDirCells counts, from the source's first slot s * R.
// One workgroup per source, four cells per thread.
static_assert(kDirCells == 4 * 1024, "k_dir_scan takes four cells per thread");
__global__ void __launch_bounds__(1024) k_dir_scan(uint32_t* __restrict__ v, long long R)
{
    __shared__ uint32_t wsum[1024 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    uint4* row = reinterpret_cast<uint4*>(v + (size_t)blockIdx.x * kDirCells);
    const uint4 c = row[t];
    const uint32_t own = c.x + c.y + c.z + c.w;
    uint32_t inc = own;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t x = __shfl_up(inc, o);
        if (lane >= o) inc += x;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    uint32_t run = (uint32_t)((long long)blockIdx.x * R) + before + inc - own;
    uint4 o;
    o.x = run;
    run += c.x;
    o.y = run;
    run += c.y;
    o.z = run;
    run += c.z;
    o.w = run;
    row[t] = o;
}

// order[slot] = the queue slot of the ray that slot traces.  Same blocks as
// k_dir_count: ranks inside the block's cells from LDS atomics, then one
// atomic per cell reserves the block's run of that cell's slots.
__global__ void __launch_bounds__(kDirThreads) k_dir_scatter(const PairDesc* __restrict__ pairs, long long R,
                                                             uint32_t* __restrict__ next,
                                                             uint32_t* __restrict__ order)
{
    __shared__ uint32_t h[kDirCells];
    const int s = blockIdx.y;
    const PairDesc& P = pairs[s];
    for (int i = threadIdx.x; i < kDirCells; i += kDirThreads) h[i] = 0u;
    __syncthreads();
    const long long j0 = (long long)blockIdx.x * kDirChunk + threadIdx.x;
    uint32_t cell[kDirChunk / kDirThreads], rank[kDirChunk / kDirThreads];
#pragma unroll
    for (int k = 0; k < kDirChunk / kDirThreads; ++k) {
        const long long j = j0 + k * kDirThreads;
        cell[k] = 0u;
        rank[k] = 0u;
        if (j < R) {
            cell[k] = dir_cell(P, (uint32_t)(P.ray_begin + j));
            rank[k] = atomicAdd(&h[cell[k]], 1u);
        }
    }
    __syncthreads();
    // all of a thread's atomics in flight at once (a cell with no ray adds 0)
    uint32_t* row = next + (size_t)s * kDirCells;
    uint32_t first[kDirCells / kDirThreads];
#pragma unroll
    for (int k = 0; k < kDirCells / kDirThreads; ++k)
        first[k] = atomicAdd(&row[threadIdx.x + k * kDirThreads], h[threadIdx.x + k * kDirThreads]);
#pragma unroll
    for (int k = 0; k < kDirCells / kDirThreads; ++k) h[threadIdx.x + k * kDirThreads] = first[k];
    __syncthreads();
    const long long total = R * (long long)gridDim.y;
#pragma unroll
    for (int k = 0; k < kDirChunk / kDirThreads; ++k) {
        const long long j = j0 + k * kDirThreads;
        if (j < R) {
            const uint32_t pos = h[cell[k]] + rank[k];
            if ((long long)pos < total) order[pos] = (uint32_t)((long long)s * R + j);
        }
    }
}

// Segment budget, second pass: from each source's segment count of the
// first N0 rays, its ray count N' = clamp(N0 + floor((B - S0) N0 / S0), N0,
// max_rays); the pair table is rewritten in place to describe rays [N0, N')
// of every source (queue slots in source order), the queue counter cleared
// and the slot total stored for the second launch.  One thread.
__global__ void k_budget_plan(PairDesc* __restrict__ pairs, int n_src, long long budget, long long n0,
                              long long max_rays, unsigned long long* __restrict__ queue,
                              long long* __restrict__ total_dev)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long run = 0;
    for (int s = 0; s < n_src; ++s) {
        PairDesc& d = pairs[s];
        const long long s0 = (long long)d.stats->n_segments;
        // floor((B - S0) N0 / S0); none when the first pass already reached the budget
        long long dn = (s0 > 0 && budget > s0) ? (budget - s0) * n0 / s0 : 0;
        dn = dn > max_rays - n0 ? max_rays - n0 : dn;
        d.ray_begin = n0;
        d.n_rays = dn;
        d.queue_begin = run;
        if (d.ray_hash) d.ray_hash += n0;
        run += dn;
    }
    *queue = 0ull;
    *total_dev = run;
}

// Segment budget, last step: every ray was emitted with 1/N0 of the energy;
// source s traced N' = N0 + n_rays (pass 2) rays, so its histograms and
// energy statistics are scaled by N0 / N'.  Grid (chunks, sources).
__global__ void k_budget_scale(const PairDesc* __restrict__ pairs, long long n0, long long hist_n, long long late_n,
                               int nb)
{
    const PairDesc& d = pairs[blockIdx.y];
    const double scale = (double)n0 / (double)(n0 + d.n_rays);
    const float fs = (float)scale;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < hist_n; i += stride) d.hist[i] *= fs;
    if (d.hist_late)
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < late_n; i += stride)
            d.hist_late[i] *= fs;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        RprIrStats* S = d.stats;
        S->e_emitted *= scale;
        for (int b = 0; b < nb; ++b) {
            S->e_class[0][b] *= scale;
            S->e_class[1][b] *= scale;
            S->e_class[2][b] *= scale;
            S->e_escaped[b] *= scale;
            S->e_alive_at_stop[b] *= scale;
            S->e_alive_at_bounce_cap[b] *= scale;
            S->e_absorbed[b] *= scale;
        }
    }
}

// Fixed-point histograms to FP32 (RPR_TRACE_DETERMINISTIC): out = fx / scale,
// per_pair cells per pair, the scale of pair j scales[j] (or `scale` for all).
__global__ void k_fx_convert(const long long* __restrict__ fx, float* __restrict__ out, long long per_pair,
                             int n_pairs, const double* __restrict__ scales, double scale)
{
    const long long n = per_pair * n_pairs;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double sc = scales ? scales[i / per_pair] : scale;
        out[i] = (float)((double)fx[i] / sc);
    }
}

__global__ void k_stats_reset(RprIrStats* __restrict__ stats, int n, unsigned long long* __restrict__ queue)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && queue) *queue = 0ull;
    if (i < n) stats_init(stats + i);
}

__global__ void k_fill(float* __restrict__ p, size_t n, float v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void __launch_bounds__(kWave) k_closest(SceneView sc, const float* __restrict__ orig,
                                                   const float* __restrict__ dir, long long n,
                                                   float* __restrict__ t_out, int32_t* __restrict__ tri_out)
{
    __shared__ int32_t stk[kMaxStack * kWave];
    const long long i = (long long)blockIdx.x * kWave + threadIdx.x;
    if (i >= n) return;
    double t;
    uint32_t id;
    const int hit = closest_hit<kMaxStack>(sc, orig[3 * i], orig[3 * i + 1], orig[3 * i + 2], dir[3 * i],
                                           dir[3 * i + 1], dir[3 * i + 2], -1, stk, threadIdx.x, t, id);
    t_out[i] = (float)t;
    tri_out[i] = hit >= 0 ? (int32_t)id : -1;
}

__global__ void k_debug_philox(const uint32_t* __restrict__ in, long long n, uint32_t* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* c = in + 6 * i;
    const uint4 r = philox4x32_10(make_uint4(c[0], c[1], c[2], c[3]), c[4], c[5]);
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

__global__ void k_debug_sh(const float* __restrict__ dirs, long long n, int order, float* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = dirs[3 * i], y = dirs[3 * i + 1], z = dirs[3 * i + 2];
    const int nc = (order + 1) * (order + 1);
    for (int c = 0; c < RPR_MAX_COEFFS; ++c) out[RPR_MAX_COEFFS * i + c] = c < nc ? sh_coeff(c, x, y, z) : 0.0f;
}

// ---------------------------------------------------------------- launch helpers
using TraceFn = void (*)(const PairDesc*, int, unsigned long long*, long long, float*, unsigned*, int,
                         const long long*, const uint32_t*);

template <int NB, int STACK, bool COUNT, bool REC = false>
TraceFn trace_fn()
{
    return k_trace<NB, STACK, COUNT, REC>;
}

struct Variant {
    TraceFn fn;
    int blocks_per_cu;
};

std::mutex g_mu;
// Stack depths of the variants, 32, 48 and 64 entries: a scene takes the
// smallest that exceeds its stack bound (LDS per wave 8 / 12 / 16 KB: 16 / 13 /
// 10 waves per CU).
inline int stack_bucket(int stack_need) { return stack_need < 32 ? 0 : (stack_need < 48 ? 1 : 2); }
Variant g_var[2][3][2];  // [bands 4/8][stack 32/48/64][count visits]
Variant g_rec[2][3];     // [bands 4/8][stack 32/48/64], with early-path records
bool g_var_init = false;
int g_cus = 0;

int ensure_variants()
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_var_init) return RPR_OK;
    int dev = 0;
    RPR_HIP_TRY(hipGetDevice(&dev));
    RPR_HIP_TRY(hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev));
    TraceFn fns[2][3][2] = {{{trace_fn<4, 32, false>(), trace_fn<4, 32, true>()},
                             {trace_fn<4, 48, false>(), trace_fn<4, 48, true>()},
                             {trace_fn<4, 64, false>(), trace_fn<4, 64, true>()}},
                            {{trace_fn<8, 32, false>(), trace_fn<8, 32, true>()},
                             {trace_fn<8, 48, false>(), trace_fn<8, 48, true>()},
                             {trace_fn<8, 64, false>(), trace_fn<8, 64, true>()}}};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 2; ++c) {
                int nb = 0;
                RPR_HIP_TRY(
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fns[a][b][c], kWave, 0));
                g_var[a][b][c] = Variant{fns[a][b][c], nb > 0 ? nb : 1};
            }
    TraceFn rfns[2][3] = {{trace_fn<4, 32, false, true>(), trace_fn<4, 48, false, true>(),
                           trace_fn<4, 64, false, true>()},
                          {trace_fn<8, 32, false, true>(), trace_fn<8, 48, false, true>(),
                           trace_fn<8, 64, false, true>()}};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            int nb = 0;
            RPR_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)rfns[a][b], kWave, 0));
            g_rec[a][b] = Variant{rfns[a][b], nb > 0 ? nb : 1};
        }
    g_var_init = true;
    return RPR_OK;
}

}  // namespace

int device_cu_count()
{
    if (ensure_variants() != RPR_OK) return 0;
    return g_cus;
}

size_t workspace_fx_offset(size_t pairs) { return (256 + sizeof(PairDesc) * (pairs ? pairs : 1) + 255) & ~(size_t)255; }

int workspace_reserve(Workspace& ws, size_t pairs, size_t fx_bytes)
{
    const size_t need = fx_bytes ? workspace_fx_offset(pairs) + fx_bytes : 256 + sizeof(PairDesc) * (pairs ? pairs : 1);
    if (ws.bytes >= need) return RPR_OK;
    if (ws.dev) {
        RPR_HIP_TRY(hipDeviceSynchronize());
        (void)hipFree(ws.dev);
        ws.dev = nullptr;
        ws.bytes = 0;
    }
    const size_t bytes = std::max(need, (size_t)4096);
    RPR_HIP_TRY(hipMalloc(&ws.dev, bytes));
    ws.bytes = bytes;
    return RPR_OK;
}

void workspace_free(Workspace& ws)
{
    if (ws.dev) (void)hipFree(ws.dev);
    if (ws.host_pin) (void)hipHostFree(ws.host_pin);
    ws = Workspace{};
}

int trace_max_waves_per_cu(int nb, int stack_need)
{
    if (ensure_variants() != RPR_OK) return 1;
    return g_var[nb <= 4 ? 0 : 1][stack_bucket(stack_need)][0].blocks_per_cu;
}

int enqueue_fill_zero(float* p, size_t n, hipStream_t stream)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<size_t>((n + 255) / 256, 16384)), dim3(256), 0, stream, p, n,
                       0.0f);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

int enqueue_fx_convert(const long long* fx, float* out, long long per_pair, int n_pairs, const double* scales,
                       double scale, hipStream_t stream)
{
    const long long n = per_pair * n_pairs;
    if (n <= 0) return RPR_OK;
    hipLaunchKernelGGL(k_fx_convert, dim3((unsigned)std::min<long long>((n + 255) / 256, 16384)), dim3(256), 0, stream,
                       fx, out, per_pair, n_pairs, scales, scale);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

int enqueue_stats_reset(RprIrStats* stats, int n, unsigned long long* queue, hipStream_t stream)
{
    hipLaunchKernelGGL(k_stats_reset, dim3((unsigned)((n + 255) / 256 + 1)), dim3(256), 0, stream, stats, n, queue);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

int launch_trace(const PairDesc* d_pairs, int n_pairs, unsigned long long* d_queue, int64_t total_rays, int nb,
                 int stack_need, bool count_visits, int waves_per_cu, int grid_override, hipStream_t stream,
                 float* rec, unsigned* rec_count, int rec_cap, const long long* total_dev, const uint32_t* order)
{
    // with total_dev, total_rays is the most slots the launch may find there (it sizes the grid)
    if (total_rays <= 0 || n_pairs <= 0) return RPR_OK;
    int rc = ensure_variants();
    if (rc != RPR_OK) return rc;
    const Variant& v = rec ? g_rec[nb <= 4 ? 0 : 1][stack_bucket(stack_need)]
                           : g_var[nb <= 4 ? 0 : 1][stack_bucket(stack_need)][count_visits ? 1 : 0];
    const int per_cu = waves_per_cu > 0 ? std::min(waves_per_cu, v.blocks_per_cu) : v.blocks_per_cu;
    long long grid = grid_override > 0 ? grid_override : (long long)g_cus * per_cu;
    const long long need = (total_rays + kWave - 1) / kWave;
    grid = std::max(1ll, std::min(grid, need));
    hipLaunchKernelGGL(v.fn, dim3((unsigned)grid), dim3(kWave), 0, stream, d_pairs, n_pairs, d_queue,
                       (long long)total_rays, rec, rec_count, rec_cap, total_dev, order);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

}  // namespace rpr

using namespace rpr;

namespace {

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

// Scratch of trace_ir_noalloc: the queue counter (first 256 bytes) and the
// pair table, in place of the scene's workspace.  Each GPU the library runs
// on holds its own copy until the process ends.
constexpr int kNoAllocMaxSources = 1024;
constexpr size_t kNoAllocScratchBytes = 256 + (size_t)kNoAllocMaxSources * sizeof(PairDesc);
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.  The array's name is a
// host-side stand-in in host code, so kernels get this address instead; it is
// looked up once per device, with that device current.
int noalloc_scratch(void** out)
{
    int dev = 0;
    RPR_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(RPR_EUNSUPPORTED, "trace_ir_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        RPR_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(RPR_EDEVICE, "trace_ir_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RPR_OK;
}

// ws: device workspace of 256 bytes (queue counter) + n_src pair descriptors,
// or null for the scene's own (grown on demand).
int trace_common(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                 const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats, uint32_t* ray_hash,
                 void* hip_stream, float* rec, unsigned* rec_count, int rec_cap, void* ws = nullptr)
{
    if (!scene || !p || !lst || (n_src > 0 && (!srcs || !hist || !stats)))
        return set_error(RPR_EINVAL, "trace_ir: null argument");
    if (n_src < 0) return set_error(RPR_EINVAL, "trace_ir: n_src=%d < 0", n_src);
    if (const int rc = scene_settle(scene); rc != RPR_OK) return rc;
    if (p->sh_order < 0 || p->sh_order > RPR_MAX_SH_ORDER)
        return set_error(RPR_EINVAL, "trace_ir: sh_order=%d not in 0..3", p->sh_order);
    if (p->n_bins < 1) return set_error(RPR_EINVAL, "trace_ir: n_bins=%d < 1", p->n_bins);
    if (!(p->bin_width_s > 0.f) || !std::isfinite(p->bin_width_s))
        return set_error(RPR_EINVAL, "trace_ir: bin_width_s must be > 0");
    if (!(p->speed_of_sound > 0.f) || !std::isfinite(p->speed_of_sound))
        return set_error(RPR_EINVAL, "trace_ir: speed_of_sound must be > 0");
    if (p->max_bounces < 0) return set_error(RPR_EINVAL, "trace_ir: max_bounces < 0");
    if (p->waves_per_cu < 0) return set_error(RPR_EINVAL, "trace_ir: waves_per_cu < 0");
    if (p->n_rays_total < 1) return set_error(RPR_EINVAL, "trace_ir: n_rays_total < 1");
    const bool budget = p->segment_budget > 0;
    const bool det = (p->flags & RPR_TRACE_DETERMINISTIC) != 0;
    if (det && (rec || ws)) return set_error(RPR_EINVAL, "trace_ir: deterministic accumulation is for trace_ir only");
    if (p->segment_budget < 0) return set_error(RPR_EINVAL, "trace_ir: segment_budget < 0");
    if (budget) {
        if (rec || ws) return set_error(RPR_EINVAL, "trace_ir: a segment budget is taken by trace_ir only");
        if (p->ray_begin != 0 || p->ray_end != p->n_rays_total)
            return set_error(RPR_EINVAL, "trace_ir: with a segment budget, ray_begin = 0 and ray_end = n_rays_total");
        if (p->max_rays < p->ray_end || p->max_rays > ((int64_t)1 << 32))
            return set_error(RPR_EINVAL, "trace_ir: max_rays must be in [ray_end, 2^32]");
        if (p->segment_budget > INT64_MAX / p->max_rays)
            return set_error(RPR_EINVAL, "trace_ir: segment_budget x max_rays overflows 64 bits");
        if (n_src > 65535) return set_error(RPR_EINVAL, "trace_ir: a segment budget takes at most 65535 sources");
    }
    if (p->ray_begin < 0 || p->ray_end < p->ray_begin || p->ray_end > ((int64_t)1 << 32))
        return set_error(RPR_EINVAL, "trace_ir: bad ray range [%lld, %lld)", (long long)p->ray_begin,
                         (long long)p->ray_end);
    if (!(lst->radius > 0.f) || !std::isfinite(lst->radius))
        return set_error(RPR_EINVAL, "trace_ir: listener radius must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(lst->pos[a])) return set_error(RPR_EINVAL, "trace_ir: non-finite listener position");
    for (int s = 0; s < n_src; ++s)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(srcs[s].pos[a])) return set_error(RPR_EINVAL, "trace_ir: non-finite source %d", s);
    if (rec_count) {  // after the argument checks, before anything else
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, (hipStream_t)hip_stream, rec_count);
        RPR_HIP_TRY(hipGetLastError());
    }
    if (n_src == 0) return RPR_OK;
    const double window = (double)p->n_bins * (double)p->bin_width_s;
    if ((double)p->max_bounces > 1e7) return set_error(RPR_EINVAL, "trace_ir: max_bounces too large");
    (void)window;

    hipStream_t st = (hipStream_t)hip_stream;
    const int nb0 = scene->n_bands;
    const int nc0 = (p->sh_order + 1) * (p->sh_order + 1);
    const size_t fx_cells = det ? (size_t)n_src * p->n_bins * nb0 * (nc0 + (hist_late ? 1 : 0)) : 0;
    // slots ordered by first direction (k_dir_*) in the scene's own workspace,
    // for launches of at most 2^26 rays (a 256 MB order): far larger ones
    // refill every lane many times, and the first segments' coherence is a
    // small part of their work
    const long long rays_all = (p->ray_end - p->ray_begin) * (long long)n_src;
    const bool by_dir = !ws && !rec && !budget && n_src <= kDirMaxSources && p->ray_end - p->ray_begin >= kWave &&
                        rays_all <= ((long long)1 << 26);
    const size_t dir_off = (fx_cells * sizeof(long long) + 255) & ~(size_t)255;
    const size_t dir_counts = by_dir ? (size_t)n_src * kDirCells : 0;
    const size_t dir_bytes = by_dir ? sizeof(uint32_t) * (dir_counts + (size_t)rays_all) : 0;
    if (!ws) {
        RprScene* sc = const_cast<RprScene*>(scene);
        const int rc = workspace_reserve(sc->ws, (size_t)n_src, dir_off + dir_bytes);
        if (rc != RPR_OK) return rc;
        ws = sc->ws.dev;
    }
    uint32_t* dir_next = by_dir ? (uint32_t*)((char*)ws + workspace_fx_offset((size_t)n_src) + dir_off) : nullptr;
    uint32_t* dir_order = by_dir ? dir_next + dir_counts : nullptr;
    unsigned long long* d_queue = (unsigned long long*)ws;
    PairDesc* d_pairs = (PairDesc*)((char*)ws + 256);

    const int nb = scene->n_bands;
    const int nc = (p->sh_order + 1) * (p->sh_order + 1);
    const long long R = p->ray_end - p->ray_begin;
    const size_t hist_stride = (size_t)p->n_bins * nb * nc;
    const size_t late_stride = (size_t)p->n_bins * nb;

    SetupArgs a;
    std::memset(&a, 0, sizeof(a));
    PairDesc& d = a.base;
    d.scene = scene->view;
    d.lst[0] = lst->pos[0];
    d.lst[1] = lst->pos[1];
    d.lst[2] = lst->pos[2];
    d.radius = lst->radius;
    d.inv_vs = (float)(1.0 / (4.0 / 3.0 * M_PI * (double)lst->radius * lst->radius * lst->radius));
    d.c = p->speed_of_sound;
    d.dt = p->bin_width_s;
    d.l_window = (float)((double)p->speed_of_sound * (double)p->n_bins * (double)p->bin_width_s);
    d.e0 = (float)(1.0 / (double)p->n_rays_total);
    d.n_bins = p->n_bins;
    d.max_bounces = p->max_bounces;
    d.sh_order = p->sh_order;
    d.n_coeffs = nc;
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.pair_id = (uint32_t)p->pair_base;
    d.flags = p->flags;
    d.ray_begin = p->ray_begin;
    d.n_rays = R;
    d.hist = hist;
    d.hist_late = hist_late;
    d.stats = stats;
    d.ray_hash = ray_hash;
    // fixed point: one cell can reach at most 4 x bands x bin width / sphere volume
    // (a ray weighs at most bands x 1/n_rays_total, |Y| < 1, a chord overlaps a bin by at most its
    // width, and a bin holds at most a few crossings per ray); 2^61 of that fits 64 bits
    const double vs = 4.0 / 3.0 * M_PI * (double)lst->radius * lst->radius * lst->radius;
    const double fx_scale = 0x1p61 * vs / (4.0 * nb * (double)p->bin_width_s);
    if (det) {
        long long* fx = (long long*)((char*)ws + workspace_fx_offset((size_t)n_src));
        d.hist_fx = fx;
        d.late_fx = hist_late ? fx + (size_t)n_src * hist_stride : nullptr;
        d.fx_scale = fx_scale;
    }
    a.rays_per_src = R;
    a.hash_stride = budget ? p->max_rays : R;
    a.hist_stride = (long long)hist_stride;
    a.late_stride = (long long)late_stride;
    a.queue = d_queue;
    // outputs cleared before the trace accumulates into them (the fixed-point
    // cells as zero bits, written as floats)
    const size_t nh = hist_stride * n_src;
    float* fx0 = det ? (float*)((char*)ws + workspace_fx_offset((size_t)n_src)) : nullptr;
    const size_t nf = det ? fx_cells * 2 : 0;
    const size_t nl = hist_late ? late_stride * n_src : 0;
    const size_t fill_blocks = std::min<size_t>(std::max({(nh + 255) / 256, (nf + 255) / 256, (nl + 255) / 256,
                                                          (size_t)1}), 16384);
    for (int s0 = 0; s0 < n_src; s0 += kSetupChunk) {
        a.s0 = s0;
        a.ns = std::min(kSetupChunk, n_src - s0);
        for (int i = 0; i < a.ns; ++i)
            for (int c = 0; c < 3; ++c) a.src[i][c] = srcs[s0 + i].pos[c];
        if (s0 + kSetupChunk < n_src)
            hipLaunchKernelGGL(k_setup, dim3(1), dim3(kSetupChunk), 0, st, a, d_pairs);
        else
            hipLaunchKernelGGL(k_setup_fill, dim3((unsigned)fill_blocks), dim3(256), 0, st, a, d_pairs, hist, nh, fx0,
                               nf, hist_late, nl, dir_next, dir_counts);
    }
    RPR_HIP_TRY(hipGetLastError());
    if (by_dir) {
        const dim3 g((unsigned)((R + kDirChunk - 1) / kDirChunk), (unsigned)n_src);
        hipLaunchKernelGGL(k_dir_count, g, dim3(kDirThreads), 0, st, d_pairs, R, dir_next);
        hipLaunchKernelGGL(k_dir_scan, dim3((unsigned)n_src), dim3(1024), 0, st, dir_next, R);
        hipLaunchKernelGGL(k_dir_scatter, g, dim3(kDirThreads), 0, st, d_pairs, R, dir_next, dir_order);
        RPR_HIP_TRY(hipGetLastError());
    }
    const bool count = (p->flags & RPR_TRACE_COUNT_VISITS) != 0 && !rec;
    // Default width of a direction-ordered launch whose rays about fill the
    // chip's resident lanes (from 3/4 to 5/4 of them): about 4/5 of the rays
    // resident, so that lanes whose rays end early take the rest from the
    // queue instead of idling through the longest rays of their wave.
    int wpc = p->waves_per_cu;
    if (wpc == 0 && by_dir) {
        const long long cus = device_cu_count(), full = trace_max_waves_per_cu(nb, scene->stack_need);
        const long long lanes = cus * full * kWave;
        if (cus > 0 && 4 * rays_all >= 3 * lanes && 4 * rays_all <= 5 * lanes)
            wpc = (int)std::max(1ll, std::min(full, (4 * rays_all + 5 * cus * kWave - 1) / (5 * cus * kWave)));
    }
    int rc = launch_trace(d_pairs, n_src, d_queue, R * n_src, nb, scene->stack_need, count, wpc, 0, st, rec,
                          rec_count, rec_cap, nullptr, dir_order);
    if (rc != RPR_OK) return rc;
    auto convert = [&]() -> int {
        if (!det) return RPR_OK;
        const long long* fx = (const long long*)((char*)ws + workspace_fx_offset((size_t)n_src));
        int rc2 = enqueue_fx_convert(fx, hist, (long long)hist_stride, n_src, nullptr, fx_scale, st);
        if (rc2 == RPR_OK && hist_late)
            rc2 = enqueue_fx_convert(fx + nh, hist_late, (long long)late_stride, n_src, nullptr, fx_scale, st);
        return rc2;
    };
    if (!budget) return convert();
    // segment budget: plan the second pass on the device from the first pass's
    // segment counts, trace it, and rescale every source to 1/N' per ray
    long long* d_total = (long long*)((char*)ws + 64);
    hipLaunchKernelGGL(k_budget_plan, dim3(1), dim3(kWave), 0, st, d_pairs, n_src, (long long)p->segment_budget,
                       (long long)R, (long long)p->max_rays, d_queue, d_total);
    RPR_HIP_TRY(hipGetLastError());
    rc = launch_trace(d_pairs, n_src, d_queue, (p->max_rays - R) * n_src, nb, scene->stack_need, count,
                      p->waves_per_cu, 0, st, nullptr, nullptr, 0, d_total);
    if (rc != RPR_OK) return rc;
    rc = convert();
    if (rc != RPR_OK) return rc;
    hipLaunchKernelGGL(k_budget_scale, dim3(64, (unsigned)n_src), dim3(256), 0, st, d_pairs, (long long)R,
                       (long long)hist_stride, hist_late ? (long long)late_stride : 0ll, nb);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

}  // namespace

extern "C" int trace_ir(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                        const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                        uint32_t* ray_hash, void* hip_stream)
{
    return trace_common(scene, srcs, n_src, lst, p, hist, hist_late, stats, ray_hash, hip_stream, nullptr, nullptr,
                        0);
}

extern "C" int trace_ir_noalloc(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                                const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                                uint32_t* ray_hash, void* hip_stream)
{
    if (n_src > kNoAllocMaxSources)
        return set_error(RPR_EINVAL, "trace_ir_noalloc: n_src=%d exceeds the static scratch's %d sources", n_src,
                         kNoAllocMaxSources);
    void* ws = nullptr;
    if (n_src > 0) {
        const int rc = noalloc_scratch(&ws);
        if (rc != RPR_OK) return rc;
    }
    return trace_common(scene, srcs, n_src, lst, p, hist, hist_late, stats, ray_hash, hip_stream, nullptr, nullptr, 0,
                        ws);
}

extern "C" int trace_ir_paths(const RprScene* scene, const RprSource* srcs, int32_t n_src, const RprListener* lst,
                              const RprTraceParams* p, float* hist, float* hist_late, RprIrStats* stats,
                              float* records, uint32_t* n_records, int32_t max_records, void* hip_stream)
{
    if (!records || !n_records || max_records < 1) return set_error(RPR_EINVAL, "trace_ir_paths: bad record buffer");
    if (n_src > 0xFFFF) return set_error(RPR_EUNSUPPORTED, "trace_ir_paths: more than 65535 sources");
    if (scene && scene->n_tris >= (int64_t)kRecNoTri)
        return set_error(RPR_EUNSUPPORTED, "trace_ir_paths: more than %u triangles", kRecNoTri - 1);
    if (p && (p->flags & RPR_TRACE_COUNT_VISITS)) return set_error(RPR_EINVAL, "trace_ir_paths: no visit counting");
    return trace_common(scene, srcs, n_src, lst, p, hist, hist_late, stats, nullptr, hip_stream, records,
                        n_records, max_records);
}

extern "C" int scene_closest_hit(const RprScene* scene, const float* orig, const float* dir, int64_t n,
                                 float* t_out, int32_t* tri_out, void* hip_stream)
{
    if (!scene || n < 0 || (n > 0 && (!orig || !dir || !t_out || !tri_out)))
        return set_error(RPR_EINVAL, "scene_closest_hit: bad argument");
    if (const int rc = scene_settle(scene); rc != RPR_OK) return rc;
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_closest, dim3((unsigned)((n + kWave - 1) / kWave)), dim3(kWave), 0,
                       (hipStream_t)hip_stream, scene->view, orig, dir, (long long)n, t_out, tri_out);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int debug_philox(const uint32_t* in, int64_t n, uint32_t* out, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!in || !out))) return set_error(RPR_EINVAL, "debug_philox: bad argument");
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, in,
                       (long long)n, out);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}

extern "C" int debug_sh_eval(const float* dirs, int64_t n, int32_t order, float* out, void* hip_stream)
{
    if (n < 0 || order < 0 || order > RPR_MAX_SH_ORDER || (n > 0 && (!dirs || !out)))
        return set_error(RPR_EINVAL, "debug_sh_eval: bad argument");
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_debug_sh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, dirs,
                       (long long)n, order, out);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
