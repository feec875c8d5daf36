// Per-pair accumulators shared by the persistent trace kernels: per-lane
// path statistics reduced over the wave by pair, deposited class energies and
// first bins, and the queue-slot to pair lookup.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

namespace rpr {
namespace {

// Per-lane band state of a ray (energy E and choice weight Q per band), in
// registers.
template <int NB>
struct BandState {
    float e[NB], q[NB];
    __device__ float& E(int b) { return e[b]; }
    __device__ float& Q(int b) { return q[b]; }
};

// Per-lane statistics of the rays one lane traced for pair `p`.  Every
// closest-hit query either escapes or ends on a surface, so the segment count
// is fin + esc.
template <int NB>
struct LaneAcc {
    int p;
    uint32_t fin, esc, rays, nodes, tris, nq;
    double len;
    float esc_e[NB], alive[NB], cap[NB], absb[NB];
};

template <int NB>
__device__ __forceinline__ void lane_acc_zero(LaneAcc<NB>& a)
{
    a.p = -1;
    a.fin = a.esc = a.rays = a.nodes = a.tris = a.nq = 0;
    a.len = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) a.esc_e[b] = a.alive[b] = a.cap[b] = a.absb[b] = 0.0f;
}

// Segmented wave reduction of every lane's accumulators by pair, one set of
// global atomics per distinct pair.
template <int NB, bool COUNT, bool NEE = false>
__device__ __forceinline__ void lane_acc_flush(LaneAcc<NB>& a, const PairDesc* __restrict__ pairs, int lane)
{
    uint64_t rem = __ballot(a.p >= 0);
    while (rem) {
        const int l0 = __ffsll((unsigned long long)rem) - 1;
        const int q = __builtin_amdgcn_readfirstlane(__shfl(a.p, l0));
        const bool in = a.p == q;
        const uint64_t m = __ballot(in);
        RprIrStats* S = pairs[q].stats;
        const int nb = pairs[q].scene.n_bands;
        const float e0 = pairs[q].e0;
        const uint32_t fin = wave_sum_u32(in ? a.fin : 0u);
        const uint32_t esc = wave_sum_u32(in ? a.esc : 0u);
        const uint32_t seg = fin + esc;
        const uint32_t rays = wave_sum_u32(in ? a.rays : 0u);
        const double len = wave_sum(in ? a.len : 0.0);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&S->n_segments, (unsigned long long)seg);
            atomicAdd((unsigned long long*)&S->n_finite_segments, (unsigned long long)fin);
            atomicAdd((unsigned long long*)&S->n_escaped, (unsigned long long)esc);
            atomicAdd((unsigned long long*)&S->n_rays, (unsigned long long)rays);
            unsafeAtomicAdd(&S->seg_len_sum, len);
            unsafeAtomicAdd(&S->e_emitted, (double)rays * (double)e0);
        }
        if (NEE) {
            const uint32_t nq = wave_sum_u32(in ? a.nq : 0u);
            if (lane == 0) atomicAdd((unsigned long long*)&S->n_next_event, (unsigned long long)nq);
        }
        if (COUNT) {
            const double nn = wave_sum(in ? (double)a.nodes : 0.0);
            const double nt = wave_sum(in ? (double)a.tris : 0.0);
            if (lane == 0) {
                atomicAdd((unsigned long long*)&S->n_node_visits, (unsigned long long)nn);
                atomicAdd((unsigned long long*)&S->n_tri_tests, (unsigned long long)nt);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nb) break;
            const double ve = wave_sum(in ? (double)a.esc_e[b] : 0.0);
            const double va = wave_sum(in ? (double)a.alive[b] : 0.0);
            const double vc = wave_sum(in ? (double)a.cap[b] : 0.0);
            const double vb = wave_sum(in ? (double)a.absb[b] : 0.0);
            if (lane == 0) {
                unsafeAtomicAdd(&S->e_escaped[b], ve);
                unsafeAtomicAdd(&S->e_alive_at_stop[b], va);
                unsafeAtomicAdd(&S->e_alive_at_bounce_cap[b], vc);
                unsafeAtomicAdd(&S->e_absorbed[b], vb);
            }
        }
        rem &= ~m;
    }
    lane_acc_zero(a);
}

// Deposited class energies of pair `p` (wave-uniform), held by lane
// cls * NB + b, plus the first arrival bins.
struct DepAcc {
    int p;
    double e;
    int fa, fl;
    uint32_t rows;  // bin rows deposited (counted by the listener-origin kernels)
};

template <int NB>
__device__ __forceinline__ void dep_acc_flush(DepAcc& d, const PairDesc* __restrict__ pairs, int lane)
{
    if (d.p >= 0) {
        RprIrStats* S = pairs[d.p].stats;
        const int nb = pairs[d.p].scene.n_bands;
        if (lane < 3 * NB && (lane % NB) < nb && d.e != 0.0) unsafeAtomicAdd(&S->e_class[lane / NB][lane % NB], d.e);
        if (lane == 0) {
            if (d.fa != INT_MAX) atomicMin(&S->first_arrival_bin, d.fa);
            if (d.fl != INT_MAX) atomicMin(&S->first_late_bin, d.fl);
            if (d.rows) atomicAdd((unsigned long long*)&S->n_deposit_rows, (unsigned long long)d.rows);
        }
    }
    d.p = -1;
    d.e = 0.0;
    d.fa = d.fl = INT_MAX;
    d.rows = 0;
}

__device__ __forceinline__ int find_pair(const PairDesc* __restrict__ pairs, int n_pairs, long long r)
{
    int lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pairs[mid].queue_begin <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace
}  // namespace rpr
