/*
 * rpr_oracle.c -- plain, slow FP64 CPU oracle for ray-parameterized
 * reverberation propagation (Schissler & Manocha, arXiv 1803.00430).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP path against an independent,
 * obviously-correct implementation.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * What it computes (paper Section 4.2 and Section 5 "Sound Propagation"):
 * stochastic rays leave each source with unit energy per frequency band split
 * over the traced rays, bounce off a triangle scene with per-band absorption
 * and scattering, and are scored at a transparent listener sphere into a
 * low-rate impulse response: per time bin, per band, per real spherical
 * harmonic (SH) coefficient of the arrival direction (Section 4.2, the IR as
 * an intensity histogram I(t) plus SH coefficients X_lm(t)).  Readings of the
 * paper where it is silent are listed at each function.
 *
 * Everything is FP64 and brute force: every segment is tested against every
 * triangle (Moller-Trumbore), SH are evaluated through associated Legendre
 * functions in spherical coordinates, and histogram updates are OpenMP atomics.
 *
 * The random stream is Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * written here from its published definition; the HIP path has its own copy.
 * Counter (ray, pair, reflection order, 0), key (seed low, seed high).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_BANDS 8
#define ORC_FNV_BASIS 2166136261u
#define ORC_FNV_PRIME 16777619u
#define ORC_HASH_ESCAPE 0xFFFFFFFFu
/* Reading (self-intersection; the paper does not discuss it): a reflected
 * segment starts 1 mm off the surface along the normal that faces the
 * incoming ray, and the triangle just hit is excluded from the next query.
 * The offset is a variable only so that a test can trace the limit of a
 * vanishing offset (orc_set_surface_offset); every other caller keeps 1 mm. */
static double orc_surface_offset = 1e-3;

void orc_set_surface_offset(double metres) { orc_surface_offset = metres; }
double orc_get_surface_offset(void) { return orc_surface_offset; }
/* early-reflection path record: [valid, order, tri1, tri2, e[8], t, d[16]] */
#define ORC_REC_W 29
#define ORC_REC_E 4
#define ORC_REC_T 12
#define ORC_REC_D 13

typedef struct {
    int64_t n_rays_total; /* energy normalisation: each ray starts with 1/n_rays_total per band */
    int64_t ray_begin;    /* absolute ray ids [ray_begin, ray_end) are traced for every source */
    int64_t ray_end;
    int32_t max_bounces;  /* K: segments of reflection order 0..K are traced */
    int32_t sh_order;     /* n in 0..3, (n+1)^2 coefficients */
    int32_t n_bins;       /* T */
    int32_t pair_base;    /* RNG counter word 1 = pair_base + source index */
    double bin_width_s;   /* dt */
    double speed_of_sound;
    uint64_t seed;
} OrcTraceParams;

typedef struct {
    int64_t n_segments;        /* closest-hit queries, including the escaping one */
    int64_t n_finite_segments; /* segments that ended on a surface */
    int64_t n_escaped;
    int64_t n_rays;
    double seg_len_sum;        /* sum of finite segment lengths */
    double e_emitted;          /* energy emitted per band = n_rays / n_rays_total */
    int32_t first_arrival_bin; /* INT32_MAX if no deposit */
    int32_t first_late_bin;    /* first bin reached by an order >= 3 segment */
    double e_class[3][ORC_MAX_BANDS]; /* time-integrated intensity: direct / early / late */
    double e_escaped[ORC_MAX_BANDS];
    double e_alive_at_stop[ORC_MAX_BANDS];
    double e_alive_at_bounce_cap[ORC_MAX_BANDS];
    double e_absorbed[ORC_MAX_BANDS];
    int64_t n_next_event;      /* listener-origin trace: next-event (shadow) queries; else 0 */
} OrcIrStats;

/* ------------------------------------------------------------------ RNG */

/* Philox4x32-10: ten rounds of the Philox S-box
 *   (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
 * with the Weyl key schedule k += (W0, W1) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits of a 32-bit word: the odd multiples
 * of 2^-24.  Exactly representable in FP32 and FP64, so both sides start every
 * decision from the same number. */
double orc_uniform(uint32_t x)
{
    return ((double)(x >> 9) * 2.0 + 1.0) * (1.0 / 16777216.0);
}

static void draw(uint64_t seed, uint32_t ray, uint32_t pair, uint32_t order, double u[4])
{
    uint32_t ctr[4] = {ray, pair, order, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform(x[i]);
}

/* ------------------------------------------------------------------ SH */

/* Real orthonormal SH (Section 2, "Spherical Harmonics") of order <= n at the
 * unit direction v, index k = l(l+1)+m.  Reading of the sign convention: the
 * Condon-Shortley phase is included in P_l^m, which is the convention under
 * which the dominant-direction formula of Section 4.1 ("Input
 * Spatialization") returns the arrival direction from the first-order
 * coefficients.  Y_l0 = K_l^0 P_l^0(cos t); Y_lm = sqrt2 K_l^m cos(m p) P_l^m
 * (m > 0); Y_l,-m = sqrt2 K_l^m sin(m p) P_l^m (m > 0), where
 * K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
void orc_sh_eval(int n, const double v[3], double *out)
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double ct = v[2] / r;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double phi = atan2(v[1], v[0]);
    double P[4][4]; /* P[l][m], m <= l */
    memset(P, 0, sizeof(P));
    /* P_m^m = (-1)^m (2m-1)!! sin^m(t);  P_{m+1}^m = (2m+1) cos(t) P_m^m;
     * P_l^m = ((2l-1) cos(t) P_{l-1}^m - (l+m-1) P_{l-2}^m) / (l-m). */
    for (int m = 0; m <= n; ++m) {
        double pmm = 1.0;
        for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * st;
        P[m][m] = pmm;
        if (m + 1 <= n) P[m + 1][m] = (2.0 * m + 1.0) * ct * pmm;
        for (int l = m + 2; l <= n; ++l)
            P[l][m] = ((2.0 * l - 1.0) * ct * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
    }
    for (int l = 0; l <= n; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double fr = 1.0; /* (l-|m|)! / (l+|m|)! */
            for (int i = l - am + 1; i <= l + am; ++i) fr /= (double)i;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fr);
            double y;
            if (m == 0) y = K * P[l][0];
            else if (m > 0) y = sqrt(2.0) * K * cos(m * phi) * P[l][m];
            else y = sqrt(2.0) * K * sin(am * phi) * P[l][am];
            out[l * (l + 1) + m] = y;
        }
    }
}

/* ------------------------------------------------------------------ geometry */

static void sub3(const double a[3], const double b[3], double o[3]) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Moller-Trumbore ray/triangle test; returns t (> 0) or INFINITY. */
static double tri_hit(const double *verts, const int32_t *tri, const double o[3], const double d[3])
{
    const double *v0 = verts + 3 * (int64_t)tri[0];
    const double *v1 = verts + 3 * (int64_t)tri[1];
    const double *v2 = verts + 3 * (int64_t)tri[2];
    double e1[3], e2[3], p[3], s[3], q[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(d, e2, p);
    double det = dot3(e1, p);
    if (det == 0.0) return INFINITY;
    double inv = 1.0 / det;
    sub3(o, v0, s);
    double u = dot3(s, p) * inv;
    if (u < 0.0 || u > 1.0) return INFINITY;
    cross3(s, e1, q);
    double v = dot3(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return INFINITY;
    double t = dot3(e2, q) * inv;
    return t > 0.0 ? t : INFINITY;
}

/* Closest hit over all triangles except `exclude`: smallest t > 0, ties to
 * the lower triangle index.  Returns the triangle index or -1. */
static int64_t closest_hit(const double *verts, const int32_t *tris, int64_t n_tris,
                           const double o[3], const double d[3], int64_t exclude, double *t_out)
{
    double best = INFINITY;
    int64_t best_i = -1;
    for (int64_t i = 0; i < n_tris; ++i) {
        if (i == exclude) continue;
        double t = tri_hit(verts, tris + 3 * i, o, d);
        if (t < best) {
            best = t;
            best_i = i;
        }
    }
    *t_out = best;
    return best_i;
}

void orc_closest_hit_batch(const double *verts, const int32_t *tris, int64_t n_tris,
                           const double *orig, const double *dir, int64_t n_rays,
                           double *t_out, int64_t *tri_out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n_rays; ++r)
        tri_out[r] = closest_hit(verts, tris, n_tris, orig + 3 * r, dir + 3 * r, -1, t_out + r);
}

/* Orthonormal basis (b1, b2, n) for a unit normal n, from Duff et al.,
 * "Building an Orthonormal Basis, Revisited" (JCGT 2017). */
static void onb(const double n[3], double b1[3], double b2[3])
{
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sg * n[0] * n[0] * a; b1[1] = sg * b; b1[2] = -sg * n[0];
    b2[0] = b; b2[1] = sg + n[1] * n[1] * a; b2[2] = -n[1];
}

/* Emission direction, uniform on the sphere (omnidirectional source). */
void orc_emission_dir(const double u[4], double d[3])
{
    double z = 1.0 - 2.0 * u[0];
    double phi = 2.0 * M_PI * u[1];
    double rxy = sqrt(fmax(0.0, 1.0 - z * z));
    d[0] = rxy * cos(phi);
    d[1] = rxy * sin(phi);
    d[2] = z;
}

/* Lambert (cosine-lobe) direction about the unit normal nf. */
void orc_diffuse_dir(const double nf[3], const double u[4], double d[3])
{
    double b1[3], b2[3];
    onb(nf, b1, b2);
    double rr = sqrt(u[2]);
    double lx = rr * cos(2.0 * M_PI * u[1]);
    double ly = rr * sin(2.0 * M_PI * u[1]);
    double lz = sqrt(fmax(0.0, 1.0 - u[2]));
    for (int i = 0; i < 3; ++i) d[i] = lx * b1[i] + ly * b2[i] + lz * nf[i];
}

/* Batch samplers over the ray streams, for the direction-moment checks:
 * out[i] = the emission direction of ray i (counter (i, pair, 0, 0)), or the
 * diffuse direction about nf drawn from counter (i, pair, order, 0). */
void orc_emission_batch(uint64_t seed, uint32_t pair, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        draw(seed, (uint32_t)i, pair, 0u, u);
        orc_emission_dir(u, out + 3 * i);
    }
}

void orc_diffuse_batch(uint64_t seed, uint32_t pair, uint32_t order, const double nf[3], int64_t n,
                       double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        draw(seed, (uint32_t)i, pair, order, u);
        orc_diffuse_dir(nf, u, out + 3 * i);
    }
}

static uint32_t fnv(uint32_t h, uint32_t w) { return (h ^ w) * ORC_FNV_PRIME; }

/* ------------------------------------------------------------------ trace */

static void atomic_min_i32(int32_t *p, int32_t v)
{
#pragma omp critical(orc_min)
    {
        if (v < *p) *p = v;
    }
}

/* Chord of the ray o + t d, 0 <= t <= tmax, through the ball (centre pc,
 * radius r): returns 1 and [*ta, *tb] when it is not empty. */
static int ball_chord(const double o[3], const double d[3], double tmax, const double pc[3], double r,
                      double *ta, double *tb)
{
    double oc[3], w[3];
    sub3(o, pc, oc);
    double bq = dot3(d, oc);
    for (int i = 0; i < 3; ++i) w[i] = oc[i] - bq * d[i];
    double disc = r * r - dot3(w, w);
    if (!(disc > 0.0)) return 0;
    double sq = sqrt(disc);
    *ta = fmax(-bq - sq, 0.0);
    *tb = fmin(-bq + sq, tmax);
    return *tb > *ta;
}

/* Track-length score of the chord [ta, tb] (metres along a segment that
 * starts at path length L) inside a ball of volume vs: the chord, in
 * propagation time, is split exactly over the histogram bins it overlaps;
 * each bin receives E_b * Y_k * (overlap in s) / vs.  Orders 0, 1-2 and >= 3
 * are the direct, early and late classes (Section 5: the first two
 * reflection orders are early, higher orders feed the late IR). */
static void score_chord(double ta, double tb, double L, int order, const double *E, int nb, double vs,
                        const double *Y, const OrcTraceParams *p, double *hist, double *hist_late,
                        OrcIrStats *st)
{
    const double c = p->speed_of_sound, dt = p->bin_width_s;
    const int T = p->n_bins;
    const int nc = (p->sh_order + 1) * (p->sh_order + 1);
    double tau_a = (L + ta) / c, tau_b = (L + tb) / c;
    int cls = order == 0 ? 0 : (order <= 2 ? 1 : 2);
    int64_t m0 = (int64_t)floor(tau_a / dt);
    for (int64_t m = m0; m < T; ++m) {
        double lo = fmax(tau_a, (double)m * dt);
        double hi = fmin(tau_b, (double)(m + 1) * dt);
        if (lo >= tau_b) break;
        double dtau = hi - lo;
        if (!(dtau > 0.0)) continue;
        double wgt = dtau / vs;
        for (int b = 0; b < nb; ++b) {
            double e = E[b] * wgt;
            for (int k = 0; k < nc; ++k) {
#pragma omp atomic
                hist[(m * nb + b) * nc + k] += e * Y[k];
            }
            if (order >= 3 && hist_late) {
#pragma omp atomic
                hist_late[m * nb + b] += e;
            }
#pragma omp atomic
            st->e_class[cls][b] += e;
        }
        if ((int32_t)m < st->first_arrival_bin) atomic_min_i32(&st->first_arrival_bin, (int32_t)m);
        if (order >= 3 && (int32_t)m < st->first_late_bin) atomic_min_i32(&st->first_late_bin, (int32_t)m);
    }
}

/* Score one segment [o, o + t_hit d) at the listener sphere (centre pl,
 * radius r) with the track-length estimator.  The arrival direction is -d
 * (the notation table defines the direction as pointing back toward the
 * source along the path). */
static void deposit(const double o[3], const double d[3], double t_hit, double L, int order,
                    const double *E, int nb, const double pl[3], double r, const OrcTraceParams *p,
                    double *hist, double *hist_late, OrcIrStats *st, double *rec)
{
    double ta, tb;
    if (!ball_chord(o, d, t_hit, pl, r, &ta, &tb)) return;
    double vs = 4.0 / 3.0 * M_PI * r * r * r;
    double md[3] = {-d[0], -d[1], -d[2]};
    double Y[16];
    orc_sh_eval(p->sh_order, md, Y);
    score_chord(ta, tb, L, order, E, nb, vs, Y, p, hist, hist_late, st);
    if (rec) {
        /* early-reflection path record (orders 1-2, Section 5): the intensity the
         * histogram received within the window, the midpoint of the chord's time
         * interval clipped to the window, and the SH directivity e_total Y */
        const double c = p->speed_of_sound, W = (double)p->n_bins * p->bin_width_s;
        double tau_a = (L + ta) / c, tau_b = fmin((L + tb) / c, W);
        if (!(tau_b > tau_a)) return;
        double et = 0.0;
        for (int b = 0; b < nb; ++b) {
            rec[ORC_REC_E + b] = E[b] * (tau_b - tau_a) / vs;
            et += rec[ORC_REC_E + b];
        }
        rec[ORC_REC_T] = 0.5 * (tau_a + tau_b);
        const int nc = (p->sh_order + 1) * (p->sh_order + 1);
        for (int k = 0; k < nc; ++k) rec[ORC_REC_D + k] = et * Y[k];
        rec[0] = 1.0;
    }
}

/* Trace rays [ray_begin, ray_end) of every source.
 *   verts [V][3], tris [T][3], tri_mat [T] (NULL = material 0)
 *   absorption, scattering [M][nb]
 * Reflection (the paper leaves the specular / diffuse mix open): each ray
 * follows one path.  Its hero band h = ray mod nb picks the kind at every
 * bounce, diffuse with probability s_h.  Every band b keeps the path's
 * probability under its own choice rule, Q_b = prod q_b with q_b = s_b
 * (diffuse) or 1 - s_b (specular).  Its energy is weighted by the balance
 * heuristic over the nb rules, Q_b / mean_j Q_j: one-sample multiple
 * importance sampling over the bands (Veach and Guibas 1995, as in hero
 * wavelength spectral sampling, Wilkie et al. 2014).  The estimate is
 * unbiased for every band and the weight stays in [0, nb] times the
 * absorption product; weights s_b / mean_j s_j alone would grow
 * geometrically with the reflection order when the bands' scattering
 * differ.  Q is kept normalised to mean 1.
 *   srcs [n_src][3], listener[4] = centre xyz, radius
 *   hist      [n_src][T][nb][(n+1)^2]  zeroed and filled
 *   hist_late [n_src][T][nb] or NULL    (orders >= 3 only)
 *   stats     [n_src]
 *   ray_hash  [n_src][ray_end-ray_begin] or NULL: FNV-1a over the sequence of
 *     hit triangle ids and bounce kinds, for finding rays whose discrete path
 *     differs between implementations.
 * Returns 0, or -1 on invalid arguments. */
static int trace_core(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                      const int32_t *tri_mat, const double *absorption, const double *scattering,
                      int32_t n_materials, int32_t nb, const double *srcs,
                      int32_t n_src, const double *listener, const OrcTraceParams *p, double *hist,
                      double *hist_late, OrcIrStats *stats, uint32_t *ray_hash, double *records);

int orc_trace_ir(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                 const int32_t *tri_mat, const double *absorption, const double *scattering,
                 int32_t n_materials, int32_t nb, const double *srcs,
                 int32_t n_src, const double *listener, const OrcTraceParams *p, double *hist,
                 double *hist_late, OrcIrStats *stats, uint32_t *ray_hash)
{
    return trace_core(verts, n_verts, tris, n_tris, tri_mat, absorption, scattering, n_materials, nb, srcs, n_src,
                      listener, p, hist, hist_late, stats, ray_hash, NULL);
}

/* orc_trace_ir that also writes the early-reflection path records (Section 5:
 * reflection orders 1 and 2 are the early reflections): records
 * [n_src][ray_end - ray_begin][2][ORC_REC_W], slot o-1 for the deposit of the
 * ray's order-o segment: [0] 1 if the segment deposited (else all zero),
 * [1] order, [2] triangle of the first reflection, [3] of the second (-1 for
 * order 1), [4..4+nb) band intensity, [12] arrival time, [13..13+nc) SH
 * directivity. */
int orc_trace_ir_paths(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                       const int32_t *tri_mat, const double *absorption, const double *scattering,
                       int32_t n_materials, int32_t nb, const double *srcs,
                       int32_t n_src, const double *listener, const OrcTraceParams *p, double *hist,
                       double *hist_late, OrcIrStats *stats, double *records)
{
    if (!records) return -1;
    return trace_core(verts, n_verts, tris, n_tris, tri_mat, absorption, scattering, n_materials, nb, srcs, n_src,
                      listener, p, hist, hist_late, stats, NULL, records);
}

static int trace_core(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                      const int32_t *tri_mat, const double *absorption, const double *scattering,
                      int32_t n_materials, int32_t nb, const double *srcs,
                      int32_t n_src, const double *listener, const OrcTraceParams *p, double *hist,
                      double *hist_late, OrcIrStats *stats, uint32_t *ray_hash, double *records)
{
    if (nb < 1 || nb > ORC_MAX_BANDS || p->sh_order < 0 || p->sh_order > 3 || p->n_bins < 1 ||
        !(p->bin_width_s > 0) || !(listener[3] > 0) || p->ray_end < p->ray_begin ||
        p->n_rays_total < 1 || n_src < 0 || n_materials < 1)
        return -1;
    for (int64_t i = 0; i < 3 * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return -1;
    const int T = p->n_bins;
    const int nc = (p->sh_order + 1) * (p->sh_order + 1);
    const int64_t R = p->ray_end - p->ray_begin;
    memset(hist, 0, sizeof(double) * (size_t)n_src * T * nb * nc);
    if (hist_late) memset(hist_late, 0, sizeof(double) * (size_t)n_src * T * nb);
    if (records) memset(records, 0, sizeof(double) * (size_t)n_src * R * 2 * ORC_REC_W);
    for (int s = 0; s < n_src; ++s) {
        memset(&stats[s], 0, sizeof(OrcIrStats));
        stats[s].first_arrival_bin = INT32_MAX;
        stats[s].first_late_bin = INT32_MAX;
    }
    const double c = p->speed_of_sound;
    const double window = (double)T * p->bin_width_s;
    const double e0 = 1.0 / (double)p->n_rays_total;

#pragma omp parallel for schedule(dynamic, 16) collapse(2)
    for (int s = 0; s < n_src; ++s) {
        for (int64_t ri = 0; ri < R; ++ri) {
            OrcIrStats *st = &stats[s];
            double *H = hist + (size_t)s * T * nb * nc;
            double *HL = hist_late ? hist_late + (size_t)s * T * nb : NULL;
            const uint32_t ray = (uint32_t)(p->ray_begin + ri);
            const uint32_t pair = (uint32_t)(p->pair_base + s);
            double u[4], o[3], d[3], E[ORC_MAX_BANDS], Q[ORC_MAX_BANDS];
            const int hero = (int)(ray % (uint32_t)nb);
            draw(p->seed, ray, pair, 0u, u);
            orc_emission_dir(u, d);
            for (int i = 0; i < 3; ++i) o[i] = srcs[3 * s + i];
            for (int b = 0; b < nb; ++b) {
                E[b] = e0;
                Q[b] = 1.0;
            }
            double L = 0.0;
            int k = 0;
            int64_t last = -1, tri1 = -1, tri2 = -1;
            uint32_t h = ORC_FNV_BASIS;
            int64_t nseg = 0, nfin = 0, nesc = 0;
            double seglen = 0.0, absorbed[ORC_MAX_BANDS] = {0};
            for (;;) {
                double t_hit;
                int64_t tri = closest_hit(verts, tris, n_tris, o, d, last, &t_hit);
                double *rec = NULL;
                if (records && (k == 1 || k == 2)) {
                    rec = records + (((size_t)s * R + ri) * 2 + (k - 1)) * ORC_REC_W;
                    rec[1] = k;
                    rec[2] = (double)tri1;
                    rec[3] = (double)tri2;
                }
                deposit(o, d, t_hit, L, k, E, nb, listener, listener[3], p, H, HL, st, rec);
                if (rec && rec[0] == 0.0) memset(rec, 0, sizeof(double) * ORC_REC_W);
                ++nseg;
                if (tri < 0) {
                    ++nesc;
                    h = fnv(h, ORC_HASH_ESCAPE);
                    for (int b = 0; b < nb; ++b) {
#pragma omp atomic
                        st->e_escaped[b] += E[b];
                    }
                    break;
                }
                L += t_hit;
                ++nfin;
                seglen += t_hit;
                h = fnv(h, (uint32_t)tri);
                if (L / c >= window || k == p->max_bounces) {
                    for (int b = 0; b < nb; ++b) {
#pragma omp atomic
                        st->e_alive_at_stop[b] += E[b];
                        if (k == p->max_bounces && !(L / c >= window)) {
#pragma omp atomic
                            st->e_alive_at_bounce_cap[b] += E[b];
                        }
                    }
                    break;
                }
                ++k;
                if (k == 1) tri1 = tri;
                if (k == 2) tri2 = tri;
                double x[3];
                for (int i = 0; i < 3; ++i) x[i] = o[i] + t_hit * d[i];
                const int32_t *tv = tris + 3 * tri;
                double e1[3], e2[3], nrm[3], nf[3];
                sub3(verts + 3 * (int64_t)tv[1], verts + 3 * (int64_t)tv[0], e1);
                sub3(verts + 3 * (int64_t)tv[2], verts + 3 * (int64_t)tv[0], e2);
                cross3(e1, e2, nrm);
                double nl = sqrt(dot3(nrm, nrm));
                for (int i = 0; i < 3; ++i) nrm[i] /= nl;
                double sgn = dot3(d, nrm) > 0.0 ? -1.0 : 1.0; /* face the incoming ray */
                for (int i = 0; i < 3; ++i) nf[i] = sgn * nrm[i];
                int mat = tri_mat ? tri_mat[tri] : 0;
                const double *al = absorption + (int64_t)mat * nb;
                const double *sc = scattering + (int64_t)mat * nb;
                draw(p->seed, ray, pair, (uint32_t)k, u);
                for (int b = 0; b < nb; ++b) absorbed[b] += al[b] * E[b];
                const int diffuse = u[0] < sc[hero];
                double q[ORC_MAX_BANDS], mean_q = 0.0;
                for (int b = 0; b < nb; ++b) {
                    q[b] = diffuse ? sc[b] : 1.0 - sc[b];
                    mean_q += Q[b] * q[b];
                }
                mean_q /= nb;
                for (int b = 0; b < nb; ++b) {
                    Q[b] *= q[b] / mean_q;
                    E[b] *= (1.0 - al[b]) * q[b] / mean_q;
                }
                if (diffuse) {
                    orc_diffuse_dir(nf, u, d);
                    h = fnv(h, 1u);
                } else {
                    double dn = dot3(d, nf);
                    for (int i = 0; i < 3; ++i) d[i] -= 2.0 * dn * nf[i];
                    h = fnv(h, 0u);
                }
                for (int i = 0; i < 3; ++i) o[i] = x[i] + orc_surface_offset * nf[i];
                last = tri;
            }
#pragma omp atomic
            st->n_segments += nseg;
#pragma omp atomic
            st->n_finite_segments += nfin;
#pragma omp atomic
            st->n_escaped += nesc;
#pragma omp atomic
            st->n_rays += 1;
#pragma omp atomic
            st->seg_len_sum += seglen;
#pragma omp atomic
            st->e_emitted += e0;
            for (int b = 0; b < nb; ++b) {
#pragma omp atomic
                st->e_absorbed[b] += absorbed[b];
            }
            if (ray_hash) ray_hash[(int64_t)s * R + ri] = h;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ listener-origin trace */

/* Direction uniform in the cone of half-angle g about the unit axis a, with
 * cg = cos g: the cosine to the axis is 1 - u0 (1 - cg), uniform in
 * [cg, 1] (equal solid angle per unit cosine), and the azimuth is 2 pi u1 in
 * the Duff et al. basis of a. */
void orc_cone_dir(const double a[3], double cg, double u0, double u1, double d[3])
{
    double b1[3], b2[3];
    onb(a, b1, b2);
    double ct = 1.0 - u0 * (1.0 - cg);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * M_PI * u1;
    for (int i = 0; i < 3; ++i) d[i] = st * cos(ph) * b1[i] + st * sin(ph) * b2[i] + ct * a[i];
}

static void draw_ctr(uint64_t seed, uint32_t ray, uint32_t pair, uint32_t order, uint32_t w3, double u[4])
{
    uint32_t ctr[4] = {ray, pair, order, w3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform(x[i]);
}

typedef struct {
    const double *verts;
    const int32_t *tris;
    int64_t n_tris;
    const double *srcs;
    int n_src;
    double r, vs;
    int nb, nc;
    uint64_t seed;
    uint32_t pair;
    const OrcTraceParams *p;
    double *hist, *hist_late;
    OrcIrStats *stats;
} OrcListenerCtx;

/* Next-event estimation ("diffuse rain", Section 5) from one vertex of a
 * listener path toward every source ball.  At a reflection the vertex is the
 * offset hit point o with facing normal nf, and band b carries
 * f_b = E_b (1 - alpha_b) s_b, the diffuse share of the reflection; at the
 * listener itself (nf == NULL, order 0) f_b = E_b and the lobe is the
 * uniform emission.  For source s a direction w is drawn uniformly in the
 * cone that the ball subtends from o (counter (ray, pair, order, 1 + s));
 * the segment from o along w is scored like any segment with the
 * track-length estimator, with weight f_b times
 *     cos(nf, w) * Omega / pi     (Lambert lobe, density cos / pi), or
 *     Omega / (4 pi)              (uniform emission, density 1 / (4 pi)),
 * Omega = 2 pi (1 - cos g) the cone's solid angle: the expectation is the
 * score of a lobe-sampled segment restricted to the directions that reach
 * the ball.  The segment stops at its first hit (nearest t > 0, the vertex's
 * own triangle excluded): a hit before the chord's entry occludes it, a hit
 * inside it shortens it.  A vertex inside a ball samples the whole lobe
 * instead (weight 1).  The SH row is the path's arrival direction at the
 * listener Y0, or, for the direct sound, that of w itself.  Each query folds
 * its outcome into the ray hash (2 clear, 3 occluded, 4 shortened). */
static void next_event(const OrcListenerCtx *X, uint32_t ray, const double o[3], const double *nf, double L,
                       int order, const double *f, int64_t exclude, const double *Y0, uint32_t *h,
                       int64_t *n_query)
{
    const OrcTraceParams *p = X->p;
    const double window = (double)p->n_bins * p->bin_width_s;
    for (int s = 0; s < X->n_src; ++s) {
        const double *ps = X->srcs + 3 * s;
        double v[4], axis[3], w[3], g;
        draw_ctr(X->seed, ray, X->pair, (uint32_t)order, 1u + (uint32_t)s, v);
        sub3(ps, o, axis);
        double rc = sqrt(dot3(axis, axis));
        if (rc <= X->r) {
            if (nf) orc_diffuse_dir(nf, v, w);
            else orc_emission_dir(v, w);
            g = 1.0;
        } else {
            double a[3] = {axis[0] / rc, axis[1] / rc, axis[2] / rc};
            double cg = sqrt(1.0 - (X->r * X->r) / (rc * rc));
            orc_cone_dir(a, cg, v[0], v[1], w);
            double omega = 2.0 * M_PI * (1.0 - cg);
            if (nf) {
                double cs = dot3(nf, w);
                if (!(cs > 0.0)) continue;
                g = cs * omega / M_PI;
            } else {
                g = omega / (4.0 * M_PI);
            }
        }
        double ta, tb;
        if (!ball_chord(o, w, INFINITY, ps, X->r, &ta, &tb)) continue;
        if ((L + ta) / p->speed_of_sound >= window) continue;
        ++*n_query;
        double t_occ;
        closest_hit(X->verts, X->tris, X->n_tris, o, w, exclude, &t_occ);
        if (t_occ <= ta) {
            *h = fnv(*h, 3u);
            continue;
        }
        if (t_occ < tb) {
            tb = t_occ;
            *h = fnv(*h, 4u);
        } else {
            *h = fnv(*h, 2u);
        }
        double e[ORC_MAX_BANDS], Yw[16];
        for (int b = 0; b < X->nb; ++b) e[b] = f[b] * g;
        const double *Y = Y0;
        if (!Y) {
            orc_sh_eval(p->sh_order, w, Yw);
            Y = Yw;
        }
        score_chord(ta, tb, L, order, e, X->nb, X->vs, Y, p, X->hist + (size_t)s * p->n_bins * X->nb * X->nc,
                    X->hist_late ? X->hist_late + (size_t)s * p->n_bins * X->nb : NULL, &X->stats[s]);
    }
}

/* Listener-origin path tracing with next-event estimation toward every
 * source (Section 5: backward path tracing from the listener, augmented with
 * diffuse rain; one set of rays serves all sources).  Each source is a ball
 * of radius listener[3] around its position; the listener is the point
 * listener[0..2].  Ray i (counter (i, pair_base, k, 0)) leaves the listener
 * uniformly on the sphere in direction w0 with 1/n_rays_total per band, and
 * reflects exactly as in orc_trace_ir (hero-band choice, balance-heuristic
 * band weights, Lambert or mirror direction, 1 mm offset, K and window
 * limits).  Its contributions:
 *   - order 0: next_event() from the listener (the direct sound; the
 *     primary segment itself is not scored);
 *   - at each reflection k (1 <= k <= K, before the window end):
 *     next_event() with the diffuse share f_b = E_b (1 - alpha_b) s_b;
 *   - each segment that follows a specular choice is scored at every source
 *     ball with the track-length estimator (the mirror share, which no
 *     next-event query can reach); a segment after a diffuse choice is not,
 *     since next_event() has already accounted for that reflection's diffuse
 *     share reaching the ball.
 * The histogram of source s then estimates, for a source spread uniformly
 * over its ball, the time-integrated energy density at the listener point
 * with the SH of the arrival direction w0 (the estimator is a forward trace
 * from the listener scored at the ball, so by the reciprocity of the room's
 * propagation it also equals the forward trace from the listener point to a
 * listener sphere at the source).
 *   srcs [n_src][3]; listener[4] = point xyz, source ball radius
 *   hist [n_src][T][nb][(n+1)^2], hist_late [n_src][T][nb] or NULL
 *   stats [n_src]: the path statistics (segments, escapes, energies,
 *     next-event queries) belong to the one ray set and are repeated in
 *     every record; e_class and the first bins are per source
 *   ray_hash [ray_end - ray_begin] or NULL: hit triangles, bounce kinds and
 *     next-event outcomes
 * Returns 0, or -1 on invalid arguments. */
int orc_trace_listener(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                       const int32_t *tri_mat, const double *absorption, const double *scattering,
                       int32_t n_materials, int32_t nb, const double *srcs, int32_t n_src, const double *listener,
                       const OrcTraceParams *p, double *hist, double *hist_late, OrcIrStats *stats,
                       uint32_t *ray_hash)
{
    if (nb < 1 || nb > ORC_MAX_BANDS || p->sh_order < 0 || p->sh_order > 3 || p->n_bins < 1 ||
        !(p->bin_width_s > 0) || !(listener[3] > 0) || p->ray_end < p->ray_begin ||
        p->n_rays_total < 1 || n_src < 0 || n_materials < 1)
        return -1;
    for (int64_t i = 0; i < 3 * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return -1;
    const int T = p->n_bins;
    const int nc = (p->sh_order + 1) * (p->sh_order + 1);
    const int64_t R = p->ray_end - p->ray_begin;
    memset(hist, 0, sizeof(double) * (size_t)n_src * T * nb * nc);
    if (hist_late) memset(hist_late, 0, sizeof(double) * (size_t)n_src * T * nb);
    for (int s = 0; s < n_src; ++s) {
        memset(&stats[s], 0, sizeof(OrcIrStats));
        stats[s].first_arrival_bin = INT32_MAX;
        stats[s].first_late_bin = INT32_MAX;
    }
    if (n_src == 0) return 0;
    const double c = p->speed_of_sound;
    const double window = (double)T * p->bin_width_s;
    const double e0 = 1.0 / (double)p->n_rays_total;
    const double r = listener[3];
    OrcListenerCtx X = {verts, tris, n_tris, srcs, n_src, r, 4.0 / 3.0 * M_PI * r * r * r, nb, nc, p->seed,
                        (uint32_t)p->pair_base, p, hist, hist_late, stats};
    OrcIrStats rs;
    memset(&rs, 0, sizeof(rs));

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ri = 0; ri < R; ++ri) {
        const uint32_t ray = (uint32_t)(p->ray_begin + ri);
        double u[4], o[3], d[3], w0[3], Y0[16], E[ORC_MAX_BANDS], Q[ORC_MAX_BANDS], f[ORC_MAX_BANDS];
        const int hero = (int)(ray % (uint32_t)nb);
        draw(p->seed, ray, X.pair, 0u, u);
        orc_emission_dir(u, w0);
        orc_sh_eval(p->sh_order, w0, Y0);
        for (int i = 0; i < 3; ++i) {
            o[i] = listener[i];
            d[i] = w0[i];
        }
        for (int b = 0; b < nb; ++b) {
            E[b] = e0;
            Q[b] = 1.0;
        }
        double L = 0.0;
        int k = 0, spec = 0;
        int64_t last = -1;
        uint32_t h = ORC_FNV_BASIS;
        int64_t nseg = 0, nfin = 0, nesc = 0, nq = 0;
        double seglen = 0.0, absorbed[ORC_MAX_BANDS] = {0};
        next_event(&X, ray, o, NULL, 0.0, 0, E, -1, NULL, &h, &nq);
        for (;;) {
            double t_hit;
            int64_t tri = closest_hit(verts, tris, n_tris, o, d, last, &t_hit);
            if (spec) {
                for (int s = 0; s < n_src; ++s) {
                    double ta, tb;
                    if (ball_chord(o, d, t_hit, srcs + 3 * s, r, &ta, &tb))
                        score_chord(ta, tb, L, k, E, nb, X.vs, Y0, p, hist + (size_t)s * T * nb * nc,
                                    hist_late ? hist_late + (size_t)s * T * nb : NULL, &stats[s]);
                }
            }
            ++nseg;
            if (tri < 0) {
                ++nesc;
                h = fnv(h, ORC_HASH_ESCAPE);
                for (int b = 0; b < nb; ++b) {
#pragma omp atomic
                    rs.e_escaped[b] += E[b];
                }
                break;
            }
            L += t_hit;
            ++nfin;
            seglen += t_hit;
            h = fnv(h, (uint32_t)tri);
            if (L / c >= window || k == p->max_bounces) {
                for (int b = 0; b < nb; ++b) {
#pragma omp atomic
                    rs.e_alive_at_stop[b] += E[b];
                    if (k == p->max_bounces && !(L / c >= window)) {
#pragma omp atomic
                        rs.e_alive_at_bounce_cap[b] += E[b];
                    }
                }
                break;
            }
            ++k;
            double x[3];
            for (int i = 0; i < 3; ++i) x[i] = o[i] + t_hit * d[i];
            const int32_t *tv = tris + 3 * tri;
            double e1[3], e2[3], nrm[3], nf[3];
            sub3(verts + 3 * (int64_t)tv[1], verts + 3 * (int64_t)tv[0], e1);
            sub3(verts + 3 * (int64_t)tv[2], verts + 3 * (int64_t)tv[0], e2);
            cross3(e1, e2, nrm);
            double nl = sqrt(dot3(nrm, nrm));
            for (int i = 0; i < 3; ++i) nrm[i] /= nl;
            double sgn = dot3(d, nrm) > 0.0 ? -1.0 : 1.0; /* face the incoming ray */
            for (int i = 0; i < 3; ++i) nf[i] = sgn * nrm[i];
            int mat = tri_mat ? tri_mat[tri] : 0;
            const double *al = absorption + (int64_t)mat * nb;
            const double *sc = scattering + (int64_t)mat * nb;
            double xo[3];
            for (int i = 0; i < 3; ++i) xo[i] = x[i] + orc_surface_offset * nf[i];
            for (int b = 0; b < nb; ++b) f[b] = E[b] * (1.0 - al[b]) * sc[b];
            next_event(&X, ray, xo, nf, L, k, f, tri, Y0, &h, &nq);
            draw(p->seed, ray, X.pair, (uint32_t)k, u);
            for (int b = 0; b < nb; ++b) absorbed[b] += al[b] * E[b];
            const int diffuse = u[0] < sc[hero];
            double q[ORC_MAX_BANDS], mean_q = 0.0;
            for (int b = 0; b < nb; ++b) {
                q[b] = diffuse ? sc[b] : 1.0 - sc[b];
                mean_q += Q[b] * q[b];
            }
            mean_q /= nb;
            for (int b = 0; b < nb; ++b) {
                Q[b] *= q[b] / mean_q;
                E[b] *= (1.0 - al[b]) * q[b] / mean_q;
            }
            if (diffuse) {
                orc_diffuse_dir(nf, u, d);
                h = fnv(h, 1u);
            } else {
                double dn = dot3(d, nf);
                for (int i = 0; i < 3; ++i) d[i] -= 2.0 * dn * nf[i];
                h = fnv(h, 0u);
            }
            spec = !diffuse;
            for (int i = 0; i < 3; ++i) o[i] = xo[i];
            last = tri;
        }
#pragma omp atomic
        rs.n_segments += nseg;
#pragma omp atomic
        rs.n_finite_segments += nfin;
#pragma omp atomic
        rs.n_escaped += nesc;
#pragma omp atomic
        rs.n_rays += 1;
#pragma omp atomic
        rs.seg_len_sum += seglen;
#pragma omp atomic
        rs.e_emitted += e0;
#pragma omp atomic
        rs.n_next_event += nq;
        for (int b = 0; b < nb; ++b) {
#pragma omp atomic
            rs.e_absorbed[b] += absorbed[b];
        }
        if (ray_hash) ray_hash[ri] = h;
    }
    for (int s = 0; s < n_src; ++s) {
        OrcIrStats *st = &stats[s];
        st->n_segments = rs.n_segments;
        st->n_finite_segments = rs.n_finite_segments;
        st->n_escaped = rs.n_escaped;
        st->n_rays = rs.n_rays;
        st->seg_len_sum = rs.seg_len_sum;
        st->e_emitted = rs.e_emitted;
        st->n_next_event = rs.n_next_event;
        for (int b = 0; b < ORC_MAX_BANDS; ++b) {
            st->e_escaped[b] = rs.e_escaped[b];
            st->e_alive_at_stop[b] = rs.e_alive_at_stop[b];
            st->e_alive_at_bounce_cap[b] = rs.e_alive_at_bounce_cap[b];
            st->e_absorbed[b] = rs.e_absorbed[b];
        }
    }
    return 0;
}

/* Cone directions for the sampling checks: out[i] = orc_cone_dir of the
 * uniforms of counter (i, pair, order, w3). */
void orc_cone_batch(uint64_t seed, uint32_t pair, uint32_t order, uint32_t w3, const double a[3], double cg,
                    int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        draw_ctr(seed, (uint32_t)i, pair, order, w3, u);
        orc_cone_dir(a, cg, u[0], u[1], out + 3 * i);
    }
}

/* Path of one ray for diagnostics: per segment k (up to max_seg), the
 * segment's origin, direction, hit distance (INFINITY on escape) and hit
 * triangle (-1 on escape).  Returns the number of segments written. */
int orc_trace_path(const double *verts, int64_t n_tris, const int32_t *tris, const int32_t *tri_mat,
                   const double *absorption, const double *scattering, int32_t nb,
                   const double src[3], uint64_t seed, uint32_t ray, uint32_t pair, int32_t max_bounces,
                   double window_len, int32_t max_seg, double *orig, double *dir, double *t_out, int64_t *tri_out)
{
    (void)absorption;
    double u[4], o[3], d[3];
    const int hero = (int)(ray % (uint32_t)nb);
    draw(seed, ray, pair, 0u, u);
    orc_emission_dir(u, d);
    for (int i = 0; i < 3; ++i) o[i] = src[i];
    double L = 0.0;
    int k = 0;
    int64_t last = -1;
    int n = 0;
    while (n < max_seg) {
        double t_hit;
        int64_t tri = closest_hit(verts, tris, n_tris, o, d, last, &t_hit);
        for (int i = 0; i < 3; ++i) {
            orig[3 * n + i] = o[i];
            dir[3 * n + i] = d[i];
        }
        t_out[n] = t_hit;
        tri_out[n] = tri;
        ++n;
        if (tri < 0) break;
        L += t_hit;
        if (L >= window_len || k == max_bounces) break;
        ++k;
        double x[3];
        for (int i = 0; i < 3; ++i) x[i] = o[i] + t_hit * d[i];
        const int32_t *tv = tris + 3 * tri;
        double e1[3], e2[3], nrm[3], nf[3];
        sub3(verts + 3 * (int64_t)tv[1], verts + 3 * (int64_t)tv[0], e1);
        sub3(verts + 3 * (int64_t)tv[2], verts + 3 * (int64_t)tv[0], e2);
        cross3(e1, e2, nrm);
        double nl = sqrt(dot3(nrm, nrm));
        for (int i = 0; i < 3; ++i) nrm[i] /= nl;
        double sgn = dot3(d, nrm) > 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i) nf[i] = sgn * nrm[i];
        int mat = tri_mat ? tri_mat[tri] : 0;
        draw(seed, ray, pair, (uint32_t)k, u);
        if (u[0] < scattering[(int64_t)mat * nb + hero]) {
            orc_diffuse_dir(nf, u, d);
        } else {
            double dn = dot3(d, nf);
            for (int i = 0; i < 3; ++i) d[i] -= 2.0 * dn * nf[i];
        }
        for (int i = 0; i < 3; ++i) o[i] = x[i] + orc_surface_offset * nf[i];
        last = tri;
    }
    return n;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
