/*
 * oracle.c -- plain FP64 CPU reference of the SDE ensemble method
 * (Januszewski & Kostur, arXiv:0903.3852).  TEST INFRASTRUCTURE ONLY: see
 * oracle.h.  Written from the paper's statements (Eq. 1, Eq. 2, Eq. 3,
 * Alg. 1, Alg. 2) and from the published definitions of Philox4x32-10
 * (Salmon et al., SC'11) and the Box-Muller transform (1958).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, "Parallel random numbers: as easy as 1, 2, 3").     */
/* A round multiplies counter words 0 and 2 by two fixed odd constants to   */
/* 64-bit products, then permutes and mixes the halves with the other two   */
/* words and the round key; the key is advanced by two Weyl increments      */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = (uint32_t)(seed & 0xffffffffu);
    uint32_t k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void oracle_philox_stream(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                          uint64_t c0_first, uint64_t count, uint32_t* out)
{
    for (uint64_t k = 0; k < count; ++k) {
        uint32_t ctr[4] = {(uint32_t)(c0_first + k), a, b, tag};
        oracle_philox(seed, ctr, out + 4 * k);
    }
}

/* Uniforms from the top 24 bits of a Philox word; both are exact in FP64. */
static double u_open0(uint32_t x) { return ((double)(x >> 8) + 1.0) * (1.0 / 16777216.0); } /* (0,1] */
static double u_closed0(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }      /* [0,1) */

/* Box-Muller on two words: g0 = rho cos(2 pi u2), g1 = rho sin(2 pi u2). */
static void box_muller(uint32_t x0, uint32_t x1, double* g0, double* g1)
{
    double u1 = u_open0(x0), u2 = u_closed0(x1);
    double rho = sqrt(-2.0 * log(u1));
    *g0 = rho * cos(2.0 * PI * u2);
    *g1 = rho * sin(2.0 * PI * u2);
}

/* The four Gaussians of block `blk` of stream (tag, a, b). */
static void gauss_block(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b, uint64_t blk,
                        double g[4])
{
    uint32_t ctr[4] = {(uint32_t)blk, a, b, tag};
    uint32_t x[4];
    oracle_philox(seed, ctr, x);
    box_muller(x[0], x[1], &g[0], &g[1]);
    box_muller(x[2], x[3], &g[2], &g[3]);
}

double oracle_gauss(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b, uint64_t n)
{
    double g[4];
    gauss_block(seed, tag, a, b, n >> 2, g);
    return g[n & 3];
}

void oracle_gauss_stream(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                         uint64_t n_first, uint64_t count, double* out)
{
    for (uint64_t k = 0; k < count; ++k) out[k] = oracle_gauss(seed, tag, a, b, n_first + k);
}

/* Cached access to one stream, one Philox block per four consecutive steps. */
typedef struct {
    uint64_t seed, blk;
    uint32_t tag, a, b;
    int valid;
    double g[4];
} gauss_stream;

static void gs_init(gauss_stream* s, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b)
{
    s->seed = seed; s->tag = tag; s->a = a; s->b = b; s->valid = 0; s->blk = 0;
}

static double gs_get(gauss_stream* s, uint64_t n)
{
    if (!s->valid || s->blk != (n >> 2)) {
        gauss_block(s->seed, s->tag, s->a, s->b, n >> 2, s->g);
        s->blk = n >> 2;
        s->valid = 1;
    }
    return s->g[n & 3];
}

/* ------------------------------------------------------------------------ */
/* One step of an additive-noise SDE  dx = f(x, t) dt + s dW  (vector form).  */
/* Heun is Alg. 2 of the paper with the noise increment added in both the   */
/* predictor and the corrector (the "+" before the noise term of the        */
/* corrector is read as intended); the second drift evaluation is taken at  */
/* t + dt.  Euler-Maruyama is the first-order variant used by the paper's    */
/* AdvanceSystem step.  `noise[i]` is the full increment s_i sqrt(dt) psi_i. */
/* ------------------------------------------------------------------------ */
typedef void (*drift_fn)(const void* ctx, double t, const double* x, double* F);

static void sde_step(int scheme, uint32_t dim, drift_fn f, const void* ctx,
                     double t, double t_next, double dt, const double* noise,
                     double* x, double* F1, double* F2, double* xp)
{
    f(ctx, t, x, F1);
    if (scheme == ORC_EULER) {
        for (uint32_t i = 0; i < dim; ++i) x[i] = x[i] + dt * F1[i] + noise[i];
        return;
    }
    for (uint32_t i = 0; i < dim; ++i) xp[i] = x[i] + dt * F1[i] + noise[i];
    f(ctx, t_next, xp, F2);
    for (uint32_t i = 0; i < dim; ++i) x[i] = x[i] + 0.5 * dt * (F1[i] + F2[i]) + noise[i];
}

static int thread_count(int n_threads)
{
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: m x'' + gamma x' = -V'(x) + a cos(w t) + f + sqrt(2 gamma D) xi(t) */
/* with -V'(x) = -sin x (Josephson form, x = phi in radians) or, for the     */
/* paper's V(x) = sin(2 pi x), -V'(x) = -2 pi cos(2 pi x) (x in periods).    */
/* State (x, v); noise acts on v only.                                       */
/* m = 0: gamma x' = -V'(x) + a cos(w t) + f + sqrt(2 gamma D) xi(t).        */
/* ------------------------------------------------------------------------ */
static double jj_potential_force(const oracle_jj_point* P, double x)
{
    return P->potential == ORC_POT_SIN2PI ? -2.0 * PI * cos(2.0 * PI * x) : -sin(x);
}

static void jj_drift(const void* ctx, double t, const double* x, double* F)
{
    const oracle_jj_point* P = (const oracle_jj_point*)ctx;
    double force = jj_potential_force(P, x[0]) + P->a * cos(P->omega * t) + P->f;
    if (P->m > 0.0) {
        F[0] = x[1];
        F[1] = (force - P->gamma * x[1]) / P->m;
    } else {
        F[0] = force / P->gamma;
    }
}

static int jj_point_valid(const oracle_jj_point* P)
{
    if (!(P->m >= 0.0) || !(P->gamma >= 0.0) || !(P->D >= 0.0) || !(P->omega > 0.0)) return 0;
    if (P->m == 0.0 && !(P->gamma > 0.0)) return 0;
    if (!isfinite(P->a) || !isfinite(P->f) || !isfinite(P->m) || !isfinite(P->gamma) ||
        !isfinite(P->D) || !isfinite(P->omega))
        return 0;
    if (P->n_paths == 0 || P->steps_per_period == 0) return 0;
    if (P->potential != ORC_POT_SIN && P->potential != ORC_POT_SIN2PI) return 0;
    return 1;
}

int oracle_jj_integrate(const oracle_jj_point* pts, uint32_t n_pts, const uint32_t* point_ids,
                        uint64_t seed, uint64_t step0, int scheme, int init_from_state,
                        double* phi, double* v, double* acc, double* point_sums,
                        uint32_t n_record, double* rec_phi, double* rec_v,
                        int n_threads)
{
    if (!pts || n_pts == 0 || !phi || !v || !acc) return -1;
    if (scheme != ORC_HEUN && scheme != ORC_EULER) return -1;
    uint64_t total = 0;
    for (uint32_t q = 0; q < n_pts; ++q) {
        if (!jj_point_valid(&pts[q])) return -1;
        total += pts[q].n_paths;
    }
    uint64_t* first = (uint64_t*)malloc(sizeof(uint64_t) * n_pts);
    if (!first) return -1;
    uint64_t off = 0;
    for (uint32_t q = 0; q < n_pts; ++q) { first[q] = off; off += pts[q].n_paths; }

    int nt = thread_count(n_threads);
    for (uint32_t q = 0; q < n_pts; ++q) {
        const oracle_jj_point* P = &pts[q];
        const double dt = 2.0 * PI / (P->omega * (double)P->steps_per_period);
        const int inertial = P->m > 0.0;
        /* noise increment amplitude per step: on v for m > 0, on phi for m = 0 */
        const double s = inertial ? sqrt(2.0 * P->gamma * P->D * dt) / P->m
                                  : sqrt(2.0 * P->D * dt / P->gamma);
        const int64_t np = (int64_t)P->n_paths;
        const uint32_t qid = point_ids ? point_ids[q] : q;
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t p = 0; p < np; ++p) {
            const uint64_t gi = first[q] + (uint64_t)p;
            double x[2], F1[2], F2[2], xp[2], noise[2];
            if (!init_from_state) {
                uint32_t ctr[4] = {0u, (uint32_t)p, qid, ORC_TAG_INIT}, r[4];
                oracle_philox(seed, ctr, r);
                /* one potential period times U: 2 pi (radians) or 1 (periods) */
                const double period = P->potential == ORC_POT_SIN2PI ? 1.0 : 2.0 * PI;
                phi[gi] = period * u_closed0(r[0]);
                v[gi] = -2.0 + 4.0 * u_closed0(r[1]);
                acc[gi] = 0.0;
            }
            x[0] = phi[gi];
            x[1] = v[gi];
            double a_sum = acc[gi];
            gauss_stream gs;
            gs_init(&gs, seed, ORC_TAG_NOISE, (uint32_t)p, qid);
            for (uint64_t k = 0; k < P->n_steps; ++k) {
                const uint64_t n = step0 + k;
                const double psi = gs_get(&gs, n);
                const double t = (double)n * dt, t1 = (double)(n + 1) * dt;
                double vel;
                if (inertial) {
                    noise[0] = 0.0;
                    noise[1] = s * psi;
                    sde_step(scheme, 2, jj_drift, P, t, t1, dt, noise, x, F1, F2, xp);
                    vel = x[1];
                } else {
                    const double before = x[0];
                    noise[0] = s * psi;
                    sde_step(scheme, 1, jj_drift, P, t, t1, dt, noise, x, F1, F2, xp);
                    vel = (x[0] - before) / dt;
                    x[1] = vel;
                }
                if (n >= P->n_transient) a_sum += vel;
                if (rec_phi && k < n_record) rec_phi[k * total + gi] = x[0];
                if (rec_v && k < n_record) rec_v[k * total + gi] = x[1];
            }
            phi[gi] = x[0];
            v[gi] = x[1];
            acc[gi] = a_sum;
        }
        if (point_sums) {
            const uint64_t end = step0 + P->n_steps;
            const double W = end > P->n_transient ? (double)(end - P->n_transient) : 0.0;
            double s1 = 0.0, s2 = 0.0;
            if (W > 0.0) {
                for (int64_t p = 0; p < np; ++p) {
                    double vb = acc[first[q] + (uint64_t)p] / W;
                    s1 += vb;
                    s2 += vb * vb;
                }
            }
            point_sums[2 * q] = s1;
            point_sums[2 * q + 1] = s2;
        }
    }
    free(first);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Ornstein-Uhlenbeck process, through the same step routine.               */
/* ------------------------------------------------------------------------ */
static void ou_drift(const void* ctx, double t, const double* x, double* F)
{
    (void)t;
    F[0] = -(*(const double*)ctx) * x[0];
}

int oracle_ou_integrate(double k, double D, double dt, uint64_t n_steps, int scheme,
                        uint64_t seed, uint32_t n_paths, double* x, int n_threads)
{
    if (!x || !(dt > 0.0) || !(D >= 0.0) || n_paths == 0) return -1;
    if (scheme != ORC_HEUN && scheme != ORC_EULER) return -1;
    const double s = sqrt(2.0 * D * dt);
    int nt = thread_count(n_threads);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t p = 0; p < (int64_t)n_paths; ++p) {
        double y[1] = {x[p]}, F1[1], F2[1], yp[1], noise[1];
        gauss_stream gs;
        gs_init(&gs, seed, ORC_TAG_NOISE, (uint32_t)p, 0);
        for (uint64_t n = 0; n < n_steps; ++n) {
            noise[0] = s * gs_get(&gs, n);
            sde_step(scheme, 1, ou_drift, &k, (double)n * dt, (double)(n + 1) * dt, dt, noise,
                     y, F1, F2, yp);
        }
        x[p] = y[0];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Kuramoto model, Eq. 2 with gamma = 1.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t N;
    double K;
    int coupling;
    const double* omega;
    const double* Kmat;
    int nt;
    double* work; /* [2N] scratch for the Eq. 3 forms of the dense coupling */
} kura_ctx;

/* F_i = omega_i + sum_j K_ij sin(x_j - x_i) */
static void kura_rhs(const kura_ctx* c, const double* x, double* F)
{
    const uint32_t N = c->N;
    const int64_t n = (int64_t)N;
    if (c->coupling == ORC_MEANFIELD) {
        /* Eq. 3: sum_j sin(x_j - x_i) = cos x_i sum_j sin x_j - sin x_i sum_j cos x_j */
        double S = 0.0, C = 0.0;
        for (uint32_t j = 0; j < N; ++j) {
            S += sin(x[j]);
            C += cos(x[j]);
        }
        const double kn = c->K / (double)N;
#pragma omp parallel for num_threads(c->nt) schedule(static)
        for (int64_t i = 0; i < n; ++i)
            F[i] = c->omega[i] + kn * (cos(x[i]) * S - sin(x[i]) * C);
    } else if (c->coupling == ORC_DIRECT) {
        /* the double sum as written in Eq. 2, with K_ij = K / N (or Kmat) */
        const double kn = c->K / (double)N;
#pragma omp parallel for num_threads(c->nt) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double sum = 0.0;
            for (uint32_t j = 0; j < N; ++j) {
                const double kij = c->Kmat ? c->Kmat[(uint64_t)i * N + j] : kn;
                sum += kij * sin(x[j] - x[i]);
            }
            F[i] = c->omega[i] + sum;
        }
    } else {
        /* explicit K_ij, each row through the Eq. 3 identity:
         * sum_j K_ij sin(x_j - x_i) = cos x_i sum_j K_ij sin x_j - sin x_i sum_j K_ij cos x_j */
        double* sx = c->work;
        double* cx = c->work + N;
        for (uint32_t j = 0; j < N; ++j) {
            sx[j] = sin(x[j]);
            cx[j] = cos(x[j]);
        }
#pragma omp parallel for num_threads(c->nt) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double* row = c->Kmat + (uint64_t)i * N;
            double S = 0.0, C = 0.0;
            for (uint32_t j = 0; j < N; ++j) {
                S += row[j] * sx[j];
                C += row[j] * cx[j];
            }
            F[i] = c->omega[i] + cos(x[i]) * S - sin(x[i]) * C;
        }
    }
}

static void kura_drift(const void* ctx, double t, const double* x, double* F)
{
    (void)t;
    kura_rhs((const kura_ctx*)ctx, x, F);
}

void oracle_kuramoto_rhs(uint32_t N, double K, int coupling, const double* phi,
                         const double* omega, const double* Kmat, double* F)
{
    double* work = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    kura_ctx c = {N, K, coupling, omega, Kmat, thread_count(0), work};
    kura_rhs(&c, phi, F);
    free(work);
}

static double order_parameter(uint32_t N, const double* x)
{
    double S = 0.0, C = 0.0;
    for (uint32_t j = 0; j < N; ++j) {
        S += sin(x[j]);
        C += cos(x[j]);
    }
    return sqrt(S * S + C * C) / (double)N;
}

int oracle_kuramoto_integrate(uint32_t N, uint32_t R, double K, double D, double dt,
                              uint64_t n_steps, uint32_t sample_every, int coupling,
                              int scheme, uint64_t seed, uint64_t step0, int init_from_state,
                              double* phi, const double* omega, const double* Kmat,
                              double* r_samples, uint32_t r_first, uint32_t r_count,
                              int n_threads)
{
    if (N == 0 || R == 0 || !(dt > 0.0) || !(D >= 0.0) || !phi || !omega) return -1;
    if (r_count == 0 || r_first + r_count > R) return -1;
    if (scheme != ORC_HEUN && scheme != ORC_EULER) return -1;
    if (coupling == ORC_DENSE && !Kmat) return -1;
    if (coupling == ORC_MEANFIELD && Kmat) return -1;
    if (r_samples && sample_every == 0) return -1;
    const uint64_t n_samples = r_samples ? n_steps / sample_every + 1 : 0;
    const double s = sqrt(2.0 * D * dt);
    double* buf = (double*)malloc(sizeof(double) * 6 * (size_t)N);
    if (!buf) return -1;
    double *F1 = buf, *F2 = buf + N, *xp = buf + 2 * (size_t)N, *noise = buf + 3 * (size_t)N;
    kura_ctx c = {N, K, coupling, omega, Kmat, thread_count(n_threads), buf + 4 * (size_t)N};

    for (uint32_t rr = 0; rr < r_count; ++rr) {
        const uint32_t r = r_first + rr;
        double* x = phi + (uint64_t)rr * N;
        if (!init_from_state) {
            for (uint32_t i = 0; i < N; ++i) {
                uint32_t ctr[4] = {0u, i, r, ORC_TAG_INIT}, w[4];
                oracle_philox(seed, ctr, w);
                x[i] = 2.0 * PI * u_closed0(w[0]);
            }
        }
        for (uint64_t k = 0;; ++k) {
            if (r_samples && k % sample_every == 0)
                r_samples[(uint64_t)rr * n_samples + k / sample_every] = order_parameter(N, x);
            if (k == n_steps) break;
            const uint64_t n = step0 + k;
#pragma omp parallel for num_threads(c.nt) schedule(static)
            for (int64_t i = 0; i < (int64_t)N; ++i)
                noise[i] = s * oracle_gauss(seed, ORC_TAG_NOISE, (uint32_t)i, r, n);
            sde_step(scheme, N, kura_drift, &c, (double)n * dt, (double)(n + 1) * dt, dt, noise,
                     x, F1, F2, xp);
        }
    }
    free(buf);
    return 0;
}
