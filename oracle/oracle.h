/*
 * oracle.h -- slow, plain FP64 CPU reference for the SDE ensemble method of
 * Januszewski & Kostur, "Accelerating numerical solution of Stochastic
 * Differential Equations with CUDA" (arXiv:0903.3852).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant table with
 * the HIP library: Philox, Box-Muller, the drifts and the Heun/Euler steps
 * are written out again here from their published definitions.
 *
 * Every routine is double precision, written for readability: loops in the
 * order the paper states them, no blocking, no fusion.  OpenMP only spreads
 * independent paths / oscillators over threads; results do not depend on the
 * thread count.
 *
 * Conventions shared with the library only through the written method
 * statement (not through code):
 *   - RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 *     (seed mod 2^32, seed >> 32), counter = (n >> 2, a, b, tag);
 *   - uniforms: u1 = ((x >> 8) + 1) * 2^-24 in (0,1], u2 = (x >> 8) * 2^-24;
 *   - Gaussians: Box-Muller (Box & Muller 1958) on (x0,x1) -> (g0,g1) and
 *     (x2,x3) -> (g2,g3); step n uses component n & 3.
 *
 * Parity status of each function is listed with it.
 */
#ifndef SDE_ORACLE_H
#define SDE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox counter word 3 ("tag") separates the independent random streams. */
enum {
    ORC_TAG_NOISE = 0,  /* per-step noise of a path / oscillator            */
    ORC_TAG_INIT = 1    /* initial conditions                               */
};

enum { ORC_HEUN = 0, ORC_EULER = 1 };
enum { ORC_MEANFIELD = 0, ORC_DIRECT = 1, ORC_DENSE = 2 };

/* ---- random numbers ---------------------------------------------------- */

/* Philox4x32-10 block: out = Philox10(key(seed), ctr).  Pinned against the
 * rocRAND library implementation and a pure-Python big-integer version. */
void oracle_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]);

/* Gaussian number n of stream (tag, a, b): component n & 3 of the Box-Muller
 * pair outputs of Philox(ctr = (n >> 2, a, b, tag)).  Pinned by moments and a
 * Kolmogorov-Smirnov test against the normal CDF. */
double oracle_gauss(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b, uint64_t n);

/* Fill out[k] for k = 0..count-1 with Philox blocks at counters
 * (c0_first + k, a, b, tag) -- bulk dump for tests. */
void oracle_philox_stream(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                          uint64_t c0_first, uint64_t count, uint32_t* out /* [count][4] */);

/* out[k] = oracle_gauss(seed, tag, a, b, n_first + k) for k < count. */
void oracle_gauss_stream(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                         uint64_t n_first, uint64_t count, double* out);

/* ---- Josephson junction / Brownian particle in a tilted washboard (Eq. 1) -
 * Two potentials:
 *   ORC_POT_SIN    m phi'' + gamma phi' = -sin phi + a cos wt + f + noise
 *                  (the Josephson-junction form; coordinate phi in radians)
 *   ORC_POT_SIN2PI m x'' + gamma x' = -V'(x) + a cos wt + f + noise with the
 *                  paper's V(x) = sin(2 pi x) (Sec. 3; x in potential periods)
 * noise = sqrt(2 gamma D) xi(t) in both. */
enum { ORC_POT_SIN = 0, ORC_POT_SIN2PI = 1 };

typedef struct {
    double m, gamma, a, omega, f, D;   /* m = 0 selects the overdamped limit */
    uint32_t n_paths, steps_per_period; /* dt = 2 pi / (omega * steps_per_period) */
    uint64_t n_steps, n_transient;      /* n_transient is an absolute step index */
    int32_t potential;                  /* ORC_POT_* */
    int32_t reserved;
} oracle_jj_point;

/*
 * Integrates every path of every point from absolute step step0 for
 * pts[q].n_steps steps with stochastic Heun (Alg. 2 applied to (phi, v)) or
 * Euler-Maruyama.  Paths of all points are laid out one after another.
 *
 *   phi, v, acc : [total paths] in/out.  phi is the point's coordinate,
 *                 NOT wrapped: radians (ORC_POT_SIN) or periods
 *                 (ORC_POT_SIN2PI); v its time derivative.  If
 *                 init_from_state is 0 they are overwritten with the
 *                 Philox INIT draw: one period times U(x0) (phi = 2 pi U or
 *                 x = U), v = -2 + 4 U(x1), acc = 0.
 *   point_sums  : [n_pts][2] out: sum_p vbar_p and sum_p vbar_p^2 where
 *                 vbar_p = acc_p / W and W = number of window steps
 *                 (absolute step n with n >= n_transient) up to step0+n_steps.
 *   rec_phi/v   : optional [n_record][total paths]: state after each of the
 *                 first n_record steps.
 *   point_ids   : optional [n_pts]: the point index b that enters the Philox
 *                 counters of point q (default q), so that a subset of a
 *                 larger batch draws the same random numbers as in the batch.
 * Returns 0, or -1 on invalid arguments.
 * Parity: pinned, for both potentials, by the equilibrium (Boltzmann)
 * moments with and without inertia (the overdamped limit at gamma != 1, so
 * the drift's and the noise's powers of gamma both matter), the relaxation
 * variance of the overdamped limit from the bottom of a well, the
 * overdamped washboard velocity and the deterministic order-2 convergence.
 */
int oracle_jj_integrate(const oracle_jj_point* pts, uint32_t n_pts, const uint32_t* point_ids,
                        uint64_t seed, uint64_t step0, int scheme, int init_from_state,
                        double* phi, double* v, double* acc, double* point_sums,
                        uint32_t n_record, double* rec_phi, double* rec_v,
                        int n_threads);

/* ---- Ornstein-Uhlenbeck: dx = -k x dt + sqrt(2 D) dW ---------------------
 * The same Heun / Euler step routine as every other model, with the linear
 * drift; noise stream (NOISE, p, 0).  x[p] in/out.  Used to pin the step
 * itself against the exact stationary variance of the discrete scheme. */
int oracle_ou_integrate(double k, double D, double dt, uint64_t n_steps, int scheme,
                        uint64_t seed, uint32_t n_paths, double* x, int n_threads);

/* ---- Kuramoto (Eq. 2 with gamma = 1, K_ij = K/N or an explicit matrix) ----
 *
 *   dphi_i = [omega_i + sum_j K_ij sin(phi_j - phi_i)] dt + sqrt(2 D) dW_i
 *
 * Realizations r_first .. r_first + r_count - 1 of R are integrated (they
 * differ in initial phases and noise; omega and K are shared).
 *   phi      : [r_count][N] radians in/out (not wrapped).  init_from_state 0
 *              draws phi = 2 pi U(Philox(0, i, r, INIT).x0).
 *   omega    : [N]
 *   Kmat     : [N][N] row-major K_ij for ORC_DENSE, else NULL (K_ij = K/N).
 *   coupling : ORC_MEANFIELD (Eq. 3 sums, uniform K only),
 *              ORC_DIRECT (the double sum over sin(phi_j - phi_i)),
 *              ORC_DENSE (explicit K_ij, evaluated through the Eq. 3 identity
 *              row by row).
 *   r_samples: [r_count][n_steps / sample_every + 1] (may be NULL): the order
 *              parameter |N^-1 sum_j exp(i phi_j)| at local steps
 *              0, sample_every, 2 sample_every, ...
 * Noise of oscillator i in realization r at absolute step n:
 * G(seed, NOISE, i, r, n).  Returns 0 or -1.
 * Parity: pinned by free-diffusion variance, the identical-oscillator
 * threshold, Adler's law for N = 2 and the Eq. 3 identity.
 */
int oracle_kuramoto_integrate(uint32_t N, uint32_t R, double K, double D, double dt,
                              uint64_t n_steps, uint32_t sample_every, int coupling,
                              int scheme, uint64_t seed, uint64_t step0, int init_from_state,
                              double* phi, const double* omega, const double* Kmat,
                              double* r_samples, uint32_t r_first, uint32_t r_count,
                              int n_threads);

/* Right-hand side F_i = omega_i + sum_j K_ij sin(phi_j - phi_i) of one
 * realization, by the chosen coupling form (for identity checks). */
void oracle_kuramoto_rhs(uint32_t N, double K, int coupling, const double* phi,
                         const double* omega, const double* Kmat, double* F);

#ifdef __cplusplus
}
#endif

#endif
