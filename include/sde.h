/*
 * sde.h -- C ABI of libsde: ensemble integration of stochastic differential
 * equations on one AMD Instinct MI355X (gfx950), after Januszewski & Kostur,
 * "Accelerating numerical solution of Stochastic Differential Equations with
 * CUDA" (arXiv:0903.3852).
 *
 * Two models of the paper are integrated:
 *   - the noisy driven Josephson junction / Stewart-McCumber equation
 *     (Eq. 1), here with the potential force -sin(phi):
 *        m phi'' + gamma phi' = -sin phi + a cos(omega t) + f + sqrt(2 gamma D) xi(t),
 *     many independent paths of many parameter points (Sec. 4.1, Alg. 1);
 *   - the noisy Kuramoto model of N globally coupled phase oscillators
 *     (Eq. 2 with gamma = 1 and D = k_B T):
 *        phi_i' = omega_i + sum_j K_ij sin(phi_j - phi_i) + sqrt(2 D) xi_i(t),
 *     with the coupling sum evaluated every step by the mean-field identity
 *     (Eq. 3), the LDS-tiled all-pairs sum (Alg. 3 / Fig. 3) or, for a dense
 *     heterogeneous K_ij, a per-step matrix product.
 * The stepper is the stochastic second-order Runge-Kutta (Heun) scheme of
 * Alg. 2, or Euler-Maruyama.  Noise comes from a counter-based Philox4x32-10
 * generator keyed by (seed, path, step) with Box-Muller Gaussians, so a run
 * can be resumed at any step with the same noise.  A Josephson-junction run
 * split into calls at a step that is a multiple of 4 and of M
 * (sample_every) reproduces the single call bit for bit; at other steps
 * the phase is re-wrapped and the window sum folded at the call boundary,
 * so the two agree to rounding.
 *
 * Conventions for every call:
 *   - Buffers marked [device] are raw HIP device pointers owned by the
 *     caller; the library never frees or retains them past the call.
 *     Descriptors and [host] buffers are host memory read during the call.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the null
 *     stream).  Calls return once the work is enqueued, except where stated.
 *   - Arguments are validated before anything is launched; on an error the
 *     output buffers are untouched and the call returns a negative status.
 *     sde_last_error() then describes the failure.
 *   - A context is used by one host thread at a time.
 *   - No C++ exception crosses this interface.
 */
#ifndef SDE_H
#define SDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
    SDE_OK = 0,
    SDE_ERR_INVALID = -1,     /* bad argument (null, zero size, non-finite, misaligned) */
    SDE_ERR_NOMEM = -2,       /* device workspace allocation failed                    */
    SDE_ERR_DEVICE = -3,      /* a HIP runtime call failed                             */
    SDE_ERR_UNSUPPORTED = -4, /* valid but not implemented (e.g. wrong GPU)            */
    SDE_ERR_NUMERIC = -5      /* the state became NaN or Inf                           */
};

/* stepper */
enum { SDE_HEUN = 0, SDE_EULER = 1 };
/* initial state */
enum { SDE_INIT_PHILOX = 0, SDE_INIT_FROM_STATE = 1 };
/* Kuramoto coupling evaluation */
enum {
    SDE_MEANFIELD = 0,   /* Eq. 3: two sums per realization and stage, K_ij = K/N      */
    SDE_TILED = 1,       /* Alg. 3: all N^2 sin terms, LDS tiles, K_ij = K/N           */
    SDE_DENSE_FP32 = 2,  /* explicit K_ij: FP32 product K [sin | cos]                  */
    SDE_DENSE_BF16X3 = 3,/* explicit K_ij: bf16 hi/lo split, 3 MFMA products, FP32 acc */
    SDE_DENSE_FP16X3 = 4 /* explicit K_ij: fp16 hi/lo split, 3 MFMA products, FP32 acc */
};
/* Philox counter word 3 of each random stream */
enum { SDE_TAG_NOISE = 0, SDE_TAG_INIT = 1 };
/* potential of a Josephson-junction / washboard point (Eq. 1) */
enum {
    SDE_POTENTIAL_SIN = 0,    /* force -sin(phi), coordinate phi in radians: the        */
                              /* Josephson-junction (Stewart-McCumber) form             */
    SDE_POTENTIAL_SIN2PI = 1  /* the paper's V(x) = sin(2 pi x) (Sec. 3): force         */
                              /* -2 pi cos(2 pi x), coordinate x in potential periods   */
};

typedef struct sde_ctx sde_ctx;

/* Creates a context on HIP device `hip_device` (makes it current).  Returns
 * SDE_ERR_UNSUPPORTED if the device is not gfx950, SDE_ERR_DEVICE if it
 * cannot be opened. */
int sde_create(int hip_device, sde_ctx** out);
/* Frees the context's workspace (after synchronizing its device). */
void sde_destroy(sde_ctx* ctx);
/* Static text for a status code. */
const char* sde_strerror(int status);
/* Text describing the last failing call on `ctx` ("" if none). */
const char* sde_last_error(const sde_ctx* ctx);
/* Synchronizes the context's device and reports SDE_ERR_NUMERIC if any
 * integration since the last check produced a NaN/Inf state, SDE_ERR_DEVICE
 * if a bounded wait inside a kernel (between the workgroups of a mean-field
 * realization, or the waves of a two-half dense workgroup) timed out. */
int sde_check(sde_ctx* ctx);

/* ---- run options shared by both models ----------------------------------- */
typedef struct {
    uint64_t seed;          /* Philox key: (seed mod 2^32, seed >> 32)                 */
    uint64_t step0;         /* absolute index of the first step (resume at any step)   */
    int32_t scheme;         /* SDE_HEUN | SDE_EULER                                    */
    int32_t init;           /* SDE_INIT_PHILOX | SDE_INIT_FROM_STATE                   */
    uint32_t sample_every;  /* M: FP32 partial sums are folded into FP64 every M       */
                            /* absolute steps (JJ); order-parameter sampling interval  */
                            /* (Kuramoto).  0 selects the paper's M = 100 (Sec. 4.1).  */
    int32_t sync;           /* nonzero: synchronize the stream before returning and    */
                            /* return SDE_ERR_NUMERIC if the state became NaN/Inf      */
} sde_run;

/* ---- Josephson junction (Eq. 1, Alg. 1, Alg. 2) -------------------------- */
typedef struct {
    double m, gamma, a, omega, f, D; /* Eq. 1: m x'' + gamma x' = -V'(x) + a cos wt  */
                                     /* + f + sqrt(2 gamma D) xi(t); m = 0 selects   */
                                     /* the overdamped limit gamma x' = ...          */
    uint32_t n_paths;                /* independent paths of this point              */
    uint32_t steps_per_period;       /* S: dt = 2 pi / (omega S); the drive phase    */
                                     /* is kept as the step index mod S (Sec. 5)     */
    uint64_t n_steps;                /* steps of this call                           */
    uint64_t n_transient;            /* absolute step index where averaging begins   */
    int32_t potential;               /* SDE_POTENTIAL_* (0, a zeroed struct: -sin)   */
    int32_t reserved;                /* must be 0                                    */
} sde_jj_point;

/*
 * Integrates every path of every point for pts[q].n_steps Heun (or Euler)
 * steps starting at absolute step run->step0, one persistent launch over
 * all (point, path-chunk) work items.
 *
 * Path p of point q (0 <= p < pts[q].n_paths) lives at index
 * off(q) + p of the per-path arrays, off(q) = sum of n_paths of points < q.
 * The coordinate is kept in units of the potential's period L (2 pi for
 * phi, 1 for x) as theta + winding:
 *   theta   [device] float,   per path, fraction of a period in [0, 1):
 *                             phi = 2 pi (theta + winding), x = theta + winding
 *   winding [device] int32,   per path, whole periods
 *   v       [device] float,   per path, velocity phi' or x' (m = 0: the
 *                             step's mean velocity (change over the step)/dt)
 *   acc     [device] double,  per path, sum of v after each window step
 *                             (absolute step n >= n_transient)
 * Each may be NULL (state not kept) unless run->init is
 * SDE_INIT_FROM_STATE, which reads all four.  With SDE_INIT_PHILOX the
 * initial state is theta = U(x0), v = -2 + 4 U(x1) from
 * Philox(ctr = (0, p, q, SDE_TAG_INIT)), winding = 0, acc = 0.
 *   point_sums [device] double [n_pts][2] or NULL: (sum_p vbar_p,
 *                             sum_p vbar_p^2) with vbar_p = acc_p / W,
 *                             W = number of window steps before
 *                             step0 + n_steps.
 * n_transient is an absolute step index, so a call that ends before it
 * (n_transient >= step0 + n_steps: a transient integrated in pieces, whose
 * state the next call resumes) is valid: its window is empty, W = 0, acc
 * is unchanged and the point sums are 0.  It is not an error.
 * The noise of path p of point q at absolute step n is component n & 3 of
 * the Box-Muller Gaussians of Philox(ctr = (n >> 2, p, q, SDE_TAG_NOISE)).
 * Points of different potentials and of m > 0 / m = 0 mix freely in one
 * call (one persistent launch per kind present).
 * Errors: SDE_ERR_INVALID for n_pts = 0, n_paths = 0, steps_per_period = 0,
 * omega <= 0, gamma < 0 (or 0 with m = 0), m < 0, D < 0, non-finite
 * parameters, an unknown potential, reserved != 0, misaligned pointers,
 * FROM_STATE with a NULL state array.
 */
int sde_jj_integrate(sde_ctx* ctx, const sde_jj_point* pts /* [host] */, uint32_t n_pts,
                     const sde_run* run, float* theta, int32_t* winding, float* v, double* acc,
                     double* point_sums, void* hip_stream);

/*
 * For callers that cannot allocate memory during a call (code that must not
 * call hipMalloc, tight serving loops, harnesses that forbid allocation):
 * sde_jj_integrate with the same arguments, results and errors, that
 * allocates nothing.  Its work-queue words, point table, work items, drive
 * tables and per-chunk partial sums live in a static device array of the
 * library (8 MiB, held by every GPU the library runs on until the process
 * ends), whose address sde_create looks up once per device; the host image
 * of the tables goes through a pinned buffer that sde_create reserves
 * (8 MiB per context).  No graphs are recorded and nothing is tuned: the
 * paths per lane are the forced option, else a choice the autotuner of
 * sde_jj_integrate cached for this shape class, else 2 (the result does not
 * depend on it).  Host-side planning uses ordinary heap memory.
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (the queue words are cleared by each call): calls that
 * overlap on one GPU -- from several contexts, or on streams not ordered
 * after each other -- race.  Calls on one context wait, before writing the
 * pinned buffer, for the previous call's copy out of it.
 * Errors: those of sde_jj_integrate, and SDE_ERR_INVALID when the call needs
 * more than 8 MiB of scratch: 96 B per point, 24 B per chunk of 64 x (paths
 * per lane) paths of a point, 4 B per drive-table entry (S + 8 per distinct
 * steps_per_period), each table rounded up to 256 B.  The 16384-point,
 * 1024-path scan needs 4.5 MiB at 2 paths per lane, 7.5 MiB at 1.
 */
int sde_jj_integrate_noalloc(sde_ctx* ctx, const sde_jj_point* pts /* [host] */, uint32_t n_pts,
                             const sde_run* run, float* theta, int32_t* winding, float* v, double* acc,
                             double* point_sums, void* hip_stream);

/*
 * sde_jj_integrate in double precision throughout (the paper's precision
 * study, Sec. 5 and Fig. 2): the same points, run options, noise streams and
 * layout, with theta and v as device double arrays and every operation of
 * the step (drift, noise, Box-Muller) in FP64.  The drive table, the
 * winding bookkeeping and the reductions are the same as in FP32.
 * Errors: as sde_jj_integrate.
 */
int sde_jj_integrate_f64(sde_ctx* ctx, const sde_jj_point* pts /* [host] */, uint32_t n_pts,
                         const sde_run* run, double* theta, int32_t* winding, double* v, double* acc,
                         double* point_sums, void* hip_stream);

/*
 * sde_jj_integrate that also streams the coarse-grained positions of every
 * path while it integrates: the ensemble's density over time in Fig. 2
 * (left panel, positions averaged over a potential period) and Sec. 5,
 * where the paper wrote every particle position to a file.  With T the
 * total number of paths of the call (row pitch) and r = 0, 1, ...:
 *   rec_winding[r * T + path_first(q) + p] = winding of path p of point q
 *   after absolute step (floor(step0 / record_every) + r + 1) * record_every,
 * for every multiple of record_every in (step0, step0 + n_steps(q)];
 * rows past a point's last step keep their contents.  The trajectory is the
 * one sde_jj_integrate computes (bit for bit).
 * record_every: a positive multiple of 4 (one noise block).  n_rows: rows
 * the caller's buffer holds; each point needs
 *   floor((step0 + n_steps) / record_every) - floor(step0 / record_every).
 * rec_winding: [device] int32 [n_rows][T], caller-owned, 4-byte aligned.
 * Errors: as sde_jj_integrate, plus SDE_ERR_INVALID for a NULL or
 * misaligned rec_winding, record_every not a positive multiple of 4, or a
 * point that needs more than n_rows rows (nothing is written).
 */
int sde_jj_integrate_recorded(sde_ctx* ctx, const sde_jj_point* pts /* [host] */, uint32_t n_pts,
                              const sde_run* run, float* theta, int32_t* winding, float* v, double* acc,
                              double* point_sums, uint32_t record_every, uint64_t n_rows,
                              int32_t* rec_winding /* [device] */, void* hip_stream);

/* ---- Kuramoto (Eq. 2, Eq. 3, Alg. 3) ------------------------------------- */
typedef struct {
    uint32_t N;            /* oscillators per realization                         */
    uint32_t R;            /* independent realizations (own phases and noise)     */
    double K;              /* uniform coupling K_ij = K / N (MEANFIELD, TILED)    */
    double D;              /* noise intensity: sqrt(2 D) xi_i                     */
    double dt;             /* step                                                */
    uint64_t n_steps;      /* steps of this call                                  */
    int32_t coupling;      /* SDE_MEANFIELD | SDE_TILED | SDE_DENSE_*             */
    int32_t reserved;      /* must be 0                                           */
} sde_kuramoto_desc;

/*
 * Integrates R realizations of N oscillators for n_steps steps.
 *   phi      [device] float [R][N], in/out: phases in revolutions
 *            (phi_i / 2 pi), kept wrapped to [0, 1).  Read only when
 *            run->init is SDE_INIT_FROM_STATE; otherwise phase i of
 *            realization r starts at U(Philox(ctr = (0, i, r, SDE_TAG_INIT)).x0).
 *   omega    [device] float [N], natural frequencies (shared by realizations)
 *   K        [device] float [N][N] row-major K_ij for SDE_DENSE_*, NULL
 *            otherwise.  The dense variants scale K by an exact power of two
 *            internally so that its largest entry lies in [1, 2).
 *   r_samples[device] double [R][n_steps / M + 1] or NULL: order parameter
 *            r = |N^-1 sum_j exp(2 pi i phi_j)| at local steps 0, M, 2M, ...
 *            (M = run->sample_every, default 100).
 * The noise of oscillator i of realization r at absolute step n is component
 * n & 3 of the Box-Muller Gaussians of Philox(ctr = (n >> 2, i, r, NOISE)).
 * Errors: SDE_ERR_INVALID for N or R = 0, dt <= 0, D < 0, non-finite K, D or
 * dt, DENSE without K or MEANFIELD/TILED with K, misaligned pointers.
 */
int sde_kuramoto_integrate(sde_ctx* ctx, const sde_kuramoto_desc* desc, const sde_run* run,
                           float* phi, const float* omega, const float* K, double* r_samples,
                           void* hip_stream);

/* ---- ensemble observables ------------------------------------------------ */
enum {
    SDE_OBS_MEAN_F32 = 0,  /* in float:  (mean, standard error of the mean)          */
    SDE_OBS_MEAN_F64 = 1,  /* in double: (mean, standard error of the mean)          */
    SDE_OBS_MEANSQ_F32 = 2,/* in float:  (mean of x^2, its standard error)           */
    SDE_OBS_ORDER = 3      /* in float revolutions: (r, psi/2pi) of the Kuramoto     */
                           /* order parameter r exp(i psi) = mean exp(2 pi i x)      */
};
/*
 * Reduces consecutive groups of a device array: group g covers counts[g]
 * elements following those of groups < g.  Sums are taken in FP64 with a
 * fixed order (wavefront shuffles, then LDS, then a second pass), so the
 * result is bitwise reproducible.  Writes host_out[g][0..1].  Synchronizes
 * `hip_stream`.  The standard error uses the n-1 sample variance (0 when
 * counts[g] < 2).  Example: <v> +- SE of each point from the per-path
 * `v` array of sde_jj_integrate (ensemble average, Sec. 4 and Sec. 5).
 */
int sde_observables(sde_ctx* ctx, int kind, const void* dev_in /* [device] */,
                    const uint32_t* counts /* [host] */, uint32_t n_groups,
                    double* host_out /* [host] [n_groups][2] */, void* hip_stream);

/*
 * Coarse-grained position histogram with one bin per potential period (the
 * distributions of Fig. 2 and Sec. 5): with x = theta + winding in periods
 * and theta in [0, 1), the bin [x0 + b, x0 + b + 1) holds exactly the paths
 * with winding == x0 + b.  Counts the n device entries of `winding` into
 *   counts[0]            winding <  x0
 *   counts[1 + b]        winding == x0 + b,  0 <= b < n_bins
 *   counts[n_bins + 1]   winding >= x0 + n_bins
 * counts: [device] uint64 [n_bins + 2], overwritten (zeroed by a kernel, so
 * the call can be recorded in a HIP graph).  Integer counts: bitwise
 * reproducible.  Asynchronous on `hip_stream`.  Errors: SDE_ERR_INVALID for
 * NULL counts, NULL winding with n > 0, n_bins = 0 or n_bins > 2^24, a
 * misaligned pointer.
 */
int sde_position_histogram(sde_ctx* ctx, const int32_t* winding /* [device] */, uint64_t n, int64_t x0,
                           uint32_t n_bins, uint64_t* counts /* [device] */, void* hip_stream);
/*
 * sde_position_histogram of n_rows rows at once (the density P(x; t) of
 * Fig. 2 from the rows sde_jj_integrate_recorded writes): row r is
 * winding[r * pitch .. r * pitch + n - 1] and its counts go to
 * counts[r * (n_bins + 2) .. (r + 1) * (n_bins + 2) - 1], laid out as above.
 * pitch >= n when n_rows > 1 (ignored for one row).  Errors: as
 * sde_position_histogram, plus SDE_ERR_INVALID for n_rows = 0 or
 * n_rows > 2^32, or pitch < n with several rows.
 */
int sde_position_histograms(sde_ctx* ctx, const int32_t* winding /* [device] */, uint64_t n, uint64_t pitch,
                            uint64_t n_rows, int64_t x0, uint32_t n_bins, uint64_t* counts /* [device] */,
                            void* hip_stream);

/*
 * Histograms of phases held in revolutions (the density P(x; t) of the
 * Kuramoto phases in Fig. 4, or of the JJ coordinate within a period): row
 * r is theta[r * pitch .. r * pitch + n - 1] (e.g. the R realizations of a
 * Kuramoto state with pitch = N) and counts[r][0 .. n_bins] receives
 *   counts[r][b]       theta in [b / n_bins, (b + 1) / n_bins), b < n_bins
 *                      (theta = 1 counts in the last bin),
 *   counts[r][n_bins]  theta outside [0, 1] or NaN.
 * The bin is floor(theta * n_bins) with the product formed in FP64 (exact),
 * so it is reproducible bit for bit.  counts: [device] uint64
 * [n_rows][n_bins + 1], overwritten by kernels (graph-safe).  pitch >= n
 * when n_rows > 1.  Asynchronous on `hip_stream`.  Errors: SDE_ERR_INVALID
 * for NULL counts, NULL theta with n > 0, n_bins = 0 or n_bins > 2^24,
 * n_rows = 0 or n_rows > 2^32, pitch < n with several rows, a misaligned
 * pointer.
 */
int sde_phase_histograms(sde_ctx* ctx, const float* theta /* [device] */, uint64_t n, uint64_t pitch,
                         uint64_t n_rows, uint32_t n_bins, uint64_t* counts /* [device] */, void* hip_stream);

/* ---- learned surrogate for the mean velocity <v> ------------------------- */
/*
 * An ensemble of small fully connected networks maps the parameters of a
 * Josephson-junction point to its time- and ensemble-averaged velocity <v>
 * (the asymptotic velocity <<v>> of Sec. 5), trained on averages the
 * integrator produces itself.  Member m (of n_members) has layers
 *   h_l = GELU(W_l h_{l-1} + b_l), l < L,   y = W_L h_{L-1} + b_L,
 * GELU(z) = z (1 + erf(z / sqrt 2)) / 2, all FP32.  Parameters of a member
 * are packed W_1, b_1, W_2, b_2, ... row-major (W_l is [w_l][w_{l-1}]).
 * Raw input features of a point are (a, omega, f, log10 D, gamma); they are
 * normalized with the scaling below before entering the network.
 * Calls on a surrogate are ordered on its context (one host thread).
 */
typedef struct sde_surrogate sde_surrogate;
typedef struct {
    float in_center[8];        /* x_i -> (x_i - in_center[i]) / in_scale[i]            */
    float in_scale[8];
    float out_mean, out_std;   /* network output y -> out_mean + out_std * y           */
    int32_t target_over_omega; /* 1: the network predicts <v> / omega (feature 1)      */
    int32_t reserved;          /* must be 0                                            */
} sde_surrogate_scaling;
typedef struct {
    uint32_t epochs;           /* passes over the samples                              */
    uint32_t batch;            /* minibatch size; a last partial batch is dropped      */
    float lr, beta1, beta2, eps; /* Adam with bias correction                          */
    uint64_t shuffle_seed;     /* each member sees its own permutation per epoch       */
} sde_train_opts;
typedef struct {
    uint64_t n_queries, n_fallback;
    double predict_ms;         /* ensemble inference (device time)                     */
    double fallback_ms;        /* simulation of the uncertain points (device time)     */
    double total_ms;           /* whole call, host wall clock                          */
} sde_scan_stats;

/* Creates a surrogate with layer widths widths[0..n_widths-1] (input width
 * first, output width 1 last), n_members members, parameters drawn
 * U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox(ctr = (k >> 2, member, 0,
 * 5), key = seed) word k & 3 for packed parameter k; identity scaling. */
int sde_surrogate_create(sde_ctx* ctx, const uint32_t* widths /* [host] */, uint32_t n_widths,
                         uint32_t n_members, uint64_t seed, sde_surrogate** out);
void sde_surrogate_destroy(sde_surrogate* s);
/* Parameters per member. */
uint64_t sde_surrogate_param_count(const sde_surrogate* s);
/* Copy one member's packed parameters from / to host memory (synchronous);
 * setting parameters also resets that member's Adam state. */
int sde_surrogate_set_params(sde_surrogate* s, uint32_t member, const float* host, uint64_t n);
int sde_surrogate_get_params(sde_surrogate* s, uint32_t member, float* host, uint64_t n);
int sde_surrogate_set_scaling(sde_surrogate* s, const sde_surrogate_scaling* sc);
int sde_surrogate_get_scaling(const sde_surrogate* s, sde_surrogate_scaling* sc);
/* Trains every member on (X [device] [n][w_0] raw features, y [device] [n]
 * targets <v>) with mean-squared error and Adam; loss_curve [host]
 * [epochs] (or NULL) receives each epoch's mean minibatch loss of member 0
 * (in normalized units).  Synchronizes. */
int sde_surrogate_train(sde_surrogate* s, const float* X, const float* y, uint64_t n,
                        const sde_train_opts* opts, float* loss_curve, void* hip_stream);
/* Ensemble prediction for X [device] [n][w_0]: mean [device] [n] and
 * spread [device] [n] (sample standard deviation over members, n - 1 in
 * the denominator), both in units of <v>. */
int sde_surrogate_predict(sde_surrogate* s, const float* X, uint64_t n, float* mean, float* spread,
                          void* hip_stream);
/* Test hook: mean-squared loss and its gradient (packed like the
 * parameters, [host] or NULL) of one member on (X, y), computed with the
 * training kernels at the member's current parameters.  Synchronizes. */
int sde_surrogate_loss_grad(sde_surrogate* s, uint32_t member, const float* X, const float* y, uint64_t n,
                            float* host_grad, double* host_loss, void* hip_stream);
/* Scan: <v> for n query points [host] (their m must be 1).  The ensemble
 * predicts every point; where its spread exceeds spread_max the point is
 * integrated instead (sde_jj_integrate with its own n_paths, n_steps,
 * n_transient and steps_per_period, and `fallback`'s seed and scheme).
 * v_out [device] [n] receives the prediction or the simulated <v>;
 * used_fallback [device] [n] (or NULL) 1 where simulated.  Synchronizes. */
int sde_surrogate_scan(sde_surrogate* s, const sde_jj_point* queries, uint64_t n, float spread_max,
                       const sde_run* fallback, double* v_out, uint8_t* used_fallback,
                       sde_scan_stats* stats, void* hip_stream);
/* Save (widths, members, scaling, parameters) to a binary file / load it. */
int sde_surrogate_save(const sde_surrogate* s, const char* path);
int sde_surrogate_load(sde_ctx* ctx, const char* path, sde_surrogate** out);

/* ---- launch layer: autotuner, graph cache, statistics --------------------- */
enum {
    SDE_OPT_AUTOTUNE = 1, /* 1 (default): on a tune-cache miss, time the candidate   */
                          /* launch configurations on a short slice of the call and  */
                          /* keep the fastest; 0: use the cached or default choice   */
    SDE_OPT_GRAPHS = 2,   /* 1 (default): record each call's launch sequence once in */
                          /* a HIP graph keyed by its arguments and replay it; 0:    */
                          /* launch kernels directly                                 */
    SDE_OPT_JJ_PPT = 3,   /* Josephson-junction paths per lane: 0 (default) = tuned, */
                          /* or 1, 2, 4 to force                                     */
    SDE_OPT_KURA_MF = 4,  /* mean-field variant: 0 (default) = registers when the    */
                          /* realization fits (N <= 2^19 on 256 CUs), else streamed  */
                          /* through HBM; 1 = always streamed; 2 = always registers  */
                          /* (SDE_ERR_UNSUPPORTED when N does not fit)               */
    SDE_OPT_KURA_JSPLIT = 5, /* all-pairs (TILED) sum split over j slices per stage */
                          /* the small-N remedy of Sec. 6: 0 (default) = automatic  */
                          /* (about 4 workgroups per CU when the plain launch has   */
                          /* fewer than 2), 1 = never, J = 2..65535 = J slices (at   */
                          /* least 64 j per slice)                                   */
    SDE_OPT_KURA_TILE = 6, /* all-pairs oscillators per lane (tile of 256 x OPT     */
                          /* phases): 0 (default) = tuned per shape class, or 1, 2, */
                          /* 4 to force                                              */
    SDE_OPT_KURA_XCD_LOCAL = 7, /* register-resident mean field: 1 (default) = the */
                          /* workgroups of a realization that run on one XCD        */
                          /* exchange their sums through that XCD's L2 (checked at  */
                          /* the start of every launch); 0 = always at device scope */
    SDE_OPT_KURA_MF_OPT = 8, /* register-resident mean field oscillators per lane   */
                          /* (512 lanes per workgroup, so N / (512 OPT) workgroups  */
                          /* per realization): 0 (default) = tuned per shape class, */
                          /* or 1, 2, 4, 8 to restrict the choice to that count     */
                          /* (SDE_ERR_UNSUPPORTED if N does not fit at it)          */
    SDE_OPT_DENSE_LAUNCH = 9, /* dense coupling launch: 0 (default) = tuned per shape */
                          /* class; 1 = 8 waves per workgroup splitting the k loop, */
                          /* row tiles dealt to XCDs in bands; 2 = 4 waves, bands;  */
                          /* 3 = 8 waves, plain order; 4 = 4 waves, plain order;    */
                          /* 5 = two workgroups per 128 x 128 tile over the two     */
                          /* halves of k (16-bit products, an even number of        */
                          /* 32-realization tiles; else as 1), bands; 6 = the same, */
                          /* plain order; 7 = 8 waves as 2 row halves x 4 k slices, */
                          /* each with two register sets of fragments (16-bit       */
                          /* products), bands; 8 = the same, plain order; 9 = 4     */
                          /* waves, K fragments double-buffered in LDS (16-bit      */
                          /* products), bands; 10 = the same, plain order; 11 = 8   */
                          /* waves as 4 k slices x 2 column halves, each pair       */
                          /* sharing its K fragments through LDS (16-bit products), */
                          /* bands; 12 = the same, plain order (FP32 always runs 4  */
                          /* waves; bands apply when the row tiles split evenly     */
                          /* over the 8 XCDs)                                       */
    SDE_OPT_KURA_MF_PAIRED = 10 /* register-resident mean field realizations per    */
                          /* workgroup: 0 (default) = tuned per shape class; 1 =    */
                          /* one; 2 = two (R even, 2 or 4 oscillators per lane, at  */
                          /* most 32 workgroups per realization: each workgroup     */
                          /* evaluates one realization's stage while the other's    */
                          /* sums are exchanged).  With this option or              */
                          /* SDE_OPT_KURA_MF_OPT set, the restricted set's default  */
                          /* is run untuned; SDE_ERR_UNSUPPORTED if it is empty     */
};
/* Sets an option of the context.  SDE_ERR_INVALID for an unknown option or
 * value. */
int sde_set_option(sde_ctx* ctx, int option, int64_t value);
/* Loads tuned launch choices from the JSON file `path` (created if missing)
 * and saves new ones there after each tuning.  NULL: keep choices in memory
 * only.  The environment variable SDE_TUNE_CACHE sets it at sde_create. */
int sde_set_tune_cache(sde_ctx* ctx, const char* path);

typedef struct {
    int32_t graph_replayed;  /* the last call replayed a cached HIP graph             */
    int32_t tuned;           /* the last call ran the autotuner                       */
    int32_t jj_paths_per_lane;
    int32_t graphs_cached;   /* HIP graphs held by the context                        */
    double tune_ms;          /* time spent tuning in the last call                    */
    uint64_t work_items;     /* work items (point, path chunk) of the last JJ call    */
    int32_t mf_streamed;     /* the last Kuramoto mean-field call streamed the state  */
                             /* through HBM (1) or held it in registers (0)           */
    int32_t kura_jsplit;     /* j slices of the last all-pairs (TILED) call           */
    int32_t kura_tile;       /* oscillators per lane of the last all-pairs call       */
    int32_t kura_mf_opt;     /* oscillators per lane of the last register-resident    */
                             /* mean-field call                                       */
    int32_t dense_waves;     /* waves per workgroup (k-loop split) of the last dense  */
                             /* call                                                  */
    int32_t dense_xcd_bands; /* its row tiles were dealt to XCDs in bands (1)         */
    int32_t kura_mf_paired;  /* the last register-resident mean-field call held two   */
                             /* realizations per workgroup (1)                        */
    int32_t dense_variant;   /* the last dense call's kernel: 0 k-sliced waves with   */
                             /* 128 x 64 tiles, 1 two workgroups per tile over the    */
                             /* halves of k (then a stage kernel), 2 row-half waves   */
                             /* with two register sets, 3 four waves with K in LDS,   */
                             /* 4 wave pairs sharing K through LDS                    */
} sde_stats;
/* Statistics of the last integration call on `ctx`. */
int sde_get_stats(const sde_ctx* ctx, sde_stats* out);

/* ---- test hooks ---------------------------------------------------------- */
/* dev_out[k][0..3] = Philox4x32-10 words at counter (ctr0_first + k, a, b, tag)
 * for k < n_blocks (the raw integers the integrators consume). */
int sde_debug_philox(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                     uint64_t ctr0_first, uint64_t n_blocks, uint32_t* dev_out /* [device] */,
                     void* hip_stream);
/* dev_out[k] = Gaussian number n_first + k of stream (tag, a, b), as the
 * integrators compute it (FP32 Box-Muller on the 24-bit uniforms). */
int sde_debug_gauss(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                    uint64_t n_first, uint64_t count, float* dev_out /* [device] */,
                    void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif
