// jj.hip -- ensemble integration of the driven, damped, noisy Brownian
// particle of Eq. 1 over many independent paths and parameter points,
// stochastic Heun (Alg. 2) or Euler-Maruyama.  Per point, either potential:
//   SDE_POTENTIAL_SIN     m phi'' + gamma phi' = -sin phi + a cos wt + f + noise
//                         (Josephson-junction form, phi in radians)
//   SDE_POTENTIAL_SIN2PI  m x'' + gamma x' = -2 pi cos(2 pi x) + a cos wt + f
//                         + noise: the paper's V(x) = sin(2 pi x), x in periods
// The state is the coordinate in units of its period (theta + winding), so
// the two differ only in the trigonometric function of the force and in
// per-point constants.
//
// Design (gfx950):
//  * One persistent launch.  Every wavefront pops work items (point, path
//    chunk of 64*PPT paths) from a device-scope counter until the queue is
//    empty; items are queued longest-first so uneven batches finish together.
//    Paths are independent (Sec. 4.1), so which wave runs an item does not
//    change any result.
//  * Per-path state stays in VGPRs for the whole item (Alg. 1 keeps x, v in
//    registers for m steps and touches global memory only at the ends); the
//    point's parameters are wave-uniform and live in SGPRs.
//  * The phase is kept in revolutions, theta in [0, 1), plus an integer
//    winding count, so the hardware v_sin_f32 (which takes revolutions) needs
//    no range reduction and FP32 never adds a tiny increment to a large phase
//    (the precision issue of Sec. 5).  The drive phase is the step index mod
//    S read from a cos table, the integer form of keeping time modulo the
//    drive period (Sec. 5).
//  * One Philox4x32-10 block per path gives the Gaussians of four
//    consecutive steps; Box-Muller uses the hardware log2/sqrt/sin/cos.
//  * The time average of v is summed in FP32 over M steps and folded into an
//    FP64 accumulator every M absolute steps (Sec. 4.1 samples every M).
//  * Per-chunk FP64 sums of vbar and vbar^2 are written without atomics and
//    combined per point in a fixed order by a second kernel, so results are
//    bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "device_common.h"
#include "sde_internal.h"

namespace sde {

// Per-point constants in the arithmetic type R of the integration (float:
// the FP32 path; double: the FP64 path).
template <typename R>
struct JJPointT {
    R dt, hdt, dtp, hdtp;          // dt, dt/2, dt/L, dt/(2L) with L the coordinate's period
                                   // (2 pi for phi, 1 for x): theta' = v / L
    R gim, kv, a_im, f_im;         // gamma/m, (force amplitude)/m, a/m, f/m with force
                                   // amplitude 1 (sin phi) or 2 pi (2 pi cos 2 pi x);
                                   // overdamped: 1/gamma for 1/m
    R c2, sig_v;                   // c2 = -2 ln2 sigma^2 with sigma the noise increment per
                                   // Gaussian: on v (inertial) or on theta in periods
                                   // (overdamped); sig_v = L / dt turns the latter into
                                   // a velocity
    uint32_t S, lut_off, n_paths, inertial;
    uint64_t path_first, n_steps, n_transient;
    double inv_W;
    uint32_t chunk_first, n_chunks;
};
using JJPointDev = JJPointT<float>;
static_assert(sizeof(JJPointT<float>) % 8 == 0 && sizeof(JJPointT<double>) % 8 == 0, "layout");

struct JJItem {
    uint32_t point, chunk;
};

struct JJArgs {
    const void* pts;      // JJPointT<R>[]
    const JJItem* items;
    const void* lut;      // R[]
    uint32_t* queue;
    int* flag;
    void* theta;          // R[]
    int32_t* winding;
    void* v;              // R[]
    double* acc;
    double* partials;
    int32_t* rec;         // optional windings every rec_every steps: [row][rec_pitch]
    uint64_t rec_pitch;   // paths of the call
    uint64_t step0;
    uint32_t key0, key1;
    uint32_t n_items, M;
    uint32_t rec_every;   // a multiple of 4 (records fall on block ends)
    int32_t init_from_state;
};

// One step n -> n + 1 of the PPT paths held by this lane.  e0, e1 are the
// uniform drive terms (a cos(w t) + f)/m at t_n and t_{n+1} (the second
// drift evaluation of Alg. 2 is taken at t + dt), ns the noise increments.
// The potential's shape at theta (in periods): sin(2 pi theta) for the
// -sin phi force, cos(2 pi theta) for -V'(x) = -2 pi cos(2 pi x).  FP32: the
// hardware v_sin/v_cos, which take revolutions; FP64: sinpi/cospi.
template <bool COSF>
__device__ __forceinline__ float jj_shape(float theta)
{
    return COSF ? cos_rev(theta) : sin_rev(theta);
}
template <bool COSF>
__device__ __forceinline__ double jj_shape(double theta)
{
    return COSF ? cospi(2.0 * theta) : sinpi(2.0 * theta);
}

__device__ __forceinline__ float fm(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return fma(a, b, c); }

// sigma * (the four Gaussians of Philox block c), c2 = -2 ln2 sigma^2.
__device__ __forceinline__ void jj_gauss4(U4 c, uint32_t k0, uint32_t k1, float c2, float g[4])
{
    gauss4_scaled(c, k0, k1, c2, g);
}
__device__ __forceinline__ void jj_gauss4(U4 c, uint32_t k0, uint32_t k1, double c2, double g[4])
{
    const U4 x = philox4x32_10(c, k0, k1);
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double u1 = (double)((w[2 * p] >> 8) + 1u) * 0x1p-24;
        const double u2 = (double)(w[2 * p + 1] >> 8) * 0x1p-24;
        const double rho = sqrt(c2 * log2(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        g[2 * p] = rho * cs;
        g[2 * p + 1] = rho * sn;
    }
}

template <typename R, int PPT, int SCHEME, bool INERTIAL, bool COSF, bool ACC>
__device__ __forceinline__ void jj_step(const JJPointT<R>& P, R e0, R e1, const R (&ns)[PPT], R (&th)[PPT],
                                        R (&vv)[PPT], R (&af)[PPT])
{
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (INERTIAL) {
            // X = (coordinate, v), F = (v, (force - gamma v + a cos wt + f)/m), noise on v
            const R F1 = fm(-P.kv, jj_shape<COSF>(th[k]), fm(-P.gim, vv[k], e0));
            if (SCHEME == SDE_HEUN) {
                const R vt = fm(P.dt, F1, vv[k]) + ns[k];
                const R tt = fm(P.dtp, vv[k], th[k]);
                const R F2 = fm(-P.kv, jj_shape<COSF>(tt), fm(-P.gim, vt, e1));
                th[k] = fm(P.hdtp, vv[k] + vt, th[k]);
                vv[k] = fm(P.hdt, F1 + F2, vv[k]) + ns[k];
            } else {
                th[k] = fm(P.dtp, vv[k], th[k]);
                vv[k] = fm(P.dt, F1, vv[k]) + ns[k];
            }
        } else {
            // overdamped: coordinate' = (force + a cos wt + f)/gamma + noise on
            // the coordinate; v reports the step's mean velocity (change / dt)
            const R F1 = fm(-P.kv, jj_shape<COSF>(th[k]), e0);
            if (SCHEME == SDE_HEUN) {
                const R tt = fm(P.dtp, F1, th[k]) + ns[k];
                const R F2 = fm(-P.kv, jj_shape<COSF>(tt), e1);
                th[k] = fm(P.hdtp, F1 + F2, th[k]) + ns[k];
                vv[k] = fm(R(0.5), F1 + F2, P.sig_v * ns[k]);
            } else {
                th[k] = fm(P.dtp, F1, th[k]) + ns[k];
                vv[k] = fm(P.sig_v, ns[k], F1);
            }
        }
        if (ACC) af[k] += vv[k];
    }
}

template <typename R, int PPT, int SCHEME, bool INERTIAL, bool COSF>
__device__ __forceinline__ void jj_item(const JJArgs& A, uint32_t q, uint32_t chunk)
{
    const JJPointT<R> P = load_uniform(static_cast<const JJPointT<R>*>(A.pts) + q);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    R* theta = static_cast<R*>(A.theta);
    R* vel = static_cast<R*>(A.v);

    R th[PPT], vv[PPT], af[PPT];
    int32_t wd[PPT];
    double ad[PPT];
    uint32_t pid[PPT];
    bool live[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        pid[k] = chunk * (kWave * PPT) + k * kWave + lane;
        live[k] = pid[k] < P.n_paths;
        const uint64_t gi = P.path_first + pid[k];
        if (A.init_from_state) {
            th[k] = live[k] ? theta[gi] : R(0);
            vv[k] = live[k] ? vel[gi] : R(0);
            wd[k] = live[k] ? A.winding[gi] : 0;
            ad[k] = live[k] ? A.acc[gi] : 0.0;
        } else {
            const U4 x = philox4x32_10(U4{0u, pid[k], q, (uint32_t)SDE_TAG_INIT}, A.key0, A.key1);
            th[k] = (R)(x.x >> 8) * R(0x1p-24);
            vv[k] = R(-2) + R(4) * ((R)(x.y >> 8) * R(0x1p-24));
            wd[k] = 0;
            ad[k] = 0.0;
        }
        af[k] = R(0);
    }

    const R* lut = static_cast<const R*>(A.lut) + P.lut_off;  // cos(2 pi k / S) for k < S + 8
    const uint64_t n_end = A.step0 + P.n_steps;
    uint64_t n = A.step0;
    uint32_t kk = (uint32_t)(n % P.S);        // drive phase index of step n
    uint32_t mc = (uint32_t)((n + 1) % A.M);  // (n + 1) mod M: fold after the step when 0
    // recording: rc = n mod rec_every; row r holds the state after the
    // (r + 1)-th multiple of rec_every past step0
    uint32_t rc = A.rec ? (uint32_t)(n % A.rec_every) : 0u;
    uint64_t row = 0;

    auto fold_tick = [&]() {
        if (mc == 0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                ad[k] += (double)af[k];
                af[k] = R(0);
            }
        }
        mc = (mc + 1 == A.M) ? 0u : mc + 1;
    };

    while (n < n_end) {
        const uint32_t j0 = (uint32_t)n & 3u;
        const uint64_t left = n_end - n;
        const uint32_t jn = left >= (uint64_t)(4u - j0) ? 4u : j0 + (uint32_t)left;
        // sigma * Gaussians of steps 4b .. 4b+3 (b = n >> 2) of each path
        R g[PPT][4];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            jj_gauss4(U4{(uint32_t)(n >> 2), pid[k], q, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, P.c2, g[k]);
        if (j0 == 0 && jn == 4) {
            R e[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) e[j] = fm(P.a_im, load_uniform(lut + kk + j), P.f_im);
            if (n >= P.n_transient) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    R ns[PPT];
#pragma unroll
                    for (int k = 0; k < PPT; ++k) ns[k] = g[k][j];
                    jj_step<R, PPT, SCHEME, INERTIAL, COSF, true>(P, e[j], e[j + 1], ns, th, vv, af);
                    fold_tick();
                }
            } else if (n + 4 <= P.n_transient) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    R ns[PPT];
#pragma unroll
                    for (int k = 0; k < PPT; ++k) ns[k] = g[k][j];
                    jj_step<R, PPT, SCHEME, INERTIAL, COSF, false>(P, e[j], e[j + 1], ns, th, vv, af);
                    fold_tick();
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    R ns[PPT];
#pragma unroll
                    for (int k = 0; k < PPT; ++k) ns[k] = g[k][j];
                    if (n + j >= P.n_transient)
                        jj_step<R, PPT, SCHEME, INERTIAL, COSF, true>(P, e[j], e[j + 1], ns, th, vv, af);
                    else
                        jj_step<R, PPT, SCHEME, INERTIAL, COSF, false>(P, e[j], e[j + 1], ns, th, vv, af);
                    fold_tick();
                }
            }
            n += 4;
            kk += 4;
            while (kk >= P.S) kk -= P.S;
        } else {
            // partial block (first or last of the call): one step at a time
            for (uint32_t j = j0; j < jn; ++j) {
                R ns[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    ns[k] = j == 0 ? g[k][0] : j == 1 ? g[k][1] : j == 2 ? g[k][2] : g[k][3];
                const R ea = fm(P.a_im, load_uniform(lut + kk), P.f_im);
                const R eb = fm(P.a_im, load_uniform(lut + kk + 1), P.f_im);
                if (n >= P.n_transient)
                    jj_step<R, PPT, SCHEME, INERTIAL, COSF, true>(P, ea, eb, ns, th, vv, af);
                else
                    jj_step<R, PPT, SCHEME, INERTIAL, COSF, false>(P, ea, eb, ns, th, vv, af);
                fold_tick();
                ++n;
                kk = (kk + 1 == P.S) ? 0u : kk + 1;
            }
        }
        // keep theta in [0, 1): move whole revolutions into the winding count
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const R fl = floor(th[k]);
            th[k] -= fl;
            wd[k] += (int32_t)fl;
        }
        // a block never crosses a multiple of 4, hence of rec_every
        if (A.rec) {
            rc += jn - j0;
            if (rc == A.rec_every) {
                rc = 0;
                int32_t* out = A.rec + row * A.rec_pitch + P.path_first;
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (live[k]) out[pid[k]] = wd[k];
                ++row;
            }
        }
    }

    double s1 = 0.0, s2 = 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        ad[k] += (double)af[k];
        if (live[k]) {
            const uint64_t gi = P.path_first + pid[k];
            if (theta) theta[gi] = th[k];
            if (A.winding) A.winding[gi] = wd[k];
            if (vel) vel[gi] = vv[k];
            if (A.acc) A.acc[gi] = ad[k];
            const double vb = ad[k] * P.inv_W;
            s1 += vb;
            s2 += vb * vb;
            bad |= !(isfinite(th[k]) && isfinite(vv[k]));
        }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
        A.partials[2 * (P.chunk_first + chunk)] = s1;
        A.partials[2 * (P.chunk_first + chunk) + 1] = s2;
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(A.flag, 1);
}

template <typename R, int PPT, int SCHEME, bool INERTIAL, bool COSF>
__global__ __launch_bounds__(256) void jj_persistent_kernel(JJArgs A)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(A.queue, 1u);
        item = uniform_u32(__shfl(item, 0, kWave));
        if (item >= A.n_items) break;
        const JJItem it = load_uniform(A.items + item);
        jj_item<R, PPT, SCHEME, INERTIAL, COSF>(A, it.point, it.chunk);
    }
}

// Stage 2: per point, the chunk partials in chunk order.
template <typename R>
__global__ void jj_point_sums_kernel(const JJPointT<R>* pts, uint32_t n_pts, const double* partials, double* out)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pts) return;
    const uint32_t first = pts[q].chunk_first, nc = pts[q].n_chunks;
    double s1 = 0.0, s2 = 0.0;
    for (uint32_t c = 0; c < nc; ++c) {
        s1 += partials[2 * (first + c)];
        s2 += partials[2 * (first + c) + 1];
    }
    out[2 * q] = s1;
    out[2 * q + 1] = s2;
}

// Test hooks: raw Philox words and the integrators' Gaussians.
__global__ void philox_dump_kernel(uint32_t k0, uint32_t k1, uint32_t tag, uint32_t a, uint32_t b,
                                   uint64_t c0, uint64_t n, uint32_t* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 x = philox4x32_10(U4{(uint32_t)(c0 + i), a, b, tag}, k0, k1);
    out[4 * i] = x.x;
    out[4 * i + 1] = x.y;
    out[4 * i + 2] = x.z;
    out[4 * i + 3] = x.w;
}

__global__ void gauss_dump_kernel(uint32_t k0, uint32_t k1, uint32_t tag, uint32_t a, uint32_t b,
                                  uint64_t n0, uint64_t n, float* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t s = n0 + i;
    float g[4];
    gauss4(U4{(uint32_t)(s >> 2), a, b, tag}, k0, k1, g);
    const uint32_t j = (uint32_t)s & 3u;
    out[i] = j == 0 ? g[0] : j == 1 ? g[1] : j == 2 ? g[2] : g[3];
}

// ------------------------------------------------------------------ host --

using JJKernel = void (*)(JJArgs);

// Paths per lane: 1, 2 or 4 in FP32; FP64 holds twice the registers per
// path and stops at 2.
template <typename R, bool INERTIAL, bool COSF>
static JJKernel pick_kernel_t(int ppt, int scheme)
{
    constexpr bool f32 = sizeof(R) == 4;
    if (scheme == SDE_HEUN) {
        if (ppt == 1) return jj_persistent_kernel<R, 1, SDE_HEUN, INERTIAL, COSF>;
        if (f32 && ppt == 4) return jj_persistent_kernel<R, f32 ? 4 : 2, SDE_HEUN, INERTIAL, COSF>;
        return jj_persistent_kernel<R, 2, SDE_HEUN, INERTIAL, COSF>;
    }
    if (ppt == 1) return jj_persistent_kernel<R, 1, SDE_EULER, INERTIAL, COSF>;
    if (f32 && ppt == 4) return jj_persistent_kernel<R, f32 ? 4 : 2, SDE_EULER, INERTIAL, COSF>;
    return jj_persistent_kernel<R, 2, SDE_EULER, INERTIAL, COSF>;
}

// Point kinds, one persistent launch each: bit 0 = overdamped, bit 1 = the
// sin(2 pi x) potential.
constexpr int kJJKinds = 4;

template <typename R>
static JJKernel pick_kernel(int kind, int ppt, int scheme)
{
    switch (kind) {
    case 0: return pick_kernel_t<R, true, false>(ppt, scheme);
    case 1: return pick_kernel_t<R, false, false>(ppt, scheme);
    case 2: return pick_kernel_t<R, true, true>(ppt, scheme);
    default: return pick_kernel_t<R, false, true>(ppt, scheme);
    }
}

static bool finite_point(const sde_jj_point& p)
{
    return std::isfinite(p.m) && std::isfinite(p.gamma) && std::isfinite(p.a) && std::isfinite(p.omega) &&
           std::isfinite(p.f) && std::isfinite(p.D);
}

// Work items of one paths-per-lane choice: chunk layout per point and the
// queue of each point kind (longest first within a kind).
template <typename R>
struct JJPlan {
    std::vector<JJPointT<R>> pts;
    std::vector<JJItem> items;
    uint32_t kind_begin[kJJKinds + 1] = {};  // items of kind k: [kind_begin[k], kind_begin[k + 1])
    uint32_t n_chunks = 0;
};

template <typename R>
static void plan_items(std::vector<JJPointT<R>>& P, const std::vector<int>& kinds, int ppt, JJPlan<R>& out)
{
    const uint32_t chunk_paths = (uint32_t)(kWave * ppt);
    std::vector<JJItem> it[kJJKinds];
    uint32_t chunk_first = 0;
    for (uint32_t q = 0; q < (uint32_t)P.size(); ++q) {
        JJPointT<R>& d = P[q];
        d.n_chunks = (d.n_paths + chunk_paths - 1) / chunk_paths;
        d.chunk_first = chunk_first;
        for (uint32_t c = 0; c < d.n_chunks; ++c) it[kinds[q]].push_back(JJItem{q, c});
        chunk_first += d.n_chunks;
    }
    auto longest_first = [&](const JJItem& x, const JJItem& y) { return P[x.point].n_steps > P[y.point].n_steps; };
    out.pts = P;
    out.items.clear();
    for (int k = 0; k < kJJKinds; ++k) {
        std::stable_sort(it[k].begin(), it[k].end(), longest_first);
        out.kind_begin[k] = (uint32_t)out.items.size();
        out.items.insert(out.items.end(), it[k].begin(), it[k].end());
    }
    out.kind_begin[kJJKinds] = (uint32_t)out.items.size();
    out.n_chunks = chunk_first;
}

struct JJLaunch {
    JJArgs A;
    uint32_t* queues;  // kJJKinds work-queue words, zeroed by each launch sequence
    int ppt;
    int scheme;
    uint32_t kind_begin[kJJKinds + 1];
    uint32_t n_items, n_pts;
    uint32_t grid[kJJKinds];
    double* point_sums;
};

template <typename R>
static int jj_grids(sde_ctx* ctx, JJLaunch& L)
{
    for (int kind = 0; kind < kJJKinds; ++kind) {
        const uint32_t count = L.kind_begin[kind + 1] - L.kind_begin[kind];
        L.grid[kind] = 0;
        if (!count) continue;
        JJKernel kern = pick_kernel<R>(kind, L.ppt, L.scheme);
        int per_cu = 0;
        SDE_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), 256, 0));
        if (per_cu < 1) per_cu = 1;
        const uint64_t want = ((uint64_t)count + 3) / 4;  // 4 waves per block, one item each at least
        L.grid[kind] = (uint32_t)std::min<uint64_t>(want, (uint64_t)per_cu * ctx->n_cu);
    }
    return SDE_OK;
}

__global__ void jj_zero_queues_kernel(uint32_t* q)
{
    if (threadIdx.x < (uint32_t)kJJKinds) q[threadIdx.x] = 0u;
}

// The launch sequence of one call: reset the queues, the persistent kernel
// of each point kind present, the per-point sums.
template <typename R>
static int jj_record(sde_ctx* ctx, const JJLaunch& L, hipStream_t s)
{
    hipLaunchKernelGGL(jj_zero_queues_kernel, dim3(1), dim3(64), 0, s, L.queues);
    SDE_HIP(ctx, hipGetLastError());
    const JJItem* all = L.A.items;
    for (int kind = 0; kind < kJJKinds; ++kind) {
        if (!L.grid[kind]) continue;
        JJArgs A = L.A;
        A.items = all + L.kind_begin[kind];
        A.n_items = L.kind_begin[kind + 1] - L.kind_begin[kind];
        A.queue = L.queues + kind;
        JJKernel kern = pick_kernel<R>(kind, L.ppt, L.scheme);
        hipLaunchKernelGGL(kern, dim3(L.grid[kind]), dim3(256), 0, s, A);
        SDE_HIP(ctx, hipGetLastError());
    }
    if (L.point_sums) {
        hipLaunchKernelGGL(jj_point_sums_kernel<R>, dim3((L.n_pts + 255) / 256), dim3(256), 0, s,
                           static_cast<const JJPointT<R>*>(L.A.pts), L.n_pts, L.A.partials, L.point_sums);
        SDE_HIP(ctx, hipGetLastError());
    }
    return SDE_OK;
}

// The graph cache key of one call: every value the recorded launches bake
// in -- each field of the kernel arguments (the per-kind item range and queue
// word are derived from kind_begin and the queue words), the kernel choice,
// the grids and the point-sum launch.  A field left out would let a later call replay a graph recorded
// with a stale value.
static std::string jj_graph_key(const char* prec, const JJLaunch& L)
{
    const JJArgs& A = L.A;
    char buf[640];
    snprintf(buf, sizeof buf,
             "jj|%s|pts%p|it%p|lut%p|q%p|fl%p|th%p|wd%p|v%p|acc%p|pa%p|rec%p/%llu/%u|n0%llu|k%u.%u|ni%u|M%u|ini%d|"
             "ppt%d|sch%d|np%u|ps%p",
             prec, A.pts, (const void*)A.items, A.lut, (void*)L.queues, (void*)A.flag, A.theta, (void*)A.winding, A.v,
             (void*)A.acc, (void*)A.partials, (void*)A.rec, (unsigned long long)A.rec_pitch, A.rec_every,
             (unsigned long long)A.step0, A.key0, A.key1, L.n_items, A.M, A.init_from_state, L.ppt, L.scheme,
             L.n_pts, (void*)L.point_sums);
    std::string k = buf;
    for (int kind = 0; kind < kJJKinds; ++kind)
        k += "|" + std::to_string(L.kind_begin[kind + 1]) + "/" + std::to_string(L.grid[kind]);
    return k;
}

template <typename R>
static int jj_upload_plan(sde_ctx* ctx, const JJPlan<R>& plan, hipStream_t stream, JJLaunch& L)
{
    int st;
    if ((st = upload(ctx, kSlotJJPoints, 0, plan.pts.data(), plan.pts.size() * sizeof(JJPointT<R>), stream)))
        return st;
    if ((st = upload(ctx, kSlotJJItems, 1, plan.items.data(), plan.items.size() * sizeof(JJItem), stream))) return st;
    void* partials = nullptr;
    if ((st = ensure_ws(ctx, kSlotJJPartials, (size_t)std::max(plan.n_chunks, 1u) * 2 * sizeof(double), &partials)))
        return st;
    if ((st = ensure_counters(ctx, kJJKinds))) return st;
    L.queues = ctx->counters;
    L.A.pts = ctx->ws[kSlotJJPoints].ptr;
    L.A.items = static_cast<const JJItem*>(ctx->ws[kSlotJJItems].ptr);
    L.A.partials = static_cast<double*>(partials);
    std::copy(plan.kind_begin, plan.kind_begin + kJJKinds + 1, L.kind_begin);
    L.n_items = (uint32_t)plan.items.size();
    L.n_pts = (uint32_t)plan.pts.size();
    return jj_grids<R>(ctx, L);
}

static int ilog2u64(uint64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

// Times the candidate paths-per-lane choices on a short slice of the call
// (same points, at most 2048 steps, no per-path outputs) and returns the
// fastest.  Nothing the caller passed is written.
template <typename R>
static int jj_tune(sde_ctx* ctx, const std::vector<JJPointT<R>>& P0, const std::vector<int>& kinds,
                   const JJLaunch& base, hipStream_t stream, int* best_ppt)
{
    std::vector<JJPointT<R>> P = P0;
    uint64_t work = 0;
    for (auto& d : P) {
        d.n_steps = std::min<uint64_t>(d.n_steps, 2048);
        work += (uint64_t)d.n_paths * d.n_steps;
    }
    if (work == 0) {
        *best_ppt = 2;
        return SDE_OK;
    }
    hipEvent_t e0, e1;
    SDE_HIP(ctx, hipEventCreate(&e0));
    SDE_HIP(ctx, hipEventCreate(&e1));
    double best = 1e300;
    int st = SDE_OK;
    const std::vector<int> cands = sizeof(R) == 4 ? std::vector<int>{1, 2, 4} : std::vector<int>{1, 2};
    for (int ppt : cands) {
        JJPlan<R> plan;
        plan_items(P, kinds, ppt, plan);
        JJLaunch L = base;
        L.ppt = ppt;
        L.point_sums = nullptr;
        L.A.theta = nullptr;
        L.A.winding = nullptr;
        L.A.v = nullptr;
        L.A.acc = nullptr;
        L.A.rec = nullptr;
        L.A.init_from_state = 0;
        L.A.flag = ctx->tune_flag;  // a trial run's NaN is not the caller's
        if ((st = jj_upload_plan(ctx, plan, stream, L))) break;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {  // first launch loads the code object
            if ((st = hipEventRecord(e0, stream) == hipSuccess ? SDE_OK : SDE_ERR_DEVICE)) break;
            if ((st = jj_record<R>(ctx, L, stream))) break;
            if ((st = hipEventRecord(e1, stream) == hipSuccess ? SDE_OK : SDE_ERR_DEVICE)) break;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = SDE_ERR_DEVICE;
                break;
            }
        }
        if (st) break;
        if (ms < best) {
            best = ms;
            *best_ppt = ppt;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == SDE_ERR_DEVICE) return fail(ctx, st, "autotuner: HIP event or launch failed");
    return st;
}

// What one call computes, from its arguments: per-point constants, point
// kinds, the drive tables, and the shape class of the call.
template <typename R>
struct JJSetup {
    std::vector<JJPointT<R>> P;
    std::vector<int> kinds;
    std::vector<R> lut;
    uint64_t path_first = 0, max_steps = 0;
    unsigned kinds_present = 0;
    uint32_t M = 100;
};

// Validates a call's arguments (nothing is launched on an error) and builds
// its per-point constants and drive tables.
template <typename R>
static int jj_setup(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run, R* theta,
                    int32_t* winding, R* v, double* acc, double* point_sums, JJSetup<R>& out)
{
    ctx->last = sde_stats{};
    if (!pts || !run || n_pts == 0) return fail(ctx, SDE_ERR_INVALID, "null points/run or n_pts = 0");
    if (run->scheme != SDE_HEUN && run->scheme != SDE_EULER)
        return fail(ctx, SDE_ERR_INVALID, "unknown scheme %d", run->scheme);
    if (run->init != SDE_INIT_PHILOX && run->init != SDE_INIT_FROM_STATE)
        return fail(ctx, SDE_ERR_INVALID, "unknown init %d", run->init);
    if (run->init == SDE_INIT_FROM_STATE && (!theta || !winding || !v || !acc))
        return fail(ctx, SDE_ERR_INVALID, "SDE_INIT_FROM_STATE needs theta, winding, v and acc");
    if (!aligned(theta, sizeof(R)) || !aligned(winding, 4) || !aligned(v, sizeof(R)) || !aligned(acc, 8) ||
        !aligned(point_sums, 8))
        return fail(ctx, SDE_ERR_INVALID, "misaligned device pointer");
    out.M = run->sample_every ? run->sample_every : 100u;

    std::vector<JJPointT<R>>& P = out.P;
    std::vector<int>& kinds = out.kinds;
    std::vector<R>& lut = out.lut;
    P.assign(n_pts, JJPointT<R>{});
    kinds.assign(n_pts, 0);
    lut.clear();
    std::map<uint32_t, uint32_t> lut_of;  // S -> offset
    uint64_t path_first = 0, max_steps = 0;
    unsigned kinds_present = 0;
    for (uint32_t q = 0; q < n_pts; ++q) {
        const sde_jj_point& p = pts[q];
        if (!finite_point(p)) return fail(ctx, SDE_ERR_INVALID, "point %u: non-finite parameter", q);
        if (p.n_paths == 0 || p.steps_per_period == 0)
            return fail(ctx, SDE_ERR_INVALID, "point %u: n_paths and steps_per_period must be > 0", q);
        if (p.n_paths > (1u << 31)) return fail(ctx, SDE_ERR_INVALID, "point %u: more than 2^31 paths", q);
        if (!(p.omega > 0) || p.m < 0 || p.gamma < 0 || p.D < 0 || (p.m == 0 && !(p.gamma > 0)))
            return fail(ctx, SDE_ERR_INVALID, "point %u: need omega > 0, m >= 0, D >= 0, gamma >= 0 "
                        "(gamma > 0 when m = 0)", q);
        if (p.potential != SDE_POTENTIAL_SIN && p.potential != SDE_POTENTIAL_SIN2PI)
            return fail(ctx, SDE_ERR_INVALID, "point %u: unknown potential %d", q, p.potential);
        if (p.reserved != 0) return fail(ctx, SDE_ERR_INVALID, "point %u: reserved must be 0", q);
        const bool sin2pi = p.potential == SDE_POTENTIAL_SIN2PI;
        const double L = sin2pi ? 1.0 : 2.0 * M_PI;   // period of the coordinate
        const double amp = sin2pi ? 2.0 * M_PI : 1.0;  // amplitude of the potential force
        const double dt = 2.0 * M_PI / (p.omega * (double)p.steps_per_period);
        JJPointT<R>& d = P[q];
        d.dt = (R)dt;
        d.hdt = (R)(0.5 * dt);
        d.dtp = (R)(dt / L);
        d.hdtp = (R)(0.5 * dt / L);
        d.inertial = p.m > 0 ? 1u : 0u;
        if (d.inertial) {
            d.kv = (R)(amp / p.m);
            d.gim = (R)(p.gamma / p.m);
            d.a_im = (R)(p.a / p.m);
            d.f_im = (R)(p.f / p.m);
            const double sig = std::sqrt(2.0 * p.gamma * p.D * dt) / p.m;
            d.c2 = (R)(-2.0 * M_LN2 * sig * sig);
            d.sig_v = (R)0;
        } else {
            const double s = std::sqrt(2.0 * p.D * dt / p.gamma);
            d.kv = (R)(amp / p.gamma);
            d.gim = (R)0;
            d.a_im = (R)(p.a / p.gamma);
            d.f_im = (R)(p.f / p.gamma);
            const double sig = s / L;
            d.c2 = (R)(-2.0 * M_LN2 * sig * sig);
            d.sig_v = (R)(L / dt);
        }
        kinds[q] = (d.inertial ? 0 : 1) + (sin2pi ? 2 : 0);
        kinds_present |= 1u << kinds[q];
        d.S = p.steps_per_period;
        auto it = lut_of.find(d.S);
        if (it == lut_of.end()) {
            const uint32_t off = (uint32_t)lut.size();
            for (uint32_t k = 0; k < d.S + 8; ++k)
                lut.push_back((R)std::cos(2.0 * M_PI * (double)(k % d.S) / (double)d.S));
            it = lut_of.emplace(d.S, off).first;
        }
        d.lut_off = it->second;
        d.n_paths = p.n_paths;
        d.path_first = path_first;
        d.n_steps = p.n_steps;
        d.n_transient = p.n_transient;
        const uint64_t end = run->step0 + p.n_steps;
        const uint64_t W = end > p.n_transient ? end - p.n_transient : 0;
        d.inv_W = W ? 1.0 / (double)W : 0.0;
        path_first += p.n_paths;
        max_steps = std::max<uint64_t>(max_steps, p.n_steps);
    }
    if (path_first / kWave > 0xffffffffull) return fail(ctx, SDE_ERR_INVALID, "too many paths in one call");
    out.path_first = path_first;
    out.max_steps = max_steps;
    out.kinds_present = kinds_present;
    return SDE_OK;
}

// The kernel arguments that come from the run options and the caller's
// buffers (the workspace pointers are filled in by the caller).
template <typename R>
static void jj_fill_args(sde_ctx* ctx, const sde_run* run, const JJSetup<R>& S, R* theta, int32_t* winding, R* v,
                         double* acc, double* point_sums, JJLaunch& L)
{
    L.scheme = run->scheme;
    L.point_sums = point_sums;
    L.A.flag = ctx->flag;
    L.A.theta = theta;
    L.A.winding = winding;
    L.A.v = v;
    L.A.acc = acc;
    L.A.step0 = run->step0;
    L.A.rec = nullptr;
    L.A.rec_pitch = S.path_first;
    L.A.rec_every = 0u;
    L.A.key0 = (uint32_t)(run->seed & 0xffffffffu);
    L.A.key1 = (uint32_t)(run->seed >> 32);
    L.A.M = S.M;
    L.A.init_from_state = run->init == SDE_INIT_FROM_STATE;
}

// Tune-cache key of a call's shape class (paths per lane).
template <typename R>
static std::string jj_tune_key(sde_ctx* ctx, const sde_run* run, const JJSetup<R>& S)
{
    char key[160];
    snprintf(key, sizeof key, "jj|%s|%s|scheme%d|kinds%x|paths2^%d|steps2^%d", ctx->arch.c_str(),
             sizeof(R) == 4 ? "f32" : "f64", run->scheme, S.kinds_present, ilog2u64(S.path_first),
             ilog2u64(std::max<uint64_t>(S.max_steps, 1)));
    return key;
}

template <typename R>
static int jj_integrate_t(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run, R* theta,
                          int32_t* winding, R* v, double* acc, double* point_sums, int32_t* rec,
                          uint32_t rec_every, uint64_t rec_rows, hipStream_t stream)
{
    JJSetup<R> S;
    int st = jj_setup<R>(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, S);
    if (st) return st;
    if (rec) {
        if (rec_every == 0 || rec_every % 4 != 0)
            return fail(ctx, SDE_ERR_INVALID, "record_every must be a positive multiple of 4");
        if (!aligned(rec, 4)) return fail(ctx, SDE_ERR_INVALID, "misaligned record buffer");
        for (uint32_t q = 0; q < n_pts; ++q) {
            const uint64_t rows = (run->step0 + pts[q].n_steps) / rec_every - run->step0 / rec_every;
            if (rows > rec_rows)
                return fail(ctx, SDE_ERR_INVALID, "point %u needs %llu record rows, the buffer has %llu", q,
                            (unsigned long long)rows, (unsigned long long)rec_rows);
        }
    }

    if ((st = upload(ctx, kSlotJJLut, 2, S.lut.data(), S.lut.size() * sizeof(R), stream))) return st;
    JJLaunch L;
    jj_fill_args<R>(ctx, run, S, theta, winding, v, acc, point_sums, L);
    L.A.lut = ctx->ws[kSlotJJLut].ptr;
    L.A.rec = rec;
    L.A.rec_every = rec ? rec_every : 0u;
    const char* prec = sizeof(R) == 4 ? "f32" : "f64";

    // paths per lane: forced, cached, or tuned on this call's shape class
    int ppt = ctx->jj_ppt;
    if (sizeof(R) == 8 && ppt == 4) ppt = 2;
    if (!ppt) {
        const std::string key = jj_tune_key<R>(ctx, run, S);
        if (!tune_lookup(ctx, key, &ppt)) {
            ppt = 2;
            if (ctx->autotune) {
                const auto t0 = std::chrono::steady_clock::now();
                if ((st = jj_tune<R>(ctx, S.P, S.kinds, L, stream, &ppt))) return st;
                ctx->last.tuned = 1;
                ctx->last.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                tune_store(ctx, key, ppt);
            }
        }
    }
    L.ppt = ppt;
    JJPlan<R> plan;
    plan_items(S.P, S.kinds, ppt, plan);
    if ((st = jj_upload_plan(ctx, plan, stream, L))) return st;
    ctx->last.jj_paths_per_lane = ppt;
    ctx->last.work_items = plan.items.size();

    if ((st = run_recorded(ctx, jj_graph_key(prec, L), stream, [&](hipStream_t s) { return jj_record<R>(ctx, L, s); })))
        return st;
    if (run->sync) return sync_and_check(ctx, stream);
    return SDE_OK;
}

int jj_integrate_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                      float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                      hipStream_t stream)
{
    return jj_integrate_t<float>(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, nullptr, 0, 0, stream);
}

int jj_integrate_recorded_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                               float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                               uint32_t record_every, uint64_t n_rows, int32_t* rec_winding, hipStream_t stream)
{
    if (!rec_winding) return fail(ctx, SDE_ERR_INVALID, "null record buffer");
    return jj_integrate_t<float>(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, rec_winding,
                                 record_every, n_rows, stream);
}

int jj_integrate_f64_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                          double* theta, int32_t* winding, double* v, double* acc, double* point_sums,
                          hipStream_t stream)
{
    return jj_integrate_t<double>(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, nullptr, 0, 0, stream);
}

// ---------------------------------------------- the no-allocation variant --
// Device scratch of sde_jj_integrate_noalloc: the queue words, point table,
// work items, drive tables and per-chunk partial sums of one call, in
// 256-byte aligned sections.  Each GPU the library runs on holds its own copy
// until the process ends; every such call on that GPU uses it.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` per device (host code must never pass the
// array's own name to a kernel or a copy: on the host it is a stand-in).
static void* g_scratch_addr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

int noalloc_setup(sde_ctx* ctx)
{
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(ctx, SDE_ERR_UNSUPPORTED, "device %d: beyond the %d devices the library tracks", ctx->device,
                    kMaxDevices);
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_addr[ctx->device]) {
            void* ptr = nullptr;
            // the caller has made ctx->device current
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(ctx, SDE_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            g_scratch_addr[ctx->device] = ptr;
        }
        ctx->noalloc_scratch = g_scratch_addr[ctx->device];
    }
    // the host image of a call's tables is staged here (pinned, so the copy
    // is asynchronous); it is never larger than the scratch
    SDE_HIP(ctx, hipHostMalloc(&ctx->noalloc_staging, kNoAllocScratchBytes, hipHostMallocDefault));
    SDE_HIP(ctx, hipEventCreateWithFlags(&ctx->noalloc_done, hipEventDisableTiming));
    return SDE_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int jj_integrate_noalloc_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                              float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                              hipStream_t stream)
{
    if (!ctx->noalloc_scratch || !ctx->noalloc_staging || !ctx->noalloc_done)
        return fail(ctx, SDE_ERR_DEVICE, "the no-allocation scratch was not set up for this context");
    JJSetup<float> S;
    int st = jj_setup<float>(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, S);
    if (st) return st;
    // paths per lane: forced, else a choice the tuner cached, else 2; never
    // tuned here (tuning allocates)
    int ppt = ctx->jj_ppt;
    if (!ppt && !tune_lookup(ctx, jj_tune_key<float>(ctx, run, S), &ppt)) ppt = 2;
    JJPlan<float> plan;
    plan_items(S.P, S.kinds, ppt, plan);

    // layout of the scratch; the tables [o_pts, o_part) are one host image
    const size_t pts_bytes = plan.pts.size() * sizeof(JJPointDev);
    const size_t items_bytes = plan.items.size() * sizeof(JJItem);
    const size_t lut_bytes = S.lut.size() * sizeof(float);
    const size_t part_bytes = (size_t)std::max(plan.n_chunks, 1u) * 2 * sizeof(double);
    const size_t o_queue = 0;
    const size_t o_pts = align256(o_queue + kJJKinds * sizeof(uint32_t));
    const size_t o_items = align256(o_pts + pts_bytes);
    const size_t o_lut = align256(o_items + items_bytes);
    const size_t o_part = align256(o_lut + lut_bytes);
    const size_t need = o_part + part_bytes;
    if (need > kNoAllocScratchBytes)
        return fail(ctx, SDE_ERR_INVALID,
                    "sde_jj_integrate_noalloc: %u points in %u path chunks need %zu bytes of scratch, the maximum "
                    "is %zu",
                    n_pts, plan.n_chunks, need, (size_t)kNoAllocScratchBytes);

    // the previous call's copy may still read the staging buffer
    if (ctx->noalloc_pending) {
        SDE_HIP(ctx, hipEventSynchronize(ctx->noalloc_done));
        ctx->noalloc_pending = false;
    }
    unsigned char* img = static_cast<unsigned char*>(ctx->noalloc_staging);
    std::memcpy(img, plan.pts.data(), pts_bytes);
    std::memcpy(img + (o_items - o_pts), plan.items.data(), items_bytes);
    std::memcpy(img + (o_lut - o_pts), S.lut.data(), lut_bytes);
    unsigned char* base = static_cast<unsigned char*>(ctx->noalloc_scratch);
    SDE_HIP(ctx, hipMemcpyAsync(base + o_pts, img, o_part - o_pts, hipMemcpyHostToDevice, stream));
    SDE_HIP(ctx, hipEventRecord(ctx->noalloc_done, stream));
    ctx->noalloc_pending = true;

    JJLaunch L;
    jj_fill_args<float>(ctx, run, S, theta, winding, v, acc, point_sums, L);
    L.ppt = ppt;
    L.queues = reinterpret_cast<uint32_t*>(base + o_queue);
    L.A.pts = base + o_pts;
    L.A.items = reinterpret_cast<const JJItem*>(base + o_items);
    L.A.lut = base + o_lut;
    L.A.partials = reinterpret_cast<double*>(base + o_part);
    std::copy(plan.kind_begin, plan.kind_begin + kJJKinds + 1, L.kind_begin);
    L.n_items = (uint32_t)plan.items.size();
    L.n_pts = (uint32_t)plan.pts.size();
    if ((st = jj_grids<float>(ctx, L))) return st;
    ctx->last.jj_paths_per_lane = ppt;
    ctx->last.work_items = plan.items.size();
    if ((st = jj_record<float>(ctx, L, stream))) return st;
    if (run->sync) return sync_and_check(ctx, stream);
    return SDE_OK;
}

int debug_philox_impl(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b, uint64_t c0,
                      uint64_t n, uint32_t* out, hipStream_t stream)
{
    if (!out || n == 0) return fail(ctx, SDE_ERR_INVALID, "null output or zero blocks");
    if (!aligned(out, 4)) return fail(ctx, SDE_ERR_INVALID, "misaligned output");
    const uint64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return fail(ctx, SDE_ERR_INVALID, "too many blocks");
    hipLaunchKernelGGL(philox_dump_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (uint32_t)seed,
                       (uint32_t)(seed >> 32), tag, a, b, c0, n, out);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int debug_gauss_impl(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b, uint64_t n0,
                     uint64_t n, float* out, hipStream_t stream)
{
    if (!out || n == 0) return fail(ctx, SDE_ERR_INVALID, "null output or zero count");
    if (!aligned(out, 4)) return fail(ctx, SDE_ERR_INVALID, "misaligned output");
    const uint64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return fail(ctx, SDE_ERR_INVALID, "count too large");
    hipLaunchKernelGGL(gauss_dump_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (uint32_t)seed,
                       (uint32_t)(seed >> 32), tag, a, b, n0, n, out);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

}  // namespace sde
