// kuramoto_dense.hip -- Kuramoto model with a dense heterogeneous coupling
// matrix K_ij (Eq. 2).  Through the Eq. 3 identity applied row by row,
//   sum_j K_ij sin(phi_j - phi_i) = cos phi_i S_i - sin phi_i C_i,
//   [S | C] = K [sin Phi | cos Phi],
// so every drift evaluation of all R realizations is one matrix product of
// the N x N coupling matrix with the N x 2R matrix of stacked sines and
// cosines, followed by an elementwise update.  Each Heun stage is one kernel:
// the product, then in the epilogue the stage's update of the phases and the
// sin/cos operand of the next product (so the phases are never re-read to
// build it).
//
// Variants:
//  * FP32: LDS-tiled FP32 FMA product (VALU).
//  * BF16X3 / FP16X3: MFMA (v_mfma_f32_16x16x32_{bf16,f16}) with FP32
//    accumulation on a hi/lo split of both operands,
//       K B ~ K_hi B_hi + K_hi B_lo + K_lo B_hi,
//    x_hi = round16(x), x_lo = round16(x - x_hi); the dropped K_lo B_lo term
//    is ~2^-16 (bf16) / 2^-22 (fp16) of each product.  K is first scaled by an
//    exact power of two so its largest entry lies in [1, 2): the fp16 lo
//    parts then stay normal, and the scaling is undone exactly afterwards.
//
// Layouts (all in the context's workspace):
//   Khi, Klo : [Mp][Np] row-major 16-bit (rows padded to 128, columns to 32)
//   K32      : [Mp][Np] row-major FP32 (FP32 variant)
//   B        : [2 Rp][Np] column-major (a column is contiguous over j):
//              column (r / 32) * 64 + (r % 32) holds sin(2 pi theta_rj),
//              32 columns later cos; Rp = R rounded up to 32.  Two buffers
//              alternate between the stages.
// A workgroup owns 128 rows x 32 realizations (64 columns), so every lane
// holds S and C of the same (i, r) in its accumulators.  Workgroups are
// dealt to XCDs so that each XCD sweeps a contiguous band of rows over all
// columns: its slice of K is read from HBM/MALL once per product and the
// whole B stays in its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "kuramoto_common.h"
#include "sde_internal.h"

namespace sde {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kDenseThreads = 256;
constexpr uint32_t kRowTile = 128;
constexpr uint32_t kRealTile = 32;
constexpr uint32_t kKStep = 32;

struct DenseArgs {
    const void* Ahi;       // [Mp][Np] 16-bit split of the scaled K, or FP32 K (A32)
    const void* Alo;
    const void* Bhi;       // [2Rp][Np] current sin/cos operand (16-bit split or FP32)
    const void* Blo;
    void* Bhi_next;        // operand for the next product
    void* Blo_next;
    const float* src;      // [R][N] phases the drift is evaluated at
    const float* base;     // [R][N] phases at the start of the step
    float* dst;            // [R][N] output phases
    float* F1;             // [R][N] stage-1 drift
    const float* omega;    // [N]
    const float* scale;    // device: {scale, 1/scale}
    uint32_t N, R, Np, Rp, Mp;
    const uint64_t* nbase; // device: absolute step of the current chunk's first step
    uint32_t k;            // step within the chunk
    uint32_t key0, key1;
    float omega_scale, hdt2pi, c2;
    int32_t stage;         // 1 predictor (or Euler step), 2 corrector
    int32_t euler;
};

__device__ __forceinline__ uint32_t bcol(uint32_t r, uint32_t kind)
{
    return (r / kRealTile) * (2 * kRealTile) + kind * kRealTile + (r % kRealTile);
}

template <typename T>
__device__ __forceinline__ void store_split(void* hi, void* lo, uint64_t idx, float x)
{
    const T h = (T)x;
    static_cast<T*>(hi)[idx] = h;
    static_cast<T*>(lo)[idx] = (T)(x - (float)h);
}

// The stage update of oscillator i of realization r given S = sum_j K_ij
// sin phi_j and C = sum_j K_ij cos phi_j; also writes the next operand.
template <typename T>
__device__ __forceinline__ void dense_update(const DenseArgs& A, uint32_t i, uint32_t r, float S, float C)
{
    const uint64_t gi = (uint64_t)r * A.N + i;
    const float ts = A.src[gi];
    const float F = fmaf(cos_rev(ts), S, fmaf(-sin_rev(ts), C, A.omega[i]));
    const uint64_t n = load_uniform(A.nbase) + A.k;
    float g[4];
    gauss4_scaled(U4{(uint32_t)(n >> 2), i, r, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2, g);
    const uint32_t j = (uint32_t)n & 3u;
    const float ns = j == 0 ? g[0] : j == 1 ? g[1] : j == 2 ? g[2] : g[3];
    const float th = A.base[gi];
    float t;
    if (A.stage == 1) {
        t = fmaf(A.omega_scale, F, th) + ns;
        if (A.euler)
            t -= floorf(t);
        else
            A.F1[gi] = F;
    } else {
        t = fmaf(A.hdt2pi, A.F1[gi] + F, th) + ns;
        t -= floorf(t);
    }
    A.dst[gi] = t;
    const uint64_t cs = (uint64_t)bcol(r, 0) * A.Np + i, cc = (uint64_t)bcol(r, 1) * A.Np + i;
    if constexpr (sizeof(T) == 4) {
        static_cast<float*>(A.Bhi_next)[cs] = sin_rev(t);
        static_cast<float*>(A.Bhi_next)[cc] = cos_rev(t);
    } else {
        store_split<T>(A.Bhi_next, A.Blo_next, cs, sin_rev(t));
        store_split<T>(A.Bhi_next, A.Blo_next, cc, cos_rev(t));
    }
}

// workgroup -> (row tile, realization tile); XCD-aware when the row tiles
// split evenly over the 8 XCDs.
__device__ __forceinline__ void tile_of(uint32_t b, uint32_t n_mt, uint32_t n_nt, uint32_t& mt, uint32_t& nt)
{
    if (n_mt % 8 == 0) {
        const uint32_t x = b & 7u, l = b >> 3;
        mt = x * (n_mt / 8) + l / n_nt;
        nt = l % n_nt;
    } else {
        mt = b / n_nt;
        nt = b % n_nt;
    }
}

// ------------------------------------------------------- split MFMA -------
template <typename T, typename V>
__device__ __forceinline__ f32x4 mfma16(V a, V b, f32x4 c)
{
    if constexpr (sizeof(T) == 2 && __is_same(T, __bf16))
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <typename T, typename V>
__global__ __launch_bounds__(kDenseThreads) void dense_mfma_kernel(DenseArgs A)
{
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, mt, nt);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t wr = wave >> 1, wc = wave & 1u;
    const uint32_t row0 = mt * kRowTile + wr * 64;      // 4 sub-tiles of 16 rows
    const uint32_t csin = nt * 2 * kRealTile + wc * 16 + (lane & 15u);
    const uint32_t ccos = csin + kRealTile;
    const uint32_t kofs = 8 * (lane >> 4);
    const T* Ahi = static_cast<const T*>(A.Ahi);
    const T* Alo = static_cast<const T*>(A.Alo);
    const T* Bhi = static_cast<const T*>(A.Bhi);
    const T* Blo = static_cast<const T*>(A.Blo);
    const uint64_t Np = A.Np;
    const T* pa_hi = Ahi + (uint64_t)(row0 + (lane & 15u)) * Np + kofs;
    const T* pa_lo = Alo + (uint64_t)(row0 + (lane & 15u)) * Np + kofs;
    const T* pbs_hi = Bhi + (uint64_t)csin * Np + kofs;
    const T* pbs_lo = Blo + (uint64_t)csin * Np + kofs;
    const T* pbc_hi = Bhi + (uint64_t)ccos * Np + kofs;
    const T* pbc_lo = Blo + (uint64_t)ccos * Np + kofs;

    f32x4 accS[4], accC[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        accS[m] = f32x4{0.f, 0.f, 0.f, 0.f};
        accC[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    V ah[4], al[4], bsh, bsl, bch, bcl;
    auto load = [&](uint32_t k0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            ah[m] = *reinterpret_cast<const V*>(pa_hi + (uint64_t)m * 16 * Np + k0);
            al[m] = *reinterpret_cast<const V*>(pa_lo + (uint64_t)m * 16 * Np + k0);
        }
        bsh = *reinterpret_cast<const V*>(pbs_hi + k0);
        bsl = *reinterpret_cast<const V*>(pbs_lo + k0);
        bch = *reinterpret_cast<const V*>(pbc_hi + k0);
        bcl = *reinterpret_cast<const V*>(pbc_lo + k0);
    };
    load(0);
    for (uint32_t k0 = 0; k0 < A.Np; k0 += kKStep) {
        V cah[4], cal[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            cah[m] = ah[m];
            cal[m] = al[m];
        }
        const V cbsh = bsh, cbsl = bsl, cbch = bch, cbcl = bcl;
        if (k0 + kKStep < A.Np) load(k0 + kKStep);  // prefetch the next k step
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            accS[m] = mfma16<T, V>(cah[m], cbsh, accS[m]);
            accC[m] = mfma16<T, V>(cah[m], cbch, accC[m]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            accS[m] = mfma16<T, V>(cah[m], cbsl, accS[m]);
            accC[m] = mfma16<T, V>(cah[m], cbcl, accC[m]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            accS[m] = mfma16<T, V>(cal[m], cbsh, accS[m]);
            accC[m] = mfma16<T, V>(cal[m], cbch, accC[m]);
        }
    }
    const float inv = A.scale[1];
    const uint32_t r = nt * kRealTile + wc * 16 + (lane & 15u);
    if (r >= A.R) return;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = row0 + m * 16 + 4 * (lane >> 4) + q;
            if (i < A.N) dense_update<T>(A, i, r, accS[m][q] * inv, accC[m][q] * inv);
        }
    }
}

// ------------------------------------------------------------ FP32 SIMT ---
// 256 lanes, tile 128 rows x 32 realizations, k step 16 through LDS; each
// lane accumulates 8 rows x (2 realizations x {sin, cos}).
constexpr uint32_t kF32K = 16;

__global__ __launch_bounds__(kDenseThreads) void dense_fp32_kernel(DenseArgs A)
{
    __shared__ float As[kF32K][kRowTile + 4];
    __shared__ float Bs[kF32K][2 * kRealTile + 4];
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, mt, nt);
    const uint32_t tx = threadIdx.x & 15u, ty = threadIdx.x >> 4;  // 16 x 16
    const float* K32 = static_cast<const float*>(A.Ahi);
    const float* B32 = static_cast<const float*>(A.Bhi);
    const uint64_t Np = A.Np;
    float accS[8][2], accC[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) accS[a][b] = accC[a][b] = 0.f;
    // global -> LDS assignment: A tile 128 x 16 = 512 float4 (2 per lane),
    // B tile 64 cols x 16 = 256 float4 (1 per lane)
    const uint32_t arow = threadIdx.x >> 2, akq = (threadIdx.x & 3u) * 4;
    const uint32_t bcolv = threadIdx.x >> 2, bkq = (threadIdx.x & 3u) * 4;
    const float* pa0 = K32 + (uint64_t)(mt * kRowTile + arow) * Np + akq;
    const float* pa1 = pa0 + 64 * Np;
    const float* pb = B32 + (uint64_t)(nt * 2 * kRealTile + bcolv) * Np + bkq;
    for (uint32_t k0 = 0; k0 < A.Np; k0 += kF32K) {
        const float4 a0 = *reinterpret_cast<const float4*>(pa0 + k0);
        const float4 a1 = *reinterpret_cast<const float4*>(pa1 + k0);
        const float4 b0 = *reinterpret_cast<const float4*>(pb + k0);
        __syncthreads();
        As[akq + 0][arow] = a0.x;
        As[akq + 1][arow] = a0.y;
        As[akq + 2][arow] = a0.z;
        As[akq + 3][arow] = a0.w;
        As[akq + 0][arow + 64] = a1.x;
        As[akq + 1][arow + 64] = a1.y;
        As[akq + 2][arow + 64] = a1.z;
        As[akq + 3][arow + 64] = a1.w;
        Bs[bkq + 0][bcolv] = b0.x;
        Bs[bkq + 1][bcolv] = b0.y;
        Bs[bkq + 2][bcolv] = b0.z;
        Bs[bkq + 3][bcolv] = b0.w;
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < kF32K; ++k) {
            float a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] = As[k][ty * 8 + q];
            const float s0 = Bs[k][2 * tx], s1 = Bs[k][2 * tx + 1];
            const float c0 = Bs[k][kRealTile + 2 * tx], c1 = Bs[k][kRealTile + 2 * tx + 1];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                accS[q][0] = fmaf(a[q], s0, accS[q][0]);
                accS[q][1] = fmaf(a[q], s1, accS[q][1]);
                accC[q][0] = fmaf(a[q], c0, accC[q][0]);
                accC[q][1] = fmaf(a[q], c1, accC[q][1]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const uint32_t r = nt * kRealTile + 2 * tx + b;
        if (r >= A.R) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t i = mt * kRowTile + ty * 8 + q;
            if (i < A.N) dense_update<float>(A, i, r, accS[q][b], accC[q][b]);
        }
    }
}

// ----------------------------------------------------------- preparation --
// max |K_ij| as the bit pattern of a non-negative float (order-independent max).
__global__ void dense_maxabs_kernel(const float* K, uint64_t n, uint32_t* out)
{
    uint32_t m = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(fabsf(K[i])));
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

__global__ void dense_zero_kernel(uint32_t* p) { *p = 0u; }

// scale = 2^-floor(log2 max|K|): the largest scaled entry lies in [1, 2).
__global__ void dense_scale_kernel(const uint32_t* maxbits, float* scale, int unit)
{
    float s = 1.f;
    const float m = __uint_as_float(*maxbits);
    if (!unit && m > 0.f && isfinite(m)) s = ldexpf(1.f, -ilogbf(m));
    scale[0] = s;
    scale[1] = 1.f / s;
}

// K -> padded [Mp][Np] scaled copy: 16-bit hi/lo split, or FP32.
template <typename T>
__global__ void dense_split_kernel(const float* K, uint32_t N, uint32_t Np, uint32_t Mp, const float* scale,
                                   void* hi, void* lo)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)Mp * Np) return;
    const uint32_t i = (uint32_t)(g / Np), j = (uint32_t)(g % Np);
    const float x = (i < N && j < N) ? K[(uint64_t)i * N + j] * scale[0] : 0.f;
    if constexpr (sizeof(T) == 4)
        static_cast<float*>(hi)[g] = x;
    else
        store_split<T>(hi, lo, g, x);
}

// theta [R][N] -> sin/cos operand [2Rp][Np] (zero in the padding).
template <typename T>
__global__ void dense_operand_kernel(const float* theta, uint32_t N, uint32_t R, uint32_t Np, uint32_t Rp, void* hi,
                                     void* lo)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)Rp * Np) return;
    const uint32_t r = (uint32_t)(g / Np), j = (uint32_t)(g % Np);
    float s = 0.f, c = 0.f;
    if (r < R && j < N) {
        const float t = theta[(uint64_t)r * N + j];
        s = sin_rev(t);
        c = cos_rev(t);
    }
    const uint64_t cs = (uint64_t)bcol(r, 0) * Np + j, cc = (uint64_t)bcol(r, 1) * Np + j;
    if constexpr (sizeof(T) == 4) {
        static_cast<float*>(hi)[cs] = s;
        static_cast<float*>(hi)[cc] = c;
    } else {
        store_split<T>(hi, lo, cs, s);
        store_split<T>(hi, lo, cc, c);
    }
}

// ------------------------------------------------------------------ host --

template <typename T>
static int dense_run_typed(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                           const float* omega, const float* K, double* r_samples, uint64_t n_samples, uint32_t M,
                           hipStream_t stream)
{
    const KuraConsts kc = kuramoto_consts(d);
    const uint32_t N = d->N, R = d->R;
    const uint32_t Np = (N + kKStep - 1) / kKStep * kKStep;
    const uint32_t Mp = (N + kRowTile - 1) / kRowTile * kRowTile;
    const uint32_t Rp = (R + kRealTile - 1) / kRealTile * kRealTile;
    const uint64_t NR = (uint64_t)N * R;
    const size_t esz = sizeof(T);
    const bool split = esz == 2;
    const size_t a_bytes = (size_t)Mp * Np * esz;
    const size_t b_bytes = (size_t)2 * Rp * Np * esz;
    void *wa = nullptr, *wb = nullptr, *wk = nullptr;
    int st;
    if ((st = ensure_ws(ctx, kSlotDenseA, a_bytes * (split ? 2 : 1), &wa))) return st;
    if ((st = ensure_ws(ctx, kSlotDenseB, b_bytes * (split ? 4 : 2) + 64, &wb))) return st;
    if ((st = ensure_ws(ctx, kSlotKuraWork, (size_t)2 * NR * sizeof(float), &wk))) return st;
    char* A0 = static_cast<char*>(wa);
    char* B0 = static_cast<char*>(wb);
    void* Ahi = A0;
    void* Alo = split ? A0 + a_bytes : nullptr;
    void* Bcur_hi = B0;
    void* Bcur_lo = split ? B0 + b_bytes : nullptr;
    void* Bnext_hi = B0 + b_bytes * (split ? 2 : 1);
    void* Bnext_lo = split ? B0 + b_bytes * 3 : nullptr;
    float* scale = reinterpret_cast<float*>(B0 + b_bytes * (split ? 4 : 2));
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(scale + 2);
    float* tilde = static_cast<float*>(wk);
    float* F1 = tilde + NR;

    // scaled, padded copy of K (split into hi/lo for the MFMA variants)
    hipLaunchKernelGGL(dense_zero_kernel, dim3(1), dim3(1), 0, stream, maxbits);
    if (split) hipLaunchKernelGGL(dense_maxabs_kernel, dim3(1024), dim3(256), 0, stream, K, (uint64_t)N * N, maxbits);
    hipLaunchKernelGGL(dense_scale_kernel, dim3(1), dim3(1), 0, stream, maxbits, scale, split ? 0 : 1);
    hipLaunchKernelGGL(dense_split_kernel<T>, dim3((uint32_t)(((uint64_t)Mp * Np + 255) / 256)), dim3(256), 0, stream,
                       K, N, Np, Mp, scale, Ahi, Alo);
    // both operand buffers get their zero padding (rows j >= N, columns of
    // realizations r >= R) here; the epilogues only ever write the live part
    for (int b = 0; b < 2; ++b)
        hipLaunchKernelGGL(dense_operand_kernel<T>, dim3((uint32_t)(((uint64_t)Rp * Np + 255) / 256)), dim3(256), 0,
                           stream, phi, N, R, Np, Rp, b ? Bnext_hi : Bcur_hi, b ? Bnext_lo : Bcur_lo);
    SDE_HIP(ctx, hipGetLastError());

    DenseArgs A;
    A.Ahi = Ahi;
    A.Alo = Alo;
    A.omega = omega;
    A.scale = scale;
    A.N = N;
    A.R = R;
    A.Np = Np;
    A.Rp = Rp;
    A.Mp = Mp;
    A.key0 = (uint32_t)run->seed;
    A.key1 = (uint32_t)(run->seed >> 32);
    A.omega_scale = kc.omega_scale;
    A.hdt2pi = kc.hdt2pi;
    A.c2 = kc.c2;
    A.F1 = F1;
    A.euler = run->scheme == SDE_EULER;
    const dim3 grid((Mp / kRowTile) * (Rp / kRealTile));
    uint64_t* nbase = nullptr;
    if ((st = step_counter(ctx, &nbase))) return st;
    A.nbase = nbase;
    auto launch = [&](hipStream_t s) -> int {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL(dense_fp32_kernel, grid, dim3(kDenseThreads), 0, s, A);
        else if constexpr (__is_same(T, __bf16))
            hipLaunchKernelGGL((dense_mfma_kernel<__bf16, bf16x8>), grid, dim3(kDenseThreads), 0, s, A);
        else
            hipLaunchKernelGGL((dense_mfma_kernel<_Float16, f16x8>), grid, dim3(kDenseThreads), 0, s, A);
        SDE_HIP(ctx, hipGetLastError());
        return SDE_OK;
    };
    // `count` steps from the device step base, then advance it.  The operand
    // buffers alternate per stage; chunks hold an even number of stages so a
    // recorded chunk always starts from the same buffer.
    void* Bb_hi[2] = {Bcur_hi, Bnext_hi};
    void* Bb_lo[2] = {Bcur_lo, Bnext_lo};
    auto record = [&](hipStream_t s, uint32_t count) -> int {
        if (r_samples) launch_order_parameter_at(phi, N, R, r_samples, n_samples, nbase, run->step0, M, s);
        int cur = 0;
        for (uint32_t k = 0; k < count; ++k) {
            A.k = k;
            // stage 1: drift at theta_n; Euler finishes the step in place
            A.stage = 1;
            A.Bhi = Bb_hi[cur];
            A.Blo = Bb_lo[cur];
            A.Bhi_next = Bb_hi[cur ^ 1];
            A.Blo_next = Bb_lo[cur ^ 1];
            A.src = phi;
            A.base = phi;
            A.dst = A.euler ? phi : tilde;
            int e = launch(s);
            if (e) return e;
            cur ^= 1;
            if (A.euler) continue;
            // stage 2: drift at the predictor; corrector into phi
            A.stage = 2;
            A.Bhi = Bb_hi[cur];
            A.Blo = Bb_lo[cur];
            A.Bhi_next = Bb_hi[cur ^ 1];
            A.Blo_next = Bb_lo[cur ^ 1];
            A.src = tilde;
            A.base = phi;
            A.dst = phi;
            if ((e = launch(s))) return e;
            cur ^= 1;
        }
        launch_step_advance(nbase, count, s);
        SDE_HIP(ctx, hipGetLastError());
        return SDE_OK;
    };
    launch_step_set(nbase, run->step0, stream);
    const uint32_t C = chunk_steps(M, d->n_steps, A.euler != 0);
    char key[320];
    snprintf(key, sizeof key, "dense%d|%p|%p|%p|%p|%p|%p|%u|%u|%u|%u|%a|%a|%a|%d|%llu|%u|%llu", d->coupling,
             (void*)phi, (void*)omega, (void*)r_samples, wa, wb, wk, N, R, A.key0, A.key1, A.omega_scale, A.hdt2pi,
             A.c2, A.euler, (unsigned long long)run->step0, M, (unsigned long long)n_samples);
    const uint64_t full = d->n_steps / C, rem = d->n_steps % C;
    for (uint64_t c = 0; c < full; ++c)
        if ((st = run_recorded(ctx, std::string(key) + "|C" + std::to_string(C), stream,
                               [&](hipStream_t s) { return record(s, C); })))
            return st;
    if (rem && (st = run_recorded(ctx, std::string(key) + "|C" + std::to_string(rem), stream,
                                  [&](hipStream_t s) { return record(s, (uint32_t)rem); })))
        return st;
    if (r_samples) launch_order_parameter_at(phi, N, R, r_samples, n_samples, nbase, run->step0, M, stream);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int dense_impl(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi, const float* omega,
               const float* K, double* r_samples, uint64_t n_samples, uint32_t M, hipStream_t stream)
{
    switch (d->coupling) {
    case SDE_DENSE_FP32: return dense_run_typed<float>(ctx, d, run, phi, omega, K, r_samples, n_samples, M, stream);
    case SDE_DENSE_BF16X3: return dense_run_typed<__bf16>(ctx, d, run, phi, omega, K, r_samples, n_samples, M, stream);
    default: return dense_run_typed<_Float16>(ctx, d, run, phi, omega, K, r_samples, n_samples, M, stream);
    }
}

}  // namespace sde
