// mlp.hip -- ensemble MLP surrogate of the mean velocity <v> of the
// Josephson junction: training (forward, back-propagation, MSE, Adam) and
// inference with hand-written FP32 kernels, and the scan that falls back to
// the integrator where the ensemble disagrees.
//
// Training works on minibatches of B samples for all members at once
// (grid.z = member).  One tiled kernel serves the three products of a layer
// -- forward Z = A W^T + b, weight gradient dW = dZ^T A, input gradient
// dA = dZ W -- on the FP32 matrix cores (v_mfma_f32_16x16x4_f32; 64 x 64
// tiles staged through LDS in 16-k slices, a 32 x 32 quarter per wave), with
// the bias/GELU (forward) and GELU' (backward) applied in its epilogue.  A
// whole epoch of steps is recorded once as a HIP graph; the Adam step count
// is read from a device counter so the same graph replays every epoch.
//
// Inference is one fused kernel for all members (mlp_infer_mfma_kernel):
// the hidden weights are packed once per call into the fragment layout of
// the FP32 MFMA (a 16 x 16 block per 1 KB run); a workgroup takes 64 queries
// whose activations stay in LDS in the operand layout of the next layer,
// each of its 4 waves computes 16 queries x all 256 outputs of a layer on
// v_mfma_f32_16x16x4_f32 with the weights streamed from L2, bias and GELU
// write the next operand, and the output layer, the members' mean and their
// sample standard deviation follow.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <new>
#include <numeric>
#include <random>

#include "device_common.h"
#include "sde_internal.h"

struct sde_surrogate {
    sde_ctx* ctx = nullptr;
    std::vector<uint32_t> widths;
    std::vector<uint64_t> w_off, b_off;  // offsets of W_l, b_l in a member's packed parameters
    uint32_t members = 0;
    uint64_t P = 0;                      // parameters per member
    float* params = nullptr;             // device [members][P]
    float* grads = nullptr;              // device [members][P]
    float* adam_m = nullptr;             // device [members][P]
    float* adam_v = nullptr;
    uint64_t* adam_t = nullptr;          // device [members] Adam step counts
    sde_surrogate_scaling sc{};
    // training workspace
    float* work = nullptr;
    size_t work_bytes = 0;
    uint32_t* perm = nullptr;            // device [members][n] sample order of the epoch
    size_t perm_cap = 0;
    // inference: hidden-layer weights in the FP32 MFMA operand layout
    float* packed = nullptr;
    size_t packed_bytes = 0;
};

namespace sde {

constexpr uint32_t kTagMlpInit = 5;
constexpr int kMaxLayers = 8;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ------------------------------------------------------------ parameters --
struct InitArgs {
    float* params;
    uint64_t P;
    uint32_t members;
    uint32_t n_layers;
    uint64_t layer_end[kMaxLayers];  // packed offset where layer l's (W, b) ends
    float bound[kMaxLayers];         // 1 / sqrt(fan_in)
    uint32_t key0, key1;
};

__global__ void mlp_init_kernel(InitArgs A)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= A.P * A.members) return;
    const uint32_t m = (uint32_t)(g / A.P);
    const uint64_t k = g % A.P;
    uint32_t l = 0;
    while (l + 1 < A.n_layers && k >= A.layer_end[l]) ++l;
    const U4 x = philox4x32_10(U4{(uint32_t)(k >> 2), m, 0u, kTagMlpInit}, A.key0, A.key1);
    const uint32_t w = (k & 3) == 0 ? x.x : (k & 3) == 1 ? x.y : (k & 3) == 2 ? x.z : x.w;
    const float u = (float)(w >> 8) * 0x1p-24f;
    A.params[g] = A.bound[l] * (2.f * u - 1.f);
}

// ------------------------------------------------------------- features --
struct NormArgs {
    const float* X;          // [n][w0] raw features
    const float* y;          // [n] targets or null
    float* Xn;               // [n][w0]
    float* yn;               // [n] or null
    uint64_t n;
    uint32_t w0;
    sde_surrogate_scaling sc;
};

__global__ void mlp_normalize_kernel(NormArgs A)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    for (uint32_t j = 0; j < A.w0; ++j)
        A.Xn[i * A.w0 + j] = (A.X[i * A.w0 + j] - A.sc.in_center[j]) / A.sc.in_scale[j];
    if (A.y) {
        float t = A.y[i];
        if (A.sc.target_over_omega) t /= A.X[i * A.w0 + 1];
        A.yn[i] = (t - A.sc.out_mean) / A.sc.out_std;
    }
}

// --------------------------------------------------------------- GEMMs ----
// C[M][N] = sum_k opA(m, k) opB(k, n) over the members in grid.z.
//  FWD: opA = X[rows ? rows[m] : m][k] (ld = K), opB = W[n][k]; epilogue
//       Z = acc + b[n], A_out = GELU(Z) (or Z for the output layer)
//  DW:  opA = dZ[k][m] (ld = M), opB = A[k][n] (ld = N); C = dW
//  DX:  opA = dZ[m][k] (ld = K), opB = W[k][n] (ld = N); epilogue
//       dZ_prev = acc * GELU'(Z_prev)
enum { kFwd = 0, kDW = 1, kDX = 2 };
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;   // tile
constexpr int kGK = 16;   // k step

struct GemmArgs {
    const float* A;  uint64_t a_mstride;   // member strides in elements
    const float* B;  uint64_t b_mstride;
    float* C;        uint64_t c_mstride;
    float* C2;       uint64_t c2_mstride;  // FWD: activation output
    const float* bias; uint64_t bias_mstride;
    const float* Zp;   uint64_t zp_mstride;  // DX: pre-activation of the previous layer
    const uint32_t* rows; uint64_t rows_mstride;  // FWD first layer: gathered sample rows
    uint32_t rows_offset;                   // first row of this minibatch in rows
    uint32_t M, N, K;
    int32_t last;                           // FWD: output layer (no GELU)
    uint32_t kslices;                       // DW: the k range is split over grid.z = member *
                                            // kslices + slice; slice s writes the M x N partial
                                            // C + member * c_mstride + s * M * N (summed later)
};

// The k range of slice ks of kslices, in whole k steps.
__device__ __forceinline__ void k_range(uint32_t K, uint32_t kslices, uint32_t ks, uint32_t& k_begin, uint32_t& k_end)
{
    const uint32_t per = ((K + kslices - 1) / kslices + kGK - 1) / kGK * kGK;
    k_begin = min(K, ks * per);
    k_end = min(K, k_begin + per);
}

template <int MODE>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g)
{
    __shared__ float As[kGK][kGT + 1];
    __shared__ float Bs[kGK][kGT + 1];
    const uint32_t ksl = MODE == kDW ? g.kslices : 1u;
    const uint32_t mem = blockIdx.z / ksl, ks = blockIdx.z % ksl;
    const float* A = g.A + mem * g.a_mstride;
    const float* B = g.B + mem * g.b_mstride;
    const uint32_t m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1u;
    uint32_t kb = 0, ke = g.K;
    if (MODE == kDW) k_range(g.K, ksl, ks, kb, ke);
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (uint32_t k0 = kb; k0 < ke; k0 += kGK) {
        // 64 x 16 elements of each operand, 4 per lane
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t idx = threadIdx.x + 256 * e;  // 0..1023
            const uint32_t kk = idx & 15u, mm = idx >> 4; // for k-contiguous loads
            const uint32_t mm2 = idx & 63u, kk2 = idx >> 6; // for m-contiguous loads
            float va = 0.f, vb = 0.f;
            if (MODE == kFwd || MODE == kDX) {
                const uint32_t m = m0 + mm, k = k0 + kk;
                if (m < g.M && k < g.K) {
                    uint64_t row = m;
                    if (MODE == kFwd && g.rows) row = g.rows[mem * g.rows_mstride + g.rows_offset + m];
                    va = A[row * g.K + k];
                }
                As[kk][mm] = va;
            } else {
                const uint32_t m = m0 + mm2, k = k0 + kk2;
                if (m < g.M && k < ke) va = A[(uint64_t)k * g.M + m];
                As[kk2][mm2] = va;
            }
            if (MODE == kFwd) {
                const uint32_t n = n0 + mm, k = k0 + kk;
                if (n < g.N && k < g.K) vb = B[(uint64_t)n * g.K + k];
                Bs[kk][mm] = vb;
            } else {
                const uint32_t n = n0 + mm2, k = k0 + kk2;
                if (n < g.N && k < ke) vb = B[(uint64_t)k * g.N + n];
                Bs[kk2][mm2] = vb;
            }
        }
        __syncthreads();
        // wave (wm, wn) takes the 32 x 32 quarter of the tile: 2 x 2 blocks of
        // v_mfma_f32_16x16x4_f32, lane l reading A[m = l % 16][k = l / 16] and
        // B[k = l / 16][n = l % 16] of each 4-k group from the LDS slices
#pragma unroll
        for (int kg = 0; kg < kGK / 4; ++kg) {
            const uint32_t k = kg * 4 + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = As[k][wm * 32 + i * 16 + (lane & 15u)];
                b[i] = Bs[k][wn * 32 + i * 16 + (lane & 15u)];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane l holds rows 4 (l / 16) + q, column l % 16 of each block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + q;
                const uint32_t n = n0 + wn * 32 + j * 16 + (lane & 15u);
                if (m >= g.M || n >= g.N) continue;
                const uint64_t o = (uint64_t)m * g.N + n;
                const float v = acc[i][j][q];
                if (MODE == kFwd) {
                    const float z = v + g.bias[mem * g.bias_mstride + n];
                    g.C[mem * g.c_mstride + o] = z;
                    g.C2[mem * g.c2_mstride + o] = g.last ? z : gelu(z);
                } else if (MODE == kDW) {
                    g.C[mem * g.c_mstride + (uint64_t)ks * g.M * g.N + o] = v;
                } else {
                    g.C[mem * g.c_mstride + o] = v * gelu_grad(g.Zp[mem * g.zp_mstride + o]);
                }
            }
}

// dW of the first layer: dW[o][j] = sum_b dZ[b][o] Xn[rows[b]][j] (gathered input rows).
__global__ __launch_bounds__(256) void mlp_gemm_dw_gather_kernel(GemmArgs g)
{
    __shared__ float As[kGK][kGT + 1];
    __shared__ float Bs[kGK][kGT + 1];
    const uint32_t mem = blockIdx.z / g.kslices, ks = blockIdx.z % g.kslices;
    const float* A = g.A + mem * g.a_mstride;
    const uint32_t m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const uint32_t tx = threadIdx.x & 15u, ty = threadIdx.x >> 4;
    uint32_t kb, ke;
    k_range(g.K, g.kslices, ks, kb, ke);
    float acc[4][4] = {};
    for (uint32_t k0 = kb; k0 < ke; k0 += kGK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t idx = threadIdx.x + 256 * e;
            const uint32_t mm2 = idx & 63u, kk2 = idx >> 6;
            const uint32_t k = k0 + kk2;
            const uint32_t m = m0 + mm2, n = n0 + mm2;
            As[kk2][mm2] = (m < g.M && k < ke) ? A[(uint64_t)k * g.M + m] : 0.f;
            float vb = 0.f;
            if (n < g.N && k < ke) {
                const uint64_t row = g.rows ? g.rows[mem * g.rows_mstride + g.rows_offset + k] : k;
                vb = g.B[row * g.N + n];
            }
            Bs[kk2][mm2] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kGK; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[k][ty * 4 + i];
                b[i] = Bs[k][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t m = m0 + ty * 4 + i;
        if (m >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t n = n0 + tx * 4 + j;
            if (n < g.N) g.C[mem * g.c_mstride + (uint64_t)ks * g.M * g.N + (uint64_t)m * g.N + n] = acc[i][j];
        }
    }
}


// db[n] = sum_b dZ[b][n] in two passes with a fixed order: slices of
// kColSlice rows summed in parallel (grid.y = slice), then the slice sums in
// slice order.  One thread per column walking all B rows alone leaves a few
// workgroups waiting out one load latency per row.
constexpr uint32_t kColSlice = 64;

__global__ void mlp_colsum_slices_kernel(const float* dZ, uint64_t dz_mstride, float* part, uint32_t B, uint32_t N)
{
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t sl = blockIdx.y, mem = blockIdx.z;
    if (n >= N) return;
    const float* p = dZ + mem * dz_mstride;
    const uint32_t b0 = sl * kColSlice, b1 = min(B, b0 + kColSlice);
    float s = 0.f;
#pragma unroll 16
    for (uint32_t b = b0; b < b1; ++b) s += p[(uint64_t)b * N + n];
    part[((uint64_t)mem * gridDim.y + sl) * N + n] = s;
}

// dW = sum of the k-slice partials of a split weight-gradient product, in
// slice order: part[member][slice][MN] -> out + member * out_mstride.
__global__ void mlp_ksum_kernel(const float* part, uint32_t kslices, uint64_t MN, float* out, uint64_t out_mstride)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mem = blockIdx.y;
    if (i >= MN) return;
    const float* p = part + (uint64_t)mem * kslices * MN + i;
    float s = 0.f;
    for (uint32_t k = 0; k < kslices; ++k) s += p[(uint64_t)k * MN];
    out[mem * out_mstride + i] = s;
}

__global__ void mlp_colsum_kernel(const float* part, uint32_t n_slices, float* db, uint64_t db_mstride, uint32_t N)
{
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mem = blockIdx.y;
    if (n >= N) return;
    const float* p = part + (uint64_t)mem * n_slices * N + n;
    float s = 0.f;
    for (uint32_t sl = 0; sl < n_slices; ++sl) s += p[(uint64_t)sl * N];
    db[mem * db_mstride + n] = s;
}

// dZ_L = 2 (y - t) / B for the output layer; loss = mean (y - t)^2 (FP64
// block sum, one workgroup per member).
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* y, uint64_t y_mstride, const float* t,
                                                       const uint32_t* rows, uint64_t rows_mstride,
                                                       uint32_t rows_offset, float* dZ, uint64_t dz_mstride,
                                                       uint32_t B, float* loss, uint32_t loss_slot,
                                                       uint32_t loss_stride)
{
    __shared__ double lds[4];
    const uint32_t mem = blockIdx.x;
    double s = 0.0;
    for (uint32_t b = threadIdx.x; b < B; b += 256) {
        const uint32_t row = rows ? rows[mem * rows_mstride + rows_offset + b] : b;
        const float r = y[mem * y_mstride + b] - t[row];
        dZ[mem * dz_mstride + b] = 2.f * r / (float)B;
        s += (double)r * (double)r;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63u) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && loss) loss[(uint64_t)mem * loss_stride + loss_slot] = (float)((lds[0] + lds[1] + lds[2] + lds[3]) / B);
}

// One Adam step (bias-corrected) of every parameter; the step count of the
// member is read from (and, by the last lane, advanced in) device memory.
struct AdamArgs {
    float* p; float* g; float* m; float* v;
    uint64_t* t;         // [members], incremented by the advance kernel
    uint64_t P;
    uint32_t members;
    float lr, b1, b2, eps;
};

__global__ void mlp_adam_kernel(AdamArgs A)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.P * A.members) return;
    const uint32_t mem = (uint32_t)(i / A.P);
    const double t = (double)(A.t[mem] + 1);
    const float bc1 = (float)(1.0 - pow((double)A.b1, t));
    const float bc2 = (float)(1.0 - pow((double)A.b2, t));
    const float g = A.g[i];
    const float m = A.b1 * A.m[i] + (1.f - A.b1) * g;
    const float v = A.b2 * A.v[i] + (1.f - A.b2) * g * g;
    A.m[i] = m;
    A.v[i] = v;
    A.p[i] -= A.lr * (m / bc1) / (sqrtf(v / bc2) + A.eps);
}

__global__ void mlp_adam_advance_kernel(uint64_t* t, uint32_t members)
{
    if (threadIdx.x < members) t[threadIdx.x] += 1;
}

// ------------------------------------------------------------ inference ---
// Fused ensemble forward for widths w0 -> H -> ... -> H -> 1 with H <= 256.
constexpr int kInfH = 256;

struct InferArgs {
    const float* X;          // [n][w0] raw features
    const float* params;     // [members][P]
    float* mean;             // [n]
    float* spread;           // [n]
    uint64_t n, P;
    uint32_t members, n_layers, w0, H;
    uint64_t w_off[kMaxLayers], b_off[kMaxLayers];
    sde_surrogate_scaling sc;
};

// FP32 MFMA forward (v_mfma_f32_16x16x4_f32).  Operands of a 16 x 16 block
// (16 rows or output columns by 16 k) are one 1 KB run: lane l = i % 16 +
// 16 * (k % 4) holds the float4 of k = k % 4 + {0, 4, 8, 12}, the operands of
// four consecutive MFMAs.  The hidden weights are packed that way once per
// call (B(k, c) = W[c][k]); the activations stay in LDS in the same layout, as
// the A operand of the next layer.
__device__ __forceinline__ uint32_t frag32_index(uint32_t i, uint32_t k, uint32_t kb16)
{
    return (((i >> 4) * kb16 + (k >> 4)) * 64 + ((i & 15u) + 16u * (k & 3u))) * 4 + ((k & 15u) >> 2);
}

struct PackArgs {
    const float* params;
    uint64_t P;
    uint32_t members, hidden, H, Hp;
    uint64_t w_off[kMaxLayers];  // of hidden layer 1 + l at index l
    float* packed;               // [members][hidden][Hp * Hp]
};

// packed[m][l] (Hp x Hp, zero padded) from the hidden weights W_{l+1} of member m
__global__ void mlp_pack_hidden_kernel(PackArgs A)
{
    const uint64_t per = (uint64_t)A.Hp * A.Hp;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)A.members * A.hidden * per) return;
    const uint32_t m = (uint32_t)(g / (A.hidden * per));
    const uint32_t l = (uint32_t)((g / per) % A.hidden);
    const uint32_t e = (uint32_t)(g % per), c = e / A.Hp, k = e % A.Hp;
    const float* W = A.params + (uint64_t)m * A.P + A.w_off[l];
    A.packed[((uint64_t)m * A.hidden + l) * per + frag32_index(c, k, A.Hp / 16)] =
        (c < A.H && k < A.H) ? W[(uint64_t)c * A.H + k] : 0.f;
}

constexpr uint32_t kInfBlocks = kInfH / 16;  // column blocks of the widest layer
// Queries per workgroup: one 16-row block per wave, so that two workgroups
// (68 KB of LDS each) share a CU and one's GELU epilogue overlaps the
// other's products.
constexpr uint32_t kInfMRows = 64;

__global__ __launch_bounds__(256, 2) void mlp_infer_mfma_kernel(InferArgs A, const float* packed, uint32_t Hp)
{
    extern __shared__ float smem[];
    float* act = smem;                      // [kInfMRows x Hp] in the operand layout
    float* xn = act + kInfMRows * kInfH;    // [kInfMRows][8] normalized features
    float* outs = xn + kInfMRows * 8;       // [kInfMRows][8] member outputs
    const uint64_t r0 = (uint64_t)blockIdx.x * kInfMRows;
    const uint32_t H = A.H, KB = Hp / 16, NB = KB;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    for (uint32_t e = threadIdx.x; e < kInfMRows * A.w0; e += 256) {
        const uint32_t row = e / A.w0, j = e % A.w0;
        const uint64_t gi = r0 + row;
        xn[row * 8 + j] = gi < A.n ? (A.X[gi * A.w0 + j] - A.sc.in_center[j]) / A.sc.in_scale[j] : 0.f;
    }
    __syncthreads();
    const uint32_t hidden = A.n_layers - 2;
    for (uint32_t mem = 0; mem < A.members; ++mem) {
        const float* prm = A.params + (uint64_t)mem * A.P;
        {   // layer 1 from the normalized features
            const float* W = prm + A.w_off[0];
            const float* b = prm + A.b_off[0];
            for (uint32_t e = threadIdx.x; e < kInfMRows * Hp; e += 256) {
                const uint32_t row = e / Hp, col = e % Hp;
                float z = 0.f;
                if (col < H) {
                    z = b[col];
                    for (uint32_t j = 0; j < A.w0; ++j) z = fmaf(W[col * A.w0 + j], xn[row * 8 + j], z);
                    z = gelu(z);
                }
                act[frag32_index(row, col, KB)] = z;
            }
            __syncthreads();
        }
        // hidden layers: wave w computes rows 16 w .. 16 w + 15, all columns
        for (uint32_t l = 0; l < hidden; ++l) {
            const float* Bp = packed + ((uint64_t)mem * hidden + l) * Hp * Hp;
            const float* b = prm + A.b_off[l + 1];
            f32x4_t acc[1][kInfBlocks];
#pragma unroll
            for (int m = 0; m < 1; ++m)
#pragma unroll
                for (int n = 0; n < (int)kInfBlocks; ++n) acc[m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            for (uint32_t kb = 0; kb < KB; ++kb) {
                f32x4_t a[1], w[kInfBlocks];
#pragma unroll
                for (int m = 0; m < 1; ++m)
                    a[m] = *reinterpret_cast<const f32x4_t*>(act + (((wave + m) * KB + kb) * 64 + lane) * 4);
#pragma unroll
                for (int n = 0; n < (int)kInfBlocks; ++n)
                    if ((uint32_t)n < NB)
                        w[n] = *reinterpret_cast<const f32x4_t*>(Bp + (((uint64_t)n * KB + kb) * 64 + lane) * 4);
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int m = 0; m < 1; ++m)
#pragma unroll
                        for (int n = 0; n < (int)kInfBlocks; ++n)
                            if ((uint32_t)n < NB)
                                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m][j], w[n][j], acc[m][n], 0, 0, 0);
            }
            __syncthreads();  // every wave has read this layer's input
#pragma unroll
            for (int m = 0; m < 1; ++m)
#pragma unroll
                for (int n = 0; n < (int)kInfBlocks; ++n) {
                    if ((uint32_t)n >= NB) continue;
                    const uint32_t col = n * 16 + (lane & 15u);
                    const float bias = col < H ? b[col] : 0.f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t row = (wave + m) * 16 + 4 * (lane >> 4) + q;
                        act[frag32_index(row, col, KB)] = col < H ? gelu(acc[m][n][q] + bias) : 0.f;
                    }
                }
            __syncthreads();
        }
        // output layer H -> 1: four lanes per row, each a quarter of the columns
        {
            const float* W = prm + A.w_off[A.n_layers - 1];
            const float bo = prm[A.b_off[A.n_layers - 1]];
            const uint32_t row = threadIdx.x >> 2, quarter = threadIdx.x & 3u;
            float part = 0.f;
            for (uint32_t col = quarter; col < H; col += 4) part = fmaf(act[frag32_index(row, col, KB)], W[col], part);
            part += __shfl_xor(part, 1, 4);
            part += __shfl_xor(part, 2, 4);
            if (quarter == 0) outs[row * 8 + mem] = part + bo;
            __syncthreads();
        }
    }
    // members' mean and sample standard deviation, in units of <v>
    if (threadIdx.x < kInfMRows) {
        const uint64_t gi = r0 + threadIdx.x;
        if (gi < A.n) {
            const float scale = A.sc.target_over_omega ? A.X[gi * A.w0 + 1] : 1.f;
            float v[8], s = 0.f;
            for (uint32_t m = 0; m < A.members; ++m) {
                v[m] = (A.sc.out_mean + A.sc.out_std * outs[threadIdx.x * 8 + m]) * scale;
                s += v[m];
            }
            const float mu = s / (float)A.members;
            float ss = 0.f;
            for (uint32_t m = 0; m < A.members; ++m) ss += (v[m] - mu) * (v[m] - mu);
            A.mean[gi] = mu;
            A.spread[gi] = A.members > 1 ? sqrtf(ss / (float)(A.members - 1)) : 0.f;
        }
    }
}

// ------------------------------------------------------------ scan glue ---
__global__ void scan_flag_kernel(const float* spread, float spread_max, uint64_t n, uint8_t* flag)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = spread[i] > spread_max ? 1 : 0;
}

__global__ void scan_merge_kernel(const float* mean, const uint8_t* flag, const uint64_t* fb_index,
                                  const double* fb_sums, const uint32_t* fb_paths, uint64_t n_fb, uint64_t n,
                                  double* v_out, uint8_t* used)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        if (!flag[i]) v_out[i] = (double)mean[i];  // flagged entries are written below
        if (used) used[i] = flag[i];
    }
    if (i < n_fb) v_out[fb_index[i]] = fb_sums[2 * i] / (double)fb_paths[i];
}

}  // namespace sde

using namespace sde;

// ------------------------------------------------------------------ host --
namespace {

int check_s(sde_surrogate* s) { return s && s->ctx ? SDE_OK : SDE_ERR_INVALID; }

void layout(sde_surrogate* s)
{
    s->w_off.clear();
    s->b_off.clear();
    uint64_t k = 0;
    for (size_t l = 0; l + 1 < s->widths.size(); ++l) {
        s->w_off.push_back(k);
        k += (uint64_t)s->widths[l + 1] * s->widths[l];
        s->b_off.push_back(k);
        k += s->widths[l + 1];
    }
    s->P = k;
}

int alloc_surrogate(sde_ctx* ctx, const uint32_t* widths, uint32_t n_widths, uint32_t members, sde_surrogate** out)
{
    if (!ctx || !widths || !out || n_widths < 2 || n_widths > (uint32_t)kMaxLayers + 1 || members == 0 || members > 8)
        return fail(ctx, SDE_ERR_INVALID, "surrogate: need 2..%d widths and 1..8 members", kMaxLayers + 1);
    if (widths[n_widths - 1] != 1) return fail(ctx, SDE_ERR_INVALID, "surrogate: the output width must be 1");
    if (widths[0] == 0 || widths[0] > 8) return fail(ctx, SDE_ERR_INVALID, "surrogate: 1..8 input features");
    for (uint32_t l = 1; l + 1 < n_widths; ++l)
        if (widths[l] == 0 || widths[l] > (uint32_t)kInfH || (l > 1 && widths[l] != widths[1]))
            return fail(ctx, SDE_ERR_INVALID, "surrogate: hidden layers must share one width <= %d", kInfH);
    sde_surrogate* s = new (std::nothrow) sde_surrogate();
    if (!s) return SDE_ERR_NOMEM;
    s->ctx = ctx;
    s->widths.assign(widths, widths + n_widths);
    s->members = members;
    layout(s);
    const size_t bytes = (size_t)members * s->P * sizeof(float);
    if (hipMalloc(&s->params, bytes) != hipSuccess || hipMalloc(&s->grads, bytes) != hipSuccess ||
        hipMalloc(&s->adam_m, bytes) != hipSuccess || hipMalloc(&s->adam_v, bytes) != hipSuccess ||
        hipMalloc(&s->adam_t, 8 * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        sde_surrogate_destroy(s);
        return fail(ctx, SDE_ERR_NOMEM, "surrogate: cannot allocate parameters");
    }
    if (hipMemset(s->adam_m, 0, bytes) != hipSuccess || hipMemset(s->adam_v, 0, bytes) != hipSuccess ||
        hipMemset(s->adam_t, 0, 8 * sizeof(uint64_t)) != hipSuccess) {
        sde_surrogate_destroy(s);
        return fail(ctx, SDE_ERR_DEVICE, "surrogate: hipMemset failed");
    }
    for (int i = 0; i < 8; ++i) {
        s->sc.in_center[i] = 0.f;
        s->sc.in_scale[i] = 1.f;
    }
    s->sc.out_mean = 0.f;
    s->sc.out_std = 1.f;
    *out = s;
    return SDE_OK;
}

int ensure_work(sde_surrogate* s, size_t bytes)
{
    if (s->work_bytes >= bytes) return SDE_OK;
    if (s->work) {
        SDE_HIP(s->ctx, hipDeviceSynchronize());
        SDE_HIP(s->ctx, hipFree(s->work));
        s->work = nullptr;
        s->work_bytes = 0;
        ++s->ctx->ws_generation;
    }
    if (hipMalloc(&s->work, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(s->ctx, SDE_ERR_NOMEM, "surrogate: cannot allocate %zu bytes of workspace", bytes);
    }
    s->work_bytes = bytes;
    ++s->ctx->ws_generation;
    return SDE_OK;
}

// Training buffers for minibatch B: per layer Z and A (outputs), dZ, plus
// the normalized inputs/targets [n].
struct TrainBufs {
    float* Xn;
    float* yn;
    std::vector<float*> Z, Aout, dZ;   // per layer l = 0..L-1, [members][B][w_{l+1}]
    std::vector<uint64_t> stride;      // member stride of layer l buffers
    float* colpart;                    // [members][B / kColSlice][max width] bias-gradient slice sums
    float* dwpart;                     // [members][kMaxKSlices][max width^2] weight-gradient slice sums
    float* loss;                       // [members][steps_per_epoch]
};

static uint32_t max_width(const sde_surrogate* s)
{
    return *std::max_element(s->widths.begin(), s->widths.end());
}

// Slices of the batch sum of a weight-gradient product: enough workgroups to
// cover the CUs (the M x N tiles alone give few), at least 64 rows each.
constexpr uint32_t kMaxKSlices = 16;
static uint32_t dw_kslices(uint32_t M, uint32_t N, uint32_t K, uint32_t members)
{
    const uint32_t tiles = ((N + kGT - 1) / kGT) * ((M + kGT - 1) / kGT) * members;
    uint32_t k = (320 + tiles - 1) / tiles;
    k = std::min(k, std::max(1u, K / 64));
    return std::max(1u, std::min(k, kMaxKSlices));
}

size_t train_bytes(const sde_surrogate* s, uint64_t n, uint32_t B, uint32_t steps)
{
    size_t e = n * (s->widths[0] + 1);
    for (size_t l = 0; l + 1 < s->widths.size(); ++l) e += 3ull * s->members * B * s->widths[l + 1];
    e += (size_t)s->members * ((B + kColSlice - 1) / kColSlice) * max_width(s);
    e += (size_t)s->members * kMaxKSlices * max_width(s) * max_width(s);
    e += (size_t)s->members * steps;
    return e * sizeof(float) + 4096;
}

void carve(sde_surrogate* s, uint64_t n, uint32_t B, TrainBufs& t)
{
    float* p = s->work;
    t.Xn = p;
    p += n * s->widths[0];
    t.yn = p;
    p += n;
    const size_t L = s->widths.size() - 1;
    t.Z.resize(L);
    t.Aout.resize(L);
    t.dZ.resize(L);
    t.stride.resize(L);
    for (size_t l = 0; l < L; ++l) {
        t.stride[l] = (uint64_t)B * s->widths[l + 1];
        t.Z[l] = p;
        p += s->members * t.stride[l];
        t.Aout[l] = p;
        p += s->members * t.stride[l];
        t.dZ[l] = p;
        p += s->members * t.stride[l];
    }
    t.colpart = p;
    p += (size_t)s->members * ((B + kColSlice - 1) / kColSlice) * max_width(s);
    t.dwpart = p;
    p += (size_t)s->members * kMaxKSlices * max_width(s) * max_width(s);
    t.loss = p;
}

template <int MODE>
int launch_gemm(sde_ctx* ctx, const GemmArgs& g, uint32_t members, hipStream_t st)
{
    dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT, members * (MODE == kDW ? g.kslices : 1u));
    hipLaunchKernelGGL(mlp_gemm_kernel<MODE>, grid, dim3(256), 0, st, g);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

// One training step (forward, loss, backward, Adam) on minibatch rows
// rows[mem][offset .. offset + B).  If adam is false only the gradient is
// formed (into s->grads).
int record_step(sde_surrogate* s, const TrainBufs& t, const uint32_t* rows, uint64_t rows_mstride, uint32_t offset,
                uint32_t B, const float* targets, uint32_t loss_slot, uint32_t loss_stride, const sde_train_opts* o,
                bool adam, hipStream_t st)
{
    sde_ctx* ctx = s->ctx;
    const size_t L = s->widths.size() - 1;
    const uint32_t M = s->members;
    int e;
    for (size_t l = 0; l < L; ++l) {
        GemmArgs g{};
        g.A = l == 0 ? t.Xn : t.Aout[l - 1];
        g.a_mstride = l == 0 ? 0 : t.stride[l - 1];
        g.B = s->params + s->w_off[l];
        g.b_mstride = s->P;
        g.C = t.Z[l];
        g.c_mstride = t.stride[l];
        g.C2 = t.Aout[l];
        g.c2_mstride = t.stride[l];
        g.bias = s->params + s->b_off[l];
        g.bias_mstride = s->P;
        g.rows = l == 0 ? rows : nullptr;
        g.rows_mstride = rows_mstride;
        g.rows_offset = offset;
        g.M = B;
        g.N = s->widths[l + 1];
        g.K = s->widths[l];
        g.last = l + 1 == L;
        if ((e = launch_gemm<kFwd>(ctx, g, M, st))) return e;
    }
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(M), dim3(256), 0, st, t.Z[L - 1], t.stride[L - 1], targets, rows,
                       rows_mstride, offset, t.dZ[L - 1], t.stride[L - 1], B, t.loss, loss_slot, loss_stride);
    SDE_HIP(ctx, hipGetLastError());
    for (size_t l = L; l-- > 0;) {
        const uint32_t out = s->widths[l + 1], in = s->widths[l];
        GemmArgs g{};
        g.A = t.dZ[l];
        g.a_mstride = t.stride[l];
        g.B = l == 0 ? t.Xn : t.Aout[l - 1];
        g.b_mstride = l == 0 ? 0 : t.stride[l - 1];
        g.M = out;
        g.N = in;
        g.K = B;
        g.kslices = dw_kslices(out, in, B, M);
        g.C = t.dwpart;
        g.c_mstride = (uint64_t)g.kslices * out * in;
        if (l > 0) {  // the first layer's inputs are gathered rows: below
            if ((e = launch_gemm<kDW>(ctx, g, M, st))) return e;
            hipLaunchKernelGGL(mlp_ksum_kernel, dim3((out * in + 255) / 256, M), dim3(256), 0, st, t.dwpart,
                               g.kslices, (uint64_t)out * in, s->grads + s->w_off[l], s->P);
        }
        const uint32_t n_slices = (B + kColSlice - 1) / kColSlice;
        hipLaunchKernelGGL(mlp_colsum_slices_kernel, dim3((out + 255) / 256, n_slices, M), dim3(256), 0, st, t.dZ[l],
                           t.stride[l], t.colpart, B, out);
        hipLaunchKernelGGL(mlp_colsum_kernel, dim3((out + 255) / 256, M), dim3(256), 0, st, t.colpart, n_slices,
                           s->grads + s->b_off[l], s->P, out);
        SDE_HIP(ctx, hipGetLastError());
        if (l > 0) {
            GemmArgs d{};
            d.A = t.dZ[l];
            d.a_mstride = t.stride[l];
            d.B = s->params + s->w_off[l];
            d.b_mstride = s->P;
            d.C = t.dZ[l - 1];
            d.c_mstride = t.stride[l - 1];
            d.Zp = t.Z[l - 1];
            d.zp_mstride = t.stride[l - 1];
            d.M = B;
            d.N = in;
            d.K = out;
            if ((e = launch_gemm<kDX>(ctx, d, M, st))) return e;
        }
    }
    // first-layer weight gradient: dW_0[o][j] = sum_b dZ_0[b][o] Xn[rows[b]][j]
    {
        GemmArgs g{};
        g.A = t.dZ[0];
        g.a_mstride = t.stride[0];
        g.B = t.Xn;
        g.b_mstride = 0;
        g.rows = rows;
        g.rows_mstride = rows_mstride;
        g.rows_offset = offset;
        g.M = s->widths[1];
        g.N = s->widths[0];
        g.K = B;
        g.kslices = dw_kslices(g.M, g.N, B, M);
        g.C = t.dwpart;
        g.c_mstride = (uint64_t)g.kslices * g.M * g.N;
        dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT, M * g.kslices);
        hipLaunchKernelGGL(mlp_gemm_dw_gather_kernel, grid, dim3(256), 0, st, g);
        hipLaunchKernelGGL(mlp_ksum_kernel, dim3((g.M * g.N + 255) / 256, M), dim3(256), 0, st, t.dwpart, g.kslices,
                           (uint64_t)g.M * g.N, s->grads + s->w_off[0], s->P);
        SDE_HIP(ctx, hipGetLastError());
    }
    if (adam) {
        AdamArgs a;
        a.p = s->params;
        a.g = s->grads;
        a.m = s->adam_m;
        a.v = s->adam_v;
        a.t = s->adam_t;
        a.P = s->P;
        a.members = M;
        a.lr = o->lr;
        a.b1 = o->beta1;
        a.b2 = o->beta2;
        a.eps = o->eps;
        const uint64_t total = s->P * M;
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, a);
        hipLaunchKernelGGL(mlp_adam_advance_kernel, dim3(1), dim3(64), 0, st, s->adam_t, M);
        SDE_HIP(ctx, hipGetLastError());
    }
    return SDE_OK;
}

int normalize(sde_surrogate* s, const float* X, const float* y, uint64_t n, const TrainBufs& t, hipStream_t st)
{
    NormArgs a;
    a.X = X;
    a.y = y;
    a.Xn = t.Xn;
    a.yn = y ? t.yn : nullptr;
    a.n = n;
    a.w0 = s->widths[0];
    a.sc = s->sc;
    hipLaunchKernelGGL(mlp_normalize_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, a);
    SDE_HIP(s->ctx, hipGetLastError());
    return SDE_OK;
}

}  // namespace

extern "C" {

int sde_surrogate_create(sde_ctx* ctx, const uint32_t* widths, uint32_t n_widths, uint32_t n_members, uint64_t seed,
                         sde_surrogate** out)
{
    if (!ctx) return SDE_ERR_INVALID;
    ctx->last_error.clear();
    sde_surrogate* s = nullptr;
    int st = alloc_surrogate(ctx, widths, n_widths, n_members, &s);
    if (st) return st;
    InitArgs a{};
    a.params = s->params;
    a.P = s->P;
    a.members = s->members;
    a.n_layers = (uint32_t)s->widths.size() - 1;
    for (uint32_t l = 0; l < a.n_layers; ++l) {
        a.layer_end[l] = s->b_off[l] + s->widths[l + 1];
        a.bound[l] = (float)(1.0 / std::sqrt((double)s->widths[l]));
    }
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    const uint64_t total = s->P * s->members;
    hipLaunchKernelGGL(mlp_init_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, 0, a);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        sde_surrogate_destroy(s);
        return fail(ctx, SDE_ERR_DEVICE, "surrogate: initialization kernel failed");
    }
    *out = s;
    return SDE_OK;
}

void sde_surrogate_destroy(sde_surrogate* s)
{
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)s->params, (void*)s->grads, (void*)s->adam_m, (void*)s->adam_v, (void*)s->adam_t,
                    (void*)s->work, (void*)s->perm, (void*)s->packed})
        if (p) (void)hipFree(p);
    delete s;
}

uint64_t sde_surrogate_param_count(const sde_surrogate* s) { return s ? s->P : 0; }

int sde_surrogate_set_params(sde_surrogate* s, uint32_t member, const float* host, uint64_t n)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    if (!host || member >= s->members || n != s->P) return fail(s->ctx, SDE_ERR_INVALID, "set_params: bad member/size");
    const size_t b = s->P * sizeof(float);
    SDE_HIP(s->ctx, hipDeviceSynchronize());
    SDE_HIP(s->ctx, hipMemcpy(s->params + member * s->P, host, b, hipMemcpyHostToDevice));
    SDE_HIP(s->ctx, hipMemset(s->adam_m + member * s->P, 0, b));
    SDE_HIP(s->ctx, hipMemset(s->adam_v + member * s->P, 0, b));
    uint64_t zero = 0;
    SDE_HIP(s->ctx, hipMemcpy(s->adam_t + member, &zero, sizeof zero, hipMemcpyHostToDevice));
    return SDE_OK;
}

int sde_surrogate_get_params(sde_surrogate* s, uint32_t member, float* host, uint64_t n)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    if (!host || member >= s->members || n != s->P) return fail(s->ctx, SDE_ERR_INVALID, "get_params: bad member/size");
    SDE_HIP(s->ctx, hipDeviceSynchronize());
    SDE_HIP(s->ctx, hipMemcpy(host, s->params + member * s->P, s->P * sizeof(float), hipMemcpyDeviceToHost));
    return SDE_OK;
}

int sde_surrogate_set_scaling(sde_surrogate* s, const sde_surrogate_scaling* sc)
{
    if (check_s(s) || !sc) return SDE_ERR_INVALID;
    for (uint32_t j = 0; j < s->widths[0]; ++j)
        if (!std::isfinite(sc->in_center[j]) || !std::isfinite(sc->in_scale[j]) || sc->in_scale[j] == 0.f)
            return fail(s->ctx, SDE_ERR_INVALID, "scaling: feature %u needs a finite center and nonzero scale", j);
    if (!std::isfinite(sc->out_mean) || !std::isfinite(sc->out_std) || sc->out_std == 0.f || sc->reserved != 0)
        return fail(s->ctx, SDE_ERR_INVALID, "scaling: bad output scaling");
    if (sc->target_over_omega && s->widths[0] < 2)
        return fail(s->ctx, SDE_ERR_INVALID, "scaling: <v>/omega needs omega as feature 1");
    s->sc = *sc;
    return SDE_OK;
}

int sde_surrogate_get_scaling(const sde_surrogate* s, sde_surrogate_scaling* sc)
{
    if (!s || !sc) return SDE_ERR_INVALID;
    *sc = s->sc;
    return SDE_OK;
}

int sde_surrogate_loss_grad(sde_surrogate* s, uint32_t member, const float* X, const float* y, uint64_t n,
                            float* host_grad, double* host_loss, void* hip_stream)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    sde_ctx* ctx = s->ctx;
    ctx->last_error.clear();
    if (!X || !y || n == 0 || n > (1u << 20) || member >= s->members)
        return fail(ctx, SDE_ERR_INVALID, "loss_grad: bad arguments");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const uint32_t B = (uint32_t)n;
    int e;
    if ((e = ensure_work(s, train_bytes(s, n, B, 1)))) return e;
    TrainBufs t;
    carve(s, n, B, t);
    if ((e = normalize(s, X, y, n, t, st))) return e;
    sde_train_opts o{};
    if ((e = record_step(s, t, nullptr, 0, 0, B, t.yn, 0, 1, &o, false, st))) return e;
    SDE_HIP(ctx, hipStreamSynchronize(st));
    if (host_grad)
        SDE_HIP(ctx, hipMemcpy(host_grad, s->grads + member * s->P, s->P * sizeof(float), hipMemcpyDeviceToHost));
    if (host_loss) {
        float l = 0.f;
        SDE_HIP(ctx, hipMemcpy(&l, t.loss + member, sizeof(float), hipMemcpyDeviceToHost));
        *host_loss = l;
    }
    return SDE_OK;
}

int sde_surrogate_train(sde_surrogate* s, const float* X, const float* y, uint64_t n, const sde_train_opts* o,
                        float* loss_curve, void* hip_stream)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    const TraceRange range("sde_surrogate_train");
    sde_ctx* ctx = s->ctx;
    ctx->last_error.clear();
    if (!X || !y || !o || n == 0 || o->epochs == 0 || o->batch == 0 || o->batch > n || n > 0xffffffffull)
        return fail(ctx, SDE_ERR_INVALID, "train: need X, y, options, 0 < batch <= n");
    if (!(o->lr > 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) || !(o->eps > 0))
        return fail(ctx, SDE_ERR_INVALID, "train: bad Adam hyper-parameters");
    try {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const uint32_t B = o->batch;
        const uint32_t steps = (uint32_t)(n / B);
        int e;
        if ((e = ensure_work(s, train_bytes(s, n, B, steps)))) return e;
        TrainBufs t;
        carve(s, n, B, t);
        if ((e = normalize(s, X, y, n, t, st))) return e;
        const size_t perm_elems = (size_t)s->members * n;
        if (s->perm_cap < perm_elems) {
            SDE_HIP(ctx, hipDeviceSynchronize());
            if (s->perm) SDE_HIP(ctx, hipFree(s->perm));
            s->perm = nullptr;
            s->perm_cap = 0;
            SDE_HIP(ctx, hipMalloc(&s->perm, perm_elems * sizeof(uint32_t)));
            s->perm_cap = perm_elems;
            ++ctx->ws_generation;
        }
        std::vector<uint32_t> perm(perm_elems);
        std::vector<float> losses(steps);
        uint32_t* hperm = nullptr;
        SDE_HIP(ctx, hipHostMalloc(&hperm, perm_elems * sizeof(uint32_t), hipHostMallocDefault));
        char key[256];
        snprintf(key, sizeof key, "mlp-epoch|%p|%p|%p|%llu|%u|%u|%a|%a|%a|%a", (void*)s, (void*)s->work, (void*)s->perm,
                 (unsigned long long)n, B, steps, o->lr, o->beta1, o->beta2, o->eps);
        for (uint32_t ep = 0; ep < o->epochs; ++ep) {
            // the sample order of this epoch, one permutation per member
            for (uint32_t m = 0; m < s->members; ++m) {
                std::mt19937_64 rng(o->shuffle_seed * 1000003ull + (uint64_t)ep * 131ull + m);
                uint32_t* p = perm.data() + (size_t)m * n;
                std::iota(p, p + n, 0u);
                std::shuffle(p, p + n, rng);
            }
            SDE_HIP(ctx, hipStreamSynchronize(st));  // the previous epoch no longer reads hperm
            std::memcpy(hperm, perm.data(), perm_elems * sizeof(uint32_t));
            SDE_HIP(ctx, hipMemcpyAsync(s->perm, hperm, perm_elems * sizeof(uint32_t), hipMemcpyHostToDevice, st));
            e = run_recorded(ctx, key, st, [&](hipStream_t cs) -> int {
                for (uint32_t k = 0; k < steps; ++k) {
                    int r = record_step(s, t, s->perm, n, k * B, B, t.yn, k, steps, o, true, cs);
                    if (r) return r;
                }
                return SDE_OK;
            });
            if (e) {
                (void)hipHostFree(hperm);
                return e;
            }
            if (loss_curve) {
                SDE_HIP(ctx, hipMemcpyAsync(losses.data(), t.loss, steps * sizeof(float), hipMemcpyDeviceToHost, st));
                SDE_HIP(ctx, hipStreamSynchronize(st));
                double sum = 0.0;
                for (float l : losses) sum += l;
                loss_curve[ep] = (float)(sum / steps);
            }
        }
        SDE_HIP(ctx, hipStreamSynchronize(st));
        SDE_HIP(ctx, hipHostFree(hperm));
        return SDE_OK;
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

static int predict_impl(sde_surrogate* s, const float* X, uint64_t n, float* mean, float* spread, hipStream_t st)
{
    sde_ctx* ctx = s->ctx;
    if (s->widths.size() - 1 < 2) return fail(ctx, SDE_ERR_UNSUPPORTED, "predict: needs at least one hidden layer");
    InferArgs a{};
    a.X = X;
    a.params = s->params;
    a.mean = mean;
    a.spread = spread;
    a.n = n;
    a.P = s->P;
    a.members = s->members;
    a.n_layers = (uint32_t)s->widths.size() - 1;
    a.w0 = s->widths[0];
    a.H = s->widths[1];
    for (uint32_t l = 0; l < a.n_layers; ++l) {
        a.w_off[l] = s->w_off[l];
        a.b_off[l] = s->b_off[l];
    }
    a.sc = s->sc;
    // hidden weights into the MFMA operand layout (Hp = H rounded up to 16)
    const uint32_t H = a.H, Hp = (H + 15u) & ~15u, hidden = a.n_layers - 2;
    if (hidden > 0) {
        const size_t need = (size_t)s->members * hidden * Hp * Hp * sizeof(float);
        if (s->packed_bytes < need) {
            if (s->packed) SDE_HIP(ctx, hipFree(s->packed));
            s->packed = nullptr;
            s->packed_bytes = 0;
            SDE_HIP(ctx, hipMalloc(&s->packed, need));
            s->packed_bytes = need;
        }
        PackArgs pk{};
        pk.params = s->params;
        pk.P = s->P;
        pk.members = s->members;
        pk.hidden = hidden;
        pk.H = H;
        pk.Hp = Hp;
        for (uint32_t l = 0; l < hidden; ++l) pk.w_off[l] = s->w_off[l + 1];
        pk.packed = s->packed;
        const uint64_t total = (uint64_t)s->members * hidden * Hp * Hp;
        hipLaunchKernelGGL(mlp_pack_hidden_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, pk);
        SDE_HIP(ctx, hipGetLastError());
    }
    const size_t lds = (size_t)(kInfMRows * kInfH + 2 * kInfMRows * 8) * sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        SDE_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_infer_mfma_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    hipLaunchKernelGGL(mlp_infer_mfma_kernel, dim3((uint32_t)((n + kInfMRows - 1) / kInfMRows)), dim3(256), lds, st, a,
                       static_cast<const float*>(s->packed), Hp);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int sde_surrogate_predict(sde_surrogate* s, const float* X, uint64_t n, float* mean, float* spread, void* hip_stream)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    const TraceRange range("sde_surrogate_predict");
    s->ctx->last_error.clear();
    if (!X || !mean || !spread || n == 0 || (n + kInfMRows - 1) / kInfMRows > 0x7fffffffull)
        return fail(s->ctx, SDE_ERR_INVALID, "predict: bad arguments");
    if (!aligned(X, 4) || !aligned(mean, 4) || !aligned(spread, 4))
        return fail(s->ctx, SDE_ERR_INVALID, "predict: misaligned pointer");
    return predict_impl(s, X, n, mean, spread, static_cast<hipStream_t>(hip_stream));
}

int sde_surrogate_scan(sde_surrogate* s, const sde_jj_point* q, uint64_t n, float spread_max, const sde_run* fb,
                       double* v_out, uint8_t* used, sde_scan_stats* stats, void* hip_stream)
{
    if (check_s(s)) return SDE_ERR_INVALID;
    const TraceRange range("sde_surrogate_scan");
    sde_ctx* ctx = s->ctx;
    ctx->last_error.clear();
    if (!q || n == 0 || !fb || !v_out || !(spread_max >= 0) || s->widths[0] != 5)
        return fail(ctx, SDE_ERR_INVALID, "scan: bad arguments (the surrogate must take 5 features)");
    if (!aligned(v_out, 8)) return fail(ctx, SDE_ERR_INVALID, "scan: misaligned v_out");
    try {
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::vector<float> feat(n * 5);
        for (uint64_t i = 0; i < n; ++i) {
            if (!(q[i].D > 0) || q[i].m != 1.0)
                return fail(ctx, SDE_ERR_INVALID, "scan: query %llu needs D > 0 and m = 1", (unsigned long long)i);
            feat[5 * i] = (float)q[i].a;
            feat[5 * i + 1] = (float)q[i].omega;
            feat[5 * i + 2] = (float)q[i].f;
            feat[5 * i + 3] = (float)std::log10(q[i].D);
            feat[5 * i + 4] = (float)q[i].gamma;
        }
        // workspace: features | mean | spread | flags
        int e = upload(ctx, kSlotMisc, 3, feat.data(), feat.size() * sizeof(float), st);
        if (e) return e;
        void* w = nullptr;
        if ((e = ensure_ws(ctx, kSlotObs, n * (2 * sizeof(float) + 1) + 256, &w))) return e;
        float* X = static_cast<float*>(ctx->ws[kSlotMisc].ptr);
        float* mean = static_cast<float*>(w);
        float* spread = mean + n;
        uint8_t* flag = reinterpret_cast<uint8_t*>(spread + n);
        hipEvent_t e0, e1, e2, e3;
        SDE_HIP(ctx, hipEventCreate(&e0));
        SDE_HIP(ctx, hipEventCreate(&e1));
        SDE_HIP(ctx, hipEventCreate(&e2));
        SDE_HIP(ctx, hipEventCreate(&e3));
        SDE_HIP(ctx, hipEventRecord(e0, st));
        if ((e = predict_impl(s, X, n, mean, spread, st))) return e;
        hipLaunchKernelGGL(scan_flag_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, spread, spread_max,
                           n, flag);
        SDE_HIP(ctx, hipEventRecord(e1, st));
        std::vector<uint8_t> hflag(n);
        SDE_HIP(ctx, hipMemcpyAsync(hflag.data(), flag, n, hipMemcpyDeviceToHost, st));
        SDE_HIP(ctx, hipStreamSynchronize(st));
        std::vector<sde_jj_point> fpts;
        std::vector<uint64_t> fidx;
        std::vector<uint32_t> fpaths;
        for (uint64_t i = 0; i < n; ++i)
            if (hflag[i]) {
                fpts.push_back(q[i]);
                fidx.push_back(i);
                fpaths.push_back(q[i].n_paths);
            }
        const uint64_t nf = fpts.size();
        // fallback simulation: one persistent launch over the uncertain points
        void* fbw = nullptr;
        if ((e = ensure_ws(ctx, kSlotTune, std::max<uint64_t>(nf, 1) * (2 * sizeof(double) + sizeof(uint64_t) + 4) + 64,
                           &fbw)))
            return e;
        double* fsums = static_cast<double*>(fbw);
        uint64_t* didx = reinterpret_cast<uint64_t*>(fsums + 2 * std::max<uint64_t>(nf, 1));
        uint32_t* dpaths = reinterpret_cast<uint32_t*>(didx + std::max<uint64_t>(nf, 1));
        SDE_HIP(ctx, hipEventRecord(e2, st));
        if (nf) {
            sde_run r = *fb;
            r.init = SDE_INIT_PHILOX;
            r.step0 = 0;
            r.sync = 0;
            if ((e = jj_integrate_impl(ctx, fpts.data(), (uint32_t)nf, &r, nullptr, nullptr, nullptr, nullptr, fsums,
                                       st)))
                return e;
            SDE_HIP(ctx, hipMemcpyAsync(didx, fidx.data(), nf * sizeof(uint64_t), hipMemcpyHostToDevice, st));
            SDE_HIP(ctx, hipMemcpyAsync(dpaths, fpaths.data(), nf * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        }
        hipLaunchKernelGGL(scan_merge_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, mean, flag, didx,
                           fsums, dpaths, nf, n, v_out, used);
        SDE_HIP(ctx, hipEventRecord(e3, st));
        SDE_HIP(ctx, hipStreamSynchronize(st));
        if (stats) {
            float a = 0.f, b = 0.f;
            SDE_HIP(ctx, hipEventElapsedTime(&a, e0, e1));
            SDE_HIP(ctx, hipEventElapsedTime(&b, e2, e3));
            stats->n_queries = n;
            stats->n_fallback = nf;
            stats->predict_ms = a;
            stats->fallback_ms = b;
            stats->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        for (hipEvent_t ev : {e0, e1, e2, e3}) (void)hipEventDestroy(ev);
        return sync_and_check(ctx, st);
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_surrogate_save(const sde_surrogate* s, const char* path)
{
    if (!s || !path) return SDE_ERR_INVALID;
    std::vector<float> p(s->P * s->members);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(p.data(), s->params, p.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(s->ctx, SDE_ERR_DEVICE, "save: cannot read parameters");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(s->ctx, SDE_ERR_INVALID, "save: cannot open %s", path);
    const uint32_t hdr[4] = {0x53444553u /* "SDES" */, 1u, (uint32_t)s->widths.size(), s->members};
    bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(s->widths.data(), sizeof(uint32_t), s->widths.size(), f) == s->widths.size() &&
              std::fwrite(&s->sc, sizeof s->sc, 1, f) == 1 && std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SDE_OK : fail(s->ctx, SDE_ERR_DEVICE, "save: write failed");
}

int sde_surrogate_load(sde_ctx* ctx, const char* path, sde_surrogate** out)
{
    if (!ctx || !path || !out) return SDE_ERR_INVALID;
    ctx->last_error.clear();
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ctx, SDE_ERR_INVALID, "load: cannot open %s", path);
    uint32_t hdr[4];
    std::vector<uint32_t> widths;
    sde_surrogate_scaling sc;
    int st = SDE_ERR_INVALID;
    sde_surrogate* s = nullptr;
    if (std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x53444553u && hdr[1] == 1u && hdr[2] >= 2 && hdr[2] <= 9) {
        widths.resize(hdr[2]);
        if (std::fread(widths.data(), sizeof(uint32_t), hdr[2], f) == hdr[2] && std::fread(&sc, sizeof sc, 1, f) == 1 &&
            (st = alloc_surrogate(ctx, widths.data(), hdr[2], hdr[3], &s)) == SDE_OK) {
            std::vector<float> p(s->P * s->members);
            if (std::fread(p.data(), sizeof(float), p.size(), f) == p.size() &&
                hipMemcpy(s->params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess) {
                s->sc = sc;
                st = SDE_OK;
            } else {
                st = SDE_ERR_INVALID;
            }
        }
    }
    std::fclose(f);
    if (st != SDE_OK) {
        sde_surrogate_destroy(s);
        return st == SDE_ERR_INVALID ? fail(ctx, st, "load: %s is not a surrogate file", path) : st;
    }
    *out = s;
    return SDE_OK;
}

}  // extern "C"
