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
//  * FP32: FP32 MFMA (v_mfma_f32_16x16x4_f32), FP32 products and accumulation.
//  * BF16X3 / FP16X3: MFMA (v_mfma_f32_16x16x32_{bf16,f16}) with FP32
//    accumulation on a hi/lo split of both operands,
//       K B ~ K_hi B_hi + K_hi B_lo + K_lo B_hi,
//    x_hi = round16(x), x_lo = round16(x - x_hi); the dropped K_lo B_lo term
//    is ~2^-16 (bf16) / 2^-22 (fp16) of each product.  K is first scaled by an
//    exact power of two so its largest entry lies in [1, 2): the fp16 lo
//    parts then stay normal, and the scaling is undone exactly afterwards.
//
// Layouts (all in the context's workspace).  Rows of K are padded to Mp (a
// multiple of 128), the k extent to Np (N rounded up to 32), realizations to
// Rp (a multiple of 32); the sin/cos operand B has 2 Rp columns, column
// (r / 32) * 64 + (r % 32) holding sin(2 pi theta_rj) and the column 32
// later cos.  Two B buffers alternate between the stages.
//   16-bit variants: K (hi and lo) and B in the fragment-packed layout of
//                    frag_off, so every MFMA operand is one contiguous 1 KB
//                    load (a row-major tile puts the 16 rows of a fragment
//                    8 KB apart, and the L1 then serves the load one lane at
//                    a time);
//   FP32 variant:    the same idea for the FP32 MFMA's operands (frag32_off):
//                    16 rows by 16 k in one contiguous 1 KB block, a lane's
//                    float4 holding the k of four consecutive MFMAs.
// A workgroup owns 128 rows x 32 realizations (64 columns), so every lane
// holds S and C of the same (i, r) in its accumulators; its waves split the
// k loop (8 or 4 waves for the 16-bit variants, 4 for FP32) and sum their
// partial tiles through LDS in a fixed order.  Workgroups are dealt to XCDs
// so that each XCD sweeps a contiguous band of rows over all columns: its
// slice of K is read from HBM/MALL once per product, B once per XCD, and the
// workgroups that share a K slab or a B column block hit in the XCD's L2.
// Four more 16-bit kernels with a whole block of load lookahead (two
// workgroups per tile over the halves of k, row-half waves with two
// register sets, 4 waves with K double-buffered in LDS, wave pairs sharing
// K through LDS) are candidates too:
// the kernel and the banding (against plain row-major order) are chosen per
// shape class by timing predictor stages of each.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

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
// s_waitcnt immediate (gfx9 encoding) waiting for LDS and scalar memory only:
// lgkmcnt(0) with vmcnt and expcnt at their maxima
constexpr int kWaitLdsOnly = (3 << 14) | (0 << 8) | (7 << 4) | 0xF;

struct DenseArgs {
    const void* K;         // scaled K, packed: 16-bit hi/lo (frag_off) or FP32 (frag32_off)
    const void* B;         // current sin/cos operand (same layout family)
    void* Bnext;           // operand for the next product
    const float* src;      // [R][N] phases the drift is evaluated at
    float* dst;            // [R][N] output phases
    float* F1;             // [R][N] the predictor's carry for the corrector: th + (dt/2) F_1 / 2 pi + noise
    const float* omega;    // [N]
    const float* scale;    // device: {scale, 1/scale}
    uint32_t N, R, Np, Rp, Mp;  // Np: k extent of the product (N rounded up to 32)
    const uint64_t* nbase; // device: absolute step of the current chunk's first step
    uint32_t k;            // step within the chunk
    uint32_t key0, key1;
    float omega_scale, hdt2pi, c2;
    int32_t stage;         // 1 predictor (or Euler step), 2 corrector
    int32_t euler;
    int32_t band;          // deal row tiles to XCDs in contiguous bands (when they split evenly)
    int* flag;             // error flag (a wave pairing that timed out in the two-half kernel)
};

__device__ __forceinline__ uint32_t bcol(uint32_t r, uint32_t kind)
{
    return (r / kRealTile) * (2 * kRealTile) + kind * kRealTile + (r % kRealTile);
}

// Fragment-packed 16-bit layout of a matrix with 32-aligned k extent Np
// (KB = Np / 32 blocks of k): the operand of one 16x16x32 MFMA -- 16 rows (A)
// or columns (B) by 32 k -- is one contiguous 1 KB block laid out as the 64
// lanes hold it (lane = row % 16 + 16 * (k % 32 / 8), 8 consecutive k per
// lane), its lo part in the next 1 KB, and consecutive k blocks of the same
// 16 rows follow each other.  A wave's fragment load is then one fully used,
// contiguous 1 KB request, and a row tile's k sweep is a sequential stream.
__device__ __forceinline__ uint64_t frag_off(uint32_t row, uint32_t k, uint32_t KB)
{
    return ((((uint64_t)(row >> 4) * KB + (k >> 5)) * 2) * 64 + ((row & 15u) + 16u * ((k >> 3) & 3u))) * 8 + (k & 7u);
}
constexpr uint32_t kFragLo = 512;  // elements from a hi fragment to its lo part

// Fragment-packed FP32 layout (k extent Np, KB16 = Np / 16 blocks of k): a
// 16 x 16 block is one contiguous 1 KB run where lane l = row % 16 +
// 16 * (k % 4) holds a float4 of k = k % 4 + {0, 4, 8, 12} -- the A (or B)
// operands of four consecutive v_mfma_f32_16x16x4_f32.
__device__ __forceinline__ uint64_t frag32_off(uint32_t row, uint32_t k, uint32_t KB16)
{
    return (((uint64_t)(row >> 4) * KB16 + (k >> 4)) * 64 + ((row & 15u) + 16u * (k & 3u))) * 4 + ((k & 15u) >> 2);
}

// x -> hi = round16(x) at p[idx], lo = round16(x - hi) at p[idx + kFragLo].
template <typename T>
__device__ __forceinline__ void store_split(T* p, uint64_t idx, float x)
{
    const T h = (T)x;
    p[idx] = h;
    p[idx + kFragLo] = (T)(x - (float)h);
}

// The stage update of oscillator i of realization r at absolute step n,
// given S = sum_j K_ij sin phi_j, C = sum_j K_ij cos phi_j, the phase ts the
// drift F is evaluated at (the predictor: the phase th at the start of the
// step) and omega_i.  Both Heun stages of a step add the same noise
// (Alg. 2), so the predictor leaves the corrector everything it needs from
// stage 1 and the step's start in one number,
// carry = th + (dt / 2) F_1 / 2 pi + noise, and the corrector neither draws
// noise nor reads th again:
//   predictor  t = th + dt F_1 / 2 pi + noise           (Euler: the step)
//   corrector  t = carry + (dt / 2) F_2 / 2 pi
// Returns the new phase; `carry` is written by the predictor, read by the
// corrector.
__device__ __forceinline__ float dense_stage(const DenseArgs& A, uint64_t n, uint32_t i, uint32_t r, float S, float C,
                                             float ts, float om, float& carry)
{
    const float F = fmaf(cos_rev(ts), S, fmaf(-sin_rev(ts), C, om));
    float t;
    if (A.stage == 1) {
        const float ns = gauss1_scaled(U4{(uint32_t)(n >> 2), i, r, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2,
                                       (uint32_t)n & 3u);
        t = fmaf(A.omega_scale, F, ts) + ns;
        if (A.euler)
            t -= floorf(t);
        else
            carry = ts + fmaf(A.hdt2pi, F, ns);  // one rounding at the phase's magnitude
    } else {
        t = fmaf(A.hdt2pi, F, carry);
        t -= floorf(t);
    }
    return t;
}

// workgroup -> (row tile, realization tile); with `band`, XCD-aware when the
// row tiles split evenly over the 8 XCDs (workgroup b runs on XCD b mod 8).
__device__ __forceinline__ void tile_of(uint32_t b, uint32_t n_mt, uint32_t n_nt, int32_t band, uint32_t& mt,
                                        uint32_t& nt)
{
    if (band && n_mt % 8 == 0) {
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

// Stage update of a 128-row x 32-realization tile whose S and C sit in LDS
// as tS[realization][row], tC[realization][row] (already unscaled), by NT
// threads.  Lane t takes the oscillators t, t + NT, ... of the tile in
// row-fastest order, so a wave's phase loads and stores cover 64 consecutive
// oscillators of one realization (256 contiguous bytes; giving each lane 8
// consecutive rows instead would put the lanes 32 bytes apart, and the L1
// would serve them one by one).  All of a lane's loads come
// before its first store: dst may be src (the in-place Euler step), so the
// compiler could not move a load above a store.  sin and cos of the new
// phase replace S and C in the tile (zero outside R x N), for the store of
// the next operand that follows.
template <uint32_t NT = kDenseThreads>
__device__ __forceinline__ void dense_tile_stage(const DenseArgs& A, uint32_t mt, uint32_t nt,
                                                 float (*tS)[kRowTile + 1], float (*tC)[kRowTile + 1])
{
    constexpr uint32_t kPer = kRowTile * kRealTile / NT;  // oscillators per lane
    static_assert(kRowTile % kWave == 0 && NT % kRowTile == 0, "a wave stays in one realization");
    const uint64_t n = load_uniform(A.nbase) + A.k;
    const bool corrector = A.stage != 1;
    float ts[kPer], cy[kPer], om[kPer];
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) {
        const uint32_t idx = threadIdx.x + e * NT;
        const uint32_t r = nt * kRealTile + idx / kRowTile, i = mt * kRowTile + idx % kRowTile;
        const bool ok = r < A.R && i < A.N;
        const uint64_t gi = ok ? (uint64_t)r * A.N + i : 0;
        ts[e] = ok ? A.src[gi] : 0.f;
        cy[e] = ok && corrector ? A.F1[gi] : 0.f;
        om[e] = ok ? A.omega[i] : 0.f;
    }
    // The lane's 16 updates are independent: read all sums first and compute
    // them branch-free (lanes outside R x N draw noise nobody uses), so the
    // compiler can interleave their Philox chains; only the stores are
    // predicated.  Each (rl, il) belongs to one lane, so reading all before
    // writing any is safe.
    float S[kPer], C[kPer], t[kPer];
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) {
        const uint32_t idx = threadIdx.x + e * NT;
        S[e] = tS[idx / kRowTile][idx % kRowTile];
        C[e] = tC[idx / kRowTile][idx % kRowTile];
    }
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) {
        const uint32_t idx = threadIdx.x + e * NT;
        const uint32_t r = nt * kRealTile + idx / kRowTile, i = mt * kRowTile + idx % kRowTile;
        t[e] = dense_stage(A, n, i, r, S[e], C[e], ts[e], om[e], cy[e]);
    }
#pragma unroll
    for (uint32_t e = 0; e < kPer; ++e) {
        const uint32_t idx = threadIdx.x + e * NT;
        const uint32_t rl = idx / kRowTile, il = idx % kRowTile;
        const uint32_t r = nt * kRealTile + rl, i = mt * kRowTile + il;
        const bool ok = r < A.R && i < A.N;
        if (ok) {
            const uint64_t gi = (uint64_t)r * A.N + i;
            if (!corrector && !A.euler) A.F1[gi] = cy[e];
            A.dst[gi] = t[e];
        }
        tS[rl][il] = ok ? sin_rev(t[e]) : 0.f;  // rows k >= N of the operand stay zero
        tC[rl][il] = ok ? cos_rev(t[e]) : 0.f;
    }
    __syncthreads();
}

// The tile's sin/cos as the next 16-bit split operand, in 16-byte rows: pass
// j sends lane -> (column c % 16, 8-row group of the 32-row block) of the
// fragment (column block, k block) = ((u >> 6) & 3, u >> 8), so a wave writes
// one whole 1 KB packed fragment (hi) and its lo part per pass.
template <typename T, typename V, uint32_t NT>
__device__ __forceinline__ void dense_tile_store(const DenseArgs& A, uint32_t mt, uint32_t nt,
                                                 const float (*tS)[kRowTile + 1], const float (*tC)[kRowTile + 1])
{
    const uint32_t KB = A.Np / kKStep;
    T* B = static_cast<T*>(A.Bnext);
#pragma unroll
    for (uint32_t j = 0; j < 2 * kRealTile * kRowTile / 8 / NT; ++j) {
        const uint32_t u = threadIdx.x + j * NT;
        const uint32_t cb = (u >> 6) & 3u, kind = cb >> 1;
        const uint32_t rl = (cb & 1u) * 16 + (u & 15u), il0 = (u >> 8) * kKStep + ((u >> 4) & 3u) * 8;
        const uint32_t r = nt * kRealTile + rl, i0 = mt * kRowTile + il0;
        if (r >= A.R || i0 >= A.N) continue;
        const float* src = kind ? &tC[rl][il0] : &tS[rl][il0];
        V hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            hi[e] = (T)src[e];
            lo[e] = (T)(src[e] - (float)hi[e]);
        }
        const uint64_t o = frag_off(bcol(r, kind), i0, KB);
        *reinterpret_cast<V*>(B + o) = hi;
        *reinterpret_cast<V*>(B + o + kFragLo) = lo;
    }
}

// The same for the FP32 operand: lane -> (column c % 16, k % 4) of the block
// (column block, 16-row block) = ((u >> 6) & 3, u >> 8); one float4 (k, k + 4,
// k + 8, k + 12) per lane, a whole 1 KB block per wave and pass.
__device__ __forceinline__ void dense_tile_store_f32(const DenseArgs& A, uint32_t mt, uint32_t nt,
                                                     const float (*tS)[kRowTile + 1], const float (*tC)[kRowTile + 1])
{
    const uint32_t KB16 = A.Np / 16;
    float* B = static_cast<float*>(A.Bnext);
#pragma unroll
    for (uint32_t j = 0; j < 2 * kRealTile * kRowTile / 4 / kDenseThreads; ++j) {
        const uint32_t u = threadIdx.x + j * kDenseThreads;
        const uint32_t cb = (u >> 6) & 3u, kind = cb >> 1;
        const uint32_t rl = (cb & 1u) * 16 + (u & 15u), il0 = (u >> 8) * 16 + ((u >> 4) & 3u);
        const uint32_t r = nt * kRealTile + rl, i0 = mt * kRowTile + il0;
        if (r >= A.R || i0 >= A.N) continue;
        const float* src = kind ? &tC[rl][il0] : &tS[rl][il0];
        const f32x4 v{src[0], src[4], src[8], src[12]};
        *reinterpret_cast<f32x4*>(B + frag32_off(bcol(r, kind), i0, KB16)) = v;
    }
}

// Sum of the FP32 kernel's four partial 128 x 64 tiles in a fixed order, times the
// exact power of two `inv`, transposed into tS/tC: waves 1..3 go through red,
// wave 0 writes its own straight into the tile, then all lanes add
// ((p1 + p2) + p3).
constexpr uint32_t kSplitK = 4;

__device__ __forceinline__ void dense_reduce_tile(const f32x4 (&acc)[8][4], f32x4 (*red)[32][kWave],
                                                  float (*tS)[kRowTile + 1], float (*tC)[kRowTile + 1], float inv)
{
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    if (wave > 0) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[wave - 1][m * 4 + n][lane] = acc[m][n];
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
                const uint32_t rl = (n & 1) * 16 + (lane & 15u);
#pragma unroll
                for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (lane >> 4) + q] = acc[m][n][q] * inv;
            }
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < 32 * kWave; p += kDenseThreads) {
        const uint32_t quad = p / kWave, l = p % kWave;
        const f32x4 sum = (red[0][quad][l] + red[1][quad][l]) + red[2][quad][l];
        const uint32_t m = quad / 4, n = quad % 4;
        float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
        const uint32_t rl = (n & 1) * 16 + (l & 15u);
#pragma unroll
        for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (l >> 4) + q] += sum[q] * inv;
    }
    __syncthreads();
}

// Split-precision product and stage update of one 128-row x 32-realization
// tile by 8 waves, two per SIMD.  The output (N x 2R = 4096 x 512 at the
// benchmark size) is too small to give each SIMD a large tile of its own, so
// the k loop is split instead: every wave computes the whole 128 x 64 tile
// (128 accumulators) over every eighth 32-k block.  Per block a wave loads
// 16 K and 8 B fragments (24 KB) for 96 MFMAs, and no fragment is loaded
// twice within the CU: 64 B per clock per CU at the MFMA rate, half of what a
// 2 x 2 grid of 64 x 32 wave tiles needs (there the L1 bounds the loop).
// Accumulators and one block of fragments fill a wave's 256 registers, so
// there is no second register set for a prefetch; instead each block is
// swept in two column passes and every fragment register is reloaded for
// the next block as soon as its last MFMA of this block is issued (the loop
// below), at least half a block ahead of its use, and the SIMD's other wave
// computes while one waits.  Per accumulator the products still enter in
// the order hi*hi, hi*lo, lo*hi of each k block.  A 4-wave variant (one
// wave per SIMD, every fourth k block) is a candidate of the autotuner too.
template <typename T, typename V, int NW>
__global__ __launch_bounds__(NW * 64, 1) void dense_mfma_kernel(DenseArgs A)
{
    static_assert(NW == 4 || NW == 8, "4 or 8 waves");
    constexpr uint32_t kThreads = NW * 64, kSplit = NW;
    // Partial tiles are summed in two rounds: waves 4-7 hand theirs to waves
    // 0-3 (red[0..2] and slot3; 8 waves only), then waves 0-3 put theirs in
    // slot3 and red[0..2] and every thread sums its share.  The transposed
    // tile [realization][row] overlays slot3, whose contents are consumed
    // before the tile is written.
    __shared__ f32x4 red[3][32][kWave];
    __shared__ __attribute__((aligned(16))) float tile[2 * kRealTile * (kRowTile + 1)];
    static_assert(sizeof(tile) >= sizeof(f32x4) * 32 * kWave, "slot3 fits under the tile");
    f32x4 (*slot3)[kWave] = reinterpret_cast<f32x4 (*)[kWave]>(tile);
    float (*tS)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile);
    float (*tC)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile + kRealTile * (kRowTile + 1));
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t KB = A.Np / kKStep;
    const uint64_t frag = 2 * 64 * 8;              // elements per k block (hi + lo)
    const uint64_t stream = (uint64_t)KB * frag;  // elements per 16-row block
    const T* pa = static_cast<const T*>(A.K) + (uint64_t)(mt * 8) * stream + lane * 8;
    const T* pb = static_cast<const T*>(A.B) + (uint64_t)(nt * 4) * stream + lane * 8;

    f32x4 acc[8][4];  // [16-row block][column block: sin 0-15, sin 16-31, cos 0-15, cos 16-31]
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    V ah[8], al[8], bh[4], bl[4];
    auto load_b = [&](uint64_t o) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            bh[n] = *reinterpret_cast<const V*>(pb + n * stream + o);
            bl[n] = *reinterpret_cast<const V*>(pb + n * stream + o + kFragLo);
        }
    };
    if (wave < KB) {
        const uint64_t o = (uint64_t)wave * frag;
        load_b(o);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            ah[m] = *reinterpret_cast<const V*>(pa + m * stream + o);
            al[m] = *reinterpret_cast<const V*>(pa + m * stream + o + kFragLo);
        }
    }
    // Two passes over the row blocks per k block: columns 0-1, then 2-3 (a
    // pair of row blocks at a time, so 4 independent accumulators separate
    // an accumulator's dependent MFMAs).  B fragments 0-1 of the next block
    // load after the first pass, 2-3 after the second, and row block m's K
    // fragments right after its last MFMAs: every load goes out at least
    // half a block before its use.  The loads are unconditional (the last
    // block loads itself again) and scheduling barriers keep them in place:
    // with a branch around them the compiler's wait counts must also cover
    // the path that issues none, and it drained every load in flight before
    // the last row block; left free, it sank them to their uses.
    for (uint32_t kb = wave; kb < KB; kb += kSplit) {
        const uint64_t on = (uint64_t)(kb + kSplit < KB ? kb + kSplit : kb) * frag;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int mp = 0; mp < 4; ++mp) {
#pragma unroll
                for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn) {
                        const int m = 2 * mp + mm, n = 2 * half + nn;
                        acc[m][n] = mfma16<T, V>(ah[m], bh[n], acc[m][n]);
                    }
#pragma unroll
                for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn) {
                        const int m = 2 * mp + mm, n = 2 * half + nn;
                        acc[m][n] = mfma16<T, V>(ah[m], bl[n], acc[m][n]);
                    }
#pragma unroll
                for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn) {
                        const int m = 2 * mp + mm, n = 2 * half + nn;
                        acc[m][n] = mfma16<T, V>(al[m], bh[n], acc[m][n]);
                    }
                if (half == 1) {
#pragma unroll
                    for (int mm = 0; mm < 2; ++mm) {
                        const int m = 2 * mp + mm;
                        ah[m] = *reinterpret_cast<const V*>(pa + m * stream + on);
                        al[m] = *reinterpret_cast<const V*>(pa + m * stream + on + kFragLo);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);  // the loads stay right behind their last MFMAs
            }
#pragma unroll
            for (int nn = 0; nn < 2; ++nn) {
                const int n = 2 * half + nn;
                bh[n] = *reinterpret_cast<const V*>(pb + n * stream + on);
                bl[n] = *reinterpret_cast<const V*>(pb + n * stream + on + kFragLo);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // round 1: wave w < 4 adds wave w + 4's partial
    if constexpr (NW == 8) {
        if (wave >= 4) {
            f32x4 (*dst)[kWave] = wave == 7 ? slot3 : red[wave - 4];
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) dst[m * 4 + n][lane] = acc[m][n];
        }
        __syncthreads();
        if (wave < 4) {
            const f32x4 (*src)[kWave] = wave == 3 ? slot3 : red[wave];
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[m][n] += src[m * 4 + n][lane];
        }
        __syncthreads();
    }
    // round 2: all four partials to LDS (wave 0's to slot3), then every
    // thread sums p0 + ((p1 + p2) + p3) for its quads, and after a barrier
    // (slot3 lies under the tile) writes them transposed into the tile,
    // times the exact power of two that undoes the scaling of K
    const float inv = A.scale[1];
    if (wave < 4) {
        f32x4 (*dst)[kWave] = wave == 0 ? slot3 : red[wave - 1];
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) dst[m * 4 + n][lane] = acc[m][n];
    }
    __syncthreads();
    constexpr uint32_t kQuads = 32 * kWave / kThreads;
    f32x4 sum[kQuads];
#pragma unroll
    for (uint32_t k = 0; k < kQuads; ++k) {
        const uint32_t p = threadIdx.x + k * kThreads, quad = p / kWave, l = p % kWave;
        sum[k] = slot3[quad][l] + ((red[0][quad][l] + red[1][quad][l]) + red[2][quad][l]);
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kQuads; ++k) {
        const uint32_t p = threadIdx.x + k * kThreads, quad = p / kWave, l = p % kWave;
        const uint32_t m = quad / 4, n = quad % 4;
        float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
        const uint32_t rl = (n & 1) * 16 + (l & 15u);
#pragma unroll
        for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (l >> 4) + q] = sum[k][q] * inv;
    }
    __syncthreads();
    dense_tile_stage<kThreads>(A, mt, nt, tS, tC);
    dense_tile_store<T, V, kThreads>(A, mt, nt, tS, tC);
}

// ------------------------------------ split MFMA, row-half waves --------
// The one-half kernel's 128 x 64 wave tiles leave no registers for a second
// set of fragments, so a block's loads can only go out as the block before
// it retires.  Here the 8 waves split the tile by rows as well: wave w
// computes the 64 x 64 half r = w & 1 of the tile over every fourth k block
// (slice s = w >> 1), with 64 accumulator registers, and holds two register
// sets of its 16 fragments (4 K and 4 B, hi and lo): each block's loads are
// issued as the block before it starts, a whole block of MFMAs ahead of
// their use.  Per block a wave loads 16 KB for 48 MFMAs (the two row-half
// waves of a slice load the same B fragments, the second from the L1).
// Per accumulator the products enter in the order hi*hi, hi*lo, lo*hi of
// each k block, and the slice partials are summed as
// p0 + ((p1 + p2) + p3).
constexpr int kRowHalfWaves = 8;

template <typename T, typename V>
__global__ __launch_bounds__(kRowHalfWaves * 64, 1) void dense_rowhalf_kernel(DenseArgs A)
{
    constexpr uint32_t kThreads = kRowHalfWaves * 64, kSlices = 4;
    __shared__ f32x4 red[2][3][16][kWave];  // [row half][slice - 1][accumulator][lane]
    __shared__ __attribute__((aligned(16))) float tile[2 * kRealTile * (kRowTile + 1)];
    float (*tS)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile);
    float (*tC)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile + kRealTile * (kRowTile + 1));
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t r = wave & 1u, sl = wave >> 1;
    const uint32_t KB = A.Np / kKStep;
    const uint64_t frag = 2 * 64 * 8;              // elements per k block (hi + lo)
    const uint64_t stream = (uint64_t)KB * frag;  // elements per 16-row block
    // wave-uniform bases (scalar registers); a lane's 16 bytes are element
    // [lane] of each 1 KB fragment, so the loads need one offset register
    const T* pa = static_cast<const T*>(A.K) + (uint64_t)(mt * 8 + 4 * r) * stream;
    const T* pb = static_cast<const T*>(A.B) + (uint64_t)(nt * 4) * stream;

    f32x4 acc[4][4];  // [16-row block of the half][column block: sin 0-15, sin 16-31, cos 0-15, cos 16-31]
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    V a0h[4], a0l[4], b0h[4], b0l[4], a1h[4], a1l[4], b1h[4], b1l[4];
    auto load_set = [&](uint32_t kb, V* ah, V* al, V* bh, V* bl) {
        const uint64_t o = (uint64_t)kb * frag;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            ah[m] = reinterpret_cast<const V*>(pa + m * stream + o)[lane];
            al[m] = reinterpret_cast<const V*>(pa + m * stream + o + kFragLo)[lane];
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            bh[n] = reinterpret_cast<const V*>(pb + n * stream + o)[lane];
            bl[n] = reinterpret_cast<const V*>(pb + n * stream + o + kFragLo)[lane];
        }
    };
    auto mfma_set = [&](const V* ah, const V* al, const V* bh, const V* bl) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah[m], bh[n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah[m], bl[n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(al[m], bh[n], acc[m][n]);
        }
    };
    // Blocks kb (set 0) and kb + 4 (set 1) per iteration; the load of block
    // kb + 8 is clamped to the last block (a spare load at the end, no
    // branch around it), and an odd last block is left in set 0.
    uint32_t kb = sl;
    if (kb < KB) load_set(kb, a0h, a0l, b0h, b0l);
    for (; kb + kSlices < KB; kb += 2 * kSlices) {
        load_set(kb + kSlices, a1h, a1l, b1h, b1l);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay a whole block ahead of their use
        mfma_set(a0h, a0l, b0h, b0l);
        __builtin_amdgcn_sched_barrier(0);
        load_set(min(kb + 2 * kSlices, KB - 1), a0h, a0l, b0h, b0l);
        __builtin_amdgcn_sched_barrier(0);
        mfma_set(a1h, a1l, b1h, b1l);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (kb < KB) mfma_set(a0h, a0l, b0h, b0l);
    // p0 + ((p1 + p2) + p3) per row half into the tile, transposed, times
    // the exact power of two that undoes the scaling of K
    const float inv = A.scale[1];
    if (sl >= 1) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[r][sl - 1][m * 4 + n][lane] = acc[m][n];
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
                const uint32_t rl = (n & 1) * 16 + (lane & 15u);
#pragma unroll
                for (int q = 0; q < 4; ++q) t[rl][(4 * r + m) * 16 + 4 * (lane >> 4) + q] = acc[m][n][q] * inv;
            }
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < 2 * 16 * kWave; p += kThreads) {
        const uint32_t h = p / (16 * kWave), quad = (p / kWave) % 16, l = p % kWave;
        const f32x4 sum = (red[h][0][quad][l] + red[h][1][quad][l]) + red[h][2][quad][l];
        const uint32_t m = 4 * h + quad / 4, n = quad % 4;
        float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
        const uint32_t rl = (n & 1) * 16 + (l & 15u);
#pragma unroll
        for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (l >> 4) + q] += sum[q] * inv;
    }
    __syncthreads();
    dense_tile_stage<kThreads>(A, mt, nt, tS, tC);
    dense_tile_store<T, V, kThreads>(A, mt, nt, tS, tC);
}

// ------------------------------ split MFMA, 4 waves, K through LDS ------
// The one-half kernel's k-sliced 128 x 64 wave tiles with a whole block of
// lookahead: one wave per SIMD, each with two LDS buffers of its own 16 K
// fragments (a block's 8 row blocks, hi and lo; 4 waves x 2 x 16 KB) that
// direct global->LDS loads fill without registers, and two register sets
// of its 8 B fragments.  Every block's loads are issued as the block before
// it starts, and row block m + 1's K fragments are read from LDS while row
// block m's 12 MFMAs issue.  A wave touches only its own buffers, so no
// wave waits for another inside the k loop.  After it the buffers hold the
// slice partials, summed as (p0 + p2) + (p1 + p3), and the tile.
constexpr int kLds4Waves = 4;

template <typename T, typename V>
__global__ __launch_bounds__(kLds4Waves * 64, 1) void dense_lds4_kernel(DenseArgs A)
{
    constexpr uint32_t kThreads = kLds4Waves * 64, kSlices = kLds4Waves;
    __shared__ V xa[kLds4Waves][2][16][kWave];  // [wave][buffer][row block m: hi 2m, lo 2m + 1][lane]
    f32x4 (*red)[32][kWave] = reinterpret_cast<f32x4 (*)[32][kWave]>(&xa[0][0][0][0]);
    float* tile = reinterpret_cast<float*>(&xa[0][0][0][0]) + 2 * 32 * kWave * 4;
    static_assert(2 * 32 * kWave * sizeof(f32x4) + 2 * kRealTile * (kRowTile + 1) * sizeof(float) <= sizeof(xa),
                  "two slice partials and the tile fit in the fragment buffers");
    float (*tS)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile);
    float (*tC)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile + kRealTile * (kRowTile + 1));
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t KB = A.Np / kKStep;
    const uint64_t frag = 2 * 64 * 8;              // elements per k block (hi + lo)
    const uint64_t stream = (uint64_t)KB * frag;  // elements per 16-row block
    const T* pa = static_cast<const T*>(A.K) + (uint64_t)(mt * 8) * stream;
    const T* pb = static_cast<const T*>(A.B) + (uint64_t)(nt * 4) * stream;

    f32x4 acc[8][4];  // [16-row block][column block: sin 0-15, sin 16-31, cos 0-15, cos 16-31]
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    V b0h[4], b0l[4], b1h[4], b1l[4];
    auto load = [&](uint32_t kb, uint32_t buf, V* bh, V* bl) {
        const uint64_t o = (uint64_t)kb * frag;
#pragma unroll
        for (int f = 0; f < 16; ++f)
            __builtin_amdgcn_global_load_lds(
                static_cast<const void*>(pa + (f >> 1) * stream + o + (f & 1) * kFragLo + lane * 8),
                (void __attribute__((address_space(3)))*)&xa[wave][buf][f][0], 16, 0, 0);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            bh[n] = reinterpret_cast<const V*>(pb + n * stream + o)[lane];
            bl[n] = reinterpret_cast<const V*>(pb + n * stream + o + kFragLo)[lane];
        }
    };
    // block kb: its K in buffer buf, its B in (bh, bl); the next block's
    // loads (clamped to the last block: a spare load at the end) go out first
    auto block = [&](uint32_t kb, uint32_t buf, const V* bh, const V* bl, V* nh, V* nl) {
        __builtin_amdgcn_s_waitcnt(0);  // block kb has landed; the reads of the other buffer are done
        load(min(kb + kSlices, KB - 1), buf ^ 1u, nh, nl);
        const V* xs = &xa[wave][buf][0][lane];
        V ah = xs[0], al = xs[kWave];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);
            V qh, ql;
            if (m < 7) {
                qh = xs[(2 * m + 2) * kWave];
                ql = xs[(2 * m + 3) * kWave];
            }
            __builtin_amdgcn_sched_barrier(0);  // the reads stay ahead of the MFMAs
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah, bh[n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah, bl[n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(al, bh[n], acc[m][n]);
            __builtin_amdgcn_sched_barrier(0);  // and the next wait stays behind them
            if (m < 7) {
                ah = qh;
                al = ql;
            }
        }
    };
    uint32_t kb = wave;
    if (kb < KB) load(kb, 0, b0h, b0l);
    for (; kb + kSlices < KB; kb += 2 * kSlices) {
        block(kb, 0, b0h, b0l, b1h, b1l);
        block(kb + kSlices, 1, b1h, b1l, b0h, b0l);
    }
    if (kb < KB) block(kb, 0, b0h, b0l, b1h, b1l);
    __builtin_amdgcn_s_waitcnt(0);  // the spare loads have landed before the buffers are reused
    __syncthreads();
    // (p0 + p2) + (p1 + p3), then the tile, transposed, times the exact power
    // of two that undoes the scaling of K
    if (wave >= 2) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[wave - 2][m * 4 + n][lane] = acc[m][n];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] += red[wave][m * 4 + n][lane];
    }
    __syncthreads();
    const float inv = A.scale[1];
    if (wave == 1) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[0][m * 4 + n][lane] = acc[m][n];
    } else if (wave == 0) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
                const uint32_t rl = (n & 1) * 16 + (lane & 15u);
#pragma unroll
                for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (lane >> 4) + q] = acc[m][n][q] * inv;
            }
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < 32 * kWave; p += kThreads) {
        const uint32_t quad = p / kWave, l = p % kWave;
        const f32x4 v = red[0][quad][l];
        const uint32_t m = quad / 4, n = quad % 4;
        float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
        const uint32_t rl = (n & 1) * 16 + (l & 15u);
#pragma unroll
        for (int q = 0; q < 4; ++q) t[rl][m * 16 + 4 * (l >> 4) + q] += v[q] * inv;
    }
    __syncthreads();
    dense_tile_stage<kThreads>(A, mt, nt, tS, tC);
    dense_tile_store<T, V, kThreads>(A, mt, nt, tS, tC);
}

// Acquire load of a workgroup-scope LDS counter (the wave-pair handshakes).
__device__ __forceinline__ uint32_t lds_acquire_u32(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------- split MFMA, wave pairs sharing K in LDS ----
// One workgroup per 128-row x 32-realization tile, as in the k-sliced
// kernel, but its 8 waves are 4 k slices x 2 column halves: wave w computes
// columns 2c, 2c + 1 (c = w & 1) of the tile over every fourth k block
// (slice s = w >> 1), with 16 accumulators, so two waves need the same K
// fragments of every block.  Each loads its four row blocks (hi and lo)
// straight into the slice's LDS buffer (global_load_lds_dwordx4, no
// registers, double-buffered), and both read all eight from there, a pair
// of row blocks ahead of the MFMAs; the B fragments go to a second register
// set.  Every block's loads are issued as the block before it starts: a
// whole block of lookahead, with the bytes per MFMA of the k-sliced kernel
// (K shared in the pair, no fragment loaded twice into the CU).  The pair
// paces itself through an LDS counter of blocks published (a wave publishes
// block j once its own loads of it have landed and its reads of block j - 1
// are done, so a partner that has seen j published may refill j - 1's
// buffer).  The slice partials are summed as p0 + ((p1 + p2) + p3).
constexpr int kPairWaves = 8;

template <typename T, typename V>
__global__ __launch_bounds__(kPairWaves * 64, 1) void dense_pair_kernel(DenseArgs A)
{
    constexpr uint32_t kThreads = kPairWaves * 64;
    constexpr size_t kXaBytes = 4 * 2 * 16 * kWave * sizeof(V);
    constexpr size_t kRedBytes = 2 * 3 * 16 * kWave * sizeof(f32x4);
    constexpr size_t kTileBytes = 2 * kRealTile * (kRowTile + 1) * sizeof(float);
    constexpr size_t kLdsBytes = kXaBytes > kRedBytes + kTileBytes ? kXaBytes : kRedBytes + kTileBytes;
    // K fragments [slice][buffer][row block m: hi 2m, lo 2m + 1][lane]; after
    // the k loop the same memory holds the partials [column half][slice - 1]
    // and, behind them, the transposed tile.
    __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
    __shared__ uint32_t pub[4][2];
    V (*xa)[2][16][kWave] = reinterpret_cast<V (*)[2][16][kWave]>(lds);
    f32x4 (*red)[3][16][kWave] = reinterpret_cast<f32x4 (*)[3][16][kWave]>(lds);
    float* tile = reinterpret_cast<float*>(lds + kRedBytes);
    float (*tS)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile);
    float (*tC)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile + kRealTile * (kRowTile + 1));
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t c = wave & 1u, s = wave >> 1;
    if (threadIdx.x < 8) (&pub[0][0])[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t KB = A.Np / kKStep;
    const uint32_t n_j = s < KB ? (KB - s + 3) / 4 : 0u;
    const uint64_t frag = 2 * 64 * 8;              // elements per k block (hi + lo)
    const uint64_t stream = (uint64_t)KB * frag;  // elements per 16-row block
    const T* pa = static_cast<const T*>(A.K) + (uint64_t)(mt * 8) * stream;
    const T* pb = static_cast<const T*>(A.B) + (uint64_t)(nt * 4 + 2 * c) * stream + lane * 8;

    f32x4 acc[8][2];  // [row block][this wave's column block: 2c, 2c + 1]
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    V bh[2][2], bl[2][2];  // B of the current block and of the next, by block parity
    // this wave's four row blocks (hi and lo) of block j into buffer j & 1
    auto load_a = [&](uint32_t j) {
        const uint64_t o = (uint64_t)(s + 4 * j) * frag;
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
            const uint32_t m = 4 * c + mm;
#pragma unroll
            for (int lo = 0; lo < 2; ++lo)
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void*>(pa + m * stream + o + lo * kFragLo + lane * 8),
                    (void __attribute__((address_space(3)))*)&xa[s][j & 1u][2 * m + lo][0], 16, 0, 0);
        }
    };
    auto load_b = [&](uint32_t j, V* dh, V* dl) {
        const uint64_t o = (uint64_t)(s + 4 * j) * frag;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            dh[n] = *reinterpret_cast<const V*>(pb + n * stream + o);
            dl[n] = *reinterpret_cast<const V*>(pb + n * stream + o + kFragLo);
        }
    };
    auto spin_until = [&](const uint32_t* p, uint32_t v) {
        uint32_t spins = 0;
        while (lds_acquire_u32(p) < v) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 24)) {  // a partner that never arrives: give up (error flag)
                if (lane == 0) atomicOr(A.flag, 2);
                break;
            }
        }
    };
    // block j with its B in register set P (= j & 1)
    auto block = [&](uint32_t j, auto parity) {
        constexpr int P = decltype(parity)::value;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of block j have landed, its reads of j - 1 are done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(&pub[s][c], j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        spin_until(&pub[s][c ^ 1u], j + 1);
        if (j + 1 < n_j) {  // the partner is done with block j - 1's buffer
            load_a(j + 1);
            load_b(j + 1, bh[P ^ 1], bl[P ^ 1]);
        }
        // a pair of row blocks' fragments is read while the previous pair's
        // 12 MFMAs issue (an LDS-only wait: the next block's loads stay in
        // flight); 4 independent accumulators per group of MFMAs
        const V* xs = &xa[s][j & 1u][0][lane];
        V a[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) a[f] = xs[f * kWave];
#pragma unroll
        for (int mp = 0; mp < 4; ++mp) {
            __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);
            V q[4];
            if (mp < 3) {
#pragma unroll
                for (int f = 0; f < 4; ++f) q[f] = xs[(4 * mp + 4 + f) * kWave];
            }
            __builtin_amdgcn_sched_barrier(0);  // the reads stay ahead of the MFMAs
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    acc[2 * mp + mm][n] = mfma16<T, V>(a[2 * mm], bh[P][n], acc[2 * mp + mm][n]);
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    acc[2 * mp + mm][n] = mfma16<T, V>(a[2 * mm], bl[P][n], acc[2 * mp + mm][n]);
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    acc[2 * mp + mm][n] = mfma16<T, V>(a[2 * mm + 1], bh[P][n], acc[2 * mp + mm][n]);
            __builtin_amdgcn_sched_barrier(0);  // and the next wait stays behind them
            if (mp < 3) {
#pragma unroll
                for (int f = 0; f < 4; ++f) a[f] = q[f];
            }
        }
    };
    if (n_j > 0) {
        load_a(0);
        load_b(0, bh[0], bl[0]);
    }
    for (uint32_t j = 0; j < n_j; j += 2) {
        block(j, std::integral_constant<int, 0>{});
        if (j + 1 < n_j) block(j + 1, std::integral_constant<int, 1>{});
    }
    __syncthreads();  // every wave is done with the fragment buffers the partials overwrite
    if (s >= 1) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) red[c][s - 1][m * 2 + n][lane] = acc[m][n];
    }
    __syncthreads();
    // p0 + ((p1 + p2) + p3), transposed into the tile, times the exact power
    // of two that undoes the scaling of K
    const float inv = A.scale[1];
    if (s == 0) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const uint32_t q = m * 2 + n;
                const f32x4 sum = acc[m][n] + ((red[c][0][q][lane] + red[c][1][q][lane]) + red[c][2][q][lane]);
                const uint32_t cb = 2 * c + n;  // column block: sin 0-15, sin 16-31, cos 0-15, cos 16-31
                float(*t)[kRowTile + 1] = (cb >> 1) ? tC : tS;
                const uint32_t rl = (cb & 1) * 16 + (lane & 15u);
#pragma unroll
                for (int e = 0; e < 4; ++e) t[rl][m * 16 + 4 * (lane >> 4) + e] = sum[e] * inv;
            }
    }
    __syncthreads();
    dense_tile_stage<kThreads>(A, mt, nt, tS, tC);
    dense_tile_store<T, V, kThreads>(A, mt, nt, tS, tC);
}

// ------------------------------------------- split MFMA, two K halves --
// The same product with twice the tile per workgroup, to halve what each
// CU loads per MFMA: a workgroup computes a 128-row x 64-realization tile (two
// realization tiles) over one half of the k range, so two workgroups share
// each tile and a second kernel adds their partial tiles (in half order)
// and runs the stage update.  Eight waves: wave w computes the 128 x 64
// tile of column half c = w & 1 over every fourth k block (slice s = w >> 1)
// of its half.  The two waves of a slice need the same K fragments: each
// loads its four row blocks (hi and lo) straight into LDS
// (global_load_lds_dwordx4, no VGPRs), double-buffered, and reads all eight
// from there row block by row block as its MFMAs go; its own B fragments
// come from global memory into a second register set.  Both loads of block
// j + 1 are issued as block j starts, a whole block of MFMAs ahead.  Per
// block a CU then loads 16 KB per wave against 24 KB in the one-half
// kernel.  The waves of a slice pace each other through an LDS counter of
// blocks published, never a workgroup barrier: a wave publishes block j once
// its own loads of it have landed and its reads of block j - 1 are done, so
// a partner that has seen block j published may refill the buffer of j - 1.
constexpr int kSplit2Waves = 8;
constexpr int kSplit2StageThreads = 512;  // the stage kernel: 8 waves, 4 partial fragments each

// Partial tiles: [half][row tile][realization tile][row block 8][column
// block 4][lane] of f32x4, each (row block, column block) the accumulator of
// one MFMA output block as a wave holds it.
__device__ __forceinline__ uint64_t split2_part(uint32_t h, uint32_t mt, uint32_t nt, uint32_t n_mt, uint32_t n_nt)
{
    return (((uint64_t)h * n_mt + mt) * n_nt + nt) * (32 * kWave);
}

template <typename T, typename V>
__global__ __launch_bounds__(kSplit2Waves * 64, 1) void dense_split2_kernel(DenseArgs A, f32x4* P)
{
    // K fragments by slice, buffer and fragment (row block m: hi at 2m, lo
    // at 2m + 1); after the k loop the same memory holds the slice partials.
    __shared__ V xa[4][2][16][kWave];
    __shared__ uint32_t pub[4][2];
    f32x4 (*red)[32][kWave] = reinterpret_cast<f32x4 (*)[32][kWave]>(&xa[0][0][0][0]);
    static_assert(sizeof(xa) >= 4 * 32 * kWave * sizeof(f32x4), "the slice partials fit in the fragment buffers");
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t c = wave & 1u, s = wave >> 1;
    if (threadIdx.x < 8) (&pub[0][0])[threadIdx.x] = 0u;
    __syncthreads();
    // workgroup -> (row tile mt, tile pair pt, k half h)
    const uint32_t n_mt = A.Mp / kRowTile, n_nt = A.Rp / kRealTile, n_pt = n_nt / 2;
    uint32_t mt, pt, h;
    {
        const uint32_t b = blockIdx.x;
        uint32_t l;
        if (A.band && n_mt % 8 == 0) {
            mt = (b & 7u) * (n_mt / 8);
            l = b >> 3;
            mt += l / (2 * n_pt);
        } else {
            mt = b / (2 * n_pt);
            l = b;
        }
        const uint32_t rem = l % (2 * n_pt);
        pt = rem >> 1;
        h = rem & 1u;
    }
    const uint32_t nt = 2 * pt + c;
    const uint32_t KB = A.Np / kKStep, KBh = (KB + 1) / 2;
    const uint32_t kb0 = h * KBh, kb1 = min(KB, kb0 + KBh);
    const uint32_t first = kb0 + s;
    const uint32_t n_j = first < kb1 ? (kb1 - first + 3) / 4 : 0u;
    const uint64_t frag = 2 * 64 * 8;              // elements per k block (hi + lo)
    const uint64_t stream = (uint64_t)KB * frag;  // elements per 16-row block
    const T* pa = static_cast<const T*>(A.K) + (uint64_t)(mt * 8) * stream;
    const T* pb = static_cast<const T*>(A.B) + (uint64_t)(nt * 4) * stream + lane * 8;

    f32x4 acc[8][4];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    V bh[2][4], bl[2][4];  // B of the current block and of the next, by block parity
    // this wave's four row blocks (hi and lo) of block j into buffer j & 1
    auto load_a = [&](uint32_t j) {
        const uint64_t o = (uint64_t)(first + 4 * j) * frag;
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
            const uint32_t m = 4 * c + mm;
#pragma unroll
            for (int lo = 0; lo < 2; ++lo)
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void*>(pa + m * stream + o + lo * kFragLo + lane * 8),
                    (void __attribute__((address_space(3)))*)&xa[s][j & 1u][2 * m + lo][0], 16, 0, 0);
        }
    };
    auto load_b = [&](uint32_t j, V* dh, V* dl) {
        const uint64_t o = (uint64_t)(first + 4 * j) * frag;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            dh[n] = *reinterpret_cast<const V*>(pb + n * stream + o);
            dl[n] = *reinterpret_cast<const V*>(pb + n * stream + o + kFragLo);
        }
    };
    auto spin_until = [&](const uint32_t* p, uint32_t v) {
        uint32_t spins = 0;
        while (lds_acquire_u32(p) < v) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 24)) {  // a partner that never arrives: give up (error flag)
                if (lane == 0) atomicOr(A.flag, 2);
                break;
            }
        }
    };
    // block j with its B in register set P (= j & 1)
    auto block = [&](uint32_t j, auto parity) {
        constexpr int P = decltype(parity)::value;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of block j have landed, its reads of j - 1 are done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(&pub[s][c], j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        spin_until(&pub[s][c ^ 1u], j + 1);
        if (j + 1 < n_j) {  // the partner is done with block j - 1's buffer
            load_a(j + 1);
            load_b(j + 1, bh[P ^ 1], bl[P ^ 1]);
        }
        // row block m + 1's fragments are read while row block m's 12 MFMAs
        // issue; the wait for row block m's reads comes before the next reads
        // are issued (an LDS-only wait: the next block's loads stay in flight)
        const V* xs = &xa[s][j & 1u][0][lane];
        V ah = xs[0], al = xs[kWave];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);
            V nh, nl;
            if (m < 7) {
                nh = xs[(2 * m + 2) * kWave];
                nl = xs[(2 * m + 3) * kWave];
            }
            __builtin_amdgcn_sched_barrier(0);  // the reads stay ahead of the MFMAs
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah, bh[P][n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(ah, bl[P][n], acc[m][n]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = mfma16<T, V>(al, bh[P][n], acc[m][n]);
            __builtin_amdgcn_sched_barrier(0);  // and the next wait stays behind them
            if (m < 7) {
                ah = nh;
                al = nl;
            }
        }
    };
    if (n_j > 0) {
        load_a(0);
        load_b(0, bh[0], bl[0]);
    }
    for (uint32_t j = 0; j < n_j; j += 2) {
        block(j, std::integral_constant<int, 0>{});
        if (j + 1 < n_j) block(j + 1, std::integral_constant<int, 1>{});
    }
    // slice partials in half order: ((s0 + s2) + (s1 + s3)) per column half
    __syncthreads();
    if (s >= 2) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[(s - 2) * 2 + c][m * 4 + n][lane] = acc[m][n];
    }
    __syncthreads();
    if (s < 2) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] += red[s * 2 + c][m * 4 + n][lane];
    }
    __syncthreads();
    if (s == 1) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) red[c][m * 4 + n][lane] = acc[m][n];
    }
    __syncthreads();
    if (s == 0) {
        f32x4* out = P + split2_part(h, mt, nt, n_mt, n_nt);
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) out[(m * 4 + n) * kWave + lane] = acc[m][n] + red[c][m * 4 + n][lane];
    }
}

// The stage of one 128-row x 32-realization tile from the two halves'
// partials: their sum (half 0 + half 1), unscaled, transposed into the LDS
// tile, then the update and the next operand as in the one-half kernel.
template <typename T, typename V>
__global__ __launch_bounds__(kSplit2StageThreads, 1) void dense_split2_stage_kernel(DenseArgs A, const f32x4* P)
{
    __shared__ __attribute__((aligned(16))) float tile[2 * kRealTile * (kRowTile + 1)];
    float (*tS)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile);
    float (*tC)[kRowTile + 1] = reinterpret_cast<float (*)[kRowTile + 1]>(tile + kRealTile * (kRowTile + 1));
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t n_mt = A.Mp / kRowTile, n_nt = A.Rp / kRealTile;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const f32x4* p0 = P + split2_part(0, mt, nt, n_mt, n_nt);
    const f32x4* p1 = P + split2_part(1, mt, nt, n_mt, n_nt);
    const float inv = A.scale[1];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t q = wave * 4 + k, m = q / 4, n = q % 4;
        const f32x4 v = p0[q * kWave + lane] + p1[q * kWave + lane];
        float(*t)[kRowTile + 1] = (n >> 1) ? tC : tS;
        const uint32_t rl = (n & 1) * 16 + (lane & 15u);
#pragma unroll
        for (int e = 0; e < 4; ++e) t[rl][m * 16 + 4 * (lane >> 4) + e] = v[e] * inv;
    }
    __syncthreads();
    dense_tile_stage<kSplit2StageThreads>(A, mt, nt, tS, tC);
    dense_tile_store<T, V, kSplit2StageThreads>(A, mt, nt, tS, tC);
}

// ------------------------------------------------------------- FP32 MFMA --
// The FP32 product on v_mfma_f32_16x16x4_f32, split over the k loop the
// same way but by 4 waves (one per SIMD): every wave computes the whole
// 128 x 64 tile over every fourth 16-k block.  Per block a wave loads 8 K and
// 4 B float4 fragments (12 KB) and issues 4 x 32 MFMAs (about 4096 cycles),
// so one block of register prefetch covers the memory latency; a second
// wave per SIMD gains nothing here.
__global__ __launch_bounds__(kDenseThreads, 1) void dense_mfma32_kernel(DenseArgs A)
{
    __shared__ f32x4 red[kSplitK - 1][32][kWave];
    __shared__ float tS[kRealTile][kRowTile + 1], tC[kRealTile][kRowTile + 1];
    uint32_t mt, nt;
    tile_of(blockIdx.x, A.Mp / kRowTile, A.Rp / kRealTile, A.band, mt, nt);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t KB16 = A.Np / 16;
    const uint64_t stream = (uint64_t)KB16 * 256;  // floats per 16-row block
    const float* pa = static_cast<const float*>(A.K) + (uint64_t)(mt * 8) * stream + lane * 4;
    const float* pb = static_cast<const float*>(A.B) + (uint64_t)(nt * 4) * stream + lane * 4;

    f32x4 acc[8][4];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 a[8], b[4];
    auto load = [&](uint64_t o) {
#pragma unroll
        for (int m = 0; m < 8; ++m) a[m] = *reinterpret_cast<const f32x4*>(pa + m * stream + o);
#pragma unroll
        for (int n = 0; n < 4; ++n) b[n] = *reinterpret_cast<const f32x4*>(pb + n * stream + o);
    };
    uint32_t kb = wave;
    if (kb < KB16) load((uint64_t)kb * 256);
    for (; kb < KB16; kb += kSplitK) {
        f32x4 ca[8], cb[4];
#pragma unroll
        for (int m = 0; m < 8; ++m) ca[m] = a[m];
#pragma unroll
        for (int n = 0; n < 4; ++n) cb[n] = b[n];
        if (kb + kSplitK < KB16) load((uint64_t)(kb + kSplitK) * 256);  // this wave's next block
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[m][j], cb[n][j], acc[m][n], 0, 0, 0);
    }
    dense_reduce_tile(acc, red, tS, tC, 1.f);
    dense_tile_stage(A, mt, nt, tS, tC);
    dense_tile_store_f32(A, mt, nt, tS, tC);
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

// K -> scaled, padded copy over Mp rows x Np columns (zero outside N x N) in
// the packed layout: FP32, or the 16-bit hi/lo split.
template <typename T>
__global__ void dense_split_kernel(const float* K, uint32_t N, uint32_t Np, uint32_t Mp, const float* scale, void* out)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)Mp * Np) return;
    const uint32_t i = (uint32_t)(g / Np), j = (uint32_t)(g % Np);
    const float x = (i < N && j < N) ? K[(uint64_t)i * N + j] * scale[0] : 0.f;
    if constexpr (sizeof(T) == 4)
        static_cast<float*>(out)[frag32_off(i, j, Np / 16)] = x;
    else
        store_split<T>(static_cast<T*>(out), frag_off(i, j, Np / kKStep), x);
}

// theta [R][N] -> sin/cos operand over 2 Rp columns x Np rows of k (zero in
// the padding) in the packed layout: FP32, or the 16-bit hi/lo split.
template <typename T>
__global__ void dense_operand_kernel(const float* theta, uint32_t N, uint32_t R, uint32_t Np, uint32_t Rp, void* out)
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
    if constexpr (sizeof(T) == 4) {
        static_cast<float*>(out)[frag32_off(bcol(r, 0), j, Np / 16)] = s;
        static_cast<float*>(out)[frag32_off(bcol(r, 1), j, Np / 16)] = c;
    } else {
        T* B = static_cast<T*>(out);
        store_split<T>(B, frag_off(bcol(r, 0), j, Np / kKStep), s);
        store_split<T>(B, frag_off(bcol(r, 1), j, Np / kKStep), c);
    }
}

// ------------------------------------------------------------------ host --
static int ilog2_dense(uint64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

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
    const bool split = sizeof(T) == 2;
    // bytes of the K copy and of one operand buffer (hi and lo for the split)
    const size_t a_bytes = (size_t)Mp * Np * sizeof(T) * (split ? 2 : 1);
    const size_t b_bytes = (size_t)2 * Rp * Np * sizeof(T) * (split ? 2 : 1);
    void *wa = nullptr, *wb = nullptr, *wk = nullptr;
    int st;
    if ((st = ensure_ws(ctx, kSlotDenseA, a_bytes, &wa))) return st;
    if ((st = ensure_ws(ctx, kSlotDenseB, 2 * b_bytes + 64, &wb))) return st;
    if ((st = ensure_ws(ctx, kSlotKuraWork, (size_t)2 * NR * sizeof(float), &wk))) return st;
    char* B0 = static_cast<char*>(wb);
    void* Bbuf[2] = {B0, B0 + b_bytes};
    float* scale = reinterpret_cast<float*>(B0 + 2 * b_bytes);
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(scale + 2);
    float* tilde = static_cast<float*>(wk);
    float* F1 = tilde + NR;

    // scaled, padded copy of K (split into hi/lo for the MFMA variants)
    hipLaunchKernelGGL(dense_zero_kernel, dim3(1), dim3(1), 0, stream, maxbits);
    if (split) hipLaunchKernelGGL(dense_maxabs_kernel, dim3(1024), dim3(256), 0, stream, K, (uint64_t)N * N, maxbits);
    hipLaunchKernelGGL(dense_scale_kernel, dim3(1), dim3(1), 0, stream, maxbits, scale, split ? 0 : 1);
    hipLaunchKernelGGL(dense_split_kernel<T>, dim3((uint32_t)(((uint64_t)Mp * Np + 255) / 256)), dim3(256), 0, stream,
                       K, N, Np, Mp, scale, wa);
    // both operand buffers get their zero padding (rows j >= N, columns of
    // realizations r >= R) here; the epilogues only ever write the live part
    for (int b = 0; b < 2; ++b)
        hipLaunchKernelGGL(dense_operand_kernel<T>, dim3((uint32_t)(((uint64_t)Rp * Np + 255) / 256)), dim3(256), 0,
                           stream, phi, N, R, Np, Rp, Bbuf[b]);
    SDE_HIP(ctx, hipGetLastError());

    DenseArgs A;
    A.K = wa;
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
    A.flag = ctx->flag;
    const uint32_t n_mt = Mp / kRowTile, n_nt = Rp / kRealTile;
    const dim3 grid(n_mt * n_nt);
    uint64_t* nbase = nullptr;
    if ((st = step_counter(ctx, &nbase))) return st;
    A.nbase = nbase;
    // The two-half kernel (16-bit products, an even number of realization
    // tiles): its partial tiles, two per output tile.
    const bool split2_ok = sizeof(T) == 2 && n_nt % 2 == 0;
    void* wpart = nullptr;
    const size_t part_bytes = (size_t)2 * n_mt * n_nt * 32 * kWave * sizeof(f32x4);
    // launch choice: bit 0 = 4 waves instead of 8 (16-bit variants), bit 1 =
    // row tiles in plain order instead of XCD bands, bit 2 = two workgroups
    // per tile over the two halves of k, bit 3 = row-half waves with two
    // register sets, bit 4 = 4 waves with K fragments through LDS (16-bit
    // variants)
    int choice = 0;
    auto launch = [&](hipStream_t s) -> int {
        A.band = (choice & 2) ? 0 : 1;
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL(dense_mfma32_kernel, grid, dim3(kDenseThreads), 0, s, A);
        } else {
            typedef typename std::conditional<__is_same(T, __bf16), bf16x8, f16x8>::type V;
            if (choice & 32) {
                hipLaunchKernelGGL((dense_pair_kernel<T, V>), grid, dim3(kPairWaves * 64), 0, s, A);
            } else if (choice & 16) {
                hipLaunchKernelGGL((dense_lds4_kernel<T, V>), grid, dim3(kLds4Waves * 64), 0, s, A);
            } else if (choice & 8) {
                hipLaunchKernelGGL((dense_rowhalf_kernel<T, V>), grid, dim3(kRowHalfWaves * 64), 0, s, A);
            } else if (choice & 4) {
                f32x4* part = static_cast<f32x4*>(wpart);
                hipLaunchKernelGGL((dense_split2_kernel<T, V>), dim3(n_mt * n_nt), dim3(kSplit2Waves * 64), 0, s, A,
                                   part);
                hipLaunchKernelGGL((dense_split2_stage_kernel<T, V>), grid, dim3(kSplit2StageThreads), 0, s, A,
                                   static_cast<const f32x4*>(part));
            } else if (choice & 1) {
                hipLaunchKernelGGL((dense_mfma_kernel<T, V, 4>), grid, dim3(256), 0, s, A);
            } else {
                hipLaunchKernelGGL((dense_mfma_kernel<T, V, 8>), grid, dim3(512), 0, s, A);
            }
        }
        SDE_HIP(ctx, hipGetLastError());
        return SDE_OK;
    };
    // The choice is tuned per shape class: predictor stages of each
    // candidate from the call's operand (the fastest of three), its phases,
    // carry and next operand going to scratch and to the operand buffer the
    // call's first stage overwrites anyway; the default (8 waves, bands) is
    // kept unless another is more than 3 % faster.
    {
        const bool band_matters = (Mp / kRowTile) % 8 == 0;
        int cands[12], nc = 0;
        for (int c : {0, 1, 2, 3, 4, 6, 8, 10, 16, 18, 32, 34}) {
            if ((c & 57) && sizeof(T) == 4) continue;
            if ((c & 2) && !band_matters) continue;
            if ((c & 4) && !split2_ok) continue;
            cands[nc++] = c;
        }
        const int n_cand = nc;
        if (split2_ok && (st = ensure_ws(ctx, kSlotDenseOut, part_bytes, &wpart))) return st;
        char tkey[160];
        snprintf(tkey, sizeof tkey, "dense%d|%s|N2^%d|R2^%d", d->coupling, ctx->arch.c_str(), ilog2_dense(N),
                 ilog2_dense(R));
        if (ctx->dense_launch) {
            static const int kForced[] = {0, 0, 1, 2, 3, 4, 6, 8, 10, 16, 18, 32, 34};
            choice = kForced[ctx->dense_launch];
        } else if (!tune_lookup(ctx, tkey, &choice)) {
            choice = 0;
            if (ctx->autotune && n_cand > 1) {
                const auto t0 = std::chrono::steady_clock::now();
                void* scratch = nullptr;
                if ((st = ensure_ws(ctx, kSlotTune, (size_t)2 * NR * sizeof(float), &scratch))) return st;
                launch_step_set(nbase, run->step0, stream);
                DenseArgs saved = A;
                A.k = 0;
                A.stage = 1;
                A.euler = 0;
                A.B = Bbuf[0];
                A.Bnext = Bbuf[1];
                A.src = phi;
                A.dst = static_cast<float*>(scratch);
                A.F1 = static_cast<float*>(scratch) + NR;
                A.flag = ctx->tune_flag;
                hipEvent_t e0, e1;
                SDE_HIP(ctx, hipEventCreate(&e0));
                if (hipEventCreate(&e1) != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    return fail(ctx, SDE_ERR_DEVICE, "dense autotuner: hipEventCreate failed");
                }
                // one untimed launch of every candidate (the first launch
                // loads the code object), then three timed rounds over all
                // of them in turn; a candidate's time is its fastest launch
                float ms[12];
                for (int c = 0; c < nc; ++c) ms[c] = 3.4e38f;
                for (int round = 0; round < 4 && st == SDE_OK; ++round) {
                    for (int c = 0; c < nc && st == SDE_OK; ++c) {
                        choice = cands[c];
                        float t = 0.f;
                        if (hipEventRecord(e0, stream) != hipSuccess) st = SDE_ERR_DEVICE;
                        if (!st) st = launch(stream);
                        if (!st && hipEventRecord(e1, stream) != hipSuccess) st = SDE_ERR_DEVICE;
                        if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                            st = SDE_ERR_DEVICE;
                        if (!st && round > 0) ms[c] = std::min(ms[c], t);
                    }
                }
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                if (st == SDE_ERR_DEVICE) return fail(ctx, st, "dense autotuner: HIP event or launch failed");
                if (st) return st;
                int best = 0;
                for (int c = 1; c < nc; ++c)
                    if (ms[c] < 0.97f * ms[best]) best = c;
                choice = cands[best];
                A = saved;
                ctx->last.tuned = 1;
                ctx->last.tune_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                tune_store(ctx, tkey, choice);
            }
        }
        if (choice < 0 || choice > 63) choice = 0;
        if (sizeof(T) == 4) choice &= 2;    // one FP32 kernel (4 waves)
        if (choice & 32) choice &= 34;      // the pair kernel: 8 waves, one workgroup per tile
        if (choice & 16) choice &= 18;      // the 4-wave LDS kernel: one workgroup per tile
        if (choice & 8) choice &= 10;       // the row-half kernel: 8 waves, one workgroup per tile
        if (!split2_ok) choice &= ~4;       // the two-half kernel needs an even number of realization tiles
        if (choice & 4) choice &= 6;        // the two-half kernel has 8 waves
        if (!band_matters) choice &= ~2;    // bands or not: the same order
    }
    ctx->last.dense_waves = sizeof(T) == 4 ? 4 : (choice & 17) ? 4 : 8;
    ctx->last.dense_xcd_bands = (choice & 2) || (Mp / kRowTile) % 8 != 0 ? 0 : 1;
    ctx->last.dense_variant = (choice & 32) ? 4 : (choice & 16) ? 3 : (choice & 8) ? 2 : (choice & 4) ? 1 : 0;
    // `count` steps from the device step base, then advance it.  The operand
    // buffers alternate per stage; chunks hold an even number of stages so a
    // recorded chunk always starts from the same buffer.
    auto record = [&](hipStream_t s, uint32_t count) -> int {
        if (r_samples) launch_order_parameter_at(phi, N, R, r_samples, n_samples, nbase, run->step0, M, s);
        int cur = 0;
        for (uint32_t k = 0; k < count; ++k) {
            A.k = k;
            // stage 1: drift at theta_n; Euler finishes the step in place
            A.stage = 1;
            A.B = Bbuf[cur];
            A.Bnext = Bbuf[cur ^ 1];
            A.src = phi;
            A.dst = A.euler ? phi : tilde;
            int e = launch(s);
            if (e) return e;
            cur ^= 1;
            if (A.euler) continue;
            // stage 2: drift at the predictor; corrector into phi
            A.stage = 2;
            A.B = Bbuf[cur];
            A.Bnext = Bbuf[cur ^ 1];
            A.src = tilde;
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
    snprintf(key, sizeof key, "dense%d|%p|%p|%p|%p|%p|%p|%u|%u|%u|%u|%a|%a|%a|%d|%llu|%u|%llu|v%d", d->coupling,
             (void*)phi, (void*)omega, (void*)r_samples, wa, wb, wk, N, R, A.key0, A.key1, A.omega_scale, A.hdt2pi,
             A.c2, A.euler, (unsigned long long)run->step0, M, (unsigned long long)n_samples, choice);
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
