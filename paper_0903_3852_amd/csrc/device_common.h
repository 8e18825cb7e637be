// device_common.h -- gfx950 device primitives shared by the integrators:
// the counter-based generator, the Gaussian transform, phase helpers and
// deterministic wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sde {

constexpr int kWave = 64;  // CDNA wavefront width

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Ten rounds; each
// round forms the two 64-bit products of counter words 0 and 2 with fixed
// multipliers (one v_mad_u64_u32 each), swaps and xors the halves with
// words 1 and 3 and the round key; the key advances by two Weyl constants.
// Counter words that are wave-uniform (step block, point, tag) keep their
// early rounds on the scalar unit: the compiler's uniformity analysis places
// them in SGPRs, so round 1 costs no VALU multiply at all.  Once the words
// are per-lane (when only counter word 1 varies across the wave, as in every
// stream here: output word 0 from the fourth round, word 2 from the fifth),
// each three-way xor is one v_bitop3_b32 (truth table 0x96) instead of two
// v_xor_b32; earlier rounds keep the plain xors so that their uniform parts
// can stay scalar.
// --------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

template <int R>
__device__ __forceinline__ uint32_t philox_xor3(uint32_t a, uint32_t b, uint32_t k)
{
    if constexpr (R >= 3)
        return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
    else
        return a ^ b ^ k;
}

template <int R>
__device__ __forceinline__ void philox_round(U4& c, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = philox_xor3<R>((uint32_t)(p1 >> 32), c.y, k0);
    n.y = (uint32_t)p1;
    n.z = philox_xor3<R - 1>((uint32_t)(p0 >> 32), c.w, k1);  // word 3 stays uniform one round longer
    n.w = (uint32_t)p0;
    c = n;
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    philox_round<0>(c, k0, k1);
    philox_round<1>(c, k0 + W0, k1 + W1);
    philox_round<2>(c, k0 + 2 * W0, k1 + 2 * W1);
    philox_round<3>(c, k0 + 3 * W0, k1 + 3 * W1);
    philox_round<4>(c, k0 + 4 * W0, k1 + 4 * W1);
    philox_round<5>(c, k0 + 5 * W0, k1 + 5 * W1);
    philox_round<6>(c, k0 + 6 * W0, k1 + 6 * W1);
    philox_round<7>(c, k0 + 7 * W0, k1 + 7 * W1);
    philox_round<8>(c, k0 + 8 * W0, k1 + 8 * W1);
    philox_round<9>(c, k0 + 9 * W0, k1 + 9 * W1);
    return c;
}

// --------------------------------------------------------------------------
// Box-Muller on 24-bit uniforms.  u1 = ((x >> 8) + 1) 2^-24 lies in (0, 1]
// and u2 = (x >> 8) 2^-24 in [0, 1); both are exact in FP32, so the GPU feeds
// the same real numbers into log and sin/cos as an FP64 reference does.
// rho = sqrt(-2 ln u1) = sqrt(-2 ln2 * log2 u1) with the hardware log2;
// v_sin/v_cos take their argument in revolutions, so u2 goes in unscaled.
// --------------------------------------------------------------------------
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, float& g0, float& g1)
{
    const float u1 = (float)((x0 >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(x1 >> 8) * 0x1p-24f;
    const float rho = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
    g0 = rho * __builtin_amdgcn_cosf(u2);
    g1 = rho * __builtin_amdgcn_sinf(u2);
}

// The four Gaussians of Philox block `c` (steps 4b .. 4b+3 of a stream).
__device__ __forceinline__ void gauss4(U4 c, uint32_t k0, uint32_t k1, float g[4])
{
    const U4 x = philox4x32_10(c, k0, k1);
    box_muller(x.x, x.y, g[0], g[1]);
    box_muller(x.z, x.w, g[2], g[3]);
}

// Box-Muller with the amplitude folded into the radius:
// sigma * rho = sqrt(c2 * log2 u1) with c2 = -2 ln2 sigma^2 (wave-uniform).
__device__ __forceinline__ void box_muller_scaled(uint32_t x0, uint32_t x1, float c2, float& g0, float& g1)
{
    const float u1 = (float)((x0 >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(x1 >> 8) * 0x1p-24f;
    const float rho = __builtin_amdgcn_sqrtf(c2 * __builtin_amdgcn_logf(u1));
    g0 = rho * __builtin_amdgcn_cosf(u2);
    g1 = rho * __builtin_amdgcn_sinf(u2);
}

// sigma * (the four Gaussians of block c), c2 = -2 ln2 sigma^2.
__device__ __forceinline__ void gauss4_scaled(U4 c, uint32_t k0, uint32_t k1, float c2, float g[4])
{
    const U4 x = philox4x32_10(c, k0, k1);
    box_muller_scaled(x.x, x.y, c2, g[0], g[1]);
    box_muller_scaled(x.z, x.w, c2, g[2], g[3]);
}

// sigma * Gaussian j (0..3) of block c alone, by the same operations that
// gauss4_scaled applies for that output (pair j / 2, cosine for even j).
// j should be wave-uniform.
__device__ __forceinline__ float gauss1_scaled(U4 c, uint32_t k0, uint32_t k1, float c2, uint32_t j)
{
    const U4 x = philox4x32_10(c, k0, k1);
    const uint32_t w1 = j < 2 ? x.x : x.z, w2 = j < 2 ? x.y : x.w;
    const float u1 = (float)((w1 >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(w2 >> 8) * 0x1p-24f;
    const float rho = __builtin_amdgcn_sqrtf(c2 * __builtin_amdgcn_logf(u1));
    return rho * ((j & 1u) ? __builtin_amdgcn_sinf(u2) : __builtin_amdgcn_cosf(u2));
}

// Load of wave-uniform read-only data through the constant address space,
// so that it becomes a scalar (SMEM) load into SGPRs.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized types only");
    typedef const __attribute__((address_space(4))) uint32_t cword;
    cword* src = (cword*)(p);
    T out;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
    return out;
}

// sin(2 pi t) for a phase t in revolutions (hardware domain |t| < 256).
__device__ __forceinline__ float sin_rev(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float cos_rev(float t) { return __builtin_amdgcn_cosf(t); }

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// --------------------------------------------------------------------------
// Deterministic FP64 wavefront sum (butterfly over the 64 lanes; every lane
// ends with the same value and the order of additions is fixed).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

}  // namespace sde
