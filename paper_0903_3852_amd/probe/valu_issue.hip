// valu_issue.hip -- issue cost of single VALU instruction forms on gfx950,
// for the ALU cost model of the benchmark, and the sustained rate of the
// MFMA forms the dense coupling uses (not part of libsde).
//
// Each mode runs one instruction form in 8 independent dependency chains per
// lane, 2048 workgroups of 256 lanes (8 waves per SIMD on 256 CUs), register
// operands only: no memory traffic inside the timed loop.  The caller turns
// the time of a launch into SIMD cycles per wave64 instruction.  The forms
// are written as inline assembly of ALU instructions (no loads), so the
// compiler can neither fold nor move them to the scalar unit.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

#define VP_CHAIN8(STMT)                 \
    {                                   \
        { const int k = 0; STMT; }      \
        { const int k = 1; STMT; }      \
        { const int k = 2; STMT; }      \
        { const int k = 3; STMT; }      \
        { const int k = 4; STMT; }      \
        { const int k = 5; STMT; }      \
        { const int k = 6; STMT; }      \
        { const int k = 7; STMT; }      \
    }

template <int MODE>
__global__ __launch_bounds__(256) void valu_issue_kernel(float* out, int iters, uint32_t su, float sf)
{
    uint32_t x[8], y[8];
    uint64_t w[8];
    double d[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = threadIdx.x * 7u + k;
        y[k] = k * 13u + 1u + threadIdx.x;
        w[k] = x[k];
        d[k] = 1e-3 * (k + threadIdx.x);
    }
    for (int it = 0; it < iters; ++it) {
        if (MODE == 0) VP_CHAIN8(asm volatile("v_add_f32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k])))
        if (MODE == 1) VP_CHAIN8(asm volatile("v_add_f32 %0, %1, %0" : "+v"(x[k]) : "s"(sf)))
        if (MODE == 2) VP_CHAIN8(asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x[k]) : "v"(y[k]), "v"(y[(k + 1) & 7])))
        if (MODE == 3) VP_CHAIN8(asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x[k]) : "s"(sf), "v"(y[k])))
        if (MODE == 4) VP_CHAIN8(asm volatile("v_mul_f32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k])))
        if (MODE == 5) VP_CHAIN8(asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k])))
        if (MODE == 6) VP_CHAIN8(asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x[k]) : "s"(su)))
        if (MODE == 7) VP_CHAIN8(asm volatile("v_add_u32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k])))
        if (MODE == 8) VP_CHAIN8(asm volatile("v_lshrrev_b32 %0, 8, %0" : "+v"(x[k])))
        if (MODE == 9) VP_CHAIN8({
            uint64_t c;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[k]), "=s"(c) : "v"(y[k]), "s"(su));
        })
        if (MODE == 10) VP_CHAIN8(asm volatile("v_mul_hi_u32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k])))
        if (MODE == 11) VP_CHAIN8(asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(x[k])))
        if (MODE == 12) VP_CHAIN8(asm volatile("v_floor_f32 %0, %0" : "+v"(x[k])))
        if (MODE == 13) VP_CHAIN8(asm volatile("v_add_f64 %0, %1, %0" : "+v"(d[k]) : "v"(d[(k + 1) & 7])))
        if (MODE == 14) VP_CHAIN8(asm volatile("v_fma_f64 %0, %1, %1, %0" : "+v"(d[k]) : "v"(d[(k + 1) & 7])))
        if (MODE == 15) VP_CHAIN8(asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d[k]) : "v"(x[(k + 1) & 7])))
        if (MODE == 16) VP_CHAIN8(asm volatile("v_sin_f32 %0, %0" : "+v"(x[k])))
        if (MODE == 17) VP_CHAIN8(asm volatile("v_cos_f32 %0, %0" : "+v"(x[k])))
        if (MODE == 18) VP_CHAIN8(asm volatile("v_log_f32 %0, %0" : "+v"(x[k])))
        if (MODE == 19) VP_CHAIN8(asm volatile("v_sqrt_f32 %0, %0" : "+v"(x[k])))
        if (MODE == 20) VP_CHAIN8(asm volatile("v_mov_b32_dpp %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf" : "=v"(x[k]) : "v"(y[k])))
        if (MODE == 21) VP_CHAIN8(asm volatile("v_mov_b32 %0, %1" : "=v"(x[k]) : "v"(y[(k + 3) & 7])))
        // the 2-cycle forms with one VGPR operand and inline constants (no
        // second VGPR read, so no register-bank conflict between operands)
        if (MODE == 22) VP_CHAIN8(asm volatile("v_add_f32 %0, 1.0, %0" : "+v"(x[k])))
        if (MODE == 23) VP_CHAIN8(asm volatile("v_fma_f32 %0, %0, 0.5, 1.0" : "+v"(x[k])))
        if (MODE == 24) VP_CHAIN8(asm volatile("v_mul_f32 %0, 0.5, %0" : "+v"(x[k])))
        if (MODE == 25) VP_CHAIN8(asm volatile("v_xor_b32 %0, 63, %0" : "+v"(x[k])))
        if (MODE == 26) VP_CHAIN8(asm volatile("v_add_u32 %0, 17, %0" : "+v"(x[k])))
    }
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += (float)x[k] + (float)y[k] + (float)w[k] + (float)d[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int MODE>
float time_mode(float* out, int iters)
{
    const int blocks = 2048;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    hipLaunchKernelGGL(valu_issue_kernel<MODE>, dim3(blocks), dim3(256), 0, 0, out, 16, 0xD2511F53u, 1e-7f);
    float best = -1.f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(valu_issue_kernel<MODE>, dim3(blocks), dim3(256), 0, 0, out, iters, 0xD2511F53u, 1e-7f);
        (void)hipEventRecord(e1, 0);
        float ms = -1.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = -1.f;
            break;
        }
        if (best < 0.f || ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

typedef float (*TimeFn)(float*, int);
const TimeFn kModes[] = {time_mode<0>,  time_mode<1>,  time_mode<2>,  time_mode<3>,  time_mode<4>,  time_mode<5>,
                         time_mode<6>,  time_mode<7>,  time_mode<8>,  time_mode<9>,  time_mode<10>, time_mode<11>,
                         time_mode<12>, time_mode<13>, time_mode<14>, time_mode<15>, time_mode<16>, time_mode<17>,
                         time_mode<18>, time_mode<19>, time_mode<20>, time_mode<21>, time_mode<22>, time_mode<23>,
                         time_mode<24>, time_mode<25>, time_mode<26>};

// Matrix-core rate: every wave issues 8 independent accumulator chains of
// one MFMA form, operands in registers, no memory traffic in the loop.
// FORM 0: v_mfma_f32_16x16x32_bf16 (16384 FLOP), 1: v_mfma_f32_16x16x32_f16,
// 2: v_mfma_f32_16x16x4_f32 (2048 FLOP).
typedef __bf16 vp_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 vp_f16x8 __attribute__((ext_vector_type(8)));
typedef float vp_f32x4 __attribute__((ext_vector_type(4)));

template <int FORM>
__global__ __launch_bounds__(256) void mfma_rate_kernel(float* out, int iters)
{
    vp_f32x4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = vp_f32x4{0.f, 0.f, 0.f, 0.f};
    const float x = 1e-3f * (float)(threadIdx.x & 15u);
    vp_bf16x8 ab, bb;
    vp_f16x8 ah, bh;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        ab[e] = (__bf16)(x + e);
        bb[e] = (__bf16)(x - e);
        ah[e] = (_Float16)(x + e);
        bh[e] = (_Float16)(x - e);
    }
    const float y = x + 1.f;
    // inline assembly keeps the accumulators in place in VGPRs (the builtins
    // let the compiler shuffle them through AGPRs every iteration); each
    // chain's next MFMA comes 8 MFMAs later, past the result latency
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (FORM == 0) asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+v"(acc[k]) : "v"(ab), "v"(bb));
            if (FORM == 1) asm volatile("v_mfma_f32_16x16x32_f16 %0, %1, %2, %0" : "+v"(acc[k]) : "v"(ah), "v"(bh));
            if (FORM == 2) asm volatile("v_mfma_f32_16x16x4_f32 %0, %1, %2, %0" : "+v"(acc[k]) : "v"(x), "v"(y));
        }
    }
    // wait states before VALU reads MFMA results (the compiler does not see
    // inside the assembly)
    asm volatile("s_nop 7\n s_nop 7\n s_nop 7" ::: "memory");
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int FORM>
float time_mfma(float* out, int blocks, int iters)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    hipLaunchKernelGGL(mfma_rate_kernel<FORM>, dim3(blocks), dim3(256), 0, 0, out, 16);
    float best = -1.f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(mfma_rate_kernel<FORM>, dim3(blocks), dim3(256), 0, 0, out, iters);
        (void)hipEventRecord(e1, 0);
        float ms = -1.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = -1.f;
            break;
        }
        if (best < 0.f || ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

typedef float (*MfmaFn)(float*, int, int);
const MfmaFn kMfmaForms[] = {time_mfma<0>, time_mfma<1>, time_mfma<2>};

// MFMAs fed from memory: per iteration a wave issues NL 1 KB fragment loads
// (global_load_dwordx4, 64 lanes x 16 B) for the next iteration into one of
// two register sets and 96 v_mfma_f32_16x16x32_bf16 on the fragments of the
// other, loaded one iteration earlier -- the data flow of the dense coupling
// kernel (24 loads per 96 MFMAs; 16 when the K fragments are shared through
// LDS).  The fragments come from a buffer of `words` 16-byte words that
// every wave sweeps at its own offset.
template <int NL>
__global__ __launch_bounds__(512) void mfma_feed_kernel(const vp_bf16x8* src, uint32_t words, float* out, int iters)
{
    const uint32_t gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
    vp_f32x4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = vp_f32x4{0.f, 0.f, 0.f, 0.f};
    vp_bf16x8 f0[NL], f1[NL];
    uint32_t pos = (gw * 7919u * 64u) % words;
    auto load = [&](vp_bf16x8* f) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            uint32_t w = pos + (uint32_t)i * 64u + lane;
            w = w < words ? w : w - words;
            f[i] = src[w];
        }
        pos += NL * 64u;
        pos = pos < words ? pos : pos - words;
    };
    auto mfmas = [&](const vp_bf16x8* f) {
#pragma unroll
        for (int q = 0; q < 96; ++q)
            acc[q & 7] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[q % NL], f[(q * 5 + 3) % NL], acc[q & 7], 0, 0, 0);
    };
    load(f0);
    for (int it = 0; it < iters; it += 2) {
        load(f1);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay a whole iteration ahead of their use
        mfmas(f0);
        __builtin_amdgcn_sched_barrier(0);
        load(f0);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(f1);
        __builtin_amdgcn_sched_barrier(0);
    }
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int NL>
float time_feed(const vp_bf16x8* src, uint32_t words, float* out, int blocks, int iters)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    hipLaunchKernelGGL(mfma_feed_kernel<NL>, dim3(blocks), dim3(512), 0, 0, src, words, out, 2);
    float best = -1.f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(mfma_feed_kernel<NL>, dim3(blocks), dim3(512), 0, 0, src, words, out, iters);
        (void)hipEventRecord(e1, 0);
        float ms = -1.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = -1.f;
            break;
        }
        if (best < 0.f || ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

typedef float (*FeedFn)(const vp_bf16x8*, uint32_t, float*, int, int);
const FeedFn kFeed[] = {time_feed<24>, time_feed<16>, time_feed<8>};
const int kFeedLoads[] = {24, 16, 8};

}  // namespace

extern "C" {

// Times MFMA form `form` (0 bf16 16x16x32, 1 f16 16x16x32, 2 f32 16x16x4):
// `blocks` workgroups of 256 lanes (4 waves), each wave `iters` iterations
// of 8 independent MFMAs; the best of three launches in milliseconds to *ms.
// Returns 0, or -1 on a bad argument or a HIP error.  Device memory: one
// float per lane, owned by the call.
int mfma_rate_time(int form, int blocks, int iters, float* ms)
{
    if (!ms || form < 0 || form >= (int)(sizeof(kMfmaForms) / sizeof(kMfmaForms[0])) || blocks < 1 ||
        blocks > 65536 || iters < 1)
        return -1;
    float* out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return -1;
    *ms = kMfmaForms[form](out, blocks, iters);
    const hipError_t e = hipDeviceSynchronize();
    (void)hipFree(out);
    return (e == hipSuccess && *ms > 0.f) ? 0 : -1;
}


// Number of instruction forms.
int valu_issue_modes(void) { return (int)(sizeof(kModes) / sizeof(kModes[0])); }

// Times form `mode` (0 <= mode < valu_issue_modes()): the best of three
// launches of `iters` loop iterations, each 8 instructions per lane, 2048
// workgroups x 256 lanes.  Writes milliseconds to *ms; returns 0, or -1 on a
// bad argument or a HIP error.  Device memory: one float per lane, owned by
// the call.
int valu_issue_time(int mode, int iters, float* ms)
{
    if (!ms || mode < 0 || mode >= valu_issue_modes() || iters < 1) return -1;
    float* out = nullptr;
    if (hipMalloc(&out, (size_t)2048 * 256 * sizeof(float)) != hipSuccess) return -1;
    *ms = kModes[mode](out, iters);
    const hipError_t e = hipDeviceSynchronize();
    (void)hipFree(out);
    return (e == hipSuccess && *ms > 0.f) ? 0 : -1;
}

// Times the memory-fed MFMA stream with `loads` (24, 16 or 8) fragment loads
// per 96 MFMAs: `blocks` workgroups of 8 waves (256 blocks: 2 waves per
// SIMD), `iters` iterations (even), fragments from a device buffer of
// `bytes` bytes (a multiple of 1 KB, at least 64 KB) that the call
// allocates and zero-fills.  Milliseconds of the best of three launches to
// *ms; returns 0, or -1 on a bad argument or a HIP error.
int mfma_feed_time(int loads, int blocks, int iters, long long bytes, float* ms)
{
    int form = -1;
    for (int i = 0; i < 3; ++i)
        if (kFeedLoads[i] == loads) form = i;
    if (!ms || form < 0 || blocks < 1 || blocks > 8192 || iters < 2 || (iters & 1) || bytes < 65536 ||
        bytes % 1024 != 0 || bytes > (1ll << 32))
        return -1;
    float* out = nullptr;
    void* src = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 512 * sizeof(float)) != hipSuccess) return -1;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess || hipMemset(src, 0, (size_t)bytes) != hipSuccess) {
        (void)hipFree(out);
        if (src) (void)hipFree(src);
        return -1;
    }
    *ms = kFeed[form](static_cast<const vp_bf16x8*>(src), (uint32_t)(bytes / 16), out, blocks, iters);
    const hipError_t e = hipDeviceSynchronize();
    (void)hipFree(out);
    (void)hipFree(src);
    return (e == hipSuccess && *ms > 0.f) ? 0 : -1;
}

}  // extern "C"
