// valu_issue.hip -- issue cost of single VALU instruction forms on gfx950,
// for the ALU cost model of the benchmark (not part of libsde).
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

}  // namespace

extern "C" {

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

}  // extern "C"
