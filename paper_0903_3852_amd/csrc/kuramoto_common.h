// kuramoto_common.h -- pieces shared by the Kuramoto translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sde_internal.h"

namespace sde {

// Per-call constants of a Kuramoto integration (phases in revolutions).
struct KuraConsts {
    float omega_scale;  // dt / (2 pi): revolutions per unit of drift
    float hdt2pi;       // dt / (4 pi)
    float kn;           // K / N (uniform coupling)
    float c2;           // -2 ln2 sigma^2 with sigma = sqrt(2 D dt) / (2 pi)
};

KuraConsts kuramoto_consts(const sde_kuramoto_desc* d);

// Order parameter of every realization of theta [R][N] into out[r*stride + col].
void launch_order_parameter(const float* theta, uint32_t N, uint32_t R, double* out, uint64_t stride,
                            uint64_t col, hipStream_t stream);
// Order parameter at local step *nbase - step0 when it is a multiple of M.
void launch_order_parameter_at(const float* theta, uint32_t N, uint32_t R, double* out, uint64_t stride,
                               const uint64_t* nbase, uint64_t step0, uint32_t M, hipStream_t stream);
void launch_step_set(uint64_t* nbase, uint64_t v, hipStream_t stream);
void launch_step_advance(uint64_t* nbase, uint32_t by, hipStream_t stream);
// Steps per recorded chunk: a divisor of M (at most 128; even if asked).
uint32_t chunk_steps(uint32_t M, uint64_t n_steps, bool even);
// theta = U(Philox(0, i, r, INIT).x0) for every oscillator.
void launch_kuramoto_init(float* theta, uint32_t N, uint32_t R, uint64_t seed, hipStream_t stream);

int dense_impl(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi, const float* omega,
               const float* K, double* r_samples, uint64_t n_samples, uint32_t M, hipStream_t stream);

}  // namespace sde
