// observables.hip -- ensemble averages of per-path / per-oscillator arrays
// (the quantities of interest of Sec. 4: averages over realizations, the
// asymptotic velocity of Sec. 5, the Kuramoto order parameter).
//
// One workgroup per group.  Thread t takes elements t, t + 256, ... in FP64;
// partial sums are combined by a wavefront butterfly and then by wave index
// through LDS, always in the same order, so results are bitwise
// reproducible.  The spread is taken about the mean in a second pass over
// the group (no cancellation from sum of squares minus squared sum).
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "sde_internal.h"

namespace sde {

constexpr int kObsThreads = 256;

__device__ double block_sum(double x, double* lds)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    x = wave_sum(x);
    if (lane == 0) lds[wid] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kObsThreads / kWave; ++w) t += lds[w];
    __syncthreads();
    return t;
}

template <typename T>
__device__ __forceinline__ double load_value(const void* in, uint64_t i, int square)
{
    const double x = (double)static_cast<const T*>(in)[i];
    return square ? x * x : x;
}

__global__ __launch_bounds__(kObsThreads) void obs_kernel(int kind, const void* in, const uint64_t* first,
                                                          const uint32_t* counts, double* out)
{
    __shared__ double lds[kObsThreads / kWave];
    const uint32_t g = blockIdx.x;
    const uint64_t base = first[g];
    const uint32_t n = counts[g];
    if (kind == SDE_OBS_ORDER) {
        double c = 0.0, s = 0.0;
        for (uint32_t i = threadIdx.x; i < n; i += kObsThreads) {
            double sn, cs;
            sincospi(2.0 * (double)static_cast<const float*>(in)[base + i], &sn, &cs);
            c += cs;
            s += sn;
        }
        c = block_sum(c, lds);
        s = block_sum(s, lds);
        if (threadIdx.x == 0) {
            const double inv = n ? 1.0 / (double)n : 0.0;
            out[2 * g] = std::sqrt(c * c + s * s) * inv;
            out[2 * g + 1] = n ? atan2(s, c) / (2.0 * M_PI) : 0.0;
        }
        return;
    }
    const int square = kind == SDE_OBS_MEANSQ_F32;
    double sum = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kObsThreads)
        sum += kind == SDE_OBS_MEAN_F64 ? load_value<double>(in, base + i, 0) : load_value<float>(in, base + i, square);
    sum = block_sum(sum, lds);
    const double mean = n ? sum / (double)n : 0.0;
    double ss = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kObsThreads) {
        const double x = kind == SDE_OBS_MEAN_F64 ? load_value<double>(in, base + i, 0)
                                                  : load_value<float>(in, base + i, square);
        ss += (x - mean) * (x - mean);
    }
    ss = block_sum(ss, lds);
    if (threadIdx.x == 0) {
        out[2 * g] = mean;
        out[2 * g + 1] = n > 1 ? std::sqrt(ss / (double)(n - 1) / (double)n) : 0.0;
    }
}

// ---- coarse-grained position histogram (one bin per potential period) ----
// With x = theta + winding and theta in [0, 1), the bin of x is its winding
// count, so the histogram is an integer histogram of `winding`.  Each
// workgroup counts its grid-stride share in LDS (32-bit; the grid keeps a
// workgroup's share below 2^31) and adds its bins to the 64-bit totals;
// more bins than fit in LDS go straight to global 64-bit atomics.  Integer
// sums: the result does not depend on the order.
constexpr uint32_t kHistLds = 8192;

__global__ void hist_zero_kernel(uint64_t* counts, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counts[i] = 0ull;
}

// Row r = blockIdx.y, blockIdx.y + gridDim.y, ... of `rows` rows of n
// windings each (row pitch `pitch`), counted into counts[r][nb + 2].
__global__ __launch_bounds__(256) void hist_kernel(const int32_t* w, uint64_t n, uint64_t pitch, uint64_t rows,
                                                   int64_t x0, uint32_t nb, uint64_t* counts)
{
    __shared__ uint32_t h[kHistLds];
    const bool lds = nb + 2 <= kHistLds;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const int32_t* wr = w + r * pitch;
        uint64_t* cr = counts + r * (uint64_t)(nb + 2);
        if (lds)
            for (uint32_t i = threadIdx.x; i < nb + 2; i += blockDim.x) h[i] = 0u;
        __syncthreads();
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const int64_t d = (int64_t)wr[i] - x0;
            const uint32_t b = d < 0 ? 0u : d >= (int64_t)nb ? nb + 1 : (uint32_t)d + 1;
            if (lds)
                atomicAdd(&h[b], 1u);
            else
                atomicAdd(reinterpret_cast<unsigned long long*>(cr + b), 1ull);
        }
        __syncthreads();
        if (lds)
            for (uint32_t i = threadIdx.x; i < nb + 2; i += blockDim.x)
                if (h[i]) atomicAdd(reinterpret_cast<unsigned long long*>(cr + i), (unsigned long long)h[i]);
        __syncthreads();  // h is cleared for the next row
    }
}

int histogram_impl(sde_ctx* ctx, const int32_t* winding, uint64_t n, uint64_t pitch, uint64_t n_rows, int64_t x0,
                   uint32_t n_bins, uint64_t* counts, hipStream_t stream)
{
    if ((!winding && n) || !counts) return fail(ctx, SDE_ERR_INVALID, "null winding or counts");
    if (n_bins == 0 || n_bins > (1u << 24)) return fail(ctx, SDE_ERR_INVALID, "n_bins must be in [1, 2^24]");
    if (n_rows == 0 || n_rows > (1ull << 32)) return fail(ctx, SDE_ERR_INVALID, "n_rows must be in [1, 2^32]");
    if (n_rows > 1 && pitch < n) return fail(ctx, SDE_ERR_INVALID, "row pitch below the row length");
    if (!aligned(winding, 4) || !aligned(counts, 8)) return fail(ctx, SDE_ERR_INVALID, "misaligned pointer");
    const uint64_t nc = (uint64_t)(n_bins + 2) * n_rows;
    const uint64_t zb = (nc + 255) / 256;
    if (zb > 0x7fffffffull) return fail(ctx, SDE_ERR_INVALID, "too many counts");
    hipLaunchKernelGGL(hist_zero_kernel, dim3((uint32_t)zb), dim3(256), 0, stream, counts, nc);
    if (n) {
        // about 4 workgroups per CU in all, at least one per row (up to 65535
        // rows in flight), at most 2^31 windings per workgroup
        const uint64_t gy = std::min<uint64_t>(n_rows, 65535);
        uint64_t gx = std::max<uint64_t>(1, (uint64_t)ctx->n_cu * 4 / gy);
        gx = std::min<uint64_t>(gx, (n + 255) / 256);
        gx = std::max<uint64_t>(gx, (n >> 31) + 1);
        hipLaunchKernelGGL(hist_kernel, dim3((uint32_t)gx, (uint32_t)gy), dim3(256), 0, stream, winding, n,
                           n_rows > 1 ? pitch : n, n_rows, x0, n_bins, counts);
    }
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

// Histogram of phases in revolutions (the density P(x; t) of Fig. 4): bin
// b = floor(theta * nb) for theta in [0, 1] (theta = 1 into the last bin),
// anything else (outside [0, 1], NaN) into bin nb.  theta * nb is formed in
// FP64, exactly for nb < 2^29, so the bin is the exact floor.  Rows and LDS
// bins as hist_kernel.
__global__ __launch_bounds__(256) void phase_hist_kernel(const float* th, uint64_t n, uint64_t pitch, uint64_t rows,
                                                         uint32_t nb, uint64_t* counts)
{
    __shared__ uint32_t h[kHistLds];
    const bool lds = nb + 1 <= kHistLds;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const float* tr = th + r * pitch;
        uint64_t* cr = counts + r * (uint64_t)(nb + 1);
        if (lds)
            for (uint32_t i = threadIdx.x; i < nb + 1; i += blockDim.x) h[i] = 0u;
        __syncthreads();
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const float t = tr[i];
            uint32_t b = nb;
            if (t >= 0.f && t <= 1.f) b = min((uint32_t)floor((double)t * (double)nb), nb - 1);
            if (lds)
                atomicAdd(&h[b], 1u);
            else
                atomicAdd(reinterpret_cast<unsigned long long*>(cr + b), 1ull);
        }
        __syncthreads();
        if (lds)
            for (uint32_t i = threadIdx.x; i < nb + 1; i += blockDim.x)
                if (h[i]) atomicAdd(reinterpret_cast<unsigned long long*>(cr + i), (unsigned long long)h[i]);
        __syncthreads();
    }
}

int phase_histogram_impl(sde_ctx* ctx, const float* theta, uint64_t n, uint64_t pitch, uint64_t n_rows,
                         uint32_t n_bins, uint64_t* counts, hipStream_t stream)
{
    if ((!theta && n) || !counts) return fail(ctx, SDE_ERR_INVALID, "null theta or counts");
    if (n_bins == 0 || n_bins > (1u << 24)) return fail(ctx, SDE_ERR_INVALID, "n_bins must be in [1, 2^24]");
    if (n_rows == 0 || n_rows > (1ull << 32)) return fail(ctx, SDE_ERR_INVALID, "n_rows must be in [1, 2^32]");
    if (n_rows > 1 && pitch < n) return fail(ctx, SDE_ERR_INVALID, "row pitch below the row length");
    if (!aligned(theta, 4) || !aligned(counts, 8)) return fail(ctx, SDE_ERR_INVALID, "misaligned pointer");
    const uint64_t nc = (uint64_t)(n_bins + 1) * n_rows;
    const uint64_t zb = (nc + 255) / 256;
    if (zb > 0x7fffffffull) return fail(ctx, SDE_ERR_INVALID, "too many counts");
    hipLaunchKernelGGL(hist_zero_kernel, dim3((uint32_t)zb), dim3(256), 0, stream, counts, nc);
    if (n) {
        const uint64_t gy = std::min<uint64_t>(n_rows, 65535);
        uint64_t gx = std::max<uint64_t>(1, (uint64_t)ctx->n_cu * 4 / gy);
        gx = std::min<uint64_t>(gx, (n + 255) / 256);
        gx = std::max<uint64_t>(gx, (n >> 31) + 1);
        hipLaunchKernelGGL(phase_hist_kernel, dim3((uint32_t)gx, (uint32_t)gy), dim3(256), 0, stream, theta, n,
                           n_rows > 1 ? pitch : n, n_rows, n_bins, counts);
    }
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int observables_impl(sde_ctx* ctx, int kind, const void* in, const uint32_t* counts, uint32_t n_groups,
                     double* host_out, hipStream_t stream)
{
    if (kind < SDE_OBS_MEAN_F32 || kind > SDE_OBS_ORDER) return fail(ctx, SDE_ERR_INVALID, "unknown kind %d", kind);
    if (!in || !counts || !host_out || n_groups == 0) return fail(ctx, SDE_ERR_INVALID, "null argument or no groups");
    if (!aligned(in, kind == SDE_OBS_MEAN_F64 ? 8 : 4)) return fail(ctx, SDE_ERR_INVALID, "misaligned input");
    // layout of the workspace: first[n_groups] (u64) | counts[n_groups] (u32) | out[n_groups][2]
    std::vector<unsigned char> meta((size_t)n_groups * 12);
    uint64_t off = 0;
    for (uint32_t g = 0; g < n_groups; ++g) {
        std::memcpy(meta.data() + 8 * (size_t)g, &off, 8);
        off += counts[g];
    }
    std::memcpy(meta.data() + 8 * (size_t)n_groups, counts, 4 * (size_t)n_groups);
    int st = upload(ctx, kSlotMisc, 3, meta.data(), meta.size(), stream);
    if (st) return st;
    void* outbuf = nullptr;
    if ((st = ensure_ws(ctx, kSlotObs, (size_t)n_groups * 2 * sizeof(double), &outbuf))) return st;
    const unsigned char* dmeta = static_cast<const unsigned char*>(ctx->ws[kSlotMisc].ptr);
    hipLaunchKernelGGL(obs_kernel, dim3(n_groups), dim3(kObsThreads), 0, stream, kind, in,
                       reinterpret_cast<const uint64_t*>(dmeta),
                       reinterpret_cast<const uint32_t*>(dmeta + 8 * (size_t)n_groups),
                       static_cast<double*>(outbuf));
    SDE_HIP(ctx, hipGetLastError());
    SDE_HIP(ctx, hipMemcpyAsync(host_out, outbuf, (size_t)n_groups * 2 * sizeof(double), hipMemcpyDeviceToHost,
                                stream));
    SDE_HIP(ctx, hipStreamSynchronize(stream));
    return SDE_OK;
}

}  // namespace sde
