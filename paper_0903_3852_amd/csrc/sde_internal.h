// sde_internal.h -- host-side context and helpers shared by the library's
// translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/sde.h"

namespace sde {

// A device buffer that only grows; freed with the context.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// A pinned host staging buffer whose last upload is fenced by an event, so
// it is never overwritten while an asynchronous copy may still read it.
struct Staging {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

}  // namespace sde

struct sde_ctx {
    int device = 0;
    int n_cu = 0;
    int xcds = 8;
    std::string arch;
    std::string last_error;
    int* flag = nullptr;          // device: nonzero once a state became NaN/Inf
    int* tune_flag = nullptr;     // device: the same for autotuner trial runs (never reported)
    uint32_t* counters = nullptr; // device: work-queue counters and barrier words
    size_t n_counters = 0;
    sde::DevBuf ws[16];           // device workspaces, by slot (see sde::Slot)
    sde::Staging staging[4];
    std::vector<unsigned char> uploaded[16];  // host copy of what each slot holds
    uint64_t ws_generation = 0;   // bumped whenever a workspace moves (invalidates graphs)
    // launch layer
    hipStream_t capture_stream = nullptr;
    std::vector<sde::GraphEntry> graphs;
    uint64_t graph_clock = 0;
    uint64_t graphs_generation = 0;  // ws_generation the cached graphs were recorded at
    int use_graphs = 1;
    int autotune = 1;
    int jj_ppt = 0;               // 0 = tuned
    int kura_mf = 0;              // mean-field variant: 0 auto, 1 streamed, 2 registers
    int kura_jsplit = 0;          // all-pairs j slices: 0 auto, else forced
    int kura_tile = 0;            // all-pairs oscillators per lane: 0 tuned, else 1, 2, 4
    int kura_xcd_local = 1;       // mean field: exchange through the XCD's L2 when possible
    int kura_mf_opt = 0;          // mean field oscillators per lane: 0 tuned, else 1, 2, 4, 8
    int kura_mf_paired = 0;       // mean field realizations per workgroup: 0 tuned, 1 one, 2 two
    int dense_launch = 0;         // dense launch: 0 tuned; 1-4: 1 + (4 waves ? 1 : 0) + (plain order ? 2 : 0);
                                  // 5, 6: two workgroups per tile over the halves of k, bands / plain order;
                                  // 7, 8: row-half waves with two register sets, bands / plain order;
                                  // 9, 10: 4 waves with K double-buffered in LDS, bands / plain order;
                                  // 11, 12: wave pairs sharing K through LDS, bands / plain order
    std::map<std::string, int> tune;
    std::string tune_path;
    sde_stats last{};
    // sde_jj_integrate_noalloc: the device's scratch (not owned), a pinned
    // staging buffer of the same size and the event fencing its last copy
    void* noalloc_scratch = nullptr;
    void* noalloc_staging = nullptr;
    hipEvent_t noalloc_done = nullptr;
    bool noalloc_pending = false;
};

namespace sde {

// Size of the static device scratch of sde_jj_integrate_noalloc, and the
// number of devices whose scratch address is tracked.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

enum Slot {
    kSlotJJPoints = 0,
    kSlotJJItems = 1,
    kSlotJJLut = 2,
    kSlotJJPartials = 3,
    kSlotObs = 4,
    kSlotKuraPartials = 5,
    kSlotKuraWork = 6,
    kSlotDenseA = 7,
    kSlotDenseB = 8,
    kSlotDenseOut = 9,
    kSlotMisc = 10,
    kSlotStep = 11,
    kSlotTune = 12,
};

// A roctx range around one C-ABI call (shown by rocprofv3 --marker-trace;
// a cheap no-op when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Status helpers -----------------------------------------------------------
inline int fail(sde_ctx* ctx, int status, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
inline int fail(sde_ctx* ctx, int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->last_error = buf;
    return status;
}

#define SDE_HIP(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::sde::fail((ctx), SDE_ERR_DEVICE, "%s failed: %s", #call,                \
                               hipGetErrorString(e_));                                       \
    } while (0)

// Grows workspace slot `slot` to at least `bytes`; returns its pointer or null.
int ensure_ws(sde_ctx* ctx, int slot, size_t bytes, void** out);
// Copies `bytes` from host `src` into workspace slot `slot` on `stream`
// unless the slot already holds exactly these bytes.  Staging buffer
// `stage` carries the asynchronous copy.
int upload(sde_ctx* ctx, int slot, int stage, const void* src, size_t bytes, hipStream_t stream);
// Resets `n` device counters starting at `first` to zero with a kernel
// (stream-ordered, safe under graph capture).
int zero_counters(sde_ctx* ctx, size_t first, size_t n, hipStream_t stream);
int ensure_counters(sde_ctx* ctx, size_t n);
// Synchronizes `stream` and reports SDE_ERR_NUMERIC if the NaN flag is set.
int sync_and_check(sde_ctx* ctx, hipStream_t stream);

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Records a launch sequence with `record(s)` on stream s.  With graphs on,
// the sequence is captured once (on the context's private stream) into a
// HIP graph stored under `key` (+ the workspace generation) and replayed on
// `stream`; otherwise `record(stream)` launches directly.  `record` must
// only enqueue kernels (no allocation, no synchronization, no memset).
int run_recorded(sde_ctx* ctx, const std::string& key, hipStream_t stream,
                 const std::function<int(hipStream_t)>& record);
// Tune cache: look up / store an integer choice under `key`.
bool tune_lookup(sde_ctx* ctx, const std::string& key, int* value);
void tune_store(sde_ctx* ctx, const std::string& key, int value);
// Small device-side counters of the step loops (one uint64 per use).
int step_counter(sde_ctx* ctx, uint64_t** out);

// Launchers implemented in the kernel translation units.
int jj_integrate_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                      float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                      hipStream_t stream);
int jj_integrate_recorded_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                               float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                               uint32_t record_every, uint64_t n_rows, int32_t* rec_winding, hipStream_t stream);
// Looks up this device's no-allocation scratch (once per device) and
// allocates the context's pinned staging buffer and event; called by
// sde_create with the device current.
int noalloc_setup(sde_ctx* ctx);
int jj_integrate_noalloc_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                              float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                              hipStream_t stream);
int jj_integrate_f64_impl(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                          double* theta, int32_t* winding, double* v, double* acc, double* point_sums,
                          hipStream_t stream);
int debug_philox_impl(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                      uint64_t c0, uint64_t n, uint32_t* out, hipStream_t stream);
int debug_gauss_impl(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                     uint64_t n0, uint64_t n, float* out, hipStream_t stream);
int observables_impl(sde_ctx* ctx, int kind, const void* in, const uint32_t* counts,
                     uint32_t n_groups, double* host_out, hipStream_t stream);
int histogram_impl(sde_ctx* ctx, const int32_t* winding, uint64_t n, uint64_t pitch, uint64_t n_rows, int64_t x0,
                   uint32_t n_bins, uint64_t* counts, hipStream_t stream);
int phase_histogram_impl(sde_ctx* ctx, const float* theta, uint64_t n, uint64_t pitch, uint64_t n_rows,
                         uint32_t n_bins, uint64_t* counts, hipStream_t stream);
int kuramoto_impl(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                  const float* omega, const float* K, double* r_samples, hipStream_t stream);

}  // namespace sde
