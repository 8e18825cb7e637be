// sde_api.hip -- the C ABI entry points: context life cycle, status text,
// workspace management, validation shared by all integrators.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <fstream>
#include <new>
#include <sstream>

#include "sde_internal.h"

namespace sde {

__global__ void zero_u32_kernel(uint32_t* p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

int ensure_ws(sde_ctx* ctx, int slot, size_t bytes, void** out)
{
    DevBuf& b = ctx->ws[slot];
    if (b.bytes < bytes) {
        if (b.ptr) {
            SDE_HIP(ctx, hipDeviceSynchronize());
            SDE_HIP(ctx, hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
            ctx->uploaded[slot].clear();
        }
        ++ctx->ws_generation;  // recorded graphs refer to the old address
        size_t cap = bytes < 4096 ? 4096 : bytes + bytes / 4;
        if (hipMalloc(&b.ptr, cap) != hipSuccess) {
            (void)hipGetLastError();
            b.ptr = nullptr;
            return fail(ctx, SDE_ERR_NOMEM, "workspace slot %d: cannot allocate %zu bytes", slot, cap);
        }
        b.bytes = cap;
    }
    *out = b.ptr;
    return SDE_OK;
}

int upload(sde_ctx* ctx, int slot, int stage, const void* src, size_t bytes, hipStream_t stream)
{
    void* dst = nullptr;
    int st = ensure_ws(ctx, slot, bytes, &dst);
    if (st) return st;
    std::vector<unsigned char>& have = ctx->uploaded[slot];
    if (have.size() == bytes && std::memcmp(have.data(), src, bytes) == 0) return SDE_OK;
    Staging& s = ctx->staging[stage];
    if (s.pending) {
        SDE_HIP(ctx, hipEventSynchronize(s.done));
        s.pending = false;
    }
    if (s.bytes < bytes) {
        if (s.host) SDE_HIP(ctx, hipHostFree(s.host));
        s.host = nullptr;
        s.bytes = 0;
        size_t cap = bytes < 65536 ? 65536 : bytes + bytes / 4;
        SDE_HIP(ctx, hipHostMalloc(&s.host, cap, hipHostMallocDefault));
        s.bytes = cap;
    }
    if (!s.done) SDE_HIP(ctx, hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    std::memcpy(s.host, src, bytes);
    SDE_HIP(ctx, hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream));
    SDE_HIP(ctx, hipEventRecord(s.done, stream));
    s.pending = true;
    have.assign(static_cast<const unsigned char*>(src), static_cast<const unsigned char*>(src) + bytes);
    return SDE_OK;
}

int ensure_counters(sde_ctx* ctx, size_t n)
{
    if (ctx->n_counters >= n) return SDE_OK;
    if (ctx->counters) {
        SDE_HIP(ctx, hipDeviceSynchronize());
        SDE_HIP(ctx, hipFree(ctx->counters));
        ctx->counters = nullptr;
        ++ctx->ws_generation;
    }
    size_t cap = n < 1024 ? 1024 : n;
    if (hipMalloc(&ctx->counters, cap * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        ctx->n_counters = 0;
        return fail(ctx, SDE_ERR_NOMEM, "cannot allocate %zu counters", cap);
    }
    SDE_HIP(ctx, hipMemset(ctx->counters, 0, cap * sizeof(uint32_t)));
    ctx->n_counters = cap;
    return SDE_OK;
}

int zero_counters(sde_ctx* ctx, size_t first, size_t n, hipStream_t stream)
{
    int st = ensure_counters(ctx, first + n);
    if (st) return st;
    const unsigned threads = 256;
    const unsigned blocks = (unsigned)((n + threads - 1) / threads);
    zero_u32_kernel<<<blocks, threads, 0, stream>>>(ctx->counters + first, n);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int sync_and_check(sde_ctx* ctx, hipStream_t stream)
{
    SDE_HIP(ctx, hipStreamSynchronize(stream));
    int flag = 0;
    SDE_HIP(ctx, hipMemcpy(&flag, ctx->flag, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) {
        SDE_HIP(ctx, hipMemset(ctx->flag, 0, sizeof(int)));
        if (flag & 2)  // a bounded wait between workgroups or waves gave up: the results are not valid
            return fail(ctx, SDE_ERR_DEVICE, "a wait between workgroups or waves timed out (results invalid)");
        return fail(ctx, SDE_ERR_NUMERIC, "the integrated state became NaN or Inf");
    }
    return SDE_OK;
}

// ---------------------------------------------------------------- graphs --
static void drop_graph(GraphEntry& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
}

int run_recorded(sde_ctx* ctx, const std::string& key, hipStream_t stream,
                 const std::function<int(hipStream_t)>& record)
{
    ctx->last.graph_replayed = 0;
    if (!ctx->use_graphs) return record(stream);
    if (ctx->graphs_generation != ctx->ws_generation) {
        // a workspace moved: every recorded graph may refer to freed memory
        for (GraphEntry& g : ctx->graphs) drop_graph(g);
        ctx->graphs.clear();
        ctx->graphs_generation = ctx->ws_generation;
    }
    const std::string& full = key;
    for (GraphEntry& g : ctx->graphs) {
        if (g.key == full) {
            g.last_use = ++ctx->graph_clock;
            SDE_HIP(ctx, hipGraphLaunch(g.exec, stream));
            ctx->last.graph_replayed = 1;
            return SDE_OK;
        }
    }
    if (!ctx->capture_stream) SDE_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    SDE_HIP(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    int st = record(ctx->capture_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (st != SDE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, SDE_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(ctx, SDE_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    // keep at most 32 graphs: drop the least recently used
    if (ctx->graphs.size() >= 32) {
        auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                    [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
        drop_graph(*lru);
        ctx->graphs.erase(lru);
    }
    GraphEntry g;
    g.key = full;
    g.exec = exec;
    g.last_use = ++ctx->graph_clock;
    ctx->graphs.push_back(g);
    SDE_HIP(ctx, hipGraphLaunch(exec, stream));
    return SDE_OK;
}

// ------------------------------------------------------------ tune cache --
// The cache file is a flat JSON object {"key": integer, ...}.
static void tune_load(sde_ctx* ctx)
{
    std::ifstream in(ctx->tune_path);
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string t = ss.str();
    size_t p = 0;
    while ((p = t.find('"', p)) != std::string::npos) {
        const size_t q = t.find('"', p + 1);
        if (q == std::string::npos) break;
        const std::string key = t.substr(p + 1, q - p - 1);
        const size_t c = t.find(':', q);
        if (c == std::string::npos) break;
        ctx->tune[key] = std::atoi(t.c_str() + c + 1);
        p = t.find_first_of(",}", c);
        if (p == std::string::npos) break;
    }
}

static void tune_save(sde_ctx* ctx)
{
    if (ctx->tune_path.empty()) return;
    const std::string tmp = ctx->tune_path + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return;
        out << "{\n";
        size_t i = 0;
        for (const auto& kv : ctx->tune)
            out << "  \"" << kv.first << "\": " << kv.second << (++i < ctx->tune.size() ? ",\n" : "\n");
        out << "}\n";
    }
    (void)std::rename(tmp.c_str(), ctx->tune_path.c_str());
}

bool tune_lookup(sde_ctx* ctx, const std::string& key, int* value)
{
    auto it = ctx->tune.find(key);
    if (it == ctx->tune.end()) return false;
    *value = it->second;
    return true;
}

void tune_store(sde_ctx* ctx, const std::string& key, int value)
{
    ctx->tune[key] = value;
    tune_save(ctx);
}

int step_counter(sde_ctx* ctx, uint64_t** out)
{
    void* p = nullptr;
    int st = ensure_ws(ctx, kSlotStep, 64, &p);
    if (st) return st;
    *out = static_cast<uint64_t*>(p);
    return SDE_OK;
}

}  // namespace sde

using namespace sde;

extern "C" {

int sde_create(int hip_device, sde_ctx** out)
{
    if (!out) return SDE_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return SDE_ERR_DEVICE;
    }
    if (hipSetDevice(hip_device) != hipSuccess) return SDE_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return SDE_ERR_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SDE_ERR_UNSUPPORTED;
    sde_ctx* ctx = new (std::nothrow) sde_ctx();
    if (!ctx) return SDE_ERR_NOMEM;
    ctx->device = hip_device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    if (hipMalloc(&ctx->flag, sizeof(int)) != hipSuccess || hipMemset(ctx->flag, 0, sizeof(int)) != hipSuccess ||
        hipMalloc(&ctx->tune_flag, sizeof(int)) != hipSuccess || ensure_counters(ctx, 1024) != SDE_OK) {
        sde_destroy(ctx);
        return SDE_ERR_NOMEM;
    }
    if (const int st = noalloc_setup(ctx)) {
        sde_destroy(ctx);
        return st;
    }
    if (const char* tc = std::getenv("SDE_TUNE_CACHE")) {
        ctx->tune_path = tc;
        tune_load(ctx);
    }
    *out = ctx;
    return SDE_OK;
}

void sde_destroy(sde_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& b : ctx->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    for (auto& s : ctx->staging) {
        if (s.host) (void)hipHostFree(s.host);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    for (auto& g : ctx->graphs) drop_graph(g);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->noalloc_staging) (void)hipHostFree(ctx->noalloc_staging);
    if (ctx->noalloc_done) (void)hipEventDestroy(ctx->noalloc_done);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->tune_flag) (void)hipFree(ctx->tune_flag);
    if (ctx->counters) (void)hipFree(ctx->counters);
    delete ctx;
}

int sde_set_option(sde_ctx* ctx, int option, int64_t value)
{
    if (!ctx) return SDE_ERR_INVALID;
    switch (option) {
    case SDE_OPT_AUTOTUNE:
        if (value != 0 && value != 1) break;
        ctx->autotune = (int)value;
        return SDE_OK;
    case SDE_OPT_GRAPHS:
        if (value != 0 && value != 1) break;
        ctx->use_graphs = (int)value;
        return SDE_OK;
    case SDE_OPT_JJ_PPT:
        if (value != 0 && value != 1 && value != 2 && value != 4) break;
        ctx->jj_ppt = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_MF:
        if (value < 0 || value > 2) break;
        ctx->kura_mf = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_JSPLIT:
        if (value < 0 || value > 65535) break;
        ctx->kura_jsplit = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_TILE:
        if (value != 0 && value != 1 && value != 2 && value != 4) break;
        ctx->kura_tile = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_XCD_LOCAL:
        if (value != 0 && value != 1) break;
        ctx->kura_xcd_local = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_MF_OPT:
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8) break;
        ctx->kura_mf_opt = (int)value;
        return SDE_OK;
    case SDE_OPT_KURA_MF_PAIRED:
        if (value < 0 || value > 2) break;
        ctx->kura_mf_paired = (int)value;
        return SDE_OK;
    case SDE_OPT_DENSE_LAUNCH:
        if (value < 0 || value > 12) break;
        ctx->dense_launch = (int)value;
        return SDE_OK;
    default: break;
    }
    return fail(ctx, SDE_ERR_INVALID, "option %d: invalid value %lld", option, (long long)value);
}

int sde_set_tune_cache(sde_ctx* ctx, const char* path)
{
    if (!ctx) return SDE_ERR_INVALID;
    ctx->tune_path = path ? path : "";
    if (path) tune_load(ctx);
    return SDE_OK;
}

int sde_get_stats(const sde_ctx* ctx, sde_stats* out)
{
    if (!ctx || !out) return SDE_ERR_INVALID;
    *out = ctx->last;
    out->graphs_cached = (int32_t)ctx->graphs.size();
    return SDE_OK;
}

const char* sde_strerror(int status)
{
    switch (status) {
    case SDE_OK: return "ok";
    case SDE_ERR_INVALID: return "invalid argument";
    case SDE_ERR_NOMEM: return "out of device memory";
    case SDE_ERR_DEVICE: return "HIP runtime error";
    case SDE_ERR_UNSUPPORTED: return "unsupported";
    case SDE_ERR_NUMERIC: return "state became NaN or Inf";
    default: return "unknown status";
    }
}

const char* sde_last_error(const sde_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int sde_check(sde_ctx* ctx)
{
    if (!ctx) return SDE_ERR_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SDE_ERR_DEVICE, "hipSetDevice failed");
    if (hipDeviceSynchronize() != hipSuccess) return fail(ctx, SDE_ERR_DEVICE, "hipDeviceSynchronize failed");
    return sync_and_check(ctx, nullptr);
}

int sde_jj_integrate(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                     float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                     void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_jj_integrate");
    ctx->last_error.clear();
    try {
        return jj_integrate_impl(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums,
                                 static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_jj_integrate_noalloc(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                             float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                             void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_jj_integrate_noalloc");
    ctx->last_error.clear();
    try {
        return jj_integrate_noalloc_impl(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums,
                                         static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_jj_integrate_f64(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                         double* theta, int32_t* winding, double* v, double* acc, double* point_sums,
                         void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_jj_integrate_f64");
    ctx->last_error.clear();
    try {
        return jj_integrate_f64_impl(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums,
                                     static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_jj_integrate_recorded(sde_ctx* ctx, const sde_jj_point* pts, uint32_t n_pts, const sde_run* run,
                              float* theta, int32_t* winding, float* v, double* acc, double* point_sums,
                              uint32_t record_every, uint64_t n_rows, int32_t* rec_winding, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_jj_integrate_recorded");
    ctx->last_error.clear();
    try {
        return jj_integrate_recorded_impl(ctx, pts, n_pts, run, theta, winding, v, acc, point_sums, record_every,
                                          n_rows, rec_winding, static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_kuramoto_integrate(sde_ctx* ctx, const sde_kuramoto_desc* desc, const sde_run* run,
                           float* phi, const float* omega, const float* K, double* r_samples,
                           void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_kuramoto_integrate");
    ctx->last_error.clear();
    try {
        return kuramoto_impl(ctx, desc, run, phi, omega, K, r_samples,
                             static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_observables(sde_ctx* ctx, int kind, const void* dev_in, const uint32_t* counts,
                    uint32_t n_groups, double* host_out, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_observables");
    ctx->last_error.clear();
    try {
        return observables_impl(ctx, kind, dev_in, counts, n_groups, host_out,
                                static_cast<hipStream_t>(hip_stream));
    } catch (...) {
        return fail(ctx, SDE_ERR_NOMEM, "host allocation failed");
    }
}

int sde_position_histogram(sde_ctx* ctx, const int32_t* winding, uint64_t n, int64_t x0, uint32_t n_bins,
                           uint64_t* counts, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_position_histogram");
    ctx->last_error.clear();
    return histogram_impl(ctx, winding, n, n, 1, x0, n_bins, counts, static_cast<hipStream_t>(hip_stream));
}

int sde_position_histograms(sde_ctx* ctx, const int32_t* winding, uint64_t n, uint64_t pitch, uint64_t n_rows,
                            int64_t x0, uint32_t n_bins, uint64_t* counts, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_position_histograms");
    ctx->last_error.clear();
    return histogram_impl(ctx, winding, n, pitch, n_rows, x0, n_bins, counts, static_cast<hipStream_t>(hip_stream));
}

int sde_phase_histograms(sde_ctx* ctx, const float* theta, uint64_t n, uint64_t pitch, uint64_t n_rows,
                         uint32_t n_bins, uint64_t* counts, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    const TraceRange range("sde_phase_histograms");
    ctx->last_error.clear();
    return phase_histogram_impl(ctx, theta, n, pitch, n_rows, n_bins, counts, static_cast<hipStream_t>(hip_stream));
}

int sde_debug_philox(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                     uint64_t ctr0_first, uint64_t n_blocks, uint32_t* dev_out, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    ctx->last_error.clear();
    return debug_philox_impl(ctx, seed, tag, a, b, ctr0_first, n_blocks, dev_out,
                             static_cast<hipStream_t>(hip_stream));
}

int sde_debug_gauss(sde_ctx* ctx, uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                    uint64_t n_first, uint64_t count, float* dev_out, void* hip_stream)
{
    if (!ctx) return SDE_ERR_INVALID;
    ctx->last_error.clear();
    return debug_gauss_impl(ctx, seed, tag, a, b, n_first, count, dev_out,
                            static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
