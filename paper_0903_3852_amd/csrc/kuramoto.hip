// kuramoto.hip -- the noisy Kuramoto model (Eq. 2 with gamma = 1):
//   dphi_i = [omega_i + sum_j K_ij sin(phi_j - phi_i)] dt + sqrt(2 D) dW_i,
// R independent realizations of N oscillators, stochastic Heun (Alg. 2) or
// Euler-Maruyama, phases kept in revolutions theta = phi / 2 pi in [0, 1).
//
// Uniform coupling K_ij = K/N is evaluated two ways:
//  * MEANFIELD (Eq. 3): per realization and stage only two sums, S = sum_j
//    sin phi_j and C = sum_j cos phi_j, then F_i = omega_i + (K/N)(cos phi_i S
//    - sin phi_i C).  One cooperative persistent launch runs every step: the
//    G workgroups of a realization hold its oscillators in registers (or,
//    beyond register capacity, stream them through HBM), publish FP64
//    partial sums as tagged words without fences, and add all G partials in
//    a fixed order (bitwise reproducible) -- directly, or through 8 group
//    leaders when G is large.  Workgroups are mapped so that each realization
//    sits on one XCD when the realizations divide evenly over the 8 XCDs
//    (workgroups are dealt to them round robin).
//  * TILED (Alg. 3, Fig. 3): all N^2 terms sin(2 pi (theta_j - theta_i)),
//    theta_j staged through LDS in tiles and read by every lane (broadcast),
//    one hardware v_sin_f32 per pair; tile size tuned, and for small N the j
//    range split over workgroups.  One launch per Heun stage; the stage
//    boundary is the global synchronization.
// The noise of oscillator i in realization r at step n is component n & 3 of
// the Box-Muller Gaussians of Philox(ctr = (n >> 2, i, r, NOISE)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "device_common.h"
#include "kuramoto_common.h"
#include "sde_internal.h"

namespace sde {

// ---------------------------------------------------------------- MF ------
// Lanes per workgroup: 8 waves for the register-resident kernel (fewer
// waves per barrier and more oscillators per lane run its stage faster than
// 16), 16 for the streamed kernel (more loads in flight).  A realization has
// at most lanes / 4 workgroups: one polling lane per exchange word.
constexpr int kMFThreads = 512;
constexpr int kMFSThreads = 1024;
constexpr uint32_t kMaxMFGroups = kMFThreads / 4;
constexpr uint32_t kMaxMFSGroups = kMFSThreads / 4;

struct MFArgs {
    float* theta;            // [R][N] revolutions, in/out (this launch's realizations)
    const float* omega;      // [N]
    double* r_samples;       // [R][n_samples] or null
    uint64_t* slots;         // [2 parities][R][G][4] tagged words (kMFWordsPerGroup), zero at launch
    uint64_t* slots2;        // [2 parities][R][8][4] group sums of the tree exchange, zero at launch
    int* flag;               // error flag (NaN state, or a barrier that timed out)
    uint32_t N, R, G, M;
    uint32_t r_base;         // global index of this launch's first realization
    uint64_t step0, n_steps, n_samples;
    uint32_t key0, key1;
    float omega_scale;       // dt / (2 pi) (revolutions per unit of F)
    float hdt2pi;            // dt / (4 pi)
    float kn;                // K / N
    float c2;                // -2 ln2 sigma^2, sigma = sqrt(2 D dt) / (2 pi)
    int32_t init_from_state;
    int32_t xcd_map;         // 1: realization r lives on XCD r / (R / 8)
    int32_t xcd_local;       // 1: exchange through the XCD's L2 where a realization's workgroups share it
    uint32_t spin_limit;     // barrier give-up bound (iterations of s_sleep)
    uint32_t tree;           // two-level exchange (G a multiple of 8)
};

// Exchange of the per-workgroup FP64 sums (s, c) of stage `epoch` among the
// G workgroups of realization r; returns the realization's S and C (the
// partials added in workgroup order, so every workgroup gets the same bits).
//
// No fences: each workgroup publishes its two doubles as four 64-bit words
// (32 data bits, 32 bits of tag = epoch + 1) with relaxed agent-scope atomic
// stores, and lane t polls word t with relaxed agent-scope atomic loads
// until its tag matches.  A 64-bit atomic is read whole or not at all, so a
// matching tag certifies its data; nothing else needs ordering.  A release
// and acquire pair instead costs a write-back and an invalidation of the
// L2 on this multi-XCD part at every stage.
//
// Flat (A.tree = 0): every workgroup polls all 4G words and adds the G
// pairs in workgroup order.  Tree (A.tree = 1, G a multiple of 8, used when
// G is large): workgroup w belongs to group w mod 8 (one XCD under the
// round-robin dispatch); the group's first workgroup polls its G/8 members,
// adds them in order and publishes the group sum as four words in slots2;
// every workgroup then polls the 8 group sums and adds them in group order.
// That replaces 4G polled words per workgroup by 32 (and 4G/8 for the
// leaders) at the price of a second round trip.
//
// Two parities of slots (and of slots2): a workgroup can only publish epoch
// e + 2 after every workgroup published e + 1, i.e. after all of them read
// epoch e -- in the tree, publishing level-one words of e + 2 requires the
// group sums of e + 1, which require every workgroup's e + 1 words.  Returns
// false if a wait exceeded the spin bound (the error flag is then set).
constexpr uint32_t kMFWordsPerGroup = 4;
constexpr uint32_t kMFTreeMinGroups = 32;  // tree exchange from this many workgroups per realization

__device__ __forceinline__ void mf_publish(uint64_t* dst, uint64_t tag, double S, double C)
{
    const uint64_t bs = (uint64_t)__double_as_longlong(S), bc = (uint64_t)__double_as_longlong(C);
    __hip_atomic_store(dst + 0, tag | (bs & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(dst + 1, tag | (bs >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(dst + 2, tag | (bc & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(dst + 3, tag | (bc >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes t < n poll the word at addr(t) until it carries `tag`, keeping its
// data bits in words[t]; returns false (all lanes) on a timed-out wait.
template <typename Args, typename Addr>
__device__ __forceinline__ bool mf_poll(const Args& A, uint32_t n, Addr addr, uint64_t tag, uint32_t* words,
                                        int* lds_ok)
{
    if (threadIdx.x < n) {
        const uint64_t* p = addr(threadIdx.x);
        uint32_t spins = 0;
        uint64_t v;
        while (((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & 0xffffffff00000000ull) !=
               tag) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > A.spin_limit) {
                atomicOr(A.flag, 2);
                *lds_ok = 0;
                break;
            }
        }
        words[threadIdx.x] = (uint32_t)v;
    }
    __syncthreads();
    return *lds_ok != 0;
}

// Sum of the n (S, C) pairs held as word quadruples in words, in order.
__device__ __forceinline__ void mf_sum_words(const uint32_t* words, uint32_t n, double& S, double& C)
{
    S = 0.0;
    C = 0.0;
#pragma unroll 4
    for (uint32_t g = 0; g < n; ++g) {
        const uint32_t* q = words + g * kMFWordsPerGroup;
        S += __longlong_as_double((long long)(((uint64_t)q[1] << 32) | q[0]));
        C += __longlong_as_double((long long)(((uint64_t)q[3] << 32) | q[2]));
    }
}

template <int NT, typename Args>
__device__ __forceinline__ bool mf_exchange(const Args& A, uint32_t r, uint32_t w, uint32_t epoch, double s,
                                            double c, double* lds, uint32_t* words, int* lds_ok, double& S,
                                            double& C)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    s = wave_sum(s);
    c = wave_sum(c);
    if (lane == 0) {
        lds[2 * wid] = s;
        lds[2 * wid + 1] = c;
    }
    __syncthreads();
    const uint64_t tag = (uint64_t)(epoch + 1) << 32;
    uint64_t* slot = A.slots + ((uint64_t)(epoch & 1u) * A.R + r) * A.G * kMFWordsPerGroup;
    if (threadIdx.x == 0) {
        double Sw = 0.0, Cw = 0.0;
#pragma unroll
        for (int k = 0; k < NT / kWave; ++k) {
            Sw += lds[2 * k];
            Cw += lds[2 * k + 1];
        }
        mf_publish(slot + (uint64_t)w * kMFWordsPerGroup, tag, Sw, Cw);
    }
    if (!A.tree) {
        if (!mf_poll(A, kMFWordsPerGroup * A.G, [&](uint32_t t) { return slot + t; }, tag, words, lds_ok))
            return false;
        mf_sum_words(words, A.G, S, C);
        __syncthreads();  // words and lds are rewritten by the next exchange
        return true;
    }
    const uint32_t x = w & 7u, g = A.G >> 3;
    uint64_t* slot2 = A.slots2 + ((uint64_t)(epoch & 1u) * A.R + r) * 8 * kMFWordsPerGroup;
    if (w < 8) {  // group leader: members x, x + 8, x + 16, ...
        if (!mf_poll(A, kMFWordsPerGroup * g,
                     [&](uint32_t t) { return slot + (uint64_t)(x + 8 * (t >> 2)) * kMFWordsPerGroup + (t & 3u); },
                     tag, words, lds_ok))
            return false;
        if (threadIdx.x == 0) {
            double Sx, Cx;
            mf_sum_words(words, g, Sx, Cx);
            mf_publish(slot2 + (uint64_t)x * kMFWordsPerGroup, tag, Sx, Cx);
        }
    }
    uint32_t* w2 = words + kMFWordsPerGroup * (NT / 4) / 2;
    if (!mf_poll(A, 8 * kMFWordsPerGroup, [&](uint32_t t) { return slot2 + t; }, tag, w2, lds_ok)) return false;
    mf_sum_words(w2, 8, S, C);
    __syncthreads();
    return true;
}

// ------------------------------------------------ MF, register-resident --
// Sum over the 64 lanes of a wave by DPP moves: swaps within quads, the
// half-row and row mirrors (every lane then holds its row's sum) and the two
// row broadcasts.  The order is fixed, the total lands in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_term(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, 0xF,
                                                                  false));
}

__device__ __forceinline__ float wave_sum_dpp(float x)
{
    x += dpp_term<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
    x += dpp_term<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
    x += dpp_term<0x141, 0xF>(x);  // row_half_mirror
    x += dpp_term<0x140, 0xF>(x);  // row_mirror
    x += dpp_term<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_term<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

constexpr int kMFWaves = kMFThreads / kWave;

// Word w of realization r's exchange (flat: [parity][R][G][4]).
__device__ __forceinline__ uint64_t* mf_word(const MFArgs& A, uint64_t* base, uint32_t per_r, uint32_t r,
                                             uint32_t epoch, uint32_t w)
{
    return base + ((uint64_t)(epoch & 1u) * A.R + r) * per_r + w;
}

// Publishes (S, C) as four tagged words.  XCD-local exchanges store at
// workgroup scope: the words land in the shared L2 of the XCD, where the
// other workgroups' agent-scope loads find them; otherwise at agent scope.
__device__ __forceinline__ void mf2_publish(uint64_t* dst, uint64_t tag, double S, double C, bool local)
{
    const uint64_t bs = (uint64_t)__double_as_longlong(S), bc = (uint64_t)__double_as_longlong(C);
    const uint64_t v[4] = {tag | (bs & 0xffffffffull), tag | (bs >> 32), tag | (bc & 0xffffffffull),
                           tag | (bc >> 32)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (local)
            __hip_atomic_store(dst + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_store(dst + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The same four words stored by lanes 0..3 of the calling wave, one each.
__device__ __forceinline__ void mf2_publish_lanes(uint64_t* dst, uint64_t tag, double S, double C, bool local)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (lane < kMFWordsPerGroup) {
        const uint64_t b = (uint64_t)__double_as_longlong(lane < 2 ? S : C);
        const uint64_t v = tag | ((lane & 1u) ? (b >> 32) : (b & 0xffffffffull));
        if (local)
            __hip_atomic_store(dst + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_store(dst + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Lane t < n of the calling wave waits for the word at p(t) to carry `tag`
// and returns its 32 data bits; false once any lane's wait exceeded the
// spin bound (the error flag is then set).  Agent-scope loads: they see both
// agent-scope stores and, within one XCD, workgroup-scope stores.
template <typename Addr>
__device__ __forceinline__ bool mf2_poll(const MFArgs& A, uint32_t n, Addr p, uint64_t tag, uint32_t& data)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    bool ok = true;
    data = 0u;
    if (lane < n) {
        const uint64_t* q = p(lane);
        uint32_t spins = 0;
        uint64_t v;
        while (((v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & 0xffffffff00000000ull) !=
               tag) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > A.spin_limit) {
                ok = false;
                break;
            }
        }
        data = (uint32_t)v;
    }
    if (__ballot(!ok) != 0) {
        if (lane == 0) atomicOr(A.flag, 2);
        return false;
    }
    return true;
}

// The (S, C) pairs the polling wave holds as words, lane 4g + j holding word
// j of pair g (zero words beyond the last pair): staged through LDS, where
// each pair reads as two doubles, and added over g = 0 .. 15 in a fixed
// pairwise order (zero pairs change nothing); every lane of the wave gets S
// and C, and every workgroup adds the same numbers to the same bits.
__device__ __forceinline__ void mf2_sum_words(uint32_t data, uint32_t* words, double& S, double& C)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    words[lane] = data;
    // the wave's own LDS writes are complete before its reads below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double2* pairs = reinterpret_cast<const double2*>(words);
    double s4[4], c4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double2 p0 = pairs[4 * q], p1 = pairs[4 * q + 1], p2 = pairs[4 * q + 2], p3 = pairs[4 * q + 3];
        s4[q] = (p0.x + p1.x) + (p2.x + p3.x);
        c4[q] = (p0.y + p1.y) + (p2.y + p3.y);
    }
    S = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    C = (c4[0] + c4[1]) + (c4[2] + c4[3]);
}

// Shared state of one workgroup of the register-resident kernel.
struct MF2Shared {
    float ws[kMFWaves], wc[kMFWaves];  // per-wave FP32 partial sums of the stage
    double S, C;                       // the realization's sums of the stage
    int ok;
    int local;                         // the realization's workgroups share one XCD
    __attribute__((aligned(8))) uint32_t words[kWave];  // the polled words of wave 0
};

// The exchange among the G workgroups of realization r, run by one wave after
// the per-wave partials are in `sh`: the workgroup's FP64 sum of its waves
// (in wave order) is published, the G workgroup sums (flat) or the 8 group
// sums of the tree (workgroup w in group w mod 8; the group's first
// workgroup adds its members in order) are collected and added in order,
// and the wave leaves S and C in `sh`.  Every workgroup of a realization adds
// the same numbers in the same order, so all get the same bits.
__device__ __forceinline__ void mf2_exchange_wave(const MFArgs& A, uint32_t r, uint32_t w, uint32_t epoch,
                                                   MF2Shared& sh)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    static_assert(kMFWaves == 8, "the pairwise order below is written for 8 waves");
    auto d = [](float x) { return (double)x; };
    const double Sw = ((d(sh.ws[0]) + d(sh.ws[1])) + (d(sh.ws[2]) + d(sh.ws[3]))) +
                      ((d(sh.ws[4]) + d(sh.ws[5])) + (d(sh.ws[6]) + d(sh.ws[7])));
    const double Cw = ((d(sh.wc[0]) + d(sh.wc[1])) + (d(sh.wc[2]) + d(sh.wc[3]))) +
                      ((d(sh.wc[4]) + d(sh.wc[5])) + (d(sh.wc[6]) + d(sh.wc[7])));
    if (A.G == 1) {  // the realization is one workgroup: nothing to exchange
        if (lane == 0) {
            sh.S = Sw;
            sh.C = Cw;
        }
        return;
    }
    const bool local = sh.local != 0;
    const uint64_t tag = (uint64_t)(epoch + 1) << 32;
    const uint32_t per1 = A.G * kMFWordsPerGroup;
    mf2_publish_lanes(mf_word(A, A.slots, per1, r, epoch, w * kMFWordsPerGroup), tag, Sw, Cw, local);
    double S, C;
    uint32_t data;
    if (!A.tree) {
        if (!mf2_poll(A, per1, [&](uint32_t t) { return mf_word(A, A.slots, per1, r, epoch, t); }, tag, data)) {
            if (lane == 0) sh.ok = 0;
            return;
        }
        mf2_sum_words(data, sh.words, S, C);
    } else {
        const uint32_t x = w & 7u, m = A.G >> 3;
        const uint32_t per2 = 8 * kMFWordsPerGroup;
        if (w < 8) {  // group leader: members x, x + 8, x + 16, ...
            if (!mf2_poll(A, m * kMFWordsPerGroup,
                          [&](uint32_t t) {
                              return mf_word(A, A.slots, per1, r, epoch, (x + 8 * (t >> 2)) * kMFWordsPerGroup + (t & 3u));
                          },
                          tag, data)) {
                if (lane == 0) sh.ok = 0;
                return;
            }
            double Sx, Cx;
            mf2_sum_words(data, sh.words, Sx, Cx);
            mf2_publish_lanes(mf_word(A, A.slots2, per2, r, epoch, x * kMFWordsPerGroup), tag, Sx, Cx, local);
        }
        if (!mf2_poll(A, per2, [&](uint32_t t) { return mf_word(A, A.slots2, per2, r, epoch, t); }, tag, data)) {
            if (lane == 0) sh.ok = 0;
            return;
        }
        mf2_sum_words(data, sh.words, S, C);
    }
    if (lane == 0) {
        sh.S = S;
        sh.C = C;
    }
}

// Whether all G workgroups of realization r run on one XCD: each publishes
// its XCD id (epoch 0, agent scope) and reads everyone's.  Run by one wave;
// the answer is the same in every workgroup of the realization.
template <typename SH>
__device__ __forceinline__ void mf2_locality(const MFArgs& A, uint32_t r, uint32_t w, SH& sh)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (A.G == 1) return;  // no exchange
    const uint32_t xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));  // HW_REG_XCC_ID[3:0]
    const uint64_t tag = 1ull << 32;
    const uint32_t per1 = A.G * kMFWordsPerGroup;
    if (lane == 0) mf2_publish(mf_word(A, A.slots, per1, r, 0, w * kMFWordsPerGroup), tag, (double)xcc, 0.0, false);
    bool same = true;
    for (uint32_t base = 0; base < A.G; base += kWave / kMFWordsPerGroup) {
        const uint32_t cnt = min(A.G - base, (uint32_t)(kWave / kMFWordsPerGroup));
        uint32_t data;
        if (!mf2_poll(A, cnt * kMFWordsPerGroup,
                      [&](uint32_t t) { return mf_word(A, A.slots, per1, r, 0, base * kMFWordsPerGroup + t); }, tag,
                      data)) {
            if (lane == 0) sh.ok = 0;
            return;
        }
        for (uint32_t g = 0; g < cnt; ++g) {
            const uint32_t s0 = __builtin_amdgcn_readlane(data, 4 * g), s1 = __builtin_amdgcn_readlane(data, 4 * g + 1);
            same &= __longlong_as_double((long long)(((uint64_t)s1 << 32) | s0)) == (double)xcc;
        }
    }
    if (lane == 0) sh.local = (same && A.xcd_local) ? 1 : 0;
}

template <int OPT, int SCHEME>
__global__ __launch_bounds__(kMFThreads, 1) void kuramoto_mf_kernel(MFArgs A)
{
    __shared__ MF2Shared sh;
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        sh.ok = 1;
        sh.local = 0;
    }
    // workgroup -> (realization r, slice w)
    uint32_t r, w;
    if (A.xcd_map) {
        const uint32_t x = blockIdx.x & 7u, l = blockIdx.x >> 3, per = A.R >> 3;
        r = x * per + l / A.G;
        w = l % A.G;
    } else {
        r = blockIdx.x / A.G;
        w = blockIdx.x % A.G;
    }
    const uint32_t N = A.N;
    float th[OPT], F1[OPT], om[OPT], sn[OPT], cs[OPT];
    uint32_t idx[OPT];
    bool live[OPT];
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
        idx[k] = (w * OPT + k) * kMFThreads + threadIdx.x;
        live[k] = idx[k] < N;
        const uint32_t i = live[k] ? idx[k] : 0u;
        om[k] = live[k] ? A.omega[i] : 0.f;
        if (A.init_from_state) {
            th[k] = live[k] ? A.theta[(uint64_t)r * N + i] : 0.f;
        } else {
            const U4 x = philox4x32_10(U4{0u, i, A.r_base + r, (uint32_t)SDE_TAG_INIT}, A.key0, A.key1);
            th[k] = (float)(x.x >> 8) * 0x1p-24f;
        }
    }
    __syncthreads();
    if (wid == 0) mf2_locality(A, r, w, sh);

    uint32_t epoch = 1;
    const double invN = 1.0 / (double)N;
    static_assert(OPT <= 8, "at most 8 oscillators per lane");
    // Noise: sigma * the Gaussians of the current block of 4 steps (g, block
    // gblk) and of the next one (gn, block gblk + 1), the latter generated
    // oscillator by oscillator while the wave waits for an exchange it does
    // not run (the exchanges rotate over the waves, so each wave has idle
    // windows); gn_done oscillators of gn are ready (wave-uniform).
    float g[OPT][4], gn[OPT][4];
    uint64_t gblk = ~0ull;
    uint32_t gn_done = 0;
    constexpr uint32_t kPrefetch = SCHEME == SDE_HEUN ? (OPT + 6) / 7 : (OPT + 2) / 3;
    auto prefetch = [&]() {
        if (gblk == ~0ull || gn_done >= (uint32_t)OPT) return;
        const uint32_t nb = (uint32_t)(gblk + 1), lo = gn_done, hi = gn_done + kPrefetch;
#pragma unroll
        for (int k = 0; k < OPT; ++k)
            if ((uint32_t)k >= lo && (uint32_t)k < hi)
                gauss4_scaled(U4{nb, idx[k], A.r_base + r, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2, gn[k]);
        gn_done = hi < (uint32_t)OPT ? hi : (uint32_t)OPT;
    };

    // sin and cos of the phases t[] (kept for the drift) and the realization's
    // sums of them: FP32 within a lane and a wave, FP64 across waves and
    // workgroups.  Exchange e is run by wave e mod 8.
    auto reduce = [&](const float (&t)[OPT], float& Sf, float& Cf, double& Sd, double& Cd) -> bool {
        float s = 0.f, c = 0.f;
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            sn[k] = live[k] ? sin_rev(t[k]) : 0.f;
            cs[k] = live[k] ? cos_rev(t[k]) : 0.f;
            s += sn[k];
            c += cs[k];
        }
        s = wave_sum_dpp(s);
        c = wave_sum_dpp(c);
        if (lane == kWave - 1) {
            sh.ws[wid] = s;
            sh.wc[wid] = c;
        }
        __syncthreads();
        if (wid == (epoch & (kMFWaves - 1))) {
            if (sh.ok) mf2_exchange_wave(A, r, w, epoch, sh);
        } else {
            prefetch();
        }
        __syncthreads();
        if (!sh.ok) return false;
        ++epoch;
        Sd = sh.S;
        Cd = sh.C;
        Sf = (float)Sd;
        Cf = (float)Cd;
        return true;
    };

    uint64_t n = A.step0;
    const uint64_t n_end = A.step0 + A.n_steps;
    uint64_t local = 0;
    for (;;) {
        // one stage-1 reduction at theta_n: the drift and, every M steps, r
        float S, C;
        double Sd, Cd;
        if (!reduce(th, S, C, Sd, Cd)) break;
        if (A.r_samples && local % A.M == 0 && w == 0 && threadIdx.x == 0)
            A.r_samples[(uint64_t)r * A.n_samples + local / A.M] = std::sqrt(Sd * Sd + Cd * Cd) * invN;
        if (n == n_end) break;
        if ((n >> 2) != gblk) {
            const uint64_t b = n >> 2;
            if (gblk != ~0ull && b == gblk + 1 && gn_done == (uint32_t)OPT) {
#pragma unroll
                for (int k = 0; k < OPT; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q) g[k][q] = gn[k][q];
            } else {
#pragma unroll
                for (int k = 0; k < OPT; ++k)
                    gauss4_scaled(U4{(uint32_t)b, idx[k], A.r_base + r, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1,
                                  A.c2, g[k]);
            }
            gblk = b;
            gn_done = 0;
        }
        const uint32_t j = (uint32_t)n & 3u;
        auto noise = [&](int k) { return j == 0 ? g[k][0] : j == 1 ? g[k][1] : j == 2 ? g[k][2] : g[k][3]; };
        float tt[OPT];
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            F1[k] = fmaf(A.kn, fmaf(cs[k], S, -sn[k] * C), om[k]);
            tt[k] = fmaf(A.omega_scale, F1[k], th[k]) + noise(k);
        }
        if (SCHEME == SDE_HEUN) {
            float S2, C2;
            double S2d, C2d;
            if (!reduce(tt, S2, C2, S2d, C2d)) break;
#pragma unroll
            for (int k = 0; k < OPT; ++k) {
                const float F2 = fmaf(A.kn, fmaf(cs[k], S2, -sn[k] * C2), om[k]);
                const float t = fmaf(A.hdt2pi, F1[k] + F2, th[k]) + noise(k);
                th[k] = t - floorf(t);
            }
        } else {
#pragma unroll
            for (int k = 0; k < OPT; ++k) th[k] = tt[k] - floorf(tt[k]);
        }
        ++n;
        ++local;
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
        if (live[k]) {
            A.theta[(uint64_t)r * N + idx[k]] = th[k];
            bad |= !isfinite(th[k]);
        }
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(A.flag, 1);
}

// ------------------------------------ MF, two realizations per workgroup --
// The register-resident mean field with the exchange latency hidden behind
// arithmetic: every workgroup holds the same slice of oscillators of two
// realizations (A = 2p and B = 2p + 1 of the launch) in eight compute waves,
// plus one exchange wave per realization.  The compute waves alternate
// between the two realizations -- while A's sums travel between the
// workgroups they evaluate B's stage, and the other way round -- and meet
// the exchange waves only through flags in LDS, so no workgroup barrier is
// on the step path.  An exchange wave adds its realization's eight wave
// partials in wave order (FP64), publishes the sum as four tagged words,
// polls the G workgroups' words (up to 32 workgroups, two words per lane),
// adds the G pairs in a fixed order -- every workgroup of a realization gets
// the same bits -- and leaves the sums in LDS.  Per realization the epochs,
// words and their two parities are those of the one-realization kernel.
constexpr int kMFPWaves = kMFWaves + 2;
constexpr int kMFPThreads = kMFPWaves * kWave;
constexpr uint32_t kMaxMFPGroups = 2 * kWave / kMFWordsPerGroup;

struct MFPShared {
    float ps[2][kMFWaves], pc[2][kMFWaves];  // per-wave FP32 partials of A and B
    double S[2], C[2];                       // the realizations' sums of the epoch in ready[]
    uint32_t arrived[2];                     // wave partials written so far (8 per epoch)
    uint32_t ready[2];                       // epoch whose sums are in S, C
    int ok;
    int local;                               // the pair's workgroups share one XCD
    __attribute__((aligned(16))) uint32_t words[2][kWave];  // each exchange wave's staged words
};

__device__ __forceinline__ uint32_t lds_acquire(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_release(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Lanes poll words t and t + 64 (t < n, n <= 128) at p(.) until both carry
// `tag`; both loads are in flight together.  False once a wait exceeded the
// spin bound (the error flag is then set).
template <typename Addr>
__device__ __forceinline__ bool mfp_poll(const MFArgs& A, uint32_t n, Addr p, uint64_t tag, uint32_t& d0,
                                         uint32_t& d1)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool has0 = lane < n, has1 = lane + kWave < n;
    const uint64_t* q0 = p(has0 ? lane : 0u);
    const uint64_t* q1 = p(has1 ? lane + kWave : 0u);
    bool ok = true, got0 = !has0, got1 = !has1;
    uint32_t spins = 0;
    d0 = d1 = 0u;
    while (!(got0 && got1)) {
        const uint64_t v0 = got0 ? tag : __hip_atomic_load(q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t v1 = got1 ? tag : __hip_atomic_load(q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!got0 && (v0 & 0xffffffff00000000ull) == tag) {
            got0 = true;
            d0 = (uint32_t)v0;
        }
        if (!got1 && (v1 & 0xffffffff00000000ull) == tag) {
            got1 = true;
            d1 = (uint32_t)v1;
        }
        if (got0 && got1) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > A.spin_limit) {
            ok = false;
            break;
        }
    }
    if (__ballot(!ok) != 0) {
        if (lane == 0) atomicOr(A.flag, 2);
        return false;
    }
    return true;
}

// Exchange wave of realization X (0 = A, 1 = B): for every epoch, the
// workgroup's sum published as soon as the eight wave partials are in, then
// the G workgroups' sums polled, added and handed to the compute waves.
__device__ __forceinline__ void mfp_exchange_loop(const MFArgs& A, int X, uint32_t r, uint32_t w, uint64_t n_epochs,
                                                  MFPShared& sh)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool local = sh.local != 0;
    const uint32_t per1 = A.G * kMFWordsPerGroup;
    auto d = [](float x) { return (double)x; };
    for (uint32_t e = 1; e <= (uint32_t)n_epochs; ++e) {
        const uint64_t tag = (uint64_t)(e + 1) << 32;
        uint32_t spins = 0;
        while (lds_acquire(&sh.arrived[X]) < kMFWaves * e) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > A.spin_limit) {
                if (lane == 0) {
                    __hip_atomic_store(&sh.ok, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    atomicOr(A.flag, 2);
                }
                return;
            }
        }
        const double Sw = ((d(sh.ps[X][0]) + d(sh.ps[X][1])) + (d(sh.ps[X][2]) + d(sh.ps[X][3]))) +
                          ((d(sh.ps[X][4]) + d(sh.ps[X][5])) + (d(sh.ps[X][6]) + d(sh.ps[X][7])));
        const double Cw = ((d(sh.pc[X][0]) + d(sh.pc[X][1])) + (d(sh.pc[X][2]) + d(sh.pc[X][3]))) +
                          ((d(sh.pc[X][4]) + d(sh.pc[X][5])) + (d(sh.pc[X][6]) + d(sh.pc[X][7])));
        uint32_t d0 = 0u, d1 = 0u;
        if (A.G > 1) {
            mf2_publish_lanes(mf_word(A, A.slots, per1, r, e, w * kMFWordsPerGroup), tag, Sw, Cw, local);
            if (!mfp_poll(A, per1, [&](uint32_t t) { return mf_word(A, A.slots, per1, r, e, t); }, tag, d0, d1)) {
                if (lane == 0) __hip_atomic_store(&sh.ok, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
        } else if (lane < kMFWordsPerGroup) {  // one workgroup: its own sums are the pair
            const uint64_t v = (uint64_t)__double_as_longlong(lane < 2 ? Sw : Cw);
            d0 = (lane & 1u) ? (uint32_t)(v >> 32) : (uint32_t)v;
        }
        double S, C;
        mf2_sum_words(d0, sh.words[X], S, C);
        if (per1 > (uint32_t)kWave) {
            double S1, C1;
            mf2_sum_words(d1, sh.words[X], S1, C1);
            S += S1;
            C += C1;
        }
        if (lane == 0) {
            sh.S[X] = S;
            sh.C[X] = C;
            lds_release(&sh.ready[X], e);
        }
    }
}

template <int OPT, int SCHEME>
__global__ __launch_bounds__(kMFPThreads, 1) void kuramoto_mfp_kernel(MFArgs A)
{
    __shared__ MFPShared sh;
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        sh.ok = 1;
        sh.local = 0;
        sh.arrived[0] = sh.arrived[1] = 0u;
        sh.ready[0] = sh.ready[1] = 0u;
    }
    // workgroup -> (pair p, slice w)
    uint32_t p, w;
    if (A.xcd_map) {
        const uint32_t x = blockIdx.x & 7u, l = blockIdx.x >> 3, per = (A.R >> 1) >> 3;
        p = x * per + l / A.G;
        w = l % A.G;
    } else {
        p = blockIdx.x / A.G;
        w = blockIdx.x % A.G;
    }
    const uint32_t rA = 2 * p;
    const uint64_t n_epochs = (SCHEME == SDE_HEUN ? 2 : 1) * A.n_steps + 1;
    __syncthreads();
    if (wid == kMFWaves && A.G > 1) mf2_locality(A, rA, w, sh);
    __syncthreads();
    if (!sh.ok) return;
    if (wid >= kMFWaves) {
        // The exchanges are the critical path: their waves issue before the
        // compute waves that share their SIMDs (those fill their waits with
        // noise generation).
        __builtin_amdgcn_s_setprio(3);
        mfp_exchange_loop(A, (int)(wid - kMFWaves), rA + (wid - kMFWaves), w, n_epochs, sh);
        return;
    }

    const uint32_t N = A.N;
    float th[2][OPT], F1[2][OPT], sn[2][OPT], cs[2][OPT], om[OPT];
    uint32_t idx[OPT];
    bool live[OPT];
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
        idx[k] = (w * OPT + k) * kMFThreads + threadIdx.x;
        live[k] = idx[k] < N;
        const uint32_t i = live[k] ? idx[k] : 0u;
        om[k] = live[k] ? A.omega[i] : 0.f;
#pragma unroll
        for (int X = 0; X < 2; ++X) {
            if (A.init_from_state) {
                th[X][k] = live[k] ? A.theta[(uint64_t)(rA + X) * N + i] : 0.f;
            } else {
                const U4 x = philox4x32_10(U4{0u, i, A.r_base + rA + X, (uint32_t)SDE_TAG_INIT}, A.key0, A.key1);
                th[X][k] = (float)(x.x >> 8) * 0x1p-24f;
            }
        }
    }
    // Noise of the current block of 4 steps (g) and of the next (gn), the
    // latter generated one (realization, oscillator) item at a time while a
    // wave waits for sums; gn_done items are ready (wave-uniform).
    float g[2][OPT][4], gn[2][OPT][4];
    uint64_t gblk = ~0ull;
    uint32_t gn_done = 0;
    // (Selects rather than a branch per item: the compiler would merge the
    // branches into one store at a computed index and move gn to scratch.)
    auto prefetch1 = [&]() {
        if (gblk == ~0ull || gn_done >= 2u * OPT) return;
        const uint32_t nb = (uint32_t)(gblk + 1), Xs = gn_done / OPT, ks = gn_done % OPT;
        uint32_t i = idx[0];
#pragma unroll
        for (int k = 1; k < OPT; ++k) i = (uint32_t)k == ks ? idx[k] : i;
        float t[4];
        gauss4_scaled(U4{nb, i, A.r_base + rA + Xs, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2, t);
#pragma unroll
        for (int X = 0; X < 2; ++X)
#pragma unroll
            for (int k = 0; k < OPT; ++k) {
                const bool mine = (uint32_t)(X * OPT + k) == gn_done;
#pragma unroll
                for (int q = 0; q < 4; ++q) gn[X][k][q] = mine ? t[q] : gn[X][k][q];
            }
        ++gn_done;
    };
    // sin and cos of realization X's phases t[] (kept for the drift) and the
    // wave's FP32 sums of them, handed to the exchange wave
    auto partial = [&](int X, const float (&t)[OPT]) {
        float s = 0.f, c = 0.f;
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            sn[X][k] = live[k] ? sin_rev(t[k]) : 0.f;
            cs[X][k] = live[k] ? cos_rev(t[k]) : 0.f;
            s += sn[X][k];
            c += cs[X][k];
        }
        s = wave_sum_dpp(s);
        c = wave_sum_dpp(c);
        if (lane == kWave - 1) {
            sh.ps[X][wid] = s;
            sh.pc[X][wid] = c;
            __hip_atomic_fetch_add(&sh.arrived[X], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    // realization X's sums of epoch e, generating noise while they are not there
    auto await = [&](int X, uint32_t e, double& Sd, double& Cd) -> bool {
        if (lds_acquire(&sh.ready[X]) != e) {
            prefetch1();
            uint32_t spins = 0;
            while (lds_acquire(&sh.ready[X]) != e) {
                if (__hip_atomic_load(&sh.ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) return false;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > A.spin_limit) {
                    if (lane == 0) atomicOr(A.flag, 2);
                    return false;
                }
            }
        }
        Sd = sh.S[X];
        Cd = sh.C[X];
        return true;
    };

#pragma unroll
    for (int X = 0; X < 2; ++X) partial(X, th[X]);
    uint32_t e = 1;
    const double invN = 1.0 / (double)N;
    uint64_t n = A.step0;
    const uint64_t n_end = A.step0 + A.n_steps;
    uint64_t local = 0;
    bool ok = true;
    for (;;) {
        const bool last = n == n_end;
        if (!last && (n >> 2) != gblk) {
            const uint64_t b = n >> 2;
            if (gblk != ~0ull && b == gblk + 1 && gn_done == 2u * OPT) {
#pragma unroll
                for (int X = 0; X < 2; ++X)
#pragma unroll
                    for (int k = 0; k < OPT; ++k)
#pragma unroll
                        for (int q = 0; q < 4; ++q) g[X][k][q] = gn[X][k][q];
            } else {
#pragma unroll
                for (int X = 0; X < 2; ++X)
#pragma unroll
                    for (int k = 0; k < OPT; ++k)
                        gauss4_scaled(U4{(uint32_t)b, idx[k], A.r_base + rA + X, (uint32_t)SDE_TAG_NOISE}, A.key0,
                                      A.key1, A.c2, g[X][k]);
            }
            gblk = b;
            gn_done = 0;
        }
        const uint32_t j = (uint32_t)n & 3u;
        auto noise = [&](int X, int k) {
            return j == 0 ? g[X][k][0] : j == 1 ? g[X][k][1] : j == 2 ? g[X][k][2] : g[X][k][3];
        };
        // stage 1 (the Euler-Maruyama step): sums at theta_n; every M steps r
#pragma unroll
        for (int X = 0; X < 2; ++X) {
            double Sd, Cd;
            if (ok && !await(X, e, Sd, Cd)) ok = false;
            if (!ok) break;
            if (A.r_samples && local % A.M == 0 && w == 0 && threadIdx.x == 0)
                A.r_samples[(uint64_t)(rA + X) * A.n_samples + local / A.M] = std::sqrt(Sd * Sd + Cd * Cd) * invN;
            if (last) continue;
            const float S = (float)Sd, C = (float)Cd;
            float tt[OPT];
#pragma unroll
            for (int k = 0; k < OPT; ++k) {
                F1[X][k] = fmaf(A.kn, fmaf(cs[X][k], S, -sn[X][k] * C), om[k]);
                tt[k] = fmaf(A.omega_scale, F1[X][k], th[X][k]) + noise(X, k);
            }
            if (SCHEME == SDE_HEUN) {
                partial(X, tt);
            } else {
#pragma unroll
                for (int k = 0; k < OPT; ++k) th[X][k] = tt[k] - floorf(tt[k]);
                partial(X, th[X]);
            }
        }
        if (!ok || last) break;
        ++e;
        if (SCHEME == SDE_HEUN) {
            // stage 2: sums at the predictor
#pragma unroll
            for (int X = 0; X < 2; ++X) {
                double S2d, C2d;
                if (ok && !await(X, e, S2d, C2d)) ok = false;
                if (!ok) break;
                const float S2 = (float)S2d, C2 = (float)C2d;
#pragma unroll
                for (int k = 0; k < OPT; ++k) {
                    const float F2 = fmaf(A.kn, fmaf(cs[X][k], S2, -sn[X][k] * C2), om[k]);
                    const float t = fmaf(A.hdt2pi, F1[X][k] + F2, th[X][k]) + noise(X, k);
                    th[X][k] = t - floorf(t);
                }
                partial(X, th[X]);
            }
            if (!ok) break;
            ++e;
        }
        ++n;
        ++local;
    }
    bool bad = false;
#pragma unroll
    for (int X = 0; X < 2; ++X)
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            if (live[k]) {
                A.theta[(uint64_t)(rA + X) * N + idx[k]] = th[X][k];
                bad |= !isfinite(th[X][k]);
            }
        }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(A.flag, 1);
}

// ------------------------------------------------------ MF, streamed ------
// The mean field for realizations too large for registers (beyond 256
// workgroups x 4096 oscillators, e.g. the 2^24 identical oscillators of
// Fig. 4): the same cooperative launch and exchange, but every workgroup
// streams its slice of theta through HBM at every stage.  Heun: the
// predictor pass reads theta and omega and writes the predictor tt and
//   carry = theta + dt/(4 pi) (F1 + omega) + noise,
// so that the corrector pass needs only tt and carry:
//   theta' = carry + dt/(4 pi) (K/N) (cos tt S2 - sin tt C2)
// (28 bytes per oscillator-step; Euler-Maruyama 12).  The noise is component
// n & 3 of the Gaussians of Philox block n >> 2, regenerated every step: the
// same stream the register-resident kernel draws once per block.
struct MFSArgs {
    float* theta;            // [R][N] revolutions, in/out (this launch's realizations)
    const float* omega;      // [N]
    float* tilde;            // [R][N] predictor (Heun)
    float* carry;            // [R][N] theta + dt/(4 pi) (F1 + omega) + noise (Heun)
    double* r_samples;       // [R][n_samples] or null
    uint64_t* slots;         // exchange words, as MFArgs
    uint64_t* slots2;
    int* flag;
    uint32_t N, R, G, M;
    uint32_t r_base;
    uint32_t chunk;          // oscillators per workgroup slice
    uint64_t step0, n_steps, n_samples;
    uint32_t key0, key1;
    float omega_scale, hdt2pi, kn, c2;
    uint32_t spin_limit;
    uint32_t tree;
};

// Each pass takes kMFSBatch oscillators per lane per iteration (stride
// kMFSThreads), all loads first, to keep several memory requests in flight.
constexpr int kMFSBatch = 4;

template <int SCHEME>
__global__ __launch_bounds__(kMFSThreads, 1) void kuramoto_mfs_kernel(MFSArgs A)
{
    __shared__ double lds[2 * kMFSThreads / kWave];
    __shared__ uint32_t words[kMFWordsPerGroup * kMaxMFSGroups];
    __shared__ int lds_ok;
    if (threadIdx.x == 0) lds_ok = 1;  // made visible by the exchange's first barrier
    const uint32_t r = blockIdx.x / A.G, w = blockIdx.x % A.G;
    const uint64_t N = A.N;
    const uint64_t i0 = (uint64_t)w * A.chunk, i1 = std::min<uint64_t>(N, i0 + A.chunk);
    float* th = A.theta + (uint64_t)r * N;
    float* tl = A.tilde + (uint64_t)r * N;
    float* cy = A.carry + (uint64_t)r * N;
    const uint32_t rr = A.r_base + r;
    constexpr uint64_t kStep = (uint64_t)kMFSBatch * kMFSThreads;
    uint32_t epoch = 0;
    auto exchange = [&](double s, double c, double& S, double& C) -> bool {
        if (!mf_exchange<kMFSThreads>(A, r, w, epoch, s, c, lds, words, &lds_ok, S, C)) return false;
        ++epoch;
        return true;
    };
    double s = 0.0, c = 0.0, S, C;
    for (uint64_t b = i0 + threadIdx.x; b < i1; b += kStep) {
        float t[kMFSBatch];
#pragma unroll
        for (int k = 0; k < kMFSBatch; ++k) {
            const uint64_t i = b + (uint64_t)k * kMFSThreads;
            t[k] = i < i1 ? th[i] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kMFSBatch; ++k)
            if (b + (uint64_t)k * kMFSThreads < i1) {
                s += (double)sin_rev(t[k]);
                c += (double)cos_rev(t[k]);
            }
    }
    if (!exchange(s, c, S, C)) return;
    const double invN = 1.0 / (double)N;
    uint64_t n = A.step0, local = 0;
    const uint64_t n_end = A.step0 + A.n_steps;
    for (;;) {
        if (A.r_samples && local % A.M == 0 && w == 0 && threadIdx.x == 0)
            A.r_samples[(uint64_t)r * A.n_samples + local / A.M] = std::sqrt(S * S + C * C) * invN;
        if (n == n_end) break;
        const uint32_t blk = (uint32_t)(n >> 2), j = (uint32_t)n & 3u;
        float Sf = (float)S, Cf = (float)C;
        s = 0.0;
        c = 0.0;
        // predictor (Heun) or the whole step (Euler-Maruyama)
        for (uint64_t b = i0 + threadIdx.x; b < i1; b += kStep) {
            float t0[kMFSBatch], om[kMFSBatch];
#pragma unroll
            for (int k = 0; k < kMFSBatch; ++k) {
                const uint64_t i = b + (uint64_t)k * kMFSThreads;
                t0[k] = i < i1 ? th[i] : 0.f;
                om[k] = i < i1 ? A.omega[i] : 0.f;
            }
#pragma unroll
            for (int k = 0; k < kMFSBatch; ++k) {
                const uint64_t i = b + (uint64_t)k * kMFSThreads;
                if (i >= i1) continue;
                const float F1 = fmaf(A.kn, fmaf(cos_rev(t0[k]), Sf, -sin_rev(t0[k]) * Cf), om[k]);
                const float ns =
                    gauss1_scaled(U4{blk, (uint32_t)i, rr, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2, j);
                const float tt = fmaf(A.omega_scale, F1, t0[k]) + ns;
                float u;
                if (SCHEME == SDE_HEUN) {
                    tl[i] = tt;
                    cy[i] = fmaf(A.hdt2pi, F1 + om[k], t0[k]) + ns;
                    u = tt;
                } else {
                    u = tt - floorf(tt);
                    th[i] = u;
                }
                s += (double)sin_rev(u);
                c += (double)cos_rev(u);
            }
        }
        if (!exchange(s, c, S, C)) return;
        if (SCHEME == SDE_HEUN) {
            Sf = (float)S;
            Cf = (float)C;
            s = 0.0;
            c = 0.0;
            for (uint64_t b = i0 + threadIdx.x; b < i1; b += kStep) {
                float tt[kMFSBatch], cv[kMFSBatch];
#pragma unroll
                for (int k = 0; k < kMFSBatch; ++k) {
                    const uint64_t i = b + (uint64_t)k * kMFSThreads;
                    tt[k] = i < i1 ? tl[i] : 0.f;
                    cv[k] = i < i1 ? cy[i] : 0.f;
                }
#pragma unroll
                for (int k = 0; k < kMFSBatch; ++k) {
                    const uint64_t i = b + (uint64_t)k * kMFSThreads;
                    if (i >= i1) continue;
                    const float t = fmaf(A.hdt2pi, A.kn * fmaf(cos_rev(tt[k]), Sf, -sin_rev(tt[k]) * Cf), cv[k]);
                    const float u = t - floorf(t);
                    th[i] = u;
                    s += (double)sin_rev(u);
                    c += (double)cos_rev(u);
                }
            }
            if (!exchange(s, c, S, C)) return;
        }
        ++n;
        ++local;
    }
    bool bad = false;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kMFSThreads) bad |= !isfinite(th[i]);
    if (__ballot(bad) != 0 && (threadIdx.x & (kWave - 1)) == 0) atomicOr(A.flag, 1);
}

__global__ void mf_zero_kernel(uint32_t* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------- TILED ------
constexpr int kTileThreads = 256;

struct TiledArgs {
    const float* src;        // [R][N] phases the coupling sum is taken over
    const float* base;       // [R][N] phases theta_n the step starts from
    float* dst;              // [R][N] output phases
    float* F1;               // [R][N] stage-1 drift (written by stage 1, read by stage 2)
    const float* omega;      // [N]
    const uint64_t* nbase;   // device: absolute step of the current chunk's first step
    uint32_t k;              // step within the chunk
    uint32_t N, R;
    uint32_t key0, key1;
    float omega_scale, hdt2pi, kn, c2;
    int32_t stage;           // 1: predictor (or Euler step), 2: corrector
    int32_t euler;
};

// The stage update of oscillator i of realization r from its coupling sum
// acc = sum_j sin(2 pi (src_j - src_i)).
__device__ __forceinline__ void tiled_stage_update(const TiledArgs& A, uint32_t r, uint32_t i, float acc, uint64_t n)
{
    const uint64_t gi = (uint64_t)r * A.N + i;
    const float F = fmaf(A.kn, acc, A.omega[i]);
    const float ns = gauss1_scaled(U4{(uint32_t)(n >> 2), i, r, (uint32_t)SDE_TAG_NOISE}, A.key0, A.key1, A.c2,
                                   (uint32_t)n & 3u);
    const float th = A.base[gi];
    if (A.stage == 1) {
        const float t = fmaf(A.omega_scale, F, th) + ns;
        A.dst[gi] = A.euler ? t - floorf(t) : t;
        if (!A.euler) A.F1[gi] = F;
    } else {
        const float t = fmaf(A.hdt2pi, A.F1[gi] + F, th) + ns;
        A.dst[gi] = t - floorf(t);
    }
}

// Coupling sums of OPT oscillators per lane over j in [j_lo, j_hi):
// tiles of src_j staged in LDS and read by all lanes (broadcast).
template <int OPT>
__device__ __forceinline__ void tiled_sums(const float* src, uint32_t N, uint32_t j_lo, uint32_t j_hi, float* tile,
                                           const float (&mine)[OPT], float (&acc)[OPT])
{
    constexpr int TILE = kTileThreads * OPT;
    for (uint32_t j0 = j_lo; j0 < j_hi; j0 += TILE) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            const uint32_t j = j0 + k * kTileThreads + threadIdx.x;
            tile[k * kTileThreads + threadIdx.x] = j < j_hi ? src[j] : 0.f;
        }
        __syncthreads();
        const uint32_t cnt = j_hi - j0 < (uint32_t)TILE ? j_hi - j0 : (uint32_t)TILE;
        if (cnt == (uint32_t)TILE) {
#pragma unroll 8
            for (int t = 0; t < TILE; ++t) {
                const float x = tile[t];
#pragma unroll
                for (int k = 0; k < OPT; ++k) acc[k] += sin_rev(x - mine[k]);
            }
        } else {
            for (uint32_t t = 0; t < cnt; ++t) {
                const float x = tile[t];
#pragma unroll
                for (int k = 0; k < OPT; ++k) acc[k] += sin_rev(x - mine[k]);
            }
        }
    }
}

// One stage for OPT oscillators per lane: F_i = omega_i + kn sum_j
// sin(2 pi (src_j - src_i)) over all j, then the stage's update.
template <int OPT>
__global__ __launch_bounds__(kTileThreads) void kuramoto_tiled_kernel(TiledArgs A)
{
    constexpr int TILE = kTileThreads * OPT;
    __shared__ float tile[TILE];
    const uint32_t r = blockIdx.y;
    const uint32_t N = A.N;
    const float* src = A.src + (uint64_t)r * N;
    float mine[OPT], acc[OPT];
    uint32_t idx[OPT];
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
        idx[k] = blockIdx.x * TILE + k * kTileThreads + threadIdx.x;
        mine[k] = idx[k] < N ? src[idx[k]] : 0.f;
        acc[k] = 0.f;
    }
    tiled_sums<OPT>(src, N, 0, N, tile, mine, acc);
    const uint64_t n = load_uniform(A.nbase) + A.k;
#pragma unroll
    for (int k = 0; k < OPT; ++k)
        if (idx[k] < N) tiled_stage_update(A, r, idx[k], acc[k], n);
}

// Small-N remedy (the paper's suggestion of less work per thread and more
// threads, Sec. 6): the j range is split into gridDim.z slices of `jlen`;
// slice z writes its partial sums to part[z][r][i] ...
template <int OPT>
__global__ __launch_bounds__(kTileThreads) void kuramoto_tiled_part_kernel(TiledArgs A, float* part, uint32_t jlen)
{
    constexpr int TILE = kTileThreads * OPT;
    __shared__ float tile[TILE];
    const uint32_t r = blockIdx.y, z = blockIdx.z;
    const uint32_t N = A.N;
    const float* src = A.src + (uint64_t)r * N;
    const uint32_t j_lo = z * jlen, j_hi = min(N, j_lo + jlen);
    float mine[OPT], acc[OPT];
    uint32_t idx[OPT];
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
        idx[k] = blockIdx.x * TILE + k * kTileThreads + threadIdx.x;
        mine[k] = idx[k] < N ? src[idx[k]] : 0.f;
        acc[k] = 0.f;
    }
    tiled_sums<OPT>(src, N, j_lo, j_hi, tile, mine, acc);
#pragma unroll
    for (int k = 0; k < OPT; ++k)
        if (idx[k] < N) part[((uint64_t)z * A.R + r) * N + idx[k]] = acc[k];
}

// ... and this kernel adds the J partials of each oscillator in slice order
// (bitwise reproducible) and applies the stage update.
__global__ __launch_bounds__(256) void kuramoto_tiled_combine_kernel(TiledArgs A, const float* part, uint32_t J)
{
    const uint64_t NR = (uint64_t)A.N * A.R;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= NR) return;
    float acc = 0.f;
    for (uint32_t z = 0; z < J; ++z) acc += part[(uint64_t)z * NR + g];
    tiled_stage_update(A, (uint32_t)(g / A.N), (uint32_t)(g % A.N), acc, load_uniform(A.nbase) + A.k);
}

__global__ __launch_bounds__(256) void order_parameter_kernel(const float* theta, uint32_t N, double* out,
                                                              uint64_t stride, uint64_t col)
{
    __shared__ double lds[2 * 256 / kWave];
    const uint32_t r = blockIdx.x;
    double s = 0.0, c = 0.0;
    for (uint32_t i = threadIdx.x; i < N; i += 256) {
        const float t = theta[(uint64_t)r * N + i];
        s += (double)sin_rev(t);
        c += (double)cos_rev(t);
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    s = wave_sum(s);
    c = wave_sum(c);
    if (lane == 0) {
        lds[2 * wid] = s;
        lds[2 * wid + 1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, C = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) {
            S += lds[2 * w];
            C += lds[2 * w + 1];
        }
        out[(uint64_t)r * stride + col] = std::sqrt(S * S + C * C) / (double)N;
    }
}

// The same, at local step l = *nbase - step0, only when l is a multiple of
// M (column l / M): lets one recorded chunk of steps sample where due.
__global__ __launch_bounds__(256) void order_parameter_at_kernel(const float* theta, uint32_t N, double* out,
                                                                 uint64_t stride, const uint64_t* nbase,
                                                                 uint64_t step0, uint32_t M)
{
    const uint64_t l = load_uniform(nbase) - step0;
    if (l % M) return;
    __shared__ double lds[2 * 256 / kWave];
    const uint32_t r = blockIdx.x;
    double s = 0.0, c = 0.0;
    for (uint32_t i = threadIdx.x; i < N; i += 256) {
        const float t = theta[(uint64_t)r * N + i];
        s += (double)sin_rev(t);
        c += (double)cos_rev(t);
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    s = wave_sum(s);
    c = wave_sum(c);
    if (lane == 0) {
        lds[2 * wid] = s;
        lds[2 * wid + 1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, C = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) {
            S += lds[2 * w];
            C += lds[2 * w + 1];
        }
        out[(uint64_t)r * stride + l / M] = std::sqrt(S * S + C * C) / (double)N;
    }
}

__global__ void step_set_kernel(uint64_t* nbase, uint64_t v) { *nbase = v; }
__global__ void step_advance_kernel(uint64_t* nbase, uint32_t by) { *nbase += by; }

__global__ void copy_f32_kernel(float* dst, const float* src, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Initial phases theta = U(Philox(0, i, r, INIT).x0), one thread per oscillator.
__global__ void kuramoto_init_kernel(float* theta, uint32_t N, uint32_t R, uint32_t key0, uint32_t key1)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)N * R) return;
    const uint32_t r = (uint32_t)(g / N), i = (uint32_t)(g % N);
    const U4 x = philox4x32_10(U4{0u, i, r, (uint32_t)SDE_TAG_INIT}, key0, key1);
    theta[g] = (float)(x.x >> 8) * 0x1p-24f;
}

// ------------------------------------------------------------------ host --

void launch_order_parameter(const float* theta, uint32_t N, uint32_t R, double* out, uint64_t stride,
                            uint64_t col, hipStream_t stream)
{
    hipLaunchKernelGGL(order_parameter_kernel, dim3(R), dim3(256), 0, stream, theta, N, out, stride, col);
}

void launch_order_parameter_at(const float* theta, uint32_t N, uint32_t R, double* out, uint64_t stride,
                               const uint64_t* nbase, uint64_t step0, uint32_t M, hipStream_t stream)
{
    hipLaunchKernelGGL(order_parameter_at_kernel, dim3(R), dim3(256), 0, stream, theta, N, out, stride, nbase, step0,
                       M);
}

void launch_step_set(uint64_t* nbase, uint64_t v, hipStream_t stream)
{
    hipLaunchKernelGGL(step_set_kernel, dim3(1), dim3(1), 0, stream, nbase, v);
}

void launch_step_advance(uint64_t* nbase, uint32_t by, hipStream_t stream)
{
    hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(1), 0, stream, nbase, by);
}

uint32_t chunk_steps(uint32_t M, uint64_t n_steps, bool even)
{
    // largest divisor of M that is at most 128 (and even if required), so
    // that every sampling step is a chunk start
    uint32_t best = 0;
    for (uint32_t c = 1; c <= 128 && c <= M; ++c)
        if (M % c == 0 && (!even || c % 2 == 0)) best = c;
    if (best == 0) best = even ? 2 : 1;
    if ((uint64_t)best > n_steps && n_steps > 0) best = (uint32_t)n_steps;
    return best;
}

void launch_kuramoto_init(float* theta, uint32_t N, uint32_t R, uint64_t seed, hipStream_t stream)
{
    const uint64_t NR = (uint64_t)N * R;
    hipLaunchKernelGGL(kuramoto_init_kernel, dim3((uint32_t)((NR + 255) / 256)), dim3(256), 0, stream, theta, N,
                       R, (uint32_t)seed, (uint32_t)(seed >> 32));
}

static int validate(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, const float* phi,
                    const float* omega, const float* K, const double* r_samples)
{
    if (!d || !run) return fail(ctx, SDE_ERR_INVALID, "null descriptor or run");
    if (d->N == 0 || d->R == 0) return fail(ctx, SDE_ERR_INVALID, "N and R must be > 0");
    if (!std::isfinite(d->K) || !std::isfinite(d->D) || !std::isfinite(d->dt) || !(d->dt > 0) || d->D < 0)
        return fail(ctx, SDE_ERR_INVALID, "need finite K, D >= 0, dt > 0");
    if (d->reserved != 0) return fail(ctx, SDE_ERR_INVALID, "reserved field must be 0");
    if (run->scheme != SDE_HEUN && run->scheme != SDE_EULER)
        return fail(ctx, SDE_ERR_INVALID, "unknown scheme %d", run->scheme);
    if (run->init != SDE_INIT_PHILOX && run->init != SDE_INIT_FROM_STATE)
        return fail(ctx, SDE_ERR_INVALID, "unknown init %d", run->init);
    if (!phi || !omega) return fail(ctx, SDE_ERR_INVALID, "phi and omega are required");
    const bool dense = d->coupling == SDE_DENSE_FP32 || d->coupling == SDE_DENSE_BF16X3 ||
                       d->coupling == SDE_DENSE_FP16X3;
    if (d->coupling < SDE_MEANFIELD || d->coupling > SDE_DENSE_FP16X3)
        return fail(ctx, SDE_ERR_INVALID, "unknown coupling %d", d->coupling);
    if (dense && !K) return fail(ctx, SDE_ERR_INVALID, "dense coupling needs K");
    if (!dense && K) return fail(ctx, SDE_ERR_INVALID, "uniform coupling takes no K matrix");
    if (!aligned(phi, 4) || !aligned(omega, 4) || !aligned(K, 16) || !aligned(r_samples, 8))
        return fail(ctx, SDE_ERR_INVALID, "misaligned device pointer");
    if ((uint64_t)d->N * d->R > (1ull << 40)) return fail(ctx, SDE_ERR_INVALID, "N * R too large");
    if (d->coupling == SDE_MEANFIELD && d->n_steps >= (1ull << 31))
        return fail(ctx, SDE_ERR_INVALID, "mean field: at most 2^31 - 1 steps per call (the exchange tags count "
                    "stages in 32 bits); split the run, it resumes bit for bit");
    return SDE_OK;
}

KuraConsts kuramoto_consts(const sde_kuramoto_desc* d)
{
    KuraConsts c;
    c.omega_scale = (float)(d->dt / (2.0 * M_PI));
    c.hdt2pi = (float)(d->dt / (4.0 * M_PI));
    c.kn = (float)(d->K / (double)d->N);
    const double sig = std::sqrt(2.0 * d->D * d->dt) / (2.0 * M_PI);
    c.c2 = (float)(-2.0 * M_LN2 * sig * sig);
    return c;
}

template <int OPT, int SCHEME>
static void* mf_kernel_ptr()
{
    return reinterpret_cast<void*>(kuramoto_mf_kernel<OPT, SCHEME>);
}

template <int OPT, int SCHEME>
static void* mfp_kernel_ptr()
{
    return reinterpret_cast<void*>(kuramoto_mfp_kernel<OPT, SCHEME>);
}

// The streamed mean field: G workgroups per realization (as many as fit
// co-resident, at most kMaxMFSGroups), each owning a contiguous slice.
static int run_meanfield_streamed(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                                  const float* omega, double* r_samples, uint64_t n_samples, uint32_t M,
                                  hipStream_t stream)
{
    const KuraConsts kc = kuramoto_consts(d);
    const bool heun = run->scheme == SDE_HEUN;
    void* kern = heun ? reinterpret_cast<void*>(kuramoto_mfs_kernel<SDE_HEUN>)
                      : reinterpret_cast<void*>(kuramoto_mfs_kernel<SDE_EULER>);
    int per_cu = 0;
    SDE_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kMFSThreads, 0));
    const uint64_t capacity = (uint64_t)std::max(per_cu, 0) * ctx->n_cu;
    if (capacity == 0) return fail(ctx, SDE_ERR_UNSUPPORTED, "streamed mean-field kernel does not fit a CU");
    const uint32_t r_per_launch = (uint32_t)std::min<uint64_t>(d->R, capacity);
    const uint64_t by_lanes = ((uint64_t)d->N + kMFSThreads - 1) / kMFSThreads;
    const uint32_t G = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>({(uint64_t)kMaxMFSGroups, capacity / r_per_launch, by_lanes}));
    const uint32_t chunk = (uint32_t)(((uint64_t)d->N + G - 1) / G);
    const uint64_t NR = (uint64_t)d->N * d->R;
    if (run->init == SDE_INIT_PHILOX) {
        launch_kuramoto_init(phi, d->N, d->R, run->seed, stream);
        SDE_HIP(ctx, hipGetLastError());
    }
    void* work = nullptr;
    int st = SDE_OK;
    if (heun && (st = ensure_ws(ctx, kSlotKuraWork, (size_t)2 * NR * sizeof(float), &work))) return st;
    void* slots = nullptr;
    const size_t slot_words = (size_t)2 * r_per_launch * G * kMFWordsPerGroup;
    const size_t slot2_words = (size_t)2 * r_per_launch * 8 * kMFWordsPerGroup;
    if ((st = ensure_ws(ctx, kSlotKuraPartials, (slot_words + slot2_words) * sizeof(uint64_t), &slots))) return st;
    for (uint32_t r0 = 0; r0 < d->R; r0 += r_per_launch) {
        const uint32_t nr = std::min(r_per_launch, d->R - r0);
        const size_t n32 = 2 * (slot_words + slot2_words);
        hipLaunchKernelGGL(mf_zero_kernel, dim3((uint32_t)((n32 + 255) / 256)), dim3(256), 0, stream,
                           static_cast<uint32_t*>(slots), n32);
        SDE_HIP(ctx, hipGetLastError());
        MFSArgs A;
        A.slots2 = static_cast<uint64_t*>(slots) + slot_words;
        A.tree = (G >= kMFTreeMinGroups && G % 8 == 0) ? 1u : 0u;
        A.theta = phi + (uint64_t)r0 * d->N;
        A.omega = omega;
        A.tilde = heun ? static_cast<float*>(work) + (uint64_t)r0 * d->N : nullptr;
        A.carry = heun ? static_cast<float*>(work) + NR + (uint64_t)r0 * d->N : nullptr;
        A.r_samples = r_samples ? r_samples + (uint64_t)r0 * n_samples : nullptr;
        A.slots = static_cast<uint64_t*>(slots);
        A.flag = ctx->flag;
        A.N = d->N;
        A.R = nr;
        A.G = G;
        A.M = M;
        A.r_base = r0;
        A.chunk = chunk;
        A.step0 = run->step0;
        A.n_steps = d->n_steps;
        A.n_samples = n_samples;
        A.key0 = (uint32_t)run->seed;
        A.key1 = (uint32_t)(run->seed >> 32);
        A.omega_scale = kc.omega_scale;
        A.hdt2pi = kc.hdt2pi;
        A.kn = kc.kn;
        A.c2 = kc.c2;
        A.spin_limit = 1u << 26;
        void* args[] = {&A};
        SDE_HIP(ctx, hipLaunchCooperativeKernel(kern, dim3(nr * G), dim3(kMFSThreads), args, 0, stream));
    }
    ctx->last.mf_streamed = 1;
    return SDE_OK;
}

static int ilog2_u64(uint64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

// The register-resident kernel at `opt` oscillators per lane: workgroups per
// realization (up to 16 flat; beyond that the two-level exchange over 8
// groups, G a multiple of 8, the workgroups past the last oscillator
// contributing zero sums), entry point, co-resident workgroups, and whether
// a realization fits (at most one polling lane per exchange word).
// The two-realization kernel (paired): the same lanes per realization and
// slice, realizations taken two at a time (R even), a flat exchange of at
// most 32 workgroups, OPT 2 or 4 (the registers of two realizations).
constexpr int kMFShapes = 6;

struct MFShape {
    int opt = 0;
    bool paired = false;
    uint32_t G = 0;
    void* kern = nullptr;
    uint32_t threads = 0;
    uint64_t capacity = 0;
    bool fits = false;
};

static int mf_shape(sde_ctx* ctx, uint32_t N, uint32_t R, int opt, bool paired, bool heun, MFShape* out)
{
    uint64_t G64 = ((uint64_t)N + (uint64_t)kMFThreads * opt - 1) / ((uint64_t)kMFThreads * opt);
    if (!paired && G64 > 16) G64 = (G64 + 7) / 8 * 8;
    if (paired) {
        switch (opt) {
        case 2: out->kern = heun ? mfp_kernel_ptr<2, SDE_HEUN>() : mfp_kernel_ptr<2, SDE_EULER>(); break;
        default: out->kern = heun ? mfp_kernel_ptr<4, SDE_HEUN>() : mfp_kernel_ptr<4, SDE_EULER>(); break;
        }
        out->threads = kMFPThreads;
    } else {
        switch (opt) {
        case 1: out->kern = heun ? mf_kernel_ptr<1, SDE_HEUN>() : mf_kernel_ptr<1, SDE_EULER>(); break;
        case 2: out->kern = heun ? mf_kernel_ptr<2, SDE_HEUN>() : mf_kernel_ptr<2, SDE_EULER>(); break;
        case 4: out->kern = heun ? mf_kernel_ptr<4, SDE_HEUN>() : mf_kernel_ptr<4, SDE_EULER>(); break;
        default: out->kern = heun ? mf_kernel_ptr<8, SDE_HEUN>() : mf_kernel_ptr<8, SDE_EULER>(); break;
        }
        out->threads = kMFThreads;
    }
    int per_cu = 0;
    SDE_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, out->kern, (int)out->threads, 0));
    out->opt = opt;
    out->paired = paired;
    out->capacity = (uint64_t)std::max(per_cu, 0) * ctx->n_cu;
    out->fits = paired ? (R % 2 == 0 && (opt == 2 || opt == 4) && G64 <= kMaxMFPGroups && out->capacity >= G64)
                       : (G64 <= kMaxMFGroups && out->capacity >= G64);
    out->G = (uint32_t)G64;
    return SDE_OK;
}

// Realizations per cooperative launch: as many as fit co-resident (pairs
// for the paired kernel).
static uint32_t mf_r_per_launch(const MFShape& sh, uint32_t R)
{
    const uint64_t units = sh.capacity / sh.G;
    return (uint32_t)std::min<uint64_t>(R, sh.paired ? 2 * units : units);
}

// Exchange words one call at this shape needs (both parities, both levels).
static size_t mf_slot_words(const MFShape& sh, uint32_t R, size_t* slot_words)
{
    const uint32_t r_per_launch = mf_r_per_launch(sh, R);
    *slot_words = (size_t)2 * r_per_launch * sh.G * kMFWordsPerGroup;
    return *slot_words + (size_t)2 * r_per_launch * 8 * kMFWordsPerGroup;
}

// All realizations of one call at shape `sh`, as many per cooperative
// launch as fit co-resident; `slots` holds mf_slot_words words.
static int mf_launch(sde_ctx* ctx, const MFShape& sh, const sde_kuramoto_desc* d, const KuraConsts& kc,
                     uint64_t seed, uint64_t step0, uint64_t n_steps, bool init_from_state, float* phi,
                     const float* omega, double* r_samples, uint64_t n_samples, uint32_t M, int* flag,
                     uint64_t* slots, hipStream_t stream)
{
    const uint32_t G = sh.G;
    const uint32_t r_per_launch = mf_r_per_launch(sh, d->R);
    size_t slot_words = 0;
    const size_t n32 = 2 * mf_slot_words(sh, d->R, &slot_words);
    for (uint32_t r0 = 0; r0 < d->R; r0 += r_per_launch) {
        const uint32_t nr = std::min(r_per_launch, d->R - r0);
        // tags start at 1: zeroed slots never match
        hipLaunchKernelGGL(mf_zero_kernel, dim3((uint32_t)((n32 + 255) / 256)), dim3(256), 0, stream,
                           reinterpret_cast<uint32_t*>(slots), n32);
        SDE_HIP(ctx, hipGetLastError());
        MFArgs A;
        A.slots2 = slots + slot_words;
        A.tree = G > 16 ? 1u : 0u;
        A.theta = phi + (uint64_t)r0 * d->N;
        A.omega = omega;
        A.r_samples = r_samples ? r_samples + (uint64_t)r0 * n_samples : nullptr;
        A.slots = slots;
        A.flag = flag;
        A.N = d->N;
        A.R = nr;
        A.G = G;
        A.M = M;
        A.step0 = step0;
        A.n_steps = n_steps;
        A.n_samples = n_samples;
        A.key0 = (uint32_t)seed;
        A.key1 = (uint32_t)(seed >> 32);
        A.omega_scale = kc.omega_scale;
        A.hdt2pi = kc.hdt2pi;
        A.kn = kc.kn;
        A.c2 = kc.c2;
        A.init_from_state = init_from_state;
        const uint32_t units = sh.paired ? nr / 2 : nr;  // realizations, or pairs of them
        A.xcd_map = (ctx->xcds == 8 && units % 8 == 0) ? 1 : 0;
        A.xcd_local = ctx->kura_xcd_local;
        A.spin_limit = 1u << 26;
        A.r_base = r0;
        void* args[] = {&A};
        SDE_HIP(ctx, hipLaunchCooperativeKernel(sh.kern, dim3(units * G), dim3(sh.threads), args, 0, stream));
    }
    return SDE_OK;
}

// Times every candidate shape on a 64-step run of the call's N and R (fresh
// phases from Philox into a scratch state, no samples, the NaN flag of the
// trials) and returns the index of the fastest; the default shape is kept
// unless another is more than 3 % faster, so that timing noise does not
// move the choice.
static int mf_tune(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, const KuraConsts& kc,
                   const float* omega, const MFShape* shapes, int n_shapes, int def, uint64_t* slots,
                   hipStream_t stream, int* best)
{
    void* scratch = nullptr;
    int st = ensure_ws(ctx, kSlotTune, (size_t)d->N * d->R * sizeof(float), &scratch);
    if (st) return st;
    hipEvent_t e0, e1;
    SDE_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SDE_ERR_DEVICE, "mean-field autotuner: hipEventCreate failed");
    }
    float ms[kMFShapes] = {};
    for (int c = 0; c < n_shapes && st == SDE_OK; ++c) {
        for (int rep = 0; rep < 2 && st == SDE_OK; ++rep) {  // the first launch loads the code object
            if (hipEventRecord(e0, stream) != hipSuccess) st = SDE_ERR_DEVICE;
            if (!st)
                st = mf_launch(ctx, shapes[c], d, kc, run->seed, 0, 64, false, static_cast<float*>(scratch), omega,
                               nullptr, 0, 100, ctx->tune_flag, slots, stream);
            if (!st && hipEventRecord(e1, stream) != hipSuccess) st = SDE_ERR_DEVICE;
            if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms[c], e0, e1) != hipSuccess))
                st = SDE_ERR_DEVICE;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == SDE_ERR_DEVICE) return fail(ctx, st, "mean-field autotuner: HIP event or launch failed");
    if (st) return st;
    int b = def;
    for (int c = 0; c < n_shapes; ++c)
        if (ms[c] < 0.97f * ms[b]) b = c;
    *best = b;
    return SDE_OK;
}

static int mf_code(const MFShape& s) { return s.opt | (s.paired ? 16 : 0); }

static int run_meanfield(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                         const float* omega, double* r_samples, uint64_t n_samples, uint32_t M,
                         hipStream_t stream)
{
    const KuraConsts kc = kuramoto_consts(d);
    const bool heun = run->scheme == SDE_HEUN;
    // The candidates: one realization per workgroup at 1, 2, 4, 8 oscillators
    // per lane (8 is the most the kernel holds in registers with its noise
    // block, its prefetched next block and the sines and cosines kept for the
    // drift), and two per workgroup at 2 or 4.  The default is the smallest
    // one-realization count that needs at most 16 workgroups per
    // realization, else the largest that fits.  The options restrict the set.
    MFShape all[kMFShapes];
    static const int kOpt[kMFShapes] = {1, 2, 4, 8, 2, 4};
    int n_fit = 0, def = -1;
    MFShape fit[kMFShapes];
    for (int c = 0; c < kMFShapes; ++c) {
        const bool paired = c >= 4;
        int st = mf_shape(ctx, d->N, d->R, kOpt[c], paired, heun, &all[c]);
        if (st) return st;
        if (!all[c].fits) continue;
        if (ctx->kura_mf_opt && kOpt[c] != ctx->kura_mf_opt) continue;
        if ((ctx->kura_mf_paired == 1 && paired) || (ctx->kura_mf_paired == 2 && !paired)) continue;
        if (def < 0 && !paired && all[c].G <= 16) def = n_fit;
        fit[n_fit++] = all[c];
    }
    if (def < 0) {
        for (int c = 0; c < n_fit; ++c)
            if (!fit[c].paired) def = c;
        if (def < 0) def = 0;
    }
    const bool forced = ctx->kura_mf_opt != 0 || ctx->kura_mf_paired != 0;
    const bool any_fit = all[0].fits || all[1].fits || all[2].fits || all[3].fits;
    if (ctx->kura_mf == 1 || (ctx->kura_mf == 0 && !any_fit))
        return run_meanfield_streamed(ctx, d, run, phi, omega, r_samples, n_samples, M, stream);
    if (!any_fit)
        return fail(ctx, SDE_ERR_UNSUPPORTED, "mean-field kernel: N = %u needs %u co-resident workgroups of %d "
                    "lanes x 8 oscillators, the device holds %llu (at most %u per realization)", d->N, all[3].G,
                    kMFThreads, (unsigned long long)all[3].capacity, kMaxMFGroups);
    if (n_fit == 0)
        return fail(ctx, SDE_ERR_UNSUPPORTED, "mean-field kernel: N = %u, R = %u does not fit the forced shape (%d "
                    "oscillators per lane, paired option %d)", d->N, d->R, ctx->kura_mf_opt, ctx->kura_mf_paired);
    // exchange words for any of the candidates
    size_t words = 0, unused = 0;
    for (int c = 0; c < n_fit; ++c) words = std::max(words, mf_slot_words(fit[c], d->R, &unused));
    void* slots = nullptr;
    int st = ensure_ws(ctx, kSlotKuraPartials, words * sizeof(uint64_t), &slots);
    if (st) return st;
    // the shape: forced (the default of the restricted set), cached, or tuned
    // on this call's shape class
    int chosen = def;
    if (!forced) {
        char key[160];
        snprintf(key, sizeof key, "meanfield|%s|N2^%d|R2^%d|%s|xcd%d", ctx->arch.c_str(), ilog2_u64(d->N),
                 ilog2_u64(d->R), heun ? "heun" : "euler", ctx->kura_xcd_local);
        int code = 0;
        if (tune_lookup(ctx, key, &code)) {
            for (int c = 0; c < n_fit; ++c)
                if (mf_code(fit[c]) == code) chosen = c;  // else made for another N or R of the class: the default
        } else if (ctx->autotune && n_fit > 1) {
            const auto t0 = std::chrono::steady_clock::now();
            if ((st = mf_tune(ctx, d, run, kc, omega, fit, n_fit, def, static_cast<uint64_t*>(slots), stream,
                              &chosen)))
                return st;
            ctx->last.tuned = 1;
            ctx->last.tune_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            tune_store(ctx, key, mf_code(fit[chosen]));
        }
    }
    ctx->last.kura_mf_opt = fit[chosen].opt;
    ctx->last.kura_mf_paired = fit[chosen].paired ? 1 : 0;
    return mf_launch(ctx, fit[chosen], d, kc, run->seed, run->step0, d->n_steps, run->init == SDE_INIT_FROM_STATE,
                     phi, omega, r_samples, n_samples, M, ctx->flag, static_cast<uint64_t*>(slots), stream);
}

// One stage: the whole j range per workgroup (J = 1), or J slices of jlen
// into `part` and the combining update.
template <int OPT>
static int launch_tiled(sde_ctx* ctx, const TiledArgs& A, uint32_t J, uint32_t jlen, float* part, hipStream_t stream)
{
    constexpr uint32_t TILE = kTileThreads * OPT;
    if (J <= 1) {
        dim3 grid((A.N + TILE - 1) / TILE, A.R);
        hipLaunchKernelGGL(kuramoto_tiled_kernel<OPT>, grid, dim3(kTileThreads), 0, stream, A);
    } else {
        dim3 grid((A.N + TILE - 1) / TILE, A.R, J);
        hipLaunchKernelGGL(kuramoto_tiled_part_kernel<OPT>, grid, dim3(kTileThreads), 0, stream, A, part, jlen);
        const uint64_t NR = (uint64_t)A.N * A.R;
        hipLaunchKernelGGL(kuramoto_tiled_combine_kernel, dim3((uint32_t)((NR + 255) / 256)), dim3(256), 0, stream, A,
                           static_cast<const float*>(part), J);
    }
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

// j slices of the all-pairs sum: forced by the context option, else enough
// to give about 4 workgroups per CU when the plain launch has fewer than 2;
// every slice holds at least 64 j.
static void tiled_split(const sde_ctx* ctx, uint32_t N, uint32_t R, uint32_t tile, uint32_t* J, uint32_t* jlen)
{
    const uint64_t wgs = (((uint64_t)N + tile - 1) / tile) * R;
    uint64_t j = 1;
    if (ctx->kura_jsplit > 0)
        j = (uint64_t)ctx->kura_jsplit;
    else if (wgs < 2 * (uint64_t)ctx->n_cu)
        j = (4 * (uint64_t)ctx->n_cu + wgs - 1) / wgs;
    j = std::min<uint64_t>({j, std::max<uint64_t>(1, N / 64), 65535});
    const uint64_t len = ((uint64_t)N + j - 1) / j;
    *jlen = (uint32_t)len;
    *J = (uint32_t)(((uint64_t)N + len - 1) / len);
}

static int launch_tiled_opt(sde_ctx* ctx, int opt, const TiledArgs& A, uint32_t J, uint32_t jlen, float* part,
                            hipStream_t s)
{
    return opt == 4 ? launch_tiled<4>(ctx, A, J, jlen, part, s)
                    : opt == 2 ? launch_tiled<2>(ctx, A, J, jlen, part, s) : launch_tiled<1>(ctx, A, J, jlen, part, s);
}

// Oscillators per lane of the all-pairs kernel (its tile: 256 x OPT phases
// in LDS): times one stage of each candidate 1, 2, 4 (with its j split) on
// copies of the state in the tuning workspace -- the caller's arrays are only
// read -- and returns the fastest.
static int tiled_tune(sde_ctx* ctx, const sde_kuramoto_desc* d, const TiledArgs& base, const float* phi,
                      hipStream_t stream, int* best_opt)
{
    const uint64_t NR = (uint64_t)d->N * d->R;
    uint32_t Jmax = 1;
    for (int opt : {1, 2, 4}) {
        uint32_t J, jlen;
        tiled_split(ctx, d->N, d->R, kTileThreads * opt, &J, &jlen);
        Jmax = std::max(Jmax, J);
    }
    void* ws = nullptr;
    int st = ensure_ws(ctx, kSlotTune, (size_t)(3 + (Jmax > 1 ? Jmax : 0)) * NR * sizeof(float), &ws);
    if (st) return st;
    float* src = static_cast<float*>(ws);
    float* dst = src + NR;
    float* F1 = dst + NR;
    float* part = F1 + NR;
    SDE_HIP(ctx, hipMemcpyAsync(src, phi, NR * sizeof(float), hipMemcpyDeviceToDevice, stream));
    TiledArgs A = base;
    A.src = src;
    A.base = src;
    A.dst = dst;
    A.F1 = F1;
    A.k = 0;
    A.stage = 1;
    A.euler = 0;
    hipEvent_t e0, e1;
    SDE_HIP(ctx, hipEventCreate(&e0));
    SDE_HIP(ctx, hipEventCreate(&e1));
    double best = 1e300;
    for (int opt : {1, 2, 4}) {
        uint32_t J, jlen;
        tiled_split(ctx, d->N, d->R, kTileThreads * opt, &J, &jlen);
        float ms = 0.f;
        for (int rep = 0; rep < 2 && st == SDE_OK; ++rep) {  // the first launch loads the code object
            if (hipEventRecord(e0, stream) != hipSuccess) st = SDE_ERR_DEVICE;
            if (!st) st = launch_tiled_opt(ctx, opt, A, J, jlen, part, stream);
            if (!st && hipEventRecord(e1, stream) != hipSuccess) st = SDE_ERR_DEVICE;
            if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = SDE_ERR_DEVICE;
        }
        if (st) break;
        if (ms < best) {
            best = ms;
            *best_opt = opt;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == SDE_ERR_DEVICE) return fail(ctx, st, "all-pairs autotuner: HIP event or launch failed");
    return st;
}

static int run_tiled(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                     const float* omega, double* r_samples, uint64_t n_samples, uint32_t M,
                     hipStream_t stream)
{
    const KuraConsts kc = kuramoto_consts(d);
    const uint64_t NR = (uint64_t)d->N * d->R;
    uint64_t* nbase = nullptr;
    int st = step_counter(ctx, &nbase);
    if (st) return st;
    TiledArgs A;
    A.omega = omega;
    A.nbase = nbase;
    A.N = d->N;
    A.R = d->R;
    A.key0 = (uint32_t)run->seed;
    A.key1 = (uint32_t)(run->seed >> 32);
    A.omega_scale = kc.omega_scale;
    A.hdt2pi = kc.hdt2pi;
    A.kn = kc.kn;
    A.c2 = kc.c2;
    // oscillators per lane: forced, cached, or tuned on this call's shape class
    int opt = ctx->kura_tile;
    if (!opt) {
        char key[160];
        snprintf(key, sizeof key, "tiled|%s|N2^%d|R2^%d|J%d", ctx->arch.c_str(), ilog2_u64(d->N), ilog2_u64(d->R),
                 ctx->kura_jsplit);
        if (!tune_lookup(ctx, key, &opt)) {
            opt = d->N >= 4096 ? 4 : 1;
            if (ctx->autotune) {
                const auto t0 = std::chrono::steady_clock::now();
                launch_step_set(nbase, run->step0, stream);
                if ((st = tiled_tune(ctx, d, A, phi, stream, &opt))) return st;
                ctx->last.tuned = 1;
                ctx->last.tune_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                tune_store(ctx, key, opt);
            }
        }
    }
    uint32_t J = 1, jlen = d->N;
    tiled_split(ctx, d->N, d->R, kTileThreads * opt, &J, &jlen);
    void* work = nullptr;
    if ((st = ensure_ws(ctx, kSlotKuraWork, (size_t)(2 + (J > 1 ? J : 0)) * NR * sizeof(float), &work))) return st;
    float* tilde = static_cast<float*>(work);
    float* F1 = tilde + NR;
    float* part = F1 + NR;
    ctx->last.kura_jsplit = (int32_t)J;
    ctx->last.kura_tile = opt;
    A.F1 = F1;
    A.euler = run->scheme == SDE_EULER;
    // `count` steps from the device step base, then advance it
    auto record = [&](hipStream_t s, uint32_t count) -> int {
        if (r_samples) launch_order_parameter_at(phi, d->N, d->R, r_samples, n_samples, nbase, run->step0, M, s);
        for (uint32_t k = 0; k < count; ++k) {
            A.k = k;
            A.stage = 1;
            A.src = phi;
            A.base = phi;
            A.dst = tilde;  // every lane reads all of src, so no step writes in place
            int e = launch_tiled_opt(ctx, opt, A, J, jlen, part, s);
            if (e) return e;
            if (A.euler) {
                hipLaunchKernelGGL(copy_f32_kernel, dim3((uint32_t)((NR + 255) / 256)), dim3(256), 0, s, phi, tilde, NR);
                continue;
            }
            A.stage = 2;
            A.src = tilde;
            A.base = phi;
            A.dst = phi;
            e = launch_tiled_opt(ctx, opt, A, J, jlen, part, s);
            if (e) return e;
        }
        launch_step_advance(nbase, count, s);
        SDE_HIP(ctx, hipGetLastError());
        return SDE_OK;
    };
    launch_step_set(nbase, run->step0, stream);
    const uint32_t C = chunk_steps(M, d->n_steps, false);
    char key[256];
    snprintf(key, sizeof key, "tiled|%p|%p|%p|%p|%u|%u|%u|%u|%a|%a|%a|%a|%d|%llu|%u|%llu|J%u/%u|opt%d", (void*)phi,
             (void*)omega, (void*)r_samples, (void*)work, d->N, d->R, A.key0, A.key1, A.omega_scale, A.hdt2pi, A.kn,
             A.c2, A.euler, (unsigned long long)run->step0, M, (unsigned long long)n_samples, J, jlen, opt);
    const uint64_t full = d->n_steps / C, rem = d->n_steps % C;
    for (uint64_t c = 0; c < full; ++c)
        if ((st = run_recorded(ctx, std::string(key) + "|C" + std::to_string(C), stream,
                               [&](hipStream_t s) { return record(s, C); })))
            return st;
    if (rem && (st = run_recorded(ctx, std::string(key) + "|C" + std::to_string(rem), stream,
                                  [&](hipStream_t s) { return record(s, (uint32_t)rem); })))
        return st;
    if (r_samples) launch_order_parameter_at(phi, d->N, d->R, r_samples, n_samples, nbase, run->step0, M, stream);
    SDE_HIP(ctx, hipGetLastError());
    return SDE_OK;
}

int kuramoto_impl(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi, const float* omega,
                  const float* K, double* r_samples, hipStream_t stream)
{
    ctx->last = sde_stats{};
    int st = validate(ctx, d, run, phi, omega, K, r_samples);
    if (st) return st;
    const uint32_t M = run->sample_every ? run->sample_every : 100u;
    const uint64_t n_samples = d->n_steps / M + 1;
    if (run->init == SDE_INIT_PHILOX && d->coupling != SDE_MEANFIELD) {
        const uint64_t NR = (uint64_t)d->N * d->R;
        hipLaunchKernelGGL(kuramoto_init_kernel, dim3((uint32_t)((NR + 255) / 256)), dim3(256), 0, stream, phi,
                           d->N, d->R, (uint32_t)run->seed, (uint32_t)(run->seed >> 32));
        SDE_HIP(ctx, hipGetLastError());
    }
    switch (d->coupling) {
    case SDE_MEANFIELD: st = run_meanfield(ctx, d, run, phi, omega, r_samples, n_samples, M, stream); break;
    case SDE_TILED: st = run_tiled(ctx, d, run, phi, omega, r_samples, n_samples, M, stream); break;
    default: st = dense_impl(ctx, d, run, phi, omega, K, r_samples, n_samples, M, stream); break;
    }
    if (st) return st;
    if (run->sync) return sync_and_check(ctx, stream);
    return SDE_OK;
}

}  // namespace sde
