// Internal helpers shared by the library's HIP translation units (gfx950,
// wave64).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pms.h"

namespace pms {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------- context
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Kernels timed by the optional profiler (pms_profile_*): HIP events are
// recorded on the context's stream around each launch of these kernels.
enum KernelId {
    K_INIT = 0, K_BETA, K_LOW, K_COLLIDE, K_SCAN, K_PIVOTS, K_XOR, K_COMPACT, K_FINAL, K_FILL, K_DEFRAG,
    K_LS_KEYS, K_SORT, K_LS_INDEX, K_BUILD_SCAN, K_LS_ROWS, K_VR_EDGES, K_VR_TRI, K_VR_INDEX, K_VR_ROWS,
    K_BACKWARD, K_CHAIN, K_CHAIN_LANE, K_CHAIN_WIDE, K_C8, K_BUDGET, K_SOLVE, K_LS_LEFT,
    K_NUM
};

struct PendingEv {
    int kid;
    hipEvent_t e0, e1;
    double bytes;   // algorithmic bytes of this launch (< 0: filled in later)
    double abytes;  // addition kernels: 4 (len t + len s + len t+s) over its additions (filled in later)
};

// Entries of the first lane chaining pass's per-lane LDS buffer: 39 x 128
// lanes x 4 bytes lets 8 two-wave blocks share a CU's 160 KB, the 4 waves per
// SIMD its registers allow.
constexpr int kLaneCap = 39;

// The chaining kernels' built-in shapes (measured on the 64^3 lower-star
// and the batched Vietoris-Rips workloads).
inline pms_tuning default_tuning()
{
    pms_tuning t;
    t.lane_blocks = 2048;  // 8 per CU
    t.chain_blocks = 512;  // 2 per CU
    t.lane_steps = 128;
    t.lane_steps_few = 0;
    t.lane_many = 65536;
    t.lane_refill = 32;
    t.lane_flush = 16;
    t.wide_blocks = 2048;
    t.lane_cap = kLaneCap;
    t.solve = 512;  // rounds that hand on a few long chains (the 64^3 lower-star's later rounds)
    return t;
}

inline bool tuning_valid(const pms_tuning &t)
{
    return t.lane_blocks >= 1 && t.lane_blocks <= 65535 && t.chain_blocks >= 1 && t.chain_blocks <= 65535 &&
           t.lane_steps >= 0 && t.lane_steps <= (1 << 30) && t.lane_steps_few >= 0 &&
           t.lane_steps_few <= (1 << 30) && t.lane_many >= 0 && t.lane_refill >= 1 && t.lane_refill <= 64 &&
           t.lane_flush >= 1 && t.lane_flush <= 64 && t.wide_blocks >= 1 && t.wide_blocks <= 65535 &&
           t.lane_cap >= 0 && t.lane_cap <= kLaneCap && t.solve >= 0 && t.solve <= (1 << 30);
}

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // the batch instances of the reduction in progress (device column
    // offsets, n_inst + 1 entries; null: one complex)
    const int64_t *inst_off = nullptr;
    int32_t n_inst = 1;
    // profiler
    bool prof_on = false;
    std::vector<PendingEv> pend;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[K_NUM] = {};
    double prof_bytes[K_NUM] = {};
    double prof_abytes[K_NUM] = {};
    int64_t prof_launches[K_NUM] = {};
    // named scratch buffers, grown on demand
    Buf b[56];
    int32_t *arena = nullptr;
    uint64_t arena_cap = 0;  // entries
    void *host_pinned = nullptr;
    // graph-mode rounds: captured and replayed on a stream of the context
    // (the caller's may be the legacy default stream, which cannot capture)
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_ev = nullptr;
    // pipelined rounds: one event per pinned counter buffer
    hipEvent_t pipe_ev[2] = {nullptr, nullptr};
    // the last captured round graph, reused while its key (the device
    // arguments and options it was captured with) is unchanged
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;
    // launch shapes and thresholds of the chaining kernels
    pms_tuning tune = default_tuning();
    // the last reduction's diagnostics (pms_options.diagnostics): one entry
    // per recorded round, and the size of the problem its estimate covers
    std::vector<pms_round_stats> diag;
    int64_t diag_m = -1;
};

enum BufId {
    B_OFF = 0, B_LEN, B_LOW, B_STATE, B_BETA, B_LEFT, B_PIV, B_T, B_NEG, B_ACT0, B_ACT1,
    B_COLL, B_AGG, B_AGG2, B_CNT, B_FLAGS, B_TMP0, B_TMP1,
    B_BUILD0, B_BUILD1, B_BUILD2, B_BUILD3, B_BUILD4, B_BUILD5, B_BUILD6, B_BUILD7,
    B_BUILD8, B_BUILD9, B_BUILD10, B_BUILD11, B_BUILD12, B_BUILD13, B_BUILD14, B_STATS, B_PART, B_CQN, B_PREC, B_WQ, B_WQ2, B_ESS,
    B_DBG_LOW, B_DBG_OFF, B_DBG_LEN, B_DBG_STATE, B_DBG_W, B_DBG_EREM, B_C8, B_INST, B_BUDH, B_BUDN,
    B_NUM
};
static_assert(B_NUM <= 56, "Ctx::b holds 56 buffers");

// Grow-only scratch: returns the buffer, reallocating (contents dropped) when
// it is smaller than `bytes`.
void *grow_scratch(Ctx *c, int id, size_t bytes);

pms_status set_err(Ctx *c, pms_status s, const std::string &msg);

hipEvent_t prof_event(Ctx *c);
// Fold finished launches into the per-kernel totals (call after a sync).
void prof_flush(Ctx *c);

// Launch `kernel` on the context's stream; with the profiler on, bracket it
// with events and remember its algorithmic bytes.
#define PMS_LAUNCH(c, kid, bytes, kernel, grid, block, ...)                                    \
    do {                                                                                        \
        hipEvent_t e0_ = nullptr;                                                               \
        if ((c)->prof_on) {                                                                     \
            e0_ = ::pms::prof_event(c);                                                         \
            (void)hipEventRecord(e0_, (c)->stream);                                             \
        }                                                                                       \
        kernel<<<(grid), (block), 0, (c)->stream>>>(__VA_ARGS__);                               \
        if ((c)->prof_on) {                                                                     \
            hipEvent_t e1_ = ::pms::prof_event(c);                                              \
            (void)hipEventRecord(e1_, (c)->stream);                                             \
            (c)->pend.push_back({(kid), e0_, e1_, (double)(bytes), 0.0});                       \
        }                                                                                       \
    } while (0)

#define PMS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::pms::set_err(c, e_ == hipErrorOutOfMemory ? PMS_ERR_OOM : PMS_ERR_HIP, \
                                  std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

inline unsigned grid_for(int64_t n, int per_block = kBlock, unsigned cap = 1u << 20)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------- device
struct I4 {
    int32_t v[4];
};

__device__ inline I4 i4_max(const I4 &a, const I4 &b)
{
    I4 r;
#pragma unroll
    for (int k = 0; k < 4; k++) r.v[k] = a.v[k] > b.v[k] ? a.v[k] : b.v[k];
    return r;
}

__device__ inline I4 i4_fill(int32_t x)
{
    I4 r;
#pragma unroll
    for (int k = 0; k < 4; k++) r.v[k] = x;
    return r;
}

// Wave64 reductions on DPP row operations (no LDS crossbar): within each
// row of 16 lanes, quad_perm [1,0,3,2] and [2,3,0,1] then row_ror 4 and 8
// leave the row total in every lane; row_bcast 15 / 31 then carry rows 0..2
// into row 3, whose lane 63 ends with the wave total.
template <int CTRL, int ROW_MASK>
__device__ inline int32_t dpp_i32(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

__device__ inline int32_t wave_sum_dpp(int32_t v)
{
    v += dpp_i32<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_i32<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_i32<0x124, 0xF>(v);  // row_ror 4
    v += dpp_i32<0x128, 0xF>(v);  // row_ror 8
    v += dpp_i32<0x142, 0xA>(v);  // row_bcast 15 -> rows 1, 3
    v += dpp_i32<0x143, 0xC>(v);  // row_bcast 31 -> rows 2, 3
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

// Max over the wave of non-negative values (rows left out of a bcast get 0
// from update_dpp's "old" operand, which must not exceed any input).
__device__ inline int32_t wave_max_dpp(int32_t v)
{
    v = max(v, dpp_i32<0xB1, 0xF>(v));
    v = max(v, dpp_i32<0x4E, 0xF>(v));
    v = max(v, dpp_i32<0x124, 0xF>(v));
    v = max(v, dpp_i32<0x128, 0xF>(v));
    v = max(v, dpp_i32<0x142, 0xA>(v));
    v = max(v, dpp_i32<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

// Broadcasts whose result the compiler knows to be wave-uniform (scalar
// registers), unlike __shfl: control flow that depends on them stays scalar.
// Workgroups are dispatched to the 8 XCDs, each with its own L2, in
// round-robin order of their index.  xcd_split gives the workgroups of XCD x
// the x-th eighth of the units [0, n), walked from `first` in steps of `step`
// up to `end`: neighbouring columns then share an XCD and its cached lines
// (a grid of fewer than 8 blocks splits into as many parts as blocks).
constexpr unsigned kXcds = 8;
struct XcdSplit {
    int64_t first, end, step;
};
__device__ inline XcdSplit xcd_split(int64_t n)
{
    const unsigned g = gridDim.x;
    const unsigned nx = g < kXcds ? g : kXcds;
    const unsigned x = blockIdx.x % nx;
    XcdSplit s;
    s.first = n * x / nx + blockIdx.x / nx;
    s.end = n * (x + 1) / nx;
    s.step = (g - x + nx - 1) / nx;  // the blocks on part x
    return s;
}

__device__ inline int32_t bcast_first(int32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ inline long long bcast_first64(long long x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ inline int32_t bcast_lane(int32_t x, int32_t l)
{
    return __builtin_amdgcn_readlane(x, l);
}

// Inclusive wave scans (wave64, __shfl_up).
__device__ inline int64_t wave_incl_sum64(int64_t x)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline int32_t wave_incl_sum32(int32_t x)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline I4 wave_incl_max4(I4 x)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        I4 y;
#pragma unroll
        for (int k = 0; k < 4; k++) y.v[k] = __shfl_up(x.v[k], d, kWave);
        if (lane >= d) x = i4_max(x, y);
    }
    return x;
}

// Block-wide exclusive sum over kThreads threads; *total receives the sum.
// Must be reached by every thread of the block.
template <int kThreads = kBlock>
__device__ inline int32_t block_excl_sum32(int32_t v, int32_t *total)
{
    constexpr int kW = kThreads / kWave;
    __shared__ int32_t s_w[kW];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int32_t inc = wave_incl_sum32(v);
    if (lane == kWave - 1) s_w[wid] = inc;
    __syncthreads();
    int32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kW; w++) {
        int32_t t = s_w[w];
        if (w < wid) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__device__ inline int64_t block_excl_sum64(int64_t v)
{
    __shared__ int64_t s_e64[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int64_t inc = wave_incl_sum64(v);
    if (lane == kWave - 1) s_e64[wid] = inc;
    __syncthreads();
    int64_t pre = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; w++)
        if (w < wid) pre += s_e64[w];
    __syncthreads();
    return pre + inc - v;
}

template <int kThreads = kBlock>
__device__ inline int64_t block_sum64(int64_t v)
{
    constexpr int kW = kThreads / kWave;
    __shared__ int64_t s_w64[kW];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int64_t inc = wave_incl_sum64(v);
    if (lane == kWave - 1) s_w64[wid] = inc;
    __syncthreads();
    int64_t tot = 0;
#pragma unroll
    for (int w = 0; w < kW; w++) tot += s_w64[w];
    __syncthreads();
    return tot;
}

// One-block exclusive scan of n values in place (1024 threads): per pass
// each thread takes kSeg consecutive values (loaded together: the index is
// clamped rather than branched on, so one wait covers them), the block scans
// the threads' sums, and each thread writes its values back.  kSeg holds 64
// bytes per thread (16 int32, 8 int64, 4 I4): more would not fit the 128
// VGPRs a 1024-thread block leaves each lane.  A pass covers 16 K int32 with
// two barriers, where a 1024-value chunk loop needs three barriers and one
// dependent load per chunk.  Returns the total.
__device__ inline int32_t shfl_up_t(int32_t x, int dd) { return __shfl_up(x, dd, kWave); }
__device__ inline int64_t shfl_up_t(int64_t x, int dd) { return __shfl_up(x, dd, kWave); }
__device__ inline I4 shfl_up_t(I4 x, int dd)
{
    I4 y;
#pragma unroll
    for (int k = 0; k < 4; k++) y.v[k] = __shfl_up(x.v[k], dd, kWave);
    return y;
}
template <typename T, typename Op>
__device__ inline T block_seg_scan(T *a, int64_t n, T ident, Op op)
{
    constexpr int kThr = 1024, kSeg = (int)(64 / sizeof(T));
    __shared__ T s_part[kThr / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    T carry = ident;
    for (int64_t base = 0; base < n; base += (int64_t)kThr * kSeg) {
        const int64_t s0 = base + (int64_t)tid * kSeg;
        T v[kSeg];
#pragma unroll
        for (int u = 0; u < kSeg; u++) v[u] = a[min(s0 + u, n - 1)];
        T loc = ident;
#pragma unroll
        for (int u = 0; u < kSeg; u++) {
            if (s0 + u >= n) v[u] = ident;
            loc = op(loc, v[u]);
        }
        T inc = loc;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
            const T y = shfl_up_t(inc, dd);
            if (lane >= dd) inc = op(inc, y);
        }
        if (lane == kWave - 1) s_part[wid] = inc;
        __syncthreads();
        T pre = carry, tot = carry;
        for (int w = 0; w < kThr / kWave; w++) {
            const T x = s_part[w];
            if (w < wid) pre = op(pre, x);
            tot = op(tot, x);
        }
        const T below = shfl_up_t(inc, 1);
        T ex = lane ? op(pre, below) : pre;
#pragma unroll
        for (int u = 0; u < kSeg; u++) {
            if (s0 + u < n) a[s0 + u] = ex;
            ex = op(ex, v[u]);
        }
        carry = tot;
        __syncthreads();  // s_part is reused by the next pass
    }
    return carry;
}

// Block-wide exclusive max-scan of I4 (identity -1); *total = block max.
__device__ inline I4 block_excl_max4(I4 v, I4 *total)
{
    __shared__ I4 s_w4[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    I4 inc = wave_incl_max4(v);
    // exclusive within the wave: shift by one lane
    I4 exc;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int32_t y = __shfl_up(inc.v[k], 1, kWave);
        exc.v[k] = lane == 0 ? -1 : y;
    }
    if (lane == kWave - 1) s_w4[wid] = inc;
    __syncthreads();
    I4 pre = i4_fill(-1), tot = i4_fill(-1);
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; w++) {
        I4 t = s_w4[w];
        if (w < wid) pre = i4_max(pre, t);
        tot = i4_max(tot, t);
    }
    __syncthreads();
    *total = tot;
    return i4_max(pre, exc);
}

}  // namespace pms
