// Stable LSD radix sort on the device (the builders' order keys).
//
// Keys are unsigned integers sorted by their bits [0, end_bit), 8 bits per
// pass from the lowest, each pass stable, so equal keys keep their input
// order and a sort by one word followed by a sort by another orders by
// (second, first).  Optional values of another unsigned type travel with
// their keys.  Per pass:
//   k_rs_count    the digit histogram of each tile of kRsTile keys (LDS
//                 atomics into one histogram per wavefront);
//   k_rs_offsets  one workgroup per digit: the exclusive sum over the tiles
//                 before, and the digit's total;
//   k_rs_scatter  each tile adds the digit's start (a block scan of the
//                 totals) to those sums, ranks its keys within their digit, in input
//                 order, by wavefront ballots (8 ballots find the lanes with
//                 the same digit; per-wave counts in LDS order the waves, a
//                 running count per digit orders the rounds), places them in
//                 LDS in digit order and writes every digit's run to its
//                 global place with consecutive threads on consecutive keys.
// Passes alternate between the two buffers; *in_b tells where the result is.
#pragma once

#include "pms_common.h"

namespace pms {

constexpr int kRsThreads = 256;  // one thread per digit value in the per-digit steps
constexpr int kRsRounds = 8;     // keys per thread per tile
constexpr int kRsTile = kRsThreads * kRsRounds;
constexpr int kRsMaxPass = 8;
static_assert(kRsThreads == 256 && kRsThreads == kBlock, "a thread per digit; block scans of kBlock threads");

template <typename K>
__device__ inline uint32_t rs_digit(K k, int shift)
{
    return (uint32_t)((unsigned long long)k >> shift) & 0xFFu;
}

// The lanes of the wavefront whose digit equals this lane's (valid lanes only).
__device__ inline uint64_t rs_match(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ inline uint64_t rs_lanes_below()
{
    const int lane = threadIdx.x & (kWave - 1);
    return lane ? (~0ull >> (kWave - lane)) : 0ull;
}

// Per tile, its digit histogram: cnt[d * ntiles + tile] (LDS atomics into
// one histogram per wavefront).
template <typename K>
__global__ void __launch_bounds__(kRsThreads) k_rs_count(const K *__restrict__ kin, int64_t n, int shift, uint32_t *cnt,
                                                         int64_t ntiles)
{
    __shared__ uint32_t h[kRsThreads / kWave][256];
    const int w = threadIdx.x / kWave;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * kRsTile;
#pragma unroll
        for (int v = 0; v < kRsThreads / kWave; v++) h[v][threadIdx.x] = 0u;
        K kr[kRsRounds];
#pragma unroll
        for (int r = 0; r < kRsRounds; r++) {
            const int64_t q = base + r * kRsThreads + threadIdx.x;
            kr[r] = kin[q < n ? q : n - 1];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsRounds; r++)
            if (base + r * kRsThreads + threadIdx.x < n) atomicAdd(&h[w][rs_digit(kr[r], shift)], 1u);
        __syncthreads();
        uint32_t v = 0;
#pragma unroll
        for (int u = 0; u < kRsThreads / kWave; u++) v += h[u][threadIdx.x];
        cnt[(int64_t)threadIdx.x * ntiles + tile] = v;
        __syncthreads();
    }
}

// Workgroup d: cnt[d][t] becomes the number of keys with digit d in the
// tiles before t; tot[d] the digit's total.  Per chunk each thread takes 16
// consecutive tiles (loaded together), and one block scan orders the threads.
static __global__ void __launch_bounds__(kRsThreads) k_rs_offsets(uint32_t *cnt, int64_t ntiles, uint32_t *tot_out)
{
    constexpr int kSeg = 16;
    const int d = blockIdx.x;
    uint32_t carry = 0;
    uint32_t *row = cnt + (int64_t)d * ntiles;
    for (int64_t t0 = 0; t0 < ntiles; t0 += (int64_t)kRsThreads * kSeg) {
        const int64_t s0 = t0 + (int64_t)threadIdx.x * kSeg;
        uint32_t v[kSeg];
        uint32_t sum = 0;
#pragma unroll
        for (int u = 0; u < kSeg; u++) {
            v[u] = s0 + u < ntiles ? row[s0 + u] : 0u;
            sum += v[u];
        }
        int32_t tot;
        uint32_t ex = carry + (uint32_t)block_excl_sum32((int32_t)sum, &tot);
#pragma unroll
        for (int u = 0; u < kSeg; u++) {
            if (s0 + u < ntiles) row[s0 + u] = ex;
            ex += v[u];
        }
        carry += (uint32_t)tot;
    }
    if (threadIdx.x == 0) tot_out[d] = carry;
}

// One pass: every key (and value) to its stable place by digit `shift`.
template <typename K, typename V, bool kVals>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const K *__restrict__ kin, K *__restrict__ kout,
                                                           const V *__restrict__ vin, V *__restrict__ vout, int64_t n,
                                                           int shift, const uint32_t *__restrict__ off,
                                                           const uint32_t *__restrict__ dtot, int64_t ntiles)
{
    // per-wave digit counts of a round, in three sets: a round writes one,
    // reads it after the barrier and clears the set of the round before, which
    // the round after next writes again (a barrier in between)
    __shared__ uint32_t cw[3][kRsThreads / kWave][256];
    __shared__ uint32_t run[2][256];  // keys per digit in the rounds so far (read one, write the other)
    __shared__ uint32_t tstart[256], goff[256];
    __shared__ K sk[kRsTile];
    __shared__ V sv[kVals ? kRsTile : 1];
    const int tid = threadIdx.x, w = tid / kWave;
    const uint64_t below = rs_lanes_below();
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * kRsTile;
        const int tn = (int)(n - base < kRsTile ? n - base : kRsTile);
#pragma unroll
        for (int s = 0; s < 3; s++)
#pragma unroll
            for (int v = 0; v < kRsThreads / kWave; v++) cw[s][v][tid] = 0u;
        run[0][tid] = 0u;
        // digit tid's first place for this tile: the keys of smaller digits
        // plus those of its digit in the tiles before
        int32_t all;
        goff[tid] = (uint32_t)block_excl_sum32((int32_t)dtot[tid], &all) + off[(int64_t)tid * ntiles + tile];
        K kr[kRsRounds];
        V vr[kRsRounds];
        uint32_t rk[kRsRounds];
#pragma unroll
        for (int r = 0; r < kRsRounds; r++) {
            const int q = r * kRsThreads + tid;
            const int64_t g = base + (q < tn ? q : tn - 1);
            kr[r] = kin[g];
            if (kVals) vr[r] = vin[g];
        }
        __syncthreads();  // the counters are cleared before round 0 writes them
#pragma unroll
        for (int r = 0; r < kRsRounds; r++) {
            const bool valid = r * kRsThreads + tid < tn;
            const uint32_t d = rs_digit(kr[r], shift);
            const uint64_t peers = rs_match(d, valid);
            const int set = r % 3, rb = r & 1;
            if (valid && !(peers & below)) cw[set][w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            uint32_t x = run[rb][d] + (uint32_t)__popcll(peers & below);
            for (int v = 0; v < w; v++) x += cw[set][v][d];
            rk[r] = x;
            // digit tid: the count after this round; the previous round's set cleared
            uint32_t s = 0;
#pragma unroll
            for (int v = 0; v < kRsThreads / kWave; v++) s += cw[set][v][tid];
            run[rb ^ 1][tid] = run[rb][tid] + s;
#pragma unroll
            for (int v = 0; v < kRsThreads / kWave; v++) cw[(r + 2) % 3][v][tid] = 0u;
        }
        __syncthreads();
        int32_t tot;
        tstart[tid] = (uint32_t)block_excl_sum32((int32_t)run[kRsRounds & 1][tid], &tot);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsRounds; r++) {
            if (r * kRsThreads + tid < tn) {
                const uint32_t slot = tstart[rs_digit(kr[r], shift)] + rk[r];
                if (slot < (uint32_t)kRsTile) {  // always (the ranks count the tile's keys); a bound, not a branch
                    sk[slot] = kr[r];
                    if (kVals) sv[slot] = vr[r];
                }
            }
        }
        __syncthreads();
        for (int s = tid; s < tn; s += kRsThreads) {
            const K k = sk[s];
            const uint32_t d = rs_digit(k, shift);
            const uint32_t pos = goff[d] + ((uint32_t)s - tstart[d]);
            if ((int64_t)pos < n) {  // always (offsets of a permutation); a bound on the write
                kout[pos] = k;
                if (kVals) vout[pos] = sv[s];
            }
        }
        __syncthreads();  // the LDS of this tile is read before the next tile writes it
    }
}

// Sorts a[0, n) (with va, when given) by bits [0, end_bit) using b (and vb)
// as the second buffer; *in_b: the result is in b / vb (else in a / va).
// cnt_id, tot_id: scratch buffers of the context.
template <typename K, typename V>
inline pms_status radix_sort(Ctx *c, K *a, K *b, V *va, V *vb, int64_t n, int end_bit, int cnt_id, int tot_id,
                             bool *in_b)
{
    *in_b = false;
    if (n <= 1 || end_bit <= 0) return PMS_OK;
    const int npass = (end_bit + 7) / 8;
    if (npass > kRsMaxPass || (int)(8 * sizeof(K)) < 8 * npass - 7)
        return set_err(c, PMS_ERR_INVALID_ARG, "internal: sort bit range wider than the key");
    const int64_t ntiles = (n + kRsTile - 1) / kRsTile;
    uint32_t *cnt = (uint32_t *)grow_scratch(c, cnt_id, (size_t)ntiles * 256 * 4);
    uint32_t *dtot = (uint32_t *)grow_scratch(c, tot_id, 256 * 4);
    if (!cnt || !dtot) return set_err(c, PMS_ERR_OOM, "sort scratch");
    hipStream_t s = c->stream;
    const unsigned gt = (unsigned)(ntiles < (1 << 20) ? ntiles : (1 << 20));
    K *src = a, *dst = b;
    V *vsrc = va, *vdst = vb;
    for (int p = 0; p < npass; p++) {
        k_rs_count<K><<<gt, kRsThreads, 0, s>>>(src, n, 8 * p, cnt, ntiles);
        k_rs_offsets<<<256, kRsThreads, 0, s>>>(cnt, ntiles, dtot);
        if (va)
            k_rs_scatter<K, V, true><<<gt, kRsThreads, 0, s>>>(src, dst, vsrc, vdst, n, 8 * p, cnt, dtot, ntiles);
        else
            k_rs_scatter<K, V, false><<<gt, kRsThreads, 0, s>>>(src, dst, nullptr, nullptr, n, 8 * p, cnt, dtot, ntiles);
        std::swap(src, dst);
        std::swap(vsrc, vdst);
        *in_b = !*in_b;
    }
    PMS_HIP(hipGetLastError());
    return PMS_OK;
}

}  // namespace pms
