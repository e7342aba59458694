// Parallel multi-scale (pms) reduction of a boundary matrix over F2 on
// gfx950.  Method: Mendoza-Smith & Tanner, arXiv 1708.04710, Alg.
// "Parallel multi-scale reduction" (Sec. 1) with the theory of Sec. 3.
//
// State (all in HBM, one entry per column j of the m x m matrix):
//   off[j], len[j]  current column: ascending rows, either a slice of the
//                   caller's CSC `rows` or (bit 62 of off set) of the arena
//   low[j]          low(j) of eq. "low" on the compressed column, -1 = empty
//   state[j]        ACTIVE (unreduced, non-zero) / PIVOT (low(j) = low*(j))
//                   / ZERO (positive, reduced to or cleared to zero) /
//                   CLEARED (zeroed this round, finalised at compaction)
//   beta[j]         beta_j of Def. "beta" (invariant, Thm. "Properties" P.2)
//   piv[i]          the pivot whose low* is i, or -1: the inverse of low*
//                   on the known pivots (the leftmost column of N(j), eq.
//                   "neighbours", for every later column with low i)
//   T[i]            round-stamped atomicMin over active columns with low i:
//                   the leftmost unreduced column with that low
//   neg             bitmask of simplices known to be negative (beta_j >= 0,
//                   Thm. "Properties" P.3, or a found pivot); their rows are
//                   deleted from every column (compression)
//
// One round (the paper's iteration: Phase I then Phase II):
//   k_low      low on every active column, skipping negative rows; T table
//   k_collide  j collides iff an earlier column shares its low
//              (low(j) in low([j-1]), Alg. "Finding local injections")
//   k_pivots   Phase I: segmented exclusive prefix max, per dimension, of the
//              lows of colliding columns (maxCollision); a non-colliding j
//              with low(j) > maxCollision, or with beta_j = low(j), is a
//              pivot (Thms. "Local injection I/II", "Properties" P.5).
//              Clearing: column low(j) of a new pivot is zeroed (Sec. 2.4).
//   k_xor      Phase II: every colliding column adds the leftmost column
//              with its low (eq. "partition": the N(j) are disjoint, so all
//              additions run at once); known-negative and top-dimension
//              columns keep adding pivots while their new low has one.
//   k_compact  stable compaction of the still-active columns.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "pms_common.h"

namespace pms {

enum : uint8_t { ST_ACTIVE = 0, ST_PIVOT = 1, ST_ZERO = 2, ST_CLEARED = 3 };

constexpr uint64_t kArenaBit = 1ull << 62;
constexpr int kScanThreads = 1024;

// Device counters of one call (zeroed at its start).
struct Counters {
    unsigned long long arena_top;
    unsigned long long additions;
    unsigned long long xor_entries;
    int32_t error;       // 1 = not compatible
    int32_t overflow;    // arena exhausted during k_xor
    int32_t n_next;      // active columns after compaction
    int32_t new_pivots;
    int32_t beta_pivots;
    int32_t topdim;
    int32_t n_pairs;
    int32_t n_ess;
    int32_t bad_source;  // a source to the right of its target (never expected)
    int32_t pad[3];
};

struct Dev {
    int64_t m;
    const int64_t *col_ptr;
    const int32_t *rows;
    const int8_t *dim;
    int64_t *off;
    int32_t *len;
    int32_t *low;
    uint8_t *state;
    int32_t *beta;
    int32_t *left;
    int32_t *piv;
    unsigned long long *T;
    uint32_t *neg;
    int32_t *low_star;
    int8_t *coll;
    int32_t *arena;
    unsigned long long arena_cap;
    Counters *cnt;
};

__device__ inline bool is_neg(const uint32_t *neg, int32_t r)
{
    return (neg[r >> 5] >> (r & 31)) & 1u;
}

__device__ inline const int32_t *col_base(const Dev &d, int64_t off)
{
    return (off & (int64_t)kArenaBit) ? d.arena + (off & ~(int64_t)kArenaBit) : d.rows + off;
}

// T holds (~round << 32 | j): newer rounds compare smaller, so atomicMin needs
// no reset between rounds.
__device__ inline unsigned long long t_key(uint32_t round, int32_t j)
{
    return ((unsigned long long)(0xFFFFFFFFu - round) << 32) | (uint32_t)j;
}

__device__ inline int32_t t_decode(unsigned long long k, uint32_t round)
{
    return (uint32_t)(k >> 32) == 0xFFFFFFFFu - round ? (int32_t)(uint32_t)k : -1;
}

__device__ inline int slot_of(const Dev &d, int32_t j)
{
    // dimensions 1..4 get their own prefix-max slot; higher ones share a slot
    // (a shared slot only makes maxCollision larger: still sound)
    return d.dim ? ((d.dim[j] - 1) & 3) : 0;
}

// ---------------------------------------------------------------- fills
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// ---------------------------------------------------------------- Phase 0
// Column headers, input checks, and left(i) (Def. "left") by atomicMin.
// The structural checks (slice inside rows[0, nnz), rows strictly ascending
// and in [0, j)) always run, so no later kernel can index out of bounds;
// `validate` adds the dimension check.
__global__ void k_init(Dev d, int64_t nnz, int validate)
{
    int top = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = d.col_ptr[j], e = d.col_ptr[j + 1];
        bool bad = e < s || s < 0 || e > nnz || (j == 0 && s != 0) || e - s > 0x7FFFFFFF;
        int32_t n = bad ? 0 : (int32_t)(e - s);
        int32_t prev = -1;
        for (int64_t p = s; p < s + n; p++) {
            const int32_t r = d.rows[p];
            if (r <= prev || (int64_t)r >= j) { bad = true; break; }
            if (validate && d.dim && d.dim[r] != d.dim[j] - 1) { bad = true; break; }
            prev = r;
            atomicMin(&d.left[r], (int32_t)j);
        }
        if (validate && d.dim && d.dim[j] < 0) bad = true;
        if (bad) { atomicExch(&d.cnt->error, 1); n = 0; }
        d.off[j] = bad ? 0 : s;
        d.len[j] = n;
        d.low[j] = n ? d.rows[s + n - 1] : -1;
        d.state[j] = n ? ST_ACTIVE : ST_ZERO;
        if (d.dim && d.dim[j] > top) top = d.dim[j];
    }
    if (d.dim) atomicMax(&d.cnt->topdim, top);
}

// beta_j = max{i : left(i) = j} (Def. "beta"); beta_j >= 0 marks column j as
// negative (Thm. "Properties of beta_j" P.3), so its row can be compressed.
__global__ void k_beta(Dev d, int compression)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = d.col_ptr[j];
        int32_t b = -1;
        for (int64_t p = s + d.len[j] - 1; p >= s; p--) {
            const int32_t r = d.rows[p];
            if (d.left[r] == (int32_t)j) { b = r; break; }  // rows ascending: first hit from the end is the max
        }
        d.beta[j] = b;
        if (compression && b >= 0) atomicOr(&d.neg[j >> 5], 1u << (j & 31));
    }
}

// ---------------------------------------------------------------- round
__global__ void k_low(Dev d, const int32_t *act, int32_t nA, uint32_t round)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nA; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = act[q];
        int32_t n = d.len[j];
        const int32_t *c = col_base(d, d.off[j]);
        // rows of known-negative simplices at the bottom of the column are
        // deleted outright (compression); the column's low is the last row left
        while (n > 0 && is_neg(d.neg, c[n - 1])) n--;
        d.len[j] = n;
        if (n == 0) {
            d.low[j] = -1;
            d.state[j] = ST_ZERO;
            continue;
        }
        const int32_t i = c[n - 1];
        d.low[j] = i;
        atomicMin(&d.T[i], t_key(round, j));
    }
}

// One tile of kBlock active positions per block.
__global__ void __launch_bounds__(kBlock) k_collide(Dev d, const int32_t *act, int32_t nA, uint32_t round, I4 *agg)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    I4 e = i4_fill(-1);
    if (q < nA) {
        const int32_t j = act[q];
        int8_t cl = 0;
        if (d.state[j] == ST_ACTIVE) {
            const int32_t i = d.low[j];
            const int32_t t = t_decode(d.T[i], round);
            cl = (d.piv[i] >= 0 || t != j) ? 1 : 0;
            if (cl) e.v[slot_of(d, j)] = i;
        }
        d.coll[q] = cl;
    }
    I4 tot;
    block_excl_max4(e, &tot);
    if (threadIdx.x == 0) agg[blockIdx.x] = tot;
}

// Exclusive max-scan of the per-block aggregates, one block of 1024 threads.
__global__ void __launch_bounds__(kScanThreads) k_scan_max4(I4 *agg, int64_t nb)
{
    __shared__ I4 s_w[kScanThreads / kWave];
    __shared__ I4 s_carry;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_carry = i4_fill(-1);
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        I4 v = i < nb ? agg[i] : i4_fill(-1);
        I4 inc = wave_incl_max4(v);
        I4 exc;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int32_t y = __shfl_up(inc.v[k], 1, kWave);
            exc.v[k] = lane == 0 ? -1 : y;
        }
        if (lane == kWave - 1) s_w[wid] = inc;
        __syncthreads();
        I4 pre = s_carry, tot = s_carry;
        for (int w = 0; w < kScanThreads / kWave; w++) {
            if (w < wid) pre = i4_max(pre, s_w[w]);
            tot = i4_max(tot, s_w[w]);
        }
        if (i < nb) agg[i] = i4_max(pre, exc);
        __syncthreads();
        if (threadIdx.x == 0) s_carry = tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sum(int32_t *cnt, int64_t nb, int32_t *total)
{
    __shared__ int32_t s_w[kScanThreads / kWave];
    __shared__ int32_t s_carry;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        int32_t v = i < nb ? cnt[i] : 0;
        int32_t inc = wave_incl_sum32(v);
        if (lane == kWave - 1) s_w[wid] = inc;
        __syncthreads();
        int32_t pre = s_carry, tot = s_carry;
        for (int w = 0; w < kScanThreads / kWave; w++) {
            if (w < wid) pre += s_w[w];
            tot += s_w[w];
        }
        if (i < nb) cnt[i] = pre + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

// Phase I + the beta test + clearing.
__global__ void __launch_bounds__(kBlock) k_pivots(Dev d, const int32_t *act, int32_t nA, const I4 *agg,
                                                   int compression, int count_beta)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    I4 e = i4_fill(-1);
    int32_t j = -1, i = -1;
    bool live = false, cl = false;
    if (q < nA) {
        j = act[q];
        live = d.state[j] == ST_ACTIVE;
        if (live) {
            i = d.low[j];
            cl = d.coll[q] != 0;
            if (cl) e.v[slot_of(d, j)] = i;
        }
    }
    I4 tot;
    I4 mc = i4_max(block_excl_max4(e, &tot), agg[blockIdx.x]);
    int np = 0, nb = 0;
    if (live && !cl) {
        const bool by_beta = d.beta[j] == i;                  // beta_j = low(j): Thm. P.5
        const bool by_li = i > mc.v[slot_of(d, j)];           // low(j) > maxCollision
        if (by_beta || by_li) {
            d.piv[i] = j;
            d.state[j] = ST_PIVOT;
            d.low_star[j] = i;
            if (compression) atomicOr(&d.neg[j >> 5], 1u << (j & 31));
            if (d.state[i] == ST_ACTIVE) d.state[i] = ST_CLEARED;  // clearing: sigma_i is positive
            np = 1;
            nb = by_beta ? 1 : 0;
        }
    }
    int32_t tnp;
    block_excl_sum32(np, &tnp);
    if (count_beta) {
        int32_t tnb;
        block_excl_sum32(nb, &tnb);
        if (threadIdx.x == 0 && tnb) atomicAdd(&d.cnt->beta_pivots, tnb);
    }
    if (threadIdx.x == 0 && tnp) atomicAdd(&d.cnt->new_pivots, tnp);
}

// Sorted symmetric difference of two ascending row lists (F2 column
// addition), dropping rows of known-negative simplices.
__device__ inline int32_t merge_add(const int32_t *__restrict__ x, int32_t nx, const int32_t *__restrict__ y, int32_t ny,
                                    int32_t *__restrict__ out, const uint32_t *neg, int compression)
{
    int32_t a = 0, b = 0, k = 0;
    while (a < nx && b < ny) {
        const int32_t u = x[a], v = y[b];
        if (u < v) {
            if (!(compression && is_neg(neg, u))) out[k++] = u;
            a++;
        } else if (v < u) {
            if (!(compression && is_neg(neg, v))) out[k++] = v;
            b++;
        } else {
            a++;
            b++;
        }
    }
    for (; a < nx; a++) {
        const int32_t u = x[a];
        if (!(compression && is_neg(neg, u))) out[k++] = u;
    }
    for (; b < ny; b++) {
        const int32_t v = y[b];
        if (!(compression && is_neg(neg, v))) out[k++] = v;
    }
    return k;
}

// Phase II.  Also counts, per tile, the positions that stay active.
__global__ void __launch_bounds__(kBlock) k_xor(Dev d, const int32_t *act, int32_t nA, uint32_t round, int variant,
                                                int compression, int chain, int tail, int32_t *keep_cnt)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t j = -1, s = -1, tlen = 0, slen = 0;
    int64_t toff = 0, soff = 0;
    bool target = false;
    if (q < nA) {
        j = act[q];
        if (d.state[j] == ST_ACTIVE && d.coll[q]) {
            const int32_t i = d.low[j];
            s = d.piv[i];
            if (s < 0 && variant == 0) {
                s = t_decode(d.T[i], round);
                if (s == j || (s >= 0 && d.state[s] == ST_CLEARED)) s = -1;
            }
            if (s >= 0) {
                target = true;
                toff = d.off[j];
                tlen = d.len[j];
                soff = d.off[s];
                slen = d.len[s];
                if (s >= j) atomicExch(&d.cnt->bad_source, 1);
            }
        }
    }
    // wave-aggregated arena allocation of a ping-pong region per target
    int64_t need = target ? 2 * (int64_t)(tlen + slen) : 0;
    int64_t inc = wave_incl_sum64(need);
    int64_t wtot = __shfl(inc, kWave - 1, kWave);
    unsigned long long wbase = 0;
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0 && wtot > 0) wbase = atomicAdd(&d.cnt->arena_top, (unsigned long long)wtot);
    wbase = __shfl(wbase, 0, kWave);
    bool fits = wbase + (unsigned long long)wtot <= d.arena_cap;
    if (target && !fits) {
        atomicExch(&d.cnt->overflow, 1);
        target = false;
    }
    int64_t adds = 0, xe = 0;
    if (target) {
        int64_t reg = (int64_t)wbase + inc - need;  // region [reg, reg + rcap)
        int64_t rcap = need;
        int half = 0;
        const bool chainable = chain && (d.beta[j] >= 0 || (d.dim && d.dim[j] == d.cnt->topdim) || nA < tail);
        while (true) {
            const int32_t *x = col_base(d, toff);
            const int32_t *y = col_base(d, soff);
            int64_t bound = (int64_t)tlen + slen;
            int64_t dst;
            if (bound <= rcap / 2) {
                dst = reg + half * (rcap / 2);
            } else {
                // region too small for this step: take a fresh, larger one
                int64_t nr = 2 * bound;
                unsigned long long o = atomicAdd(&d.cnt->arena_top, (unsigned long long)nr);
                if (o + (unsigned long long)nr > d.arena_cap) {
                    atomicExch(&d.cnt->overflow, 1);
                    break;  // header still describes a valid column
                }
                reg = (int64_t)o;
                rcap = nr;
                half = 0;
                dst = reg;
            }
            int32_t *out = d.arena + dst;
            const int32_t k = merge_add(x, tlen, y, slen, out, d.neg, compression);
            adds++;
            xe += (int64_t)tlen + slen;
            toff = dst | (int64_t)kArenaBit;
            tlen = k;
            d.off[j] = toff;
            d.len[j] = k;
            if (k == 0) {
                d.low[j] = -1;
                d.state[j] = ST_ZERO;  // column j is positive
                break;
            }
            const int32_t nl = out[k - 1];
            d.low[j] = nl;
            if (!chainable) break;
            s = d.piv[nl];
            if (s < 0) break;
            soff = d.off[s];
            slen = d.len[s];
            half ^= 1;
        }
    }
    const int keep = (q < nA && d.state[j] == ST_ACTIVE) ? 1 : 0;
    int32_t tk;
    block_excl_sum32(keep, &tk);
    int64_t badds = block_sum64(adds);
    int64_t bxe = block_sum64(xe);
    if (threadIdx.x == 0) {
        keep_cnt[blockIdx.x] = tk;
        if (badds) {
            atomicAdd(&d.cnt->additions, (unsigned long long)badds);
            atomicAdd(&d.cnt->xor_entries, (unsigned long long)bxe);
        }
    }
}

// Stable compaction of the active list; finalises cleared columns.
__global__ void __launch_bounds__(kBlock) k_compact(Dev d, const int32_t *act, int32_t nA, const int32_t *keep_off,
                                                    int32_t *act_next)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int keep = 0;
    int32_t j = -1;
    if (q < nA) {
        j = act[q];
        const uint8_t st = d.state[j];
        if (st == ST_CLEARED) {
            d.state[j] = ST_ZERO;
            d.len[j] = 0;
            d.low[j] = -1;
        }
        keep = st == ST_ACTIVE;
    }
    int32_t tot;
    const int32_t pos = block_excl_sum32(keep, &tot);
    if (keep) act_next[keep_off[blockIdx.x] + pos] = j;
}

// Arena regrowth: copy every live arena column into a new arena.
__global__ void k_defrag(Dev d, int32_t *dst, unsigned long long *dst_top)
{
    for (int64_t j0 = blockIdx.x * (int64_t)blockDim.x; j0 < d.m; j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        int64_t n = 0, off = 0;
        if (j < d.m) {
            off = d.off[j];
            const uint8_t st = d.state[j];
            if ((off & (int64_t)kArenaBit) && (st == ST_ACTIVE || st == ST_PIVOT)) n = d.len[j];
        }
        int64_t inc = wave_incl_sum64(n);
        int64_t wtot = __shfl(inc, kWave - 1, kWave);
        unsigned long long base = 0;
        if ((threadIdx.x & (kWave - 1)) == 0 && wtot) base = atomicAdd(dst_top, (unsigned long long)wtot);
        base = __shfl(base, 0, kWave);
        if (n) {
            const int64_t o = (int64_t)base + inc - n;
            const int32_t *src = d.arena + (off & ~(int64_t)kArenaBit);
            for (int64_t k = 0; k < n; k++) dst[o + k] = src[k];
            d.off[j] = o | (int64_t)kArenaBit;
        }
    }
}

// ---------------------------------------------------------------- finalize
__global__ void __launch_bounds__(kBlock) k_fin_count(Dev d, int32_t *cnt_pairs, int32_t *cnt_ess)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int dp = 0, de = 0;
    if (j < d.m) {
        dp = d.low_star[j] >= 0;
        de = d.low_star[j] < 0 && d.piv[j] < 0;
    }
    int32_t tp, te;
    block_excl_sum32(dp, &tp);
    block_excl_sum32(de, &te);
    if (threadIdx.x == 0) {
        cnt_pairs[blockIdx.x] = tp;
        cnt_ess[blockIdx.x] = te;
    }
}

__global__ void __launch_bounds__(kBlock) k_fin_scatter(Dev d, const int32_t *off_pairs, const int32_t *off_ess,
                                                        int32_t *birth, int32_t *death, int32_t *ess)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int dp = 0, de = 0;
    int32_t ls = -1;
    if (j < d.m) {
        ls = d.low_star[j];
        dp = ls >= 0;
        de = ls < 0 && d.piv[j] < 0;
    }
    int32_t tp, te;
    const int32_t pp = block_excl_sum32(dp, &tp);
    const int32_t pe = block_excl_sum32(de, &te);
    if (dp && birth) {
        birth[off_pairs[blockIdx.x] + pp] = ls;
        death[off_pairs[blockIdx.x] + pp] = (int32_t)j;
    }
    if (de && ess) ess[off_ess[blockIdx.x] + pe] = (int32_t)j;
}

// ---------------------------------------------------------------- host
void *scratch(Ctx *c, int id, size_t bytes)
{
    Buf &b = c->b[id];
    if (b.bytes >= bytes && b.p) return b.p;
    if (b.p) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    want = want + want / 4;  // headroom so slightly larger calls reuse it
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        return nullptr;
    }
    b.bytes = want;
    return b.p;
}

pms_status set_err(Ctx *c, pms_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

static pms_status grow_arena(Ctx *c, Dev &d, Counters *h, bool defrag_only_if_needed)
{
    (void)defrag_only_if_needed;
    unsigned long long new_cap = c->arena_cap * 2;
    int32_t *na = nullptr;
    PMS_HIP(hipMalloc(&na, new_cap * sizeof(int32_t)));
    unsigned long long *top = (unsigned long long *)scratch(c, B_TMP1, 64);
    if (!top) { (void)hipFree(na); return set_err(c, PMS_ERR_OOM, "scratch alloc"); }
    PMS_HIP(hipMemsetAsync(top, 0, sizeof(unsigned long long), c->stream));
    k_defrag<<<grid_for(d.m, kBlock, 65536), kBlock, 0, c->stream>>>(d, na, top);
    PMS_HIP(hipGetLastError());
    unsigned long long ntop = 0;
    PMS_HIP(hipMemcpyAsync(&ntop, top, sizeof(ntop), hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    PMS_HIP(hipFree(c->arena));
    c->arena = na;
    c->arena_cap = new_cap;
    d.arena = na;
    d.arena_cap = new_cap;
    h->arena_top = ntop;
    h->overflow = 0;
    PMS_HIP(hipMemcpyAsync(&d.cnt->arena_top, &h->arena_top, sizeof(unsigned long long), hipMemcpyHostToDevice, c->stream));
    PMS_HIP(hipMemsetAsync(&d.cnt->overflow, 0, sizeof(int32_t), c->stream));
    return PMS_OK;
}

static pms_status reduce_impl(Ctx *c, const pms_boundary *bnd, const pms_options *opt, pms_result *res)
{
    const int64_t m = bnd->m;
    res->n_pairs = res->n_essential = 0;
    res->rounds = 0;
    res->phase0_pivots = 0;
    res->additions = res->xor_entries = 0;
    if (m == 0) return PMS_OK;

    // nnz (host needs it only to size the arena)
    int64_t nnz = 0;
    PMS_HIP(hipMemcpyAsync(&nnz, bnd->col_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    if (nnz < 0) return set_err(c, PMS_ERR_INVALID_ARG, "col_ptr[m] < 0");

    const int64_t nblk = (m + kBlock - 1) / kBlock;
    const int64_t nwords = (m + 31) / 32;
    Dev d{};
    d.m = m;
    d.col_ptr = bnd->col_ptr;
    d.rows = bnd->rows;
    d.dim = bnd->dim;
    d.off = (int64_t *)scratch(c, B_OFF, m * 8);
    d.len = (int32_t *)scratch(c, B_LEN, m * 4);
    d.low = (int32_t *)scratch(c, B_LOW, m * 4);
    d.state = (uint8_t *)scratch(c, B_STATE, m);
    d.beta = (int32_t *)scratch(c, B_BETA, m * 4);
    d.left = (int32_t *)scratch(c, B_LEFT, m * 4);
    d.piv = (int32_t *)scratch(c, B_PIV, m * 4);
    d.T = (unsigned long long *)scratch(c, B_T, m * 8);
    d.neg = (uint32_t *)scratch(c, B_NEG, nwords * 4);
    d.coll = (int8_t *)scratch(c, B_COLL, m);
    d.cnt = (Counters *)scratch(c, B_CNT, sizeof(Counters));
    d.low_star = res->low_star;
    int32_t *act0 = (int32_t *)scratch(c, B_ACT0, m * 4);
    int32_t *act1 = (int32_t *)scratch(c, B_ACT1, m * 4);
    I4 *agg = (I4 *)scratch(c, B_AGG, nblk * sizeof(I4));
    int32_t *keep = (int32_t *)scratch(c, B_AGG2, (nblk + 1) * 4);
    int32_t *keep2 = (int32_t *)scratch(c, B_FLAGS, (nblk + 1) * 4);
    if (!d.off || !d.len || !d.low || !d.state || !d.beta || !d.left || !d.piv || !d.T || !d.neg || !d.coll ||
        !d.cnt || !act0 || !act1 || !agg || !keep || !keep2)
        return set_err(c, PMS_ERR_OOM, "scratch allocation failed");

    // arena: sized for the first rounds' fill-in, grown on demand
    unsigned long long want = (unsigned long long)(4 * nnz) + (1ull << 22);
    if (opt->arena_entries > 0) want = (unsigned long long)opt->arena_entries;
    if (c->arena_cap < want || (opt->arena_entries > 0 && c->arena_cap != want)) {
        if (c->arena) PMS_HIP(hipFree(c->arena));
        c->arena = nullptr;
        c->arena_cap = 0;
        PMS_HIP(hipMalloc(&c->arena, want * sizeof(int32_t)));
        c->arena_cap = want;
    }
    d.arena = c->arena;
    d.arena_cap = c->arena_cap;

    hipStream_t st = c->stream;
    const unsigned gm = grid_for(m, kBlock, 65536);
    PMS_HIP(hipMemsetAsync(d.cnt, 0, sizeof(Counters), st));
    k_fill_i32<<<gm, kBlock, 0, st>>>(d.left, m, 0x7FFFFFFF);
    k_fill_i32<<<gm, kBlock, 0, st>>>(d.piv, m, -1);
    k_fill_i32<<<gm, kBlock, 0, st>>>(d.low_star, m, -1);
    k_fill_i32<<<grid_for(nwords, kBlock, 65536), kBlock, 0, st>>>((int32_t *)d.neg, nwords, 0);
    k_fill_u64<<<gm, kBlock, 0, st>>>(d.T, m, ~0ull);
    k_init<<<gm, kBlock, 0, st>>>(d, nnz, opt->validate);
    k_beta<<<gm, kBlock, 0, st>>>(d, opt->compression);
    k_iota<<<gm, kBlock, 0, st>>>(act0, m);
    PMS_HIP(hipGetLastError());

    Counters *h = (Counters *)c->host_pinned;
    PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    PMS_HIP(hipStreamSynchronize(st));
    if (h->error) return set_err(c, PMS_ERR_NOT_COMPATIBLE, "boundary matrix is not that of a compatible filtration "
                                                            "(rows must ascend, lie above the diagonal and be facets)");

    int32_t nA = (int32_t)m;
    uint32_t round = 0;
    int32_t *act = act0, *act_next = act1;
    while (nA > 0) {
        if (opt->max_rounds > 0 && (int32_t)round >= opt->max_rounds) {
            res->rounds = (int32_t)round;
            return set_err(c, PMS_ERR_NOT_CONVERGED, "max_rounds reached before the reduction converged");
        }
        const int64_t tiles = (nA + kBlock - 1) / kBlock;
        const unsigned gA = grid_for(nA, kBlock, 65536);
        k_low<<<gA, kBlock, 0, st>>>(d, act, nA, round);
        k_collide<<<(unsigned)tiles, kBlock, 0, st>>>(d, act, nA, round, agg);
        k_scan_max4<<<1, kScanThreads, 0, st>>>(agg, tiles);
        k_pivots<<<(unsigned)tiles, kBlock, 0, st>>>(d, act, nA, agg, opt->compression, round == 0);
        k_xor<<<(unsigned)tiles, kBlock, 0, st>>>(d, act, nA, round, opt->variant, opt->compression, opt->chain,
                                                  opt->tail_active, keep);
        k_scan_sum<<<1, kScanThreads, 0, st>>>(keep, tiles, &d.cnt->n_next);
        k_compact<<<(unsigned)tiles, kBlock, 0, st>>>(d, act, nA, keep, act_next);
        PMS_HIP(hipGetLastError());
        PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
        PMS_HIP(hipStreamSynchronize(st));
        round++;
        if (h->bad_source) return set_err(c, PMS_ERR_HIP, "internal: a column was added a column to its right");
        if (h->overflow) {
            pms_status s = grow_arena(c, d, h, true);
            if (s != PMS_OK) return s;
        }
        nA = h->n_next;
        std::swap(act, act_next);
    }
    res->rounds = (int32_t)round;
    res->additions = (int64_t)h->additions;
    res->xor_entries = (int64_t)h->xor_entries;
    res->phase0_pivots = h->beta_pivots;

    // pairs and essential simplices, canonical order
    int32_t *cp = keep, *ce = keep2;
    k_fin_count<<<(unsigned)nblk, kBlock, 0, st>>>(d, cp, ce);
    k_scan_sum<<<1, kScanThreads, 0, st>>>(cp, nblk, &d.cnt->n_pairs);
    k_scan_sum<<<1, kScanThreads, 0, st>>>(ce, nblk, &d.cnt->n_ess);
    PMS_HIP(hipGetLastError());
    PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    PMS_HIP(hipStreamSynchronize(st));
    res->n_pairs = h->n_pairs;
    res->n_essential = h->n_ess;
    const bool want_pairs = res->pair_birth && res->pair_death;
    const bool want_ess = res->essential != nullptr;
    if ((want_pairs && res->cap_pairs < res->n_pairs) || (want_ess && res->cap_essential < res->n_essential))
        return set_err(c, PMS_ERR_CAPACITY, "output capacity too small (n_pairs / n_essential hold the sizes)");
    if (want_pairs || want_ess) {
        k_fin_scatter<<<(unsigned)nblk, kBlock, 0, st>>>(d, cp, ce, want_pairs ? res->pair_birth : nullptr,
                                                         want_pairs ? res->pair_death : nullptr,
                                                         want_ess ? res->essential : nullptr);
        PMS_HIP(hipGetLastError());
        PMS_HIP(hipStreamSynchronize(st));
    }
    return PMS_OK;
}

}  // namespace pms

// ==================================================================== ABI
struct pms_ctx : pms::Ctx {};

extern "C" {

const char *pms_version(void) { return "pms-gfx950 0.1"; }

pms_options pms_default_options(void)
{
    pms_options o;
    o.variant = 0;
    o.compression = 1;
    o.max_rounds = 0;
    o.chain = 1;
    o.tail_active = 1024;
    o.validate = 1;
    o.arena_entries = 0;
    return o;
}

pms_status pms_create(pms_ctx **ctx, int device, void *stream)
{
    if (!ctx) return PMS_ERR_INVALID_ARG;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PMS_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return PMS_ERR_HIP;
    pms_ctx *c = new (std::nothrow) pms_ctx();
    if (!c) return PMS_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipHostMalloc(&c->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return PMS_ERR_OOM;
    }
    *ctx = c;
    return PMS_OK;
}

void pms_destroy(pms_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->b)
        if (b.p) (void)hipFree(b.p);
    if (c->arena) (void)hipFree(c->arena);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    delete c;
}

const char *pms_last_error(const pms_ctx *c)
{
    if (!c) return "no context";
    return c->err.c_str();
}

pms_status pms_reduce(pms_ctx *c, const pms_boundary *bnd, const pms_options *opt, pms_result *res)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!bnd || !res) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null boundary or result");
    if (bnd->m < 0 || bnd->m >= 0x7FFFFFFF) return pms::set_err(c, PMS_ERR_INVALID_ARG, "m out of range");
    if (bnd->m > 0 && (!bnd->col_ptr || !bnd->rows || !res->low_star))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "null col_ptr / rows / low_star");
    pms_options o = opt ? *opt : pms_default_options();
    if (o.variant < 0 || o.variant > 1 || o.max_rounds < 0 || o.arena_entries < 0)
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "bad options");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    pms_status s = pms::reduce_impl(c, bnd, &o, res);
    if (s != PMS_OK && s != PMS_ERR_CAPACITY && s != PMS_ERR_NOT_CONVERGED) {
        res->n_pairs = res->n_essential = 0;
    }
    return s;
}

}  // extern "C"
