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

#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pms_common.h"

namespace pms {

enum : uint8_t { ST_ACTIVE = 0, ST_PIVOT = 1, ST_ZERO = 2, ST_CLEARED = 3 };
constexpr int8_t kNotLive = 2;  // coll[q]: column act[q] was not active when the round's collisions were taken
constexpr int8_t kWaits = 3;    // coll[q]: column act[q] collides but waits for a later round (round_budget)

constexpr uint64_t kArenaBit = 1ull << 62;
constexpr int kScanThreads = 1024;

enum StatId {
    S_ADDS = 0, S_XE, S_XBYTES, S_CBYTES, S_NEWPIV, S_BETAPIV,
    // opt-in trace of k_chain (PMS_TRACE=1): steps by path, working-column
    // length, shader cycles per phase of a short-pivot step, flushes, lows from P
    S_T_SHORT, S_T_LONG, S_T_GLOBAL, S_T_SUML, S_T_CTOG, S_T_CNEXT, S_T_CFLUSH, S_T_FLUSHES, S_T_QUEUED,
    S_T_LANE, S_T_BAIL, S_LBYTES, S_T_FROMP, S_T_DEL, S_T_LSUML, S_T_LGT16, S_T_LGT32,
    S_WBYTES, S_T_WIDE, S_T_TOWIDE, S_T_LITER, S_T_LREFILL, S_T_LFLUSH, S_T_LBUSY, S_T_LLONG, S_T_LTOG, S_T_LTROUND,
    // bytes of the additions by the unit cost of one column addition,
    // 4 (len t + len s + len t+s), per kernel
    S_ABYTES_XOR, S_ABYTES_LANE, S_ABYTES_WIDE, S_ABYTES_CHAIN,
    // k_chain_solve: algorithmic bytes, bytes of its additions as multi-way sums, sweeps,
    // columns solved, columns handed to k_chain
    S_SBYTES, S_ABYTES_SOLVE, S_T_SWEEPS, S_T_SOLVED, S_T_SFALL,
    // trace of k_chain_solve: shader cycles in set-up, the two passes, the toggles and the
    // write-back (thread 0, summed over columns), membership changes
    S_T_SINIT, S_T_SA, S_T_SB, S_T_SC, S_T_SOUT, S_T_SDELTA, S_T_SLONG, S_T_SLONGE, S_T_SDEFER,
    // k_pivots: bytes a new pivot moves (its record, the column entries it copies, the tables)
    S_PBYTES,
    S_NUM
};

// Device counters of one call (zeroed at its start).
struct Counters {
    unsigned long long additions;    // column additions (folded from the stripes)
    unsigned long long xor_entries;  // entries read by them
    unsigned long long xor_bytes;    // algorithmic bytes moved by k_xor
    unsigned long long chain_bytes;  // algorithmic bytes moved by k_chain
    unsigned long long lane_bytes;   // algorithmic bytes moved by k_chain_lane
    unsigned long long wide_bytes;   // algorithmic bytes moved by k_chain_wide
    // 4 (len t + len s + len t+s) summed over the additions of k_xor, the two
    // lane passes and k_chain (the bytes of a column addition by itself)
    unsigned long long abytes_xor, abytes_lane, abytes_wide, abytes_chain;
    unsigned long long solve_bytes;  // algorithmic bytes moved by k_chain_solve
    unsigned long long pivot_bytes;  // bytes k_pivots moves for its new pivots
    // its additions as multi-way sums: 4 (len c + the pivots' lengths + len out) per column
    unsigned long long abytes_solve;
    unsigned long long active_sum;   // sum over rounds of the round's active columns
    unsigned long long diag_low_l1;  // diagnostics: sum_j (low(j) + 1)
    unsigned long long diag_ess;     // diagnostics: |E|
    unsigned long long diag_active;  // diagnostics: columns neither pivot nor zero
    unsigned long long arena_free;   // arena entries still free at the end of the round
    unsigned long long c8_cleared;   // columns cleared by Lemma "Clearing by local compression"
    int32_t error;       // 1 = not compatible
    int32_t overflow;    // an arena partition ran out during this round
    int32_t n_next;      // active columns after compaction
    int32_t new_pivots;
    int32_t beta_pivots;
    int32_t topdim;
    int32_t n_pairs;
    int32_t n_ess;
    int32_t bad_source;  // internal invariant broken (never expected)
    int32_t max_chain;   // trace: most additions one column made in k_chain this round
    int32_t max_sweeps;  // most sweeps one column took in k_chain_solve this round
    int32_t max_solve_us;  // trace: longest time one column took in k_chain_solve this round (us)
    int32_t n_cur;       // active columns of the current round (read by the round kernels)
    uint32_t round;      // rounds that did work so far
    int32_t dbg_flags;   // debug_invariants: the invariants found broken (DbgBit)
    int32_t dbg_col;     // a column or row that broke one
    int32_t bad_info[4]; // where k_chain set bad_source: column, low, previous low, step
    unsigned long long trace[S_NUM];  // folded stripes (trace output)
};

static_assert(sizeof(Counters) % 8 == 0, "Counters is cleared as 64-bit words");

// debug_invariants: one bit per property checked
enum DbgBit : int32_t {
    DBG_LOW_ROSE = 1,        // a column's low increased
    DBG_BETA_ABOVE = 2,      // beta_j > low(j) (P.5)
    DBG_BETA_ZERO = 4,       // beta_j defined but column j zero (P.3)
    DBG_PIVOT_CHANGED = 8,   // a pivot column changed, or stopped being one
    DBG_PIVOT_TABLE = 16,    // piv / low_star do not name a pivot
    DBG_DOUBLE_WRITE = 32,   // a column written twice by one kernel launch
    DBG_ESS_REMOVED = 64,    // an essential simplex left the estimate E
    DBG_FINAL = 128          // low* is not the last low seen, or beta_j > low*(j)
};

// Everything a chained addition needs about row i, in one 32-byte record
// (one load, one cache line): s >= 0 is the pivot of row i (written once,
// when column s becomes the pivot: its low is i and stays i) with its length
// k and, when short, the entries below its low; s = -1 with k = -1 marks a
// row known to be negative (compression), s = -1 with k = 0 any other row.
constexpr int kRecInline = 6;
struct __align__(32) PivRec {
    int32_t s;                // the pivot column
    int32_t k;                // its length, low included
    int32_t e[kRecInline];    // the k-1 entries below the low, ascending, when k-1 <= kRecInline
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
    // high-rate counters, striped over cache lines: stats[(id*kStripe + slot)*16]
    unsigned long long *stats;
    // arena bump pointers, one cache line each: part[p*16]; partition p owns
    // [part_base + p*part_size, part_base + (p+1)*part_size) (the last one ends at arena_cap)
    unsigned long long *part;
    unsigned long long part_base, part_size;
    PivRec *prec;      // [m] pivot records by row
    int32_t *cq;       // chain queue, kPart slices of cq_slice entries
    int32_t *cq_n;     // entries per slice, one cache line each: cq_n[p*32]; cq_n[kPart*32] = wq entries,
                       // cq_n[(kPart+1)*32] = wq2 entries, cq_n[(kPart+2)*32] = wq2 entries k_chain_solve
                       // hands to k_chain (after the wide pass has read the first ones)
    int64_t cq_slice;
    int32_t *wq;       // columns handed from the lane chain passes to the wavefront kernel
    int32_t *wq2;      // columns the first lane pass hands to the wide one (too long for its buffer)
    uint32_t *ess;     // diagnostics: the essential estimate E as a bitmask (null when off)
    // Lemma "Clearing by local compression" (null when off): the complexes
    // (batch instances, column / row ranges inst_off[k] .. inst_off[k+1]) and,
    // per instance and dimension e < kC8Dims, the first row of dimension e
    // not yet paired
    const int64_t *inst_off;
    int32_t n_inst;
    int32_t *c8_first;
    // debug_invariants (null when off): the last round's low, header and
    // state of every column, writes per column in the current kernel, and
    // the round at which each index left the essential estimate
    int32_t *dbg_low;
    int64_t *dbg_off;
    int32_t *dbg_len;
    uint8_t *dbg_state;
    int32_t *dbg_w;
    int32_t *dbg_erem;
};

// debug_invariants: one more write of column j by the current kernel
__device__ inline void dbg_write(const Dev &d, int64_t j)
{
    if (d.dbg_w) atomicAdd(&d.dbg_w[j], 1);
}

__device__ inline void dbg_fail(const Dev &d, int32_t bit, int64_t j)
{
    if (atomicOr(&d.cnt->dbg_flags, bit) == 0) d.cnt->dbg_col = (int32_t)j;
}

constexpr int kStripe = 64;
constexpr int kPart = 64;

__device__ inline void stat_add(const Dev &d, int id, unsigned long long v, unsigned slot)
{
    if (v) atomicAdd(&d.stats[((unsigned)id * kStripe + (slot & (kStripe - 1))) * 16], v);
}

// Bump allocation of n entries in partition p; -1 when the partition is full.
// n entries from partition p, or, when p is full, from the next partition
// with room (skipped by a plain read when full, so exhausted partitions take
// no further atomics); -1 when every partition is full
__device__ inline int64_t arena_alloc(const Dev &d, unsigned p, int64_t n)
{
    for (unsigned t = 0; t < (unsigned)kPart; t++) {
        const unsigned q = (p + t) & (kPart - 1);
        const unsigned long long end =
            q == kPart - 1 ? d.arena_cap : d.part_base + (unsigned long long)(q + 1) * d.part_size;
        if (t > 0 &&
            __hip_atomic_load(&d.part[q * 16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + (unsigned long long)n > end)
            continue;
        const unsigned long long o = atomicAdd(&d.part[q * 16], (unsigned long long)n);
        if (o + (unsigned long long)n <= end) return (int64_t)o;
    }
    return -1;
}

// Marks column j known negative (bit j of neg) where f holds; every lane of
// the wave calls it.  When the active lanes hold 64 consecutive columns from
// a 64-aligned base (one column per lane in index order), their bits are
// combined per 32-bit word, one atomic per word instead of one per lane.
__device__ inline void mark_neg(uint32_t *neg, int64_t j, bool f)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int64_t jb = j - lane;
    const int64_t jb0 = bcast_first64(jb);
    if (__ballot(jb != jb0) == 0 && jb0 >= 0 && (jb0 & (kWave - 1)) == 0) {
        const uint64_t bits = __ballot(f);
        const uint32_t half = lane < 32 ? (uint32_t)bits : (uint32_t)(bits >> 32);
        if (f && (lane & 31) == __ffs(half) - 1) atomicOr(&neg[(jb0 >> 5) + (lane >> 5)], half);
    } else if (f) {
        atomicOr(&neg[j >> 5], 1u << (j & 31));
    }
}

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
// given = 1: left and beta come with the boundary (a builder made them), so
// the atomics on left are skipped and beta's consequences (a known-negative
// row's record, its bit in neg) are written here instead of in k_beta.
__global__ void k_init(Dev d, int64_t nnz, int validate, int given, int compression)
{
    int top = 0;
    const int lane = threadIdx.x & (kWave - 1);
    const XcdSplit xs = xcd_split((d.m + blockDim.x - 1) / blockDim.x);
    for (int64_t t = xs.first; t < xs.end; t += xs.step) {
        const int64_t j = t * blockDim.x + threadIdx.x;
        const bool inr = j < d.m;
        const int64_t s = inr ? d.col_ptr[j] : 0, e = inr ? d.col_ptr[j + 1] : 0;
        bool bad = e < s || s < 0 || e > nnz || (j == 0 && s != 0) || e - s > 0x7FFFFFFF;
        int32_t n = bad ? 0 : (int32_t)(e - s);
        // Neighbouring columns often share their last row (VR triangles with
        // one longest edge are consecutive in the order), and would all take
        // the atomic on left at once; the first column of such a run has the
        // smallest index, so the others leave that row to it.
        const int32_t last = n > 0 ? d.rows[s + n - 1] : -1 - lane;
        const int32_t prev_last = __shfl_up(last, 1, kWave);
        const bool skip_last = lane > 0 && prev_last == last;
        const bool negb = given && compression && inr && d.beta[j] >= 0;
        if (given) mark_neg(d.neg, j, negb);  // every lane of the wave takes part
        if (!inr) continue;
        const int dj = validate && d.dim ? d.dim[j] : 0;
        // the rows four at a time: their loads (and the facets' dimensions)
        // go out together instead of one dependent chain per row
        int32_t prev = -1;
        const int32_t nscan = given && !validate ? 0 : n;  // the rows are read to check them or for left
        for (int32_t p0 = 0; p0 < nscan; p0 += 4) {
            int32_t r[4];
#pragma unroll
            for (int u = 0; u < 4; u++) r[u] = p0 + u < n ? d.rows[s + p0 + u] : 0x7FFFFFFF;
            int dr[4] = {0, 0, 0, 0};
            if (validate && d.dim) {
#pragma unroll
                for (int u = 0; u < 4; u++) dr[u] = p0 + u < n && r[u] >= 0 && (int64_t)r[u] < j ? d.dim[r[u]] : dj - 1;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (p0 + u >= n) break;
                if (r[u] <= prev || (int64_t)r[u] >= j || (validate && d.dim && dr[u] != dj - 1)) bad = true;
                prev = r[u];
            }
            if (bad) break;
            if (!given) {
#pragma unroll
                for (int u = 0; u < 4; u++)  // left only decreases
                    if (p0 + u < n && !(skip_last && p0 + u == n - 1) && (int32_t)j < d.left[r[u]])
                        atomicMin(&d.left[r[u]], (int32_t)j);
            }
        }
        if (validate && d.dim && dj < 0) bad = true;
        if (bad) { atomicExch(&d.cnt->error, 1); n = 0; }
        d.off[j] = bad ? 0 : s;
        d.len[j] = n;
        d.low[j] = n ? d.rows[s + n - 1] : -1;
        d.state[j] = n ? ST_ACTIVE : ST_ZERO;
        // row j: no pivot, not known negative (the whole 32-byte record, so
        // the stores fill whole memory sectors)
        int4 *pr = reinterpret_cast<int4 *>(&d.prec[j]);
        pr[0] = make_int4(-1, negb ? -1 : 0, 0, 0);  // with beta given: known negative rows marked here
        pr[1] = make_int4(0, 0, 0, 0);
        if (d.dim && d.dim[j] > top) top = d.dim[j];
    }
    if (d.dim) {
        for (int o = kWave / 2; o > 0; o >>= 1) top = max(top, __shfl_xor(top, o, kWave));
        // read first: once the maximum is in, almost no wave needs the atomic
        if ((threadIdx.x & (kWave - 1)) == 0 && top > *(volatile int32_t *)&d.cnt->topdim)
            atomicMax(&d.cnt->topdim, top);
    }
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
        if (compression && b >= 0) d.prec[j].k = -1;  // a negative row never gets a pivot record
        if (compression) mark_neg(d.neg, j, b >= 0);
    }
}

// ---------------------------------------------------------------- round
__global__ void k_low(Dev d, const int32_t *act)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    const int lane = threadIdx.x & (kWave - 1);
    const XcdSplit xs = xcd_split(((int64_t)nA + blockDim.x - 1) / blockDim.x);
    for (int64_t t = xs.first; t < xs.end; t += xs.step) {
        const int64_t q = t * blockDim.x + threadIdx.x;
        int32_t j = -1, i = -1 - lane;  // (distinct in every lane without a low)
        if (q < nA) {
            j = act[q];
            dbg_write(d, j);
            int32_t n = d.len[j];
            const int32_t *c = col_base(d, d.off[j]);
            // rows of known-negative simplices at the bottom of the column are
            // deleted outright (compression); the column's low is the last row left
            while (n > 0 && is_neg(d.neg, c[n - 1])) n--;
            d.len[j] = n;
            if (n == 0) {
                d.low[j] = -1;
                d.state[j] = ST_ZERO;
            } else {
                i = c[n - 1];
                d.low[j] = i;
            }
        }
        // T (the leftmost column per low) is read only for lows without a
        // known pivot (a pivot's low collides, and Phase II adds the pivot);
        // T only ever decreases, so a plain read that already shows a
        // smaller key saves the atomic, and of neighbouring positions with
        // one low (the active list ascends) only the first, the smallest
        // column, takes it
        const int32_t prev_i = __shfl_up(i, 1, kWave);
        if (i >= 0 && !(lane > 0 && prev_i == i) && d.piv[i] < 0) {
            const unsigned long long key = t_key(round, j);
            if (key < d.T[i]) atomicMin(&d.T[i], key);
        }
    }
}

// One tile of kBlock active positions per block.
__global__ void __launch_bounds__(kBlock) k_collide(Dev d, const int32_t *act, I4 *agg)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    if (blockIdx.x == 0 && threadIdx.x <= kPart + 2) d.cq_n[threadIdx.x * 32] = 0;  // the chain queues start empty
    if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt->max_chain = d.cnt->max_sweeps = d.cnt->max_solve_us = 0;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    const XcdSplit xs = xcd_split(tiles);
    for (int64_t tile = xs.first; tile < xs.end; tile += xs.step) {
    const int64_t q = tile * kBlock + threadIdx.x;
    I4 e = i4_fill(-1);
    if (q < nA) {
        const int32_t j = act[q];
        int8_t cl = kNotLive;  // the state as of this kernel, for the rest of the round
        if (d.state[j] == ST_ACTIVE) {
            const int32_t i = d.low[j];
            // a known pivot of the low makes j collide; else T decides (k_low
            // updated it for such lows this round)
            cl = (d.piv[i] >= 0 || t_decode(d.T[i], round) != j) ? 1 : 0;
            if (cl) e.v[slot_of(d, j)] = i;
        }
        d.coll[q] = cl;
    }
    I4 tot;
    block_excl_max4(e, &tot);
    if (threadIdx.x == 0) agg[tile] = tot;
    __syncthreads();
    }
}

// Exclusive max-scan of the per-block aggregates, one block of 1024 threads.
__global__ void __launch_bounds__(kScanThreads) k_scan_max4(I4 *agg, const int32_t *n_cur)
{
    const int64_t nb = ((int64_t)*n_cur + kBlock - 1) / kBlock;  // one aggregate per tile of the round
    block_seg_scan(agg, nb, i4_fill(-1), [](const I4 &x, const I4 &y) { return i4_max(x, y); });
}

// nb entries, or, when n_cur is given, one entry per tile of *n_cur columns
__global__ void __launch_bounds__(kScanThreads) k_scan_sum(int32_t *cnt, int64_t nb, const int32_t *n_cur,
                                                           int32_t *total)
{
    if (n_cur) nb = ((int64_t)*n_cur + kBlock - 1) / kBlock;
    const int32_t tot = block_seg_scan(cnt, nb, 0, [](int32_t x, int32_t y) { return x + y; });
    if (threadIdx.x == 0) *total = tot;
}

// Two independent scans of nb entries in one launch: workgroup 0 scans a
// (total to *ta), workgroup 1 scans b (total to *tb).
__global__ void __launch_bounds__(kScanThreads) k_scan_sum2(int32_t *a, int32_t *b, int64_t nb, int32_t *ta,
                                                            int32_t *tb)
{
    int32_t *x = blockIdx.x ? b : a;
    const int32_t tot = block_seg_scan(x, nb, 0, [](int32_t u, int32_t v) { return u + v; });
    if (threadIdx.x == 0) *(blockIdx.x ? tb : ta) = tot;
}

// Phase I + the beta test + clearing.
__global__ void __launch_bounds__(kBlock) k_pivots(Dev d, const int32_t *act, const I4 *agg, int compression)
{
    const int32_t nA = d.cnt->n_cur;
    const int count_beta = d.cnt->round == 0;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t q = tile * kBlock + threadIdx.x;
    I4 e = i4_fill(-1);
    int32_t j = -1, i = -1;
    bool live = false, cl = false;
    if (q < nA) {
        j = act[q];
        // liveness as k_collide saw it: columns cleared by other threads of
        // this kernel stay in the test, so the pivots found do not depend on
        // timing (a cleared column is positive and never passes it)
        const int8_t c0 = d.coll[q];
        live = c0 != kNotLive;
        if (live) {
            i = d.low[j];
            cl = c0 == 1;
            if (cl) e.v[slot_of(d, j)] = i;
        }
    }
    I4 tot;
    I4 mc = i4_max(block_excl_max4(e, &tot), agg[tile]);
    int np = 0, nb = 0;
    int64_t pb = 0;  // a new pivot: piv, its 32-byte record and the entries copied into it (+ off),
                     // low_star, its state, its row's record head, the cleared column's state
    if (live && !cl) {
        const bool by_beta = d.beta[j] == i;                  // beta_j = low(j): Thm. P.5
        const bool by_li = i > mc.v[slot_of(d, j)];           // low(j) > maxCollision
        if (by_beta || by_li) {
            d.piv[i] = j;
            PivRec r;
            r.s = j;
            r.k = d.len[j];
            pb = 4 + 32 + 8 + 4 + 1 + 4 + 2;
            if (r.k - 1 <= kRecInline) {
                const int32_t *c = col_base(d, d.off[j]);
                for (int t = 0; t < r.k - 1; t++) r.e[t] = c[t];
                pb += 4 * (int64_t)(r.k - 1);
            }
            d.prec[i] = r;
            d.state[j] = ST_PIVOT;
            dbg_write(d, j);
            d.low_star[j] = i;
            if (compression) d.prec[j].k = -1;
            if (d.state[i] == ST_ACTIVE) {
                d.state[i] = ST_CLEARED;  // clearing: sigma_i is positive
                dbg_write(d, i);
            }
            np = 1;
            nb = by_beta ? 1 : 0;
        }
    }
    if (compression) mark_neg(d.neg, j, np != 0);
    int32_t tnp;
    block_excl_sum32(np, &tnp);
    if (count_beta) {
        int32_t tnb;
        block_excl_sum32(nb, &tnb);
        if (threadIdx.x == 0) stat_add(d, S_BETAPIV, (unsigned long long)tnb, (unsigned)tile);
    }
    const int64_t bpb = block_sum64(pb);
    if (threadIdx.x == 0) {
        stat_add(d, S_NEWPIV, (unsigned long long)tnp, (unsigned)tile);
        stat_add(d, S_PBYTES, (unsigned long long)bpb, (unsigned)tile);
    }
    __syncthreads();
    }
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

// The same symmetric difference for one lane with long inputs in global
// memory: both lists are read in blocks of kMB entries held in registers
// (a block's loads are independent, so one memory latency per block rather
// than per entry, and the next block is requested while the current one is
// merged), the negative-row bits of a block fetched when it becomes current;
// the head of each list is element 0 of its block, consumed by shifting.
constexpr int kMB = 4;
__device__ inline int32_t merge_add_stream(const int32_t *__restrict__ x, int32_t nx, const int32_t *__restrict__ y,
                                           int32_t ny, int32_t *__restrict__ out, const uint32_t *neg, int compression)
{
    constexpr int32_t kEnd = 0x7FFFFFFF;
    // per list: the block being merged (b, with its negative-row flags n) and
    // the next block (q, raw entries), requested one block ahead so that its
    // entries arrive while the current block is consumed
    int32_t xb[kMB], yb[kMB], xn[kMB], yn[kMB], xq[kMB], yq[kMB];
    // Loads without conditions, so that a block's loads go out together and
    // are waited for once: positions past the end read the list's last entry
    // (kEnd is put in when the block becomes current), the end marker's flag
    // word is word 0, and the flag words are read even without compression.
    auto fetch = [&](const int32_t *a, int32_t n, int32_t pos, int32_t *q) {
        const int32_t *src = n > 0 ? a : reinterpret_cast<const int32_t *>(neg);  // an empty list reads a valid word
        const int32_t last = n > 0 ? n - 1 : 0;
#pragma unroll
        for (int u = 0; u < kMB; u++) q[u] = src[min(pos + u, last)];
    };
    auto current = [&](const int32_t *q, int32_t n, int32_t pos, int32_t *b) {
#pragma unroll
        for (int u = 0; u < kMB; u++) b[u] = pos + u < n ? q[u] : kEnd;
    };
    // a block's flag words (loaded), then its flags (the words used)
    auto words = [&](const int32_t *b, uint32_t *w) {
#pragma unroll
        for (int u = 0; u < kMB; u++) w[u] = neg[(b[u] != kEnd ? b[u] : 0) >> 5];
    };
    auto flags = [&](const int32_t *b, const uint32_t *w, int32_t *nb) {
#pragma unroll
        for (int u = 0; u < kMB; u++)
            nb[u] = (compression && b[u] != kEnd) ? (int32_t)((w[u] >> (b[u] & 31)) & 1u) : 0;
    };
    uint32_t wx[kMB], wy[kMB];
    fetch(x, nx, 0, xq);
    fetch(y, ny, 0, yq);
    current(xq, nx, 0, xb);
    current(yq, ny, 0, yb);
    words(xb, wx);
    words(yb, wy);
    __builtin_amdgcn_sched_barrier(0);  // the flag words go out before the next blocks: loads complete in order
    fetch(x, nx, kMB, xq);
    fetch(y, ny, kMB, yq);
    __builtin_amdgcn_sched_barrier(0);
    flags(xb, wx, xn);
    flags(yb, wy, yn);
    int32_t xp = 2 * kMB, yp = 2 * kMB, k = 0;  // the next positions to request
    while (xb[0] != kEnd || yb[0] != kEnd) {
        const int32_t u = xb[0], v = yb[0];
        if (u < v) {
            if (!xn[0]) out[k++] = u;
        } else if (v < u) {
            if (!yn[0]) out[k++] = v;
        }  // equal: 1 + 1 = 0
        if (u <= v) {
#pragma unroll
            for (int t = 0; t < kMB - 1; t++) {
                xb[t] = xb[t + 1];
                xn[t] = xn[t + 1];
            }
            xb[kMB - 1] = kEnd;
            xn[kMB - 1] = 0;
            if (xb[0] == kEnd && xp - kMB < nx) {
                current(xq, nx, xp - kMB, xb);
                uint32_t w[kMB];
                words(xb, w);
                __builtin_amdgcn_sched_barrier(0);
                fetch(x, nx, xp, xq);
                __builtin_amdgcn_sched_barrier(0);
                flags(xb, w, xn);
                xp += kMB;
            }
        }
        if (v <= u) {
#pragma unroll
            for (int t = 0; t < kMB - 1; t++) {
                yb[t] = yb[t + 1];
                yn[t] = yn[t + 1];
            }
            yb[kMB - 1] = kEnd;
            yn[kMB - 1] = 0;
            if (yb[0] == kEnd && yp - kMB < ny) {
                current(yq, ny, yp - kMB, yb);
                uint32_t w[kMB];
                words(yb, w);
                __builtin_amdgcn_sched_barrier(0);
                fetch(y, ny, yp, yq);
                __builtin_amdgcn_sched_barrier(0);
                flags(yb, w, yn);
                yp += kMB;
            }
        }
    }
    return k;
}

// The column a colliding active column j adds this round (-1: none): the
// known pivot of its low, else (variant 0) the leftmost column with that low
// unless it was cleared.
__device__ inline int32_t xor_source(const Dev &d, int32_t j, int variant, uint32_t round)
{
    const int32_t i = d.low[j];
    int32_t s = d.piv[i];
    if (s < 0 && variant == 0) {
        s = t_decode(d.T[i], round);
        if (s == j || (s >= 0 && d.state[s] == ST_CLEARED)) s = -1;
    }
    return s;
}

// ------------------------------------------------ priority with a budget
// Sec. 3.4: with fewer processors than colliding columns only some of them
// add in a round, chosen by a priority.  Each colliding column with a source
// gets a key h in [0, 255] (larger first): 0 for all (column order), 1 for
// the columns known negative (Sec. 3.4 "N(j) and Neg"), or the size of its
// set N -- the colliding columns with its low, served by one pivot --
// capped at 255 (Sec. 3.4 "sets N(j) with large cardinality").  With t the
// largest key at which the columns of key >= t reach the budget, the columns
// of key > t add, those of key t add in column order up to what is left, and
// the rest wait (their collision flag is cleared for this round).
constexpr int kBudKeys = 256;

__device__ inline bool bud_target(const Dev &d, const int32_t *act, int64_t q, int variant, uint32_t round,
                                  bool waiting = false)
{
    const int32_t j = act[q];
    const int8_t c = d.coll[q];
    return d.state[j] == ST_ACTIVE && (c == 1 || (waiting && c == kWaits)) && xor_source(d, j, variant, round) >= 0;
}

__device__ inline int bud_key(const Dev &d, int32_t j, int prio, const int32_t *ncount)
{
    if (prio == 2) return d.beta[j] >= 0 ? 1 : 0;
    if (prio == 1) return min(ncount[d.low[j]], kBudKeys - 1);
    return 0;
}

// |N| per low (priority 1): one count per colliding column with a source;
// sign = -1 takes them back out after the round's choice (the waiting
// columns included)
__global__ void __launch_bounds__(kBlock) k_bud_ncount(Dev d, const int32_t *act, int variant, int32_t *ncount,
                                                       int sign)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < nA; q += (int64_t)gridDim.x * kBlock)
        if (bud_target(d, act, q, variant, round, sign < 0)) atomicAdd(&ncount[d.low[act[q]]], sign);
}

// key histogram (hist[kBudKeys + 2] is zeroed by the previous round's choice)
__global__ void __launch_bounds__(kBlock) k_bud_hist(Dev d, const int32_t *act, int variant, int prio,
                                                     const int32_t *ncount, int32_t *hist)
{
    __shared__ int32_t s_h[kBudKeys];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < nA; q += (int64_t)gridDim.x * kBlock)
        if (bud_target(d, act, q, variant, round)) atomicAdd(&s_h[bud_key(d, act[q], prio, ncount)], 1);
    __syncthreads();
    if (s_h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], s_h[threadIdx.x]);
}

// the threshold key t (hist[kBudKeys]) and the budget left for key t
// (hist[kBudKeys + 1]); the histogram is cleared for the next round
__global__ void k_bud_thresh(int32_t *hist, int32_t budget)
{
    if (threadIdx.x != 0) return;
    int32_t above = 0, t = -1;  // t = -1: every column fits the budget
    for (int h = kBudKeys - 1; h >= 0; h--) {
        if (above + hist[h] >= budget) {
            t = h;
            break;
        }
        above += hist[h];
    }
    for (int h = 0; h < kBudKeys; h++) hist[h] = 0;
    hist[kBudKeys] = t;
    hist[kBudKeys + 1] = budget - above;  // ranks of key t below this add (all of them when the total fits)
}

// per tile: colliding columns of key t
__global__ void __launch_bounds__(kBlock) k_bud_count(Dev d, const int32_t *act, int variant, int prio,
                                                      const int32_t *ncount, const int32_t *hist, int32_t *tcnt)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    const int32_t t = hist[kBudKeys];
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t q = tile * kBlock + threadIdx.x;
        const int tie = (q < nA && bud_target(d, act, q, variant, round) && bud_key(d, act[q], prio, ncount) == t);
        int32_t tot;
        block_excl_sum32(tie, &tot);
        if (threadIdx.x == 0) tcnt[tile] = tot;
        __syncthreads();
    }
}

// the choice: colliding columns past the budget wait
__global__ void __launch_bounds__(kBlock) k_bud_apply(Dev d, const int32_t *act, int variant, int prio,
                                                      const int32_t *ncount, const int32_t *hist,
                                                      const int32_t *toff)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    const int32_t t = hist[kBudKeys], left = hist[kBudKeys + 1];
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t q = tile * kBlock + threadIdx.x;
        const bool tg = q < nA && bud_target(d, act, q, variant, round);
        const int key = tg ? bud_key(d, act[q], prio, ncount) : -1;
        const int tie = key == t;
        int32_t tot;
        const int32_t r = toff[tile] + block_excl_sum32(tie, &tot);
        if (tg && (key < t || (tie && r >= left))) d.coll[q] = kWaits;
        __syncthreads();
    }
}

// Phase II, first addition of every colliding column (one lane per
// column: most columns are a few entries long).  A column that may keep
// adding known pivots (chaining) and whose new low has one is queued for
// k_chain.
constexpr int32_t kXorDefer = 128;  // merges longer than this go to the chain kernels in tail rounds

__global__ void __launch_bounds__(kBlock) k_xor(Dev d, const int32_t *act, int variant, int compression, int chain,
                                                int tail)
{
    const int32_t nA = d.cnt->n_cur;
    const uint32_t round = d.cnt->round;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    // strided: per-tile work varies widely (long merges cluster), so fixed parts would leave a tail
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t q = tile * kBlock + threadIdx.x;
    int32_t j = -1, s = -1, tlen = 0, slen = 0;
    int64_t toff = 0, soff = 0;
    bool target = false, push = false;
    if (q < nA) {
        j = act[q];
        if (d.state[j] == ST_ACTIVE && d.coll[q] == 1) {
            s = xor_source(d, j, variant, round);
            if (s >= 0) {
                target = true;
                toff = d.off[j];
                tlen = d.len[j];
                soff = d.off[s];
                slen = d.len[s];
                if (s >= j) atomicExch(&d.cnt->bad_source, 1);
                // a long merge with the low's known pivot in a round where every
                // column chains: it is the chain's first step, left to the chain
                // kernels (one lane merging thousands of entries would hold the round)
                if (chain && nA < tail && tlen + slen > kXorDefer && d.piv[d.low[j]] == s) {
                    target = false;
                    push = true;
                }
            }
        }
    }
    // block-aggregated arena allocation (at most tlen + slen - 2 entries
    // survive), from this block's arena partition
    __shared__ int64_t s_base;
    const int64_t need = target ? (int64_t)tlen + slen : 0;
    const int64_t excl = block_excl_sum64(need);
    const int64_t btot = block_sum64(need);
    if (threadIdx.x == 0) s_base = btot ? arena_alloc(d, (unsigned)tile, btot) : 0;
    __syncthreads();
    const int64_t bbase = s_base;
    if (threadIdx.x == 0 && bbase < 0) atomicExch(&d.cnt->overflow, 1);  // once per block: one flag for all
    if (target && bbase < 0) target = false;  // the column stays as it is this round
    int64_t adds = 0, xe = 0, by = q < nA ? 6 : 0, ab = 0;  // act, state, coll
    if (target) {
        const int64_t dst = bbase + excl;
        int32_t *out = d.arena + dst;
        const int32_t k = merge_add_stream(col_base(d, toff), tlen, col_base(d, soff), slen, out, d.neg, compression);
        adds = 1;
        xe = (int64_t)tlen + slen;
        by += 42 + 4 * ((int64_t)tlen + slen + k) + 16;  // headers, low, piv/T, beta, dim; data in and out
        ab = 4 * ((int64_t)tlen + slen + k);
        dbg_write(d, j);
        d.off[j] = dst | (int64_t)kArenaBit;
        d.len[j] = k;
        if (k == 0) {
            d.low[j] = -1;
            d.state[j] = ST_ZERO;  // column j is positive
        } else {
            const int32_t nl = out[k - 1];
            d.low[j] = nl;
            const bool chainable = chain && (d.beta[j] >= 0 || (d.dim && d.dim[j] == d.cnt->topdim) || nA < tail);
            push = chainable && d.piv[nl] >= 0;
        }
    }
    // block-aggregated push onto this block's slice of the chain queue
    __shared__ int32_t s_q;
    int32_t npush;
    const int32_t qpos = block_excl_sum32(push ? 1 : 0, &npush);
    const unsigned qp = (unsigned)tile & (kPart - 1);
    if (threadIdx.x == 0) s_q = npush ? atomicAdd(&d.cq_n[qp * 32], npush) : 0;
    __syncthreads();
    if (push) d.cq[(int64_t)qp * d.cq_slice + s_q + qpos] = j;
    const int64_t badds = block_sum64(adds);
    const int64_t bxe = block_sum64(xe);
    const int64_t bby = block_sum64(by);
    const int64_t bab = block_sum64(ab);
    if (threadIdx.x == 0) {
        stat_add(d, S_XBYTES, (unsigned long long)bby, (unsigned)tile);
        stat_add(d, S_ABYTES_XOR, (unsigned long long)bab, (unsigned)tile);
        stat_add(d, S_ADDS, (unsigned long long)badds, (unsigned)tile);
        stat_add(d, S_XE, (unsigned long long)bxe, (unsigned)tile);
    }
    __syncthreads();
    }
}

// ---------------------------------------------------------------- chaining
constexpr int kChainWaves = 4;
constexpr int kCapW = 1520;  // LDS entries per working buffer (two per wave); two blocks fit a CU
constexpr int kCapS = 512;   // LDS entries for the pivot column

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int32_t lower_bound_i32(const int32_t *a, int32_t n, int32_t x)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Everything a chain step needs about row i: its record, one load.
struct Look {
    int32_t s, k;  // k < 0: the row is known negative
    int32_t e[kRecInline];
};

__device__ inline Look look_up(const Dev &d, int32_t i)
{
    const PivRec rec = d.prec[i];
    Look r;
    r.s = rec.s;
    r.k = rec.k;
#pragma unroll
    for (int t = 0; t < kRecInline; t++) r.e[t] = rec.e[t];
    return r;
}

// median of three (selected to v_med3_i32 from this min/max form)
__device__ __forceinline__ int32_t med3_i32(int32_t a, int32_t b, int32_t c)
{
    return max(min(a, b), min(max(a, b), c));
}

__device__ inline int32_t wave_sum32(int32_t x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ inline uint32_t wave_or32(uint32_t x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x |= __shfl_xor(x, o, kWave);
    return x;
}

// Lane chaining: one lane per queued column.  The column is W = B xor P:
// B, its sorted base, sits in a per-lane LDS buffer (entry e of lane t at
// sL[e * kLaneThreads + t], so a wave's lanes hit consecutive banks) and
// only loses entries at its top; P, at most kLaneP pending toggles, lives in
// registers in descending order (P[0] is its largest entry, -1 = empty) and
// is updated by fixed compare-select networks.  A step removes the low and
// toggles the pivot's entries below it (at most kRecInline, from its record)
// into P, so its cost does not depend on the column's length; B and P are
// merged in place when P is full.  Lanes work independently: each loop
// iteration every busy lane takes one step, and a lane whose chain ends
// writes its column back merged into the arena (from a chunk its wave
// claimed) and takes the wave's next queued column, so short and long chains
// share a wave without idling it.  A pivot with more entries than its record
// holds is merged from its stored column into B in the merge phase, when B
// has room for the result.  Columns that chain longer than the step cap go on
// to the wavefront kernel.  The kernel runs in
// two passes: the first (k_chain_lane, kLaneCap = 39 entries per lane, two waves per
// block) takes the round's queued columns and hands those that outgrow its
// buffer to the second (k_chain_wide, 80 entries per lane, one wave per
// block: fewer lanes per CU, for the fewer long columns); what outgrows that
// goes to the wavefront kernel too.  Both passes wait on one record load per
// step, so their speed follows the lanes resident per CU: the buffer sizes
// are those at which LDS allows as many waves as the registers do.
constexpr int kLaneThreads = 128;
constexpr int kWideThreads = 64;
constexpr int kWideCap = 80;
constexpr int kLaneP = 16;
// The grid, the step caps and the refill / merge thresholds come from the
// context's pms_tuning.  A lane hands a longer chain to a wavefront, whose
// steps are faster: with many queued columns (at least tn.lane_many) lanes
// keep chains longer (throughput, tn.lane_steps), with few the long chains
// move on early (they are the critical path, tn.lane_steps_few).
constexpr int kLaneChunk = 1024;   // arena entries a wave claims at a time for its write-backs

template <int kCap, int kThreads, bool kWide, bool kTrace>
__device__ __forceinline__ void lane_chain(const Dev &d, int compression, const pms_tuning &tn)
{
    constexpr bool trace = kTrace;  // the trace counters exist only in the traced instantiation
    __shared__ int32_t sL[kCap * kThreads];
    __shared__ int32_t s_pre[kPart];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const uint64_t below = lane ? (~0ull >> (kWave - lane)) : 0ull;  // the lanes under this one
#define LW(e) sL[(e) * kThreads + tid]
    int32_t total;
    if (!kWide) {  // the round's queue: kPart slices
        if (tid < kPart) s_pre[tid] = d.cq_n[tid * 32];
        __syncthreads();
        if (tid == 0)
            for (int p = 1; p < kPart; p++) s_pre[p] += s_pre[p - 1];  // inclusive prefix of the slice sizes
        __syncthreads();
        total = s_pre[kPart - 1];
    } else {  // the first pass's hand-overs, one list
        total = d.cq_n[(kPart + 1) * 32];
    }
    const int32_t step_cap = total >= tn.lane_many ? tn.lane_steps : tn.lane_steps_few;
    // entries a lane's buffer may hold: the first pass may use less than its
    // LDS room (tn.lane_cap), handing longer columns to the wide pass
    const int32_t cap = kWide ? kCap : min(kCap, tn.lane_cap);
    const unsigned gwave = blockIdx.x * (kThreads / kWave) + (unsigned)bcast_first(tid / kWave);
    // per-lane counts (32 bits: a lane makes a few thousand steps per launch;
    // the wave sums below are 64-bit)
    uint32_t adds = 0, xe = 0, by = 0, bails = 0, towide = 0, ab = 0;
    int64_t tsl = 0, tg16 = 0, tg32 = 0;
    // wave state (uniform): unassigned tasks [tb, te) and the arena chunk [cb, ce);
    // the wave's tasks are the 64-task chunks gwave, gwave + nwaves, ... (shared
    // by the whole grid: chain lengths vary, and fixed parts would idle at the end)
    const int64_t nwaves = (int64_t)gridDim.x * (kThreads / kWave);
    int64_t kc = gwave;
    int32_t tb = 0, te = 0;
    bool drained = false;
    long long cb = 0, ce = 0;
    // lane state
    int32_t j = -1, LB = 0, np = 0, i = -1, steps = 0;
    int32_t p[kLaneP];
#pragma unroll
    for (int u = 0; u < kLaneP; u++) p[u] = -1;
    bool dirty = false;
    Look lk{};
    // the low of W: an equal pair on top of P cancels (1 + 1 = 0), and so do
    // equal tops of B and P.  Not unrolled: peeled copies of this loop turn
    // into chains of register copies of P on the common path.
    auto top = [&]() -> int32_t {
#pragma clang loop unroll(disable)
        for (;;) {
            if (p[0] >= 0 && p[0] == p[1]) {
#pragma unroll
                for (int u = 0; u < kLaneP - 2; u++) p[u] = p[u + 2];
                p[kLaneP - 2] = p[kLaneP - 1] = -1;
                np -= 2;
                continue;
            }
            const int32_t bt = LB > 0 ? LW(LB - 1) : -1;
            if (p[0] != bt) return p[0] > bt ? p[0] : bt;
            if (bt < 0) return -1;
#pragma unroll
            for (int u = 0; u < kLaneP - 1; u++) p[u] = p[u + 1];
            p[kLaneP - 1] = -1;
            np--;
            LB--;
        }
    };
    // P := P + {x}: x is inserted in order even when P holds it already, the
    // equal entries then sit side by side and cancel when they reach the top
    // of P or are merged (P is W's toggles counted mod 2).  Slot u of the
    // result is the median of x and the old slots u and u-1 (x clamped into
    // [P[u], P[u-1]]): one v_med3 per slot, updated from the bottom up so P
    // stays in the same registers.  x = -2 (above the -1 padding, below
    // every row) leaves P as it is, so lanes with fewer toggles run the same
    // instructions.
    auto toggle = [&](int32_t x) {
#pragma unroll
        for (int u = kLaneP - 1; u >= 1; u--) p[u] = med3_i32(p[u], x, p[u - 1]);
        p[0] = max(p[0], x);
        np += x < 0 ? 0 : 1;
    };
    // B := B xor P in place, from the top down (needs LB + np <= cap);
    // cancelled pairs close the gap by moving the merged top part down
    auto flush = [&]() {
        int32_t r = LB - 1, w = LB + np - 1, c = 0;
        bool pair = false;  // p[u] is the second of an equal pair of P, skipped with the first
#pragma unroll
        for (int u = 0; u < kLaneP; u++) {
            if (u < np && pair) {
                pair = false;
            } else if (u < np && u + 1 < np && p[u] == p[(u + 1) & (kLaneP - 1)]) {
                pair = true;  // x + x = 0: neither enters B (counted like a cancellation)
                c++;
            } else if (u < np) {
                const int32_t x = p[u];
                int32_t y = r >= 0 ? LW(r) : -1;
                while (y > x) {
                    LW(w) = y;
                    w--;
                    r--;
                    y = r >= 0 ? LW(r) : -1;
                }
                if (y == x) {  // 1 + 1 = 0
                    r--;
                    c++;
                } else {
                    LW(w) = x;
                    w--;
                }
            }
        }
        const int32_t topi = LB + np - 1;
        if (c)
            for (int32_t e = w + 1; e <= topi; e++) LW(e - 2 * c) = LW(e);
        LB = LB + np - 2 * c;
#pragma unroll
        for (int u = 0; u < kLaneP; u++) p[u] = -1;
        np = 0;
    };
    bool fin = true, bail = false;  // fin: no column in progress (finished, or never given one)
    bool roomb = false;             // the bail is for want of buffer room (first pass: to the wide one)
    bool wantf = false;             // P is full: this lane waits for a merge phase
    bool wantl = false;             // a long pivot: merged from its column in the merge phase
    int64_t titer = 0, trefill = 0, tflush = 0, tbusy = 0;  // trace: wave iterations, phases, busy lanes
    int64_t tlong = 0;                                       // trace: long-pivot steps
    int64_t ttog = 0, ttround = 0;                           // trace: toggles (per lane), toggle rounds (per wave)
    for (;;) {
        if (trace) titer++;
        // finished lanes are written back and refilled together, once at
        // least tn.lane_refill of them (or every lane) are waiting: the wave-wide
        // work is shared by many columns
        const uint64_t finm = __ballot(fin);
        const bool more = !(drained && tb >= te);  // tasks left for this wave
        const uint64_t want = __ballot(fin && (j >= 0 || more));
        if (__popcll(want) >= tn.lane_refill || finm == ~0ull) {
            if (trace) trefill++;
            // write back (B and P merged from the bottom up) from the wave's arena chunk
            const bool wr = fin && j >= 0 && dirty;
            const int32_t need = wr ? LB + np : 0;
            const int32_t incl = wave_incl_sum32(need);
            const int32_t wtot = bcast_lane(incl, kWave - 1);
            if (wtot > 0 && ce - cb < wtot) {
                const int32_t claim = wtot > kLaneChunk ? wtot : kLaneChunk;
                long long o = 0;
                if (lane == 0) o = arena_alloc(d, gwave, claim);
                o = bcast_first64(o);
                if (o < 0) {
                    cb = ce = 0;
                } else {
                    cb = o;
                    ce = o + claim;
                }
            }
            const bool room = wtot == 0 || ce - cb >= wtot;
            // progress dropped; the stored columns stay valid (one flag per wave)
            if (!room && lane == 0) atomicExch(&d.cnt->overflow, 1);
            if (wr && room) {
                dbg_write(d, j);
                const long long o = cb + incl - need;
                int32_t *out = d.arena + o;
                int32_t w = 0, r = 0;
                bool pair = false;  // as in the merge phase: equal pairs of P cancel
#pragma unroll
                for (int u = kLaneP - 1; u >= 0; u--) {
                    if (u < np && pair) {
                        pair = false;
                    } else if (u < np && u >= 1 && p[u] == p[(u + kLaneP - 1) & (kLaneP - 1)]) {
                        pair = true;
                    } else if (u < np) {
                        const int32_t x = p[u];
                        while (r < LB && LW(r) < x) out[w++] = LW(r++);
                        if (r < LB && LW(r) == x) r++;  // 1 + 1 = 0
                        else out[w++] = x;
                    }
                }
                while (r < LB) out[w++] = LW(r++);
                if (w > 0) {
                    d.off[j] = o | (int64_t)kArenaBit;
                    d.len[j] = w;
                    d.low[j] = out[w - 1];
                } else {
                    d.len[j] = 0;
                    d.low[j] = -1;
                    d.state[j] = ST_ZERO;  // column j is positive
                }
                by += 4u * (uint32_t)w + 16u;
            }
            if (room) cb += wtot;
            // hand the bailing columns over to the wavefront kernel, or (first
            // pass, too long for the buffer) to the wide pass
            const uint64_t bal = __ballot(fin && bail && !roomb);
            if (bal) {
                int32_t qb = 0;
                if (lane == 0) qb = atomicAdd(&d.cq_n[kPart * 32], (int32_t)__popcll(bal));
                qb = bcast_first(qb);
                if (fin && bail && !roomb) d.wq[qb + __popcll(bal & below)] = j;
                bails += (fin && bail && !roomb) ? 1 : 0;
            }
            if (!kWide) {
                const uint64_t balw = __ballot(fin && bail && roomb);
                if (balw) {
                    int32_t qb = 0;
                    if (lane == 0) qb = atomicAdd(&d.cq_n[(kPart + 1) * 32], (int32_t)__popcll(balw));
                    qb = bcast_first(qb);
                    if (fin && bail && roomb) d.wq2[qb + __popcll(balw & below)] = j;
                    towide += (fin && bail && roomb) ? 1 : 0;
                }
            }
            if (fin) {
                j = -1;
                bail = false;
                roomb = false;
            }
            // refill: the wave's next tasks to the free lanes
            uint64_t idle = finm;
            for (int pass = 0; pass < 2 && idle && !(drained && tb >= te); pass++) {
                if (tb >= te && !drained) {  // the wave's next chunk of 64 tasks
                    const int64_t nb = kc * kWave;
                    kc += nwaves;
                    if (nb >= total) {
                        drained = true;
                        break;
                    }
                    tb = (int32_t)nb;
                    te = (int32_t)min(nb + kWave, (int64_t)total);
                }
                const int32_t rank = __popcll(idle & below);
                const int32_t avail = te - tb;
                if (((idle >> lane) & 1ull) && rank < avail) {
                    const int32_t t = tb + rank;
                    if (kWide) {
                        j = d.wq2[t];
                    } else {
                        int lo = 0, hi = kPart - 1;  // first slice whose prefix exceeds t
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (s_pre[mid] > t) hi = mid;
                            else lo = mid + 1;
                        }
                        const int32_t before = lo > 0 ? s_pre[lo - 1] : 0;
                        j = d.cq[(int64_t)lo * d.cq_slice + (t - before)];
                    }
                    fin = false;
                }
                tb += min(__popcll(idle), avail);
                idle = __ballot(fin);
            }
            if (__ballot(!fin) == 0) break;  // every lane free and the queue drained
            // load the new columns (all new lanes at once, 8 loads in flight each)
            const bool fresh = ((finm >> lane) & 1ull) && !fin;
            if (fresh) {
                const int32_t L = d.len[j];
                by += 16u + 4u * (uint32_t)L;
                np = 0;
#pragma unroll
                for (int u = 0; u < kLaneP; u++) p[u] = -1;
                dirty = false;
                wantf = false;
                wantl = false;
                steps = 0;
                if (L > cap) {
                    bail = true;  // too long for a lane: straight to the next pass
                    roomb = !kWide;
                    fin = true;
                    LB = 0;
                } else {
                    const int32_t *g = col_base(d, d.off[j]);
                    for (int32_t e0 = 0; e0 < L; e0 += 8) {
                        int32_t v[8];
#pragma unroll
                        for (int u = 0; u < 8; u++) v[u] = e0 + u < L ? g[e0 + u] : 0;
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            if (e0 + u < L) LW(e0 + u) = v[u];
                    }
                    LB = L;
                    i = top();
                    lk = look_up(d, i >= 0 ? i : 0);
                }
            }
        }
        // lanes whose P is full are merged together, once enough of them
        // wait (the merge loop's trip count varies from lane to lane)
        {
            const uint64_t busy = __ballot(!fin);
            const uint64_t nf = __ballot(!fin && (wantf || wantl));
            if (trace) tbusy += __popcll(busy);
            if (nf && (__popcll(nf) >= tn.lane_flush || nf == busy)) {
                if (trace) tflush++;
                if (wantf) {
                    flush();
                    wantf = false;
                }
                if (wantl) {
                    // a long pivot: W = B now, its top is the low.  Remove it
                    // and merge the pivot's entries below its low (read from
                    // the stored column) into B, from the top down
                    wantl = false;
                    if (LB <= 0 || LW(LB - 1) != i) {
                        atomicExch(&d.cnt->bad_source, 3);
                        dirty = false;
                        fin = true;
                    } else {
                        LB--;
                        const int32_t kk = lk.k - 1;
                        const int32_t *g = col_base(d, d.off[lk.s]);
                        int32_t r = LB - 1, w = LB + kk - 1, c = 0;
                        for (int32_t q0 = kk - 1; q0 >= 0; q0 -= 8) {
                            int32_t v[8];
#pragma unroll
                            for (int u = 0; u < 8; u++) v[u] = g[max(q0 - u, 0)];
#pragma unroll
                            for (int u = 0; u < 8; u++) {
                                if (q0 - u >= 0) {
                                    const int32_t x = v[u];
                                    int32_t y = r >= 0 ? LW(r) : -1;
                                    while (y > x) {
                                        LW(w) = y;
                                        w--;
                                        r--;
                                        y = r >= 0 ? LW(r) : -1;
                                    }
                                    if (y == x) {  // 1 + 1 = 0
                                        r--;
                                        c++;
                                    } else {
                                        LW(w) = x;
                                        w--;
                                    }
                                }
                            }
                        }
                        const int32_t topi = LB + kk - 1;
                        if (c)
                            for (int32_t e = w + 1; e <= topi; e++) LW(e - 2 * c) = LW(e);
                        steps++;
                        adds++;
                        xe += (uint32_t)(LB + kk + 2);
                        by += 44u + 4u * (uint32_t)lk.k;
                        ab += 4u * (uint32_t)((LB + 1) + lk.k + (LB + kk - 2 * c));
                        if (trace) {
                            tsl += LB + 1;
                            tlong++;
                        }
                        LB = LB + kk - 2 * c;
                        dirty = true;
                        const int32_t ni = top();
                        if (ni >= i) {  // the low must drop; stop rather than spin
                            atomicExch(&d.cnt->bad_source, 3);
                            dirty = false;
                            fin = true;
                        } else {
                            i = ni;
                            if (i >= 0) lk = look_up(d, i);
                        }
                    }
                }
            }
        }
        // one step for every lane with a column in progress.  The pending-set
        // updates are selects run by every lane (per-lane branches around
        // them cost more in exec-mask handling and register copies than the
        // selects themselves); only the search for the next low branches.
        {
            const bool act = !fin && !wantf && !wantl;
            const int32_t kk = lk.k - 1;
            const bool has = act && i >= 0;
            const bool piv = has && lk.s >= 0;
            const bool del = has && lk.s < 0 && compression && lk.k < 0;  // a known-negative row: delete it
            // W is zero, or no pivot owns its low: the chain ends here
            if (act && !piv && !del) fin = true;
            // a longer pivot than its record holds is merged from its stored
            // column in the wave's next merge phase (after P's merge), when B
            // has room for the result
            const bool lng = piv && kk > kRecInline;
            const bool capx = piv && steps >= step_cap;
            const bool roomx = piv && !capx && (lng ? LB + np + kk - 1 > cap : (np + kk > kLaneP && LB + np > cap));
            const bool over = capx || roomx;
            if (over) {
                bail = true;
                roomb = !kWide && roomx;  // only room is lacking
                fin = true;
            }
            const bool full = piv && !over && (lng || np + kk > kLaneP);
            if (full) {  // wait for the wave's next merge phase
                wantf = np > 0 || !lng;
                wantl = lng;
            }
            const bool go = piv && !over && !full;
            if (go) {
                steps++;
                adds++;
                xe += (uint32_t)(LB + np + kk + 1);
                by += 32;
                ab += 4u * (uint32_t)(2 * (LB + np + kk + 1) - 2);
                if (trace) {
                    tsl += LB + np;
                    tg16 += LB + np > 16 ? 1 : 0;
                    tg32 += LB + np > 32 ? 1 : 0;
                }
            }
            // the low leaves W: from P when it is P's top, else from B's top
            const bool rm = go || del;
            const bool fromp = rm && p[0] == i;
#pragma unroll
            for (int u = 0; u < kLaneP; u++) p[u] = fromp ? (u + 1 < kLaneP ? p[u + 1] : -1) : p[u];
            np -= fromp ? 1 : 0;
            LB -= (rm && !fromp) ? 1 : 0;
            // the pivot's entries below the low, as many rounds as the wave's
            // longest record needs
#pragma unroll
            for (int q = 0; q < kRecInline; q++) {
                if (__ballot(go && q < kk) == 0) break;
                if (trace) {
                    ttog += go && q < kk ? 1 : 0;
                    ttround++;
                }
                toggle(go && q < kk ? lk.e[q] : -2);
            }
            if (rm) {
                dirty = true;
                const int32_t ni = top();
                if (ni >= i) {  // the low must drop; stop rather than spin
                    atomicExch(&d.cnt->bad_source, 3);
                    dirty = false;
                    fin = true;
                } else {
                    i = ni;
                    if (i >= 0) lk = look_up(d, i);
                }
            }
        }
    }
#undef LW
    // counters: lane sums -> one atomic per wave
    const int64_t wadds = wave_incl_sum64((int64_t)adds), wxe = wave_incl_sum64((int64_t)xe),
                  wby = wave_incl_sum64((int64_t)by), wb = wave_incl_sum64((int64_t)bails),
                  wab = wave_incl_sum64((int64_t)ab);
    const int64_t wsl = trace ? wave_incl_sum64(tsl) : 0, wg16 = trace ? wave_incl_sum64(tg16) : 0,
                  wg32 = trace ? wave_incl_sum64(tg32) : 0, wtw = trace ? wave_incl_sum64((int64_t)towide) : 0,
                  wlg = trace ? wave_incl_sum64(tlong) : 0, wtg = trace ? wave_incl_sum64(ttog) : 0;
    if (lane == kWave - 1) {
        stat_add(d, S_ADDS, (unsigned long long)wadds, gwave);
        stat_add(d, S_XE, (unsigned long long)wxe, gwave);
        stat_add(d, kWide ? S_WBYTES : S_LBYTES, (unsigned long long)wby, gwave);
        stat_add(d, kWide ? S_ABYTES_WIDE : S_ABYTES_LANE, (unsigned long long)wab, gwave);
        if (trace) {
            stat_add(d, kWide ? S_T_WIDE : S_T_LANE, (unsigned long long)wadds, gwave);
            stat_add(d, S_T_TOWIDE, (unsigned long long)wtw, gwave);
            if (!kWide) {  // wave-uniform counts, once per wave
                stat_add(d, S_T_LITER, (unsigned long long)titer, gwave);
                stat_add(d, S_T_LREFILL, (unsigned long long)trefill, gwave);
                stat_add(d, S_T_LFLUSH, (unsigned long long)tflush, gwave);
                stat_add(d, S_T_LBUSY, (unsigned long long)tbusy, gwave);
            }
            stat_add(d, S_T_BAIL, (unsigned long long)wb, gwave);
            stat_add(d, S_T_LSUML, (unsigned long long)wsl, gwave);
            stat_add(d, S_T_LGT16, (unsigned long long)wg16, gwave);
            stat_add(d, S_T_LGT32, (unsigned long long)wg32, gwave);
            stat_add(d, S_T_LLONG, (unsigned long long)wlg, gwave);
            stat_add(d, S_T_LTOG, (unsigned long long)wtg, gwave);
            if (!kWide) stat_add(d, S_T_LTROUND, (unsigned long long)ttround, gwave);
        }
    }
}

template <bool kTrace>
__global__ void __launch_bounds__(kLaneThreads) k_chain_lane(Dev d, int compression, pms_tuning tn)
{
    lane_chain<kLaneCap, kLaneThreads, false, kTrace>(d, compression, tn);
}

template <bool kTrace>
__global__ void __launch_bounds__(kWideThreads) k_chain_wide(Dev d, int compression, pms_tuning tn)
{
    lane_chain<kWideCap, kWideThreads, true, kTrace>(d, compression, tn);
}

// Wavefront chaining, for the columns the lane kernel hands over (long
// chains, long columns, long pivots).  The working column is W = B xor P:
// B, a sorted base array (in LDS while it fits, else in the arena), only
// ever loses entries at its top; P, a set of at most 64 pending row
// toggles, lives one entry per lane (stored as row + 1, 0 = empty).  A step
// with a short pivot removes the low and toggles the pivot's entries below
// it into P, one ballot and one lane select per entry, so its cost does not
// grow with the length of W; one wave-wide max finds the next low.  The
// pivot records of every P entry and of the 64 topmost B entries are copied
// ahead, memory to LDS without passing through registers, into one LDS slot
// per lane: the next low's record is an LDS read, at most one load latency
// after the step that inserted it.  Known-negative lows are deleted while
// the next low is searched.  B and P are merged into a new B when P is full,
// before a long pivot (whose column is merged as a whole) and at the end.
// A step issues few instructions on purpose: one wavefront runs one chain,
// so its instruction issue rate bounds the chain's speed.
typedef __attribute__((address_space(3))) void lds_void_t;

// copy this lane's record of row i to LDS slot (lane) of ra / rb (16 bytes each)
__device__ inline void rec_to_lds(const Dev &d, int32_t i, int4 *ra, int4 *rb)
{
    const int4 *src = reinterpret_cast<const int4 *>(d.prec + i);
    __builtin_amdgcn_global_load_lds(src, (lds_void_t *)ra, 16, 0, 0);
    __builtin_amdgcn_global_load_lds(src + 1, (lds_void_t *)rb, 16, 0, 0);
}

__device__ inline void wait_vmem()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copies to LDS have landed
}

// With solve_max > 0 and at most that many columns handed over, only those
// k_chain_solve passes on (wq2); else the lane passes' hand-over queue (wq).
template <bool kTrace>
__global__ void __launch_bounds__(kChainWaves *kWave) k_chain(Dev d, int compression, int32_t solve_max)
{
    __shared__ int32_t sW[kChainWaves][2][kCapW];
    __shared__ int32_t sS[kChainWaves][kCapS];
    __shared__ int32_t sE[kChainWaves][kCapS + 1];
    __shared__ int4 sRP[kChainWaves][2][kWave];  // records of the P entries (two halves), slot = lane
    __shared__ int4 sRW[kChainWaves][2][kWave];  // records of the window entries
    const int w = bcast_first(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);  // w: uniform by construction
    const unsigned gw = blockIdx.x * kChainWaves + w, nw = gridDim.x * kChainWaves;
    int4 *RPa = sRP[w][0], *RPb = sRP[w][1], *RWa = sRW[w][0], *RWb = sRW[w][1];
    const bool fallback = solve_max > 0 && d.cq_n[kPart * 32] <= solve_max;
    const int32_t *queue = fallback ? d.wq2 : d.wq;
    const int32_t total = d.cq_n[(fallback ? kPart + 2 : kPart) * 32];
    int64_t adds = 0, xe = 0, by = 0, ab = 0;
    // trace: short, long, global, sum |W|, toggle / next / flush cycles, flushes, queued, lows from P, deletions
    unsigned long long tr[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (kTrace && gw == 0) tr[8] = (unsigned long long)total;
    for (int32_t t = (int32_t)gw; t < total; t += (int32_t)nw) {
        const int32_t j = queue[t];
        const int32_t L0 = d.len[j];
        by += 4 + 12 + 4 * (int64_t)L0;  // queue entry, header, column in
        const int32_t *g = col_base(d, d.off[j]);
        int cur = 0;
        bool in_lds = L0 <= kCapW;
        const int32_t *Bg = g;  // B when it is not in LDS
        if (in_lds)
            for (int32_t a = lane; a < L0; a += kWave) sW[w][0][a] = g[a];
        wave_sync();
        int32_t LB = L0;
        uint64_t valid = 0;       // lanes holding an entry of P
        int32_t pq = 0;           // this lane's entry of P, plus one (0: none)
        int32_t pm1 = 0;          // max(P) + 1 (0: P empty), when !pdirty
        bool pdirty = false;
        int32_t wb = 0, wv = -1;  // window: this lane holds B[wb + lane] (-1: none)
        int32_t i = -1, pl = 0;   // the low, and its lane when it is in P
        bool from_p = false;
        int32_t ls = -1, lk = 0;  // the low's record: pivot, length
        int4 lea, leb;            // and entries (e[0], e[1] in lea.z, lea.w; e[2..5] in leb)
        bool dirty = false, failed = false;
        int32_t cadds = 0, cxe = 0, cby = 0;  // this column's counters (32-bit: cheap in the loop)
        int64_t cab = 0;

        auto Bp = [&]() -> const int32_t * { return in_lds ? (const int32_t *)sW[w][cur] : Bg; };
        auto refill = [&]() {
            wb = LB > kWave ? LB - kWave : 0;
            const int32_t a = wb + lane;
            wv = a < LB ? Bp()[a] : -1;
            if (wv >= 0) rec_to_lds(d, wv, RWa, RWb);
            wait_vmem();  // window records are read without a wait
        };
        auto read_rec = [&](const int4 *ra, const int4 *rb, int32_t l, bool wait) {
            if (wait) wait_vmem();  // the copies of the P records issued since
            lea = ra[l];
            leb = rb[l];
            ls = bcast_first(lea.x);
            lk = bcast_first(lea.y);
        };
        // the low of W: the larger of max(B) and max(P), equal tops cancel;
        // known-negative lows are deleted on the way
        auto next = [&]() {
            const int64_t c0 = kTrace ? clock64() : 0;
            for (;;) {
                if (LB > 0 && LB - 1 < wb) refill();
                if (pdirty) {
                    pm1 = valid ? wave_max_dpp(pq) : 0;
                    pdirty = false;
                }
                const int32_t bt = LB > 0 ? __builtin_amdgcn_readlane(wv, LB - 1 - wb) : -1;
                if (pm1 > bt + 1) {
                    const int32_t l = (int32_t)__builtin_ctzll(__ballot(pq == pm1));
                    i = pm1 - 1;
                    pl = l;
                    from_p = true;
                    read_rec(RPa, RPb, l, true);
                    if (compression && ls < 0 && lk < 0) {  // a negative row: delete it
                        valid &= ~(1ull << l);
                        pq = lane == l ? 0 : pq;
                        pdirty = true;
                        if (kTrace) tr[10]++;
                        continue;
                    }
                    if (kTrace) tr[9]++;
                    break;
                }
                if (bt < 0) {
                    i = -1;
                    break;
                }
                if (pm1 == bt + 1) {  // 1 + 1 = 0
                    const int32_t l = (int32_t)__builtin_ctzll(__ballot(pq == pm1));
                    valid &= ~(1ull << l);
                    pq = lane == l ? 0 : pq;
                    pdirty = true;
                    LB--;
                    continue;
                }
                i = bt;
                from_p = false;
                read_rec(RWa, RWb, LB - 1 - wb, false);
                if (compression && ls < 0 && lk < 0) {  // max(P) is unchanged
                    LB--;
                    if (kTrace) tr[10]++;
                    continue;
                }
                break;
            }
            if (kTrace) tr[5] += clock64() - c0;
        };
        // remove the low, toggle its pivot's entries e[0, kk) into P (needs
        // kk free lanes) and start the copies of the new entries' records
        auto step = [&](int32_t kk) {
            const int64_t c0 = kTrace ? clock64() : 0;
            if (from_p) {
                valid &= ~(1ull << pl);
                pq = lane == pl ? 0 : pq;
                pdirty = true;  // the low was max(P)
            } else {
                LB--;
            }
            const int32_t ev[kRecInline] = {lea.z, lea.w, leb.x, leb.y, leb.z, leb.w};
            uint64_t fresh = 0;
#pragma unroll
            for (int q = 0; q < kRecInline; q++) {
                if (q < kk) {
                    const int32_t x1 = ev[q] + 1;
                    const uint64_t m = __ballot(pq == x1);
                    if (m) {
                        const int32_t l = (int32_t)__builtin_ctzll(m);
                        valid &= ~(1ull << l);
                        fresh &= ~(1ull << l);
                        if (x1 == pm1) pdirty = true;
                        pq = lane == l ? 0 : pq;
                    } else {
                        const int32_t f = (int32_t)__builtin_ctzll(~valid);
                        valid |= 1ull << f;
                        fresh |= 1ull << f;
                        pm1 = max(pm1, x1);
                        pq = lane == f ? x1 : pq;
                    }
                }
            }
            if ((fresh >> lane) & 1ull) rec_to_lds(d, pq - 1, RPa, RPb);
            if (kTrace) tr[4] += clock64() - c0;
        };
        // B := B xor P (P emptied), into the free LDS buffer or the arena
        auto flush = [&]() -> bool {
            const int64_t c0 = kTrace ? clock64() : 0;
            const int32_t np = __popcll(valid);
            const int32_t cap = LB + np;
            const int nb = in_lds ? cur ^ 1 : 0;
            int32_t *dst;
            const bool dst_lds = cap <= kCapW;
            if (dst_lds) {
                dst = sW[w][nb];
            } else {
                long long o = 0;
                if (lane == 0) o = arena_alloc(d, gw, cap);
                o = bcast_first64(o);
                if (o < 0) {
                    if (lane == 0) atomicExch(&d.cnt->overflow, 1);
                    return false;  // keep the stored column; redo next round
                }
                dst = d.arena + o;
            }
            const int32_t *B = Bp();
            int32_t *sc = sE[w];  // [0,64) P by lane, [64,128) P sorted, [128,192) cancel flags, [192,256) their prefix
            const bool pvld = pq > 0;
            const int32_t my = pvld ? pq - 1 : 0x7FFFFFFF;
            wave_sync();
            sc[lane] = my;
            wave_sync();
            int32_t rk = 0;
            for (int u = 0; u < kWave; u++) rk += sc[u] < my ? 1 : 0;
            int32_t q = 0;
            bool cq = false;
            if (pvld) {
                q = lower_bound_i32(B, LB, my);
                cq = q < LB && B[q] == my;
                sc[64 + rk] = my;
                sc[128 + rk] = cq ? 1 : 0;
            }
            wave_sync();
            const int32_t ct = lane < np ? sc[128 + lane] : 0;
            const int32_t incl = wave_incl_sum32(ct);
            const int32_t totc = __builtin_amdgcn_readlane(incl, kWave - 1);
            sc[192 + lane] = incl - ct;
            wave_sync();
            const int32_t nL = cap - 2 * totc;
            if (pvld && !cq) {
                const int32_t o = q + rk - 2 * sc[192 + rk];
                if (o >= 0 && o < nL) dst[o] = my;
            }
            const int32_t cs = ((LB + kWave - 1) / kWave) | 1;  // odd chunks: lanes start in different banks
            const int32_t a0 = lane * cs, a1 = min(a0 + cs, LB);
            if (a0 < a1) {
                int32_t r = lower_bound_i32(sc + 64, np, B[a0]);
                for (int32_t a = a0; a < a1; a++) {
                    const int32_t x = B[a];
                    while (r < np && sc[64 + r] < x) r++;
                    if (r < np && sc[64 + r] == x) continue;
                    const int32_t o = a + r - 2 * (r < np ? sc[192 + r] : totc);
                    if (o >= 0 && o < nL) dst[o] = x;
                }
            }
            if (!dst_lds) __threadfence();
            wave_sync();
            valid = 0;
            pq = 0;
            pm1 = 0;
            pdirty = false;
            LB = nL;
            if (dst_lds) {
                in_lds = true;
                cur = nb;
            } else {
                in_lds = false;
                Bg = dst;
            }
            refill();
            if (kTrace) {
                tr[6] += clock64() - c0;
                tr[7]++;
            }
            return true;
        };

        refill();
        next();
        while (i >= 0 && ls >= 0) {  // a low without a pivot ends the chain
            const int32_t pi = i;
            const int32_t kk = lk - 1;
            cadds++;
            cxe += LB + lk;
            if (kk <= kRecInline) {
                if (__popcll(valid) + kk > kWave) {
                    if (!flush()) {
                        failed = true;
                        break;
                    }
                    from_p = false;  // W is unchanged: its low is now the top of B
                }
                cby += 32;  // the record of the low
                cab += 4 * (2 * (int64_t)(LB + __popcll(valid) + lk) - 2);
                if (kTrace) {
                    tr[0]++;
                    tr[3] += LB + __popcll(valid);
                }
                step(kk);
                dirty = true;
            } else {
                // long pivot: merge its whole column into W = B
                if (valid && !flush()) {
                    failed = true;
                    break;
                }
                const int32_t k = lk, L = LB;
                const int32_t *W = Bp();
                cby += 32 + 12 + 4 * k;
                if (kTrace) {
                    tr[3] += L;
                    if (in_lds && L + k <= kCapW && k <= kCapS) tr[1]++;
                    else tr[2]++;
                }
                const int32_t *Sg = col_base(d, d.off[ls]);
                if (in_lds && L + k <= kCapW && k <= kCapS) {
                    for (int32_t b = lane; b < k; b += kWave) sS[w][b] = Sg[b];
                    wave_sync();
                    const int32_t *S = sS[w];
                    int32_t *Wn = sW[w][cur ^ 1];
                    // cancelled pairs: exclusive prefix count over S
                    int32_t carry = 0;
                    for (int32_t base = 0; base < k; base += kWave) {
                        const int32_t b = base + lane;
                        int32_t e = 0;
                        if (b < k) {
                            const int32_t qq = lower_bound_i32(W, L, S[b]);
                            e = (qq < L && W[qq] == S[b]) ? 1 : 0;
                        }
                        const int32_t inc = wave_incl_sum32(e);
                        if (b < k) sE[w][b] = carry + inc - e;
                        carry += bcast_lane(inc, kWave - 1);
                    }
                    if (lane == 0) sE[w][k] = carry;
                    wave_sync();
                    // an entry's output position: its own index plus its
                    // rank in the other list minus twice the number of
                    // cancelled pairs below it
                    for (int32_t a = lane; a < L; a += kWave) {
                        const int32_t x = W[a];
                        const int32_t r = lower_bound_i32(S, k, x);
                        if (!(r < k && S[r] == x)) Wn[a + r - 2 * sE[w][r]] = x;
                    }
                    for (int32_t b = lane; b < k; b += kWave) {
                        const int32_t x = S[b];
                        const int32_t qq = lower_bound_i32(W, L, x);
                        if (!(qq < L && W[qq] == x)) Wn[b + qq - 2 * sE[w][b]] = x;
                    }
                    LB = L + k - 2 * carry;
                    cab += 4 * ((int64_t)L + k + LB);
                    wave_sync();
                    cur ^= 1;
                } else {
                    // too long for LDS: lane 0 merges in global memory
                    long long o = 0;
                    const int64_t need = (int64_t)L + k;
                    if (lane == 0) o = arena_alloc(d, gw, need);
                    o = bcast_first64(o);
                    if (o < 0) {
                        if (lane == 0) atomicExch(&d.cnt->overflow, 1);
                        failed = true;  // keep the stored column; redo next round
                        break;
                    }
                    int32_t *out = d.arena + o;
                    int32_t nL = 0;
                    if (lane == 0) nL = merge_add(W, L, Sg, k, out, d.neg, compression);
                    nL = bcast_first(nL);
                    __threadfence();  // lane 0's global writes, then every lane reads them
                    wave_sync();
                    Bg = out;
                    in_lds = false;
                    LB = nL;
                    cab += 4 * ((int64_t)L + k + nL);
                }
                dirty = true;
                refill();
            }
            next();
            if (i >= pi) {  // the low must drop; stop rather than spin
                if (lane == 0) {  // never expected
                    d.cnt->bad_info[0] = j;
                    d.cnt->bad_info[1] = i;
                    d.cnt->bad_info[2] = pi;
                    d.cnt->bad_info[3] = cadds;
                    atomicExch(&d.cnt->bad_source, 2);
                }
                failed = true;
                break;
            }
        }
        if (!failed && valid && !flush()) failed = true;
        wait_vmem();  // no record copy may land after this column is done
        adds += cadds;
        xe += cxe;
        by += cby;
        ab += cab;
        if (kTrace && lane == 0) atomicMax(&d.cnt->max_chain, cadds);
        if (failed || !dirty) continue;
        // write the result back
        if (LB == 0) {
            if (lane == 0) {
                dbg_write(d, j);
                d.len[j] = 0;
                d.low[j] = -1;
                d.state[j] = ST_ZERO;  // column j is positive
            }
            continue;
        }
        int64_t dst;
        if (in_lds) {
            long long o = 0;
            if (lane == 0) o = arena_alloc(d, gw, LB);
            o = bcast_first64(o);
            if (o < 0) {
                if (lane == 0) atomicExch(&d.cnt->overflow, 1);
                continue;  // progress of this chain is dropped; the stored column is still valid
            }
            const int32_t *W = sW[w][cur];
            for (int32_t a = lane; a < LB; a += kWave) d.arena[o + a] = W[a];
            dst = (int64_t)o;
        } else {
            if (Bg == g) {  // only deletions at the top: the stored column, shortened
                if (lane == 0) {
                    dbg_write(d, j);
                    d.len[j] = LB;
                    d.low[j] = Bg[LB - 1];
                }
                continue;
            }
            dst = (int64_t)(Bg - d.arena);
        }
        by += 4 * (int64_t)LB + 16;  // column and header out
        if (lane == 0) {
            dbg_write(d, j);
            d.off[j] = dst | (int64_t)kArenaBit;
            d.len[j] = LB;
            d.low[j] = in_lds ? sW[w][cur][LB - 1] : Bg[LB - 1];
        }
        wave_sync();
    }
    // per-wave counters (every lane holds the same values)
    if (lane == 0) {
        stat_add(d, S_ADDS, (unsigned long long)adds, gw);
        stat_add(d, S_XE, (unsigned long long)xe, gw);
        stat_add(d, S_CBYTES, (unsigned long long)by, gw);
        stat_add(d, S_ABYTES_CHAIN, (unsigned long long)ab, gw);
        if (kTrace) {
            for (int q = 0; q < 9; q++) stat_add(d, S_T_SHORT + q, tr[q], gw);
            stat_add(d, S_T_FROMP, tr[9], gw);
            stat_add(d, S_T_DEL, tr[10], gw);
        }
    }
}

// ------------------------------------------ chaining as a triangular solve
// The pivots a chained column j adds are fixed by a unit-triangular system
// over F2 (the inner loop of Alg. "Standard reduction", on known pivots).
// Let c be the column, P_s the pivot column of a row s that has a known pivot
// (its low is s: every other entry lies below s) and S the rows whose pivot
// gets added.  With v(r) = c(r) + the sum of P_s(r) over s in S with s > r,
// row r is in S exactly when it has a known pivot, v(r) = 1 and r lies above
// L, the highest row with v = 1 and no known pivot (the chain ends there: it
// is the new low; with no such row the column reduces to zero).  The result
// is c + the sum of P_s over S, and low(j) becomes L.  Whether r is in S
// depends only on rows above r, so the system has one solution, and the
// sweep "S from v, then v from S" is exact on every row whose dependencies
// are: it reaches the solution after as many sweeps as the longest path of
// dependencies among the rows involved.  The serial walk (k_chain) makes one
// dependent addition per step: thousands on the longest columns of a 64^3
// lower-star filtration, whose dependency paths are 10 to 80 rows long.
//
// One workgroup per column.  The rows the column touches are kept in LDS as
// a dense list (row, one byte of flags) in the order they were met, found
// through a hash table of list positions, so a pass costs the rows touched,
// not the table.  A sweep is a pass that finds L, a pass that flips the
// membership of the rows whose test changed (into a list of changes), and a
// pass that toggles the entries of those rows' pivots (from their records,
// one load each).  The head of each entry's own record (pivot, length) is
// loaded before it is toggled: rows known to be negative are left out
// (compression deletes them), and a new row enters the list with its flags.
// The result is written back sorted.  A column whose rows overfill the list
// goes to k_chain.
constexpr int kSolveThreads = 512;
constexpr int kSolveH = 8192;            // hash slots (list positions, -1 = free)
constexpr int kSolveMaxU = 6144;         // rows one column may touch (list length)
constexpr int kSolveDelta = 2048;        // membership changes applied per sweep
constexpr int kSolveSweeps = 4096;       // a column still changing then goes to k_chain
constexpr int kSolveLong = 64;           // long pivots a sweep spreads over the workgroup (more: per thread)
constexpr int kSolvePer = kSolveMaxU / 4 / kSolveThreads;  // flag words (4 rows each) per thread
static_assert(kSolveMaxU % (4 * kSolveThreads) == 0 && kSolveMaxU < kSolveH && (kSolveH & (kSolveH - 1)) == 0,
              "k_chain_solve: whole flag words per thread; probes always end; the result sorts in the table");
// flags of a row
constexpr uint32_t kSV = 1;   // v(r)
constexpr uint32_t kSX = 2;   // r is in S
constexpr uint32_t kSP = 4;   // r has a known pivot
constexpr uint32_t kSR = 8;   // r's pivot lies right of column j (never expected in S)

struct SolveLds {
    int32_t *hk;       // hash slot -> list position
    int32_t *key;      // list position -> row
    uint32_t *flag;    // flags, byte (position & 3) of word position / 4
    int32_t *n;        // list length (positions handed out)
    int32_t *fail;
};

__device__ inline uint32_t solve_hash(int32_t r)
{
    return ((uint32_t)r * 2654435761u) >> 19;  // 13 bits: kSolveH slots
}

// Toggles v(e), appending row e with flags fl when it is new.  A full list
// sets *fail (the column then goes to the serial kernel).  A new row's list
// entry is written before its position is published in the hash table, so a
// thread that finds the position finds the row: LDS performs one wave's
// operations in issue order, so only the compiler must keep them in order
// (a fence would also wait for this thread's global loads in flight).
__device__ inline void solve_toggle(const SolveLds &t, int32_t e, uint32_t fl)
{
    uint32_t h = solve_hash(e);
    int32_t mine = -1;
    for (;;) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t x = __hip_atomic_load(&t.hk[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (x >= 0) {
            if (t.key[x] == e) {
                if (mine >= 0) t.key[mine] = -1;  // reserved for nothing: a dead entry (flags 0)
                atomicXor(&t.flag[x >> 2], kSV << (8 * (x & 3)));
                return;
            }
            h = (h + 1) & (kSolveH - 1);
            continue;
        }
        if (mine < 0) {
            mine = atomicAdd(t.n, 1);
            if (mine >= kSolveMaxU) {
                atomicExch(t.fail, 1);
                return;
            }
            t.key[mine] = e;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t old = atomicCAS(&t.hk[h], -1, mine);
        if (old == -1) {
            atomicXor(&t.flag[mine >> 2], (fl | kSV) << (8 * (mine & 3)));
            return;
        }
        // the slot was taken meanwhile: look at it again
    }
}

// Toggles the rows rows[u] with bit u of use set: each row's pivot (piv) and
// known-negative bit (neg; both dense, so mostly cache hits) are loaded
// together first (row 0 stands in for unused slots: the loads are
// unconditional and the group waits once); known-negative rows are skipped.
template <int kN>
__device__ inline void solve_toggle_n(const Dev &d, const SolveLds &t, const int32_t (&rows)[kN], uint32_t use,
                                      int32_t j, int compression)
{
    int32_t pv[kN];
    uint32_t nw[kN];
#pragma unroll
    for (int u = 0; u < kN; u++) {
        const int32_t r = (use >> u) & 1u ? rows[u] : 0;
        pv[u] = d.piv[r];
        nw[u] = d.neg[r >> 5];
    }
#pragma unroll
    for (int u = 0; u < kN; u++) {
        const bool negative = compression && ((nw[u] >> (rows[u] & 31)) & 1u);
        if (((use >> u) & 1u) && !negative)
            solve_toggle(t, rows[u], pv[u] >= 0 ? (pv[u] < j ? kSP : (kSP | kSR)) : 0u);
    }
}

// The kernel takes the handed-over columns when there are at most solve_max
// of them (a round of few, long chains, bound by its longest one); more
// columns are walked by k_chain, whose waves hold more columns per CU.
template <bool kTrace>
__global__ void __launch_bounds__(kSolveThreads) k_chain_solve(Dev d, int compression, int32_t solve_max)
{
    __shared__ __align__(16) int32_t hk[kSolveH];        // hash table; then the result, sorted
    __shared__ __align__(16) int32_t key[kSolveMaxU];    // the rows touched, in the order met (-1: dead)
    __shared__ uint32_t flag[kSolveMaxU / 4];            // their flags, 4 per word
    __shared__ int32_t dl[kSolveDelta];                  // this sweep's changes of S: r (joins) or ~r (leaves)
    __shared__ int32_t s_n, s_fail, s_bad, s_L[2], s_nd[2];
    __shared__ long long s_o;
    __shared__ long long s_loff[kSolveLong];  // this sweep's long pivots: stored column, entries below the low
    __shared__ int32_t s_lpre[kSolveLong + 1], s_nl;
    const SolveLds t{hk, key, flag, &s_n, &s_fail};
    const int4 *key4 = reinterpret_cast<const int4 *>(key);
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int32_t total = d.cq_n[kPart * 32];  // columns the lane passes handed over
    if (total > solve_max) return;             // k_chain takes them all
    int64_t adds = 0, pk = 0, by = 0, ab = 0, sweeps = 0;  // pk: entries read (column and added pivots)
    int32_t nsolved = 0, nfall = 0;
    // trace: set-up, pass A, pass B, toggles, out cycles; changes; long pivots, their entries;
    // changes left for the next sweep (more than kSolveDelta in one)
    unsigned long long tr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    long long c0 = 0;
    auto tick = [&](int q) {
        if (kTrace) {
            const long long c1 = clock64();
            tr[q] += (unsigned long long)(c1 - c0);
            c0 = c1;
        }
    };
    auto hand_on = [&](int32_t j) {
        if (tid == 0) d.wq2[atomicAdd(&d.cq_n[(kPart + 2) * 32], 1)] = j;
        nfall++;
    };
    for (int32_t q0 = (int32_t)blockIdx.x; q0 < total; q0 += (int32_t)gridDim.x) {
        __syncthreads();  // the previous column's last reads of LDS are done
        const int32_t j = d.wq[q0];
        const int32_t L0 = d.len[j];
        const int32_t *g = col_base(d, d.off[j]);
        if (L0 > kSolveMaxU / 2) {
            hand_on(j);
            continue;
        }
        if (kTrace) c0 = clock64();
        const long long w0 = kTrace ? wall_clock64() : 0;
        for (int a = tid; a < kSolveH / 4; a += kSolveThreads) reinterpret_cast<int4 *>(hk)[a] = make_int4(-1, -1, -1, -1);
        for (int a = tid; a < kSolveMaxU / 4; a += kSolveThreads) flag[a] = 0;
        if (tid == 0) {
            s_n = 0;
            s_fail = 0;
            s_bad = 0;
            s_L[0] = s_L[1] = 0;
            s_nd[0] = s_nd[1] = 0;
        }
        __syncthreads();
        // v = c
        for (int32_t a0 = 0; a0 < L0; a0 += 4 * kSolveThreads) {
            int32_t rows[4];
            int32_t n = 0;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int32_t a = a0 + u * kSolveThreads + tid;
                rows[u] = a < L0 ? g[a] : -1;
                n += a < L0 ? 1 : 0;
            }
            solve_toggle_n<4>(d, t, rows, (1u << n) - 1u, j, compression);
        }
        __syncthreads();
        tick(0);
        bool ok = false;
        int64_t cxe = 0;  // entries of the pivots in S (this thread's share)
        for (int it = 0;; it++) {
            const int p = it & 1;
            const int32_t nwords = (min(s_n, kSolveMaxU) + 3) >> 2;
            // this thread's rows, read once for both passes (nothing writes them in between)
            uint32_t fw[kSolvePer];
            int32_t kw[kSolvePer][4];
#pragma unroll
            for (int u = 0; u < kSolvePer; u++) {
                const int w = u * kSolveThreads + tid;
                fw[u] = 0;
                kw[u][0] = kw[u][1] = kw[u][2] = kw[u][3] = -1;
                if (w < nwords) {
                    fw[u] = flag[w];
                    const int4 k4 = key4[w];
                    kw[u][0] = k4.x;
                    kw[u][1] = k4.y;
                    kw[u][2] = k4.z;
                    kw[u][3] = k4.w;
                }
            }
            // L + 1 (0: no row with v = 1 lacks a pivot)
            int32_t lm = 0;
#pragma unroll
            for (int u = 0; u < kSolvePer; u++)
#pragma unroll
                for (int b = 0; b < 4; b++)
                    lm = ((fw[u] >> (8 * b)) & (kSV | kSP)) == kSV ? max(lm, kw[u][b] + 1) : lm;
            lm = wave_max_dpp(lm);
            if (lane == 0 && lm > 0) atomicMax(&s_L[p], lm);
            __syncthreads();
            tick(1);
            const int32_t Lp1 = s_L[p];
            // the membership test; at most kSolveDelta changes a sweep (the rest wait for the next)
            uint32_t chg = 0;  // bit 4u + b: row b of word u changes
#pragma unroll
            for (int u = 0; u < kSolvePer; u++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const uint32_t fb = fw[u] >> (8 * b);
                    const bool want = (fb & (kSV | kSP)) == (kSV | kSP) && kw[u][b] >= Lp1;
                    chg |= (uint32_t)(want != ((fb & kSX) != 0)) << (4 * u + b);
                }
            if (tid == 0) s_nl = 0;
            if (chg) {
                int32_t q = atomicAdd(&s_nd[p], __popc(chg));
                while (chg) {
                    const int i = __builtin_ctz(chg);
                    chg &= chg - 1;
                    const int w = (i >> 2) * kSolveThreads + tid, b = i & 3;
                    if (q < kSolveDelta) {
                        const int32_t r = key[4 * w + b];
                        const bool has = ((flag[w] >> (8 * b)) & kSX) != 0;  // it leaves S, else joins
                        dl[q] = has ? ~r : r;
                        flag[w] ^= kSX << (8 * b);  // this thread's word: no other writer in this pass
                    } else if (kTrace) {
                        tr[8]++;
                    }
                    q++;
                }
            }
            __syncthreads();
            tick(2);
            const int32_t nd = min(s_nd[p], kSolveDelta);
            tr[5] += kTrace ? nd : 0;
            if (s_fail || nd == 0 || it >= kSolveSweeps) {
                ok = !s_fail && nd == 0;
                sweeps += it;
                if (tid == 0) atomicMax(&d.cnt->max_sweeps, it);
                break;
            }
            if (tid == 0) {
                s_L[p ^ 1] = 0;
                s_nd[p ^ 1] = 0;
            }
            // toggle the entries of the changed rows' pivots.  G lanes share a changed
            // row (G = 8 when the changes are few: each lane then toggles one entry,
            // so the probe chains run side by side; G = 1 when they are many); the
            // lanes of a row load its record together, then their entries' pivots
            // and known-negative bits, then toggle
            {
                const int32_t G = nd <= kSolveThreads / 8 ? 8 : nd <= kSolveThreads / 4 ? 4
                                : nd <= kSolveThreads / 2 ? 2 : 1;
                const int32_t sub = tid & (G - 1), grp = tid / G, per = kSolveThreads / G;
                for (int32_t q0 = 0; q0 < nd; q0 += per) {
                    const int32_t q = q0 + grp;
                    const int32_t code = q < nd ? dl[q] : 0;
                    const int32_t sign = q < nd ? (code >= 0 ? 1 : -1) : 0;
                    const PivRec rec = d.prec[code >= 0 ? code : ~code];  // row 0 stands in for no row
                    const int32_t k = sign ? rec.k : 1;  // the pivot's length, its low included
                    const bool inl = k - 1 <= kRecInline;
                    // this lane's entries: e[sub], e[sub + G], ...
                    int32_t ent[kRecInline];
                    uint32_t use = 0;
#pragma unroll
                    for (int i = 0; i < kRecInline; i++) {
                        const int32_t u = sub + i * G;
                        int32_t x = rec.e[0];
#pragma unroll
                        for (int c = 1; c < kRecInline; c++) x = u == c ? rec.e[c] : x;
                        ent[i] = x;
                        use |= (uint32_t)(inl && u < k - 1) << i;
                    }
                    solve_toggle_n<kRecInline>(d, t, ent, use, j, compression);
                    if (sub == 0 && sign) {
                        cxe += sign * k;
                        by += 32;
                        if (!inl) {  // a long pivot: its entries from its stored column
                            const int64_t off = d.off[rec.s];
                            by += 12 + 4 * (int64_t)k;
                            if (kTrace) {
                                tr[6]++;
                                tr[7] += k - 1;
                            }
                            const int32_t li = atomicAdd(&s_nl, 1);
                            if (li < kSolveLong) {  // the workgroup toggles its entries below
                                s_loff[li] = off;
                                s_lpre[li + 1] = k - 1;
                            } else {
                                const int32_t *pc = col_base(d, off);
                                for (int32_t a0 = 0; a0 < k - 1; a0 += 4) {
                                    int32_t rows[4];
                                    int32_t n = 0;
#pragma unroll
                                    for (int u = 0; u < 4; u++) {
                                        rows[u] = a0 + u < k - 1 ? pc[a0 + u] : -1;
                                        n += a0 + u < k - 1 ? 1 : 0;
                                    }
                                    solve_toggle_n<4>(d, t, rows, (1u << n) - 1u, j, compression);
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
            const int32_t nl = min(s_nl, kSolveLong);
            if (nl > 0) {  // the long pivots' entries, spread over every thread
                if (tid < kWave) {
                    const int32_t c = tid < nl ? s_lpre[tid + 1] : 0;
                    const int32_t incl = wave_incl_sum32(c);
                    if (tid < nl) s_lpre[tid + 1] = incl;
                    if (tid == 0) s_lpre[0] = 0;
                }
                __syncthreads();
                const int32_t tot = s_lpre[nl];
                for (int32_t e0 = tid; e0 < tot; e0 += 4 * kSolveThreads) {
                    int32_t rows[4];
                    int32_t n = 0;
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int32_t ei = e0 + u * kSolveThreads;
                        const int32_t ec = min(ei, tot - 1);  // loaded unconditionally: one wait
                        int32_t lo = 0, hi = nl - 1;          // the pivot whose entries hold ec
                        while (lo < hi) {
                            const int32_t mid = (lo + hi + 1) >> 1;
                            if (s_lpre[mid] <= ec) lo = mid;
                            else hi = mid - 1;
                        }
                        rows[u] = col_base(d, s_loff[lo])[ec - s_lpre[lo]];
                        n += ei < tot ? 1 : 0;
                    }
                    solve_toggle_n<4>(d, t, rows, (1u << n) - 1u, j, compression);
                }
                __syncthreads();
            }
            tick(3);
        }
        if (!ok) {
            hand_on(j);
            continue;
        }
        // the result: the rows with v = 1 outside S, sorted
        const int32_t nwords = (min(s_n, kSolveMaxU) + 3) >> 2;
        int32_t nw = 0, ns = 0;
        bool bad = false;
        for (int w = tid; w < nwords; w += kSolveThreads) {
            const uint32_t f = flag[w];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const uint32_t fb = f >> (8 * b);
                nw += (fb & (kSV | kSX)) == kSV ? 1 : 0;
                ns += (fb & kSX) ? 1 : 0;
                bad = bad || (fb & (kSX | kSR)) == (kSX | kSR);
            }
        }
        if (bad) s_bad = 1;
        int32_t tot_w, tot_s;
        int32_t o = block_excl_sum32<kSolveThreads>(nw, &tot_w);  // its barriers end every use of the hash table
        block_excl_sum32<kSolveThreads>(ns, &tot_s);
        if (s_bad) {  // a pivot right of the column would be added: never expected
            if (tid == 0) {
                d.cnt->bad_info[0] = j;
                d.cnt->bad_info[1] = -1;
                d.cnt->bad_info[2] = L0;
                d.cnt->bad_info[3] = tot_s;
                atomicExch(&d.cnt->bad_source, 4);
            }
            continue;
        }
        nsolved++;
        pk += cxe;
        for (int w = tid; w < nwords; w += kSolveThreads) {
            const uint32_t f = flag[w];
            const int4 k4 = key4[w];
            const int32_t kk[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
            for (int b = 0; b < 4; b++)
                if (((f >> (8 * b)) & (kSV | kSX)) == kSV) hk[o++] = kk[b];
        }
        int32_t n2 = 1;
        while (n2 < tot_w) n2 <<= 1;  // <= kSolveMaxU rounded up <= kSolveH
        for (int32_t a = tot_w + tid; a < n2; a += kSolveThreads) hk[a] = 0x7FFFFFFF;
        __syncthreads();
        // bitonic sort of hk[0, n2)
        for (int32_t kk = 2; kk <= n2; kk <<= 1)
            for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int32_t a = tid; a < n2; a += kSolveThreads) {
                    const int32_t b = a ^ jj;
                    if (b > a) {
                        const int32_t x = hk[a], y = hk[b];
                        if ((x > y) == ((a & kk) == 0)) {
                            hk[a] = y;
                            hk[b] = x;
                        }
                    }
                }
                __syncthreads();
            }
        if (tid == 0) {
            adds += tot_s;
            by += 4 + 12 + 4 * (int64_t)L0;  // queue entry, header, column in
            ab += 4 * (int64_t)tot_w;        // + 4 (len c + the pivots' lengths) from pk
            pk += L0;
        }
        if (tot_w == 0) {
            if (tid == 0) {
                dbg_write(d, j);
                d.len[j] = 0;
                d.low[j] = -1;
                d.state[j] = ST_ZERO;  // column j is positive
            }
            continue;
        }
        if (tid == 0) s_o = arena_alloc(d, blockIdx.x, tot_w);
        __syncthreads();
        const long long oa = s_o;
        if (oa < 0) {
            if (tid == 0) atomicExch(&d.cnt->overflow, 1);
            continue;  // progress of this column is dropped; the stored column is still valid
        }
        for (int32_t a = tid; a < tot_w; a += kSolveThreads) d.arena[oa + a] = hk[a];
        tick(4);
        if (kTrace && tid == 0) atomicMax(&d.cnt->max_solve_us, (int32_t)((wall_clock64() - w0) / 100));  // 100 MHz
        if (tid == 0) {
            by += 4 * (int64_t)tot_w + 16;  // column and header out
            dbg_write(d, j);
            d.off[j] = (int64_t)oa | (int64_t)kArenaBit;
            d.len[j] = tot_w;
            d.low[j] = hk[tot_w - 1];
        }
    }
    // the additions' bytes as one multi-way sum: 4 (len c + the pivots' lengths + len out)
    const int64_t b_adds = block_sum64<kSolveThreads>(adds), b_xe = block_sum64<kSolveThreads>(pk), b_by = block_sum64<kSolveThreads>(by);
    const int64_t b_ab = block_sum64<kSolveThreads>(ab) + 4 * b_xe;
    const int64_t b_sw = block_sum64<kSolveThreads>(sweeps) / kSolveThreads;
    if (kTrace) {  // per-thread counts (the cycle counts are thread 0's)
        tr[6] = (unsigned long long)block_sum64<kSolveThreads>((int64_t)tr[6]);
        tr[7] = (unsigned long long)block_sum64<kSolveThreads>((int64_t)tr[7]);
        tr[8] = (unsigned long long)block_sum64<kSolveThreads>((int64_t)tr[8]);
    }
    if (tid == 0) {
        stat_add(d, S_ADDS, (unsigned long long)b_adds, blockIdx.x);
        stat_add(d, S_XE, (unsigned long long)b_xe, blockIdx.x);
        stat_add(d, S_SBYTES, (unsigned long long)b_by, blockIdx.x);
        stat_add(d, S_ABYTES_SOLVE, (unsigned long long)b_ab, blockIdx.x);
        stat_add(d, S_T_SWEEPS, (unsigned long long)b_sw, blockIdx.x);
        stat_add(d, S_T_SOLVED, (unsigned long long)nsolved, blockIdx.x);
        stat_add(d, S_T_SFALL, (unsigned long long)nfall, blockIdx.x);
        if (kTrace)
            for (int q = 0; q < 9; q++) stat_add(d, S_T_SINIT + q, tr[q], blockIdx.x);
    }
}

// ------------------------------------------------- clearing by compression
// Lemma "Clearing by local compression" (Sec. 3.2) with its Corollary, the
// case L_j = {0}: low*(j) lies in {0} and the (d-1)-simplices of
// [beta_j, low(j)] that are not paired yet (d = dim(j)).  For a column with
// no beta_j the range is [first row of its complex, low(j)], so when every
// (d-1)-simplex of the complex up to low(j) is paired, low*(j) = 0: column j
// is positive, and is cleared like a column cleared by a pivot.  A row i is
// paired once it is known negative (beta_i defined, or a found pivot) or is
// the low* of a found pivot (piv[i]).
constexpr int kC8Dims = 8;

__device__ inline bool c8_paired(const Dev &d, int64_t i)
{
    return d.beta[i] >= 0 || d.state[i] == ST_PIVOT || d.piv[i] >= 0;
}

// The first unpaired row of each dimension below the top one, per instance,
// in three steps.  Rows only ever become paired and lows only decrease, so
// each round scans [start, end] of an instance: start = the smallest first
// unpaired row of the last round, end = the largest low among the columns
// the last clearing pass looked at (a row above every low decides no
// column; a twist-order stage starts over from the instance's end).  The
// range is split over many blocks.  Per instance, c8_first holds the
// kC8Dims first rows, then start, this round's end and the next round's end.
constexpr int kC8Stride = kC8Dims + 3;
constexpr int kC8Start = kC8Dims, kC8End = kC8Dims + 1, kC8Next = kC8Dims + 2;

__global__ void k_c8_range(Dev d)
{
    const int32_t nd = min(d.cnt->topdim, kC8Dims);  // row dimensions 0 .. topdim-1 are needed
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < d.n_inst; k += gridDim.x * blockDim.x) {
        int32_t *f = d.c8_first + (int64_t)k * kC8Stride;
        const int64_t lo = d.inst_off[k], hi = d.inst_off[k + 1];
        int64_t start = hi;
        for (int e = 0; e < nd; e++) start = min(start, (int64_t)f[e]);
        f[kC8Start] = (int32_t)max(start, lo);
        f[kC8End] = (int32_t)min((int64_t)f[kC8Next], hi - 1);
        f[kC8Next] = -1;  // the clearing pass raises it to the largest low it keeps
        for (int e = 0; e < kC8Dims; e++) f[e] = 0x7FFFFFFF;
    }
}

template <int kChunks>
__global__ void __launch_bounds__(kBlock) k_c8_scan(Dev d)
{
    __shared__ int32_t s_first[kC8Dims];
    const int32_t nd = min(d.cnt->topdim, kC8Dims);
    for (int64_t bk = blockIdx.x; bk < (int64_t)d.n_inst * kChunks; bk += gridDim.x) {
        const int32_t k = (int32_t)(bk / kChunks), ch = (int32_t)(bk % kChunks);
        int32_t *f = d.c8_first + (int64_t)k * kC8Stride;
        const int64_t start = f[kC8Start], end = f[kC8End];
        if (threadIdx.x < kC8Dims) s_first[threadIdx.x] = 0x7FFFFFFF;
        __syncthreads();
        if (end >= start) {
            const int64_t per = (end - start + kChunks) / kChunks;
            const int64_t a = start + ch * per, b = min(a + per, end + 1);
            for (int64_t i = a + threadIdx.x; i < b; i += kBlock) {
                const int e = d.dim[i];
                if (e < nd && !c8_paired(d, i)) atomicMin(&s_first[e], (int32_t)i);
            }
        }
        __syncthreads();
        if (threadIdx.x < nd && s_first[threadIdx.x] != 0x7FFFFFFF) atomicMin(&f[threadIdx.x], s_first[threadIdx.x]);
        __syncthreads();
    }
}

// a dimension with no unpaired row in [start, end]: its first one lies past
// end (past start, nothing known, when the range is empty)
__global__ void k_c8_fold(Dev d)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < d.n_inst; k += gridDim.x * blockDim.x) {
        int32_t *f = d.c8_first + (int64_t)k * kC8Stride;
        const int32_t past = f[kC8End] >= f[kC8Start] ? f[kC8End] + 1 : f[kC8Start];
        for (int e = 0; e < kC8Dims; e++)
            if (f[e] == 0x7FFFFFFF) f[e] = past;
    }
}

// the next round scans up to each instance's end (start of a reduction or
// of a twist-order stage: the columns are new to the clearing pass)
__global__ void k_c8_reset_end(Dev d)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < d.n_inst; k += gridDim.x * blockDim.x)
        d.c8_first[(int64_t)k * kC8Stride + kC8Next] = 0x7FFFFFFE;
}

// The active columns with L_j = {0}: cleared (positive); the others raise
// the next round's scan end to their low.
__global__ void __launch_bounds__(kBlock) k_c8_clear(Dev d, const int32_t *act)
{
    const int32_t nA = d.cnt->n_cur;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    const XcdSplit xs = xcd_split(tiles);
    for (int64_t tile = xs.first; tile < xs.end; tile += xs.step) {
        const int64_t q = tile * kBlock + threadIdx.x;
        int cleared = 0;
        if (q < nA) {
            const int32_t j = act[q];
            const int e = d.dim[j] - 1;
            if (e >= 0 && e < kC8Dims && d.state[j] == ST_ACTIVE && d.beta[j] < 0) {
                int32_t a = 0, b = d.n_inst - 1;  // the instance: inst_off[a] <= j < inst_off[a + 1]
                while (a < b) {
                    const int32_t mid = (a + b + 1) >> 1;
                    if (d.inst_off[mid] <= j) a = mid;
                    else b = mid - 1;
                }
                int32_t *f = d.c8_first + (int64_t)a * kC8Stride;
                const int32_t lo = d.low[j];
                if (lo <= f[kC8End] && lo < f[e]) {
                    dbg_write(d, j);
                    d.state[j] = ST_CLEARED;
                    cleared = 1;
                } else if (lo > f[kC8Next]) {
                    atomicMax(&f[kC8Next], lo);  // the next round's scan end
                }
            }
        }
        int32_t tot;
        block_excl_sum32(cleared, &tot);
        if (threadIdx.x == 0 && tot) atomicAdd(&d.cnt->c8_cleared, (unsigned long long)tot);
    }
}

// Per-tile count of the positions that stay active.
// (dimsel >= 0: only the active columns of that dimension stay, for the
// first list of a twist-order stage)
__global__ void __launch_bounds__(kBlock) k_keep_count(Dev d, const int32_t *act, int32_t *keep_cnt, int dimsel)
{
    const int32_t nA = d.cnt->n_cur;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    const XcdSplit xs = xcd_split(tiles);
    for (int64_t tile = xs.first; tile < xs.end; tile += xs.step) {
        const int64_t q = tile * kBlock + threadIdx.x;
        const int keep =
            (q < nA && d.state[act[q]] == ST_ACTIVE && (dimsel < 0 || d.dim[act[q]] == dimsel)) ? 1 : 0;
        int32_t tk;
        block_excl_sum32(keep, &tk);
        if (threadIdx.x == 0) keep_cnt[tile] = tk;
        __syncthreads();
    }
}

// Stable compaction of the active list; finalises cleared columns.
__global__ void __launch_bounds__(kBlock) k_compact(Dev d, const int32_t *act, const int32_t *keep_off,
                                                    int32_t *act_next, int dimsel)
{
    const int32_t nA = d.cnt->n_cur;
    const int64_t tiles = ((int64_t)nA + kBlock - 1) / kBlock;
    const XcdSplit xs = xcd_split(tiles);
    for (int64_t tile = xs.first; tile < xs.end; tile += xs.step) {
    const int64_t q = tile * kBlock + threadIdx.x;
    int keep = 0;
    int32_t j = -1;
    if (q < nA) {
        j = act[q];
        const uint8_t st = d.state[j];
        if (st == ST_CLEARED) {
            dbg_write(d, j);
            d.state[j] = ST_ZERO;
            d.len[j] = 0;
            d.low[j] = -1;
        }
        keep = st == ST_ACTIVE && (dimsel < 0 || d.dim[j] == dimsel);
    }
    int32_t tot;
    const int32_t pos = block_excl_sum32(keep, &tot);
    if (keep) act_next[keep_off[tile] + pos] = j;
    __syncthreads();
    }
}

// ---------------------------------------------------------------- diagnostics
__global__ void k_diag_reset(Dev d)
{
    d.cnt->diag_low_l1 = 0;
    d.cnt->diag_ess = 0;
    d.cnt->diag_active = 0;
}

// low^l of every column (-1 for zero and cleared columns; an active column's
// low with known-negative rows trimmed, as k_low will), summed as
// low^l(j) + 1; E loses the columns known negative (pivots, beta_j defined)
// and every low^l(j): the paired rows of the pivots and the lows of the
// columns still active (eq. "essential_iteration").
__global__ void __launch_bounds__(kBlock) k_diag_update(Dev d, int compression)
{
    int64_t l1 = 0, act = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t st = d.state[j];
        int32_t lo = -1;
        if (st == ST_PIVOT) {
            lo = d.low[j];
        } else if (st == ST_ACTIVE) {
            int32_t n = d.len[j];
            const int32_t *c = col_base(d, d.off[j]);
            if (compression)
                while (n > 0 && is_neg(d.neg, c[n - 1])) n--;
            lo = n > 0 ? c[n - 1] : -1;
            act += lo >= 0 ? 1 : 0;
        }
        l1 += (int64_t)lo + 1;
        if (st == ST_PIVOT || d.beta[j] >= 0) atomicAnd(&d.ess[j >> 5], ~(1u << (j & 31)));
        if (lo >= 0) atomicAnd(&d.ess[lo >> 5], ~(1u << (lo & 31)));
    }
    const int64_t bl1 = block_sum64(l1), bact = block_sum64(act);
    if (threadIdx.x == 0) {
        atomicAdd(&d.cnt->diag_low_l1, (unsigned long long)bl1);
        atomicAdd(&d.cnt->diag_active, (unsigned long long)bact);
    }
}

__global__ void __launch_bounds__(kBlock) k_diag_count(Dev d, int64_t nwords)
{
    int64_t n = 0;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nwords; w += (int64_t)gridDim.x * blockDim.x)
        n += __popc(d.ess[w]);
    const int64_t bn = block_sum64(n);
    if (threadIdx.x == 0) atomicAdd(&d.cnt->diag_ess, (unsigned long long)bn);
}

// E^0 = [m]: every bit of the first m set
__global__ void k_diag_init(uint32_t *ess, int64_t m, int64_t nwords)
{
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nwords; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rest = m - w * 32;
        ess[w] = rest >= 32 ? ~0u : ((1u << rest) - 1u);
    }
}

// ---------------------------------------------------------------- debug_invariants
// The current low of column j as the round kernels see it: a pivot's low, an
// active column's last row that is not known negative, -1 otherwise.
__device__ inline int32_t dbg_cur_low(const Dev &d, int64_t j, uint8_t st, int compression)
{
    if (st == ST_PIVOT) return d.low[j];
    if (st != ST_ACTIVE) return -1;
    int32_t n = d.len[j];
    const int32_t *c = col_base(d, d.off[j]);
    if (compression)
        while (n > 0 && is_neg(d.neg, c[n - 1])) n--;
    return n > 0 ? c[n - 1] : -1;
}

// After Phase 0 (first = 1: records the starting state) and after every
// round: lows never rise (Sec. 3.1), beta_j <= low(j) and beta_j defined =>
// column j not zero (Thm. "Properties of beta_j" P.5, P.3), a pivot column is
// frozen and named by piv and low_star; and the indices that leave the
// essential estimate this round (known negative columns and every current
// low, eq. "essential_iteration") get the round as their stamp.
__global__ void __launch_bounds__(kBlock) k_dbg_round(Dev d, int compression, int first, int32_t round)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t st = d.state[j];
        const int32_t lo = dbg_cur_low(d, j, st, compression);
        const int32_t b = d.beta[j];
        if (!first) {
            if (lo > d.dbg_low[j]) dbg_fail(d, DBG_LOW_ROSE, j);
            if (d.dbg_state[j] == ST_PIVOT &&
                (st != ST_PIVOT || d.off[j] != d.dbg_off[j] || d.len[j] != d.dbg_len[j] || lo != d.dbg_low[j]))
                dbg_fail(d, DBG_PIVOT_CHANGED, j);
        }
        if (b >= 0 && (st == ST_ZERO || st == ST_CLEARED)) dbg_fail(d, DBG_BETA_ZERO, j);
        if (b >= 0 && lo >= 0 && b > lo) dbg_fail(d, DBG_BETA_ABOVE, j);
        if (st == ST_PIVOT && (lo < 0 || d.piv[lo] != (int32_t)j || d.low_star[j] != lo))
            dbg_fail(d, DBG_PIVOT_TABLE, j);
        d.dbg_low[j] = lo;
        d.dbg_state[j] = st;
        d.dbg_off[j] = d.off[j];
        d.dbg_len[j] = d.len[j];
        if (st == ST_PIVOT || b >= 0) atomicMin(&d.dbg_erem[j], round);
        if (lo >= 0) atomicMin(&d.dbg_erem[lo], round);
    }
}

// After each kernel that writes columns: no column was written twice.
__global__ void __launch_bounds__(kBlock) k_dbg_writes(Dev d)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        if (d.dbg_w[j] > 1) dbg_fail(d, DBG_DOUBLE_WRITE, j);
        d.dbg_w[j] = 0;
    }
}

// After finalisation: low*(j) is the last low seen, beta_j <= low*(j), and no
// essential simplex (low*(i) = -1 and no column's low*) ever left E.
__global__ void __launch_bounds__(kBlock) k_dbg_final(Dev d)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.m; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t ls = d.low_star[j];
        if (ls != d.dbg_low[j] || (d.beta[j] >= 0 && d.beta[j] > ls)) dbg_fail(d, DBG_FINAL, j);
        if (ls >= 0 && d.piv[ls] != (int32_t)j) dbg_fail(d, DBG_PIVOT_TABLE, j);
        if (ls < 0 && d.piv[j] < 0 && d.dbg_erem[j] != 0x7FFFFFFF) dbg_fail(d, DBG_ESS_REMOVED, j);
    }
}

// Twist-order stages: the list to filter has n entries; a stage starts from
// the filtered list and treats its dimension as the top one (nothing can
// clear its columns any more: the dimension above is reduced).
__global__ void k_set_active(Dev d, int32_t n) { d.cnt->n_cur = n; }

__global__ void k_stage_start(Dev d, int32_t topd)
{
    d.cnt->n_cur = d.cnt->n_next;
    d.cnt->topdim = topd;
}

// One complex: instance offsets {0, m}.
__global__ void k_one_instance(int64_t *off, int64_t m)
{
    off[0] = 0;
    off[1] = m;
}

// End of a round: the compacted list is the next round's; a round that did
// work advances the round number (the T table's stamp).
// One wavefront: lane p reads partition p's fill.
__global__ void __launch_bounds__(kWave) k_round_end(Dev d)
{
    static_assert(kPart == kWave, "one lane per arena partition");
    const int p = threadIdx.x;
    const unsigned long long end =
        p == kPart - 1 ? d.arena_cap : d.part_base + (unsigned long long)(p + 1) * d.part_size;
    const unsigned long long cur = d.part[p * 16];
    unsigned long long fr = cur < end ? end - cur : 0;  // a partition past its end is full
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) fr += __shfl_xor(fr, o, kWave);
    if (p == 0) {
        d.cnt->active_sum += (unsigned long long)d.cnt->n_cur;
        if (d.cnt->n_cur > 0) d.cnt->round = d.cnt->round + 1;
        d.cnt->n_cur = d.cnt->n_next;
        d.cnt->arena_free = fr;
    }
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
            // debug_invariants: the move keeps the column's entries (a pivot
            // column that moves has not changed)
            if (d.dbg_off) d.dbg_off[j] = o | (int64_t)kArenaBit;
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

// Partition bump pointers after (re)allocation: partition p starts at
// part_base + p * part_size.
// The reduction's state before Phase 0, in one pass: counters and stripes
// cleared, arena partitions set, and per column left = none, no pivot, no
// low*, the leftmost table empty, the active list 0..m-1; the negative
// bitmask cleared; the round counters (count m, round 0) after the clear.
__global__ void __launch_bounds__(kBlock) k_setup(Dev d, int32_t *act0, int64_t nwords, int64_t nstats, int fill_left)
{
    const int64_t gid = blockIdx.x * (int64_t)kBlock + threadIdx.x, gstride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = gid; j < d.m; j += gstride) {
        if (fill_left) d.left[j] = 0x7FFFFFFF;
        d.piv[j] = -1;
        d.low_star[j] = -1;
        d.T[j] = ~0ull;
        act0[j] = (int32_t)j;
    }
    for (int64_t w = gid; w < nwords; w += gstride) d.neg[w] = 0u;
    for (int64_t w = gid; w < nstats; w += gstride) d.stats[w] = 0ull;
    if (blockIdx.x == 0) {
        unsigned long long *cw = reinterpret_cast<unsigned long long *>(d.cnt);
        for (int w = threadIdx.x; w < (int)(sizeof(Counters) / 8); w += kBlock) cw[w] = 0ull;
        if (threadIdx.x < kPart) d.part[threadIdx.x * 16] = d.part_base + (unsigned long long)threadIdx.x * d.part_size;
        __syncthreads();
        if (threadIdx.x == 0) {
            d.cnt->n_cur = (int32_t)d.m;
            d.cnt->round = 0;
        }
    }
}

__global__ void k_part_init(Dev d)
{
    const int p = threadIdx.x;
    if (p < kPart) d.part[p * 16] = d.part_base + (unsigned long long)p * d.part_size;
}

// Fold the striped counters into the call's Counters.
__global__ void k_stats_fold(Dev d)
{
    __shared__ unsigned long long s_sum[S_NUM];
    if (threadIdx.x < S_NUM) s_sum[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < S_NUM * kStripe; i += blockDim.x)
        atomicAdd(&s_sum[i / kStripe], d.stats[(unsigned)i * 16]);
    __syncthreads();
    if (threadIdx.x == 0) {
        d.cnt->additions = s_sum[S_ADDS];
        d.cnt->xor_entries = s_sum[S_XE];
        d.cnt->xor_bytes = s_sum[S_XBYTES];
        d.cnt->chain_bytes = s_sum[S_CBYTES];
        d.cnt->lane_bytes = s_sum[S_LBYTES];
        d.cnt->wide_bytes = s_sum[S_WBYTES];
        d.cnt->abytes_xor = s_sum[S_ABYTES_XOR];
        d.cnt->abytes_lane = s_sum[S_ABYTES_LANE];
        d.cnt->abytes_wide = s_sum[S_ABYTES_WIDE];
        d.cnt->abytes_chain = s_sum[S_ABYTES_CHAIN];
        d.cnt->solve_bytes = s_sum[S_SBYTES];
        d.cnt->pivot_bytes = s_sum[S_PBYTES];
        d.cnt->abytes_solve = s_sum[S_ABYTES_SOLVE];
        d.cnt->new_pivots = (int32_t)s_sum[S_NEWPIV];
        d.cnt->beta_pivots = (int32_t)s_sum[S_BETAPIV];
        for (int q = 0; q < S_NUM; q++) d.cnt->trace[q] = s_sum[q];
    }
}

// Self-test of the DPP wave reductions against __shfl-based ones on a few
// patterns; writes the number of mismatches.
__global__ void k_selftest(int32_t *bad)
{
    const int lane = threadIdx.x & (kWave - 1);
    int32_t nbad = 0;
    for (int pat = 0; pat < 6; pat++) {
        int32_t v;
        switch (pat) {
        case 0: v = lane; break;
        case 1: v = (lane * 37 + 11) & 1023; break;
        case 2: v = lane == 63 ? 5000 : 0; break;
        case 3: v = lane == 0 ? 7 : 0; break;
        case 4: v = (lane & 15) == 15 ? lane : 1; break;
        default: v = 1 << (lane % 20); break;
        }
        int32_t ref_sum = v, ref_max = v;
        for (int o = 1; o < kWave; o <<= 1) {
            ref_sum += __shfl_xor(ref_sum, o, kWave);
            ref_max = max(ref_max, __shfl_xor(ref_max, o, kWave));
        }
        if (wave_sum_dpp(v) != ref_sum) nbad++;
        if (wave_max_dpp(v) != ref_max) nbad++;
    }
    if (lane == 0) atomicAdd(bad, nbad);
}

// ---------------------------------------------------------------- host
void *grow_scratch(Ctx *c, int id, size_t bytes)
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

// the message for a broken internal invariant reported by a kernel
static std::string bad_source_text(const Counters &h)
{
    if (h.bad_source == 1) return "internal: a column was added a column to its right";
    if (h.bad_source == 4)
        return "internal: k_chain_solve would add a pivot right of column " + std::to_string(h.bad_info[0]);
    std::string m = "internal: a chained addition did not lower the low (";
    if (h.bad_source == 2)
        m += "k_chain: column " + std::to_string(h.bad_info[0]) + ", low " + std::to_string(h.bad_info[1]) +
             " after " + std::to_string(h.bad_info[2]) + ", step " + std::to_string(h.bad_info[3]);
    else
        m += "k_chain_lane or k_chain_wide";
    return m + ")";
}

hipEvent_t prof_event(Ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_flush(Ctx *c)
{
    for (auto &p : c->pend) {
        float ms = 0.f;
        if (p.e0 && p.e1 && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            c->prof_ms[p.kid] += ms;
            c->prof_launches[p.kid] += 1;
            if (p.bytes > 0) c->prof_bytes[p.kid] += p.bytes;
            c->prof_abytes[p.kid] += p.abytes;
        }
        if (p.e0) c->ev_pool.push_back(p.e0);
        if (p.e1) c->ev_pool.push_back(p.e1);
    }
    c->pend.clear();
}

static void set_partitions(Dev &d, unsigned long long used)
{
    d.part_base = used;
    d.part_size = (d.arena_cap - used) / kPart;
}

// Arena regrowth: copy the live columns into an arena at least twice as
// large (and at least min_cap entries), then split the free space into
// fresh partitions.
// Where a reduction's scratch comes from: the context's grow-only buffers
// (allocated on growth), or one fixed device region carved front to back,
// with the column arena taking what is left (the allocation-free entry
// point; then nothing is allocated and the arena cannot grow).
struct ScratchSource {
    Ctx *c = nullptr;
    char *base = nullptr;  // the fixed region, or null for the context's buffers
    size_t cap = 0, used = 0;
    void *get(int id, size_t bytes)
    {
        if (!base) return grow_scratch(c, id, bytes);
        const size_t a = (used + 255) & ~(size_t)255;
        if (a > cap || bytes > cap - a) return nullptr;
        used = a + bytes;
        return base + a;
    }
};

static pms_status grow_arena(Ctx *c, Dev &d, Counters *h, const ScratchSource &S, unsigned long long min_cap = 0)
{
    if (S.base)
        return set_err(c, PMS_ERR_TOO_LARGE,
                       "the column arena of the allocation-free region is full (its fill-in outgrew it); "
                       "use pms_reduce, whose arena grows");
    unsigned long long new_cap = std::max<unsigned long long>(c->arena_cap * 2, min_cap);
    int32_t *na = nullptr;
    PMS_HIP(hipMalloc(&na, new_cap * sizeof(int32_t)));
    unsigned long long *top = (unsigned long long *)grow_scratch(c, B_TMP1, 64);
    if (!top) { (void)hipFree(na); return set_err(c, PMS_ERR_OOM, "scratch alloc"); }
    PMS_LAUNCH(c, K_FILL, 0, k_fill_u64, 1, kBlock, top, 1, 0ull);
    PMS_LAUNCH(c, K_DEFRAG, 0, k_defrag, grid_for(d.m, kBlock, 65536), kBlock, d, na, top);
    PMS_HIP(hipGetLastError());
    unsigned long long ntop = 0;
    PMS_HIP(hipMemcpyAsync(&ntop, top, sizeof(ntop), hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    PMS_HIP(hipFree(c->arena));
    c->arena = na;
    c->arena_cap = new_cap;
    d.arena = na;
    d.arena_cap = new_cap;
    set_partitions(d, ntop);
    PMS_LAUNCH(c, K_FILL, 0, k_part_init, 1, kPart, d);
    h->overflow = 0;
    PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, 1, kBlock, &d.cnt->overflow, 1, 0);
    return PMS_OK;
}

// the options added after the first ones: ranges, and dim where they need it
static bool extra_options_ok(const pms_options &o, const pms_boundary *bnd)
{
    if (o.c8 < 0 || o.c8 > 1 || o.sweep < 0 || o.sweep > 1 || o.priority < 0 || o.priority > 2 ||
        o.round_budget < 0 || o.reserved != 0)
        return false;
    return (bnd->dim || (!o.c8 && !o.sweep)) && (!bnd->left) == (!bnd->beta);
}

static pms_status reduce_impl(Ctx *c, const pms_boundary *bnd, const pms_options *opt, pms_result *res,
                              ScratchSource &S, const int64_t *inst_off, int32_t n_inst)
{
    const int64_t m = bnd->m;
    res->n_pairs = res->n_essential = 0;
    res->rounds = 0;
    res->phase0_pivots = 0;
    res->additions = res->xor_entries = 0;
    res->active_sum = res->addition_bytes = 0;
    c->diag.clear();
    c->diag_m = -1;
    const bool diag = opt->diagnostics != 0;
    const bool dbg = opt->debug_invariants != 0;
    if (m == 0) {
        if (diag) {
            c->diag.push_back(pms_round_stats{0, 0, 0, 0, 0, 0, 0, 0});
            c->diag_m = 0;
        }
        return PMS_OK;
    }

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
    d.off = (int64_t *)S.get(B_OFF, m * 8);
    d.len = (int32_t *)S.get(B_LEN, m * 4);
    d.low = (int32_t *)S.get(B_LOW, m * 4);
    d.state = (uint8_t *)S.get(B_STATE, m);
    // left and beta: the caller's when a builder gave them (read only), else computed in Phase 0
    const bool given_lb = bnd->left && bnd->beta;
    d.beta = given_lb ? const_cast<int32_t *>(bnd->beta) : (int32_t *)S.get(B_BETA, m * 4);
    d.left = given_lb ? const_cast<int32_t *>(bnd->left) : (int32_t *)S.get(B_LEFT, m * 4);
    d.piv = (int32_t *)S.get(B_PIV, m * 4);
    d.T = (unsigned long long *)S.get(B_T, m * 8);
    d.neg = (uint32_t *)S.get(B_NEG, nwords * 4);
    d.coll = (int8_t *)S.get(B_COLL, m);
    d.cnt = (Counters *)S.get(B_CNT, sizeof(Counters));
    d.low_star = res->low_star;
    int32_t *act0 = (int32_t *)S.get(B_ACT0, m * 4);
    int32_t *act1 = (int32_t *)S.get(B_ACT1, m * 4);
    I4 *agg = (I4 *)S.get(B_AGG, nblk * sizeof(I4));
    int32_t *keep = (int32_t *)S.get(B_AGG2, (nblk + 1) * 4);
    int32_t *keep2 = (int32_t *)S.get(B_FLAGS, (nblk + 1) * 4);
    d.cq_slice = (nblk + kPart - 1) / kPart * kBlock;  // a slice takes every kPart-th tile
    d.cq = (int32_t *)S.get(B_TMP0, (size_t)kPart * d.cq_slice * 4);
    d.cq_n = (int32_t *)S.get(B_CQN, (kPart + 3) * 32 * 4);
    d.wq = (int32_t *)S.get(B_WQ, (size_t)m * 4);
    d.wq2 = (int32_t *)S.get(B_WQ2, (size_t)m * 4);
    d.stats = (unsigned long long *)S.get(B_STATS, (size_t)S_NUM * kStripe * 16 * 8);
    d.part = (unsigned long long *)S.get(B_PART, kPart * 16 * 8);
    d.prec = (PivRec *)S.get(B_PREC, (size_t)m * sizeof(PivRec));
    if (!d.off || !d.len || !d.low || !d.state || !d.beta || !d.left || !d.piv || !d.T || !d.neg || !d.coll ||
        !d.cnt || !act0 || !act1 || !agg || !keep || !keep2 || !d.cq || !d.cq_n || !d.stats || !d.part || !d.prec || !d.wq ||
        !d.wq2)
        return S.base ? set_err(c, PMS_ERR_TOO_LARGE, "the matrix does not fit the allocation-free region; use pms_reduce")
                      : set_err(c, PMS_ERR_OOM, "scratch allocation failed");
    if (dbg) {
        d.dbg_low = (int32_t *)S.get(B_DBG_LOW, m * 4);
        d.dbg_off = (int64_t *)S.get(B_DBG_OFF, m * 8);
        d.dbg_len = (int32_t *)S.get(B_DBG_LEN, m * 4);
        d.dbg_state = (uint8_t *)S.get(B_DBG_STATE, m);
        d.dbg_w = (int32_t *)S.get(B_DBG_W, m * 4);
        d.dbg_erem = (int32_t *)S.get(B_DBG_EREM, m * 4);
        if (!d.dbg_low || !d.dbg_off || !d.dbg_len || !d.dbg_state || !d.dbg_w || !d.dbg_erem)
            return set_err(c, S.base ? PMS_ERR_TOO_LARGE : PMS_ERR_OOM, "debug scratch allocation failed");
    }

    // arena: sized for the first rounds' fill-in, grown on demand; in a
    // fixed region, everything the other buffers left
    if (S.base) {
        const size_t a = (S.used + 255) & ~(size_t)255;
        const unsigned long long avail = a < S.cap ? (S.cap - a) / sizeof(int32_t) : 0;
        const unsigned long long need = (unsigned long long)(4 * nnz) + (1ull << 20);
        if (avail < need)
            return set_err(c, PMS_ERR_TOO_LARGE,
                           "the matrix does not fit the allocation-free region (its per-column state and an "
                           "arena of 4 nnz + 2^20 entries); use pms_reduce");
        d.arena = (int32_t *)(S.base + a);
        d.arena_cap = avail;
        S.used = S.cap;
    } else {
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
    }
    set_partitions(d, 0);

    hipStream_t st = c->stream;
    const unsigned gm = grid_for(m, kBlock, 65536);
    const double dm = (double)m, dz = (double)nnz;
    // left, piv, low*, T, the active list; the negative bitmask
    PMS_LAUNCH(c, K_FILL, (given_lb ? 20 : 24) * dm + 4.0 * nwords, k_setup, gm, kBlock, d, act0, (int64_t)nwords,
               (int64_t)S_NUM * kStripe * 16, given_lb ? 0 : 1);
    // col_ptr, rows, left updates, dims (facets and columns), headers out
    // + the 32-byte record of every row (no pivot, not known negative); with
    // left and beta given, no left updates (rows read only to check them) but beta read
    if (given_lb)
        PMS_LAUNCH(c, K_INIT, 8 * dm + (opt->validate ? 4 * dz + (bnd->dim ? dm + dz : 0) : 4 * dm) + 25 * dm + 32 * dm +
                                  4 * dm + dm / 8,
                   k_init, gm, kBlock, d, nnz, opt->validate, 1, opt->compression);
    else
        PMS_LAUNCH(c, K_INIT, 8 * dm + 8 * dz + (bnd->dim ? dm + dz : 0) + 25 * dm + 32 * dm, k_init, gm, kBlock, d,
                   nnz, opt->validate, 0, opt->compression);
    // col_ptr, len, rows, left, beta out, neg bits
    if (!given_lb)
        PMS_LAUNCH(c, K_BETA, 12 * dm + 8 * dz + 4 * dm + dm / 8, k_beta, gm, kBlock, d, opt->compression);
    // priority with a budget: the key histogram (and threshold) and, for
    // priority 1, the sizes of the sets N per low
    const bool budget = opt->round_budget > 0;
    int32_t *bud_h = nullptr, *bud_n = nullptr;
    if (budget) {
        bud_h = (int32_t *)S.get(B_BUDH, (kBudKeys + 3) * 4);
        if (opt->priority == 1) bud_n = (int32_t *)S.get(B_BUDN, (size_t)m * 4);
        if (!bud_h || (opt->priority == 1 && !bud_n)) return set_err(c, PMS_ERR_OOM, "round budget scratch");
        PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, 1, kBlock, bud_h, (int64_t)kBudKeys + 3, 0);
        if (bud_n) PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, gm, kBlock, bud_n, m, 0);
    }
    // clearing by local compression: the complexes and their first unpaired rows
    const bool c8on = opt->c8 != 0;
    d.inst_off = nullptr;
    d.n_inst = 0;
    d.c8_first = nullptr;
    if (c8on) {
        if (!inst_off) {
            int64_t *one = (int64_t *)S.get(B_INST, 16);
            if (!one) return set_err(c, PMS_ERR_OOM, "instance offsets");
            PMS_LAUNCH(c, K_FILL, 0, k_one_instance, 1, 1, one, m);
            inst_off = one;
            n_inst = 1;
        }
        d.inst_off = inst_off;
        d.n_inst = n_inst;
        d.c8_first = (int32_t *)S.get(B_C8, (size_t)n_inst * kC8Stride * 4);
        if (!d.c8_first) return set_err(c, PMS_ERR_OOM, "clearing-by-compression scratch");
        // first rows 0 (scan from each instance's start); end: every row (m)
        PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, grid_for((int64_t)n_inst * kC8Stride), kBlock, d.c8_first,
                   (int64_t)n_inst * kC8Stride, 0);
        PMS_LAUNCH(c, K_FILL, 0, k_c8_reset_end, grid_for(n_inst), kBlock, d);
    }
    if (dbg) {
        PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, gm, kBlock, d.dbg_w, m, 0);
        PMS_LAUNCH(c, K_FILL, 0, k_fill_i32, gm, kBlock, d.dbg_erem, m, 0x7FFFFFFF);
        PMS_LAUNCH(c, K_FILL, 0, k_dbg_round, gm, kBlock, d, opt->compression, 1, 0);
    }
    PMS_HIP(hipGetLastError());

    Counters *h = (Counters *)c->host_pinned;
    PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    PMS_HIP(hipStreamSynchronize(st));
    if (h->error) return set_err(c, PMS_ERR_NOT_COMPATIBLE, "boundary matrix is not that of a compatible filtration "
                                                            "(rows must ascend, lie above the diagonal and be facets)");
    // debug_invariants: the first broken property, by name
    auto dbg_check = [&](const char *where, int32_t r) -> pms_status {
        if (!h->dbg_flags) return PMS_OK;
        static const char *const names[] = {
            "a column's low increased (lows only decrease, Sec. 3.1)",
            "beta_j > low(j) (Thm. \"Properties of beta_j\" P.5)",
            "a column with beta_j defined became zero (Thm. \"Properties of beta_j\" P.3)",
            "a pivot column changed after it was found",
            "piv / low_star do not name a pivot column",
            "a column was written twice by one kernel launch",
            "an essential simplex left the essential estimate (Lemma \"Essential estimation\")",
            "low* differs from the last low, or beta_j > low*(j)"};
        int bit = 0;
        while (!((h->dbg_flags >> bit) & 1)) bit++;
        return set_err(c, PMS_ERR_INVARIANT,
                       std::string("invariant broken ") + where + " " + std::to_string(r) + ": " + names[bit] +
                           " (column or row " + std::to_string(h->dbg_col) + ", flags " +
                           std::to_string(h->dbg_flags) + ")");
    };
    {
        const pms_status sdb = dbg_check("after Phase 0, round", 0);
        if (sdb != PMS_OK) return sdb;
    }

    int32_t nA = (int32_t)m;
    uint32_t round = 0;
    unsigned long long xor_bytes_prev = 0, chain_bytes_prev = 0, lane_bytes_prev = 0, wide_bytes_prev = 0;
    unsigned long long solve_bytes_prev = 0, pivot_bytes_prev = 0;
    unsigned long long ab_prev[5] = {0, 0, 0, 0, 0};
    const char *tr_env = getenv("PMS_TRACE");
    const int trace = tr_env && tr_env[0] == '1';
    unsigned long long tprev[S_NUM] = {};
    int32_t nA_prev = 0;
    int32_t *act = act0, *act_next = act1;
    // One round (Phase I, Phase II, compaction) on the list `a` into `an`.
    // The kernels read the round's active count and number from the device
    // (they loop over tiles), so `grid_tiles` only bounds their grids: the
    // exact tile count when the host knows it, a fixed size in a graph.
    size_t xor_slot = 0, lane_slot = 0, wide_slot = 0, chain_slot = 0, solve_slot = 0, pivots_slot = 0;
    double pivots_base = 0;
    const pms_tuning tn = c->tune;
    auto launch_round = [&](const int32_t *a, int32_t *an, int64_t grid_tiles, double dA) -> pms_status {
        const unsigned gT = (unsigned)(grid_tiles > 0 ? grid_tiles : 1);
        // the chaining kernels take queued columns (at most the active ones)
        // in wavefront-sized chunks over any grid: with the active count known
        // (dA > 0), no more workgroups than it can use
        auto chain_grid = [&](int64_t tuned, int64_t cols_per_block) -> unsigned {
            if (dA <= 0) return (unsigned)tuned;
            const int64_t need = ((int64_t)dA + cols_per_block - 1) / cols_per_block;
            return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tuned, need));
        };
        const unsigned g_lane = chain_grid(tn.lane_blocks, kLaneThreads), g_wide = chain_grid(tn.wide_blocks, kWideThreads);
        const unsigned g_solve = chain_grid(tn.chain_blocks, 1), g_chain = chain_grid(tn.chain_blocks, kChainWaves);
        const unsigned gA = grid_for(grid_tiles * kBlock, kBlock, 65536);
        const double dt = (double)grid_tiles;
        // act, len, off, last row, low out, T atomic
        PMS_LAUNCH(c, K_LOW, 32 * dA, k_low, gA, kBlock, d, a);
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        // act, state, low, T, piv, coll out, dim; block aggregates
        PMS_LAUNCH(c, K_COLLIDE, 23 * dA + 16 * dt, k_collide, gT, kBlock, d, a, agg);
        PMS_LAUNCH(c, K_SCAN, 32 * dt, k_scan_max4, 1, kScanThreads, agg, &d.cnt->n_cur);
        // act, state, low, coll, dim, beta; aggregates
        PMS_LAUNCH(c, K_PIVOTS, -1.0, k_pivots, gT, kBlock, d, a, agg, opt->compression);
        pivots_slot = c->pend.size() - 1;
        pivots_base = 15 * dA + 16 * dt;  // act, coll, low, beta, dim, scan aggregates; + the new pivots' bytes
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        if (c8on) {
            // the first unpaired rows (a scan from the last ones, usually short); act, dim, beta, state, low
            const unsigned gi = grid_for(d.n_inst, kBlock, 4096);
            PMS_LAUNCH(c, K_C8, 0, k_c8_range, gi, kBlock, d);
            if (d.n_inst >= 512) PMS_LAUNCH(c, K_C8, 0, k_c8_scan<2>, (unsigned)std::min<int64_t>(2LL * d.n_inst, 4096), kBlock, d);
            else if (d.n_inst >= 16) PMS_LAUNCH(c, K_C8, 0, k_c8_scan<32>, (unsigned)std::min<int64_t>(32LL * d.n_inst, 4096), kBlock, d);
            else PMS_LAUNCH(c, K_C8, 0, k_c8_scan<1024>, (unsigned)std::min<int64_t>(1024LL * d.n_inst, 4096), kBlock, d);
            PMS_LAUNCH(c, K_C8, 0, k_c8_fold, gi, kBlock, d);
            PMS_LAUNCH(c, K_C8, 14 * dA, k_c8_clear, gT, kBlock, d, a);
            if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        }
        if (budget) {  // which colliding columns add this round
            const int pr = opt->priority, va = opt->variant;
            if (pr == 1) PMS_LAUNCH(c, K_BUDGET, 0, k_bud_ncount, gA, kBlock, d, a, va, bud_n, 1);
            PMS_LAUNCH(c, K_BUDGET, 0, k_bud_hist, gA, kBlock, d, a, va, pr, bud_n, bud_h);
            PMS_LAUNCH(c, K_BUDGET, 0, k_bud_thresh, 1, kWave, bud_h, opt->round_budget);
            PMS_LAUNCH(c, K_BUDGET, 0, k_bud_count, gT, kBlock, d, a, va, pr, bud_n, bud_h, keep2);
            PMS_LAUNCH(c, K_SCAN, 0, k_scan_sum, 1, kScanThreads, keep2, 0, &d.cnt->n_cur, bud_h + kBudKeys + 2);
            PMS_LAUNCH(c, K_BUDGET, 0, k_bud_apply, gT, kBlock, d, a, va, pr, bud_n, bud_h, keep2);
            if (pr == 1) PMS_LAUNCH(c, K_BUDGET, 0, k_bud_ncount, gA, kBlock, d, a, va, bud_n, -1);
        }
        PMS_LAUNCH(c, K_XOR, -1.0, k_xor, gT, kBlock, d, a, opt->variant, opt->compression, opt->chain,
                   opt->tail_active);
        xor_slot = c->pend.size() - 1;
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        if (trace)
            PMS_LAUNCH(c, K_CHAIN_LANE, -1.0, k_chain_lane<true>, g_lane, kLaneThreads, d, opt->compression, tn);
        else
            PMS_LAUNCH(c, K_CHAIN_LANE, -1.0, k_chain_lane<false>, g_lane, kLaneThreads, d, opt->compression, tn);
        lane_slot = c->pend.size() - 1;
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        if (trace)
            PMS_LAUNCH(c, K_CHAIN_WIDE, -1.0, k_chain_wide<true>, g_wide, kWideThreads, d, opt->compression, tn);
        else
            PMS_LAUNCH(c, K_CHAIN_WIDE, -1.0, k_chain_wide<false>, g_wide, kWideThreads, d, opt->compression, tn);
        wide_slot = c->pend.size() - 1;
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        if (tn.solve > 0) {  // few handed-over columns: by sweeps; what does not fit, serially
            if (trace)
                PMS_LAUNCH(c, K_SOLVE, -1.0, k_chain_solve<true>, g_solve, kSolveThreads, d, opt->compression,
                           tn.solve);
            else
                PMS_LAUNCH(c, K_SOLVE, -1.0, k_chain_solve<false>, g_solve, kSolveThreads, d, opt->compression,
                           tn.solve);
            solve_slot = c->pend.size() - 1;
            if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        }
        if (trace)
            PMS_LAUNCH(c, K_CHAIN, -1.0, k_chain<true>, g_chain, kChainWaves * kWave, d, opt->compression, tn.solve);
        else
            PMS_LAUNCH(c, K_CHAIN, -1.0, k_chain<false>, g_chain, kChainWaves * kWave, d, opt->compression, tn.solve);
        chain_slot = c->pend.size() - 1;
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        PMS_LAUNCH(c, K_COMPACT, 5 * dA, k_keep_count, gT, kBlock, d, a, keep, -1);
        PMS_LAUNCH(c, K_SCAN, 8 * dt, k_scan_sum, 1, kScanThreads, keep, 0, &d.cnt->n_cur, &d.cnt->n_next);
        // act, state, act_next
        PMS_LAUNCH(c, K_COMPACT, 9 * dA, k_compact, gT, kBlock, d, a, keep, an, -1);
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_writes, gm, kBlock, d);
        if (c->prof_on || trace || diag) PMS_LAUNCH(c, K_FILL, 0, k_stats_fold, 1, 256, d);
        PMS_LAUNCH(c, K_FILL, 0, k_round_end, 1, kWave, d);
        return PMS_OK;
    };
    // diagnostics after Phase 0 and after each round: low^l's l1 norm, the
    // unreduced columns and the essential estimate, read with the round's counters
    auto launch_diag = [&]() -> pms_status {
        PMS_LAUNCH(c, K_FILL, 0, k_diag_reset, 1, 1, d);
        PMS_LAUNCH(c, K_FILL, 13.0 * dm, k_diag_update, gm, kBlock, d, opt->compression);
        PMS_LAUNCH(c, K_FILL, 4.0 * nwords, k_diag_count, grid_for(nwords, kBlock, 65536), kBlock, d, nwords);
        return PMS_OK;
    };
    unsigned long long diag_adds = 0, diag_xe = 0, diag_np = 0, diag_c8 = 0;
    auto record_diag = [&](int32_t r) {
        pms_round_stats e;
        e.round = r;
        e.active = (int32_t)h->diag_active;
        e.new_pivots = (int64_t)((unsigned long long)h->new_pivots - diag_np);
        e.additions = (int64_t)(h->additions - diag_adds);
        e.xor_entries = (int64_t)(h->xor_entries - diag_xe);
        e.low_l1 = (int64_t)h->diag_low_l1;
        e.ess_estimate = (int64_t)h->diag_ess;
        e.c8_cleared = (int64_t)(h->c8_cleared - diag_c8);
        diag_c8 = h->c8_cleared;
        diag_np = (unsigned long long)h->new_pivots;
        diag_adds = h->additions;
        diag_xe = h->xor_entries;
        c->diag.push_back(e);
    };
    if (diag) {
        d.ess = (uint32_t *)S.get(B_ESS, (size_t)nwords * 4);
        if (!d.ess) return set_err(c, PMS_ERR_OOM, "diagnostics scratch");
        PMS_LAUNCH(c, K_FILL, 4.0 * nwords, k_diag_init, grid_for(nwords, kBlock, 65536), kBlock, d.ess, m, nwords);
        pms_status sd = launch_diag();
        if (sd != PMS_OK) return sd;
        PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
        PMS_HIP(hipStreamSynchronize(st));
        record_diag(0);
        c->diag_m = m;
    }

    // The arena grows (live columns copied into one twice as large) when a
    // round runs it out, which drops that round's remaining progress, and
    // before that happens: when the free part left after a round (or a graph
    // replay of rounds) is less than twice what it took.
    // Grown early, it takes at least what is in use plus four times the last
    // round's take, so the rounds after it (and later calls, which start from
    // the kept arena) do not grow it again.
    unsigned long long free_prev = d.arena_cap - d.part_base, want_cap = 0;
    auto grow_early = [&](int32_t n_left, const Counters *hc) {
        const unsigned long long took = free_prev > hc->arena_free ? free_prev - hc->arena_free : 0;
        free_prev = hc->arena_free;
        want_cap = (d.arena_cap - hc->arena_free) + 4 * took;
        return n_left > 0 && hc->arena_free < 2 * took;
    };

    // Graph mode: `graph_rounds` rounds (rounded up to even, so the active
    // list ends where it started) captured once into a HIP graph and
    // replayed, one host synchronisation per replay; rounds after
    // convergence find no active column and return at once.
    const int graph_k = (opt->graph_rounds > 0 && !c->prof_on && !trace && !diag && !dbg && opt->max_rounds == 0)
                            ? (opt->graph_rounds + 1) & ~1 : 0;
    // Twist order (pms_options.sweep): one stage per dimension, from the top
    // down; a stage's first list holds the active columns of its dimension,
    // and the stage runs rounds until none is left.  Without it one stage
    // holds every column.
    int32_t sd = opt->sweep ? h->topdim : -1;
    auto stage_build = [&](int32_t dsel) -> pms_status {
        const int64_t tiles_m = (m + kBlock - 1) / kBlock;
        const unsigned gTm = (unsigned)(tiles_m > 0 ? tiles_m : 1);
        PMS_LAUNCH(c, K_FILL, 4 * dm, k_iota, gm, kBlock, act1, m);
        PMS_LAUNCH(c, K_FILL, 0, k_set_active, 1, 1, d, (int32_t)m);
        PMS_LAUNCH(c, K_COMPACT, 6 * dm, k_keep_count, gTm, kBlock, d, act1, keep, (int)dsel);
        PMS_LAUNCH(c, K_SCAN, 8.0 * tiles_m, k_scan_sum, 1, kScanThreads, keep, 0, &d.cnt->n_cur, &d.cnt->n_next);
        PMS_LAUNCH(c, K_COMPACT, 10 * dm, k_compact, gTm, kBlock, d, act1, keep, act0, (int)dsel);
        PMS_LAUNCH(c, K_FILL, 0, k_stage_start, 1, 1, d, dsel);
        if (c8on) PMS_LAUNCH(c, K_FILL, 0, k_c8_reset_end, grid_for(d.n_inst), kBlock, d);
        PMS_HIP(hipGetLastError());
        PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
        PMS_HIP(hipStreamSynchronize(st));
        act = act0;
        act_next = act1;
        nA = h->n_cur;
        return PMS_OK;
    };
    if (sd >= 0) {
        const pms_status sb = stage_build(sd);
        if (sb != PMS_OK) return sb;
    }
    for (;;) {
    if (graph_k > 0 && nA > 0) {
        // fixed grids: enough blocks to fill the device, looping over tiles
        const int64_t gtiles = std::min<int64_t>((m + kBlock - 1) / kBlock, 2048);
        if (!c->graph_stream) PMS_HIP(hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking));
        if (!c->graph_ev) PMS_HIP(hipEventCreateWithFlags(&c->graph_ev, hipEventDisableTiming));
        hipStream_t gs = c->graph_stream;
        // the graph runs after everything issued on the caller's stream so far
        PMS_HIP(hipEventRecord(c->graph_ev, st));
        PMS_HIP(hipStreamWaitEvent(gs, c->graph_ev, 0));
        // everything the captured launches depend on
        auto make_key = [&]() {
            std::vector<unsigned char> k(sizeof(Dev) + sizeof(pms_options) + sizeof(pms_tuning) + 5 * sizeof(void *) +
                                         2 * sizeof(int64_t));
            unsigned char *p = k.data();
            memcpy(p, &d, sizeof(Dev));
            p += sizeof(Dev);
            memcpy(p, &tn, sizeof(tn));
            p += sizeof(tn);
            pms_options o2 = *opt;
            memcpy(p, &o2, sizeof(o2));
            p += sizeof(o2);
            const void *ptrs[5] = {act0, act1, agg, keep, (const void *)(intptr_t)graph_k};
            memcpy(p, ptrs, sizeof(ptrs));
            p += sizeof(ptrs);
            const int64_t sz[2] = {gtiles, m};
            memcpy(p, sz, sizeof(sz));
            return k;
        };
        auto capture = [&]() -> pms_status {
            if (c->graph_exec) {
                (void)hipGraphExecDestroy(c->graph_exec);
                c->graph_exec = nullptr;
                c->graph_key.clear();
            }
            hipGraph_t graph = nullptr;
            PMS_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
            c->stream = gs;  // PMS_LAUNCH issues on c->stream
            pms_status sr = PMS_OK;
            for (int r = 0; r < graph_k && sr == PMS_OK; r++)
                sr = (r & 1) ? launch_round(act1, act0, gtiles, 0.0) : launch_round(act0, act1, gtiles, 0.0);
            c->stream = st;
            const hipError_t ec = hipStreamEndCapture(gs, &graph);
            if (sr != PMS_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return sr;
            }
            PMS_HIP(ec);
            hipGraphExec_t exec = nullptr;
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            PMS_HIP(ei);
            c->graph_exec = exec;
            c->graph_key = make_key();
            return PMS_OK;
        };
        if (!c->graph_exec || c->graph_key != make_key()) {
            pms_status sg = capture();
            if (sg != PMS_OK) return sg;
        }
        for (;;) {
            hipError_t e = hipGraphLaunch(c->graph_exec, gs);
            if (e == hipSuccess) e = hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, gs);
            if (e == hipSuccess) e = hipStreamSynchronize(gs);
            if (e != hipSuccess) return set_err(c, PMS_ERR_HIP, std::string("graph round: ") + hipGetErrorString(e));
            round = h->round;
            if (h->bad_source) return set_err(c, PMS_ERR_HIP, bad_source_text(*h));
            if (h->overflow || (!S.base && grow_early(h->n_cur, h))) {  // the arena moves: grow it (on the caller's stream) and capture again
                pms_status s = grow_arena(c, d, h, S, h->overflow ? 0 : want_cap);
                if (s != PMS_OK) return s;
                free_prev = d.arena_cap - d.part_base;
                PMS_HIP(hipEventRecord(c->graph_ev, st));
                PMS_HIP(hipStreamWaitEvent(gs, c->graph_ev, 0));
                s = capture();
                if (s != PMS_OK) return s;
                continue;
            }
            if (h->n_cur == 0) break;
        }
        nA = 0;
    }
    // Pipelined rounds: once few columns are active, the next round is queued
    // before this one's counters reach the host.  The active list only
    // shrinks, so the count a round started with bounds the next round's grid
    // (an oversized grid costs little at that size), and a round queued after
    // convergence finds no active column and returns at once.  Consecutive
    // rounds' counters land in two pinned buffers, each behind its own event.
    // Off where the host acts on every round before the next may start
    // (profiling, traces, diagnostics, invariant checks, a round cap) and for
    // the c8 and budget options.
    constexpr int32_t kPipeCols = 1 << 18;
    if (nA > 0 && !c->prof_on && !trace && !diag && !dbg && opt->max_rounds == 0 && !c8on && !budget) {
        Counters *hb[2] = {h, h + 1};
        auto queue = [&](const int32_t *a, int32_t *an, int32_t bound, int q) -> pms_status {
            const pms_status sr = launch_round(a, an, (bound + kBlock - 1) / kBlock, (double)bound);
            if (sr != PMS_OK) return sr;
            PMS_HIP(hipGetLastError());
            PMS_HIP(hipMemcpyAsync(hb[q], d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
            PMS_HIP(hipEventRecord(c->pipe_ev[q], st));
            return PMS_OK;
        };
        int q = 0;
        pms_status sr = queue(act, act_next, nA, q);
        if (sr != PMS_OK) return sr;
        bool grown = false;  // the round read next ran before the arena moved
        for (;;) {
            // the round reading `act` is queued, its counters going to hb[q]
            const bool ahead = nA <= kPipeCols;
            if (ahead) {  // queue the one after it
                sr = queue(act_next, act, nA, q ^ 1);
                if (sr != PMS_OK) return sr;
            }
            PMS_HIP(hipEventSynchronize(c->pipe_ev[q]));
            const Counters *hr = hb[q];
            round++;
            if (hr->bad_source) return set_err(c, PMS_ERR_HIP, bad_source_text(*hr));
            const int32_t nn = hr->n_next;
            if (grown) {
                grown = false;  // its arena figures are the old arena's
            } else if (hr->overflow || (!S.base && grow_early(nn, hr))) {
                // the arena moves once a queued round is done (grow_arena waits for it)
                const pms_status s = grow_arena(c, d, hb[q], S, hr->overflow ? 0 : want_cap);
                if (s != PMS_OK) return s;
                free_prev = d.arena_cap - d.part_base;
                grown = ahead;
            }
            if (nn == 0) break;  // a queued round finds no active column
            std::swap(act, act_next);
            nA = nn;
            q ^= 1;
            if (!ahead) {  // the next round, its grid from the count just read
                sr = queue(act, act_next, nA, q);
                if (sr != PMS_OK) return sr;
            }
        }
        nA = 0;
    }
    while (nA > 0) {
        if (opt->max_rounds > 0 && (int32_t)round >= opt->max_rounds) {
            res->rounds = (int32_t)round;
            return set_err(c, PMS_ERR_NOT_CONVERGED, "max_rounds reached before the reduction converged");
        }
        nA_prev = nA;
        const int64_t tiles = (nA + kBlock - 1) / kBlock;
        pms_status sr = launch_round(act, act_next, tiles, (double)nA);
        if (sr != PMS_OK) return sr;
        if (diag) {
            sr = launch_diag();
            if (sr != PMS_OK) return sr;
        }
        if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_round, gm, kBlock, d, opt->compression, 0, (int32_t)round + 1);
        PMS_HIP(hipGetLastError());
        PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
        PMS_HIP(hipStreamSynchronize(st));
        round++;
        if (diag) record_diag((int32_t)round);
        if (c->prof_on) {
            c->pend[xor_slot].bytes = (double)(h->xor_bytes - xor_bytes_prev);
            xor_bytes_prev = h->xor_bytes;
            c->pend[pivots_slot].bytes = pivots_base + (double)(h->pivot_bytes - pivot_bytes_prev);
            pivot_bytes_prev = h->pivot_bytes;
            c->pend[chain_slot].bytes = (double)(h->chain_bytes - chain_bytes_prev);
            chain_bytes_prev = h->chain_bytes;
            c->pend[lane_slot].bytes = (double)(h->lane_bytes - lane_bytes_prev);
            lane_bytes_prev = h->lane_bytes;
            c->pend[wide_slot].bytes = (double)(h->wide_bytes - wide_bytes_prev);
            wide_bytes_prev = h->wide_bytes;
            const unsigned long long abn[5] = {h->abytes_xor, h->abytes_lane, h->abytes_wide, h->abytes_chain,
                                               h->abytes_solve};
            const size_t slots[5] = {xor_slot, lane_slot, wide_slot, chain_slot, solve_slot};
            const int nslots = tn.solve > 0 ? 5 : 4;
            if (tn.solve > 0) {
                c->pend[solve_slot].bytes = (double)(h->solve_bytes - solve_bytes_prev);
                solve_bytes_prev = h->solve_bytes;
            }
            for (int q = 0; q < nslots; q++) {
                c->pend[slots[q]].abytes = (double)(abn[q] - ab_prev[q]);
                ab_prev[q] = abn[q];
            }
            prof_flush(c);
        }
        if (trace) {
            unsigned long long dl[S_NUM];
            for (int q = 0; q < S_NUM; q++) { dl[q] = h->trace[q] - tprev[q]; tprev[q] = h->trace[q]; }
            const double st = (double)(dl[S_T_SHORT] ? dl[S_T_SHORT] : 1);
            fprintf(stderr,
                    "pms round %u: active %d -> %d, new pivots %llu, additions %llu, lane steps %llu, to the wide "
                    "pass %llu, wide steps %llu, handed to waves "
                    "%llu, chain steps short %llu long %llu global %llu, mean |W| %.1f, lows from P %llu, flushes "
                    "%llu, deletions %llu, longest chain %d, cycles/short step: toggle %.0f next %.0f flush %.0f; lane steps: "
                    "mean L %.1f, L>16 %llu, L>32 %llu, long-pivot steps %llu, toggles %llu; first lane pass: toggle rounds %llu, wave iterations %llu, refill phases %llu, "
                    "merge phases %llu, busy lanes per iteration %.1f, steps per iteration %.1f; solve: columns %llu, "
                    "sweeps %llu, most sweeps %d, to k_chain %llu, cycles: set-up %llu, pass A %llu, pass B %llu, "
                    "toggles %llu, out %llu, changes %llu, longest column %d us, long pivots %llu (entries %llu), deferred changes %llu\n",
                    round, nA_prev, h->n_next, dl[S_NEWPIV], dl[S_ADDS], dl[S_T_LANE], dl[S_T_TOWIDE], dl[S_T_WIDE],
                    dl[S_T_QUEUED], dl[S_T_SHORT],
                    dl[S_T_LONG], dl[S_T_GLOBAL],
                    (double)dl[S_T_SUML] / (double)((dl[S_T_SHORT] + dl[S_T_LONG] + dl[S_T_GLOBAL]) ? (dl[S_T_SHORT] + dl[S_T_LONG] + dl[S_T_GLOBAL]) : 1),
                    dl[S_T_FROMP], dl[S_T_FLUSHES], dl[S_T_DEL], h->max_chain, dl[S_T_CTOG] / st, dl[S_T_CNEXT] / st, dl[S_T_CFLUSH] / st,
                    (double)dl[S_T_LSUML] / (double)(dl[S_T_LANE] ? dl[S_T_LANE] : 1), dl[S_T_LGT16], dl[S_T_LGT32], dl[S_T_LLONG], dl[S_T_LTOG], dl[S_T_LTROUND],
                    dl[S_T_LITER], dl[S_T_LREFILL], dl[S_T_LFLUSH],
                    (double)dl[S_T_LBUSY] / (double)(dl[S_T_LITER] ? dl[S_T_LITER] : 1),
                    (double)dl[S_T_LANE] / (double)(dl[S_T_LITER] ? dl[S_T_LITER] : 1), dl[S_T_SOLVED],
                    dl[S_T_SWEEPS], h->max_sweeps, dl[S_T_SFALL], dl[S_T_SINIT], dl[S_T_SA], dl[S_T_SB], dl[S_T_SC],
                    dl[S_T_SOUT], dl[S_T_SDELTA], h->max_solve_us, dl[S_T_SLONG], dl[S_T_SLONGE], dl[S_T_SDEFER]);
        }
        if (h->bad_source) return set_err(c, PMS_ERR_HIP, bad_source_text(*h));
        {
            const pms_status sdb = dbg_check("in round", (int32_t)round);
            if (sdb != PMS_OK) return sdb;
        }
        if (h->overflow || (!S.base && grow_early(h->n_next, h))) {
            pms_status s = grow_arena(c, d, h, S, h->overflow ? 0 : want_cap);
            if (s != PMS_OK) return s;
            free_prev = d.arena_cap - d.part_base;
        }
        nA_prev = h->n_next;
        nA = h->n_next;
        std::swap(act, act_next);
    }
    if (sd <= 0) break;
    sd--;
    const pms_status sb = stage_build(sd);
    if (sb != PMS_OK) return sb;
    }
    PMS_LAUNCH(c, K_FILL, 0, k_stats_fold, 1, 256, d);
    if (dbg) PMS_LAUNCH(c, K_FILL, 0, k_dbg_final, gm, kBlock, d);
    PMS_HIP(hipMemcpyAsync(h, d.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    PMS_HIP(hipStreamSynchronize(st));
    {
        const pms_status sdb = dbg_check("at the end, after round", (int32_t)round);
        if (sdb != PMS_OK) return sdb;
    }
    res->rounds = (int32_t)round;
    res->additions = (int64_t)h->additions;
    res->xor_entries = (int64_t)h->xor_entries;
    res->active_sum = (int64_t)h->active_sum;
    res->addition_bytes =
        (int64_t)(h->abytes_xor + h->abytes_lane + h->abytes_wide + h->abytes_chain + h->abytes_solve);
    res->phase0_pivots = h->beta_pivots;

    // pairs and essential simplices, canonical order
    int32_t *cp = keep, *ce = keep2;
    PMS_LAUNCH(c, K_FINAL, 8 * dm, k_fin_count, (unsigned)nblk, kBlock, d, cp, ce);
    PMS_LAUNCH(c, K_SCAN, 16.0 * nblk, k_scan_sum2, 2, kScanThreads, cp, ce, nblk, &d.cnt->n_pairs, &d.cnt->n_ess);
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
        PMS_LAUNCH(c, K_FINAL, 8 * dm + 8.0 * res->n_pairs + 4.0 * res->n_essential, k_fin_scatter,
                   (unsigned)nblk, kBlock, d, cp, ce, want_pairs ? res->pair_birth : nullptr,
                   want_pairs ? res->pair_death : nullptr, want_ess ? res->essential : nullptr);
        PMS_HIP(hipGetLastError());
        PMS_HIP(hipStreamSynchronize(st));
    }
    if (c->prof_on) prof_flush(c);
    return PMS_OK;
}

}  // namespace pms

// ==================================================================== ABI
struct pms_ctx : pms::Ctx {};

// The device region of the allocation-free entry point (pms_reduce_noalloc):
// PMS_NOALLOC_BYTES bytes on every device the library runs on, held until the
// process ends.  In host code this name is a host-side stand-in, not a device
// address: the device address of each device's copy comes from
// hipGetSymbolAddress (in pms_create, with that device current) and is kept
// in noalloc_ptr[device]; only that pointer is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[PMS_NOALLOC_BYTES];
constexpr int kNoAllocDevices = 64;
static void *noalloc_ptr[kNoAllocDevices];
static std::mutex noalloc_mu;

namespace pms {

__device__ inline int64_t lower_bound_i64(const int32_t *a, int64_t n, int64_t x)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Where each instance's pairs and essential simplices start: the outputs are
// ascending in the death (resp. essential) index and instance b owns the
// columns [col_off[b], col_off[b+1]), so one lower bound per instance.
__global__ void k_inst_offsets(int32_t count, const int64_t *col_off, const int32_t *pair_death, int64_t n_pairs,
                               const int32_t *essential, int64_t n_ess, int64_t *pair_off, int64_t *ess_off)
{
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= count; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = col_off[b];
        if (pair_off) pair_off[b] = pair_death ? lower_bound_i64(pair_death, n_pairs, c) : 0;
        if (ess_off) ess_off[b] = essential ? lower_bound_i64(essential, n_ess, c) : 0;
    }
}

// The instance of every pair (the one owning its death column).
__global__ void k_pair_inst(int32_t count, const int64_t *col_off, const int32_t *pair_death, int64_t n_pairs,
                            int32_t *pair_inst)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_pairs; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = pair_death[k];
        int32_t lo = 0, hi = count - 1;  // last instance whose first column is <= j
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (col_off[mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        pair_inst[k] = lo;
    }
}

}  // namespace pms

extern "C" {

const char *pms_version(void) { return "pms-gfx950 0.2"; }

pms_options pms_default_options(void)
{
    pms_options o;
    o.variant = 0;
    o.compression = 1;
    o.max_rounds = 0;
    o.chain = 1;
    o.tail_active = 1024;
    o.validate = 1;
    o.graph_rounds = 0;
    o.diagnostics = 0;
    o.arena_entries = 0;
    o.debug_invariants = 0;
    o.c8 = 0;
    o.sweep = 0;
    o.priority = 0;
    o.round_budget = 0;
    o.reserved = 0;
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
    if (hipHostMalloc(&c->host_pinned, 2 * sizeof(pms::Counters), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return PMS_ERR_OOM;
    }
    for (int q = 0; q < 2; q++)
        if (hipEventCreateWithFlags(&c->pipe_ev[q], hipEventDisableTiming) != hipSuccess) {
            for (int k = 0; k < q; k++) (void)hipEventDestroy(c->pipe_ev[k]);
            (void)hipHostFree(c->host_pinned);
            delete c;
            return PMS_ERR_HIP;
        }
    // once per device: the device address of its copy of the allocation-free region
    if (device < kNoAllocDevices) {
        std::lock_guard<std::mutex> lk(noalloc_mu);
        if (!noalloc_ptr[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                for (int q = 0; q < 2; q++) (void)hipEventDestroy(c->pipe_ev[q]);
                (void)hipHostFree(c->host_pinned);
                delete c;
                return PMS_ERR_HIP;
            }
            noalloc_ptr[device] = p;
        }
    }
    *ctx = c;
    return PMS_OK;
}

void pms_destroy(pms_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    pms::prof_flush(c);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto &b : c->b)
        if (b.p) (void)hipFree(b.p);
    if (c->arena) (void)hipFree(c->arena);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph_ev) (void)hipEventDestroy(c->graph_ev);
    for (auto e : c->pipe_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->graph_stream) (void)hipStreamDestroy(c->graph_stream);
    delete c;
}

static const char *const kKernelNames[pms::K_NUM] = {
    "k_init", "k_beta", "k_low", "k_collide", "k_scan", "k_pivots", "k_xor", "k_compact", "k_finalize", "k_fill",
    "k_defrag", "k_ls_keys", "k_sort", "k_ls_index", "k_build_scan", "k_ls_rows", "k_vr_edges", "k_vr_tri",
    "k_vr_index", "k_vr_rows", "k_backward", "k_chain", "k_chain_lane", "k_chain_wide", "k_c8", "k_budget",
    "k_chain_solve", "k_ls_left"};

pms_status pms_profile_enable(pms_ctx *c, int enable)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(c->stream);
    pms::prof_flush(c);
    for (int k = 0; k < pms::K_NUM; k++) {
        c->prof_ms[k] = 0;
        c->prof_bytes[k] = 0;
        c->prof_abytes[k] = 0;
        c->prof_launches[k] = 0;
    }
    c->prof_on = enable != 0;
    return PMS_OK;
}

int pms_profile_kernels(void) { return pms::K_NUM; }

// The debug_invariants detectors on fabricated states of an 8-column
// matrix (column j >= 1 holds the single row j - 1): a consistent state
// raises nothing, and each state that breaks one property raises exactly
// that property's bit.
static pms_status debug_selftest(pms::Ctx *c)
{
    using namespace pms;
    constexpr int M = 8;
    struct Host {
        int64_t off[M], dbg_off[M];
        int32_t rows[M], len[M], low[M], beta[M], piv[M], low_star[M], dbg_low[M], dbg_len[M], dbg_w[M],
            dbg_erem[M];
        uint32_t neg[1];
        uint8_t state[M], dbg_state[M];
    };
    Host h0{};
    for (int j = 0; j < M; j++) {
        h0.rows[j] = j;  // column j >= 1 is rows[j-1 .. j) = {j - 1}
        h0.off[j] = h0.dbg_off[j] = j > 0 ? j - 1 : 0;
        h0.len[j] = h0.dbg_len[j] = j > 0 ? 1 : 0;
        h0.low[j] = h0.dbg_low[j] = j - 1;
        h0.state[j] = h0.dbg_state[j] = j > 0 ? ST_ACTIVE : ST_ZERO;
        h0.beta[j] = h0.piv[j] = h0.low_star[j] = -1;
        h0.dbg_w[j] = 0;
        h0.dbg_erem[j] = 0x7FFFFFFF;
    }
    h0.neg[0] = 0;
    Host *dv = (Host *)grow_scratch(c, B_TMP0, sizeof(Host) + sizeof(Counters) + 256);
    if (!dv) return set_err(c, PMS_ERR_OOM, "scratch");
    Counters *cnt = (Counters *)((char *)dv + ((sizeof(Host) + 255) / 256) * 256);
    Dev d{};
    d.m = M;
    d.rows = dv->rows;
    d.off = dv->off;
    d.len = dv->len;
    d.low = dv->low;
    d.state = dv->state;
    d.beta = dv->beta;
    d.piv = dv->piv;
    d.low_star = dv->low_star;
    d.neg = dv->neg;
    d.cnt = cnt;
    d.dbg_low = dv->dbg_low;
    d.dbg_off = dv->dbg_off;
    d.dbg_len = dv->dbg_len;
    d.dbg_state = dv->dbg_state;
    d.dbg_w = dv->dbg_w;
    d.dbg_erem = dv->dbg_erem;
    // kind 0: the round check, 1: the write check, 2: the final check
    auto run = [&](const Host &h, int kind, int32_t want) -> pms_status {
        PMS_HIP(hipMemcpyAsync(dv, &h, sizeof(Host), hipMemcpyHostToDevice, c->stream));
        PMS_HIP(hipMemsetAsync(cnt, 0, sizeof(Counters), c->stream));
        if (kind == 0) k_dbg_round<<<1, kBlock, 0, c->stream>>>(d, 1, 0, 1);
        else if (kind == 1) k_dbg_writes<<<1, kBlock, 0, c->stream>>>(d);
        else k_dbg_final<<<1, kBlock, 0, c->stream>>>(d);
        PMS_HIP(hipGetLastError());
        int32_t got = -1;
        PMS_HIP(hipMemcpyAsync(&got, &cnt->dbg_flags, 4, hipMemcpyDeviceToHost, c->stream));
        PMS_HIP(hipStreamSynchronize(c->stream));
        if (got != want)
            return set_err(c, PMS_ERR_HIP, "debug_invariants detector self-test: kind " + std::to_string(kind) +
                                               " raised " + std::to_string(got) + ", expected " +
                                               std::to_string(want));
        return PMS_OK;
    };
    pms_status s;
    Host h = h0;
    if ((s = run(h, 0, 0)) != PMS_OK) return s;
    h = h0; h.dbg_low[5] = 2;  // column 5's low is 4 now: it rose
    if ((s = run(h, 0, DBG_LOW_ROSE)) != PMS_OK) return s;
    h = h0; h.beta[5] = 5;     // above low(5) = 4
    if ((s = run(h, 0, DBG_BETA_ABOVE)) != PMS_OK) return s;
    h = h0; h.beta[0] = 0;     // column 0 is zero
    if ((s = run(h, 0, DBG_BETA_ZERO)) != PMS_OK) return s;
    h = h0; h.dbg_state[3] = ST_PIVOT;  // a pivot that is active again
    if ((s = run(h, 0, DBG_PIVOT_CHANGED)) != PMS_OK) return s;
    h = h0; h.state[3] = ST_PIVOT;      // a pivot no table names
    if ((s = run(h, 0, DBG_PIVOT_TABLE)) != PMS_OK) return s;
    h = h0;
    if ((s = run(h, 1, 0)) != PMS_OK) return s;
    h.dbg_w[6] = 2;
    if ((s = run(h, 1, DBG_DOUBLE_WRITE)) != PMS_OK) return s;
    Host f = h0;  // a finished reduction with every column zero
    for (int j = 0; j < M; j++) f.dbg_low[j] = -1;
    if ((s = run(f, 2, 0)) != PMS_OK) return s;
    h = f; h.dbg_erem[7] = 1;  // simplex 7 is essential but left E in round 1
    if ((s = run(h, 2, DBG_ESS_REMOVED)) != PMS_OK) return s;
    h = f; h.low_star[3] = 2; h.piv[2] = 3; h.dbg_low[3] = 1;  // low* is not the last low
    if ((s = run(h, 2, DBG_FINAL)) != PMS_OK) return s;
    return PMS_OK;
}

pms_status pms_selftest(pms_ctx *c)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    int32_t *bad = (int32_t *)pms::grow_scratch(c, pms::B_TMP1, 64);
    if (!bad) return pms::set_err(c, PMS_ERR_OOM, "scratch");
    PMS_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    pms::k_selftest<<<4, 256, 0, c->stream>>>(bad);
    PMS_HIP(hipGetLastError());
    int32_t h = -1;
    PMS_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    if (h != 0) return pms::set_err(c, PMS_ERR_HIP, "wave reduction self-test failed");
    return debug_selftest(c);
}

const char *pms_profile_kernel_name(int k) { return (k >= 0 && k < pms::K_NUM) ? kKernelNames[k] : nullptr; }

pms_status pms_profile_read(pms_ctx *c, int k, double *total_ms, int64_t *launches, double *bytes)
{
    if (!c || k < 0 || k >= pms::K_NUM) return PMS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PMS_ERR_HIP;
    pms::prof_flush(c);
    if (total_ms) *total_ms = c->prof_ms[k];
    if (launches) *launches = c->prof_launches[k];
    if (bytes) *bytes = c->prof_bytes[k];
    return PMS_OK;
}

pms_status pms_profile_read_addition_bytes(pms_ctx *c, int k, double *bytes)
{
    if (!c || k < 0 || k >= pms::K_NUM || !bytes) return PMS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PMS_ERR_HIP;
    pms::prof_flush(c);
    *bytes = c->prof_abytes[k];
    return PMS_OK;
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
    if (o.variant < 0 || o.variant > 1 || o.max_rounds < 0 || o.arena_entries < 0 || o.graph_rounds < 0 ||
        o.graph_rounds > 1024 || o.diagnostics < 0 || o.diagnostics > 1 || o.debug_invariants < 0 ||
        o.debug_invariants > 1 || !pms::extra_options_ok(o, bnd))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "bad options (c8 and sweep need dim; left and beta come together)");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    pms::ScratchSource S;
    S.c = c;
    pms_status s = pms::reduce_impl(c, bnd, &o, res, S, c->inst_off, c->n_inst);
    if (s != PMS_OK && s != PMS_ERR_CAPACITY && s != PMS_ERR_NOT_CONVERGED) {
        res->n_pairs = res->n_essential = 0;
    }
    return s;
}

pms_status pms_reduce_noalloc(pms_ctx *c, const pms_boundary *bnd, const pms_options *opt, pms_result *res)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!bnd || !res) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null boundary or result");
    if (bnd->m < 0 || bnd->m >= 0x7FFFFFFF) return pms::set_err(c, PMS_ERR_INVALID_ARG, "m out of range");
    if (bnd->m > 0 && (!bnd->col_ptr || !bnd->rows || !res->low_star))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "null col_ptr / rows / low_star");
    const pms_options o = opt ? *opt : pms_default_options();
    if (o.variant < 0 || o.variant > 1 || o.max_rounds < 0 || o.arena_entries != 0 || o.graph_rounds != 0 ||
        o.diagnostics != 0 || o.debug_invariants < 0 || o.debug_invariants > 1 || !pms::extra_options_ok(o, bnd))
        return pms::set_err(c, PMS_ERR_INVALID_ARG,
                            "bad options (without allocation: no graph rounds, no diagnostics, arena_entries 0)");
    if (c->prof_on) return pms::set_err(c, PMS_ERR_INVALID_ARG, "the profiler is on (it creates events)");
    void *base = c->device < kNoAllocDevices ? noalloc_ptr[c->device] : nullptr;
    if (!base) return pms::set_err(c, PMS_ERR_INVALID_ARG, "no allocation-free region on this device");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    pms::ScratchSource S;
    S.c = c;
    S.base = (char *)base;
    S.cap = PMS_NOALLOC_BYTES;
    pms_status s = pms::reduce_impl(c, bnd, &o, res, S, nullptr, 1);
    if (s != PMS_OK && s != PMS_ERR_CAPACITY && s != PMS_ERR_NOT_CONVERGED) res->n_pairs = res->n_essential = 0;
    return s;
}

pms_status pms_round_stats_read(pms_ctx *c, int32_t cap, pms_round_stats *out, int32_t *count)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!count || cap < 0 || (cap > 0 && !out))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "null count, negative cap, or null out with cap > 0");
    *count = (int32_t)c->diag.size();
    const int32_t n = cap < *count ? cap : *count;
    for (int32_t i = 0; i < n; i++) out[i] = c->diag[(size_t)i];
    return PMS_OK;
}

pms_status pms_essential_estimate(pms_ctx *c, int64_t m, uint32_t *bits)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (c->diag_m < 0) return pms::set_err(c, PMS_ERR_INVALID_ARG, "no reduction with diagnostics on this context");
    if (m != c->diag_m) return pms::set_err(c, PMS_ERR_INVALID_ARG, "m is not that of the last reduction with diagnostics");
    if (m == 0) return PMS_OK;
    if (!bits) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null bits");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    const size_t bytes = (size_t)((m + 31) / 32) * 4;
    PMS_HIP(hipMemcpyAsync(bits, c->b[pms::B_ESS].p, bytes, hipMemcpyDeviceToDevice, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    return PMS_OK;
}

pms_tuning pms_default_tuning(void) { return pms::default_tuning(); }

pms_status pms_set_tuning(pms_ctx *c, const pms_tuning *t)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    const pms_tuning v = t ? *t : pms::default_tuning();
    if (!pms::tuning_valid(v)) return pms::set_err(c, PMS_ERR_INVALID_ARG, "tuning field out of range");
    c->tune = v;
    return PMS_OK;
}

pms_status pms_get_tuning(pms_ctx *c, pms_tuning *t)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!t) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null tuning");
    *t = c->tune;
    return PMS_OK;
}

pms_status pms_autotune(pms_ctx *c, const pms_boundary *bnd, int32_t n, const pms_options *opts,
                        const pms_tuning *tunes, int32_t reps, pms_result *res, double *ms, int32_t *best)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!bnd || !res || !tunes || !best || n < 1 || reps < 1 || reps > 64)
        return pms::set_err(c, PMS_ERR_INVALID_ARG,
                            "null boundary / result / candidates / best, n < 1, or reps outside 1..64");
    for (int32_t i = 0; i < n; i++)
        if (!pms::tuning_valid(tunes[i]))
            return pms::set_err(c, PMS_ERR_INVALID_ARG,
                                "candidate " + std::to_string(i) + ": tuning field out of range");
    const pms_tuning before = c->tune;
    auto fail = [&](int32_t i, pms_status s) {
        c->tune = before;
        c->err = "candidate " + std::to_string(i) + ": " + c->err;
        return s;
    };
    std::vector<double> score((size_t)n), t((size_t)reps);
    for (int32_t i = 0; i < n; i++) {
        c->tune = tunes[i];
        const pms_options *o = opts ? &opts[i] : nullptr;
        // one untimed run (scratch growth, graph capture), then the timed ones
        for (int32_t r = -1; r < reps; r++) {
            const auto t0 = std::chrono::steady_clock::now();
            const pms_status s = pms_reduce(c, bnd, o, res);
            const auto t1 = std::chrono::steady_clock::now();
            if (s != PMS_OK) return fail(i, s);
            if (r >= 0) t[(size_t)r] = std::chrono::duration<double, std::milli>(t1 - t0).count();
        }
        std::sort(t.begin(), t.end());
        score[(size_t)i] = (reps & 1) ? t[(size_t)reps / 2] : 0.5 * (t[(size_t)reps / 2 - 1] + t[(size_t)reps / 2]);
        if (ms) ms[i] = score[(size_t)i];
    }
    int32_t b = 0;
    for (int32_t i = 1; i < n; i++)
        if (score[(size_t)i] < score[(size_t)b]) b = i;
    c->tune = tunes[b];
    const pms_status s = pms_reduce(c, bnd, opts ? &opts[b] : nullptr, res);
    if (s != PMS_OK) return fail(b, s);
    *best = b;
    return PMS_OK;
}

pms_status pms_reduce_batched(pms_ctx *c, int32_t count, const int64_t *inst_col_off, const pms_boundary *bnd,
                              const pms_options *opt, pms_result *res, int64_t *inst_pair_off, int64_t *inst_ess_off,
                              int32_t *pair_inst)
{
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!bnd || !res || count < 1 || !inst_col_off)
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "null boundary / result / offsets, or count < 1");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    {
        // the offsets: count + 1 entries, ascending from 0 to m
        std::vector<int64_t> h((size_t)count + 1);
        PMS_HIP(hipMemcpyAsync(h.data(), inst_col_off, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
        PMS_HIP(hipStreamSynchronize(c->stream));
        bool ok = h[0] == 0 && h[count] == bnd->m;
        for (int32_t b = 0; ok && b < count; b++) ok = h[b] <= h[b + 1];
        if (!ok)
            return pms::set_err(c, PMS_ERR_INVALID_ARG,
                                "inst_col_off must ascend from 0 to m (count + 1 entries)");
    }
    c->inst_off = inst_col_off;  // the complexes, for clearing by local compression
    c->n_inst = count;
    pms_status s = pms_reduce(c, bnd, opt, res);
    c->inst_off = nullptr;
    c->n_inst = 1;
    if (s != PMS_OK) return s;
    const bool pairs = res->pair_birth && res->pair_death;
    if (inst_pair_off || inst_ess_off)
        PMS_LAUNCH(c, pms::K_FINAL, 16.0 * (count + 1), pms::k_inst_offsets, pms::grid_for(count + 1), pms::kBlock,
                   count, inst_col_off, pairs ? res->pair_death : nullptr, res->n_pairs, res->essential,
                   res->n_essential, inst_pair_off, inst_ess_off);
    if (pair_inst && pairs && res->n_pairs > 0)
        PMS_LAUNCH(c, pms::K_FINAL, 8.0 * res->n_pairs, pms::k_pair_inst, pms::grid_for(res->n_pairs, pms::kBlock, 65536),
                   pms::kBlock, count, inst_col_off, res->pair_death, res->n_pairs, pair_inst);
    PMS_HIP(hipGetLastError());
    PMS_HIP(hipStreamSynchronize(c->stream));
    if (c->prof_on) pms::prof_flush(c);
    return PMS_OK;
}

}  // extern "C"
