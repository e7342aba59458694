// Vietoris-Rips filtrations (dimension <= 3) of batches of point clouds,
// built on the GPU.
//
// A simplex of a cloud is present when its squared diameter is at most the
// cloud's threshold (Sec. 2.2: diam <= 2r is monotone in the squared
// diameter); its value is that squared diameter.  Each cloud's filtration
// is ordered compatibly by (value, dimension, lexicographic vertex tuple).
// To dimension 2 the order is one 64-bit key:
//   integer clouds : [63:29] squared distance (< 2^35), [28:27] dim, [26:0] lex
//   FP32 clouds    : [63:32] FP32 bits (values >= 0),   [31:30] dim, [29:0] lex
// with lex = a (vertex), a*n + b (edge a<b), a*n^2 + b*n + c (triangle
// a<b<c).  To dimension 3 (lex of a tetrahedron a<b<c<d: ((a*n + b)*n + c)*n
// + d) the key takes two words, (cloud, value, dim) and lex, sorted by two
// stable radix passes (lex first).  The FP32 squared distance is rounded
// step by step in coordinate order, d = x_a - x_b, s = s + d*d, with no
// fused multiply-add.
//
// The clouds are concatenated block-diagonally: cloud b owns the columns
// [col_base_b, col_base_b + m_b) and its rows stay inside that range, so the
// batch is reduced as one matrix and every cloud's pairs come out exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <algorithm>
#include <cstring>

#include <vector>

#include "pms_build.h"
#include "pms_sort.h"
#include "pms_common.h"

namespace pms {

struct VrInst {
    int32_t n, D;
    int64_t pt_off;     // index of cloud b's first coordinate in pts
    int64_t pbase;      // global id of its point 0
    int64_t slot_base;  // start of its n x n slot grid
    int64_t adj_base;   // start of its adjacency bitmask rows (words per row)
    int32_t words;      // 64-bit words per adjacency row
    int32_t has_thr;
    int64_t thr_i;
    float thr_f;
    int32_t pad;
    int64_t col_base;   // first column of cloud b
    int64_t e_first;    // scan value of the edge counts at its first slot
    int64_t t_first;    // same for the triangle counts
    int64_t E, T;       // edges and triangles of cloud b
    int64_t q_first;    // scan value of the tetrahedron counts at its first slot
    int64_t Q;          // tetrahedra of cloud b
};

// The order key (value, dimension, lexicographic vertex tuple) in one
// unsigned 64-bit word: the value on top (raw bits of a non-negative FP32
// value, 31 bits; an integer squared distance, < 2^35), then 2 bits of
// dimension, then lexb bits of the vertex tuple's rank a*n^2 + b*n + c
// (lexb: enough for the batch's largest n^3).  A batch sorted in one pass
// also carries its cloud above the key.
constexpr int kValueBitsF = 31, kValueBitsI = 35;

__device__ inline unsigned long long vr_key(unsigned long long value, int dim, unsigned long long lex, int lexb)
{
    return (value << (lexb + 2)) | ((unsigned long long)dim << lexb) | lex;
}

// Squared distances and adjacency, one thread per slot (a, b), a < b.
template <bool F32>
__global__ void k_vr_dist(const VrInst *inst, const void *pts, unsigned long long *val, unsigned long long *adj,
                          int32_t *err)
{
    const VrInst I = inst[blockIdx.y];
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= (int64_t)I.n * I.n) return;
    const int32_t a = (int32_t)(sl / I.n), b = (int32_t)(sl % I.n);
    if (a >= b) return;
    unsigned long long v;
    bool adjacent;
    if (F32) {
        const float *p = (const float *)pts + I.pt_off;
        float s = 0.0f;
        for (int k = 0; k < I.D; k++) {
            const float dk = __fsub_rn(p[(int64_t)a * I.D + k], p[(int64_t)b * I.D + k]);
            s = __fadd_rn(s, __fmul_rn(dk, dk));
        }
        if (!(s >= 0.0f) || s == INFINITY) atomicExch(err, 1);  // NaN or overflow
        v = __float_as_uint(s);
        adjacent = !I.has_thr || s <= I.thr_f;
    } else {
        const int32_t *p = (const int32_t *)pts + I.pt_off;
        long long s = 0;
        for (int k = 0; k < I.D; k++) {
            const long long dk = (long long)p[(int64_t)a * I.D + k] - (long long)p[(int64_t)b * I.D + k];
            s += dk * dk;
        }
        if (s >= (1ll << 35)) atomicExch(err, 2);  // does not fit the key's value field
        v = (unsigned long long)s;
        adjacent = !I.has_thr || s <= I.thr_i;
    }
    val[I.slot_base + sl] = v;
    if (adjacent) {
        atomicOr(&adj[I.adj_base + (int64_t)a * I.words + (b >> 6)], 1ull << (b & 63));
        atomicOr(&adj[I.adj_base + (int64_t)b * I.words + (a >> 6)], 1ull << (a & 63));
    }
}

// Per slot (a < b): 1 if the edge is present, the number of triangles
// (a, b, c), c > b, whose three edges are present, and (maxdim 3) the number
// of tetrahedra (a, b, c, d), d > c > b, whose six edges are present.
__global__ void k_vr_count(const VrInst *inst, const unsigned long long *adj, int64_t *ecnt, int64_t *tcnt,
                           int64_t *qcnt, int maxdim)
{
    const VrInst I = inst[blockIdx.y];
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= (int64_t)I.n * I.n) return;
    const int32_t a = (int32_t)(sl / I.n), b = (int32_t)(sl % I.n);
    int64_t e = 0, t = 0, q = 0;
    if (a < b) {
        const unsigned long long *ra = adj + I.adj_base + (int64_t)a * I.words;
        const unsigned long long *rb = adj + I.adj_base + (int64_t)b * I.words;
        if (maxdim >= 1 && ((ra[b >> 6] >> (b & 63)) & 1ull)) {
            e = 1;
            if (maxdim >= 2)
                for (int w = (b + 1) >> 6; w < I.words; w++) {
                    unsigned long long x = ra[w] & rb[w];
                    if (w == ((b + 1) >> 6)) x &= ~0ull << ((b + 1) & 63);
                    t += __popcll(x);
                    while (maxdim >= 3 && x) {
                        const int c = w * 64 + __ffsll((long long)x) - 1;
                        x &= x - 1;
                        const unsigned long long *rc = adj + I.adj_base + (int64_t)c * I.words;
                        for (int w2 = (c + 1) >> 6; w2 < I.words; w2++) {
                            unsigned long long y = ra[w2] & rb[w2] & rc[w2];
                            if (w2 == ((c + 1) >> 6)) y &= ~0ull << ((c + 1) & 63);
                            q += __popcll(y);
                        }
                    }
                }
        }
    }
    ecnt[I.slot_base + sl] = e;
    tcnt[I.slot_base + sl] = t;
    if (qcnt) qcnt[I.slot_base + sl] = q;
}

// Per cloud: scan values at its first slot and at the end of the grid.
__global__ void k_vr_bounds(VrInst *inst, int32_t B, const int64_t *escan, const int64_t *tscan,
                            const int64_t *qscan, int64_t e_total, int64_t t_total, int64_t q_total, int64_t nslots)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t s0 = inst[b].slot_base;
    const int64_t s1 = b + 1 < B ? inst[b + 1].slot_base : nslots;
    const int64_t e0 = s0 < nslots ? escan[s0] : e_total, e1 = s1 < nslots ? escan[s1] : e_total;
    const int64_t t0 = s0 < nslots ? tscan[s0] : t_total, t1 = s1 < nslots ? tscan[s1] : t_total;
    inst[b].e_first = e0;
    inst[b].t_first = t0;
    inst[b].E = e1 - e0;
    inst[b].T = t1 - t0;
    if (qscan) {
        const int64_t q0 = s0 < nslots ? qscan[s0] : q_total, q1 = s1 < nslots ? qscan[s1] : q_total;
        inst[b].q_first = q0;
        inst[b].Q = q1 - q0;
    } else {
        inst[b].q_first = 0;
        inst[b].Q = 0;
    }
}

// The order keys of every simplex, at its slot's place in the unsorted
// array.  kWide (dimension 3): keys[p] = lex and hi[p] = (cloud, value,
// dim) with the value above 2 bits of dimension; else one word, with the
// cloud above the key (cshift > 0, batches sorted in one pass) or in cl
// (batches sorted in two passes).
template <bool F32, bool kWide>
__global__ void k_vr_emit(const VrInst *inst, const unsigned long long *val, const unsigned long long *adj,
                          const int64_t *escan, const int64_t *tscan, const int64_t *qscan, unsigned long long *keys,
                          unsigned long long *hi, uint32_t *cl, int maxdim, int lexb, int cshift)
{
    const VrInst I = inst[blockIdx.y];
    const uint32_t cb = blockIdx.y;
    const unsigned long long ck = cshift > 0 ? (unsigned long long)blockIdx.y << cshift : 0ull;
    constexpr int kVb = F32 ? kValueBitsF : kValueBitsI;
    const unsigned long long chi = (unsigned long long)blockIdx.y << (kVb + 2);
    auto put = [&](int64_t pos, unsigned long long v, int dm, unsigned long long lex) {
        if (kWide) {
            keys[pos] = lex;
            hi[pos] = chi | (v << 2) | (unsigned long long)dm;
        } else {
            keys[pos] = ck | vr_key(v, dm, lex, lexb);
            if (cl) cl[pos] = cb;
        }
    };
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl < I.n) put(I.col_base + sl, 0, 0, (unsigned long long)sl);  // vertex sl
    if (sl >= (int64_t)I.n * I.n) return;
    const int32_t a = (int32_t)(sl / I.n), b = (int32_t)(sl % I.n);
    if (a >= b) return;
    const unsigned long long *ra = adj + I.adj_base + (int64_t)a * I.words;
    const unsigned long long *rb = adj + I.adj_base + (int64_t)b * I.words;
    if (maxdim < 1 || !((ra[b >> 6] >> (b & 63)) & 1ull)) return;
    const unsigned long long n = (unsigned long long)I.n;
    const unsigned long long vab = val[I.slot_base + sl];
    put(I.col_base + I.n + (escan[I.slot_base + sl] - I.e_first), vab, 1,
        (unsigned long long)a * n + (unsigned long long)b);
    if (maxdim < 2) return;
    int64_t pos = I.col_base + I.n + I.E + (tscan[I.slot_base + sl] - I.t_first);
    int64_t qpos = kWide ? I.col_base + I.n + I.E + I.T + (qscan[I.slot_base + sl] - I.q_first) : 0;
    for (int w = (b + 1) >> 6; w < I.words; w++) {
        unsigned long long x = ra[w] & rb[w];
        if (w == ((b + 1) >> 6)) x &= ~0ull << ((b + 1) & 63);
        while (x) {
            const int c = w * 64 + __ffsll((long long)x) - 1;
            x &= x - 1;
            unsigned long long v = vab;
            const unsigned long long vac = val[I.slot_base + (int64_t)a * I.n + c];
            const unsigned long long vbc = val[I.slot_base + (int64_t)b * I.n + c];
            // FP32 values are >= 0, so their bit patterns order like the values
            v = v > vac ? v : vac;
            v = v > vbc ? v : vbc;
            const unsigned long long labc = ((unsigned long long)a * n + (unsigned long long)b) * n + (unsigned long long)c;
            put(pos++, v, 2, labc);
            if (!kWide || maxdim < 3) continue;
            const unsigned long long *rc = adj + I.adj_base + (int64_t)c * I.words;
            for (int w2 = (c + 1) >> 6; w2 < I.words; w2++) {
                unsigned long long y = ra[w2] & rb[w2] & rc[w2];
                if (w2 == ((c + 1) >> 6)) y &= ~0ull << ((c + 1) & 63);
                while (y) {
                    const int dd = w2 * 64 + __ffsll((long long)y) - 1;
                    y &= y - 1;
                    unsigned long long u = v;
                    const unsigned long long vad = val[I.slot_base + (int64_t)a * I.n + dd];
                    const unsigned long long vbd = val[I.slot_base + (int64_t)b * I.n + dd];
                    const unsigned long long vcd = val[I.slot_base + (int64_t)c * I.n + dd];
                    u = u > vad ? u : vad;
                    u = u > vbd ? u : vbd;
                    u = u > vcd ? u : vcd;
                    put(qpos++, u, 3, labc * n + (unsigned long long)dd);
                }
            }
        }
    }
}

__device__ inline int find_inst(const int64_t *col_base, int32_t B, int64_t p)
{
    int lo = 0, hi = B - 1;  // last cloud whose first column is <= p
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (col_base[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Value, dimension and lex of the sorted simplex p (one-word or two-word keys).
template <bool F32, bool kWide>
__device__ inline void vr_decode(const unsigned long long *keys, const unsigned long long *hi, int64_t p, int lexb,
                                 unsigned long long &lex, int &dm, unsigned long long &v)
{
    constexpr int kVb = F32 ? kValueBitsF : kValueBitsI;
    if (kWide) {
        lex = keys[p];
        const unsigned long long h = hi[p];
        dm = (int)(h & 3ull);
        v = (h >> 2) & ((1ull << kVb) - 1ull);
    } else {
        const unsigned long long key = keys[p];
        lex = key & ((1ull << lexb) - 1ull);
        dm = (int)((key >> lexb) & 3ull);
        v = (key >> (lexb + 2)) & ((1ull << kVb) - 1ull);
    }
}

// The dm+1 vertices (ascending, within the cloud) of a simplex from its lex.
__device__ inline void lex_vertices(unsigned long long lex, int dm, unsigned long long n, int32_t x[4])
{
    for (int k = 0; k < 4; k++) x[k] = -1;
    for (int k = dm; k >= 0; k--) {
        x[k] = (int32_t)(lex % n);
        lex /= n;
    }
}

// Decode the sorted keys: per-cloud index tables, dim, value, vertices and
// the facet counts of each tile (for col_ptr).
template <bool F32, bool kWide>
__global__ void __launch_bounds__(kBlock) k_vr_index(const VrInst *inst, const int64_t *col_base, int32_t B,
                                                     const unsigned long long *keys, const unsigned long long *hi,
                                                     int64_t m, int lexb, int32_t *vidx, int32_t *eidx, int8_t *dim,
                                                     void *value, int32_t *verts, int64_t *tile_sum)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    if (p < m) {
        const int b = find_inst(col_base, B, p);
        const VrInst &I = inst[b];
        unsigned long long lex, v;
        int dm;
        vr_decode<F32, kWide>(keys, hi, p, lexb, lex, dm, v);
        int32_t x[4];
        lex_vertices(lex, dm, (unsigned long long)I.n, x);
        if (dm == 0) vidx[I.pbase + x[0]] = (int32_t)p;
        if (dm == 1) eidx[I.slot_base + (int64_t)x[0] * I.n + x[1]] = (int32_t)p;
        dim[p] = (int8_t)dm;
        if (F32) ((float *)value)[p] = __uint_as_float((uint32_t)v);
        else ((int64_t *)value)[p] = (int64_t)v;
        for (int k = 0; k < 4; k++) verts[4 * p + k] = k <= dm ? (int32_t)(I.pbase + x[k]) : -1;
        nf = dm > 0 ? dm + 1 : 0;
    }
    const int64_t tot = block_sum64(nf);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Index of the triangle (a < b < c) of a cloud whose columns are [lo, hi_end):
// its key is known (the value is the largest of its edges' values), so a
// binary search over the cloud's sorted two-word keys finds it; -1 if absent.
template <bool F32>
__device__ inline int32_t find_triangle(const unsigned long long *keys, const unsigned long long *hi, int64_t lo,
                                        int64_t hi_end, unsigned long long khi, unsigned long long klo)
{
    int64_t l = lo, r = hi_end;
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        const unsigned long long h = hi[mid];
        if (h < khi || (h == khi && keys[mid] < klo)) l = mid + 1;
        else r = mid;
    }
    return (l < hi_end && hi[l] == khi && keys[l] == klo) ? (int32_t)l : -1;
}

template <bool F32, bool kWide>
__global__ void __launch_bounds__(kBlock) k_vr_rows(const VrInst *inst, const int64_t *col_base, int32_t B,
                                                    const unsigned long long *keys, const unsigned long long *hi,
                                                    const unsigned long long *val, int64_t m, int lexb, int64_t nnz,
                                                    const int32_t *vidx, const int32_t *eidx, const int64_t *tile_off,
                                                    int64_t *col_ptr, int32_t *rows, int32_t *crit, int32_t *err)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    int b = 0, dm = 0;
    int32_t x[4] = {0, 0, 0, 0};
    if (p < m) {
        b = find_inst(col_base, B, p);
        unsigned long long lex, v;
        vr_decode<F32, kWide>(keys, hi, p, lexb, lex, dm, v);
        lex_vertices(lex, dm, (unsigned long long)inst[b].n, x);
        nf = dm > 0 ? dm + 1 : 0;
    }
    const int64_t start = tile_off[blockIdx.x] + block_excl_sum64(nf);
    if (p < m && start + nf <= nnz) {
        const VrInst &I = inst[b];
        const int64_t g = I.slot_base;
        col_ptr[p] = start;
        if (p == m - 1) col_ptr[m] = start + nf;
        int32_t ca = -1, cb = -1;
        if (dm == 1) {
            const int32_t r0 = vidx[I.pbase + x[0]], r1 = vidx[I.pbase + x[1]];
            rows[start] = r0 < r1 ? r0 : r1;
            rows[start + 1] = r0 < r1 ? r1 : r0;
            ca = (int32_t)(I.pbase + x[0]);
            cb = (int32_t)(I.pbase + x[1]);
        } else if (dm >= 2) {
            // the edge latest in the filtration fixes the value (the critical
            // edge); for a triangle it is also its low before any reduction
            int32_t best = -1;
            for (int u = 0; u < dm; u++)
                for (int w = u + 1; w <= dm; w++) {
                    const int32_t e = eidx[g + (int64_t)x[u] * I.n + x[w]];
                    if (e > best) {
                        best = e;
                        ca = (int32_t)(I.pbase + x[u]);
                        cb = (int32_t)(I.pbase + x[w]);
                    }
                }
            int32_t r[4] = {-1, -1, -1, -1};
            if (dm == 2) {
                r[0] = eidx[g + (int64_t)x[1] * I.n + x[2]];
                r[1] = eidx[g + (int64_t)x[0] * I.n + x[2]];
                r[2] = eidx[g + (int64_t)x[0] * I.n + x[1]];
            } else if (kWide) {  // dm == 3: the four triangles, each found by its key
                constexpr int kVb = F32 ? kValueBitsF : kValueBitsI;
                const unsigned long long n = (unsigned long long)I.n;
                const int64_t lo = col_base[b], end = b + 1 < B ? col_base[b + 1] : m;
                const unsigned long long chi = (unsigned long long)b << (kVb + 2);
                for (int k = 0; k < 4; k++) {
                    int32_t f[3];
                    for (int u = 0, t = 0; u < 4; u++)
                        if (u != k) f[t++] = x[u];
                    unsigned long long fv = val[g + (int64_t)f[0] * I.n + f[1]];
                    const unsigned long long v02 = val[g + (int64_t)f[0] * I.n + f[2]];
                    const unsigned long long v12 = val[g + (int64_t)f[1] * I.n + f[2]];
                    fv = fv > v02 ? fv : v02;
                    fv = fv > v12 ? fv : v12;
                    const unsigned long long flex =
                        ((unsigned long long)f[0] * n + (unsigned long long)f[1]) * n + (unsigned long long)f[2];
                    r[k] = find_triangle<F32>(keys, hi, lo, end, chi | (fv << 2) | 2ull, flex);
                    if (r[k] < 0) atomicExch(err, 3);
                }
            } else {  // one-word keys never hold a tetrahedron
                atomicExch(err, 3);
            }
            for (int u = 1; u <= dm; u++) {
                const int32_t y = r[u];
                int w = u - 1;
                while (w >= 0 && r[w] > y) {
                    r[w + 1] = r[w];
                    w--;
                }
                r[w + 1] = y;
            }
            for (int u = 0; u <= dm; u++) rows[start + u] = r[u];
        }
        crit[2 * p] = ca;
        crit[2 * p + 1] = cb;
    }
}

__global__ void k_vr_colbase(const VrInst *inst, int32_t B, int64_t *col_base, int32_t *seg_lo, int32_t *seg_hi)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) {
        col_base[b] = inst[b].col_base;
        seg_lo[b] = (int32_t)inst[b].col_base;
        seg_hi[b] = (int32_t)(inst[b].col_base + inst[b].n + inst[b].E + inst[b].T + inst[b].Q);
    }
}

// ---------------------------------------------------------------- host
static pms_status build_vr(Ctx *c, const void *pts, bool f32, const int32_t *n, const int32_t *D,
                           const int64_t *pt_off, const void *thr, int32_t B, int32_t maxdim, Filtration **out,
                           int64_t *inst_col_off)
{
    if (!out || !n || !D || !pt_off || B < 1 || maxdim < 0 || maxdim > 3)
        return set_err(c, PMS_ERR_INVALID_ARG, "bad Vietoris-Rips arguments (maxdim must be 0..3)");
    // to dimension 3 the order key takes two words: (cloud, value, dim) and lex
    const bool wide = maxdim >= 3;
    if (wide && (f32 ? kValueBitsF : kValueBitsI) + 2 + 32 - __builtin_clz((unsigned)B) > 64)
        return set_err(c, PMS_ERR_INVALID_ARG, "too many clouds for one dimension-3 batch");
    std::vector<VrInst> h(B);
    int64_t slots = 0, adjw = 0, pbase = 0, maxnn = 0;
    const int nmax = f32 ? 1023 : 511;  // n^3 must fit the lex field
    for (int b = 0; b < B; b++) {
        if (n[b] < 0 || n[b] > nmax || D[b] < 1 || pt_off[b] < 0 || (n[b] > 0 && !pts))
            return set_err(c, PMS_ERR_INVALID_ARG, "cloud size out of range (n <= 511 for int32, 1023 for FP32)");
        VrInst &I = h[b];
        memset(&I, 0, sizeof(I));
        I.n = n[b];
        I.D = D[b];
        I.pt_off = pt_off[b];
        I.pbase = pbase;
        I.slot_base = slots;
        I.words = (n[b] + 63) / 64;
        I.adj_base = adjw;
        if (f32) {
            const float t = thr ? ((const float *)thr)[b] : -1.0f;
            I.has_thr = t >= 0.0f;
            I.thr_f = t;
        } else {
            const int64_t t = thr ? ((const int64_t *)thr)[b] : -1;
            I.has_thr = t >= 0;
            I.thr_i = t;
        }
        pbase += n[b];
        slots += (int64_t)n[b] * n[b];
        adjw += (int64_t)n[b] * I.words;
        if ((int64_t)n[b] * n[b] > maxnn) maxnn = (int64_t)n[b] * n[b];
    }
    if (pbase >= 0x7FFFFFFF) return set_err(c, PMS_ERR_INVALID_ARG, "too many points");
    hipStream_t s = c->stream;
    const int64_t S = slots > 0 ? slots : 1;
    VrInst *dinst = (VrInst *)grow_scratch(c, B_BUILD6, (size_t)B * sizeof(VrInst));
    unsigned long long *val = (unsigned long long *)grow_scratch(c, B_BUILD7, S * 8);
    unsigned long long *adj = (unsigned long long *)grow_scratch(c, B_BUILD8, (adjw > 0 ? adjw : 1) * 8);
    int64_t *ecnt = (int64_t *)grow_scratch(c, B_BUILD9, (S + 1) * 8);
    int64_t *tcnt = (int64_t *)grow_scratch(c, B_BUILD10, (S + 1) * 8);
    int64_t *tmp = (int64_t *)grow_scratch(c, B_BUILD11, ((S + kBlock - 1) / kBlock + 2) * 8);
    int32_t *err = (int32_t *)grow_scratch(c, B_BUILD4, 64);
    int64_t *qcnt = wide ? (int64_t *)grow_scratch(c, B_BUILD14, (S + 1) * 8) : nullptr;
    if (!dinst || !val || !adj || !ecnt || !tcnt || !tmp || !err || (wide && !qcnt))
        return set_err(c, PMS_ERR_OOM, "builder scratch");
    PMS_HIP(hipMemcpyAsync(dinst, h.data(), (size_t)B * sizeof(VrInst), hipMemcpyHostToDevice, s));
    PMS_HIP(hipMemsetAsync(adj, 0, (adjw > 0 ? adjw : 1) * 8, s));
    PMS_HIP(hipMemsetAsync(err, 0, 4, s));
    const dim3 g2((unsigned)((maxnn + kBlock - 1) / kBlock > 0 ? (maxnn + kBlock - 1) / kBlock : 1), (unsigned)B);
    if (f32) PMS_LAUNCH(c, K_VR_EDGES, 12.0 * slots, k_vr_dist<true>, g2, kBlock, dinst, pts, val, adj, err);
    else PMS_LAUNCH(c, K_VR_EDGES, 12.0 * slots, k_vr_dist<false>, g2, kBlock, dinst, pts, val, adj, err);
    PMS_LAUNCH(c, K_VR_TRI, 16.0 * slots, k_vr_count, g2, kBlock, dinst, adj, ecnt, tcnt, qcnt, maxdim);
    int64_t etot = 0, ttot = 0, qtot = 0;
    pms_status st = scan_i64(c, ecnt, slots, tmp, &etot);
    if (st != PMS_OK) return st;
    st = scan_i64(c, tcnt, slots, tmp, &ttot);
    if (st != PMS_OK) return st;
    if (wide) {
        st = scan_i64(c, qcnt, slots, tmp, &qtot);
        if (st != PMS_OK) return st;
    }
    PMS_LAUNCH(c, K_FILL, 0, k_vr_bounds, (unsigned)((B + 255) / 256), 256, dinst, B, ecnt, tcnt, qcnt, etot, ttot,
               qtot, slots);
    PMS_HIP(hipMemcpyAsync(h.data(), dinst, (size_t)B * sizeof(VrInst), hipMemcpyDeviceToHost, s));
    int32_t herr = 0;
    PMS_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    PMS_HIP(hipStreamSynchronize(s));
    if (herr == 1) return set_err(c, PMS_ERR_INVALID_ARG, "non-finite FP32 squared distance");
    if (herr == 2) return set_err(c, PMS_ERR_INVALID_ARG, "squared distance >= 2^35 does not fit the order key");
    int64_t m = 0, nnz = 0;
    for (int b = 0; b < B; b++) {
        h[b].col_base = m;
        if (inst_col_off) inst_col_off[b] = m;
        m += h[b].n + h[b].E + h[b].T + h[b].Q;
        nnz += 2 * h[b].E + 3 * h[b].T + 4 * h[b].Q;
    }
    if (inst_col_off) inst_col_off[B] = m;
    if (m >= 0x7FFFFFFF) return set_err(c, PMS_ERR_INVALID_ARG, "too many simplices for 32-bit indices");
    Filtration *f = *out;
    st = filtration_reserve(c, &f, m, nnz, f32 ? 1 : 0);
    if (st != PMS_OK) return st;
    *out = f;
    f->m = m;
    f->nnz = nnz;
    f->value_is_f32 = f32 ? 1 : 0;
    const int64_t M = m > 0 ? m : 1;
    unsigned long long *keys = (unsigned long long *)grow_scratch(c, B_BUILD0, M * 8);
    unsigned long long *keys2 = (unsigned long long *)grow_scratch(c, B_BUILD1, M * 8);
    int32_t *vidx = (int32_t *)grow_scratch(c, B_BUILD2, (pbase > 0 ? pbase : 1) * 4);
    int32_t *eidx = (int32_t *)grow_scratch(c, B_BUILD3, S * 4);
    int64_t *colb = (int64_t *)grow_scratch(c, B_TMP0, (size_t)(B + 1) * 8);
    int32_t *seg = (int32_t *)grow_scratch(c, B_TMP1, (size_t)(2 * B + 2) * 4);
    const int64_t tiles = (m + kBlock - 1) / kBlock;
    int64_t *tsum = (int64_t *)grow_scratch(c, B_BUILD5, (tiles + 1) * 8);
    if (!keys || !keys2 || !vidx || !eidx || !colb || !seg || !tsum) return set_err(c, PMS_ERR_OOM, "builder scratch");
    PMS_HIP(hipMemcpyAsync(dinst, h.data(), (size_t)B * sizeof(VrInst), hipMemcpyHostToDevice, s));
    if (m == 0) {
        int64_t zero = 0;
        PMS_HIP(hipMemcpyAsync(f->col_ptr, &zero, 8, hipMemcpyHostToDevice, s));
        PMS_HIP(hipStreamSynchronize(s));
        return PMS_OK;
    }
    const dim3 g3((unsigned)((maxnn + kBlock - 1) / kBlock > 0 ? (maxnn + kBlock - 1) / kBlock : 1), (unsigned)B);
    int64_t n_hi = 1;
    for (int b = 0; b < B; b++) n_hi = std::max<int64_t>(n_hi, h[b].n);
    int cbits = 1;
    while ((1 << cbits) < B) cbits++;
    PMS_LAUNCH(c, K_FILL, 0, k_vr_colbase, (unsigned)((B + 255) / 256), 256, dinst, B, colb, seg, seg + B);
    const unsigned long long *sorted = keys2, *sorted_hi = nullptr;
    int lexb = 1;
    if (wide) {
        // two words, two stable radix passes: by lex, then by (cloud, value, dim)
        while (lexb < 63 && (1ll << lexb) < n_hi * n_hi * n_hi * n_hi) lexb++;
        const int hibits = (f32 ? kValueBitsF : kValueBitsI) + 2 + (B > 1 ? cbits : 0);
        unsigned long long *hw = (unsigned long long *)grow_scratch(c, B_BUILD12, M * 8);
        unsigned long long *hw2 = (unsigned long long *)grow_scratch(c, B_BUILD13, M * 8);
        if (!hw || !hw2) return set_err(c, PMS_ERR_OOM, "builder scratch");
        if (f32)
            PMS_LAUNCH(c, K_VR_TRI, 16.0 * m, (k_vr_emit<true, true>), g3, kBlock, dinst, val, adj, ecnt, tcnt, qcnt,
                       keys, hw, nullptr, maxdim, lexb, 0);
        else
            PMS_LAUNCH(c, K_VR_TRI, 16.0 * m, (k_vr_emit<false, true>), g3, kBlock, dinst, val, adj, ecnt, tcnt, qcnt,
                       keys, hw, nullptr, maxdim, lexb, 0);
        hipEvent_t e0 = nullptr;
        if (c->prof_on) { e0 = prof_event(c); (void)hipEventRecord(e0, s); }
        // by lex, then (stable) by (cloud, value, dim)
        bool in_b = false;
        pms_status ss = radix_sort(c, keys, keys2, hw, hw2, m, lexb, B_AGG, B_AGG2, &in_b);
        if (ss != PMS_OK) return ss;
        unsigned long long *lx = in_b ? keys2 : keys, *lx2 = in_b ? keys : keys2;
        unsigned long long *hx = in_b ? hw2 : hw, *hx2 = in_b ? hw : hw2;
        ss = radix_sort(c, hx, hx2, lx, lx2, m, hibits, B_AGG, B_AGG2, &in_b);
        if (ss != PMS_OK) return ss;
        if (c->prof_on) {
            hipEvent_t e1 = prof_event(c);
            (void)hipEventRecord(e1, s);
            c->pend.push_back({K_SORT, e0, e1, 64.0 * m});
        }
        sorted = in_b ? lx2 : lx;
        sorted_hi = in_b ? hx2 : hx;
    } else {
        // key widths: lex for the largest cloud's n^3, the value's bits, and the
        // cloud's when a batch is sorted in one pass
        while (lexb < 62 && (1ll << lexb) < n_hi * n_hi * n_hi) lexb++;
        const int keybits = (f32 ? kValueBitsF : kValueBitsI) + 2 + lexb;
        // batches: the whole device sorts, not one workgroup per cloud.  When the
        // cloud fits above the key, one sort of (cloud, key) words; else one
        // stable sort of all keys (carrying their cloud) by key, then a stable
        // sort by cloud, so each cloud's columns come out in key order
        const bool one_pass = B > 1 && keybits + cbits <= 64;
        const bool by_cloud = B > 1 && !one_pass;
        uint32_t *cl = nullptr, *cl2 = nullptr;
        if (by_cloud) {
            cl = (uint32_t *)grow_scratch(c, B_BUILD12, M * 4);
            cl2 = (uint32_t *)grow_scratch(c, B_BUILD13, M * 4);
            if (!cl || !cl2) return set_err(c, PMS_ERR_OOM, "builder scratch");
        }
        if (f32)
            PMS_LAUNCH(c, K_VR_TRI, 8.0 * m, (k_vr_emit<true, false>), g3, kBlock, dinst, val, adj, ecnt, tcnt, qcnt,
                       keys, nullptr, cl, maxdim, lexb, one_pass ? keybits : 0);
        else
            PMS_LAUNCH(c, K_VR_TRI, 8.0 * m, (k_vr_emit<false, false>), g3, kBlock, dinst, val, adj, ecnt, tcnt, qcnt,
                       keys, nullptr, cl, maxdim, lexb, one_pass ? keybits : 0);
        hipEvent_t e0 = nullptr;
        if (c->prof_on) { e0 = prof_event(c); (void)hipEventRecord(e0, s); }
        bool in_b = false;
        if (!by_cloud) {
            const int bits = keybits + (one_pass ? cbits : 0);
            const pms_status ss = radix_sort<unsigned long long, uint32_t>(c, keys, keys2, nullptr, nullptr, m, bits,
                                                                           B_AGG, B_AGG2, &in_b);
            if (ss != PMS_OK) return ss;
            sorted = in_b ? keys2 : keys;
        } else {
            // by key (carrying the cloud), then stable by cloud
            pms_status ss = radix_sort(c, keys, keys2, cl, cl2, m, keybits, B_AGG, B_AGG2, &in_b);
            if (ss != PMS_OK) return ss;
            unsigned long long *kx = in_b ? keys2 : keys, *kx2 = in_b ? keys : keys2;
            uint32_t *cx = in_b ? cl2 : cl, *cx2 = in_b ? cl : cl2;
            ss = radix_sort(c, cx, cx2, kx, kx2, m, cbits, B_AGG, B_AGG2, &in_b);
            if (ss != PMS_OK) return ss;
            sorted = in_b ? kx2 : kx;
        }
        if (c->prof_on) {
            hipEvent_t e1 = prof_event(c);
            (void)hipEventRecord(e1, s);
            c->pend.push_back({K_SORT, e0, e1, by_cloud ? 48.0 * m : 16.0 * m});
        }
    }
#define VR_INDEX(F, W)                                                                                            \
    PMS_LAUNCH(c, K_VR_INDEX, (F ? 41.0 : 45.0) * m + (W ? 8.0 * m : 0.0), (k_vr_index<F, W>), (unsigned)tiles,    \
               kBlock, dinst, colb, B, sorted, sorted_hi, m, lexb, vidx, eidx, f->dim, f->value, f->verts, tsum)
#define VR_ROWS(F, W)                                                                                             \
    PMS_LAUNCH(c, K_VR_ROWS, 24.0 * m + 8.0 * nnz, (k_vr_rows<F, W>), (unsigned)tiles, kBlock, dinst, colb, B, sorted, \
               sorted_hi, val, m, lexb, nnz, vidx, eidx, tsum, f->col_ptr, f->rows, f->crit, err)
    if (f32 && wide) VR_INDEX(true, true);
    else if (f32) VR_INDEX(true, false);
    else if (wide) VR_INDEX(false, true);
    else VR_INDEX(false, false);
    PMS_LAUNCH(c, K_BUILD_SCAN, 16.0 * tiles, k_scan_i64, 1, 1024, tsum, tiles);
    if (f32 && wide) VR_ROWS(true, true);
    else if (f32) VR_ROWS(true, false);
    else if (wide) VR_ROWS(false, true);
    else VR_ROWS(false, false);
#undef VR_INDEX
#undef VR_ROWS
    PMS_HIP(hipGetLastError());
    PMS_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    PMS_HIP(hipStreamSynchronize(s));
    if (c->prof_on) prof_flush(c);
    if (herr == 3) return set_err(c, PMS_ERR_HIP, "internal: a tetrahedron's face was not found");
    return PMS_OK;
}

pms_status build_vr_batch(Ctx *c, const void *pts, bool f32, const int32_t *n, const int32_t *D, const int64_t *pt_off,
                          const void *thr, int32_t B, int32_t maxdim, Filtration **out, int64_t *inst_col_off)
{
    return build_vr(c, pts, f32, n, D, pt_off, thr, B, maxdim, out, inst_col_off);
}

}  // namespace pms
