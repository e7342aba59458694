// Vietoris-Rips filtrations (dimension <= 2) of batches of point clouds,
// built on the GPU.
//
// A simplex of a cloud is present when its squared diameter is at most the
// cloud's threshold (Sec. 2.2: diam <= 2r is monotone in the squared
// diameter); its value is that squared diameter.  Each cloud's filtration
// is ordered compatibly by (value, dimension, lexicographic vertex tuple),
// encoded as one 64-bit key:
//   integer clouds : [63:29] squared distance (< 2^35), [28:27] dim, [26:0] lex
//   FP32 clouds    : [63:32] FP32 bits (values >= 0),   [31:30] dim, [29:0] lex
// with lex = a (vertex), a*n + b (edge a<b), a*n^2 + b*n + c (triangle
// a<b<c).  The FP32 squared distance is rounded step by step in coordinate
// order, d = x_a - x_b, s = s + d*d, with no fused multiply-add.
//
// The clouds are concatenated block-diagonally: cloud b owns the columns
// [col_base_b, col_base_b + m_b) and its rows stay inside that range, so the
// batch is reduced as one matrix and every cloud's pairs come out exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <vector>

#include "pms_build.h"
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

// Per slot (a < b): 1 if the edge is present, and the number of triangles
// (a, b, c), c > b, whose three edges are present.
__global__ void k_vr_count(const VrInst *inst, const unsigned long long *adj, int64_t *ecnt, int64_t *tcnt,
                           int maxdim)
{
    const VrInst I = inst[blockIdx.y];
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= (int64_t)I.n * I.n) return;
    const int32_t a = (int32_t)(sl / I.n), b = (int32_t)(sl % I.n);
    int64_t e = 0, t = 0;
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
                }
        }
    }
    ecnt[I.slot_base + sl] = e;
    tcnt[I.slot_base + sl] = t;
}

// Per cloud: scan values at its first slot and at the end of the grid.
__global__ void k_vr_bounds(VrInst *inst, int32_t B, const int64_t *escan, const int64_t *tscan, int64_t e_total,
                            int64_t t_total, int64_t nslots)
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
}

template <bool F32>
__global__ void k_vr_emit(const VrInst *inst, const unsigned long long *val, const unsigned long long *adj,
                          const int64_t *escan, const int64_t *tscan, unsigned long long *keys, uint16_t *cl,
                          int maxdim, int lexb, int cshift)
{
    // cl (batches sorted in two passes): the cloud of every key; cshift > 0
    // (batches sorted in one): the cloud goes into the key's bits from cshift
    const VrInst I = inst[blockIdx.y];
    const uint16_t cb = (uint16_t)blockIdx.y;
    const unsigned long long ck = cshift > 0 ? (unsigned long long)blockIdx.y << cshift : 0ull;
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl < I.n) {
        keys[I.col_base + sl] = ck | vr_key(0, 0, (unsigned long long)sl, lexb);  // vertex sl
        if (cl) cl[I.col_base + sl] = cb;
    }
    if (sl >= (int64_t)I.n * I.n) return;
    const int32_t a = (int32_t)(sl / I.n), b = (int32_t)(sl % I.n);
    if (a >= b) return;
    const unsigned long long *ra = adj + I.adj_base + (int64_t)a * I.words;
    const unsigned long long *rb = adj + I.adj_base + (int64_t)b * I.words;
    if (maxdim < 1 || !((ra[b >> 6] >> (b & 63)) & 1ull)) return;
    const unsigned long long n = (unsigned long long)I.n;
    const unsigned long long vab = val[I.slot_base + sl];
    const int64_t pe = I.col_base + I.n + (escan[I.slot_base + sl] - I.e_first);
    keys[pe] = ck | vr_key(vab, 1, (unsigned long long)a * n + (unsigned long long)b, lexb);
    if (cl) cl[pe] = cb;
    if (maxdim < 2) return;
    int64_t pos = I.col_base + I.n + I.E + (tscan[I.slot_base + sl] - I.t_first);
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
            if (cl) cl[pos] = cb;
            keys[pos++] = ck | vr_key(v, 2, ((unsigned long long)a * n + (unsigned long long)b) * n + (unsigned long long)c, lexb);
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

// Decode the sorted keys: per-cloud index tables, dim, value, vertices and
// the facet counts of each tile (for col_ptr).
template <bool F32>
__global__ void __launch_bounds__(kBlock) k_vr_index(const VrInst *inst, const int64_t *col_base, int32_t B,
                                                     const unsigned long long *keys, int64_t m, int lexb,
                                                     int32_t *vidx, int32_t *eidx, int8_t *dim, void *value,
                                                     int32_t *verts, int64_t *tile_sum)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    if (p < m) {
        const int b = find_inst(col_base, B, p);
        const VrInst &I = inst[b];
        const unsigned long long key = keys[p];
        const unsigned long long lex = key & ((1ull << lexb) - 1ull);
        const int dm = (int)((key >> lexb) & 3ull);
        const unsigned long long v = (key >> (lexb + 2)) & ((1ull << (F32 ? kValueBitsF : kValueBitsI)) - 1ull);
        const unsigned long long n = (unsigned long long)I.n;
        int32_t x[3] = {-1, -1, -1};
        if (dm == 0) x[0] = (int32_t)lex;
        else if (dm == 1) { x[0] = (int32_t)(lex / n); x[1] = (int32_t)(lex % n); }
        else { x[0] = (int32_t)(lex / (n * n)); x[1] = (int32_t)((lex / n) % n); x[2] = (int32_t)(lex % n); }
        if (dm == 0) vidx[I.pbase + x[0]] = (int32_t)p;
        if (dm == 1) eidx[I.slot_base + (int64_t)x[0] * I.n + x[1]] = (int32_t)p;
        dim[p] = (int8_t)dm;
        if (F32) ((float *)value)[p] = __uint_as_float((uint32_t)v);
        else ((int64_t *)value)[p] = (int64_t)v;
        for (int k = 0; k < 4; k++) verts[4 * p + k] = (k <= dm && k < 3) ? (int32_t)(I.pbase + x[k]) : -1;
        nf = dm > 0 ? dm + 1 : 0;
    }
    const int64_t tot = block_sum64(nf);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

template <bool F32>
__global__ void __launch_bounds__(kBlock) k_vr_rows(const VrInst *inst, const int64_t *col_base, int32_t B,
                                                    const unsigned long long *keys, int64_t m, int lexb, int64_t nnz,
                                                    const int32_t *vidx, const int32_t *eidx, const int64_t *tile_off,
                                                    int64_t *col_ptr, int32_t *rows, int32_t *crit)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    int b = 0, dm = 0;
    int32_t x[3] = {0, 0, 0};
    if (p < m) {
        b = find_inst(col_base, B, p);
        const unsigned long long key = keys[p];
        const unsigned long long lex = key & ((1ull << lexb) - 1ull);
        dm = (int)((key >> lexb) & 3ull);
        const unsigned long long n = (unsigned long long)inst[b].n;
        if (dm == 1) { x[0] = (int32_t)(lex / n); x[1] = (int32_t)(lex % n); }
        if (dm == 2) { x[0] = (int32_t)(lex / (n * n)); x[1] = (int32_t)((lex / n) % n); x[2] = (int32_t)(lex % n); }
        nf = dm > 0 ? dm + 1 : 0;
    }
    const int64_t start = tile_off[blockIdx.x] + block_excl_sum64(nf);
    if (p < m && start + nf <= nnz) {
        const VrInst &I = inst[b];
        col_ptr[p] = start;
        if (p == m - 1) col_ptr[m] = start + nf;
        int32_t ca = -1, cb = -1;
        if (dm == 1) {
            const int32_t r0 = vidx[I.pbase + x[0]], r1 = vidx[I.pbase + x[1]];
            rows[start] = r0 < r1 ? r0 : r1;
            rows[start + 1] = r0 < r1 ? r1 : r0;
            ca = (int32_t)(I.pbase + x[0]);
            cb = (int32_t)(I.pbase + x[1]);
        } else if (dm == 2) {
            const int64_t g = I.slot_base;
            int32_t r[3] = {eidx[g + (int64_t)x[1] * I.n + x[2]], eidx[g + (int64_t)x[0] * I.n + x[2]],
                            eidx[g + (int64_t)x[0] * I.n + x[1]]};
            // the facet edge latest in the filtration fixes the value: it is
            // the triangle's low before any reduction
            const int32_t ends[3][2] = {{x[1], x[2]}, {x[0], x[2]}, {x[0], x[1]}};
            int hi = 0;
            for (int k = 1; k < 3; k++)
                if (r[k] > r[hi]) hi = k;
            ca = (int32_t)(I.pbase + ends[hi][0]);
            cb = (int32_t)(I.pbase + ends[hi][1]);
            for (int u = 1; u < 3; u++) {
                const int32_t y = r[u];
                int v = u - 1;
                while (v >= 0 && r[v] > y) { r[v + 1] = r[v]; v--; }
                r[v + 1] = y;
            }
            rows[start] = r[0];
            rows[start + 1] = r[1];
            rows[start + 2] = r[2];
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
        seg_hi[b] = (int32_t)(inst[b].col_base + inst[b].n + inst[b].E + inst[b].T);
    }
}

// ---------------------------------------------------------------- host
static pms_status build_vr(Ctx *c, const void *pts, bool f32, const int32_t *n, const int32_t *D,
                           const int64_t *pt_off, const void *thr, int32_t B, int32_t maxdim, Filtration **out,
                           int64_t *inst_col_off)
{
    if (!out || !n || !D || !pt_off || B < 1 || maxdim < 0 || maxdim > 2)
        return set_err(c, PMS_ERR_INVALID_ARG, "bad Vietoris-Rips arguments (maxdim must be 0..2)");
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
    VrInst *dinst = (VrInst *)scratch(c, B_BUILD6, (size_t)B * sizeof(VrInst));
    unsigned long long *val = (unsigned long long *)scratch(c, B_BUILD7, S * 8);
    unsigned long long *adj = (unsigned long long *)scratch(c, B_BUILD8, (adjw > 0 ? adjw : 1) * 8);
    int64_t *ecnt = (int64_t *)scratch(c, B_BUILD9, (S + 1) * 8);
    int64_t *tcnt = (int64_t *)scratch(c, B_BUILD10, (S + 1) * 8);
    int64_t *tmp = (int64_t *)scratch(c, B_BUILD11, ((S + kBlock - 1) / kBlock + 2) * 8);
    int32_t *err = (int32_t *)scratch(c, B_BUILD4, 64);
    if (!dinst || !val || !adj || !ecnt || !tcnt || !tmp || !err) return set_err(c, PMS_ERR_OOM, "builder scratch");
    PMS_HIP(hipMemcpyAsync(dinst, h.data(), (size_t)B * sizeof(VrInst), hipMemcpyHostToDevice, s));
    PMS_HIP(hipMemsetAsync(adj, 0, (adjw > 0 ? adjw : 1) * 8, s));
    PMS_HIP(hipMemsetAsync(err, 0, 4, s));
    const dim3 g2((unsigned)((maxnn + kBlock - 1) / kBlock > 0 ? (maxnn + kBlock - 1) / kBlock : 1), (unsigned)B);
    if (f32) PMS_LAUNCH(c, K_VR_EDGES, 12.0 * slots, k_vr_dist<true>, g2, kBlock, dinst, pts, val, adj, err);
    else PMS_LAUNCH(c, K_VR_EDGES, 12.0 * slots, k_vr_dist<false>, g2, kBlock, dinst, pts, val, adj, err);
    PMS_LAUNCH(c, K_VR_TRI, 16.0 * slots, k_vr_count, g2, kBlock, dinst, adj, ecnt, tcnt, maxdim);
    int64_t etot = 0, ttot = 0;
    pms_status st = scan_i64(c, ecnt, slots, tmp, &etot);
    if (st != PMS_OK) return st;
    st = scan_i64(c, tcnt, slots, tmp, &ttot);
    if (st != PMS_OK) return st;
    PMS_LAUNCH(c, K_FILL, 0, k_vr_bounds, (unsigned)((B + 255) / 256), 256, dinst, B, ecnt, tcnt, etot, ttot, slots);
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
        m += h[b].n + h[b].E + h[b].T;
        nnz += 2 * h[b].E + 3 * h[b].T;
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
    unsigned long long *keys = (unsigned long long *)scratch(c, B_BUILD0, M * 8);
    unsigned long long *keys2 = (unsigned long long *)scratch(c, B_BUILD1, M * 8);
    int32_t *vidx = (int32_t *)scratch(c, B_BUILD2, (pbase > 0 ? pbase : 1) * 4);
    int32_t *eidx = (int32_t *)scratch(c, B_BUILD3, S * 4);
    int64_t *colb = (int64_t *)scratch(c, B_TMP0, (size_t)(B + 1) * 8);
    int32_t *seg = (int32_t *)scratch(c, B_TMP1, (size_t)(2 * B + 2) * 4);
    const int64_t tiles = (m + kBlock - 1) / kBlock;
    int64_t *tsum = (int64_t *)scratch(c, B_BUILD5, (tiles + 1) * 8);
    if (!keys || !keys2 || !vidx || !eidx || !colb || !seg || !tsum) return set_err(c, PMS_ERR_OOM, "builder scratch");
    PMS_HIP(hipMemcpyAsync(dinst, h.data(), (size_t)B * sizeof(VrInst), hipMemcpyHostToDevice, s));
    if (m == 0) {
        int64_t zero = 0;
        PMS_HIP(hipMemcpyAsync(f->col_ptr, &zero, 8, hipMemcpyHostToDevice, s));
        PMS_HIP(hipStreamSynchronize(s));
        return PMS_OK;
    }
    const dim3 g3((unsigned)((maxnn + kBlock - 1) / kBlock > 0 ? (maxnn + kBlock - 1) / kBlock : 1), (unsigned)B);
    // key widths: lex for the largest cloud's n^3, the value's bits, and the
    // cloud's when a batch is sorted in one pass
    int64_t n_hi = 1;
    for (int b = 0; b < B; b++) n_hi = std::max<int64_t>(n_hi, h[b].n);
    int lexb = 1;
    while (lexb < 62 && (1ll << lexb) < n_hi * n_hi * n_hi) lexb++;
    const int keybits = (f32 ? kValueBitsF : kValueBitsI) + 2 + lexb;
    int cbits = 1;
    while ((1 << cbits) < B) cbits++;
    // batches: the whole device sorts, not one workgroup per cloud.  When the
    // cloud fits above the key, one sort of (cloud, key) words; else one
    // stable sort of all keys (carrying their cloud) by key, then a stable
    // sort by cloud, so each cloud's columns come out in key order
    const bool one_pass = B > 1 && keybits + cbits <= 64;
    const bool by_cloud = B > 1 && !one_pass && B <= 65536;
    uint16_t *cl = nullptr, *cl2 = nullptr;
    if (by_cloud) {
        cl = (uint16_t *)scratch(c, B_BUILD12, M * 2);
        cl2 = (uint16_t *)scratch(c, B_BUILD13, M * 2);
        if (!cl || !cl2) return set_err(c, PMS_ERR_OOM, "builder scratch");
    }
    if (f32)
        PMS_LAUNCH(c, K_VR_TRI, 8.0 * m, k_vr_emit<true>, g3, kBlock, dinst, val, adj, ecnt, tcnt, keys, cl, maxdim,
                   lexb, one_pass ? keybits : 0);
    else
        PMS_LAUNCH(c, K_VR_TRI, 8.0 * m, k_vr_emit<false>, g3, kBlock, dinst, val, adj, ecnt, tcnt, keys, cl, maxdim,
                   lexb, one_pass ? keybits : 0);
    PMS_LAUNCH(c, K_FILL, 0, k_vr_colbase, (unsigned)((B + 255) / 256), 256, dinst, B, colb, seg, seg + B);
    const unsigned long long *sorted = keys2;
    {
        hipEvent_t e0 = nullptr;
        if (c->prof_on) { e0 = prof_event(c); (void)hipEventRecord(e0, s); }
        size_t tb = 0;
        if (B == 1 || one_pass) {
            const int bits = keybits + (one_pass ? cbits : 0);
            PMS_HIP(rocprim::radix_sort_keys(nullptr, tb, keys, keys2, (size_t)m, 0, bits, s));
            void *tmps = scratch(c, B_AGG, tb);
            if (!tmps) return set_err(c, PMS_ERR_OOM, "sort scratch");
            PMS_HIP(rocprim::radix_sort_keys(tmps, tb, keys, keys2, (size_t)m, 0, bits, s));
        } else if (by_cloud) {
            size_t tb2 = 0;
            PMS_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys, keys2, cl, cl2, (size_t)m, 0, keybits, s));
            PMS_HIP(rocprim::radix_sort_pairs(nullptr, tb2, cl2, cl, keys2, keys, (size_t)m, 0, cbits, s));
            void *tmps = scratch(c, B_AGG, tb > tb2 ? tb : tb2);
            if (!tmps) return set_err(c, PMS_ERR_OOM, "sort scratch");
            PMS_HIP(rocprim::radix_sort_pairs(tmps, tb, keys, keys2, cl, cl2, (size_t)m, 0, keybits, s));
            PMS_HIP(rocprim::radix_sort_pairs(tmps, tb2, cl2, cl, keys2, keys, (size_t)m, 0, cbits, s));
            sorted = keys;
        } else {
            PMS_HIP(rocprim::segmented_radix_sort_keys(nullptr, tb, keys, keys2, (unsigned)m, (unsigned)B, seg,
                                                       seg + B, 0, keybits, s));
            void *tmps = scratch(c, B_AGG, tb);
            if (!tmps) return set_err(c, PMS_ERR_OOM, "sort scratch");
            PMS_HIP(rocprim::segmented_radix_sort_keys(tmps, tb, keys, keys2, (unsigned)m, (unsigned)B, seg, seg + B,
                                                       0, keybits, s));
        }
        if (c->prof_on) {
            hipEvent_t e1 = prof_event(c);
            (void)hipEventRecord(e1, s);
            c->pend.push_back({K_SORT, e0, e1, by_cloud ? 40.0 * m : 16.0 * m});
        }
    }
    if (f32)
        PMS_LAUNCH(c, K_VR_INDEX, 41.0 * m, k_vr_index<true>, (unsigned)tiles, kBlock, dinst, colb, B, sorted, m, lexb, vidx,
                   eidx, f->dim, f->value, f->verts, tsum);
    else
        PMS_LAUNCH(c, K_VR_INDEX, 45.0 * m, k_vr_index<false>, (unsigned)tiles, kBlock, dinst, colb, B, sorted, m, lexb, vidx,
                   eidx, f->dim, f->value, f->verts, tsum);
    PMS_LAUNCH(c, K_BUILD_SCAN, 16.0 * tiles, k_scan_i64, 1, 1024, tsum, tiles);
    if (f32)
        PMS_LAUNCH(c, K_VR_ROWS, 24.0 * m + 8.0 * nnz, k_vr_rows<true>, (unsigned)tiles, kBlock, dinst, colb, B, sorted,
                   m, lexb, nnz, vidx, eidx, tsum, f->col_ptr, f->rows, f->crit);
    else
        PMS_LAUNCH(c, K_VR_ROWS, 24.0 * m + 8.0 * nnz, k_vr_rows<false>, (unsigned)tiles, kBlock, dinst, colb, B, sorted,
                   m, lexb, nnz, vidx, eidx, tsum, f->col_ptr, f->rows, f->crit);
    PMS_HIP(hipGetLastError());
    PMS_HIP(hipStreamSynchronize(s));
    if (c->prof_on) prof_flush(c);
    return PMS_OK;
}

pms_status build_vr_batch(Ctx *c, const void *pts, bool f32, const int32_t *n, const int32_t *D, const int64_t *pt_off,
                          const void *thr, int32_t B, int32_t maxdim, Filtration **out, int64_t *inst_col_off)
{
    return build_vr(c, pts, f32, n, D, pt_off, thr, B, maxdim, out, inst_col_off);
}

}  // namespace pms
