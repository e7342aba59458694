// Lower-star filtration of the Freudenthal triangulation of a 3-D vertex
// grid, built on the GPU.
//
// The simplices of the triangulation are the chains v0 < v1 < ... < vk of
// grid vertices whose successive steps are non-zero 0/1 vectors with
// disjoint supports (k <= 3).  A simplex is stored as (anchor v0, shape),
// where the shape is the sequence of steps: 1 shape of dimension 0, 7 of
// dimension 1, 12 of dimension 2 and 6 of dimension 3.  Its value is the
// largest vertex value (lower-star filtration), and the filtration order is
// compatible (Sec. 2.2): by value, then dimension, then the lexicographic
// order of the ascending vertex tuple.  Because a simplex's vertices are the
// anchor plus fixed offsets, the lexicographic order is (anchor, rank of the
// shape's offset tuple), so the whole order is one key of b + 38 bits, b the
// bits of a vertex id (nx ny nz <= 2^b, b <= 26), sorted by those bits only:
//
//   [b+37:b+6] value, as order-preserving bits of the FP32 (-0 read as +0)
//   [b+5 :b+4] dimension
//   [b+3 :  4] anchor vertex id
//   [3   :  0] rank of the shape among the shapes of its dimension
//
// The boundary matrix (eq. "def:boundary_matrix") follows from a dense
// (anchor, shape) -> filtration index table: the facets of (v, s) are
// (v + delta, s') with delta and s' read from a per-shape table.  The same
// table read the other way gives each simplex's cofaces, so the builder also
// returns left (Def. "left": the first column holding a row, the first
// coface in the order) and beta (Def. "beta": the largest row of a column
// whose left is that column), which the reduction would otherwise compute
// with one atomic per nonzero.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pms_common.h"
#include "pms_build.h"
#include "pms_sort.h"

namespace pms {

constexpr int kShapes = 26;

struct ShapeTab {
    int32_t nx, ny, nz;
    int8_t dim[kShapes];
    int8_t ext[kShapes];      // OR of the steps: axes the shape advances along
    int8_t rank[kShapes];     // lexicographic rank within its dimension
    int32_t cum[kShapes][4];  // vertex offsets from the anchor (cum[0] = 0)
    int8_t by_rank[4][16];    // shape id of (dim, rank)
    int8_t facet[kShapes][4]; // facet shape id after removing vertex k
    int32_t fdelta[kShapes][4];  // anchor shift of that facet
    // cofaces: the shapes one dimension up with this shape as a facet, and the
    // step (axis mask, 0: none) from their anchor to this one
    int8_t ncof[kShapes];
    int8_t cof_s[kShapes][14];
    int8_t cof_e[kShapes][14];
    int32_t vbits;  // bits of an anchor index in the order key (nx ny nz <= 2^vbits)
};

__device__ inline uint32_t f32_order_bits(float x)
{
    if (x == 0.0f) x = 0.0f;  // -0 and +0 are one value
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ inline float f32_from_order_bits(uint32_t u)
{
    const uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __uint_as_float(b);
}

// One key per (anchor, shape); shapes that leave the grid get ~0 (sorted
// last).  The shape tables sit in LDS (a thread's shape differs from its
// neighbours'), 32-bit index arithmetic (nv * 26 < 2^31), and the value's
// up to four vertex reads are issued together (clamped to the anchor).
__global__ void __launch_bounds__(kBlock) k_ls_keys(ShapeTab t, const float *__restrict__ grid, int64_t nv,
                                                    unsigned long long *keys, int32_t *err)
{
    __shared__ int32_t s_cum[kShapes][4];
    __shared__ int8_t s_dim[kShapes], s_ext[kShapes], s_rank[kShapes];
    for (int k = threadIdx.x; k < kShapes * 4; k += kBlock) s_cum[k / 4][k % 4] = t.cum[k / 4][k % 4];
    if (threadIdx.x < kShapes) {
        s_dim[threadIdx.x] = t.dim[threadIdx.x];
        s_ext[threadIdx.x] = t.ext[threadIdx.x];
        s_rank[threadIdx.x] = t.rank[threadIdx.x];
    }
    __syncthreads();
    const uint32_t n = (uint32_t)(nv * kShapes), nx = (uint32_t)t.nx, nxy = (uint32_t)(t.nx * t.ny);
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint32_t v = i / kShapes;
        const int s = (int)(i - v * kShapes);
        const uint32_t z = v / nxy, r = v - z * nxy, y = r / nx, x = r - y * nx;
        const int e = s_ext[s], dm = s_dim[s];
        unsigned long long key = ~0ull;
        if (!((e & 1) && x + 1 >= nx) && !((e & 2) && y + 1 >= (uint32_t)t.ny) && !((e & 4) && z + 1 >= (uint32_t)t.nz)) {
            float g[4];
#pragma unroll
            for (int k = 0; k < 4; k++) g[k] = grid[v + (k <= dm ? s_cum[s][k] : 0)];
            float val = g[0];
#pragma unroll
            for (int k = 1; k < 4; k++) val = k <= dm ? fmaxf(val, g[k]) : val;
            if (val != val) atomicExch(err, 1);  // NaN has no place in an order
            key = ((unsigned long long)f32_order_bits(val) << (t.vbits + 6)) |
                  ((unsigned long long)dm << (t.vbits + 4)) | ((unsigned long long)v << 4) |
                  (unsigned long long)s_rank[s];
        }
        keys[i] = key;
    }
}

// Decode the sorted keys: index table, dimension, value, critical vertex,
// vertex tuple, and the per-tile facet counts for col_ptr.
__global__ void __launch_bounds__(kBlock) k_ls_index(ShapeTab t, const float *__restrict__ grid,
                                                     const unsigned long long *__restrict__ keys, int64_t m, int64_t nv,
                                                     int32_t *idx_tab, int8_t *dim, float *value, int32_t *crit,
                                                     int32_t *verts, int64_t *tile_sum, int32_t *err)
{
    // the shape tables in LDS: neighbouring simplices have different shapes
    __shared__ int32_t s_cum[kShapes][4];
    __shared__ int8_t s_shape[4][16];
    for (int k = threadIdx.x; k < kShapes * 4; k += kBlock) s_cum[k / 4][k % 4] = t.cum[k / 4][k % 4];
    if (threadIdx.x < 64) s_shape[threadIdx.x / 16][threadIdx.x % 16] = t.by_rank[threadIdx.x / 16][threadIdx.x % 16];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    const unsigned long long key = p < m ? keys[p] : ~0ull;
    const unsigned long long vmask = (1ull << t.vbits) - 1;
    if (p < m && (key == ~0ull || (int64_t)((key >> 4) & vmask) >= nv)) atomicExch(err, 2);
    else if (p < m) {
        const int32_t v = (int32_t)((key >> 4) & vmask);
        const int dm = (int)((key >> (t.vbits + 4)) & 3u);
        const int s = s_shape[dm][key & 15u];
        idx_tab[(int64_t)v * kShapes + s] = (int32_t)p;
        dim[p] = (int8_t)dm;
        value[p] = f32_from_order_bits((uint32_t)(key >> (t.vbits + 6)));
        // the vertices (k > dm: the anchor again), their values read together
        int32_t u[4];
        float gu[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            u[k] = v + (k <= dm ? s_cum[s][k] : 0);
            gu[k] = grid[u[k]];
        }
        // argmax vertex by (value, id): the vertex whose value the simplex takes
        int32_t best = v;
        float bv = gu[0];
#pragma unroll
        for (int k = 1; k < 4; k++)
            if (k <= dm && (gu[k] > bv || (gu[k] == bv && u[k] > best))) { best = u[k]; bv = gu[k]; }
        reinterpret_cast<int2 *>(crit)[p] = make_int2(best, -1);
        if (verts)
            reinterpret_cast<int4 *>(verts)[p] =
                make_int4(u[0], dm >= 1 ? u[1] : -1, dm >= 2 ? u[2] : -1, dm >= 3 ? u[3] : -1);
        nf = dm > 0 ? dm + 1 : 0;
    }
    const int64_t tot = block_sum64(nf);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_ls_rows(ShapeTab t, const unsigned long long *__restrict__ keys, int64_t m,
                                                    int64_t nv, int64_t nnz, const int32_t *__restrict__ idx_tab,
                                                    const int64_t *tile_off, int64_t *col_ptr, int32_t *rows,
                                                    const int32_t *__restrict__ left, int32_t *beta)
{
    // the shape tables in LDS: neighbouring simplices have different shapes
    __shared__ int32_t s_fdelta[kShapes][4];
    __shared__ int8_t s_facet[kShapes][4], s_shape[4][16];
    for (int k = threadIdx.x; k < kShapes * 4; k += kBlock) {
        s_fdelta[k / 4][k % 4] = t.fdelta[k / 4][k % 4];
        s_facet[k / 4][k % 4] = t.facet[k / 4][k % 4];
    }
    if (threadIdx.x < 64) s_shape[threadIdx.x / 16][threadIdx.x % 16] = t.by_rank[threadIdx.x / 16][threadIdx.x % 16];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t nf = 0;
    int32_t v = 0;
    int s = 0, dm = 0;
    bool ok = false;
    if (p < m) {
        const unsigned long long key = keys[p];
        const unsigned long long vmask = (1ull << t.vbits) - 1;
        ok = key != ~0ull && (int64_t)((key >> 4) & vmask) < nv;
        v = (int32_t)((key >> 4) & vmask);
        dm = (int)((key >> (t.vbits + 4)) & 3u);
        s = s_shape[dm][key & 15u];
        nf = (ok && dm > 0) ? dm + 1 : 0;
    }
    const int64_t start = tile_off[blockIdx.x] + block_excl_sum64(nf);
    if (p < m && start + nf <= nnz) {
        col_ptr[p] = start;
        if (p == m - 1) col_ptr[m] = start + nf;
        // the facets' indices, read together (k >= nf: the simplex's own entry)
        int32_t r[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            r[k] = idx_tab[k < nf ? (int64_t)(v + s_fdelta[s][k]) * kShapes + s_facet[s][k]
                                  : (int64_t)v * kShapes + s];
        for (int a = 1; a < nf; a++) {  // ascending rows
            const int32_t x = r[a];
            int b = a - 1;
            while (b >= 0 && r[b] > x) { r[b + 1] = r[b]; b--; }
            r[b + 1] = x;
        }
        for (int k = 0; k < nf; k++) rows[start + k] = r[k];
        // beta: the largest row whose first column is this one (loads together, then the scan)
        int32_t lf[4];
#pragma unroll
        for (int k = 0; k < 4; k++) lf[k] = left[k < nf ? r[k] : 0];
        int32_t b = -1;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (k < nf && lf[k] == (int32_t)p) b = r[k];  // rows ascending: the last hit is the largest
        beta[p] = b;
    }
}

// left of every simplex (Def. "left"): the smallest filtration index among
// its cofaces (none: 2^31 - 1).  A coface of (v, s) is anchored at v minus a
// step e (a subset of the axes), so a workgroup that handles the anchors
// v0 .. v0 + kLeftV - 1 needs the index-table rows of four planes, v - b and
// v - b - 1 for b in {0, nx, nx ny, nx ny + nx}: it stages them into LDS with
// coalesced loads (rows padded to an odd stride), then takes its (anchor,
// shape) pairs shape-major, so a wavefront holds one shape and reads the
// coface tables as scalars.  The one scattered access is the write of left at
// the simplex's filtration index.
constexpr int kLeftV = 64;                                  // anchors per tile
constexpr int kLeftRow = kShapes + 1;                       // LDS row stride
constexpr int kLeftPlane = (kLeftV + 1) * kShapes;          // staged entries per plane
constexpr int kLeftPer = (kLeftPlane + kBlock - 1) / kBlock;

// The smallest staged index among the cofaces of (v0 + vl, s), kN >= the
// shape's coface count (a vertex has 14, an edge at most 6, a triangle 2);
// the LDS reads are issued together.
template <int kN>
__device__ inline int32_t ls_first_coface(const ShapeTab &t, int s, int vl, int back, int fwd,
                                          const int32_t (*seg)[(kLeftV + 1) * kLeftRow])
{
    const int nc = t.ncof[s];
    int32_t got[kN];
    bool ok[kN];
#pragma unroll
    for (int c = 0; c < kN; c++) {
        const int sp = c < nc ? t.cof_s[s][c] : s;
        const int e = c < nc ? t.cof_e[s][c] : 0;
        // the coface's anchor v - e is on the grid, and the coface fits there
        ok[c] = c < nc && !(e & ~back) && !(t.ext[sp] & ~e & ~fwd);
        got[c] = seg[(e >> 1) & 3][(vl + 1 - (e & 1)) * kLeftRow + sp];
    }
    int32_t best = 0x7FFFFFFF;
#pragma unroll
    for (int c = 0; c < kN; c++)
        if (ok[c]) best = min(best, got[c]);
    return best;
}

__global__ void __launch_bounds__(kBlock) k_ls_left(ShapeTab t, int64_t nv, int64_t m,
                                                    const int32_t *__restrict__ idx_tab, int32_t *left)
{
    static_assert(kLeftV == 64 && kBlock % kLeftV == 0, "one shape per wavefront");
    __shared__ int32_t seg[4][(kLeftV + 1) * kLeftRow];
    __shared__ uint8_t nb[kLeftV];  // back | fwd << 3: axes with a grid neighbour below / above
    const int32_t nx = t.nx, ny = t.ny, nz = t.nz, nxy = nx * ny;
    for (int64_t v0 = (int64_t)blockIdx.x * kLeftV; v0 < nv; v0 += (int64_t)gridDim.x * kLeftV) {
        // plane g holds the kLeftV + 1 rows from v0 - b_g - 1 on: one
        // contiguous run of the table starting at a uniform entry
        int32_t val[4][kLeftPer];
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const int64_t start = (v0 - ((g & 1 ? nx : 0) + (g & 2 ? nxy : 0)) - 1) * kShapes;
#pragma unroll
            for (int q = 0; q < kLeftPer; q++) {
                const int r = q * kBlock + (int)threadIdx.x;
                const int64_t e = start + r;
                const bool in = r < kLeftPlane && e >= 0 && e < nv * kShapes;
                val[g][q] = idx_tab[in ? e : 0];
                if (!in) val[g][q] = -1;
            }
        }
#pragma unroll
        for (int g = 0; g < 4; g++)
#pragma unroll
            for (int q = 0; q < kLeftPer; q++) {
                const int r = q * kBlock + (int)threadIdx.x;
                const int j = r / kShapes;
                if (r < kLeftPlane) seg[g][j * kLeftRow + (r - j * kShapes)] = val[g][q];
            }
        if (threadIdx.x < kLeftV) {
            const int64_t v = v0 + threadIdx.x;
            const int32_t z = (int32_t)(v / nxy), rem = (int32_t)(v - (int64_t)z * nxy), y = rem / nx, x = rem - y * nx;
            const int fwd = (x + 1 < nx ? 1 : 0) | (y + 1 < ny ? 2 : 0) | (z + 1 < nz ? 4 : 0);
            const int back = (x > 0 ? 1 : 0) | (y > 0 ? 2 : 0) | (z > 0 ? 4 : 0);
            nb[threadIdx.x] = (uint8_t)(back | fwd << 3);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kShapes * kLeftV; k += kBlock) {
            const int s = __builtin_amdgcn_readfirstlane(k / kLeftV);  // k / 64 is one value per wavefront
            const int vl = k % kLeftV;
            const int bits = nb[vl], back = bits & 7, fwd = bits >> 3;
            if (v0 + vl >= nv || (t.ext[s] & ~fwd)) continue;  // past the end, or the shape leaves the grid
            const int32_t p = seg[0][(vl + 1) * kLeftRow + s];
            int32_t best = 0x7FFFFFFF;
            switch (t.dim[s]) {
            case 0: best = ls_first_coface<14>(t, s, vl, back, fwd, seg); break;
            case 1: best = ls_first_coface<6>(t, s, vl, back, fwd, seg); break;
            case 2: best = ls_first_coface<2>(t, s, vl, back, fwd, seg); break;
            default: break;
            }
            if ((uint64_t)(uint32_t)p < (uint64_t)m) left[p] = best;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host
static int step_offset(int e, int nx, int ny)
{
    return (e & 1) + ((e >> 1) & 1) * nx + ((e >> 2) & 1) * nx * ny;
}

static void make_tables(ShapeTab &t, int nx, int ny, int nz)
{
    t.nx = nx;
    t.ny = ny;
    t.nz = nz;
    t.vbits = 1;
    while ((1ll << t.vbits) < (long long)nx * ny * nz) t.vbits++;
    std::vector<std::vector<int>> shapes;
    shapes.push_back({});
    for (int e = 1; e < 8; e++) shapes.push_back({e});
    for (int e1 = 1; e1 < 8; e1++)
        for (int e2 = 1; e2 < 8; e2++)
            if (!(e1 & e2)) shapes.push_back({e1, e2});
    const int perm[6][3] = {{1, 2, 4}, {1, 4, 2}, {2, 1, 4}, {2, 4, 1}, {4, 1, 2}, {4, 2, 1}};
    for (auto &p : perm) shapes.push_back({p[0], p[1], p[2]});
    auto find = [&](const std::vector<int> &st) {
        for (size_t i = 0; i < shapes.size(); i++)
            if (shapes[i] == st) return (int)i;
        return -1;
    };
    for (int s = 0; s < kShapes; s++) {
        const auto &st = shapes[s];
        t.dim[s] = (int8_t)st.size();
        int e = 0, c = 0;
        t.cum[s][0] = 0;
        for (size_t k = 0; k < st.size(); k++) {
            e |= st[k];
            c += step_offset(st[k], nx, ny);
            t.cum[s][k + 1] = c;
        }
        for (size_t k = st.size() + 1; k < 4; k++) t.cum[s][k] = 0;
        t.ext[s] = (int8_t)e;
        for (int k = 0; k < 4; k++) { t.facet[s][k] = 0; t.fdelta[s][k] = 0; }
        const int d = (int)st.size();
        if (d >= 1)
            for (int k = 0; k <= d; k++) {
                std::vector<int> f;
                int delta = 0;
                if (k == 0) {
                    f.assign(st.begin() + 1, st.end());
                    delta = step_offset(st[0], nx, ny);
                } else if (k < d) {
                    for (int q = 0; q < d; q++) {
                        if (q == k - 1) f.push_back(st[q] | st[q + 1]);
                        else if (q != k) f.push_back(st[q]);
                    }
                } else {
                    f.assign(st.begin(), st.end() - 1);
                }
                t.facet[s][k] = (int8_t)find(f);
                t.fdelta[s][k] = delta;
            }
    }
    // lexicographic rank of the offset tuple within each dimension
    for (int d = 0; d < 4; d++) {
        std::vector<int> ids;
        for (int s = 0; s < kShapes; s++)
            if (t.dim[s] == d) ids.push_back(s);
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
            for (int k = 1; k <= d; k++)
                if (t.cum[a][k] != t.cum[b][k]) return t.cum[a][k] < t.cum[b][k];
            return false;
        });
        for (int r = 0; r < 16; r++) t.by_rank[d][r] = 0;
        for (size_t r = 0; r < ids.size(); r++) {
            t.rank[ids[r]] = (int8_t)r;
            t.by_rank[d][r] = (int8_t)ids[r];
        }
    }
    // cofaces: facet k of (v', s') is (v' + step, facet[s'][k]), the step being
    // the shape's first step when k = 0 and none otherwise
    for (int s = 0; s < kShapes; s++) t.ncof[s] = 0;
    for (int sp = 0; sp < kShapes; sp++) {
        const int d = t.dim[sp];
        for (int k = 0; d >= 1 && k <= d; k++) {
            const int f = t.facet[sp][k];
            const int n = t.ncof[f]++;
            t.cof_s[f][n] = (int8_t)sp;
            t.cof_e[f][n] = (int8_t)(k == 0 ? shapes[sp][0] : 0);
        }
    }
}

// Number of simplices and facets (closed form: a shape fits at an anchor iff
// every axis it advances along has room).
static void ls_sizes(const ShapeTab &t, int64_t *m, int64_t *nnz)
{
    int64_t M = 0, Z = 0;
    for (int mask = 0; mask < 8; mask++) {
        int64_t anchors = 1;
        const int32_t ext[3] = {t.nx, t.ny, t.nz};
        for (int a = 0; a < 3; a++) anchors *= (mask >> a & 1) ? (int64_t)(ext[a] - 1) : 1;
        if (anchors <= 0) continue;
        for (int s = 0; s < kShapes; s++) {
            if ((t.ext[s] & ~mask) != 0) continue;
            // anchors whose availability mask is exactly `mask`
            M += anchors;
            Z += anchors * (t.dim[s] > 0 ? t.dim[s] + 1 : 0);
        }
    }
    *m = M;
    *nnz = Z;
}

pms_status build_lowerstar(Ctx *c, const float *grid, int32_t nx, int32_t ny, int32_t nz, Filtration **out)
{
    if (!grid || !out || nx < 1 || ny < 1 || nz < 1) return set_err(c, PMS_ERR_INVALID_ARG, "bad grid arguments");
    const int64_t nv = (int64_t)nx * ny * nz;
    if (nv >= (1ll << 26)) return set_err(c, PMS_ERR_INVALID_ARG, "grid too large for the 26-bit anchor field");
    ShapeTab t;
    make_tables(t, nx, ny, nz);
    int64_t m = 0, nnz = 0;
    ls_sizes(t, &m, &nnz);
    Filtration *f = *out;
    pms_status st = filtration_reserve(c, &f, m, nnz, /*f32*/ 1);
    if (st != PMS_OK) return st;
    *out = f;
    f->m = m;
    f->nnz = nnz;
    f->value_is_f32 = 1;
    hipStream_t s = c->stream;
    const int64_t nk = nv * kShapes;
    unsigned long long *keys = (unsigned long long *)grow_scratch(c, B_BUILD0, nk * 8);
    unsigned long long *keys2 = (unsigned long long *)grow_scratch(c, B_BUILD1, nk * 8);
    int32_t *idx = (int32_t *)grow_scratch(c, B_BUILD2, nk * 4);
    const int64_t tiles = (m + kBlock - 1) / kBlock;
    int64_t *tsum = (int64_t *)grow_scratch(c, B_BUILD3, (tiles + 1) * 8);
    int32_t *err = (int32_t *)grow_scratch(c, B_BUILD4, 64);
    if (!keys || !keys2 || !idx || !tsum || !err) return set_err(c, PMS_ERR_OOM, "builder scratch");
    PMS_HIP(hipMemsetAsync(err, 0, 4, s));
    // grid reads are cache resident; the key write is the stream
    PMS_LAUNCH(c, K_LS_KEYS, 8.0 * nk + 4.0 * nv, k_ls_keys, grid_for(nk, kBlock, 1u << 16), kBlock, t, grid, nv, keys,
               err);
    {
        hipEvent_t e0 = nullptr;
        if (c->prof_on) { e0 = prof_event(c); (void)hipEventRecord(e0, s); }
        bool in_b = false;
        // bits: value, dim, anchor, shape rank (keys of shapes off the grid are all ones)
        const pms_status ss = radix_sort<unsigned long long, uint32_t>(c, keys, keys2, nullptr, nullptr, nk, t.vbits + 38, B_BUILD5,
                                                                       B_BUILD6, &in_b);
        if (ss != PMS_OK) return ss;
        if (!in_b) std::swap(keys, keys2);  // keys2: the sorted keys
        if (c->prof_on) {
            hipEvent_t e1 = prof_event(c);
            (void)hipEventRecord(e1, s);
            c->pend.push_back({K_SORT, e0, e1, 16.0 * nk});
        }
    }
    PMS_LAUNCH(c, K_LS_INDEX, 8.0 * m + 4.0 * m + 1.0 * m + 4.0 * m + 8.0 * m + 16.0 * m, k_ls_index,
               (unsigned)tiles, kBlock, t, grid, keys2, m, nv, idx, f->dim, (float *)f->value, f->crit, f->verts, tsum,
               err);
    PMS_LAUNCH(c, K_BUILD_SCAN, 16.0 * tiles, k_scan_i64, 1, 1024, tsum, tiles);
    // the simplex's and its cofaces' table entries, left out
    PMS_LAUNCH(c, K_LS_LEFT, 4.0 * m + 4.0 * nnz + 4.0 * m, k_ls_left, grid_for(nv, kLeftV, 65536), kBlock, t, nv, m,
               idx, f->left);
    // + the facets' left, beta out
    PMS_LAUNCH(c, K_LS_ROWS, 8.0 * m + 4.0 * nnz + 4.0 * nnz + 8.0 * m + 4.0 * nnz + 4.0 * m, k_ls_rows,
               (unsigned)tiles, kBlock, t, keys2, m, nv, nnz, idx, tsum, f->col_ptr, f->rows, f->left, f->beta);
    f->has_left_beta = 1;
    PMS_HIP(hipGetLastError());
    int32_t herr = 0;
    PMS_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    PMS_HIP(hipStreamSynchronize(s));
    if (c->prof_on) prof_flush(c);
    if (herr == 1) return set_err(c, PMS_ERR_INVALID_ARG, "grid holds NaN");
    if (herr) return set_err(c, PMS_ERR_HIP, "internal: simplex count mismatch in the lower-star builder");
    return PMS_OK;
}

}  // namespace pms
