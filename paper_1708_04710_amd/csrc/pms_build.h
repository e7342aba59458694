// Internal: library-owned filtrations produced by the GPU builders.
#pragma once

#include "pms_common.h"

namespace pms {

// Device arrays of one filtration in compatible order (owned by the library).
struct Filtration {
    int device = 0;
    int64_t m = 0, nnz = 0;
    int64_t cap_m = 0, cap_nnz = 0;
    int64_t *col_ptr = nullptr;  // [m+1]
    int32_t *rows = nullptr;     // [nnz]
    int8_t *dim = nullptr;       // [m]
    void *value = nullptr;       // [m] float or int64
    int32_t *crit = nullptr;     // [2m] critical vertex / critical edge endpoints
    int32_t *verts = nullptr;    // [4m] ascending vertex ids, -1 padded
    int32_t *left = nullptr;     // [m] Def. "left" (2^31 - 1: no column holds the row), when has_left_beta
    int32_t *beta = nullptr;     // [m] Def. "beta" (-1: none), when has_left_beta
    int value_is_f32 = 1;
    int has_left_beta = 0;       // the builder wrote left and beta
};

// (Re)allocate *f for m simplices and nnz facets; reuses it when big enough.
pms_status filtration_reserve(Ctx *c, Filtration **f, int64_t m, int64_t nnz, int f32);

pms_status build_lowerstar(Ctx *c, const float *grid, int32_t nx, int32_t ny, int32_t nz, Filtration **out);
pms_status build_vr_batch(Ctx *c, const void *pts, bool f32, const int32_t *n, const int32_t *D, const int64_t *pt_off,
                          const void *thr, int32_t B, int32_t maxdim, Filtration **out, int64_t *inst_col_off);

// In-place exclusive scan of n int64 on ctx's stream; *total receives the
// sum (the call synchronises).  tmp holds ceil(n / kBlock) + 2 entries.
pms_status scan_i64(Ctx *c, int64_t *data, int64_t n, int64_t *tmp, int64_t *total);

// Exclusive scan of n int64 in place, one block of 1024 threads.
static __global__ void __launch_bounds__(1024) k_scan_i64(int64_t *a, int64_t n)
{
    block_seg_scan(a, n, (int64_t)0, [](int64_t x, int64_t y) { return x + y; });
}

}  // namespace pms
