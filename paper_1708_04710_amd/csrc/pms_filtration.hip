// Library-owned filtrations: allocation, views and the builder entry points
// of the C ABI.
#include <hip/hip_runtime.h>

#include <new>

#include "pms_build.h"

namespace pms {

static void filtration_release(Filtration *f)
{
    if (!f) return;
    (void)hipFree(f->col_ptr);
    (void)hipFree(f->rows);
    (void)hipFree(f->dim);
    (void)hipFree(f->value);
    (void)hipFree(f->crit);
    (void)hipFree(f->verts);
    (void)hipFree(f->left);
    (void)hipFree(f->beta);
    f->left = f->beta = nullptr;
    f->col_ptr = nullptr;
    f->rows = nullptr;
    f->dim = nullptr;
    f->value = nullptr;
    f->crit = nullptr;
    f->verts = nullptr;
    f->cap_m = f->cap_nnz = 0;
}

pms_status filtration_reserve(Ctx *c, Filtration **pf, int64_t m, int64_t nnz, int f32)
{
    Filtration *f = *pf;
    if (!f) {
        f = new (std::nothrow) Filtration();
        if (!f) return set_err(c, PMS_ERR_OOM, "filtration");
        f->device = c->device;
        *pf = f;
    }
    f->has_left_beta = 0;  // until a builder writes them
    if (f->cap_m >= m && f->cap_nnz >= nnz && f->device == c->device) return PMS_OK;
    (void)hipStreamSynchronize(c->stream);
    filtration_release(f);
    f->device = c->device;
    const int64_t M = m > 0 ? m : 1, Z = nnz > 0 ? nnz : 1;
    PMS_HIP(hipMalloc(&f->col_ptr, (M + 1) * 8));
    PMS_HIP(hipMalloc(&f->rows, Z * 4));
    PMS_HIP(hipMalloc(&f->dim, M));
    PMS_HIP(hipMalloc(&f->value, M * 8));
    PMS_HIP(hipMalloc(&f->crit, M * 8));
    PMS_HIP(hipMalloc(&f->verts, M * 16));
    PMS_HIP(hipMalloc(&f->left, M * 4));
    PMS_HIP(hipMalloc(&f->beta, M * 4));
    f->cap_m = M;
    f->cap_nnz = Z;
    (void)f32;
    return PMS_OK;
}

__global__ void __launch_bounds__(kBlock) k_tile_sums(const int64_t *data, int64_t n, int64_t *tmp)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t t = block_sum64(i < n ? data[i] : 0);
    if (threadIdx.x == 0) tmp[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_tile_apply(int64_t *data, int64_t n, const int64_t *tmp, int64_t *total)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t v = i < n ? data[i] : 0;
    const int64_t e = tmp[blockIdx.x] + block_excl_sum64(v);
    if (i < n) data[i] = e;
    if (i == n - 1) *total = e + v;
}

pms_status scan_i64(Ctx *c, int64_t *data, int64_t n, int64_t *tmp, int64_t *total)
{
    *total = 0;
    if (n <= 0) return PMS_OK;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    PMS_LAUNCH(c, K_BUILD_SCAN, 8.0 * n, k_tile_sums, (unsigned)tiles, kBlock, data, n, tmp);
    PMS_LAUNCH(c, K_BUILD_SCAN, 16.0 * tiles, k_scan_i64, 1, 1024, tmp, tiles);
    PMS_LAUNCH(c, K_BUILD_SCAN, 16.0 * n, k_tile_apply, (unsigned)tiles, kBlock, data, n, tmp, tmp + tiles + 1);
    PMS_HIP(hipGetLastError());
    PMS_HIP(hipMemcpyAsync(total, tmp + tiles + 1, 8, hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    return PMS_OK;
}

}  // namespace pms


extern "C" {

pms_status pms_build_lowerstar(pms_ctx *ctx, const float *grid, int32_t nx, int32_t ny, int32_t nz,
                               pms_filtration **f)
{
    pms::Ctx *c = reinterpret_cast<pms::Ctx *>(ctx);
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!f) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null filtration handle");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    pms::Filtration *pf = reinterpret_cast<pms::Filtration *>(*f);
    pms_status s = pms::build_lowerstar(c, grid, nx, ny, nz, &pf);
    *f = reinterpret_cast<pms_filtration *>(pf);
    return s;
}

static pms_status vr_entry(pms_ctx *ctx, const void *pts, bool f32, int32_t count, const int32_t *n,
                           const int32_t *D, const int64_t *pt_off, const void *thr, int32_t maxdim, pms_filtration **f,
                           int64_t *inst_col_off)
{
    pms::Ctx *c = reinterpret_cast<pms::Ctx *>(ctx);
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!f) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null filtration handle");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    pms::Filtration *pf = reinterpret_cast<pms::Filtration *>(*f);
    pms_status s = pms::build_vr_batch(c, pts, f32, n, D, pt_off, thr, count, maxdim, &pf, inst_col_off);
    *f = reinterpret_cast<pms_filtration *>(pf);
    return s;
}

pms_status pms_build_vr_i32(pms_ctx *ctx, const int32_t *pts, int32_t count, const int32_t *n, const int32_t *D,
                            const int64_t *pt_off, const int64_t *thr_sqd, int32_t maxdim, pms_filtration **f,
                            int64_t *inst_col_off)
{
    return vr_entry(ctx, pts, false, count, n, D, pt_off, thr_sqd, maxdim, f, inst_col_off);
}

pms_status pms_build_vr_f32(pms_ctx *ctx, const float *pts, int32_t count, const int32_t *n, const int32_t *D,
                            const int64_t *pt_off, const float *thr_sqd, int32_t maxdim, pms_filtration **f,
                            int64_t *inst_col_off)
{
    return vr_entry(ctx, pts, true, count, n, D, pt_off, thr_sqd, maxdim, f, inst_col_off);
}

pms_status pms_filtration_view_get(const pms_filtration *fh, pms_filtration_view *v)
{
    const pms::Filtration *f = reinterpret_cast<const pms::Filtration *>(fh);
    if (!f || !v) return PMS_ERR_INVALID_ARG;
    v->m = f->m;
    v->nnz = f->nnz;
    v->col_ptr = f->col_ptr;
    v->rows = f->rows;
    v->dim = f->dim;
    v->value_f32 = f->value_is_f32 ? (const float *)f->value : nullptr;
    v->value_i64 = f->value_is_f32 ? nullptr : (const int64_t *)f->value;
    v->crit = f->crit;
    v->verts = f->verts;
    v->left = f->has_left_beta ? f->left : nullptr;
    v->beta = f->has_left_beta ? f->beta : nullptr;
    return PMS_OK;
}

pms_status pms_filtration_copy_left_beta(pms_ctx *ctx, const pms_filtration *fh, int32_t *left, int32_t *beta)
{
    pms::Ctx *c = reinterpret_cast<pms::Ctx *>(ctx);
    const pms::Filtration *f = reinterpret_cast<const pms::Filtration *>(fh);
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (!f || !f->has_left_beta) return pms::set_err(c, PMS_ERR_INVALID_ARG, "the filtration has no left / beta");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    const size_t n = (size_t)f->m * 4;
    if (left && n) PMS_HIP(hipMemcpyAsync(left, f->left, n, hipMemcpyDeviceToDevice, c->stream));
    if (beta && n) PMS_HIP(hipMemcpyAsync(beta, f->beta, n, hipMemcpyDeviceToDevice, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    return PMS_OK;
}

pms_status pms_filtration_copy_out(pms_ctx *ctx, const pms_filtration *fh, int64_t *col_ptr, int32_t *rows,
                                   int8_t *dim, void *value, int32_t *crit, int32_t *verts)
{
    pms::Ctx *c = reinterpret_cast<pms::Ctx *>(ctx);
    const pms::Filtration *f = reinterpret_cast<const pms::Filtration *>(fh);
    if (!c || !f) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (col_ptr) PMS_HIP(hipMemcpyAsync(col_ptr, f->col_ptr, (f->m + 1) * 8, k, c->stream));
    if (rows && f->nnz) PMS_HIP(hipMemcpyAsync(rows, f->rows, f->nnz * 4, k, c->stream));
    if (dim && f->m) PMS_HIP(hipMemcpyAsync(dim, f->dim, f->m, k, c->stream));
    if (value && f->m) PMS_HIP(hipMemcpyAsync(value, f->value, f->m * (f->value_is_f32 ? 4 : 8), k, c->stream));
    if (crit && f->m) PMS_HIP(hipMemcpyAsync(crit, f->crit, f->m * 8, k, c->stream));
    if (verts && f->m) PMS_HIP(hipMemcpyAsync(verts, f->verts, f->m * 16, k, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    return PMS_OK;
}

void pms_filtration_free(pms_filtration *f)
{
    if (!f) return;
    pms::Filtration *pf = reinterpret_cast<pms::Filtration *>(f);
    (void)hipSetDevice(pf->device);
    (void)hipDeviceSynchronize();
    pms::filtration_release(pf);
    delete pf;
}

}  // extern "C"
