// Values of chosen simplices and the backward pass through a fixed pairing.
//
// With the pairing fixed, a persistence loss depends on the input only
// through the filtration values of the paired simplices.  The value of a
// lower-star simplex is the value of its critical vertex (the argmax by
// (value, id)), so dL/dvalue goes to that grid value.  The value of a
// Vietoris-Rips simplex is the squared length of its critical edge (a, b)
// (its latest facet edge), so d value / d x_a = 2 (x_a - x_b) and
// d value / d x_b = -2 (x_a - x_b).  Contributions are accumulated with
// FP32 atomics into caller-zeroed gradient buffers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms_build.h"
#include "pms_common.h"

namespace pms {

__global__ void k_gather(const Filtration f, int64_t n, const int32_t *simplex, void *values, int8_t *dims,
                         int32_t *err)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = simplex[k];
        if (j < 0 || (int64_t)j >= f.m) {
            atomicExch(err, 1);
            continue;
        }
        if (values) {
            if (f.value_is_f32) ((float *)values)[k] = ((const float *)f.value)[j];
            else ((int64_t *)values)[k] = ((const int64_t *)f.value)[j];
        }
        if (dims) dims[k] = f.dim[j];
    }
}

// Each paired simplex's gradient goes to its critical vertex.  Pairs come
// in ascending order of death, and a vertex's lower star is contiguous in
// the filtration, so neighbouring lanes often add to the same vertex: a
// segmented sum over each run of equal vertices in neighbouring lanes (only
// the run's own values are added) leaves one atomic per run.
__global__ void __launch_bounds__(kBlock) k_backward_lowerstar(const Filtration f, int64_t n, const int32_t *simplex,
                                                              const float *grad, float *grad_grid, int64_t nv,
                                                              int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t k0 = blockIdx.x * (int64_t)kBlock; k0 < n; k0 += (int64_t)gridDim.x * kBlock) {
        const int64_t k = k0 + threadIdx.x;
        int32_t v = -1;
        float g = 0.0f;
        if (k < n) {
            const int32_t j = simplex[k];
            if (j < 0 || (int64_t)j >= f.m) {
                atomicExch(err, 1);
            } else {
                g = grad[k];
                if (g != 0.0f) {  // nothing to add otherwise: no gather of the critical vertex
                    const int32_t c = f.crit[2 * (int64_t)j];
                    if (c >= 0 && c < nv) v = c;
                }
            }
        }
        if (v < 0) g = 0.0f;
        const int32_t vprev = __shfl_up(v, 1, kWave), vnext = __shfl_down(v, 1, kWave);
        const uint64_t heads = __ballot(lane == 0 || vprev != v);
        const int start = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));  // the run's first lane
        float inc = g;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const float y = __shfl_up(inc, o, kWave);
            if (lane - o >= start) inc += y;
        }
        if (v >= 0 && (lane == kWave - 1 || vnext != v) && inc != 0.0f) atomicAdd(&grad_grid[v], inc);
    }
}

__global__ void k_backward_vr(const Filtration f, int64_t n, const int32_t *simplex, const float *grad,
                              const float *pts, int32_t D, int64_t npts, float *grad_pts, int32_t *err)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = simplex[k];
        if (j < 0 || (int64_t)j >= f.m) {
            atomicExch(err, 1);
            continue;
        }
        const float g = grad[k];
        if (g == 0.0f) continue;  // nothing to add: no gather of the critical edge
        const int32_t a = f.crit[2 * (int64_t)j], b = f.crit[2 * (int64_t)j + 1];
        if (a < 0 || b < 0) continue;  // vertices: value 0, no dependence
        if ((int64_t)a >= npts || (int64_t)b >= npts) {
            atomicExch(err, 1);
            continue;
        }
        for (int t = 0; t < D; t++) {
            const float d = pts[(int64_t)a * D + t] - pts[(int64_t)b * D + t];
            const float w = 2.0f * g * d;
            atomicAdd(&grad_pts[(int64_t)a * D + t], w);
            atomicAdd(&grad_pts[(int64_t)b * D + t], -w);
        }
    }
}

}  // namespace pms

extern "C" {

static pms_status bw_prologue(pms_ctx *ctx, const pms_filtration *fh, pms::Ctx **pc, const pms::Filtration **pf)
{
    pms::Ctx *c = reinterpret_cast<pms::Ctx *>(ctx);
    if (!c) return PMS_ERR_INVALID_ARG;
    c->err.clear();
    const pms::Filtration *f = reinterpret_cast<const pms::Filtration *>(fh);
    if (!f) return pms::set_err(c, PMS_ERR_INVALID_ARG, "null filtration");
    if (hipSetDevice(c->device) != hipSuccess) return pms::set_err(c, PMS_ERR_HIP, "hipSetDevice failed");
    *pc = c;
    *pf = f;
    return PMS_OK;
}

static pms_status bw_epilogue(pms::Ctx *c, int32_t *err)
{
    PMS_HIP(hipGetLastError());
    int32_t h = 0;
    PMS_HIP(hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, c->stream));
    PMS_HIP(hipStreamSynchronize(c->stream));
    if (c->prof_on) pms::prof_flush(c);
    if (h) return pms::set_err(c, PMS_ERR_INVALID_ARG, "simplex or vertex index out of range");
    return PMS_OK;
}

pms_status pms_gather(pms_ctx *ctx, const pms_filtration *fh, int64_t n, const int32_t *simplex, void *values,
                      int8_t *dims)
{
    pms::Ctx *c;
    const pms::Filtration *f;
    pms_status s = bw_prologue(ctx, fh, &c, &f);
    if (s != PMS_OK) return s;
    if (n < 0 || (n > 0 && !simplex)) return pms::set_err(c, PMS_ERR_INVALID_ARG, "bad gather arguments");
    int32_t *err = (int32_t *)pms::grow_scratch(c, pms::B_TMP1, 64);
    if (!err) return pms::set_err(c, PMS_ERR_OOM, "scratch");
    PMS_HIP(hipMemsetAsync(err, 0, 4, c->stream));
    if (n > 0)
        PMS_LAUNCH(c, pms::K_FINAL, 13.0 * n, pms::k_gather, pms::grid_for(n, pms::kBlock, 65536), pms::kBlock, *f, n,
                   simplex, values, dims, err);
    return bw_epilogue(c, err);
}

pms_status pms_backward_lowerstar(pms_ctx *ctx, const pms_filtration *fh, int64_t n, const int32_t *simplex,
                                  const float *grad, float *grad_grid, int64_t n_vertices)
{
    pms::Ctx *c;
    const pms::Filtration *f;
    pms_status s = bw_prologue(ctx, fh, &c, &f);
    if (s != PMS_OK) return s;
    if (n < 0 || (n > 0 && (!simplex || !grad || !grad_grid)))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "bad backward arguments");
    int32_t *err = (int32_t *)pms::grow_scratch(c, pms::B_TMP1, 64);
    if (!err) return pms::set_err(c, PMS_ERR_OOM, "scratch");
    PMS_HIP(hipMemsetAsync(err, 0, 4, c->stream));
    if (n > 0)
        PMS_LAUNCH(c, pms::K_BACKWARD, 20.0 * n, pms::k_backward_lowerstar, pms::grid_for(n, pms::kBlock, 65536),
                   pms::kBlock, *f, n, simplex, grad, grad_grid, n_vertices, err);
    return bw_epilogue(c, err);
}

pms_status pms_backward_vr_f32(pms_ctx *ctx, const pms_filtration *fh, int64_t n, const int32_t *simplex,
                               const float *grad, const float *pts, int32_t D, int64_t n_points, float *grad_pts)
{
    pms::Ctx *c;
    const pms::Filtration *f;
    pms_status s = bw_prologue(ctx, fh, &c, &f);
    if (s != PMS_OK) return s;
    if (n < 0 || D < 1 || (n > 0 && (!simplex || !grad || !pts || !grad_pts)))
        return pms::set_err(c, PMS_ERR_INVALID_ARG, "bad backward arguments");
    int32_t *err = (int32_t *)pms::grow_scratch(c, pms::B_TMP1, 64);
    if (!err) return pms::set_err(c, PMS_ERR_OOM, "scratch");
    PMS_HIP(hipMemsetAsync(err, 0, 4, c->stream));
    if (n > 0)
        PMS_LAUNCH(c, pms::K_BACKWARD, (20.0 + 16.0 * D) * n, pms::k_backward_vr,
                   pms::grid_for(n, pms::kBlock, 65536), pms::kBlock, *f, n, simplex, grad, pts, D, n_points,
                   grad_pts, err);
    return bw_epilogue(c, err);
}

}  // extern "C"
