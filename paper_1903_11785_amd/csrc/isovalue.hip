// The paper's own isovalue of the crossing edges (Sec. II-C, Eq. (2)-(3)) on
// gfx950: in each camera the last foreground pixel of the Bresenham line from
// the occupied end's pixel to the other end's, the image-space ratio of
// Eq. (2), and the minimum over cameras of Eq. (3).  The readings of the
// points the paper leaves open are those stated in include/fvv.h
// (fvv_isovalue).  The exit-point bisection is the path's estimator; this is
// the paper's, for comparison.
//
// One lane per edge.  The ends' projections are the occupancy test's fp32
// rows; pixel indices are exact floors (rcp quotient corrected by fma
// residuals), the far end's clamped to [-8, dim + 8].  lambda_i^2 is the IEEE
// double quotient of two integer squared lengths, so the minimum and its
// correctly rounded square root do not depend on how the walk was evaluated.
#include "fvv_internal.h"

namespace fvv {

// Exact floor of a/w (w > 0), clamped to [-8, dim + 8].  The rcp quotient is
// first clamped to +-2^20, where it is within 1 of a/w; beyond that the
// clamp to the image margin gives the same result either way.
__device__ __forceinline__ int line_pixel(float a, float w, int dim) {
    float q;
    if (w >= 0x1p-64f)
        q = a * __builtin_amdgcn_rcpf(w);
    else
        q = a / w;
    q = __builtin_amdgcn_fmed3f(q, -0x1p20f, 0x1p20f);
    const int n = exact_floor(a, w, q);
    return n < -8 ? -8 : (n > dim + 8 ? dim + 8 : n);
}

__device__ __forceinline__ bool sil_fg(const uint32_t* __restrict__ sil, int W, int H, int wpr,
                                       int x, int y) {
    const bool in = ((unsigned)x < (unsigned)W) & ((unsigned)y < (unsigned)H);
    const uint32_t word = sil[in ? y * wpr + (x >> 5) : 0];
    return in & (((word >> (x & 31)) & 1u) != 0u);
}

// lambda_i^2 for the pixel line (x0, y0) -> (x1, y1): Bresenham's integer
// walk (error term dx - dy; a step along x when twice the error is at least
// -dy, along y when it is at most dx), stopping at the first pixel that is
// background or off the image; 1 when the line is foreground to its end, 0
// when its start is not foreground.
__device__ __forceinline__ double line_lambda2(const uint32_t* __restrict__ sil, int W, int H,
                                               int wpr, int x0, int y0, int x1, int y1) {
    if (!sil_fg(sil, W, H, wpr, x0, y0))
        return 0.0;
    const int dx = abs(x1 - x0), dy = abs(y1 - y0);
    const int sx = x0 < x1 ? 1 : -1, sy = y0 < y1 ? 1 : -1;
    int err = dx - dy;
    int x = x0, y = y0, lx = x0, ly = y0;
    while (x != x1 || y != y1) {
        const int e2 = 2 * err;
        if (e2 >= -dy) {
            err -= dy;
            x += sx;
        }
        if (e2 <= dx) {
            err += dx;
            y += sy;
        }
        if (!sil_fg(sil, W, H, wpr, x, y)) {
            const int64_t ax = lx - x0, ay = ly - y0, bx = x1 - x0, by = y1 - y0;
            return (double)(ax * ax + ay * ay) / (double)(bx * bx + by * by);
        }
        lx = x;
        ly = y;
    }
    return 1.0;
}

__global__ __launch_bounds__(kBlock) void isovalue_kernel(const fvv_grid g,
                                                          const uint8_t* __restrict__ occ,
                                                          const CamSet cams,
                                                          const uint32_t* __restrict__ sils,
                                                          const uint32_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ n_keys_p,
                                                          uint32_t max_keys,
                                                          float* __restrict__ lambda,
                                                          float* __restrict__ xyz) {
    const uint32_t nk_all = *n_keys_p;
    const uint32_t nk = nk_all < max_keys ? nk_all : max_keys;
    const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1], nz = (uint32_t)g.dims[2];
    const int W = cams.W, H = cams.H, wpr = cams.wpr;
    const size_t sil_stride = (size_t)H * wpr;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < nk; e += gridDim.x * kBlock) {
        const uint32_t key = keys[e];
        const uint32_t lin = key / 3u, axis = key - 3u * lin;
        const uint32_t r = lin / nx, i = lin - r * nx;
        const uint32_t k = r / ny, j = r - k * ny;
        // a key must name an edge of the lattice (both samples inside)
        const bool ok = k < nz && (axis == 0 ? i + 1 < nx : axis == 1 ? j + 1 < ny : k + 1 < nz);
        if (!ok) {
            lambda[e] = __builtin_nanf("");
            if (xyz)
                xyz[3 * (size_t)e] = xyz[3 * (size_t)e + 1] = xyz[3 * (size_t)e + 2] =
                    __builtin_nanf("");
            continue;
        }
        const bool p_on = occ[lin] != 0;
        const int32_t ga[3] = {g.lo[0] + (int32_t)i, g.lo[1] + (int32_t)j, g.lo[2] + (int32_t)k};
        const int32_t gax = axis == 0 ? ga[0] : (axis == 1 ? ga[1] : ga[2]);
        const int32_t g_on = p_on ? gax : gax + 1;
        const int32_t g_off = p_on ? gax + 1 : gax;
        const float o_ax = axis == 0 ? g.origin[0] : (axis == 1 ? g.origin[1] : g.origin[2]);
        float Xon[3], Xoff[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            Xon[a] = Xoff[a] = __builtin_fmaf((float)ga[a], g.h, g.origin[a]);
        const float c_on = __builtin_fmaf((float)g_on, g.h, o_ax);
        const float c_off = __builtin_fmaf((float)g_off, g.h, o_ax);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Xon[a] = (uint32_t)a == axis ? c_on : Xon[a];
            Xoff[a] = (uint32_t)a == axis ? c_off : Xoff[a];
        }
        double best = 1.0;
        for (int c = 0; c < cams.n; ++c) {
            const float* p = cams.P[c];
            const float a0 = __builtin_fmaf(p[2], Xon[2], __builtin_fmaf(p[1], Xon[1], __builtin_fmaf(p[0], Xon[0], p[3])));
            const float b0 = __builtin_fmaf(p[6], Xon[2], __builtin_fmaf(p[5], Xon[1], __builtin_fmaf(p[4], Xon[0], p[7])));
            const float w0 = __builtin_fmaf(p[10], Xon[2], __builtin_fmaf(p[9], Xon[1], __builtin_fmaf(p[8], Xon[0], p[11])));
            const float a1 = __builtin_fmaf(p[2], Xoff[2], __builtin_fmaf(p[1], Xoff[1], __builtin_fmaf(p[0], Xoff[0], p[3])));
            const float b1 = __builtin_fmaf(p[6], Xoff[2], __builtin_fmaf(p[5], Xoff[1], __builtin_fmaf(p[4], Xoff[0], p[7])));
            const float w1 = __builtin_fmaf(p[10], Xoff[2], __builtin_fmaf(p[9], Xoff[1], __builtin_fmaf(p[8], Xoff[0], p[11])));
            double l2 = 0.0;   // an end behind the camera
            if (w1 > 0.0f && w0 > 0.0f)
                l2 = line_lambda2(sils + c * sil_stride, W, H, wpr, line_pixel(a0, w0, W),
                                  line_pixel(b0, w0, H), line_pixel(a1, w1, W),
                                  line_pixel(b1, w1, H));
            best = l2 < best ? l2 : best;
        }
        const float lam = (float)__builtin_sqrt(best);
        lambda[e] = lam;
        if (xyz) {
            const float d = p_on ? 1.0f : -1.0f;
            const float q = __builtin_fmaf((float)g_on + d * lam, g.h, o_ax);
            xyz[3 * (size_t)e + 0] = axis == 0 ? q : Xon[0];
            xyz[3 * (size_t)e + 1] = axis == 1 ? q : Xon[1];
            xyz[3 * (size_t)e + 2] = axis == 2 ? q : Xon[2];
        }
    }
}

hipError_t launch_isovalue(fvv_ctx* ctx, const fvv_grid& g, const uint8_t* occ, const CamSet& cams,
                           const uint32_t* sils, const uint32_t* keys, const uint32_t* n_keys,
                           uint32_t max_keys, float* lambda, float* xyz, hipStream_t s) {
    const int64_t want = ((int64_t)max_keys + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)ctx->n_cus * 8;
    hipLaunchKernelGGL(isovalue_kernel, dim3((unsigned)(want < cap ? want : cap)), dim3(kBlock), 0,
                       s, g, occ, cams, sils, keys, n_keys, max_keys, lambda, xyz);
    return hipGetLastError();
}

}  // namespace fvv
