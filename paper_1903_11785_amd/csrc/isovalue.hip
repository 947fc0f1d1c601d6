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

constexpr int kIsoGroup = 4;   // cameras whose first pixel loads are issued together

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

// One camera's pixel line: its ends and the walk's state after the first
// step (Bresenham's integer walk: error term dx - dy; a step along x when
// twice the error is at least -dy, along y when it is at most dx).
struct PixelLine {
    int x0, y0, x1, y1;
    int x, y, err, dx, dy, sx, sy;
};

__device__ __forceinline__ void line_step(PixelLine& l) {
    const int e2 = 2 * l.err;
    if (e2 >= -l.dy) {
        l.err -= l.dy;
        l.x += l.sx;
    }
    if (e2 <= l.dx) {
        l.err += l.dx;
        l.y += l.sy;
    }
}

__device__ __forceinline__ PixelLine line_start(int x0, int y0, int x1, int y1) {
    PixelLine l;
    l.x0 = x0;
    l.y0 = y0;
    l.x1 = x1;
    l.y1 = y1;
    l.dx = abs(x1 - x0);
    l.dy = abs(y1 - y0);
    l.sx = x0 < x1 ? 1 : -1;
    l.sy = y0 < y1 ? 1 : -1;
    l.err = l.dx - l.dy;
    l.x = x0;
    l.y = y0;
    if (x0 != x1 || y0 != y1)
        line_step(l);
    return l;
}

__device__ __forceinline__ double ratio2(int ax, int ay, int bx, int by) {
    return (double)((int64_t)ax * ax + (int64_t)ay * ay) /
           (double)((int64_t)bx * bx + (int64_t)by * by);
}

// min(best, lambda_i^2) for a line whose start and first-step pixels have
// been tested (fg0, fg1): the walk goes on from the first step while its
// pixels are foreground, stopping early once the ratio at the current pixel
// reaches `best` (it only grows along the line, so lambda_i^2 >= best).
__device__ __forceinline__ double line_min(const uint32_t* __restrict__ sil, int W, int H, int wpr,
                                           PixelLine l, bool fg0, bool fg1, double best) {
    if (!fg0)
        return 0.0;
    if (l.x0 == l.x1 && l.y0 == l.y1)
        return best;                               // lambda_i = 1
    const int bx = l.x1 - l.x0, by = l.y1 - l.y0;
    if (!fg1)
        return 0.0;                                // P_i = P_on
    int lx = l.x, ly = l.y;
    while (l.x != l.x1 || l.y != l.y1) {
        if (ratio2(lx - l.x0, ly - l.y0, bx, by) >= best)
            return best;
        line_step(l);
        if (!sil_fg(sil, W, H, wpr, l.x, l.y)) {
            const double r = ratio2(lx - l.x0, ly - l.y0, bx, by);
            return r < best ? r : best;
        }
        lx = l.x;
        ly = l.y;
    }
    return best;                                   // foreground to its end: lambda_i = 1
}

// lambda of one crossing edge of lattice g (axis-aligned from sample
// (i, j, k) along `axis`, p_on: whether that first sample is the occupied
// one), and the point there.
__device__ __forceinline__ float edge_isovalue(const fvv_grid& g, uint32_t i, uint32_t j,
                                               uint32_t k, uint32_t axis, bool p_on,
                                               const CamSet& cams,
                                               const uint32_t* __restrict__ sils, float xyz[3]) {
    const int W = cams.W, H = cams.H, wpr = cams.wpr;
    const size_t sil_stride = (size_t)H * wpr;
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
    // cameras in groups of kIsoGroup: every line's start and first-step
    // pixels are loaded together, then the walks go on one by one; an edge
    // stops at lambda = 0, which no camera can lower
    double best = 1.0;
    for (int c0 = 0; c0 < cams.n && best > 0.0; c0 += kIsoGroup) {
        PixelLine ln[kIsoGroup];
        bool live[kIsoGroup], fg0[kIsoGroup], fg1[kIsoGroup];
#pragma unroll
        for (int q = 0; q < kIsoGroup; ++q) {
            const int c = c0 + q < cams.n ? c0 + q : c0;
            const float* p = cams.P[c];
            const float a0 = __builtin_fmaf(p[2], Xon[2], __builtin_fmaf(p[1], Xon[1], __builtin_fmaf(p[0], Xon[0], p[3])));
            const float b0 = __builtin_fmaf(p[6], Xon[2], __builtin_fmaf(p[5], Xon[1], __builtin_fmaf(p[4], Xon[0], p[7])));
            const float w0 = __builtin_fmaf(p[10], Xon[2], __builtin_fmaf(p[9], Xon[1], __builtin_fmaf(p[8], Xon[0], p[11])));
            const float a1 = __builtin_fmaf(p[2], Xoff[2], __builtin_fmaf(p[1], Xoff[1], __builtin_fmaf(p[0], Xoff[0], p[3])));
            const float b1 = __builtin_fmaf(p[6], Xoff[2], __builtin_fmaf(p[5], Xoff[1], __builtin_fmaf(p[4], Xoff[0], p[7])));
            const float w1 = __builtin_fmaf(p[10], Xoff[2], __builtin_fmaf(p[9], Xoff[1], __builtin_fmaf(p[8], Xoff[0], p[11])));
            live[q] = c0 + q < cams.n;
            const bool front = w0 > 0.0f && w1 > 0.0f;   // else lambda_i = 0
            ln[q] = front ? line_start(line_pixel(a0, w0, W), line_pixel(b0, w0, H),
                                       line_pixel(a1, w1, W), line_pixel(b1, w1, H))
                          : line_start(-1, -1, -1, -1);
            const uint32_t* sil = sils + c * sil_stride;
            fg0[q] = sil_fg(sil, W, H, wpr, ln[q].x0, ln[q].y0);
            fg1[q] = sil_fg(sil, W, H, wpr, ln[q].x, ln[q].y);
        }
#pragma unroll
        for (int q = 0; q < kIsoGroup; ++q)
            if (live[q] && best > 0.0)
                best = line_min(sils + (c0 + q) * sil_stride, W, H, wpr, ln[q], fg0[q], fg1[q],
                                best);
    }
    const float lam = (float)__builtin_sqrt(best);
    const float d = p_on ? 1.0f : -1.0f;
    const float q = __builtin_fmaf((float)g_on + d * lam, g.h, o_ax);
    xyz[0] = axis == 0 ? q : Xon[0];
    xyz[1] = axis == 1 ? q : Xon[1];
    xyz[2] = axis == 2 ? q : Xon[2];
    return lam;
}

// The keys of one lattice (fvv_isovalue).
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
        float pt[3];
        lambda[e] = edge_isovalue(g, i, j, k, axis, occ[lin] != 0, cams, sils, pt);
        if (xyz) {
            xyz[3 * (size_t)e + 0] = pt[0];
            xyz[3 * (size_t)e + 1] = pt[1];
            xyz[3 * (size_t)e + 2] = pt[2];
        }
    }
}

// The crossing edges of a frame's jobs (ROI-major keys with point_off): the
// points at the paper's isovalue in place of the bisection's.  xyz[3e] holds
// the edge pass's side mark (+1: the key's sample is the occupied one).
__global__ __launch_bounds__(kBlock) void isovalue_jobs_kernel(
    const fvv_job* __restrict__ jobs, const uint32_t* __restrict__ n_jobs_p,
    const uint32_t* __restrict__ point_off, const CamSet cams, const uint32_t* __restrict__ sils,
    const uint32_t* __restrict__ keys, float* __restrict__ xyz, uint32_t max_points) {
    __shared__ uint32_t s_off[kJobTable + 1];
    const int nj = (int)*n_jobs_p;
    const bool lds = nj < kJobTable;
    if (lds)
        for (int j = threadIdx.x; j <= nj; j += kBlock)
            s_off[j] = point_off[j];
    __syncthreads();
    const uint32_t total = lds ? s_off[nj] : point_off[nj];
    const uint32_t E = total < max_points ? total : max_points;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < E; e += gridDim.x * kBlock) {
        const int jb = lds ? upper_job([&](int m) { return (uint64_t)s_off[m]; }, nj, e)
                           : upper_job([&](int m) { return (uint64_t)point_off[m]; }, nj, e);
        const fvv_grid g = jobs[jb].grid;
        const uint32_t key = keys[e];
        const uint32_t lin = key / 3u, axis = key - 3u * lin;
        const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1];
        const uint32_t r = lin / nx, i = lin - r * nx;
        const uint32_t k = r / ny, j = r - k * ny;
        const bool p_on = xyz[3 * (size_t)e] > 0.0f;
        float pt[3];
        edge_isovalue(g, i, j, k, axis, p_on, cams, sils, pt);
        xyz[3 * (size_t)e + 0] = pt[0];
        xyz[3 * (size_t)e + 1] = pt[1];
        xyz[3 * (size_t)e + 2] = pt[2];
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

hipError_t launch_isovalue_jobs(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                                const uint32_t* point_off, const CamSet& cams,
                                const uint32_t* sils, const uint32_t* keys, float* xyz,
                                uint32_t max_points, hipStream_t s, hipEvent_t k_start,
                                hipEvent_t k_stop) {
    const int64_t want = ((int64_t)max_points + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)ctx->n_cus * 8;
    hipExtLaunchKernelGGL(isovalue_jobs_kernel, dim3((unsigned)(want < cap ? want : cap)),
                          dim3(kBlock), 0, s, k_start, k_stop, 0, jobs, n_jobs_dev, point_off,
                          cams, sils, keys, xyz, max_points);
    return hipGetLastError();
}

}  // namespace fvv
