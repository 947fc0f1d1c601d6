// Depth images and visibility of a triangle mesh in every camera (Sec. II-D,
// Eq. (4)) on gfx950, with the readings stated in include/fvv.h
// (fvv_visibility): a triangle covers the pixels whose centres lie on the same
// side of its three projected edges, at the camera-plane distance of its
// centroid; a pixel keeps the minimum; a triangle is visible in a camera when
// its centroid projects into the image and its distance exceeds the depth
// there by at most T_v.
//
// Depth: one thread per triangle, its vertices loaded once and rastered in
// every camera in turn (a wave's triangles, listed cell by cell, touch
// neighbouring pixels of each image); the minimum is an atomicMin on the
// float's bits (the distances are positive, so their bit patterns order like
// the values and the result does not depend on the order of the updates).  Visibility: one thread per triangle
// over all cameras, one mask word each.  All arithmetic is fp32 in a fixed
// order with IEEE division, as the reading defines it.
#include <algorithm>

#include "fvv_internal.h"

namespace fvv {

constexpr uint32_t kInfBits = 0x7f800000u;   // +inf

__global__ __launch_bounds__(kBlock) void depth_clear_kernel(uint32_t* __restrict__ depth,
                                                             size_t n) {
    for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < n;
         q += (size_t)gridDim.x * kBlock)
        depth[q] = kInfBits;
}

__device__ __forceinline__ void project3(const float* p, const float X[3], float& a, float& b,
                                         float& w) {
    a = __builtin_fmaf(p[2], X[2], __builtin_fmaf(p[1], X[1], __builtin_fmaf(p[0], X[0], p[3])));
    b = __builtin_fmaf(p[6], X[2], __builtin_fmaf(p[5], X[1], __builtin_fmaf(p[4], X[0], p[7])));
    w = __builtin_fmaf(p[10], X[2], __builtin_fmaf(p[9], X[1], __builtin_fmaf(p[8], X[0], p[11])));
}

// The triangle's vertices, or false when it names a vertex past nv.
__device__ __forceinline__ bool load_triangle(const float* __restrict__ xyz,
                                              const uint32_t* __restrict__ tris, uint32_t m,
                                              uint32_t nv, float V[3][3]) {
    const uint32_t t0 = tris[3 * (size_t)m], t1 = tris[3 * (size_t)m + 1],
                   t2 = tris[3 * (size_t)m + 2];
    if (t0 >= nv || t1 >= nv || t2 >= nv)
        return false;
    const uint32_t t[3] = {t0, t1, t2};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            V[k][a] = xyz[3 * (size_t)t[k] + a];
    return true;
}

// Camera-plane distance of the centroid ((v0 + v1) + v2) / 3 and its image
// position.
__device__ __forceinline__ void centroid(const float* p, const float V[3][3], float& u, float& v,
                                         float& w) {
    float G[3], a, b;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        G[k] = ((V[0][k] + V[1][k]) + V[2][k]) / 3.0f;
    project3(p, G, a, b, w);
    u = a / w;
    v = b / w;
}

__device__ __forceinline__ float edge_fn(float x0, float y0, float x1, float y1, float px,
                                         float py) {
    return (x1 - x0) * (py - y0) - (y1 - y0) * (px - x0);
}

// The pixels of one triangle (vertices V) in one camera: skipped when a vertex
// is behind the camera, the projected area is zero, the centroid's distance is
// not positive or the box misses the image; else atomicMin of the distance's
// bits into each covered pixel of the camera's depth image D.
__device__ __forceinline__ void raster_one(const float* p, const float V[3][3], int W, int H,
                                           uint32_t* __restrict__ D) {
    float u[3], v[3];
    bool front = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float a, b, w;
        project3(p, V[k], a, b, w);
        front &= w > 0.0f;
        u[k] = a / w;
        v[k] = b / w;
    }
    if (!front || edge_fn(u[0], v[0], u[1], v[1], u[2], v[2]) == 0.0f)
        return;
    float gu, gv, d;
    centroid(p, V, gu, gv, d);
    if (!(d > 0.0f))
        return;
    const float lo_u = fminf(u[0], fminf(u[1], u[2])), hi_u = fmaxf(u[0], fmaxf(u[1], u[2]));
    const float lo_v = fminf(v[0], fminf(v[1], v[2])), hi_v = fmaxf(v[0], fmaxf(v[1], v[2]));
    if (!(hi_u >= 0.0f && hi_v >= 0.0f && lo_u < (float)W && lo_v < (float)H))
        return;
    // pixels whose centres could be inside (the edge test decides)
    const int x0 = lo_u < 0.0f ? 0 : (int)lo_u;
    const int y0 = lo_v < 0.0f ? 0 : (int)lo_v;
    const int x1 = hi_u >= (float)(W - 1) ? W - 1 : (int)hi_u;
    const int y1 = hi_v >= (float)(H - 1) ? H - 1 : (int)hi_v;
    const uint32_t dbits = __float_as_uint(d);
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            const float px = (float)x + 0.5f, py = (float)y + 0.5f;
            const float e0 = edge_fn(u[0], v[0], u[1], v[1], px, py);
            const float e1 = edge_fn(u[1], v[1], u[2], v[2], px, py);
            const float e2 = edge_fn(u[2], v[2], u[0], v[0], px, py);
            const bool in = (e0 >= 0.0f && e1 >= 0.0f && e2 >= 0.0f) ||
                            (e0 <= 0.0f && e1 <= 0.0f && e2 <= 0.0f);
            if (in)
                atomicMin(&D[(size_t)y * W + x], dbits);
        }
}

__global__ __launch_bounds__(kBlock) void depth_raster_kernel(
    const CamSet cams, const float* __restrict__ xyz, const uint32_t* __restrict__ n_vert_p,
    uint32_t max_vert, const uint32_t* __restrict__ tris, const uint32_t* __restrict__ n_tris_p,
    uint32_t max_tris, uint32_t* __restrict__ depth) {
    const uint32_t nv_all = *n_vert_p, nt_all = *n_tris_p;
    const uint32_t nv = nv_all < max_vert ? nv_all : max_vert;
    const uint32_t T = nt_all < max_tris ? nt_all : max_tris;
    const int W = cams.W, H = cams.H;
    for (uint64_t mm = (uint64_t)blockIdx.x * kBlock + threadIdx.x; mm < T;
         mm += (uint64_t)gridDim.x * kBlock) {
        float V[3][3];
        if (!load_triangle(xyz, tris, (uint32_t)mm, nv, V))
            continue;
        for (int c = 0; c < cams.n; ++c)
            raster_one(cams.P[c], V, W, H, depth + (size_t)c * W * H);
    }
}

__global__ __launch_bounds__(kBlock) void visibility_kernel(
    const CamSet cams, const float* __restrict__ xyz, const uint32_t* __restrict__ n_vert_p,
    uint32_t max_vert, const uint32_t* __restrict__ tris, const uint32_t* __restrict__ n_tris_p,
    uint32_t max_tris, const float* __restrict__ depth, float t_v, uint32_t* __restrict__ vis) {
    const uint32_t nv_all = *n_vert_p, nt_all = *n_tris_p;
    const uint32_t nv = nv_all < max_vert ? nv_all : max_vert;
    const uint32_t T = nt_all < max_tris ? nt_all : max_tris;
    const int W = cams.W, H = cams.H;
    for (uint32_t m = blockIdx.x * kBlock + threadIdx.x; m < T; m += gridDim.x * kBlock) {
        float V[3][3];
        uint32_t mask = 0;
        if (load_triangle(xyz, tris, m, nv, V))
            for (int c = 0; c < cams.n; ++c) {
                float u, v, d;
                centroid(cams.P[c], V, u, v, d);
                if (!(d > 0.0f))
                    continue;
                const float fx = __builtin_floorf(u), fy = __builtin_floorf(v);
                if (!(fx >= 0.0f && fy >= 0.0f && fx < (float)W && fy < (float)H))
                    continue;
                const float D = depth[((size_t)c * H + (size_t)fy) * W + (size_t)fx];
                if (d - D <= t_v)
                    mask |= 1u << c;
            }
        vis[m] = mask;
    }
}

hipError_t launch_visibility(fvv_ctx* ctx, const CamSet& cams, const float* xyz,
                             const uint32_t* n_vert, uint32_t max_vert, const uint32_t* tris,
                             const uint32_t* n_tris, uint32_t max_tris, float t_v, float* depth,
                             uint32_t* vis, hipStream_t s) {
    const size_t n = (size_t)cams.n * cams.W * cams.H;
    const int64_t cap = (int64_t)ctx->n_cus * 8;
    hipLaunchKernelGGL(depth_clear_kernel,
                       dim3((unsigned)std::min<int64_t>(((int64_t)n + kBlock - 1) / kBlock, cap)),
                       dim3(kBlock), 0, s, reinterpret_cast<uint32_t*>(depth), n);
    hipLaunchKernelGGL(depth_raster_kernel,
                       dim3((unsigned)std::min<int64_t>(((int64_t)max_tris + kBlock - 1) / kBlock,
                                                        cap)),
                       dim3(kBlock), 0, s, cams, xyz, n_vert, max_vert, tris, n_tris, max_tris,
                       reinterpret_cast<uint32_t*>(depth));
    hipLaunchKernelGGL(visibility_kernel,
                       dim3((unsigned)std::min<int64_t>(((int64_t)max_tris + kBlock - 1) / kBlock,
                                                        cap)),
                       dim3(kBlock), 0, s, cams, xyz, n_vert, max_vert, tris, n_tris, max_tris,
                       depth, t_v, vis);
    return hipGetLastError();
}

}  // namespace fvv
