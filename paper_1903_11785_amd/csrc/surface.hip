// Crossing-edge compaction and exit-point bisection (Sec. II-C) for gfx950.
//
// Crossing edges: work items are chunks of kEdgeChunk consecutive samples of
// one ROI, eight consecutive samples per thread.  A first pass counts each
// item's edges, one workgroup scans the counts, and a second pass writes keys
// 3*lin+axis in ascending order (a thread's keys are in order, and a block
// scan orders the threads).  Exit points: a group of four lanes per edge, each
// owning a quarter of the cameras; a first pass keeps the cameras that can
// reject some point of the edge at all, and the n_steps bisection steps test
// only those at each bracket midpoint.
#include "fvv_internal.h"

namespace fvv {

// The single job of fvv_surface, from the kernel arguments.
__global__ void surface_single_kernel(const fvv_job job, fvv_job* __restrict__ dst,
                                      JobPrefix* __restrict__ pre, uint32_t* __restrict__ counts) {
    if (threadIdx.x == 0) {
        dst[0] = job;
        const uint64_t V = (uint64_t)job.grid.dims[0] * job.grid.dims[1] * job.grid.dims[2];
        pre[0].item_off = 0;
        pre[1].item_off = (uint32_t)((V + kEdgeChunk - 1) / kEdgeChunk);
        counts[3] = 1;
    }
}

hipError_t launch_surface_prepare_single(fvv_ctx* ctx, const fvv_job& job, hipStream_t s) {
    hipLaunchKernelGGL(surface_single_kernel, dim3(1), dim3(64), 0, s, job, ctx->d_job_single,
                       ctx->d_prefix, ctx->d_counts_single);
    return hipGetLastError();
}

// ------------------------------------------------------------------ crossing edges
constexpr int kEdgeRun = kEdgeChunk / kBlock;   // consecutive samples per thread

struct ItemRef {
    int job;
    uint32_t lin0;
};

__device__ __forceinline__ ItemRef locate_item(const JobPrefix* __restrict__ pre, int nj,
                                               uint32_t item) {
    const int jb = upper_job([&](int m) { return (uint64_t)pre[m].item_off; }, nj, item);
    return {jb, (item - pre[jb].item_off) * (uint32_t)kEdgeChunk};
}

// Crossing bits (x, y, z in bits 3s, 3s+1, 3s+2) of this thread's kEdgeRun
// consecutive samples starting at lin; samples at or past V give 0.
__device__ __forceinline__ uint32_t run_bits(const uint8_t* __restrict__ occ, uint32_t lin,
                                             uint32_t V, int dx, int dy, int dz) {
    if (lin >= V)
        return 0;
    const uint32_t sx = (uint32_t)dx, sxy = (uint32_t)dx * (uint32_t)dy;
    uint32_t i = lin % sx;
    const uint32_t r = lin / sx;
    uint32_t j = r % (uint32_t)dy;
    uint32_t k = r / (uint32_t)dy;
    uint8_t o[kEdgeRun + 1], oy[kEdgeRun], oz[kEdgeRun];
#pragma unroll
    for (int s = 0; s <= kEdgeRun; ++s)
        o[s] = lin + s < V ? occ[lin + s] : 0;
#pragma unroll
    for (int s = 0; s < kEdgeRun; ++s) {
        oy[s] = lin + s + sx < V ? occ[lin + s + sx] : 0;
        oz[s] = lin + s + sxy < V ? occ[lin + s + sxy] : 0;
    }
    uint32_t bits = 0;
#pragma unroll
    for (int s = 0; s < kEdgeRun; ++s) {
        if (lin + s < V) {
            const bool c = o[s] != 0;
            if (i + 1 < sx && (o[s + 1] != 0) != c)
                bits |= 1u << (3 * s);
            if (j + 1 < (uint32_t)dy && (oy[s] != 0) != c)
                bits |= 2u << (3 * s);
            if (k + 1 < (uint32_t)dz && (oz[s] != 0) != c)
                bits |= 4u << (3 * s);
        }
        if (++i == sx) {
            i = 0;
            if (++j == (uint32_t)dy) {
                j = 0;
                ++k;
            }
        }
    }
    return bits;
}

__global__ __launch_bounds__(kBlock) void edge_count_kernel(const fvv_job* __restrict__ jobs,
                                                            const JobPrefix* __restrict__ pre,
                                                            const uint32_t* __restrict__ n_jobs_p,
                                                            const uint8_t* __restrict__ occ_base,
                                                            uint32_t* __restrict__ item_cnt) {
    __shared__ uint32_t scratch[kBlock / kWave];
    const int nj = (int)*n_jobs_p;
    const uint32_t n_items = pre[nj].item_off;
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const ItemRef ref = locate_item(pre, nj, item);
        const fvv_job job = jobs[ref.job];
        const uint32_t V = (uint32_t)job.grid.dims[0] * job.grid.dims[1] * job.grid.dims[2];
        const uint32_t bits = run_bits(occ_base + job.out_offset, ref.lin0 + threadIdx.x * kEdgeRun,
                                       V, job.grid.dims[0], job.grid.dims[1], job.grid.dims[2]);
        uint32_t total;
        block_exclusive_sum<kBlock>((uint32_t)__popc(bits), scratch, &total);
        if (threadIdx.x == 0)
            item_cnt[item] = total;
    }
}

// One workgroup: exclusive scan of the item counts, first edge of every job,
// and the total.
__global__ __launch_bounds__(1024) void edge_scan_kernel(const JobPrefix* __restrict__ pre,
                                                         const uint32_t* __restrict__ n_jobs_p,
                                                         const uint32_t* __restrict__ item_cnt,
                                                         uint32_t* __restrict__ item_base,
                                                         uint32_t* __restrict__ point_off,
                                                         uint32_t* __restrict__ n_points,
                                                         uint32_t max_points,
                                                         uint32_t* __restrict__ status) {
    __shared__ uint64_t scratch[1024 / kWave];
    const int nj = (int)*n_jobs_p;
    const uint32_t n_items = pre[nj].item_off;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n_items; base += 1024) {
        const uint32_t it = base + threadIdx.x;
        const uint64_t c = it < n_items ? item_cnt[it] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_sum64<1024>(c, scratch, &total);
        if (it < n_items)
            item_base[it] = (uint32_t)min(carry + ex, (uint64_t)0xffffffffull);
        carry += total;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nj; j += 1024)
        point_off[j] = item_base[pre[j].item_off];
    if (threadIdx.x == 0) {
        const uint32_t tot = (uint32_t)min(carry, (uint64_t)0xffffffffull);
        point_off[nj] = tot;
        *n_points = tot;
        if (carry > max_points)
            atomicOr(status, kFlagCapacity);
    }
}

__global__ __launch_bounds__(kBlock) void edge_write_kernel(const fvv_job* __restrict__ jobs,
                                                            const JobPrefix* __restrict__ pre,
                                                            const uint32_t* __restrict__ n_jobs_p,
                                                            const uint8_t* __restrict__ occ_base,
                                                            const uint32_t* __restrict__ item_base,
                                                            uint32_t* __restrict__ keys,
                                                            uint32_t max_points) {
    __shared__ uint32_t scratch[kBlock / kWave];
    const int nj = (int)*n_jobs_p;
    const uint32_t n_items = pre[nj].item_off;
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const ItemRef ref = locate_item(pre, nj, item);
        const fvv_job job = jobs[ref.job];
        const uint32_t V = (uint32_t)job.grid.dims[0] * job.grid.dims[1] * job.grid.dims[2];
        const uint32_t lin = ref.lin0 + threadIdx.x * kEdgeRun;
        uint32_t bits = run_bits(occ_base + job.out_offset, lin, V, job.grid.dims[0],
                                 job.grid.dims[1], job.grid.dims[2]);
        uint32_t total;
        uint32_t pos = item_base[item] + block_exclusive_sum<kBlock>((uint32_t)__popc(bits),
                                                                     scratch, &total);
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            if (pos < max_points)
                keys[pos] = 3u * (lin + (uint32_t)(b / 3)) + (uint32_t)(b % 3);
            ++pos;
        }
    }
}

// ------------------------------------------------------------------ exit points
constexpr int kLanesPerEdge = 4;

// Whether camera c accepts every point of the edge X0-X1: the pixel rectangle
// of the edge's projection, widened by cams.pad[c], lies inside the image and
// is entirely foreground.  The projection of a segment is the segment between
// the projections of its ends, and pad[c] bounds the distance between the real
// quotient of any point of the lattice's box and the rounded quotient the
// occupancy test floors (the ends' quotients here come from rcp, whose error
// pad[c] also covers).  Rectangles of more than 2 rows or 2 words are not
// examined (the camera then stays in the bisection).
__device__ __forceinline__ bool camera_accepts_edge(const CamSet& cams, int c,
                                                    const uint32_t* __restrict__ sil,
                                                    const float* X0, const float* X1) {
    const float* P = &cams.P[c][0];
    const float pad = cams.pad[c];
    float x[2], y[2];
    bool front = true;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float* X = e ? X1 : X0;
        const float a = __builtin_fmaf(P[2], X[2], __builtin_fmaf(P[1], X[1], __builtin_fmaf(P[0], X[0], P[3])));
        const float b = __builtin_fmaf(P[6], X[2], __builtin_fmaf(P[5], X[1], __builtin_fmaf(P[4], X[0], P[7])));
        const float w = __builtin_fmaf(P[10], X[2], __builtin_fmaf(P[9], X[1], __builtin_fmaf(P[8], X[0], P[11])));
        const float r = __builtin_amdgcn_rcpf(w);
        front = front && w > 0.0f;
        x[e] = a * r;
        y[e] = b * r;
    }
    const float fx0 = __builtin_floorf(fminf(x[0], x[1]) - pad);
    const float fx1 = __builtin_floorf(fmaxf(x[0], x[1]) + pad);
    const float fy0 = __builtin_floorf(fminf(y[0], y[1]) - pad);
    const float fy1 = __builtin_floorf(fmaxf(y[0], y[1]) + pad);
    const bool small = front && fx0 >= 0.0f && fy0 >= 0.0f && fx1 < (float)cams.W &&
                       fy1 < (float)cams.H && fx1 - fx0 <= 31.0f && fy1 - fy0 <= 1.0f;
    const int x0 = small ? (int)fx0 : 0, x1 = small ? (int)fx1 : 0;
    const int y0 = small ? (int)fy0 : 0, y1 = small ? (int)fy1 : 0;
    const int w0 = x0 >> 5, w1 = x1 >> 5;
    const uint32_t m0 = w0 == w1 ? (2u << (x1 & 31)) - (1u << (x0 & 31)) : 0u - (1u << (x0 & 31));
    const uint32_t m1 = w0 == w1 ? 0u : (2u << (x1 & 31)) - 1u;
    // the four words are loaded together (unused ones repeat a used one)
    const uint32_t* r0 = sil + y0 * cams.wpr;
    const uint32_t* r1 = sil + y1 * cams.wpr;
    const uint32_t a00 = r0[w0], a01 = r0[w1], a10 = r1[w0], a11 = r1[w1];
    return small && (a00 & m0) == m0 && (a01 & m1) == m1 && (a10 & m0) == m0 &&
           (a11 & m1) == m1;
}

// One crossing edge per group of kLanesPerEdge lanes; lane `sub` of the group
// owns cameras sub, sub + kLanesPerEdge, ...  Each lane first keeps the ones of
// its cameras that can reject some point of the edge, then every bisection
// step tests the midpoint against those, and a wave ballot ANDs the group.
__global__ __launch_bounds__(kBlock) void bisect_kernel(const fvv_job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ n_jobs_p,
                                                        const uint32_t* __restrict__ point_off,
                                                        const uint8_t* __restrict__ occ_base,
                                                        const CamSet cams,
                                                        const uint32_t* __restrict__ sils,
                                                        int n_steps,
                                                        const uint32_t* __restrict__ keys,
                                                        float* __restrict__ xyz,
                                                        uint32_t max_points) {
    constexpr int kPerLane = (FVV_MAX_CAMS + kLanesPerEdge - 1) / kLanesPerEdge;
    constexpr uint32_t kGroupMask = (1u << kLanesPerEdge) - 1u;
    constexpr uint32_t kEdgesPerBlock = kBlock / kLanesPerEdge;
    const int nj = (int)*n_jobs_p;
    const uint32_t total = point_off[nj];
    const uint32_t E = total < max_points ? total : max_points;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    const int sub = lane_id() % kLanesPerEdge;
    const int shift = lane_id() - sub;
    for (uint32_t base = blockIdx.x * kEdgesPerBlock; base < E; base += gridDim.x * kEdgesPerBlock) {
        const uint32_t e = base + threadIdx.x / kLanesPerEdge;
        const bool act = e < E;
        const uint32_t ee = act ? e : E - 1;
        const int jb = upper_job([&](int m) { return (uint64_t)point_off[m]; }, nj, ee);
        const fvv_grid g = jobs[jb].grid;
        const int64_t out_offset = jobs[jb].out_offset;
        const uint32_t key = keys[ee];
        const uint32_t lin = key / 3u;
        const int axis = (int)(key - 3u * lin);
        const uint32_t i = lin % (uint32_t)g.dims[0];
        const uint32_t r = lin / (uint32_t)g.dims[0];
        const uint32_t j = r % (uint32_t)g.dims[1];
        const uint32_t k = r / (uint32_t)g.dims[1];
        const int gidx[3] = {g.lo[0] + (int)i, g.lo[1] + (int)j, g.lo[2] + (int)k};
        const bool p_on = occ_base[out_offset + lin] != 0;
        const int g_on = gidx[axis] + (p_on ? 0 : 1);
        const float d = p_on ? 1.0f : -1.0f;
        float c[3] = {lattice_coord(gidx[0], g.h, g.origin[0]),
                      lattice_coord(gidx[1], g.h, g.origin[1]),
                      lattice_coord(gidx[2], g.h, g.origin[2])};
        float X0[3] = {c[0], c[1], c[2]}, X1[3] = {c[0], c[1], c[2]};
        X1[axis] = lattice_coord(gidx[axis] + 1, g.h, g.origin[axis]);
        uint32_t mine = 0;   // bit q: camera sub + q*kLanesPerEdge can reject
#pragma unroll
        for (int q = 0; q < kPerLane; ++q) {
            const int cam = sub + q * kLanesPerEdge;
            if (cam < cams.n && !camera_accepts_edge(cams, cam, sils + cam * cam_words, X0, X1))
                mine |= 1u << q;
        }
        float lo = 0.0f, hi = 1.0f;
        for (int s = 0; s < n_steps; ++s) {
            const float m = 0.5f * (lo + hi);
            const float q = (float)g_on + d * m;
            const float ax = __builtin_fmaf(q, g.h, g.origin[axis]);
            const float X = axis == 0 ? ax : c[0];
            const float Y = axis == 1 ? ax : c[1];
            const float Z = axis == 2 ? ax : c[2];
            bool in = true;
            for (uint32_t rest = mine; rest; rest &= rest - 1) {
                const int cam = sub + (__ffs(rest) - 1) * kLanesPerEdge;
                in = in && seen_inside(&cams.P[cam][0], X, Y, Z, sils + cam * cam_words, cams.W,
                                       cams.H, cams.wpr);
            }
            const uint64_t fail = __ballot(!in);
            if ((((uint32_t)(fail >> shift)) & kGroupMask) == 0)
                lo = m;
            else
                hi = m;
        }
        if (act && sub == 0) {
            const float t = 0.5f * (lo + hi);
            const float q = (float)g_on + d * t;
            c[axis] = __builtin_fmaf(q, g.h, g.origin[axis]);
            xyz[3 * (int64_t)e + 0] = c[0];
            xyz[3 * (int64_t)e + 1] = c[1];
            xyz[3 * (int64_t)e + 2] = c[2];
        }
    }
}

hipError_t launch_surface(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                          uint32_t max_jobs, const uint8_t* occ_fine, const CamSet& cams,
                          const uint32_t* sils, int n_steps, uint32_t* keys, float* xyz,
                          uint32_t max_points, uint32_t* point_off, uint32_t* n_points,
                          hipEvent_t edges_done, hipStream_t s) {
    (void)max_jobs;
    const unsigned blocks = (unsigned)(ctx->n_cus * 8);
    hipLaunchKernelGGL(edge_count_kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, ctx->d_prefix,
                       n_jobs_dev, occ_fine, ctx->d_item_cnt);
    hipLaunchKernelGGL(edge_scan_kernel, dim3(1), dim3(1024), 0, s, ctx->d_prefix, n_jobs_dev,
                       ctx->d_item_cnt, ctx->d_item_base, point_off, n_points, max_points,
                       ctx->d_status);
    hipLaunchKernelGGL(edge_write_kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, ctx->d_prefix,
                       n_jobs_dev, occ_fine, ctx->d_item_base, keys, max_points);
    if (edges_done)
        (void)hipEventRecord(edges_done, s);
    hipLaunchKernelGGL(bisect_kernel, dim3(ctx->n_cus * 16), dim3(kBlock), 0, s, jobs, n_jobs_dev,
                       point_off, occ_fine, cams, sils, n_steps, keys, xyz, max_points);
    return hipGetLastError();
}

}  // namespace fvv
