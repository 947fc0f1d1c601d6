// ROI -> fine lattices (Sec. II-B-3), crossing-edge compaction and exit-point
// bisection (Sec. II-C) for gfx950.
//
// Crossing edges: work items are chunks of kEdgeChunk consecutive samples of
// one ROI.  A first pass counts each item's edges, one workgroup scans the
// counts, and a second pass writes keys 3*lin+axis in ascending order: within
// an item a workgroup walks its samples in 8 passes of 256, and a block scan
// of the per-lane counts (0..3 axes each) places every key.  Exit points: one
// edge per lane, n_steps bisection steps, each testing all cameras with the
// same occupancy test as carving.
#include "fvv_internal.h"

namespace fvv {

// ------------------------------------------------------------------ fine jobs of a frame
// One workgroup: map each kept ROI to its fine lattice (integer micrometres,
// one-coarse-cell dilation, clamped to the coarse lattice's extent), lay the
// carried ROIs out back to back in the fine occupancy buffer, and build the
// tile and work-item prefixes of the batched carve and the surface passes.
__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

__device__ __forceinline__ int64_t ceil_div64(int64_t a, int64_t b) { return -floor_div64(-a, b); }

constexpr int64_t kMaxKeyedSamples = 1431655765;  // 3*lin+axis must fit 32 bits

__global__ __launch_bounds__(kBlock) void frame_jobs_kernel(
    const CamSet cams, const fvv_grid coarse, int64_t hc_um, int64_t hf_um, float h_fine,
    const fvv_roi* __restrict__ rois, const uint32_t* __restrict__ n_rois, uint32_t max_rois,
    fvv_job* __restrict__ jobs, int64_t max_fine, uint32_t* __restrict__ counts, int tile_x,
    int tile_z, JobPrefix* __restrict__ pre, uint32_t* __restrict__ counter, uint32_t blocks,
    fvv_camera* __restrict__ dcams, uint32_t* __restrict__ status) {
    __shared__ uint64_t scratch[kBlock / kWave];
    __shared__ uint64_t c_vox, c_tiles, c_items;
    __shared__ uint32_t carried;
    for (int c = threadIdx.x; c < cams.n; c += kBlock) {
        fvv_camera cam;
        for (int e = 0; e < 12; ++e)
            cam.P[e] = cams.P[c][e];
        cam.width = cams.W;
        cam.height = cams.H;
        dcams[c] = cam;
    }
    const uint32_t K_all = *n_rois;
    const uint32_t K = K_all < max_rois ? K_all : max_rois;
    if (threadIdx.x == 0) {
        c_vox = c_tiles = c_items = 0;
        carried = K;
    }
    __syncthreads();
    for (uint32_t base = 0; base < K; base += kBlock) {
        const uint32_t t = base + threadIdx.x;
        fvv_grid fg;
        int64_t V = 0;
        if (t < K) {
            const fvv_roi r = rois[t];
            V = 1;
            for (int a = 0; a < 3; ++a) {
                const int64_t A = (int64_t)coarse.lo[a] + r.lo[a] - 1;
                const int64_t B = (int64_t)coarse.lo[a] + r.hi[a] + 1;
                int64_t f0 = floor_div64(A * hc_um, hf_um);
                int64_t f1 = ceil_div64(B * hc_um, hf_um);
                const int64_t fmin = ceil_div64((int64_t)coarse.lo[a] * hc_um, hf_um);
                const int64_t fmax =
                    floor_div64(((int64_t)coarse.lo[a] + coarse.dims[a] - 1) * hc_um, hf_um);
                f0 = f0 < fmin ? fmin : f0;
                f1 = f1 > fmax ? fmax : f1;
                fg.origin[a] = coarse.origin[a];
                fg.lo[a] = (int32_t)f0;
                fg.dims[a] = (int32_t)(f1 - f0 + 1);
                V *= (f1 - f0 + 1);
            }
            fg.h = h_fine;
        }
        uint64_t tot_v;
        const uint64_t ex_v = block_exclusive_sum64<kBlock>((uint64_t)V, scratch, &tot_v);
        const uint64_t off = c_vox + ex_v;
        const bool fits = t < K && off + (uint64_t)V <= (uint64_t)max_fine && V <= kMaxKeyedSamples &&
                          t < carried;
        const uint64_t tiles = fits ? tiles_of_grid(fg, tile_x, tile_z) : 0;
        const uint64_t items = fits ? ((uint64_t)V + kEdgeChunk - 1) / kEdgeChunk : 0;
        uint64_t tot_t, tot_i;
        const uint64_t ex_t = block_exclusive_sum64<kBlock>(tiles, scratch, &tot_t);
        const uint64_t ex_i = block_exclusive_sum64<kBlock>(items, scratch, &tot_i);
        if (fits) {
            fvv_job j;
            j.grid = fg;
            j.cam_base = 0;
            j.n_cams = cams.n;
            j.width = cams.W;
            j.height = cams.H;
            j.sil_base = 0;
            j.out_offset = (int64_t)off;
            jobs[t] = j;
            pre[t].tile_off = c_tiles + ex_t;
            pre[t].item_off = (uint32_t)(c_items + ex_i);
        }
        // the carried ROIs are the prefix that fits: the first misfit ends it
        if (t < K && !fits)
            atomicMin(&carried, t);
        __syncthreads();
        if (threadIdx.x == 0) {
            c_vox += tot_v;
            c_tiles += tot_t;
            c_items += tot_i;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const uint32_t n = carried;
        // totals over the carried prefix only
        uint64_t vox = 0, tiles = 0, items = 0;
        if (n > 0) {
            const fvv_job& last = jobs[n - 1];
            const uint64_t Vl = (uint64_t)last.grid.dims[0] * last.grid.dims[1] * last.grid.dims[2];
            vox = (uint64_t)last.out_offset + Vl;
            tiles = pre[n - 1].tile_off + tiles_of_grid(last.grid, tile_x, tile_z);
            items = pre[n - 1].item_off + (Vl + kEdgeChunk - 1) / kEdgeChunk;
        }
        pre[n].tile_off = tiles;
        pre[n].item_off = (uint32_t)items;
        counts[0] = K_all;
        counts[1] = (uint32_t)(vox > 0xffffffffull ? 0xffffffffull : vox);
        counts[3] = n;
        const uint64_t per = (tiles + (uint64_t)blocks * 8 - 1) / ((uint64_t)blocks * 8);
        counter[0] = 0;
        counter[1] = (uint32_t)(per < 1 ? 1 : per);
        counter[2] = n;
        if (n < K_all)
            atomicOr(status, kFlagCapacity);
    }
}

hipError_t launch_frame_jobs(fvv_ctx* ctx, const CamSet& cams, const fvv_grid& coarse,
                             int64_t hc_um, int64_t hf_um, float h_fine, const fvv_roi* rois,
                             const uint32_t* n_rois, uint32_t max_rois, fvv_job* jobs,
                             int64_t max_fine, uint32_t* counts, TileShape fine_tile, int blocks,
                             hipStream_t s) {
    hipLaunchKernelGGL(frame_jobs_kernel, dim3(1), dim3(kBlock), 0, s, cams, coarse, hc_um, hf_um,
                       h_fine, rois, n_rois, max_rois, jobs, max_fine, counts, fine_tile.tx,
                       fine_tile.tz, ctx->d_prefix, ctx->d_counter, (uint32_t)blocks, ctx->d_cams,
                       ctx->d_status);
    return hipGetLastError();
}

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
// Bits 0..2: the edges along x, y, z from sample lin of a dims lattice.
__device__ __forceinline__ uint32_t crossing_bits(const uint8_t* __restrict__ occ, uint32_t lin,
                                                  int dx, int dy, int dz) {
    const uint32_t i = lin % (uint32_t)dx;
    const uint32_t r = lin / (uint32_t)dx;
    const uint32_t j = r % (uint32_t)dy;
    const uint32_t k = r / (uint32_t)dy;
    const bool o = occ[lin] != 0;
    uint32_t bits = 0;
    if (i + 1 < (uint32_t)dx && (occ[lin + 1] != 0) != o)
        bits |= 1u;
    if (j + 1 < (uint32_t)dy && (occ[lin + dx] != 0) != o)
        bits |= 2u;
    if (k + 1 < (uint32_t)dz && (occ[lin + (uint32_t)dx * dy] != 0) != o)
        bits |= 4u;
    return bits;
}

struct ItemRef {
    int job;
    uint32_t lin0;
};

__device__ __forceinline__ ItemRef locate_item(const JobPrefix* __restrict__ pre, int nj,
                                               uint32_t item) {
    const int jb = upper_job([&](int m) { return (uint64_t)pre[m].item_off; }, nj, item);
    return {jb, (item - pre[jb].item_off) * (uint32_t)kEdgeChunk};
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
        const uint8_t* occ = occ_base + job.out_offset;
        uint32_t cnt = 0;
        for (int it = 0; it < kEdgeChunk / kBlock; ++it) {
            const uint32_t lin = ref.lin0 + it * kBlock + threadIdx.x;
            if (lin < V)
                cnt += __popc(crossing_bits(occ, lin, job.grid.dims[0], job.grid.dims[1],
                                            job.grid.dims[2]));
        }
        uint32_t total;
        block_exclusive_sum<kBlock>(cnt, scratch, &total);
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
        const uint8_t* occ = occ_base + job.out_offset;
        uint32_t running = item_base[item];
        for (int it = 0; it < kEdgeChunk / kBlock; ++it) {
            const uint32_t lin = ref.lin0 + it * kBlock + threadIdx.x;
            const uint32_t bits = lin < V ? crossing_bits(occ, lin, job.grid.dims[0],
                                                          job.grid.dims[1], job.grid.dims[2])
                                          : 0u;
            uint32_t total;
            uint32_t pos = running + block_exclusive_sum<kBlock>(__popc(bits), scratch, &total);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (bits & (1u << a)) {
                    if (pos < max_points)
                        keys[pos] = 3u * lin + (uint32_t)a;
                    ++pos;
                }
            }
            running += total;
        }
    }
}

// ------------------------------------------------------------------ exit points
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
    const int nj = (int)*n_jobs_p;
    const uint32_t total = point_off[nj];
    const uint32_t E = total < max_points ? total : max_points;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < E; e += gridDim.x * kBlock) {
        const int jb = upper_job([&](int m) { return (uint64_t)point_off[m]; }, nj, e);
        const fvv_job& job = jobs[jb];
        const fvv_grid g = job.grid;
        const uint32_t key = keys[e];
        const uint32_t lin = key / 3u;
        const int axis = (int)(key - 3u * lin);
        const uint32_t i = lin % (uint32_t)g.dims[0];
        const uint32_t r = lin / (uint32_t)g.dims[0];
        const uint32_t j = r % (uint32_t)g.dims[1];
        const uint32_t k = r / (uint32_t)g.dims[1];
        const int gidx[3] = {g.lo[0] + (int)i, g.lo[1] + (int)j, g.lo[2] + (int)k};
        const bool p_on = occ_base[job.out_offset + lin] != 0;
        const int g_on = gidx[axis] + (p_on ? 0 : 1);
        const float d = p_on ? 1.0f : -1.0f;
        float c[3] = {lattice_coord(gidx[0], g.h, g.origin[0]),
                      lattice_coord(gidx[1], g.h, g.origin[1]),
                      lattice_coord(gidx[2], g.h, g.origin[2])};
        float lo = 0.0f, hi = 1.0f;
        for (int s = 0; s < n_steps; ++s) {
            const float m = 0.5f * (lo + hi);
            const float q = (float)g_on + d * m;
            const float ax = __builtin_fmaf(q, g.h, g.origin[axis]);
            const float X = axis == 0 ? ax : c[0];
            const float Y = axis == 1 ? ax : c[1];
            const float Z = axis == 2 ? ax : c[2];
            bool in = true;
            for (int cam = 0; cam < cams.n && in; ++cam)
                in = seen_inside(&cams.P[cam][0], X, Y, Z, sils + cam * cam_words, cams.W, cams.H,
                                 cams.wpr);
            if (in)
                lo = m;
            else
                hi = m;
        }
        const float t = 0.5f * (lo + hi);
        const float q = (float)g_on + d * t;
        c[axis] = __builtin_fmaf(q, g.h, g.origin[axis]);
        xyz[3 * (int64_t)e + 0] = c[0];
        xyz[3 * (int64_t)e + 1] = c[1];
        xyz[3 * (int64_t)e + 2] = c[2];
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
    hipLaunchKernelGGL(bisect_kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, n_jobs_dev,
                       point_off, occ_fine, cams, sils, n_steps, keys, xyz, max_points);
    return hipGetLastError();
}

}  // namespace fvv
