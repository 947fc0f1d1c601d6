// Internal declarations of the gfx950 visual-hull library: device helpers
// shared by the kernels, the context layout and the launch functions each
// kernel file provides to the C ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvv.h"

namespace fvv {

constexpr int kWave = 64;
constexpr int kBlock = 256;              // threads per workgroup everywhere
constexpr int kEdgeChunk = 2048;         // fine samples per crossing-edge work item
constexpr int kRootChunk = 16384;        // coarse samples per root-numbering block
constexpr uint32_t kFlagCapacity = 1u;   // sticky device status bits

// Projections of a camera rig passed by value in the kernel arguments.
struct CamSet {
    float P[FVV_MAX_CAMS][12];
    int32_t n, W, H, wpr;
};

// Tile of the carving kernels: TX*TY == 256 threads, TZ samples per thread.
struct TileShape {
    int tx, ty, tz;
};

// ------------------------------------------------------------------ pixel test
// Index of the pixel holding the image coordinate a/w along an axis of `dim`
// pixels, or -1 when outside [0, dim).  Requires w > 0 and finite a, w.
// q = a * rcp(w) is within a few ulp of the real quotient, so floor(q) is the
// exact floor or off by one; the sign of the residual a - n*w, which a single
// fma rounds without changing, decides which.  The result is the floor of the
// real quotient whatever the rounding of q.  The IEEE division serves the
// (never seen) w below 2^-64, where rcp could overflow.
__device__ __forceinline__ int pixel_index(float a, float w, int dim) {
    float q = (w >= 0x1p-64f) ? a * __builtin_amdgcn_rcpf(w) : a / w;
    int n = (int)__builtin_floorf(q);
    float nf = (float)n;
    if (__builtin_fmaf(-nf, w, a) < 0.0f)
        n -= 1;
    else if (__builtin_fmaf(-(nf + 1.0f), w, a) >= 0.0f)
        n += 1;
    return ((unsigned)n < (unsigned)dim) ? n : -1;
}

// World coordinate of global lattice index g on one axis.
__device__ __forceinline__ float lattice_coord(int g, float h, float o) {
    return __builtin_fmaf((float)g, h, o);
}

// Test of one sample against camera P (12 floats): 1 if it projects into a
// foreground pixel of `sil` (this camera's [H][wpr] rows), else 0.
__device__ __forceinline__ bool seen_inside(const float* __restrict__ P, float X, float Y, float Z,
                                            const uint32_t* __restrict__ sil, int W, int H,
                                            int wpr) {
    float a = __builtin_fmaf(P[2], Z, __builtin_fmaf(P[1], Y, __builtin_fmaf(P[0], X, P[3])));
    float b = __builtin_fmaf(P[6], Z, __builtin_fmaf(P[5], Y, __builtin_fmaf(P[4], X, P[7])));
    float w = __builtin_fmaf(P[10], Z, __builtin_fmaf(P[9], Y, __builtin_fmaf(P[8], X, P[11])));
    if (!(w > 0.0f))
        return false;
    int px = pixel_index(a, w, W);
    int py = pixel_index(b, w, H);
    if ((px | py) < 0)
        return false;
    uint32_t word = sil[py * wpr + (px >> 5)];
    return (word >> (px & 31)) & 1u;
}

// ------------------------------------------------------------------ wave/block helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below_mask() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum over a wave.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t u = __shfl_up(v, d, kWave);
        if (lane_id() >= d)
            v += u;
    }
    return v;
}

// Exclusive prefix sum over a 256- or 1024-thread block; *total = block sum.
// `scratch` holds one uint32 per wave.  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* scratch,
                                                        uint32_t* total) {
    constexpr int NW = NT / kWave;
    uint32_t inc = wave_inclusive_sum(v);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1)
        scratch[w] = inc;
    __syncthreads();
    uint32_t base = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint32_t s = scratch[i];
        base += (i < w) ? s : 0u;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

__device__ __forceinline__ uint64_t wave_inclusive_sum64(uint64_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t u = __shfl_up((unsigned long long)v, d, kWave);
        if (lane_id() >= d)
            v += u;
    }
    return v;
}

template <int NT>
__device__ __forceinline__ uint64_t block_exclusive_sum64(uint64_t v, uint64_t* scratch,
                                                          uint64_t* total) {
    constexpr int NW = NT / kWave;
    uint64_t inc = wave_inclusive_sum64(v);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1)
        scratch[w] = inc;
    __syncthreads();
    uint64_t base = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint64_t s = scratch[i];
        base += (i < w) ? s : 0ull;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v = min(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

// Carving tiles of lattice g for a TX x (256/TX) x TZ tile.
__host__ __device__ inline uint64_t tiles_of_grid(const fvv_grid& g, int tx, int tz) {
    const int ty = kBlock / tx;
    return (uint64_t)((g.dims[0] + tx - 1) / tx) * (uint64_t)((g.dims[1] + ty - 1) / ty) *
           (uint64_t)((g.dims[2] + tz - 1) / tz);
}

// ------------------------------------------------------------------ device-side job prefix data
// Per job of a batched carve / surface: first carving tile and first
// crossing-edge work item (exclusive prefix sums over the job table).
struct JobPrefix {
    uint64_t tile_off;   // first tile of the job
    uint32_t item_off;   // first crossing-edge work item of the job
    uint32_t pad;
};

// Largest j in [0, n) with off(j) <= x, for ascending offsets (binary search).
template <typename F>
__device__ __forceinline__ int upper_job(F off, int n, uint64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off(mid) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

}  // namespace fvv

// ------------------------------------------------------------------ context
struct fvv_ctx {
    fvv_limits lim;
    int device;
    // status and counters
    uint32_t* d_status;          // sticky flags
    uint32_t* d_counter;         // persistent-kernel work counter [0] and grab size [1]
    // labelling
    int32_t* d_parent;           // union-find forest over coarse samples
    int32_t* d_rid;              // root number of each root sample
    uint64_t* d_rootbits;        // root flags, one bit per sample
    uint32_t* d_blk_cnt;         // roots per numbering block
    uint32_t* d_n_roots;         // number of components
    int32_t* d_stats;            // per root: count, lo[3], hi[3], root index
    int32_t* d_keep;             // per root: final label or 0
    int64_t root_cap;
    // batched carve / frame
    fvv::JobPrefix* d_prefix;    // per job (max(max_jobs, max_rois) + 1)
    fvv_job* d_job_single;       // the job of a single-ROI fvv_surface call
    fvv_camera* d_cams;          // camera table of fvv_frame
    uint32_t* d_item_cnt;        // crossing edges per work item
    uint32_t* d_item_base;       // first edge of each work item
    uint32_t* d_point_off_single;
    uint32_t* d_counts_single;
    int64_t item_cap;
    int64_t job_cap;
    int n_cus;
};

namespace fvv {

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_pack(int n, int W, int H, const uint8_t* masks, uint32_t* sils, hipStream_t s);
hipError_t launch_carve(const CamSet& cams, const uint32_t* sils, const fvv_grid& g,
                        TileShape t, uint8_t* occ, hipStream_t s);
hipError_t launch_carve_batched(fvv_ctx* ctx, const fvv_job* jobs, uint32_t n_jobs,
                                const fvv_camera* cams, const uint32_t* sils, uint8_t* out,
                                TileShape t, int blocks, bool jobs_prepared, hipStream_t s);
hipError_t launch_label(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                        uint32_t t_np, uint32_t t_nb, fvv_roi* rois, uint32_t max_rois,
                        uint32_t* n_rois, hipStream_t s);
hipError_t launch_frame_jobs(fvv_ctx* ctx, const CamSet& cams, const fvv_grid& coarse,
                             int64_t hc_um, int64_t hf_um, float h_fine, const fvv_roi* rois,
                             const uint32_t* n_rois, uint32_t max_rois, fvv_job* jobs,
                             int64_t max_fine, uint32_t* counts, TileShape fine_tile, int blocks,
                             hipStream_t s);
hipError_t launch_surface(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                          uint32_t max_jobs, const uint8_t* occ_fine, const CamSet& cams,
                          const uint32_t* sils, int n_steps, uint32_t* keys, float* xyz,
                          uint32_t max_points, uint32_t* point_off, uint32_t* n_points,
                          hipEvent_t edges_done, hipStream_t s);
hipError_t launch_surface_prepare_single(fvv_ctx* ctx, const fvv_job& job, hipStream_t s);

}  // namespace fvv
