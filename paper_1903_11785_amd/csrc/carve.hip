// Silhouette packing and volumetric visual-hull carving (Sec. II-B-1 over the
// whole volume, Sec. II-B-3 inside ROIs) for gfx950.
//
// Carving is one sample per lane: a workgroup of 256 threads owns a tile of
// TX x TY x TZ samples, TX consecutive x-samples per row so each wave writes
// contiguous occupancy bytes, and each thread carries TZ samples stacked in z.
// The two inner fma terms of each projection row (P0*X + P3, then + P1*Y) do
// not depend on z, so they are computed once per thread and camera; the same
// fused chain in the same order as a per-sample evaluation, hence bit-equal.
// Cameras are tested in index order and a wave stops as soon as none of its
// samples is still inside every camera tested so far.
#include "fvv_internal.h"

namespace fvv {

// ------------------------------------------------------------------ packing
// One lane per 32-pixel word.  Fast path: rows of a multiple of 32 pixels
// whose 32 bytes per word are read with two 16-byte loads.
__global__ __launch_bounds__(kBlock) void pack_kernel(const uint8_t* __restrict__ masks,
                                                      uint32_t* __restrict__ sils, int n, int W,
                                                      int H, int wpr) {
    const int64_t total = (int64_t)n * H * wpr;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t row = idx / wpr;
        int word = (int)(idx - row * wpr);
        const uint8_t* src = masks + row * W + (int64_t)word * 32;
        uint32_t bits = 0;
        if ((W & 31) == 0) {
            const uint4* v = reinterpret_cast<const uint4*>(src);
            uint4 q[2] = {v[0], v[1]};
            const uint32_t* d = reinterpret_cast<const uint32_t*>(q);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                uint32_t x = d[k];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bits |= (uint32_t)(((x >> (8 * b)) & 0xffu) != 0u) << (4 * k + b);
            }
        } else {
            int nb = min(32, W - word * 32);
            for (int b = 0; b < nb; ++b)
                bits |= (uint32_t)(src[b] != 0) << b;
        }
        sils[idx] = bits;
    }
}

hipError_t launch_pack(int n, int W, int H, const uint8_t* masks, uint32_t* sils, hipStream_t s) {
    int wpr = (W + 31) / 32;
    int64_t total = (int64_t)n * H * wpr;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, masks, sils, n, W,
                       H, wpr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ carving tile
// Carve tile `tile` of lattice g.  getP(c) returns camera c's 12 floats (a
// wave-uniform address); sil_of(c) its silhouette rows.
template <int TX, int TZ, typename GetP, typename GetSil>
__device__ __forceinline__ void carve_tile(GetP getP, GetSil sil_of, int ncam, int W, int H,
                                           int wpr, const fvv_grid& g, uint64_t tile,
                                           uint8_t* __restrict__ out) {
    constexpr int TY = kBlock / TX;
    const int ntx = (g.dims[0] + TX - 1) / TX;
    const int nty = (g.dims[1] + TY - 1) / TY;
    const int bx = (int)(tile % (uint64_t)ntx);
    const uint64_t r = tile / (uint64_t)ntx;
    const int by = (int)(r % (uint64_t)nty);
    const int bz = (int)(r / (uint64_t)nty);
    const int i = bx * TX + (int)(threadIdx.x % TX);
    const int j = by * TY + (int)(threadIdx.x / TX);
    const int k0 = bz * TZ;
    const bool in_xy = i < g.dims[0] && j < g.dims[1];

    const float X = lattice_coord(g.lo[0] + i, g.h, g.origin[0]);
    const float Y = lattice_coord(g.lo[1] + j, g.h, g.origin[1]);
    float Z[TZ];
    uint32_t alive = 0;
#pragma unroll
    for (int z = 0; z < TZ; ++z) {
        Z[z] = lattice_coord(g.lo[2] + k0 + z, g.h, g.origin[2]);
        if (in_xy && k0 + z < g.dims[2])
            alive |= 1u << z;
    }

    for (int c = 0; c < ncam; ++c) {
        if (__ballot(alive != 0) == 0)
            break;
        const float* __restrict__ P = getP(c);
        const float p0 = P[0], p1 = P[1], p2 = P[2], p3 = P[3];
        const float p4 = P[4], p5 = P[5], p6 = P[6], p7 = P[7];
        const float p8 = P[8], p9 = P[9], p10 = P[10], p11 = P[11];
        const float ba = __builtin_fmaf(p1, Y, __builtin_fmaf(p0, X, p3));
        const float bb = __builtin_fmaf(p5, Y, __builtin_fmaf(p4, X, p7));
        const float bw = __builtin_fmaf(p9, Y, __builtin_fmaf(p8, X, p11));
        const uint32_t* __restrict__ sil = sil_of(c);
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
            if (alive & (1u << z)) {
                const float a = __builtin_fmaf(p2, Z[z], ba);
                const float b = __builtin_fmaf(p6, Z[z], bb);
                const float w = __builtin_fmaf(p10, Z[z], bw);
                bool ok = w > 0.0f;
                const int px = pixel_index(a, w, W);
                const int py = pixel_index(b, w, H);
                ok = ok && (px | py) >= 0;
                const uint32_t word = sil[ok ? py * wpr + (px >> 5) : 0];
                ok = ok && ((word >> (px & 31)) & 1u);
                if (!ok)
                    alive &= ~(1u << z);
            }
        }
    }

    if (in_xy) {
        const uint64_t plane = (uint64_t)g.dims[0] * (uint64_t)g.dims[1];
        uint8_t* o = out + (uint64_t)j * g.dims[0] + i;
#pragma unroll
        for (int z = 0; z < TZ; ++z)
            if (k0 + z < g.dims[2])
                o[(uint64_t)(k0 + z) * plane] = (uint8_t)((alive >> z) & 1u);
    }
}

template <int TX, int TZ>
__device__ __forceinline__ uint64_t tiles_of(const fvv_grid& g) {
    constexpr int TY = kBlock / TX;
    return (uint64_t)((g.dims[0] + TX - 1) / TX) * (uint64_t)((g.dims[1] + TY - 1) / TY) *
           (uint64_t)((g.dims[2] + TZ - 1) / TZ);
}

// ------------------------------------------------------------------ one lattice
template <int TX, int TZ>
__global__ __launch_bounds__(kBlock) void carve_kernel(const CamSet cams,
                                                       const uint32_t* __restrict__ sils,
                                                       const fvv_grid g, uint8_t* __restrict__ occ) {
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    carve_tile<TX, TZ>([&](int c) { return &cams.P[c][0]; },
                       [&](int c) { return sils + c * cam_words; }, cams.n, cams.W, cams.H,
                       cams.wpr, g, blockIdx.x, occ);
}

// ------------------------------------------------------------------ batched, persistent
// Prefix sums of tile counts over a host-given job table; resets the work
// counter.  counter[0] = next work item, [1] = tiles per item, [2] = jobs.
template <int TX, int TZ>
__global__ __launch_bounds__(kBlock) void batched_prepare_kernel(const fvv_job* __restrict__ jobs,
                                                                 uint32_t n_jobs,
                                                                 JobPrefix* __restrict__ pre,
                                                                 uint32_t* __restrict__ counter,
                                                                 uint32_t blocks) {
    __shared__ uint64_t scratch[kBlock / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n_jobs; base += kBlock) {
        uint32_t j = base + threadIdx.x;
        uint64_t t = j < n_jobs ? tiles_of<TX, TZ>(jobs[j].grid) : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_sum64<kBlock>(t, scratch, &tot);
        uint64_t c0 = carry;
        if (j < n_jobs)
            pre[j].tile_off = c0 + ex;
        __syncthreads();
        if (threadIdx.x == 0)
            carry = c0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t total = carry;
        pre[n_jobs].tile_off = total;
        uint64_t per = (total + (uint64_t)blocks * 8 - 1) / ((uint64_t)blocks * 8);
        counter[0] = 0;
        counter[1] = (uint32_t)(per < 1 ? 1 : per);
        counter[2] = n_jobs;
    }
}

template <int TX, int TZ>
__global__ __launch_bounds__(kBlock) void carve_persistent_kernel(
    const fvv_job* __restrict__ jobs, const JobPrefix* __restrict__ pre,
    uint32_t* __restrict__ counter, const fvv_camera* __restrict__ cams,
    const uint32_t* __restrict__ sils, uint8_t* __restrict__ out) {
    __shared__ uint32_t s_item;
    const uint32_t nj = counter[2];
    const uint64_t per = counter[1];
    const uint64_t total = pre[nj].tile_off;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = atomicAdd(&counter[0], 1u);
        __syncthreads();
        const uint64_t t0 = (uint64_t)s_item * per;
        __syncthreads();
        if (t0 >= total)
            break;
        const uint64_t t1 = t0 + per < total ? t0 + per : total;
        for (uint64_t t = t0; t < t1; ++t) {
            const int jb = upper_job([&](int m) { return pre[m].tile_off; }, (int)nj, t);
            const fvv_job job = jobs[jb];
            const int wpr = (job.width + 31) / 32;
            const int64_t cam_words = (int64_t)job.height * wpr;
            const fvv_camera* jc = cams + job.cam_base;
            const uint32_t* js = sils + job.sil_base;
            carve_tile<TX, TZ>([&](int c) { return &jc[c].P[0]; },
                               [&](int c) { return js + c * cam_words; }, job.n_cams, job.width,
                               job.height, wpr, job.grid, t - pre[jb].tile_off,
                               out + job.out_offset);
        }
    }
}

// ------------------------------------------------------------------ dispatch
#define FVV_TILE_CASES(X)                                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(32, 1) X(32, 2) X(32, 4) X(32, 8) X(16, 1)     \
    X(16, 2) X(16, 4) X(16, 8)

static inline uint64_t host_tiles(const fvv_grid& g, TileShape t) {
    return (uint64_t)((g.dims[0] + t.tx - 1) / t.tx) * (uint64_t)((g.dims[1] + t.ty - 1) / t.ty) *
           (uint64_t)((g.dims[2] + t.tz - 1) / t.tz);
}

hipError_t launch_carve(const CamSet& cams, const uint32_t* sils, const fvv_grid& g, TileShape t,
                        uint8_t* occ, hipStream_t s) {
    uint64_t tiles = host_tiles(g, t);
    if (tiles == 0)
        return hipSuccess;
    if (tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
#define X(TXV, TZV)                                                                           \
    if (t.tx == TXV && t.tz == TZV) {                                                         \
        hipLaunchKernelGGL((carve_kernel<TXV, TZV>), dim3((unsigned)tiles), dim3(kBlock), 0, s, \
                           cams, sils, g, occ);                                               \
        return hipGetLastError();                                                             \
    }
    FVV_TILE_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_carve_batched(fvv_ctx* ctx, const fvv_job* jobs, uint32_t n_jobs,
                                const fvv_camera* cams, const uint32_t* sils, uint8_t* out,
                                TileShape t, int blocks, bool jobs_prepared, hipStream_t s) {
#define X(TXV, TZV)                                                                            \
    if (t.tx == TXV && t.tz == TZV) {                                                          \
        if (!jobs_prepared)                                                                    \
            hipLaunchKernelGGL((batched_prepare_kernel<TXV, TZV>), dim3(1), dim3(kBlock), 0, s, \
                               jobs, n_jobs, ctx->d_prefix, ctx->d_counter, (uint32_t)blocks);  \
        hipLaunchKernelGGL((carve_persistent_kernel<TXV, TZV>), dim3(blocks), dim3(kBlock), 0, \
                           s, jobs, ctx->d_prefix, ctx->d_counter, cams, sils, out);           \
        return hipGetLastError();                                                              \
    }
    FVV_TILE_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace fvv
