// Connected components of the coarse occupancy, size filter and ROI boxes
// (Sec. II-B-2) for gfx950.
//
// The paper splits the volume into blocks labelled locally and then globally,
// with 26-adjacency in both stages.  Here:
//   local    one workgroup per 16x4x4 block: union-find in LDS over each
//            sample's 13 earlier neighbours inside the block;
//   merge    samples on block faces unite with their earlier neighbours in
//            other blocks (global union-find, atomicMin links);
//   flatten  every sample points straight at its root; root flags are
//            gathered with wave ballots into a bitmap;
//   number   roots are numbered in ascending linear order (per-block counts,
//            then a block scan) -- the canonical label order;
//   stats    count and bounding box per root, aggregated per wave before
//            the atomics;
//   filter   one workgroup applies T_np <= N(S) <= T_nb and numbers the kept
//            components 1..K in root order, writing the ROI table;
//   write    labels and the filtered occupancy.
// Links always hang the larger root under the smaller, so every root is the
// smallest linear index of its component whatever the interleaving of the
// atomics: labels and boxes are identical from run to run.
#include "fvv_internal.h"

namespace fvv {

constexpr int BX = 16, BY = 4, BZ = 4;

// ------------------------------------------------------------------ union-find
__device__ __forceinline__ int32_t find_root(volatile int32_t* P, int32_t x) {
    int32_t p = P[x];
    while (p != x) {
        x = p;
        p = P[x];
    }
    return x;
}

// Unite the trees of a and b: the larger root is linked under the smaller
// with atomicMin; if that root was linked meanwhile, retry from its new parent.
__device__ __forceinline__ void unite(int32_t* P, int32_t a, int32_t b) {
    for (;;) {
        a = find_root(P, a);
        b = find_root(P, b);
        if (a == b)
            return;
        if (a < b) {
            int32_t old = atomicMin(&P[b], a);
            if (old == b)
                return;
            b = old;
        } else {
            int32_t old = atomicMin(&P[a], b);
            if (old == a)
                return;
            a = old;
        }
    }
}

// The 13 neighbours that precede a sample in raster order (dz = -1: 9, dz = 0,
// dy = -1: 3, dz = 0, dy = 0, dx = -1: 1).
__device__ __forceinline__ void earlier_neighbour(int n, int& dx, int& dy, int& dz) {
    if (n < 9) {
        dz = -1;
        dy = n / 3 - 1;
        dx = n % 3 - 1;
    } else if (n < 12) {
        dz = 0;
        dy = -1;
        dx = n - 10;
    } else {
        dz = 0;
        dy = 0;
        dx = -1;
    }
}

__global__ __launch_bounds__(kBlock) void ccl_local_kernel(const uint8_t* __restrict__ occ,
                                                           int32_t* __restrict__ parent, int nx,
                                                           int ny, int nz) {
    __shared__ int32_t L[BX * BY * BZ];
    const int t = threadIdx.x;
    const int lx = t % BX, ly = (t / BX) % BY, lz = t / (BX * BY);
    const int x = blockIdx.x * BX + lx, y = blockIdx.y * BY + ly, z = blockIdx.z * BZ + lz;
    const bool in = x < nx && y < ny && z < nz;
    const int32_t gi = in ? x + nx * (y + ny * z) : 0;
    const bool on = in && occ[gi] != 0;
    L[t] = on ? t : -1;
    if (__syncthreads_or(on) == 0) {
        if (in)
            parent[gi] = -1;
        return;
    }
    if (on) {
        for (int n = 0; n < 13; ++n) {
            int dx, dy, dz;
            earlier_neighbour(n, dx, dy, dz);
            const int ax = lx + dx, ay = ly + dy, az = lz + dz;
            if (ax < 0 || ax >= BX || ay < 0 || ay >= BY || az < 0)
                continue;
            const int nt = ax + BX * (ay + BY * az);
            if (L[nt] >= 0)
                unite(L, t, nt);
        }
    }
    __syncthreads();
    if (on) {
        const int r = find_root(L, t);
        const int rx = blockIdx.x * BX + r % BX;
        const int ry = blockIdx.y * BY + (r / BX) % BY;
        const int rz = blockIdx.z * BZ + r / (BX * BY);
        parent[gi] = rx + nx * (ry + ny * rz);
    } else if (in) {
        parent[gi] = -1;
    }
}

__global__ __launch_bounds__(kBlock) void ccl_merge_kernel(int32_t* __restrict__ parent, int nx,
                                                           int ny, int nz) {
    const int t = threadIdx.x;
    const int lx = t % BX, ly = (t / BX) % BY, lz = t / (BX * BY);
    const int x = blockIdx.x * BX + lx, y = blockIdx.y * BY + ly, z = blockIdx.z * BZ + lz;
    if (x >= nx || y >= ny || z >= nz)
        return;
    if (lx != 0 && lx != BX - 1 && ly != 0 && ly != BY - 1 && lz != 0)
        return;  // every earlier neighbour is in the same block
    const int32_t gi = x + nx * (y + ny * z);
    if (parent[gi] < 0)
        return;
    for (int n = 0; n < 13; ++n) {
        int dx, dy, dz;
        earlier_neighbour(n, dx, dy, dz);
        const int ax = x + dx, ay = y + dy, az = z + dz;
        if (ax < 0 || ax >= nx || ay < 0 || ay >= ny || az < 0)
            continue;
        if (ax / BX == (int)blockIdx.x && ay / BY == (int)blockIdx.y && az / BZ == (int)blockIdx.z)
            continue;
        const int32_t ni = ax + nx * (ay + ny * az);
        if (parent[ni] >= 0)
            unite(parent, gi, ni);
    }
}

// Point every sample at its root; root bitmap; roots per kRootChunk block.
__global__ __launch_bounds__(kBlock) void ccl_flatten_kernel(int32_t* __restrict__ parent,
                                                             int32_t V,
                                                             uint64_t* __restrict__ rootbits,
                                                             uint32_t* __restrict__ blk_cnt) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kRootChunk;
    uint32_t cnt = 0;
    for (int it = 0; it < kRootChunk / kBlock; ++it) {
        const int64_t v = base + (int64_t)it * kBlock + threadIdx.x;
        bool root = false;
        if (v < V) {
            const int32_t p = parent[v];
            if (p >= 0) {
                const int32_t r = find_root(parent, (int32_t)v);
                if (r != p)
                    parent[v] = r;
                root = (r == (int32_t)v);
            }
        }
        const uint64_t m = __ballot(root);
        if (lane_id() == 0) {
            rootbits[(base + (int64_t)it * kBlock) / kWave + threadIdx.x / kWave] = m;
            cnt += (uint32_t)__popcll(m);
        }
    }
    if (lane_id() == 0)
        wsum[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kBlock / kWave; ++w)
            s += wsum[w];
        blk_cnt[blockIdx.x] = s;
    }
}

// Number the roots in ascending linear order: root number = roots in earlier
// blocks + roots earlier in this block.  Initialises each root's stats row.
__global__ __launch_bounds__(kBlock) void ccl_number_kernel(const uint64_t* __restrict__ rootbits,
                                                            const uint32_t* __restrict__ blk_cnt,
                                                            int32_t* __restrict__ rid,
                                                            int32_t* __restrict__ stats,
                                                            uint32_t* __restrict__ n_roots) {
    __shared__ uint32_t scratch[kBlock / kWave];
    uint32_t part = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kBlock)
        part += blk_cnt[i];
    uint32_t base;
    block_exclusive_sum<kBlock>(part, scratch, &base);
    uint64_t m = rootbits[(int64_t)blockIdx.x * (kRootChunk / kWave) + threadIdx.x];
    uint32_t total;
    uint32_t id = base + block_exclusive_sum<kBlock>((uint32_t)__popcll(m), scratch, &total);
    while (m) {
        const int bit = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int32_t v = (int32_t)((int64_t)blockIdx.x * kRootChunk + threadIdx.x * kWave + bit);
        rid[v] = (int32_t)id;
        int32_t* s = stats + 8 * (int64_t)id;
        s[0] = 0;
        s[1] = s[2] = s[3] = 0x7fffffff;
        s[4] = s[5] = s[6] = -1;
        s[7] = v;
        ++id;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *n_roots = base + total;
}

// Count and bounding box per component, one set of atomics per (wave, root).
__global__ __launch_bounds__(kBlock) void ccl_stats_kernel(const int32_t* __restrict__ parent,
                                                           const int32_t* __restrict__ rid,
                                                           int32_t* __restrict__ stats, int nx,
                                                           int ny, int32_t V) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t p = v < V ? parent[v] : -1;
    const bool on = p >= 0;
    const int32_t id = on ? rid[p] : -1;
    const uint32_t uv = (uint32_t)v;
    const int i = (int)(uv % (uint32_t)nx);
    const int j = (int)((uv / (uint32_t)nx) % (uint32_t)ny);
    const int k = (int)(uv / ((uint32_t)nx * (uint32_t)ny));
    uint64_t pending = __ballot(on);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lid = __shfl(id, leader, kWave);
        const bool mine = on && id == lid;
        const uint64_t mm = __ballot(mine);
        const int lo_i = wave_min(mine ? i : 0x7fffffff);
        const int lo_j = wave_min(mine ? j : 0x7fffffff);
        const int lo_k = wave_min(mine ? k : 0x7fffffff);
        const int hi_i = wave_max(mine ? i : -1);
        const int hi_j = wave_max(mine ? j : -1);
        const int hi_k = wave_max(mine ? k : -1);
        if (lane_id() == leader) {
            int32_t* s = stats + 8 * (int64_t)lid;
            atomicAdd(&s[0], (int32_t)__popcll(mm));
            atomicMin(&s[1], lo_i);
            atomicMin(&s[2], lo_j);
            atomicMin(&s[3], lo_k);
            atomicMax(&s[4], hi_i);
            atomicMax(&s[5], hi_j);
            atomicMax(&s[6], hi_k);
        }
        pending &= ~mm;
    }
}

// Eq. (1) filter and canonical numbering, in one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void ccl_filter_kernel(const int32_t* __restrict__ stats,
                                                          const uint32_t* __restrict__ n_roots,
                                                          int32_t* __restrict__ keep,
                                                          uint32_t t_np, uint32_t t_nb,
                                                          fvv_roi* __restrict__ rois,
                                                          uint32_t max_rois,
                                                          uint32_t* __restrict__ n_rois,
                                                          uint32_t* __restrict__ status) {
    __shared__ uint32_t scratch[1024 / kWave];
    const uint32_t n = *n_roots;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t id = base + threadIdx.x;
        bool kept = false;
        uint32_t cnt = 0;
        if (id < n) {
            cnt = (uint32_t)stats[8 * (int64_t)id];
            kept = t_np <= cnt && cnt <= t_nb;
        }
        uint32_t total;
        const uint32_t ex = block_exclusive_sum<1024>(kept ? 1u : 0u, scratch, &total);
        const uint32_t label = carry + ex + 1;
        if (id < n)
            keep[id] = kept ? (int32_t)label : 0;
        if (kept && label <= max_rois) {
            const int32_t* s = stats + 8 * (int64_t)id;
            fvv_roi r;
            r.lo[0] = s[1];
            r.lo[1] = s[2];
            r.lo[2] = s[3];
            r.hi[0] = s[4];
            r.hi[1] = s[5];
            r.hi[2] = s[6];
            r.count = cnt;
            r.min_index = (uint32_t)s[7];
            rois[label - 1] = r;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        *n_rois = carry;
        if (carry > max_rois)
            atomicOr(status, kFlagCapacity);
    }
}

__global__ __launch_bounds__(kBlock) void ccl_write_kernel(const int32_t* __restrict__ parent,
                                                           const int32_t* __restrict__ rid,
                                                           const int32_t* __restrict__ keep,
                                                           uint8_t* __restrict__ occ,
                                                           int32_t* __restrict__ labels,
                                                           int32_t V) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= V)
        return;
    const int32_t p = parent[v];
    if (p >= 0) {
        const int32_t lab = keep[rid[p]];
        labels[v] = lab;
        if (lab == 0)
            occ[v] = 0;
    } else {
        labels[v] = 0;
    }
}

hipError_t launch_label(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                        uint32_t t_np, uint32_t t_nb, fvv_roi* rois, uint32_t max_rois,
                        uint32_t* n_rois, hipStream_t s) {
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const int32_t V = nx * ny * nz;
    const dim3 blocks3((nx + BX - 1) / BX, (ny + BY - 1) / BY, (nz + BZ - 1) / BZ);
    const unsigned chunks = (unsigned)((V + kRootChunk - 1) / kRootChunk);
    const unsigned vblocks = (unsigned)((V + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(ccl_local_kernel, blocks3, dim3(kBlock), 0, s, occ, ctx->d_parent, nx, ny,
                       nz);
    hipLaunchKernelGGL(ccl_merge_kernel, blocks3, dim3(kBlock), 0, s, ctx->d_parent, nx, ny, nz);
    hipLaunchKernelGGL(ccl_flatten_kernel, dim3(chunks), dim3(kBlock), 0, s, ctx->d_parent, V,
                       ctx->d_rootbits, ctx->d_blk_cnt);
    hipLaunchKernelGGL(ccl_number_kernel, dim3(chunks), dim3(kBlock), 0, s, ctx->d_rootbits,
                       ctx->d_blk_cnt, ctx->d_rid, ctx->d_stats, ctx->d_n_roots);
    hipLaunchKernelGGL(ccl_stats_kernel, dim3(vblocks), dim3(kBlock), 0, s, ctx->d_parent,
                       ctx->d_rid, ctx->d_stats, nx, ny, V);
    hipLaunchKernelGGL(ccl_filter_kernel, dim3(1), dim3(1024), 0, s, ctx->d_stats, ctx->d_n_roots,
                       ctx->d_keep, t_np, t_nb, rois, max_rois, n_rois, ctx->d_status);
    hipLaunchKernelGGL(ccl_write_kernel, dim3(vblocks), dim3(kBlock), 0, s, ctx->d_parent,
                       ctx->d_rid, ctx->d_keep, occ, labels, V);
    return hipGetLastError();
}

}  // namespace fvv
