// Silhouette packing and volumetric visual-hull carving (Sec. II-B-1 over the
// whole volume, Sec. II-B-3 inside ROIs) for gfx950.
//
// A workgroup of 256 threads carves a tile of TX x TY x TZ lattice samples
// (TX * TY = 256).  The tile keeps, in LDS, the list of its samples that are
// still inside every camera tested so far.  Each pass tests the listed samples
// against the next kCamGroup cameras (independent loads, one memory round trip
// per pass) and appends the survivors to the other list, so every lane of a
// pass works on a live sample: samples outside the lattice never enter the
// list and rejected ones leave it at once.  The tile is done when a pass
// leaves no survivor or the cameras run out; the survivors are the occupied
// samples.  The occupancy is the AND over all cameras, so neither the passes
// nor the order in which samples are listed change a result.  Each test
// evaluates the full fused projection chain of the sample, bit-equal to the
// definition.
#include "fvv_internal.h"

namespace fvv {

constexpr int kCamGroup = 2;

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
constexpr int log2_of(int v) { return v <= 1 ? 0 : 1 + log2_of(v / 2); }

// Append val to an LDS list for the lanes where pred holds (one LDS atomic
// per wave).
__device__ __forceinline__ void lds_append(bool pred, uint16_t val, uint16_t* list,
                                           uint32_t* count) {
    const uint64_t m = __ballot(pred);
    if (m == 0)
        return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader)
        base = atomicAdd(count, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if (pred)
        list[base + lane_rank(m)] = val;
}

// Carve tile `tile` of lattice g.  getP(c) returns camera c's 12 floats (a
// wave-uniform address); sil_of(c) its silhouette rows.  With kRows, the
// occupancy is also ORed into the labelling's row bitmap: the TX lanes of one
// tile row cover TX consecutive x inside one bitmap word (TX divides 64), so
// each tile row costs one atomic, and none where it is empty.
template <int TX, int TZ, bool kRows, typename GetP, typename GetSil>
__device__ __forceinline__ void carve_tile(GetP getP, GetSil sil_of, int ncam, int W, int H,
                                           int wpr, const fvv_grid& g, uint64_t tile,
                                           uint8_t* __restrict__ out, const RowBits& rb) {
    constexpr int TY = kBlock / TX;
    constexpr int TV = TX * TY * TZ;
    constexpr int LX = log2_of(TX), LY = log2_of(TY);
    __shared__ uint16_t s_list[2][TV];
    __shared__ uint32_t s_cnt[3];
    __shared__ uint32_t s_alive[TV / 32];

    const int ntx = (g.dims[0] + TX - 1) / TX;
    const int nty = (g.dims[1] + TY - 1) / TY;
    const int bx = (int)(tile % (uint64_t)ntx);
    const uint64_t r = tile / (uint64_t)ntx;
    const int by = (int)(r % (uint64_t)nty);
    const int bz = (int)(r / (uint64_t)nty);
    const int i0 = bx * TX, j0 = by * TY, k0 = bz * TZ;

    __syncthreads();   // the previous tile of this workgroup is done with the LDS
    if (threadIdx.x < 3)
        s_cnt[threadIdx.x] = 0;
    for (int w = threadIdx.x; w < TV / 32; w += kBlock)
        s_alive[w] = 0;
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < TZ; ++rr) {
        const int s = rr * kBlock + (int)threadIdx.x;
        const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
        const bool valid = i0 + lx < g.dims[0] && j0 + ly < g.dims[1] && k0 + lz < g.dims[2];
        lds_append(valid, (uint16_t)s, s_list[0], &s_cnt[0]);
    }
    __syncthreads();

    int cur = 0;
    for (int c0 = 0; c0 < ncam; c0 += kCamGroup) {
        const uint32_t n = s_cnt[cur % 3];
        if (n == 0)
            break;
        if (threadIdx.x == 0)
            s_cnt[(cur + 2) % 3] = 0;   // last read a pass ago, next appended to a pass on
        const float* P[kCamGroup];
        const uint32_t* sil[kCamGroup];
#pragma unroll
        for (int q = 0; q < kCamGroup; ++q) {
            const int c = c0 + q < ncam ? c0 + q : c0;   // wave-uniform
            P[q] = getP(c);
            sil[q] = sil_of(c);
        }
        const uint16_t* src = s_list[cur & 1];
        uint16_t* dst = s_list[(cur + 1) & 1];
        uint32_t* dcnt = &s_cnt[(cur + 1) % 3];
        // each wave takes 64 consecutive entries per round and stops as soon
        // as its next slice starts past the end of the list
        const uint32_t wave0 = (threadIdx.x / kWave) * kWave;
        for (uint32_t base = wave0; base < n; base += kBlock) {
            const uint32_t idx = base + lane_id();
            const bool act = idx < n;
            const int s = act ? src[idx] : 0;
            const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
            const float X = lattice_coord(g.lo[0] + i0 + lx, g.h, g.origin[0]);
            const float Y = lattice_coord(g.lo[1] + j0 + ly, g.h, g.origin[1]);
            const float Z = lattice_coord(g.lo[2] + k0 + lz, g.h, g.origin[2]);
            // all tests of the group are issued unconditionally (a camera past
            // the last one repeats camera c0 and cannot change the result), so
            // their silhouette loads are in flight together
            const bool in = group_inside<kCamGroup>(P, X, Y, Z, sil, W, H, wpr);
            lds_append(act && in, (uint16_t)s, dst, dcnt);
        }
        __syncthreads();
        ++cur;
    }

    const uint32_t n_in = s_cnt[cur % 3];
    const uint16_t* surv = s_list[cur & 1];
    for (uint32_t base = 0; base < n_in; base += kBlock) {
        const uint32_t idx = base + threadIdx.x;
        const bool act = idx < n_in;
        const int s = act ? surv[idx] : 0;
        if (act)
            atomicOr(&s_alive[s >> 5], 1u << (s & 31));
    }
    __syncthreads();
    const uint64_t plane = (uint64_t)g.dims[0] * (uint64_t)g.dims[1];
#pragma unroll
    for (int rr = 0; rr < TZ; ++rr) {
        const int s = rr * kBlock + (int)threadIdx.x;
        const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
        const int i = i0 + lx, j = j0 + ly, k = k0 + lz;
        const bool valid = i < g.dims[0] && j < g.dims[1] && k < g.dims[2];
        const uint32_t bit = (s_alive[s >> 5] >> (s & 31)) & 1u;
        if (valid)
            out[(uint64_t)k * plane + (uint64_t)j * g.dims[0] + i] = (uint8_t)bit;
        if (kRows) {
            // lanes [TX*q, TX*q + TX) of the wave hold one tile row (lx = 0..TX-1)
            const uint64_t m = __ballot(valid && bit != 0u);
            const int q = lane_id() / TX;
            const uint64_t bits = TX == 64 ? m : (m >> (q * TX)) & ((1ull << (TX & 63)) - 1);
            if (lx == 0 && bits != 0) {
                const int64_t row = (int64_t)j + (int64_t)g.dims[1] * k;
                atomicOr((unsigned long long*)&rb.words[row * rb.wr + (i0 >> 6)],
                         (unsigned long long)(bits << (i0 & 63)));
                atomicOr((unsigned long long*)&rb.rowmask[row >> 6], 1ull << (row & 63));
            }
        }
    }
}

// ------------------------------------------------------------------ one lattice
template <int TX, int TZ, bool kRows>
__global__ __launch_bounds__(kBlock) void carve_kernel(const CamSet cams,
                                                       const uint32_t* __restrict__ sils,
                                                       const fvv_grid g, uint8_t* __restrict__ occ,
                                                       const RowBits rb) {
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    carve_tile<TX, TZ, kRows>([&](int c) { return &cams.P[c][0]; },
                              [&](int c) { return sils + c * cam_words; }, cams.n, cams.W, cams.H,
                              cams.wpr, g, blockIdx.x, occ, rb);
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
        uint64_t t = j < n_jobs ? tiles_of_grid(jobs[j].grid, TX, TZ) : 0;
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
        counter[0] = 0;
        counter[1] = grab_size(total, blocks);
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
    const RowBits no_rows{};
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
            carve_tile<TX, TZ, false>([&](int c) { return &jc[c].P[0]; },
                                      [&](int c) { return js + c * cam_words; }, job.n_cams,
                                      job.width, job.height, wpr, job.grid, t - pre[jb].tile_off,
                                      out + job.out_offset, no_rows);
        }
    }
}

// ------------------------------------------------------------------ dispatch
#define FVV_TILE_CASES(X)                                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(32, 1) X(32, 2) X(32, 4) X(32, 8) X(16, 1)     \
    X(16, 2) X(16, 4) X(16, 8)

hipError_t launch_carve(const CamSet& cams, const uint32_t* sils, const fvv_grid& g, TileShape t,
                        uint8_t* occ, const RowBits* rows, hipStream_t s) {
    const uint64_t tiles = tiles_of_grid(g, t.tx, t.tz);
    if (tiles == 0)
        return hipSuccess;
    if (tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
    const RowBits rb = rows ? *rows : RowBits{};
#define X(TXV, TZV)                                                                           \
    if (t.tx == TXV && t.tz == TZV) {                                                         \
        if (rows)                                                                             \
            hipLaunchKernelGGL((carve_kernel<TXV, TZV, true>), dim3((unsigned)tiles),         \
                               dim3(kBlock), 0, s, cams, sils, g, occ, rb);                   \
        else                                                                                  \
            hipLaunchKernelGGL((carve_kernel<TXV, TZV, false>), dim3((unsigned)tiles),        \
                               dim3(kBlock), 0, s, cams, sils, g, occ, rb);                   \
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
