// Connected components of the coarse occupancy, size filter, ROI boxes
// (Sec. II-B-2) and, in a frame, the fine lattice of every ROI (Sec. II-B-3)
// for gfx950.
//
// The coarse hull of a sports scene occupies well under 1 % of the volume, so
// the work is organised around the list of occupied samples rather than the
// grid.  Occupied samples are appended to a list, each with a union-find
// parent (itself), its list position and a stats row; the coarse carve of a
// frame does this as it writes the occupancy, fvv_label with a seed pass.
//
// Small lists (up to kLdsCap samples, the usual case) are labelled by ONE
// workgroup with the whole forest in LDS: union-find over list positions,
// linking the root with the larger linear index under the smaller with a CAS,
// then flattening, per-root count and bounding box, and the selection below
// -- one launch, no global round trips between the union steps.  Larger lists
// take a global path of three kernels (unite, flatten, select) with the same
// rules on the linear indices in global memory (atomicMin links).  Each path's
// kernels return at once when the list belongs to the other.
//
// Selection: roots flag themselves in a two-level bitmap; the non-zero words
// are walked in ascending order, so components are numbered 1..K by smallest
// linear index without a sort, after the Eq. (1) filter T_np <= N(S) <= T_nb.
// The selection clears the bitmap words it reads and the list count, so the
// scratch is ready for the next call without a memset.  A final grid pass
// writes the labels and the filtered occupancy.  Every root is the smallest
// linear index of its component whatever the interleaving of the atomics, so
// labels and boxes are identical from run to run.
#include "fvv_internal.h"

namespace fvv {

constexpr int kListBlocksPerCU = 4;
constexpr int kSelectThreads = 256;
constexpr int kSmallThreads = 512;
constexpr int kLdsCap = 8192;

// ------------------------------------------------------------------ helpers
// Root of x with path halving: each visited node is re-pointed at its
// grandparent.  Links only ever change roots (by CAS or atomicMin on a node
// that was a root), and a re-pointed node still reaches the same root through
// an ancestor, so halving races with neither links nor other finds.
__device__ __forceinline__ int32_t find_root(volatile int32_t* P, int32_t x) {
    for (;;) {
        const int32_t p = P[x];
        if (p == x)
            return x;
        const int32_t gp = P[p];
        if (gp == p)
            return p;
        P[x] = gp;
        x = gp;
    }
}

// Global forest over linear indices: the larger root is linked under the
// smaller with atomicMin; if that root was linked meanwhile, retry.
__device__ __forceinline__ void unite_global(int32_t* P, int32_t a, int32_t b) {
    for (;;) {
        a = find_root(P, a);
        b = find_root(P, b);
        if (a == b)
            return;
        if (a < b) {
            const int32_t old = atomicMin(&P[b], a);
            if (old == b)
                return;
            b = old;
        } else {
            const int32_t old = atomicMin(&P[a], b);
            if (old == a)
                return;
            a = old;
        }
    }
}

// LDS forest over list positions ordered by their linear indices L[]: the
// root with the larger linear index is linked under the other with a CAS that
// only succeeds while it is still a root.
__device__ __forceinline__ void unite_lds(int32_t* P, const int32_t* L, int32_t a, int32_t b) {
    for (;;) {
        a = find_root(P, a);
        b = find_root(P, b);
        if (a == b)
            return;
        if (L[a] < L[b]) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&P[a], a, b) == a)
            return;
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

__device__ __forceinline__ void coords_of(int32_t v, int nx, int ny, int& i, int& j, int& k) {
    const uint32_t uv = (uint32_t)v;
    i = (int)(uv % (uint32_t)nx);
    j = (int)((uv / (uint32_t)nx) % (uint32_t)ny);
    k = (int)(uv / ((uint32_t)nx * (uint32_t)ny));
}

// Add each active lane's sample (i, j, k) to the stats row of its root r: one
// set of atomics per (wave, root).
__device__ __forceinline__ void accumulate_stats(int32_t* __restrict__ stats, bool act, int32_t r,
                                                 int i, int j, int k) {
    uint64_t pending = __ballot(act);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lr = __shfl(r, leader, kWave);
        const bool mine = act && r == lr;
        const uint64_t mm = __ballot(mine);
        const int lo_i = wave_min(mine ? i : 0x7fffffff);
        const int lo_j = wave_min(mine ? j : 0x7fffffff);
        const int lo_k = wave_min(mine ? k : 0x7fffffff);
        const int hi_i = wave_max(mine ? i : -1);
        const int hi_j = wave_max(mine ? j : -1);
        const int hi_k = wave_max(mine ? k : -1);
        if (lane_id() == leader) {
            int32_t* s = stats + (int64_t)kStatsRow * lr;
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

// Load of a value other waves produced with device atomics, from L2 (not a
// possibly stale L1 line).
template <typename T>
__device__ __forceinline__ T coherent_load(T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_root(uint64_t* __restrict__ bits0, uint64_t* __restrict__ bits1,
                                          uint32_t v) {
    atomicOr((unsigned long long*)&bits0[v >> 6], 1ull << (v & 63));
    atomicOr((unsigned long long*)&bits1[v >> 12], 1ull << ((v >> 6) & 63));
}

// ------------------------------------------------------------------ fine jobs of a frame
__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

__device__ __forceinline__ int64_t ceil_div64(int64_t a, int64_t b) { return -floor_div64(-a, b); }

constexpr int64_t kMaxKeyedSamples = 1431655765;  // 3*lin+axis must fit 32 bits

// Map each ROI to its fine lattice (integer micrometres, one-coarse-cell
// dilation, clamped to the coarse lattice's extent), lay the carried ROIs out
// back to back in the fine occupancy buffer (the longest prefix that fits
// max_fine), and build the tile and work-item prefixes of the batched carve
// and the surface passes.  counts: [0] K, [1] fine samples, [3] ROIs carried.
template <int NT>
__device__ __forceinline__ void build_fine_jobs(const FrameJobs& fj,
                                                const fvv_roi* __restrict__ rois, uint32_t K_all,
                                                uint32_t max_rois, JobPrefix* __restrict__ pre,
                                                uint32_t* __restrict__ counter,
                                                fvv_camera* __restrict__ dcams,
                                                uint32_t* __restrict__ status) {
    __shared__ uint64_t scratch[NT / kWave];
    __shared__ uint64_t c_vox, c_tiles, c_items;
    __shared__ uint32_t carried;
    for (int c = threadIdx.x; c < fj.cams.n; c += NT) {
        fvv_camera cam;
        for (int e = 0; e < 12; ++e)
            cam.P[e] = fj.cams.P[c][e];
        cam.width = fj.cams.W;
        cam.height = fj.cams.H;
        dcams[c] = cam;
    }
    const uint32_t K = K_all < max_rois ? K_all : max_rois;
    if (threadIdx.x == 0) {
        c_vox = c_tiles = c_items = 0;
        carried = K;
    }
    __syncthreads();
    for (uint32_t base = 0; base < K; base += NT) {
        const uint32_t t = base + threadIdx.x;
        fvv_grid fg;
        int64_t V = 0;
        if (t < K) {
            const fvv_roi r = rois[t];
            V = 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t A = (int64_t)fj.coarse.lo[a] + r.lo[a] - 1;
                const int64_t B = (int64_t)fj.coarse.lo[a] + r.hi[a] + 1;
                int64_t f0 = floor_div64(A * fj.hc_um, fj.hf_um);
                int64_t f1 = ceil_div64(B * fj.hc_um, fj.hf_um);
                const int64_t fmin = ceil_div64((int64_t)fj.coarse.lo[a] * fj.hc_um, fj.hf_um);
                const int64_t fmax = floor_div64(
                    ((int64_t)fj.coarse.lo[a] + fj.coarse.dims[a] - 1) * fj.hc_um, fj.hf_um);
                f0 = f0 < fmin ? fmin : f0;
                f1 = f1 > fmax ? fmax : f1;
                fg.origin[a] = fj.coarse.origin[a];
                fg.lo[a] = (int32_t)f0;
                fg.dims[a] = (int32_t)(f1 - f0 + 1);
                V *= (f1 - f0 + 1);
            }
            fg.h = fj.h_fine;
        }
        uint64_t tot_v;
        const uint64_t ex_v = block_exclusive_sum64<NT>((uint64_t)V, scratch, &tot_v);
        const uint64_t off = c_vox + ex_v;
        const bool fits = t < K && off + (uint64_t)V <= (uint64_t)fj.max_fine &&
                          V <= kMaxKeyedSamples && t < carried;
        const uint64_t tiles = fits ? tiles_of_grid(fg, fj.tile_x, fj.tile_z) : 0;
        const uint64_t items = fits ? ((uint64_t)V + kEdgeChunk - 1) / kEdgeChunk : 0;
        uint64_t tot_t, tot_i;
        const uint64_t ex_t = block_exclusive_sum64<NT>(tiles, scratch, &tot_t);
        const uint64_t ex_i = block_exclusive_sum64<NT>(items, scratch, &tot_i);
        if (fits) {
            fvv_job j;
            j.grid = fg;
            j.cam_base = 0;
            j.n_cams = fj.cams.n;
            j.width = fj.cams.W;
            j.height = fj.cams.H;
            j.sil_base = 0;
            j.out_offset = (int64_t)off;
            fj.jobs[t] = j;
            pre[t].tile_off = c_tiles + ex_t;
            pre[t].item_off = (uint32_t)(c_items + ex_i);
        }
        if (t < K && !fits)
            atomicMin(&carried, t);     // the carried ROIs are the prefix that fits
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
        uint64_t vox = 0, tiles = 0, items = 0;   // totals over the carried prefix
        if (n > 0) {
            const fvv_job& last = fj.jobs[n - 1];
            const uint64_t Vl =
                (uint64_t)last.grid.dims[0] * last.grid.dims[1] * last.grid.dims[2];
            vox = (uint64_t)last.out_offset + Vl;
            tiles = pre[n - 1].tile_off + tiles_of_grid(last.grid, fj.tile_x, fj.tile_z);
            items = pre[n - 1].item_off + (Vl + kEdgeChunk - 1) / kEdgeChunk;
        }
        pre[n].tile_off = tiles;
        pre[n].item_off = (uint32_t)items;
        fj.counts[0] = K_all;
        fj.counts[1] = (uint32_t)(vox > 0xffffffffull ? 0xffffffffull : vox);
        fj.counts[3] = n;
        counter[0] = 0;
        counter[1] = grab_size(tiles, fj.blocks);
        counter[2] = n;
        if (n < K_all)
            atomicOr(status, kFlagCapacity);
    }
}

// ------------------------------------------------------------------ selection
struct SelectArgs {
    int32_t V;
    uint64_t* bits0;
    uint64_t* bits1;
    uint32_t* words;
    int32_t* stats;
    uint32_t t_np, t_nb;
    fvv_roi* rois;
    uint32_t max_rois;
    uint32_t* n_rois;
    uint32_t* list_count;
    uint32_t* status;
    JobPrefix* pre;
    uint32_t* counter;
    fvv_camera* dcams;
};

// Roots in ascending linear order -> Eq. (1) filter, labels 1..K, ROI table;
// then, in a frame, the fine jobs.  Run by one workgroup of NT threads.
template <int NT, bool kJobs>
__device__ __forceinline__ void select_roots(const SelectArgs& a, const FrameJobs& fj) {
    __shared__ uint32_t scratch[NT / kWave];
    const uint32_t n1 = (uint32_t)((a.V + 4095) / 4096);
    uint32_t nw = 0;
    for (uint32_t base = 0; base < n1; base += NT) {
        const uint32_t i = base + threadIdx.x;
        uint64_t w1 = 0;
        if (i < n1) {
            w1 = coherent_load(&a.bits1[i]);
            if (w1)
                a.bits1[i] = 0;
        }
        uint32_t total;
        uint32_t pos = nw + block_exclusive_sum<NT>((uint32_t)__popcll(w1), scratch, &total);
        while (w1) {
            const int b = __ffsll((unsigned long long)w1) - 1;
            w1 &= w1 - 1;
            a.words[pos++] = i * 64 + (uint32_t)b;
        }
        nw += total;
    }
    __syncthreads();
    uint32_t K = 0;
    for (uint32_t base = 0; base < nw; base += NT) {
        const uint32_t j = base + threadIdx.x;
        uint64_t w0 = 0;
        uint32_t wi = 0;
        if (j < nw) {
            wi = a.words[j];
            w0 = coherent_load(&a.bits0[wi]);
            a.bits0[wi] = 0;
        }
        uint32_t kc = 0;
        for (uint64_t m = w0; m; m &= m - 1) {
            const uint32_t v = wi * 64 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
            const uint32_t cnt = (uint32_t)coherent_load(&a.stats[(int64_t)kStatsRow * v]);
            kc += (a.t_np <= cnt && cnt <= a.t_nb) ? 1u : 0u;
        }
        uint32_t total;
        uint32_t lab = K + block_exclusive_sum<NT>(kc, scratch, &total);
        for (uint64_t m = w0; m; m &= m - 1) {
            const uint32_t v = wi * 64 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
            int32_t* s = a.stats + (int64_t)kStatsRow * v;
            const uint32_t cnt = (uint32_t)coherent_load(&s[0]);
            if (a.t_np <= cnt && cnt <= a.t_nb) {
                ++lab;
                s[7] = (int32_t)lab;
                if (lab <= a.max_rois) {
                    fvv_roi r;
                    r.lo[0] = coherent_load(&s[1]);
                    r.lo[1] = coherent_load(&s[2]);
                    r.lo[2] = coherent_load(&s[3]);
                    r.hi[0] = coherent_load(&s[4]);
                    r.hi[1] = coherent_load(&s[5]);
                    r.hi[2] = coherent_load(&s[6]);
                    r.count = cnt;
                    r.min_index = v;
                    a.rois[lab - 1] = r;
                }
            }
        }
        K += total;
    }
    if (threadIdx.x == 0) {
        *a.n_rois = K;
        *a.list_count = 0;
        if (K > a.max_rois)
            atomicOr(a.status, kFlagCapacity);
    }
    if (kJobs) {
        __syncthreads();
        build_fine_jobs<NT>(fj, a.rois, K, a.max_rois, a.pre, a.counter, a.dcams, a.status);
    }
}

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(kBlock) void ccl_seed_kernel(const uint8_t* __restrict__ occ,
                                                          int32_t V, const LabelSeed seed) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool on = v < V && occ[v] != 0;
    const uint64_t m = __ballot(on);
    if (m == 0)
        return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader)
        base = atomicAdd(seed.count, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if (on)
        seed_sample(seed, (int32_t)v, base + lane_rank(m));
}

// Global forest, one thread per (listed sample, earlier neighbour) from
// `first` in steps of `stride`.
__device__ __forceinline__ void unite_listed(const uint8_t* __restrict__ occ, int32_t* parent,
                                             const int32_t* __restrict__ list, uint32_t n, int nx,
                                             int ny, uint64_t first, uint64_t stride) {
    const uint64_t pairs = (uint64_t)n * 13;
    for (uint64_t idx = first; idx < pairs; idx += stride) {
        const int32_t v = list[idx / 13];
        const int q = (int)(idx % 13);
        int x, y, z, dx, dy, dz;
        coords_of(v, nx, ny, x, y, z);
        earlier_neighbour(q, dx, dy, dz);
        const int ax = x + dx, ay = y + dy, az = z + dz;
        if (ax < 0 || ax >= nx || ay < 0 || ay >= ny || az < 0)
            continue;
        const int32_t u = ax + nx * (ay + ny * az);
        if (occ[u] != 0)
            unite_global(parent, v, u);
    }
}

// Global forest: every listed sample points at its root, adds itself to the
// root's stats, and roots flag themselves.  Entry base + tid for base = first,
// first + stride, ...; whole waves iterate together.
__device__ __forceinline__ void flatten_listed(int32_t* parent, int32_t* __restrict__ stats,
                                               const int32_t* __restrict__ list, uint32_t n,
                                               uint64_t* bits0, uint64_t* bits1, int nx, int ny,
                                               uint32_t first, uint32_t stride, uint32_t tid) {
    for (uint32_t base = first; base < n; base += stride) {
        const uint32_t idx = base + tid;
        const bool act = idx < n;
        const int32_t v = act ? list[idx] : 0;
        const int32_t r = act ? find_root(parent, v) : -1;
        if (act && r != v)
            parent[v] = r;
        int i, j, k;
        coords_of(v, nx, ny, i, j, k);
        accumulate_stats(stats, act, r, i, j, k);
        if (act && r == v)
            flag_root(bits0, bits1, (uint32_t)v);
    }
}

// The whole labelling in one workgroup.  Lists of up to kLdsCap samples keep
// the forest in LDS; longer ones (kFallback) use the global forest with the
// same rules, still in this workgroup, or are left to the multi-workgroup
// kernels below (!kFallback).
template <bool kJobs, bool kFallback>
__global__ __launch_bounds__(kSmallThreads) void ccl_small_kernel(
    const uint8_t* __restrict__ occ, int32_t* __restrict__ parent,
    const int32_t* __restrict__ list, const int32_t* __restrict__ slot,
    const uint32_t* __restrict__ count, int nx, int ny, int nz, const SelectArgs sa,
    const FrameJobs fj) {
    __shared__ int32_t L[kLdsCap];
    __shared__ int32_t P[kLdsCap];
    const uint32_t n = *count;
    if (n > (uint32_t)kLdsCap) {
        if (!kFallback)
            return;
        unite_listed(occ, parent, list, n, nx, ny, threadIdx.x, kSmallThreads);
        __threadfence();
        __syncthreads();
        flatten_listed(parent, sa.stats, list, n, sa.bits0, sa.bits1, nx, ny, 0, kSmallThreads,
                       threadIdx.x);
        __threadfence();
        __syncthreads();
        select_roots<kSmallThreads, kJobs>(sa, fj);
        return;
    }
    for (uint32_t c = threadIdx.x; c < n; c += kSmallThreads) {
        L[c] = list[c];
        P[c] = (int32_t)c;
    }
    __syncthreads();
    for (uint32_t c = threadIdx.x; c < n; c += kSmallThreads) {
        const int32_t v = L[c];
        int x, y, z;
        coords_of(v, nx, ny, x, y, z);
        int32_t nb[13];
        bool on[13];
#pragma unroll
        for (int q = 0; q < 13; ++q) {
            int dx, dy, dz;
            earlier_neighbour(q, dx, dy, dz);
            const int ax = x + dx, ay = y + dy, az = z + dz;
            const bool in = ax >= 0 && ax < nx && ay >= 0 && ay < ny && az >= 0;
            nb[q] = in ? ax + nx * (ay + ny * az) : v;
            on[q] = in && occ[nb[q]] != 0;
        }
        int32_t other[13];
#pragma unroll
        for (int q = 0; q < 13; ++q)
            other[q] = on[q] ? slot[nb[q]] : (int32_t)c;
#pragma unroll
        for (int q = 0; q < 13; ++q)
            if (other[q] != (int32_t)c)
                unite_lds(P, L, (int32_t)c, other[q]);
    }
    __syncthreads();
    for (uint32_t base = 0; base < n; base += kSmallThreads) {
        const uint32_t c = base + threadIdx.x;
        const bool act = c < n;
        int32_t v = 0, r = 0;
        if (act) {
            v = L[c];
            r = L[find_root(P, (int32_t)c)];
            parent[v] = r;
            if (r == v)
                flag_root(sa.bits0, sa.bits1, (uint32_t)v);
        }
        int i, j, k;
        coords_of(v, nx, ny, i, j, k);
        accumulate_stats(sa.stats, act, r, i, j, k);
    }
    // one workgroup: the barrier orders the atomics above before the
    // selection's (L2-coherent) loads of their results
    __syncthreads();
    select_roots<kSmallThreads, kJobs>(sa, fj);
}

// Global path: one thread per (listed sample, earlier neighbour).
__global__ __launch_bounds__(kBlock) void ccl_unite_kernel(const uint8_t* __restrict__ occ,
                                                           int32_t* __restrict__ parent,
                                                           const int32_t* __restrict__ list,
                                                           const uint32_t* __restrict__ count,
                                                           int nx, int ny, int nz) {
    (void)nz;
    const uint32_t n = *count;
    if (n <= (uint32_t)kLdsCap)
        return;
    unite_listed(occ, parent, list, n, nx, ny, (uint64_t)blockIdx.x * kBlock + threadIdx.x,
                 (uint64_t)gridDim.x * kBlock);
}

__global__ __launch_bounds__(kBlock) void ccl_flatten_kernel(int32_t* __restrict__ parent,
                                                             int32_t* __restrict__ stats,
                                                             const int32_t* __restrict__ list,
                                                             const uint32_t* __restrict__ count,
                                                             uint64_t* __restrict__ bits0,
                                                             uint64_t* __restrict__ bits1, int nx,
                                                             int ny) {
    const uint32_t n = *count;
    if (n <= (uint32_t)kLdsCap)
        return;
    flatten_listed(parent, stats, list, n, bits0, bits1, nx, ny, blockIdx.x * kBlock,
                   gridDim.x * kBlock, threadIdx.x);
}

template <bool kJobs>
__global__ __launch_bounds__(kSelectThreads) void ccl_select_kernel(const uint32_t* __restrict__ count,
                                                                    const SelectArgs sa,
                                                                    const FrameJobs fj) {
    if (*count <= (uint32_t)kLdsCap)
        return;
    select_roots<kSelectThreads, kJobs>(sa, fj);
}

__global__ __launch_bounds__(kBlock) void ccl_write_kernel(const int32_t* __restrict__ parent,
                                                           const int32_t* __restrict__ stats,
                                                           uint8_t* __restrict__ occ,
                                                           int32_t* __restrict__ labels,
                                                           int32_t V) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= V)
        return;
    if (occ[v]) {
        const int32_t lab = stats[(int64_t)kStatsRow * parent[v] + 7];
        labels[v] = lab;
        if (lab == 0)
            occ[v] = 0;
    } else {
        labels[v] = 0;
    }
}

LabelSeed label_seed(fvv_ctx* ctx) {
    return LabelSeed{ctx->d_parent, ctx->d_stats, ctx->d_list, ctx->d_slot, ctx->d_list_count};
}

hipError_t launch_label(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                        uint32_t t_np, uint32_t t_nb, fvv_roi* rois, uint32_t max_rois,
                        uint32_t* n_rois, bool seeded, const FrameJobs* frame, hipStream_t s) {
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const int32_t V = nx * ny * nz;
    const unsigned vblocks = (unsigned)((V + kBlock - 1) / kBlock);
    const unsigned lblocks = (unsigned)(ctx->n_cus * kListBlocksPerCU);
    const LabelSeed seed = label_seed(ctx);
    SelectArgs sa;
    sa.V = V;
    sa.bits0 = ctx->d_bits0;
    sa.bits1 = ctx->d_bits1;
    sa.words = ctx->d_words;
    sa.stats = ctx->d_stats;
    sa.t_np = t_np;
    sa.t_nb = t_nb;
    sa.rois = rois;
    sa.max_rois = max_rois;
    sa.n_rois = n_rois;
    sa.list_count = ctx->d_list_count;
    sa.status = ctx->d_status;
    sa.pre = ctx->d_prefix;
    sa.counter = ctx->d_counter;
    sa.dcams = ctx->d_cams;
    const FrameJobs fj = frame ? *frame : FrameJobs{};
    if (!seeded)
        hipLaunchKernelGGL(ccl_seed_kernel, dim3(vblocks), dim3(kBlock), 0, s, occ, V, seed);
    if (frame) {
        // a frame's list is labelled by one workgroup whatever its length
        hipLaunchKernelGGL((ccl_small_kernel<true, true>), dim3(1), dim3(kSmallThreads), 0, s,
                           occ, ctx->d_parent, ctx->d_list, ctx->d_slot, ctx->d_list_count, nx, ny,
                           nz, sa, fj);
    } else {
        hipLaunchKernelGGL((ccl_small_kernel<false, false>), dim3(1), dim3(kSmallThreads), 0, s,
                           occ, ctx->d_parent, ctx->d_list, ctx->d_slot, ctx->d_list_count, nx, ny,
                           nz, sa, fj);
        hipLaunchKernelGGL(ccl_unite_kernel, dim3(lblocks), dim3(kBlock), 0, s, occ,
                           ctx->d_parent, ctx->d_list, ctx->d_list_count, nx, ny, nz);
        hipLaunchKernelGGL(ccl_flatten_kernel, dim3(lblocks), dim3(kBlock), 0, s, ctx->d_parent,
                           ctx->d_stats, ctx->d_list, ctx->d_list_count, ctx->d_bits0,
                           ctx->d_bits1, nx, ny);
        hipLaunchKernelGGL((ccl_select_kernel<false>), dim3(1), dim3(kSelectThreads), 0, s,
                           ctx->d_list_count, sa, fj);
    }
    if (!labels)
        return hipGetLastError();
    return launch_label_write(ctx, g, occ, labels, s);
}

// Labels and filtered occupancy of every sample (after launch_label).
hipError_t launch_label_write(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                              hipStream_t s) {
    const int32_t V = g.dims[0] * g.dims[1] * g.dims[2];
    const unsigned vblocks = (unsigned)((V + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(ccl_write_kernel, dim3(vblocks), dim3(kBlock), 0, s, ctx->d_parent,
                       ctx->d_stats, occ, labels, V);
    return hipGetLastError();
}

}  // namespace fvv
